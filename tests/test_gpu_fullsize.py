"""Full-size workloads: sampled-cell parity and whole-batch cross-precision checks."""
import numpy as np
import pytest

from gpu_common import dev, invariant_indices, rel_err, say, torch
from oracle import apply as oapply
from oracle import core as ocore
from oracle_cache import coo

import paper_2605_28475_amd as wefq
from paper_2605_28475_amd import synth

pytestmark = pytest.mark.gpu


def _full(K, L, model, gamma, B, seed, sample, tol32, tol16):
    d = dev()
    say(f"[full] K={K} L={L} {model} B={B}")
    core = wefq.Core(model, K, L, gamma=gamma, device=0)
    c = synth.perturbed_maxwellian(K, L, B, seed=seed)
    f64 = torch.tensor(c, device=d)
    f32 = f64.float()
    q64 = core.apply_Q(f64)
    q32 = core.apply_Q(f32)
    q16 = core.apply_Q(f32, precision="bf16x3")
    torch.cuda.synchronize()
    ref = q64.cpu().numpy()
    e32 = rel_err(q32.cpu().numpy().astype(np.float64), ref)
    e16 = rel_err(q16.cpu().numpy().astype(np.float64), ref)
    say(f"[full] fp32 vs fp64 {e32:.3e}  bf16x3 vs fp64 {e16:.3e}")
    assert e32 < tol32 and e16 < tol16
    for q in (q64, q32, q16):
        assert core.check_conservation(q, precision="fp64" if q.dtype == torch.float64 else "fp32") == 0.0
    T = coo(L)
    R = ocore.zero_invariants(ocore.core_exact(K, L, gamma, table=T), T["channels"])
    idx = np.unique(np.linspace(0, B - 1, sample).astype(int))
    o = oapply.apply_q(R, T, c[idx], K)
    e64 = rel_err(ref[idx], o)
    say(f"[full] fp64 vs oracle on {len(idx)} cells {e64:.3e}")
    assert e64 < 1e-12
    core.close()


def test_k8_batch_maxwell_and_hard_sphere():
    _full(8, 8, "mm", 0.0, 4096, synth.BASE_SEED + 2, 64, 1e-5, 3e-5)
    _full(8, 8, "hs", 1.0, 4096, synth.BASE_SEED + 2, 64, 1e-5, 3e-5)


def test_k12_batch_vhs_B65536():
    _full(12, 12, "vhs", 0.5, 65536, synth.BASE_SEED + 3, 8, 1e-5, 3e-5)

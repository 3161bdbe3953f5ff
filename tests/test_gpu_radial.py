"""The radial-first ordering (wefq_apply_Q_radial, FP64) against the oracle and against the
angular-first kernel."""
import ctypes

import numpy as np
import pytest

from gpu_common import dev, invariant_indices, rel_err, say, torch
from oracle import apply as oapply
from oracle_cache import coo, core_zeroed

import paper_2605_28475_amd as wefq
from paper_2605_28475_amd import _lib, synth

pytestmark = pytest.mark.gpu
_cores = {}


def gpu_core(model, K, L, gamma):
    key = (model, K, L, gamma)
    if key not in _cores:
        say(f"[build] {key}")
        _cores[key] = wefq.Core(model, K, L, gamma=gamma, device=0, precisions=("fp64", "radial"))
    return _cores[key]


@pytest.mark.parametrize("K,L,model,gamma,B", [(3, 3, "hs", 1.0, 7), (4, 6, "vhs", 0.5, 70), (2, 5, "mm", 0.0, 3),
                                               (5, 2, "hs", 1.0, 130), (0, 4, "hs", 1.0, 5), (6, 0, "vhs", 0.5, 9)])
def test_radial_first_matches_oracle(K, L, model, gamma, B):
    core = gpu_core(model, K, L, gamma)
    c = synth.perturbed_maxwellian(K, L, B, seed=synth.BASE_SEED + 101 + K + L)
    say(f"[radial] K={K} L={L} {model} B={B}")
    got = core.apply_Q_radial(torch.tensor(c, device=dev())).cpu().numpy()
    ref = oapply.apply_q(core_zeroed(K, L, gamma), coo(L), c, K)
    assert rel_err(got, ref) < 1e-12
    assert np.all(got[:, invariant_indices(K, L)] == 0.0)


@pytest.mark.parametrize("K,L", [(4, 13), (12, 12)])
def test_radial_first_matches_angular_first(K, L):
    """At the sizes of the ordering comparison (K = 4, L = 13) and of the headline (K = L = 12):
    against the FP64 angular-first kernel, a different ordering of the same sum."""
    core = gpu_core("hs", K, L, 1.0)
    f = torch.tensor(synth.perturbed_maxwellian(K, L, 67, seed=9), device=dev())
    a = core.apply_Q(f, precision="fp64").cpu().numpy()
    r = core.apply_Q_radial(f).cpu().numpy()
    say(f"[radial vs angular] K={K} L={L}: {rel_err(r, a):.2e}")
    assert rel_err(r, a) < 1e-12


def test_radial_first_chunking_is_bitwise_neutral():
    """Every cell is computed in the same order whatever the chunk, so a batch split into
    64-cell chunks equals the same batch in one chunk, bit for bit."""
    K, L = 4, 5
    core = gpu_core("vhs", K, L, 0.5)
    f = torch.tensor(synth.perturbed_maxwellian(K, L, 200, seed=10), device=dev())
    one = core.apply_Q_radial(f, chunk=256)
    small = torch.empty(core.radial_workspace_bytes(64), dtype=torch.uint8, device=dev())
    many = core.apply_Q_radial(f, work=small)
    assert torch.equal(one, many)
    alone = core.apply_Q_radial(f[133:134].contiguous())
    assert torch.equal(alone[0], one[133])


def test_radial_first_errors():
    K, L = 3, 3
    core = gpu_core("hs", K, L, 1.0)
    N = core.N
    f = torch.tensor(synth.perturbed_maxwellian(K, L, 4, seed=1), device=dev())
    Q = torch.empty_like(f)
    per64 = core.radial_workspace_bytes(64)
    assert per64 == 64 * 8 * (N + core.info["radial_groups"] * (K + 1))
    assert core.radial_workspace_bytes(1) == per64 and core.radial_workspace_bytes(65) == 2 * per64
    work = torch.empty(2 * per64 + 256, dtype=torch.uint8, device=dev())
    L_ = _lib.lib()
    s = ctypes.c_void_p(torch.cuda.current_stream(dev()).cuda_stream)
    fp, qp, wp = (ctypes.c_void_p(t.data_ptr()) for t in (f, Q, work))
    h = core.handle
    assert L_.wefq_apply_Q_radial(h, fp, qp, 4, N, N, wp, per64 - 8, s) == _lib.WEFQ_EINVAL      # too small
    assert L_.wefq_apply_Q_radial(h, fp, qp, 4, N, N, ctypes.c_void_p(work.data_ptr() + 8), per64, s) == \
        _lib.WEFQ_EINVAL                                                                        # misaligned
    assert L_.wefq_apply_Q_radial(h, fp, fp, 4, N, N, wp, per64, s) == _lib.WEFQ_EINVAL          # f aliases Q
    assert L_.wefq_apply_Q_radial(h, fp, qp, 4, N, N, fp, per64, s) == _lib.WEFQ_EINVAL          # f in the workspace
    assert L_.wefq_apply_Q_radial(h, fp, qp, 4, N - 1, N, wp, per64, s) == _lib.WEFQ_EINVAL
    assert L_.wefq_apply_Q_radial(h, fp, qp, 0, N, N, wp, per64, s) == _lib.WEFQ_OK
    assert L_.wefq_apply_Q_radial(h, fp, qp, 4, N, N, wp, per64, s) == _lib.WEFQ_OK
    plain = wefq.Core("hs", K, L, device=0, precisions=("fp64",))
    n = ctypes.c_int64()
    assert L_.wefq_radial_workspace(plain.handle, 64, ctypes.byref(n)) == _lib.WEFQ_EINVAL
    assert L_.wefq_apply_Q_radial(plain.handle, fp, qp, 4, N, N, wp, per64, s) == _lib.WEFQ_EINVAL
    plain.close()
    torch.cuda.synchronize()


def test_radial_first_at_largest_truncation():
    """K = L = 16: 430,529 groups, 58.5 MB of workspace per cell; 70 cells in two chunks,
    against the FP64 angular-first kernel."""
    K = L = 16
    core = wefq.Core("hs", K, L, device=0, precisions=("fp64", "radial"))
    assert core.info["radial_groups"] > 400000
    f = torch.tensor(synth.perturbed_maxwellian(K, L, 70, seed=12), device=dev())
    a = core.apply_Q(f, precision="fp64").cpu().numpy()
    r = core.apply_Q_radial(f, chunk=64).cpu().numpy()
    say(f"[radial vs angular] K=L=16: {rel_err(r, a):.2e}")
    assert rel_err(r, a) < 1e-12
    assert np.all(r[:, invariant_indices(K, L)] == 0.0)
    core.close()

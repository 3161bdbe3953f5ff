"""The HIP path against stored oracle values (tests/golden/, written by make_golden.py, which
calls only oracle/):

* the single hard-sphere cell at K = L = 3 against the plain 8-D weak-form definition
  (Section 2.3), not the factorized oracle;
* K = L = 16, hard spheres and gamma = 0.5: sampled channels of the GPU-built core and
  Q(f, f) of two cells in every precision, alone in a batch, inside an uneven plan and
  through the continuous-batching server (eq. full_discrete_sum, Section 4.5).
"""
import os

import numpy as np
import pytest

from gpu_common import dev, invariant_indices, say, torch
from oracle_cache import golden

import paper_2605_28475_amd as wefq
from paper_2605_28475_amd import serve, synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
# max |GPU - oracle| / max |oracle| per precision (BF16x3: about twice its error model, the
# dropped lo x lo product and the rounding of the lo halves, about 2^-16 of each term)
TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 3e-5}
_cores = {}


def gpu_core(model, K, gamma):
    key = (model, K, gamma)
    if key not in _cores:
        say(f"[build] {key}")
        _cores[key] = wefq.Core(model, K, K, gamma=gamma, device=0)
    return _cores[key]


def k16_golden(model):
    z = np.load(os.path.join(GOLDEN, f"oracle_K16L16_{model}.npz"), allow_pickle=False)
    c = synth.perturbed_maxwellian(16, 16, len(z["Q"]), seed=int(z["seed"]))
    assert np.allclose(c.sum(axis=1), z["c_sum"], rtol=0, atol=1e-12), "seeded input generator drifted"
    return float(z["gamma"]), z["channels"], z["R"], c, z["Q"]


def rel(a, ref):
    return float(np.abs(np.asarray(a, dtype=np.float64) - ref).max() / np.abs(ref).max())


def run(core, c, prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    return core.apply_Q(torch.tensor(c, dtype=dt, device=dev()), precision=prec).cpu().numpy().astype(np.float64)


# ---------------------------------------------------------------- K = L = 3 vs the 8-D definition
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_single_cell_matches_weak_form_definition(prec):
    rows = np.array(golden("config1_hs_K3L3_weakform.txt"), dtype=np.float64)
    w = synth.WORKLOADS["single_cell"]
    c = synth.perturbed_maxwellian(3, 3, 1, seed=w["seed"])
    assert np.array_equal(rows[:, 1], c[0])
    ref = rows[:, 2]
    inv = invariant_indices(3, 3)
    assert np.abs(ref[inv]).max() < 5e-14 * np.abs(ref).max()       # the definition conserves (rounding)
    say(f"[config1] {prec}")
    q = run(gpu_core("hs", 3, 1.0), c, prec)[0]
    assert np.all(q[inv] == 0.0)                                     # the factorized path: exactly
    assert rel(q, ref) < TOL[prec]


# ---------------------------------------------------------------- K = L = 16
@pytest.mark.parametrize("model", ["hs", "vhs"])
def test_k16_core_sampled_channels(model):
    gamma, chans, Rref, _, _ = k16_golden(model)
    say(f"[k16 core] {model}")
    R = gpu_core(model, 16, gamma).download_R()
    # The two FP64 quadratures (GPU and oracle: different frames, rules and summation order)
    # sum polynomials of degree 3(2K + L) = 144 whose terms cancel; at K = L = 16 their rounding
    # differs by up to about 3e-12 of a channel's largest entry (1e-12 up to K = L = 12).
    # Q(f, f) still agrees to 1e-12 (test_k16_apply_matches_oracle).
    for i, ch in enumerate(chans):
        err = rel(R[ch], Rref[i])
        say(f"[k16 core] {model} channel {int(ch)}: {err:.2e}")
        assert err < 5e-12, int(ch)


def _batch(c_gold, n, seed):
    """n seeded cells with the oracle cells at rows 0 and n - 1 (a ragged last tile)."""
    c = synth.perturbed_maxwellian(16, 16, n, seed=seed)
    c[0], c[n - 1] = c_gold[0], c_gold[1]
    return c


@pytest.mark.parametrize("model", ["hs", "vhs"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_k16_apply_matches_oracle(model, prec):
    gamma, _, _, cg, qg = k16_golden(model)
    core = gpu_core(model, 16, gamma)
    c = _batch(cg, 13, seed=5)
    say(f"[k16 apply] {model} {prec}")
    q = run(core, c, prec)
    got = q[[0, 12]]
    assert rel(got, qg) < TOL[prec]
    assert np.all(q[:, invariant_indices(16, 16)] == 0.0)
    # the oracle cells alone (one cell per launch) are bitwise the rows of the batch
    alone = run(core, c[12:13], prec)
    assert np.array_equal(alone[0], q[12])


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_k16_plan_segment_matches_oracle(prec):
    """An uneven plan whose K = L = 16 segments carry the oracle cells, mixed with other cores."""
    d = dev()
    dt = torch.float64 if prec == "fp64" else torch.float32
    segs, gold = [], []
    for i, model in enumerate(("hs", "vhs")):
        gamma, _, _, cg, qg = k16_golden(model)
        c = _batch(cg, 21, seed=40 + i)
        f = torch.tensor(c, dtype=dt, device=d)
        segs.append((gpu_core(model, 16, gamma), f, torch.empty_like(f)))
        gold.append(qg)
    for K, model, gamma, B in ((4, "hs", 1.0, 45), (12, "vhs", 0.5, 30), (8, "hs", 1.0, 7)):
        f = torch.tensor(synth.perturbed_maxwellian(K, K, B, seed=60 + K), dtype=dt, device=d)
        segs.append((gpu_core(model, K, gamma), f, torch.empty_like(f)))
    plan = wefq.Plan(segs, precision=prec)
    say(f"[k16 plan] {prec} items={plan.info['work_items']}")
    plan.launch()
    torch.cuda.synchronize()
    for i, qg in enumerate(gold):
        q = segs[i][2].cpu().numpy().astype(np.float64)
        assert rel(q[[0, 20]], qg) < TOL[prec]
    for core, f, q in segs:
        assert torch.equal(q, core.apply_Q(f, precision=prec))


def test_k16_server_matches_oracle():
    """Requests served in a mix (K = L = 8 and 16, hard spheres, FP32) against the oracle cells
    and bitwise against standalone applies."""
    gamma, _, _, cg, qg = k16_golden("hs")
    d = dev()
    cores = [gpu_core("hs", 8, 1.0), gpu_core("hs", 16, 1.0)]
    pool16 = synth.perturbed_maxwellian(16, 16, 64, seed=71)
    pool16[10], pool16[11] = cg[0], cg[1]
    pools = [torch.tensor(synth.perturbed_maxwellian(8, 8, 256, seed=70), dtype=torch.float32, device=d),
             torch.tensor(pool16, dtype=torch.float32, device=d)]
    srv = serve.Server(torch, cores, pools, budget_bytes=64 << 20, streams=3)
    # (arrival s, core index, cells, pool offset): the oracle cells arrive inside two requests
    trace = [(0.0, 0, 100, 3), (0.0, 1, 2, 10), (0.0005, 0, 7, 200), (0.001, 1, 17, 0), (0.001, 0, 256, 0),
             (0.0015, 1, 1, 11), (0.002, 1, 40, 5), (0.002, 0, 1, 9)]
    say("[k16 serve]")
    res = srv.run(trace, keep_outputs=True)
    out = {r: res["outputs"][r].cpu().numpy().astype(np.float64) for r in range(len(trace))}
    assert rel(out[1], qg) < TOL["fp32"]
    assert rel(out[5][0], qg[1]) < TOL["fp32"]
    assert rel(out[3][10:12], qg) < TOL["fp32"]
    for rid, (_, k, n, off) in enumerate(trace):
        assert torch.equal(res["outputs"][rid], cores[k].apply_Q(pools[k][off:off + n])), rid

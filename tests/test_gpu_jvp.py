"""Two-input forms on the GPU against the oracle: the Jacobian-vector product
J(c) d = Q(c, d) + Q(d, c) (wefq_apply_J) and the bilinear form Q(f, g) (wefq_apply_Qfg)."""
import ctypes

import numpy as np
import pytest

from gpu_common import dev, invariant_indices, rel_err, say, torch
from oracle import apply as oapply
from oracle_cache import coo, core_raw, core_zeroed

import paper_2605_28475_amd as wefq
from paper_2605_28475_amd import _lib, synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}
_cores = {}


def gpu_core(model, K, L, gamma):
    key = (model, K, L, gamma)
    if key not in _cores:
        say(f"[build] {key}")
        _cores[key] = wefq.Core(model, K, L, gamma=gamma, device=0, precisions=("fp64", "fp32", "bilinear"))
    return _cores[key]


def tensor(c, prec):
    return torch.tensor(c, dtype=torch.float64 if prec == "fp64" else torch.float32, device=dev())


def jvp(core, c, d, prec):
    return core.apply_J(tensor(c, prec), tensor(d, prec), precision=prec).cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("K,L,model,gamma,B", [(3, 3, "hs", 1.0, 7), (4, 4, "vhs", 0.5, 19), (8, 8, "mm", 0.0, 5),
                                               (5, 2, "hs", 1.0, 3), (2, 6, "vhs", 0.5, 4), (0, 3, "hs", 1.0, 6),
                                               (4, 0, "vhs", 0.5, 5)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_jvp_matches_oracle(K, L, model, gamma, B, prec):
    core = gpu_core(model, K, L, gamma)
    c = synth.perturbed_maxwellian(K, L, B, seed=synth.BASE_SEED + 61 + K)
    rng = np.random.default_rng(K * 100 + L)
    d = 0.05 * rng.standard_normal(c.shape)
    say(f"[jvp] K={K} L={L} {model} B={B} {prec}")
    c_in = tensor(c, prec).cpu().numpy().astype(np.float64)      # as stored in the run's precision
    d_in = tensor(d, prec).cpu().numpy().astype(np.float64)
    ref = oapply.apply_jvp(core_zeroed(K, L, gamma), coo(L), c_in, d_in, K)
    got = jvp(core, c, d, prec)
    assert rel_err(got, ref) < TOL[prec]
    assert np.all(got[:, invariant_indices(K, L)] == 0.0)


@pytest.mark.parametrize("K,L,model,gamma", [(11, 11, "vhs", 0.5), (12, 12, "vhs", 0.5), (13, 13, "mm", 0.0),
                                             (14, 14, "hs", 1.0), (15, 15, "hs", 1.0), (16, 16, "hs", 1.0)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_jvp_polarization_large(K, L, model, gamma, prec):
    """At sizes the oracle does not reach in seconds: J(c) d = Q(c + d) - Q(c) - Q(d), with
    the three Q from the FP64 apply kernel (a different kernel: one input, full tiles)."""
    core = gpu_core(model, K, L, gamma)
    c = synth.perturbed_maxwellian(K, L, 3, seed=synth.BASE_SEED + 71)
    d = 0.05 * np.random.default_rng(K).standard_normal(c.shape)
    c_in = tensor(c, prec).cpu().numpy().astype(np.float64)
    d_in = tensor(d, prec).cpu().numpy().astype(np.float64)
    q = lambda x: core.apply_Q(tensor(x, "fp64"), precision="fp64").cpu().numpy()
    ref = q(c_in + d_in) - q(c_in) - q(d_in)
    got = jvp(core, c, d, prec)
    assert rel_err(got, ref) < max(TOL[prec], 1e-11)
    assert np.all(got[:, invariant_indices(K, L)] == 0.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_jvp_consistency_with_apply(prec):
    """J(c) c = 2 Q(c); J is linear in d (J(c)(2d) = 2 J(c) d bitwise); results per cell do
    not depend on the batch."""
    K = L = 6
    core = gpu_core("vhs", K, L, 0.5)
    c = synth.perturbed_maxwellian(K, L, 21, seed=13)
    d = synth.perturbed_maxwellian(K, L, 21, seed=14) - synth.unit_maxwellian(K, L, 21)
    q = core.apply_Q(tensor(c, prec), precision=prec).cpu().numpy().astype(np.float64)
    jcc = jvp(core, c, c, prec)
    assert rel_err(jcc, 2 * q) < TOL[prec]
    j1 = jvp(core, c, d, prec)
    j2 = jvp(core, c, 2 * d, prec)
    assert np.array_equal(j2, 2 * j1)
    one = jvp(core, c[7:8], d[7:8], prec)
    assert np.array_equal(one[0], j1[7])


def test_linearized_operator_from_jvp_matches_oracle():
    """Columns J(e_000) e_j of the linearized operator, all N in one batch (hard spheres)."""
    K = L = 4
    core = gpu_core("hs", K, L, 1.0)
    N = core.N
    c = np.zeros((N, N))
    c[:, 0] = 1.0
    d = np.eye(N)
    Lgpu = jvp(core, c, d, "fp64").T                  # column j = J(e0) e_j
    Lref = oapply.apply_jvp(core_zeroed(K, L, 1.0), coo(L), c, d, K).T
    assert rel_err(Lgpu, Lref) < 1e-12
    ev = np.linalg.eigvalsh(0.5 * (Lgpu + Lgpu.T))
    assert np.abs(Lgpu - Lgpu.T).max() < 1e-12 * np.abs(Lgpu).max()   # self-adjoint
    assert ev.max() < 1e-12 and np.sum(np.abs(ev) < 1e-12) == 5        # H-theorem, 5 invariants


def test_jvp_errors():
    K = L = 3
    core = gpu_core("hs", K, L, 1.0)
    N = core.N
    c = tensor(synth.perturbed_maxwellian(K, L, 4, seed=1), "fp64")
    out = torch.empty_like(c)
    s = ctypes.c_void_p(torch.cuda.current_stream(dev()).cuda_stream)
    L_ = _lib.lib()
    cp, op = ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(out.data_ptr())
    assert L_.wefq_apply_J(core.handle, _lib.BF16X3, cp, cp, op, 4, N, N, N, s) == _lib.WEFQ_EINVAL
    assert L_.wefq_apply_J(core.handle, _lib.FP64, cp, cp, cp, 4, N, N, N, s) == _lib.WEFQ_EINVAL
    assert L_.wefq_apply_J(core.handle, _lib.FP64, cp, None, op, 4, N, N, N, s) == _lib.WEFQ_EINVAL
    assert L_.wefq_apply_J(core.handle, _lib.FP64, cp, cp, op, 4, N, N, N - 1, s) == _lib.WEFQ_EINVAL
    assert L_.wefq_apply_J(core.handle, _lib.FP64, cp, cp, op, 0, N, N, N, s) == _lib.WEFQ_OK


def qfg(core, f, g, prec):
    return core.apply_Qfg(tensor(f, prec), tensor(g, prec), precision=prec).cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("K,L,model,gamma,B", [(3, 3, "hs", 1.0, 6), (4, 4, "vhs", 0.5, 9), (8, 8, "mm", 0.0, 3),
                                               (2, 6, "vhs", 0.5, 4), (5, 2, "hs", 1.0, 3), (0, 3, "hs", 1.0, 4),
                                               (4, 0, "mm", 0.0, 3)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_bilinear_matches_oracle(K, L, model, gamma, B, prec):
    """Q(f, g) against the oracle's literal bilinear sum with the core before the zeroing
    (the momentum and energy rows of Q(f, g) are not zero)."""
    core = gpu_core(model, K, L, gamma)
    f = synth.perturbed_maxwellian(K, L, B, seed=synth.BASE_SEED + 81 + K)
    g = synth.perturbed_maxwellian(K, L, B, seed=synth.BASE_SEED + 91 + K)
    g[:, 1:] += 0.1 * np.random.default_rng(K).standard_normal(g[:, 1:].shape)
    say(f"[qfg] K={K} L={L} {model} B={B} {prec}")
    f_in = tensor(f, prec).cpu().numpy().astype(np.float64)
    g_in = tensor(g, prec).cpu().numpy().astype(np.float64)
    ref = oapply.apply_bilinear(core_raw(K, L, gamma), coo(L), f_in, g_in, K)
    got = qfg(core, f, g, prec)
    assert rel_err(got, ref) < TOL[prec]
    assert np.all(got[:, 0] == 0.0)
    mom = invariant_indices(K, L)[1:]
    assert np.abs(ref[:, mom]).max() > 1e-3 * np.abs(ref).max()      # the rows are really there


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_bilinear_identities(prec):
    """Q(f, f) = Q(f); Q(f, g) + Q(g, f) = J(f) g; and for Maxwell molecules
    Q(f, g) - Q(g, f) = f_000 g - g_000 f (b0 = 1/(4 pi)) on every row."""
    K = L = 8
    core = gpu_core("mm", K, L, 0.0)
    f = synth.perturbed_maxwellian(K, L, 5, seed=21)
    g = synth.perturbed_maxwellian(K, L, 5, seed=22)
    g[:, 0] = 0.7
    tol = 1e-12 if prec == "fp64" else 1e-5
    q = core.apply_Q(tensor(f, prec), precision=prec).cpu().numpy().astype(np.float64)
    assert rel_err(qfg(core, f, f, prec), q) < tol
    fg, gf = qfg(core, f, g, prec), qfg(core, g, f, prec)
    assert rel_err(fg + gf, jvp(core, f, g, prec)) < tol
    f_in = tensor(f, prec).cpu().numpy().astype(np.float64)
    g_in = tensor(g, prec).cpu().numpy().astype(np.float64)
    anti = f_in[:, :1] * g_in - g_in[:, :1] * f_in
    anti[:, 0] = 0.0
    assert rel_err(fg - gf, anti) < 10 * tol


def test_bilinear_needs_prepared_tables():
    core = wefq.Core("hs", 3, 3, device=0, precisions=("fp64",))
    c = tensor(synth.perturbed_maxwellian(3, 3, 2, seed=1), "fp64")
    with pytest.raises(wefq.WefqError) as err:
        core.apply_Qfg(c, c, precision="fp64")
    assert err.value.status == _lib.WEFQ_EINVAL
    core.close()


@pytest.mark.parametrize("K,L", [(13, 13), (15, 15), (16, 16)])
def test_bilinear_large_fp64_against_fp32_and_identities(K, L):
    """FP64 Q(f, g) where it runs on tiles of 2 cells: Q(f, f) = Q(f) (the FP64 apply),
    Q(f, g) + Q(g, f) = J(f) g, and agreement with the FP32 bilinear form."""
    core = gpu_core("hs", K, L, 1.0)
    f = synth.perturbed_maxwellian(K, L, 5, seed=41)
    g = synth.perturbed_maxwellian(K, L, 5, seed=42)
    q = core.apply_Q(tensor(f, "fp64"), precision="fp64").cpu().numpy()
    assert rel_err(qfg(core, f, f, "fp64"), q) < 1e-12
    fg, gf = qfg(core, f, g, "fp64"), qfg(core, g, f, "fp64")
    assert rel_err(fg + gf, jvp(core, f, g, "fp64")) < 1e-12
    assert rel_err(qfg(core, f, g, "fp32"), fg) < 1e-5

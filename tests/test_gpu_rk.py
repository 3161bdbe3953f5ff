"""Batched explicit Runge-Kutta stepping on the GPU (wefq_rk_integrate) against the oracle."""
import ctypes
import math

import numpy as np
import pytest

from gpu_common import dev, invariant_indices, rel_err, say, torch
from oracle import rk as ork
from oracle_cache import coo, core_zeroed

import paper_2605_28475_amd as wefq
from paper_2605_28475_amd import _lib, synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp64_naive": 1e-12, "fp32": 1e-5, "bf16x3": 3e-5}
_cores = {}


def gpu_core(model, K, L, gamma):
    key = (model, K, L, gamma)
    if key not in _cores:
        say(f"[build] {key}")
        _cores[key] = wefq.Core(model, K, L, gamma=gamma, device=0)
    return _cores[key]


def tensor(c, prec):
    dt = torch.float64 if prec in ("fp64", "fp64_naive") else torch.float32
    return torch.tensor(c, dtype=dt, device=dev())


@pytest.mark.parametrize("scheme", ["euler", "heun", "ssp3", "rk4"])
@pytest.mark.parametrize("prec", ["fp64", "fp64_naive", "fp32", "bf16x3"])
def test_rk_matches_oracle(scheme, prec):
    K, L, B, dt, n = 3, 3, 5, 0.05, 3
    core = gpu_core("hs", K, L, 1.0)
    # start both sides from the coefficients as stored in the run's precision
    c0 = tensor(synth.perturbed_maxwellian(K, L, B, seed=synth.BASE_SEED + 41), prec).cpu().numpy().astype(np.float64)
    say(f"[rk] {scheme} {prec}")
    ref = ork.integrate(core_zeroed(K, L, 1.0), coo(L), c0, K, dt, n, scheme)
    c = tensor(c0, prec)
    inv = core.rk_integrate(c, dt, n, scheme=scheme, precision=prec)
    got = c.cpu().numpy().astype(np.float64)
    # The change over the run is what the operator contributes; compare it.  In FP32 storage
    # every step's update of c rounds c itself (unit roundoff 2^-24 of |c| ~ 1, once per step),
    # which the increment's relative error inherits; the bound is twice the precision's
    # tolerance plus that rounding.
    store = 0.0 if prec.startswith("fp64") else n * 2.0 ** -24 * np.abs(c0).max() / np.abs(ref - c0).max()
    err = rel_err(got - c0, ref - c0)
    say(f"[rk] {scheme} {prec}: increment error {err:.2e}, storage rounding {store:.2e}")
    assert err < 2 * (TOL[prec] + store)
    assert inv == 0.0
    idx = invariant_indices(K, L)
    assert np.array_equal(got[:, idx], c0[:, idx])


def test_rk4_follows_bkw_closed_form_on_gpu():
    """Maxwell molecules, K=L=8: RK4 from the BKW state at K0 = 0.6 to t = 1.2 lands on
    the closed form c(K(t)) within the oracle-measured RK4 error at that step."""
    from test_oracle import _bkw_coeffs
    kmax = L = 8
    core = gpu_core("mm", kmax, L, 0.0)
    K0, t_end, n = 0.6, 1.2, 12
    c0 = np.zeros((2, core.N))
    c0[:, :kmax + 1] = _bkw_coeffs(K0, kmax)
    exact = _bkw_coeffs(1.0 - (1.0 - K0) * math.exp(-t_end / 6.0), kmax)
    c = tensor(c0, "fp64")
    inv = core.rk_integrate(c, t_end / n, n, scheme="rk4", precision="fp64")
    got = c.cpu().numpy()
    assert inv == 0.0
    assert np.abs(got[:, :kmax + 1] - exact).max() < 2e-8        # RK4 error at dt = 0.1 is ~7e-9
    assert np.abs(got[:, kmax + 1:]).max() < 1e-13               # stays isotropic


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rk_cell_independent_of_batch(prec):
    K = L = 6
    core = gpu_core("vhs", K, L, 0.5)
    c0 = synth.perturbed_maxwellian(K, L, 33, seed=77)
    full = tensor(c0, prec)
    core.rk_integrate(full, 0.02, 2, precision=prec)
    one = tensor(c0[12:13], prec)
    core.rk_integrate(one, 0.02, 2, precision=prec)
    assert torch.equal(one[0], full[12])


def test_rk_strided_input_and_errors():
    K = L = 3
    core = gpu_core("hs", K, L, 1.0)
    N = core.N
    c0 = synth.perturbed_maxwellian(K, L, 4, seed=5)
    pad = torch.zeros((4, N + 7), dtype=torch.float64, device=dev())
    pad[:, :N] = tensor(c0, "fp64")
    ref = tensor(c0, "fp64")
    core.rk_integrate(ref, 0.1, 2, precision="fp64")
    core.rk_integrate(pad[:, :N], 0.1, 2, precision="fp64")
    assert torch.equal(pad[:, :N], ref)
    assert torch.all(pad[:, N:] == 0)
    h = core.handle
    L_ = _lib.lib()
    need = core.rk_workspace_bytes(4, "rk4", "fp64")
    work = torch.empty(need, dtype=torch.uint8, device=dev())
    c = tensor(c0, "fp64")
    cp = ctypes.c_void_p(c.data_ptr())
    wp = ctypes.c_void_p(work.data_ptr())
    s = ctypes.c_void_p(torch.cuda.current_stream(dev()).cuda_stream)
    res = ctypes.c_double()
    assert L_.wefq_rk_integrate(h, _lib.FP64, 9, cp, 4, N, 0.1, 1, wp, need, ctypes.byref(res), s) == _lib.WEFQ_EINVAL
    assert L_.wefq_rk_integrate(h, _lib.FP64, 4, cp, 4, N, 0.1, 1, wp, need - 8, ctypes.byref(res), s) == _lib.WEFQ_EINVAL
    assert L_.wefq_rk_integrate(h, _lib.FP64, 4, cp, 4, N, 0.1, 1, ctypes.c_void_p(work.data_ptr() + 8), need - 8,
                                ctypes.byref(res), s) == _lib.WEFQ_EINVAL
    assert L_.wefq_rk_integrate(h, _lib.FP64, 4, cp, 4, N - 1, 0.1, 1, wp, need, ctypes.byref(res), s) == _lib.WEFQ_EINVAL
    assert L_.wefq_rk_integrate(h, _lib.FP64, 4, cp, 4, N, float("nan"), 1, wp, need, ctypes.byref(res), s) == _lib.WEFQ_EINVAL
    assert L_.wefq_rk_integrate(h, _lib.FP64, 4, wp, 4, N, 0.1, 1, wp, need, ctypes.byref(res), s) == _lib.WEFQ_EINVAL
    # nothing ran: c is untouched
    assert torch.equal(c, tensor(c0, "fp64"))
    # zero steps or zero cells are no-ops
    assert L_.wefq_rk_integrate(h, _lib.FP64, 4, cp, 4, N, 0.1, 0, wp, need, ctypes.byref(res), s) == _lib.WEFQ_OK
    assert L_.wefq_rk_integrate(h, _lib.FP64, 4, cp, 0, N, 0.1, 3, None, 0, ctypes.byref(res), s) == _lib.WEFQ_OK
    assert torch.equal(c, tensor(c0, "fp64"))

"""Cores with an angular factor, B = b0 u^gamma beta(cos chi), on the GPU against the oracle
(the beta-weighted gain quadrature of the core build, and every apply path on such a core)."""
import math

import numpy as np
import pytest
from scipy.special import eval_legendre, roots_legendre

from gpu_common import dev, invariant_indices, rel_err, say, torch
from oracle import apply as oapply
from oracle_cache import coo, core_zeroed

import paper_2605_28475_amd as wefq
from paper_2605_28475_amd import _lib, synth

pytestmark = pytest.mark.gpu

BETA = (1.0, 0.5, 0.3, 0.1)                    # positive on [-1, 1]
EVEN = (0.8, 0.0, 0.4, 0.0, 0.2)
FORWARD = (1.0, 0.9, 0.6, 0.3, 0.12, 0.03, 0.005)   # degree 6, weighted to small deflections
_cores = {}


def gpu_core(model, K, L, gamma, beta):
    key = (model, K, L, gamma, beta)
    if key not in _cores:
        say(f"[build] {key}")
        _cores[key] = wefq.Core(model, K, L, gamma=gamma, device=0, beta=beta,
                                precisions=("fp64", "fp32", "bf16x3", "bilinear"))
    return _cores[key]


@pytest.mark.parametrize("K,L,model,gamma,beta", [(2, 2, "hs", 1.0, BETA), (3, 4, "mm", 0.0, EVEN),
                                                  (4, 3, "vhs", 0.5, BETA), (5, 5, "hs", 1.0, FORWARD),
                                                  (3, 6, "vhs", 1.5, BETA), (6, 1, "hs", 1.0, EVEN)])
def test_angular_core_matches_oracle(K, L, model, gamma, beta):
    dev()
    core = gpu_core(model, K, L, gamma, beta)
    assert core.beta == beta
    R = core.download_R()
    ref = core_zeroed(K, L, gamma, beta=beta).reshape(R.shape)
    say(f"[core] K={K} L={L} {model} beta={beta}: {rel_err(R, ref):.2e}")
    assert rel_err(R, ref) < 1e-12


def test_constant_factor_reproduces_isotropic_core():
    """beta = (1,) takes the direct beta-weighted gain quadrature and must agree with the
    isotropic closed form (Funk-Hecke) to rounding; beta = (b,) scales the core by b."""
    dev()
    K = L = 6
    iso = wefq.Core("vhs", K, L, gamma=0.5, device=0, precisions=("fp64",))
    one = gpu_core("vhs", K, L, 0.5, (1.0,))
    two = gpu_core("vhs", K, L, 0.5, (2.5,))
    Ri = iso.download_R()
    assert rel_err(one.download_R(), Ri) < 1e-13
    assert rel_err(two.download_R(), 2.5 * Ri) < 1e-13
    iso.close()


@pytest.mark.parametrize("prec", ["fp64", "fp64_naive", "fp32", "bf16x3"])
def test_angular_apply_matches_oracle(prec):
    K, L = 5, 4
    core = gpu_core("hs", K, L, 1.0, BETA)
    c = synth.perturbed_maxwellian(K, L, 37, seed=synth.BASE_SEED + 5)
    dt = torch.float64 if prec.startswith("fp64") else torch.float32
    f = torch.tensor(c, dtype=dt, device=dev())
    ref = oapply.apply_q(core_zeroed(K, L, 1.0, beta=BETA), coo(L), f.cpu().numpy().astype(np.float64), K)
    got = core.apply_Q(f, precision=prec).cpu().numpy().astype(np.float64)
    tol = {"fp64": 1e-12, "fp64_naive": 1e-12, "fp32": 1e-5, "bf16x3": 3e-5}[prec]
    assert rel_err(got, ref) < tol
    assert np.all(got[:, invariant_indices(K, L)] == 0.0)


def test_angular_bilinear_matches_oracle():
    K, L = 4, 4
    core = gpu_core("vhs", K, L, 0.5, BETA)
    from oracle_cache import core_raw
    f = synth.perturbed_maxwellian(K, L, 6, seed=31)
    g = synth.perturbed_maxwellian(K, L, 6, seed=32)
    ref = oapply.apply_bilinear(core_raw(K, L, 0.5, beta=BETA), coo(L), f, g, K)
    got = core.apply_Qfg(torch.tensor(f, device=dev()), torch.tensor(g, device=dev()), precision="fp64")
    assert rel_err(got.cpu().numpy(), ref) < 1e-12


def test_only_even_part_enters_q_on_gpu():
    """beta(t) and beta(-t) give different cores but the same Q(f, f) (post-collision
    velocities swapped); the bilinear form tells them apart."""
    K, L = 6, 6
    flip = tuple(b * (-1) ** j for j, b in enumerate(BETA))
    a, b = gpu_core("hs", K, L, 1.0, BETA), gpu_core("hs", K, L, 1.0, flip)
    assert rel_err(a.download_R(), b.download_R()) > 0.1
    f = torch.tensor(synth.perturbed_maxwellian(K, L, 9, seed=4), device=dev())
    g = torch.flip(f, dims=[0]).contiguous()
    qa = a.apply_Q(f, precision="fp64").cpu().numpy()
    qb = b.apply_Q(f, precision="fp64").cpu().numpy()
    assert rel_err(qa, qb) < 1e-12
    ga = a.apply_Qfg(f, g, precision="fp64").cpu().numpy()
    gb = b.apply_Qfg(f, g, precision="fp64").cpu().numpy()
    assert rel_err(ga, gb) > 1e-3


def _wcu_beta(k, l, beta, b0=1.0 / (4 * math.pi)):
    t, w = roots_legendre(60)
    c, s = np.sqrt((1 + t) / 2), np.sqrt((1 - t) / 2)
    f = c ** (2 * k + l) * eval_legendre(l, c) + s ** (2 * k + l) * eval_legendre(l, s) - 1 - (k == 0 and l == 0)
    bt = sum(bj * eval_legendre(j, t) for j, bj in enumerate(beta))
    return 2 * math.pi * b0 * float(w @ (bt * f))


@pytest.mark.parametrize("beta", [BETA, FORWARD])
def test_maxwell_spectrum_at_full_size(beta):
    """Maxwell molecules, K = L = 12 (2,197 modes): the linearized operator J(e_000), all
    columns in one FP64 batch, is diagonal with the Wang Chang-Uhlenbeck eigenvalues of the
    angular factor (a closed form, independent of the oracle)."""
    K = L = 12
    core = gpu_core("mm", K, L, 0.0, beta)
    N = core.N
    c = torch.zeros((N, N), dtype=torch.float64, device=dev())
    c[:, 0] = 1.0
    d = torch.eye(N, dtype=torch.float64, device=dev())
    Lm = core.apply_J(c, d, precision="fp64").cpu().numpy().T
    lam = np.array([_wcu_beta(k, l, beta) for l in range(L + 1) for m in range(-l, l + 1) for k in range(K + 1)])
    scale = np.abs(lam).max()
    err_diag = np.abs(np.diag(Lm) - lam).max() / scale
    err_off = np.abs(Lm - np.diag(np.diag(Lm))).max() / scale
    say(f"[wcu] K=L=12 beta={beta}: diag {err_diag:.2e} off {err_off:.2e}")
    assert err_diag < 1e-12 and err_off < 1e-12


def test_angular_core_serialization(tmp_path):
    dev()
    a = gpu_core("vhs", 4, 4, 0.5, BETA)
    path = tmp_path / "angular.wefq"
    a.save(path)
    b = wefq.Core.load(path, precisions=("fp64",), device=0)
    assert b.beta == BETA and b.gamma == a.gamma
    assert np.array_equal(a.download_R(), b.download_R())
    b.close()


def test_maxwell_spectrum_at_largest_truncation():
    """K = L = 16 (4,913 modes), where the two-input FP64 kernel does not fit LDS: the
    linearized operator by polarization of the FP64 apply, L e_j = Q(e0 + e_j) - Q(e0) - Q(e_j),
    against the Wang Chang-Uhlenbeck eigenvalues of the angular factor."""
    K = L = 16
    beta = EVEN
    core = wefq.Core("mm", K, L, device=0, beta=beta, precisions=("fp64",))
    N = core.N
    e0 = torch.zeros((N, N), dtype=torch.float64, device=dev())
    e0[:, 0] = 1.0
    d = torch.eye(N, dtype=torch.float64, device=dev())
    q = lambda x: core.apply_Q(x, precision="fp64")
    Lm = (q(e0 + d) - q(e0) - q(d)).cpu().numpy().T
    lam = np.array([_wcu_beta(k, l, beta) for l in range(L + 1) for m in range(-l, l + 1) for k in range(K + 1)])
    scale = np.abs(lam).max()
    err_diag = np.abs(np.diag(Lm) - lam).max() / scale
    err_off = np.abs(Lm - np.diag(np.diag(Lm))).max() / scale
    say(f"[wcu] K=L=16 beta={beta}: diag {err_diag:.2e} off {err_off:.2e}")
    assert err_diag < 1e-11 and err_off < 1e-11
    core.close()


def test_largest_angular_degree_and_zero_kernel():
    """n_beta = WEFQ_MAX_BETA (degree 32) against the oracle; beta = 0 gives a zero operator."""
    dev()
    K, L = 2, 3
    beta = tuple(1.0 / (1 + j) ** 2 for j in range(_lib.MAX_BETA))
    core = wefq.Core("hs", K, L, device=0, beta=beta, precisions=("fp64",))
    assert core.beta == beta
    R = core.download_R()
    ref = core_zeroed(K, L, 1.0, beta=beta).reshape(R.shape)
    say(f"[core] degree 32: {rel_err(R, ref):.2e}")
    assert rel_err(R, ref) < 1e-12
    core.close()
    zero = wefq.Core("vhs", 4, 4, gamma=0.5, device=0, beta=(0.0,), precisions=("fp64", "fp32"))
    assert np.all(zero.download_R() == 0.0)
    f = torch.tensor(synth.perturbed_maxwellian(4, 4, 3, seed=2), device=dev())
    assert torch.all(zero.apply_Q(f, precision="fp64") == 0)
    zero.close()

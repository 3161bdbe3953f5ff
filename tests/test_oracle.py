"""Pins of the FP64 oracle against what the paper and the mathematics fix."""
import math

import numpy as np
import pytest
from scipy.special import factorial, roots_genlaguerre, roots_hermite, roots_legendre, eval_legendre

from oracle import apply, basis, core, gaunt, rk, weakform
from oracle_cache import coo, core_raw, core_zeroed, golden

B0 = 1.0 / (4 * math.pi)


# ---------------------------------------------------------------- basis
def test_basis_orthonormal_under_reference_maxwellian():
    """Identity mass matrix (Section 2.3) and the closed forms of the invariants."""
    K, L = 3, 3
    x, w = roots_hermite(12)
    X = math.sqrt(2) * np.stack(np.meshgrid(x, x, x, indexing="ij"), -1).reshape(-1, 3)
    W = math.pi ** -1.5 * np.einsum("i,j,k->ijk", w, w, w).ravel()
    P = basis.basis_all(K, L, X)
    gram = (P * W[:, None]).T @ P
    assert np.abs(gram - np.eye(P.shape[1])).max() < 1e-13
    v2 = np.sum(X * X, axis=1)
    assert np.allclose(P[:, basis.mode_index(K, 0, 0, 0)], 1.0, atol=1e-14)
    assert np.allclose(P[:, basis.mode_index(K, 1, 0, 0)], math.sqrt(2 / 3) * (1.5 - v2 / 2), atol=1e-12)
    for m, comp in ((1, 0), (-1, 1), (0, 2)):       # momentum modes are v_x, v_y, v_z
        assert np.allclose(P[:, basis.mode_index(K, 0, 1, m)], X[:, comp], atol=1e-12)


# ---------------------------------------------------------------- Gaunt / COO
def test_table1_coo_rows_and_channel_count():
    T = coo(4)
    assert len(T["g"]) == 1158 and len(T["channels"]) == 42
    for z, q1, q2, q3, c, g in golden("table1_coo_L4.txt"):
        i = int(z) - 1
        assert (T["q1"][i] + 1, T["q2"][i] + 1, T["q3"][i] + 1, T["c"][i] + 1) == \
            (int(q1), int(q2), int(q3), int(c))
        assert round(T["g"][i], 4) == float(g)


def test_table6_gaunt_nonzeros_and_dofs():
    for L, dofs, nnz, naive_gb in golden("table6_counts.txt"):
        L = int(L)
        assert basis.num_modes(4, L) == int(dofs)
        if L <= 12:
            assert len(coo(L)["g"]) == int(nnz)
        # the printed dense size is N^3 FP64 values in GiB, to within its rounding
        assert basis.num_modes(4, L) ** 3 * 8 / 2 ** 30 == pytest.approx(float(naive_gb), rel=0.012)


def _threej000(l1, l2, l3):
    J = l1 + l2 + l3
    if J % 2:
        return 0.0
    g = J // 2
    f = factorial
    return (-1) ** g * math.sqrt(f(J - 2 * l1) * f(J - 2 * l2) * f(J - 2 * l3) / f(J + 1)) * \
        f(g) / (f(g - l1) * f(g - l2) * f(g - l3))


def test_gaunt_closed_form_norms():
    """sum over m of g^2 per channel = (2l1+1)(2l2+1)(2l3+1)/(4pi) (l1 l2 l3;0 0 0)^2."""
    L = 8
    T = coo(L)
    S = np.bincount(T["c"], weights=T["g"] ** 2)
    for ci, (l1, l2, l3) in enumerate(T["channels"]):
        ref = (2 * l1 + 1) * (2 * l2 + 1) * (2 * l3 + 1) / (4 * math.pi) * _threej000(l1, l2, l3) ** 2
        assert abs(S[ci] - ref) < 1e-13 * ref
    # g(q, q, Y00) = 1/sqrt(4 pi) for every q
    sel = T["q3"] == 0
    assert np.allclose(T["g"][sel], 1 / math.sqrt(4 * math.pi), atol=1e-15)
    assert np.array_equal(T["q1"][sel], T["q2"][sel])


# ---------------------------------------------------------------- 8-D definition
@pytest.mark.parametrize("gamma", [0.0, 0.5, 1.0])
def test_bruteforce_conservation_and_equilibrium(gamma):
    K, L = 2, 2
    N = basis.num_modes(K, L)
    e0 = np.zeros(N); e0[0] = 1.0
    assert np.abs(weakform.q_bruteforce(e0, K, L, gamma)).max() < 1e-14
    c = e0 + 0.1 * np.random.default_rng(7).standard_normal(N)
    Q = weakform.q_bruteforce(c, K, L, gamma)
    inv = [basis.mode_index(K, 0, 0, 0), basis.mode_index(K, 1, 0, 0)] + \
        [basis.mode_index(K, 0, 1, m) for m in (-1, 0, 1)]
    assert np.abs(Q[inv]).max() < 1e-14 * np.abs(Q).max()
    assert np.abs(Q).max() > 1e-3


def test_factorization_is_exact_and_core_matches_definition():
    """C = R^{(c)} g entry-wise (eq. wigner-eckart-factorization); exact core = C/g."""
    K, L, gamma = 2, 2, 1.0
    C = weakform.c_tensor_bruteforce(K, L, gamma)
    T = coo(L)
    Rb = core.core_from_tensor(C, K, L, T)
    Re = core_raw(K, L, gamma)
    scale = np.abs(Rb).max()
    assert np.abs(Rb - Re).max() < 1e-14 * scale
    NK, ks = K + 1, np.arange(K + 1)
    Cr = np.zeros_like(C)
    for q1, q2, q3, c, g in zip(T["q1"], T["q2"], T["q3"], T["c"], T["g"]):
        Cr[np.ix_(q1 * NK + ks, q2 * NK + ks, q3 * NK + ks)] += g * Rb[c]
    assert np.abs(C - Cr).max() < 1e-14 * np.abs(C).max()


@pytest.mark.parametrize("gamma", [0.0, 0.5])
def test_bruteforce_q_matches_factorized_sum(gamma):
    K, L = 2, 2
    N = basis.num_modes(K, L)
    c = np.zeros(N); c[0] = 1.0
    c += 0.05 * np.random.default_rng(3).standard_normal(N)
    Qd = weakform.q_bruteforce(c, K, L, gamma)
    Qf = apply.apply_q(core_zeroed(K, L, gamma), coo(L), c, K)
    assert np.abs(Qd - Qf).max() < 2e-14 * np.abs(Qd).max()


def test_bruteforce_core_matches_reduced_core_beyond_l3():
    """The 8-D definition against the reduced quadrature entry-wise at L = 4 (channels up to
    l = 4, gamma = 0.5): R = sum_m g C / sum_m g^2 of the brute-force tensor equals core_exact."""
    K, L, gamma = 1, 4, 0.5
    T = coo(L)
    Rb = core.core_from_tensor(weakform.c_tensor_bruteforce(K, L, gamma), K, L, T)
    Re = core_raw(K, L, gamma)
    assert max(max(ch) for ch in T["channels"]) == 4
    assert np.abs(Rb - Re).max() < 1e-14 * np.abs(Rb).max()


def test_single_cell_golden_matches_factorized_oracle():
    """The stored 8-D weak-form Q of the single hard-sphere cell at K = L = 3 (written by
    golden/make_golden.py from oracle/weakform.py) equals the factorized sum with the reduced
    core, and its invariant rows vanish up to rounding (Section 4.4)."""
    rows = np.array(golden("config1_hs_K3L3_weakform.txt"), dtype=np.float64)
    c, Qd = rows[:, 1], rows[:, 2]
    Qf = apply.apply_q(core_zeroed(3, 3, 1.0), coo(3), c, 3)
    scale = np.abs(Qd).max()
    assert np.abs(Qd - Qf).max() < 1e-13 * scale
    inv = [basis.mode_index(3, 0, 0, 0), basis.mode_index(3, 1, 0, 0)] + \
        [basis.mode_index(3, 0, 1, m) for m in (-1, 0, 1)]
    assert np.abs(Qd[inv]).max() < 5e-14 * scale and np.all(Qf[inv] == 0.0)


def test_gain_sphere_vs_funk_hecke_and_truncation_independence():
    T = coo(3)
    a = core.core_exact(2, 3, 0.5, table=T)
    b = core.core_exact(2, 3, 0.5, table=T, gain="sphere")
    assert np.abs(a - b).max() < 1e-14 * np.abs(a).max()
    big = core_raw(5, 4, 0.5)
    chans4 = coo(4)["channels"]
    for ci, ch in enumerate(T["channels"]):
        blk = big[chans4.index(ch)][:3, :3, :3]
        assert np.abs(blk - a[ci]).max() < 2e-14 * np.abs(a).max()


# ---------------------------------------------------------------- zeroing
def test_zeroed_rows_and_exact_invariants_of_factorized_sum():
    K, L = 3, 3
    R = core_zeroed(K, L, 1.0)
    T = coo(L)
    N = basis.num_modes(K, L)
    c = np.zeros(N); c[0] = 1.0
    assert np.all(apply.apply_q(R, T, c, K) == 0.0)                     # Q(M, M) = 0
    c += 0.05 * np.random.default_rng(1).standard_normal(N)
    Q = apply.apply_q(R, T, c, K)
    inv = [basis.mode_index(K, 0, 0, 0), basis.mode_index(K, 1, 0, 0)] + \
        [basis.mode_index(K, 0, 1, m) for m in (-1, 0, 1)]
    assert np.all(Q[inv] == 0.0)


# ---------------------------------------------------------------- Maxwell molecules
def test_maxwell_degree_triangularity():
    """For gamma = 0, C vanishes unless deg(a2) + deg(a3) <= deg(a1), deg = 2k + l."""
    K = L = 8
    R = core_raw(K, L, 0.0)
    chans = coo(L)["channels"]
    k = np.arange(K + 1)
    scale = np.abs(R).max()
    for ci, (l1, l2, l3) in enumerate(chans):
        d1 = 2 * k[:, None, None] + l1
        d23 = 2 * k[None, :, None] + l2 + 2 * k[None, None, :] + l3
        assert np.abs(R[ci][d23 > d1]).max(initial=0.0) < 1e-13 * scale


def _wcu(k, l, b0=B0):
    t, w = roots_legendre(40)
    c, s = np.sqrt((1 + t) / 2), np.sqrt((1 - t) / 2)
    f = c ** (2 * k + l) * eval_legendre(l, c) + s ** (2 * k + l) * eval_legendre(l, s) - 1 - (k == 0 and l == 0)
    return 2 * math.pi * b0 * float(w @ f)


def _linearized(R, chans, K, L):
    N = basis.num_modes(K, L)
    NK = K + 1
    Lm = np.zeros((N, N))
    for i, (k1, l1, m1) in enumerate(basis.mode_table(K, L)):
        q = l1 * l1 + l1 + m1
        a, b = chans.index((l1, 0, l1)), chans.index((l1, l1, 0))
        Lm[i, q * NK:(q + 1) * NK] = (R[a][k1, 0, :] + R[b][k1, :, 0]) / math.sqrt(4 * math.pi)
    return Lm


def test_wang_chang_uhlenbeck_spectrum_table3():
    K, L = 4, 6
    Lm = _linearized(core_zeroed(K, L, 0.0), coo(L)["channels"], K, L)
    modes = basis.mode_table(K, L)
    lam = np.array([_wcu(k, l) for k, l, m in modes])
    assert np.abs(Lm - np.diag(lam)).max() < 2e-14
    ev = np.linalg.eigvals(Lm)
    assert np.abs(ev.imag).max() < 1e-14
    ev = np.sort(ev.real)[::-1]
    ratio = ev / abs(ev[5])
    # twice the printed bound, floored at 2e-14: the FP64 rounding of the operator's entries
    # (lambda_6 = -1/3 comes out 4e-15 off) exceeds the printed 3e-15 of the -1 group
    for first, last, r, bound in golden("table3_wcu.txt"):
        seg = ratio[int(first) - 1:int(last)]
        assert np.abs(seg - float(r)).max() <= max(2 * float(bound), 2e-14)
    assert ratio.min() >= -3.0                   # WCU lower bound
    assert abs(ev[5] - (-4 * math.pi * B0 / 3)) < 1e-14


def _bkw_coeffs(Kt, kmax):
    """c_k(K) = int f_K phi_{k00} d^3v for the BKW profile (Section 5.2.1)."""
    x, w = roots_genlaguerre(kmax + 3, 0.5)
    v = np.sqrt(2 * Kt * x)
    pref = math.sqrt(4 * math.pi) * (2 * math.pi * Kt) ** -1.5 * Kt * math.sqrt(2 * Kt)
    poly = (5 * Kt - 3) / (2 * Kt) + (1 - Kt) * x / Kt
    return np.array([pref * np.sum(w * poly * basis.radial(k, 0, v)) for k in range(kmax + 1)])


def test_bkw_identity():
    """Q(c(K))_{k00} = (2 pi b0 / 3)(1 - K) dc_k/dK for every k (exact for gamma = 0)."""
    kmax, L = 8, 2
    R = core_zeroed(kmax, L, 0.0)
    T = coo(L)
    Ks = np.linspace(0.55, 1.05, kmax + 4)
    coefs = np.array([_bkw_coeffs(Kt, kmax) for Kt in Ks])
    for Kt in (0.6, 0.8, 0.95):
        ck = _bkw_coeffs(Kt, kmax)
        dck = np.array([np.polyval(np.polyder(np.polyfit(Ks, coefs[:, k], kmax + 2)), Kt)
                        for k in range(kmax + 1)])
        f = np.zeros(basis.num_modes(kmax, L))
        f[:kmax + 1] = ck                          # l = 0 block, n = k
        Q = apply.apply_q(R, T, f, kmax)
        rhs = 2 * math.pi * B0 / 3 * (1 - Kt) * dck
        assert np.abs(Q[:kmax + 1] - rhs).max() < 1e-10 * max(1.0, np.abs(rhs).max())
        assert np.abs(Q[kmax + 1:]).max() < 1e-14


def test_bilinear_form_and_jacobian():
    """Q(f, g) reduces to Q(f) on the diagonal, and the Jacobian-vector product obeys the
    polarization identity Q(c + d) - Q(c) - Q(d) = J(c) d (exact for a quadratic form);
    the collision tensor is not symmetric in its two inputs (the loss term), so the
    bilinear form is not either."""
    K, L = 3, 3
    R = core_zeroed(K, L, 1.0)
    T = coo(L)
    rng = np.random.default_rng(3)
    c = rng.standard_normal(basis.num_modes(K, L))
    d = rng.standard_normal(basis.num_modes(K, L))
    qc = apply.apply_q(R, T, c, K)
    assert np.abs(apply.apply_bilinear(R, T, c, c, K) - qc).max() < 1e-13 * np.abs(qc).max()
    j = apply.apply_jvp(R, T, c, d, K)
    pol = apply.apply_q(R, T, c + d, K) - qc - apply.apply_q(R, T, d, K)
    assert np.abs(j - pol).max() < 1e-12 * np.abs(j).max()
    assert np.abs(apply.apply_jvp(R, T, c, c, K) - 2 * qc).max() < 1e-13 * np.abs(qc).max()
    asym = apply.apply_bilinear(R, T, c, d, K) - apply.apply_bilinear(R, T, d, c, K)
    assert np.abs(asym).max() > 1e-3 * np.abs(j).max()


def test_bilinear_antisymmetric_part_maxwell_molecules():
    """For Maxwell molecules (B = b0 constant) the gain term is symmetric in the two inputs
    and the loss term of Q(f, g) is -4 pi b0 g_000 f, so with the unzeroed core
    Q(f, g) - Q(g, f) = 4 pi b0 (f_000 g - g_000 f) on every row, momentum and energy included."""
    K, L = 3, 2
    R = core_raw(K, L, 0.0)
    T = coo(L)
    rng = np.random.default_rng(11)
    f = rng.standard_normal(basis.num_modes(K, L))
    g = rng.standard_normal(basis.num_modes(K, L))
    lhs = apply.apply_bilinear(R, T, f, g, K) - apply.apply_bilinear(R, T, g, f, K)
    rhs = 4 * math.pi * B0 * (f[0] * g - g[0] * f)
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()


def test_rk_schemes_reach_bkw_at_their_order():
    """The BKW coefficients c(K(t)), K(t) = 1 - (1 - K0) exp(-t/6), solve the truncated
    system dc/dt = Q(c) exactly (Maxwell molecules, b0 = 1/(4 pi)), so the integration
    error is the scheme's alone: halving dt divides it by 2^p for a scheme of order p."""
    kmax, L = 6, 0
    R = core_zeroed(kmax, L, 0.0)
    T = coo(L)
    K0, t_end = 0.6, 1.2
    exact = _bkw_coeffs(1.0 - (1.0 - K0) * math.exp(-t_end / 6.0), kmax)
    c0 = _bkw_coeffs(K0, kmax)
    for scheme, order in (("euler", 1), ("heun", 2), ("ssp3", 3), ("rk4", 4)):
        errs = []
        for n in (6, 12):
            c = rk.integrate(R, T, c0, kmax, t_end / n, n, scheme)
            assert c[0] == c0[0] and c[1] == c0[1]          # mass and energy rows
            errs.append(np.abs(c - exact).max())
        ratio = errs[0] / errs[1]
        assert 0.8 * 2 ** order < ratio < 1.25 * 2 ** order, (scheme, errs)
    assert errs[1] < 1e-8                                   # rk4 at dt = 0.1


# ---------------------------------------------------------------- hard spheres
def test_chapman_enskog_viscosity_table4():
    Kmax = 8
    chans = coo(2)["channels"]
    R = core_zeroed(Kmax, 2, 1.0)
    L2 = (R[chans.index((2, 0, 2))][:, 0, :] + R[chans.index((2, 2, 0))][:, :, 0]) / math.sqrt(4 * math.pi)
    fmu = [L2[0, 0] * np.linalg.inv(L2[:K + 1, :K + 1])[0, 0] for K in range(Kmax + 1)]
    table = golden("table4_viscosity.txt")
    for K, val in table[:-1]:
        assert abs(fmu[int(K)] - float(val)) <= 5e-7
    assert abs(fmu[1] - 205 / 202) < 1e-13
    assert all(b > a for a, b in zip(fmu, fmu[1:]))
    assert 1.016028 < fmu[8] <= float(table[-1][1]) + 5e-7


@pytest.mark.parametrize("gamma", [0.5, 1.0])
def test_linearized_symmetric_negative_semidefinite(gamma):
    K, L = 4, 4
    Lm = _linearized(core_zeroed(K, L, gamma), coo(L)["channels"], K, L)
    assert np.abs(Lm - Lm.T).max() < 1e-13
    ev = np.linalg.eigvalsh(0.5 * (Lm + Lm.T))
    assert np.sum(np.abs(ev) < 1e-12) == 5
    assert ev.max() < 1e-12


def test_galilean_shift_table5():
    """Invariant rows of Q(c_U) are exactly 0 and the residual grows like U^8."""
    K, L = 4, 6
    R = core_zeroed(K, L, 0.0)
    T = coo(L)
    x, w = roots_hermite(10)
    X = np.stack(np.meshgrid(x, x, x, indexing="ij"), -1).reshape(-1, 3)
    W = np.einsum("i,j,k->ijk", w, w, w).ravel()
    inv = [basis.mode_index(K, 0, 0, 0), basis.mode_index(K, 1, 0, 0)] + \
        [basis.mode_index(K, 0, 1, m) for m in (-1, 0, 1)]
    norms = {}
    for U, _, cons in golden("table5_galilean.txt"):
        c = math.pi ** -1.5 * W @ basis.basis_all(K, L, np.array([float(U), 0, 0]) + math.sqrt(2) * X)
        Q = apply.apply_q(R, T, c, K)
        assert np.all(Q[inv] == 0.0) and float(cons) == 0.0
        norms[float(U)] = np.linalg.norm(Q)
    assert norms[0.0] < 1e-14
    assert abs(math.log(norms[0.3] / norms[0.1]) / math.log(3) - 8) < 0.05
    assert abs(math.log(norms[0.6] / norms[0.3]) / math.log(2) - 8) < 0.1


def test_rotation_equivariance_of_factorized_sum():
    """Q(D c) = D Q(c) for a random rotation (isotropic kernel, SO(3) covariance)."""
    from rotation import random_rotation, rotate, wigner_blocks
    K, L = 3, 4
    R = core_zeroed(K, L, 0.5)
    T = coo(L)
    blocks = wigner_blocks(L, random_rotation(5))
    for D in blocks:
        assert np.abs(D @ D.T - np.eye(len(D))).max() < 1e-13
    c = np.zeros((2, basis.num_modes(K, L))); c[:, 0] = 1.0
    c += 0.05 * np.random.default_rng(2).standard_normal(c.shape)
    Qc = apply.apply_q(R, T, c, K)
    Qr = apply.apply_q(R, T, rotate(c, K, L, blocks), K)
    assert np.abs(Qr - rotate(Qc, K, L, blocks)).max() < 1e-14 * np.abs(Qc).max() * 10


# ---------------------------------------------------------------- anisotropic scattering
BETA = (1.0, 0.5, 0.3, 0.1)          # beta(t) = 1 + 0.5 P1 + 0.3 P2 + 0.1 P3 > 0 on [-1, 1]


def test_anisotropic_core_matches_bruteforce_definition():
    """B = b0 u^gamma beta(cos chi): the reduced quadrature (relative-velocity frame, beta-weighted
    sphere rule per node) equals the 8-D definition taken literally (Section 2.3)."""
    K, L, gamma = 2, 2, 1.0
    T = coo(L)
    Rb = core.core_from_tensor(weakform.c_tensor_bruteforce(K, L, gamma, beta=BETA), K, L, T)
    Re = core_raw(K, L, gamma, beta=BETA)
    assert np.abs(Rb - Re).max() < 1e-14 * np.abs(Rb).max()
    # the angular factor really changed the core; beta = 1 is the isotropic kernel
    assert np.abs(Re - core_raw(K, L, gamma)).max() > 0.1 * np.abs(Re).max()
    iso = core.core_exact(K, L, gamma, table=T, beta=[1.0])
    assert np.abs(iso - core_raw(K, L, gamma)).max() < 1e-14 * np.abs(iso).max()


def _wcu_beta(k, l, beta, b0=B0):
    t, w = roots_legendre(40)
    c, s = np.sqrt((1 + t) / 2), np.sqrt((1 - t) / 2)
    f = c ** (2 * k + l) * eval_legendre(l, c) + s ** (2 * k + l) * eval_legendre(l, s) - 1 - (k == 0 and l == 0)
    bt = sum(bj * eval_legendre(j, t) for j, bj in enumerate(beta))
    return 2 * math.pi * b0 * float(w @ (bt * f))


def test_anisotropic_maxwell_spectrum_wang_chang_uhlenbeck():
    """Maxwell molecules with any angular factor: the linearized operator is diagonal in the
    Burnett basis with lambda_kl = 2 pi b0 int beta(t) [c^{2k+l} P_l(c) + s^{2k+l} P_l(s)
    - 1 - delta_k0 delta_l0] dt, c = cos(chi/2), s = sin(chi/2) (Wang Chang and Uhlenbeck)."""
    K, L = 3, 4
    Lm = _linearized(core_zeroed(K, L, 0.0, beta=BETA), coo(L)["channels"], K, L)
    lam = np.array([_wcu_beta(k, l, BETA) for k, l, m in basis.mode_table(K, L)])
    assert np.abs(Lm - np.diag(lam)).max() < 1e-14
    assert np.abs(lam - np.array([_wcu(k, l) for k, l, m in basis.mode_table(K, L)])).max() > 0.02


def test_anisotropic_only_even_part_enters_q():
    """Swapping the post-collision velocities (n -> -n) turns beta(t) into beta(-t) and leaves
    Q(f, f) unchanged, while the unsymmetrized core and Q(f, g) do change."""
    K, L = 3, 3
    flip = tuple(b * (-1) ** j for j, b in enumerate(BETA))
    T = coo(L)
    rng = np.random.default_rng(7)
    c = np.zeros((2, basis.num_modes(K, L))); c[:, 0] = 1.0
    c += 0.1 * rng.standard_normal(c.shape)
    qa = apply.apply_q(core_zeroed(K, L, 0.5, beta=BETA), T, c, K)
    qb = apply.apply_q(core_zeroed(K, L, 0.5, beta=flip), T, c, K)
    assert np.abs(qa - qb).max() < 1e-14 * np.abs(qa).max()
    Ra, Rb = core_raw(K, L, 0.5, beta=BETA), core_raw(K, L, 0.5, beta=flip)
    assert np.abs(Ra - Rb).max() > 0.1 * np.abs(Ra).max()
    ga = apply.apply_bilinear(Ra, T, c[0], c[1], K)
    gb = apply.apply_bilinear(Rb, T, c[0], c[1], K)
    assert np.abs(ga - gb).max() > 1e-3 * np.abs(ga).max()


def test_anisotropic_conservation_before_zeroing():
    """Mass, momentum and energy are collision invariants for any B: with the unzeroed core
    the five invariant rows of Q vanish to rounding, and so does Q of the Maxwellian."""
    K, L = 3, 3
    R = core_raw(K, L, 1.0, beta=BETA)
    T = coo(L)
    c = np.zeros(basis.num_modes(K, L)); c[0] = 1.0
    e0 = c.copy()
    c += 0.1 * np.random.default_rng(8).standard_normal(c.shape)
    Q = apply.apply_q(R, T, c, K)
    inv = [basis.mode_index(K, 0, 0, 0), basis.mode_index(K, 1, 0, 0)] + \
        [basis.mode_index(K, 0, 1, m) for m in (-1, 0, 1)]
    assert np.abs(Q[inv]).max() < 1e-14 * np.abs(Q).max()
    assert np.abs(apply.apply_q(R, T, e0, K)).max() < 1e-14


def test_anisotropic_maxwell_antisymmetric_part():
    """Maxwell molecules with an even angular factor: the gain of Q(f, g) is symmetric in
    the inputs and the loss is -4 pi b0 beta_0 g_000 f, so
    Q(f, g) - Q(g, f) = 4 pi b0 beta_0 (f_000 g - g_000 f) with the unzeroed core."""
    K, L = 3, 2
    beta = (0.8, 0.0, 0.4, 0.0, 0.2)
    R = core_raw(K, L, 0.0, beta=beta)
    T = coo(L)
    rng = np.random.default_rng(12)
    f = rng.standard_normal(basis.num_modes(K, L))
    g = rng.standard_normal(basis.num_modes(K, L))
    lhs = apply.apply_bilinear(R, T, f, g, K) - apply.apply_bilinear(R, T, g, f, K)
    rhs = 4 * math.pi * B0 * beta[0] * (f[0] * g - g[0] * f)
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()


@pytest.mark.parametrize("model", ["hs", "vhs"])
def test_k16_golden_consistent_with_small_truncation(model):
    """The stored K = L = 16 oracle values (golden/make_golden.py): entries of R do not depend
    on the truncation, so the k, l <= 3 block of the stored (0,0,0) channel equals the K = L = 3
    core (Section 4.1: R depends on the channel and the radial indices only); the stored Q has
    exactly zero invariant rows (Section 4.4 zeroing)."""
    import os
    z = np.load(os.path.join(os.path.dirname(__file__), "golden", f"oracle_K16L16_{model}.npz"),
                allow_pickle=False)
    gamma = float(z["gamma"])
    assert int(z["channels"][0]) == 0 and coo(16)["channels"][0] == (0, 0, 0)
    small = core_zeroed(3, 3, gamma)[0]
    assert np.abs(z["R"][0][:4, :4, :4] - small).max() < 1e-13 * np.abs(small).max()
    inv = [basis.mode_index(16, 0, 0, 0), basis.mode_index(16, 1, 0, 0)] + \
        [basis.mode_index(16, 0, 1, m) for m in (-1, 0, 1)]
    assert np.all(z["Q"][:, inv] == 0.0) and np.abs(z["Q"]).max() > 1e-4

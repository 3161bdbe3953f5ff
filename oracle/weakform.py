"""Brute-force quadrature of the 8-D weak form (Section 2.3, eqs. for C+ and C-).

Definition followed:
    C_{a1 a2 a3} = int dv int dw int du' B(u) [phi_a1(v') - phi_a1(v)]
                   phi_a2(v) phi_a3(w) M(v) M(w),       v' = (v + w + u u')/2,
    Q_a1(c)      = sum_{a2,a3} C_{a1 a2 a3} c_a2 c_a3          (Section 2.3),
with B = b0 u^gamma beta(cos chi) (Grad cut-off) and M the reference Maxwellian.
cos chi = u_hat . u' is the deflection angle (Section 2.1).  beta is a polynomial
given by its Legendre coefficients, beta(t) = sum_j beta_j P_j(t); beta = None
is the isotropic kernel beta = 1.

Exact evaluation (no singular quadrature is needed in these variables):
with G = (v+w)/2 and u = v - w = rho u_hat (unit Jacobian),
    M(v)M(w) = (2pi)^-3 exp(-|G|^2 - rho^2/4),  v' = G + (rho/2) n, n in S^2,
    C = b0 (2pi)^-3 int dG e^{-|G|^2} int_0^inf rho^{2+gamma} e^{-rho^2/4} drho
        int du_hat [A_a1(G,rho) - 4pi phi_a1(v)] phi_a2(v) phi_a3(w),
    A_a1(G,rho) = int dn phi_a1(G + (rho/2) n).
With an angular factor the gain and loss weights become int dn beta(u_hat . n)
phi_a1(G + (rho/2) n) and phi_a1(v) int dn beta(u_hat . n), both taken literally
at every (G, u_hat) node.
Everything except the weights is a polynomial of total degree <= 3D, D = 2K+L:
  * G: tensor Gauss-Hermite (weight e^{-x^2}) exact to degree 3D per axis;
  * rho: s = rho^2/4 turns rho^{2+gamma} drho into 2^{2+gamma} s^{(1+gamma)/2} ds;
    the u_hat-integrated integrand is even in rho, so generalized Gauss-Laguerre
    in s (alpha = (1+gamma)/2) is exact;
  * u_hat: product sphere rule exact to degree 3D + J (J the degree of beta);
    n: exact to degree D + J.
The result is therefore exact up to FP64 rounding, for any gamma >= 0.
"""
import math

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy.special import roots_genlaguerre, roots_hermite

from .basis import basis_all, num_modes
from .gaunt import sphere_rule

B0_DEFAULT = 1.0 / (4.0 * math.pi)


def angular_factor(beta, t):
    """beta(t) = sum_j beta_j P_j(t); beta = None is the isotropic factor 1."""
    t = np.asarray(t, dtype=np.float64)
    if beta is None:
        return np.ones_like(t)
    return npleg.legval(t, np.asarray(beta, dtype=np.float64))


def _degree(beta):
    return 0 if beta is None else len(beta) - 1


def _rules(K, L, gamma, beta=None):
    D = 2 * K + L
    J = _degree(beta)
    xg, wg = roots_hermite(3 * D // 2 + 1)
    G = np.stack(np.meshgrid(xg, xg, xg, indexing="ij"), axis=-1).reshape(-1, 3)
    WG = np.einsum("i,j,k->ijk", wg, wg, wg).ravel()
    s, ws = roots_genlaguerre((3 * D) // 2 // 2 + 1, 0.5 * (1.0 + gamma))
    U, WU = sphere_rule(3 * D + J)
    Nn, WN = sphere_rule(D + J)
    return G, WG, s, ws, U, WU, Nn, WN


def _sweep(K, L, gamma, b0, consume, chunk=48, beta=None):
    """Visit all quadrature points; call consume(W, dA, phi_v, phi_w)."""
    G, WG, s, ws, U, WU, Nn, WN = _rules(K, L, gamma, beta)
    pref = b0 * (2 * math.pi) ** -3 * 2.0 ** (2.0 + gamma)
    nU, nN = len(WU), len(WN)
    # scattering weights beta(u_hat . n) dn for every (u_hat, n) pair, and their sums
    Bn = angular_factor(beta, U @ Nn.T) * WN[None, :]            # (nU, nN)
    loss = Bn.sum(axis=1)                                          # int dn beta, per u_hat
    for si in range(len(s)):
        rho = 2.0 * math.sqrt(s[si])
        for g0 in range(0, len(WG), chunk):
            Gc = G[g0:g0 + chunk]
            nc = len(Gc)
            # gain: weighted sphere average of the test function around G
            Pn = Gc[:, None, :] + 0.5 * rho * Nn[None, :, :]
            phn = basis_all(K, L, Pn.reshape(-1, 3)).reshape(nc, nN, -1)
            A = np.einsum("gnj,un->guj", phn, Bn).reshape(nc * nU, -1)
            V = (Gc[:, None, :] + 0.5 * rho * U[None, :, :]).reshape(-1, 3)
            Wv = (Gc[:, None, :] - 0.5 * rho * U[None, :, :]).reshape(-1, 3)
            phv = basis_all(K, L, V)
            phw = basis_all(K, L, Wv)
            dA = A - np.tile(loss, nc)[:, None] * phv
            W = pref * ws[si] * np.outer(WG[g0:g0 + chunk], WU).ravel()
            consume(W, dA, phv, phw)


def q_bruteforce(c, K, L, gamma, b0=B0_DEFAULT, beta=None):
    """Q(c, c) from the 8-D definition; c is a length-N coefficient vector."""
    c = np.asarray(c, dtype=np.float64)
    Q = np.zeros(num_modes(K, L))

    def consume(W, dA, phv, phw):
        Q[:] += (W * (phv @ c) * (phw @ c)) @ dA

    _sweep(K, L, gamma, b0, consume, beta=beta)
    return Q


def c_tensor_bruteforce(K, L, gamma, b0=B0_DEFAULT, beta=None):
    """Full tensor C[a1, a2, a3] from the 8-D definition (tiny bases only)."""
    N = num_modes(K, L)
    C = np.zeros((N, N * N))

    def consume(W, dA, phv, phw):
        kr = (phv[:, :, None] * phw[:, None, :]).reshape(len(W), N * N)
        C[:] += (dA * W[:, None]).T @ kr

    _sweep(K, L, gamma, b0, consume, chunk=16, beta=beta)
    return C.reshape(N, N, N)

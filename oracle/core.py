"""Radial kinematic core R^{(c)}_{k1 k2 k3} (Sections 3.2-3.3 and 4.1, 4.4).

R is defined convention-free from the weak-form tensor C of Section 2.3 and the
real Gaunt weights g of Section 4.1 through the factorization C = R^{(c)} g:
    R^{(c)}_{k1k2k3} = sum_{m's} g_{q1q2q3} C_{(k1q1)(k2q2)(k3q3)} / S_c,
    S_c = sum_{m's} g_{q1q2q3}^2   (sums over the channel's COO rows).
Two independent evaluations are provided:

core_from_tensor   applies this definition to a brute-force C (weakform.py).
core_exact         evaluates the same sum directly.  sum_m g C is a rotation
    invariant 8-D integral; with G = (v+w)/2, u = rho u_hat it becomes
      b0 (2pi)^-3 int dG e^{-G^2} int rho^{2+gamma} e^{-rho^2/4} drho int du_hat T
    and invariance lets u_hat = z_hat (factor 4 pi) and G = (G_perp, 0, G_z)
    (factor 2 pi, G_perp dG_perp = dG_perp^2 / 2).  The integrand is a
    polynomial in (G_perp^2, G_z, rho^2) times the weights, so Gauss-Laguerre
    in G_perp^2, Gauss-Hermite in G_z and generalized Gauss-Laguerre in
    rho^2/4 are exact.  At each node the invariant Gaunt sum
      sum_z g_z Y_q1(a) Y_q2(b) Y_q3(c)
    is evaluated in the frame where v is along z_hat and w lies in the x-z
    plane (the privileged frame of Section 3.1).  The gain sphere average of
    the test function, int dn phi_{k l m}(G + r n), equals h_kl(|G|, r) Y_lm(G_hat)
    (it commutes with rotations), and h_kl is a 1-D Gauss-Legendre integral
    (gain="funk_hecke"); gain="sphere" integrates over n directly instead.
With an angular factor, B = b0 u^gamma beta(cos chi) and cos chi = u_hat . n
(Sections 2.1, 4.3), the gain average int dn beta(u_hat . n) phi(G + r n) is not
a function of G alone, so only gain="sphere" applies: it weights the sphere
rule by beta at every node, and the loss by int dn beta(u_hat . n).
No quantity here is truncated or regularized: the result is exact up to FP64
rounding for any gamma >= 0.
"""
import math

import numpy as np
from scipy.sparse import csr_matrix
from scipy.special import roots_genlaguerre, roots_hermite, roots_legendre

from .basis import basis_all, num_modes, q_index, radial, real_sh_all, real_sph_harm
from .gaunt import coo, l_of_q, sphere_rule
from .weakform import B0_DEFAULT, angular_factor


def core_from_tensor(C, K, L, table=None):
    """R[c, k1, k2, k3] from a full weak-form tensor C[a1, a2, a3]."""
    table = table or coo(L)
    NK = K + 1
    NT = len(table["channels"])
    num = np.zeros((NT, NK, NK, NK))
    S = np.zeros(NT)
    ks = np.arange(NK)
    for q1, q2, q3, c, g in zip(table["q1"], table["q2"], table["q3"], table["c"], table["g"]):
        i1 = q1 * NK + ks
        i2 = q2 * NK + ks
        i3 = q3 * NK + ks
        num[c] += g * C[np.ix_(i1, i2, i3)]
        S[c] += g * g
    return num / S[:, None, None, None]


def _outer_rules(K, L, gamma):
    D = 2 * K + L
    n_half = (3 * D) // 2 // 2 + 1
    gp, wgp = roots_genlaguerre(n_half, 0.0)     # G_perp^2, weight e^{-x}
    gz, wgz = roots_hermite(3 * D // 2 + 1)      # G_z, weight e^{-x^2}
    s, ws = roots_genlaguerre(n_half, 0.5 * (1.0 + gamma))
    A, Bz, S = np.meshgrid(gp, gz, s, indexing="ij")
    W = np.einsum("i,j,k->ijk", wgp, wgz, ws).ravel()
    W = W * 0.5 * 2.0 ** (2.0 + gamma) * 4 * math.pi * 2 * math.pi
    return A.ravel(), Bz.ravel(), S.ravel(), W


def _frames(gperp2, gz, s):
    """Privileged-frame vectors at each node: v along z, w in the x-z plane."""
    rho = 2.0 * np.sqrt(s)
    G = np.stack([np.sqrt(gperp2), np.zeros_like(gz), gz], axis=-1)
    V = G.copy(); V[:, 2] += 0.5 * rho
    Wv = G.copy(); Wv[:, 2] -= 0.5 * rho
    vn = np.linalg.norm(V, axis=1)
    wn = np.linalg.norm(Wv, axis=1)
    cb = np.clip(np.sum(V * Wv, axis=1) / (vn * wn), -1.0, 1.0)
    sb = np.sqrt(1.0 - cb * cb)
    w_f = np.stack([wn * sb, np.zeros_like(wn), wn * cb], axis=-1)
    v_f = np.stack([np.zeros_like(vn), np.zeros_like(vn), vn], axis=-1)
    G_f = 0.5 * (v_f + w_f)
    return vn, wn, w_f, G_f, 0.5 * rho


def _gain_h(K, L, Gn, r):
    """h[p, l, k] with int dn phi_{k l m}(G + r n) = h_kl(|G|, r) Y_lm(G_hat)."""
    nu, wnu = roots_legendre((K + L) // 2 + 1)
    P = len(Gn)
    h = np.zeros((P, L + 1, K + 1))
    for j in range(len(nu)):
        x = np.sqrt(1.0 - nu[j] ** 2)
        X = np.stack([r * x, np.zeros(P), Gn + r * nu[j]], axis=-1)
        xn = np.linalg.norm(X, axis=1)
        th = np.arccos(np.clip(X[:, 2] / np.where(xn > 0, xn, 1.0), -1, 1))
        for l in range(L + 1):
            y = real_sph_harm(l, 0, th, np.zeros(P)) / math.sqrt((2 * l + 1) / (4 * math.pi))
            for k in range(K + 1):
                h[:, l, k] += 2 * math.pi * wnu[j] * radial(k, l, xn) * y
    return h


def core_exact(K, L, gamma, b0=B0_DEFAULT, gain="auto", table=None,
               chunk=8192, subset=None, beta=None):
    """R[c, k1, k2, k3] (no zeroing) by the exact reduced quadrature.

    subset: optional list of channel indices; other channels are left zero.
    beta:   Legendre coefficients of the angular factor beta(cos chi), or None
            for the isotropic kernel.
    """
    if gain == "auto":
        gain = "funk_hecke" if beta is None else "sphere"
    if beta is not None and gain != "sphere":
        raise ValueError("an angular factor needs gain='sphere'")
    J = 0 if beta is None else len(beta) - 1
    table = table or coo(L)
    chans = table["channels"]
    NT, NK = len(chans), K + 1
    want = np.zeros(NT, bool)
    want[list(range(NT)) if subset is None else list(subset)] = True
    gp, gz, s, W = _outer_rules(K, L, gamma)
    W = W * b0 * (2 * math.pi) ** -3
    vn, wn, w_f, G_f, r = _frames(gp, gz, s)
    P = len(W)
    v_f = np.stack([np.zeros_like(vn), np.zeros_like(vn), vn], axis=-1)
    uhat = (v_f - w_f) / (2.0 * r)[:, None]                    # relative-velocity direction
    Rv = np.stack([np.stack([radial(k, l, vn) for k in range(NK)], -1)
                   for l in range(L + 1)], 1)                  # (P, L+1, NK)
    Rw = np.stack([np.stack([radial(k, l, wn) for k in range(NK)], -1)
                   for l in range(L + 1)], 1)
    Yz = real_sh_all(L, np.array([[0.0, 0.0, 1.0]]))[0]       # (NQ,)
    Yw = real_sh_all(L, w_f)                                   # (P, NQ)
    q1, q2, q3, cz, g = (table[k] for k in ("q1", "q2", "q3", "c", "g"))
    S = np.bincount(cz, weights=g * g, minlength=NT)
    lc = np.array([c[0] for c in chans])
    # invariant Gaunt sums in the privileged frame (v along z_hat):
    #   J[p, c]  = sum_{z in c} g_z Y_q1(G_hat) Y_q2(z_hat) Y_q3(w_hat)   (gain)
    #   JL[p, c] = sum_{z in c} g_z Y_q1(z_hat) Y_q2(z_hat) Y_q3(w_hat)   (loss)
    keep = (np.abs(Yz[q2]) > 1e-14) & want[cz]
    keepL = keep & (np.abs(Yz[q1]) > 1e-14)
    SL = csr_matrix((g[keepL] * Yz[q1[keepL]] * Yz[q2[keepL]],
                     (np.arange(keepL.sum()), cz[keepL])), shape=(keepL.sum(), NT))
    JL = np.asarray((SL.T @ Yw[:, q3[keepL]].T).T)
    lossw = np.full(P, 4 * math.pi)                             # int dn beta(u_hat . n)
    if gain == "funk_hecke":
        Gn = np.linalg.norm(G_f, axis=1)
        Hrad = _gain_h(K, L, Gn, r)                            # (P, L+1, NK)
        Yg = real_sh_all(L, G_f)
        Sg = csr_matrix((g[keep] * Yz[q2[keep]], (np.arange(keep.sum()), cz[keep])),
                        shape=(keep.sum(), NT))
        J = np.empty((P, NT))
        for p0 in range(0, P, chunk):
            sl = slice(p0, p0 + chunk)
            M = Yg[sl][:, q1[keep]] * Yw[sl][:, q3[keep]]
            J[sl] = np.asarray((Sg.T @ M.T).T)

        def gain_block(cs):
            return J[:, cs, None] * Hrad[:, lc[cs], :]
    elif gain == "sphere":
        Nn, WN = sphere_rule(2 * K + L + J)
        N = num_modes(K, L)
        Hm = np.empty((P, (L + 1) ** 2, NK))
        for p0 in range(0, P, 64):
            sl = slice(p0, p0 + 64)
            pts = G_f[sl][:, None, :] + r[sl][:, None, None] * Nn[None]
            Wn = angular_factor(beta, uhat[sl] @ Nn.T) * WN[None, :]   # beta(u_hat . n) dn
            lossw[sl] = Wn.sum(axis=1)
            Hm[sl] = np.einsum("pnj,pn->pj", basis_all(K, L, pts.reshape(-1, 3))
                               .reshape(len(pts), len(WN), N), Wn).reshape(-1, NQ_of(L), NK)
        fac = (g[keep] * Yz[q2[keep]]) * Yw[:, q3[keep]]               # (P, z)
        Xg_all = np.zeros((P, NT, NK))
        for zi, (c, qa) in enumerate(zip(cz[keep], q1[keep])):
            Xg_all[:, c, :] += fac[:, zi, None] * Hm[:, qa, :]

        def gain_block(cs):
            return Xg_all[:, cs, :]
    else:
        raise ValueError(gain)
    R = np.zeros((NT, NK, NK, NK))
    pairs = {}
    for ci, (l1, l2, l3) in enumerate(chans):
        if want[ci]:
            pairs.setdefault((l2, l3), []).append(ci)
    for (l2, l3), cs in pairs.items():
        cs = np.array(cs)
        X = gain_block(cs) - lossw[:, None, None] * JL[:, cs, None] * Rv[:, lc[cs], :]
        X *= W[:, None, None]
        E = (Rv[:, l2, :, None] * Rw[:, l3, None, :]).reshape(P, NK * NK)
        R[cs] = (X.reshape(P, len(cs) * NK).T @ E).reshape(len(cs), NK, NK, NK)
    S = np.where(S > 0, S, 1.0)
    return R / S[:, None, None, None]


def NQ_of(L):
    return (L + 1) ** 2


def zero_invariants(R, chans):
    """Null-space and detailed-balance zeroing (Section 4.4).

    l1 = 0: rows k1 = 0 (mass) and k1 = 1 (energy) of R^{(c)} are set to 0;
    l1 = 1: row k1 = 0 (momentum); channel (0,0,0): R_{k1,0,0} = 0 for all k1.
    """
    R = R.copy()
    for ci, (l1, l2, l3) in enumerate(chans):
        if l1 in (0, 1):
            R[ci, 0] = 0.0
        if l1 == 0 and R.shape[1] > 1:
            R[ci, 1] = 0.0
        if (l1, l2, l3) == (0, 0, 0):
            R[ci, :, 0, 0] = 0.0
    return R

"""Spectral basis of Section 2.2 (phi_alpha = R_kl(v) Y_lm(v_hat)).

Conventions (the paper fixes the ingredients but not every sign or scale):
  * alpha = (k, l, m); angular index q = l*l + l + m (0-based); flat index
    n = q * NK + k with NK = K + 1 (the paper's f_{k,q}).
  * R_kl(v) = N_kl v^l L_k^{(l+1/2)}(v^2/2): associated Laguerre radial part,
    orthonormal under the reference Maxwellian (2 pi)^{-3/2} exp(-v^2/2) of
    Section 2.3, so the Galerkin mass matrix is the identity and phi_000 = 1.
  * Real spherical harmonics built from the Condon-Shortley complex ones:
    Y_{l,0} = Y_l^0, Y_{l,m>0} = sqrt2 (-1)^m Re Y_l^m,
    Y_{l,m<0} = sqrt2 (-1)^m Im Y_l^{|m|}  (so Y_{1,1} ~ +x, Y_{1,-1} ~ +y).
Special functions come from scipy (library primitives); nothing here is shared
with the GPU library.
"""
import math

import numpy as np
from scipy.special import eval_genlaguerre, gammaln, sph_harm_y


def num_modes(K, L):
    """N = (K+1)(L+1)^2 (Section 4.6, box truncation)."""
    return (K + 1) * (L + 1) ** 2


def q_index(l, m):
    return l * l + l + m


def mode_index(K, k, l, m):
    return q_index(l, m) * (K + 1) + k


def mode_table(K, L):
    """Array (N, 3) of (k, l, m) in flat order n = q*NK + k."""
    out = []
    for l in range(L + 1):
        for m in range(-l, l + 1):
            for k in range(K + 1):
                out.append((k, l, m))
    return np.array(out, dtype=np.int64)


def radial_norm(k, l):
    """N_kl with N_kl^2 = (2 pi)^{3/2} k! / (2^{l+1/2} Gamma(k+l+3/2))."""
    logn2 = 1.5 * math.log(2 * math.pi) + math.lgamma(k + 1) \
        - (l + 0.5) * math.log(2.0) - float(gammaln(k + l + 1.5))
    return math.exp(0.5 * logn2)


def radial(k, l, v):
    """R_kl(v) = N_kl v^l L_k^{(l+1/2)}(v^2/2)."""
    v = np.asarray(v, dtype=np.float64)
    return radial_norm(k, l) * v ** l * eval_genlaguerre(k, l + 0.5, 0.5 * v * v)


def real_sph_harm(l, m, theta, phi):
    """Real spherical harmonic Y_lm at polar angle theta, azimuth phi."""
    am = abs(m)
    y = sph_harm_y(l, am, theta, phi)
    if m == 0:
        return np.real(y)
    s = math.sqrt(2.0) * (-1.0) ** am
    return s * (np.real(y) if m > 0 else np.imag(y))


def _angles(X):
    X = np.asarray(X, dtype=np.float64)
    r = np.sqrt(np.sum(X * X, axis=-1))
    rs = np.where(r > 0, r, 1.0)
    ct = np.clip(X[..., 2] / rs, -1.0, 1.0)
    theta = np.arccos(ct)
    phi = np.arctan2(X[..., 1], X[..., 0])
    return r, theta, phi


def real_sh_all(L, X):
    """Y_q(x_hat) for all q < (L+1)^2 at points X (..., 3) -> (..., NQ)."""
    _, theta, phi = _angles(X)
    cols = []
    for l in range(L + 1):
        for m in range(-l, l + 1):
            cols.append(real_sph_harm(l, m, theta, phi))
    return np.stack(cols, axis=-1)


def basis_all(K, L, X):
    """phi_alpha(x) for all alpha in flat order at points X (P, 3) -> (P, N)."""
    X = np.asarray(X, dtype=np.float64)
    r, _, _ = _angles(X)
    Y = real_sh_all(L, X)                      # (P, NQ)
    NK = K + 1
    out = np.empty(X.shape[:-1] + (num_modes(K, L),))
    for l in range(L + 1):
        for k in range(NK):
            rad = radial(k, l, r)
            for m in range(-l, l + 1):
                out[..., mode_index(K, k, l, m)] = rad * Y[..., q_index(l, m)]
    return out


def maxwellian_ref(v):
    """Reference Maxwellian (2 pi)^{-3/2} exp(-v^2/2) (Section 2.3)."""
    v = np.asarray(v, dtype=np.float64)
    return (2 * math.pi) ** -1.5 * np.exp(-0.5 * v * v)

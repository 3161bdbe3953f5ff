"""Angular geometry of Sections 4.1-4.2: channels, real Gaunt table, COO list.

The real Gaunt weight g(q1,q2,q3) = int_{S^2} Y_q1 Y_q2 Y_q3 dOmega is computed
here by an exact product rule on the sphere (Gauss-Legendre in cos(theta) times
the trapezoid rule in phi, exact for polynomials of degree 3L), not by the 3j
closed form used in the product library.
"""
import math

import numpy as np
from scipy.special import roots_legendre

from .basis import real_sh_all


def sphere_rule(degree):
    """Nodes (P,3) and weights (P,) exact for polynomials of the given degree."""
    nt = degree // 2 + 1
    nph = degree + 1
    x, w = roots_legendre(nt)
    ph = 2 * math.pi * np.arange(nph) / nph
    st = np.sqrt(1.0 - x * x)
    X = np.stack([np.outer(st, np.cos(ph)), np.outer(st, np.sin(ph)),
                  np.outer(x, np.ones(nph))], axis=-1).reshape(-1, 3)
    W = np.outer(w, np.full(nph, 2 * math.pi / nph)).ravel()
    return X, W


def channels(L):
    """Valid (l1,l2,l3) triplets, l1 outer, l2 middle, l3 inner (Section 4.6).

    Triangle rule |l1-l2| <= l3 <= l1+l2, even l1+l2+l3, all degrees <= L.
    Index c here is 0-based; the paper's channel number is c+1.
    """
    out = []
    for l1 in range(L + 1):
        for l2 in range(L + 1):
            for l3 in range(abs(l1 - l2), min(l1 + l2, L) + 1):
                if (l1 + l2 + l3) % 2 == 0:
                    out.append((l1, l2, l3))
    return out


def gaunt_dense(L):
    """Dense real Gaunt tensor g[q1,q2,q3], shape (NQ,NQ,NQ)."""
    X, W = sphere_rule(3 * L)
    Y = real_sh_all(L, X).T                  # (NQ, P)
    NQ = Y.shape[0]
    g = np.empty((NQ, NQ, NQ))
    for a in range(NQ):
        g[a] = (Y * (Y[a] * W)) @ Y.T
    return g


def l_of_q(q):
    return int(math.isqrt(int(q)))


def coo(L, tol=1e-12):
    """COO routing table in the paper's order (Table 1): q3 slowest, q1 fastest.

    Returns dict of int64 arrays q1,q2,q3,c (0-based) and float64 g, plus the
    channel list.  Entries with |g| <= tol are structural zeros.
    """
    g = gaunt_dense(L)
    chans = channels(L)
    cid = {t: i for i, t in enumerate(chans)}
    NQ = (L + 1) ** 2
    lq = np.array([l_of_q(q) for q in range(NQ)])
    rows = []
    for q3 in range(NQ):
        for q2 in range(NQ):
            for q1 in range(NQ):
                val = g[q1, q2, q3]
                if abs(val) > tol:
                    c = cid[(lq[q1], lq[q2], lq[q3])]
                    rows.append((q1, q2, q3, c, val))
    a = np.array(rows, dtype=object)
    return {
        "q1": a[:, 0].astype(np.int64), "q2": a[:, 1].astype(np.int64),
        "q3": a[:, 2].astype(np.int64), "c": a[:, 3].astype(np.int64),
        "g": a[:, 4].astype(np.float64), "channels": chans,
    }


def num_slices(table):
    """N_S: number of distinct (channel, q1) pairs (Section 4.7)."""
    return len(set(zip(table["c"].tolist(), table["q1"].tolist())))

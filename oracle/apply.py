"""The factorized discrete sum of Section 4.5 (eq. full_discrete_sum), literally.

    Q_{k1, q1z} += g_z sum_{k2, k3} R^{(c_z)}_{k1 k2 k3} f_{k2, q2z} f_{k3, q3z}

for every COO row z, scattered to the row's test state q1z.  Coefficients use
the flat layout n = q * NK + k.  This is the paper's "naive" ordering, chosen
here because it is the plainest reading of the sum; the product library uses a
different ordering and never calls this code.
"""
import numpy as np


def apply_q(R, table, f, K, zchunk=8192):
    """Q(f, f) for one cell (f shape (N,)) or a batch (shape (B, N))."""
    f = np.asarray(f, dtype=np.float64)
    if f.ndim == 2:
        return np.stack([apply_q(R, table, fb, K, zchunk) for fb in f])
    NK = K + 1
    F = f.reshape(-1, NK)                    # F[q, k]
    Q = np.zeros_like(F)
    q1, q2, q3, c, g = (table[k] for k in ("q1", "q2", "q3", "c", "g"))
    for z0 in range(0, len(g), zchunk):
        sl = slice(z0, z0 + zchunk)
        Rz = R[c[sl]].reshape(-1, NK * NK, NK)             # [z, (k1 k2), k3]
        t = (Rz @ F[q3[sl]][:, :, None]).reshape(-1, NK, NK)   # [z, k1, k2]
        t = (t @ F[q2[sl]][:, :, None])[:, :, 0]                # [z, k1]
        t *= g[sl][:, None]
        for k in range(NK):
            Q[:, k] += np.bincount(q1[sl], weights=t[:, k], minlength=F.shape[0])
    return Q.reshape(-1)


def apply_bilinear(R, table, f, g, K, zchunk=8192):
    """The bilinear form Q(f, g) = sum_z g_z sum_{k2,k3} R^{(c_z)}_{k1 k2 k3} f_{k2,q2z} g_{k3,q3z}
    scattered to q1z (the same sum with the second factor taken from g), one cell or a batch."""
    f = np.asarray(f, dtype=np.float64)
    gg = np.asarray(g, dtype=np.float64)
    if f.ndim == 2:
        return np.stack([apply_bilinear(R, table, fb, gb, K, zchunk) for fb, gb in zip(f, gg)])
    NK = K + 1
    F = f.reshape(-1, NK)
    G = gg.reshape(-1, NK)
    Q = np.zeros_like(F)
    q1, q2, q3, c, w = (table[k] for k in ("q1", "q2", "q3", "c", "g"))
    for z0 in range(0, len(w), zchunk):
        sl = slice(z0, z0 + zchunk)
        Rz = R[c[sl]].reshape(-1, NK * NK, NK)
        t = (Rz @ G[q3[sl]][:, :, None]).reshape(-1, NK, NK)
        t = (t @ F[q2[sl]][:, :, None])[:, :, 0]
        t *= w[sl][:, None]
        for k in range(NK):
            Q[:, k] += np.bincount(q1[sl], weights=t[:, k], minlength=F.shape[0])
    return Q.reshape(-1)


def apply_jvp(R, table, c, d, K):
    """J(c) d = Q(c, d) + Q(d, c): the derivative of Q(f, f) at c in the direction d."""
    return apply_bilinear(R, table, c, d, K) + apply_bilinear(R, table, d, c, K)

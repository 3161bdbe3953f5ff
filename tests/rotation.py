"""Real Wigner rotation matrices of the coefficient space (test helper).

For a rotation matrix Rm, f_rot(v) = f(Rm^T v) has coefficients c_rot = D c with
D block diagonal in l (identity in k): D^l_{m m'} = int Y_lm(n) Y_lm'(Rm^T n) dn,
computed with an exact product rule on the sphere (scipy harmonics).
"""
import numpy as np
from scipy.spatial.transform import Rotation

from oracle.basis import real_sh_all
from oracle.gaunt import sphere_rule


def random_rotation(seed):
    return Rotation.random(random_state=seed).as_matrix()


def wigner_blocks(L, Rm):
    X, W = sphere_rule(2 * L)
    Y = real_sh_all(L, X)                  # (P, NQ)
    Yr = real_sh_all(L, X @ Rm)            # Y(Rm^T n): rows of X are n^T, n^T Rm = (Rm^T n)^T
    full = (Y * W[:, None]).T @ Yr         # (NQ, NQ), block diagonal in l
    return [full[l * l:(l + 1) ** 2, l * l:(l + 1) ** 2] for l in range(L + 1)]


def rotate(c, K, L, blocks):
    """Apply D to coefficient rows c (B, N) in the layout n = q*(K+1) + k."""
    NK = K + 1
    c = np.asarray(c)
    out = np.empty_like(c)
    C = c.reshape(c.shape[0], -1, NK)       # [b, q, k]
    O = out.reshape(c.shape[0], -1, NK)
    for l, D in enumerate(blocks):
        sl = slice(l * l, (l + 1) ** 2)
        O[:, sl, :] = np.einsum("mp,bpk->bmk", D, C[:, sl, :])
    return out

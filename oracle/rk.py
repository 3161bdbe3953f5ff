"""Explicit Runge-Kutta integration of the Galerkin system dc/dt = Q(c), in FP64.

Test infrastructure only (see the package header).  With the identity mass
matrix of Section 2.3 the weak form is an ODE system per cell; the relaxation
experiments of Section 5 integrate it with an explicit Runge-Kutta scheme whose
order the paper does not state.  Four textbook schemes are written out from
their Butcher tableaux, each stage evaluating Q with the oracle's literal sum:

  euler  forward Euler                          b = (1)
  heun   Heun's second-order method             a21 = 1;            b = (1/2, 1/2)
  ssp3   third-order strong-stability-preserving (Shu and Osher)
                                                a21 = 1; a31 = a32 = 1/4;  b = (1/6, 1/6, 2/3)
  rk4    the classic fourth-order method        a21 = a32 = 1/2; a43 = 1;  b = (1/6, 1/3, 1/3, 1/6)

Pinned in tests by the order of convergence of each scheme on the BKW solution
and by the BKW closed form itself.
"""
import numpy as np

from . import apply

TABLEAUX = {
    "euler": ([], [1.0]),
    "heun": ([[1.0]], [0.5, 0.5]),
    "ssp3": ([[1.0], [0.25, 0.25]], [1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0]),
    "rk4": ([[0.5], [0.0, 0.5], [0.0, 0.0, 1.0]], [1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0]),
}


def integrate(R, table, c, K, dt, nsteps, scheme="rk4"):
    """c after nsteps steps of size dt; c has shape (N,) or (B, N)."""
    a, b = TABLEAUX[scheme]
    c = np.array(c, dtype=np.float64)
    for _ in range(nsteps):
        ks = []
        for s in range(len(b)):
            y = c.copy()
            for j in range(s):
                y = y + dt * a[s - 1][j] * ks[j]
            ks.append(apply.apply_q(R, table, y, K))
        for j in range(len(b)):
            c = c + dt * b[j] * ks[j]
    return c

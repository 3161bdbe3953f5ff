"""Memoized oracle products shared by tests (all computed by oracle/ only)."""
import functools
import math

from oracle import core, gaunt


@functools.lru_cache(maxsize=None)
def coo(L):
    return gaunt.coo(L)


@functools.lru_cache(maxsize=None)
def core_zeroed(K, L, gamma, b0=1.0 / (4 * math.pi), beta=None):
    """beta: a tuple of Legendre coefficients of the angular factor, or None."""
    T = coo(L)
    return core.zero_invariants(core_raw(K, L, gamma, b0, beta), T["channels"])


@functools.lru_cache(maxsize=None)
def core_raw(K, L, gamma, b0=1.0 / (4 * math.pi), beta=None):
    return core.core_exact(K, L, gamma, b0=b0, table=coo(L), beta=None if beta is None else list(beta))


def golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    rows = []
    for line in open(path):
        line = line.split("#")[0].strip()
        if line:
            rows.append(line.split())
    return rows

"""Helpers shared by the GPU tests."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_err(a, ref):
    """max |a - ref| / max |ref| over the whole array."""
    return float(np.abs(np.asarray(a) - np.asarray(ref)).max() / max(np.abs(ref).max(), 1e-300))


def invariant_indices(K, L):
    idx = [0]
    if K >= 1:
        idx.append(1)
    if L >= 1:
        idx += [1 * (K + 1), 2 * (K + 1), 3 * (K + 1)]
    return np.array(idx)

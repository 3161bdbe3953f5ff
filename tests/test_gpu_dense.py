"""The dense Cartesian contraction (Section 4.5.1) on the GPU: the assembled tensor C against the
oracle's C = g R, Q(f, f) against the oracle, and against the angular-first apply at the largest
size of the paper's ordering comparison (K = 4, L = 13)."""
import ctypes

import numpy as np
import pytest

from gpu_common import dev, invariant_indices, rel_err, say, torch
from oracle import apply as oapply
from oracle_cache import coo, core_zeroed

import paper_2605_28475_amd as wefq
from paper_2605_28475_amd import _lib, synth

pytestmark = pytest.mark.gpu


def _unlayout(raw, N):
    """C[a1, a2, a3] from the matrix-core operand layout of wefq_dense_assemble: element
    (a1, kappa = a2 N4 + a3) at ((a1/16) KC + kappa/4) 64 + a1 % 16 + 16 (kappa % 4)."""
    NA, N4 = (N + 15) // 16 * 16, (N + 3) // 4 * 4
    KC = N * N4 // 4
    x = raw.view(np.float64).reshape(NA // 16, KC, 4, 16)          # [a1 tile][kappa/4][kappa%4][a1%16]
    x = x.transpose(0, 3, 1, 2).reshape(NA, N, N4)                  # [a1][a2][a3]
    assert np.all(x[N:] == 0.0) and np.all(x[:, :, N:] == 0.0)      # padding stays zero
    return x[:N, :, :N]


def test_assembled_tensor_is_g_times_R():
    K, L, gamma = 2, 3, 1.0
    core = wefq.Core("hs", K, L, device=0, precisions=("fp64",))
    C = core.dense_assemble()
    torch.cuda.synchronize()
    got = _unlayout(C.cpu().numpy(), core.N)
    R, T, NK = core_zeroed(K, L, gamma), coo(L), K + 1
    ks = np.arange(NK)
    ref = np.zeros((core.N,) * 3)
    for q1, q2, q3, c, g in zip(T["q1"], T["q2"], T["q3"], T["c"], T["g"]):
        ref[np.ix_(q1 * NK + ks, q2 * NK + ks, q3 * NK + ks)] += g * R[c]
    assert np.abs(got - ref).max() < 1e-14 * np.abs(ref).max()
    core.close()


@pytest.mark.parametrize("K,L,model,gamma,B", [(4, 2, "hs", 1.0, 19), (4, 3, "vhs", 0.5, 33), (4, 4, "mm", 0.0, 5),
                                               (2, 5, "hs", 1.0, 17), (0, 3, "hs", 1.0, 3), (3, 0, "vhs", 0.5, 1)])
def test_dense_matches_oracle(K, L, model, gamma, B):
    say(f"[dense] K={K} L={L} {model} B={B}")
    core = wefq.Core(model, K, L, gamma=gamma, device=0, precisions=("fp64",))
    C = core.dense_assemble()
    c = synth.perturbed_maxwellian(K, L, B, seed=synth.BASE_SEED + 300 + 7 * K + L)
    q = core.apply_Q_dense(C, torch.tensor(c, device=dev())).cpu().numpy()
    ref = oapply.apply_q(core_zeroed(K, L, gamma), coo(L), c, K)
    assert rel_err(q, ref) < 1e-12
    assert np.all(q[:, invariant_indices(K, L)] == 0.0)
    core.close()


def test_dense_matches_angular_first_at_K4_L13():
    """The largest size of the paper's Fig. 6 comparison: 7.6 GB of C."""
    K, L, B = 4, 13, 40
    core = wefq.Core("hs", K, L, device=0, precisions=("fp64",))
    say(f"[dense] K={K} L={L}: C {core.dense_bytes() / 2**30:.2f} GiB")
    C = core.dense_assemble()
    f = torch.tensor(synth.perturbed_maxwellian(K, L, B, seed=77), device=dev())
    qd = core.apply_Q_dense(C, f).cpu().numpy()
    qa = core.apply_Q(f, precision="fp64").cpu().numpy()
    assert rel_err(qd, qa) < 1e-12
    del C
    core.close()


def test_dense_argument_errors():
    L_ = _lib.lib()
    core32 = wefq.Core("hs", 2, 2, device=0, precisions=("fp32",))
    n = ctypes.c_int64()
    assert L_.wefq_dense_bytes(core32.handle, ctypes.byref(n)) == _lib.WEFQ_EINVAL      # no FP64 tables
    core32.close()
    big = wefq.Core("hs", 12, 12, device=0, precisions=("fp64",))
    assert L_.wefq_dense_bytes(big.handle, ctypes.byref(n)) == _lib.WEFQ_EUNSUPPORTED   # N = 2197
    big.close()
    core = wefq.Core("hs", 2, 2, device=0, precisions=("fp64",))
    nb = core.dense_bytes()
    C = torch.zeros(nb + 512, dtype=torch.uint8, device=dev())
    f = torch.zeros((3, core.N), dtype=torch.float64, device=dev())
    q = torch.full_like(f, 9.0)
    cp, fp, qp = ctypes.c_void_p(C.data_ptr()), ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(q.data_ptr())
    assert L_.wefq_dense_assemble(core.handle, cp, nb - 8, None) == _lib.WEFQ_EINVAL    # too small
    assert L_.wefq_dense_assemble(core.handle, ctypes.c_void_p(C.data_ptr() + 8), nb, None) == _lib.WEFQ_EINVAL
    assert L_.wefq_apply_Q_dense(core.handle, cp, nb, fp, qp, -1, core.N, core.N, None) == _lib.WEFQ_EINVAL
    assert L_.wefq_apply_Q_dense(core.handle, cp, nb, fp, qp, 3, core.N - 1, core.N, None) == _lib.WEFQ_EINVAL
    assert L_.wefq_apply_Q_dense(core.handle, cp, nb, fp, fp, 3, core.N, core.N, None) == _lib.WEFQ_EINVAL
    assert L_.wefq_apply_Q_dense(core.handle, cp, nb, fp, cp, 3, core.N, core.N, None) == _lib.WEFQ_EINVAL
    assert L_.wefq_apply_Q_dense(core.handle, cp, nb, fp, qp, 0, core.N, core.N, None) == _lib.WEFQ_OK
    torch.cuda.synchronize()
    assert torch.all(q == 9.0)
    core.close()

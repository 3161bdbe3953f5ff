"""wefq_rk_integrate_noalloc (fixed device scratch, allocates nothing) against
wefq_rk_integrate (caller workspace), through the C ABI: bitwise equal results on two
calls in a row, the second with a smaller batch; refusal of a batch beyond the scratch."""
import ctypes

import numpy as np
import pytest

from gpu_common import dev, say, torch

import paper_2605_28475_amd as wefq
from paper_2605_28475_amd import _lib, synth

pytestmark = pytest.mark.gpu


def _noalloc(core, prec, scheme, c, dt, nsteps, stream):
    res = ctypes.c_double(-1.0)
    st = _lib.lib().wefq_rk_integrate_noalloc(core.handle, prec, scheme, ctypes.c_void_p(c.data_ptr()), c.shape[0],
                                              c.stride(0), dt, nsteps, ctypes.byref(res),
                                              ctypes.c_void_p(stream.cuda_stream))
    return st, res.value


def _with_workspace(core, prec, scheme, c, dt, nsteps, stream):
    need = ctypes.c_int64()
    _lib.check(_lib.lib().wefq_rk_workspace(core.handle, prec, scheme, c.shape[0], ctypes.byref(need)))
    work = torch.empty(need.value, dtype=torch.uint8, device=c.device)
    res = ctypes.c_double(-1.0)
    _lib.check(_lib.lib().wefq_rk_integrate(core.handle, prec, scheme, ctypes.c_void_p(c.data_ptr()), c.shape[0],
                                            c.stride(0), dt, nsteps, ctypes.c_void_p(work.data_ptr()), need.value,
                                            ctypes.byref(res), ctypes.c_void_p(stream.cuda_stream)))
    torch.cuda.synchronize()
    return res.value


@pytest.mark.parametrize("prec,K", [("fp32", 8), ("fp64", 5), ("bf16x3", 12)])
def test_noalloc_matches_workspace_entry_point(prec, K):
    d = dev()
    stream = torch.cuda.current_stream(d)
    core = wefq.Core("hs", K, K, device=0, precisions=(prec,))
    p = wefq.PRECISIONS[prec]
    dt_ = torch.float64 if prec == "fp64" else torch.float32
    for B, scheme, nsteps in ((300, _lib.RK_CLASSIC4, 3), (37, _lib.RK_SSP3, 2)):     # second call smaller
        say(f"[noalloc] {prec} K={K} B={B} scheme={scheme}")
        c0 = torch.tensor(synth.perturbed_maxwellian(K, K, B, seed=900 + B), dtype=dt_, device=d)
        ref = c0.clone()
        inv_ref = _with_workspace(core, p, scheme, ref, 0.05, nsteps, stream)
        got = c0.clone()
        st, inv = _noalloc(core, p, scheme, got, 0.05, nsteps, stream)
        torch.cuda.synchronize()
        assert st == _lib.WEFQ_OK, _lib.lib().wefq_last_error()
        assert torch.equal(got, ref)
        assert inv == inv_ref == 0.0
        assert not torch.equal(got, c0)
    core.close()


def test_noalloc_refuses_batches_beyond_the_scratch():
    d = dev()
    stream = torch.cuda.current_stream(d)
    core = wefq.Core("hs", 12, 12, device=0, precisions=("fp32",))
    per_cell = 5 * core.N * 4                                  # RK4: 4 stages + the stage input
    B = (_lib.RK_NOALLOC_BYTES - 256) // per_cell + 1          # one cell too many
    c = torch.zeros((B, core.N), dtype=torch.float32, device=d)
    c[:, 0] = 1.0
    st, _ = _noalloc(core, _lib.FP32, _lib.RK_CLASSIC4, c, 0.05, 1, stream)
    assert st == _lib.WEFQ_EBUDGET
    assert b"scratch" in _lib.lib().wefq_last_error()
    torch.cuda.synchronize()
    assert torch.all(c[:, 1:] == 0.0) and torch.all(c[:, 0] == 1.0)  # nothing ran
    st, _ = _noalloc(core, _lib.FP32, _lib.RK_CLASSIC4, c[:B - 1], 0.05, 1, stream)   # the largest that fits
    torch.cuda.synchronize()
    assert st == _lib.WEFQ_OK
    core.close()

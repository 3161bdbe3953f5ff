"""The rate probe behind the measured peaks of the benchmark: every kind returns a plausible
rate through the C ABI, and bad arguments are rejected with EINVAL."""
import ctypes

import pytest

from gpu_common import say

import paper_2605_28475_amd as wefq
from paper_2605_28475_amd import _lib

pytestmark = pytest.mark.gpu

# datasheet dense rates of the MI355X, TFLOP/s (the vector FP32 figure counts packed
# instructions, which this library does not use; the probe issues unpacked ones)
DATASHEET = {"mfma_f32": 157.3, "mfma_f64": 78.6, "mfma_bf16": 2500.0, "valu_f32": 157.3, "valu_f64": 78.6}


@pytest.mark.parametrize("kind", sorted(DATASHEET))
def test_probe_rate_is_plausible(kind):
    rate = wefq.peak_probe(kind, device=0)
    say(f"[probe] {kind}: {rate:.1f} TFLOP/s")
    # a probe that loses most of the pipe, or counts FLOPs twice, falls outside this band
    assert 0.4 * DATASHEET[kind] < rate < 1.15 * DATASHEET[kind]


def test_probe_rejects_bad_arguments():
    L_ = _lib.lib()
    out = ctypes.c_double(-1.0)
    assert L_.wefq_peak_probe(0, 5, ctypes.byref(out), None) == _lib.WEFQ_EINVAL
    assert out.value == 0.0
    assert L_.wefq_peak_probe(0, -1, ctypes.byref(out), None) == _lib.WEFQ_EINVAL
    assert L_.wefq_peak_probe(0, _lib.PROBE_MFMA_F32, None, None) == _lib.WEFQ_EINVAL
    assert L_.wefq_peak_probe(4096, _lib.PROBE_MFMA_F32, ctypes.byref(out), None) == _lib.WEFQ_EINVAL
    assert b"device" in L_.wefq_last_error()

"""Failure paths forced from the host: an injected device-allocation failure at several
points of a core build (test hook WEFQ_TEST_FAIL_DEVICE_ALLOC) returns WEFQ_ENOMEM with a
message, releases what was allocated, and leaves the library usable."""
import numpy as np
import pytest

from gpu_common import dev, invariant_indices, say, torch

import paper_2605_28475_amd as wefq
from paper_2605_28475_amd import _lib, synth

pytestmark = pytest.mark.gpu

ALL = ("fp64", "fp32", "bf16x3", "bilinear", "radial")


def test_injected_allocation_failures_release_everything(monkeypatch):
    d = dev()
    K = L = 6
    wefq.Core("hs", K, L, device=0, precisions=ALL).close()          # module load, warm caches
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(0)[0]
    for n in (1, 2, 5, 12):
        monkeypatch.setenv("WEFQ_TEST_FAIL_DEVICE_ALLOC", str(n))
        say(f"[fail] allocation {n}")
        with pytest.raises(wefq.WefqError) as err:
            wefq.Core("hs", K, L, device=0, precisions=ALL)
        assert err.value.status == _lib.WEFQ_ENOMEM
        assert "allocation" in str(err.value)
    monkeypatch.delenv("WEFQ_TEST_FAIL_DEVICE_ALLOC")
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info(0)[0]
    assert free0 - free1 < (64 << 20)                                  # nothing held on
    core = wefq.Core("hs", K, L, device=0, precisions=ALL)
    f = torch.tensor(synth.perturbed_maxwellian(K, L, 5, seed=3), dtype=torch.float32, device=d)
    q = core.apply_Q(f).cpu().numpy()
    assert np.isfinite(q).all() and np.all(q[:, invariant_indices(K, L)] == 0.0)
    core.close()

"""Core serialization (wefq_core_save / wefq_core_load) on the GPU."""
import numpy as np
import pytest

from gpu_common import dev, say, torch

import paper_2605_28475_amd as wefq
from paper_2605_28475_amd import _lib, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("model,K,L,gamma", [("vhs", 6, 6, 0.5), ("hs", 12, 4, 1.0)])
def test_saved_core_reloads_bitwise(tmp_path, model, K, L, gamma):
    dev()
    say(f"[serialize] {model} K={K} L={L}")
    a = wefq.Core(model, K, L, gamma=gamma, device=0, precisions=("fp64", "fp32", "bilinear"))
    path = tmp_path / "core.wefq"
    a.save(path)
    b = wefq.Core.load(path, precisions=("fp64", "fp32", "bilinear"), device=0)
    assert (b.K, b.L, b.model, b.gamma) == (a.K, a.L, a.model, a.gamma)
    assert b.info["b0"] == a.info["b0"] and b.info["quad_nodes"] == a.info["quad_nodes"]
    assert np.array_equal(a.download_R(), b.download_R())
    c = synth.perturbed_maxwellian(K, L, 5, seed=3)
    for prec, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
        f = torch.tensor(c, dtype=dt, device=dev())
        g = torch.flip(f, dims=[0]).contiguous()
        assert torch.equal(a.apply_Q(f, precision=prec), b.apply_Q(f, precision=prec))
        assert torch.equal(a.apply_Qfg(f, g, precision=prec), b.apply_Qfg(f, g, precision=prec))
    # a flipped payload byte fails the checksum; a truncated file fails the size check
    raw = bytearray(path.read_bytes())
    raw[-9] ^= 0x40
    bad = tmp_path / "bad.wefq"
    bad.write_bytes(bytes(raw))
    with pytest.raises(wefq.WefqError) as err:
        wefq.Core.load(bad, device=0)
    assert err.value.status == _lib.WEFQ_EINVAL
    bad.write_bytes(path.read_bytes()[:-8])
    with pytest.raises(wefq.WefqError):
        wefq.Core.load(bad, device=0)
    a.close()
    b.close()

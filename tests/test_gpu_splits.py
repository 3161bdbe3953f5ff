"""Launch-shape choices never change results: batches whose launches split their cell tiles
over several workgroups (a second workgroup per compute unit at K = L = 8, partial last
rounds at K = L = 12 and 16) give bitwise the rows of the same cells in a batch of whole
rounds, which runs unsplit."""
import pytest

from gpu_common import dev, say, torch

import paper_2605_28475_amd as wefq
from paper_2605_28475_amd import synth

pytestmark = pytest.mark.gpu

# (K, precisions, small batch sizes, whole-round batch size): 16-cell tiles at K = 8 and 12,
# 8-cell FP32 tiles and 4-cell FP64 tiles at K = 16, on 256 compute units
CASES = [
    (8, ("fp32", "bf16x3"), (4096,), 8192),
    (12, ("fp32", "fp64"), (4500, 6000), 8192),
    (16, ("fp32",), (2516, 3072), 8192),
    (16, ("fp64",), (2516,), 4096),
]


@pytest.mark.parametrize("K,precs,small,whole", CASES)
def test_split_launches_match_whole_rounds(K, precs, small, whole):
    d = dev()
    core = wefq.Core("hs", K, K, device=0, precisions=("fp32", "fp64", "bf16x3"))
    c = torch.tensor(synth.perturbed_maxwellian(K, K, whole, seed=synth.BASE_SEED + 61), device=d)
    for prec in precs:
        f = c if prec == "fp64" else c.float()
        big = core.apply_Q(f, precision=prec)
        for B in small:
            say(f"[split] K={K} {prec} {B} of {whole} cells")
            part = core.apply_Q(f[:B].contiguous(), precision=prec)
            torch.cuda.synchronize()
            assert torch.equal(part, big[:B]), (K, prec, B)
    core.close()

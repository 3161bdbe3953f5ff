"""The apply entry points allocate nothing and record no memset, so a caller can capture them
into a HIP graph (torch.cuda.graph): replays, with eager work between them, give bitwise the
eager results."""
import numpy as np
import pytest

from gpu_common import dev, say, torch

import paper_2605_28475_amd as wefq
from paper_2605_28475_amd import synth

pytestmark = pytest.mark.gpu


def test_captured_apply_and_jvp_replay_bitwise():
    d = dev()
    K = L = 8
    core = wefq.Core("hs", K, L, device=0, precisions=("fp32", "bf16x3"))
    f = torch.tensor(synth.perturbed_maxwellian(K, L, 300, seed=21), dtype=torch.float32, device=d)
    g = torch.tensor(synth.perturbed_maxwellian(K, L, 300, seed=22), dtype=torch.float32, device=d)
    q, q16, j = torch.empty_like(f), torch.empty_like(f), torch.empty_like(f)
    ref_q = core.apply_Q(f).clone()
    ref_16 = core.apply_Q(f, precision="bf16x3").clone()
    ref_j = core.apply_J(f, g).clone()
    # warm the kernels (attributes, code objects) on a side stream before capture
    s = torch.cuda.Stream(device=d)
    s.wait_stream(torch.cuda.current_stream(d))
    with torch.cuda.stream(s):
        core.apply_Q(f, out=q)
        core.apply_Q(f, out=q16, precision="bf16x3")
        core.apply_J(f, g, out=j)
    torch.cuda.current_stream(d).wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        core.apply_Q(f, out=q)
        core.apply_Q(f, out=q16, precision="bf16x3")
        core.apply_J(f, g, out=j)
    for replay in range(3):
        for t in (q, q16, j):
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        say(f"[graph] replay {replay}")
        assert torch.equal(q, ref_q) and torch.equal(q16, ref_16) and torch.equal(j, ref_j), replay
        torch.ones(4096, device=d).cumsum(0)[-1].item()          # unrelated eager work
    del graph
    core.close()

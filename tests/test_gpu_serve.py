"""Continuous-batching server: results alone vs in the mix; admission under a small budget."""
import pytest

from gpu_common import dev, say, torch

from paper_2605_28475_amd import serve

pytestmark = pytest.mark.gpu


def test_server_results_equal_standalone_applies():
    say("[serve] mix")
    srv = serve.make_server(torch, sizes=(4, 8, 12), pool_cells=512, budget_gb=0.25, streams=3)
    trace = serve.poisson_trace(3000.0, 0.05, (4, 8, 12), 512, seed=7, pool_cells=512)
    assert len(trace) > 20
    res = srv.run(trace, keep_outputs=True)
    assert res["requests"] == len(trace) and res["p99_ms"] >= res["p50_ms"] > 0
    for rid, (t, k, n, off) in enumerate(trace):
        alone = srv.cores[k].apply_Q(srv.pools[k][off:off + n])
        assert torch.equal(res["outputs"][rid], alone), rid
    assert srv.arena.used == 0


def test_admission_waits_for_memory():
    """A budget that holds only a few requests at once still serves every request."""
    srv = serve.make_server(torch, sizes=(8,), pool_cells=256, budget_gb=0.02, streams=2)
    trace = serve.poisson_trace(5000.0, 0.02, (8,), 256, seed=11, pool_cells=256)
    res = srv.run(trace, keep_outputs=True)
    assert res["requests"] == len(trace)
    assert res["arena_peak_bytes"] <= 0.02 * 2 ** 30
    for rid, (t, k, n, off) in enumerate(trace):
        assert torch.equal(res["outputs"][rid], srv.cores[0].apply_Q(srv.pools[0][off:off + n]))

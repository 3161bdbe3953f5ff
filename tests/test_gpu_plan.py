"""Uneven batches in one persistent, graph-captured launch; autotuner."""
import numpy as np
import pytest

from gpu_common import dev, say, torch

import paper_2605_28475_amd as wefq
from paper_2605_28475_amd import _lib, autotune, synth

pytestmark = pytest.mark.gpu

_cores = {}


def core(model, K, gamma=None):
    key = (model, K, gamma)
    if key not in _cores:
        say(f"[build] {key}")
        _cores[key] = wefq.Core(model, K, K, gamma=gamma, device=0)
    return _cores[key]


def segments(prec, specs):
    d = dev()
    dt = torch.float64 if prec == "fp64" else torch.float32
    out = []
    for i, (model, K, gamma, B) in enumerate(specs):
        c = core(model, K, gamma)
        f = torch.tensor(synth.perturbed_maxwellian(K, K, B, seed=1000 + i), dtype=dt, device=d)
        out.append((c, f, torch.empty_like(f)))
    return out


MIX = [("hs", 4, None, 37), ("vhs", 8, 0.5, 1), ("hs", 12, None, 130), ("vhs", 16, 0.5, 9),
       ("mm", 3, None, 64), ("hs", 16, None, 17), ("vhs", 12, 0.5, 33), ("hs", 8, None, 5)]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp64"])
def test_plan_matches_single_segment_applies(prec):
    say(f"[plan] {prec}")
    segs = segments(prec, MIX if prec == "fp32" else MIX[:4])
    refs = [c.apply_Q(f, precision=prec).clone() for c, f, _ in segs]
    plan = wefq.Plan(segs, precision=prec)
    assert plan.info["work_items"] > 0
    for replay in range(3):
        for _, _, q in segs:
            q.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for (c, f, q), r in zip(segs, refs):
            assert torch.equal(q, r), f"replay {replay} K={c.K}"
        # unrelated eager work between replays
        torch.ones(1000, device=dev()).sum().item()
    for _, _, q in segs:
        q.zero_()
    plan.launch(graph=False)
    torch.cuda.synchronize()
    for (c, f, q), r in zip(segs, refs):
        assert torch.equal(q, r)
    plan.close()


@pytest.mark.parametrize("prec,slots", [("fp32", 2), ("fp32", 4), ("fp64", 2), ("fp64", 4)])
def test_plan_tiles_without_pad_rows_match_padded_standalone_tiles(prec, slots):
    """8- and 4-cell tiles of even NK and even H (K = 3, 7, 15): the standalone kernels stage
    them with a pad row per q block, the persistent kernel without.  Only LDS addresses
    differ, so the results are bitwise equal."""
    specs = [("hs", 3, None, 29), ("vhs", 7, 0.5, 21)]
    if not (prec == "fp64" and slots == 2):          # (that K = 15 tile does not fit in LDS)
        specs.append(("hs", 15, None, 6))
    say(f"[plan pad] {prec} slots={slots}")
    segs = segments(prec, specs)
    refs = []
    for c, f, _ in segs:
        old = c.tune_get(prec)
        c.tune_set(prec, slots, old[1])
        try:
            refs.append(c.apply_Q(f, precision=prec).clone())
        finally:
            c.tune_set(prec, *old)
    plan = wefq.Plan([(c, f, q, slots) for c, f, q in segs], precision=prec)
    plan.launch()
    torch.cuda.synchronize()
    for (c, _, q), r in zip(segs, refs):
        assert torch.equal(q, r), f"K={c.K}"
    plan.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp64"])
def test_plan_tile_shape_override_keeps_results(prec):
    """Non-default tile shapes (4-cell tiles): in BF16x3 and FP64 they take the build of the
    persistent kernel that holds every shape, not the default-shape one."""
    segs = segments(prec, [("hs", 4, None, 40), ("vhs", 8, 0.5, 23)])
    refs = [c.apply_Q(f, precision=prec).clone() for c, f, _ in segs]
    plan = wefq.Plan([(c, f, q, 4) for c, f, q in segs], precision=prec, block=256)
    plan.launch()
    torch.cuda.synchronize()
    for (_, _, q), r in zip(segs, refs):
        assert torch.equal(q, r)
    plan.close()


def test_autotuner_picks_valid_shape_and_keeps_results():
    c = core("vhs", 8, 0.5)
    f = torch.tensor(synth.perturbed_maxwellian(8, 8, 300, seed=4), dtype=torch.float32, device=dev())
    before = c.apply_Q(f).clone()
    s, b, timings = autotune.tune(c, "fp32", cells=256, reps=2, use_cache=False)
    assert (s, b) == c.tune_get("fp32") and len(timings) >= 2
    assert torch.equal(c.apply_Q(f), before)
    c.tune_set("fp32", 1, 512)


def test_plan_rejects_bad_segments():
    c = core("hs", 4)
    f = torch.zeros((4, c.N), dtype=torch.float32, device=dev())
    with pytest.raises(wefq.WefqError):
        wefq.Plan([(c, f, torch.empty_like(f))], precision="fp32", block=300)
    with pytest.raises(wefq.WefqError):
        wefq.Plan([(c, f, torch.empty_like(f), 3)], precision="fp32")


def test_plan_with_anisotropic_cores():
    """Segments whose cores carry an angular factor run in the same persistent launch and
    give bitwise the standalone results."""
    d = dev()
    aniso = wefq.Core("hs", 8, 8, device=0, beta=(1.0, 0.5, 0.3, 0.1))
    iso = core("vhs", 12, 0.5)
    segs = []
    for i, (c, K, B) in enumerate(((aniso, 8, 70), (iso, 12, 40), (aniso, 8, 3))):
        f = torch.tensor(synth.perturbed_maxwellian(K, K, B, seed=2000 + i), dtype=torch.float32, device=d)
        segs.append((c, f, torch.empty_like(f)))
    refs = [c.apply_Q(f).clone() for c, f, _ in segs]
    plan = wefq.Plan(segs, precision="fp32")
    for replay in range(2):
        for _, _, q in segs:
            q.fill_(float("nan"))
        plan.launch()
        torch.cuda.synchronize()
        for (c, f, q), r in zip(segs, refs):
            assert torch.equal(q, r), f"replay {replay}"
    plan.close()
    aniso.close()


def test_twelve_wave_plan_matches_single_segment_applies():
    """Plans of 768 threads run the 12-wave persistent kernel: the default FP32 shapes of
    K = 3, 4, 8, 12 and 16 are among its tile shapes; results stay bitwise those of the
    standalone applies, over graph replays and a direct launch."""
    segs = segments("fp32", MIX)
    refs = [c.apply_Q(f).clone() for c, f, _ in segs]
    plan = wefq.Plan(segs, precision="fp32", block=768)
    assert plan.info["block"] == 768 and plan.info["work_items"] > 0
    for replay in range(3):
        for _, _, q in segs:
            q.fill_(float("nan"))
        plan.launch()
        torch.cuda.synchronize()
        for (c, f, q), r in zip(segs, refs):
            assert torch.equal(q, r), f"replay {replay} K={c.K}"
        torch.ones(1000, device=dev()).sum().item()
    for _, _, q in segs:
        q.zero_()
    plan.launch(graph=False)
    torch.cuda.synchronize()
    for (c, f, q), r in zip(segs, refs):
        assert torch.equal(q, r)
    plan.close()


def test_second_twelve_wave_build_matches_single_segment_applies():
    """The other 12-wave build: 6x6 quadrants (K = 10, 11) and 7x7 and 8x8 with two output
    states (K = 13, 14, 15), bitwise equal to the standalone applies."""
    segs = segments("fp32", [("hs", 10, None, 37), ("vhs", 11, 0.5, 16), ("hs", 13, None, 9),
                             ("vhs", 14, 0.5, 12), ("hs", 15, None, 5)])
    refs = [c.apply_Q(f).clone() for c, f, _ in segs]
    plan = wefq.Plan(segs, precision="fp32", block=768)
    for replay in range(2):
        for _, _, q in segs:
            q.fill_(float("nan"))
        plan.launch()
        torch.cuda.synchronize()
        for (c, f, q), r in zip(segs, refs):
            assert torch.equal(q, r), f"replay {replay} K={c.K}"
    plan.close()


def test_twelve_wave_plan_refuses_other_shapes_and_precisions():
    """768 threads take FP32 plans whose tile shapes all belong to one 12-wave build (EINVAL
    before any allocation or launch otherwise)."""
    other = segments("fp32", [("hs", 10, None, 20), ("hs", 12, None, 20)])     # one shape of each build
    with pytest.raises(wefq.WefqError) as err:
        wefq.Plan(other, precision="fp32", block=768)
    assert err.value.status == _lib.WEFQ_EINVAL
    c, f, q = segments("fp32", [("hs", 4, None, 20)])[0]
    with pytest.raises(wefq.WefqError):
        wefq.Plan([(c, f, q, 4)], precision="fp32", block=768)         # 4-cell tiles of 3x3
    with pytest.raises(wefq.WefqError):
        wefq.Plan(segments("fp64", [("hs", 4, None, 20)]), precision="fp64", block=768)
    with pytest.raises(wefq.WefqError):
        wefq.Runner(0, "fp64", block=768)


def test_twelve_wave_runner_falls_back_for_other_shapes():
    """A runner of 768 threads launches a 12-wave build for batches whose tile shapes it covers
    and the 8-wave kernel of 512 threads for the others; all bitwise equal to standalone
    applies."""
    segs = segments("fp32", MIX[:4] + [("hs", 10, None, 21)])
    refs = [c.apply_Q(f).clone() for c, f, _ in segs]
    run = wefq.Runner(0, "fp32", max_segments=64, max_items=1 << 16, block=768)
    stream = torch.cuda.current_stream(dev())
    for pick in (range(4), range(5), [4], range(4)):
        for i in pick:
            segs[i][2].fill_(float("nan"))
        run.launch([segs[i] for i in pick], stream=stream)
        torch.cuda.synchronize()
        for i in pick:
            assert torch.equal(segs[i][2], refs[i]), (list(pick), i)
    run.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_runner_launches_match_single_segment_applies(prec):
    """wefq_runner_launch: one persistent launch per call over a changing mix of segments,
    six calls in a row (every ring slot reused), bitwise equal to standalone applies."""
    say(f"[runner] {prec}")
    segs = segments(prec, MIX if prec == "fp32" else MIX[:4])
    refs = [c.apply_Q(f, precision=prec).clone() for c, f, _ in segs]
    run = wefq.Runner(0, prec, max_segments=64, max_items=1 << 16)
    stream = torch.cuda.current_stream(dev())
    for call in range(6):
        # a different subset and different cell ranges each call
        pick = [i for i in range(len(segs)) if (i + call) % 3 != 0]
        for i in pick:
            segs[i][2].fill_(float("nan"))
        parts = []
        for i in pick:
            c, f, q = segs[i]
            cut = (call * 5) % max(1, f.shape[0])
            parts += [(c, f[:cut], q[:cut]), (c, f[cut:], q[cut:])] if 0 < cut < f.shape[0] else [(c, f, q)]
        run.launch(parts, stream=stream)
        torch.cuda.synchronize()
        for i in pick:
            assert torch.equal(segs[i][2], refs[i]), (call, i)
    run.launch([], stream=stream)                         # nothing to do
    small = wefq.Runner(0, prec, max_segments=4, max_items=2)
    c, f, q = segs[2]
    with pytest.raises(wefq.WefqError) as err:
        small.launch([(c, f, q)], stream=stream)          # more work items than the runner holds
    assert err.value.status == _lib.WEFQ_EBUDGET
    with pytest.raises(ValueError):
        small.launch([(c, f, q)] * 5, stream=stream)      # more segments than it holds
    small.close()
    run.close()


def test_plan_autotuner_times_whole_plans_and_keeps_results():
    """autotune.tune_plan picks shapes by timing whole plans; the chosen plan's results equal
    standalone applies bitwise, and the default shapes are among the candidates."""
    segs = segments("fp32", [("hs", 4, None, 64), ("vhs", 8, 0.5, 40), ("hs", 12, None, 33)])
    refs = [c.apply_Q(f).clone() for c, f, _ in segs]
    slots, block, tried = autotune.tune_plan(segs, "fp32", reps=2)
    assert block in (256, 512, 768) and len(slots) == len(segs)
    assert "block=512 slots=0,0,0" in tried and np.isfinite(min(tried.values()))
    plan = wefq.Plan([(c, f, q, s) for (c, f, q), s in zip(segs, slots)], precision="fp32", block=block)
    plan.launch()
    torch.cuda.synchronize()
    for (c, f, q), r in zip(segs, refs):
        assert torch.equal(q, r)

"""Continuous-batching server for Q(f,f) requests on one GPU.

Requests (core = model, K, L; n cells) arrive over time.  The cores of every size are
resident, and so are the cells' coefficient states (a pool per core).  The scheduler runs a
loop whose tick is one persistent launch over every core at once (wefq_runner_launch):

  1. completed launches are retired, their requests' completion events recorded and their
     HBM blocks freed;
  2. arrived requests are admitted in arrival order while their output block (n N floats)
     fits a first-fit arena carved from a fixed HBM budget (head-of-line order is kept);
     requests of fewer than two cell tiles take no block of their own;
  3. while fewer than `max_inflight` launches are on the device, the next tick is built:
     every admitted request with cells left gets an equal share of the tick's work (its
     next cells, in whole cell tiles, read in place from its pool into its output block),
     what is left of the tick goes to the oldest requests, and the small requests of each
     core are packed into one staging block (device-to-device copies) so that they share
     cell tiles; the whole tick is one launch of the persistent kernel, cores mixed;
  4. launches go to one HIP stream (default priority), so consecutive ticks run back to
     back while the host builds the next one.

A request of thousands of K = L = 16 cells is thus served over several ticks, interleaved
with the small requests that arrive meanwhile, instead of holding the device for its whole
duration.  Completion times come from HIP events (device clock, relative to a reference
event recorded at the start), so latencies are arrival -> device completion.  Per-cell
results are bitwise independent of the batch, chunk or tick a cell lands in.
"""
import bisect
import math
import sys
import time

import numpy as np

from . import synth


class Arena:
    """First-fit allocator over a device float32 buffer (offsets in floats)."""

    def __init__(self, torch, nfloats, device):
        self.buf = torch.empty(int(nfloats), dtype=torch.float32, device=device)
        self.free = [(0, int(nfloats))]            # sorted (offset, size)
        self.size = int(nfloats)
        self.used = 0
        self.peak = 0

    def alloc(self, n):
        n = int((n + 63) // 64 * 64)               # 256-byte alignment
        for i, (off, sz) in enumerate(self.free):
            if sz >= n:
                if sz == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + n, sz - n)
                self.used += n
                self.peak = max(self.peak, self.used)
                return off, n
        return None

    def release(self, off, n):
        self.used -= n
        i = bisect.bisect_left(self.free, (off, 0))
        self.free.insert(i, (off, n))
        # coalesce neighbours
        j = max(i - 1, 0)
        while j < len(self.free) - 1:
            a, b = self.free[j], self.free[j + 1]
            if a[0] + a[1] == b[0]:
                self.free[j] = (a[0], a[1] + b[1])
                self.free.pop(j + 1)
            else:
                j += 1


def poisson_trace(rate, duration, sizes, max_cells, seed, pool_cells):
    """Arrival times (s), core size index, cell count and pool offset per request."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        n = int(min(max(math.floor(math.exp(rng.uniform(0.0, math.log(max_cells)))), 1), max_cells))
        k = int(rng.integers(len(sizes)))
        off = int(rng.integers(0, pool_cells - n + 1))
        out.append((t, k, n, off))
    return out


class Server:
    """Continuous batching over resident cores and cell pools (see the module notes).

    tick_ms and rate_tflops size a tick: about tick_ms of work at rate_tflops of algorithmic
    FLOPs.  streams is accepted for compatibility: ticks run on one stream."""

    def __init__(self, torch, cores, pools, budget_bytes, streams=1, max_inflight=2, device=0, tick_ms=32.0,
                 rate_tflops=140.0, precision="fp32", pack_tiles=2, block=None):
        import paper_2605_28475_amd as wefq
        self.torch = torch
        self.cores = cores                 # list of Core
        self.pools = pools                 # list of device tensors [pool_cells, N]
        self.dev = torch.device("cuda", device)
        self.arena = Arena(torch, budget_bytes // 4, self.dev)
        self.stream = torch.cuda.Stream(device=self.dev)
        self.depth = max(1, int(max_inflight))
        # threads per workgroup of the persistent kernel: 768 in FP32 (the 12-wave kernel, for
        # ticks whose cores all have its tile shapes; the runner takes the 8-wave kernel of 512
        # threads for the others), else 512.  Measured on this module's bench workload (K = 8, 12
        # and 16): saturation 146.8 against 135.7 TFLOP/s, p99 at 1,250 req/s 122 against 188 ms.
        self.block = int(block) if block else (768 if precision == "fp32" else 512)
        self.runner = wefq.Runner(device, precision, block=self.block)
        self.tile = [16 // c.tune_get(precision)[0] for c in cores]
        self.fpc = [float(c.info["flop_alg_per_cell"]) for c in cores]
        self.tick_flop = tick_ms * 1e-3 * rate_tflops * 1e12
        self.pack = int(pack_tiles)

    def _tick(self, active, state):
        """Segments of the next launch: (segments, finished [(rid, q view)], blocks to free)."""
        torch = self.torch
        plan, used = {}, 0.0
        share = self.tick_flop / max(1, len(active))
        for r in active:
            k, n, off, done, blk, _ = state[r]
            rem, tb, fpc = n - done, self.tile[k], self.fpc[k]
            m = rem if blk is None else min(rem, max(tb, int(share / fpc / tb) * tb))
            plan[r] = m
            used += m * fpc
        left = self.tick_flop - used
        for r in active:                   # what is left of the tick: oldest first
            if left <= 0:
                break
            k, n, off, done, blk, _ = state[r]
            rem = n - done - plan[r]
            if blk is None or rem <= 0:
                continue
            tb, fpc = self.tile[k], self.fpc[k]
            extra = min(rem, int(left / fpc / tb) * tb)
            if extra > 0:
                plan[r] += extra
                left -= extra * fpc
        segs, fin, blks, small = [], [], [], {}
        for r in active:
            k, n, off, done, blk, q = state[r]
            m = plan[r]
            if blk is None:
                small.setdefault(k, []).append(r)
                continue
            pool = self.pools[k]
            segs.append((self.cores[k], pool[off + done:off + done + m], q[done:done + m]))
            state[r][3] = done + m
            if done + m == n:
                fin.append((r, q))
                blks.append(blk)
        for k, rids in small.items():      # small requests of one core share cell tiles
            core, pool, N = self.cores[k], self.pools[k], self.cores[k].N
            cells = sum(state[r][1] for r in rids)
            blk = self.arena.alloc(2 * cells * N)
            if blk is None:
                continue                   # they wait for memory
            o = blk[0]
            sf = self.arena.buf[o:o + cells * N].view(cells, N)
            sq = self.arena.buf[o + cells * N:o + 2 * cells * N].view(cells, N)
            row = 0
            with torch.cuda.stream(self.stream):
                for r in rids:
                    _, n, off, _, _, _ = state[r]
                    sf[row:row + n].copy_(pool[off:off + n], non_blocking=True)
                    fin.append((r, sq[row:row + n]))
                    state[r][3] = n
                    row += n
            segs.append((core, sf, sq))
            blks.append(blk)
        return segs, fin, blks

    def run(self, trace, keep_outputs=False):
        torch = self.torch
        ref = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize(self.dev)
        ref.record(self.stream)
        t0 = time.perf_counter()
        pending = list(range(len(trace)))[::-1]   # not yet admitted; the next one is last
        state = {}                                # rid -> [core, n, pool offset, cells scheduled, block, q]
        active = []                               # admitted, cells left to schedule, arrival order
        inflight = []                             # (event, finished requests, blocks), oldest first
        done_ev, outputs = {}, {}
        max_queue = launches = 0
        while pending or active or inflight:
            # 1. retire completed launches, oldest first
            while inflight and inflight[0][0].query():
                ev, fin, blks = inflight.pop(0)
                with torch.cuda.stream(self.stream):
                    for r, q in fin:
                        done_ev[r] = ev
                        if keep_outputs:
                            outputs[r] = q.clone()      # ordered before any reuse of the block
                for b in blks:
                    self.arena.release(*b)
            now = time.perf_counter() - t0
            # 2. admit arrived requests in arrival order while their output block fits
            while pending and trace[pending[-1]][0] <= now:
                r = pending[-1]
                _, k, n, off = trace[r]
                N = self.cores[k].N
                if n < self.pack * self.tile[k]:
                    state[r] = [k, n, off, 0, None, None]
                else:
                    blk = self.arena.alloc(n * N)
                    if blk is None:
                        break
                    state[r] = [k, n, off, 0, blk, self.arena.buf[blk[0]:blk[0] + n * N].view(n, N)]
                active.append(r)
                pending.pop()
            max_queue = max(max_queue, len(active) + sum(len(x[1]) for x in inflight))
            # 3. the next tick: one persistent launch over every core
            if active and len(inflight) < self.depth:
                segs, fin, blks = self._tick(active, state)
                if segs:
                    with torch.cuda.stream(self.stream):
                        self.runner.launch(segs, stream=self.stream)
                        ev = torch.cuda.Event(enable_timing=True)
                        ev.record(self.stream)
                    inflight.append((ev, fin, blks))
                    launches += 1
                    active = [r for r in active if state[r][3] < state[r][1]]
                    continue
            # 4. nothing to launch now: wait for a completion or the next arrival
            if not inflight and pending and not active:
                wait = trace[pending[-1]][0] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.001))
            elif not inflight and active:
                raise RuntimeError("requests need more memory than the HBM budget")
            else:
                time.sleep(2e-5)
        torch.cuda.synchronize(self.dev)
        wall = time.perf_counter() - t0
        t_done = {r: ref.elapsed_time(ev) * 1e-3 for r, ev in done_ev.items()}
        lat = np.array([t_done[r] - trace[r][0] for r in range(len(trace))])
        end = max(t_done.values()) if t_done else 0.0
        cells = sum(t[2] for t in trace)
        # algorithmic FLOPs served (Section 4.7 count of each request's core) over the makespan
        flop = sum(t[2] * self.fpc[t[1]] for t in trace)
        res = {"requests": len(trace), "cells": int(cells), "launches": launches,
               "flop_alg": float(flop), "achieved_tflops": float(flop / end / 1e12) if end > 0 else 0.0,
               "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
               "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3),
               "makespan_s": float(end), "throughput_cells_per_s": float(cells / end) if end > 0 else 0.0,
               "max_queue": int(max_queue), "arena_peak_bytes": int(self.arena.peak * 4), "host_wall_s": wall}
        if keep_outputs:
            torch.cuda.synchronize(self.dev)
            res["outputs"] = outputs
        return res


def make_server(torch, sizes=(8, 12, 16), model="hs", pool_cells=4096, budget_gb=8.0, streams=1, device=0,
                precision="fp32", **server_args):
    """Resident hard-sphere cores K = L in sizes and seeded resident cell pools; server_args go
    to Server (tick_ms, max_inflight, rate_tflops, pack_tiles, block)."""
    import paper_2605_28475_amd as wefq
    dev = torch.device("cuda", device)
    cores, pools = [], []
    for K in sizes:
        c = wefq.Core(model, K, K, device=device, precisions=(precision,))
        cores.append(c)
        pools.append(torch.tensor(synth.perturbed_maxwellian(K, K, pool_cells, seed=synth.BASE_SEED + 50 + K),
                                  dtype=torch.float32, device=dev))
    return Server(torch, cores, pools, int(budget_gb * 2 ** 30), streams=streams, device=device, precision=precision,
                  **server_args)


def bench(args):
    """Serving under Poisson arrivals: 1-4096 cells per request (log-uniform), K = L in {8, 12, 16},
    hard spheres, FP32."""
    import torch
    cfg = synth.WORKLOADS["serving"]
    tick_ms = float(getattr(args, "tick_ms", 32.0))
    depth = int(getattr(args, "serve_depth", 2))
    extra = {}
    if getattr(args, "serve_tflops", None):
        extra["rate_tflops"] = float(args.serve_tflops)
    if getattr(args, "serve_block", None):
        extra["block"] = int(args.serve_block)
    srv = make_server(torch, sizes=cfg["sizes"], pool_cells=cfg["max_cells"], tick_ms=tick_ms, max_inflight=depth,
                      **extra)
    # warm up every core once
    for c, p in zip(srv.cores, srv.pools):
        c.apply_Q(p[:64])
    torch.cuda.synchronize()
    runs = {}
    rates = getattr(args, "serve_rates", None) or (250.0, 500.0, 750.0, 1000.0, 1250.0, 1500.0, 1750.0, cfg["rate"])
    for rate in rates:
        dur = 1.0 if rate < cfg["rate"] else 2.0
        tr = poisson_trace(rate, dur, cfg["sizes"], cfg["max_cells"], cfg["seed"] + int(rate), cfg["max_cells"])
        runs[rate] = srv.run(tr)
        runs[rate]["trace_s"] = dur
        print(f"[serve] rate {rate:.0f}/s: p50 {runs[rate]['p50_ms']:.1f} ms, p99 {runs[rate]['p99_ms']:.1f} ms, "
              f"makespan {runs[rate]['makespan_s']:.2f} s, {runs[rate]['achieved_tflops']:.1f} TFLOP/s, "
              f"{runs[rate]['launches']} launches", file=sys.stderr, flush=True)
    main = runs[max(runs)]
    # sustainable: the queue does not build up over the trace (the run ends within 0.25 s
    # of the trace, so the device keeps pace with arrivals) and p99 stays below 250 ms
    sustainable = max([r for r, v in runs.items()
                       if v["makespan_s"] <= v["trace_s"] + 0.25 and v["p99_ms"] < 250.0] + [0.0])
    out = {"metric": "serving p50/p99 latency (ms) and throughput, Poisson arrivals", "value": main["p99_ms"],
           "unit": "ms (p99)", "n_gpus": 1, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": cfg["name"], "rate_req_per_s": max(runs), "sizes": list(cfg["sizes"]),
                      "cells_per_request": "log-uniform 1..4096", "model": "hard spheres",
                      "tick_ms": tick_ms, "launches_in_flight": depth, "block": srv.block,
                      "tick_rate_tflops": srv.tick_flop / (tick_ms * 1e-3) / 1e12},
           "p50_ms": main["p50_ms"], "p99_ms": main["p99_ms"], "throughput_cells_per_s": main["throughput_cells_per_s"],
           # algorithmic FLOPs of the served requests over the makespan, against the dense FP32
           # MFMA peak of 157.3 TFLOP/s; arrivals, not the device, bound it below saturation
           "roofline": {"bound": "mfma", "achieved": main["achieved_tflops"], "peak": 157.3, "unit": "TFLOP/s",
                        "frac": main["achieved_tflops"] / 157.3, "traffic": None},
           "runs": {str(int(r)): {k: v for k, v in res.items()} for r, res in runs.items()},
           "sustainable_rate_req_per_s": sustainable,
           "sustainable_rule": "highest tested rate whose run ends within 0.25 s of its trace, with p99 < 250 ms"}
    return out

"""Continuous-batching server for Q(f,f) requests on one GPU.

Requests (model, K, L, n cells) arrive over time.  The cores of every size are
resident, and so are the cells' coefficient states (a pool per core).  The
scheduler runs in a loop:

  1. completed launches are retired and their HBM blocks freed;
  2. every request that has arrived is admitted in arrival order as long as its
     staging + output block (2 n N floats) fits in a first-fit arena carved from
     a fixed HBM budget (head-of-line order is kept);
  3. requests admitted in the same tick that share a core are fused into one
     contiguous batch: their cells are copied next to each other in the block
     (device-to-device) and one wefq_apply_Q launch serves them all; a lone
     request is applied straight on its resident cells; when the whole group
     does not fit, its longest prefix that does is admitted;
  4. launches rotate over several HIP streams, so work of different requests
     overlaps on the device while new requests keep being admitted.

Completion times come from HIP events (device clock, relative to a reference
event recorded at the start), so latencies are arrival -> device completion
and do not depend on how often the host polls.  Per-cell results are bitwise
independent of the batch a cell lands in.
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
    def __init__(self, torch, cores, pools, budget_bytes, streams=4, max_inflight=64, device=0):
        self.torch = torch
        self.cores = cores                 # list of Core
        self.pools = pools                 # list of device tensors [pool_cells, N]
        self.dev = torch.device("cuda", device)
        self.arena = Arena(torch, budget_bytes // 4, self.dev)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(streams)]
        self.max_inflight = max_inflight

    def run(self, trace, keep_outputs=False, scan=256):
        torch = self.torch
        ref = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize(self.dev)
        ref.record(torch.cuda.current_stream(self.dev))
        t0 = time.perf_counter()
        pending = list(range(len(trace)))  # not yet admitted, arrival order
        inflight = []                      # (done_event, [(rid, q view)], arena block)
        done_ev, outputs = {}, {}
        max_queue = si = launches = 0
        while pending or inflight:
            now = time.perf_counter() - t0
            # 1. retire finished launches and free their blocks
            still = []
            for ev, qs, blk in inflight:
                if ev.query():
                    for r, q in qs:
                        done_ev[r] = ev
                        if keep_outputs:
                            outputs[r] = q.clone()
                    if keep_outputs:
                        # the clones run on this stream; the block may be reused by a launch
                        # on another stream as soon as it is released, so they finish first
                        torch.cuda.current_stream(self.dev).synchronize()
                    self.arena.release(*blk)
                else:
                    still.append((ev, qs, blk))
            inflight = still
            # 2. arrived requests (queue head), grouped per core in arrival order
            groups = {}
            for r in pending[:scan]:
                if trace[r][0] > now:
                    break
                groups.setdefault(trace[r][1], []).append(r)
            max_queue = max(max_queue, sum(len(g) for g in groups.values()))
            admitted = set()
            for k, rids in groups.items():
                if len(inflight) >= self.max_inflight:
                    break
                core, pool = self.cores[k], self.pools[k]
                N = core.N
                take, blk = len(rids), None
                while take > 0:                    # whole group, else the longest prefix that fits
                    cells = sum(trace[r][2] for r in rids[:take])
                    blk = self.arena.alloc((cells if take == 1 else 2 * cells) * N)
                    if blk is not None:
                        break
                    take -= 1
                if blk is None:
                    continue
                group = rids[:take]
                off0 = blk[0]
                s = self.streams[si % len(self.streams)]
                si += 1
                with torch.cuda.stream(s):
                    if take == 1:                  # apply straight on the resident cells
                        _, _, n, off = trace[group[0]]
                        qout = self.arena.buf[off0:off0 + n * N].view(n, N)
                        core.apply_Q(pool[off:off + n], out=qout, stream=s)
                        qs = [(group[0], qout)]
                    else:                          # fuse: gather the cells next to each other
                        stage = self.arena.buf[off0:off0 + cells * N].view(cells, N)
                        qout = self.arena.buf[off0 + cells * N:off0 + 2 * cells * N].view(cells, N)
                        row, qs = 0, []
                        for r in group:
                            _, _, n, off = trace[r]
                            stage[row:row + n].copy_(pool[off:off + n], non_blocking=True)
                            qs.append((r, qout[row:row + n]))
                            row += n
                        core.apply_Q(stage, out=qout, stream=s)
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(s)
                inflight.append((ev, qs, blk))
                admitted.update(group)
                launches += 1
            if admitted:
                pending = [r for r in pending if r not in admitted]
            elif not inflight and pending:
                head = pending[0]
                if trace[head][0] <= now:
                    raise RuntimeError("request %d needs more memory than the HBM budget" % head)
                wait = trace[head][0] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.001))
        torch.cuda.synchronize(self.dev)
        wall = time.perf_counter() - t0
        t_done = {r: ref.elapsed_time(ev) * 1e-3 for r, ev in done_ev.items()}
        lat = np.array([t_done[r] - trace[r][0] for r in range(len(trace))])
        end = max(t_done.values()) if t_done else 0.0
        cells = sum(t[2] for t in trace)
        # algorithmic FLOPs served (Section 4.7 count of each request's core) over the makespan
        flop = sum(t[2] * self.cores[t[1]].info["flop_alg_per_cell"] for t in trace)
        res = {"requests": len(trace), "cells": int(cells), "launches": launches,
               "flop_alg": float(flop), "achieved_tflops": float(flop / end / 1e12) if end > 0 else 0.0,
               "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
               "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3),
               "makespan_s": float(end), "throughput_cells_per_s": float(cells / end) if end > 0 else 0.0,
               "max_queue": int(max_queue), "arena_peak_bytes": int(self.arena.peak * 4), "host_wall_s": wall}
        if keep_outputs:
            res["outputs"] = outputs
        return res


def make_server(torch, sizes=(8, 12, 16), model="hs", pool_cells=4096, budget_gb=8.0, streams=4, device=0,
                precision="fp32"):
    """Resident hard-sphere cores K = L in sizes and seeded resident cell pools."""
    import paper_2605_28475_amd as wefq
    dev = torch.device("cuda", device)
    cores, pools = [], []
    for K in sizes:
        c = wefq.Core(model, K, K, device=device, precisions=(precision,))
        cores.append(c)
        pools.append(torch.tensor(synth.perturbed_maxwellian(K, K, pool_cells, seed=synth.BASE_SEED + 50 + K),
                                  dtype=torch.float32, device=dev))
    return Server(torch, cores, pools, int(budget_gb * 2 ** 30), streams=streams, device=device)


def bench(args):
    """Serving under Poisson arrivals: 1-4096 cells per request (log-uniform), K = L in {8, 12, 16},
    hard spheres, FP32."""
    import torch
    cfg = synth.WORKLOADS["serving"]
    # the library's default tile shapes (largest LDS tiles): under load, requests of one
    # core are fused into batches of thousands of cells, where those are the fastest
    srv = make_server(torch, sizes=cfg["sizes"], pool_cells=cfg["max_cells"])
    # warm up every core once
    for c, p in zip(srv.cores, srv.pools):
        c.apply_Q(p[:64])
    torch.cuda.synchronize()
    runs = {}
    for rate in (250.0, 500.0, 750.0, 1000.0, 1250.0, 1500.0, cfg["rate"]):
        dur = 1.0 if rate < cfg["rate"] else 2.0
        tr = poisson_trace(rate, dur, cfg["sizes"], cfg["max_cells"], cfg["seed"] + int(rate), cfg["max_cells"])
        runs[rate] = srv.run(tr)
        runs[rate]["trace_s"] = dur
        print(f"[serve] rate {rate:.0f}/s: p50 {runs[rate]['p50_ms']:.1f} ms, p99 {runs[rate]['p99_ms']:.1f} ms, "
              f"makespan {runs[rate]['makespan_s']:.2f} s", file=sys.stderr, flush=True)
    main = runs[cfg["rate"]]
    # sustainable: the queue does not build up over the trace (the run ends within 0.25 s
    # of the trace, so the device keeps pace with arrivals) and p99 stays below 250 ms
    sustainable = max([r for r, v in runs.items()
                       if v["makespan_s"] <= v["trace_s"] + 0.25 and v["p99_ms"] < 250.0] + [0.0])
    out = {"metric": "serving p50/p99 latency (ms) and throughput, Poisson arrivals", "value": main["p99_ms"],
           "unit": "ms (p99)", "n_gpus": 1, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": cfg["name"], "rate_req_per_s": cfg["rate"], "sizes": list(cfg["sizes"]),
                      "cells_per_request": "log-uniform 1..4096", "model": "hard spheres"},
           "p50_ms": main["p50_ms"], "p99_ms": main["p99_ms"], "throughput_cells_per_s": main["throughput_cells_per_s"],
           # algorithmic FLOPs of the served requests over the makespan, against the dense FP32
           # MFMA peak of 157.3 TFLOP/s; arrivals, not the device, bound it below saturation
           "roofline": {"bound": "mfma", "achieved": main["achieved_tflops"], "peak": 157.3, "unit": "TFLOP/s",
                        "frac": main["achieved_tflops"] / 157.3, "traffic": None},
           "runs": {str(int(r)): {k: v for k, v in res.items()} for r, res in runs.items()},
           "sustainable_rate_req_per_s": sustainable,
           "sustainable_rule": "highest tested rate whose run ends within 0.25 s of its trace, with p99 < 250 ms"}
    return out

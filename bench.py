"""Benchmark: Q(f,f) cell evaluations per second at Kmax = Lmax = 12 on one MI355X.

Workload: variable-hard-sphere core (gamma = 0.5), Kmax = Lmax = 12 (N = 2197 modes),
B = 65536 cells of seeded perturbed Maxwellians, coefficients resident in HBM.
One step = one pass of the hot path over the batch: wefq_apply_Q (FP32 angular
coupling + FP32 MFMA radial contraction, invariant rows written as exact zeros)
followed by the FP64 conservation check of the invariant rows.  Beside it the
plain FP64 GPU apply (the comparator) and the split BF16x3 apply are timed, and
the FP64 CPU oracle is timed on a bounded sample of the same cells.

Prints one JSON line.  Only one GPU is supported (--gpus 1).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32": 157.3, "fp64": 78.6, "bf16x3": 2500.0}   # TFLOP/s, MI355X dense


KERNEL_SOURCES = ["paper_2605_28475_amd/csrc/apply_tile.h", "paper_2605_28475_amd/csrc/apply.hip",
                  "paper_2605_28475_amd/csrc/capi.cpp", "paper_2605_28475_amd/csrc/wefq_core.h"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, precision="fp32", K=12, L=12, cells=65536):
    """HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE passes recorded under profiles/
    by `--workload traffic` (each scaled by a plain copy of known size), or None when the
    kernel sources changed since the counters were taken."""
    try:
        with open(traffic_file(precision, K, L, cells)) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("workload") != workload or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def profile_workload(args):
    model = args.model
    g = {"hs": 1.0, "mm": 0.0}.get(model, args.gamma)
    name = f"{model}{g:g}_K{args.K}L{args.L}_B{args.cells}" if model == "vhs" else f"{model}_K{args.K}L{args.L}_B{args.cells}"
    return name, g


def traffic_file(precision, K, L, cells):
    return os.path.join(ROOT, "profiles", f"traffic_apply_{precision}_K{K}L{L}_B{cells}.json")


def profile_run(args, torch, wefq, synth):
    """A few launches of one apply and one plain copy of f: the program that the rocprofv3
    counter passes run (the copy moves a known byte count, which scales the counters)."""
    name, gamma = profile_workload(args)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    core = wefq.Core(args.model, args.K, args.L, gamma=gamma, device=0, precisions=(args.precision,))
    dt = torch.float64 if args.precision == "fp64" else torch.float32
    f = torch.tensor(synth.perturbed_maxwellian(args.K, args.L, args.cells, seed=synth.BASE_SEED + 3), dtype=dt,
                     device=dev)
    q = torch.empty_like(f)
    dst = torch.empty_like(f)
    # calibration: a copy of f reads and writes f.numel() * elem bytes; 2 GiB written first push
    # f out of the caches (f was just uploaded, and a cache-resident f would read short)
    flush = torch.empty(1 << 29, dtype=torch.float32, device=dev)
    flush.fill_(1.0)
    del flush
    dst.copy_(f)
    ms, _ = time_steps(lambda: core.apply_Q(f, out=q, precision=args.precision), args.launches, stream, torch)
    print(json.dumps({"workload": name, "precision": args.precision, "launches": args.launches,
                      "kernel_ms": float(np.mean(ms)), "copy_bytes": f.numel() * f.element_size(),
                      "algorithmic_bytes_per_launch": 2 * f.numel() * f.element_size(),
                      "source_hash": kernel_source_hash()}), flush=True)
    core.close()


def _counter_rows(folder, counter):
    """(kernel name, dispatch id, value) per dispatch from a rocprofv3 counter-collection CSV
    (values summed over the rows of one dispatch and counter)."""
    import csv
    import glob
    paths = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if not paths:
        raise SystemExit(f"no counter_collection.csv under {folder}")
    agg = {}
    for path in paths:
        with open(path) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                key = (row["Kernel_Name"], row.get("Dispatch_Id") or row.get("Correlation_Id"))
                agg[key] = agg.get(key, 0.0) + float(row["Counter_Value"])
    return [(k[0], k[1], v) for k, v in agg.items()]


def traffic_from_counters(args):
    """HBM bytes per launch of the apply kernel from the FETCH_SIZE and WRITE_SIZE passes of a
    profile run, each scaled by what the same counter reads for the plain copy of f (its bytes
    are known), written to profiles/traffic_apply_<precision>_K<K>L<L>_B<cells>.json."""
    name, _ = profile_workload(args)
    elem = 8 if args.precision == "fp64" else 4
    N = (args.K + 1) * (args.L + 1) ** 2
    copy_bytes = args.cells * N * elem
    out = {"kernel": f"apply_mfma_kernel ({args.precision})", "workload": name, "precision": args.precision,
           "source_hash": kernel_source_hash(), "algorithmic_bytes_per_launch": 2 * copy_bytes}
    for counter, folder, key in (("FETCH_SIZE", args.fetch_dir, "fetch"), ("WRITE_SIZE", args.write_dir, "write")):
        rows = _counter_rows(folder, counter)
        apply_kib = [v for k, _, v in rows if "apply_mfma_kernel" in k]
        copy_kib = [v for k, _, v in rows if "apply" not in k and "copy" in k.lower()]
        if not apply_kib or not copy_kib:
            raise SystemExit(f"{counter}: apply or copy dispatch missing in {folder}")
        scale = copy_bytes / (max(copy_kib) * 1024.0)
        out[f"{key}_kib_per_launch"] = float(np.mean(apply_kib))
        out[f"{key}_copy_kib"] = float(max(copy_kib))
        out[f"{key}_scale"] = scale
        out[f"{key}_bytes_per_launch"] = float(np.mean(apply_kib)) * 1024.0 * scale
    out["traffic_bytes_per_launch"] = out["fetch_bytes_per_launch"] + out["write_bytes_per_launch"]
    out["traffic_over_algorithmic"] = out["traffic_bytes_per_launch"] / out["algorithmic_bytes_per_launch"]
    out["commands"] = [
        f"rocprofv3 --pmc {c} --kernel-trace --output-format csv -d <out>/{d} -o run -- python3 bench.py "
        f"--workload profile --model {args.model} --K {args.K} --L {args.L} --cells {args.cells} "
        f"--precision {args.precision}" for c, d in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write"))]
    path = traffic_file(args.precision, args.K, args.L, args.cells)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out), flush=True)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_steps(fn, steps, stream, torch):
    """Per-step device time from HIP events recorded on the launch stream."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = np.array([a.elapsed_time(b) for a, b in evs])
    return ms, wall


def _oracle_cells(job):
    """The oracle's literal factorized sum (Section 4.5 as written) over cells until the time
    budget runs out, with one BLAS thread; returns (cells done, seconds, their Q rows)."""
    R, T, K, cells, budget = job
    from threadpoolctl import threadpool_limits
    from oracle import apply as oapply
    out = []
    with threadpool_limits(limits=1):
        done, t0 = 0, time.perf_counter()
        while done < len(cells) and time.perf_counter() - t0 < budget:
            out.append(oapply.apply_q(R, T, cells[done], K))
            done += 1
        return done, time.perf_counter() - t0, np.array(out).reshape(done, -1)


def cpu_baseline(K, L, gamma, c, budget_s, single_budget_s=5.0, max_workers=16):
    """The oracle on the host: one worker process per core (at most max_workers), each on its
    own cells of the batch for budget_s, and one thread alone for single_budget_s.  Runs
    before the GPU is initialized, so the workers are plain CPU processes.  Returns the
    record and the oracle's Q for the cells it finished (batch indices, rows), which the GPU
    results are then checked against."""
    import multiprocessing
    from oracle import core as ocore, gaunt as ogaunt
    T = ogaunt.coo(L)
    R = ocore.zero_invariants(ocore.core_exact(K, L, gamma, table=T), T["channels"])
    done1, dt1, _ = _oracle_cells((R, T, K, c[:64], single_budget_s))
    workers = max(1, min(os.cpu_count() or 1, max_workers))
    cap = min(len(c), 256 * workers)
    jobs = [(R, T, K, np.ascontiguousarray(c[i:cap:workers]), budget_s) for i in range(workers)]
    with multiprocessing.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_oracle_cells, jobs)
    done, dt = sum(r[0] for r in res), max(r[1] for r in res)
    idx = np.concatenate([np.arange(i, cap, workers)[:r[0]] for i, r in enumerate(res)])
    qref = np.concatenate([r[2] for r in res])
    rec = {"value": done / dt, "unit": "cells/s", "cores": workers, "kind": "oracle",
           "sample": f"{done} cells of the same batch over {workers} worker processes with one thread each "
                     f"(oracle factorized sum, Section 4.5 as written), {dt:.1f} s",
           "single_thread": {"value": done1 / dt1, "unit": "cells/s", "cores": 1,
                             "sample": f"{done1} cells, {dt1:.1f} s"}}
    return rec, (idx, qref)


def mode_errors(q, ref):
    """Error per output mode alpha, e_alpha = max_b |q_b,alpha - ref_b,alpha| / max_{b,alpha'} |ref|,
    summarized as its maximum and median over modes, and the normwise relative error."""
    q = np.asarray(q, dtype=np.float64)
    scale = np.abs(ref).max()
    e = np.abs(q - ref).max(axis=0) / scale
    return {"max_mode": float(e.max()), "median_mode": float(np.median(e)),
            "normwise": float(np.linalg.norm(q - ref) / np.linalg.norm(ref))}


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def measured_peaks(wefq, stream):
    """Attainable rates (TFLOP/s) from the library's rate probe, beside the datasheet figures."""
    return {kind: wefq.peak_probe(kind, device=0, stream=stream) for kind in wefq.PROBES}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cells", type=int, default=65536)
    ap.add_argument("--K", type=int, default=12)
    ap.add_argument("--L", type=int, default=12)
    ap.add_argument("--gamma", type=float, default=0.5)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--naive-cells", type=int, default=2048)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64/BF16x3 comparison legs")
    ap.add_argument("--workload", choices=["k12", "uneven", "serve", "rk", "jvp", "build", "orderings", "profile",
                                           "traffic"],
                    default="k12",
                    help="k12: the headline batch; uneven: one persistent launch over a mix of cores; "
                         "serve: continuous-batching server under Poisson arrivals; "
                         "rk: batched RK4 time stepping (anisotropic stress relaxation, hard spheres); "
                         "jvp: Jacobian-vector products J(c) d on the headline batch; "
                         "build: radial core build times, isotropic and with angular factors, and reload; "
                         "orderings: naive, radial-first and angular-first FP64 at K = 4, L = 2..13; "
                         "profile: a few launches of one apply (--K --L --cells --precision) and a plain "
                         "copy of f, the command to run under rocprofv3 counter passes; "
                         "traffic: HBM bytes per launch from the FETCH_SIZE and WRITE_SIZE passes "
                         "(--fetch-dir, --write-dir) of a profile run, written to profiles/ (no GPU)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3", "fp64"],
                    help="profile/traffic: the apply precision")
    ap.add_argument("--launches", type=int, default=2, help="profile: launches of the apply")
    ap.add_argument("--model", default="vhs", help="profile/traffic: collision model (gamma from --gamma)")
    ap.add_argument("--fetch-dir", default=None, help="traffic: output folder of the FETCH_SIZE pass")
    ap.add_argument("--write-dir", default=None, help="traffic: output folder of the WRITE_SIZE pass")
    ap.add_argument("--tick-ms", type=float, default=32.0, help="serve: work per scheduling tick, in ms")
    ap.add_argument("--serve-depth", type=int, default=2, help="serve: launches in flight")
    ap.add_argument("--serve-rates", type=float, nargs="*", default=None, help="serve: arrival rates (req/s)")
    ap.add_argument("--serve-tflops", type=float, default=None, help="serve: rate that sizes a tick (TFLOP/s)")
    ap.add_argument("--serve-block", type=int, default=None,
                    help="serve: threads per workgroup (256, 512 or 768; default 768 in FP32)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain device copy of f (known byte count) for counter scaling")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the operator is applied per cell with no exchange between "
              "GPUs, and this build runs on a single MI355X (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    if args.workload == "traffic":
        return traffic_from_counters(args)
    import torch
    import paper_2605_28475_amd as wefq
    from paper_2605_28475_amd import synth
    if args.workload == "profile":
        return profile_run(args, torch, wefq, synth)
    if args.workload == "uneven":
        return bench_uneven(args, torch, wefq, synth)
    if args.workload == "serve":
        from paper_2605_28475_amd import serve
        print(json.dumps(serve.bench(args)), flush=True)
        return
    if args.workload == "rk":
        return bench_rk(args, torch, wefq, synth)
    if args.workload == "jvp":
        return bench_jvp(args, torch, wefq, synth)
    if args.workload == "build":
        return bench_build(args, torch, wefq)
    if args.workload == "orderings":
        return bench_orderings(args, torch, wefq, synth)

    K, L, B, gamma = args.K, args.L, args.cells, args.gamma
    workload = f"vhs{gamma:g}_K{K}L{L}_B{B}"
    c = synth.perturbed_maxwellian(K, L, B, seed=synth.BASE_SEED + 3)
    cpu = oracle_q = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle), before the GPU is initialized")
        cpu, oracle_q = cpu_baseline(K, L, gamma, c, args.cpu_budget)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    log(f"[bench] building core {workload}")
    t0 = time.perf_counter()
    core = wefq.Core("vhs", K, L, gamma=gamma, device=0)
    build_s = time.perf_counter() - t0
    info = core.info
    N = core.N
    f64 = torch.tensor(c, device=dev)
    f32 = f64.float()
    q32 = torch.empty_like(f32)
    check = {}

    def step():
        core.apply_Q(f32, out=q32)
        check["max"] = core.check_conservation(q32, precision="fp32")

    if args.calibrate_copy:
        dst = torch.empty_like(f32)
        dst.copy_(f32)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {f32.numel() * 4} bytes read, {f32.numel() * 4} bytes written")
        del dst
    log("[bench] warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    # kernel-only times (apply alone) from events on the launch stream
    kms, _ = time_steps(lambda: core.apply_Q(f32, out=q32), args.steps, stream, torch)
    value = B / (wall / args.steps)
    flop_cell = info["flop_alg_per_cell"]
    achieved = flop_cell * B / (np.mean(kms) * 1e-3) / 1e12
    out = {
        "metric": "Q(f,f) cell-evals/sec at Kmax=Lmax=12 vs plain FP64 GPU; p50/p99 latency",
        "value": value, "unit": "cells/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": workload, "Kmax": K, "Lmax": L, "gamma": gamma, "cells": B, "modes": N,
                   "precision": "fp32 coupling + fp32 MFMA contraction"},
        "p50_ms": float(np.percentile(kms, 50)), "p99_ms": float(np.percentile(kms, 99)),
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK["fp32"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK["fp32"], "traffic": measured_traffic(workload, "fp32", K, L, B),
                     "flop_per_cell": flop_cell, "kernel_ms": float(np.mean(kms)),
                     "algorithmic_bytes": 2.0 * B * N * 4},
        "conservation_max_abs": check["max"],
        "core_build_s": build_s, "quad_nodes": info["quad_nodes"],
    }
    if not args.no_compare:
        q64 = torch.empty_like(f64)
        log("[bench] fp64 comparator (same tiled kernel in FP64 with FP64 MFMA)")
        core.apply_Q(f64, out=q64, precision="fp64")
        ms64, _ = time_steps(lambda: core.apply_Q(f64, out=q64, precision="fp64"), args.fp64_steps, stream, torch)
        nb = min(args.naive_cells, B)
        log(f"[bench] fp64 naive ordering on {nb} cells")
        qn = torch.empty_like(f64[:nb])
        msn, _ = time_steps(lambda: core.apply_Q(f64[:nb], out=qn, precision="fp64_naive"), 1, stream, torch)
        naive_err = float((qn - q64[:nb]).abs().max().item() / q64[:nb].abs().max().item())
        q16 = torch.empty_like(f32)
        core.apply_Q(f32, out=q16, precision="bf16x3")
        ms16, _ = time_steps(lambda: core.apply_Q(f32, out=q16, precision="bf16x3"), args.steps, stream, torch)
        core.apply_Q(f32, out=q32)
        torch.cuda.synchronize()
        ref = q64.cpu().numpy()
        h32, h16 = q32.cpu().numpy(), q16.cpu().numpy()
        fp64_naive_cps = nb / (np.mean(msn) * 1e-3)
        out["fp64_tiled"] = {"cells_per_s": B / (np.mean(ms64) * 1e-3), "kernel_ms": float(np.mean(ms64)),
                             "roofline_frac": flop_cell * B / (np.mean(ms64) * 1e-3) / 1e12 / PEAK["fp64"],
                             "kernel": "angular-first tiles, FP64 coupling + FP64 MFMA (the same kernel as "
                                       "the FP32 path, in FP64)"}
        out["fp64_naive"] = {"cells_per_s": fp64_naive_cps, "cells": nb,
                             "kernel": "plain FP64 GPU apply: the naive ordering of the factorized sum "
                                       "(every COO row contracts its K^3 block), one thread per output",
                             "max_rel_diff_vs_fp64_tiled": naive_err}
        # the metric's comparator, the plain FP64 GPU apply, is the naive ordering; the tiled
        # FP64 kernel is the same optimized kernel as the headline, in FP64
        out["speedup_fp32_vs_fp64_naive"] = float(value / fp64_naive_cps)
        out["speedup_fp32_vs_fp64_tiled"] = float(np.mean(ms64) / np.mean(kms))
        out["bf16x3"] = {"cells_per_s": B / (np.mean(ms16) * 1e-3), "kernel_ms": float(np.mean(ms16)),
                         # algorithmic rate; no single peak bounds it (BF16 MFMA contraction, FP32 VALU coupling)
                         "achieved_tflops_alg": flop_cell * B / (np.mean(ms16) * 1e-3) / 1e12,
                         "p50_ms": float(np.percentile(ms16, 50)), "p99_ms": float(np.percentile(ms16, 99))}
        # accuracy: per output mode against the FP64 CPU oracle on the cells the CPU leg finished,
        # and against the GPU FP64 tiled apply on every cell of the batch
        if oracle_q is not None:
            idx, qo = oracle_q
            out["error_vs_oracle"] = {"cells": int(len(idx)), "reference": "FP64 CPU oracle (factorized sum "
                                      "with the oracle's own core) on the cells of the cpu_baseline leg",
                                      "fp32": mode_errors(h32[idx], qo), "bf16x3": mode_errors(h16[idx], qo),
                                      "fp64_tiled": mode_errors(ref[idx], qo)}
        out["error_vs_fp64_tiled"] = {"cells": B, "fp32": mode_errors(h32, ref), "bf16x3": mode_errors(h16, ref)}
        del q64
        out["single_cell_latency"] = bench_single_cell(torch, wefq, synth, stream)
        out["k8_batch"] = bench_k8(torch, wefq, synth, stream)
        log("[bench] measured peaks (rate probe)")
        mp = measured_peaks(wefq, stream)
        out["measured_peaks_tflops"] = mp
        out["roofline"]["measured_peak"] = mp["mfma_f32"]
        out["roofline"]["frac_measured_peak"] = achieved / mp["mfma_f32"]
        out["fp64_tiled"]["roofline_frac_measured_peak"] = out["fp64_tiled"]["roofline_frac"] * PEAK["fp64"] / mp["mfma_f64"]
    if cpu is not None:
        out["cpu_baseline"] = cpu
    out["host_cpu"] = {"cpu_count": os.cpu_count(), "model": host_cpu_model()}
    core.close()
    print(json.dumps(out), flush=True)


def bench_single_cell(torch, wefq, synth, stream):
    """One hard-sphere cell at K = L = 3 in FP64: launch-to-completion latency of apply_Q
    (HIP events around each call, 200 calls) and the conservation check."""
    dev = torch.device("cuda:0")
    core = wefq.Core("hs", 3, 3, device=0, precisions=("fp64",))
    f = torch.tensor(synth.perturbed_maxwellian(3, 3, 1, seed=synth.BASE_SEED + 1), device=dev)
    q = torch.empty_like(f)
    core.apply_Q(f, out=q, precision="fp64")
    ms, _ = time_steps(lambda: core.apply_Q(f, out=q, precision="fp64"), 200, stream, torch)
    cons = core.check_conservation(q, precision="fp64")
    flop = core.info["flop_alg_per_cell"]
    core.close()
    # one cell is latency-bound: the FP64 fraction states how far from it the launch is
    return {"workload": "hs_K3L3_B1_fp64", "p50_ms": float(np.percentile(ms, 50)),
            "p99_ms": float(np.percentile(ms, 99)), "conservation_max_abs": cons,
            "roofline_frac_fp64": flop / (np.percentile(ms, 50) * 1e-3) / 1e12 / PEAK["fp64"]}


def bench_k8(torch, wefq, synth, stream):
    """Maxwell molecules and hard spheres at K = L = 8, 4,096 cells: FP32 and FP64 (the same
    tiled kernel) cells/s and the FP32 error against FP64."""
    dev = torch.device("cuda:0")
    res = {}
    for name, gamma in (("mm", 0.0), ("hs", 1.0)):
        core = wefq.Core(name, 8, 8, device=0, precisions=("fp64", "fp32"))
        f64 = torch.tensor(synth.perturbed_maxwellian(8, 8, 4096, seed=synth.BASE_SEED + 2), device=dev)
        f32 = f64.float()
        q64, q32 = torch.empty_like(f64), torch.empty_like(f32)
        core.apply_Q(f64, out=q64, precision="fp64")
        core.apply_Q(f32, out=q32, precision="fp32")
        ms64, _ = time_steps(lambda: core.apply_Q(f64, out=q64, precision="fp64"), 50, stream, torch)
        ms32, _ = time_steps(lambda: core.apply_Q(f32, out=q32, precision="fp32"), 50, stream, torch)
        err = float((q32.double() - q64).abs().max().item() / q64.abs().max().item())
        flop = core.info["flop_alg_per_cell"] * 4096
        res[name] = {"fp32_cells_per_s": 4096 / (np.mean(ms32) * 1e-3), "fp64_cells_per_s": 4096 / (np.mean(ms64) * 1e-3),
                     "fp32_roofline_frac": flop / (np.mean(ms32) * 1e-3) / 1e12 / PEAK["fp32"],
                     "fp64_roofline_frac": flop / (np.mean(ms64) * 1e-3) / 1e12 / PEAK["fp64"],
                     "fp32_p99_ms": float(np.percentile(ms32, 99)), "fp64_p99_ms": float(np.percentile(ms64, 99)),
                     "fp32_max_rel_err_vs_fp64": err}
        core.close()
    return {"workload": "mm_and_hs_K8L8_B4096"} | res


# angular factors of the build workload: Legendre coefficients of beta(cos chi)
BUILD_BETAS = {"isotropic": None, "deg3": (1.0, 0.5, 0.3, 0.1),
               "deg8": (1.0, 0.8, 0.55, 0.35, 0.2, 0.1, 0.05, 0.02, 0.005)}


def bench_build(args, torch, wefq):
    """Wall time of wefq_build_core (FP64 quadrature on the GPU plus the apply tables of all
    precisions) for hard spheres at K = L = 8, 12, 16, isotropic and with two angular factors,
    and of wefq_core_load of the same core from a file."""
    import tempfile
    torch.cuda.set_device(0)
    wefq.Core("hs", 2, 2, device=0, precisions=("fp64",)).close()      # context and module load
    rows = []
    with tempfile.TemporaryDirectory() as tmp:
        for K in (8, 12, 16):
            for name, beta in BUILD_BETAS.items():
                log(f"[build] K=L={K} {name}")
                t0 = time.perf_counter()
                core = wefq.Core("hs", K, K, device=0, beta=beta)
                t_build = time.perf_counter() - t0
                row = {"K": K, "L": K, "beta": name, "build_s": t_build,
                       "quad_nodes": core.info["quad_nodes"], "device_bytes": core.info["device_bytes"]}
                if beta is None:
                    path = os.path.join(tmp, f"k{K}.wefq")
                    core.save(path)
                    t0 = time.perf_counter()
                    wefq.Core.load(path, device=0).close()
                    row["load_s"] = time.perf_counter() - t0
                core.close()
                rows.append(row)
    k12 = [r for r in rows if r["K"] == 12 and r["beta"] == "isotropic"][0]
    out = {"metric": "radial core build time, hard spheres, K = L = 12 (FP64 on the GPU)",
           "value": k12["build_s"], "unit": "s", "n_gpus": 1, "higher_is_better": False,
           "dtype": "f64", "data": "synthetic", "config": {"workload": "core_build_hs"}, "builds": rows}
    print(json.dumps(out), flush=True)


def bench_orderings(args, torch, wefq, synth):
    """The orderings of the factorized sum (Section 4.5) on one GPU, FP64, hard spheres,
    K = 4 and L = 2..13, 16,384 cells: naive (every table row contracts its NK^3 block; on
    2,048 cells), radial-first (the dense intermediate Psi through HBM, then one pass over the
    table), angular-first (the tiled MFMA kernel) and the dense Cartesian contraction of
    Section 4.5.1 (the full N^3 tensor C assembled in HBM, 2 N^3 FLOPs per cell on the FP64
    matrix cores; on 2,048 cells).  One more point compares radial-first with angular-first at
    K = L = 12 (VHS 0.5, 1,024 cells)."""
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    K, B, nb_naive, nb_dense = 4, 16384, 2048, 2048
    rows = []
    for L in (2, 4, 6, 8, 10, 12, 13):
        log(f"[orderings] K={K} L={L}")
        core = wefq.Core("hs", K, L, device=0, precisions=("fp64", "radial"))
        info = core.info
        N, NK = core.N, K + 1
        f = torch.tensor(synth.perturbed_maxwellian(K, L, B, seed=synth.BASE_SEED + 17), device=dev)
        q = torch.empty_like(f)
        core.apply_Q(f, out=q, precision="fp64")
        ms_a, _ = time_steps(lambda: core.apply_Q(f, out=q, precision="fp64"), 10, stream, torch)
        per64 = core.radial_workspace_bytes(64)
        chunk = max(64, min(B, (4 << 30) // per64 * 64))
        work = torch.empty(core.radial_workspace_bytes(chunk), dtype=torch.uint8, device=dev)
        qr = torch.empty_like(f)
        core.apply_Q_radial(f, out=qr, work=work)
        ms_r, _ = time_steps(lambda: core.apply_Q_radial(f, out=qr, work=work), 3, stream, torch)
        fn, qn = f[:nb_naive], torch.empty_like(f[:nb_naive])
        core.apply_Q(fn, out=qn, precision="fp64_naive")
        ms_n, _ = time_steps(lambda: core.apply_Q(fn, out=qn, precision="fp64_naive"), 2, stream, torch)
        log(f"[orderings] dense, C {core.dense_bytes() / 2**30:.2f} GiB")
        Cd = torch.empty(core.dense_bytes(), dtype=torch.uint8, device=dev)
        ms_asm, _ = time_steps(lambda: core.dense_assemble(Cd), 1, stream, torch)
        fd, qd = f[:nb_dense], torch.empty_like(f[:nb_dense])
        core.apply_Q_dense(Cd, fd, out=qd)
        ms_d, _ = time_steps(lambda: core.apply_Q_dense(Cd, fd, out=qd), 3, stream, torch)
        scale = q.abs().max().item()
        err_r = (qr - q).abs().max().item() / scale
        err_n = (qn - q[:nb_naive]).abs().max().item() / scale
        err_d = (qd - q[:nb_dense]).abs().max().item() / scale
        t_a, t_r, t_n, t_d = (float(np.mean(m)) * 1e-3 for m in (ms_a, ms_r, ms_n, ms_d))
        dense_tflops = 2.0 * N ** 3 * nb_dense / t_d / 1e12
        groups = info["radial_groups"]
        psi_bytes = 2.0 * groups * NK * 8 + 2.0 * N * 8          # Psi and the transposed f, written and read
        rows.append({"L": L, "N": N, "N_G": info["N_G"], "N_S": info["N_S"], "radial_groups": groups,
                     "angular_first_cells_per_s": B / t_a, "radial_first_cells_per_s": B / t_r,
                     "naive_cells_per_s": nb_naive / t_n,
                     "dense_cells_per_s": nb_dense / t_d, "dense_tflops": dense_tflops,
                     "dense_frac_fp64_peak": dense_tflops / PEAK["fp64"], "dense_assembly_ms": float(ms_asm[0]),
                     "dense_tensor_gib": core.dense_bytes() / 2 ** 30,
                     "angular_vs_dense": (B / t_a) / (nb_dense / t_d),
                     "angular_vs_naive": (B / t_a) / (nb_naive / t_n), "angular_vs_radial": t_r / t_a,
                     "radial_vs_naive": (B / t_r) / (nb_naive / t_n),
                     "flop_per_cell": {"angular_first": info["flop_alg_per_cell"],
                                       "radial_first": 2.0 * groups * (NK ** 3 + NK ** 2) + 2.0 * NK * info["N_G"],
                                       "naive": 2.0 * NK ** 3 * info["N_G"], "dense": 2.0 * N ** 3},
                     "radial_first_hbm_gb_s": psi_bytes * B / t_r / 1e9, "radial_chunk_cells": chunk,
                     "rel_err_vs_angular": {"radial_first": err_r, "naive": err_n, "dense": err_d}})
        log(f"[orderings] L={L}: angular {B / t_a:.3e}, radial {B / t_r:.3e}, naive {nb_naive / t_n:.3e}, "
            f"dense {nb_dense / t_d:.3e} cells/s ({dense_tflops:.1f} TFLOP/s)")
        del f, q, qr, work, fn, qn, Cd, fd, qd
        core.close()
    # the headline truncation: which ordering an apply should use at K = L = 12
    log("[orderings] K=L=12 (1,024 cells)")
    core = wefq.Core("vhs", 12, 12, gamma=0.5, device=0, precisions=("fp64", "radial"))
    f = torch.tensor(synth.perturbed_maxwellian(12, 12, 1024, seed=synth.BASE_SEED + 18), device=dev)
    q, qr = torch.empty_like(f), torch.empty_like(f)
    core.apply_Q(f, out=q, precision="fp64")
    ms_a, _ = time_steps(lambda: core.apply_Q(f, out=q, precision="fp64"), 5, stream, torch)
    work = torch.empty(core.radial_workspace_bytes(256), dtype=torch.uint8, device=dev)
    core.apply_Q_radial(f, out=qr, work=work)
    ms_r, _ = time_steps(lambda: core.apply_Q_radial(f, out=qr, work=work), 2, stream, torch)
    k12 = {"K": 12, "L": 12, "cells": 1024, "model": "vhs0.5",
           "angular_first_cells_per_s": 1024 / (np.mean(ms_a) * 1e-3),
           "radial_first_cells_per_s": 1024 / (np.mean(ms_r) * 1e-3),
           "angular_vs_radial": float(np.mean(ms_r) / np.mean(ms_a)),
           "rel_err_radial_vs_angular": (qr - q).abs().max().item() / q.abs().max().item()}
    del f, q, qr, work
    core.close()
    last = rows[-1]
    out = {"metric": "FP64 Q(f,f) cell-evals/sec by ordering, hard spheres, K = 4, L = 13",
           "value": last["angular_first_cells_per_s"], "unit": "cells/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "f64", "data": "synthetic", "config": {"workload": f"orderings_hs_K{K}_L2-13_B{B}", "cells": B},
           "orderings": rows, "headline_truncation": k12}
    print(json.dumps(out), flush=True)


def bench_jvp(args, torch, wefq, synth):
    """J(c) d = Q(c, d) + Q(d, c) on the headline batch (VHS 0.5, K = L = 12, 65,536 cells),
    FP32 and FP64, against one apply of Q on the same cells.  Algorithmic count: the
    coupling doubles (two outer products per row), the radial contraction does not."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    K, L, B, gamma = args.K, args.L, args.cells, args.gamma
    core = wefq.Core("vhs", K, L, gamma=gamma, device=0, precisions=("fp64", "fp32", "bilinear"))
    info = core.info
    NK = K + 1
    flop_cell = 2.0 * 2 * NK * NK * info["N_G"] + 2.0 * NK ** 3 * info["N_S"]
    c = synth.perturbed_maxwellian(K, L, B, seed=synth.BASE_SEED + 3)
    d = synth.perturbed_maxwellian(K, L, B, seed=synth.BASE_SEED + 8) - synth.unit_maxwellian(K, L, B)
    res = {}
    for prec, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        ct, dd = torch.tensor(c, dtype=dt, device=dev), torch.tensor(d, dtype=dt, device=dev)
        out = torch.empty_like(ct)
        core.apply_J(ct, dd, out=out, precision=prec)
        n = args.steps if prec == "fp32" else max(3, args.steps // 20)
        ms, _ = time_steps(lambda: core.apply_J(ct, dd, out=out, precision=prec), n, stream, torch)
        msq, _ = time_steps(lambda: core.apply_Q(ct, out=out, precision=prec), max(3, n // 4), stream, torch)
        msb, _ = time_steps(lambda: core.apply_Qfg(ct, dd, out=out, precision=prec), max(3, n // 4), stream, torch)
        t = float(np.mean(ms)) * 1e-3
        res[prec] = {"cells_per_s": B / t, "kernel_ms": 1e3 * t, "p50_ms": float(np.percentile(ms, 50)),
                     "p99_ms": float(np.percentile(ms, 99)), "apply_Q_ms": float(np.mean(msq)),
                     "bilinear_Qfg_ms": float(np.mean(msb)), "tflops": flop_cell * B / t / 1e12}
        del ct, dd, out
    t32 = res["fp32"]["kernel_ms"] * 1e-3
    out = {"metric": "J(c) d cell-evals/sec at Kmax=Lmax=12", "value": B / t32, "unit": "cells/s", "n_gpus": 1,
           "steps": args.steps, "warmup": 1, "ms_per_step": 1e3 * t32, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"jvp_vhs{gamma:g}_K{K}L{L}_B{B}", "cells": B},
           "roofline": {"bound": "mfma", "achieved": res["fp32"]["tflops"], "peak": PEAK["fp32"], "unit": "TFLOP/s",
                        "frac": res["fp32"]["tflops"] / PEAK["fp32"], "traffic": None, "flop_per_cell": flop_cell},
           "fp32": res["fp32"], "fp64": res["fp64"] | {"roofline_frac_fp64": res["fp64"]["tflops"] / PEAK["fp64"]}}
    core.close()
    print(json.dumps(out), flush=True)


def bench_rk(args, torch, wefq, synth):
    """Batched RK4 stepping of dc/dt = Q(c): hard spheres, K = L = 12, 65,536 cells, each a
    Maxwellian with an anisotropic stress perturbation in the (k, l) = (0, 2) modes plus the
    seeded perturbation law, FP32; one step = 4 applies + fused combinations + FP64 checks."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    K = L = 12
    B, dt, nsteps = args.cells, 0.05, 4
    core = wefq.Core("hs", K, L, gamma=1.0, device=0, precisions=("fp32",))
    c = synth.perturbed_maxwellian(K, L, B, seed=synth.BASE_SEED + 6)
    NK = K + 1
    for m, amp in zip(range(-2, 3), (0.0, 0.0, 0.3, 0.0, 0.15)):     # q = 4 + 2 + m, k = 0
        c[:, (6 + m) * NK] += amp
    c0 = torch.tensor(c, dtype=torch.float32, device=dev)
    x = c0.clone()
    work = torch.empty(core.rk_workspace_bytes(B, "rk4", "fp32"), dtype=torch.uint8, device=dev)
    log(f"[rk] {B} cells, RK4 dt={dt}, {nsteps} steps per timed call")
    core.rk_integrate(x, dt, 1, work=work)                            # warm-up
    x.copy_(c0)
    torch.cuda.synchronize()
    reps = max(1, args.steps // 20)
    ms = []
    for _ in range(reps):                                             # timed: no host readback
        a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        core.rk_integrate(x, dt, nsteps, work=work, check=False)
        e.record(stream)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(e))
    x.copy_(c0)
    t0 = time.perf_counter()
    inv = core.rk_integrate(x, dt, nsteps, work=work)                 # checked run from t = 0
    wall = time.perf_counter() - t0
    xs = x.cpu().numpy()
    idx = [0, 1, NK, 2 * NK, 3 * NK]
    drift = float(np.abs(xs[:, idx] - c0.cpu().numpy()[:, idx]).max())
    shear0 = float(np.abs(c[:, 6 * NK]).mean())                     # (k, l, m) = (0, 2, 0)
    shear1 = float(np.abs(xs[:, 6 * NK]).mean())
    ms_apply, _ = time_steps(lambda: core.apply_Q(c0, out=torch.empty_like(c0)), 5, stream, torch)
    step_ms = float(np.median(ms)) / nsteps
    flop = core.info["flop_alg_per_cell"] * B * 4
    out = {"metric": "RK4 cell-steps/sec, hard-sphere stress relaxation", "value": B / (step_ms * 1e-3),
           "unit": "cell-steps/s", "n_gpus": 1, "steps": reps * nsteps, "warmup": 1, "ms_per_step": step_ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "rk4_hs_K12L12_stress", "cells": B, "dt": dt, "scheme": "rk4"},
           "roofline": {"bound": "mfma", "achieved": flop / (step_ms * 1e-3) / 1e12, "peak": PEAK["fp32"],
                        "unit": "TFLOP/s", "frac": flop / (step_ms * 1e-3) / 1e12 / PEAK["fp32"], "traffic": None},
           "apply_ms": float(np.mean(ms_apply)), "overhead_vs_4_applies": step_ms / (4 * float(np.mean(ms_apply))),
           "checked_run_wall_ms": 1e3 * wall, "max_invariant_Q": inv, "invariant_coefficient_drift": drift,
           "mean_abs_shear_mode": {"t0": shear0, f"t{nsteps * dt:g}": shear1}}
    core.close()
    print(json.dumps(out), flush=True)


def bench_uneven(args, torch, wefq, synth):
    """20000 cells, K = L drawn from {4, 8, 12, 16}, hard spheres or VHS 0.5, FP32, one
    persistent graph-captured launch with tile shapes chosen by the autotuner on whole plans,
    against the default shapes and against separate launches."""
    from paper_2605_28475_amd import autotune
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    cfg = synth.WORKLOADS["uneven"]
    rng = np.random.Generator(np.random.PCG64(cfg["seed"]))
    total = cfg["cells"]
    size = rng.choice(np.array(cfg["sizes"]), size=total)
    model = rng.choice(np.array(["hs", "vhs"]), size=total)
    segs, flop = [], 0.0
    for K in cfg["sizes"]:
        for m in ("hs", "vhs"):
            B = int(np.sum((size == K) & (model == m)))
            if B == 0:
                continue
            log(f"[uneven] core {m} K=L={K}, {B} cells")
            core = wefq.Core(m, K, K, gamma=1.0 if m == "hs" else 0.5, device=0, precisions=("fp32",))
            f = torch.tensor(synth.perturbed_maxwellian(K, K, B, seed=cfg["seed"] + 10 * K + (m == "hs")),
                             dtype=torch.float32, device=dev)
            segs.append((core, f, torch.empty_like(f)))
            flop += core.info["flop_alg_per_cell"] * B
    log("[uneven] autotuning whole plans")
    slots, blk, tried = autotune.tune_plan(segs, "fp32")
    # the tuner's starting point: every core's default shape at its first block size
    zeros = "slots=" + ",".join("0" for _ in segs)
    default_key = next(k for k in tried if k.endswith(zeros))
    default_ms = tried[default_key]
    segs_used = [(c, f, q, s if s else c.tune_get("fp32")[0]) for (c, f, q), s in zip(segs, slots)]
    plan = wefq.Plan(segs_used, precision="fp32", block=blk)
    shape_name = "autotuned on whole plans"
    for _ in range(args.warmup):
        plan.launch()
    ms, wall = time_steps(lambda: plan.launch(), args.steps, stream, torch)
    ms_direct, _ = time_steps(lambda: plan.launch(graph=False), args.steps, stream, torch)

    def separate():
        for core, f, q, _ in segs_used:
            core.apply_Q(f, out=q)
    ms_sep, _ = time_steps(separate, args.steps, stream, torch)
    t = float(np.mean(ms)) * 1e-3
    out = {"metric": "Q(f,f) cell-evals/sec, uneven batch in one persistent launch", "value": total / t,
           "unit": "cells/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": float(np.mean(ms)), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "uneven_20000_K4-16_hs_vhs", "cells": total,
                      "segments": [{"model": c.model, "K": c.K, "cells": f.shape[0], "slots": s}
                                   for c, f, _, s in segs_used],
                      "tile_shapes": shape_name, "block": blk, "plan": plan.info},
           "p50_ms": float(np.percentile(ms, 50)), "p99_ms": float(np.percentile(ms, 99)),
           "roofline": {"bound": "mfma", "achieved": flop / t / 1e12, "peak": PEAK["fp32"], "unit": "TFLOP/s",
                        "frac": flop / t / 1e12 / PEAK["fp32"], "traffic": None},
           "graph_ms": float(np.mean(ms)), "direct_ms": float(np.mean(ms_direct)),
           "separate_launches_ms": float(np.mean(ms_sep)), "default_shapes_ms": default_ms,
           "default_shapes": default_key,
           "autotune_candidates_ms": tried}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

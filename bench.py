#!/usr/bin/env python3
"""Benchmark: SaCD outer iterations on one MI355X.

A step is one outer iteration of Alg. 1 (sweeps of modes 0, 1, 2: MTTKRP,
Gram-Hadamard H and L, gradient and Lipschitz importance, saturation
selection, projected Gauss-Seidel update, Gram and FP64 objective) over the
whole tensor, with the tensor and factors resident in HBM.  The metric is
nnz * R / (seconds per step).

Prints one JSON line.  Progress goes to stderr.

    python bench.py [--steps K] [--warmup W] [--workload zipf|small|uniform64|uniform128]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "zipf": "ZIPF_UIT",
    "small": "SMALL_UNIFORM",
    "uniform64": "UNIFORM_20M_R64",
    "uniform128": "UNIFORM_20M_R128",
}

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(w, dims, idx, vals, budget_s: float):
    """The FP64 oracle on the same tensor: whole iterations until the time
    budget is used (at least one), single thread."""
    from oracle import oracle as O
    t0 = time.perf_counter()
    T = O.Tensor(dims, idx, vals)
    m = O.Model(T, w.rank, seed=w.init_seed)
    log(f"[bench] oracle ingest {time.perf_counter() - t0:.1f} s")
    iters, spent = 0, 0.0
    while True:
        t1 = time.perf_counter()
        for n in range(3):
            m.sweep(n)
        spent += time.perf_counter() - t1
        iters += 1
        log(f"[bench] oracle iteration {iters}: {spent / iters:.2f} s/iter")
        if spent >= budget_s or iters >= 20:
            break
    per_iter = spent / iters
    return {
        "value": T.nnz * w.rank / per_iter,
        "unit": "nnz*R/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{iters} outer iteration(s) of the full tensor ({T.nnz} entries, R={w.rank}), "
                  f"FP64 C oracle, single thread, ingest excluded; {per_iter:.3f} s/iteration",
    }


def measured_traffic(workload: str):
    """HBM bytes per MTTKRP launch from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the plain-copy calibration),
    or None when no summary exists for this workload or the kernel source has
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_mttkrp_{workload.lower()}_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    try:
        blob = text[text.index("```json") + 7:]
        rec = json.loads(blob[:blob.index("```")])
    except ValueError:
        return None
    src = os.path.join(ROOT, "paper_2003_03572_amd", "csrc", "mttkrp.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec.get("mttkrp_hip_sha256"):
        return None
    return rec.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="zipf", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--kernel-reps", type=int, default=10)
    ap.add_argument("--data-cache", default="",
                    help="directory to keep the generated tensor in (reused when present)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                          "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2003_03572_amd import gen, sacd

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    sacd.lib()
    w = getattr(gen, WORKLOADS[args.workload])
    t0 = time.perf_counter()
    cache = os.path.join(args.data_cache, w.name + ".npz") if args.data_cache else None
    if cache and os.path.exists(cache):
        import numpy as np
        z = np.load(cache)
        dims, idx, vals = tuple(int(d) for d in z["dims"]), z["idx"], z["vals"]
    else:
        dims, idx, vals = gen.make(w)
        if cache:
            import numpy as np
            os.makedirs(args.data_cache, exist_ok=True)
            np.savez(cache, dims=np.array(dims), idx=idx, vals=vals)
    log(f"[bench] generated {w.name}: dims {dims}, nnz {idx.shape[0]} in {time.perf_counter() - t0:.1f} s")

    t0 = time.perf_counter()
    T = sacd.Tensor.from_numpy(dims, idx, vals)
    nnz = T.nnz
    torch.cuda.synchronize()
    t_ingest = time.perf_counter() - t0
    m = sacd.Model(T, w.rank, seed=w.init_seed)
    m.synchronize()
    log(f"[bench] GPU ingest {t_ingest:.3f} s (incl. host->device copy), model ready")

    stream = T.stream
    m.iterate(args.warmup)
    m.timing_prepare(args.steps)  # event creation, before the timed region
    m.synchronize()
    log(f"[bench] warmup {args.warmup} iterations done")

    # timed region: K outer iterations, enqueued launch by launch with HIP
    # events around the MTTKRP launches (same kernels and stream as the graph
    # replay of Model.iterate, which is timed after the region for reference)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    mt_ms = m.iterate_timed(args.steps)
    e1.record(stream)
    m.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    ms_per_step = 1e3 * wall / args.steps
    value = nnz * w.rank / (wall / args.steps)
    fit, f = m.fit()
    log(f"[bench] {args.steps} iterations: wall {1e3 * wall:.3f} ms, events {gpu_ms:.3f} ms, "
        f"fit {fit:.6f}")

    # dominant kernel: MTTKRP, 3 launches per step, timed inside the region
    mt_bytes_mode = [m.kernel_bytes(0, n) for n in range(3)]
    mt_time = sum(sum(r) for r in mt_ms) * 1e-3
    mt_bytes = args.steps * sum(mt_bytes_mode)
    achieved = mt_bytes / mt_time / 1e9
    mt_avg_us = [1e3 * sum(r[n] for r in mt_ms) / args.steps for n in range(3)]
    log(f"[bench] MTTKRP in the timed region: " +
        ", ".join(f"mode {n} {mt_avg_us[n]:.1f} us" for n in range(3)) +
        f"; {achieved:.0f} GB/s algorithmic")

    # other kernels, timed after the region (HIP events on the library stream)
    ktimes = {}
    for which, name in [(2, "importance"), (1, "select_update")]:
        for n in range(3):
            ktimes[(name, n)] = m.time_kernel(which, n, args.kernel_reps)
    for n in range(3):
        ktimes[("mttkrp", n)] = mt_avg_us[n] * 1e-3
    for (name, n), ms in ktimes.items():
        log(f"[bench] kernel {name} mode {n}: {1e3 * ms:.1f} us")
    traffic = measured_traffic(w.name)

    # the same iterations replayed from the captured graph (reference only)
    e0.record(stream)
    m.iterate(args.steps)
    e1.record(stream)
    m.synchronize()
    graph_ms = e0.elapsed_time(e1) / args.steps
    log(f"[bench] graph replay: {graph_ms:.3f} ms per iteration")

    out = {
        "metric": "nnz*R SaCD updates/sec per sweep",
        "value": value,
        "unit": "nnz*R/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "dims": list(dims), "nnz": nnz, "rank": w.rank,
                   "step": "one outer iteration (sweeps of modes 0, 1, 2) incl. FP64 objective",
                   "gpu_event_ms_per_step": gpu_ms / args.steps,
                   "graph_replay_ms_per_step": graph_ms,
                   "kernel_us": {f"{k[0]}_mode{k[1]}": round(1e3 * v, 2) for k, v in ktimes.items()}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_mttkrp (3 launches per step, one per mode, averaged)",
                     "algorithmic_bytes_per_launch": sum(mt_bytes_mode) / 3.0,
                     "avg_launch_us": sum(mt_avg_us) / 3.0},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, dims, idx, vals, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

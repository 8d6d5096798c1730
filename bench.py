#!/usr/bin/env python3
"""Benchmark: SaCD outer iterations on one MI355X.

A step is one outer iteration of Alg. 1 (sweeps of modes 0, 1, 2: MTTKRP,
Gram-Hadamard H and L, gradient and Lipschitz importance, saturation
selection, projected Gauss-Seidel update, Gram and FP64 objective) over the
whole tensor, with the tensor and factors resident in HBM.  The metric is
nnz * R / (seconds per step).

Prints one JSON line.  Progress goes to stderr.

    python bench.py [--steps K] [--warmup W] [--workload zipf|small|uniform64|uniform128]
                    [--precision fp32|mixed]
    python bench.py --workload batched     # 256 uneven jobs to tolerance, batched vs serial
    python bench.py --workload serving     # Poisson arrivals, served vs serial, p50/p99
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
                  f"FP64 C oracle, single thread, ingest excluded; {per_iter:.3f} s/iteration; "
                  f"host {host_cpu()}, {os.cpu_count()} hardware threads",
    }


def host_cpu() -> str:
    """The host CPU model (from /proc/cpuinfo), for the CPU baseline's record."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def mixed_vs_fp32(sacd, T, w, m_mixed, iters: int):
    """Objective, fit and factors of the mixed run against the FP32 GPU path
    (itself within 1e-5 of the FP64 oracle per sweep) after the same number
    of iterations from the same initial factors."""
    import numpy as np
    m32 = sacd.Model(T, w.rank, seed=w.init_seed)
    m32.iterate(iters)
    fit_b, f_b = m_mixed.fit()
    fit_a, f_a = m32.fit()
    rel = []
    for n in range(3):
        a = m32.factor(n).double().cpu().numpy()
        b = m_mixed.factor(n).double().cpu().numpy()
        rel.append(float(np.linalg.norm(b - a) / max(np.linalg.norm(a), 1e-300)))
    return {"iterations": iters, "f_rel": abs(f_b - f_a) / abs(f_a), "fit_mixed": fit_b, "fit_fp32": fit_a,
            "factor_rel": rel}


def _pool(gen, n_jobs: int, cache_dir: str):
    """The batched workload's job pool (generated, or loaded from the cache)."""
    import numpy as np
    specs = gen.job_specs(n_jobs)
    path = os.path.join(cache_dir, f"jobs{n_jobs}.npz") if cache_dir else None
    if path and os.path.exists(path):
        z = np.load(path)
        return [(sp, tuple(int(d) for d in z[f"d{j}"]), z[f"i{j}"], z[f"v{j}"]) for j, sp in enumerate(specs)]
    t0 = time.perf_counter()
    out = []
    for sp in specs:
        dims, idx, vals = gen.job_tensor(sp)
        out.append((sp, dims, idx, vals))
    log(f"[bench] generated {n_jobs} jobs in {time.perf_counter() - t0:.1f} s")
    if path:
        os.makedirs(cache_dir, exist_ok=True)
        arrs = {}
        for j, (sp, dims, idx, vals) in enumerate(out):
            arrs[f"d{j}"], arrs[f"i{j}"], arrs[f"v{j}"] = np.array(dims), idx, vals
        np.savez(path, **arrs)
    return out


def _serial(sacd, pool, prec, tol, max_iter):
    """The plain path: each job alone (ingest, factors, run to tolerance),
    one after the other.  Returns per-job (seconds, iterations, fit)."""
    import torch
    res = []
    for sp, dims, idx, vals in pool:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T = sacd.Tensor.from_numpy(dims, idx, vals)
        m = sacd.Model(T, sp.rank, seed=sp.seed, precision=prec)
        it, fit = m.run_until(tol, max_iter)
        res.append((time.perf_counter() - t0, it, fit))
        del m, T
    return res


def _pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def run_many(args):
    """Batched (all jobs at once) or served (Poisson arrivals) form against
    the plain one-job-at-a-time GPU path, at equal final fit."""
    import numpy as np
    import torch
    from paper_2003_03572_amd import gen, sacd
    tol, max_iter = 1e-4, 500
    serving = args.workload == "serving"
    prec_name = args.precision or ("mixed" if serving else "fp32")
    prec = sacd.PREC_MIXED_BF16 if prec_name == "mixed" else sacd.PREC_FP32
    pool = _pool(gen, args.jobs, args.data_cache)
    nnzR = [idx.shape[0] * sp.rank for sp, dims, idx, vals in pool]
    # warm the library (first launches, code objects) before timing
    _serial(sacd, pool[:2], prec, tol, 5)
    ser = _serial(sacd, pool, prec, tol, max_iter)
    ser_t = [r[0] for r in ser]
    log(f"[bench] serial path: {sum(ser_t):.2f} s for {len(pool)} jobs, "
        f"iterations {min(r[1] for r in ser)}..{max(r[1] for r in ser)}")
    base = {"n_gpus": 1, "higher_is_better": not serving, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32" if prec == sacd.PREC_FP32 else "bf16-mfma+f32", "data": "synthetic",
            "steps": None, "warmup": None}
    if not serving:
        budget = 16 << 30
        S = sacd.Server(budget, max_slots=len(pool), max_iter=max_iter, tol=tol, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tickets = [S.submit(dims, idx, vals, sp.rank, sp.seed) for sp, dims, idx, vals in pool]
        steps = 0
        while True:
            running, queued = S.step()
            steps += 1
            if running == 0 and queued == 0:
                break
        T_b = time.perf_counter() - t0
        polls = [S.poll(t) for t in tickets]
        equal = all(p["iters"] == r[1] and p["fit"] == r[2] for p, r in zip(polls, ser))
        work = sum(nr * p["iters"] for nr, p in zip(nnzR, polls))
        st = S.stats()
        out = dict(base)
        out.update({
            "metric": "nnz*R SaCD updates/sec, 256 uneven jobs run to tolerance",
            "value": work / T_b, "unit": "nnz*R/s", "ms_per_step": 1e3 * T_b / max(steps, 1),
            "steps": steps,
            "config": {"workload": f"batched-{len(pool)}-jobs-zipf1.1-r8to64", "tol": tol, "max_iter": max_iter,
                       "precision": prec_name, "batched_seconds": T_b, "serial_seconds": sum(ser_t),
                       "serial_value": work / sum(ser_t), "speedup_vs_serial": sum(ser_t) / T_b,
                       "results_equal_to_serial": equal, "total_nnz": int(sum(p[2].shape[0] for p in pool)),
                       "iterations_p50": _pct([p["iters"] for p in polls], 50),
                       "iterations_max": max(p["iters"] for p in polls),
                       "jobs_at_max_iter": sum(p["iters"] >= max_iter for p in polls),
                       "server": st,
                       "note": "batched: every job submitted at t=0 and resident at once; time includes "
                               "upload and ingest of every job; serial: each job alone, one after the other"},
        })
        print(json.dumps(out), flush=True)
        return
    # serving
    rates = [float(x) for x in args.rates.split(",")]
    sizes = [sum(sacd.job_bytes(dims, idx.shape[0], sp.rank, prec)) for sp, dims, idx, vals in pool]
    budget = int(args.budget_mb * 2**20) if args.budget_mb > 0 else int(24 * np.mean(sizes))
    per_rate = {}
    for lam in rates:
        rng = np.random.Generator(np.random.PCG64(3000 + int(lam)))
        arr = gen.poisson_arrivals(lam, args.requests, 3000 + int(lam))
        pick = rng.integers(0, len(pool), size=args.requests)
        # serial: one job at a time, first come first served, from the measured service times
        fin, lat_s = 0.0, []
        for a, j in zip(arr, pick):
            fin = max(fin, a) + ser_t[j]
            lat_s.append(fin - a)
        S = sacd.Server(budget, max_slots=256, max_iter=max_iter, tol=tol, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nxt, lat, done_t, info = 0, {}, {}, {}
        max_running = 0
        while len(done_t) < args.requests:
            now = time.perf_counter() - t0
            while nxt < args.requests and arr[nxt] <= now:
                sp, dims, idx, vals = pool[pick[nxt]]
                tk = S.submit(dims, idx, vals, sp.rank, sp.seed)
                info[tk] = nxt
                nxt += 1
            running, queued = S.step()
            max_running = max(max_running, running)
            t_now = time.perf_counter() - t0
            for tk in S.finished():
                k = info[tk]
                done_t[k] = t_now
                p = S.poll(tk)
                lat[k] = (t_now - arr[k], p["iters"], p["fit"])
                S.release(tk)
            if running == 0 and queued == 0 and nxt < args.requests:
                wait = arr[nxt] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
        T_total = time.perf_counter() - t0
        st = S.stats()
        S.close()
        lat_v = [lat[k][0] for k in range(args.requests)]
        equal = all(lat[k][1] == ser[pick[k]][1] and lat[k][2] == ser[pick[k]][2] for k in range(args.requests))
        per_rate[str(int(lam))] = {
            "served_p50_ms": 1e3 * _pct(lat_v, 50), "served_p99_ms": 1e3 * _pct(lat_v, 99),
            "serial_p50_ms": 1e3 * _pct(lat_s, 50), "serial_p99_ms": 1e3 * _pct(lat_s, 99),
            "served_jobs_per_s": args.requests / T_total, "serial_jobs_per_s": args.requests / fin,
            "served_nnzR_per_s": sum(nnzR[pick[k]] * lat[k][1] for k in range(args.requests)) / T_total,
            "max_running": max_running, "peak_bytes": st["peak_bytes"], "steps": st["steps"],
            "graph_launches": st["graph_launches"], "eager_launches": st["eager_launches"],
            "results_equal_to_serial": equal}
        log(f"[bench] rate {lam:.0f}/s: served p50 {per_rate[str(int(lam))]['served_p50_ms']:.1f} ms "
            f"p99 {per_rate[str(int(lam))]['served_p99_ms']:.1f} ms; serial p50 "
            f"{per_rate[str(int(lam))]['serial_p50_ms']:.1f} ms p99 {per_rate[str(int(lam))]['serial_p99_ms']:.1f} ms; "
            f"max running {max_running}")
    top = per_rate[str(int(rates[-1]))]
    out = dict(base)
    out.update({
        "metric": f"p99 time-to-tolerance (ms), served, {rates[-1]:.0f} req/s",
        "value": top["served_p99_ms"], "unit": "ms", "ms_per_step": None,
        "config": {"workload": f"serving-poisson-{args.requests}req-pool{len(pool)}", "tol": tol,
                   "max_iter": max_iter, "precision": prec_name, "budget_bytes": budget,
                   "rates": per_rate,
                   "note": "latency from arrival to result, incl. upload, ingest and queueing; serial: "
                           "one job at a time, first come first served, from each job's measured time alone"},
    })
    print(json.dumps(out), flush=True)


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
    ap.add_argument("--workload", default="zipf", choices=sorted(WORKLOADS) + ["batched", "serving"])
    ap.add_argument("--precision", default=None, choices=["fp32", "mixed"],
                    help="arithmetic of the dense products (default: fp32; serving: mixed)")
    ap.add_argument("--jobs", type=int, default=256, help="batched / serving: job pool size")
    ap.add_argument("--requests", type=int, default=2000, help="serving: requests per arrival rate")
    ap.add_argument("--rates", default="50,200,800", help="serving: arrival rates (1/s)")
    ap.add_argument("--budget-mb", type=float, default=0.0,
                    help="serving: HBM budget of the server (MB); 0 picks one that binds at the top rate")
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
        print(f"bench.py runs on one GPU only: this implementation has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2003_03572_amd import gen, sacd

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    sacd.lib()
    if args.workload in ("batched", "serving"):
        return run_many(args)
    prec = sacd.PREC_MIXED_BF16 if args.precision == "mixed" else sacd.PREC_FP32
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
    m = sacd.Model(T, w.rank, seed=w.init_seed, precision=prec)
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
    which_of = {"mttkrp": 0, "select_update": 1, "importance": 2}
    kernel_gbps = {f"{name}_mode{n}": round(m.kernel_bytes(which_of[name], n) / (ms * 1e-3) / 1e9, 1)
                   for (name, n), ms in ktimes.items()}
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
        "dtype": "f32" if prec == sacd.PREC_FP32 else "bf16-mfma+f32",
        "data": "synthetic",
        "config": {"workload": w.name, "dims": list(dims), "nnz": nnz, "rank": w.rank,
                   "step": "one outer iteration (sweeps of modes 0, 1, 2) incl. FP64 objective",
                   "gpu_event_ms_per_step": gpu_ms / args.steps,
                   "graph_replay_ms_per_step": graph_ms,
                   "kernel_us": {f"{k[0]}_mode{k[1]}": round(1e3 * v, 2) for k, v in ktimes.items()},
                   # algorithmic bytes of each launch over its measured time
                   "kernel_gbps_algorithmic": kernel_gbps},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_mttkrp (3 launches per step, one per mode, averaged)",
                     "algorithmic_bytes_per_launch": sum(mt_bytes_mode) / 3.0,
                     "avg_launch_us": sum(mt_avg_us) / 3.0},
    }
    if prec != sacd.PREC_FP32:
        out["config"]["precision"] = "mixed: Gram and A*H on BF16 MFMA, FP32 accumulation"
        out["config"]["vs_fp32_gpu"] = mixed_vs_fp32(sacd, T, w, m, args.warmup + 2 * args.steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, dims, idx, vals, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

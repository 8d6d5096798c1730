#!/usr/bin/env python3
"""Benchmark: SaCD outer iterations on one MI355X.

A step is one outer iteration of Alg. 1 (sweeps of modes 0, 1, 2: MTTKRP,
Gram-Hadamard H and L, gradient and Lipschitz importance, saturation
selection, projected Gauss-Seidel update, Gram and FP64 objective) over the
whole tensor, with the tensor and factors resident in HBM.  The metric is
nnz * R / (seconds per step).

The default run prints one JSON line whose headline is the largest
single-GPU configuration, the 2e7-entry uniform tensor at R = 128 in FP32,
with per-mode values; its `config` also carries the Zipf user x item x tag
tensor (1e7 entries, R = 32), its 4-way extension with a day mode, and the
served-vs-serial latencies to tolerance
(Poisson arrivals at 50, 200 and 800 requests/s, both paths run live).
Progress goes to stderr.

    python bench.py [--steps K] [--warmup W]              # headline + extras
    python bench.py --workload zipf|small|uniform64|uniform128 [--precision fp32|mixed]
    python bench.py --workload nway        # the 4-way Zipf tensor (1e7 entries, R = 32)
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
# FP32 vector peak of MI355X: 256 CUs x 128 FP32 lanes (packed FMA) x 2 flops x 2.4 GHz
FP32_VECTOR_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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


def cpu_baseline(w, dims, idx, vals, budget_s: float, threads: int = 1):
    """The FP64 oracle on the same tensor: whole iterations until the time
    budget is used (at least one), on `threads` threads of the host (0: all
    the OpenMP runtime offers).  Results are bit-identical for any count."""
    from oracle import oracle as O
    prev = O.set_threads(0)
    used = O.set_threads(threads if threads > 0 else prev)
    try:
        t0 = time.perf_counter()
        T = O.Tensor(dims, idx, vals)
        m = O.Model(T, w.rank, seed=w.init_seed)
        log(f"[bench] oracle ingest {time.perf_counter() - t0:.1f} s ({used} threads)")
        iters, spent = 0, 0.0
        while True:
            t1 = time.perf_counter()
            for n in range(3):
                m.sweep(n)
            spent += time.perf_counter() - t1
            iters += 1
            log(f"[bench] oracle iteration {iters} ({used} threads): {spent / iters:.2f} s/iter")
            if spent >= budget_s or iters >= 20:
                break
    finally:
        O.set_threads(prev)
    per_iter = spent / iters
    return {
        "value": T.nnz * w.rank / per_iter,
        "unit": "nnz*R/s",
        "cores": used,
        "kind": "oracle",
        "sample": f"{iters} outer iteration(s) of the full tensor ({T.nnz} entries, R={w.rank}), "
                  f"FP64 C oracle, {used} thread(s) (OpenMP over independent slices, rows and Gram "
                  f"entries), ingest excluded; {per_iter:.3f} s/iteration; host {host_cpu()}, "
                  f"{os.cpu_count()} hardware threads visible",
    }


def mixed_vs_fp32(sacd, T, w, m_mixed, iters: int):
    """Objective, fit and factors of the mixed run against the FP32 GPU path
    after the same number of iterations from the same initial factors (the
    errors of both against the FP64 oracle are stated by the mixed-form
    tests)."""
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


def _median(xs):
    s = sorted(xs)
    k = len(s)
    return 0.5 * (s[(k - 1) // 2] + s[k // 2]) if k else None


def load_workload(gen, w, data_cache: str):
    import numpy as np
    t0 = time.perf_counter()
    cache = os.path.join(data_cache, w.name + ".npz") if data_cache else None
    if cache and os.path.exists(cache):
        z = np.load(cache)
        dims, idx, vals = tuple(int(d) for d in z["dims"]), z["idx"], z["vals"]
    else:
        dims, idx, vals = gen.make(w)
        if cache:
            os.makedirs(data_cache, exist_ok=True)
            np.savez(cache, dims=np.array(dims), idx=idx, vals=vals)
    log(f"[bench] generated {w.name}: dims {dims}, nnz {idx.shape[0]} in {time.perf_counter() - t0:.1f} s")
    return dims, idx, vals


def run_tensor(sacd, gen, w, prec, args, with_cpu: bool):
    """One tensor workload: K timed iterations (launch by launch, HIP events
    around every MTTKRP launch and at the end of every sweep), the kernels
    timed one by one, the graph replay; returns the JSON record."""
    import torch
    dims, idx, vals = load_workload(gen, w, args.data_cache)
    t0 = time.perf_counter()
    T = sacd.Tensor.from_numpy(dims, idx, vals)
    nnz = T.nnz
    torch.cuda.synchronize()
    t_ingest = time.perf_counter() - t0
    m = sacd.Model(T, w.rank, seed=w.init_seed, precision=prec, columns=args.columns)
    m.synchronize()
    log(f"[bench] GPU ingest {t_ingest:.3f} s (incl. host->device copy), model ready "
        f"({m.device_bytes() / 2**20:.1f} MiB of model state)")

    stream = T.stream
    m.iterate(args.warmup)
    m.timing_prepare(args.steps)  # event creation, before the timed region
    m.synchronize()
    log(f"[bench] warmup {args.warmup} iterations done")

    # timed region: K outer iterations, enqueued launch by launch with HIP
    # events around the MTTKRP launches and after every sweep (same kernels
    # and stream as the graph replay of Model.iterate, timed afterwards)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    mt_ms, sw_ms = m.iterate_timed(args.steps, sweeps=True)
    e1.record(stream)
    m.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    ms_per_step = 1e3 * wall / args.steps
    value = nnz * w.rank / (wall / args.steps)
    fit, f = m.fit()
    log(f"[bench] {w.name}: {args.steps} iterations: wall {1e3 * wall:.3f} ms, events {gpu_ms:.3f} ms, "
        f"fit {fit:.6f}")

    # dominant kernel: MTTKRP, 3 launches per step, timed inside the region
    mt_bytes_mode = [m.kernel_bytes(0, n) for n in range(3)]
    mt_flops_mode = 3.0 * w.rank * nnz  # per launch: per entry and column one product and one FMA
    mt_time = sum(sum(r) for r in mt_ms) * 1e-3
    mt_avg_us = [1e3 * sum(r[n] for r in mt_ms) / args.steps for n in range(3)]
    achieved_gbs = args.steps * sum(mt_bytes_mode) / mt_time / 1e9
    achieved_tflops = args.steps * 3 * mt_flops_mode / mt_time / 1e12
    log(f"[bench] MTTKRP in the timed region: " +
        ", ".join(f"mode {n} {mt_avg_us[n]:.1f} us" for n in range(3)) +
        f"; {achieved_gbs:.0f} GB/s algorithmic, {achieved_tflops:.2f} TFLOP/s")
    per_mode = {}
    for n in range(3):
        sw_med = _median([r[n] for r in sw_ms])
        per_mode[f"mode{n}"] = {"sweep_ms_median": sw_med,
                                "mttkrp_us_median": 1e3 * _median([r[n] for r in mt_ms]),
                                "nnzR_per_s_sweep": nnz * w.rank / (sw_med * 1e-3)}
    step_ms = [sum(r) for r in sw_ms]

    # other kernels, timed after the region (HIP events on the library stream)
    ktimes = {}
    for which, name in ([(2, "importance"), (1, "select_update")] if not args.columns else []):
        for n in range(3):
            ktimes[(name, n)] = m.time_kernel(which, n, args.kernel_reps)
    for n in range(3):
        ktimes[("mttkrp", n)] = mt_avg_us[n] * 1e-3
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

    # the roofline that bounds the MTTKRP: HBM (algorithmic bytes) or the FP32
    # vector units (3 R flops per entry), whichever gives the longer time
    alg_bytes = sum(mt_bytes_mode) / 3.0
    t_hbm = alg_bytes / (HBM_PEAK_GBS * 1e9)
    t_alu = mt_flops_mode / (FP32_VECTOR_PEAK_TFLOPS * 1e12)
    if t_alu > t_hbm:
        roof = {"bound": "alu", "achieved": achieved_tflops, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS}
    else:
        roof = {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved_gbs / HBM_PEAK_GBS}
    roof.update({"traffic": traffic,
                 "kernel": "k_mttkrp (3 launches per step, one per mode, averaged)",
                 "algorithmic_bytes_per_launch": alg_bytes, "flops_per_launch": mt_flops_mode,
                 "avg_launch_us": sum(mt_avg_us) / 3.0,
                 "hbm_gbs_algorithmic": achieved_gbs, "hbm_frac_algorithmic": achieved_gbs / HBM_PEAK_GBS,
                 "fp32_tflops": achieved_tflops, "fp32_frac": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS})

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
                   "gpu_event_ms_per_step_median": _median(step_ms),
                   "graph_replay_ms_per_step": graph_ms,
                   "per_mode": per_mode,
                   "kernel_us": {f"{k[0]}_mode{k[1]}": round(1e3 * v, 2) for k, v in ktimes.items()},
                   # algorithmic bytes of each launch over its measured time
                   "kernel_gbps_algorithmic": kernel_gbps,
                   "ingest_s_incl_upload": t_ingest,
                   "model_device_bytes": m.device_bytes()},
        "roofline": roof,
    }
    if args.columns:
        out["config"]["form"] = (f"column-at-a-time, {args.columns} columns per block: the MTTKRP interval covers "
                                 f"both passes over the column blocks")
    if prec != sacd.PREC_FP32:
        out["config"]["precision"] = "mixed: Gram and A*H on BF16 MFMA, FP32 accumulation"
        out["config"]["vs_fp32_gpu"] = mixed_vs_fp32(sacd, T, w, m, args.warmup + 2 * args.steps)
    del m, T
    torch.cuda.synchronize()
    if with_cpu:
        out["cpu_baseline"] = cpu_baseline(w, dims, idx, vals, args.cpu_budget, threads=0)
        one = cpu_baseline(w, dims, idx, vals, args.cpu_budget, threads=1)
        out["config"]["cpu_baseline_1_thread"] = one
    return out


def run_nway(sacd, gen, w, args):
    """An N-way tensor (Sec. 3 for N modes): K timed outer iterations (sweeps
    of modes 0, ..., N - 1, launch by launch with HIP events around every
    MTTKRP launch and at the end of every sweep) and the graph replay;
    returns the record that goes into the headline's config."""
    import torch
    dims, idx, vals = load_workload(gen, w, args.data_cache)
    N = len(dims)
    T = sacd.NTensor.from_numpy(dims, idx, vals)
    nnz = T.nnz
    m = sacd.NModel(T, w.rank, seed=w.init_seed)
    m.iterate(args.warmup)
    m.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mt_ms, sw_ms = m.iterate_timed(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fit = m.fit()[0]
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(T.stream)
    m.iterate(args.steps)
    e1.record(T.stream)
    m.synchronize()
    graph_ms = e0.elapsed_time(e1) / args.steps
    R = w.rank
    # MTTKRP of mode n: 12 B per entry (key, value), each row of the N - 1
    # other factors read once and M written once (4 R B per row); N R flops
    # per entry (N - 2 products of rows, one by x, one add)
    mt_bytes = [12.0 * nnz + 4.0 * R * (sum(dims) - dims[n]) + 4.0 * R * dims[n] for n in range(N)]
    mt_us = [1e3 * _median([float(r[n]) for r in mt_ms]) for n in range(N)]
    mt_time = float(mt_ms.sum()) * 1e-3
    gbs = args.steps * sum(mt_bytes) / mt_time / 1e9
    log(f"[bench] {w.name}: {1e3 * wall / args.steps:.3f} ms per iteration (graph {graph_ms:.3f}), MTTKRP " +
        ", ".join(f"{u:.1f} us" for u in mt_us) + f", {gbs:.0f} GB/s algorithmic, fit {fit:.6f}")
    return {"workload": w.name, "dims": list(dims), "nnz": nnz, "rank": R, "modes": N,
            "value": nnz * R / (wall / args.steps), "unit": "nnz*R/s", "ms_per_step": 1e3 * wall / args.steps,
            "graph_replay_ms_per_step": graph_ms, "fit_after": fit,
            "per_mode": {f"mode{n}": {"sweep_ms_median": _median([float(r[n]) for r in sw_ms]),
                                      "mttkrp_us_median": mt_us[n]} for n in range(N)},
            "mttkrp_roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": gbs / HBM_PEAK_GBS, "kernel": "k_mttkrp_n (one launch per mode)",
                                "algorithmic_bytes_per_launch": sum(mt_bytes) / N}}


# ------------------------------------------------------------- many jobs ----

def _gen_job(spec):
    from paper_2003_03572_amd import gen
    dims, idx, vals = gen.job_tensor(spec)
    return dims, idx, vals


def _pool(gen, n_jobs: int, cache_dir: str):
    """The batched workload's job pool (generated in worker processes, or
    loaded from the cache)."""
    import numpy as np
    specs = gen.job_specs(n_jobs)
    path = os.path.join(cache_dir, f"jobs{n_jobs}.npz") if cache_dir else None
    if path and os.path.exists(path):
        z = np.load(path)
        return [(sp, tuple(int(d) for d in z[f"d{j}"]), z[f"i{j}"], z[f"v{j}"]) for j, sp in enumerate(specs)]
    t0 = time.perf_counter()
    import concurrent.futures as cf
    import multiprocessing as mp
    workers = max(1, min(16, os.cpu_count() or 1))
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        tensors = list(ex.map(_gen_job, specs, chunksize=4))
    out = [(sp, dims, idx, vals) for sp, (dims, idx, vals) in zip(specs, tensors)]
    log(f"[bench] generated {n_jobs} jobs in {time.perf_counter() - t0:.1f} s ({workers} processes)")
    if path:
        os.makedirs(cache_dir, exist_ok=True)
        arrs = {}
        for j, (sp, dims, idx, vals) in enumerate(out):
            arrs[f"d{j}"], arrs[f"i{j}"], arrs[f"v{j}"] = np.array(dims), idx, vals
        np.savez(path, **arrs)
    return out


def _one_job(sacd, job, prec, tol, max_iter):
    sp, dims, idx, vals = job
    T = sacd.Tensor.from_numpy(dims, idx, vals)
    m = sacd.Model(T, sp.rank, seed=sp.seed, precision=prec)
    it, fit = m.run_until(tol, max_iter)
    del m, T
    return it, fit


def _serial(sacd, pool, prec, tol, max_iter):
    """The plain path: each job alone (ingest, factors, run to tolerance),
    one after the other.  Returns per-job (seconds, iterations, fit)."""
    import torch
    res = []
    for job in pool:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, fit = _one_job(sacd, job, prec, tol, max_iter)
        res.append((time.perf_counter() - t0, it, fit))
    return res


def _serial_live(sacd, pool, arr, pick, prec, tol, max_iter):
    """The plain path under the same arrivals, run live: one job at a time,
    first come first served; latency from arrival to result."""
    t0 = time.perf_counter()
    lat, res = [], []
    for a, j in zip(arr, pick):
        now = time.perf_counter() - t0
        if now < a:
            time.sleep(a - now)
        it, fit = _one_job(sacd, pool[j], prec, tol, max_iter)
        lat.append(time.perf_counter() - t0 - a)
        res.append((it, fit))
    return lat, res, time.perf_counter() - t0


def _pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def run_served(sacd, gen, pool, prec, rates, requests, budget_mb, tol, max_iter):
    """Poisson arrivals at each rate against the server (continuous batching)
    and against the plain path, both live.  Returns (per-rate dict, budget)."""
    import numpy as np
    import torch
    sizes = [sum(sacd.job_bytes(dims, idx.shape[0], sp.rank, prec)) for sp, dims, idx, vals in pool]
    budget = int(budget_mb * 2**20) if budget_mb > 0 else int(24 * np.mean(sizes))
    nnzR = [idx.shape[0] * sp.rank for sp, dims, idx, vals in pool]
    per_rate = {}
    for lam in rates:
        rng = np.random.Generator(np.random.PCG64(3000 + int(lam)))
        arr = gen.poisson_arrivals(lam, requests, 3000 + int(lam))
        pick = rng.integers(0, len(pool), size=requests)
        S = sacd.Server(budget, max_slots=256, max_iter=max_iter, tol=tol, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nxt, lat, info = 0, {}, {}
        max_running = 0
        sec_submit = 0.0
        while len(lat) < requests:
            now = time.perf_counter() - t0
            while nxt < requests and arr[nxt] <= now:
                sp, dims, idx, vals = pool[pick[nxt]]
                ts = time.perf_counter()
                tk = S.submit(dims, idx, vals, sp.rank, sp.seed)
                sec_submit += time.perf_counter() - ts
                info[tk] = nxt
                nxt += 1
            running, queued = S.step()
            max_running = max(max_running, running)
            t_now = time.perf_counter() - t0
            for tk in S.finished():
                k = info[tk]
                p = S.poll(tk)
                lat[k] = (t_now - arr[k], p["iters"], p["fit"])
                S.release(tk)
            if running == 0 and queued == 0 and nxt < requests:
                wait = arr[nxt] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
        T_total = time.perf_counter() - t0
        st = S.stats()
        S.close()
        lat_v = [lat[k][0] for k in range(requests)]
        lat_s, res_s, T_serial = _serial_live(sacd, pool, arr, pick, prec, tol, max_iter)
        equal = all(lat[k][1] == res_s[k][0] and lat[k][2] == res_s[k][1] for k in range(requests))
        r = {"served_p50_ms": 1e3 * _pct(lat_v, 50), "served_p99_ms": 1e3 * _pct(lat_v, 99),
             "serial_p50_ms": 1e3 * _pct(lat_s, 50), "serial_p99_ms": 1e3 * _pct(lat_s, 99),
             "served_jobs_per_s": requests / T_total, "serial_jobs_per_s": requests / T_serial,
             "served_nnzR_per_s": sum(nnzR[pick[k]] * lat[k][1] for k in range(requests)) / T_total,
             "max_running": max_running, "peak_bytes": st["peak_bytes"], "steps": st["steps"],
             "graph_launches": st["graph_launches"], "eager_launches": st["eager_launches"],
             "host_seconds": {"submit": sec_submit, "admit": st["sec_admit"], "tables": st["sec_tables"],
                              "iterate": st["sec_iterate"], "retire": st["sec_retire"], "total": T_total},
             "results_equal_to_serial": equal}
        per_rate[str(int(lam))] = r
        log(f"[bench] rate {lam:.0f}/s: served p50 {r['served_p50_ms']:.1f} ms p99 {r['served_p99_ms']:.1f} ms "
            f"({r['served_jobs_per_s']:.0f} jobs/s); serial p50 {r['serial_p50_ms']:.1f} ms p99 "
            f"{r['serial_p99_ms']:.1f} ms ({r['serial_jobs_per_s']:.0f} jobs/s); max running {max_running}")
    return per_rate, budget


def run_many(args, pool):
    """Batched (all jobs at once) or served (Poisson arrivals) form against
    the plain one-job-at-a-time GPU path, at equal final fit."""
    import torch
    from paper_2003_03572_amd import gen, sacd
    tol, max_iter = 1e-4, 500
    serving = args.workload == "serving"
    prec_name = args.precision or ("mixed" if serving else "fp32")
    prec = sacd.PREC_MIXED_BF16 if prec_name == "mixed" else sacd.PREC_FP32
    nnzR = [idx.shape[0] * sp.rank for sp, dims, idx, vals in pool]
    _serial(sacd, pool[:2], prec, tol, 5)  # first launches, code objects
    base = {"n_gpus": 1, "higher_is_better": not serving, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32" if prec == sacd.PREC_FP32 else "bf16-mfma+f32", "data": "synthetic",
            "steps": None, "warmup": None}
    if not serving:
        ser = _serial(sacd, pool, prec, tol, max_iter)
        ser_t = [r[0] for r in ser]
        log(f"[bench] serial path: {sum(ser_t):.2f} s for {len(pool)} jobs")
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
                       "server": S.stats(),
                       "note": "batched: every job submitted at t=0 and resident at once; time includes "
                               "upload and ingest of every job; serial: each job alone, one after the other"},
        })
        print(json.dumps(out), flush=True)
        return
    rates = [float(x) for x in args.rates.split(",")]
    per_rate, budget = run_served(sacd, gen, pool, prec, rates, args.requests, args.budget_mb, tol, max_iter)
    top = per_rate[str(int(rates[-1]))]
    out = dict(base)
    out.update({
        "metric": f"p99 time-to-tolerance (ms), served, {rates[-1]:.0f} req/s",
        "value": top["served_p99_ms"], "unit": "ms", "ms_per_step": None,
        "config": {"workload": f"serving-poisson-{args.requests}req-pool{len(pool)}", "tol": tol,
                   "max_iter": max_iter, "precision": prec_name, "budget_bytes": budget, "rates": per_rate,
                   "note": "latency from arrival to result, incl. upload, ingest and queueing; serial: the "
                           "plain path run live under the same arrivals, one job at a time, first come first "
                           "served"},
    })
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="headline",
                    choices=["headline"] + sorted(WORKLOADS) + ["nway", "batched", "serving"],
                    help="headline (default): the uniform R = 128 FP32 line with the Zipf tensor and the "
                         "served-vs-serial latencies in its config")
    ap.add_argument("--precision", default=None, choices=["fp32", "mixed"],
                    help="arithmetic of the dense products (default: fp32; serving: mixed)")
    ap.add_argument("--jobs", type=int, default=256, help="batched / serving: job pool size")
    ap.add_argument("--requests", type=int, default=None,
                    help="serving: requests per arrival rate (default 2000; 500 in the headline run)")
    ap.add_argument("--rates", default="50,200,800", help="serving: arrival rates (1/s)")
    ap.add_argument("--budget-mb", type=float, default=0.0,
                    help="serving: HBM budget of the server (MB); 0 picks one that binds at the top rate")
    ap.add_argument("--columns", type=int, default=0,
                    help="tensor workloads: the column-at-a-time form with blocks of this many columns")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline: skip the Zipf and serving legs")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--kernel-reps", type=int, default=10)
    ap.add_argument("--data-cache", default="",
                    help="directory to keep the generated tensors in (reused when present)")
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

    from paper_2003_03572_amd import gen
    # the job pool is drawn by worker processes before this process touches
    # the GPU (no process is started from one that has initialised it)
    pool = None
    if args.workload in ("batched", "serving") or (args.workload == "headline" and not args.no_extras):
        pool = _pool(gen, args.jobs, args.data_cache)

    import torch
    from paper_2003_03572_amd import sacd

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    sacd.lib()
    if args.workload in ("batched", "serving"):
        if args.requests is None:
            args.requests = 2000
        return run_many(args, pool)
    if args.workload == "nway":
        print(json.dumps(run_nway(sacd, gen, gen.ZIPF_UITD, args)), flush=True)
        return
    prec = sacd.PREC_MIXED_BF16 if args.precision == "mixed" else sacd.PREC_FP32
    name = "uniform128" if args.workload == "headline" else args.workload
    w = getattr(gen, WORKLOADS[name])
    out = run_tensor(sacd, gen, w, prec, args, with_cpu=not args.no_cpu_baseline)
    if args.workload == "headline" and not args.no_extras:
        z = run_tensor(sacd, gen, gen.ZIPF_UIT, sacd.PREC_FP32, args, with_cpu=False)
        out["config"]["zipf_r32"] = {
            "workload": z["config"]["workload"], "value": z["value"], "unit": z["unit"],
            "ms_per_step": z["ms_per_step"], "roofline": z["roofline"], "per_mode": z["config"]["per_mode"],
            "kernel_us": z["config"]["kernel_us"], "graph_replay_ms_per_step": z["config"]["graph_replay_ms_per_step"]}
        out["config"]["nway_4mode_r32"] = run_nway(sacd, gen, gen.ZIPF_UITD, args)
        _serial(sacd, pool[:2], sacd.PREC_MIXED_BF16, 1e-4, 5)  # first launches, code objects
        per_rate, budget = run_served(sacd, gen, pool, sacd.PREC_MIXED_BF16,
                                      [float(x) for x in args.rates.split(",")], args.requests or 500,
                                      args.budget_mb, 1e-4, 500)
        out["config"]["serving"] = {
            "workload": f"serving-poisson-{args.requests or 500}req-pool{len(pool)}-mixed", "tol": 1e-4,
            "budget_bytes": budget, "rates": per_rate,
            "note": "p50/p99 time to tolerance from arrival (upload, ingest and queueing included), the "
                    "server (continuous batching, mixed form) against the plain path run live under the "
                    "same arrivals"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark: SPD HSS construction + PCG solve on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step = spdhss_build + ulv_factor + pcg_solve (to the workload's relative
residual) on an H^2 matrix that is already resident in HBM; the H^2 matrix is
built once beforehand and its construction time reported separately.  The
default workload is the N = 1M Gaussian configuration (l = 0.2, + 1e-3 I,
leaf 400, 16 right-hand sides) with eps_H = 1e-8, tau = 1e-2 and r = 200
(see workloads.HEADLINE for why these differ from 1e-6, 1e-1 and 100).  One
step takes about a minute or more, so the defaults are one step and no
warm-up (the H^2 build before the timed region loads every kernel).  Prints
one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2011_07632_amd/csrc/kernels.hip", "paper_2011_07632_amd/csrc/runtime.cpp",
                  "paper_2011_07632_amd/csrc/h2.cpp"]


def source_hash() -> str:
    """Hash of the sources that determine the product's kernels and launches."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload: str, pass_name: str):
    """HBM bytes per launch of a pass of the product measured with rocprofv3
    counters (profiles/hbm_traffic_<workload>.json, one entry per pass), or
    None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    p = rec.get("passes", {}).get(pass_name)
    if rec.get("source_sha") != source_hash() or p is None:
        return None
    return round(p["fetch_bytes"] + p["write_bytes"], 1)


def h2_sampled_error(P, h2, w, Xg, nrows: int = 200) -> float:
    """Realized accuracy of the H^2 matrix: relative error of the product on a
    random vector over sampled rows, each row of sigma*I + K formed directly."""
    import torch
    if w.kernel == "rpy":
        return None  # rows of the tensor matrix are not formed here
    rng = np.random.default_rng(11)
    x = rng.standard_normal(w.n)
    xg = P.binding.cols_like(w.n, 1, "cuda").copy_(torch.from_numpy(x[:, None]))
    y = P.h2_matvec(h2, xg).cpu().numpy()[:, 0]
    X = Xg.cpu().numpy()
    rows = rng.choice(w.n, size=nrows, replace=False)
    d = np.sqrt(((X[rows, None, :] - X[None, :, :]) ** 2).sum(-1))
    if w.kernel == "matern32":
        t = np.sqrt(3.0) * d / w.ell
        K = (1.0 + t) * np.exp(-t)
    elif w.kernel == "gaussian":
        K = np.exp(-(d / w.ell) ** 2)
    elif w.kernel == "exponential":
        K = np.exp(-d / w.ell)
    else:
        K = 1.0 / np.sqrt(d * d + w.ell * w.ell)
    ref = K @ x + w.shift * x[rows]
    return float(np.linalg.norm(y[rows] - ref) / np.linalg.norm(ref))


def hbm_practical(torch) -> dict:
    """What plain streaming reaches on this GPU, for scale beside the peak: a
    4 GiB FP64 sum (read only) and a 2 GiB device copy (read + write), each
    timed with events over 5 repetitions after a warm-up."""
    x = torch.ones(1 << 29, dtype=torch.float64, device="cuda")
    y = torch.empty(1 << 28, dtype=torch.float64, device="cuda")
    out = {}
    for name, fn, nbytes in (("read_gbs", lambda: x.sum(), x.numel() * 8),
                             ("copy_gbs", lambda: y.copy_(x[: y.numel()]), 2 * y.numel() * 8)):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(5):
            fn()
        b.record()
        b.synchronize()
        out[name] = round(nbytes * 5 / (a.elapsed_time(b) * 1e-3) / 1e9, 1)
    del x, y
    torch.cuda.empty_cache()
    return out


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_facts() -> dict:
    """nproc, CPU model and RAM of the host the CPU baseline ran on."""
    model, ram = "unknown", 0
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    ram = int(line.split()[1]) * 1024
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    return {"nproc": aff, "cpu_model": model, "ram_bytes": ram}


def cpu_baseline(w, n_sample: int, iters_gpu: int, iters_sample: int = 40) -> dict:
    """The CPU oracle, unchanged, on a bounded sample of the workload: the same
    kernel, shift, tolerances and ranks on n_sample points of the same point
    set, run end to end (H^2 build, SPD-HSS build, iters_sample PCG
    iterations), with BLAS on every host core.  The measured times are
    reported as they are; `value` extrapolates them to the full workload
    (SPD-HSS build by N log N, one iteration by N, times the GPU's iteration
    count), so it is an estimate, labelled as such.  Beside it, the oracle is
    timed unscaled, end to end, on the small configuration."""
    from threadpoolctl import threadpool_info
    from oracle.h2 import H2 as OH2
    from oracle.pcg import pcg as opcg
    from oracle.spdhss import SPDHSS as OHSS
    ws = w.with_(n=n_sample)
    X = ws.points()
    t0 = time.perf_counter()
    h = OH2(X, ws.kernel, ws.ell, ws.shift, ws.leaf, ws.h2_tol, eta=ws.eta)
    t_h2 = time.perf_counter() - t0
    om = ws.omega()[h.tree.perm]
    t0 = time.perf_counter()
    s = OHSS(h, om, ws.hss_tol, ws.max_rank, "chol")
    t_build = time.perf_counter() - t0
    b = ws.rhs()[h.tree.perm]
    t0 = time.perf_counter()
    _, it, _ = opcg(h.matvec, s.solve, b, 0.0, iters_sample)
    t_pcg = time.perf_counter() - t0
    t_it = t_pcg / max(int(it.max()), 1)
    scale_n = w.n / n_sample
    build_full = t_build * scale_n * np.log(w.n) / np.log(n_sample)
    solve_full = t_it * scale_n * iters_gpu
    small = oracle_small_end_to_end()
    cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    return {"value": round(build_full + solve_full, 1), "unit": "s", "cores": cores, "kind": "oracle",
            "extrapolated": True,
            "sample": (f"the oracle end to end at N={n_sample} of the same workload: H^2 build "
                       f"{t_h2:.2f} s, SPD-HSS build {t_build:.2f} s, {int(it.max())} PCG iterations of "
                       f"{w.nrhs} columns {t_it * 1e3:.1f} ms each; value = build x (N log N ratio) + "
                       f"iteration x (N ratio) x {iters_gpu} GPU iterations"),
            "sample_n": n_sample, "sample_seconds": round(t_h2 + t_build + t_pcg, 2),
            "sample_build_s": round(t_build, 3), "sample_iteration_s": round(t_it, 4),
            "small_config_end_to_end": small, "host": host_facts()}


def oracle_small_end_to_end() -> dict:
    """The oracle, unchanged and unscaled, on the small configuration
    (workloads.SMALL, N = 2,000): H^2 build, SPD-HSS build and PCG to its
    tolerance, timed end to end."""
    from oracle.h2 import H2 as OH2
    from oracle.pcg import pcg as opcg
    from oracle.spdhss import SPDHSS as OHSS
    w = workloads.SMALL
    t0 = time.perf_counter()
    h = OH2(w.points(), w.kernel, w.ell, w.shift, w.leaf, w.h2_tol, eta=w.eta)
    s = OHSS(h, w.omega()[h.tree.perm], w.hss_tol, w.max_rank, "chol")
    _, it, res = opcg(h.matvec, s.solve, w.rhs()[h.tree.perm], w.pcg_tol, 5000)
    return {"workload": w.name, "n": w.n, "nrhs": w.nrhs, "seconds": round(time.perf_counter() - t0, 3),
            "pcg_iterations": int(np.max(it)), "relres_max": float(np.max(res))}


def run_batch(args, torch, P):
    """Independent instances (N log-uniform in [5k, 50k], three kernels, cube and
    sphere, 4 right-hand sides, FP64 build and FP32 solve operators): all of
    them one at a time (one worker), then concurrently; the results of the two
    runs must agree bit for bit."""
    from paper_2011_07632_amd.binding import cols_like
    dev = "cuda"
    ws = workloads.batch_instances(args.batch)
    reqs = []
    for w in ws:
        reqs.append(dict(points=torch.from_numpy(w.points()).to(dev), kernel=w.kernel, ell=w.ell, shift=w.shift,
                         leaf=w.leaf, tree=w.tree, h2_tol=w.h2_tol, hss_tol=w.hss_tol, max_rank=w.max_rank,
                         oversample=w.oversample, b=cols_like(w.rows, w.nrhs, dev).copy_(torch.from_numpy(w.rhs())),
                         omega=cols_like(w.rows, w.s, dev).copy_(torch.from_numpy(w.omega())),
                         rtol=w.pcg_tol, maxit=5000, precision="f32"))
    P.binding.solve_batch(reqs[:2], workers=2)  # warm-up
    torch.cuda.synchronize()
    runs = {}
    for workers in (1, args.workers):
        t0 = time.perf_counter()
        out = P.binding.solve_batch(reqs, workers=workers)
        torch.cuda.synchronize()
        runs[workers] = (time.perf_counter() - t0, out)
        log(f"[bench] batch of {len(ws)} with {workers} worker(s): {runs[workers][0]:.3f} s")
    t1, o1 = runs[1]
    tw, ow = runs[args.workers]
    same = all(np.array_equal(a["x"].cpu().numpy(), b["x"].cpu().numpy()) and
               a["iters"].tolist() == b["iters"].tolist() for a, b in zip(o1, ow))
    status = {}
    for o in ow:
        status[o["status"]] = status.get(o["status"], 0) + 1
    line = {"metric": "batched SPD-HSS build + PCG solves per second", "value": round(len(ws) / tw, 3),
            "unit": "solves/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64 build, f32 solve operators",
            "data": "synthetic",
            "config": {"workload": f"batch-{len(ws)}-N5k-50k-mixed-kernels", "instances": len(ws),
                       "points_total": int(sum(w.n for w in ws)), "nrhs_each": 4, "leaf": 128,
                       "hss_tol": 1e-2, "pcg_tol": 1e-8, "workers": args.workers},
            "seconds_concurrent": round(tw, 3), "seconds_one_at_a_time": round(t1, 3),
            "speedup": round(t1 / tw, 3), "results_identical": bool(same), "status_counts": status,
            "iterations_max": int(max(int(o["iters"].max()) for o in ow)),
            "relres_max": float(max(float(o["relres"].max()) for o in ow)),
            "seconds_h2_sum": round(sum(o["seconds_h2"] for o in o1), 3),
            "seconds_build_sum": round(sum(o["seconds_build"] for o in o1), 3),
            "seconds_solve_sum": round(sum(o["seconds_solve"] for o in o1), 3),
            "seconds_longest_instance": round(max(o["seconds_h2"] + o["seconds_build"] + o["seconds_solve"]
                                                  for o in o1), 3),
            "instances": [{"name": w.name, "n": w.n, "iters": int(o["iters"].max()),
                           "relres": float(f"{float(o['relres'].max()):.3e}"), "status": o["status"],
                           "seconds": round(o["seconds_h2"] + o["seconds_build"] + o["seconds_solve"], 3)}
                          for w, o in zip(ws, o1)]}
    print(json.dumps(line), flush=True)


def run_serve(args, torch, P):
    """Requests of uneven size, kernel and width arrive with Poisson gaps and
    are submitted to the request loop at their arrival times; latency is
    completion minus arrival."""
    from paper_2011_07632_amd.binding import cols_like
    dev = "cuda"
    trace = workloads.serve_requests(args.serve, n_hi=args.serve_nmax, repeat=args.serve_repeat)
    reqs = []
    for _, w, _ in trace:
        reqs.append(dict(points=torch.from_numpy(w.points()).to(dev), kernel=w.kernel, ell=w.ell,
                         shift=w.shift, leaf=w.leaf, tree=w.tree, h2_tol=w.h2_tol, hss_tol=w.hss_tol,
                         max_rank=w.max_rank,
                         oversample=w.oversample, b=cols_like(w.rows, w.nrhs, dev).copy_(torch.from_numpy(w.rhs())),
                         rtol=w.pcg_tol, maxit=3000, seed=w.seed_base))
    torch.cuda.synchronize()
    S = P.binding.Server(workers=args.workers, hbm_budget_bytes=200 << 30)
    t0 = time.perf_counter()
    tickets = []
    for (arr, w, key), r in zip(trace, reqs):
        dt = arr - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        # every request names its matrix, so a later request on the same
        # matrix solves on the device-resident state
        tickets.append(S.submit(r, key=key))
    done = {}
    phase = {}
    while len(done) < len(tickets):
        for k, t in enumerate(tickets):
            if k in done:
                continue
            p = S.phase(t)
            if p != phase.get(k) and p in ("building", "solving"):
                log(f"[bench] {trace[k][1].name}: {p} at {time.perf_counter() - t0:.1f} s")
            phase[k] = p
            r = S.wait(t, block=False)
            if r is not None:
                done[k] = r
                log(f"[bench] served {len(done)}/{len(tickets)}: {trace[k][1].name} {r['status']} "
                    f"latency {r['seconds_total']:.2f} s (h2 {r['seconds_h2']:.1f} s, build "
                    f"{r['seconds_build']:.1f} s, solve {r['seconds_solve']:.1f} s, "
                    f"{int(r['iters'].max())} iterations)")
        time.sleep(0.05)
    res = [done[k] for k in range(len(tickets))]
    span = time.perf_counter() - t0
    S.close()
    lat = np.array([r["seconds_total"] for r in res])
    status = {}
    for r in res:
        status[r["status"]] = status.get(r["status"], 0) + 1
    ok = [r for r in res if r["status"] == "SPD_OK"]
    line = {"metric": "served p50 latency, s (request loop)", "value": round(float(np.percentile(lat, 50)), 3),
            "unit": "s", "p99_s": round(float(np.percentile(lat, 99)), 3), "higher_is_better": False,
            "solves_per_s": round(len(res) / span, 3), "n_gpus": 1, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"serve-{len(res)}-poisson20-N10k-{args.serve_nmax // 1000}k"
                                   f"-repeat{args.serve_repeat:g}", "requests": len(res),
                       "arrival_rate_per_s": 20.0, "n_range": [10000, args.serve_nmax], "leaf": 400,
                       "repeat_fraction": args.serve_repeat, "workers": args.workers,
                       "hbm_budget_bytes": 200 << 30},
            "seconds_makespan": round(span, 3), "status_counts": status,
            "queued_p50_s": round(float(np.percentile([r["seconds_queued"] for r in res], 50)), 3),
            "relres_max_converged": float(max([float(r["relres"].max()) for r in ok], default=0.0)),
            "reused_state": sum(1 for r in res if r["seconds_h2"] == 0.0 and r["seconds_solve"] > 0.0),
            "requests": [{"name": w.name, "n": w.n, "nrhs": w.nrhs, "key": key, "arrival_s": round(a, 3),
                          "latency_s": round(r["seconds_total"], 3), "queued_s": round(r["seconds_queued"], 3),
                          "h2_s": round(r["seconds_h2"], 3), "build_s": round(r["seconds_build"], 3),
                          "solve_s": round(r["seconds_solve"], 3), "iters": int(r["iters"].max()),
                          "relres": float(r["relres"].max()), "status": r["status"]}
                         for (a, w, key), r in zip(trace, res)]}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default=workloads.HEADLINE.name, choices=list(workloads.BY_NAME))
    ap.add_argument("--maxit", type=int, default=20000)
    ap.add_argument("--cpu-sample", type=int, default=4000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision step")
    ap.add_argument("--mixed", action="store_true",
                    help="run the mixed-precision forms also for 5-16 right-hand sides (three more solves)")
    ap.add_argument("--batch", type=int, default=0, metavar="COUNT",
                    help="batched mode: COUNT independent instances of uneven sizes, run one at a time "
                         "and then concurrently (spd_solve_batch); prints its own JSON line")
    ap.add_argument("--workers", type=int, default=8, help="worker threads of the batched and served modes")
    ap.add_argument("--serve", type=int, default=0, metavar="COUNT",
                    help="served mode: a seeded trace of COUNT requests with Poisson arrivals (20/s) "
                         "through the request loop; prints p50/p99 latency and solves/s")
    ap.add_argument("--serve-nmax", type=int, default=1_000_000,
                    help="largest N of the served trace (log-uniform from 10,000)")
    ap.add_argument("--serve-repeat", type=float, default=0.25,
                    help="fraction of served requests on an earlier request's matrix")
    ap.add_argument("--counters-build", action="store_true",
                    help="build the H^2 matrix, then one SPD-HSS build + ULV factor, and exit (for counter runs)")
    ap.add_argument("--counters", action="store_true",
                    help="counter-collection mode: build the H^2 matrix, run a 2 GiB copy (counter "
                         "calibration) and one product, then exit; run under rocprofv3 --pmc")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2011_07632_amd as P
    from paper_2011_07632_amd.binding import cols_like

    if args.batch:
        run_batch(args, torch, P)
        return
    if args.serve:
        run_serve(args, torch, P)
        return
    w = workloads.BY_NAME[args.workload]
    dev = "cuda"
    X = torch.from_numpy(w.points()).to(dev)
    om = cols_like(w.rows, w.s, dev).copy_(torch.from_numpy(w.omega()))
    b = cols_like(w.rows, w.nrhs, dev).copy_(torch.from_numpy(w.rhs()))
    x = cols_like(w.rows, w.nrhs, dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h2 = P.h2_build(X, w.kernel, w.ell, w.shift, leaf=w.leaf, tol=w.h2_tol, eta=w.eta, tree=w.tree)
    torch.cuda.synchronize()
    t_h2 = time.perf_counter() - t0
    log(f"[bench] {w.name}: h2_build {t_h2:.3f} s, levels {h2.levels}")
    if args.counters:
        # calibration dispatches of known traffic: a fill that writes 2 GiB
        # and a column sum that reads the same 2 GiB (both torch kernels)
        src = torch.ones(1 << 28, dtype=torch.float64, device=dev)   # 2 GiB written
        torch.cuda.synchronize()
        tot = src.view(1 << 14, 1 << 14).sum(dim=0)                   # 2 GiB read
        torch.cuda.synchronize()
        del tot
        P.h2_matvec(h2, b)
        torch.cuda.synchronize()
        log(f"[bench] counters mode done (source {source_hash()})")
        return
    if args.counters_build:
        # one SPD-HSS build and ULV factor (the MFMA-bound phase), for counter runs
        torch.cuda.synchronize()
        hss = P.spdhss_build(h2, w.hss_tol, w.max_rank, w.oversample, omega=om)
        ulv = P.ulv_factor(hss)
        torch.cuda.synchronize()
        log(f"[bench] build counters mode done ({ulv is not None})")
        return

    def step(precision="f64", op="f64"):
        t0 = time.perf_counter()
        hss = P.spdhss_build(h2, w.hss_tol, w.max_rank, w.oversample, omega=om)
        ulv = P.ulv_factor(hss, precision=precision)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, it, res = P.pcg_solve(h2, ulv, b, rtol=w.pcg_tol, maxit=args.maxit, out=x, op_precision=op,
                                 raise_on_nonconvergence=False)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        step.ulv, step.hss = ulv, hss
        return t1 - t0, t2 - t1, it, res

    for i in range(args.warmup):
        tb, ts, it, res = step()
        log(f"[bench] warmup {i}: build {tb:.3f} s solve {ts:.3f} s iterations {int(it.max())}")
    torch.cuda.synchronize()
    builds, solves = [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        tb, ts, it, res = step()
        builds.append(tb)
        solves.append(ts)
        log(f"[bench] step {i}: build {tb:.3f} s solve {ts:.3f} s iterations {int(it.max())} "
            f"relres {float(res.max()):.2e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = 1e3 * wall / args.steps
    ulv64 = step.ulv
    # HSS ranks per tree level (leaves are level 1, as in the paper) and how
    # many nodes reached the rank cap, from the last timed step
    r = step.hss.ranks()
    depth = np.floor(np.log2(np.arange(1, len(r) + 1))).astype(int)
    top = int(depth.max())
    hss_ranks = {"by_level_min_mean_max": {str(top + 1 - d): [int(r[depth == d].min()), round(float(r[depth == d].mean()), 1),
                                                             int(r[depth == d].max())] for d in range(top, 0, -1)},
                 "max_rank": w.max_rank, "rank_cap_hits": int((r[1:] >= w.max_rank).sum()), "nodes": int(len(r) - 1)}
    step.hss = None

    # mixed-precision forms, one step each beside the plain form (not part of
    # `value`): the FP32-block product inside PCG with FP64 residual
    # replacement, FP32 solve operators, and both; each with its error against
    # the FP64 operator it replaces and the true residual reached (FP64 product)
    mixed = None
    if w.nrhs <= 16 and (args.mixed or (w.nrhs <= 4 and not args.no_mixed)):
        v = cols_like(w.rows, 1, dev).copy_(torch.from_numpy(workloads.gaussian_matrix(w.rows, 1, 4242)))
        y64 = P.h2_matvec(h2, v)
        y32 = P.h2_matvec(h2, v, precision="f32")
        pdiff = float(torch.linalg.norm(y32 - y64) / torch.linalg.norm(y64))
        a64 = P.ulv_apply(ulv64, v)
        forms = {}
        for name, pre, op, desc in (
                ("product_f32", "f64", "f32", "FP32 near and coupling blocks in the PCG product (FP64 "
                 "accumulation), FP64 residual replacement; FP64 preconditioner, vectors and dots"),
                ("solve_ops_f32", "f32", "f64", "FP32 solve operators; FP64 product, vectors and dots"),
                ("both_f32", "f32", "f32", "FP32 blocks in the PCG product and FP32 solve operators")):
            tb, ts, itm, resm = step(pre, op)
            a32 = P.ulv_apply(step.ulv, v)
            adiff = float(torch.linalg.norm(a32 - a64) / torch.linalg.norm(a64))
            forms[name] = {"value": round(tb + ts, 4), "build_s": round(tb, 4), "solve_s": round(ts, 4),
                           "pcg_iterations": int(itm.max()), "relres_max": float(resm.max()),
                           "converged": bool(float(resm.max()) <= w.pcg_tol),
                           "precision": desc,
                           "product_rel_diff_vs_f64": float(f"{pdiff:.3e}") if op == "f32" else 0.0,
                           "apply_rel_diff_vs_f64": float(f"{adiff:.3e}")}
            log(f"[bench] mixed {name}: build {tb:.3f} s solve {ts:.3f} s iterations {int(itm.max())} "
                f"relres {float(resm.max()):.2e}")
        # the fastest form that reached the tolerance (equal final accuracy)
        ok = [k for k in forms if forms[k]["converged"]] or list(forms)
        best = min(ok, key=lambda k: forms[k]["value"])
        mixed = {"value": forms[best]["value"], "unit": "s", "form": best,
                 "vs_plain": round(forms[best]["value"] / (wall / args.steps), 4), "forms": forms}

    # dominant kernel of the timed region: the slowest launch of the H^2 product
    # that PCG calls every iteration, timed with HIP events on its stream
    launches = P.binding.product_launch_times(h2, w.nrhs, reps=10)
    dom = max(launches, key=lambda d: d["ms"])
    acc = {}
    for d in launches:
        ms_, by_ = acc.get(d["pass"], (0.0, 0.0))
        acc[d["pass"]] = (ms_ + d["ms"], by_ + d["bytes"])
    passes = {k: {"ms": round(v[0], 4), "gbs": round(v[1] / v[0] / 1e6, 1)} for k, v in acc.items()}
    kern = ("k_symv (symmetric-pair streaming product)" if w.nrhs <= 4 else
            "k_symm16 (symmetric-pair product on FP64 MFMA)" if w.nrhs <= 16 else "k_gemm (MFMA)")
    roofline = {"bound": "hbm", "achieved": round(dom["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dom["gbs"] / HBM_PEAK_GBS, 4),
                "traffic": recorded_traffic(w.name, dom["pass"]),
                "kernel": f"{kern}: {dom['pass']} of h2_matvec",
                "bytes_per_launch": dom["bytes"], "ms_per_launch": round(dom["ms"], 4),
                "product_passes_ms": passes, "practical": hbm_practical(torch)}
    h2_err = h2_sampled_error(P, h2, w, X)
    log(f"[bench] sampled-row error of the H^2 product vs sigma*I + K: {h2_err}")
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_sample, int(it.max()))
    out = {
        "metric": f"SPD-HSS build s + PCG solve s to 1e-8 resid at N={w.n // 1000000}M" if w.n >= 1000000
                  else f"SPD-HSS build s + PCG solve s to 1e-8 resid at N={w.n // 1000}k",
        "value": round(wall / args.steps, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "kernel": w.kernel, "ell": w.ell, "shift": w.shift,
                   "leaf": w.leaf, "h2_tol": w.h2_tol, "hss_tol": w.hss_tol, "max_rank": w.max_rank,
                   "oversample": w.oversample, "nrhs": w.nrhs, "pcg_tol": w.pcg_tol},
        "build_s": round(float(np.mean(builds)), 4),
        "solve_s": round(float(np.mean(solves)), 4),
        "pcg_iterations": int(it.max()),
        "relres_max": float(res.max()),
        "converged": bool(float(res.max()) <= w.pcg_tol and int(it.max()) < args.maxit),
        "h2_build_s": round(t_h2, 3),
        "h2_rel_err_sampled": None if h2_err is None else float(f"{h2_err:.3e}"),
        "hss_ranks": hss_ranks,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "mixed": mixed,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

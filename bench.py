"""Benchmark: DOFs solved per second by PCG + multigrid V-cycle to relative
residual 1e-8 on one MI355X, mixed precision (FP32 inner solves inside FP64
iterative refinement) against the plain FP64 solver, with solve-latency
percentiles, the roofline of the banded stiffness apply and the FP64 oracle
timed on the host.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--precision both|fp64|mixed] [--no-cpu-baseline] [--no-serve]
                    [--profile-steps 3] [--secondary square4x4_p4]
    python bench.py --serve-full [--serve-rate R]     # the full serving recipe instead
    python bench.py --fichera-table 2,3 [--fichera-levels 1,2]   # Fichera iteration counts instead

A step is one complete solve of the workload from u = 0 to ||f - A u|| <= 1e-8
||f|| (setup excluded; inputs resident in HBM).  The default workload is the
64-patch p=5 cube (2.87M free dofs), the largest single-GPU configuration; the
2D 16-patch p=4 square is timed beside it in the `secondary` object.  Prints one JSON line; `value`
is the mixed-precision rate when both precisions run.  The `serving` object
reports continuous-batching throughput and p50/p99 latency over a seeded mix of
resident problems (see paper_1804_02539_amd/serve.py).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "square4x4_p4": "2D Poisson, 4x4 biquadratic patches with seeded interior control points, "
                    "p=4, 64x64 elements per patch, 6 levels, Dirichlet left/bottom, seeded U[-1,1] rhs",
    "cube2x2x2_p3": "3D Poisson, 2x2x2 trilinear patches with the centre vertex seeded-perturbed, "
                    "p=3, 32^3 elements per patch, 6 levels, full Dirichlet, f = 3 pi^2 sin sin sin",
    "square2x2_p2": "2D Poisson, 2x2 identity patches, p=2, 16x16 elements per patch, 4 levels",
    "cube4x4x4_p5": "3D Poisson, 4x4x4 trilinear patches with seeded-perturbed interior vertices, per-slab "
                    "element counts drawn from {8,16,24,32,48} (seed 4; N in [2e6,4e6]), p=5, 4 levels, "
                    "full Dirichlet, seeded U[-1,1] rhs",
}


def make_problem(name):
    from paper_1804_02539_amd import workloads as W
    return {"square4x4_p4": W.square_4x4_bezier, "cube2x2x2_p3": W.cube_2x2x2_trilinear,
            "square2x2_p2": W.unit_square_2x2, "cube4x4x4_p5": W.batched_patch_cube}[name]()


def rhs_for(prob, solver):
    from paper_1804_02539_amd import workloads as W
    src = prob.meta["source"]
    if src[0] == "random":
        return W.random_rhs(solver.N, src[1])
    return solver.load_vector(src[1], src[2])


def kernel_sha():
    """Hash of the banded kernel's source (its section of kernels.hip, from its
    header comment to the smoother section) and of the layout header: counter
    summaries taken on other source are not reported."""
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1804_02539_amd", "csrc", "kernels.hip")) as fh:
        txt = fh.read()
    h.update(txt[txt.index("// banded stiffness apply"):txt.index("// smoother kernels over 2D tensors")].encode())
    with open(os.path.join(ROOT, "paper_1804_02539_amd", "csrc", "layout.hpp"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload, precision):
    """HBM bytes per launch of the finest apply from committed rocprofv3 counter
    summaries, if they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"band_apply_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_sha") != kernel_sha():
        return None
    return t.get(precision, {}).get("hbm_bytes_per_launch")


def _host_cores():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count() or 1


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def traffic_summary(workload, fetch_csv, write_csv, fetch_cmd, write_cmd):
    """HBM bytes per launch of the finest-level banded apply from two
    rocprofv3 --pmc runs of the same bench command with --copy-calibration
    (FETCH_SIZE, then WRITE_SIZE; csv output).  Each counter is scaled by what
    it reads for the 256 MiB device copy of the calibration; the finest level
    is the band launch with the largest grid.  An apply in scatter form is
    its two kernels (k_band_sym_scatter, k_band_sym_reduce), each at its own
    largest grid, summed.  Written beside the kernel source hash, so that
    bench.py reports it only for the kernels measured."""
    import csv
    copy_bytes = 256 << 20

    def read(path, counter):
        rows = []
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") == counter:
                    grid = r.get("Grid_Size", r.get("Grid_Size_X", "0"))
                    rows.append((r["Kernel_Name"], int(grid), float(r["Counter_Value"])))
        # the calibration copy: the copy dispatch whose counter is within a
        # factor of 4 of its size (FETCH_SIZE counts half of it, WRITE_SIZE all)
        copies = [v for n, g, v in rows if "copyBuffer" in n and 0.25 < v * 1024.0 / copy_bytes < 4.0]
        if not copies:
            raise SystemExit(f"{path}: no copy-calibration dispatch")
        out = {"copy_kib": max(copies)}

        def finest(key, typ):
            band = [(g, v) for n, g, v in rows if key in n and typ in n]
            if not band:
                return None
            gmax = max(g for g, _ in band)
            vals = [v for g, v in band if g == gmax]
            return sum(vals) / len(vals), len(vals)

        for prec, key, typ in (("fp64", "k_band_half<", "double"), ("mixed", "k_band_full<", "float")):
            sc, rd = finest("k_band_sym_scatter<", typ), finest("k_band_sym_reduce<", typ)
            if sc and rd:
                out[prec] = (sc[0] + rd[0], sc[1], "k_band_sym_scatter + k_band_sym_reduce")
            elif finest(key, typ):
                out[prec] = finest(key, typ) + (key.rstrip("<"),)
        return out

    fe, wr = read(fetch_csv, "FETCH_SIZE"), read(write_csv, "WRITE_SIZE")
    fs, ws = copy_bytes / (fe["copy_kib"] * 1024.0), copy_bytes / (wr["copy_kib"] * 1024.0)
    res = {"kernel_sha": kernel_sha(),
           "kernel_sha_covers": "the banded kernels' section of kernels.hip and layout.hpp",
           "workload": workload, "copy_bytes": copy_bytes,
           "fetch_copy_kib": fe["copy_kib"], "fetch_scale": fs, "fetch_command": fetch_cmd,
           "write_copy_kib": wr["copy_kib"], "write_scale": ws, "write_command": write_cmd}
    for prec in ("fp64", "mixed"):
        if prec in fe and prec in wr:
            res[prec] = {"kernels": fe[prec][2],
                         "fetch_kib_per_launch": fe[prec][0], "fetch_launches": fe[prec][1],
                         "write_kib_per_launch": wr[prec][0], "write_launches": wr[prec][1],
                         "hbm_bytes_per_launch": 1024.0 * (fe[prec][0] * fs + wr[prec][0] * ws)}
    path = os.path.join(ROOT, "profiles", f"band_apply_{workload}_traffic.json")
    with open(path, "w") as fh:
        json.dump(res, fh, indent=1)
    return res


def cpu_baseline(prob, rhs, min_seconds=10.0, max_solves=50):
    """The oracle's PCG solve of the same workload on the host (setup
    excluded), repeated until about min_seconds of solving have elapsed."""
    from oracle.multigrid import Hierarchy
    cores = _host_cores()
    t0 = time.perf_counter()
    H = Hierarchy(prob)
    t_setup = time.perf_counter() - t0
    solves, it = 0, 0
    t0 = time.perf_counter()
    while True:
        u, it, hist = H.pcg(rhs, tol=1e-8)
        solves += 1
        t = time.perf_counter() - t0
        if t >= min_seconds or solves >= max_solves:
            break
    return {"value": H.finest.N * solves / t, "unit": "DOF/s", "cores": int(cores), "kind": "oracle",
            "cpu_model": _cpu_model(),
            "sample": f"{solves} full PCG solves of the same workload (N={H.finest.N}, {it} iterations each, "
                      f"{t:.1f} s of solving; oracle setup {t_setup:.1f} s excluded)",
            "iterations": it, "solve_s": t / solves}


def cpu_baseline_sampled(prob_replica, iterations_full, n_full, seconds=20.0):
    """The oracle on a bounded sample of a workload too large for it: the
    replica with every element count divided by 4 (same patches, degree,
    geometry and coarsest level).  A number of its PCG iterations is timed
    (about ``seconds`` of CPU work, oracle setup excluded); the rate is then
    scaled to the full workload as N / (iterations_full * t_iter * N / N_rep),
    i.e. it assumes the oracle's time per iteration grows linearly with the
    number of unknowns, and takes the full workload's FP64 iteration count."""
    from oracle.multigrid import Hierarchy
    from paper_1804_02539_amd import workloads as W
    cores = _host_cores()
    t0 = time.perf_counter()
    H = Hierarchy(prob_replica)
    t_setup = time.perf_counter() - t0
    n_rep = H.finest.N
    rhs = W.random_rhs(n_rep, prob_replica.meta["source"][1])
    t0 = time.perf_counter()
    H.finest.apply(H.vcycle(rhs))
    t_one = time.perf_counter() - t0
    k = int(max(2, min(40, seconds / max(t_one, 1e-3))))
    t0 = time.perf_counter()
    _, it, hist = H.pcg(rhs, tol=1e-8, maxit=k)
    t = time.perf_counter() - t0
    t_iter = t / max(it, 1)
    value = n_rep / (iterations_full * t_iter)
    return {"value": value, "unit": "DOF/s", "cores": int(cores), "kind": "oracle", "cpu_model": _cpu_model(),
            "sample": f"{it} PCG iterations of the oracle on the replica with element counts / 4 "
                      f"(N_rep={n_rep}, {t:.1f} s, {t_iter:.2f} s per iteration; oracle setup {t_setup:.1f} s "
                      f"excluded), scaled to the full workload (N={n_full}) as linear time per unknown and "
                      f"{iterations_full} iterations (the GPU FP64 solve's count)",
            "replica_n_free": int(n_rep), "replica_s_per_iteration": t_iter, "replica_iterations_run": int(it),
            "replica_rel_residual_after_sample": float(hist[-1])}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run(workload, prob, precision, steps, warmup, dev, fd_mfma=0, profile_steps=3, persistent=0):
    import torch
    from paper_1804_02539_amd import igamg
    opts = igamg.default_options(precision=igamg.MIXED if precision == "mixed" else igamg.FP64, fd_mfma=fd_mfma,
                                 persistent=persistent)
    t0 = time.perf_counter()
    S = igamg.Solver(prob, opts, device=dev)
    setup_s = time.perf_counter() - t0
    log(f"{workload} {precision}{' fd_mfma' if fd_mfma else ''}{' persistent' if persistent else ''}: "
        f"setup {setup_s:.1f} s, N = {S.N}")
    f = torch.as_tensor(rhs_for(prob, S), device=dev)
    u = torch.empty_like(f)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        S.solve(f, tol=1e-8, u=u)
    # timed pass: the product path (each PCG iteration replayed as HIP graphs)
    lat, iters = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(steps):
        t1 = time.perf_counter()
        _, info = S.solve(f, tol=1e-8, u=u, stream=stream)
        lat.append(time.perf_counter() - t1)
        iters.append((info.iterations, info.outer_iterations))
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    log(f"  timed pass: {1e3 * total / steps:.2f} ms/solve")
    # second timed pass of the same solves with a HIP event pair around every
    # banded-apply launch (direct launches: HIP does not time events in graphs)
    S.profile(True)
    torch.cuda.synchronize()
    t_p = time.perf_counter()
    psteps = max(1, min(profile_steps, steps))
    for _ in range(psteps):
        S.solve(f, tol=1e-8, u=u, stream=stream)
    torch.cuda.synchronize()
    total_prof = time.perf_counter() - t_p
    S.profile(False)
    log(f"  profiled pass: {1e3 * total_prof / psteps:.2f} ms/solve")
    cnt, ms, by = S.profile_read()
    nl = prob.levels
    Lf = nl - 1
    # dominant banded kernel: FP32 finest level for mixed, FP64 finest otherwise
    k = Lf + nl if precision == "mixed" else Lf
    avg_ms = ms[k] / max(cnt[k], 1)
    bytes_launch = by[k] / max(cnt[k], 1)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    res = {
        "value": S.N * steps / total,
        "ms_per_step": 1e3 * total / steps,
        "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                       "p99": 1e3 * float(np.percentile(lat, 99)),
                       "mean": 1e3 * float(np.mean(lat))},
        "iterations": int(np.median([i for i, _ in iters])),
        "refinements": int(np.median([o for _, o in iters])),
        "final_rel_residual": info.rel_residual,
        "converged": bool(info.converged),
        "smoother_variant_finest": igamg.FD_NAMES[S.tuning(-1, precision == "mixed")],
        "setup_s": setup_s,
        "roofline": {"bound": "hbm",
                     "kernel": (("finest-level FP32 banded residual/apply (inner solves)" if precision == "mixed"
                                 else "finest-level FP64 banded residual/apply")
                                + (": k_band_sym_scatter + k_band_sym_reduce (half band, scatter form)"
                                   if S.band_form(-1) == igamg.BAND_SCATTER else
                                   ": k_band_full (full FP32 band)" if precision == "mixed"
                                   else ": k_band_half (half band, gather form)")),
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_from_profiles(workload, precision),
                     "avg_launch_us": 1e3 * avg_ms,
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "launches_per_step": float(cnt[k]) / psteps,
                     "band_ms_per_step_fp64_all_levels": float(ms[:nl].sum()) / psteps,
                     "band_ms_per_step_fp32_all_levels": float(ms[nl:].sum()) / psteps,
                     "measured_over": f"a second timed pass of {psteps} of the same solves, direct launches, "
                                      f"each banded launch timed by HIP events attached to its dispatch "
                                      f"({1e3 * total_prof / psteps:.2f} ms/solve)"},
    }
    return S, res


def copy_bandwidth(dev, nbytes=2 << 30, reps=5):
    """Measured device-to-device copy rate (bytes read plus written per
    second) of a 2 GiB buffer, median of a few copies timed by HIP events: the
    practical streaming ceiling beside the published HBM peak."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    x.fill_(1.0)
    y = torch.empty_like(x)
    y.copy_(x)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * nbytes / float(np.median(ts)) / 1e9


def serving(precision, n_requests, n_families, seed, dev):
    """Continuous-batching serving of a seeded request mix: first every request
    at once with the hierarchies resident (saturated throughput), then the same
    number of fresh requests arriving as a Poisson process at 0.7x that rate
    (latency percentiles).  Setup runs once, before both timed phases."""
    import torch
    from paper_1804_02539_amd import igamg, serve
    opts = igamg.default_options(precision=igamg.MIXED if precision == "mixed" else igamg.FP64)
    free, total = torch.cuda.mem_get_info()
    budget = int(0.75 * free)
    S = serve.Server(budget, opts=opts, device=dev, handles_per_key=2, keep_results=False)
    fams, _ = serve.request_mix(0, seed=seed, n_families=n_families)
    warm = [serve.Request(f, lambda n: np.ones(n)) for f in fams for _ in range(2)]
    t0 = time.perf_counter()
    S.run([(0.0, r) for r in warm])              # builds two resident hierarchies per family
    setup_s = time.perf_counter() - t0
    burst = serve.requests_for(fams, n_requests, seed + 100)
    S.finished.clear()
    S.steps = 0
    t_sat = S.run([(0.0, r) for r in burst])
    sat = S.stats(t_sat)
    rate = 0.7 * sat["requests_per_s"]
    pois = serve.requests_for(fams, n_requests, seed + 200)
    S.finished.clear()
    S.steps = 0
    offs = serve.poisson_offsets(n_requests, rate, seed=seed)
    t_p = S.run([(float(o), r) for o, r in zip(offs, pois)])
    lat = S.stats(t_p)
    S.close()
    sizes = sorted(f_n for f_n in {r.n for r in burst + pois})
    return {"requests": n_requests, "families": n_families, "precision": precision,
            "family_sizes_free_dofs": [int(sizes[0]), int(sizes[-1])],
            "hbm_budget_bytes": budget, "resident_bytes": S.used, "setup_s": setup_s,
            "saturated": {"requests_per_s": sat["requests_per_s"], "dofs_per_s": sat["dofs_per_s"],
                          "makespan_s": sat["makespan_s"], "steps": sat["steps"],
                          "latency_ms": sat["latency_ms"]},
            "poisson": {"arrival_rate_per_s": rate, "requests_per_s": lat["requests_per_s"],
                        "dofs_per_s": lat["dofs_per_s"], "latency_ms": lat["latency_ms"],
                        "steps": lat["steps"], "failed": lat["failed"] + sat["failed"]},
            "description": "seeded mix of 2D/3D multi-patch problems, p in 2..6, N log-uniform in "
                           "[1e4, 3e5] free dofs per family, fresh U[-1,1] rhs per request"}


def serving_full(n_requests, n_families, rate, seed, dev, precision="mixed", workers=2):
    """The full serving recipe: ``n_requests`` seeded requests over
    ``n_families`` problem families (2D with 4-16 patches, 3D with 8-64, p in
    2..6, N log-uniform in [1e4, 4e6]) arriving as a Poisson process at
    ``rate`` per second into a cold server.  Every hierarchy is set up inside
    the served time (device assembly, on two worker threads), under an HBM
    budget of 80% of the free device memory; idle hierarchies are evicted
    least recently used first when a new one does not fit."""
    import torch
    from paper_1804_02539_amd import igamg, serve
    opts = igamg.default_options(precision=igamg.MIXED if precision == "mixed" else igamg.FP64)
    fams, reqs = serve.request_mix(n_requests, seed=seed, n_families=n_families, n_min=1e4, n_max=4e6,
                                   band_bytes_max=60e9, n0_max=8000)
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    ws = [igamg.workspace_size(f, opts) for f in fams]
    log(f"serve-full: {n_families} families, workspaces {min(ws) / 1e6:.0f} MB .. {max(ws) / 1e9:.1f} GB "
        f"(sum {sum(ws) / 1e9:.0f} GB), budget {budget / 1e9:.0f} GB, {n_requests} requests at {rate}/s")
    S = serve.Server(budget, opts=opts, device=dev, handles_per_key=1, setup_workers=workers, keep_results=False)
    offs = serve.poisson_offsets(n_requests, rate, seed=seed)

    def progress(srv, t):
        log(f"serve-full: {t:.0f} s, {len(srv.finished)} done, {len(srv.pending)} waiting, "
            f"{len(srv.setups)} setting up, {len(srv.running)} running, {srv.used / 1e9:.0f} GB held")

    t = S.run([(float(o), r) for o, r in zip(offs, reqs)], timeout=1000.0, progress=progress)
    S.close()
    st = S.stats(t)
    n = np.array(sorted(r.n for r in S.finished))
    lat = np.array([r.latency for r in S.finished])
    big = lat[np.array([r.n for r in S.finished]) >= 1e6]
    setups = sum(1 for e in S.events if e[1] == "resident")
    out = {"requests": n_requests, "families": n_families, "precision": precision, "arrival_rate_per_s": rate,
           "setup_workers": workers,
           "finished": st["requests"], "rejected": st["rejected"], "failed": st["failed"],
           "free_dofs": {"min": int(n[0]), "median": int(np.median(n)), "max": int(n[-1]),
                         "requests_over_1e6": int((n >= 1e6).sum())},
           "hbm_budget_bytes": budget, "peak_held_bytes": S.peak_used, "setups": setups,
           "evictions": st["evictions"], "makespan_s": t, "requests_per_s": st["requests_per_s"],
           "dofs_per_s": st["dofs_per_s"], "latency_ms": st["latency_ms"],
           "rejections": sorted({str(r.error)[:160] for r in S.rejected}),
           "setup_errors": [e[2][:160] for e in S.events if e[1] == "setup_error"],
           "latency_ms_over_1e6_dofs": {"p50": 1e3 * float(np.percentile(big, 50)),
                                        "p99": 1e3 * float(np.percentile(big, 99))} if len(big) else None,
           "description": "cold server: latency = arrival to solution, including queueing, setup (when the "
                          "family is not resident) and the solve to 1e-8"}
    log(f"serve-full: {st['requests']} finished in {t:.1f} s, {st['requests_per_s']:.2f} req/s, "
        f"p50 {st['latency_ms']['p50']:.0f} ms, p99 {st['latency_ms']['p99']:.0f} ms, {setups} setups, "
        f"{st['evictions']} evictions")
    return {"serving_full": out}


# readings of the smoother's constants, as options on top of the library's
# default (omega = 1, K + sigma M on S1)
READINGS = {
    "library": {},
    "s1_K": {"s1_sigma": 0},
    "omega_mean": {"geometry_scaling": 1},
    "omega_mean_s1_K": {"geometry_scaling": 1, "s1_sigma": 0},
    "mult": {"iface_multiplicity": 1},
    "direct": {"iface_direct": 1},
    "physh": {"physical_h": 1},
}


def fichera_table(degrees, levels, dev, reading="library"):
    """FP64 PCG iteration counts on the Fichera corner with K=448 patches
    (Sec. 5: 7 unit cubes split into 4^3 patches each, 1 element per patch on
    the coarsest level, f = 75 pi^2 sin 5 pi x sin 5 pi y sin 5 pi z), beside
    the counts the paper prints for the same cases."""
    import torch
    from paper_1804_02539_amd import igamg, workloads as W
    with open(os.path.join(ROOT, "tests", "golden", "iteration_counts.json")) as fh:
        paper = json.load(fh)["fichera_K448"]
    rows = []
    for p in degrees:
        for lev in levels:
            prob = W.fichera(p, lev + 1, split=4)
            t0 = time.perf_counter()
            S = igamg.Solver(prob, igamg.default_options(**READINGS[reading]), device=dev)
            setup = time.perf_counter() - t0
            f = torch.as_tensor(S.load_vector(75.0 * np.pi ** 2, 5.0), device=dev)
            u, info = S.solve(f, tol=1e-8)
            ref = paper.get(str(lev), {}).get(str(p))
            rows.append({"p": p, "level": lev, "reading": reading, "N": S.N, "N0": int(S.num_dofs(0)[0]),
                         "iterations": info.iterations, "paper": ref, "converged": bool(info.converged),
                         "rel_residual": info.rel_residual, "setup_s": round(setup, 1),
                         "solve_ms": round(info.solve_ms, 1)})
            log(f"fichera {reading} p={p} l={lev}: N={S.N}, {info.iterations} it (paper {ref}), setup {setup:.1f} s, "
                f"solve {info.solve_ms:.0f} ms")
            del S, u, f
            torch.cuda.empty_cache()
    return {"fichera_K448": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cube4x4x4_p5", choices=sorted(WORKLOADS))
    ap.add_argument("--profile-steps", type=int, default=3,
                    help="solves in the second, per-launch timed pass (roofline)")
    ap.add_argument("--secondary", default="square4x4_p4",
                    help="comma-separated workloads also timed (FP64 and mixed) in a secondary object; '' for none")
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-full", action="store_true",
                    help="instead of the benchmark line, run the full serving recipe (cold server, 256 requests, "
                         "1e4..4e6 dofs, Poisson arrivals) and print its statistics")
    ap.add_argument("--serve-full-requests", type=int, default=256)
    ap.add_argument("--serve-full-families", type=int, default=64)
    ap.add_argument("--serve-rate", type=float, default=2.0, help="arrivals per second for --serve-full")
    ap.add_argument("--serve-workers", type=int, default=2, help="setup worker threads for --serve-full")
    ap.add_argument("--fichera-table", default="",
                    help="instead of the benchmark line, print FP64 iteration counts on the Fichera corner "
                         "(K=448) for these degrees, e.g. 2,3,4, on the levels --fichera-levels")
    ap.add_argument("--fichera-levels", default="1,2,3,4")
    ap.add_argument("--fichera-readings", default="library",
                    help="comma-separated readings of the smoother constants for --fichera-table: "
                         + ", ".join(READINGS))
    ap.add_argument("--fd-mfma", action="store_true",
                    help="also time the mixed solver with the smoother's mode products on the matrix cores, with "
                         "FP32 operands (fd_mfma = 1) and with bfloat16 operands (fd_mfma = 3)")
    ap.add_argument("--persistent", action="store_true",
                    help="also time every solve with the persistent coarse cycle (options.persistent = 1)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first fill and copy a 256 MiB buffer: dispatches of known size against "
                         "which hardware byte counters are scaled")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="instead of the benchmark line, write profiles/band_apply_<workload>_traffic.json from the "
                         "counter_collection.csv files of two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE)")
    ap.add_argument("--traffic-commands", nargs=2, default=["", ""], metavar=("FETCH_CMD", "WRITE_CMD"),
                    help="the two rocprofv3 commands, recorded in the summary")
    ap.add_argument("--serve-requests", type=int, default=96)
    ap.add_argument("--serve-families", type=int, default=12)
    a = ap.parse_args()
    if a.traffic_summary:
        print(json.dumps(traffic_summary(a.workload, a.traffic_summary[0], a.traffic_summary[1],
                                         a.traffic_commands[0], a.traffic_commands[1])))
        return
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(sharding patches across GPUs is described, not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch  # noqa: F401

    dev = "cuda:0"
    if a.serve_full:
        print(json.dumps(serving_full(a.serve_full_requests, a.serve_full_families, a.serve_rate, 21, dev,
                                      workers=a.serve_workers)), flush=True)
        return
    if a.fichera_table:
        degrees = [int(x) for x in a.fichera_table.split(",")]
        levels = [int(x) for x in a.fichera_levels.split(",")]
        out = {"fichera_K448": []}
        for rd in a.fichera_readings.split(","):
            out["fichera_K448"] += fichera_table(degrees, levels, dev, rd)["fichera_K448"]
        print(json.dumps(out), flush=True)
        return
    if a.copy_calibration:
        x = torch.empty(64 << 20, dtype=torch.float32, device=dev)
        x.fill_(1.0)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    prob = make_problem(a.workload)
    runs = {}
    if a.precision in ("both", "fp64"):
        S, runs["fp64"] = run(a.workload, prob, "fp64", a.steps, a.warmup, dev, profile_steps=a.profile_steps)
        N_free, N_local = S.N, S.N_local
        rhs_cpu = rhs_for(prob, S)
        del S
        torch.cuda.empty_cache()
        if a.persistent:
            _, runs["fp64_persistent"] = run(a.workload, prob, "fp64", a.steps, a.warmup, dev, persistent=1,
                                             profile_steps=a.profile_steps)
    if a.precision in ("both", "mixed"):
        S, runs["mixed"] = run(a.workload, prob, "mixed", a.steps, a.warmup, dev, profile_steps=a.profile_steps)
        N_free, N_local = S.N, S.N_local
        if a.fd_mfma:
            _, runs["mixed_fd_mfma"] = run(a.workload, prob, "mixed", a.steps, a.warmup, dev, fd_mfma=1,
                                           profile_steps=a.profile_steps)
            _, runs["mixed_fd_bf16"] = run(a.workload, prob, "mixed", a.steps, a.warmup, dev, fd_mfma=3,
                                           profile_steps=a.profile_steps)
        if a.persistent:
            _, runs["mixed_persistent"] = run(a.workload, prob, "mixed", a.steps, a.warmup, dev, persistent=1,
                                              profile_steps=a.profile_steps)
        rhs_cpu = rhs_for(prob, S)
        del S
        torch.cuda.empty_cache()
    head = "mixed" if ("mixed" in runs and runs["mixed"]["converged"]) else "fp64"
    h = runs[head]
    out = {
        "metric": "DOFs solved/s to rel. residual 1e-8",
        "value": h["value"],
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 inner / f64 refinement" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "description": WORKLOADS[a.workload],
                   "n_free_dofs": N_free, "n_local_dofs": N_local, "degree": prob.degree,
                   "patches": prob.npatch, "levels": prob.levels, "precision": head,
                   "solver": "PCG, one V-cycle (1+1 smoothing, tau=0.25, sigma=5/h^2) per iteration"},
        "latency_ms": h["latency_ms"],
        "iterations": h["iterations"],
        "final_rel_residual": h["final_rel_residual"],
        "roofline": dict(h["roofline"]),
    }
    if not a.copy_calibration:    # a counter run keeps its copies to the calibration
        cbw = copy_bandwidth(dev)
        out["roofline"]["copy_GBps_measured"] = cbw
        out["roofline"]["frac_of_measured_copy"] = out["roofline"]["achieved"] / cbw
    for k, v in runs.items():
        out[k] = {kk: vv for kk, vv in v.items() if kk != "roofline"}
        out[k]["band_roofline_frac"] = v["roofline"]["frac"]
        out[k]["band_avg_launch_us"] = v["roofline"]["avg_launch_us"]
        out[k]["band_bytes_per_launch"] = v["roofline"]["algorithmic_bytes_per_launch"]
        out[k]["band_traffic_bytes_per_launch"] = v["roofline"]["traffic"]
    if "fp64" in runs and "mixed" in runs:
        out["speedup_mixed_vs_fp64"] = runs["mixed"]["value"] / runs["fp64"]["value"]
    if "mixed_fd_mfma" in runs and "mixed" in runs:
        out["mixed_fd_mfma_vs_default"] = runs["mixed_fd_mfma"]["value"] / runs["mixed"]["value"]
        out["mixed_fd_bf16_vs_default"] = runs["mixed_fd_bf16"]["value"] / runs["mixed"]["value"]
    for prec in ("fp64", "mixed"):
        if f"{prec}_persistent" in runs and prec in runs:
            out[f"{prec}_persistent_vs_default"] = runs[f"{prec}_persistent"]["value"] / runs[prec]["value"]
    secondary = {}
    for wname in [w for w in a.secondary.split(",") if w and w != a.workload]:
        sprob = make_problem(wname)
        srun = {}
        for prec in ("fp64", "mixed"):
            Ss, r = run(wname, sprob, prec, a.steps, a.warmup, dev, profile_steps=a.profile_steps)
            srun[prec] = {kk: vv for kk, vv in r.items() if kk != "roofline"}
            srun[prec]["n_free_dofs"] = Ss.N
            srun[prec]["band_roofline_frac"] = r["roofline"]["frac"]
            srun[prec]["band_avg_launch_us"] = r["roofline"]["avg_launch_us"]
            del Ss
        srun["speedup_mixed_vs_fp64"] = srun["mixed"]["value"] / srun["fp64"]["value"]
        srun["description"] = WORKLOADS[wname]
        secondary[wname] = srun
    if secondary:
        out["secondary"] = secondary
    if not a.no_serve:
        log("serving")
        out["serving"] = serving("mixed" if head == "mixed" else "fp64", a.serve_requests,
                                 a.serve_families, 5, dev)
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle)")
        if a.workload == "cube4x4x4_p5":
            from paper_1804_02539_amd import workloads as W
            it_full = runs["fp64"]["iterations"] if "fp64" in runs else h["iterations"]
            out["cpu_baseline"] = cpu_baseline_sampled(W.batched_patch_cube(divide=4), it_full, N_free)
        else:
            out["cpu_baseline"] = cpu_baseline(prob, rhs_cpu)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

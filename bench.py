#!/usr/bin/env python3
"""Sorted-sequence SKR throughput on one MI355X.

Workload (seeded, synthetic; stands in for the paper's Darcy dataset): 2-D Darcy
-div(a grad u) = 1 on the unit square, 256 x 256 interior grid (n = 65,536, 326,656 nnz CSR FP64),
5-point harmonic-mean finite differences, a = exp(GRF) with spectral density (9 + |k|^2)^-2,
400 systems. One step = the whole hot path on that batch: greedy nearest-neighbour sort of the
400 parameter fields (Alg. 1) and GCRO-DR(60, 20) along the sorted chain (Alg. 2), every system to
relative residual 1e-8, inputs resident in HBM before the timed region.

Printed: one JSON line with systems/s (converged systems only), the roofline of the dominant
Arnoldi-step kernel (sampled hipEvent timings inside the timed region), GMRES(60) on the same GPU
for a prefix of the sorted chain, SpMV bandwidth, and the CPU oracle timed on a bounded sample.

Secondary modes, each printing its own JSON line:
--dim 3     3-D Darcy on a 128^3 grid (n = 2,097,152; 7-point operator, CSR or matrix-free), 8 systems
            by default, GCRO-DR(80, 20). Its working set (basis about 1.7 GB) is far beyond the 256 MB
            Infinity Cache, so its kernel rates are HBM rates. No oracle sample.
--mixed     FP32-stored basis and recycle space, FP64 arithmetic and refinement (any mode).
--chains C  the sorted order split into C contiguous chains solved concurrently.
--serve     Darcy systems of several grid sizes arriving one at a time (Poisson) through the serving
            runtime: capacity, throughput and latency.
--advdiff   time-stepping advection-diffusion chains (512^2, 64 chains x 32 backward-Euler steps).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_m_traffic_darcy256.txt")
STEP_SOURCES = [os.path.join(ROOT, "paper_2401_09516_amd", "csrc", f) for f in ("skr_solver.hip", "skr_internal.hpp")]


def step_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the dominant step kernel (k_step_m, the merged kernel of the two-kernel
    Arnoldi step at this size) from the committed FETCH_SIZE / WRITE_SIZE summary, or None when
    the summary is missing or was taken on a different version of the step-kernel source."""
    try:
        kv = dict(ln.split(":", 1) for ln in open(TRAFFIC_FILE) if ":" in ln and not ln.startswith("#"))
    except OSError:
        return None
    if kv.get("source_sha256", "").strip() != step_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--systems", type=int, default=None, help="default 400 in 2-D, 8 in 3-D")
    ap.add_argument("--dim", type=int, choices=[2, 3], default=2,
                    help="2: the 2-D Darcy workload; 3: 3-D Darcy on a grid^3 mesh (7-point), a secondary mode")
    ap.add_argument("--grid", type=int, default=None, help="grid side (default 256 in 2-D, 128 in 3-D)")
    ap.add_argument("--m", type=int, default=None, help="default 60 in 2-D, 80 in 3-D")
    ap.add_argument("--k", type=int, default=20)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=40000)
    ap.add_argument("--matrix", choices=["csr", "stencil"], default="csr")
    ap.add_argument("--mixed", action="store_true",
                    help="FP32-stored Arnoldi vectors and recycle space, FP64 arithmetic and residuals, "
                         "one refinement step per cycle (SKR_FLAG_MIXED)")
    ap.add_argument("--chains", type=int, default=1,
                    help="split the sorted order into this many contiguous chains, solved concurrently on "
                         "their own contexts and streams (the sorted-partition parallel scheme, App. E)")
    ap.add_argument("--chains-form", choices=["batched", "streams"], default="batched",
                    help="--chains C > 1: all chains in lockstep through skr_solve_chains, one call per round "
                         "of systems (default), or one host thread and stream per chain")
    ap.add_argument("--gmres-systems", type=int, default=40, help="prefix of the sorted chain solved by GMRES(m)")
    ap.add_argument("--cpu-systems", type=int, default=8, help="oracle sample: first systems of the sorted chain")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the untimed identity-order solve of the same systems (the sort ablation)")
    ap.add_argument("--spmv-grid", type=int, default=4096,
                    help="grid of the SpMV bandwidth cases whose working sets exceed the 256 MB Infinity Cache")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="untimed: one pass of the hot path over --systems systems, then a device copy of "
                         "--copy-mib MiB (the reference kernel that scales hardware byte counters); for "
                         "rocprofv3 --pmc runs")
    ap.add_argument("--copy-mib", type=int, default=512)
    ap.add_argument("--serve", action="store_true",
                    help="serving mode: Darcy systems of several grid sizes arrive one at a time (Poisson) and "
                         "are admitted by skr_submit into nearest chains; prints throughput and latency")
    ap.add_argument("--serve-sizes", default="64,128,256,512,1024")
    ap.add_argument("--serve-systems", type=int, default=30, help="systems submitted per run (sizes round-robin)")
    ap.add_argument("--serve-load", type=float, default=0.7, help="arrival rate as a fraction of the measured capacity")
    ap.add_argument("--serve-sweep", default="0.3,0.5,0.9,1.2",
                    help="further arrival rates (fractions of the capacity) swept after the main Poisson run; "
                         "empty for none")
    ap.add_argument("--serve-workers", type=int, default=4)
    ap.add_argument("--serve-chains", type=int, default=8)
    ap.add_argument("--serve-chain-cap", type=int, default=0,
                    help="systems a chain takes before a new chain of the same shape is started (0: no limit)")
    ap.add_argument("--advdiff", action="store_true",
                    help="time-stepping mode: unsteady advection-diffusion, --chains chains of --steps-per-chain "
                         "backward-Euler steps on a --grid^2 mesh, each chain solved as a chain of the serving runtime")
    ap.add_argument("--steps-per-chain", type=int, default=32)
    ap.add_argument("--advdiff-form", choices=["both", "batched", "serve"], default="both",
                    help="--advdiff: all chains in lockstep (skr_solve_chains, one call per time step), the "
                         "serving runtime (one submission per step and chain), or both")
    a = ap.parse_args()
    if a.grid is None:
        a.grid = 256 if a.dim == 2 else 128
    if a.systems is None:
        a.systems = 400 if a.dim == 2 else 8
    if a.m is None:
        a.m = 60 if a.dim == 2 else 80
    if a.dim == 3:
        a.spmv_grid = 0          # the 3-D matrix at the config grid is already the HBM-sized case
    return a


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def serve_bench(a):
    """Continuous batching: capacity from a saturation run (every system submitted at once), then
    a Poisson arrival run at --serve-load times that capacity, then the rates of --serve-sweep.
    Latency = completion - submission."""
    import threading

    import numpy as np
    import torch

    from paper_2401_09516_amd import skr
    from workloads import darcy_sequence
    from workloads.device import upload_systems

    skr.load_library()
    sizes = [int(v) for v in a.serve_sizes.split(",")]
    per = -(-a.serve_systems // len(sizes))
    pool = []
    for N in sizes:
        t = time.perf_counter()
        for s_ in darcy_sequence(N, per, first_seed=1000 * N):
            pool.append(s_)
        log(f"generated {per} systems of {N}x{N} in {time.perf_counter() - t:.1f}s")
    rng = np.random.default_rng(2401)
    order = [int(i) for i in rng.permutation(len(pool))[:a.serve_systems]]
    ops, bs, xs = upload_systems(pool, "cuda:0", a.matrix)
    params = [torch.from_numpy(np.ascontiguousarray(s_.a.ravel())).cuda() for s_ in pool]
    mode = skr.SKR_FLAG_MIXED if a.mixed else 0

    def run(gaps):
        ctx = skr.skr_ctx_create(0, torch.cuda.current_stream().cuda_stream)
        skr.skr_serve_start(ctx, max_chains=a.serve_chains, workers=a.serve_workers,
                            max_chain_systems=a.serve_chain_cap)
        sub, done, res, tickets = {}, {}, {}, {}
        lock = threading.Lock()
        finished = threading.Event()

        def poller():
            while True:
                with lock:
                    pending = [(i, t) for i, t in tickets.items() if i not in done]
                    all_sent = len(tickets) == len(order)
                for i, t in pending:
                    r = skr.skr_poll(ctx, t)
                    if r is not None:
                        with lock:
                            done[i] = time.perf_counter()
                            res[i] = r
                if all_sent and not pending:
                    finished.set()
                    return
                time.sleep(0.0005)
        th = threading.Thread(target=poller)
        t0 = time.perf_counter()
        th.start()
        nxt = t0
        for q, i in enumerate(order):
            nxt += gaps[q]
            while time.perf_counter() < nxt:
                time.sleep(min(0.001, max(0.0, nxt - time.perf_counter())))
            ts = time.perf_counter()
            t = skr.skr_submit(ctx, ops[i], params[i], params[i].numel(), bs[i], xs[i], m=a.m, k=a.k, rtol=a.rtol,
                               maxit=a.maxit, flags=mode)
            with lock:
                sub[i], tickets[i] = ts, t
        finished.wait()
        th.join()
        wall = max(done.values()) - t0
        stats = skr.skr_serve_stats_get(ctx)
        skr.skr_serve_stop(ctx)
        skr.skr_ctx_destroy(ctx)
        lat = {i: done[i] - sub[i] for i in order}
        return wall, lat, res, stats

    log("saturation run (capacity)")
    wall_sat, _, res_sat, st_sat = run([0.0] * len(order))
    capacity = len(order) / wall_sat
    lam = a.serve_load * capacity
    gaps = list(np.random.default_rng(2402).exponential(1.0 / lam, len(order)))
    log(f"capacity {capacity:.2f} systems/s; Poisson run at {lam:.2f} systems/s")
    wall, lat, res, st = run(gaps)
    conv = sum(r["status"] in (skr.SKR_CONVERGED, skr.SKR_BREAKDOWN) for r in res.values())
    L = np.array([lat[i] for i in order]) * 1e3
    by_size = {}
    for N in sizes:
        idx = [i for i in order if pool[i].N_g == N]
        if idx:
            v = np.array([lat[i] for i in idx]) * 1e3
            by_size[str(N)] = dict(systems=len(idx), p50_ms=round(float(np.percentile(v, 50)), 1),
                                   p99_ms=round(float(np.percentile(v, 99)), 1),
                                   iters_mean=float(np.mean([res[i]["iters"] for i in idx])))
    out = {
        "metric": "serving: systems/s and latency, Poisson arrivals of Darcy systems of mixed grid sizes",
        "value": round(conv / wall, 3), "unit": "systems/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"darcy2d-serving-{'-'.join(map(str, sizes))}-{len(order)}sys-gcrodr({a.m},{a.k})"
                               + ("-fp32basis" if a.mixed else ""),
                   "sizes": sizes, "systems": len(order), "m": a.m, "k": a.k, "rtol": a.rtol,
                   "workers": a.serve_workers, "max_chains": a.serve_chains,
                   "max_chain_systems": a.serve_chain_cap, "load": a.serve_load},
        "capacity_systems_per_s": round(capacity, 3), "arrival_rate": round(lam, 3),
        "latency_ms": {"p50": round(float(np.percentile(L, 50)), 1), "p99": round(float(np.percentile(L, 99)), 1),
                       "max": round(float(L.max()), 1)},
        "latency_by_size": by_size, "converged": conv,
        "max_relres": max(r["relres_true"] for r in res.values()),
        "chains": {"created": st["chains_created"], "retired": st["chains_retired"]},
        "saturation_wall_s": round(wall_sat, 2), "poisson_wall_s": round(wall, 2),
    }
    sweep = []
    for f in [float(v) for v in a.serve_sweep.split(",") if v.strip()]:
        rate = f * capacity
        g = list(np.random.default_rng(2403).exponential(1.0 / rate, len(order)))
        log(f"sweep: Poisson run at {f:.2f} x capacity ({rate:.2f} systems/s)")
        w_, lat_, res_, _ = run(g)
        L_ = np.array([lat_[i] for i in order]) * 1e3
        c_ = sum(r["status"] in (skr.SKR_CONVERGED, skr.SKR_BREAKDOWN) for r in res_.values())
        sweep.append(dict(load=f, arrival_rate=round(rate, 3), throughput=round(c_ / w_, 3), converged=c_,
                          p50_ms=round(float(np.percentile(L_, 50)), 1), p99_ms=round(float(np.percentile(L_, 99)), 1)))
    if sweep:
        out["rate_sweep"] = sweep
    print(json.dumps(out), flush=True)


def advdiff_bench(a):
    """Backward-Euler chains A x^{t+1} = x^t / dt in two forms. Batched: one skr_solve_chains call
    per time step advances every chain by one step in lockstep (each launch covers all chains; the
    recycle spaces stay on the context between calls). Serving: one host thread per chain submits
    each step when the previous one is done; the serving runtime keeps each chain's recycle space
    resident and runs up to --serve-workers chains at once on their own streams."""
    import threading

    import numpy as np
    import torch

    from paper_2401_09516_amd import skr
    from workloads.advdiff import advdiff_chains
    from workloads.device import upload_systems

    skr.load_library()
    N, C, T = a.grid, a.chains, a.steps_per_chain
    t = time.perf_counter()
    chains = advdiff_chains(N, C, first_seed=0)
    log(f"generated {C} chains of {N}x{N} in {time.perf_counter() - t:.1f}s")
    ops, _, _ = upload_systems(chains, "cuda:0")
    params = [torch.from_numpy(c.params).cuda() for c in chains]
    x0 = [torch.from_numpy(c.x0).cuda() for c in chains]
    torch.cuda.synchronize()          # the chain threads read these on their own streams
    mode = skr.SKR_FLAG_MIXED if a.mixed else 0

    def run(nch, nsteps, k):
        ctx = skr.skr_ctx_create(0, torch.cuda.current_stream().cuda_stream)
        skr.skr_serve_start(ctx, max_chains=max(nch, 1), workers=a.serve_workers, split_d2_rel=1e-12)
        res = [[None] * nsteps for _ in range(nch)]
        errs = []

        def chain_loop(c):
            try:
                st = torch.cuda.Stream()
                with torch.cuda.stream(st):
                    xa = torch.empty_like(x0[c])
                    xb = torch.empty_like(x0[c])
                    b = torch.empty_like(x0[c])
                    prev = x0[c]
                    for q in range(nsteps):
                        torch.div(prev, chains[c].dt, out=b)
                        st.synchronize()
                        x = xa if q % 2 == 0 else xb
                        tk = skr.skr_submit(ctx, ops[c], params[c], params[c].numel(), b, x, m=a.m, k=k,
                                            rtol=a.rtol, maxit=a.maxit, flags=mode)
                        res[c][q] = skr.skr_wait(ctx, tk)
                        prev = x
            except BaseException as e:     # re-raised in the calling thread
                errs.append(e)
        th = [threading.Thread(target=chain_loop, args=(c,)) for c in range(nch)]
        t0 = time.perf_counter()
        for x_ in th:
            x_.start()
        for x_ in th:
            x_.join()
        wall = time.perf_counter() - t0
        stats = skr.skr_serve_stats_get(ctx)
        skr.skr_serve_stop(ctx)
        skr.skr_ctx_destroy(ctx)
        if errs:
            raise errs[0]
        flat = [r for rc in res for r in rc]
        conv = sum(r["status"] in (skr.SKR_CONVERGED, skr.SKR_BREAKDOWN) for r in flat)
        return dict(wall=wall, value=conv / wall, converged=conv, solves=len(flat),
                    iters_mean=float(np.mean([r["iters"] for r in flat])),
                    iters_first=float(np.mean([rc[0]["iters"] for rc in res])),
                    iters_later=float(np.mean([r["iters"] for rc in res for r in rc[1:]])) if nsteps > 1 else None,
                    max_relres=max(r["relres_true"] for r in flat), chains=stats["chains_created"])

    def run_batched(nch, nsteps, k):
        ctx = skr.skr_ctx_create(0, torch.cuda.current_stream().cuda_stream)
        bufs = [[torch.empty_like(x0[c]) for _ in range(3)] for c in range(nch)]   # b, x (two, alternating)
        prev = [x0[c] for c in range(nch)]
        starts = list(range(nch + 1))
        res = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for q in range(nsteps):
            bs, xs = [], []
            for c in range(nch):
                torch.div(prev[c], chains[c].dt, out=bufs[c][0])
                bs.append(bufs[c][0])
                xs.append(bufs[c][1 + q % 2])
            rc, r = skr.skr_solve_chains(ctx, starts, ops[:nch], bs, xs, None, m=a.m, k=k, rtol=a.rtol,
                                         maxit=a.maxit, flags=mode | (skr.SKR_FLAG_CONTINUE if q else 0))
            res.append(r)
            prev = xs
            log(f"  batched time step {q} of {nch} chains done")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        skr.skr_ctx_destroy(ctx)
        flat = [x for r in res for x in r]
        conv = sum(r_["status"] in (skr.SKR_CONVERGED, skr.SKR_BREAKDOWN) for r_ in flat)
        return dict(wall=wall, value=conv / wall, converged=conv, solves=len(flat),
                    iters_mean=float(np.mean([r_["iters"] for r_ in flat])),
                    iters_first=float(np.mean([r_["iters"] for r_ in res[0]])),
                    iters_later=float(np.mean([r_["iters"] for r in res[1:] for r_ in r])) if nsteps > 1 else None,
                    max_relres=max(r_["relres_true"] for r_ in flat), chains=nch)

    forms = ["batched", "serve"] if a.advdiff_form == "both" else [a.advdiff_form]
    runner = {"batched": run_batched, "serve": run}
    sub_c, sub_t = min(C, 8), min(T, 8)
    results = {}
    for f in forms:
        log(f"[{f}] warm-up")
        runner[f](min(C, 4), 2, a.k)
        log(f"[{f}] timed run: {C} chains x {T} steps")
        main = runner[f](C, T, a.k)
        log(f"[{f}] {main['value']:.1f} systems/s; GMRES(m) and GCRO-DR on {sub_c} chains x {sub_t} steps")
        g = runner[f](sub_c, sub_t, 0)
        s_ = runner[f](sub_c, sub_t, a.k)
        results[f] = dict(run=main, subset={"chains": sub_c, "steps": sub_t, "gmres": g, "gcrodr": s_,
                                            "speedup_vs_gmres": round(s_["value"] / g["value"], 2)
                                            if g["value"] > 0 else None})
    head = forms[0]
    out = {
        "metric": "systems/s of backward-Euler advection-diffusion chains (GCRO-DR recycling along each chain)",
        "value": round(results[head]["run"]["value"], 3), "unit": "systems/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"advdiff2d-{N}x{N}-{C}chains-x{T}steps-gcrodr({a.m},{a.k})"
                               + ("-fp32basis" if a.mixed else ""),
                   "grid": N, "n": N * N, "chains": C, "steps": T, "dt": chains[0].dt, "m": a.m, "k": a.k,
                   "rtol": a.rtol, "form": head, "workers": a.serve_workers},
        "run": results[head]["run"], "subset": results[head]["subset"],
    }
    if len(forms) > 1:
        other = forms[1]
        out[other] = results[other]
        out[f"{head}_over_{other}"] = round(results[head]["run"]["value"] / results[other]["run"]["value"], 3)
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.serve and a.gpus == 1:
        serve_bench(a)
        return
    if a.advdiff and a.gpus == 1:
        if a.grid is None or a.grid == 256 and "--grid" not in sys.argv:
            a.grid = 512
        if "--chains" not in sys.argv:
            a.chains = 64
        advdiff_bench(a)
        return
    if a.gpus != 1:
        print(f"bench.py: --gpus {a.gpus} is not supported: the benchmark measures one GPU. Sorted chains "
              "would shard across GPUs without communication (contiguous slices of the sorted order).",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2401_09516_amd import skr
    from workloads import darcy3d_system, darcy_sequence, darcy_system, param_matrix
    from workloads.device import upload_systems

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    skr.load_library()
    dev = "cuda:0"
    t = time.perf_counter()
    if a.dim == 2:
        systems = darcy_sequence(a.grid, a.systems)
    else:
        systems = []
        for i in range(a.systems):
            systems.append(darcy3d_system(a.grid, i, with_csr=(a.matrix == "csr")))
            log(f"generated 3-D system {i}")
    P = param_matrix(systems)
    log(f"generated {a.systems} systems of n={systems[0].n} in {time.perf_counter() - t:.1f}s")
    Pd = torch.from_numpy(P).to(dev)
    ops, bs, xs = upload_systems(systems, dev, a.matrix)
    G = a.grid
    nnz = 5 * G * G - 4 * G if a.dim == 2 else 7 * G ** 3 - 6 * G * G     # nonzeros of the assembled operator
    stream = torch.cuda.current_stream()
    ctx = skr.skr_ctx_create(0, stream.cuda_stream)
    N, p = P.shape
    mode = skr.SKR_FLAG_MIXED if a.mixed else 0

    if a.pmc_probe:
        order, _ = skr.skr_sort(ctx, Pd, N, p, 0, want_dist=False)
        rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, order, m=a.m, k=a.k, rtol=a.rtol, maxit=a.maxit,
                                         flags=skr.SKR_FLAG_PROFILE | mode)
        torch.cuda.synchronize()
        sa = skr.skr_profile_get(ctx)["kernels"]["step_a"]
        nb = a.copy_mib << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        skr.skr_ctx_destroy(ctx)
        print(json.dumps({"pmc_probe": True, "systems": a.systems, "iters": [r["iters"] for r in res],
                          "first_step_kernel_algorithmic_bytes_per_launch": sa["bytes"] / max(sa["launches"], 1),
                          "copy_bytes_read": nb, "copy_bytes_written": nb, "copies": 3,
                          "step_source_sha256": step_source_hash()}), flush=True)
        return

    C = max(1, min(a.chains, N))
    streams = [stream] + [torch.cuda.Stream() for _ in range(C - 1)]
    ctxs = [ctx] + [skr.skr_ctx_create(0, st.cuda_stream) for st in streams[1:]]

    def solve_chains(order, flags):
        if C == 1:
            return skr.skr_solve_sequence(ctx, ops, bs, xs, order, m=a.m, k=a.k, rtol=a.rtol, maxit=a.maxit,
                                          flags=flags | mode)
        slices = [[int(i) for i in sl] for sl in np.array_split(np.asarray(order), C)]
        if a.chains_form == "batched":
            # round t gives every chain its t-th system; the chains carry their recycle spaces from
            # round to round (SKR_FLAG_CONTINUE), which solves each chain as one uninterrupted call would
            res = [None] * N
            rc = 0
            for t_ in range(max(len(sl) for sl in slices)):
                idx = [sl[t_] for sl in slices if t_ < len(sl)]
                starts = np.concatenate([[0], np.cumsum([1 if t_ < len(sl) else 0 for sl in slices])])
                rc_, r = skr.skr_solve_chains(ctx, starts, [ops[i] for i in idx], [bs[i] for i in idx],
                                              [xs[i] for i in idx], None, m=a.m, k=a.k, rtol=a.rtol,
                                              maxit=a.maxit, flags=flags | mode | (skr.SKR_FLAG_CONTINUE if t_ else 0))
                rc = max(rc, rc_)
                for i, r_ in zip(idx, r):
                    res[i] = r_
                if a.dim == 3:
                    log(f"  round {t_}: {len(idx)} systems done")
            return rc, res
        import threading
        out = [None] * C

        def run(c):
            try:
                sl = slices[c]
                out[c] = skr.skr_solve_sequence(ctxs[c], [ops[i] for i in sl], [bs[i] for i in sl],
                                                [xs[i] for i in sl], None, m=a.m, k=a.k, rtol=a.rtol,
                                                maxit=a.maxit, flags=flags | mode)
            except BaseException as e:   # re-raised in the calling thread
                out[c] = e
        th = [threading.Thread(target=run, args=(c,)) for c in range(C)]
        for t_ in th:
            t_.start()
        for t_ in th:
            t_.join()
        res = [None] * N
        rc = 0
        for c in range(C):
            if isinstance(out[c], BaseException):
                raise out[c]
            rc = max(rc, out[c][0])
            for i, r in zip(slices[c], out[c][1]):
                res[i] = r
        return rc, res

    def step(flags):
        order, _ = skr.skr_sort(ctx, Pd, N, p, 0, want_dist=False)
        rc, res = solve_chains(order, flags)
        return order, rc, res

    for w in range(a.warmup):
        t = time.perf_counter()
        step(0)
        log(f"warmup step {w}: {time.perf_counter() - t:.2f}s")
    for c_ in ctxs:
        skr.skr_profile_reset(c_)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_ in range(a.steps):
        order, rc, res = step(skr.SKR_FLAG_PROFILE)
        log(f"timed step {s_} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    converged = sum(r["status"] in (skr.SKR_CONVERGED, skr.SKR_BREAKDOWN) for r in res)
    maxit_hits = sum(r["status"] == skr.SKR_MAXIT for r in res)
    value = a.steps * converged / elapsed
    iters = [r["iters"] for r in res]
    secs = np.array([r["seconds"] for r in res]) * 1e3
    per_system_ms = dict(p50=round(float(np.percentile(secs, 50)), 2), p99=round(float(np.percentile(secs, 99)), 2),
                         max=round(float(secs.max()), 2), first=round(float(secs[int(order[0])]), 2)) if len(secs) else None
    prof = skr.skr_profile_get(ctx)
    kern = {}
    for name, kst in prof["kernels"].items():
        if kst["launches"]:
            avg_ms = kst["ms"] / kst["launches"]
            kern[name] = dict(launches_timed=kst["launches"], avg_us=1e3 * avg_ms,
                              avg_bytes=kst["bytes"] / kst["launches"],
                              gbs=kst["bytes"] / (kst["ms"] * 1e-3) / 1e9)
    dom = max(kern, key=lambda k_: kern[k_]["avg_us"]) if kern else None
    # FP64 basis on at most 256 workgroups: two kernels per step, the first the merged kernel k_step_m
    # (pass A only at step 0 of a cycle); otherwise passes A, B and C
    merged = (not a.mixed) and (systems[0].n + 255) // 256 <= 256
    kernel_names = {"step_a": "k_step_m" if merged else "k_step_a", "step_b": "k_step_b", "step_c": "k_step_c"}
    roofline = None
    if dom:
        ach = kern[dom]["gbs"]
        traffic = (measured_traffic() if dom == "step_a" and merged and a.dim == 2 and G == 256 else None)
        basis_bytes = (a.k + a.m + 1) * systems[0].n * (4 if a.mixed else 8)
        roofline = dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(ach / HBM_PEAK_GBS, 4),
                        traffic=round(traffic) if traffic is not None else None, kernel=kernel_names[dom],
                        avg_us=round(kern[dom]["avg_us"], 2), bytes_per_launch=round(kern[dom]["avg_bytes"]),
                        working_set_bytes=basis_bytes,
                        memory_level="the basis fits the 256 MB Infinity Cache: memory-bound kernel fed "
                                     "partly from that cache, priced against the HBM peak"
                        if basis_bytes <= (256 << 20) else "HBM (basis beyond the 256 MB Infinity Cache)")
    # the sort ablation (Sec. 4.1): the same systems as one chain in their original order, untimed by
    # the bench line; the library call is the same, only the order differs
    ablation = None
    if not a.no_ablation and a.dim == 2 and C == 1:
        torch.cuda.synchronize()
        ta = time.perf_counter()
        rci, resi = skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=a.m, k=a.k, rtol=a.rtol, maxit=a.maxit,
                                           flags=mode)
        torch.cuda.synchronize()
        ta = time.perf_counter() - ta
        convi = sum(r["status"] in (skr.SKR_CONVERGED, skr.SKR_BREAKDOWN) for r in resi)
        ablation = dict(order="identity (unsorted)", value=round(convi / ta, 3), unit="systems/s", converged=convi,
                        iters_total=int(np.sum([r["iters"] for r in resi])),
                        iters_total_sorted=int(np.sum(iters)),
                        iters_ratio_unsorted_over_sorted=round(float(np.sum([r["iters"] for r in resi]))
                                                               / max(1, int(np.sum(iters))), 4))
        log(f"ablation: identity order {ablation['value']} systems/s, iterations x{ablation['iters_ratio_unsorted_over_sorted']}")

    # timing of the sort alone
    torch.cuda.synchronize()
    ts = time.perf_counter()
    skr.skr_sort(ctx, Pd, N, p, 0, want_dist=False)
    sort_ms = 1e3 * (time.perf_counter() - ts)

    # GMRES(m) on the same GPU, prefix of the sorted chain
    g = a.gmres_systems
    gmres = None
    if g > 0:
        pre = [int(i) for i in order[:g]]
        gops = [ops[i] for i in pre]
        gbs = [bs[i] for i in pre]
        gxs = [torch.zeros_like(bs[i]) for i in pre]
        torch.cuda.synchronize()
        tg = time.perf_counter()
        rcg, resg = skr.skr_solve_sequence(ctx, gops, gbs, gxs, None, m=a.m, k=0, rtol=a.rtol, maxit=a.maxit,
                                           flags=mode)
        torch.cuda.synchronize()
        tg = time.perf_counter() - tg
        gconv = sum(r["status"] == skr.SKR_CONVERGED for r in resg)
        gmres = dict(value=round(gconv / tg, 3), unit="systems/s", systems=g, converged=gconv,
                     iters_mean=float(np.mean([r["iters"] for r in resg])),
                     sample="first systems of the sorted chain, GMRES(m) = same library call with k = 0")
        skr_prefix_iters = float(np.mean([res[i]["iters"] for i in pre]))
        gmres["skr_iters_mean_same_systems"] = skr_prefix_iters

    # SpMV bandwidth. 2-D: the config matrix (fits the 256 MB Infinity Cache) and a > 256 MB matrix.
    # 3-D: the 7-point operator at the config grid, matrix-free and CSR.
    def spmv_bytes(kind, dim, G_, nnz_):
        n_ = G_ ** dim
        if kind == "csr":
            return 12.0 * nnz_ + 4.0 * (n_ + 1) + 16.0 * n_
        return 8.0 * dim * G_ ** (dim - 1) * (G_ + 1) + 16.0 * n_

    def time_spmv(op, n_, reps):
        xd = torch.rand(n_, dtype=torch.float64, device=dev)
        yd = torch.empty_like(xd)
        return skr.skr_spmv_repeat(ctx, op, xd, yd, reps)

    # A rate is labelled an HBM rate (frac_hbm) only when the working set exceeds the 256 MB Infinity
    # Cache; repeated launches on a smaller operator are served partly by that cache (effective rates).
    MALL_BYTES = 256 << 20

    def spmv_entry(ms_, byt_):
        e = dict(us=round(1e3 * ms_, 2), gbs=round(byt_ / (ms_ * 1e-3) / 1e9, 1), bytes=byt_)
        if byt_ > MALL_BYTES:
            e["frac_hbm"] = round(byt_ / (ms_ * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)
        else:
            e["note"] = ("working set under the 256 MB Infinity Cache, repeated launches on one operator: "
                         "an effective rate, not an HBM rate")
        return e

    spmv = {}
    n0 = systems[0].n
    ms = time_spmv(ops[0], n0, 200 if a.dim == 2 else 50)
    spmv[f"{a.matrix}{'' if a.dim == 2 else '7'}_{G}"] = spmv_entry(ms, spmv_bytes(a.matrix, a.dim, G, nnz))
    if a.dim == 3:
        other = "stencil" if a.matrix == "csr" else "csr"
        from workloads.darcy3d import darcy3d_from_nodes
        s0 = darcy3d_from_nodes(systems[0].a, with_csr=(other == "csr"))
        oops, _, _ = upload_systems([s0], dev, other)
        ms = time_spmv(oops[0], n0, 50)
        spmv[f"{other}7_{G}"] = spmv_entry(ms, spmv_bytes(other, 3, G, nnz))
        del oops, s0
    if a.spmv_grid:
        big = darcy_system(a.spmv_grid, 999)
        bn, bnnz = big.n, int(big.A.nnz)
        for kind in ("csr", "stencil"):
            bops, _, _ = upload_systems([big], dev, kind)
            ms = time_spmv(bops[0], bn, 20)
            spmv[f"{kind}_{a.spmv_grid}"] = spmv_entry(ms, spmv_bytes(kind, 2, a.spmv_grid, bnnz))
            del bops
        del big
    # the practical ceiling: a plain device copy of 512 MiB (read + write) in the same process
    src = torch.ones((512 << 20) // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    cms = e0.elapsed_time(e1) / 10
    spmv["copy_512MiB"] = dict(us=round(1e3 * cms, 1), gbs=round(2 * (512 << 20) / (cms * 1e-3) / 1e9, 1),
                               frac_hbm=round(2 * (512 << 20) / (cms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3),
                               note="torch device copy, bytes read + written: the practical HBM ceiling")
    del src, dst
    for c_ in ctxs:
        skr.skr_ctx_destroy(c_)

    cpu = None
    if not a.no_cpu and a.cpu_systems > 0 and a.dim == 2:
        import oracle
        try:
            from threadpoolctl import threadpool_info
            cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
        except Exception:
            cores = len(os.sched_getaffinity(0))
        pre = [int(i) for i in order[:a.cpu_systems]]
        tc = time.perf_counter()
        ref = oracle.solve_sequence([systems[i].A for i in pre], [systems[i].b for i in pre], None,
                                    a.m, a.k, a.rtol, a.maxit, basis_fp32=a.mixed)
        tc = time.perf_counter() - tc
        cpu = dict(value=round(len(pre) / tc, 4), unit="systems/s", cores=int(cores), kind="oracle",
                   sample=f"first {len(pre)} systems of the sorted chain (the first starts without a recycle "
                          f"space), {tc:.1f} s; oracle iterations {[r.iters for r in ref]}",
                   extrapolated_s_for_all=round(tc / len(pre) * N, 1),
                   extrapolation=f"per-system mean of the sample x {N} systems (an extrapolation, not a run)")

    out = {
        "metric": "systems/sec to rel-res 1e-8, SKR vs plain GMRES on 1 GPU; SpMV HBM GB/s",
        "value": round(value, 3),
        "unit": "systems/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(1e3 * elapsed / a.steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"darcy2d-{G}x{G}" if a.dim == 2 else f"darcy3d-{G}x{G}x{G}")
                               + f"-{a.systems}sys-sorted-gcrodr({a.m},{a.k})-{a.matrix}"
                               + ("-fp32basis" if a.mixed else "")
                               + (f"-{C}chains" if C > 1 else ""),
                   "dim": a.dim, "grid": a.grid, "n": systems[0].n, "nnz": nnz, "systems": a.systems, "m": a.m, "k": a.k,
                   "rtol": a.rtol, "matrix": a.matrix, "chains": C,
                   "basis_storage": "fp32 (FP64 arithmetic and refinement)" if a.mixed else "fp64",
                   "parallelism": "single chain" if C == 1 else (
                       f"{C} contiguous chains of the sorted order advanced in lockstep (skr_solve_chains: one "
                       "launch per kernel covers every chain)" if a.chains_form == "batched" else
                       f"{C} contiguous chains of the sorted order, one host thread and stream each")},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "converged": converged,
        "maxit_hits": maxit_hits,
        "per_system_ms": per_system_ms,
        "iters_mean": float(np.mean(iters)),
        "iters_total": int(np.sum(iters)),
        "sort_ms": round(sort_ms, 2),
        "gmres": gmres,
        "speedup_vs_gmres": round(value / gmres["value"], 2) if gmres and gmres["value"] > 0 else None,
        # the paper's own figures, on CPUs and other workloads: context, not a target
        "paper_context": {
            "darcy_skr_vs_gmres_tol1e-8": {"time_x": 2.70, "iterations_x": 19.1, "n": 6400,
                                           "hardware": "dual Intel Xeon Gold 6154, 72 MPI ranks, PETSc",
                                           "source": "Table 1"},
            "headline_up_to": {"time_x": 13.9, "iterations_x": 30.0,
                               "workload": "Helmholtz n = 10^4, ASM preconditioner, tol 1e-7",
                               "hardware": "dual Intel Xeon Gold 6154, 72 MPI ranks, PETSc",
                               "source": "abstract, Table 1"}},
        "sort_ablation": ablation,
        "kernels": kern,
        "arnoldi_steps_profiled": prof["steps"],
        "arnoldi_step_bytes_total": prof["step_bytes"],
        "spmv": spmv,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

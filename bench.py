"""Throughput benchmark: solved degrees of freedom per second to a 1e-8
relative residual for the shifted-HSS Helmholtz solver on one MI355X.

One step = one complete helm_solve (outer FP64 FGMRES, shifted-HSS
preconditioner with ceil(k) HSS steps, each inner solve a fixed number of
V(2,2) cycles chosen from the measured cycle rate, all right-hand sides)
with the load vectors already resident in HBM.

Headline workload (`value`): the largest one-GPU configuration, 3D Q1 on a
256^3 hexahedral mesh (N = 257^3 = 16,974,593 nodes), k = 40, delta = 0,
delta_hat = k, 6 multigrid levels, one Gaussian source (sigma 0.03) at a
seeded uniform centre, plain complex FP64 on the GPU.  The same mesh is
solved with FP32 multigrid and FP64 outer iteration (`fp32_mg`, with the
FP64/FP32-MG DoF/s ratio), and the 2D P1 configurations 64^2 (k = 10),
1024^2 (k = 100, four right-hand sides) and 2048^2 (k = 200) are reported
in `workloads`, each in both precision modes with its error against the
oracle's direct solve (64^2 in process; 1024^2 and 2048^2 in CPU worker
processes that run beside the GPU work).

--steps and --warmup are caps: the run plans its solves against a
wall-clock budget (--budget-s, measured from process start, default 450 s)
and reports the number of headline solves it actually warmed up and timed.
At least one full warm-up solve and one timed solve always run.

Prints ONE JSON line on stdout; progress goes to stderr.
"""

import argparse
import hashlib
import re
import json
import os
import platform
import subprocess
import sys
import time

T_PROC0 = time.time()

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "solved DOFs/s to 1e-8 rel residual (FP32-MG vs FP64), %HBM peak; p50/p99 latency"
PROFILES = os.path.join(ROOT, "profiles")
HEADLINE = "q1-256-k40"


def log(*a):
    print("[%6.1fs]" % (time.time() - T_PROC0), *a, file=sys.stderr, flush=True)


def elapsed():
    return time.time() - T_PROC0


# The dominant kernel of each mesh dimension and the source files its
# counter record depends on.  2D: the finest-level prolongation, four Jacobi
# sweeps (cycle q's post-smoothing and cycle q+1's pre-smoothing) and the
# residual restriction in one register-streaming pass.  3D: the
# finest-level prolongation and the post-smoothing Jacobi sweep(s) of one
# z-marching pass (one sweep in FP64, two in FP32; the cycles before the
# last of each HSS step).
DOMINANT = {
    2: {"tag": "k_stream_sweeps4", "sources": ("kernels2d_stream.hip", "helm_common.h", "stencil_rows.h"),
        "desc": "finest-level prolongation + four Jacobi sweeps + residual restriction "
                "(k_stream_sweeps<S=4>); x, b, e_c read, x', b_c written"},
    3: {"tag": "k3_pass_prolong", "sources": ("kernels3d_fused.hip", "helm_common.h", "launch.h"),
        "desc": "finest-level prolongation + Jacobi sweep(s) in one z-marching pass "
                "(k3_pass<F_JAC, stages, prolong>: one sweep in FP64, two in FP32); "
                "x, b, e_c read, x' written: 3.125 S N"},
}


def code_tokens(text):
    """Source text without comments and with whitespace runs collapsed, so
    that an edit of a comment does not count as a change of the kernel."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(dim):
    h = hashlib.sha256()
    for f in DOMINANT[dim]["sources"]:
        with open(os.path.join(ROOT, "paper_2506_18694_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(code_tokens(fh.read()).encode())
    return h.hexdigest()[:16]


def stored_traffic(dim, workload, precision):
    """HBM traffic per launch of the dominant kernel from committed rocprofv3
    counter runs (FETCH_SIZE and WRITE_SIZE, copy-calibrated); null when the
    kernel source changed since they were taken."""
    path = os.path.join(PROFILES, "traffic_%s_%s_%s.json" % (DOMINANT[dim]["tag"], workload, precision))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_hash") != kernel_source_hash(dim):
        return None
    return rec.get("bytes_per_launch")


def host_info():
    """Core count and CPU model of the host the CPU baseline runs on."""
    model = platform.processor() or "unknown"
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except Exception:
        affinity = os.cpu_count()
    return {"nproc": affinity, "cpu_count": os.cpu_count(), "cpu_model": model}


def make_solver(W, name, precision, **kw):
    from paper_2506_18694_amd import Solver
    w = W.WORKLOADS[name]
    return Solver(w["dim"], w["n"], w["levels"], w["k"], w["delta"], w["delta_hat"],
                  precision=precision, **kw)


def measure(W, name, precision, warmup_max, steps_max, tol, deadline_fn=None, full_warmup=True,
            streaming=True, split=False, keep_x=False):
    """Warm up and time complete solves of one workload on one handle.

    full_warmup: the first warm-up is a complete solve (its time estimates
    a step); otherwise the warm-up is one preconditioner application on the
    same handle and workspace (it measures the cycle rate and the segment
    heights that the timed solve then reuses).  deadline_fn(t_solve) returns
    how many more solves of t_solve seconds fit the budget."""
    import torch
    s = make_solver(W, name, precision, profile=True, streaming=streaming, split=split)
    f = torch.from_numpy(W.workload_sources(name)).cuda().contiguous()
    b = s.load_nodal(f)
    x = torch.empty_like(b)
    ws = s.workspace(b.shape[0])
    log("[bench] %s %s: N=%d nrhs=%d workspace %.1f GB" % (name, precision, s.N, b.shape[0],
                                                           ws.numel() / 1e9))
    t_est = None
    warm = 0
    if full_warmup:
        _, st = s.solve(b, x, tol=tol, workspace=ws)
        warm = 1
        t_est = st["solve_ms"] / 1e3
        log("[bench] warmup 0: %.1f ms, outer its %d, true rel res %.2e"
            % (st["solve_ms"], st["outer_its"], st["true_rel_residual"]))
    else:
        _ = s.precondition(b)
        torch.cuda.synchronize()
        log("[bench] warmup: one preconditioner application")
    steps = steps_max
    if deadline_fn is not None and t_est is not None:
        fit = deadline_fn(t_est)
        steps = max(1, min(steps_max, fit))
        extra = max(0, min(warmup_max - warm, fit - steps))
        for i in range(extra):
            _, st = s.solve(b, x, tol=tol, workspace=ws)
            warm += 1
            log("[bench] warmup %d: %.1f ms" % (warm - 1, st["solve_ms"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(steps):
        _, st = s.solve(b, x, tol=tol, workspace=ws)
        stats.append(st)
        log("[bench] step %d: %.1f ms, outer its %d, true rel res %.2e"
            % (i, st["solve_ms"], st["outer_its"], st["true_rel_residual"]))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ok = all(st["converged"] == 1 and st["true_rel_residual"] <= tol for st in stats)
    xh = x.cpu().numpy() if keep_x else None
    N, nrhs = s.N, b.shape[0]
    s.close()
    s._ws.clear()
    del ws, b, x, s
    torch.cuda.empty_cache()
    ms = el / steps * 1e3
    last = stats[-1]
    return dict(N=N, nrhs=nrhs, elapsed=el, steps=steps, warmup=warm, stats=stats, ok=ok,
                ms=ms, value=N * nrhs / (ms / 1e3), x=xh,
                summary={"value": N * nrhs / (ms / 1e3), "ms_per_step": ms, "steps": steps,
                         "warmup": warm if full_warmup else "one preconditioner application",
                         "outer_its": max(st["outer_its"] for st in stats),
                         "mg_cycles": last["mg_cycles"], "hss_steps": last["hss_steps"],
                         "vcycle_rate": last["vcycle_rate"],
                         "true_rel_residual": max(st["true_rel_residual"] for st in stats),
                         "converged": ok})


def roofline(dim, name, precision, stats):
    """HBM roofline of the dominant kernel from the HIP-event timings that
    the timed solves took of its launches (every tenth HSS step)."""
    sw_ms = sum(st["sweep_ms"] for st in stats)
    sw_n = sum(st["sweep_launches"] for st in stats)
    sw_b = sum(st["sweep_bytes"] for st in stats)
    achieved = sw_b / (sw_ms / 1e3) / 1e9 if sw_ms > 0 else None
    per_launch = sw_b / sw_n if sw_n else None
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": stored_traffic(dim, name, precision),
            "kernel": DOMINANT[dim]["desc"], "bytes_per_launch": per_launch,
            "avg_launch_us": sw_ms / sw_n * 1e3 if sw_n else None, "launches_timed": sw_n}


# ---------------------------------------------------------------- oracle side --
def _oracle_direct_worker(name, out_path, threads):
    """CPU worker: the oracle's direct solves B_0 u = b of a workload's
    right-hand sides (sparse LU), saved for the error of the GPU solves.
    Its BLAS threads are capped (set before numpy loads): with every
    worker's threads plus the GPU process's on the same cores, spinning BLAS
    threads slowed the factorisation by more than ten times."""
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = str(threads)
    import numpy as np
    from oracle import solver as osolver
    import workloads as W
    log("[oracle worker %s] started" % name)
    w = W.WORKLOADS[name]
    pr = osolver.Problem(w["dim"], w["n"], w["k"], w["delta_hat"], levels=1)
    log("[oracle worker %s] assembled" % name)
    f = W.workload_sources(name)
    U = np.stack([pr.solve_direct((pr.M @ fi).astype(np.complex128)) for fi in f])
    np.save(out_path + ".tmp.npy", U)
    os.replace(out_path + ".tmp.npy", out_path)
    log("[oracle worker %s] direct solves done" % name)


def start_oracle_worker(name, tmpdir, threads=4):
    import multiprocessing as mp
    out = os.path.join(tmpdir, "oracle_%s.npy" % name)
    if os.path.exists(out):
        os.remove(out)
    p = mp.get_context("spawn").Process(target=_oracle_direct_worker, args=(name, out, threads),
                                        daemon=True)
    p.start()
    return p, out


def oracle_error(x, u):
    """Relative l2 error of each column of x against the oracle's u (max)."""
    import numpy as np
    return float(max(np.linalg.norm(xi - ui) / np.linalg.norm(ui) for xi, ui in zip(x, u)))


def _baseline_column_worker(args):
    """One right-hand side's oracle HSS steps, timed (CPU worker)."""
    dim, n, k, dh, levels, cycles, centre, sigma, steps = args
    import numpy as np
    from oracle import solver as osolver, hss
    import workloads as W
    pr = osolver.Problem(dim, n, k, dh, levels=levels, cycles=cycles)
    _ = pr.hierarchy
    R = pr.M @ W.gaussian_nodal(dim, n, centre, sigma)
    t0 = time.perf_counter()
    hss.hss_correction(pr.Bdh, R, k, steps, pr.mg_solve)
    return (time.perf_counter() - t0) / steps


def cpu_baseline(W, name, outer_its, cycles, sample_steps, info):
    """The oracle (plain CSR, complex FP64) timed on the host: its HSS step
    in correction form with the same number of CSR V(2,2) cycles per inner
    solve as the GPU run, extrapolated to the whole solve with the GPU's
    outer iteration count (the oracle's own FGMRES orthogonalisation is left
    out, which flatters the CPU).  Independent right-hand sides run in
    parallel worker processes, one per column (at most one per core).  A 3D
    mesh too large for the oracle's assembly within the sample's budget is
    sampled on a 64^3 mesh with the same k, delta_hat, cycles and coarsest
    mesh, and its cost per node and step carried over (the oracle's CSR
    passes cost the same per node at any size)."""
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    w = W.WORKLOADS[name]
    dim, nrhs = w["dim"], w["nrhs"]
    n_s, lev_s = w["n"], w["levels"]
    if dim == 3 and w["n"] > 64:
        n_s = 64
        lev_s = w["levels"] - 2
    centres = W.workload_centres(name)
    jobs = [(dim, n_s, w["k"], w["delta_hat"], lev_s, cycles, tuple(c), w["sigma"], sample_steps)
            for c in centres]
    workers = max(1, min(len(jobs), info["nproc"]))
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        t_steps = list(ex.map(_baseline_column_worker, jobs))
    import math
    hss_steps = int(math.ceil(w["k"]))
    N = (w["n"] + 1) ** dim
    N_s = (n_s + 1) ** dim
    t_step = sum(t_steps) / len(t_steps) * (N / N_s)  # one column's HSS step at full size
    # the columns run concurrently on `workers` cores
    t_solve = outer_its * hss_steps * t_step * math.ceil(nrhs / workers)
    return {"value": N * nrhs / t_solve, "unit": "DoF/s", "cores": workers,
            "host_cores": info["nproc"], "cpu_model": info["cpu_model"], "kind": "oracle",
            "sample": "%d HSS steps (%d CSR V(2,2) cycles each) per right-hand side on the %s "
                      "mesh%s, %d column(s) on %d core(s), %.3f s per full-size step; "
                      "extrapolated to %d outer its x %d HSS steps"
                      % (sample_steps, cycles, name,
                         (" reduced to %d^3 (%d levels), cost per node carried over" % (n_s, lev_s))
                         if n_s != w["n"] else "", nrhs, workers, t_step, outer_its, hss_steps)}


def run_serving(W, count, sizes, rate, max_cols, budget_gb, precision, seed=1, restart=0,
                time_cap=None, arrival_cap=None):
    """Continuous-batching run: requests arrive by a seeded Poisson process
    and are submitted when their arrival time passes; the server steps
    continuously.  Latency = completion - arrival (wall clock).  With
    arrival_cap, the stream is cut after the arrivals up to that time and
    every request that arrived runs to completion (exact latencies of that
    prefix of the stream)."""
    import numpy as np
    import torch
    from paper_2506_18694_amd import Server, Solver
    reqs = W.serving_stream(count, sizes=sizes, max_rhs=8, rate=rate, seed=seed)
    if arrival_cap is not None:
        reqs = [r for r in reqs if r["arrival"] <= arrival_cap]
    # load vectors b = M f on the device (set-up, untimed)
    loaders = {}
    rhs = []
    for r in reqs:
        n = r["n"]
        if n not in loaders:
            loaders[n] = Solver(2, n, r["levels"], r["k"], 0.0, r["k"], precision=precision)
        f = np.stack([W.gaussian_nodal(2, n, c, r["sigma"]) for c in r["centres"]])
        rhs.append(loaders[n].load_nodal(torch.from_numpy(f).cuda()))
    torch.cuda.synchronize()
    for s in loaders.values():
        s.close()
    srv = Server(hbm_budget_bytes=budget_gb * 1e9, max_cols=max_cols, precision=precision,
                 restart=restart)
    ids, lat, its, conv = {}, {}, [], []
    t0 = time.perf_counter()
    nxt = 0
    done = 0
    dof = 0
    while done < len(reqs):
        now = time.perf_counter() - t0
        while nxt < len(reqs) and reqs[nxt]["arrival"] <= now:
            r = reqs[nxt]
            ids[nxt], _ = srv.submit(rhs[nxt], r["n"], r["levels"], r["k"], tol=1e-8)
            nxt += 1
        if not ids or (nxt < len(reqs) and sum(srv.load()[:2]) == 0):
            # nothing queued or running: wait for the next arrival
            time.sleep(max(0.0, reqs[nxt]["arrival"] - now))
            continue
        srv.step()
        t = time.perf_counter() - t0
        for i, rid in ids.items():
            if i in lat:
                continue
            info = srv.query(rid)
            if info["status"] == 2:
                lat[i] = t - reqs[i]["arrival"]
                its.append(info["outer_its"])
                conv.append(info["converged"])
                dof += (reqs[i]["n"] + 1) ** 2 * reqs[i]["nrhs"]
                done += 1
                if done % 8 == 0:
                    q, run, used = srv.load()
                    log("[serving] %d/%d done at %.1f s, queued %d running %d, %.1f GB in use"
                        % (done, len(reqs), t, q, run, used / 1e9))
        if nxt == len(reqs) and not ids:
            break
        if time_cap is not None and time.perf_counter() - t0 > time_cap:
            log("[serving] time cap reached with %d of %d requests done" % (done, len(reqs)))
            break
    makespan = time.perf_counter() - t0
    srv.close()
    finished = sorted(lat)
    L = np.array([lat[i] for i in finished])
    by_size = {}
    for i in finished:
        by_size.setdefault(reqs[i]["n"], []).append(lat[i])
    return {"requests": len(reqs), "stream_requests": count, "arrival_cap_s": arrival_cap,
            "completed": len(finished), "sizes": list(sizes),
            "rate_per_s": rate, "max_cols": max_cols, "restart": restart,
            "precision": precision, "p50_latency_s": float(np.percentile(L, 50)),
            "p99_latency_s": float(np.percentile(L, 99)), "mean_latency_s": float(L.mean()),
            "p50_by_size_s": {str(k): float(np.percentile(v, 50)) for k, v in sorted(by_size.items())},
            "p99_by_size_s": {str(k): float(np.percentile(v, 99)) for k, v in sorted(by_size.items())},
            "makespan_s": makespan, "dofs_per_s": dof / makespan,
            "mean_outer_its": float(np.mean(its)), "all_converged": bool(all(conv))}


# The paper's FGMRES counts with multigrid inner solves (primal formulation,
# uniform source; its table of FGMRES iterations with one W-cycle per HSS
# step), its measured HSS and outer rates with multigrid inner solves, and
# nu_s: context for the GPU runs at the same settings (a different cycle and
# smoother, so the counts need not match).
PAPER_MG = {16.0: {"fgmres": {0.5: 29, 1.0: 8, 1.5: 6}, "eta_s": 0.8778, "eta_h": 0.2264},
            32.0: {"fgmres": {0.5: 38, 1.0: 6, 1.5: 4}, "eta_s": 0.9376, "eta_h": 0.1410},
            64.0: {"fgmres": {0.5: 55, 1.0: 6, 1.5: 2}, "eta_s": 0.9681, "eta_h": 0.1225},
            128.0: {"fgmres": {0.5: 66, 1.0: 6, 1.5: 2}, "eta_s": 0.9844, "eta_h": 0.1130}}


# the same for the mixed formulation (two W-cycles with GMRES(4) smoothing
# per HSS step in the paper)
PAPER_MG_MIXED = {16.0: {"fgmres": {0.5: 38, 1.0: 9, 1.5: 7}, "eta_s": 0.8806, "eta_h": 0.2830},
                  32.0: {"fgmres": {0.5: 50, 1.0: 8, 1.5: 6}, "eta_s": 0.9373, "eta_h": 0.2386},
                  64.0: {"fgmres": {0.5: 72, 1.0: 8, 1.5: 5}, "eta_s": 0.9687, "eta_h": 0.2083},
                  128.0: {"fgmres": {0.5: 85, 1.0: 7, 1.5: 3}, "eta_s": 0.9842, "eta_h": 0.1796}}


# The paper's weak-scaling convergence tables (box source, FGMRES runs):
# measured HSS rate eta_s, its bound nu_s and the multigrid rate eta_mg of
# its W-cycle, for 2D k = 64..1024 and 3D k = 20, 40, 80.
PAPER_WEAK = {(2, 64.0): (0.9677, 0.00336), (2, 128.0): (0.9837, 0.00199),
              (2, 256.0): (0.9920, 0.00109), (2, 512.0): (0.9960, 0.00072),
              (2, 1024.0): (0.9980, 0.00057),
              (3, 20.0): (0.9029, 0.01931), (3, 40.0): (0.9492, 0.01507),
              (3, 80.0): (0.9748, 0.00950)}


def run_paper_rates(W, dims=(2, 3), seed=3):
    """The HSS and multigrid rates of the paper's weak-scaling runs on one
    GPU (delta_hat = 2, box source, ceil(k) HSS steps with the library's
    V(2,2) cycles): eta_s from the per-step HSS residuals of one
    preconditioner application to the random guess's residual, eta_mg as
    the residual contraction of one cycle on a random right-hand side."""
    import torch
    from paper_2506_18694_amd import Solver
    rows = []
    for dim in dims:
        meshes = W.WEAK_MESHES_2D if dim == 2 else W.WEAK_MESHES_3D
        for k, (n, levels) in meshes.items():
            t0 = time.perf_counter()
            s = Solver(dim, n, levels, k, 0.0, 2.0, restart=1)
            N = s.N
            f = torch.from_numpy(W.box_source(n, dim)).to("cuda").reshape(1, N)
            b = s.load_nodal(f)
            x0 = torch.from_numpy(W.paper_initial_guess(N, seed)).to("cuda").reshape(1, N)
            R = (b - s.apply("B0", x0)).contiguous()
            _, res = s.hss_history(R)
            steps = res.shape[1] - 1
            g = torch.Generator(device="cuda").manual_seed(seed)
            rb = torch.randn(1, N, dtype=torch.complex128, device="cuda", generator=g)
            rx = s.vcycle(rb)
            eta_mg = float(torch.linalg.vector_norm(rb - s.apply("L", rx)) /
                           torch.linalg.vector_norm(rb))
            torch.cuda.synchronize()
            p_eta, p_mg = PAPER_WEAK[(dim, k)]
            row = {"dim": dim, "k": k, "n": n, "levels": levels, "dofs": N,
                   "eta_s": float((res[0, -1] / res[0, 0]) ** (1.0 / steps)),
                   "nu_s": (k - 1.0) / (k + 1.0), "paper_eta_s": p_eta,
                   "eta_mg_vcycle": eta_mg, "paper_eta_mg_wcycle": p_mg,
                   "s": time.perf_counter() - t0}
            log("[rates] %dD k=%g n=%d: eta_s %.4f (nu_s %.4f, paper %.4f), one V-cycle %.3f, %.1fs"
                % (dim, k, n, row["eta_s"], row["nu_s"], p_eta, eta_mg, row["s"]))
            rows.append(row)
            s.close()
            del s
            torch.cuda.empty_cache()
    return rows


def run_paper(W, ks, precision, rtol_ref="r0", cycle="v", outers=("fgmres", "richardson"), seed=3,
              form="primal"):
    """The paper's experiment of Sec. 5.3 on the GPU path: delta_hat = 2,
    c0 k^(3/2) cells, uniform and box sources, seeded random initial guess,
    relative tolerance 1e-6, ceil(k^theta) HSS steps for theta in
    {1/2, 1, 3/2}, FGMRES and preconditioned Richardson; plus the measured
    HSS residual rate eta_s (on the random guess's residual) and outer rate
    eta_h at theta = 1.  The paper does not say what its tolerance is
    relative to: rtol_ref "b" stops at |r| <= 1e-6 |b|, "r0" at
    |r| <= 1e-6 |r_0|, r_0 = b - B_0 x_0, run as the solve of B_0 e = r_0
    from e = 0 (x = x_0 + e: the same Krylov spaces and Richardson
    iterates as the solve from x_0).  cycle "w" runs the paper's own
    multigrid (one W-cycle per HSS step, GMRES(5)-Jacobi smoothing on 4
    levels) instead of the library's V(2,2) Jacobi cycles, and reports the
    cycle's residual contraction eta_mg on a random right-hand side.  form
    "mixed" solves the mixed [DG0]^2 x P1 system instead (sigma eliminated
    in every HSS step)."""
    import math
    import torch
    from paper_2506_18694_amd import Solver
    rows = []
    for k in ks:
        n, levels = W.PAPER_MESHES[k]
        if cycle == "w":
            levels = 4  # the paper's hierarchy: 4 levels, 64x fewer coarsest DoFs
        N = (n + 1) ** 2
        NV = N + (4 * n * n if form == "mixed" else 0)
        x0 = torch.from_numpy(W.paper_initial_guess(NV, seed)).to("cuda").reshape(1, NV)
        mix = form == "mixed"
        sys_op = "MIXED" if mix else "B0"
        for source in ("uniform", "box"):
            f = W.uniform_source(2, n) if source == "uniform" else W.box_source(n)
            row = {"k": k, "n": n, "levels": levels, "dofs": NV, "source": source, "form": form}
            for theta in (0.5, 1.0, 1.5):
                steps = int(math.ceil(k ** theta))
                for outer in outers:
                    t0 = time.perf_counter()
                    s = Solver(2, n, levels, k, 0.0, 2.0, precision=precision, hss_steps=steps,
                               outer=outer, x0_given=rtol_ref == "b",
                               restart=(120 if mix else 200) if outer == "fgmres" else 0,
                               max_outer=2000, cycle=cycle, mixed=mix)
                    b = s.load_nodal(torch.from_numpy(f).to("cuda").reshape(1, N))
                    if rtol_ref == "r0":
                        x, st = s.solve((b - s.apply(sys_op, x0)).contiguous(), tol=1e-6)
                    else:
                        x, st = s.solve(b, tol=1e-6, x0=x0)
                    torch.cuda.synchronize()
                    key = "%s_theta%s" % (outer, {0.5: "1/2", 1.0: "1", 1.5: "3/2"}[theta])
                    row[key] = {"its": st["outer_its"], "hss_total": st["outer_its"] * steps,
                                "cycles_total": st["vcycles"], "mg_cycles": st["mg_cycles"],
                                "eta_h": st["outer_rate"], "converged": st["converged"],
                                "s": time.perf_counter() - t0}
                    log("[paper] k=%g %s %s: %d its (%d cycles/HSS step), eta_h %.4f, %.1fs"
                        % (k, source, key, st["outer_its"], st["mg_cycles"], st["outer_rate"],
                           time.perf_counter() - t0))
                    if theta == 1.0 and outer == "fgmres":
                        R = b - s.apply(sys_op, x0)
                        _, res = s.hss_history(R.contiguous())
                        row["eta_s"] = float((res[0, -1] / res[0, 0]) ** (1.0 / steps))
                        # one cycle on a random right-hand side: residual contraction
                        g = torch.Generator(device="cuda").manual_seed(seed)
                        rb = torch.randn(1, N, dtype=torch.complex128, device="cuda", generator=g)
                        rx = s.vcycle(rb)
                        row["eta_mg"] = float(torch.linalg.vector_norm(rb - s.apply("L", rx)) /
                                              torch.linalg.vector_norm(rb))
                    s.close()
            row["nu_s"] = (k - 1.0) / (k + 1.0)
            ref = PAPER_MG_MIXED if mix else PAPER_MG
            row["paper_mg"] = {"fgmres_uniform": {str(t): c for t, c in ref[k]["fgmres"].items()},
                               "eta_s": ref[k]["eta_s"], "eta_h": ref[k]["eta_h"]}
            rows.append(row)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1,
                    help="cap on the timed headline solves (the wall-clock budget may allow fewer)")
    ap.add_argument("--warmup", type=int, default=1,
                    help="cap on the headline's full warm-up solves (at least one runs)")
    ap.add_argument("--budget-s", type=float, default=450.0,
                    help="wall-clock budget of the whole run in seconds, from process start")
    ap.add_argument("--workload", default=HEADLINE)
    ap.add_argument("--precision", choices=("fp64", "fp32"), default="fp64",
                    help="precision mode of the headline solves (the other mode is reported "
                         "beside them)")
    ap.add_argument("--only-headline", action="store_true",
                    help="skip the 2D configurations")
    ap.add_argument("--no-oracle-error", action="store_true",
                    help="skip the error of the 2D solves against the oracle's direct solve")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--split", action="store_true",
                    help="run the preconditioner's right-hand sides as two groups on two "
                         "streams (for comparison; the default is one batch on one stream)")
    ap.add_argument("--lds-kernels", action="store_true",
                    help="run the large 2D levels with the LDS-tiled kernels instead of the "
                         "register-streaming ones (for comparison)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=10)
    ap.add_argument("--profile-run", action="store_true",
                    help="short run for counter collection: 3 outer iterations of the "
                         "headline workload, no extras")
    ap.add_argument("--serving", action="store_true",
                    help="run the continuous-batching serving workload instead (one JSON line)")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--sizes", default="128,256,512,1024")
    ap.add_argument("--rate", default="auto",
                    help="Poisson arrival rate (requests/s), or 'auto': 0.8 of the capacity "
                         "measured by a saturating batch of requests first")
    ap.add_argument("--max-cols", type=int, default=8)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--serving-restart", type=int, default=0,
                    help="FGMRES basis per column in the serving groups (0: the library's "
                         "3 ceil(k) + 30 for each group's k)")
    ap.add_argument("--probe-requests", type=int, default=32,
                    help="size of the saturating batch that measures capacity (rate auto)")
    ap.add_argument("--time-cap", type=float, default=None,
                    help="stop the serving run after this many seconds (latencies of the "
                         "completed requests are reported with the completed count)")
    ap.add_argument("--arrival-cap", type=float, default=None,
                    help="serve only the requests of the stream that arrive within this many "
                         "seconds, each to completion")
    ap.add_argument("--paper", action="store_true",
                    help="run the paper's own settings (delta_hat = 2, uniform and box sources, "
                         "theta sweep, FGMRES and Richardson) and print their counts and rates")
    ap.add_argument("--paper-k", default="16,32,64,128")
    ap.add_argument("--paper-rates", action="store_true",
                    help="HSS and multigrid rates at the meshes of the paper's weak-scaling runs")
    ap.add_argument("--paper-precision", default="fp64")
    ap.add_argument("--paper-cycle", choices=("v", "w"), default="v",
                    help="v: the library's V(2,2) Jacobi cycles; w: the paper's W-cycle with "
                         "GMRES(5)-Jacobi smoothing on 4 levels")
    ap.add_argument("--paper-outer", default="fgmres,richardson")
    ap.add_argument("--paper-form", choices=("primal", "mixed"), default="primal")
    ap.add_argument("--paper-rtol", choices=("r0", "b"), default="r0",
                    help="the 1e-6 tolerance relative to the initial residual (r0) or to |b|")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X and "
              "this build has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.paper_rates:
        t0 = time.perf_counter()
        rows = run_paper_rates(W)
        out = {"metric": "HSS and multigrid contraction rates at the paper's weak-scaling meshes",
               "value": None, "unit": "rate", "n_gpus": 1, "steps": 1, "warmup": 0,
               "ms_per_step": (time.perf_counter() - t0) * 1e3, "higher_is_better": False,
               "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
               "config": {"workload": "paper-weak-scaling-meshes-delta_hat2"}, "table": rows}
        print(json.dumps(out), flush=True)
        return
    if args.paper:
        ks = [float(v) for v in args.paper_k.split(",")]
        t0 = time.perf_counter()
        rows = run_paper(W, ks, args.paper_precision, args.paper_rtol, args.paper_cycle,
                         tuple(args.paper_outer.split(",")), form=args.paper_form)
        out = {"metric": "outer iterations and measured rates at the paper's settings",
               "value": None, "unit": "iterations", "n_gpus": 1, "steps": 1, "warmup": 0,
               "ms_per_step": (time.perf_counter() - t0) * 1e3, "higher_is_better": False,
               "scaling": "weak", "vs_baseline": None,
               "dtype": "f64" if args.paper_precision == "fp64" else "f32+f64",
               "data": "synthetic",
               "config": {"workload": "paper-2d-p1-delta_hat2", "tol": 1e-6,
                          "tol_relative_to": args.paper_rtol, "cycle": args.paper_cycle,
                          "form": args.paper_form,
                          "precision": args.paper_precision},
               "table": rows}
        print(json.dumps(out), flush=True)
        return
    if args.serving:
        sizes = tuple(int(v) for v in args.sizes.split(","))
        capacity = None
        if args.rate == "auto":
            # capacity: a batch of requests all queued at t = 0 (another seed)
            probe = run_serving(W, args.probe_requests, sizes, None, args.max_cols,
                                args.budget_gb, "fp32", seed=2, restart=args.serving_restart)
            capacity = probe["requests"] / probe["makespan_s"]
            rate = 0.8 * capacity
            log("[serving] capacity %.2f requests/s; offered load 0.8 -> %.2f requests/s"
                % (capacity, rate))
        else:
            rate = float(args.rate)
        res = run_serving(W, args.requests, sizes, rate, args.max_cols, args.budget_gb, "fp32",
                          restart=args.serving_restart, time_cap=args.time_cap,
                          arrival_cap=args.arrival_cap)
        res["capacity_req_per_s"] = capacity
        res["offered_load"] = rate / capacity if capacity else None
        out = {"metric": "serving p50/p99 latency (continuous batching, FP32-MG/FP64-outer)",
               "value": res["p99_latency_s"], "unit": "s (p99)", "n_gpus": 1, "steps": 1,
               "warmup": 0, "ms_per_step": res["makespan_s"] * 1e3, "higher_is_better": False,
               "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
               "config": {"workload": "serving-2d-p1", **{k: v for k, v in res.items()
                                                          if k in ("requests", "stream_requests",
                                                                   "arrival_cap_s", "completed", "sizes",
                                                                   "rate_per_s", "max_cols",
                                                                   "restart", "precision",
                                                                   "offered_load")}},
               "serving": res}
        print(json.dumps(out), flush=True)
        return
    if args.profile_run:
        # counter collection: a handle capped at 3 outer iterations, eager
        w = W.WORKLOADS[args.workload]
        prec = args.precision
        s = make_solver(W, args.workload, prec, profile=True, max_outer=3, restart=3,
                        streaming=not args.lds_kernels)
        f = torch.from_numpy(W.workload_sources(args.workload)).cuda().contiguous()
        b = s.load_nodal(f)
        _, st = s.solve(b, tol=args.tol)
        torch.cuda.synchronize()
        log("[bench] profile run: %d outer its, %.1f ms" % (st["outer_its"], st["solve_ms"]))
        print(json.dumps({"profile_run": args.workload, "precision": prec,
                          "outer_its": st["outer_its"], "solve_ms": st["solve_ms"],
                          "roofline": roofline(w["dim"], args.workload, prec, [st])}), flush=True)
        return
    # ---- the default run: headline + the other configurations -----------------
    import tempfile
    budget = args.budget_s
    info = host_info()
    tmpdir = tempfile.mkdtemp(prefix="helm_bench_")
    w_head = W.WORKLOADS[args.workload]
    head_prec = args.precision
    other = [] if args.only_headline else [n for n in ("p1-64-k10", "p1-1024-k100", "p1-2048-k200")
                                           if n != args.workload]
    # the oracle's direct solves of the 1024^2 and 2048^2 meshes (sparse LU in
    # nested-dissection order: ~15 s and ~1.5 min) run beside the GPU work
    workers = {}
    if not args.no_oracle_error:
        for name in other:
            if name in ("p1-1024-k100", "p1-2048-k200"):
                workers[name] = start_oracle_worker(name, tmpdir)
                log("[bench] oracle direct-solve worker started for %s" % name)
    # time the rest of the run needs after the headline's FP64 solves, in
    # units of one headline solve (FP32-MG: a cheaper solve, no full warm-up)
    # plus the fixed-size parts (2D configurations, CPU baseline, margin)
    fixed_rest = (0 if args.only_headline else 75.0) + (0 if args.no_cpu_baseline else 25.0) + 20.0

    def fits(t_solve):
        rest = fixed_rest + (0 if args.no_fp32 else 1.0 * t_solve)
        return int(max(0.0, budget - elapsed() - rest) // max(t_solve, 1e-3))

    r = measure(W, args.workload, head_prec, args.warmup, args.steps, args.tol, deadline_fn=fits,
                streaming=not args.lds_kernels, split=args.split, keep_x=not args.no_fp32)
    dim = w_head["dim"]
    out = {"metric": METRIC, "value": r["value"], "unit": "DoF/s", "n_gpus": 1,
           "steps": r["steps"], "warmup": r["warmup"], "ms_per_step": r["ms"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if head_prec == "fp64" else "f32+f64", "data": "synthetic",
           "config": {"workload": args.workload, "dim": dim, "n": w_head["n"], "dofs": r["N"],
                      "nrhs": r["nrhs"], "k": w_head["k"], "delta_hat": w_head["delta_hat"],
                      "levels": w_head["levels"], "precision": head_prec, "tol": args.tol,
                      "outer_its": r["summary"]["outer_its"],
                      "hss_steps": r["summary"]["hss_steps"],
                      "mg_cycles": r["summary"]["mg_cycles"],
                      "vcycle_rate": r["summary"]["vcycle_rate"],
                      "true_rel_residual": r["summary"]["true_rel_residual"],
                      "converged": r["ok"], "budget_s": budget,
                      "requested_steps": args.steps, "requested_warmup": args.warmup},
           "roofline": roofline(dim, args.workload, head_prec, r["stats"]),
           "breakdown": {"solve_ms": sum(st["solve_ms"] for st in r["stats"]) / len(r["stats"]),
                         "precond_ms": sum(st["precond_ms"] for st in r["stats"]) / len(r["stats"])}}
    if not args.no_fp32:
        import numpy as np
        other_prec = "fp32" if head_prec == "fp64" else "fp64"
        r2 = measure(W, args.workload, other_prec, 1, 1, args.tol, full_warmup=False,
                     streaming=not args.lds_kernels, split=args.split, keep_x=True)
        sub = dict(r2["summary"])
        a, b = (r["x"], r2["x"]) if head_prec == "fp64" else (r2["x"], r["x"])
        sub["rel_l2_vs_fp64_solution"] = oracle_error(b, a)
        if head_prec == "fp64":
            sub["ratio_vs_fp64"] = r2["value"] / r["value"]
            out["fp32_mg"] = sub
        else:
            sub["ratio_fp32mg_over_fp64"] = r["value"] / r2["value"]
            out["fp64"] = sub
        del a, b
    r.pop("x", None)
    # ---- the 2D configurations: both precision modes, error vs the oracle ------
    subs = {}
    for name in other:
        if elapsed() > budget - fixed_rest + 60.0:
            log("[bench] skipping %s: budget" % name)
            subs[name] = {"skipped": "wall-clock budget"}
            continue
        import numpy as np
        w = W.WORKLOADS[name]
        ent = {"dim": w["dim"], "n": w["n"], "dofs": (w["n"] + 1) ** w["dim"], "nrhs": w["nrhs"],
               "k": w["k"], "levels": w["levels"]}
        xs = {}
        for prec in ("fp64", "fp32"):
            m = measure(W, name, prec, 1, 1, args.tol, full_warmup=False,
                        streaming=not args.lds_kernels, keep_x=True)
            xs[prec] = m["x"]
            ent["fp64" if prec == "fp64" else "fp32_mg"] = m["summary"]
        ent["ratio_fp32mg_vs_fp64"] = ent["fp32_mg"]["value"] / ent["fp64"]["value"]
        ent["fp32mg_rel_l2_vs_fp64_solution"] = oracle_error(xs["fp32"], xs["fp64"])
        if not args.no_oracle_error:
            U = None
            if name == "p1-64-k10":
                from oracle import solver as osolver
                pr = osolver.Problem(2, w["n"], w["k"], w["delta_hat"], levels=1)
                U = np.stack([pr.solve_direct((pr.M @ fi).astype(np.complex128))
                              for fi in W.workload_sources(name)])
            elif name in workers:
                p, path = workers[name]
                # the remaining configurations take a few seconds; keep the
                # CPU baseline's share and a margin of the budget
                p.join(timeout=max(1.0, budget - elapsed() - 60.0))
                if os.path.exists(path):
                    U = np.load(path)
                else:
                    log("[bench] oracle direct solve of %s not finished (worker %s)"
                        % (name, "running" if p.is_alive() else "exited %s" % p.exitcode))
            if U is not None:
                ent["rel_l2_error_vs_oracle_direct"] = {"fp64": oracle_error(xs["fp64"], U),
                                                        "fp32_mg": oracle_error(xs["fp32"], U)}
            else:
                ent["rel_l2_error_vs_oracle_direct"] = None
        subs[name] = ent
        log("[bench] %s: fp64 %.3g DoF/s, fp32-mg %.3g DoF/s (ratio %.2f)"
            % (name, ent["fp64"]["value"], ent["fp32_mg"]["value"], ent["ratio_fp32mg_vs_fp64"]))
    if subs:
        out["workloads"] = subs
    for p, _ in workers.values():
        if p.is_alive():
            p.terminate()
    if not args.no_cpu_baseline:
        log("[bench] oracle CPU baseline sample ...")
        out["cpu_baseline"] = cpu_baseline(W, args.workload, out["config"]["outer_its"],
                                           out["config"]["mg_cycles"], args.cpu_sample_steps, info)
    out["host"] = info
    out["wall_s"] = elapsed()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

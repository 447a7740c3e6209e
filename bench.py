"""Throughput benchmark: solved degrees of freedom per second to a 1e-8
relative residual for the shifted-HSS Helmholtz solver on one MI355X.

One step = one complete helm_solve (outer FP64 FGMRES, shifted-HSS
preconditioner with ceil(k) HSS sweeps, each inner solve a fixed number of
V(2,2) cycles chosen from the measured cycle rate, all right-hand sides)
with the load vectors already resident in HBM.

Default workload: 2D P1, 1024 x 1024 right-diagonal mesh (N = 1,050,625
nodes), k = 100, delta = 0, delta_hat = k, 8 multigrid levels, four
Gaussian sources (sigma 0.02) at seeded uniform centres, plain complex
FP64 on the GPU.  The same workload is also solved with FP32 multigrid and
FP64 outer iteration, reported as `fp32_mg`.

Prints ONE JSON line on stdout; progress goes to stderr.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "solved DOFs/s to 1e-8 rel residual (FP32-MG vs FP64), %HBM peak; p50/p99 latency"
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the dominant kernel: finest-level prolongation, four Jacobi sweeps (cycle
# q's post-smoothing and cycle q+1's pre-smoothing) and the residual
# restriction in one register-streaming pass
DOMINANT = {"tag": "k_stream_sweeps4", "source": "kernels2d_stream.hip",
            "desc": "finest-level prolongation + four Jacobi sweeps + residual restriction "
                    "(k_stream_sweeps<S=4>)"}


# in 3D the timed pass is one finest-level Jacobi sweep: the z-marching
# column-tile kernel on the interior nodes plus the boundary-node kernel
DOMINANT_3D = ("finest-level Jacobi sweep (k_stencil3d_tile + k_stencil3d_bnd); "
               "x, b read, x' written")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in (DOMINANT["source"], "helm_common.h", "stencil_rows.h"):
        with open(os.path.join(ROOT, "paper_2506_18694_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(workload, precision):
    """HBM traffic per launch of the dominant kernel from committed rocprofv3
    counter runs; null when the kernel source changed since they were taken."""
    path = os.path.join(PROFILES, "traffic_%s_%s_%s.json" % (DOMINANT["tag"], workload, precision))
    if workload.startswith("q1"):
        return None
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def run_solves(W, name, precision, steps, warmup, tol, max_outer=0, streaming=True, split=False):
    import torch
    from paper_2506_18694_amd import Solver
    w = W.WORKLOADS[name]
    s = Solver(w["dim"], w["n"], w["levels"], w["k"], w["delta"], w["delta_hat"],
               precision=precision, profile=True, max_outer=max_outer,
               restart=max_outer if max_outer else 0, streaming=streaming, split=split)
    f = torch.from_numpy(W.workload_sources(name)).cuda().contiguous()
    b = s.load_nodal(f)
    x = torch.empty_like(b)
    ws = s.workspace(b.shape[0])
    log("[bench] %s %s: N=%d nrhs=%d workspace %.1f GB" % (name, precision, s.N, b.shape[0],
                                                           ws.numel() / 1e9))
    for i in range(warmup):
        _, st = s.solve(b, x, tol=tol, workspace=ws)
        log("[bench] warmup %d: %.1f ms, outer its %d, true rel res %.2e"
            % (i, st["solve_ms"], st["outer_its"], st["true_rel_residual"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(steps):
        _, st = s.solve(b, x, tol=tol, workspace=ws)
        stats.append(st)
        log("[bench] step %d: %.1f ms, outer its %d, true rel res %.2e"
            % (i, st["solve_ms"], st["outer_its"], st["true_rel_residual"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ok = all(st["converged"] == 1 and st["true_rel_residual"] <= tol for st in stats)
    s.close()
    return dict(N=s.N, nrhs=b.shape[0], elapsed=elapsed, stats=stats, ok=ok, w=w)


def cpu_baseline(W, name, outer_its, cycles, sample_steps):
    """The oracle's HSS step (correction form, `cycles` CSR V(2,2) cycles per
    inner solve, as the GPU run used) timed on the host for one right-hand
    side, extrapolated to the full solve with the GPU's outer iteration count
    (the oracle's own FGMRES orthogonalisation is left out, which flatters
    the CPU)."""
    from oracle import solver as osolver, hss
    w = W.WORKLOADS[name]
    pr = osolver.Problem(w["dim"], w["n"], w["k"], w["delta_hat"], levels=w["levels"],
                         cycles=cycles)
    f = W.workload_sources(name)[0]
    R = pr.M @ f
    _ = pr.hierarchy
    t0 = time.perf_counter()
    hss.hss_correction(pr.Bdh, R, w["k"], sample_steps, pr.mg_solve)
    t_step = (time.perf_counter() - t0) / sample_steps
    nrhs = w["nrhs"]
    t_solve = nrhs * outer_its * pr.hss_steps() * t_step
    N = (w["n"] + 1) ** w["dim"]
    return {"value": N * nrhs / t_solve, "unit": "DoF/s", "cores": 1, "kind": "oracle",
            "sample": "%d HSS steps (%d CSR V(2,2) cycles each) for 1 of %d right-hand sides on "
                      "the %s mesh, %.3f s per step, extrapolated to %d outer its x %d steps x "
                      "%d rhs" % (sample_steps, cycles, nrhs, name, t_step, outer_its,
                                  pr.hss_steps(), nrhs)}


def run_serving(W, count, sizes, rate, max_cols, budget_gb, precision, seed=1):
    """Continuous-batching run: requests arrive by a seeded Poisson process
    and are submitted when their arrival time passes; the server steps
    continuously.  Latency = completion - arrival (wall clock)."""
    import numpy as np
    import torch
    from paper_2506_18694_amd import Server, Solver
    reqs = W.serving_stream(count, sizes=sizes, max_rhs=8, rate=rate, seed=seed)
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
    srv = Server(hbm_budget_bytes=budget_gb * 1e9, max_cols=max_cols, precision=precision)
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
        if not ids:
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
    makespan = time.perf_counter() - t0
    srv.close()
    L = np.array([lat[i] for i in range(len(reqs))])
    return {"requests": len(reqs), "sizes": list(sizes), "rate_per_s": rate, "max_cols": max_cols,
            "precision": precision, "p50_latency_s": float(np.percentile(L, 50)),
            "p99_latency_s": float(np.percentile(L, 99)), "mean_latency_s": float(L.mean()),
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
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="p1-1024-k100")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--split", action="store_true",
                    help="run the preconditioner's right-hand sides as two groups on two "
                         "streams (for comparison; the default is one batch on one stream)")
    ap.add_argument("--lds-kernels", action="store_true",
                    help="run the large 2D levels with the LDS-tiled kernels instead of the "
                         "register-streaming ones (for comparison)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=20)
    ap.add_argument("--profile-run", action="store_true",
                    help="short run for counter collection: 3 outer iterations, no extras")
    ap.add_argument("--serving", action="store_true",
                    help="run the continuous-batching serving workload instead (one JSON line)")
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--sizes", default="128,256,512")
    ap.add_argument("--rate", default="auto",
                    help="Poisson arrival rate (requests/s), or 'auto': 0.8 of the capacity "
                         "measured by a saturating batch of requests first")
    ap.add_argument("--max-cols", type=int, default=16)
    ap.add_argument("--budget-gb", type=float, default=120.0)
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
            probe = run_serving(W, max(16, args.requests // 4), sizes, None, args.max_cols,
                                args.budget_gb, "fp32", seed=2)
            capacity = probe["requests"] / probe["makespan_s"]
            rate = 0.8 * capacity
            log("[serving] capacity %.2f requests/s; offered load 0.8 -> %.2f requests/s"
                % (capacity, rate))
        else:
            rate = float(args.rate)
        res = run_serving(W, args.requests, sizes, rate, args.max_cols, args.budget_gb, "fp32")
        res["capacity_req_per_s"] = capacity
        res["offered_load"] = rate / capacity if capacity else None
        out = {"metric": "serving p50/p99 latency (continuous batching, FP32-MG/FP64-outer)",
               "value": res["p99_latency_s"], "unit": "s (p99)", "n_gpus": 1, "steps": 1,
               "warmup": 0, "ms_per_step": res["makespan_s"] * 1e3, "higher_is_better": False,
               "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
               "config": {"workload": "serving-2d-p1", **{k: v for k, v in res.items()
                                                          if k in ("requests", "sizes", "rate_per_s",
                                                                   "max_cols", "precision",
                                                                   "offered_load")}},
               "serving": res}
        print(json.dumps(out), flush=True)
        return
    name = args.workload
    prec = W.WORKLOADS[name]["precision"]
    main_prec = "fp64" if prec == "fp64" else "fp32"
    if args.profile_run:
        args.no_fp32 = args.no_cpu_baseline = True
    r = run_solves(W, name, main_prec, args.steps, args.warmup, args.tol,
                   max_outer=3 if args.profile_run else 0, streaming=not args.lds_kernels,
                   split=args.split)
    ms = r["elapsed"] / args.steps * 1e3
    value = r["N"] * r["nrhs"] / (ms / 1e3)
    sw_ms = sum(st["sweep_ms"] for st in r["stats"])
    sw_n = sum(st["sweep_launches"] for st in r["stats"])
    sw_b = sum(st["sweep_bytes"] for st in r["stats"])
    achieved = sw_b / (sw_ms / 1e3) / 1e9 if sw_ms > 0 else None
    per_launch = sw_b / sw_n if sw_n else None
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": stored_traffic(name, main_prec),
            "kernel": DOMINANT["desc"] if r["w"]["dim"] == 2 else DOMINANT_3D,
            "bytes_per_launch": per_launch,
            "avg_launch_us": sw_ms / sw_n * 1e3 if sw_n else None}
    w = r["w"]
    out = {"metric": METRIC, "value": value, "unit": "DoF/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if main_prec == "fp64" else "f32+f64",
           "data": "synthetic",
           "config": {"workload": name, "dim": w["dim"], "n": w["n"], "dofs": r["N"],
                      "nrhs": r["nrhs"], "k": w["k"], "delta_hat": w["delta_hat"],
                      "levels": w["levels"], "precision": main_prec, "tol": args.tol,
                      "outer_its": max(st["outer_its"] for st in r["stats"]),
                      "hss_steps": r["stats"][0]["hss_steps"],
                      "mg_cycles": r["stats"][0]["mg_cycles"],
                      "vcycle_rate": r["stats"][0]["vcycle_rate"],
                      "true_rel_residual": max(st["true_rel_residual"] for st in r["stats"]),
                      "converged": r["ok"]},
           "roofline": roof,
           # where a solve's time goes: device time inside the preconditioner
           # (HSS loop) against the whole solve's wall time
           "breakdown": {"solve_ms": sum(st["solve_ms"] for st in r["stats"]) / len(r["stats"]),
                         "precond_ms": sum(st["precond_ms"] for st in r["stats"]) / len(r["stats"])}}
    if not args.no_fp32 and main_prec == "fp64":
        r32 = run_solves(W, name, "fp32", 1, 1, args.tol, streaming=not args.lds_kernels,
                         split=args.split)
        ms32 = r32["elapsed"] * 1e3
        v32 = r32["N"] * r32["nrhs"] / (ms32 / 1e3)
        s32 = r32["stats"][0]
        out["fp32_mg"] = {"value": v32, "ms_per_step": ms32, "ratio_vs_fp64": v32 / value,
                          "outer_its": s32["outer_its"],
                          "true_rel_residual": s32["true_rel_residual"],
                          "sweep_GBs": s32["sweep_bytes"] / (s32["sweep_ms"] / 1e3) / 1e9
                          if s32["sweep_ms"] > 0 else None,
                          "converged": r32["ok"]}
    if not args.no_cpu_baseline:
        log("[bench] oracle CPU baseline sample ...")
        out["cpu_baseline"] = cpu_baseline(W, name, out["config"]["outer_its"],
                                           out["config"]["mg_cycles"], args.cpu_sample_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

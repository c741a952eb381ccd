"""Throughput of the polarized-traces solver on one MI355X.

Workload (default): the 200^3 layered-dipping model with a 15-point absorbing
layer, 8 points per wavelength at c_min = 1.5, L = 20 layers, R = 64 point
sources on an 8 x 8 surface grid at depth 16; complex64 fronts and
substitutions on the matrix cores with FP64 iterative refinement (GMRES on
the interface traces in FP64).

A step is one online solve of the 64-column batch (Algorithm 2: local solves
of the source, GMRES with the polarized sweeps, reconstruction, FP64
residual and refinement) with the factors resident in HBM, as the paper
times its "online" stage; the factorization (Algorithm 1) is timed once and
reported beside it.  The FP64 path (complex128 fronts) is run on the same
batch first: it supplies the reference each mixed-precision column is
checked against (relative l2 error <= 1e-6) and the RHS/s of the plain FP64
GPU path.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solved RHS/s at n=200³, rel.err≤1e-6, mixed vs FP64; p50/p99 latency"
PEAK = {"fp32_mfma": 157.3e12, "fp64_mfma": 78.6e12, "hbm": 8.0e12}
# Mixed-precision refinement settings of every mixed run here: GMRES to 5e-4
# in the first solve and to 2e-4 in the refinement steps, FP64 residual
# tolerance 1e-10, stop on an estimated error of 1e-6 (at 200^3 every column
# then stops after two solves; with 1e-3 / 2e-4 ten of 64 took a third)
MIXED_KW = dict(ir_tol=1e-10, inner_tol=5e-4, inner_tol_refine=2e-4, err_target=1e-6,
                ir_max_steps=4)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="layered-200")
    ap.add_argument("--rhs", type=int, default=64)
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--fp64-warmup", type=int, default=1)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--fp64-loose-tol", default="1e-6,1e-7",
                    help="GMRES tolerances of the FP64 runs compared at equal accuracy: "
                         "the fastest whose error meets the mixed path's target counts")
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="GMRES tolerance of the first mixed-precision solve "
                         "(default: that of MIXED_KW)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", action="store_true", default=True,
                    help="time kernel classes with HIP events (roofline)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="tile widths from the batch width instead of measured per depth")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this size first (counter calibration)")
    ap.add_argument("--serve", action="store_true",
                    help="serving run instead: 3 resident 160^3 models, Poisson requests")
    ap.add_argument("--serve-requests", type=int, default=12)
    ap.add_argument("--batch", action="store_true",
                    help="batched run instead: independent problems n in [64, 160]")
    ap.add_argument("--batch-count", type=int, default=32)
    ap.add_argument("--batch-resident", type=int, default=0,
                    help="at most this many problems resident at once (0: as many as "
                         "memory admits; 1: one after the other, no overlap)")
    ap.add_argument("--slots", type=int, default=32)
    ap.add_argument("--depth-rates", action="store_true",
                    help="per-depth substitution GEMM rates of one interior layer's solve "
                         "(the measured tile-width launches against each depth's flops)")
    ap.add_argument("--rhs-scaling", action="store_true",
                    help="RHS/s against the number of right-hand sides R = 1, 2, ..., 64 "
                         "on one factorization of the workload")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_solves(s, srcs, steps, warmup, torch):
    out = None
    for _ in range(warmup):
        out = s.solve_points(srcs, out=out)
    torch.cuda.synchronize()
    s.kernel_stats(reset=True)
    lat = []
    info = None
    t0 = time.perf_counter()
    for _ in range(steps):
        t1 = time.perf_counter()
        out, info = s.solve_points(srcs, info=True, out=out)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    return out, info, total, lat


def percentile(v, q):
    v = sorted(v)
    if not v:
        return None
    i = min(len(v) - 1, max(0, int(round(q / 100.0 * (len(v) - 1)))))
    return v[i]


def measured_traffic(kernel_class, workload):
    """HBM bytes per launch of a kernel class from the calibrated rocprofv3
    FETCH_SIZE / WRITE_SIZE runs kept in profiles/, if they were taken on the
    current kernel sources (else None)."""
    from paper_1801_08655_amd.rocprof_summary import kernel_sources_hash, read_traffic
    t = read_traffic(os.path.join(ROOT, "profiles", f"traffic_{kernel_class}_{workload}.txt"))
    if not t or t.get("sources_sha256") != kernel_sources_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def roofline(stats, precision, workload):
    """Dominant (longest) kernel class: achieved flops per launch-second vs
    the matrix-core peak of its arithmetic type."""
    best = max(stats.items(), key=lambda kv: kv[1]["total_ms"])
    name, st = best
    avg_ms = st["total_ms"] / max(st["launches"], 1)
    flops_per_launch = st["flops"] / max(st["launches"], 1)
    bytes_per_launch = st["bytes"] / max(st["launches"], 1)
    traffic = measured_traffic(name, workload)
    if flops_per_launch > 0:
        achieved = flops_per_launch / (avg_ms * 1e-3)
        peak = PEAK["fp32_mfma"] if precision == "mixed" else PEAK["fp64_mfma"]
        return {"kernel": name, "bound": "mfma", "achieved": achieved / 1e12,
                "peak": peak / 1e12, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": traffic, "launches": st["launches"],
                "avg_launch_ms": avg_ms,
                "flops_per_launch": flops_per_launch,
                "bytes_per_launch": bytes_per_launch,
                "traffic_over_algorithmic": (traffic / bytes_per_launch) if traffic else None}
    achieved = bytes_per_launch / (avg_ms * 1e-3)
    return {"kernel": name, "bound": "hbm", "achieved": achieved / 1e9,
            "peak": PEAK["hbm"] / 1e9, "unit": "GB/s", "frac": achieved / PEAK["hbm"],
            "traffic": traffic, "launches": st["launches"], "avg_launch_ms": avg_ms}


def small_k_probe(s, wl, torch, layer=None, reps=3):
    """One-column local solves of an interior layer (layer 5, or the middle
    one when there are fewer than 10; the HBM-bound regime of the
    substitutions): algorithmic bytes of the forward / backward GEMM classes
    per event-timed second, against the 8 TB/s HBM peak."""
    if layer is None:
        layer = min(5, wl.n_layers // 2)
    _, _, lo, hi = s.layer_info(layer)
    r = torch.randn((1, hi - lo + 1, wl.n[1], wl.n[0]), dtype=torch.complex128,
                    device="cuda")
    s.layer_solve(layer, r)
    torch.cuda.synchronize()
    s.kernel_stats(reset=True)
    for _ in range(reps):
        s.layer_solve(layer, r)
    torch.cuda.synchronize()
    ks = s.kernel_stats(reset=True)
    out = {"layer": layer, "k": 1, "solves": reps}
    for name in ("solve_fwd_gemm", "solve_bwd_gemm"):
        st = ks[name]
        gbs = st["bytes"] / max(st["total_ms"], 1e-9) / 1e6
        out[name] = {"ms_per_solve": st["total_ms"] / reps, "GB/s": gbs,
                     "frac_hbm": gbs * 1e9 / PEAK["hbm"]}
    return out


def cpu_baseline():
    """The oracle (global sparse assembly + SuperLU direct solve, complex128)
    on the same workload recipe at the largest grid it finishes in ~15 s.
    Returns the record and the oracle's solution (for the same-input GPU
    comparison)."""
    import numpy as np
    from helm_inputs import workload
    from oracle.direct import SparseLU
    from oracle.discretization import Problem, point_source_rhs
    wl = workload("layered-32")
    pb = Problem(wl.m(), wl.h, wl.omega, wl.pml, wl.pml_C)
    F = point_source_rhs(pb.shape, wl.sources, wl.h)
    t0 = time.perf_counter()
    H = pb.operator()
    lu = SparseLU(H)
    t1 = time.perf_counter()
    U = lu.solve(F)
    t2 = time.perf_counter()
    assert np.isfinite(U).all()
    R = F.shape[1]
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    return {"value": R / (t2 - t0), "unit": "RHS/s", "cores": cores, "kind": "oracle",
            "value_solve_only": R / (t2 - t1), "workload": wl.name,
            "factor_s": t1 - t0, "solve_s": t2 - t1,
            "sample": f"oracle global direct solve (scipy SuperLU with threaded BLAS, "
                      f"complex128) of the {wl.n[0]}^3 layered-dipping workload of "
                      f"the same recipe (8 ppw, {wl.pml}-pt PML) with R={R} surface "
                      f"point sources; assembly+factorization {t1 - t0:.1f}s, solves "
                      f"{t2 - t1:.1f}s; value = R / (factorization + solves). The "
                      "oracle cannot factor the 200^3 grid on the host in bounded time."}, U


def same_input_gpu(pt, torch, U_oracle):
    """The GPU path on the oracle's own input (the layered recipe at 32^3, all
    of its sources), both precisions: RHS/s including the factorization (as
    the oracle's value) and for the solves alone, and each column's error
    against the oracle's solution."""
    import numpy as np
    from helm_inputs import workload
    wl = workload("layered-32")
    out = {"workload": wl.name, "rhs": len(wl.sources)}
    R = len(wl.sources)
    for prec in ("mixed", "fp64"):
        kw = dict(gmres_tol=1e-10) if prec == "fp64" else dict(MIXED_KW)
        # one untimed run first: code objects loaded, device warm
        s = pt.Solver(wl.m(), wl.h, wl.omega, wl.pml, wl.n_layers, precision=prec,
                      pml_local=wl.pml_local, pml_C=wl.pml_C, **kw)
        s.solve_points(wl.sources)
        s.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = pt.Solver(wl.m(), wl.h, wl.omega, wl.pml, wl.n_layers, precision=prec,
                      pml_local=wl.pml_local, pml_C=wl.pml_C, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        u = s.solve_points(wl.sources)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        uh = u.cpu().numpy().reshape(R, -1).T
        err = np.linalg.norm(uh - U_oracle, axis=0) / np.linalg.norm(U_oracle, axis=0)
        out[prec] = {"value": R / (t2 - t0), "value_solve_only": R / (t2 - t1),
                     "factor_s": t1 - t0, "solve_s": t2 - t1,
                     "err_vs_oracle_max": float(err.max())}
        s.close()
    return out


def serve_bench(args, torch, pt):
    """Request server on three resident factorizations of one 160^3 layered
    model (16-pt PML, L = 16) at 6, 8 and 10 points per wavelength; requests
    of R ~ U{1..128} surface sources at a random model, Poisson arrivals.
    Phase 1 offers the nominal 50 requests/s (far above one GPU's capacity,
    so it measures saturated throughput and queueing latency); phase 2
    offers 75% of the capacity measured in phase 1."""
    from helm_inputs import poisson_requests, serving_models
    from paper_1801_08655_amd.serving import Server
    models = serving_models()
    srv = Server(slots=args.slots)
    solvers, factor_s = [], []
    for w in models:
        log(f"[serve] factorize {w.name}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = pt.Solver(w.m(), w.h, w.omega, w.pml, w.n_layers, precision="mixed",
                      pml_local=w.pml_local, pml_C=w.pml_C, **MIXED_KW)
        torch.cuda.synchronize()
        factor_s.append(time.perf_counter() - t0)
        srv.add_model(s)
        solvers.append(s)
    cands = models[0].sources
    for mid in range(len(models)):          # warm-up: graphs, Krylov basis
        srv.submit(mid, cands[:1]).wait()

    def run(reqs, label):
        log(f"[serve] {label}: {len(reqs)} requests")
        t0 = time.perf_counter()
        pending = []
        for r in reqs:
            dt = r.t - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            pending.append(srv.submit(r.model, r.sources))
        infos = []
        for q in pending:
            _, inf = q.wait()
            infos.append(inf)
            q.u = q._result = None           # release the output volume
        total = time.perf_counter() - t0
        lat = [i["latency_ms"] for i in infos]
        cols = sum(len(r.sources) for r in reqs)
        log(f"[serve] {label}: {cols} columns in {total:.1f}s")
        return {"requests": len(reqs), "columns": cols, "wall_s": total,
                "rhs_per_s": cols / total,
                "offered_req_per_s": len(reqs) / max(reqs[-1].t, 1e-9),
                "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99),
                               "mean": sum(lat) / len(lat)},
                "queue_ms_p50": percentile([i["t_first_ms"] - i["t_submit_ms"]
                                            for i in infos], 50),
                "est_error_max": max(i["est_error_max"] for i in infos),
                "rel_residual_max": max(i["rel_residual_max"] for i in infos),
                "all_ok": all(i["status"] == 0 for i in infos)}

    nominal = run(poisson_requests(args.serve_requests, 50.0, len(models), cands, seed=1806),
                  "nominal rate")
    mean_r = 64.5
    rate = 0.75 * nominal["rhs_per_s"] / mean_r
    scaled = run(poisson_requests(args.serve_requests, rate, len(models), cands, seed=1807),
                 "75% of capacity")
    # an idle server: one single-source request per model at a time (the
    # lane runs it at width 1)
    idle = []
    for mid in range(len(models)):
        _, inf = srv.submit(mid, cands[17:18]).wait()
        idle.append(inf["latency_ms"])
    st = srv.stats()
    srv.close()
    for s in solvers:
        s.close()
    out = {
        "metric": "serving: request latency p50/p99 and solved RHS/s, 3 resident models",
        "value": scaled["rhs_per_s"], "unit": "RHS/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "c64 fronts + f64 refinement",
        "data": "synthetic",
        "config": {"workload": "serving 3 x layered-160 (ppw 6/8/10), 16-pt PML, L=16",
                   "slots_per_model": args.slots, "rel_err_target": 1e-6,
                   "requests_per_phase": args.serve_requests},
        "factor_s": factor_s,
        "nominal_rate_50_per_s": nominal,
        "scaled_rate": dict(scaled, rate_req_per_s=rate),
        "idle_single_source_latency_ms": idle,
        "server": st,
    }
    print(json.dumps(out), flush=True)


def depth_rates_bench(args, torch, pt):
    """Per-depth rates of the substitution GEMMs in one interior layer's
    local solve of R columns: the first solve of the layer measures every
    tile width of each depth's launches (HELM_FLAG_AUTOTUNE, start and stop
    events recorded by each launch); the kept width's time against the
    depth's algorithmic flops (8 real flops per complex multiply-add:
    sum (s + b) s forward, sum b s backward, times R)."""
    from helm_inputs import workload
    wl = workload(args.workload)
    s = pt.Solver(wl.m(), wl.h, wl.omega, wl.pml, wl.n_layers, precision="mixed",
                  pml_local=wl.pml_local, pml_C=wl.pml_C, max_rhs=args.rhs,
                  flags=pt._lib.HELM_FLAG_AUTOTUNE)
    layer = wl.n_layers // 4
    _, _, lo, hi = s.layer_info(layer)
    r = torch.randn((args.rhs, hi - lo + 1, wl.n[1], wl.n[0]), dtype=torch.complex128,
                    device="cuda")
    s.layer_solve(layer, r)   # the first solve of the layer set measures the widths
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        s.layer_solve(layer, r)
    torch.cuda.synchronize()
    solve_ms = (time.perf_counter() - t0) / 3 * 1e3
    col = {1: 0, 16: 1, 32: 2, 64: 3}
    rows = []
    for c in sorted(s.tile_choices(), key=lambda c: c["depth"]):
        if c["set_layers"] != 1 or c["k"] != args.rhs:
            continue
        tf = c["t_fwd_us"][col[c["fwd_bn"]]]
        tb = c["t_bwd_us"][col[c["bwd_bn"]]]
        gf = 8.0 * args.rhs * c["fwd_elems"] / 1e9
        gb = 8.0 * args.rhs * c["bwd_elems"] / 1e9
        rows.append({"depth": c["depth"], "fronts": c["fronts"], "mean_s": c["mean_s"],
                     "mean_b": c["mean_b"], "fwd_bn": c["fwd_bn"], "fwd_us": tf,
                     "fwd_gflop": gf, "fwd_tflops": gf / tf * 1e3 if tf > 0 else None,
                     "bwd_bm": c["bwd_bm"], "bwd_bn": c["bwd_bn"], "bwd_us": tb,
                     "bwd_gflop": gb, "bwd_tflops": gb / tb * 1e3 if tb > 0 else None,
                     "tuned": c["tuned"]})
    s.close()
    print(json.dumps({"metric": "per-depth substitution GEMM rates of one layer solve",
                      "workload": wl.name, "layer": layer, "rhs": args.rhs,
                      "layer_solve_ms": solve_ms, "depths": rows}), flush=True)


def rhs_scaling_bench(args, torch, pt):
    """Throughput against the batch width R on one mixed-precision
    factorization: R columns share every layer solve (the substitution GEMMs
    take them as the N dimension), so RHS/s grows with R until the
    substitutions reach the matrix-core bound."""
    from helm_inputs import workload
    wl = workload(args.workload)
    m = wl.m()
    log(f"[rhs-scaling] factorize {wl.name}")
    s = pt.Solver(m, wl.h, wl.omega, wl.pml, wl.n_layers, precision="mixed",
                  **MIXED_KW, pml_local=wl.pml_local, pml_C=wl.pml_C, max_rhs=64,
                  flags=0 if args.no_autotune else pt._lib.HELM_FLAG_AUTOTUNE)
    points = []
    for R in (1, 2, 4, 8, 16, 32, 64):
        srcs = wl.point_sources(R)
        _, info, total, lat = timed_solves(s, srcs, args.steps, args.warmup, torch)
        pt_ = {"rhs": R, "rhs_per_s": R * args.steps / total,
               "ms_per_step": 1e3 * total / args.steps,
               "layer_solves_per_step": info["layer_solves"],
               "ms_per_layer_solve": 1e3 * total / args.steps / max(1, info["layer_solves"]),
               "gmres_iters": info["gmres_iters"], "est_error_max": info["est_error_max"],
               "ir_width": info["ir_width"]}
        log(f"[rhs-scaling] {pt_}")
        points.append(pt_)
    s.close()
    print(json.dumps({"metric": "RHS/s against the batch width R (mixed)",
                      "unit": "RHS/s", "steps": args.steps, "warmup": args.warmup,
                      "data": "synthetic", "config": {"workload": wl.name, "n": list(wl.n),
                                                      "layers": wl.n_layers},
                      "points": points}), flush=True)


def batch_bench(args, torch, pt):
    """Independent problems in one batched call: n ~ U{64..160} cubes with an
    8-pt PML, smooth random media (c in [0.8, 1.2]), 10 ppw, L = round(n/10),
    R ~ U{1..256} surface sources each; complex64 fronts with FP64
    refinement, measured tile widths.  The throughput counts the whole call:
    every factorization and every solve (the problems do not all fit the
    device at once, so factorizations are part of the stream of work)."""
    from helm_inputs import batched_problems
    from paper_1801_08655_amd.batch import Problem, solve_batch
    wls = batched_problems(count=args.batch_count)
    log(f"[batch] building {len(wls)} models")
    probs = [Problem(w.m(), w.h, w.omega, w.pml, w.n_layers, w.sources) for w in wls]
    log("[batch] solving")
    res, summ = solve_batch(probs, slots=args.slots, max_resident=args.batch_resident,
                            host_output=True, precision="mixed",
                            pml_local=4, **MIXED_KW,
                            flags=pt._lib.HELM_FLAG_AUTOTUNE)
    infos = [r[1] for r in res]
    out = {
        "metric": "batched independent problems: solved RHS/s incl. factorization",
        "value": summ["rhs_per_s"], "unit": "RHS/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "c64 fronts + f64 refinement",
        "data": "synthetic",
        "config": {"workload": f"{len(wls)} problems, n in [64,160], 8-pt PML, smooth random "
                               "c in [0.8,1.2], 10 ppw, L=round(n/10), R in [1,256]",
                   "slots_per_problem": args.slots, "max_resident": args.batch_resident,
                   "n": [w.n[0] for w in wls],
                   "rhs": [len(w.sources) for w in wls]},
        "summary": summ,
        "all_ok": all(i["status"] == 0 for i in infos),
        "failed": {i: inf["status"] for i, inf in enumerate(infos) if inf["status"] != 0},
        "est_error_max": max(i["est_error_max"] for i in infos),
        "rel_residual_max": max(i["rel_residual_max"] for i in infos),
        "factor_ms": [i["factor_ms"] for i in infos],
        "done_ms": [i["t_done_ms"] for i in infos],
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the solver runs on exactly one GPU; sharding the layers over "
              "several GPUs is a design, not a measured path", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1801_08655_amd as pt
    from helm_inputs import workload
    from helm_inputs.models import checksum

    if args.serve:
        serve_bench(args, torch, pt)
        return
    if args.rhs_scaling:
        rhs_scaling_bench(args, torch, pt)
        return
    if args.depth_rates:
        depth_rates_bench(args, torch, pt)
        return
    if args.batch:
        if args.slots == 32:
            args.slots = 64
        batch_bench(args, torch, pt)
        return
    log("[calibration] attainable device rates")
    attain = pt.device_peaks(0)
    wl = workload(args.workload)
    m = wl.m()
    srcs = wl.point_sources(args.rhs)
    R = len(srcs)
    if args.copy_calibration_mib:
        x = torch.ones(args.copy_calibration_mib << 17, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    # The factorizations and the one-column probe time every kernel class.
    # The timed steps run with the default flags (substitution sequences
    # replayed from captured HIP graphs, no timing events); a separate step
    # after them times the forward substitution GEMM launches (the roofline's
    # kernel) with events, launch by launch.
    tune = 0 if args.no_autotune else pt._lib.HELM_FLAG_AUTOTUNE
    flags = (pt._lib.HELM_FLAG_PROFILE if args.profile else 0) | tune
    step_flags = tune
    # (every refinement step of the profiled pass at the full batch width, so
    # that the timed class holds the 64-column launches only)
    prof_flags = (pt._lib.HELM_FLAG_PROFILE_FWD if args.profile else 0) | tune | \
        pt._lib.HELM_FLAG_NO_NARROW
    common = dict(pml_local=wl.pml_local, pml_C=wl.pml_C, max_rhs=64, flags=flags)
    mixed_kw = dict(MIXED_KW)
    if args.inner_tol is not None:
        mixed_kw["inner_tol"] = args.inner_tol
    extra = {}

    log(f"[mixed] factorize {wl.name}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = pt.Solver(m, wl.h, wl.omega, wl.pml, wl.n_layers, precision="mixed",
                  **mixed_kw, **common)
    torch.cuda.synchronize()
    factor_s = time.perf_counter() - t0
    log(f"[mixed] factorized in {factor_s:.2f}s; warmup {args.warmup}, steps {args.steps}")
    fstats = s.kernel_stats(reset=True)
    finfo = s.factor_info()
    s.set_options(flags=step_flags)
    u, info, total, lat = timed_solves(s, srcs, args.steps, args.warmup, torch)
    value = R * args.steps / total
    log(f"[mixed] {value:.2f} RHS/s ({1e3 * total / args.steps:.0f} ms per step)")
    # the profiled step (forward GEMM launches timed one by one)
    s.set_options(flags=prof_flags)
    s.kernel_stats(reset=True)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    u, _ = s.solve_points(srcs, info=True, out=u)
    torch.cuda.synchronize()
    tp = time.perf_counter() - tp
    kstats = s.kernel_stats()
    s.set_options(flags=flags)
    # the same step with the 64 solution volumes handed back to host memory
    # (pinned): the PCIe-inclusive rate, reported beside the HBM-resident one
    u_host = torch.empty(u.shape, dtype=u.dtype, pin_memory=True)
    torch.cuda.synchronize()
    t_copy = time.perf_counter()
    u_host.copy_(u)
    t_copy = time.perf_counter() - t_copy
    pcie = {"d2h_s": t_copy, "bytes": u.numel() * u.element_size(),
            "rhs_per_s": R / (total / args.steps + t_copy)}
    rl = roofline({k: v for k, v in kstats.items() if k.startswith("solve_")}, "mixed",
                  wl.name)
    rl["profiled_step_ms"] = 1e3 * tp
    small = small_k_probe(s, wl, torch)
    s.close()
    del s
    del u   # kept in u_host: the FP64 handle needs the room
    torch.cuda.empty_cache()
    # FP64 reference after the mixed handle is released, so that the
    # headline factorization runs in a fresh process (an allocation right
    # after a ~130 GB release takes seconds of host time)
    u_ref = None
    fp64 = None
    fp64_loose = None
    if not args.no_fp64:
        log(f"[fp64] factorize {wl.name}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s64 = pt.Solver(m, wl.h, wl.omega, wl.pml, wl.n_layers, precision="fp64",
                        gmres_tol=1e-10, **common)
        torch.cuda.synchronize()
        f64_factor = time.perf_counter() - t0
        log(f"[fp64] factorized in {f64_factor:.2f}s; solving R={R}")
        extra["fp64_factor_kernels"] = s64.kernel_stats(reset=True)
        extra["fp64_factor_info"] = s64.factor_info()
        s64.set_options(flags=step_flags)
        u_ref, info64, tot64, lat64 = timed_solves(s64, srcs, args.fp64_steps,
                                                   args.fp64_warmup, torch)
        fp64 = {"value": R * args.fp64_steps / tot64, "factor_s": f64_factor,
                "gmres_tol": 1e-10,
                "ms_per_step": 1e3 * tot64 / args.fp64_steps,
                "gmres_iters": info64["gmres_iters"],
                "rel_residual_max": info64["rel_residual_max"]}
        log(f"[fp64] {fp64}")
        # the FP64 path stopped early: the fastest such run whose error still
        # meets the mixed path's target (1e-6 for every column) gives the
        # speed-up of the precision alone, at equal accuracy
        loose = []
        for tol in (float(x) for x in args.fp64_loose_tol.split(",")):
            s64.set_options(gmres_tol=tol)
            u_l, info_l, tot_l, _ = timed_solves(s64, srcs, 1, 0, torch)
            d = (u_l - u_ref).reshape(R, -1).norm(dim=1) / u_ref.reshape(R, -1).norm(dim=1)
            loose.append({"value": R / tot_l, "gmres_tol": tol,
                          "gmres_iters": info_l["gmres_iters"],
                          "err_vs_fp64_max": float(d.max())})
            log(f"[fp64 loose] {loose[-1]}")
            del u_l
        ok = [x for x in loose if x["err_vs_fp64_max"] <= mixed_kw["err_target"]]
        fp64_loose = max(ok, key=lambda x: x["value"]) if ok else \
            min(loose, key=lambda x: x["gmres_tol"])
        extra["fp64_at_tolerances"] = loose
        s64.close()
        del s64
        torch.cuda.empty_cache()

    err = None
    if u_ref is not None:
        u = u_host.cuda()
        d = (u - u_ref).reshape(R, -1).norm(dim=1) / u_ref.reshape(R, -1).norm(dim=1)
        err = float(d.max())
        del u, u_host, u_ref
        torch.cuda.empty_cache()
    rl["attainable_peak"] = attain["mfma_f32_tflops"]
    rl["frac_of_attainable"] = rl["achieved"] / attain["mfma_f32_tflops"]
    for name in ("solve_fwd_gemm", "solve_bwd_gemm"):
        small[name]["frac_of_attainable_read"] = small[name]["GB/s"] / attain["hbm_read_gbps"]
    # factorization: the LU count over the time of every factor kernel
    fk_ms = sum(v["total_ms"] for k, v in fstats.items() if k.startswith("factor_"))
    sw = fstats.get("factor_sweep_gemm", {})
    factor_roofline = {
        "lu_flops": finfo["lu_flops"], "gj_flops_executed": finfo["gj_flops"],
        "kernel_s": fk_ms * 1e-3,
        "achieved_tflops": finfo["lu_flops"] / max(fk_ms * 1e-3, 1e-12) / 1e12,
        "frac": finfo["lu_flops"] / max(fk_ms * 1e-3, 1e-12) / PEAK["fp32_mfma"],
        "executed_tflops": finfo["gj_flops"] / max(fk_ms * 1e-3, 1e-12) / 1e12,
        "sweep_gemm_s": sw.get("total_ms", 0.0) * 1e-3,
        "sweep_gemm_lu_share_tflops": sw.get("flops", 0.0) / max(sw.get("total_ms", 0.0)
                                                                 * 1e-3, 1e-12) / 1e12,
        "pivot_min": finfo["pivot_min"], "pivot_max": finfo["pivot_max"],
        "pivot_growth": finfo["pivot_growth"],
        # wall time of helm_factorize by phase (host plans, device set-up,
        # numeric factorization, single-layer launch lists)
        "phases_s": {"symbolic": finfo["symbolic_seconds"], "setup": finfo["setup_seconds"],
                     "numeric": finfo["seconds"], "lists": finfo["lists_seconds"]}}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 fronts + f64 refinement",
        "data": "synthetic",
        "config": {"workload": wl.name, "n": list(wl.n), "pml": wl.pml,
                   "layers": wl.n_layers, "pml_local": wl.pml_local, "rhs": R,
                   "ppw": wl.ppw, "omega": wl.omega, "precision": "mixed",
                   "model_checksum": checksum(m)},
        "latency_ms": {"p50": 1e3 * percentile(lat, 50), "p99": 1e3 * percentile(lat, 99)},
        "err_vs_fp64_max": err,
        "fp64": fp64,
        "speedup_vs_fp64": (value / fp64["value"]) if fp64 else None,
        "fp64_at_matched_accuracy": fp64_loose,
        "speedup_vs_fp64_matched_accuracy": (value / fp64_loose["value"]) if fp64_loose
        else None,
        "factor_s": factor_s,
        "factor": factor_roofline,
        "gmres_iters": info["gmres_iters"],
        "ir_steps": info["ir_steps"],
        "rel_residual_max": info["rel_residual_max"],
        "est_error_max": info["est_error_max"],
        "ir_residual": info["ir_residual"],
        "ir_gmres_iters": info["ir_gmres_iters"],
        "ir_width": info["ir_width"],
        "narrow_products": info["narrow_products"],
        "layer_solves_per_step": info["layer_solves"],
        "pcie_inclusive": pcie,
        "roofline": rl,
        "hbm_bound_k1": small,
        "attainable": attain,
        "kernels": kstats,
        "factor_kernels": fstats,
    }
    out.update(extra)
    if not args.no_cpu_baseline:
        log("[cpu] oracle baseline")
        cb, U32 = cpu_baseline()
        out["cpu_baseline"] = cb
        log("[gpu] the oracle's input on the GPU")
        same = same_input_gpu(pt, torch, U32)
        same["mixed_over_oracle"] = same["mixed"]["value"] / cb["value"]
        same["fp64_over_oracle"] = same["fp64"]["value"] / cb["value"]
        out["same_input"] = same
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

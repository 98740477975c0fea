#!/usr/bin/env python3
"""Benchmark: DPP solve time and DOF/s to 1e-8 relative residual on one MI355X.

One step = one solve of the assembled CG-VMS four-field system from a zero
initial guess to ||f - K x|| <= 1e-8 ||f|| (flexible GMRES with the Schur
fieldsplit / multigrid preconditioner).  Assembly and preconditioner setup are
timed separately, as the paper reports assembly and solver times separately.
Inputs are synthetic (seeded log-normal permeability fields and the
manufactured-solution boundary data of the paper's 3D study), already resident
in HBM when the timed region starts.

Default workload: the 96^3 log-normal box (7,301,384 DOF), FP64; the same line
carries the mixed-precision (FP32 inner solve, FP64 refinement) timing, every
field's error against the CPU oracle's solution of the same system, the
roofline of the dominant kernel and the oracle's own solve rate on the host.

Prints one JSON line (metric, value, ..., roofline, cpu_baseline).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "DPP solve time & DOF/s to 1e-8 rel residual; SpMV HBM GB/s vs peak"
WORKLOADS = {
    "c2_3d64": "3D unit cube, 64^3 hexahedra x 6 Kuhn tetrahedra (65^3 nodes), CG-VMS P1, "
               "8 unknowns/node = 2,197,000 DOF; k1=1, k2=1e-2, beta=mu=1; manufactured-solution "
               "pressure data on all faces; FP64 flexible GMRES + Schur fieldsplit + MG V-cycles",
    "c3_3d96_grf": "3D unit cube 96^3 x 6 tetrahedra (97^3 nodes) = 7,301,384 DOF; log-normal "
                   "per-hex k1, k2 (Gaussian random field, correlation length 0.1, seeds 1001/1002)",
    "c5_3d48_grf": "3D unit cube 48^3 x 6 tetrahedra (49^3 nodes) = 941,192 DOF; log-normal k1, k2",
    "c1_2d16": "2D unit square 16^2 x 2 triangles (289 nodes) = 1,734 DOF; k1=1, k2=0.1, beta=mu=1",
    "c2f_3d64_flux": "the 64^3 workload with velocity (flux) faces: network 1 prescribes u.n on the "
                     "x faces, network 2 on the y faces and z = 0 (essential), pressures weakly "
                     "on the rest",
    "c2p_3d64_pureflux": "the 64^3 workload with velocity faces on every face of both networks "
                         "(singular K: consistent right-hand side, pressures normalised to "
                         "int p1 = 0)",
    "h2_3d64_q1": "3D unit cube, 64^3 hexahedra with Q1 elements (65^3 nodes, the HEX columns of the "
                  "3D study) = 2,197,000 DOF; k1=1, k2=1e-2, beta=mu=1; manufactured-solution pressure "
                  "data on all faces",
    "h3_3d96_grf_q1": "3D unit cube 96^3 hexahedra with Q1 elements = 7,301,384 DOF; log-normal per-hex "
                      "k1, k2 (seeds 1001/1002)",
    "g2_3d20_dg": "3D unit cube 20^3 x 6 tetrahedra with DG-VMS (discontinuous P1, 4 vertex slots per "
                  "simplex) = 1,536,000 DOF (the largest TET row of the DG h-size study); k1=1, k2=0.1, "
                  "beta=mu=1; manufactured-solution pressure data on all faces",
    "g1_2d160_dg": "2D unit square 160^2 x 2 triangles with DG-VMS = 921,600 DOF (the largest TRI row of "
                   "the DG h-size study); k1=1, k2=0.1, beta=mu=1",
    "c4_batch64": "64 independent 2D unit-square instances, n ~ U{32..256} cells per side (seed 2024), "
                  "beta ~ logU[0.1,10], k2/k1 ~ logU[1e-3,1]; one batched launch per phase",
}
PRECISION = {0: "f64", 1: "f64+f32 refinement", 2: "f64 Krylov, f32 preconditioner"}


# profiling families that are one kernel each (the roofline reports the one
# with the largest share of the solve; the others group several kernels)
SINGLE_KERNEL_FAMILIES = ("spmv_K", "cheb_S_l0", "resid_S_l0", "schur_rhs", "schur_vel", "dg_vel")


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("mg.hip", "ops.hip", "krylov.hip", "common.h", "stencil.h", "mvec.h", "batch.hip", "batch.h",
              "dg.hip"):
        with open(os.path.join(ROOT, "paper_1808_08328_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_name(family, dim, pc, flux=False, dg=False):
    """rocprofv3 name of a single-kernel family's FP64 kernel (flux: the
    instances for problems with velocity faces; dg: DG-VMS problems)."""
    if dg:
        return {"spmv_K": "k_dg_spmv<%d>", "dg_vel": "k_dg_vcheb<%d, double>"}[family] % dim
    if family in ("cheb_S_l0", "resid_S_l0"):
        lanes, sym = pc.shape(0)
        k = "k_cheb" if family == "cheb_S_l0" else "k_lspmv"
        return "%s<%d, double, double, %d, %s, true>" % (k, dim, lanes, "true" if sym else "false")
    bc = "true" if flux else "false"
    # the K product: node pairs without velocity faces, one node per thread with them
    return {"spmv_K": "k_spmv_K1<%d, double>" if flux else "k_spmv_K<%d, double>",
            "schur_rhs": "k_schur_rhs<%d, double, double, " + bc + ">",
            "schur_vel": "k_schur_vel<%d, double, double, " + bc + ">"}[family] % dim


def stencil_tag(prob):
    """Template tag of the library's stencil kernels: the dimension, plus 10
    for Q1 box cells."""
    return prob.dim + (10 if getattr(prob, "elem", "p1") == "q1" else 0)


def measured_traffic(workload, family):
    """HBM bytes per launch of a single-kernel family on a workload, from the
    committed rocprofv3 counter summary (profiles/traffic_counters.json), if it
    was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_sha") != kernel_source_sha():
        return None
    ent = d.get("workloads", {}).get(workload, {}).get("families", {}).get(family)
    return None if ent is None else ent.get("bytes_per_launch")


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def oracle_leg(prob, gpu_iters, sample_iters, solutions, ref_rtol=1e-11):
    """The CPU oracle (FP64 numpy/scipy + its OpenMP C loops; its own
    assembly, fieldsplit and flexible GMRES of the same definition) on the
    same system.

    cpu_baseline: the oracle's FGMRES from x = 0 toward 1e-8 with its OpenMP
    CSR product as the operator, timed over at most `sample_iters` iterations
    (a bounded sample), scaled to the iterations it needs when it stops early.
    Reference: the same FGMRES continued (restarted from its iterate) to
    ref_rtol; each GPU solution in `solutions` gets its per-field error against
    it and the oracle's own residual ||f - K_oracle x|| / ||f||."""
    import numpy as np

    from oracle import dpp as odpp
    from oracle import solver as osolver
    dg = getattr(prob, "elem", "p1") == "dg"
    t0 = time.perf_counter()
    if dg:
        from oracle import dg as odg
        S = odg.assemble(prob)
        t1 = time.perf_counter()
        F = odg.FieldSplitDG(S, prob)
        fs = odg.fields(prob.dim, S.S)
    else:
        S = odpp.assemble(prob)
        t1 = time.perf_counter()
        F = osolver.FieldSplit(S)
        fs = odpp.fields(prob.dim, S.N)
    t2 = time.perf_counter()
    log("oracle assembly %.1f s, fieldsplit setup %.1f s" % (t1 - t0, t2 - t1))
    mv = lambda v: odpp.spmv(S.K, v)
    x, its, res = osolver.fgmres(S.K, S.f, F.apply, restart=30, rtol=1e-8, maxiter=sample_iters,
                                 matvec=mv)
    t3 = time.perf_counter()
    t_sample = t3 - t2
    full = res <= 1e-8
    n_dof = S.K.shape[0]
    log("oracle sample: %d iterations in %.1f s (rel. residual %.2e)" % (its, t_sample, res))
    # the reference continues restart cycle by restart cycle (the same
    # iteration as one call), with a line after each
    xr, its2, res2 = x, 0, res
    while res2 > ref_rtol and its2 < 600:
        xr, k, res2 = osolver.fgmres(S.K, S.f, F.apply, restart=30, rtol=ref_rtol, maxiter=30,
                                     x0=xr, matvec=mv)
        its2 += k
        log("oracle reference: %d more iterations, rel. residual %.2e" % (its2, res2))
        if k == 0:
            break
    # a sample stopped at its bound is scaled to the iteration count of the
    # GPU solve (the same preconditioner definition; the oracle orthogonalises
    # by modified Gram-Schmidt, so the counts can differ by rounding)
    its_full = its if full else gpu_iters
    t_est = t_sample if full else t_sample / max(its, 1) * its_full
    fn = np.linalg.norm(S.f)
    errs = {"reference": "CPU oracle FGMRES (FP64) to rel. residual %.0e (reached %.2e)"
                         % (ref_rtol, res2)}
    for name, xg in solutions.items():
        errs[name] = {f: float(np.linalg.norm(xg[fs[f]] - xr[fs[f]]) / np.linalg.norm(xr[fs[f]]))
                      for f in ("u1", "p1", "u2", "p2")}
        errs[name]["oracle_residual"] = float(np.linalg.norm(S.f - mv(xg)) / fn)
    threads = odpp.threads()
    pc_kind = "block-Jacobi Chebyshev, S_q steps, V-cycles" if dg else "V-cycles"
    base = {
        "value": n_dof / t_est, "unit": "DOF/s", "cores": threads, "kind": "oracle",
        "sample": ("oracle FGMRES solve of the same %d-DOF system to 1e-8 from x = 0: %d iterations "
                   "in %.2f s (assembly %.1f s and fieldsplit setup %.1f s not counted); CSR "
                   "products on %d OpenMP threads, %s and vector updates in numpy/scipy"
                   % (n_dof, its, t_sample, t1 - t0, t2 - t1, threads, pc_kind)) if full else
                  ("first %d oracle FGMRES iterations on the same %d-DOF system (%.2f s), scaled to "
                   "the %d iterations of the GPU solve to 1e-8; CSR products on %d OpenMP threads, "
                   "%s and vector updates in numpy/scipy"
                   % (its, n_dof, t_sample, its_full, threads, pc_kind)),
        "solve_s": t_est, "iters": its_full, "gpu_iters": gpu_iters,
    }
    return base, errs


def oracle_batch_leg(probs, budget_s):
    """cpu_baseline of the batch: the oracle solves instances one after
    another (FGMRES to 1e-8 with its OpenMP CSR product) until `budget_s` of
    solve time is spent; DOF/s over the instances it finished."""
    from oracle import dpp as odpp
    from oracle import solver as osolver
    dof, t, done = 0, 0.0, 0
    for pr in probs:
        S = odpp.assemble(pr)
        F = osolver.FieldSplit(S)
        t0 = time.perf_counter()
        x, its, res = osolver.fgmres(S.K, S.f, F.apply, restart=30, rtol=1e-8, maxiter=400,
                                     matvec=lambda v: odpp.spmv(S.K, v))
        t += time.perf_counter() - t0
        dof += S.K.shape[0]
        done += 1
        if t >= budget_s:
            break
    threads = odpp.threads()
    return {"value": dof / t, "unit": "DOF/s", "cores": threads, "kind": "oracle",
            "sample": ("the first %d of the %d instances solved one after another by the oracle's "
                       "FGMRES to 1e-8 (%d DOF, %.2f s of solve time; assembly and setup not "
                       "counted); CSR products on %d OpenMP threads" % (done, len(probs), dof, t, threads)),
            "solve_s": t}


def measured_copy_gbs(torch):
    """HBM bandwidth of a plain device copy (1 GiB read + 1 GiB written), the
    practical ceiling next to the 8 TB/s peak."""
    src = torch.ones(128 * 1024 * 1024, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * src.numel() * 8 * 5 / (e0.elapsed_time(e1) * 1e6)
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def profiled(dpp, run, steps):
    """Per-family HIP-event timings of `steps` runs -> {family: stats}."""
    dpp.profile_enable(True)
    for _ in range(steps):
        run()
    import torch
    torch.cuda.synchronize()
    prof = dpp.profile_read()
    dpp.profile_enable(False)
    tot_ms = sum(v[1] for v in prof.values())
    kernels = {}
    for name, (n, t, by) in prof.items():
        if n:
            kernels[name] = {"launches_per_solve": n / steps, "ms_per_solve": t / steps,
                             "avg_us": 1e3 * t / n, "GBps": by / (t * 1e6) if t > 0 else None,
                             "share": t / tot_ms if tot_ms else None,
                             "_raw": (n, t, by)}
    return kernels


def roofline(kernels, candidates, copy_gbs, name_of, workload):
    """Roofline object of the candidate family with the largest time share;
    traffic: its measured HBM bytes per launch on this workload (counters)."""
    dom = max((k for k in kernels if k in candidates), key=lambda k: kernels[k]["ms_per_solve"])
    n, t, by = kernels[dom]["_raw"]
    achieved = by / (t * 1e6)
    per_launch = by / n
    traffic = measured_traffic(workload, dom)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
            "traffic_over_algorithmic": round(traffic / per_launch, 3) if traffic else None,
            "kernel": dom, "kernel_name": name_of(dom),
            "algorithmic_bytes_per_launch": per_launch, "avg_launch_us": 1e3 * t / n,
            "copy_ceiling": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)}


def strip_raw(kernels):
    return {k: {a: b for a, b in v.items() if a != "_raw"} for k, v in kernels.items()}


def timed(torch, run, steps, warmup):
    """Mean wall time (ms) of `steps` runs after `warmup` untimed ones, with
    a device synchronisation on both sides; returns (ms, last result)."""
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    tb = time.perf_counter()
    out = None
    for _ in range(steps):
        out = run()
    torch.cuda.synchronize()
    return (time.perf_counter() - tb) * 1e3 / steps, out


BATCH_FAMILIES = ("batch_spmv_K", "batch_cheb_S_l0")


def bench_batch(args, torch, I, dpp):
    """64 uneven 2D instances: batched solve vs the same instances solved one
    after another with the single-problem path."""
    probs = I.batch_configs(64, seed=2024)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B = dpp.assemble_batch(probs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    opts = dict(rtol=1e-8, precision=args.precision, use_graph=1)
    ms, (x, st) = timed(torch, lambda: B.solve(**opts), args.steps, args.warmup)
    log("batched solve %.2f ms" % ms)
    line = {
        "metric": METRIC, "value": B.n_dof / (ms / 1e3), "unit": "DOF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == 0 else "f64/f32",
        "data": "synthetic",
        "config": {"workload": "c4_batch64", "description": WORKLOADS["c4_batch64"],
                   "n_dof": B.n_dof, "instances": len(probs), "rtol": 1e-8,
                   "precision": PRECISION[args.precision], "graph": True},
        "iters_max": max(s.iters for s in st), "iters_min": min(s.iters for s in st),
        "all_converged": all(s.converged for s in st),
        "setup_ms": (t1 - t0) * 1e3, "lanes_per_level": B.lanes(),
    }
    if args.precision == 0:
        # the other precisions of the same batch, timed the same way
        for prec in (2, 1):
            try:
                msp, (_, stp) = timed(torch, lambda: B.solve(**{**opts, "precision": prec}),
                                      args.steps, args.warmup)
                line["precision_%d" % prec] = {
                    "precision": PRECISION[prec], "ms_per_step": msp, "value": B.n_dof / (msp / 1e3),
                    "iters_max": max(s.iters for s in stp), "refinements_max": max(s.refinements for s in stp)}
            except dpp.DppError as e:
                line["precision_%d" % prec] = {"error": str(e)}
    # reference: the single-problem FP64 path, instance by instance
    singles = []
    for pr in probs:
        P = dpp.assemble_problem(pr)
        singles.append((P, P.setup_precond()))
    for P, pc in singles[:4]:
        P.solve(pc, rtol=1e-8)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for P, pc in singles:
        P.solve(pc, rtol=1e-8)
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - ts) * 1e3
    del singles
    line["sequential_single_fp64_ms"] = seq_ms
    line["speedup_vs_sequential"] = seq_ms / ms
    if not args.no_profile:
        copy_gbs = measured_copy_gbs(torch)
        # the profiled runs replay no graphs (each launch is bracketed by events)
        kernels = profiled(dpp, lambda: B.solve(**{**opts, "use_graph": 0}), args.steps)
        line["roofline"] = roofline(kernels, BATCH_FAMILIES, copy_gbs,
                                    lambda k: {"batch_spmv_K": "kb_spmv_K<2, double, false>",
                                               "batch_cheb_S_l0": "kb_cheb<2, double, double, L> "
                                               "(finest levels; L = lanes per row)"}[k], args.config)
        line["kernels"] = strip_raw(kernels)
    else:
        line["roofline"] = None
    if not args.no_cpu_baseline:
        log("oracle batch sample")
        line["cpu_baseline"] = oracle_batch_leg(probs, args.cpu_budget)
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c3_3d96_grf", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", type=int, default=0, choices=[0, 1, 2])
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision timing carried next to the FP64 line")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (CPU baseline and the per-field errors against it)")
    ap.add_argument("--cpu-sample-iters", type=int, default=40,
                    help="oracle FGMRES iterations timed for the CPU baseline")
    ap.add_argument("--cpu-budget", type=float, default=20.0,
                    help="seconds of oracle solve time for the batch's CPU baseline")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--shapes", default=None,
                    help="JSON file of per-level kernel shapes: written after autotuning when "
                         "absent, applied instead of the autotuner's choice when present "
                         "(so profiler runs time the same kernels)")
    ap.add_argument("--graph", type=int, default=0, choices=[0, 1],
                    help="replay each Arnoldi step from a captured hipGraph")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 512 MiB device copy first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU (no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import dpp_inputs as I
    import paper_1808_08328_amd as dpp
    assert torch.cuda.is_available(), "no GPU"
    dpp.lib()  # fail loudly if the HIP library is missing

    if args.calibrate_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.config == "c4_batch64":
        return bench_batch(args, torch, I, dpp)
    prob = I.make_config(args.config)
    dg = prob.elem == "dg"
    if dg and (args.precision == 1 or args.shapes):
        print("bench.py: DG-VMS solves run in FP64 or with the FP32 preconditioner (--precision 0 or 2), "
              "with the default shapes (no --shapes)", file=sys.stderr)
        sys.exit(2)
    # load the library's code objects on a small box first, so that the
    # assembly and setup times below are the work itself
    Pw = dpp.assemble_problem(I.mms_problem(prob.dim, 4, elem=prob.elem))
    Pw.solve(Pw.setup_precond(), rtol=1e-6)
    del Pw
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = dpp.assemble_problem(prob)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pc = P.setup_precond()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    if args.shapes:
        nlev = pc.info()["levels"]
        if os.path.exists(args.shapes):
            for lvl, (lanes, sym) in enumerate(json.load(open(args.shapes))["shapes"]):
                pc.set_shape(lvl, lanes, sym)
        else:
            json.dump({"workload": args.config, "shapes": [list(pc.shape(lvl)) for lvl in range(nlev - 1)]},
                      open(args.shapes, "w"))
    opts = dict(rtol=1e-8, precision=args.precision, use_graph=args.graph)
    ms, (x, st) = timed(torch, lambda: P.solve(pc, **opts), args.steps, args.warmup)
    iters = st.iters
    value = P.n_dof / (ms / 1e3)
    log("%s precision %d: %.3f ms per solve, %d iterations" % (args.config, args.precision, ms, iters))
    solutions = {"precision_%d" % args.precision: x.cpu().numpy()}

    line = {
        "metric": METRIC, "value": value, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == 0 else "f64/f32",
        "data": "synthetic",
        "config": {"workload": args.config, "description": WORKLOADS[args.config],
                   "n_dof": P.n_dof, "rtol": 1e-8, "precision": PRECISION[args.precision],
                   "graph": bool(args.graph)},
        "iters": iters, "rel_residual": st.rel_residual,
        "assemble_ms": (t1 - t0) * 1e3, "setup_ms": (t2 - t1) * 1e3,
    }
    if args.precision == 0 and not args.no_mixed:
        # the mixed-precision solve of the same system, timed the same way
        # (DG-VMS: the FP32 preconditioner; iterative refinement is CG-VMS only)
        mp = 2 if dg else 1
        msm, (xm, stm) = timed(torch, lambda: P.solve(pc, **{**opts, "precision": mp}),
                               args.steps, args.warmup)
        log("precision %d: %.3f ms per solve, %d iterations" % (mp, msm, stm.iters))
        line["mixed"] = {"precision": PRECISION[mp], "ms_per_step": msm, "value": P.n_dof / (msm / 1e3),
                         "iters": stm.iters, "refinements": stm.refinements,
                         "rel_residual": stm.rel_residual, "speedup_vs_fp64": ms / msm}
        solutions["precision_%d" % mp] = xm.cpu().numpy()

    copy_gbs = measured_copy_gbs(torch)
    if not args.no_profile:
        kernels = profiled(dpp, lambda: P.solve(pc, **opts), args.steps)
        line["roofline"] = roofline(kernels, SINGLE_KERNEL_FAMILIES, copy_gbs,
                                    lambda k: kernel_name(k, stencil_tag(prob), pc,
                                                          flux=getattr(prob, "face_bc", None) is not None,
                                                          dg=dg),
                                    args.config)
        line["kernels"] = strip_raw(kernels)
    else:
        line["roofline"] = None
    if not args.no_cpu_baseline:
        del pc, P
        torch.cuda.empty_cache()
        log("oracle leg")
        base, errs = oracle_leg(prob, iters, args.cpu_sample_iters, solutions)
        line["cpu_baseline"] = base
        line["field_error_vs_oracle"] = errs
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark: one-cell inversion on one MI355X, on the 200,000-cell S_64 problem.

Workload (the large seeded problem): 64 regions, 200,000 cells, S_64,
sigma_t lognormal(0, 1) clipped to [0.01, 10] with dx = 1, c ~ U[0.5, 0.99],
Q ~ U[0, 1], reflecting left / vacuum right, dt = 0.05, v = 1, 50 time steps,
stopping tolerance 1e-6.  One bench step = one full solve from the initial
condition: rebuild every region's cell operator (oci_refactor), reset the
state, then the 50 time steps of plain FP64 OCI to tolerance (oci_solve, the
scalar flux of every step into a device tensor).  The metric: OCI cell-angle
updates per second (sum over iterations of J*N over wall time) and the time
to the 1e-6 tolerance per time step; the same solve in mixed precision
(FP64 defect correction, FP32 inner iterations) and source iteration are
reported beside it, each with its error against the FP64 oracle on the first
steps.  The 10,000-cell S_32 problem (100 steps, tol 1e-10), the ensemble
and the learned corrector follow as secondary fields.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-secondary]
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "OCI cell·angle updates/s + time-to-1e-6 per step: learned/mixed vs plain OCI"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_MFMA_TFLOPS = 78.6


def algorithmic_bytes_per_cell_iteration(n_angles):
    """Values one OCI iteration must move per cell, 8 bytes each: incident
    fluxes in (2N), the step constant of the outgoing fluxes in (2N),
    outgoing fluxes out (2N), new scalar flux out (4) and old scalar flux in
    (4) for the residual: 6N + 8 (the kernels also read the scalar flux's own
    step constant, 4 values more, not counted)."""
    return 8 * (6 * n_angles + 8)


# the iteration kernel by iterates per launch (the library's launch shape)
ITERATION_KERNELS = {1: "k_oci_iterate", 2: "k_oci_iterate2", 3: "k_oci_iterateK<3>",
                     4: "k_oci_iterateK<4>"}


def roofline_launch_seconds(oci, prob, stream, steps=9, k=None):
    """Per-launch time of the iteration kernel of k iterates per launch (default:
    the library's launch shape) on the workload's cells, regions and angles,
    with v = inf and tol = 0 so that every launch does the full work (the
    kernel's work does not depend on the values).  Steps of two and of one
    full launches (four and two with fewer than three iterates per launch:
    all within the eight iterates one ring of iterate buffers takes at least)
    each run as one replayed graph (the launches and the end of step), timed
    with HIP events on the library's stream; the per-launch time is the
    difference of the median step times over the extra launches, which
    removes the end of step.  It is launch to launch: the kernel's duration
    plus the dispatch gap between two graph nodes.  Returns (seconds, k)."""
    import dataclasses
    roof = dataclasses.replace(prob, speed=float("inf"), name=prob.name + ", v = inf")
    with oci.OciContext(roof, stream=stream) as cq:
        k = cq.iterates_per_launch if k is None else min(k, cq.iterates_per_launch)
    hi_launches = 2 if k >= 3 else 4
    lo_launches = hi_launches // 2
    hi, lo = hi_launches * k, lo_launches * k
    med = {}
    for n in (hi, lo):
        with oci.OciContext(roof, stream=stream, tol=0.0, max_iters=n) as cr:
            cr.set_iterates_per_launch(k)   # (a fresh context's default may differ)
            cr.step()
            ms = []
            for _ in range(steps):
                rc, info = cr.step()
                if info["launches"] != n or info["iterations"] != n:
                    raise RuntimeError("roofline step did not run %d full launches: %r"
                                       % (n, info))
                ms.append(info["ms"])
            med[n] = float(np.median(ms))
    return (med[hi] - med[lo]) * 1e-3 / (hi_launches - lo_launches), k


def copy_calibration(torch, mib):
    """A plain device-to-device copy of `mib` MiB (3 times), the reference
    kernel for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    n = mib * (1 << 20) // 8
    src = torch.rand(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return n * 8


KERNEL_SOURCES = ("oci_step.hip", "oci_device.h", "oci_kernels.h")


def traffic_profile(k, tag):
    name = ITERATION_KERNELS[k].replace("<", "").replace(">", "")
    return os.path.join(ROOT, "profiles", "%s_%s_hbm_traffic.txt" % (name, tag))


def measured_traffic(k, tag):
    """HBM bytes per launch of the iteration kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when there is
    none or the kernel sources have changed since the counters were taken."""
    import hashlib
    try:
        fields = dict(line.split(":", 1) for line in open(traffic_profile(k, tag))
                      if line.startswith(("traffic_bytes_per_launch:", "kernel_sources_sha256:")))
    except OSError:
        return None
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2305_13555_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != fields.get("kernel_sources_sha256", "").strip():
        return None
    return float(fields["traffic_bytes_per_launch"])


def on_box_peaks(torch):
    """Achievable rates on this GPU: a 2 GiB device-to-device copy (read +
    written bytes per second, far past the 256 MB last-level cache) and an
    8192^3 FP64 matrix product (rocBLAS on the FP64 matrix cores), best of 5
    after a warm-up."""
    n = (2 << 30) // 8
    src = torch.rand(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    best = float("inf")
    for _ in range(6):
        torch.cuda.synchronize()
        t = time.perf_counter()
        dst.copy_(src)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    copy_gbs = 2 * n * 8 / best / 1e9
    del src, dst
    m = 8192
    a = torch.rand((m, m), dtype=torch.float64, device="cuda")
    b = torch.rand((m, m), dtype=torch.float64, device="cuda")
    best = float("inf")
    for _ in range(6):
        torch.cuda.synchronize()
        t = time.perf_counter()
        c = a @ b
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    del a, b, c
    torch.cuda.empty_cache()
    return {"hbm_copy_gbs": copy_gbs, "fp64_gemm_tflops": 2.0 * m ** 3 / best / 1e12,
            "spec_hbm_gbs": PEAK_HBM_GBS, "spec_fp64_mfma_tflops": PEAK_FP64_MFMA_TFLOPS,
            "how": "2 GiB device copy (read + written bytes) and an 8192^3 FP64 torch "
                   "matmul, best of 5 after a warm-up"}


def cpu_baseline(prob, n_steps):
    """The oracle's OCI (per-region LU + multi-right-hand-side solves) timed
    on the host for the first n_steps of the workload at its tolerance, then
    (untimed) the first step continued to e <= 1e-13 as the converged FP64
    reference.  Returns (cpu_baseline record, oracle steps, converged phi of
    the first step)."""
    from oracle import oci as ooci
    from oracle.problem import cell_data, initial_edge_state
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    cd = cell_data(prob)
    t0 = time.perf_counter()
    res = ooci.run_oci(prob, cd, n_steps, tol=prob.tol, max_iters=prob.max_iters)
    dt = time.perf_counter() - t0
    its = sum(r["iterations"] for r in res)
    updates = its * cd.J * cd.n
    f = ooci.RegionFactors(cd)
    conv = ooci.oci_step(cd, f, initial_edge_state(prob, cd), res[0]["psi"], 1e-13, 1000)
    rec = {"value": updates / dt, "unit": "cell·angle updates/s", "cores": int(threads),
           "kind": "oracle",
           "sample": "first %d of %d time steps of the same workload at tol %g (%d iterations, "
                     "%.1f s), operator factorisation included" % (
                         n_steps, prob.n_steps, prob.tol, its, dt),
           "host_cpu_count": os.cpu_count()}
    return rec, res, conv["phi"]


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def timed_solves(oci, torch, ctx, prob, phi_dev, n, refactor=True):
    """n full solves of prob on ctx (operator rebuild, reset, all steps);
    returns (wall seconds, infos of every solve)."""
    T = prob.n_steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = []
    for _ in range(n):
        if refactor:
            ctx.refactor(prob)
        ctx.set_state(None, 0)
        rc, infos = ctx.solve(T, phi_dev)
        if rc < 0 or any(i["status"] != oci.OCI_OK for i in infos):
            raise RuntimeError("solve failed: rc=%d" % rc)
        out.append(infos)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, out


def si_steps(oci, prob, stream, tol, n=5):
    """Source iteration step by step on the same problem: ms and sweeps per step."""
    with oci.OciContext(prob, stream=stream, tol=tol) as cs:
        ms, its = [], []
        for _ in range(n):
            rc, info = cs.si_step()
            ms.append(info["ms"])
            its.append(info["iterations"])
    return float(np.mean(ms)), float(np.mean(its))


def secondary_case(oci, torch, stream, steps=5):
    """The 10,000-cell S_32 problem (16 regions, 100 steps, tol 1e-10): plain
    FP64 OCI updates/s and ms per step, the iteration kernel's roofline,
    source iteration and the OCI/SI speedup, mixed precision, and the scalar
    flux against the oracle on the first 3 steps."""
    from paper_2305_13555_amd import workloads
    from oracle import oci as ooci
    from oracle.problem import cell_data
    prob = workloads.config2()
    J, N, T = prob.n_cells, prob.n_angles, prob.n_steps
    phi = torch.zeros((T, J, 4), dtype=torch.float64, device="cuda")
    with oci.OciContext(prob, stream=stream) as ctx:
        timed_solves(oci, torch, ctx, prob, phi, 2)
        wall, infos = timed_solves(oci, torch, ctx, prob, phi, steps)
        shape = ctx.iterates_per_launch
    iters = sum(i["iterations"] for inf in infos for i in inf)
    ms_step = wall * 1e3 / (steps * T)
    t, k = roofline_launch_seconds(oci, prob, stream)
    nbytes = algorithmic_bytes_per_cell_iteration(N) * J * k
    si_ms, si_its = si_steps(oci, prob, stream, prob.tol, 10)
    with oci.OciContext(prob, stream=stream, precision=oci.OCI_PREC_FP32) as cm:
        timed_solves(oci, torch, cm, prob, phi, 2)   # (warm-up and timing as plain)
        mwall, _ = timed_solves(oci, torch, cm, prob, phi, steps)
    ref = ooci.run_oci(prob, cell_data(prob), 3, tol=prob.tol, max_iters=prob.max_iters)
    with oci.OciContext(prob, stream=stream) as ctx:
        ctx.solve(3, phi)
    got = phi[:3].cpu().numpy()
    mixed_ms = mwall * 1e3 / (steps * T)
    return {
        "workload": prob.name + ", tol 1e-10",
        "cell_angle_updates_per_s": iters * J * N / wall,
        "oci_ms_per_time_step": ms_step,
        "iterations_per_time_step": iters / (steps * T),
        "iterates_per_launch": shape,
        "iteration_kernel": {"kernel": ITERATION_KERNELS[k], "us_per_launch": t * 1e6,
                             "bytes_per_launch": nbytes,
                             "hbm_frac": nbytes / t / 1e9 / PEAK_HBM_GBS,
                             "traffic": measured_traffic(k, "c2")},
        "si_ms_per_time_step": si_ms, "si_iterations_per_time_step": si_its,
        "oci_over_si_speedup": si_ms / ms_step,
        "mixed_ms_per_time_step": mixed_ms,
        "mixed_speedup_vs_plain": ms_step / mixed_ms,
        "parity_vs_oracle_rel_first_3_steps": max(rel_err(got[i], ref[i]["phi"])
                                                  for i in range(3)),
    }


def learned_case(oci, torch, stream, n_steps=2, tol=1e-6, first=10, period=20):
    """The learned corrector inside the iteration on the thin-cell evaluation
    problem (100,000 cells, S128, 64 regions, optical thickness 0.01 - 0.5,
    c = 0.9 - 0.999, dt = 1, v = 4: hundreds of OCI iterations per step), with
    the weights trained on the seeded thin-cell problems (train_corrector.py;
    the record of that training travels with the weights).  Time to the
    stopping tolerance per step, first n_steps steps: plain FP64 OCI (queued
    solve), the same iterates driven from the host (the driver the corrections
    use), and learned (corrections at iterates first, first + period, ...,
    kept only when the next plain iterate changes less than a plain one
    would).  Each result's largest difference to the plain solve at tol 1e-11
    is reported."""
    from paper_2305_13555_amd import corrector as C
    from paper_2305_13555_amd import workloads
    w, c_in, meta = C.load_weights(os.path.join(ROOT, "paper_2305_13555_amd",
                                                "corrector_weights.json"))
    prob = workloads.config4_eval(n_steps=n_steps)
    J, N = prob.n_cells, prob.n_angles
    phi = torch.zeros((n_steps, J, 4), dtype=torch.float64, device="cuda")
    with oci.OciContext(prob, stream=stream, tol=1e-11) as cr:
        cr.solve(n_steps, phi)
        ref = phi.cpu().numpy()

    def run(mode):
        with oci.OciContext(prob, stream=stream, tol=tol) as cx:
            k = None
            if mode == "learned":
                k = oci.Corrector(c_in, C.C_OUT, 1, J, stream=stream)
                k.set_weights(w)
                cx.set_corrector(k, first=first, period=period)
            cx.solve(1)                      # warm-up: graphs, caches
            cx.set_state(None, 0)
            torch.cuda.synchronize()
            t = time.perf_counter()
            if mode == "host_plain":
                infos = []
                for s in range(n_steps):
                    rc, info, _ = cx.step_history(0)
                    phi[s].copy_(torch.from_numpy(cx.flux()).to("cuda"))
                    infos.append(info)
            else:
                rc, infos = cx.solve(n_steps, phi)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t
            cx.set_corrector(None)
            if k is not None:
                k.close()
        got = phi.cpu().numpy()
        return {"ms_per_time_step": sec * 1e3 / n_steps,
                "iterations_per_step": [i["iterations"] for i in infos],
                "launches_per_step": [i["launches"] for i in infos],
                "corrections_per_step": [i["corrections"] for i in infos],
                "rel_vs_tight_solve": max(rel_err(got[s], ref[s]) for s in range(n_steps))}

    out = {"workload": prob.name + ", first %d steps, tol %g" % (n_steps, tol),
           "corrections_at": "iterates %d, %d, ... (every %d)" % (first, first + period, period),
           "training": {k2: meta.get(k2) for k2 in ("problems", "generator", "samples",
                                                     "cell_samples", "epochs", "loss_first_last")},
           "input_channels": c_in,
           "inference": "FP32 on the matrix cores (v_mfma_f32_16x16x4f32)"}
    for mode in ("plain", "host_plain", "learned"):
        out[mode] = run(mode)
    out["learned_speedup_vs_plain"] = out["plain"]["ms_per_time_step"] / \
        out["learned"]["ms_per_time_step"]
    out["applied_in_iteration"] = True
    return out


def ensemble_case(oci, torch, n_problems=512, chunk=128, n_check=8,
                  modes=("sequential", "threads", "ensemble")):
    """The batched ensemble: problems 0 .. n_problems-1 of the ensemble
    generator (500 - 100,000 cells log-uniform, S8 - S128, 16 regions, 20
    steps, tol 1e-10), in groups of `chunk` contexts (compact iterate rings;
    all 512 side by side would need about 150 GB).  Per group, after a warm-up
    of each mode, the same 20 steps of every problem: one problem after
    another (each context's own queued solve), driven by host threads (one
    stream per context), and as one ensemble (oci_solve_ensemble: one launch
    per iteration over the work queue of all the group's tiles).  Cell-angle
    updates per second over all problems, and the ensemble's scalar flux of
    the first two steps of n_check sampled problems against the oracle.
    `modes` restricts the timed forms (for a profile of one of them)."""
    from paper_2305_13555_amd import workloads
    from oracle import oci as ooci
    from oracle.problem import cell_data
    probs = [workloads.config5(i) for i in range(n_problems)]
    T = probs[0].n_steps
    # sampled problems for the oracle: small enough for it (J * N <= 1e6)
    check = [i for i, p in enumerate(probs) if p.n_cells * p.n_angles <= 1e6][:n_check]
    secs = {k: 0.0 for k in modes}
    upd = {k: 0 for k in secs}
    worst = 0.0
    for g0 in range(0, n_problems, chunk):
        group = list(range(g0, min(n_problems, g0 + chunk)))
        streams = [torch.cuda.Stream() for _ in group]
        ctxs = [oci.OciContext(probs[i], stream=s, compact=True) for i, s in zip(group, streams)]
        outs = [torch.zeros((2, probs[i].n_cells, 4), dtype=torch.float64, device="cuda")
                if i in check else None for i in group]
        try:
            for mode in modes:
                for rep in range(2):   # a warm-up, then the timed run
                    for c in ctxs:
                        c.set_state(None, 0)
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    if mode == "sequential":
                        infos = [c.solve(T)[1] for c in ctxs]
                    elif mode == "threads":
                        infos = oci.oci_solve_batch(ctxs, T)[1]
                    else:
                        infos = oci.oci_solve_ensemble(ctxs, T)[1]
                    torch.cuda.synchronize()
                    if rep == 1:
                        secs[mode] += time.perf_counter() - t
                        upd[mode] += sum(inf["iterations"] * probs[i].n_cells * probs[i].n_angles
                                         for i, per in zip(group, infos) for inf in per)
            if any(i in check for i in group):   # the ensemble's first two steps vs the oracle
                for c in ctxs:
                    c.set_state(None, 0)
                oci.oci_solve_ensemble(ctxs, 2, outs)
                for i, o in zip(group, outs):
                    if o is None:
                        continue
                    ref = ooci.run_oci(probs[i], cell_data(probs[i]), 2, tol=1e-10,
                                       max_iters=1000)
                    got = o.cpu().numpy()
                    worst = max(worst, max(rel_err(got[k], ref[k]["phi"]) for k in range(2)))
        finally:
            for c in ctxs:
                c.close()
            torch.cuda.empty_cache()
    out = {"workload": "%d ensemble problems (S8 - S128, 16 regions, %d - %d cells, %d in all), "
                       "%d steps each, tol 1e-10, in groups of %d" % (
                           n_problems, min(p.n_cells for p in probs),
                           max(p.n_cells for p in probs), sum(p.n_cells for p in probs), T, chunk),
           "oracle_check": {"problems": check, "steps": 2, "max_rel_vs_oracle": worst}}
    for k in secs:
        out[k] = {"seconds": secs[k], "cell_angle_updates_per_s": upd[k] / secs[k]}
    if "sequential" in secs and "ensemble" in secs:
        out["ensemble_speedup_vs_sequential"] = secs["sequential"] / secs["ensemble"]
    if "sequential" in secs and "threads" in secs:
        out["threads_speedup_vs_sequential"] = secs["sequential"] / secs["threads"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 10,000-cell S_32 problem, the ensemble and the corrector")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the iteration kernel's roofline batches on the workload and a "
                         "64 MiB copy (for hardware-counter runs)")
    ap.add_argument("--learned-only", action="store_true",
                    help="only the learned corrector on the thin-cell evaluation problem")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="only the 512-problem ensemble")
    ap.add_argument("--ensemble-modes", default="sequential,threads,ensemble",
                    help="with --ensemble-only: the forms timed, comma-separated")
    ap.add_argument("--skip-ensemble", action="store_true",
                    help="the secondary cases without the 512-problem ensemble")
    ap.add_argument("--workload", choices=["large", "bench16"], default="large",
                    help="with --roofline-only: the 200,000-cell S_64 problem or the "
                         "10,000-cell S_32 one")
    ap.add_argument("--k", type=int, default=None,
                    help="with --roofline-only: iterates per launch (default: the launch shape)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the OCI path here is single-GPU "
              "(multi-GPU sharding is described, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    modes = tuple(m for m in args.ensemble_modes.split(",") if m)
    if not modes or set(modes) - {"sequential", "threads", "ensemble"}:
        print("--ensemble-modes: a comma-separated subset of sequential,threads,ensemble",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2305_13555_amd import oci, workloads

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.roofline_only:
        prob = workloads.config3() if args.workload == "large" else workloads.config2()
        t, k = roofline_launch_seconds(oci, prob, stream, steps=3, k=args.k)
        nbytes = copy_calibration(torch, 64)
        b = algorithmic_bytes_per_cell_iteration(prob.n_angles) * prob.n_cells * k
        print(json.dumps({"workload": prob.name, "kernel": ITERATION_KERNELS[k],
                          "us_per_launch": t * 1e6, "algorithmic_bytes_per_launch": b,
                          "GB/s": b / t / 1e9, "copy_bytes": nbytes}))
        return

    if args.learned_only:
        print(json.dumps(learned_case(oci, torch, stream)))
        return
    if args.ensemble_only:
        print(json.dumps(ensemble_case(oci, torch, modes=modes)))
        return
    prob = workloads.config3()
    J, N, T = prob.n_cells, prob.n_angles, prob.n_steps
    print("bench: %s, tol %g" % (prob.name, prob.tol), file=sys.stderr, flush=True)
    from paper_2305_13555_amd import tune
    ctx = oci.OciContext(prob, stream=stream)
    phi_dev = torch.zeros((T, J, 4), dtype=torch.float64, device="cuda")
    # the launch configuration from the autotuner (short solves from the
    # initial state), then the warm-up and timed full solves
    shape, shape_ms = tune.tune(ctx, torch, n_steps=8, repeats=2, use_cache=False)
    fused, fused_ms = tune.tune_fusion(ctx, torch, n_steps=8, repeats=2, use_cache=False)
    timed_solves(oci, torch, ctx, prob, phi_dev, args.warmup)
    wall, all_infos = timed_solves(oci, torch, ctx, prob, phi_dev, args.steps)
    iters = sum(i["iterations"] for infos in all_infos for i in infos)
    value = iters * J * N / wall
    plain_ms = wall * 1e3 / (args.steps * T)
    plain_phi = phi_dev[:max(args.cpu_steps, 1)].cpu().numpy()
    bounds = [i["err_bound"] for i in all_infos[-1]]
    print("bench: plain %.4f ms per time step" % plain_ms, file=sys.stderr, flush=True)

    # mixed precision, same workload and stopping rule
    nm = max(args.steps // 2, 1)
    with oci.OciContext(prob, stream=stream, precision=oci.OCI_PREC_FP32) as cm:
        inner, inner_ms = tune.tune(cm, torch, n_steps=8, repeats=2, use_cache=False)
        mfused, mfused_ms = tune.tune_fusion(cm, torch, n_steps=8, repeats=2, use_cache=False)
        timed_solves(oci, torch, cm, prob, phi_dev, args.warmup)   # (the same warm-up as plain)
        mwall, minfos = timed_solves(oci, torch, cm, prob, phi_dev, nm)
    mixed_ms = mwall * 1e3 / (nm * T)
    mixed_phi = phi_dev[:1].cpu().numpy()
    print("bench: mixed %.4f ms per time step" % mixed_ms, file=sys.stderr, flush=True)

    # the iteration kernel the timed solves run most: with the end of step
    # fused, a step's first iterate comes with the previous step's end and the
    # rest in launches of up to the launch shape; unfused, all of them
    k_main = max(1, min(ctx.iterates_per_launch,
                        max(i["iterations"] for i in all_infos[-1]) - (1 if fused else 0)))
    roof_steps = 15
    per_launch_s, k_launch = roofline_launch_seconds(oci, prob, stream, steps=roof_steps,
                                                     k=k_main)
    kernel = ITERATION_KERNELS[k_launch]
    bytes_launch = algorithmic_bytes_per_cell_iteration(N) * J * k_launch
    achieved = bytes_launch / per_launch_s / 1e9
    si_ms, si_its = si_steps(oci, prob, stream, prob.tol, 5)

    cpu, parity = None, None
    if not args.no_cpu:
        ncpu = max(1, min(args.cpu_steps, T))
        print("bench: oracle on the first %d steps" % ncpu, file=sys.stderr, flush=True)
        cpu, ref, conv = cpu_baseline(prob, ncpu)
        parity = {
            "plain_vs_oracle_same_rule_rel": [rel_err(plain_phi[i], ref[i]["phi"])
                                              for i in range(ncpu)],
            "plain_iterations": [i["iterations"] for i in all_infos[-1][:ncpu]],
            "oracle_iterations": [r["iterations"] for r in ref],
            "plain_vs_converged_oracle_rel_step1": rel_err(plain_phi[0], conv),
            "mixed_vs_converged_oracle_rel_step1": rel_err(mixed_phi[0], conv),
            "converged_reference": "oracle OCI, first step continued to e <= 1e-13",
        }
    peaks = on_box_peaks(torch)
    secondary = ensemble = learned = None
    if not args.no_secondary:
        print("bench: secondary cases", file=sys.stderr, flush=True)
        secondary = secondary_case(oci, torch, stream)
        ensemble = None if args.skip_ensemble else ensemble_case(oci, torch)
        learned = learned_case(oci, torch, stream)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "cell·angle updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "plain FP64 OCI, %s; sigma_t lognormal(0,1) clipped to [0.01, 10] with "
                        "dx = 1, c ~ U[0.5, 0.99], Q ~ U[0, 1], reflecting left / vacuum right, "
                        "dt = 0.05, v = 1, tol 1e-6 (seeded)" % prob.name,
            "cells": J, "angles": N, "regions": prob.n_regions, "time_steps": T,
            "tol": prob.tol, "step": "operator rebuild + %d time steps (one full solve)" % T,
            "driver": "queued solve (whole steps replayed from cached HIP graphs)",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kernel,
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": measured_traffic(k_launch, "c3"),
            "bytes_per_launch": bytes_launch,
            "us_per_launch": per_launch_s * 1e6,
            "iterations_per_launch": k_launch,
            "measured": "(median step time at 2 full launches - at 1) (at 4 - at 2 for "
                        "fewer than 3 iterates per launch), %d steps each, HIP events on the "
                        "library's stream (launch to launch, dispatch gap included)"
                        % roof_steps,
        },
        "cpu_baseline": cpu,
        "time_to_1e-6_ms_per_step": {
            "plain_fp64": plain_ms, "mixed": mixed_ms,
            "learned_thin_cell_eval": None if learned is None else {
                "plain_fp64": learned["plain"]["ms_per_time_step"],
                "learned": learned["learned"]["ms_per_time_step"]}},
        "mixed_speedup_vs_plain": plain_ms / mixed_ms,
        "iterations_per_time_step": iters / (args.steps * T),
        "mixed_fp64_iterations_per_time_step": float(np.mean(
            [i["iterations"] for inf in minfos for i in inf])),
        "mixed_launches_per_time_step": float(np.mean(
            [i["launches"] for inf in minfos for i in inf])),
        "plain_err_bound_max": max(bounds),
        "autotuned": {"iterates_per_launch": shape,
                      "iterates_per_launch_ms_per_step": {str(k): v for k, v in shape_ms.items()},
                      "mixed_inner_iterations": inner,
                      "mixed_inner_ms_per_step": {str(k): v for k, v in inner_ms.items()},
                      "end_fusion": fused, "end_fusion_ms_per_step": fused_ms,
                      "mixed_end_fusion": mfused, "mixed_end_fusion_ms_per_step": mfused_ms,
                      "how": "8-step solves from the initial state, best of 2 per candidate"},
        "parity_vs_oracle": parity,
        "si_ms_per_time_step": si_ms,
        "si_iterations_per_time_step": si_its,
        "oci_over_si_speedup": si_ms / plain_ms,
        "on_box_peaks": peaks,
        "bench16": secondary,
        "ensemble": ensemble,
        "learned": learned,
    }
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()

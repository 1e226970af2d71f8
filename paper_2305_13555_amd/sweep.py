"""OCI against SI across quadrature orders and problem parameters.

The paper's quadrature study (Sec. "GPU Explorations Across Quadrature Sets")
runs a homogeneous slab (width 10, Sigma = 2, Q = 0.1, vacuum on both sides,
zero initial flux, five time steps) with both iterations on the GPU and
reports the wall-clock speedup t_SI / t_OCI over the scattering ratio c, the
cell optical thickness Sigma*dx and the time step, for S_2 .. S_256.  The
figure's grid values are not printed; this sweep uses log-spaced grids (see
GRID) and v = 1.

Each point solves the five steps once with OCI (queued solve) and once with
SI (step by step) on one context each, after a warm-up solve, and records the
wall times, the iterations per step and the largest relative difference of
the two final scalar fluxes.  Both stop by the strict rule (change e <= tol
and the a-posteriori bound e rho / (1 - rho) <= tol), so both reach the same
accuracy even where one contracts far more slowly than the other.  With
check_oracle, the point's five steps are also solved by the FP64 oracle's OCI
(same rule, tol 1e-12) and each method's final scalar flux is compared with
it.

Usage: python -m paper_2305_13555_amd.sweep [--quick] [--out FILE] [--check]
Prints one JSON object per point and a speedup table per N; --check compares
one point per N (c = 0.9, sigma*dx = 0.1, dt = 0.1) with the oracle.
"""
import argparse
import itertools
import json
import sys
import time

import numpy as np

from . import workloads

GRID = {
    "n_angles": [2, 4, 8, 16, 32, 64, 128, 256],
    "c": [0.5, 0.9, 0.99],
    "sigma_dx": [0.01, 0.1, 1.0],   # cells: 20 / sigma_dx = 2000, 200, 20
    "dt": [0.01, 0.1, 1.0],
}
QUICK = {"n_angles": [4, 32, 256], "c": [0.9], "sigma_dx": [0.1], "dt": [0.1]}
WIDTH, SIGMA_T, SOURCE, STEPS, TOL = 10.0, 2.0, 0.1, 5, 1e-9


def problem(n_angles, c, sigma_dx, dt):
    n_cells = int(round(WIDTH * SIGMA_T / sigma_dx))
    return workloads.homogeneous_slab(n_angles, n_cells, c, sigma_dx, dt, speed=1.0,
                                      sigma_t=SIGMA_T, source=SOURCE, n_steps=STEPS,
                                      width=WIDTH)


CHECK = {"c": 0.9, "sigma_dx": 0.1, "dt": 0.1}


def run_point(oci, torch, n_angles, c, sigma_dx, dt, max_iters=200000, check_oracle=False):
    prob = problem(n_angles, c, sigma_dx, dt)
    stream = torch.cuda.current_stream()
    out = {"n_angles": n_angles, "c": c, "sigma_dx": sigma_dx, "dt": dt,
           "cells": prob.n_cells, "tol": TOL, "rule": "strict"}
    with oci.OciContext(prob, stream=stream, tol=TOL, max_iters=max_iters, strict=True) as ctx:
        ctx.solve(STEPS)                      # warm-up: graphs, caches
        ctx.set_state(None, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, infos = ctx.solve(STEPS)
        torch.cuda.synchronize()
        out["oci_s"] = time.perf_counter() - t0
        out["oci_iters"] = [i["iterations"] for i in infos]
        out["oci_rc"] = rc
        phi_oci = ctx.flux().copy()
    with oci.OciContext(prob, stream=stream, tol=TOL, max_iters=max_iters, strict=True) as ctx:
        ctx.si_step()
        ctx.set_state(None, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, rcs = [], []
        for _ in range(STEPS):
            rc, info = ctx.si_step()
            its.append(info["iterations"])
            rcs.append(rc)
        torch.cuda.synchronize()
        out["si_s"] = time.perf_counter() - t0
        out["si_iters"] = its
        out["si_rc"] = max(rcs)
        phi_si = ctx.flux().copy()
    out["speedup_si_over_oci"] = out["si_s"] / out["oci_s"]
    out["oci_vs_si_rel"] = float(np.max(np.abs(phi_oci - phi_si)) / np.max(np.abs(phi_si)))
    if check_oracle:
        from oracle import oci as ooci
        from oracle.problem import cell_data
        ref = ooci.run_oci(prob, cell_data(prob), STEPS, tol=1e-12, max_iters=max_iters,
                           strict=True)[-1]["phi"]
        scale = float(np.max(np.abs(ref)))
        out["oci_vs_oracle_rel"] = float(np.max(np.abs(phi_oci - ref))) / scale
        out["si_vs_oracle_rel"] = float(np.max(np.abs(phi_si - ref))) / scale
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="three points only")
    ap.add_argument("--out", default=None, help="also write the JSON lines here")
    ap.add_argument("--check", action="store_true",
                    help="compare one point per N with the FP64 oracle")
    args = ap.parse_args(argv)
    import torch
    from . import oci
    grid = QUICK if args.quick else GRID
    rows = []
    sink = open(args.out, "w") if args.out else None
    for n, c, sdx, dt in itertools.product(grid["n_angles"], grid["c"], grid["sigma_dx"],
                                           grid["dt"]):
        chk = args.check and (c, sdx, dt) == (CHECK["c"], CHECK["sigma_dx"], CHECK["dt"])
        r = run_point(oci, torch, n, c, sdx, dt, check_oracle=chk)
        rows.append(r)
        line = json.dumps(r)
        print(line, flush=True)
        if sink:
            sink.write(line + "\n")
            sink.flush()
    if sink:
        sink.close()
    print("\nspeedup t_SI / t_OCI (min / median / max over c, sigma*dx, dt):", file=sys.stderr)
    for n in grid["n_angles"]:
        s = [r["speedup_si_over_oci"] for r in rows if r["n_angles"] == n]
        print("  S%-4d %6.2f %6.2f %6.2f" % (n, min(s), float(np.median(s)), max(s)),
              file=sys.stderr)
    return rows


if __name__ == "__main__":
    main()

"""Train the learned iterate corrector on the seeded thin-cell problems.

Usage: python -m paper_2305_13555_amd.train_corrector [--problems 48] [--epochs 150]
                                                      [--out FILE] [--windows 'f,n;f,n']

For each training problem (workloads.config4(i), i < problems: 1k - 50k
cells, S16 - S64, 16 regions of optical thickness 0.01 - 0.5 and scattering
ratio 0.9 - 0.999) the library solves three time steps at tol 1e-10 with
oci_step_history, recording the scalar flux of a window of 16 iterates per
step (iterates 1 - 16, 24 - 39 and 80 - 95: early, middle and late in slow
steps); the converged step gives the target phi^(inf).  Up to eight samples
per window, spread over it, form one training set per window; Adam runs over
all sets (one step per set and epoch, FP64 training kernels).  The weights
and the training record go to a JSON file that bench.py and the tests read.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "corrector_weights.json")
WINDOWS = ((1, 16), (24, 16), (80, 16))   # (first iterate, iterates) per step


def collect(torch, oci, C, workloads, n_problems, per_window=8, windows=WINDOWS):
    sets, info = [], []
    for i in range(n_problems):
        p = workloads.config4(i)
        with oci.OciContext(p, tol=1e-10) as ctx:
            for first, nh in windows:
                phis, ref, st = C.step_history(ctx, nh, first)
                x, t, _, used = C.samples(phis, ref, range(first + 2, first + nh), first)
                info.append({"problem": i, "cells": p.n_cells, "angles": p.n_angles,
                             "first": first, "step_iterations": st["iterations"],
                             "samples": 0 if x is None else min(per_window, len(used))})
                if x is None:
                    continue
                pick = np.unique(np.linspace(0, len(used) - 1, min(per_window, len(used)))
                                 .round().astype(int))
                sets.append((torch.from_numpy(np.ascontiguousarray(x[pick])).to("cuda"),
                             torch.from_numpy(np.ascontiguousarray(t[pick])).to("cuda")))
        print("problem %d: %s, step iterations %s" % (
            i, p.name, [r["step_iterations"] for r in info[-len(windows):]]), flush=True)
    return sets, info


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--problems", type=int, default=48)
    ap.add_argument("--epochs", type=int, default=150)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--windows", default=None,
                    help="first iterate and length of each window, e.g. '1,16;40,16'")
    args = ap.parse_args()
    windows = WINDOWS if args.windows is None else tuple(
        tuple(int(v) for v in w.split(",")) for w in args.windows.split(";"))
    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch
    from paper_2305_13555_amd import corrector as C
    from paper_2305_13555_amd import oci, workloads

    t0 = time.perf_counter()
    sets, info = collect(torch, oci, C, workloads, args.problems, windows=windows)
    t_hist = time.perf_counter() - t0
    k, hist, t_train = C.train_sets(torch, sets, epochs=args.epochs, lr=args.lr,
                                    max_cells=workloads.config4_eval().n_cells)
    w = k.weights()
    k.close()
    meta = {"problems": args.problems, "generator": "workloads.config4(0 .. problems-1)",
            "windows": windows, "training_sets": len(sets),
            "samples": int(sum(int(x.shape[0]) for x, _ in sets)),
            "cell_samples": int(sum(int(x.shape[0]) * int(x.shape[2]) for x, _ in sets)),
            "epochs": args.epochs, "lr": args.lr, "loss_first_last": [hist[0], hist[-1]],
            "history_s": t_hist, "train_s": t_train, "steps": info}
    C.save_weights(args.out, w, meta, c_in=int(sets[0][0].shape[1]))
    print(json.dumps({k2: v for k2, v in meta.items() if k2 != "steps"}))


if __name__ == "__main__":
    main()

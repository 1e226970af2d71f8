"""Launch-shape autotuner for queued FP64 solves.

The one knob that changes the speed of a solve but not its results is the
launch shape: how many OCI iterates one iteration kernel computes (2 up to
what the problem allows, oci_set_iterates_per_launch).  More iterates per
launch save launches and re-reads of the previous iterate but recompute
halo cells and hold more LDS per work-group; which wins depends on N, the
mesh and the region layout.  tune() times a short solve per candidate from
the context's current state (restored afterwards), keeps the fastest, and
remembers it per (N, J, regions, precision) in a process-wide cache that can
be saved to and loaded from a JSON file.
"""
import json
import time

from . import oci

_cache = {}


def cache_key(ctx):
    return "N%d_J%d_R%d_%s" % (ctx.n_angles, ctx.n_cells, ctx.n_regions,
                               "fp32" if ctx.precision == oci.OCI_PREC_FP32 else "fp64")


def fastest(times):
    """The candidate with the smallest time (the smaller shape on a tie)."""
    return min(sorted(times), key=lambda k: times[k])


def tune(ctx, torch, n_steps=8, repeats=3, use_cache=True):
    """Pick and set the fastest launch shape for ctx; returns (shape, times
    in ms per step by candidate; empty when the cache answered)."""
    key = cache_key(ctx)
    if use_cache and key in _cache:
        return ctx.set_iterates_per_launch(_cache[key]), {}
    top = ctx.set_iterates_per_launch(64)   # the most the problem allows
    if top <= 2:
        _cache[key] = top
        return top, {}
    psi, step = ctx.state()
    times = {}
    for k in range(2, top + 1):
        ctx.set_iterates_per_launch(k)
        best = float("inf")
        for r in range(repeats + 1):   # the first run builds the graphs
            ctx.set_state(psi, step)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.solve(n_steps)
            torch.cuda.synchronize()
            if r > 0:
                best = min(best, (time.perf_counter() - t0) * 1e3 / n_steps)
        times[k] = best
    ctx.set_state(psi, step)
    k = fastest(times)
    _cache[key] = k
    return ctx.set_iterates_per_launch(k), times


def save_cache(path):
    with open(path, "w") as f:
        json.dump(_cache, f, indent=1, sort_keys=True)


def load_cache(path):
    with open(path) as f:
        data = json.load(f)
    for k, v in data.items():
        if not isinstance(k, str) or not isinstance(v, int) or v < 1:
            raise ValueError("bad tuning cache entry %r: %r" % (k, v))
    _cache.update(data)

"""Autotuner of the launch configuration of queued solves.

Two knobs change the speed of a solve but not what it converges to:

* FP64 contexts: the launch shape, how many OCI iterates one iteration kernel
  computes (1 up to what the problem allows, oci_set_iterates_per_launch).
  More iterates per launch save launches and re-reads of the previous iterate
  but recompute halo cells and hold more LDS per work-group.
* Mixed-precision contexts: the FP32 inner iterations per correction
  (oci_set_inner_iterations, 1 .. 4 tried).  More make each correction more
  complete (fewer FP64 iterates per step) at the cost of the inner launches.
* Both: whether the end of a queued step also computes the next step's first
  iterate (oci_set_end_fusion): one launch fewer per step against a longer
  end-of-step kernel (and, for FP64, one iterate fewer in the launches that
  follow it).

Which wins depends on N, the mesh, the region layout and the tolerance.
tune() times a short solve per candidate from the context's current state
(restored afterwards), keeps the fastest, and remembers it per (N, J,
regions, precision) in a process-wide cache that can be saved to and loaded
from a JSON file; tune_fusion() does the same for the end-of-step fusion at
the context's current setting of the first knob.  The tile (16 cells, the
MFMA block's columns) and the waves per work-group (min(2N/16, 4): the
scalar-flux rows' k-steps split over the waves, one angle per thread in the
per-angle phases) are fixed by the kernels' data layout and are not tuned.
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


INNER_CANDIDATES = (1, 2, 3, 4)


def _time_solves(ctx, torch, n_steps, repeats, psi, step):
    best = float("inf")
    for r in range(repeats + 1):   # the first run builds the graphs
        ctx.set_state(psi, step)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.solve(n_steps)
        torch.cuda.synchronize()
        if r > 0:
            best = min(best, (time.perf_counter() - t0) * 1e3 / n_steps)
    return best


def tune(ctx, torch, n_steps=8, repeats=3, use_cache=True):
    """Pick and set the fastest configuration for ctx: the launch shape of an
    FP64 context, the inner iterations of a mixed-precision one.  Returns
    (value set, times in ms per step by candidate; empty when the cache
    answered or there was nothing to choose)."""
    key = cache_key(ctx)
    mixed = ctx.precision == oci.OCI_PREC_FP32
    setter = ctx.set_inner_iterations if mixed else ctx.set_iterates_per_launch
    if use_cache and key in _cache:
        return setter(_cache[key]), {}
    if mixed:
        cands = INNER_CANDIDATES
    else:
        top = ctx.set_iterates_per_launch(64)   # the most the problem allows
        cands = range(1, top + 1)
    psi, step = ctx.state()
    times = {}
    for k in cands:
        setter(k)
        times[k] = _time_solves(ctx, torch, n_steps, repeats, psi, step)
    ctx.set_state(psi, step)
    k = fastest(times)
    _cache[key] = k
    return setter(k), times


def tune_fusion(ctx, torch, n_steps=8, repeats=3, use_cache=True):
    """Pick and set the faster end-of-step fusion for ctx (at its current
    launch shape or inner iterations).  Returns (fused: bool, ms per step by
    candidate {"fused": t, "unfused": t}; empty when the cache answered)."""
    key = cache_key(ctx) + "_fusion"
    if use_cache and key in _cache:
        return ctx.set_end_fusion(bool(_cache[key])), {}
    psi, step = ctx.state()
    times = {}
    for name, on in (("fused", True), ("unfused", False)):
        ctx.set_end_fusion(on)
        times[name] = _time_solves(ctx, torch, n_steps, repeats, psi, step)
    ctx.set_state(psi, step)
    on = times["fused"] <= times["unfused"]
    _cache[key] = 1 if on else 0
    return ctx.set_end_fusion(on), times


def save_cache(path):
    with open(path, "w") as f:
        json.dump(_cache, f, indent=1, sort_keys=True)


def load_cache(path):
    with open(path) as f:
        data = json.load(f)
    for k, v in data.items():
        lo = 0 if isinstance(k, str) and k.endswith("_fusion") else 1
        if not isinstance(k, str) or not isinstance(v, int) or v < lo or (lo == 0 and v > 1):
            raise ValueError("bad tuning cache entry %r: %r" % (k, v))
    _cache.update(data)

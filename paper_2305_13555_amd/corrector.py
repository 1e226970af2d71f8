"""Training data, training and use of the learned iterate corrector.

The corrector (oci_corrector_* in the C ABI) maps the two latest differences
of OCI's scalar-flux iterates and the latest one extrapolated with the
iteration's observed contraction, per cell,
    x = [phi^(l) - phi^(l-1), phi^(l-1) - phi^(l-2), a (phi^(l) - phi^(l-1))]
        (12 channels; a = rho / (1 - rho), rho = e_l / e_{l-1} in [0, 0.9999],
        e_l = max|phi^(l) - phi^(l-1)| / max|phi^(l)|, the library's residual),
to the iterate's remaining error, phi^(inf) - phi^(l) (4 channels); the
8-channel form (without the extrapolated difference) is also accepted by the
library.  The network is positively homogeneous, so each training sample is
scaled by s = (1 + a) max |phi^(l) - phi^(l-1)| (which leaves the prediction
for the unscaled input exact up to rounding) and every sample weighs alike in
the loss.

The histories come from the library itself: oci_step_history runs an
ordinary OCI step from the context's state and copies out the scalar flux of
a window of its iterates as they are formed (one solve per step, no re-runs);
the step, converged to a tight tolerance, gives phi^(inf) and advances the
state as any step does.  Inside the iteration the library applies the
trained network itself (oci_set_corrector): it corrects every scalar-flux
iterate it is applied to together with the outgoing fluxes, and keeps the
correction only when the next plain iterate changes less than a plain one
would (backing off after corrections it rejects).
"""
import json
import time

import numpy as np

from . import oci

C_IN, C_OUT = 12, 4
RHO_MAX = 0.9999


def step_history(ctx, n_hist, first=1):
    """One OCI step of ctx (at its tolerance) with the scalar flux of its
    iterates first .. first + n_hist - 1: returns (the recorded iterates
    [n] x [J][4], n <= n_hist of them computed, the step's converged phi, its
    step info)."""
    rc, info, hist = ctx.step_history(n_hist, first=first)
    n = max(0, min(n_hist, info["iterations"] - first + 1))
    return [hist[i] for i in range(n)], ctx.flux().copy(), info


def extrapolation_factor(p0, p1, p2):
    """rho / (1 - rho) with rho = e_l / e_{l-1} clamped to [0, RHO_MAX], from the
    scalar fluxes of iterates l, l-1, l-2 (the library's residual e)."""
    def e(a, b):
        den = float(np.max(np.abs(a)))
        return float(np.max(np.abs(a - b))) / den if den > 0 else 0.0
    e0, em = e(p0, p1), e(p1, p2)
    rho = min(max(e0 / em, 0.0), RHO_MAX) if em > 0 else 0.0
    return rho / (1.0 - rho)


def features(p0, p1, p2, c_in=C_IN):
    """The corrector's unscaled input [c_in][J] for iterate l from the scalar
    fluxes of iterates l, l-1, l-2 ([J][4] each), and the extrapolation factor."""
    d1, d2 = (p0 - p1).T, (p1 - p2).T
    if c_in == 8:
        return np.concatenate([d1, d2]), 0.0
    a = extrapolation_factor(p0, p1, p2)
    return np.concatenate([d1, d2, a * d1]), a


def samples(phis, ref, ls, first=1, c_in=C_IN):
    """Inputs [B][c_in][J], targets [B][4][J] and scales [B] for iterates l in
    ls (phis[i] is iterate first + i; l >= first + 2); samples whose last
    difference is zero are skipped."""
    xs, ts, ss, used = [], [], [], []
    for l in ls:
        i = l - first
        if i < 2 or i >= len(phis):
            continue
        x, a = features(phis[i], phis[i - 1], phis[i - 2], c_in)
        s = float(np.max(np.abs(phis[i] - phis[i - 1]))) * (1.0 + a)
        if not s > 0.0:
            continue
        xs.append(x / s)
        ts.append((ref - phis[i]).T / s)
        ss.append(s)
        used.append(l)
    if not xs:
        return None, None, np.zeros(0), []
    return (np.ascontiguousarray(np.stack(xs)), np.ascontiguousarray(np.stack(ts)), np.array(ss),
            used)


def init_weights(n_in, n_out, seed=0):
    """He-scaled normal weights for the four layers; the last layer 10x smaller
    (the first predictions stay near zero, i.e. near the plain iterate)."""
    rng = np.random.default_rng(seed)
    chans = [n_in, 32, 32, 32, n_out]
    out = []
    for l in range(4):
        std = np.sqrt(2.0 / (chans[l] * 5))
        if l == 3:
            std *= 0.1
        out.append(rng.normal(0.0, std, chans[l + 1] * chans[l] * 5))
    return np.concatenate(out)


def train(torch, x, t, epochs=400, lr=2e-3, seed=0, stream=None):
    """Full-batch Adam on device tensors x [B][c_in][J], t [B][4][J]; returns the
    corrector, the loss history and the training time in seconds."""
    B, c_in, J = x.shape
    k = oci.Corrector(c_in, C_OUT, B, J, stream=stream)
    k.set_weights(init_weights(c_in, C_OUT, seed))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = [k.train_step(x, t, lr) for _ in range(epochs)]
    torch.cuda.synchronize()
    return k, losses, time.perf_counter() - t0


def train_sets(torch, sets, epochs=200, lr=2e-3, seed=0, max_cells=None):
    """Adam over several data sets of different cell counts (one step per set
    and epoch, the sets in a seeded shuffled order each epoch); sets: list of
    (x [B][c_in][J], t [B][4][J]) device tensors.  Returns (corrector, mean
    loss per epoch, seconds).  The corrector is sized for the largest set (and
    at least max_cells cells of one sample, for inference on a larger mesh)."""
    mb = max(int(x.shape[0]) for x, _ in sets)
    mc = max(int(x.shape[2]) for x, _ in sets)
    c_in = int(sets[0][0].shape[1])
    if max_cells is not None:
        mc = max(mc, -(-int(max_cells) // mb))
    k = oci.Corrector(c_in, C_OUT, mb, mc)
    k.set_weights(init_weights(c_in, C_OUT, seed))
    rng = np.random.default_rng(seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = []
    for _ in range(epochs):
        ls = [k.train_step(sets[i][0], sets[i][1], lr) for i in rng.permutation(len(sets))]
        hist.append(float(np.mean(ls)))
    torch.cuda.synchronize()
    return k, hist, time.perf_counter() - t0


def evaluate(torch, k, phis, ref, ls, first=1, c_in=None):
    """Per iterate l: the plain error max|phi^(inf) - phi^(l)|, the corrected
    error max|phi^(inf) - (phi^(l) + s f(x))|, and the plain iterate count
    whose error first falls to the corrected one (None past the history)."""
    x, _, s, used = samples(phis, ref, ls, first, c_in=k.c_in if c_in is None else c_in)
    if x is None:
        return []
    y = k.forward(torch.from_numpy(np.ascontiguousarray(x)).to("cuda")).cpu().numpy()
    plain_all = [float(np.max(np.abs(ref - p))) for p in phis]
    rows = []
    for b, l in enumerate(used):
        corr = phis[l - first] + s[b] * y[b].T
        ec = float(np.max(np.abs(ref - corr)))
        eq = next((i + first for i, e in enumerate(plain_all) if e <= ec), None)
        rows.append({"l": l, "plain": plain_all[l - first], "corrected": ec,
                     "plain_equivalent": eq})
    return rows


def save_weights(path, w, meta, c_in=C_IN):
    with open(path, "w") as f:
        json.dump({"c_in": c_in, "c_out": C_OUT, "weights": [float(v) for v in w],
                   "meta": meta}, f)


def load_weights(path):
    """(weights, c_in, training record) from a file written by save_weights."""
    with open(path) as f:
        d = json.load(f)
    if d.get("c_in") not in (8, 12) or d.get("c_out") != C_OUT:
        raise ValueError("weights for another network shape")
    return np.array(d["weights"], dtype=np.float64), int(d["c_in"]), d.get("meta", {})

"""Training data and training for the learned iterate corrector.

The corrector (oci_corrector_* in the C ABI) maps the two latest differences
of OCI's scalar-flux iterates, per cell,
    x = [phi^(l) - phi^(l-1), phi^(l-1) - phi^(l-2)]       (8 channels),
to the iterate's remaining error, phi^(inf) - phi^(l) (4 channels).  The
network is positively homogeneous, so each sample is scaled by
s = max |phi^(l) - phi^(l-1)| (which leaves the prediction for the unscaled
input exact up to rounding) and every sample weighs alike in the loss.

The histories come from the library itself: the context's state is saved,
each iterate count l is run as a step of exactly l OCI iterations (tol 0,
max_iters l) from the saved state, and the converged step (tol tol_ref)
then advances the state.  The correction is evaluated on the scalar flux;
the iteration's own iterates (the outgoing fluxes) are not changed by it.
"""
import time

import numpy as np

from . import oci

C_IN, C_OUT = 8, 4


def step_history(ctx, prob, n_iter, tol_ref=1e-13, max_ref=100_000):
    """phi^(1) .. phi^(n_iter) of the context's current time step ([J][4] each),
    its converged phi, and the converged step's iteration count; the state
    ends advanced by the converged step."""
    psi, step = ctx.state()
    phis = []
    for l in range(1, n_iter + 1):
        ctx.set_state(psi, step)
        ctx.refactor(prob, tol=0.0, max_iters=l)
        ctx.step()
        phis.append(ctx.flux().copy())
    ctx.set_state(psi, step)
    ctx.refactor(prob, tol=tol_ref, max_iters=max_ref)
    _, info = ctx.step()
    return phis, ctx.flux().copy(), info


def samples(phis, ref, ls):
    """Inputs [B][8][J], targets [B][4][J] and scales [B] for iterates l in ls
    (1-based, l >= 3); samples whose last difference is zero are skipped."""
    xs, ts, ss, used = [], [], [], []
    for l in ls:
        d1 = phis[l - 1] - phis[l - 2]
        d2 = phis[l - 2] - phis[l - 3]
        s = float(np.max(np.abs(d1)))
        if not s > 0.0:
            continue
        xs.append(np.concatenate([d1.T, d2.T]) / s)
        ts.append((ref - phis[l - 1]).T / s)
        ss.append(s)
        used.append(l)
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
    """Full-batch Adam on device tensors x [B][8][J], t [B][4][J]; returns the
    corrector, the loss history and the training time in seconds."""
    B, _, J = x.shape
    k = oci.Corrector(C_IN, C_OUT, B, J, stream=stream)
    k.set_weights(init_weights(C_IN, C_OUT, seed))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = [k.train_step(x, t, lr) for _ in range(epochs)]
    torch.cuda.synchronize()
    return k, losses, time.perf_counter() - t0


def evaluate(torch, k, phis, ref, ls):
    """Per iterate l: the plain error max|phi^(inf) - phi^(l)|, the corrected
    error max|phi^(inf) - (phi^(l) + s f(x))|, and the plain iterate count
    whose error first falls to the corrected one (None past the history)."""
    x, _, s, used = samples(phis, ref, ls)
    y = k.forward(torch.from_numpy(np.ascontiguousarray(x)).to("cuda")).cpu().numpy()
    plain_all = [float(np.max(np.abs(ref - p))) for p in phis]
    rows = []
    for b, l in enumerate(used):
        corr = phis[l - 1] + s[b] * y[b].T
        ec = float(np.max(np.abs(ref - corr)))
        eq = next((i + 1 for i, e in enumerate(plain_all) if e <= ec), None)
        rows.append({"l": l, "plain": plain_all[l - 1], "corrected": ec, "plain_equivalent": eq})
    return rows

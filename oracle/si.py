"""Source iteration (SI), as the paper's SI subsection states it (oracle).

TEST INFRASTRUCTURE ONLY.

The scattering source is lagged: with the scalar flux phi^{(l)} of the previous
iteration, every angle is swept through the mesh along its direction, and each
cell solves the local 4x4 system A^+ x = b^+ (mu > 0) or A^- x = b^- (mu < 0),
where b carries (dx/4)(Sigma_s phi^{(l)} + Q), the previous time edge
psi_{k-1/2} and the flux entering from the upstream cell just computed in the
same sweep.  The new scalar flux is sum_n w_n psi_n, and iterations continue
until it stops changing (rule in ``stopping``).

Readings where the paper is silent:
* sweep order with reflection: with a reflecting left edge the mu < 0 angles
  are swept first and the mu > 0 sweep starts from their outgoing flux at
  x = 0 (exact, same iteration); with only the right edge reflecting the order
  is reversed; with both reflecting the mu < 0 sweep starts from the mu > 0
  outgoing flux at x = X of the previous iteration (lagged);
* first iterate: phi^(0) = 0 in the first step, the previous step's converged
  phi afterwards (warm start); the lagged right-edge reflection starts at 0.
"""
import numpy as np

from .oci import A_minus, A_plus
from .problem import INCIDENT, REFLECT, initial_edge_state
from .stopping import accept, relative_change


class AngleMatrices:
    """A^+ / A^- per region and angle, [R][N][4][4]."""

    def __init__(self, cd):
        regs = []
        start = 0
        reg = cd.region
        self.first_cell = []
        for r in range(int(reg.max()) + 1):
            cnt = int(np.sum(reg == r))
            self.first_cell.append(start)
            j0 = start
            start += cnt
            mats = np.zeros((cd.n, 4, 4))
            for m in range(cd.n):
                mu = cd.mu[m]
                f = A_plus if mu > 0 else A_minus
                mats[m] = f(mu, cd.dx[j0], cd.sig[j0], cd.a)
            regs.append(mats)
        self.mats = np.array(regs)


def _local_source(cd, phi, psi_prev):
    """b without the upstream term, [J][N][4] (same for all angles but the time term)."""
    J, n = cd.J, cd.n
    s = (cd.dx / 4.0)[:, None] * (cd.sigs[:, None] * phi + cd.q[:, None])   # [J][4]
    t2 = (cd.dx * cd.a / 2.0)[:, None]
    b = np.repeat(s[:, None, :], n, axis=1)
    b[:, :, 0] += t2 * psi_prev[:, :, 0]
    b[:, :, 1] += t2 * psi_prev[:, :, 1]
    return b


def _sweep(cd, mats, b, angles, incoming_k, incoming_h, psi):
    """Sweep the given angles (all of one sign) through the mesh in place.

    incoming_*: [len(angles)] flux entering the first cell of the sweep.
    Returns the outgoing flux at the last edge (level k, level k+1/2).
    """
    mu = cd.mu[angles]
    J = cd.J
    positive = mu[0] > 0
    order = range(J) if positive else range(J - 1, -1, -1)
    in_k = np.array(incoming_k, dtype=np.float64)
    in_h = np.array(incoming_h, dtype=np.float64)
    for j in order:
        r = cd.region[j]
        rhs = b[j, angles].copy()
        if positive:
            rhs[:, 0] += mu * in_k          # + mu psi_{k,j-1,R}
            rhs[:, 2] += mu * in_h          # + mu psi_{k+1/2,j-1,R}
        else:
            rhs[:, 1] -= mu * in_k          # - mu psi_{k,j+1,L}
            rhs[:, 3] -= mu * in_h          # - mu psi_{k+1/2,j+1,L}
        x = np.linalg.solve(mats[r][angles], rhs[:, :, None])[:, :, 0]
        psi[j, angles] = x
        if positive:
            in_k, in_h = x[:, 1], x[:, 3]
        else:
            in_k, in_h = x[:, 0], x[:, 2]
    return in_k, in_h


def si_sweep(cd, am, phi, psi_prev, lag_right):
    """One source iteration: all angles swept with the lagged scalar flux phi.

    lag_right: [N/2][2] previous iteration's mu > 0 outgoing flux at x = X
    (levels k, k+1/2), used only when both edges reflect.  Returns
    (psi [J][N][4], new lag_right).
    """
    n, J = cd.n, cd.J
    neg = np.arange(n // 2)              # mu < 0, ascending
    pos = np.arange(n // 2, n)           # mu > 0
    mirror_of_pos = n - 1 - pos          # the mu < 0 partner of each mu > 0 angle
    b = _local_source(cd, phi, psi_prev)
    psi = np.zeros((J, n, 4))

    def right_in():
        if cd.bc_right == INCIDENT:
            v = cd.inc_right[neg]
            return v, v
        return np.zeros(n // 2), np.zeros(n // 2)

    def left_in():
        if cd.bc_left == INCIDENT:
            v = cd.inc_left[pos]
            return v, v
        return np.zeros(n // 2), np.zeros(n // 2)

    new_lag = lag_right
    if cd.bc_left == REFLECT:
        if cd.bc_right == REFLECT:
            # entering angle m at x = X is leaving angle N-1-m, from the last iteration
            k_in = lag_right[::-1, 0]
            h_in = lag_right[::-1, 1]
        else:
            k_in, h_in = right_in()
        out_k, out_h = _sweep(cd, am.mats, b, neg, k_in, h_in, psi)
        # leaving at x = 0 in angle m' (mu < 0) enters in angle N-1-m' (mu > 0)
        idx = mirror_of_pos               # for each mu>0 angle, its mu<0 partner index in neg
        o_k, o_h = _sweep(cd, am.mats, b, pos, out_k[idx], out_h[idx], psi)
        new_lag = np.stack([o_k, o_h], axis=1)
    elif cd.bc_right == REFLECT:
        k_in, h_in = left_in()
        o_k, o_h = _sweep(cd, am.mats, b, pos, k_in, h_in, psi)
        # leaving at x = X in angle m (mu > 0) enters in angle N-1-m (mu < 0)
        _sweep(cd, am.mats, b, neg, o_k[::-1], o_h[::-1], psi)
    else:
        k_in, h_in = right_in()
        _sweep(cd, am.mats, b, neg, k_in, h_in, psi)
        k_in, h_in = left_in()
        _sweep(cd, am.mats, b, pos, k_in, h_in, psi)
    return psi, new_lag


def scalar_flux(cd, psi):
    return np.einsum("n,jnc->jc", cd.w, psi)


def si_step(cd, am, psi_prev, phi_start, lag_right, tol, max_iters, strict=False):
    phi = phi_start
    hist = []
    converged = False
    psi = None
    it = 0
    while it < max_iters:
        psi, lag_right = si_sweep(cd, am, phi, psi_prev, lag_right)
        it += 1
        phi_new = scalar_flux(cd, psi)
        hist.append(relative_change(phi_new, phi))
        phi = phi_new
        if accept(hist, tol, strict):
            converged = True
            break
    return {"psi": psi, "phi": phi, "iterations": it,
            "residual": hist[-1] if hist else None, "converged": converged,
            "history": hist, "lag_right": lag_right}


def run_si(prob, cd, n_steps, tol, max_iters, strict=False):
    am = AngleMatrices(cd)
    psi_prev = initial_edge_state(prob, cd)
    phi = np.zeros((cd.J, 4))
    lag = np.zeros((cd.n // 2, 2))
    out = []
    for _ in range(n_steps):
        res = si_step(cd, am, psi_prev, phi, lag, tol, max_iters, strict)
        phi = res["phi"]
        lag = res["lag_right"]
        psi_prev = res["psi"][:, :, 2:4].copy()
        res["psi_edge"] = psi_prev
        out.append(res)
    return out

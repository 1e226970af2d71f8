"""One-cell inversion (OCI), as the paper's OCI subsection states it (oracle).

TEST INFRASTRUCTURE ONLY.

Per cell j, all 4N angular fluxes (N angles; L and R half cells; levels k and
k+1/2) solve (A - S) Psi = c, where

* A = blockdiag(A_1 .. A_N), A_m = A^+ for mu_m > 0 and A^- for mu_m < 0,
  the 4x4 matrices printed in the SI subsection;
* S has entries (dx_j Sigma_{s,j} / 4) w_n.  Reading of the garbled index
  "S_{l,n}": the entry couples row (m, c) to column (n, c) of the same
  component c, i.e. S = (dx Sigma_s / 4) (1 w^T) (x) I_4, which is the
  scattering term (dx/4) Sigma_s phi_c of b^+/b^- with phi_c = sum_n w_n psi_{n,c};
* c = [c_1 .. c_N], c_m = c^+ or c^-: the source, the previous time edge
  psi_{k-1/2} and the incident fluxes from the neighbouring cells taken at the
  previous iterate l.

Each iteration solves every cell independently (parallel block Jacobi).  The
dense solve is LU with partial pivoting (LAPACK gesv in the paper); cells of a
region share A - S, so the factorisation is done once per region and every
cell of the region is one right-hand-side column of the solve.

Readings where the paper is silent:
* boundary: vacuum / prescribed incident fluxes enter c like a neighbour's
  value; a reflecting edge takes the mirror angle's outgoing flux of the
  boundary cell from the previous iterate (lagged, like every other incident
  flux of OCI);
* first iterate: zero in the first time step; in later steps the previous
  step's converged Psi (warm start);
* stopping rule: see ``stopping``.
"""
import numpy as np
import scipy.linalg as sla

from .problem import INCIDENT, REFLECT, initial_edge_state
from .stopping import accept, relative_change


def A_plus(mu, dx, sig, a):
    """A^+ of the SI subsection (mu > 0); a = 1/(v dt), so dx/(v dt) = dx*a."""
    d = (mu + dx * sig) / 2.0
    t = dx * a
    return np.array([
        [d, mu / 2.0, t / 2.0, 0.0],
        [-mu / 2.0, d, 0.0, t / 2.0],
        [-t, 0.0, t + d, mu / 2.0],
        [0.0, -t, -mu / 2.0, t + d],
    ])


def A_minus(mu, dx, sig, a):
    """A^- of the SI subsection (mu < 0): diagonal (-mu + dx Sigma)/2, off-diagonal mu/2."""
    d = (-mu + dx * sig) / 2.0
    t = dx * a
    return np.array([
        [d, mu / 2.0, t / 2.0, 0.0],
        [-mu / 2.0, d, 0.0, t / 2.0],
        [-t, 0.0, t + d, mu / 2.0],
        [0.0, -t, -mu / 2.0, t + d],
    ])


def cell_matrix(cd, dx, sig, sigs):
    """A - S for a cell with width dx and cross sections sig, sigs (4N x 4N)."""
    n = cd.n
    A = np.zeros((4 * n, 4 * n))
    for m in range(n):
        mu = cd.mu[m]
        blk = A_plus(mu, dx, sig, cd.a) if mu > 0 else A_minus(mu, dx, sig, cd.a)
        A[4 * m:4 * m + 4, 4 * m:4 * m + 4] = blk
    S = np.zeros((4 * n, 4 * n))
    for m in range(n):
        for nn in range(n):
            for c in range(4):
                S[4 * m + c, 4 * nn + c] = dx * sigs / 4.0 * cd.w[nn]
    return A - S


def incident_from_iterate(cd, psi):
    """Incident fluxes each cell sees from the iterate psi [J][N][4].

    Returns (up_k, up_h, dn_k, dn_h), each [J][N]:
    up_*[j, m] = psi^{(l)}_{m,level,j-1,R} (used for mu_m > 0),
    dn_*[j, m] = psi^{(l)}_{m,level,j+1,L} (used for mu_m < 0),
    with the boundary conditions in place of the missing neighbours.
    """
    J, n = cd.J, cd.n
    up_k = np.zeros((J, n))
    up_h = np.zeros((J, n))
    dn_k = np.zeros((J, n))
    dn_h = np.zeros((J, n))
    up_k[1:] = psi[:-1, :, 1]
    up_h[1:] = psi[:-1, :, 3]
    dn_k[:-1] = psi[1:, :, 0]
    dn_h[:-1] = psi[1:, :, 2]
    mirror = np.arange(n)[::-1]
    if cd.bc_left == REFLECT:
        # the flux entering at x = 0 in angle m is the flux leaving in angle N-1-m
        up_k[0] = psi[0, mirror, 0]
        up_h[0] = psi[0, mirror, 2]
    elif cd.bc_left == INCIDENT:
        up_k[0] = cd.inc_left
        up_h[0] = cd.inc_left
    if cd.bc_right == REFLECT:
        dn_k[-1] = psi[-1, mirror, 1]
        dn_h[-1] = psi[-1, mirror, 3]
    elif cd.bc_right == INCIDENT:
        dn_k[-1] = cd.inc_right
        dn_h[-1] = cd.inc_right
    return up_k, up_h, dn_k, dn_h


def rhs(cd, psi_prev, psi_iter):
    """c for every cell, [J][N][4], from c^+ / c^- of the OCI subsection."""
    J, n = cd.J, cd.n
    mu = cd.mu
    pos = mu > 0
    q4 = (cd.dx * cd.q / 4.0)[:, None]          # dx/4 * Q
    t2 = (cd.dx * cd.a / 2.0)[:, None]          # dx/(2 v dt)
    up_k, up_h, dn_k, dn_h = incident_from_iterate(cd, psi_iter)
    c = np.zeros((J, n, 4))
    c[:, :, 0] = q4 + t2 * psi_prev[:, :, 0]
    c[:, :, 1] = q4 + t2 * psi_prev[:, :, 1]
    c[:, :, 2] = q4
    c[:, :, 3] = q4
    # c^+: + mu psi^{(l)}_{k,j-1,R} in row 1 and + mu psi^{(l)}_{k+1/2,j-1,R} in row 3
    c[:, pos, 0] += mu[pos] * up_k[:, pos]
    c[:, pos, 2] += mu[pos] * up_h[:, pos]
    # c^-: - mu psi^{(l)}_{k,j+1,L} in row 2 and - mu psi^{(l)}_{k+1/2,j+1,L} in row 4
    neg = ~pos
    c[:, neg, 1] -= mu[neg] * dn_k[:, neg]
    c[:, neg, 3] -= mu[neg] * dn_h[:, neg]
    return c


class RegionFactors:
    """LU factors of A - S, one per region (cells of a region share it)."""

    def __init__(self, cd):
        self.cell_ranges = []
        self.lu = []
        start = 0
        reg = cd.region
        for r in range(int(reg.max()) + 1 if reg.size else 0):
            cnt = int(np.sum(reg == r))
            j0 = start
            start += cnt
            self.cell_ranges.append((j0, start))
            if cnt == 0:
                self.lu.append(None)
                continue
            M = cell_matrix(cd, cd.dx[j0], cd.sig[j0], cd.sigs[j0])
            self.lu.append(sla.lu_factor(M))


def sweep_cells(cd, factors, psi_prev, psi_iter):
    """One OCI iteration: every cell solved with incident fluxes from psi_iter."""
    J, n = cd.J, cd.n
    c = rhs(cd, psi_prev, psi_iter)
    out = np.empty((J, n, 4))
    for (j0, j1), lu in zip(factors.cell_ranges, factors.lu):
        if j1 == j0:
            continue
        C = c[j0:j1].reshape(j1 - j0, 4 * n).T     # one column per cell
        X = sla.lu_solve(lu, C)
        out[j0:j1] = X.T.reshape(j1 - j0, n, 4)
    return out


def scalar_flux(cd, psi):
    return np.einsum("n,jnc->jc", cd.w, psi)


def oci_step(cd, factors, psi_prev, psi_start, tol, max_iters, strict=False):
    """Iterate one time step to the stopping rule.

    Returns dict: psi (last iterate), phi, iterations, residual (e of the last
    iterate, None if undefined), converged, history.
    """
    psi = psi_start
    phi_old = None
    hist = []
    converged = False
    it = 0
    while it < max_iters:
        psi = sweep_cells(cd, factors, psi_prev, psi)
        it += 1
        phi = scalar_flux(cd, psi)
        hist.append(None if phi_old is None else relative_change(phi, phi_old))
        phi_old = phi
        if accept(hist, tol, strict):
            converged = True
            break
    if it == 0:
        phi_old = scalar_flux(cd, psi)
    return {"psi": psi, "phi": phi_old, "iterations": it,
            "residual": hist[-1] if hist else None,
            "converged": converged, "history": hist}


def run_oci(prob, cd, n_steps, tol, max_iters, strict=False, psi_prev=None, psi_start=None):
    """Step the problem n_steps times with OCI (warm start between steps)."""
    factors = RegionFactors(cd)
    if psi_prev is None:
        psi_prev = initial_edge_state(prob, cd)
    psi = np.zeros((cd.J, cd.n, 4)) if psi_start is None else psi_start
    out = []
    for _ in range(n_steps):
        res = oci_step(cd, factors, psi_prev, psi, tol, max_iters, strict)
        psi = res["psi"]
        psi_prev = psi[:, :, 2:4].copy()
        res["psi_edge"] = psi_prev
        out.append(res)
    return out

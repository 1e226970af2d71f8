"""The MB-SCB balance equations of one time step, and their direct solution.

TEST INFRASTRUCTURE ONLY.

This module is the plain definition of the result.  Each time step of the
method is the linear system formed by, for every cell j and angle m:

* the four half-cell balances eq:scb-mb-a .. eq:scb-mb-d (Sec. "Derivation of
  MB-SCB"): time-average balance on the left and right half cells, and the
  auxiliary half-step balance on both halves;
* the first closure: the cell-midpoint flux is the average of the two
  half-cell fluxes, at both time levels;
* the second closure: the cell-edge flux is taken upstream (the left cell's
  R value for mu > 0, the right cell's L value for mu < 0), at both levels;
* the boundary conditions: prescribed incident flux at x = 0 for mu > 0 and
  at x = X for mu < 0 (vacuum = zero); a reflecting edge sets the incoming
  flux equal to the outgoing flux of the mirror angle at the same edge and the
  same time level.

The equations are written term by term exactly as printed (each multiplied
through by nothing: dx/2 * (1/v) * (.)/dt becomes h*a*(.), with h = dx/2 and
a = 1/(v dt); the half-step equations carry (.)/(dt/2), i.e. h*2a*(.)).

Unknowns per cell and angle, in the order of the paper's psi_n vector (OCI
subsection): c = 0: psi_{k,L}, 1: psi_{k,R}, 2: psi_{k+1/2,L}, 3: psi_{k+1/2,R}.
Global index ((j*N) + m)*4 + c (cell-major, angles ascending).

``solve_sparse`` uses a library sparse LU on the assembled system (tiny
meshes); ``solve_block_tridiagonal`` eliminates cell by cell with dense 4N x 4N
blocks (block Gaussian elimination, library LU for each pivot block) for
medium meshes.  Tests check that both agree.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .problem import INCIDENT, REFLECT, mirror

KL, KR, HL, HR = 0, 1, 2, 3   # c index: time level k / k+1/2, half cell L / R
LEVEL_COMPS = {0: (KL, KR), 1: (HL, HR)}   # level 0 = k, level 1 = k+1/2


def _edge(cd, j, m, level, side):
    """Resolve the cell-edge flux psi_{m,level,j+-1/2} by the upstream closure.

    side = -1 for the left edge j-1/2, +1 for the right edge j+1/2.
    Returns ('u', dj, mm, c) for an unknown of cell j+dj, or ('k', value) for a
    boundary constant.
    """
    n, J = cd.n, cd.J
    L_c, R_c = LEVEL_COMPS[level]
    mu = cd.mu[m]
    if side < 0:                       # edge j - 1/2
        if mu < 0:
            return ("u", 0, m, L_c)    # upstream is this cell's left half
        if j > 0:
            return ("u", -1, m, R_c)   # upstream is the left neighbour's right half
        # x = 0, incoming direction
        if cd.bc_left == REFLECT:
            return ("u", 0, mirror(n, m), L_c)   # outgoing mirror angle at x = 0
        return ("k", cd.inc_left[m] if cd.bc_left == INCIDENT else 0.0)
    else:                              # edge j + 1/2
        if mu > 0:
            return ("u", 0, m, R_c)
        if j < J - 1:
            return ("u", 1, m, L_c)
        if cd.bc_right == REFLECT:
            return ("u", 0, mirror(n, m), R_c)
        return ("k", cd.inc_right[m] if cd.bc_right == INCIDENT else 0.0)


def local_equations(cd, j, psi_prev_j):
    """The 4N balance equations of cell j.

    Returns (D, Lm, Up, b): coefficient blocks on the unknowns of cells j, j-1
    and j+1 (each 4N x 4N, row/col index m*4 + c) and the right-hand side.
    psi_prev_j is [N][2]: psi_{m,k-1/2} at the L and R half cells.
    """
    n = cd.n
    size = 4 * n
    D = np.zeros((size, size))
    Lm = np.zeros((size, size))
    Up = np.zeros((size, size))
    b = np.zeros(size)
    h = 0.5 * cd.dx[j]
    a = cd.a
    sig, sigs, q = cd.sig[j], cd.sigs[j], cd.q[j]
    blocks = {-1: Lm, 0: D, 1: Up}

    def add(row, dj, mm, c, coef):
        blocks[dj][row, mm * 4 + c] += coef

    def add_edge(row, coef, m, level, side):
        e = _edge(cd, j, m, level, side)
        if e[0] == "u":
            add(row, e[1], e[2], e[3], coef)
        else:
            b[row] -= coef * e[1]

    for m in range(n):
        mu = cd.mu[m]
        r = m * 4
        # eq:scb-mb-a  (time average, left half)
        row = r + KL
        add(row, 0, m, HL, h * a)
        b[row] += h * a * psi_prev_j[m, 0]
        add(row, 0, m, KL, 0.5 * mu)
        add(row, 0, m, KR, 0.5 * mu)
        add_edge(row, -mu, m, 0, -1)
        add(row, 0, m, KL, h * sig)
        # eq:scb-mb-b  (time average, right half)
        row = r + KR
        add(row, 0, m, HR, h * a)
        b[row] += h * a * psi_prev_j[m, 1]
        add_edge(row, mu, m, 0, +1)
        add(row, 0, m, KL, -0.5 * mu)
        add(row, 0, m, KR, -0.5 * mu)
        add(row, 0, m, KR, h * sig)
        # eq:scb-mb-c  (half step, left half)
        row = r + HL
        add(row, 0, m, HL, h * 2.0 * a)
        add(row, 0, m, KL, -h * 2.0 * a)
        add(row, 0, m, HL, 0.5 * mu)
        add(row, 0, m, HR, 0.5 * mu)
        add_edge(row, -mu, m, 1, -1)
        add(row, 0, m, HL, h * sig)
        # eq:scb-mb-d  (half step, right half)
        row = r + HR
        add(row, 0, m, HR, h * 2.0 * a)
        add(row, 0, m, KR, -h * 2.0 * a)
        add_edge(row, mu, m, 1, +1)
        add(row, 0, m, HL, -0.5 * mu)
        add(row, 0, m, HR, -0.5 * mu)
        add(row, 0, m, HR, h * sig)
    # right side of every one of the four equations:
    # (dx/2)(1/2)(Sigma_s sum_n w_n psi_{n,c} + Q), scattering moved to the left
    for c in (KL, KR, HL, HR):
        D[c::4, c::4] -= h * 0.5 * sigs * cd.w[None, :]
    b += h * 0.5 * q
    return D, Lm, Up, b


def assemble(cd, psi_prev):
    """Global sparse matrix and right-hand side of one time step (tiny meshes)."""
    J, n = cd.J, cd.n
    size = 4 * n
    rows, cols, vals = [], [], []
    rhs = np.zeros(J * size)
    for j in range(J):
        D, Lm, Up, b = local_equations(cd, j, psi_prev[j])
        rhs[j * size:(j + 1) * size] = b
        for dj, blk in ((-1, Lm), (0, D), (1, Up)):
            if not (0 <= j + dj < J):
                assert not np.any(blk)
                continue
            rr, cc = np.nonzero(blk)
            rows.append(rr + j * size)
            cols.append(cc + (j + dj) * size)
            vals.append(blk[rr, cc])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(J * size, J * size))
    return A, rhs


def solve_sparse(cd, psi_prev):
    """Psi [J][N][4] of one time step by a sparse direct solve."""
    A, rhs = assemble(cd, psi_prev)
    x = spla.spsolve(A.tocsc(), rhs)
    return x.reshape(cd.J, cd.n, 4)


def solve_block_tridiagonal(cd, psi_prev):
    """Psi [J][N][4] of one time step by block Gaussian elimination over cells.

    Forward sweep: D'_0 = D_0, D'_j = D_j - L_j D'_{j-1}^{-1} U_{j-1};
    back substitution from the last cell.
    """
    J, n = cd.J, cd.n
    size = 4 * n
    ys = []          # D'^{-1}-applied right-hand sides
    zs = []          # D'^{-1} U_j, kept on the nonzero columns of U_j only
    zcols = []
    for j in range(J):
        D, Lm, Up, b = local_equations(cd, j, psi_prev[j])
        if j > 0:
            D = D.copy()
            D[:, zcols[-1]] -= Lm @ zs[-1]
            b = b - Lm @ ys[-1]
        lu = sla.lu_factor(D)
        ys.append(sla.lu_solve(lu, b))
        cols = np.nonzero(np.any(Up != 0.0, axis=0))[0]
        zcols.append(cols)
        zs.append(sla.lu_solve(lu, Up[:, cols]) if cols.size else np.zeros((size, 0)))
    x = np.zeros((J, size))
    x[J - 1] = ys[J - 1]
    for j in range(J - 2, -1, -1):
        x[j] = ys[j] - zs[j] @ x[j + 1][zcols[j]]
    return x.reshape(J, n, 4)


def scalar_flux(cd, psi):
    """phi_c = sum_n w_n psi_{n,c} for each cell, [J][4] (SI subsection)."""
    return np.einsum("n,jnc->jc", cd.w, psi)


def edge_state(psi):
    """psi_{k+1/2} at the L and R half cells, [J][N][2]: the next step's psi_{k-1/2}."""
    return psi[:, :, [HL, HR]].copy()


def run_direct(prob, cd, n_steps, psi_prev=None, solver="auto"):
    """Step the problem n_steps times by direct solves.

    Returns a list of dicts with phi [J][4], psi [J][N][4] and the next state.
    """
    from .problem import initial_edge_state
    if psi_prev is None:
        psi_prev = initial_edge_state(prob, cd)
    out = []
    for _ in range(n_steps):
        if solver == "sparse" or (solver == "auto" and cd.J * cd.n <= 4096):
            psi = solve_sparse(cd, psi_prev)
        else:
            psi = solve_block_tridiagonal(cd, psi_prev)
        psi_prev = edge_state(psi)
        out.append({"phi": scalar_flux(cd, psi), "psi": psi, "psi_edge": psi_prev})
    return out

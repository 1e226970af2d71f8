"""Per-cell data of a slab problem, derived from its region table (oracle).

TEST INFRASTRUCTURE ONLY.

A problem is any object with these attributes (the seeded generators in the
package's ``workloads`` module produce one; the oracle reads it duck-typed and
imports nothing from the package):

* ``n_angles``            N, even
* ``mu``, ``w``           optional [N] quadrature override (ascending mu)
* ``cells``               [R] cells per region; region r is uniform with
                          dx_r = width_r / cells_r
* ``width``, ``sigma_t``, ``sigma_s``, ``source``   [R]
* ``dt``, ``speed``       time step and particle speed; speed = inf gives the
                          steady equations (the 1/(v dt) terms vanish)
* ``bc_left``, ``bc_right``   0 vacuum, 1 reflecting, 2 prescribed incident
* ``inc_left``            [N/2] incident psi at x = 0 for the mu > 0 angles
                          (ascending mu), ``inc_right`` [N/2] at x = X for the
                          mu < 0 angles; time-constant
* ``psi0``                optional [J][N][2] initial psi at the L and R half
                          cells (None = 0)

Data model: Sec. "Derivation of MB-SCB" (S_N equation with Sigma(x),
Sigma_s(x), Q(x); initial and boundary conditions) and the region-wise data of
Sec. "Transient Reed's Problem".  Reading of the time levels of the data: the
source and incident fluxes are time-constant, so Q_k = Q_{k+1/2} and the
incident flux is the same at both time levels; the half-cell sources
Q_{j,L} = Q_{j,R} equal the region's Q.
"""
from dataclasses import dataclass

import numpy as np

from .quadrature import gauss_legendre

VACUUM, REFLECT, INCIDENT = 0, 1, 2


@dataclass
class CellData:
    n: int            # angles
    mu: np.ndarray    # [N]
    w: np.ndarray     # [N]
    dx: np.ndarray    # [J]
    sig: np.ndarray   # [J] total cross section
    sigs: np.ndarray  # [J] scattering cross section
    q: np.ndarray     # [J] isotropic source Q
    region: np.ndarray  # [J] region index
    a: float          # 1/(v dt), 0 for steady
    bc_left: int
    bc_right: int
    inc_left: np.ndarray   # [N] (entries for mu > 0 used)
    inc_right: np.ndarray  # [N] (entries for mu < 0 used)

    @property
    def J(self):
        return self.dx.shape[0]


def cell_data(prob):
    n = int(prob.n_angles)
    if n < 2 or n % 2:
        raise ValueError("the number of angles must be even (odd Gauss-Legendre sets hold mu = 0)")
    mu = getattr(prob, "mu", None)
    w = getattr(prob, "w", None)
    if mu is None or w is None:
        mu, w = gauss_legendre(n)
    mu = np.asarray(mu, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    cells = np.asarray(prob.cells, dtype=np.int64)
    width = np.asarray(prob.width, dtype=np.float64)
    region = np.repeat(np.arange(cells.shape[0]), cells)
    dx = (width / cells)[region]
    sig = np.asarray(prob.sigma_t, dtype=np.float64)[region]
    sigs = np.asarray(prob.sigma_s, dtype=np.float64)[region]
    q = np.asarray(prob.source, dtype=np.float64)[region]
    speed = float(prob.speed)
    a = 0.0 if np.isinf(speed) else 1.0 / (speed * float(prob.dt))
    inc_l = np.zeros(n)
    inc_r = np.zeros(n)
    if prob.bc_left == INCIDENT:
        inc_l[n // 2:] = np.asarray(prob.inc_left, dtype=np.float64)
    if prob.bc_right == INCIDENT:
        inc_r[: n // 2] = np.asarray(prob.inc_right, dtype=np.float64)
    return CellData(n, mu, w, dx, sig, sigs, q, region, a,
                    int(prob.bc_left), int(prob.bc_right), inc_l, inc_r)


def initial_edge_state(prob, cd):
    """psi at the L and R half cells at t = 0, [J][N][2] (zero if psi0 is None)."""
    psi0 = getattr(prob, "psi0", None)
    if psi0 is None:
        return np.zeros((cd.J, cd.n, 2))
    return np.array(psi0, dtype=np.float64).reshape(cd.J, cd.n, 2)


def mirror(n, m):
    """Index of the angle with mu = -mu_m in an ascending symmetric set."""
    return n - 1 - m

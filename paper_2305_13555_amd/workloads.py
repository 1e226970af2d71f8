"""Seeded synthetic slab problems (input generation only, no method arithmetic).

The paper's workloads are a transient multi-region Reed-type problem (region
data only in a figure) and a homogeneous slab swept over c, Sigma*dx, dt and
N (Sec. "GPU Explorations Across Quadrature Sets").  No data set ships with
the paper, so these generators stand in for them: region tables drawn from a
fixed-seed generator, with the shapes and ranges stated per config.

This module is shared by the tests, the benchmark, the oracle's callers and
the GPU binding's callers; it holds no part of the transport method.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

VACUUM, REFLECT, INCIDENT = 0, 1, 2
SEED = 230513555


@dataclass
class SlabProblem:
    n_angles: int
    cells: np.ndarray            # [R] int
    width: np.ndarray            # [R]
    sigma_t: np.ndarray          # [R]
    sigma_s: np.ndarray          # [R]
    source: np.ndarray           # [R]
    dt: float
    speed: float
    bc_left: int = VACUUM
    bc_right: int = VACUUM
    inc_left: Optional[np.ndarray] = None    # [N/2], mu > 0 angles ascending
    inc_right: Optional[np.ndarray] = None   # [N/2], mu < 0 angles ascending
    psi0: Optional[np.ndarray] = None        # [J][N][2]
    n_steps: int = 1
    tol: float = 1e-10
    max_iters: int = 1000
    strict: bool = False
    mu: Optional[np.ndarray] = None
    w: Optional[np.ndarray] = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_cells(self):
        return int(np.sum(self.cells))

    @property
    def n_regions(self):
        return int(len(self.cells))


def _rng(cfg, idx=0):
    return np.random.default_rng([SEED, cfg, idx])


def split_cells(J, R):
    """Regions split the cells evenly: J_r = J//R + (r < J%R)."""
    return np.array([J // R + (1 if r < J % R else 0) for r in range(R)], dtype=np.int32)


def _draw_regions(rng, R, tau_lo=0.01, tau_hi=10.0):
    """Per-region sigma_t, c, Q (vectorised draws in this order)."""
    sigma_t = np.clip(rng.lognormal(0.0, 1.0, R), tau_lo, tau_hi)
    c = rng.uniform(0.5, 0.99, R)
    q = rng.uniform(0.0, 1.0, R)
    return sigma_t, c, q


def config1():
    """Homogeneous slab, width 10, 100 cells, S_8, sigma_t = 1, c = 0.9, Q = 1,
    vacuum both sides, zero initial flux, v = 1, dt = 0.1, 10 steps, tol 1e-10."""
    return SlabProblem(
        n_angles=8, cells=np.array([100], np.int32), width=np.array([10.0]),
        sigma_t=np.array([1.0]), sigma_s=np.array([0.9]), source=np.array([1.0]),
        dt=0.1, speed=1.0, bc_left=VACUUM, bc_right=VACUUM, n_steps=10, tol=1e-10,
        name="homogeneous slab, 100 cells, S8, 10 steps")


def config2(paper_regime=False, n_cells=10_000, n_regions=16, n_angles=32, n_steps=100):
    """16 regions, 10,000 cells, S_32, sigma_t lognormal(0, 1) clipped to
    [0.01, 10] with dx = 1 (cell optical thickness 0.01-10 mfp), c ~ U[0.5, 0.99],
    Q ~ U[0, 1] per region, reflecting left / vacuum right, dt = 0.05, v = 1
    (paper_regime: v = 80 so 1/(v dt) = 0.25), 100 steps, tol 1e-10."""
    rng = _rng(2)
    sigma_t, c, q = _draw_regions(rng, n_regions)
    cells = split_cells(n_cells, n_regions)
    return SlabProblem(
        n_angles=n_angles, cells=cells, width=cells.astype(np.float64) * 1.0,
        sigma_t=sigma_t, sigma_s=c * sigma_t, source=q,
        dt=0.05, speed=80.0 if paper_regime else 1.0,
        bc_left=REFLECT, bc_right=VACUUM, n_steps=n_steps, tol=1e-10,
        name="16 regions, %d cells, S%d, reflect/vacuum, %d steps%s" % (
            n_cells, n_angles, n_steps, ", 1/(v dt)=0.25" if paper_regime else ""))


def config3(n_steps=50):
    """64 regions, 200,000 cells, S_64, draws as config 2, 50 steps, tol 1e-6."""
    rng = _rng(3)
    R, J = 64, 200_000
    sigma_t, c, q = _draw_regions(rng, R)
    cells = split_cells(J, R)
    return SlabProblem(
        n_angles=64, cells=cells, width=cells.astype(np.float64),
        sigma_t=sigma_t, sigma_s=c * sigma_t, source=q, dt=0.05, speed=1.0,
        bc_left=REFLECT, bc_right=VACUUM, n_steps=n_steps, tol=1e-6,
        name="64 regions, 200000 cells, S64, 50 steps")


def _config4_problem(rng, J, N, R, name, n_steps):
    """Thin-cell, highly scattering slab: per region sigma_t lognormal(0, 1)
    clipped to [0.01, 10], c ~ U[0.9, 0.999], Q ~ U[0, 1] (drawn in that order),
    then the cell optical thickness tau ~ logU[0.01, 0.5] (dx = tau / sigma_t);
    reflecting left / vacuum right, dt = 1, v = 4 (1/(v dt) = 0.25)."""
    sigma_t = np.clip(rng.lognormal(0.0, 1.0, R), 0.01, 10.0)
    c = rng.uniform(0.9, 0.999, R)
    q = rng.uniform(0.0, 1.0, R)
    tau = np.exp(rng.uniform(np.log(0.01), np.log(0.5), R))
    cells = split_cells(J, R)
    dx = tau / sigma_t
    return SlabProblem(
        n_angles=N, cells=cells, width=cells * dx, sigma_t=sigma_t, sigma_s=c * sigma_t,
        source=q, dt=1.0, speed=4.0, bc_left=REFLECT, bc_right=VACUUM, n_steps=n_steps,
        tol=1e-6, max_iters=200_000, name=name)


def config4(idx, n_steps=5):
    """Training problem idx of the learned corrector: J = round(exp U[ln 1e3,
    ln 5e4]) cells, N uniform in {16, 32, 64}, 16 regions, thin cells (optical
    thickness 0.01 - 0.5) with scattering ratio 0.9 - 0.999, dt = 1, v = 4,
    5 steps.  Each problem has its own generator (config 4, index idx)."""
    rng = _rng(4, idx)
    J = int(round(np.exp(rng.uniform(np.log(1e3), np.log(5e4)))))
    N = int(rng.choice([16, 32, 64]))
    return _config4_problem(rng, J, N, 16, "thin-cell problem %d: %d cells, S%d, 16 regions"
                            % (idx, J, N), n_steps)


def config4_eval(n_steps=5, n_cells=100_000, n_angles=128, n_regions=64):
    """Evaluation problem of the learned corrector (config 4, index 10,000):
    100,000 cells, S_128, 64 regions, draws as config4."""
    rng = _rng(4, 10_000)
    return _config4_problem(rng, n_cells, n_angles, n_regions,
                            "thin-cell evaluation problem: %d cells, S%d, %d regions"
                            % (n_cells, n_angles, n_regions), n_steps)


def config5(idx, n_steps=20):
    """Problem idx of the ensemble: J = round(exp U[ln 500, ln 1e5]) cells, N
    uniform in {8, 16, 32, 64, 128}, 16 regions with draws as config 2
    (dx = 1), reflecting left / vacuum right, dt = 0.05, v = 1, 20 steps,
    tol 1e-10.  Each problem has its own generator (config 5, index idx)."""
    rng = _rng(5, idx)
    J = int(round(np.exp(rng.uniform(np.log(500.0), np.log(1e5)))))
    N = int(rng.choice([8, 16, 32, 64, 128]))
    R = 16
    sigma_t, c, q = _draw_regions(rng, R)
    cells = split_cells(J, R)
    return SlabProblem(
        n_angles=N, cells=cells, width=cells.astype(np.float64),
        sigma_t=sigma_t, sigma_s=c * sigma_t, source=q, dt=0.05, speed=1.0,
        bc_left=REFLECT, bc_right=VACUUM, n_steps=n_steps, tol=1e-10,
        name="ensemble problem %d: %d cells, S%d, 16 regions" % (idx, J, N))


def homogeneous_slab(n_angles, n_cells, c, sigma_dx, dt, speed=1.0, sigma_t=2.0,
                     source=0.1, n_steps=5, width=None):
    """The paper's quadrature-sweep slab: sigma_t = 2, Q = 0.1, vacuum both
    sides, zero initial flux, 5 steps; width follows from sigma*dx and J."""
    dx = sigma_dx / sigma_t
    w = dx * n_cells if width is None else width
    return SlabProblem(
        n_angles=n_angles, cells=np.array([n_cells], np.int32), width=np.array([w]),
        sigma_t=np.array([sigma_t]), sigma_s=np.array([c * sigma_t]),
        source=np.array([source]), dt=dt, speed=speed, n_steps=n_steps,
        name="homogeneous slab S%d J=%d c=%g sdx=%g dt=%g" % (n_angles, n_cells, c, sigma_dx, dt))


def random_small(seed, n_cells=None, n_regions=None, n_angles=None, bc=None,
                 dt=None, speed=None, incident=True, psi0=True):
    """Small random multi-region problem for parity tests (mixed BCs, psi0)."""
    rng = np.random.default_rng([SEED, 99, seed])
    R = int(n_regions if n_regions is not None else rng.integers(1, 5))
    J = int(n_cells if n_cells is not None else rng.integers(R, 40))
    N = int(n_angles if n_angles is not None else rng.choice([2, 4, 8]))
    cells = np.array(rng.multinomial(J - R, np.ones(R) / R) + 1, dtype=np.int32)
    dx = np.exp(rng.uniform(np.log(0.02), np.log(3.0), R))
    sigma_t = np.exp(rng.uniform(np.log(0.2), np.log(4.0), R))
    c = rng.uniform(0.0, 0.99, R)
    q = rng.uniform(0.0, 1.0, R)
    if bc is None:
        bl, br = int(rng.integers(0, 3)), int(rng.integers(0, 3))
    else:
        bl, br = bc
    inc_l = rng.uniform(0.0, 1.0, N // 2) if (bl == INCIDENT and incident) else None
    inc_r = rng.uniform(0.0, 1.0, N // 2) if (br == INCIDENT and incident) else None
    if bl == INCIDENT and inc_l is None:
        inc_l = np.zeros(N // 2)
    if br == INCIDENT and inc_r is None:
        inc_r = np.zeros(N // 2)
    p0 = rng.uniform(0.0, 0.5, (J, N, 2)) if psi0 else None
    return SlabProblem(
        n_angles=N, cells=cells, width=dx * cells, sigma_t=sigma_t,
        sigma_s=c * sigma_t, source=q,
        dt=float(dt if dt is not None else np.exp(rng.uniform(np.log(0.01), np.log(2.0)))),
        speed=float(speed if speed is not None else np.exp(rng.uniform(np.log(0.5), np.log(10.0)))),
        bc_left=bl, bc_right=br, inc_left=inc_l, inc_right=inc_r, psi0=p0,
        n_steps=3, tol=1e-12, max_iters=20000, name="random small #%d" % seed)


def layout_case(seed, sizes, n_angles, bc, dt=0.3, speed=2.0, psi0=True):
    """Multi-region problem with the given cells per region (tiny regions put
    tile and halo edges next to region and domain edges); per-region data
    drawn as in random_small."""
    rng = np.random.default_rng([SEED, 77, seed])
    cells = np.array(sizes, dtype=np.int32)
    R, J, N = len(sizes), int(np.sum(sizes)), int(n_angles)
    dx = np.exp(rng.uniform(np.log(0.05), np.log(2.0), R))
    sigma_t = np.exp(rng.uniform(np.log(0.2), np.log(4.0), R))
    c = rng.uniform(0.0, 0.99, R)
    q = rng.uniform(0.0, 1.0, R)
    bl, br = bc
    inc_l = rng.uniform(0.0, 1.0, N // 2) if bl == INCIDENT else None
    inc_r = rng.uniform(0.0, 1.0, N // 2) if br == INCIDENT else None
    p0 = rng.uniform(0.0, 0.5, (J, N, 2)) if psi0 else None
    return SlabProblem(
        n_angles=N, cells=cells, width=dx * cells, sigma_t=sigma_t, sigma_s=c * sigma_t,
        source=q, dt=dt, speed=speed, bc_left=bl, bc_right=br, inc_left=inc_l,
        inc_right=inc_r, psi0=p0, n_steps=3, tol=1e-12, max_iters=20000,
        name="layout case #%d (%d regions, %d cells, S%d)" % (seed, R, J, N))

"""Pins for the oracle's discrete equations, direct solve, OCI and SI.

Every test here checks the oracle against something other than itself: the
paper's printed matrices, closed forms of the discrete scheme, exact
properties of the iterations, or an independent algorithm.
"""
import dataclasses

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import balance, oci, si, spectral
from oracle.problem import cell_data
from paper_2305_13555_amd import workloads as W


def _slab(**kw):
    base = dict(n_angles=4, cells=np.array([5]), width=np.array([5.0]),
                sigma_t=np.array([1.0]), sigma_s=np.array([0.5]), source=np.array([1.0]),
                dt=0.1, speed=1.0)
    base.update(kw)
    return W.SlabProblem(**base)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# --------------------------------------------------------------------------
# P2: balance equations == the printed A^+/A^-, S, c^+/c^- of the OCI section
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(6))
def test_balance_blocks_equal_printed_oci_system(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.choice([2, 4, 8]))
    p = _slab(n_angles=n, cells=np.array([3]), width=np.array([3 * rng.uniform(0.05, 2)]),
              sigma_t=np.array([rng.uniform(0.1, 3)]), sigma_s=np.array([rng.uniform(0, 1)]),
              source=np.array([rng.uniform(0, 2)]), dt=rng.uniform(0.01, 1), speed=rng.uniform(0.5, 5))
    cd = cell_data(p)
    prev = rng.uniform(0, 1, (3, n, 2))
    D, Lm, Up, b = balance.local_equations(cd, 1, prev[1])
    M = oci.cell_matrix(cd, cd.dx[1], cd.sig[1], cd.sigs[1])
    np.testing.assert_allclose(D, M, rtol=1e-14, atol=1e-15)
    # For any iterate, the middle cell's balance residual equals (A - S) Psi_j - c_j
    psi = rng.uniform(-1, 1, (3, n, 4))
    lhs = D @ psi[1].ravel() + Lm @ psi[0].ravel() + Up @ psi[2].ravel() - b
    c = oci.rhs(cd, prev, psi)[1].ravel()
    np.testing.assert_allclose(lhs, M @ psi[1].ravel() - c, rtol=1e-13, atol=1e-14)


def test_printed_A_plus_minus_from_unified_form():
    # A^- is A^+ with |mu| on the diagonal; off-diagonals keep the signed mu/2.
    mu, dx, sig, a = 0.7, 0.3, 1.7, 2.0
    Ap = oci.A_plus(mu, dx, sig, a)
    Am = oci.A_minus(-mu, dx, sig, a)
    np.testing.assert_allclose(np.diag(Ap), np.diag(Am))
    off = ~np.eye(4, dtype=bool)
    np.testing.assert_allclose(Ap[off] * np.where(np.abs(Ap[off]) == mu / 2, -1, 1), Am[off])


# --------------------------------------------------------------------------
# Direct solvers agree; OCI and SI converge to the direct solution (P6)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(8))
def test_direct_oci_si_share_the_fixed_point(seed):
    p = W.random_small(seed)
    cd = cell_data(p)
    d = balance.run_direct(p, cd, 2, solver="sparse")
    blk = balance.run_direct(p, cd, 2, solver="block")
    o = oci.run_oci(p, cd, 2, 1e-13, 50000, strict=True)
    s = si.run_si(p, cd, 2, 1e-13, 50000, strict=True)
    for k in range(2):
        assert _rel(blk[k]["phi"], d[k]["phi"]) < 1e-13
        assert o[k]["converged"] and s[k]["converged"]
        assert _rel(o[k]["phi"], d[k]["phi"]) < 5e-12
        assert _rel(s[k]["phi"], d[k]["phi"]) < 5e-12
        assert _rel(o[k]["psi_edge"], d[k]["psi_edge"]) < 5e-12


# --------------------------------------------------------------------------
# P3: flat infinite medium (reflecting both edges), closed form per step
# --------------------------------------------------------------------------
def _flat_step(Q, sig, sigs, a, phi_minus):
    sa = sig - sigs
    det = sa * sa + 2 * a * sa + 2 * a * a
    phik = ((Q + a * phi_minus) * (2 * a + sa) - a * Q) / det
    phih = (sa * Q + 2 * a * (Q + a * phi_minus)) / det
    return phik, phih


@pytest.mark.parametrize("n,J,c", [(2, 3, 0.5), (8, 7, 0.9), (16, 4, 1.0)])
def test_flat_infinite_medium_closed_form(n, J, c):
    Q, sig, v, dt, phi0 = 0.7, 1.3, 2.0, 0.25, 0.4
    p = _slab(n_angles=n, cells=np.array([J]), width=np.array([J * 0.37]),
              sigma_t=np.array([sig]), sigma_s=np.array([c * sig]), source=np.array([Q]),
              dt=dt, speed=v, bc_left=W.REFLECT, bc_right=W.REFLECT,
              psi0=np.full((J, n, 2), phi0 / 2.0))
    cd = cell_data(p)
    a = 1.0 / (v * dt)
    d = balance.run_direct(p, cd, 4)
    o = oci.run_oci(p, cd, 4, 1e-14, 100000, strict=True)
    s = si.run_si(p, cd, 4, 1e-14, 100000, strict=True)
    phim = phi0
    for k in range(4):
        phik, phih = _flat_step(Q, sig, c * sig, a, phim)
        expect = np.tile([phik, phik, phih, phih], (J, 1))
        for res, tol in ((d[k], 2e-14), (o[k], 1e-12), (s[k], 1e-12)):
            np.testing.assert_allclose(res["phi"], expect, rtol=tol)
        phim = phih


# --------------------------------------------------------------------------
# P4 and spatial order: MB is second order in time, SCB second order in space
# --------------------------------------------------------------------------
def test_mb_second_order_in_time():
    Q, sig, c, v, T = 1.0, 1.0, 0.5, 1.0, 2.0
    sa = sig * (1 - c)
    exact = Q / sa * (1 - np.exp(-v * sa * T))
    errs = []
    for dt in (0.2, 0.1, 0.05, 0.025):
        p = _slab(n_angles=4, cells=np.array([3]), width=np.array([3.0]), sigma_t=np.array([sig]),
                  sigma_s=np.array([c * sig]), source=np.array([Q]), dt=dt, speed=v,
                  bc_left=W.REFLECT, bc_right=W.REFLECT)
        cd = cell_data(p)
        r = balance.run_direct(p, cd, int(round(T / dt)))
        errs.append(abs(r[-1]["phi"][0, 2] - exact))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(ratios > 3.8) and np.all(ratios < 4.2), ratios


@pytest.mark.parametrize("n", [2, 8])
def test_scb_second_order_in_space(n):
    # steady pure absorber lit from the left: psi_m(x) = exp(-Sigma x / mu_m)
    errs, exits = [], []
    for J in (20, 40, 80, 160):
        p = _slab(n_angles=n, cells=np.array([J]), width=np.array([2.0]), sigma_t=np.array([1.0]),
                  sigma_s=np.array([0.0]), source=np.array([0.0]), dt=1.0, speed=np.inf,
                  bc_left=W.INCIDENT, bc_right=W.VACUUM, inc_left=np.ones(n // 2))
        cd = cell_data(p)
        psi = balance.solve_sparse(cd, np.zeros((J, n, 2)))
        x = np.linspace(0, 2, J + 1)
        mu = cd.mu[n // 2:]
        dx = 2.0 / J
        cell_avg = np.stack([m / dx * (np.exp(-x[:-1] / m) - np.exp(-x[1:] / m)) for m in mu], 1)
        got = 0.5 * (psi[:, n // 2:, 0] + psi[:, n // 2:, 1])
        errs.append(np.max(np.abs(got - cell_avg)))
        exits.append(np.max(np.abs(psi[-1, n // 2:, 1] - np.exp(-2.0 / mu))))
        assert np.max(np.abs(psi[:, : n // 2])) < 1e-15     # nothing travels left
    r1 = errs[-2] / errs[-1]
    r2 = exits[-2] / exits[-1]
    assert 3.4 < r1 < 4.4 and 3.7 < r2 < 4.3, (errs, exits)


# --------------------------------------------------------------------------
# P5: without scattering, OCI is exact after exactly J iterations; SI after one
# --------------------------------------------------------------------------
@pytest.mark.parametrize("J,n", [(6, 4), (9, 2), (5, 8)])
def test_oci_nilpotent_without_scattering(J, n):
    rng = np.random.default_rng(J)
    p = W.SlabProblem(n_angles=n, cells=np.array([2, J - 2]), width=np.array([0.6, 2.0]),
                      sigma_t=np.array([1.0, 2.5]), sigma_s=np.zeros(2), source=np.array([1.0, 0.3]),
                      dt=0.2, speed=1.5, bc_left=W.INCIDENT, bc_right=W.VACUUM,
                      inc_left=rng.uniform(0.2, 1.0, n // 2), psi0=rng.uniform(0, 1, (J, n, 2)))
    cd = cell_data(p)
    ref = balance.solve_sparse(cd, np.asarray(p.psi0))
    f = oci.RegionFactors(cd)
    psi = rng.uniform(-5, 5, (J, n, 4))            # any start
    for it in range(1, J + 1):
        psi = oci.sweep_cells(cd, f, np.asarray(p.psi0), psi)
        if it == J - 1:
            assert _rel(psi, ref) > 1e-10     # not yet exact one iteration earlier
    assert _rel(psi, ref) < 1e-13


@pytest.mark.parametrize("bc", [(W.REFLECT, W.VACUUM), (W.VACUUM, W.REFLECT), (W.INCIDENT, W.INCIDENT)])
def test_si_exact_after_one_sweep_without_scattering(bc):
    p = W.random_small(3, bc=bc)
    p = dataclasses.replace(p, sigma_s=np.zeros_like(p.sigma_s))
    cd = cell_data(p)
    ref = balance.solve_sparse(cd, np.asarray(p.psi0))
    am = si.AngleMatrices(cd)
    psi, _ = si.si_sweep(cd, am, np.full((cd.J, 4), 3.0), np.asarray(p.psi0), np.zeros((cd.n // 2, 2)))
    assert _rel(psi, ref) < 1e-13


# --------------------------------------------------------------------------
# P7: a reflecting edge is a mirror: half of the symmetric doubled slab
# --------------------------------------------------------------------------
def test_reflecting_edge_is_a_mirror():
    p = W.random_small(11, bc=(W.REFLECT, W.VACUUM), n_angles=8, psi0=False)
    cd = cell_data(p)
    half = balance.run_direct(p, cd, 3)
    R = p.n_regions
    rev = slice(None, None, -1)
    dbl = W.SlabProblem(n_angles=p.n_angles,
                        cells=np.concatenate([p.cells[rev], p.cells]),
                        width=np.concatenate([p.width[rev], p.width]),
                        sigma_t=np.concatenate([p.sigma_t[rev], p.sigma_t]),
                        sigma_s=np.concatenate([p.sigma_s[rev], p.sigma_s]),
                        source=np.concatenate([p.source[rev], p.source]),
                        dt=p.dt, speed=p.speed, bc_left=W.VACUUM, bc_right=W.VACUUM)
    cdd = cell_data(dbl)
    full = balance.run_direct(dbl, cdd, 3)
    J = cd.J
    assert R >= 1
    for k in range(3):
        assert _rel(full[k]["phi"][J:], half[k]["phi"]) < 1e-12
        # and the left half is the mirror image (L <-> R swapped)
        assert _rel(full[k]["phi"][:J][::-1][:, [1, 0, 3, 2]], half[k]["phi"]) < 1e-12


# --------------------------------------------------------------------------
# P8: particle balance of every cell, at both time levels
# --------------------------------------------------------------------------
def _edge_currents(cd, psi, level):
    """Net current sum_m w_m mu_m psi_edge at the J+1 edges (upstream closure)."""
    J, n = cd.J, cd.n
    Lc, Rc = (0, 1) if level == 0 else (2, 3)
    pos = cd.mu > 0
    edge = np.zeros((J + 1, n))
    edge[1:, pos] = psi[:, pos, Rc]
    edge[:-1, ~pos] = psi[:, ~pos, Lc]
    mir = np.arange(n)[::-1]
    if cd.bc_left == W.REFLECT:
        edge[0, pos] = psi[0, mir, Lc][pos]
    else:
        edge[0, pos] = cd.inc_left[pos]
    if cd.bc_right == W.REFLECT:
        edge[J, ~pos] = psi[-1, mir, Rc][~pos]
    else:
        edge[J, ~pos] = cd.inc_right[~pos]
    return edge @ (cd.w * cd.mu)


@pytest.mark.parametrize("seed", range(5))
def test_particle_balance(seed):
    p = W.random_small(seed + 20)
    cd = cell_data(p)
    prev = np.asarray(p.psi0)
    psi = balance.solve_sparse(cd, prev)
    phi = np.einsum("n,jnc->jc", cd.w, psi)
    phi_prev = np.einsum("n,jnc->jc", cd.w, prev)
    sa = cd.sig - cd.sigs
    Jk = _edge_currents(cd, psi, 0)
    Jh = _edge_currents(cd, psi, 1)
    h = cd.dx / 2
    bal_k = (h * cd.a * (phi[:, 2] - phi_prev[:, 0] + phi[:, 3] - phi_prev[:, 1])
             + (Jk[1:] - Jk[:-1]) + h * sa * (phi[:, 0] + phi[:, 1]) - cd.dx * cd.q)
    bal_h = (h * 2 * cd.a * (phi[:, 2] - phi[:, 0] + phi[:, 3] - phi[:, 1])
             + (Jh[1:] - Jh[:-1]) + h * sa * (phi[:, 2] + phi[:, 3]) - cd.dx * cd.q)
    scale = np.max(np.abs(phi)) * np.max(cd.dx * (cd.sig + cd.a) + 1)
    assert np.max(np.abs(bal_k)) < 1e-13 * scale
    assert np.max(np.abs(bal_h)) < 1e-13 * scale


# --------------------------------------------------------------------------
# P9: the cell solve by Woodbury (blockdiag A_m plus rank-4 scattering) == LU
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 8, 32])
def test_cell_solve_woodbury_equals_lu(n):
    rng = np.random.default_rng(n)
    p = _slab(n_angles=n, sigma_s=np.array([0.95]), dt=0.3, speed=0.7)
    cd = cell_data(p)
    dx, sig, sigs = 0.4, 1.0, 0.95
    M = oci.cell_matrix(cd, dx, sig, sigs)
    c = rng.uniform(-1, 1, 4 * n)
    x_lu = sla.lu_solve(sla.lu_factor(M), c)
    # M = A - U V with U = (dx sigs / 4)(1_N (x) I4), V = (w^T (x) I4)
    Ainv_blocks = [np.linalg.inv(oci.A_plus(mu, dx, sig, cd.a) if mu > 0 else
                                 oci.A_minus(mu, dx, sig, cd.a)) for mu in cd.mu]
    def Ainv(v):
        v = v.reshape(n, 4, -1)
        return np.concatenate([Ainv_blocks[m] @ v[m] for m in range(n)]).reshape(4 * n, -1)
    U = np.kron(np.ones((n, 1)), np.eye(4)) * dx * sigs / 4
    V = np.kron(cd.w[None, :], np.eye(4))
    y = Ainv(c)
    AU = Ainv(U)
    cap = np.eye(4) - V @ AU
    x_w = (y + AU @ np.linalg.solve(cap, V @ y)).ravel()
    np.testing.assert_allclose(x_w, x_lu, rtol=1e-12, atol=1e-13)


# --------------------------------------------------------------------------
# P10: the spectral-radius trends of Fig. 1 (steady, S_4, reflecting both edges)
# --------------------------------------------------------------------------
def _rho(sdx, c, J=6, speed=np.inf, dt=1.0):
    p = _slab(n_angles=4, cells=np.array([J]), width=np.array([J * sdx]), sigma_t=np.array([1.0]),
              sigma_s=np.array([c]), source=np.array([1.0]), dt=dt, speed=speed,
              bc_left=W.REFLECT, bc_right=W.REFLECT)
    cd = cell_data(p)
    return (spectral.spectral_radius(spectral.oci_iteration_matrix(cd)),
            spectral.spectral_radius(spectral.si_iteration_matrix(cd)))


def test_spectral_radius_trends():
    sdx = [0.01, 0.1, 1.0, 10.0]
    o9 = [_rho(s, 0.9) for s in sdx]
    oci9 = [r[0] for r in o9]
    # OCI falls steeply with cell optical thickness
    assert all(a > b for a, b in zip(oci9, oci9[1:])), oci9
    assert oci9[0] > 0.99 and oci9[-1] < 0.5
    # SI is governed by c: for many-mfp problems it is nearly c, whatever the cell size
    assert abs(o9[-1][1] - 0.9) < 0.01 and abs(o9[-2][1] - 0.9) < 0.02
    # thin cells: OCI slower than SI; thick cells: faster
    assert o9[0][0] > o9[0][1] and o9[-1][0] < o9[-1][1]
    # both converge faster with less scattering
    o5 = [_rho(s, 0.5) for s in (0.1, 1.0)]
    assert o5[0][0] < o9[1][0] and o5[1][0] < o9[2][0]
    assert o5[1][1] < o9[2][1]
    # the time term (1/(v dt) > 0) lowers OCI's spectral radius
    assert _rho(0.01, 0.99, speed=1.0, dt=0.05)[0] < _rho(0.01, 0.99)[0] - 0.1

"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Tolerances (FP64 path):
* same number of iterations on both sides (max_iters fixed, tol = 0): the two
  compute the same iterates in a different order of rounding; the library
  also applies (A - S)^{-1} through its precomputed rows, whose error is
  ~cond(A - S) * eps < 1e-13.  Bound: 1e-11 relative to max|phi|.
* converged steps: library and oracle OCI use the same stopping rule and
  agree to the same bound; against the direct solve (the exact fixed point)
  the stopping rule leaves an error of order tol * rho/(1-rho): bound 1e-10
  relative for the paper-sized tolerance 1e-10 cases run strict, 1e-9 otherwise.
"""
import dataclasses

import numpy as np
import pytest

from oracle import balance
from oracle import oci as ooci
from oracle import si as osi
from oracle.problem import cell_data, initial_edge_state
from paper_2305_13555_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_13555_amd import oci
    return oci


def rel(a, b):
    s = float(np.max(np.abs(b))) if np.size(b) else 0.0
    return float(np.max(np.abs(a - b))) / (s if s > 0 else 1.0)


def gpu_run(lib, prob, n_steps, method="oci", **kw):
    out = []
    with lib.OciContext(prob, **kw) as ctx:
        for _ in range(n_steps):
            rc, info = ctx.step() if method == "oci" else ctx.si_step()
            info["rc"] = rc
            info["phi"] = ctx.flux().copy()
            info["psi_edge"] = ctx.state()[0]
            out.append(info)
    return out


# ---------------------------------------------------------------------------
# a1: the per-region operator equals rows of (A - S)^{-1} [B | T | q]
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 8, 32])
def test_operator_matches_cell_inverse(lib, n):
    p = W.random_small(5, n_angles=n, n_regions=3, n_cells=20)
    cd = cell_data(p)
    with lib.OciContext(p) as ctx:
        for r in range(3):
            op = ctx.operator(r)
            j = int(np.sum(p.cells[:r]))
            M = ooci.cell_matrix(cd, cd.dx[j], cd.sig[j], cd.sigs[j])
            N = n
            C = np.zeros((4 * N, 4 * N + 1))
            for m in range(N):
                for t in range(2):
                    i = 2 * m + t
                    cin = (1 if t == 0 else 3) if cd.mu[m] < 0 else (0 if t == 0 else 2)
                    C[4 * m + cin, i] = abs(cd.mu[m])
                for s in range(2):
                    C[4 * m + s, 2 * N + 2 * m + s] = cd.dx[j] * cd.a / 2
            C[:, 4 * N] = cd.dx[j] * cd.q[j] / 4
            Y = np.linalg.solve(M, C)
            rows = []
            for m in range(N):
                for t in range(2):
                    c = (0 if t == 0 else 2) if cd.mu[m] < 0 else (1 if t == 0 else 3)
                    rows.append(Y[4 * m + c])
            for c in range(4):
                rows.append(sum(cd.w[m] * Y[4 * m + c] for m in range(N)))
            for m in range(N):
                for s in range(2):
                    rows.append(Y[4 * m + 2 + s])
            expect = np.array(rows)
            assert rel(op, expect) < 1e-13


# ---------------------------------------------------------------------------
# a2-a6: identical iterates for a fixed number of iterations
# ---------------------------------------------------------------------------
CASES = [(s, None) for s in range(8)] + [
    (100, dict(n_angles=2, n_cells=1, n_regions=1)),
    (101, dict(n_angles=16, n_cells=17, n_regions=1)),
    (102, dict(n_angles=8, n_cells=33, n_regions=2, bc=(W.REFLECT, W.REFLECT))),
    (103, dict(n_angles=4, n_cells=40, n_regions=3, bc=(W.INCIDENT, W.INCIDENT))),
    (104, dict(n_angles=6, n_cells=23, n_regions=2, bc=(W.REFLECT, W.INCIDENT))),
    (105, dict(n_angles=64, n_cells=20, n_regions=2, bc=(W.VACUUM, W.REFLECT))),
    (106, dict(n_angles=128, n_cells=9, n_regions=1, bc=(W.REFLECT, W.VACUUM))),
    (107, dict(n_angles=256, n_cells=5, n_regions=1, bc=(W.INCIDENT, W.REFLECT))),
    # several tiles per region at the angle counts of the multi-iterate
    # launches, with incident and vacuum edges (halo cells at fixed ghosts)
    (108, dict(n_angles=16, n_cells=70, n_regions=3, bc=(W.INCIDENT, W.INCIDENT))),
    (109, dict(n_angles=32, n_cells=53, n_regions=2, bc=(W.VACUUM, W.INCIDENT))),
    (110, dict(n_angles=8, n_cells=45, n_regions=4, bc=(W.INCIDENT, W.VACUUM))),
]


@pytest.mark.parametrize("seed,kw", CASES)
@pytest.mark.parametrize("iters", [1, 4, 7])
def test_fixed_iterations_match_oracle_oci(lib, seed, kw, iters):
    p = W.random_small(seed, **(kw or {}))
    cd = cell_data(p)
    ref = ooci.run_oci(p, cd, 3, tol=0.0, max_iters=iters)
    got = gpu_run(lib, p, 3, tol=0.0, max_iters=iters)
    for k in range(3):
        # tol = 0 stops only at the limit, or where an iterate repeats the
        # one before bit for bit (e = 0: a small problem converged to
        # rounding), which the two sides may reach one iterate apart
        assert ref[k]["iterations"] <= iters
        if ref[k]["iterations"] == iters:
            assert got[k]["iterations"] == iters
        else:
            assert abs(got[k]["iterations"] - ref[k]["iterations"]) <= 1
        assert got[k]["rc"] in (lib.OCI_NOT_CONVERGED, lib.OCI_OK)
        assert rel(got[k]["phi"], ref[k]["phi"]) < 1e-11, (seed, k)
        assert rel(got[k]["psi_edge"], ref[k]["psi_edge"]) < 1e-11, (seed, k)


# Tile layouts: regions of one or two cells (halo cells in other regions,
# halo cells next to a reflecting edge: a tile starting at cell 1 or ending
# at cell J-2), the four-wave split of the scalar-flux rows (N = 32), the
# shared scalar-flux row tile (N = 12), and more regions than the region
# table in the kernel arguments holds (tile table path).
LAYOUTS = [
    (0, [1, 17, 1, 2, 30, 1], 8, (W.REFLECT, W.REFLECT)),
    (1, [3, 40, 1, 20], 32, (W.INCIDENT, W.REFLECT)),
    (2, [1 + (r * 7) % 6 for r in range(40)], 4, (W.REFLECT, W.VACUUM)),
    (3, [5, 33, 2], 12, (W.VACUUM, W.INCIDENT)),
    (4, [16, 16, 1, 15], 16, (W.REFLECT, W.INCIDENT)),
    # S_64 with regions of 3 .. 40 cells: the multi-iterate launches with the
    # halo cells' tables of other regions read from memory
    (5, [3, 20, 3, 33, 5], 64, (W.REFLECT, W.REFLECT)),
    (6, [4, 40, 17, 3], 64, (W.INCIDENT, W.VACUUM)),
]


@pytest.mark.parametrize("case", LAYOUTS, ids=lambda c: "layout%d" % c[0])
@pytest.mark.parametrize("iters", [1, 2, 3, 4, 5])
def test_tile_layouts_fixed_iterations(lib, case, iters):
    seed, sizes, n, bc = case
    p = W.layout_case(seed, sizes, n, bc)
    cd = cell_data(p)
    ref = ooci.run_oci(p, cd, 3, tol=0.0, max_iters=iters)
    got = gpu_run(lib, p, 3, tol=0.0, max_iters=iters)
    for k in range(3):
        assert got[k]["iterations"] == iters
        assert rel(got[k]["phi"], ref[k]["phi"]) < 1e-11, (seed, iters, k)
        assert rel(got[k]["psi_edge"], ref[k]["psi_edge"]) < 1e-11, (seed, iters, k)


@pytest.mark.parametrize("case", LAYOUTS, ids=lambda c: "layout%d" % c[0])
def test_tile_layouts_converged(lib, case):
    seed, sizes, n, bc = case
    p = W.layout_case(seed, sizes, n, bc)
    cd = cell_data(p)
    direct = balance.run_direct(p, cd, 2)
    got = gpu_run(lib, p, 2, tol=1e-12, max_iters=50000, strict=True)
    for k in range(2):
        assert got[k]["rc"] == lib.OCI_OK
        assert rel(got[k]["phi"], direct[k]["phi"]) < 1e-10


@pytest.mark.parametrize("seed,kw", CASES[:12])
def test_fixed_iterations_match_oracle_si(lib, seed, kw):
    p = W.random_small(seed, **(kw or {}))
    cd = cell_data(p)
    ref = osi.run_si(p, cd, 3, tol=0.0, max_iters=3)
    got = gpu_run(lib, p, 3, method="si", tol=0.0, max_iters=3)
    for k in range(3):
        assert got[k]["iterations"] == 3
        assert rel(got[k]["phi"], ref[k]["phi"]) < 1e-11, (seed, k)
        assert rel(got[k]["psi_edge"], ref[k]["psi_edge"]) < 1e-11, (seed, k)


# ---------------------------------------------------------------------------
# converged steps: against oracle OCI (same rule) and the direct solve
# ---------------------------------------------------------------------------
def test_config1_ten_steps(lib):
    p = W.config1()
    cd = cell_data(p)
    ref = ooci.run_oci(p, cd, 10, tol=1e-10, max_iters=1000)
    direct = balance.run_direct(p, cd, 10)
    got = gpu_run(lib, p, 10)
    its_g = [g["iterations"] for g in got]
    its_o = [r["iterations"] for r in ref]
    assert all(abs(a - b) <= 1 for a, b in zip(its_g, its_o)), (its_g, its_o)
    assert sum(a == b for a, b in zip(its_g, its_o)) >= 8
    for k in range(10):
        assert got[k]["rc"] == lib.OCI_OK
        assert got[k]["residual"] <= 1e-10
        assert rel(got[k]["phi"], ref[k]["phi"]) < 1e-10
        assert rel(got[k]["phi"], direct[k]["phi"]) < 1e-9


@pytest.mark.parametrize("seed", range(6))
def test_strict_converged_matches_direct(lib, seed):
    p = W.random_small(seed + 40)
    cd = cell_data(p)
    direct = balance.run_direct(p, cd, 2)
    got = gpu_run(lib, p, 2, tol=1e-12, max_iters=50000, strict=True)
    for k in range(2):
        assert got[k]["rc"] == lib.OCI_OK
        assert rel(got[k]["phi"], direct[k]["phi"]) < 1e-10
        # the strict rule accepted the iterate on the bound the step reports
        assert 0.0 <= got[k]["err_bound"] <= 1e-12
    got_si = gpu_run(lib, p, 2, method="si", tol=1e-12, max_iters=50000, strict=True)
    for k in range(2):
        assert got_si[k]["rc"] == lib.OCI_OK
        assert rel(got_si[k]["phi"], direct[k]["phi"]) < 1e-10
        assert 0.0 <= got_si[k]["err_bound"] <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_many_tiles_match_oracle(lib, precision):
    """40,000 cells (2,500 tiles): the last iterate's residual is reduced once
    before the end of step instead of by every work-group."""
    p = W.config2(n_cells=40000, n_regions=4, n_angles=8, n_steps=3)
    ref = ooci.run_oci(p, cell_data(p), 3, tol=1e-10, max_iters=1000)
    prec = lib.OCI_PREC_FP64 if precision == "fp64" else lib.OCI_PREC_FP32
    with lib.OciContext(p, precision=prec) as ctx:
        phi = np.zeros((3, p.n_cells, 4))
        rc, infos = ctx.solve(3, phi)
    assert rc == lib.OCI_OK
    for k in range(3):
        if precision == "fp64":
            assert abs(infos[k]["iterations"] - ref[k]["iterations"]) <= 1
        assert rel(phi[k], ref[k]["phi"]) < 1e-9


def test_config2_full_size_first_steps(lib):
    """Full-size multi-region problem (10,000 cells, S_32): first 3 steps."""
    p = W.config2(n_steps=3)
    cd = cell_data(p)
    ref = ooci.run_oci(p, cd, 3, tol=1e-10, max_iters=1000)
    got = gpu_run(lib, p, 3)
    for k in range(3):
        assert abs(got[k]["iterations"] - ref[k]["iterations"]) <= 1
        assert rel(got[k]["phi"], ref[k]["phi"]) < 1e-10
        assert got[k]["rc"] == lib.OCI_OK


def test_flat_infinite_medium_closed_form(lib):
    n, J, c, Q, sig, v, dt, phi0 = 16, 37, 0.9, 0.7, 1.3, 2.0, 0.25, 0.4
    p = W.SlabProblem(n_angles=n, cells=np.array([J]), width=np.array([J * 0.37]),
                      sigma_t=np.array([sig]), sigma_s=np.array([c * sig]), source=np.array([Q]),
                      dt=dt, speed=v, bc_left=W.REFLECT, bc_right=W.REFLECT,
                      psi0=np.full((J, n, 2), phi0 / 2.0))
    got = gpu_run(lib, p, 3, tol=1e-13, max_iters=100000, strict=True)
    a = 1.0 / (v * dt)
    sa = sig * (1 - c)
    det = sa * sa + 2 * a * sa + 2 * a * a
    phim = phi0
    for k in range(3):
        phik = ((Q + a * phim) * (2 * a + sa) - a * Q) / det
        phih = (sa * Q + 2 * a * (Q + a * phim)) / det
        expect = np.tile([phik, phik, phih, phih], (J, 1))
        assert rel(got[k]["phi"], expect) < 1e-11
        phim = phih


# ---------------------------------------------------------------------------
# API behaviour
# ---------------------------------------------------------------------------
def test_not_converged_and_state_advances(lib):
    p = W.config1()
    with lib.OciContext(p, max_iters=2, tol=1e-14) as ctx:
        rc, info = ctx.step()
        assert rc == lib.OCI_NOT_CONVERGED and info["iterations"] == 2
        assert ctx.state()[1] == 1


def test_nonfinite_detected(lib):
    p = W.random_small(3, n_angles=4, n_cells=10, n_regions=1, psi0=True)
    p.psi0 = np.full((10, 4, 2), 1.7e308)
    p.speed, p.dt = 1e-3, 1e-3
    with lib.OciContext(p) as ctx:
        with pytest.raises(lib.OciError) as ei:
            ctx.step()
        assert ei.value.code == lib.OCI_ENONFINITE
        assert ctx.state()[1] == 0


def test_deterministic_and_checkpoint_resume(lib):
    p = W.random_small(7, n_angles=8, n_cells=50, n_regions=3)
    a = gpu_run(lib, p, 4)
    b = gpu_run(lib, p, 4)
    for k in range(4):
        assert np.array_equal(a[k]["phi"], b[k]["phi"])          # bitwise repeatable
    with lib.OciContext(p) as ctx:
        ctx.step()
        ctx.step()
        psi, step = ctx.state()
        assert step == 2
    with lib.OciContext(p) as ctx:
        ctx.set_state(psi, step)
        for k in range(2):
            ctx.step()
            assert rel(ctx.flux(), a[2 + k]["phi"]) < 1e-9
        assert ctx.state()[1] == 4


def test_solve_to_device_tensor_and_mixed_si(lib):
    import torch
    p = W.random_small(9, n_angles=8, n_cells=30)
    cd = cell_data(p)
    direct = balance.run_direct(p, cd, 4)
    with lib.OciContext(p, tol=1e-12, max_iters=100000, strict=True) as ctx:
        out = torch.zeros((2, ctx.n_cells, 4), dtype=torch.float64, device="cuda")
        rc, infos = ctx.solve(2, out)
        assert rc == lib.OCI_OK and len(infos) == 2
        got = out.cpu().numpy()
        for k in range(2):
            assert rel(got[k], direct[k]["phi"]) < 1e-10
        ctx.si_step()
        assert rel(ctx.flux(), direct[2]["phi"]) < 1e-10
        ctx.step()
        assert rel(ctx.flux(), direct[3]["phi"]) < 1e-10


def test_quadrature_and_steady(lib):
    p = W.random_small(12, n_angles=8, n_cells=12, n_regions=2)
    p = dataclasses.replace(p, speed=np.inf, psi0=None)
    cd = cell_data(p)
    direct = balance.run_direct(p, cd, 1)
    with lib.OciContext(p, tol=1e-13, max_iters=200000, strict=True) as ctx:
        mu, w = ctx.quadrature()
        np.testing.assert_allclose(mu, cd.mu, atol=1e-15)
        ctx.step()
        assert rel(ctx.flux(), direct[0]["phi"]) < 1e-10


@pytest.mark.parametrize("which", ["config1", "config2_small"])
def test_queued_solve_matches_step_by_step(lib, which):
    """oci_solve queues every step with a fixed batch of iteration launches;
    steps that need more stall the queue and are resumed from the host.  The
    result must equal stepping one at a time, bit for bit (same tile
    arithmetic, same decisions).  config1 needs ~19 iterations per step, so
    the first queue (batch 2) stalls at every step."""
    import torch
    p = W.config1() if which == "config1" else W.config2(n_steps=4, n_cells=700, n_regions=5,
                                                           n_angles=16)
    steps = 4
    a = gpu_run(lib, p, steps)
    with lib.OciContext(p) as ctx:
        out = torch.zeros((steps, ctx.n_cells, 4), dtype=torch.float64, device="cuda")
        rc, infos = ctx.solve(steps, out)
        assert rc == lib.OCI_OK
        got = out.cpu().numpy()
        psi = ctx.state()[0]
        assert ctx.state()[1] == steps
    for k in range(steps):
        assert infos[k]["iterations"] == a[k]["iterations"]
        assert np.array_equal(got[k], a[k]["phi"])
    assert np.array_equal(psi, a[-1]["psi_edge"])


@pytest.mark.parametrize("cap", ["1", "2", "3"])
def test_launch_shape_cap_agrees(lib, monkeypatch, cap):
    """Iterates per launch (up to four: halo cells recomputed level by level)
    change only the rounding order at tile edges: capping the launch shape
    with OCI_ITERATES_PER_LAUNCH gives the same steps to rounding."""
    import torch
    p = W.config2(n_steps=6, n_cells=700, n_regions=5, n_angles=32)
    steps = 6

    def run():
        with lib.OciContext(p) as ctx:
            out = torch.zeros((steps, ctx.n_cells, 4), dtype=torch.float64, device="cuda")
            rc, infos = ctx.solve(steps, out)
            assert rc == lib.OCI_OK
            return ctx.iterates_per_launch, out.cpu().numpy(), infos

    k0, phi0, inf0 = run()
    assert k0 == 4
    monkeypatch.setenv("OCI_ITERATES_PER_LAUNCH", cap)
    k1, phi1, inf1 = run()
    assert k1 == int(cap)
    for k in range(steps):
        assert abs(inf1[k]["iterations"] - inf0[k]["iterations"]) <= 1
        assert rel(phi1[k], phi0[k]) < 1e-11
    ref = ooci.run_oci(p, cell_data(p), steps, tol=p.tol, max_iters=p.max_iters)
    for k in range(steps):
        assert rel(phi1[k], ref[k]["phi"]) < 1e-9


# The angle-lane SI sweep over many segments and regions (segments of ~4 cells
# per chunk, chunks of regions' edges, the entering-flux scan across
# segments), every boundary kind, the cross-row lane sums of N = 64 and 128
@pytest.mark.parametrize("n,bc", [(64, (W.REFLECT, W.REFLECT)), (64, (W.INCIDENT, W.VACUUM)),
                                  (128, (W.VACUUM, W.REFLECT)), (16, (W.REFLECT, W.INCIDENT))])
def test_si_many_segments_match_oracle(lib, n, bc):
    p = W.random_small(200 + n, n_cells=700, n_regions=5, n_angles=n, bc=bc)
    cd = cell_data(p)
    ref = osi.run_si(p, cd, 2, tol=0.0, max_iters=3)
    got = gpu_run(lib, p, 2, method="si", tol=0.0, max_iters=3)
    for k in range(2):
        assert got[k]["iterations"] == 3
        assert rel(got[k]["phi"], ref[k]["phi"]) < 1e-11, (n, k)
        assert rel(got[k]["psi_edge"], ref[k]["psi_edge"]) < 1e-11, (n, k)

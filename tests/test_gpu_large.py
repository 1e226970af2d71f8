"""GPU parity at the kernel instances large problems run, against the FP64 oracle.

Problems with more than 768 tiles read their tile descriptors from a table
(not the kernel arguments), and past 2,048 tiles the end of step reduces the
last iterate's residual records in a separate launch.  The angle counts 64
and 128 have kernels built for them.  The 200,000-cell S_64 problem (64
regions, reflecting left / vacuum right, tol 1e-6) runs exactly these
instances, so they are compared here with the oracle element by element:

* fixed iteration counts (tol = 0): same iterates in another rounding order,
  1e-11 relative to max|phi|;
* converged steps with the same stopping rule: 1e-10 relative and iteration
  counts within one;
* the large problem's first step itself, plain FP64 at tol 1e-10 against the
  oracle at the same rule, and plain and mixed precision at tol 1e-6 against
  the oracle's step converged to 1e-13 (the mixed path's bound is 1e-6).
"""
import numpy as np
import pytest

from oracle import oci as ooci
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


def gpu_steps(lib, prob, n_steps, **kw):
    """n_steps queued steps (oci_solve into a host array), with their records."""
    with lib.OciContext(prob, **kw) as ctx:
        phi = np.zeros((n_steps, prob.n_cells, 4))
        rc, infos = ctx.solve(n_steps, phi)
        psi = ctx.state()[0]
    return rc, phi, infos, psi


def n_tiles(prob):
    return int(sum((int(c) + 15) // 16 for c in prob.cells))


# 64 regions and S_64 like the large problem, 40,000 cells: 2,560 tiles
def n64_problem():
    return W.config2(n_cells=40_000, n_regions=64, n_angles=64, n_steps=3)


# S_128 with table tiles and the separate record reduction: 34,000 cells, 2,128 tiles
def n128_problem():
    return W.config2(n_cells=34_000, n_regions=16, n_angles=128, n_steps=2)


# S_128 with table tiles and records reduced by the end of step: 13,000 cells, 816 tiles
def n128_table_problem():
    return W.config2(n_cells=13_000, n_regions=16, n_angles=128, n_steps=2)


def test_problem_sizes_reach_the_large_instances():
    assert n_tiles(n64_problem()) > 2048
    assert n_tiles(n128_problem()) > 2048
    assert 768 < n_tiles(n128_table_problem()) <= 2048
    assert n_tiles(W.config3()) > 2048


@pytest.mark.parametrize("iters", [3, 6])
def test_n64_many_tiles_fixed_iterations(lib, iters):
    p = n64_problem()
    cd = cell_data(p)
    ref = ooci.run_oci(p, cd, 3, tol=0.0, max_iters=iters)
    rc, phi, infos, psi = gpu_steps(lib, p, 3, tol=0.0, max_iters=iters)
    assert rc == lib.OCI_NOT_CONVERGED
    for k in range(3):
        assert infos[k]["iterations"] == iters == ref[k]["iterations"]
        assert rel(phi[k], ref[k]["phi"]) < 1e-11, (iters, k)
    assert rel(psi, ref[-1]["psi_edge"]) < 1e-11


def test_n64_many_tiles_converged(lib):
    p = n64_problem()
    cd = cell_data(p)
    ref = ooci.run_oci(p, cd, 3, tol=1e-10, max_iters=1000)
    rc, phi, infos, _ = gpu_steps(lib, p, 3, tol=1e-10)
    assert rc == lib.OCI_OK
    for k in range(3):
        assert abs(infos[k]["iterations"] - ref[k]["iterations"]) <= 1
        assert infos[k]["residual"] <= 1e-10
        assert rel(phi[k], ref[k]["phi"]) < 1e-10, k


def test_n64_many_tiles_mixed(lib):
    p = n64_problem()
    cd = cell_data(p)
    ref = ooci.run_oci(p, cd, 3, tol=1e-12, max_iters=1000)
    rc, phi, infos, _ = gpu_steps(lib, p, 3, tol=1e-10, precision=lib.OCI_PREC_FP32)
    assert rc == lib.OCI_OK
    for k in range(3):
        assert rel(phi[k], ref[k]["phi"]) < 1e-9, k


@pytest.mark.parametrize("make", [n128_problem, n128_table_problem],
                         ids=["reduced_before_end", "reduced_by_end"])
def test_n128_many_tiles_fixed_iterations(lib, make):
    p = make()
    cd = cell_data(p)
    ref = ooci.run_oci(p, cd, 2, tol=0.0, max_iters=3)
    rc, phi, infos, psi = gpu_steps(lib, p, 2, tol=0.0, max_iters=3)
    for k in range(2):
        assert infos[k]["iterations"] == 3 == ref[k]["iterations"]
        assert rel(phi[k], ref[k]["phi"]) < 1e-11, k
    assert rel(psi, ref[-1]["psi_edge"]) < 1e-11


# ---------------------------------------------------------------------------
# the 200,000-cell S_64 problem itself: its first time step
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def large_reference():
    """Oracle OCI on the large problem's first step, one sequence of iterates
    from zero: the iterate the stopping rule accepts at tol 1e-6 and at 1e-10
    (with its iteration count), and the sequence continued until e <= 1e-13."""
    from oracle.stopping import accept, relative_change
    p = W.config3(n_steps=1)
    cd = cell_data(p)
    f = ooci.RegionFactors(cd)
    psi_prev = initial_edge_state(p, cd)
    psi = np.zeros((cd.J, cd.n, 4))
    hist, phi_old, found = [], None, {}
    for it in range(1, 200):
        psi = ooci.sweep_cells(cd, f, psi_prev, psi)
        phi = ooci.scalar_flux(cd, psi)
        hist.append(None if phi_old is None else relative_change(phi, phi_old))
        phi_old = phi
        for tol in (1e-6, 1e-10, 1e-13):
            if tol not in found and accept(hist, tol, False):
                found[tol] = {"phi": phi, "iterations": it}
        if 1e-13 in found:
            break
    return p, found[1e-6], found[1e-10], found[1e-13]


@pytest.mark.slow
def test_large_problem_first_step_plain(lib, large_reference):
    p, r6, r10, conv = large_reference
    rc, phi, infos, _ = gpu_steps(lib, p, 1, tol=1e-10)
    assert rc == lib.OCI_OK
    assert abs(infos[0]["iterations"] - r10["iterations"]) <= 1
    assert rel(phi[0], r10["phi"]) < 1e-10
    assert rel(phi[0], conv["phi"]) < 1e-10
    rc, phi6, infos6, _ = gpu_steps(lib, p, 1, tol=1e-6)
    assert rc == lib.OCI_OK
    assert abs(infos6[0]["iterations"] - r6["iterations"]) <= 1
    if infos6[0]["iterations"] == r6["iterations"]:   # the same iterate
        assert rel(phi6[0], r6["phi"]) < 1e-11
    assert rel(phi6[0], conv["phi"]) < 1e-6


@pytest.mark.slow
def test_large_problem_first_step_mixed(lib, large_reference):
    p, _, _, conv = large_reference
    rc, phi, infos, _ = gpu_steps(lib, p, 1, tol=1e-6, precision=lib.OCI_PREC_FP32)
    assert rc == lib.OCI_OK
    assert rel(phi[0], conv["phi"]) < 1e-6
    rc, phi, infos, _ = gpu_steps(lib, p, 1, tol=1e-10, precision=lib.OCI_PREC_FP32)
    assert rc == lib.OCI_OK
    assert rel(phi[0], conv["phi"]) < 1e-9

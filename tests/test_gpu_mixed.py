"""Mixed precision (OCI_PREC_FP32): FP64 defect correction with FP32 inner
iterations, through the C ABI, against the FP64 oracle.

Every accepted iterate is an FP64 application of the OCI operator to a point
y (an FP64 iterate plus an FP32 correction) and is judged by the same
stopping rule as plain OCI, so a converged mixed step is as close to the
step's exact solution as a converged plain step: with the rule's change e
below tol, the accepted iterate is within about tol * rho / (1 - rho) of the
fixed point (rho the iteration's contraction).  The tests compare with the
direct solve of each step's linear system (the exact fixed point) at
tol = 1e-13, where that bound is below 1e-11 for every case here (rho <=
0.99), and use 1e-10 relative to max|phi|; with the paper's tol 1e-10 against
oracle OCI (same rule, FP64 throughout) the bound is 1e-9.
"""
import dataclasses

import numpy as np
import pytest

from oracle import balance
from oracle import oci as ooci
from oracle.problem import cell_data
from paper_2305_13555_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_13555_amd import oci
    return oci


def rel(a, b):
    return float(np.max(np.abs(a - b))) / float(np.max(np.abs(b)))


def run(lib, prob, n_steps, **kw):
    out = []
    with lib.OciContext(prob, precision=lib.OCI_PREC_FP32, **kw) as ctx:
        for _ in range(n_steps):
            rc, info = ctx.step()
            info["rc"] = rc
            info["phi"] = ctx.flux().copy()
            info["psi_edge"] = ctx.state()[0]
            out.append(info)
    return out


MIXED_CASES = [
    (0, None), (1, None), (2, None), (3, None),
    (100, dict(n_angles=2, n_cells=1, n_regions=1)),
    (101, dict(n_angles=16, n_cells=17, n_regions=1)),
    (102, dict(n_angles=8, n_cells=33, n_regions=2, bc=(W.REFLECT, W.REFLECT))),
    (103, dict(n_angles=4, n_cells=40, n_regions=3, bc=(W.INCIDENT, W.INCIDENT))),
    (104, dict(n_angles=6, n_cells=23, n_regions=2, bc=(W.REFLECT, W.INCIDENT))),
    (105, dict(n_angles=64, n_cells=20, n_regions=2, bc=(W.VACUUM, W.REFLECT))),
    (106, dict(n_angles=128, n_cells=9, n_regions=1, bc=(W.REFLECT, W.VACUUM))),
    (107, dict(n_angles=256, n_cells=5, n_regions=1, bc=(W.INCIDENT, W.REFLECT))),
]


@pytest.mark.parametrize("seed,kw", MIXED_CASES)
def test_mixed_converged_matches_direct(lib, seed, kw):
    p = W.random_small(seed, **(kw or {}))
    cd = cell_data(p)
    direct = balance.run_direct(p, cd, 3)
    got = run(lib, p, 3, tol=1e-13, max_iters=5000)
    for k in range(3):
        assert got[k]["rc"] == lib.OCI_OK, (seed, k, got[k])
        assert rel(got[k]["phi"], direct[k]["phi"]) < 1e-10, (seed, k)
        assert rel(got[k]["psi_edge"], direct[k]["psi_edge"]) < 1e-10, (seed, k)


@pytest.mark.parametrize("case", [
    (0, [1, 17, 1, 2, 30, 1], 8, (W.REFLECT, W.REFLECT)),
    (1, [3, 40, 1, 20], 32, (W.INCIDENT, W.REFLECT)),
    (3, [5, 33, 2], 12, (W.VACUUM, W.INCIDENT)),
], ids=lambda c: "layout%d" % c[0])
def test_mixed_tile_layouts_match_direct(lib, case):
    seed, sizes, n, bc = case
    p = W.layout_case(seed, sizes, n, bc)
    direct = balance.run_direct(p, cell_data(p), 2)
    got = run(lib, p, 2, tol=1e-13, max_iters=5000)
    for k in range(2):
        assert got[k]["rc"] == lib.OCI_OK
        assert rel(got[k]["phi"], direct[k]["phi"]) < 1e-10


def test_mixed_config2_first_steps_match_oracle(lib):
    """Full-size multi-region problem (10,000 cells, S_32), tol 1e-10."""
    p = W.config2(n_steps=3)
    ref = ooci.run_oci(p, cell_data(p), 3, tol=1e-10, max_iters=1000)
    got = run(lib, p, 3)
    for k in range(3):
        assert got[k]["rc"] == lib.OCI_OK
        assert rel(got[k]["phi"], ref[k]["phi"]) < 1e-9
        # FP64 iterates: the first gives the defect, later ones check corrections
        assert 2 <= got[k]["iterations"] <= ref[k]["iterations"]
        assert got[k]["launches"] > got[k]["iterations"]


def test_mixed_queued_solve_matches_direct_on_slow_problem(lib):
    """Optically thin cells, c = 0.99 (contraction near 1): the inner
    iterations grow, and steps are resumed past their queued launches."""
    p = dataclasses.replace(W.homogeneous_slab(4, 200, 0.99, 0.01, 1.0), n_steps=3)
    cd = cell_data(p)
    direct = balance.run_direct(p, cd, 3)
    with lib.OciContext(p, precision=lib.OCI_PREC_FP32, tol=1e-12, max_iters=100000) as ctx:
        phi = np.zeros((3, p.n_cells, 4))
        rc, infos = ctx.solve(3, phi)
    assert rc == lib.OCI_OK
    for k in range(3):
        assert rel(phi[k], direct[k]["phi"]) < 1e-8, k
        assert infos[k]["status"] == lib.OCI_OK


def test_mixed_and_plain_agree_and_interleave_with_si(lib):
    p = W.random_small(11, n_angles=8, n_cells=60, n_regions=3, bc=(W.REFLECT, W.VACUUM))
    with lib.OciContext(p, tol=1e-13, max_iters=5000) as a, \
            lib.OciContext(p, tol=1e-13, max_iters=5000, precision=lib.OCI_PREC_FP32) as b:
        for kind in ("oci", "si", "oci", "oci"):
            if kind == "si":
                a.si_step()
                b.si_step()
            else:
                a.step()
                b.step()
            assert rel(b.flux(), a.flux()) < 1e-10, kind


def test_mixed_iteration_limit_and_strict_rejected(lib):
    p = W.config1()
    with lib.OciContext(p, precision=lib.OCI_PREC_FP32, max_iters=1, tol=1e-14) as ctx:
        rc, info = ctx.step()
        assert rc == lib.OCI_NOT_CONVERGED and info["iterations"] == 1
        assert ctx.state()[1] == 1
    with pytest.raises(lib.OciError) as ei:
        lib.OciContext(p, precision=lib.OCI_PREC_FP32, strict=True)
    assert ei.value.code == lib.OCI_EINVAL


@pytest.mark.parametrize("n_angles", [16, 64])
def test_mixed_queued_windows_match_oracle(lib, n_angles):
    """Queued windows of several steps: the end of every step but a window's
    last also forms the next step's first FP64 iterate and its defect, and
    the next step's first inner iteration opens it."""
    p = W.config2(n_steps=8, n_cells=700, n_regions=5, n_angles=n_angles)
    ref = ooci.run_oci(p, cell_data(p), 8, tol=1e-12, max_iters=1000)
    with lib.OciContext(p, precision=lib.OCI_PREC_FP32, tol=1e-10) as ctx:
        phi = np.zeros((8, p.n_cells, 4))
        rc, infos = ctx.solve(8, phi)
        import torch
        dev = torch.zeros((8, p.n_cells, 4), dtype=torch.float64, device="cuda")
        ctx.set_state(None, 0)
        rc2, infos2 = ctx.solve(8, dev)
    assert rc == lib.OCI_OK and rc2 == lib.OCI_OK
    got = dev.cpu().numpy()
    for k in range(8):
        assert rel(phi[k], ref[k]["phi"]) < 1e-9, k
        assert rel(got[k], ref[k]["phi"]) < 1e-9, k

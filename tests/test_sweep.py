"""The OCI-vs-SI quadrature sweep: its problem family (CPU) and one point run
on the GPU through the C ABI."""
import pytest

from paper_2305_13555_amd import sweep
from paper_2305_13555_amd import workloads as W


def test_sweep_problem_family():
    p = sweep.problem(8, 0.9, 0.1, 0.01)
    assert p.n_angles == 8 and p.n_cells == 200 and p.n_steps == 5
    assert float(p.width[0]) == pytest.approx(10.0)
    assert float(p.sigma_t[0]) == 2.0 and float(p.sigma_s[0]) == pytest.approx(1.8)
    assert float(p.source[0]) == 0.1
    assert p.bc_left == W.VACUUM and p.bc_right == W.VACUUM and p.psi0 is None
    # the cell optical thickness is the grid's sigma*dx
    assert float(p.sigma_t[0] * p.width[0] / p.n_cells) == pytest.approx(0.1)
    for n in sweep.GRID["n_angles"]:
        assert n % 2 == 0


@pytest.mark.gpu
def test_sweep_point_runs_both_iterations():
    import torch
    assert torch.cuda.is_available()
    from paper_2305_13555_amd import oci
    r = sweep.run_point(oci, torch, 4, 0.9, 1.0, 0.1, check_oracle=True)
    assert r["cells"] == 20 and r["oci_rc"] == 0 and r["si_rc"] == 0
    assert len(r["oci_iters"]) == sweep.STEPS and len(r["si_iters"]) == sweep.STEPS
    assert r["oci_s"] > 0 and r["si_s"] > 0
    # both stop by the strict rule at 1e-9: within that of the oracle (FP64
    # OCI, strict, 1e-12), up to the bound's estimate of the contraction
    assert r["oci_vs_oracle_rel"] < 1e-8 and r["si_vs_oracle_rel"] < 1e-8

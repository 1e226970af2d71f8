"""Steps that take thousands of iterations (GPU, through the C ABI).

A step not decided within its queued launches is resumed in batches that
grow 1, 1, 2, 4, ... up to 64 launches; a step of a few thousand iterations
runs dozens of such batches.  These cases check the resumed path against the
oracle far beyond the growth phase, for OCI and for SI.

* OCI: the quadrature-sweep slab at S_2 with the thinnest cells
  (Sigma*dx = 0.01, 2000 cells), c = 0.99 and dt = 1: about 1800 iterations.
* SI: a reflecting slab of thick cells, c = 0.999 and dt = 100: about 2700
  sweeps (the spectral radius is c*Sigma/(Sigma + 1/(v dt)) ~ 0.994).

Both sides take the same iterates and the same stopping rule, so the counts
agree to within one (a rounding-level difference in e at the threshold) and
the fluxes to 1e-8 relative (one iteration's change at tol 1e-9 near the
end is ~1e-9 of max|phi| per unit of rho/(1-rho) <= 10).
"""
import dataclasses

import numpy as np
import pytest

from oracle import oci as ooci
from oracle import si as osi
from oracle.problem import cell_data
from paper_2305_13555_amd import sweep
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


def test_oci_step_of_thousands_of_iterations(lib):
    p = dataclasses.replace(sweep.problem(2, 0.99, 0.01, 1.0), n_steps=1)
    ref = ooci.run_oci(p, cell_data(p), 1, tol=1e-9, max_iters=200000)[0]
    assert ref["iterations"] > 1700
    with lib.OciContext(p, tol=1e-9, max_iters=200000) as ctx:
        rc, info = ctx.step()
        phi = ctx.flux()
    assert rc == lib.OCI_OK
    assert abs(info["iterations"] - ref["iterations"]) <= 1
    assert info["launches"] >= info["iterations"]
    assert rel(phi, ref["phi"]) < 1e-8


def test_si_step_of_thousands_of_sweeps(lib):
    base = W.homogeneous_slab(2, 10, 0.999, 2.0, 100.0, speed=1.0, n_steps=1)
    p = dataclasses.replace(base, bc_left=W.REFLECT, bc_right=W.REFLECT)
    ref = osi.run_si(p, cell_data(p), 1, tol=1e-9, max_iters=200000)[0]
    assert ref["iterations"] > 2000
    with lib.OciContext(p, tol=1e-9, max_iters=200000) as ctx:
        rc, info = ctx.si_step()
        phi = ctx.flux()
        # the OCI step that follows starts from the SI iterate
        rc2, info2 = ctx.step()
    assert rc == lib.OCI_OK and rc2 == lib.OCI_OK
    assert abs(info["iterations"] - ref["iterations"]) <= 1
    assert rel(phi, ref["phi"]) < 1e-8
    assert info2["iterations"] >= 2

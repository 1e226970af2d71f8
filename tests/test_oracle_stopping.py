"""Pins for the stopping rule and for iteration counts of the oracle."""
import math

import numpy as np

from oracle import oci
from oracle.problem import cell_data
from oracle.stopping import accept, relative_change
from paper_2305_13555_amd import workloads as W


def test_relative_change_definition():
    a = np.array([[1.0, -4.0, 2.0, 0.5]])
    b = np.array([[1.5, -3.0, 2.0, 0.5]])
    assert relative_change(a, b) == 1.0 / 4.0
    z = np.zeros((2, 4))
    assert relative_change(z, z) == 0.0
    assert math.isinf(relative_change(z, a[:, :].repeat(2, 0)))


def test_accept_rules():
    assert not accept([None], 1e-3, False)
    assert accept([None, 1e-4], 1e-3, False)
    assert not accept([None, 1e-2], 1e-3, False)
    # strict: rho = 0.9 -> bound 9e-4 * 9 > 1e-3
    assert not accept([1e-3, 9e-4], 1e-3, True)
    # rho = 0.1 -> bound 1e-4 * 0.111 < 1e-3
    assert accept([1e-3, 1e-4], 1e-3, True)
    assert not accept([None, 1e-4], 1e-3, True)


def test_strict_rule_bounds_the_true_error():
    # thin cells, high scattering: slow OCI where a plain change test under-reports
    p = W.homogeneous_slab(4, 40, c=0.99, sigma_dx=0.02, dt=1.0, speed=0.25)
    cd = cell_data(p)
    from oracle import balance
    ref = balance.run_direct(p, cd, 1)[0]["phi"]
    tol = 1e-8
    plain = oci.run_oci(p, cd, 1, tol, 200000, strict=False)[0]
    strict = oci.run_oci(p, cd, 1, tol, 200000, strict=True)[0]
    e_strict = np.max(np.abs(strict["phi"] - ref)) / np.max(np.abs(ref))
    assert strict["iterations"] > plain["iterations"]
    assert e_strict <= 2 * tol

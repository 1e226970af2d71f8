"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, computes the quadrature on the host, and rejects invalid
problems before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "oci.h")
LIB = os.path.join(ROOT, "paper_2305_13555_amd", "liboci.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b((?:oci|si)_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("oci_setup", "oci_step", "si_step", "oci_solve", "oci_get_flux",
                     "oci_get_state", "oci_set_state", "oci_destroy", "oci_strerror",
                     "oci_last_error", "oci_gauss_legendre", "oci_get_operator"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build first: python -m paper_2305_13555_amd.build"
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.parametrize("n", [2, 4, 8, 16, 32, 64, 128, 256])
def test_library_quadrature_matches_oracle(n):
    from oracle.quadrature import gauss_legendre
    from paper_2305_13555_amd import oci
    mu, w = oci.oci_gauss_legendre(n)
    rmu, rw = gauss_legendre(n)
    np.testing.assert_allclose(mu, rmu, atol=2e-16 * 4)
    np.testing.assert_allclose(w, rw, rtol=1e-12)   # both ~4e-13 from the exact weights at N = 256


def _valid():
    from paper_2305_13555_amd import workloads as W
    return W.random_small(1, n_angles=4)


@pytest.mark.parametrize("mutate,why", [
    (lambda p: setattr(p, "n_angles", 3), "odd"),
    (lambda p: setattr(p, "n_angles", 0), "zero angles"),
    (lambda p: setattr(p, "n_angles", 512), "too many angles"),
    (lambda p: setattr(p, "dt", 0.0), "dt"),
    (lambda p: setattr(p, "dt", -1.0), "dt<0"),
    (lambda p: setattr(p, "speed", 0.0), "speed"),
    (lambda p: setattr(p, "sigma_t", p.sigma_t * 0.0), "sigma_t"),
    (lambda p: setattr(p, "sigma_s", p.sigma_s * 0.0 - 1.0), "sigma_s<0"),
    (lambda p: setattr(p, "source", p.source * 0.0 - 1.0), "Q<0"),
    (lambda p: setattr(p, "cells", p.cells * 0), "no cells"),
    (lambda p: setattr(p, "max_iters", 0), "max_iters"),
    (lambda p: setattr(p, "tol", -1.0), "tol"),
    (lambda p: (setattr(p, "bc_left", 2), setattr(p, "inc_left", None)), "incident array"),
    (lambda p: setattr(p, "bc_right", 7), "bc"),
    (lambda p: setattr(p, "psi0", np.full_like(p.psi0, np.nan)), "psi0 nan"),
])
def test_setup_rejects_invalid_problems_on_host(mutate, why):
    from paper_2305_13555_amd import oci
    p = _valid()
    p.psi0 = np.zeros((p.n_cells, p.n_angles, 2))
    mutate(p)
    if getattr(p, "n_angles", 4) in (3, 0, 512):
        p.psi0 = None
    with pytest.raises(oci.OciError) as ei:
        oci.oci_setup(p, stream=0)
    assert ei.value.code == oci.OCI_EINVAL, why


def test_strerror_covers_codes():
    from paper_2305_13555_amd import oci
    for code in (0, 1, -1, -2, -3, -4, -5):
        assert oci.oci_strerror(code) != "unknown error code"
    assert oci.oci_strerror(42) == "unknown error code"


@pytest.mark.parametrize("args", [(3, 4, 1, 10), (8, 6, 1, 10), (8, 4, 0, 10), (8, 4, 1, 0),
                                  (2048, 4, 1, 10)])
def test_corrector_create_rejects_bad_shapes_on_host(args):
    import ctypes
    from paper_2305_13555_amd import oci
    h = ctypes.c_void_p()
    assert oci._lib.oci_corrector_create(*args, None, ctypes.byref(h)) == oci.OCI_EINVAL
    assert not h.value

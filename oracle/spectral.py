"""Spectral radii of the OCI and SI iteration operators by brute force (oracle).

TEST INFRASTRUCTURE ONLY.

Fig. 1 of the paper reports the spectral radius of both iterations for an
infinite medium (reflecting both edges), steady state, S_4, against the cell
optical thickness Sigma dx and the scattering ratio c.  Both iterations are
affine maps; their linear part is obtained here by applying one iteration with
all sources, previous-time terms and incident fluxes set to zero to every unit
vector of the iterate, and the spectral radius is the largest eigenvalue
modulus of that matrix.  Small meshes only.
"""
import dataclasses

import numpy as np

from .oci import RegionFactors, sweep_cells
from .si import AngleMatrices, si_sweep


def _homogeneous(cd):
    return dataclasses.replace(cd, q=np.zeros_like(cd.q),
                               inc_left=np.zeros_like(cd.inc_left),
                               inc_right=np.zeros_like(cd.inc_right))


def oci_iteration_matrix(cd):
    """Linear part of Psi^(l) -> Psi^(l+1), size 4NJ."""
    h = _homogeneous(cd)
    f = RegionFactors(h)
    J, n = h.J, h.n
    size = J * n * 4
    prev = np.zeros((J, n, 2))
    T = np.zeros((size, size))
    for i in range(size):
        e = np.zeros(size)
        e[i] = 1.0
        T[:, i] = sweep_cells(h, f, prev, e.reshape(J, n, 4)).ravel()
    return T


def si_iteration_matrix(cd):
    """Linear part of the SI state map (phi [J][4], lagged right reflection [N/2][2])."""
    h = _homogeneous(cd)
    am = AngleMatrices(h)
    J, n = h.J, h.n
    nphi = J * 4
    nlag = n  # N/2 angles x 2 levels
    size = nphi + nlag
    prev = np.zeros((J, n, 2))
    T = np.zeros((size, size))
    for i in range(size):
        e = np.zeros(size)
        e[i] = 1.0
        phi = e[:nphi].reshape(J, 4)
        lag = e[nphi:].reshape(n // 2, 2)
        psi, lag_new = si_sweep(h, am, phi, prev, lag)
        T[:nphi, i] = np.einsum("n,jnc->jc", h.w, psi).ravel()
        T[nphi:, i] = np.asarray(lag_new).ravel()
    return T


def spectral_radius(T):
    return float(np.max(np.abs(np.linalg.eigvals(T))))

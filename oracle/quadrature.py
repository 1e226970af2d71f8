"""Gauss-Legendre S_N quadrature for the oracle (test infrastructure only).

The paper uses Gauss-Legendre quadrature in all its explorations (Sec.
"ONE-CELL INVERSION (OCI)", discussion of Fig. 1).  The transport equation of
Sec. "Derivation of MB-SCB" writes the scattering source as
1/2 * Sigma_s * sum_n w_n psi_n, so the weights integrate 1 over mu in [-1, 1]
to 2.

Nodes are the roots of the Legendre polynomial P_N, found by Newton's method
on the three-term recurrence; weights are 2 / ((1 - mu^2) P_N'(mu)^2).
Returned in ascending mu, so for even N the first N/2 nodes are negative and
node N-1-m mirrors node m.

Pinned by tests/test_oracle_quadrature.py: polynomial exactness up to degree
2N-1 (a property of the Gauss rule), symmetry, sum(w) = 2, and agreement with
an independent library routine.
"""
import math

import numpy as np


def _legendre_and_derivative(n, x):
    """P_n(x) and P_n'(x) by the recurrences
    (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}  and  P'_{k+1} = P'_{k-1} + (2k+1) P_k."""
    p_prev, p = np.ones_like(x), x.copy()
    d_prev, d = np.zeros_like(x), np.ones_like(x)
    if n == 0:
        return p_prev, d_prev
    for k in range(1, n):
        p_prev, p = p, ((2 * k + 1) * x * p - k * p_prev) / (k + 1)
        d_prev, d = d, d_prev + (2 * k + 1) * p_prev
    return p, d


def gauss_legendre(n):
    """Return (mu, w), float64 arrays of length n, mu ascending."""
    if n < 1:
        raise ValueError("n must be >= 1")
    i = np.arange(1, n + 1, dtype=np.float64)
    x = np.cos(math.pi * (i - 0.25) / (n + 0.5))  # Tricomi-style first guess
    for _ in range(100):
        p, dp = _legendre_and_derivative(n, x)
        dx = p / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    p, dp = _legendre_and_derivative(n, x)
    w = 2.0 / ((1.0 - x * x) * dp * dp)
    order = np.argsort(x)
    return x[order].copy(), w[order].copy()

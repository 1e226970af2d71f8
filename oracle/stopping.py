"""Scalar-flux stopping rule shared by the oracle's OCI and SI (test infrastructure only).

The paper stops source iteration when the scalar-flux vector stops changing
(end of the SI subsection) and one-cell inversion when the angular-flux vector
stops changing (end of the OCI subsection); its disabled backward-Euler study
iterates to a change of 1e-9; it never names the norm.  Reading taken here,
for both iterations, on the scalar flux of all four components
(phi_{k,L}, phi_{k,R}, phi_{k+1/2,L}, phi_{k+1/2,R}) of every cell:

    e_l = max |phi^(l) - phi^(l-1)| / max |phi^(l)|      (0/0 -> 0, x/0 -> inf)

and iterate l is accepted when e_l <= tol.  With ``strict`` the estimated
contraction rho = e_l / e_{l-1} (clamped to [0, 0.9999]) must also give an
a-posteriori error bound e_l * rho / (1 - rho) <= tol; l = 1 of OCI has no
predecessor within the step and is never accepted.
"""
import numpy as np

RHO_CLAMP = 0.9999


def relative_change(phi_new, phi_old):
    num = float(np.max(np.abs(phi_new - phi_old))) if phi_new.size else 0.0
    den = float(np.max(np.abs(phi_new))) if phi_new.size else 0.0
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return num / den


def accept(e_hist, tol, strict):
    """Decide from the residual history (e_1 .. e_l, None where undefined)."""
    e = e_hist[-1]
    if e is None or not (e <= tol):
        return False
    if not strict:
        return True
    if len(e_hist) < 2 or e_hist[-2] is None:
        return False
    prev = e_hist[-2]
    rho = 0.0 if prev == 0.0 else min(max(e / prev, 0.0), RHO_CLAMP)
    return e * rho / (1.0 - rho) <= tol

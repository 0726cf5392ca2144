"""Newton iterations for the nonlinear Crouzeix-Raviart scheme (test infrastructure).

Section 3.1 approximates the nonlinear system by the Newton method: each
iteration solves the linear system of one Newton step about the current
iterate ubar, J(ubar) u + D^t P = R_f + b_h(ubar, ubar) (J = S (x) I + the
Jacobian of the convection form b_h, eq. defbh), whose solution u is the next
iterate.  Here each step is the oracle's coupled sparse LU solve; the
iteration stops when max|u - ubar| <= tol max|u|.  Boundary data (gbnd) are
imposed on the exterior faces in every step, and the exterior faces of ubar
take them too.
"""
from __future__ import annotations

import numpy as np

from . import cr


def newton(coords, elems, mu, nu, fbar, gbnd=None, u_prev=None, u0=None, tol=1e-10, maxit=30):
    """Returns (U [nf, d], P [ne], increments) with increments[i] = max|u_{i+1} - u_i| / max|u_{i+1}|."""
    m = cr.build_mesh(coords, elems)
    ubar = np.zeros((m.nf, m.d)) if u0 is None else np.asarray(u0, dtype=np.float64).copy()
    inc = []
    U, Pk = ubar, np.zeros(m.ne)
    for _ in range(maxit):
        P = cr.make_problem(coords, elems, mu, nu, fbar, u_prev=u_prev, ulin=ubar, gbnd=gbnd)
        U, Pk = cr.solve_coupled(P, refine=1)
        inc.append(np.abs(U - ubar).max() / max(np.abs(U).max(), 1e-300))
        ubar = U
        if inc[-1] <= tol:
            break
    return U, Pk, inc


def nonlinear_residual(coords, elems, mu, nu, fbar, U, Pk, gbnd=None, u_prev=None):
    """Relative residual of the nonlinear scheme at (U, P): the Newton system about
    ubar = U evaluated at u = U (it equals S U + b_h(U, U) + D^t P - R_f, since
    J(U) U = S U + 2 b_h(U, U))."""
    P = cr.make_problem(coords, elems, mu, nu, fbar, u_prev=u_prev, ulin=U, gbnd=gbnd)
    res, div = cr.coupled_residual(P, U, Pk)
    return res, div

"""Newton iterations of the nonlinear Crouzeix-Raviart scheme on the GPU.

Section 3.1 approximates the nonlinear system of the Navier-Stokes scheme by
the Newton method; every Newton iteration is one linear system
J(ubar) u + D^t P = R_f + b_h(ubar, ubar) about the current iterate ubar, and
the hybrid method of Section 3.2 solves it.  This module only orders the
library calls: per iteration cr_eliminate with u_lin = ubar (the exterior faces
of ubar take the boundary data of cr_set_boundary), cr_solve with the W of the
previous linear solve as its initial guess (cr_export_W_device; across time
steps too: W changes little from one Newton step to the next), cr_recover; the
iterate becomes the recovered U until max|U - ubar| <= tol max|U|.  Every step
of the path runs in the HIP library.
"""
from __future__ import annotations

import time

from ._binding import System


class NewtonSolver:
    """A Navier-Stokes system (steady: mu = 0, or one backward-Euler step:
    mu = 1/dt) solved by Newton iterations, each one hybridised Newton step."""

    def __init__(self, coords, elems, mu, nu, k0=0, lambda_scale=0.0, stream=None):
        import torch
        self.torch = torch
        self.sys = System(coords, elems, mu, nu, k0=k0, problem="ns", lambda_scale=lambda_scale, stream=stream)
        self.dim = self.sys.dim
        self._W = None  # W of the last linear solve, the next one's initial guess

    def set_boundary(self, g):
        self.sys.set_boundary(g)

    def solve(self, f_mean, u_prev=None, u0=None, tol=1e-10, maxit=30, method="bicgstab2", precision="fp64",
              lin_tol=1e-11, lin_maxit=400000):
        """Returns (U, P, record): U [n_int_faces, dim], P [n_elements] on the
        device; record: increments, linear iterations and times per iteration,
        and the status of each linear solve."""
        torch = self.torch
        s = self.sys
        f = s._dev(f_mean, (s.n_elements, self.dim))
        up = s._dev(u_prev, (s.n_int_faces, self.dim))
        if u0 is None:
            ubar = torch.zeros((s.n_int_faces, self.dim), dtype=torch.float64, device="cuda")
        else:
            ubar = s._dev(u0, (s.n_int_faces, self.dim)).clone()
        rec = dict(increments=[], linear_iters=[], linear_status=[], times_ms=[])
        U = P = None
        for it in range(maxit):
            t0 = time.perf_counter()
            s.eliminate(f, up, ubar)
            info = s.solve(method, precision, tol=lin_tol, maxit=lin_maxit, w0=self._W, raise_on_error=False)
            # a failed solve's W is no guess for the next one
            self._W = s.export_W_device(self._W) if info["status"] == 0 else None
            U, P = s.recover()
            inc = (torch.max(torch.abs(U - ubar)) / torch.clamp(torch.max(torch.abs(U)), min=1e-300)).item()
            rec["times_ms"].append(1e3 * (time.perf_counter() - t0))
            rec["increments"].append(inc)
            rec["linear_iters"].append(info["iters"])
            rec["linear_status"].append(info["status"])
            ubar = U
            if inc <= tol:
                break
        rec["converged"] = bool(rec["increments"] and rec["increments"][-1] <= tol)
        return U, P, rec

    def close(self):
        self.sys.close()

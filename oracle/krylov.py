"""Plain FP64 Jacobi-preconditioned conjugate gradient on G (Section 3.2 item 6).

Test infrastructure only.  Used where a sparse direct factorisation of the
system is too large: Section 3.2 shows G is symmetric positive definite when
mu > 0 and there is no convection, so CG applies ("hybrid method", step 2).
Textbook PCG, no blocking or fusion.
"""
from __future__ import annotations

import numpy as np


def pcg(G, b, tol=1e-12, maxit=100000, x0=None, callback=None):
    """Solve G x = b to ||b - G x|| <= tol ||b||.  Returns (x, iterations, history).

    callback(iteration, relative recursive residual), if given, is called after
    every iteration (progress reporting only)."""
    dinv = 1.0 / G.diagonal()
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - G @ x
    z = dinv * r
    p = z.copy()
    rz = r @ z
    nb = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / nb]
    it = 0
    while hist[-1] > tol and it < maxit:
        q = G @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
        hist.append(np.linalg.norm(r) / nb)
        if callback is not None:
            callback(it, hist[-1])
    return x, it, hist

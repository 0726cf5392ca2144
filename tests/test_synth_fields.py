"""Pins of the synthetic exact fields (CPU only).

The Green-Taylor vortex of Section 4.1 (eqs. gretayvel, gretaypre) is used as
an exact solution with zero force; these tests check, by central differences
independent of the closed-form derivatives in synth.fields, that it is one:
div u = 0 and du/dt + (u.grad) u - nu Lap u + grad p = 0, and that the stated
gradients and forces agree with the fields.
"""
from __future__ import annotations

import numpy as np

from synth.fields import GreenTaylor2D


def _pts(n=64, seed=3):
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(n, 2))


def _grad_fd(fn, x, h=1e-5):
    """[m, comps, 2] central differences of fn (values [m] or [m, comps])."""
    out = []
    for j in range(2):
        e = np.zeros(2)
        e[j] = h
        out.append((np.atleast_2d((fn(x + e) - fn(x - e)).T).T) / (2 * h))
    return np.stack(out, axis=-1)


def test_green_taylor_solves_unforced_navier_stokes():
    nu, amp = 0.5, 20.0
    gt = GreenTaylor2D(amp=amp, nu=nu)
    x = _pts()
    t = 0.013
    h = 1e-4
    u = gt.u(x, t)
    du_dt = (gt.u(x, t + h) - gt.u(x, t - h)) / (2 * h)
    g = _grad_fd(lambda y: gt.u(y, t), x, h)            # [m, 2, 2]
    lap = np.zeros_like(u)
    for j in range(2):
        e = np.zeros(2)
        e[j] = h
        lap += (gt.u(x + e, t) - 2 * u + gt.u(x - e, t)) / h ** 2
    gp = _grad_fd(lambda y: gt.p(y, t), x, h)[:, 0, :]  # [m, 2]
    conv = np.einsum("mj,mij->mi", u, g)
    res = du_dt + conv - nu * lap + gp
    scale = np.abs(du_dt).max() + np.abs(conv).max() + np.abs(nu * lap).max()
    assert np.abs(res).max() < 1e-5 * scale
    assert np.abs(g[:, 0, 0] + g[:, 1, 1]).max() < 1e-7 * np.abs(g).max()
    # the time dependence is not trivial: each term is of the scale of the others
    assert np.abs(du_dt).max() > 0.05 * scale and np.abs(conv).max() > 0.05 * scale


def test_green_taylor_closed_forms_match_differences():
    gt = GreenTaylor2D(amp=2.0, nu=0.3)
    x = _pts(seed=5)
    t = 0.02
    gu = _grad_fd(lambda y: gt.u(y, t), x)
    assert np.abs(gt.grad_u(x, t) - gu).max() < 1e-6 * np.abs(gu).max()
    gp = _grad_fd(lambda y: gt.p(y, t), x)[:, 0, :]
    assert np.abs(gt.grad_p(x, t) - gp).max() < 1e-6 * np.abs(gp).max()
    # forces: Stokes f = mu u - nu Lap u + grad p, steady NS f = -nu Lap u + u.grad u + grad p
    h = 1e-4
    lap = sum((gt.u(x + e, t) - 2 * gt.u(x, t) + gt.u(x - e, t)) / h ** 2 for e in (np.array([h, 0.0]), np.array([0.0, h])))
    mu = 5.0
    fs = mu * gt.u(x, t) - gt.nu * lap + gt.grad_p(x, t)
    assert np.abs(gt.stokes_force(mu, t)(x) - fs).max() < 1e-5 * np.abs(fs).max()
    fn = -gt.nu * lap + np.einsum("mj,mij->mi", gt.u(x, t), gt.grad_u(x, t)) + gt.grad_p(x, t)
    assert np.abs(gt.steady_ns_force(t)(x) - fn).max() < 1e-5 * np.abs(fn).max()


def test_green_taylor_paper_constants():
    """k = 2 pi, the velocity amplitude is the Reynolds number and the decay
    rates are 2 nu k^2 (velocity) and 4 nu k^2 (pressure)."""
    gt = GreenTaylor2D(amp=100.0, nu=1.0)
    x = np.array([[0.0, 0.0], [0.3, 0.8]])
    u0 = gt.u(x, 0.0)
    assert abs(np.abs(gt.u(np.array([[0.75, 0.75]]), 0.0)).max() - 100.0) < 1e-12
    t = 0.001
    k2 = (2 * np.pi) ** 2
    assert np.allclose(gt.u(x, t), u0 * np.exp(-2 * k2 * t), rtol=1e-14, atol=0)
    assert np.allclose(gt.p(x, t), gt.p(x, 0.0) * np.exp(-4 * k2 * t), rtol=1e-14, atol=0)


def test_green_taylor_3d_solves_unforced_navier_stokes():
    """The 3D extension (third component zero, no x3 dependence) by central
    differences in all three directions."""
    from synth.fields import GreenTaylor3D
    nu = 0.5
    gt = GreenTaylor3D(amp=20.0, nu=nu)
    x = np.random.default_rng(7).uniform(0.0, 1.0, size=(48, 3))
    t, h = 0.004, 1e-4
    u = gt.u(x, t)
    assert u.shape == (48, 3) and np.all(u[:, 2] == 0.0)
    du_dt = (gt.u(x, t + h) - gt.u(x, t - h)) / (2 * h)
    g = np.zeros((len(x), 3, 3))
    lap = np.zeros_like(u)
    gp = np.zeros((len(x), 3))
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        g[:, :, j] = (gt.u(x + e, t) - gt.u(x - e, t)) / (2 * h)
        lap += (gt.u(x + e, t) - 2 * u + gt.u(x - e, t)) / h ** 2
        gp[:, j] = (gt.p(x + e, t) - gt.p(x - e, t)) / (2 * h)
    res = du_dt + np.einsum("mj,mij->mi", u, g) - nu * lap + gp
    assert np.abs(res).max() < 1e-5 * (np.abs(du_dt).max() + np.abs(nu * lap).max())
    assert np.abs(np.trace(g, axis1=1, axis2=2)).max() < 1e-7 * np.abs(g).max()
    assert np.abs(gt.grad_u(x, t) - g).max() < 1e-6 * np.abs(g).max()
    assert np.abs(gt.grad_p(x, t) - gp).max() < 1e-6 * np.abs(gp).max()

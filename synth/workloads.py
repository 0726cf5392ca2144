"""Named synthetic workloads: meshes, coefficients and forcing data.

Each builder returns a plain dict of numpy arrays and scalars, identical for the
HIP path and the oracle.  Coefficients follow the strong form of Section 2:
mu = 1/dt for a transient step (mu = 0 for the steady Newton step), nu = 1/Re.

Workloads (structured stand-ins for the paper's meshes, Section 4):
  square16   2D unit square 16x16 cells x2 triangles, mu = 100, nu = 1
  square512j 2D 512x512 cells x2, interior vertices jittered by up to 0.2 h,
             mu = 1000, nu = 1
  cube64     3D 64^3 cubes x6 tetrahedra, mu = 100, nu = 1
  ns256      2D 256x256 cells x2, steady (mu = 0), nu = 0.01, Newton step
             about a seeded divergence-free velocity (8 Fourier modes)
  ns_cube(n) 3D n^3 cubes x6, steady, nu = 0.01, Newton step about a seeded
             divergence-free velocity (curl of an 8-mode vector potential)
The right-hand side is the element mean of the force implied by a seeded
smooth manufactured velocity (Manufactured).
"""
from __future__ import annotations

import numpy as np

from .fields import LinearisationField2D, LinearisationField3D, Manufactured, element_means
from .mesh import cube_mesh, square_mesh


def interior_face_list(elems):
    """Interior faces as sorted vertex tuples in lexicographic order.

    This is the canonical face order of the solver interface: it is used here
    only to place per-face input values (previous velocity, linearisation
    velocity) in that order.
    """
    d1 = elems.shape[1]
    loc = np.stack([np.delete(elems, j, axis=1) for j in range(d1)], axis=1)
    keys = np.sort(loc.reshape(-1, d1 - 1), axis=1)
    uniq, counts = np.unique(keys, axis=0, return_counts=True)
    return uniq[counts == 2].astype(np.int32)


def exterior_face_list(elems):
    """Exterior (boundary) faces as sorted vertex tuples in lexicographic order:
    the order of the boundary data of the solver interface."""
    d1 = elems.shape[1]
    loc = np.stack([np.delete(elems, j, axis=1) for j in range(d1)], axis=1)
    keys = np.sort(loc.reshape(-1, d1 - 1), axis=1)
    uniq, counts = np.unique(keys, axis=0, return_counts=True)
    return uniq[counts == 1].astype(np.int32)


def transient_stokes(mesh, mu, nu, seed=0, quad=4):
    coords, elems = mesh
    dim = coords.shape[1]
    man = Manufactured(dim, seed=seed, mu=mu, nu=nu)
    fbar = element_means(coords, elems, man.f, n=quad)
    return dict(coords=coords, elems=elems, mu=float(mu), nu=float(nu), fbar=fbar,
                problem="stokes", manufactured=man)


def square(n, mu, nu, jitter=0.0, seed=0, quad=4):
    return transient_stokes(square_mesh(n, jitter=jitter, seed=seed), mu, nu, seed=seed, quad=quad)


def square16():
    return square(16, mu=100.0, nu=1.0)


def square512j():
    return square(512, mu=1000.0, nu=1.0, jitter=0.2, seed=0, quad=3)


def cube(n, mu=100.0, nu=1.0, seed=0, quad=2):
    return transient_stokes(cube_mesh(n), mu, nu, seed=seed, quad=quad)


def cube64():
    return cube(64)


def ns_square(n, nu=0.01, seed=0, quad=3):
    coords, elems = square_mesh(n)
    man = Manufactured(2, seed=seed, mu=0.0, nu=nu)
    fbar = element_means(coords, elems, man.f, n=quad)
    lin = LinearisationField2D(seed=seed)
    faces = interior_face_list(elems)
    ubar = lin.face_means(coords, faces)
    return dict(coords=coords, elems=elems, mu=0.0, nu=float(nu), fbar=fbar,
                problem="ns", ulin=ubar, faces=faces)


def ns256():
    return ns_square(256)


def ns_cube(n, nu=0.01, seed=0, quad=2):
    """3D steady Navier-Stokes Newton step on n^3 cubes x 6 tetrahedra: manufactured
    force, linearisation velocity = face means of a seeded divergence-free field
    (LinearisationField3D, max|u| = 1, so nu = 1/Re)."""
    coords, elems = cube_mesh(n)
    man = Manufactured(3, seed=seed, mu=0.0, nu=nu)
    fbar = element_means(coords, elems, man.f, n=quad)
    lin = LinearisationField3D(seed=seed)
    faces = interior_face_list(elems)
    ubar = lin.face_means(coords, faces)
    return dict(coords=coords, elems=elems, mu=0.0, nu=float(nu), fbar=fbar,
                problem="ns", ulin=ubar, faces=faces)


def serving_sessions(n_requests=2000, seed=1, n_min=32, n_max=512, rate=20.0, dt_range=(1e-3, 1e-1),
                     max_steps=20, quad=2, nu=1.0):
    """Transient-Stokes serving workload: sessions arrive as a Poisson process
    (rate per second); each has an N x N x 2 mesh with N log-uniform in
    [n_min, n_max], a time step dt uniform in dt_range (mu = 1/dt), 1 to
    max_steps backward-Euler steps, and the force of one seeded manufactured
    velocity.  Sessions are drawn until their steps total n_requests.
    Returns a list of dicts (n, dt, steps, arrival, coords, elems, fbar)."""
    rng = np.random.default_rng(seed)
    man = Manufactured(2, seed=seed, mu=1.0, nu=nu)
    meshes = {}
    out = []
    total, t = 0, 0.0
    while total < n_requests:
        n = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max)))))
        dt = float(rng.uniform(*dt_range))
        steps = int(min(rng.integers(1, max_steps + 1), n_requests - total))
        t += float(rng.exponential(1.0 / rate))
        if n not in meshes:
            meshes[n] = square_mesh(n)
        coords, elems = meshes[n]
        fbar = element_means(coords, elems, man.force(1.0 / dt, nu), n=quad)
        out.append(dict(n=n, dt=dt, steps=steps, arrival=t, coords=coords, elems=elems, fbar=fbar, nu=nu))
        total += steps
    return out

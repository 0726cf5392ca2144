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
The right-hand side is the element mean of the force implied by a seeded
smooth manufactured velocity (Manufactured).
"""
from __future__ import annotations

import numpy as np

from .fields import LinearisationField2D, Manufactured, element_means
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

"""Seeded synthetic simplicial meshes (triangles in 2D, tetrahedra in 3D).

These are input generators only: they produce vertex coordinates and element
vertex lists and hold none of the discretisation's arithmetic.  Both the HIP
path and the CPU oracle consume the arrays they return.

The paper's workloads run on the FVCA "Mesh1" triangle family and on cubes cut
into six tetrahedra (Section 4.1, Section 4.2).  The triangle family is not
available here; a structured square grid with every cell cut along one
diagonal, with optional seeded jitter of the interior vertices, stands in for
it.  The cube split is the Kuhn (Freudenthal) split into six tetrahedra around
the main diagonal, which is conforming across cubes.
"""
from __future__ import annotations

import itertools

import numpy as np


def square_mesh(n: int, jitter: float = 0.0, seed: int = 0):
    """Unit square, n x n cells, each cut into two triangles.

    Vertex (i, j) (x index i, y index j) has id j*(n+1)+i.  Cell (i, j) is cut
    along its diagonal from (i, j) to (i+1, j+1) into a lower triangle
    (v00, v10, v11) and an upper triangle (v00, v11, v01); elements are listed
    cell by cell (x fastest), lower before upper.

    ``jitter`` moves every interior vertex by an independent uniform draw in
    [-jitter*h, jitter*h] in each coordinate (h = 1/n), boundary vertices stay
    fixed.  With jitter <= 0.2 every triangle keeps a positive area.
    Returns (coords float64 [(n+1)^2, 2], elems int32 [2 n^2, 3]).
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    h = 1.0 / n
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    coords = np.stack([ii.ravel() * h, jj.ravel() * h], axis=1).astype(np.float64)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        disp = rng.uniform(-jitter * h, jitter * h, size=coords.shape)
        interior = ((ii.ravel() > 0) & (ii.ravel() < n) & (jj.ravel() > 0) & (jj.ravel() < n))
        coords = coords + disp * interior[:, None]
    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ci = ci.ravel()
    cj = cj.ravel()
    v00 = cj * (n + 1) + ci
    v10 = v00 + 1
    v01 = v00 + (n + 1)
    v11 = v01 + 1
    lower = np.stack([v00, v10, v11], axis=1)
    upper = np.stack([v00, v11, v01], axis=1)
    elems = np.stack([lower, upper], axis=1).reshape(-1, 3).astype(np.int32)
    return coords, elems


def cube_mesh(n: int):
    """Unit cube, n^3 cubes, each cut into six tetrahedra (Kuhn split).

    Vertex (i, j, k) has id (k*(n+1)+j)*(n+1)+i.  For every permutation
    (a, b, c) of the axes, the tetrahedron is the path 000 -> e_a -> e_a+e_b ->
    111 through the cube.  Elements are listed cube by cube (x fastest), the six
    permutations in lexicographic order.
    Returns (coords float64 [(n+1)^3, 3], elems int32 [6 n^3, 4]).
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    h = 1.0 / n
    m = n + 1
    kk, jj, ii = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    coords = np.stack([ii.ravel() * h, jj.ravel() * h, kk.ravel() * h], axis=1).astype(np.float64)
    ck, cj, ci = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ci = ci.ravel()
    cj = cj.ravel()
    ck = ck.ravel()

    def vid(di, dj, dk):
        return ((ck + dk) * m + (cj + dj)) * m + (ci + di)

    tets = []
    for perm in itertools.permutations(range(3)):
        step = [0, 0, 0]
        path = [vid(0, 0, 0)]
        for ax in perm:
            step[ax] = 1
            path.append(vid(*step))
        tets.append(np.stack(path, axis=1))
    elems = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    return coords, elems

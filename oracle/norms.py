"""Error norms of a discrete CR solution against a smooth exact solution.

Test infrastructure only.  The discrete velocity is affine on each element,
u_h|_K = sum_sigma U_sigma phi_sigma with the CR basis of Section 2 item 1
(U = 0, or the given boundary data, on exterior faces); the discrete pressure is constant per element
(Section 2 item 5) and is compared after removing its |K|-weighted mean, as
Section 2 item 5 suggests for retrieving an element of L^2_0.
"""
from __future__ import annotations

import numpy as np

from .cr import Mesh, boundary_local_values, cr_basis, local_face_values


def errors(m: Mesh, U, Pk, exact_u, exact_grad, exact_p, quad, gbnd=None):
    """Broken L2 and H1 velocity errors and L2 pressure error.

    quad = (barycentric points [nq, d+1], weights [nq] summing to 1).
    gbnd: the velocity on the exterior faces [nbf, d] (None: zero).
    Returns dict(l2u, h1u, l2p) of absolute errors.
    """
    lam, wt = quad
    c, grad = cr_basis(m)
    X = m.coords[m.elems]
    pts = np.einsum("qj,ejd->eqd", lam, X)
    ne, nq, d = pts.shape
    Ul = local_face_values(m, U)                                   # [ne, d1, d]
    if gbnd is not None:
        Ul = Ul + boundary_local_values(m, gbnd)
    phi = c[:, None, :] + np.einsum("eqd,esd->eqs", pts - m.xK[:, None, :], grad)
    uh = np.einsum("eqs,esi->eqi", phi, Ul)
    guh = np.einsum("esi,esj->eij", Ul, grad)                       # d u_i / d x_j
    flat = pts.reshape(-1, d)
    ue = exact_u(flat).reshape(ne, nq, d)
    ge = exact_grad(flat).reshape(ne, nq, d, d)
    pe = exact_p(flat).reshape(ne, nq)
    w = wt[None, :] * m.vol[:, None]
    l2u = np.sqrt((w[:, :, None] * (ue - uh) ** 2).sum())
    h1u = np.sqrt((w[:, :, None, None] * (ge - guh[:, None]) ** 2).sum())
    area = m.vol.sum()
    pe_mean = (w * pe).sum() / area
    ph_mean = (m.vol * Pk).sum() / area
    l2p = np.sqrt((w * ((pe - pe_mean) - (Pk[:, None] - ph_mean)) ** 2).sum())
    return dict(l2u=l2u, h1u=h1u, l2p=l2p)

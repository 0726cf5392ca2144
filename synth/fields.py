"""Seeded smooth fields and simplex quadrature used to build solver inputs.

Input generators only: a manufactured velocity/pressure pair and the body
force it implies through the strong form (Section 2, first display:
mu u - nu Lap u + grad p = f), per-element means of a field (the forcing data
the right-hand side of the scheme consumes, Section 2 item 4), point values at
face centroids (previous time-step velocity), and a discretely
divergence-free linearisation velocity for the Newton step of the
Navier-Stokes case.  None of the scheme's arithmetic lives here.
"""
from __future__ import annotations

import math

import numpy as np
import sympy as sp

# ---------------------------------------------------------------------------
# Quadrature on simplices: collapsed (Duffy) tensor Gauss-Legendre rules.
# ---------------------------------------------------------------------------


def _gl01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def simplex_rule(dim: int, n: int):
    """Barycentric points [nq, dim+1] and weights [nq] (sum 1) on a simplex.

    Collapsed Gauss-Legendre rule with n points per direction; exact for
    polynomials of total degree 2n-1-dim+1 at least (2n-2 in 2D, 2n-3 in 3D).
    """
    t, w = _gl01(n)
    if dim == 2:
        u, v = np.meshgrid(t, t, indexing="ij")
        wu, wv = np.meshgrid(w, w, indexing="ij")
        l1 = u
        l2 = v * (1.0 - u)
        wt = 2.0 * wu * wv * (1.0 - u)
        lam = np.stack([1.0 - l1 - l2, l1, l2], axis=-1).reshape(-1, 3)
        return lam, wt.ravel()
    if dim == 3:
        u, v, s = np.meshgrid(t, t, t, indexing="ij")
        wu, wv, ws = np.meshgrid(w, w, w, indexing="ij")
        l1 = u
        l2 = v * (1.0 - u)
        l3 = s * (1.0 - u) * (1.0 - v)
        wt = 6.0 * wu * wv * ws * (1.0 - u) ** 2 * (1.0 - v)
        lam = np.stack([1.0 - l1 - l2 - l3, l1, l2, l3], axis=-1).reshape(-1, 4)
        return lam, wt.ravel()
    raise ValueError("dim must be 2 or 3")


def element_points(coords, elems, lam):
    """Physical quadrature points [n_e, nq, dim] for barycentric points lam."""
    X = coords[elems]  # [ne, dim+1, dim]
    return np.einsum("qj,ejd->eqd", lam, X)


def element_means(coords, elems, fn, n: int = 4, chunk: int = 1 << 20):
    """Mean value over each element of a vector field fn(points [N, dim]) -> [N, k].

    Evaluated in chunks of elements so that large meshes stay within memory.
    """
    dim = coords.shape[1]
    lam, wt = simplex_rule(dim, n)
    nq = len(wt)
    ne = elems.shape[0]
    per = max(1, chunk // nq)
    out = None
    for s in range(0, ne, per):
        e = elems[s:s + per]
        pts = element_points(coords, e, lam).reshape(-1, dim)
        vals = np.asarray(fn(pts), dtype=np.float64)
        k = vals.shape[1]
        if out is None:
            out = np.empty((ne, k), dtype=np.float64)
        out[s:s + per] = np.einsum("eqk,q->ek", vals.reshape(len(e), nq, k), wt)
    return out


def face_centroids(coords, face_vertices):
    return coords[face_vertices].mean(axis=1)


# ---------------------------------------------------------------------------
# Manufactured solution: u = curl(psi) with psi vanishing to second order on
# the boundary (so u = 0 there), a seeded cosine pressure, and
# f = mu u - nu Lap u + grad p.
# ---------------------------------------------------------------------------


class Manufactured:
    """Seeded smooth divergence-free velocity, pressure and implied force."""

    def __init__(self, dim: int, seed: int = 0, mu: float = 1.0, nu: float = 1.0):
        self.dim = dim
        self.mu = float(mu)
        self.nu = float(nu)
        rng = np.random.default_rng(seed)
        X = sp.symbols("x0:%d" % dim, real=True)
        self._X = X
        bubble = sp.Integer(1)
        for x in X:
            bubble = bubble * x * (1 - x)
        scale = 4 ** (2 * dim)  # max of bubble^2 becomes 1
        pi = sp.pi

        def smooth(nterm):
            g = sp.Integer(1)
            for _ in range(nterm):
                c = sp.Float(rng.uniform(-0.5, 0.5))
                freq = [int(rng.integers(1, 4)) for _ in range(dim)]
                th = sp.Float(rng.uniform(0.0, 2.0 * math.pi))
                g = g + c * sp.sin(pi * sum(fq * x for fq, x in zip(freq, X)) + th)
            return g

        if dim == 2:
            psi = scale * bubble ** 2 * smooth(4)
            u = [sp.diff(psi, X[1]), -sp.diff(psi, X[0])]
        elif dim == 3:
            A = [scale * bubble ** 2 * smooth(3) for _ in range(3)]
            x, y, z = X
            u = [sp.diff(A[2], y) - sp.diff(A[1], z),
                 sp.diff(A[0], z) - sp.diff(A[2], x),
                 sp.diff(A[1], x) - sp.diff(A[0], y)]
        else:
            raise ValueError("dim must be 2 or 3")
        p = sp.Integer(0)
        for _ in range(3):
            c = sp.Float(rng.uniform(-1.0, 1.0))
            freq = [int(rng.integers(1, 3)) for _ in range(dim)]
            th = sp.Float(rng.uniform(0.0, 2.0 * math.pi))
            p = p + c * sp.cos(pi * sum(fq * x for fq, x in zip(freq, X)) + th)
        lap = [sum(sp.diff(ui, x, 2) for x in X) for ui in u]
        f = [self.mu * ui - self.nu * li + sp.diff(p, x) for ui, li, x in zip(u, lap, X)]
        grad = [[sp.diff(ui, x) for x in X] for ui in u]
        self._u = sp.lambdify(X, u, modules="numpy", cse=True)
        self._p = sp.lambdify(X, p, modules="numpy", cse=True)
        self._f = sp.lambdify(X, f, modules="numpy", cse=True)
        self._g = sp.lambdify(X, [g for row in grad for g in row], modules="numpy", cse=True)
        # the pieces of f separately, for forces with other coefficients
        self._parts = sp.lambdify(X, u + lap + [sp.diff(p, x) for x in X], modules="numpy", cse=True)

    def _eval(self, fn, pts, k):
        cols = [pts[:, i] for i in range(self.dim)]
        vals = fn(*cols)
        out = np.empty((pts.shape[0], k), dtype=np.float64)
        for i, v in enumerate(vals if k > 1 else [vals]):
            out[:, i] = v
        return out

    def u(self, pts):
        return self._eval(self._u, pts, self.dim)

    def p(self, pts):
        return self._eval(self._p, pts, 1)[:, 0]

    def f(self, pts):
        return self._eval(self._f, pts, self.dim)

    def force(self, mu, nu):
        """f = mu u - nu Lap u + grad p for other coefficients than the constructor's."""
        d = self.dim

        def fn(pts):
            v = self._eval(self._parts, pts, 3 * d)
            return mu * v[:, :d] - nu * v[:, d:2 * d] + v[:, 2 * d:]
        return fn

    def grad_u(self, pts):
        return self._eval(self._g, pts, self.dim * self.dim).reshape(-1, self.dim, self.dim)


def constant_force(value):
    """A constant body force, for which the exact discrete velocity is zero."""
    value = np.asarray(value, dtype=np.float64)

    def fn(pts):
        return np.broadcast_to(value, (pts.shape[0], value.shape[0])).copy()

    return fn


# ---------------------------------------------------------------------------
# Linearisation velocity for the Newton step (2D): u = curl(psi) with
# psi = S * bubble^2 * sum_k a_k sin(2 pi (m_k x + n_k y) + theta_k), 8 modes,
# scaled so that max |u| is 1 on a sample grid.  Face means: the normal part is
# exact (difference of psi between the face end points), the tangential part
# uses 5-point Gauss-Legendre; the normal fluxes therefore sum to zero around
# every element.
# ---------------------------------------------------------------------------


class LinearisationField2D:
    def __init__(self, seed: int = 0, modes: int = 8):
        rng = np.random.default_rng(seed)
        x, y = sp.symbols("x y", real=True)
        bubble = x * (1 - x) * y * (1 - y)
        s = sp.Integer(0)
        for _ in range(modes):
            a = sp.Float(rng.normal())
            m = int(rng.integers(1, 5))
            n = int(rng.integers(1, 5))
            th = sp.Float(rng.uniform(0.0, 2.0 * math.pi))
            s = s + a * sp.sin(2 * sp.pi * (m * x + n * y) + th)
        psi = 256 * bubble ** 2 * s
        u = [sp.diff(psi, y), -sp.diff(psi, x)]
        psi_f = sp.lambdify((x, y), psi, modules="numpy")
        u_f = sp.lambdify((x, y), u, modules="numpy")
        g = np.linspace(0.0, 1.0, 201)
        gx, gy = np.meshgrid(g, g, indexing="ij")
        uu = np.asarray(u_f(gx, gy))
        self.scale = 1.0 / float(np.sqrt((uu ** 2).sum(axis=0)).max())
        self._psi = psi_f
        self._u = u_f

    def psi(self, pts):
        return self.scale * np.asarray(self._psi(pts[:, 0], pts[:, 1]), dtype=np.float64)

    def u(self, pts):
        v = self._u(pts[:, 0], pts[:, 1])
        return self.scale * np.stack([np.broadcast_to(v[0], pts[:, 0].shape),
                                      np.broadcast_to(v[1], pts[:, 0].shape)], axis=1)

    def face_means(self, coords, face_vertices):
        """Mean of u over each face [nf, 2]; face_vertices [nf, 2] (any order).

        The end points are taken in increasing vertex-id order so that the
        value of a face does not depend on which element lists it.
        """
        fv = np.sort(np.asarray(face_vertices), axis=1)
        a = coords[fv[:, 0]]
        b = coords[fv[:, 1]]
        e = b - a
        L = np.sqrt((e ** 2).sum(axis=1))
        t = e / L[:, None]
        nrm = np.stack([t[:, 1], -t[:, 0]], axis=1)
        un = (self.psi(b) - self.psi(a)) / L
        q, w = _gl01(5)
        ut = np.zeros(len(fv))
        for qi, wi in zip(q, w):
            pts = a + qi * e
            ut += wi * (self.u(pts) * t).sum(axis=1)
        return un[:, None] * nrm + ut[:, None] * t


class LinearisationField3D:
    """Seeded smooth divergence-free velocity on the unit cube, u = curl A with
    a vector potential A = bubble^2 x (8 Fourier modes per component), scaled to
    max|u| = 1, and its face means with exact normal fluxes: the flux of u
    through a triangle is the circulation of A around its edges (Stokes'
    theorem), each edge integral computed once per edge, so that the face
    values are discretely divergence-free on every tetrahedron up to rounding.
    The tangential part is the face mean of u by quadrature."""

    def __init__(self, seed: int = 0, modes: int = 8):
        rng = np.random.default_rng(seed)
        X = sp.symbols("x0:3", real=True)
        bubble = X[0] * (1 - X[0]) * X[1] * (1 - X[1]) * X[2] * (1 - X[2])
        A = []
        for _ in range(3):
            s = sp.Integer(0)
            for _ in range(modes):
                a = sp.Float(rng.normal())
                k = [int(rng.integers(1, 4)) for _ in range(3)]
                th = sp.Float(rng.uniform(0.0, 2.0 * math.pi))
                s = s + a * sp.sin(2 * sp.pi * (k[0] * X[0] + k[1] * X[1] + k[2] * X[2]) + th)
            A.append(4096 * bubble ** 2 * s)
        u = [sp.diff(A[2], X[1]) - sp.diff(A[1], X[2]),
             sp.diff(A[0], X[2]) - sp.diff(A[2], X[0]),
             sp.diff(A[1], X[0]) - sp.diff(A[0], X[1])]
        self._A = sp.lambdify(X, A, modules="numpy")
        self._u = sp.lambdify(X, u, modules="numpy")
        g = np.linspace(0.0, 1.0, 41)
        gx, gy, gz = np.meshgrid(g, g, g, indexing="ij")
        pts = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
        self.scale = 1.0
        self.scale = 1.0 / float(np.sqrt((self.u(pts) ** 2).sum(axis=1)).max())

    @staticmethod
    def _vec(fn, pts):
        v = fn(pts[:, 0], pts[:, 1], pts[:, 2])
        return np.stack([np.broadcast_to(np.asarray(c, dtype=np.float64), pts[:, 0].shape) for c in v], axis=1)

    def A(self, pts):
        return self.scale * self._vec(self._A, pts)

    def u(self, pts):
        return self.scale * self._vec(self._u, pts)

    def _edge(self, a, b):
        """Integral of A . dl along the straight edge from a to b (5-point Gauss)."""
        q, w = _gl01(5)
        e = b - a
        out = np.zeros(len(a))
        for qi, wi in zip(q, w):
            out += wi * (self.A(a + qi * e) * e).sum(axis=1)
        return out

    def face_means(self, coords, face_vertices):
        """Mean of u over each triangle [nf, 3]; face_vertices [nf, 3] (any order)."""
        fv = np.sort(np.asarray(face_vertices), axis=1)
        p0, p1, p2 = coords[fv[:, 0]], coords[fv[:, 1]], coords[fv[:, 2]]
        nv = 0.5 * np.cross(p1 - p0, p2 - p0)
        area = np.sqrt((nv ** 2).sum(axis=1))
        n = nv / area[:, None]
        # circulation along p0 -> p1 -> p2 -> p0, every edge taken from its lower to
        # its higher vertex id (the same number wherever the edge appears)
        circ = self._edge(p0, p1) + self._edge(p1, p2) - self._edge(p0, p2)
        un = circ / area
        lam, wq = simplex_rule(2, 4)
        um = np.zeros((len(fv), 3))
        for l, wi in zip(lam, wq):
            um += wi * self.u(l[0] * p0 + l[1] * p1 + l[2] * p2)
        ut = um - (um * n).sum(axis=1)[:, None] * n
        return un[:, None] * n + ut


def face_means(coords, faces, fn, n: int = 5):
    """Mean of a vector field fn(pts [m, dim]) -> [m, k] over each face [nf, dim]
    (vertex ids): Gauss-Legendre on segments (2D), the collapsed rule on triangles (3D)."""
    faces = np.asarray(faces)
    dim = coords.shape[1]
    P = coords[faces]  # [nf, dim(vertices), dim]
    if dim == 2:
        q, w = _gl01(n)
        out = None
        for qi, wi in zip(q, w):
            v = wi * np.asarray(fn(P[:, 0] + qi * (P[:, 1] - P[:, 0])))
            out = v if out is None else out + v
        return out
    lam, w = simplex_rule(2, n)
    out = None
    for l, wi in zip(lam, w):
        v = wi * np.asarray(fn(l[0] * P[:, 0] + l[1] * P[:, 1] + l[2] * P[:, 2]))
        out = v if out is None else out + v
    return out


class GreenTaylor2D:
    """The Green-Taylor vortex of the paper's 2D convergence test (Section 4.1,
    eqs. gretayvel and gretaypre), an exact solution of the Navier-Stokes
    equations with zero force and viscosity nu:
      u = amp (-cos(k (x + 1/4)) sin(k (y + 1/2)), sin(k (x + 1/4)) cos(k (y + 1/2))) exp(-2 k^2 nu t),
      p = -amp^2 (cos(2k (x + 1/4)) + cos(2k (y + 1/2))) / 4 exp(-4 k^2 nu t),
    with k = 2 pi (the paper: amp = Re = 100, nu = 1).  Its velocity does not
    vanish on the boundary of the unit square (non-homogeneous Dirichlet data,
    zero net flux).  u.grad u + grad p = 0, so (u, p) also solves the steady
    problem -nu Lap u + u.grad u + grad p = 2 k^2 nu u, and the Stokes problem
    mu u - nu Lap u + grad p = f with f = (mu + 2 k^2 nu) u + grad p."""

    def __init__(self, amp: float = 1.0, nu: float = 1.0, k: float = 2.0 * math.pi):
        self.amp = float(amp)
        self.nu = float(nu)
        self.k = float(k)

    def _decay(self, t, m=2):
        return math.exp(-m * self.k ** 2 * self.nu * t)

    def _xy(self, pts):
        return self.k * (pts[:, 0] + 0.25), self.k * (pts[:, 1] + 0.5)

    def u(self, pts, t=0.0):
        X, Y = self._xy(pts)
        e = self.amp * self._decay(t)
        return np.stack([-np.cos(X) * np.sin(Y), np.sin(X) * np.cos(Y)], axis=1) * e

    def grad_u(self, pts, t=0.0):
        """[m, 2 (component), 2 (derivative)]"""
        X, Y = self._xy(pts)
        e = self.amp * self._decay(t) * self.k
        g = np.empty((len(X), 2, 2))
        g[:, 0, 0] = np.sin(X) * np.sin(Y) * e
        g[:, 0, 1] = -np.cos(X) * np.cos(Y) * e
        g[:, 1, 0] = np.cos(X) * np.cos(Y) * e
        g[:, 1, 1] = -np.sin(X) * np.sin(Y) * e
        return g

    def p(self, pts, t=0.0):
        X, Y = self._xy(pts)
        return -self.amp ** 2 * (np.cos(2 * X) + np.cos(2 * Y)) / 4.0 * self._decay(t, 4)

    def grad_p(self, pts, t=0.0):
        X, Y = self._xy(pts)
        c = self.amp ** 2 * self.k / 2.0 * self._decay(t, 4)
        return np.stack([np.sin(2 * X), np.sin(2 * Y)], axis=1) * c

    def stokes_force(self, mu, t=0.0):
        """f = mu u - nu Lap u + grad p at time t (Lap u = -2 k^2 u)."""
        def fn(pts):
            return (mu + 2.0 * self.k ** 2 * self.nu) * self.u(pts, t) + self.grad_p(pts, t)
        return fn

    def steady_ns_force(self, t=0.0):
        """f = -nu Lap u + u.grad u + grad p = 2 k^2 nu u (the convection and the
        pressure gradient cancel)."""
        def fn(pts):
            return 2.0 * self.k ** 2 * self.nu * self.u(pts, t)
        return fn


class GreenTaylor3D(GreenTaylor2D):
    """The 3D extension of the Green-Taylor vortex used by the paper's 3D tests
    (Section 4.1): the first two velocity components and the pressure are those
    of the 2D vortex in (x1, x2), independent of x3, and the third component is
    zero.  It solves the unforced 3D Navier-Stokes equations on the unit cube
    (non-homogeneous Dirichlet data on every face)."""

    def u(self, pts, t=0.0):
        u2 = super().u(pts[:, :2], t)
        return np.concatenate([u2, np.zeros((len(pts), 1))], axis=1)

    def grad_u(self, pts, t=0.0):
        g2 = super().grad_u(pts[:, :2], t)
        g = np.zeros((len(pts), 3, 3))
        g[:, :2, :2] = g2
        return g

    def p(self, pts, t=0.0):
        return super().p(pts[:, :2], t)

    def grad_p(self, pts, t=0.0):
        g2 = super().grad_p(pts[:, :2], t)
        return np.concatenate([g2, np.zeros((len(pts), 1))], axis=1)

"""Oracle: Crouzeix-Raviart scheme, coupled system and hybrid method in plain FP64.

Test infrastructure only (see the package docstring).  Local numbering inside
an element: face j is the face opposite local vertex j; local velocity unknowns
are ordered face-major, index = face * d + component.  Global velocity unknowns
use the canonical interior-face order (faces as sorted vertex tuples, sorted
lexicographically) and the same face-major layout.  Pressures are indexed by
element (caller order); the pinned element K0 carries P = 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla


class MeshError(ValueError):
    pass


# ---------------------------------------------------------------------------
# Topology and geometry (Section 2, item 1)
# ---------------------------------------------------------------------------


@dataclass
class Mesh:
    coords: np.ndarray          # [nv, d]
    elems: np.ndarray           # [ne, d+1]
    d: int
    faces: np.ndarray           # [nf, d] interior faces, sorted vertex ids, canonical order
    elem_face: np.ndarray       # [ne, d+1] canonical interior face of local face j, -1 if exterior
    face_elems: np.ndarray      # [nf, 2] (K, L) with K < L
    vol: np.ndarray             # [ne] |K|
    xK: np.ndarray              # [ne, d] centre of gravity of K
    xs: np.ndarray              # [ne, d+1, d] centre of gravity of local face j
    a: np.ndarray               # [ne, d+1, d] a_{K,sigma} = |sigma| n_{K,sigma}, outward
    area: np.ndarray            # [ne, d+1] |sigma|
    sign: np.ndarray = field(default=None)  # [ne, d+1] C_K entry of local face j (0 if exterior)
    bfaces: np.ndarray = field(default=None)      # [nbf, d] exterior faces, sorted vertex ids, lexicographic
    elem_bface: np.ndarray = field(default=None)  # [ne, d+1] exterior face of local face j, -1 if interior

    @property
    def ne(self):
        return self.elems.shape[0]

    @property
    def nf(self):
        return self.faces.shape[0]

    def interior_mask(self):
        return self.elem_face >= 0


def build_mesh(coords, elems) -> Mesh:
    """Faces, interior/exterior split, M_sigma, x_K, x_sigma and a_{K,sigma}.

    Section 2 item 1: every element has d+1 faces (no hanging nodes); a face is
    interior iff it belongs to two elements, exterior iff to one.  a_{K,sigma}
    is |sigma| times the unit normal to sigma pointing out of K, computed here
    from its geometric definition (edge rotation in 2D, half cross product in
    3D), oriented by the sign of (x_sigma - x_K).
    """
    coords = np.asarray(coords, dtype=np.float64)
    elems = np.asarray(elems, dtype=np.int64)
    ne, d1 = elems.shape
    d = d1 - 1
    if coords.shape[1] != d or d not in (2, 3):
        raise MeshError("coordinates/element arity mismatch")
    loc = np.stack([np.delete(elems, j, axis=1) for j in range(d1)], axis=1)  # [ne, d1, d]
    keys = np.sort(loc, axis=2).reshape(-1, d)
    uniq, inv, counts = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
    inv = inv.reshape(-1)
    if (counts > 2).any():
        raise MeshError("a face is shared by more than two elements")
    interior = counts == 2
    canon = -np.ones(len(uniq), dtype=np.int64)
    canon[interior] = np.arange(int(interior.sum()))
    elem_face = canon[inv].reshape(ne, d1)
    faces = uniq[interior]
    nf = faces.shape[0]
    owners = np.full((nf, 2), -1, dtype=np.int64)
    kk, jj = np.nonzero(elem_face >= 0)
    ff = elem_face[kk, jj]
    order = np.lexsort((kk, ff))
    ff_s, kk_s = ff[order], kk[order]
    owners[:, 0] = kk_s[0::2]
    owners[:, 1] = kk_s[1::2]
    assert (ff_s[0::2] == np.arange(nf)).all() and (ff_s[1::2] == np.arange(nf)).all()

    X = coords[elems]                           # [ne, d1, d]
    xK = X.mean(axis=1)
    xs = (X.sum(axis=1)[:, None, :] - X) / d    # centroid of the face opposite vertex j
    E = X[:, 1:, :] - X[:, :1, :]
    vol = np.abs(np.linalg.det(E)) / math.factorial(d)
    if (vol <= 0).any() or not np.isfinite(vol).all():
        raise MeshError("zero-volume element")
    a = np.zeros((ne, d1, d))
    for j in range(d1):
        fv = X[:, [m for m in range(d1) if m != j], :]
        if d == 2:
            t = fv[:, 1] - fv[:, 0]
            n = np.stack([t[:, 1], -t[:, 0]], axis=1)
        else:
            n = 0.5 * np.cross(fv[:, 1] - fv[:, 0], fv[:, 2] - fv[:, 0])
        s = np.sign(((xs[:, j] - xK) * n).sum(axis=1))
        a[:, j] = n * s[:, None]
    area = np.sqrt((a ** 2).sum(axis=2))
    m = Mesh(coords=coords, elems=elems, d=d, faces=faces, elem_face=elem_face,
             face_elems=owners, vol=vol, xK=xK, xs=xs, a=a, area=area)
    m.sign = default_signs(m)
    bcanon = -np.ones(len(uniq), dtype=np.int64)
    bcanon[~interior] = np.arange(int((~interior).sum()))
    m.bfaces = uniq[~interior]
    m.elem_bface = bcanon[inv].reshape(ne, d1)
    return m


def default_signs(m: Mesh):
    """C_K of eq. propc: +1 on the lower-index element of a face, -1 on the other.

    Section 3.2 asks only that the two entries of a face are opposite and
    non-zero; this fixes the choice.
    """
    sign = np.zeros(m.elem_face.shape)
    for j in range(m.d + 1):
        f = m.elem_face[:, j]
        ok = f >= 0
        k = np.nonzero(ok)[0]
        sign[k, j] = np.where(m.face_elems[f[ok], 0] == k, 1.0, -1.0)
    return sign


# ---------------------------------------------------------------------------
# Crouzeix-Raviart basis and element matrices (Section 2 items 1-3, Section 3.1)
# ---------------------------------------------------------------------------


def cr_basis(m: Mesh):
    """Affine CR basis on each element from its defining conditions.

    Section 2 item 1: phi_sigma restricted to K is affine with mean 1 on sigma
    and 0 on the other faces of K.  For an affine function the face mean is
    its value at the face centre of gravity, so with
    phi(x) = c + g.(x - x_K) the conditions are a (d+1)x(d+1) linear system.
    Returns (c [ne, d1], grad [ne, d1 (sigma), d]).
    """
    d1 = m.d + 1
    M = np.concatenate([np.ones((m.ne, d1, 1)), m.xs - m.xK[:, None, :]], axis=2)
    coef = np.linalg.solve(M, np.broadcast_to(np.eye(d1), (m.ne, d1, d1)))
    c = coef[:, 0, :]
    grad = np.transpose(coef[:, 1:, :], (0, 2, 1))
    return c, grad


def mass_matrix(m: Mesh, quad_rule=None):
    """Element matrix of int_K Pi_h phi_sigma Pi_h phi_sigma' (Section 2 item 3).

    2D: Pi_h is the identity; the integral of the product of two affine basis
    functions is computed with a quadrature rule exact for quadratics.
    3D: Pi_h phi_sigma is the indicator of the cones D_{K,sigma} (base sigma,
    apex x_K), so the element matrix is diagonal with the cone volumes
    |sigma| * dist(x_K, sigma) / d.
    """
    d1 = m.d + 1
    if m.d == 2:
        if quad_rule is None:
            # degree-2 exact rule at the edge midpoints of a triangle
            lam = np.array([[0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])
            wt = np.full(3, 1.0 / 3.0)
        else:
            lam, wt = quad_rule
        c, grad = cr_basis(m)
        X = m.coords[m.elems]
        pts = np.einsum("qj,ejd->eqd", lam, X)                       # [ne, nq, d]
        phi = c[:, None, :] + np.einsum("eqd,esd->eqs", pts - m.xK[:, None, :], grad)
        return np.einsum("q,eqs,eqt->est", wt, phi, phi) * m.vol[:, None, None]
    height = ((m.xs - m.xK[:, None, :]) * m.a).sum(axis=2) / m.area
    cone = m.area * height / m.d
    Mm = np.zeros((m.ne, d1, d1))
    idx = np.arange(d1)
    Mm[:, idx, idx] = cone
    return Mm


def stiffness_matrix(m: Mesh):
    """Element matrix of int_K grad phi_sigma . grad phi_sigma' (Section 3.1)."""
    _, grad = cr_basis(m)
    return np.einsum("esd,etd->est", grad, grad) * m.vol[:, None, None]


def element_S(m: Mesh, mu, nu, quad_rule=None):
    """S_K = mu * mass + nu * stiffness over all d+1 local faces (Section 3.1).

    Rows and columns of exterior faces are removed later (restrict()).
    """
    return mu * mass_matrix(m, quad_rule) + nu * stiffness_matrix(m)


def element_D(m: Mesh):
    """(D_K)_{sigma,i} = -a^{(i)}_{K,sigma} (Section 3.1), face-major flattened."""
    return -m.a.reshape(m.ne, -1)


def element_R(m: Mesh, fbar, mu=0.0, u_prev=None):
    """(R_K)_{sigma,i} = a^{(i)}_{K,sigma} fbar_K.(x_sigma - x_K)  (eq. defrhs, Section 3.1).

    fbar [ne, d] is the element mean of the force.  When u_prev (the previous
    time-step velocity on the interior faces, [nf, d]) is given, the transient
    data enters through the same lumped mass as the mu term of S_K:
    + mu * |D_{K,sigma}| * U^{n-1}_{sigma,i}.  Exterior faces carry zero.
    """
    proj = ((m.xs - m.xK[:, None, :]) * fbar[:, None, :]).sum(axis=2)   # [ne, d1]
    R = m.a * proj[:, :, None]
    if u_prev is not None and mu != 0.0:
        Mm = mass_matrix(m)
        diag = np.einsum("ess->es", Mm)
        up = np.where(m.elem_face[:, :, None] >= 0, np.asarray(u_prev)[np.maximum(m.elem_face, 0)], 0.0)
        R = R + mu * diag[:, :, None] * up
    return R.reshape(m.ne, -1)


# ---------------------------------------------------------------------------
# Convection form b_h (Section 2 item 6, eq. defbh) and its Newton Jacobian
# ---------------------------------------------------------------------------


def local_face_values(m: Mesh, U):
    """Gather interior-face values [nf, d] into [ne, d1, d] with zeros on exterior faces."""
    U = np.asarray(U)
    return np.where(m.elem_face[:, :, None] >= 0, U[np.maximum(m.elem_face, 0)], 0.0)


def fluxes(m: Mesh, W):
    """F_{sigma,sigma'}(w) for every element and ordered face pair, [ne, d1, d1].

    Uses the closed form of Section 2 item 6: the flux through tau_{sigma,sigma'}
    of the affine w_K equals (W_s + W_s' - sum W / (d+1)) . (a_s' - a_s)/(d+1).
    W: local face values [ne, d1, d].
    """
    d1 = m.d + 1
    mean = W.sum(axis=1, keepdims=True) / d1
    val = W[:, :, None, :] + W[:, None, :, :] - mean[:, :, None, :]       # at x_{s,s'}
    g = (m.a[:, None, :, :] - m.a[:, :, None, :]) / d1                     # [ne, s, s', d]
    return (val * g).sum(axis=3)


def convection(m: Mesh, Wflux, Z):
    """Element vector N_K(w, z)_{sigma,i} = 1/2 sum_{s' != s} F_{s,s'}(w) (Z_{s',i} - Z_{s,i}).

    This is the test-function-sigma coefficient of b_h (second form of eq.
    defbh); its sum over elements gives b_h(w, z) against v.  Local face values
    [ne, d1, d] in, [ne, d1*d] out.
    """
    F = fluxes(m, Wflux)
    d1 = m.d + 1
    off = 1.0 - np.eye(d1)
    diff = Z[:, None, :, :] - Z[:, :, None, :]                              # [ne, s, s', i]
    out = 0.5 * np.einsum("est,esti->esi", F * off, diff)
    return out.reshape(m.ne, -1)


def convection_jacobian(m: Mesh, Ubar):
    """d/du of N_K(u, u) at u = ubar: N_K(ubar, .) + N_K(., ubar), [ne, d1*d, d1*d].

    Differentiates the closed form of fluxes()/convection(): F is linear in w
    with dF_{s,s'}/dW_{r,j} = (delta_{rs} + delta_{rs'} - 1/(d+1)) g^{(j)}_{s,s'}.
    """
    d, d1 = m.d, m.d + 1
    F = fluxes(m, Ubar) * (1.0 - np.eye(d1))
    g = (m.a[:, None, :, :] - m.a[:, :, None, :]) / d1                     # [ne, s, s', j]
    I = np.eye(d1)
    J = np.zeros((m.ne, d1, d, d1, d))
    # N(ubar, u): 1/2 sum_{s'} F_{s s'} (delta_{r s'} - delta_{r s}) delta_ij
    T1 = 0.5 * (F[:, :, :] - np.diag(np.ones(d1))[None] * F.sum(axis=2)[:, :, None])  # [ne, s, r]
    for i in range(d):
        J[:, :, i, :, i] += T1
    # N(u, ubar): 1/2 sum_{s'} dF_{s s'}/dU_{r j} (ubar_{s' i} - ubar_{s i})
    dU = Ubar[:, None, :, :] - Ubar[:, :, None, :]                          # [ne, s, s', i]
    coef = I[None, :, None, :] + I[None, None, :, :] - 1.0 / d1             # [1, s, s', r]
    offm = (1.0 - np.eye(d1))[None, :, :, None]
    cm = np.broadcast_to(coef * offm, (m.ne, d1, d1, d1))
    J += 0.5 * np.einsum("estr,estj,esti->esirj", cm, g, dU)
    return J.reshape(m.ne, d1 * d, d1 * d)


# ---------------------------------------------------------------------------
# Element matrices A_K, restriction to interior faces
# ---------------------------------------------------------------------------


@dataclass
class Problem:
    mesh: Mesh
    mu: float
    nu: float
    A: np.ndarray          # [ne, d1*d, d1*d] element velocity matrices (all local faces)
    D: np.ndarray          # [ne, d1*d]
    R: np.ndarray          # [ne, d1*d]
    k0: int = 0
    ulin: np.ndarray = None
    lam_scale: float = 2.0    # lambda_K = lam_scale * ||A_K||_inf on M1 (mu = 0), see element_E
    e: np.ndarray = None      # [ne] right-hand side of D_K^t U_K = e_K (boundary data; None: zero)
    gbnd: np.ndarray = None   # [nbf, d] velocity on the exterior faces (None: zero)

    def ediv(self):
        return np.zeros(self.mesh.ne) if self.e is None else self.e

    @property
    def d(self):
        return self.mesh.d

    def dof_mask(self):
        """[ne, d1*d] True for local unknowns on interior faces."""
        if getattr(self, "_mask", None) is None:
            self._mask = np.repeat(self.mesh.interior_mask(), self.d, axis=1)
        return self._mask

    def local_to_global(self):
        """[ne, d1*d] global velocity index (face * d + i), -1 on exterior faces."""
        if getattr(self, "_l2g", None) is None:
            ef = self.mesh.elem_face
            g = ef[:, :, None] * self.d + np.arange(self.d)[None, None, :]
            self._l2g = np.where(ef[:, :, None] >= 0, g, -1).reshape(self.mesh.ne, -1)
        return self._l2g


def boundary_local_values(m: Mesh, gbnd):
    """Exterior-face values [nbf, d] gathered into [ne, d1, d], zeros on interior faces."""
    g = np.asarray(gbnd)
    return np.where(m.elem_bface[:, :, None] >= 0, g[np.maximum(m.elem_bface, 0)], 0.0)


def make_problem(coords, elems, mu, nu, fbar, u_prev=None, ulin=None, k0=0, quad_rule=None, lam_scale=2.0,
                 gbnd=None):
    """Element data of eq. syslin: A_K, D_K, R_K (Section 3.1).

    Stokes: A_K = S_K on each diagonal component block.  Navier-Stokes Newton
    step about ulin (interior face values, [nf, d]): A_K is completed by the
    Jacobian of the convection form and R_K by N_K(ulin, ulin); this is the
    linear system J(ubar) u + D^t P = R_f + b(ubar, ubar) of one Newton step for
    S u + b(u, u) + D^t P = R_f.  (The Newton right-hand-side completion is a
    reading of Section 3.1, which only says that R_K "is completed by the
    non-linear terms issued from the Newton method".)
    """
    m = build_mesh(coords, elems)
    d = m.d
    S = element_S(m, mu, nu, quad_rule)
    A = np.einsum("est,ij->esitj", S, np.eye(d)).reshape(m.ne, (d + 1) * d, (d + 1) * d)
    R = element_R(m, np.asarray(fbar, dtype=np.float64), mu, u_prev)
    Gl = None if gbnd is None else boundary_local_values(m, gbnd)
    if ulin is not None:
        Ub = local_face_values(m, ulin)
        if Gl is not None:
            Ub = Ub + Gl  # the linearisation velocity takes the boundary data on exterior faces
        A = A + convection_jacobian(m, Ub)
        R = R + convection(m, Ub, Ub)
    D = element_D(m)
    e = None
    if Gl is not None:
        # known exterior-face values move to the right-hand side: the velocity
        # rows lose A_K[., bnd] g, and the divergence row of K reads
        # D_K^t U_K = -D_K[bnd] . g =: e_K over its interior faces
        g = Gl.reshape(m.ne, -1)
        R = R - np.einsum("eab,eb->ea", A, g)
        e = -(D * g).sum(axis=1)
    return Problem(mesh=m, mu=float(mu), nu=float(nu), A=A, D=D, R=R, k0=int(k0),
                   ulin=None if ulin is None else np.asarray(ulin), lam_scale=float(lam_scale), e=e,
                   gbnd=None if gbnd is None else np.asarray(gbnd, dtype=np.float64))


def restrict(P: Problem, k):
    """Interior-face restriction of element k: (A_K, D_K, R_K, global indices)."""
    mask = P.dof_mask()[k]
    idx = np.nonzero(mask)[0]
    return (P.A[k][np.ix_(idx, idx)], P.D[k][idx], P.R[k][idx], P.local_to_global()[k][idx], idx)


# ---------------------------------------------------------------------------
# Coupled system (eq. syslin) and its direct solution
# ---------------------------------------------------------------------------


def assemble_coupled(P: Problem):
    """A = sum H_K A_K H_K^t, D = sum_{K != K0} F_K D_K^t H_K^t, R = sum H_K R_K (Section 3.1).

    Returns (A csr [n, n], D csr [ne-1, n], R [n], prow) with prow[K] the row of
    P_K in D (-1 for K0).  n = d * #F_int.
    """
    m = P.mesh
    n = m.nf * P.d
    mask = P.dof_mask()
    g = P.local_to_global()
    rows, cols, vals = [], [], []
    for k in range(m.ne):
        idx = np.nonzero(mask[k])[0]
        gi = g[k][idx]
        rows.append(np.repeat(gi, len(gi)))
        cols.append(np.tile(gi, len(gi)))
        vals.append(P.A[k][np.ix_(idx, idx)].ravel())
    A = sps.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    prow = -np.ones(m.ne, dtype=np.int64)
    others = np.array([k for k in range(m.ne) if k != P.k0], dtype=np.int64)
    prow[others] = np.arange(len(others))
    kk, ll = np.nonzero(mask)
    keep = prow[kk] >= 0
    D = sps.csr_matrix((P.D[kk, ll][keep], (prow[kk][keep], g[kk, ll][keep])), shape=(m.ne - 1, n))
    R = np.zeros(n)
    np.add.at(R, g[mask], P.R[mask])
    return A, D, R, prow


def divergence_rhs(P: Problem, prow):
    """Right-hand side of the divergence rows (K != K0, row order prow): e_K."""
    e = np.zeros(P.mesh.ne - 1)
    keep = prow >= 0
    e[prow[keep]] = P.ediv()[keep]
    return e


def solve_coupled(P: Problem, refine=0):
    """Solve [A D^t; D 0][U; P] = [R; 0] with sparse LU (SuperLU).

    refine > 0 adds that many steps of iterative refinement with the same
    factors, x += LU^{-1} (b - M x), all in FP64: on large, badly scaled
    systems (transient Stokes with mu |K| far below nu) the plain LU solution
    leaves divergence residuals of 1e-8 relative, which refinement removes.
    Returns (U [nf, d], P [ne] with P[K0] = 0).
    """
    A, D, R, prow = assemble_coupled(P)
    n = A.shape[0]
    M = sps.bmat([[A, D.T], [D, None]], format="csc")
    rhs = np.concatenate([R, divergence_rhs(P, prow)])
    lu = spla.splu(M, permc_spec="COLAMD")
    sol = lu.solve(rhs)
    for _ in range(int(refine)):
        sol = sol + lu.solve(rhs - M @ sol)
    U = sol[:n].reshape(-1, P.d)
    Pk = np.zeros(P.mesh.ne)
    Pk[prow >= 0] = sol[n:][prow[prow >= 0]]
    return U, Pk


# ---------------------------------------------------------------------------
# Hybridisation (Section 3.2)
# ---------------------------------------------------------------------------


def mis_partition(m: Mesh):
    """M1 of Section 3.2 item 7: a maximal independent set of elements.

    Greedy in caller element order: K joins M1 unless a face-neighbour is
    already in M1.  Every other element then has a neighbour in M1, so
    M2 = complement of M1 is the set of neighbours of M1.
    """
    nb = -np.ones((m.ne, m.d + 1), dtype=np.int64)
    for j in range(m.d + 1):
        f = m.elem_face[:, j]
        ok = f >= 0
        k = np.nonzero(ok)[0]
        fe = m.face_elems[f[ok]]
        nb[k, j] = np.where(fe[:, 0] == k, fe[:, 1], fe[:, 0])
    in1 = np.zeros(m.ne, dtype=bool)
    for k in range(m.ne):
        ns = nb[k][nb[k] >= 0]
        if not in1[ns].any():
            in1[k] = True
    return in1, nb


def element_E(P: Problem):
    """Diagonal E_K of eq. prope, as [ne, d1*d] (Section 3.2, items 6 and 7).

    mu > 0: E_K = 0.  mu = 0: K in M1 gets E_K = -lambda_K Id
    with lambda_K = c ||A_K||_inf (interior rows; c = P.lam_scale > 1, 2 by
    default), which exceeds the modulus of every eigenvalue of A_K; K in M2 gets +lambda_L on each face shared with an
    M1 element L and 0 elsewhere, so that E_K + E_L = 0 on every face.  (A
    per-element lambda is a reading: the paper names one lambda larger than the
    eigenvalues of A_K.)
    """
    m = P.mesh
    d = P.d
    E = np.zeros((m.ne, (m.d + 1) * d))
    if P.mu > 0.0:
        return E
    in1, nb = mis_partition(m)
    mask = P.dof_mask()
    lam = np.zeros(m.ne)
    for k in np.nonzero(in1)[0]:
        idx = np.nonzero(mask[k])[0]
        lam[k] = P.lam_scale * np.abs(P.A[k][np.ix_(idx, idx)]).sum(axis=1).max()
        E[k, idx] = -lam[k]
    for k in np.nonzero(~in1)[0]:
        for j in range(m.d + 1):
            L = nb[k, j]
            if L >= 0 and in1[L]:
                E[k, j * d:(j + 1) * d] = lam[L]
    return E


@dataclass
class Hybrid:
    G: sps.csr_matrix
    S: np.ndarray
    Ainv: list
    l: list
    r: list
    B: np.ndarray
    C: list
    Rl: list
    Dl: list
    gidx: list


def eliminate(P: Problem, E=None, signs=None):
    """Element-wise elimination of (U^, P) from eq. syslinhyb (Section 3.2 items 4-5).

    For every element: A^_K = A_K + E_K, its inverse (numpy.linalg.inv, no
    structure used), B_K = D_K^t A^_K^{-1} D_K, and
        G_K = C_K (A^_K^{-1} - A^_K^{-1} D_K D_K^t A^_K^{-1} / B_K) C_K   (K != K0)
        G_K0 = C_K0 A^_K0^{-1} C_K0
        s_K  = C_K (A^_K^{-1} R_K - A^_K^{-1} D_K (D_K^t A^_K^{-1} R_K - e_K) / B_K)
    with the non-symmetric reading A^{-1} D D^t A^{-1} = l r^t, l = A^{-1} D,
    r = A^{-t} D, which is what the elimination computes.  G = sum H_K G_K H_K^t
    and S = sum H_K s_K.
    """
    m = P.mesh
    d = P.d
    if E is None:
        E = element_E(P)
    if signs is None:
        signs = m.sign
    n = m.nf * d
    ek = P.ediv()
    rows, cols, vals = [], [], []
    S = np.zeros(n)
    out = Hybrid(G=None, S=None, Ainv=[], l=[], r=[], B=np.zeros(m.ne), C=[], Rl=[], Dl=[], gidx=[])
    for k in range(m.ne):
        Ak, Dk, Rk, gk, idx = restrict(P, k)
        if len(idx) == 0:
            raise MeshError("element without interior face")
        Ek = np.diag(E[k][idx])
        Ck = np.diag(np.repeat(signs[k], d)[idx])
        Ainv = np.linalg.inv(Ak + Ek)
        l = Ainv @ Dk
        r = Ainv.T @ Dk
        B = Dk @ l
        if k != P.k0:
            Gk = Ck @ (Ainv - np.outer(l, r) / B) @ Ck
            sk = Ck @ (Ainv @ Rk - l * (r @ Rk - ek[k]) / B)
        else:
            Gk = Ck @ Ainv @ Ck
            sk = Ck @ Ainv @ Rk
        rows.append(np.repeat(gk, len(gk)))
        cols.append(np.tile(gk, len(gk)))
        vals.append(Gk.ravel())
        np.add.at(S, gk, sk)
        out.Ainv.append(Ainv)
        out.l.append(l)
        out.r.append(r)
        out.B[k] = B
        out.C.append(Ck)
        out.Rl.append(Rk)
        out.Dl.append(Dk)
        out.gidx.append(gk)
    out.G = sps.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    out.S = S
    return out


def recover(P: Problem, H: Hybrid, W):
    """Recovery of P and U^ from W (Section 3.2, items 2 and 4).

    P_K = (r_K^t (R_K - C_K W_K) - e_K) / B_K for K != K0 (the divergence row
    D_K^t U^_K = e_K solved for P_K; e_K = 0 without boundary data), P_K0 = 0, and
    U^_K = A^_K^{-1} (R_K - D_K P_K - C_K W_K), W_K = H_K^t W.
    Returns (U [nf, d] taken from the copy of the element with C = +1,
    P [ne], Uhat list of local copies).
    """
    m = P.mesh
    d = P.d
    W = np.asarray(W).ravel()
    U = np.zeros(m.nf * d)
    Pk = np.zeros(m.ne)
    ek = P.ediv()
    Uhat = []
    for k in range(m.ne):
        Wk = W[H.gidx[k]]
        rhs = H.Rl[k] - H.C[k] @ Wk
        if k != P.k0:
            Pk[k] = (H.r[k] @ rhs - ek[k]) / H.B[k]
        uk = H.Ainv[k] @ (rhs - H.Dl[k] * Pk[k])
        Uhat.append(uk)
        own = np.diag(H.C[k]) > 0
        U[H.gidx[k][own]] = uk[own]
    return U.reshape(-1, d), Pk, Uhat


def solve_hybrid(P: Problem, E=None, signs=None, direct=True):
    """The hybrid method of Section 3.2: eliminate, solve G W = S directly, recover."""
    H = eliminate(P, E, signs)
    if direct:
        W = spla.splu(H.G.tocsc(), permc_spec="COLAMD").solve(H.S)
    else:
        raise ValueError("use oracle.krylov for iterative solves")
    U, Pk, Uhat = recover(P, H, W)
    return U, Pk, W, H, Uhat


def jump(P: Problem, H: Hybrid, Uhat):
    """C^ U^ = sum_K H_K C_K U^_K: the mismatch between the two copies of a face value."""
    n = P.mesh.nf * P.d
    J = np.zeros(n)
    for k in range(P.mesh.ne):
        np.add.at(J, H.gidx[k], H.C[k] @ Uhat[k])
    return J


def divergence(P: Problem, U):
    """D_K^t H_K^t U for every element (including K0), [ne]."""
    Ul = local_face_values(P.mesh, U).reshape(P.mesh.ne, -1)
    return (P.D * Ul).sum(axis=1)


def coupled_residual(P: Problem, U, Pk):
    """Relative residuals of eq. syslin: (||R - A U - D^t P|| / ||R||, max_K |D_K U - e_K| / max|D_K|)."""
    A, D, R, prow = assemble_coupled(P)
    Pv = Pk[prow >= 0][np.argsort(prow[prow >= 0])]
    u = np.asarray(U).ravel()
    r1 = R - A @ u - D.T @ Pv
    div = divergence(P, U) - P.ediv()
    scale = np.abs(P.D).max() * np.abs(u).max() if np.abs(u).max() > 0 else 1.0
    return np.linalg.norm(r1) / np.linalg.norm(R), np.abs(div).max() / scale

"""Pins of the CPU oracle against what the paper and mathematics fix (CPU only).

Each test names the passage of the paper (Chenier & Eymard, arXiv 2101.03777)
or the mathematical fact it checks.  None of them re-types an oracle formula:
they compare the oracle with an independent computation (quadrature of the
basis functions, direct geometry, brute force on tiny meshes, finite
differences, closed-form exact solutions) or with a property the paper proves.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import synth
import synth.workloads as wl
from oracle import brute, cr, krylov, norms

RNG = np.random.default_rng(1234)


def small2d(n=6, jitter=0.2, mu=50.0, nu=1.0, seed=3):
    coords, elems = synth.square_mesh(n, jitter=jitter, seed=seed)
    fbar = np.random.default_rng(seed).normal(size=(len(elems), 2))
    return cr.make_problem(coords, elems, mu, nu, fbar)


def small3d(n=2, mu=30.0, nu=1.0, seed=5):
    coords, elems = synth.cube_mesh(n)
    fbar = np.random.default_rng(seed).normal(size=(len(elems), 3))
    return cr.make_problem(coords, elems, mu, nu, fbar)


# --------------------------------------------------------------------------
# Quadrature used by the pins themselves
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim,n", [(2, 3), (2, 5), (3, 3), (3, 4)])
def test_simplex_rule_monomials(dim, n):
    """Mean of x^a y^b (z^c) over the unit simplex is a! b! c! d! / (a+b+c+d)!."""
    lam, wt = synth.simplex_rule(dim, n)
    pts = lam[:, 1:]
    deg = 2 * n - dim
    for exps in np.ndindex(*([deg + 1] * dim)):
        if sum(exps) > deg:
            continue
        val = (wt * np.prod(pts ** np.array(exps), axis=1)).sum()
        exact = math.factorial(dim) * np.prod([math.factorial(e) for e in exps]) / math.factorial(sum(exps) + dim)
        assert abs(val - exact) < 1e-14


# --------------------------------------------------------------------------
# Mesh and geometry (Section 2 item 1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("P", [small2d(), small3d()], ids=["2d", "3d"])
def test_geometry(P):
    m = P.mesh
    # closed surface: sum of outward face vectors vanishes
    assert np.abs(m.a.sum(axis=1)).max() < 1e-14
    # outward
    assert (((m.xs - m.xK[:, None, :]) * m.a).sum(axis=2) > 0).all()
    # |a| equals the face measure computed from the vertices
    X = m.coords[m.elems]
    for j in range(m.d + 1):
        fv = X[:, [q for q in range(m.d + 1) if q != j]]
        if m.d == 2:
            meas = np.linalg.norm(fv[:, 1] - fv[:, 0], axis=1)
        else:
            meas = 0.5 * np.linalg.norm(np.cross(fv[:, 1] - fv[:, 0], fv[:, 2] - fv[:, 0]), axis=1)
        assert np.allclose(m.area[:, j], meas, rtol=1e-14, atol=0)
    # elements tile the unit domain
    assert abs(m.vol.sum() - 1.0) < 1e-13
    # every interior face has two distinct owners and appears in both element lists
    fe = m.face_elems
    assert (fe[:, 0] < fe[:, 1]).all()
    for s in range(2):
        k = fe[:, s]
        assert ((m.elem_face[k] == np.arange(m.nf)[:, None]).sum(axis=1) == 1).all()


def test_faces_match_generator_order():
    coords, elems = synth.square_mesh(5, jitter=0.1, seed=2)
    m = cr.build_mesh(coords, elems)
    assert (m.faces == wl.interior_face_list(elems)).all()


def test_interior_face_counts_structured():
    """#F_int = 3N^2 - 2N in 2D (N x N cells x2) and 2D sizing of the hybridised system."""
    for n in (2, 5, 16):
        m = cr.build_mesh(*synth.square_mesh(n))
        assert m.nf == 3 * n * n - 2 * n


def test_mesh_errors():
    coords, elems = synth.square_mesh(2)
    bad = np.concatenate([elems, elems[:1]])     # a face now belongs to 3 elements
    with pytest.raises(cr.MeshError):
        cr.build_mesh(coords, bad)
    flat = coords.copy()
    flat[:, 1] = 0.0
    with pytest.raises(cr.MeshError):
        cr.build_mesh(flat, elems)


# --------------------------------------------------------------------------
# CR basis and element matrices (Section 2 items 1-3, Section 3.1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("P", [small2d(), small3d()], ids=["2d", "3d"])
def test_cr_basis_face_means(P):
    """phi_sigma has mean 1 on sigma and 0 on the other faces (checked by face quadrature)."""
    m = P.mesh
    c, grad = cr.cr_basis(m)
    X = m.coords[m.elems]
    lamf, wtf = synth.simplex_rule(m.d - 1, 3) if m.d == 3 else (None, None)
    for j in range(m.d + 1):
        fv = X[:, [q for q in range(m.d + 1) if q != j]]
        if m.d == 2:
            t, w = np.polynomial.legendre.leggauss(3)
            t = 0.5 * (t + 1)
            w = 0.5 * w
            pts = fv[:, None, 0] + t[None, :, None] * (fv[:, None, 1] - fv[:, None, 0])
        else:
            pts = np.einsum("qj,ejd->eqd", lamf, fv)
            w = wtf
        phi = c[:, None, :] + np.einsum("eqd,esd->eqs", pts - m.xK[:, None, :], grad)
        mean = np.einsum("q,eqs->es", w, phi)
        target = np.zeros(m.d + 1)
        target[j] = 1.0
        assert np.abs(mean - target).max() < 1e-12


@pytest.mark.parametrize("P", [small2d(), small3d()], ids=["2d", "3d"])
def test_basis_gradient_is_face_vector(P):
    """grad phi_sigma = a_{K,sigma} / |K| (divergence theorem on the affine basis)."""
    m = P.mesh
    _, grad = cr.cr_basis(m)
    assert np.abs(grad - m.a / m.vol[:, None, None]).max() < 1e-9 * np.abs(grad).max()


def test_mass_2d_diagonal():
    """Section 2 item 3: in 2D the CR mass matrix is already diagonal (|K|/3 on the diagonal)."""
    P = small2d()
    m = P.mesh
    hi = cr.mass_matrix(m, quad_rule=synth.simplex_rule(2, 4))
    lo = cr.mass_matrix(m)
    assert np.abs(hi - lo).max() < 1e-15
    off = hi - np.einsum("ess->es", hi)[:, :, None] * np.eye(3)
    assert np.abs(off).max() < 1e-15
    assert np.abs(np.einsum("ess->es", hi) - m.vol[:, None] / 3).max() < 1e-15


def test_mass_3d_cones():
    """Section 2 item 3: the cones D_{K,sigma} partition K; each has volume |K|/4."""
    m = small3d().mesh
    Mm = cr.mass_matrix(m)
    diag = np.einsum("ess->es", Mm)
    assert np.abs(diag.sum(axis=1) - m.vol).max() < 1e-15
    assert np.abs(diag - m.vol[:, None] / 4).max() < 1e-15


@pytest.mark.parametrize("P", [small2d(), small3d()], ids=["2d", "3d"])
def test_stiffness_partition_of_unity(P):
    """The basis functions of K sum to 1, so every stiffness row sums to 0; the matrix is PSD."""
    K = cr.stiffness_matrix(P.mesh)
    assert np.abs(K.sum(axis=2)).max() < 1e-13 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    assert ev.min() > -1e-12 * ev.max()


# --------------------------------------------------------------------------
# Exact solutions and the coupled system (Section 3.1, Section 4.1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim", [2, 3])
def test_constant_force_exact(dim):
    """Section 4.1 first paragraph: constant force gives U = 0 and P_K = c.(x_K - x_K0) exactly."""
    if dim == 2:
        coords, elems = synth.square_mesh(7, jitter=0.2, seed=9)
        c = np.array([0.7, -1.3])
    else:
        coords, elems = synth.cube_mesh(2)
        c = np.array([0.4, -0.9, 1.7])
    fbar = np.tile(c, (len(elems), 1))
    for mu in (0.0, 25.0):
        P = cr.make_problem(coords, elems, mu, 1.0, fbar, k0=3)
        exact = (P.mesh.xK - P.mesh.xK[3]) @ c
        U, Pk = cr.solve_coupled(P)
        assert np.abs(U).max() < 1e-12
        assert np.abs(Pk - exact).max() < 1e-12
        Uh, Ph, *_ = cr.solve_hybrid(P)
        assert np.abs(Uh).max() < 1e-11
        assert np.abs(Ph - exact).max() < 1e-11


def test_steady_state_is_fixed_point_of_transient_step():
    """Reading of 'f includes a term from the velocity at the start of the step' (Section 2):
    if U^{n-1} is the steady solution, the transient step returns it unchanged."""
    coords, elems = synth.square_mesh(6, jitter=0.15, seed=4)
    fbar = np.random.default_rng(4).normal(size=(len(elems), 2))
    Ps = cr.make_problem(coords, elems, 0.0, 1.0, fbar)
    Us, Pss = cr.solve_coupled(Ps)
    Pt = cr.make_problem(coords, elems, 80.0, 1.0, fbar, u_prev=Us)
    Ut, Pt_ = cr.solve_coupled(Pt)
    assert np.abs(Ut - Us).max() < 1e-12 * np.abs(Us).max()
    assert np.abs(Pt_ - Pss).max() < 1e-11 * np.abs(Pss).max()


def _orders(errs):
    return [{k: math.log2(a[k] / b[k]) for k in a} for a, b in zip(errs[:-1], errs[1:])]


def _paper_orders():
    vals = {}
    with open(__file__.replace("test_oracle.py", "golden/paper_orders.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def test_manufactured_orders_2d():
    """Section 4.1, Table tab0: velocity L2 order -> 2, pressure order > 1; broken H1 order 1."""
    quad = synth.simplex_rule(2, 5)
    errs = []
    for n in (8, 16, 32, 64):
        w = wl.square(n, mu=100.0, nu=1.0)
        P = cr.make_problem(w["coords"], w["elems"], w["mu"], w["nu"], w["fbar"])
        U, Pk = cr.solve_coupled(P)
        man = w["manufactured"]
        errs.append(norms.errors(P.mesh, U, Pk, man.u, man.grad_u, man.p, quad))
    o = _orders(errs)
    paper = _paper_orders()
    assert o[-1]["l2u"] > min(paper["tab0_velocity_l2_ratio_fine1"], paper["tab0_velocity_l2_ratio_fine2"]) - 0.1
    assert 0.9 < o[-1]["h1u"] < 1.2
    assert o[-1]["l2p"] > 1.0 and o[-2]["l2p"] > 1.0
    assert all(e1["l2u"] > e2["l2u"] for e1, e2 in zip(errs[:-1], errs[1:]))


def test_manufactured_orders_3d():
    """Section 4.1, 3D Stokes table: velocity L2 order -> 2, broken H1 -> 1, pressure > 1.

    64^3-scale meshes are out of reach of a CPU test; on n = 4, 8, 12, 16 cubes x 6
    tetrahedra the observed orders (log of the error ratio over log of the h ratio)
    rise with every refinement, and the finest pair is within 0.3 of the velocity
    ratio the paper prints and above its pressure ratio.  The oracle's hybrid path
    with its own CG solves the systems (equal to the coupled solve by the
    hybrid = coupled pins; a direct solve at n = 16 takes minutes)."""
    quad = synth.simplex_rule(3, 4)
    ns = (4, 8, 12, 16)
    errs = []
    for n in ns:
        w = wl.cube(n, mu=100.0)
        P = cr.make_problem(w["coords"], w["elems"], w["mu"], w["nu"], w["fbar"])
        H = cr.eliminate(P)
        W, it, hist = krylov.pcg(H.G, H.S, tol=1e-12)
        assert hist[-1] <= 1e-12
        U, Pk, _ = cr.recover(P, H, W)
        man = w["manufactured"]
        errs.append(norms.errors(P.mesh, U, Pk, man.u, man.grad_u, man.p, quad))
    o = [{k: math.log(a[k] / b[k]) / math.log(n2 / n1) for k in a}
         for (n1, a), (n2, b) in zip(zip(ns[:-1], errs[:-1]), zip(ns[1:], errs[1:]))]
    paper = _paper_orders()
    for key in ("l2u", "h1u", "l2p"):
        assert all(a[key] < b[key] for a, b in zip(o[:-1], o[1:])), (key, o)
    assert o[-1]["l2u"] > paper["tab3dstokes_velocity_l2_ratio_fine"] - 0.3
    assert o[-1]["h1u"] > 0.8
    assert o[-1]["l2p"] > paper["tab3dstokes_pressure_ratio_fine"]


def test_error_norms_of_zero_discrete_solution():
    """norms.errors with U = 0, P = 0 against closed-form integrals on the unit square and
    cube: u = x (componentwise), grad u = I, p = x give ||u||^2 = d/3, ||grad u||^2 = d,
    ||p - mean p||^2 = 1/12."""
    for dim in (2, 3):
        if dim == 2:
            coords, elems = synth.square_mesh(5, jitter=0.2, seed=2)
        else:
            coords, elems = synth.cube_mesh(3)
        m = cr.build_mesh(coords, elems)
        e = norms.errors(m, np.zeros((m.nf, dim)), np.zeros(m.ne),
                         lambda x: x.copy(),
                         lambda x: np.broadcast_to(np.eye(dim), (len(x), dim, dim)),
                         lambda x: x[:, 0], synth.simplex_rule(dim, 3))
        assert abs(e["l2u"] ** 2 - dim / 3.0) < 1e-13
        assert abs(e["h1u"] ** 2 - dim) < 1e-13
        assert abs(e["l2p"] ** 2 - 1.0 / 12.0) < 1e-13


def test_error_norms_of_discrete_field_closed_form():
    """norms.errors with the exact solution zero against closed forms of the discrete field.

    CR basis phi_s = 1 - d lambda_s (face s opposite vertex s) and the simplex integrals
    int lambda_i = |K|/(d+1), int lambda_i lambda_j = |K| (1 + delta_ij) / ((d+1)(d+2)) give
    int phi_s phi_t = |K| (1 - 2d/(d+1) + d^2 (1 + delta_st) / ((d+1)(d+2))), i.e. |K|/3
    on the diagonal and 0 off it in 2D, 2|K|/5 and -|K|/20 in 3D; grad phi_s = a_s / |K|.
    The pressure error is that of P minus its |K|-weighted mean."""
    for dim in (2, 3):
        if dim == 2:
            coords, elems = synth.square_mesh(4, jitter=0.2, seed=6)
        else:
            coords, elems = synth.cube_mesh(2)
        m = cr.build_mesh(coords, elems)
        rng = np.random.default_rng(40 + dim)
        U = rng.normal(size=(m.nf, dim))
        Pk = rng.normal(size=m.ne)
        Ul = cr.local_face_values(m, U)                     # [ne, d1, d], zero on exterior faces
        d1 = dim + 1
        Mref = np.array([[1 - 2 * dim / d1 + dim * dim * (1 + (s == t)) / (d1 * (d1 + 1))
                          for t in range(d1)] for s in range(d1)])
        l2 = sum(m.vol[k] * np.einsum("si,st,ti->", Ul[k], Mref, Ul[k]) for k in range(m.ne))
        h1 = sum(np.sum(np.einsum("si,sj->ij", Ul[k], m.a[k]) ** 2) / m.vol[k] for k in range(m.ne))
        pm = (m.vol * Pk).sum() / m.vol.sum()
        l2p = (m.vol * (Pk - pm) ** 2).sum()
        zero = lambda x: np.zeros((len(x), dim))
        e = norms.errors(m, U, Pk, zero, lambda x: np.zeros((len(x), dim, dim)), lambda x: np.zeros(len(x)),
                         synth.simplex_rule(dim, 3))
        assert abs(e["l2u"] ** 2 - l2) < 1e-12 * l2
        assert abs(e["h1u"] ** 2 - h1) < 1e-12 * h1
        assert abs(e["l2p"] ** 2 - l2p) < 1e-12 * l2p


# --------------------------------------------------------------------------
# Hybridisation (Section 3.2)
# --------------------------------------------------------------------------

def _cases():
    coords, elems = synth.square_mesh(8, jitter=0.2, seed=11)
    f2 = np.random.default_rng(11).normal(size=(len(elems), 2))
    c3, e3 = synth.cube_mesh(2)
    f3 = np.random.default_rng(12).normal(size=(len(e3), 3))
    ns = wl.ns_square(8, nu=0.02, seed=3)
    ns3 = wl.ns_cube(2, nu=0.05, seed=4)
    return {
        "stokes2d": cr.make_problem(coords, elems, 200.0, 1.0, f2, k0=5),
        "stokes3d": cr.make_problem(c3, e3, 40.0, 1.0, f3),
        "steady2d": cr.make_problem(coords, elems, 0.0, 1.0, f2),
        "ns2d": cr.make_problem(ns["coords"], ns["elems"], 0.0, ns["nu"], ns["fbar"], ulin=ns["ulin"]),
        "ns2d_transient": cr.make_problem(ns["coords"], ns["elems"], 30.0, ns["nu"], ns["fbar"], ulin=ns["ulin"]),
        "ns3d": cr.make_problem(ns3["coords"], ns3["elems"], 0.0, ns3["nu"], ns3["fbar"], ulin=5.0 * ns3["ulin"]),
        "ns3d_transient": cr.make_problem(ns3["coords"], ns3["elems"], 20.0, ns3["nu"], ns3["fbar"],
                                          ulin=5.0 * ns3["ulin"]),
    }


CASES = _cases()


@pytest.mark.parametrize("name", list(CASES))
def test_hybrid_equals_coupled(name):
    """Section 3.2 item 2: the hybrid system's (U, P) is the coupled solution (P^ = P)."""
    P = CASES[name]
    U, Pk = cr.solve_coupled(P)
    Uh, Ph, W, H, Uhat = cr.solve_hybrid(P)
    assert np.abs(Uh - U).max() <= 1e-10 * np.abs(U).max()
    assert np.abs(Ph - Pk).max() <= 1e-10 * np.abs(Pk).max()
    # incompressibility on every element, K0 included (global flux balance)
    div = cr.divergence(P, Uh)
    assert np.abs(div).max() < 1e-11 * np.abs(P.D).max() * np.abs(Uh).max()
    assert Ph[P.k0] == 0.0
    # copies agree: C^ U^ = 0 up to the solve's rounding
    assert np.abs(cr.jump(P, H, Uhat)).max() < 1e-10 * np.abs(U).max()


@pytest.mark.parametrize("name", list(CASES))
def test_residual_is_copy_mismatch(name):
    """For any W, S - G W equals C^ U^ with U^, P recovered from W (substituting the recovery
    relations of Section 3.2 item 4 into the C^ row of eq. syslinhyb)."""
    P = CASES[name]
    H = cr.eliminate(P)
    W = np.random.default_rng(7).normal(size=H.S.shape)
    _, _, Uhat = cr.recover(P, H, W)
    lhs = H.S - H.G @ W
    rhs = cr.jump(P, H, Uhat)
    assert np.abs(lhs - rhs).max() < 1e-10 * np.abs(lhs).max()


def test_spd_transient_stokes():
    """Section 3.2 item 6: mu > 0, b_h = 0 -> G symmetric positive definite (Cholesky succeeds)."""
    for name in ("stokes2d", "stokes3d"):
        H = cr.eliminate(CASES[name])
        G = H.G.toarray()
        assert np.abs(G - G.T).max() < 1e-13 * np.abs(G).max()
        scipy.linalg.cholesky(G)


def test_steady_stokes_symmetric_indefinite():
    """Abstract / Section 3.2 item 7: steady Stokes gives a symmetric invertible, indefinite G."""
    H = cr.eliminate(CASES["steady2d"])
    G = H.G.toarray()
    assert np.abs(G - G.T).max() < 1e-13 * np.abs(G).max()
    ev = np.linalg.eigvalsh(G)
    assert ev.min() < 0 < ev.max()
    assert np.abs(ev).min() > 1e-10 * np.abs(ev).max()


def test_navier_stokes_nonsymmetric():
    H = cr.eliminate(CASES["ns2d"])
    G = H.G.toarray()
    assert np.abs(G - G.T).max() > 1e-3 * np.abs(G).max()


def test_local_schur_positive_kronecker():
    """Section 3.2 item 4: B_K > 0; for Stokes A^_K = S_K (x) I_d, so
    B_K = sum_i a^(i)t S_K^{-1} a^(i) over the interior faces."""
    P = CASES["stokes2d"]
    H = cr.eliminate(P)
    m = P.mesh
    S = cr.element_S(m, P.mu, P.nu)
    assert (H.B > 0).all()
    for k in range(0, m.ne, 7):
        idx = np.nonzero(m.elem_face[k] >= 0)[0]
        Sk = S[k][np.ix_(idx, idx)]
        ak = m.a[k][idx]
        Bk = sum(ak[:, i] @ np.linalg.solve(Sk, ak[:, i]) for i in range(m.d))
        assert abs(Bk - H.B[k]) < 1e-12 * Bk


@pytest.mark.parametrize("n,blocks", [(2, 28), (16, 3556)])
def test_stencil_of_G(n, blocks):
    """Section 3.2 item 5: G has the block stencil of A: one dxd block per pair of interior
    faces sharing an element, plus the diagonal: #blocks = #F_int + sum_K s_K (s_K - 1)."""
    coords, elems = synth.square_mesh(n)
    fbar = RNG.normal(size=(len(elems), 2))
    P = cr.make_problem(coords, elems, 10.0, 1.0, fbar)
    H = cr.eliminate(P)
    G = H.G.tocsr()
    G.sum_duplicates()
    sK = (P.mesh.elem_face >= 0).sum(axis=1)
    assert P.mesh.nf + (sK * (sK - 1)).sum() == blocks
    assert G.nnz == blocks * 4          # structural entries
    A, D, R, _ = cr.assemble_coupled(P)
    A.sum_duplicates()
    # A is block diagonal per component; its face-pair pattern is the block stencil of G
    rA, cA = A.tocoo().row, A.tocoo().col
    rG, cG = G.tocoo().row, G.tocoo().col
    bA = set(zip(rA // 2, cA // 2))
    bG = set(zip(rG // 2, cG // 2))
    assert bA == bG and len(bG) == blocks


def test_brute_force_three_field():
    """Section 3.2 eq. syslinhyb on a 2x2-cell mesh: sizes 32 + 7 + 16 = 55, copies equal
    (eq. ukl), (U, P^) equals the coupled solution, W^ equals the eliminated solve, J C^t = 0."""
    coords, elems = synth.square_mesh(2, jitter=0.0)
    fbar = RNG.normal(size=(8, 2))
    for mu, ulin in ((10.0, None), (0.0, None)):
        P = cr.make_problem(coords, elems, mu, 1.0, fbar, ulin=ulin)
        B = brute.three_field(P)
        assert B["size"] == (32, 7, 16)
        assert np.abs(B["Chat"] @ B["Uhat"]).max() < 1e-13
        U, Pk = cr.solve_coupled(P)
        assert np.abs(B["U"] - U).max() < 1e-12 * np.abs(U).max()
        assert np.abs(B["P"] - Pk).max() < 1e-12 * np.abs(Pk).max()
        _, _, W, _, _ = cr.solve_hybrid(P)
        assert np.abs(B["W"] - W).max() < 1e-11 * np.abs(W).max()
        assert np.abs(B["J"] @ B["Chat"].T).max() == 0.0


def test_brute_force_navier_stokes():
    ns = wl.ns_square(2, nu=0.05, seed=1)
    P = cr.make_problem(ns["coords"], ns["elems"], 0.0, ns["nu"], ns["fbar"], ulin=ns["ulin"])
    B = brute.three_field(P)
    U, Pk = cr.solve_coupled(P)
    assert np.abs(B["U"] - U).max() < 1e-11 * np.abs(U).max()
    _, _, W, _, _ = cr.solve_hybrid(P)
    assert np.abs(B["W"] - W).max() < 1e-10 * np.abs(W).max()


def test_gauge_invariances():
    """Flipping C on faces negates W there; changing K0 shifts P by a constant; changing
    E (steady case) changes G and W but not (U, P) (Section 1 and Section 3.2 item 7)."""
    P = CASES["stokes2d"]
    U, Pk, W, H, _ = cr.solve_hybrid(P)
    flip = RNG.random(P.mesh.nf) < 0.5
    sg = P.mesh.sign.copy()
    for j in range(P.d + 1):
        f = P.mesh.elem_face[:, j]
        ok = f >= 0
        sg[ok, j] *= np.where(flip[f[ok]], -1.0, 1.0)
    U2, P2, W2, _, _ = cr.solve_hybrid(P, signs=sg)
    assert np.abs(U2 - U).max() < 1e-11 * np.abs(U).max()
    assert np.abs(P2 - Pk).max() < 1e-11 * np.abs(Pk).max()
    fl = np.repeat(np.where(flip, -1.0, 1.0), P.d)
    assert np.abs(W2 - fl * W).max() < 1e-10 * np.abs(W).max()
    # K0
    P_k = cr.make_problem(P.mesh.coords, P.mesh.elems, P.mu, P.nu, np.zeros((P.mesh.ne, 2)), k0=0)
    P_k.R = P.R.copy()
    U3, P3, *_ = cr.solve_hybrid(P_k)
    assert np.abs(U3 - U).max() < 1e-11 * np.abs(U).max()
    shift = P3 - Pk
    assert np.abs(shift - shift.mean()).max() < 1e-11 * np.abs(Pk).max()
    # E in the steady case
    Ps = CASES["steady2d"]
    E = cr.element_E(Ps)
    U4, P4, W4, _, _ = cr.solve_hybrid(Ps, E=E)
    U5, P5, W5, _, _ = cr.solve_hybrid(Ps, E=3.0 * E)
    assert np.abs(U5 - U4).max() < 1e-10 * np.abs(U4).max()
    assert np.abs(P5 - P4).max() < 1e-10 * np.abs(P4).max()
    assert np.abs(W5 - W4).max() > 1e-3 * np.abs(W4).max()


def test_E_satisfies_prope():
    """eq. prope: (E_K)_sigma + (E_L)_sigma = 0 on every interior face; M1 independent, M2 = its neighbours."""
    P = CASES["ns2d"]
    m = P.mesh
    E = cr.element_E(P)
    tot = np.zeros((m.nf, P.d))
    for j in range(m.d + 1):
        f = m.elem_face[:, j]
        ok = f >= 0
        np.add.at(tot, f[ok], E[ok, j * P.d:(j + 1) * P.d])
    assert np.abs(tot).max() == 0.0
    in1, nb = cr.mis_partition(m)
    for k in range(m.ne):
        ns = nb[k][nb[k] >= 0]
        if in1[k]:
            assert not in1[ns].any()
        else:
            assert in1[ns].any()
    # lower triangles form M1 on the single-diagonal structured mesh
    assert in1[0::2].all() and not in1[1::2].any()


# --------------------------------------------------------------------------
# Convection form (Section 2 item 6)
# --------------------------------------------------------------------------

def _geometric_flux(m, Ul, s, t):
    """F_{s,t}(u) = integral over tau_{s,t} of u_K . n_{s,t}, from the co-volume geometry
    (2D: tau is the segment from x_K to the vertex shared by faces s and t; 3D: the
    triangle from x_K to their shared edge), n oriented from the cone D_{K,s} to D_{K,t}.
    u_K is affine (CR basis from its face-mean conditions), so the integral is its value
    at the centroid of tau times the measure of tau."""
    d1 = m.d + 1
    c, grad = cr.cr_basis(m)
    X = m.coords[m.elems]
    xK = m.xK
    V = X[:, [q for q in range(d1) if q not in (s, t)]]
    if m.d == 2:
        v = V[:, 0]
        e = v - xK
        n = np.stack([e[:, 1], -e[:, 0]], axis=1)      # |tau| * unit normal
        cen = 0.5 * (xK + v)
    else:
        n = 0.5 * np.cross(V[:, 0] - xK, V[:, 1] - xK)
        cen = (xK + V[:, 0] + V[:, 1]) / 3.0
    # cone centroids to orient from D_s to D_t
    cs = (xK + X[:, [q for q in range(d1) if q != s]].sum(axis=1)) / d1
    ct = (xK + X[:, [q for q in range(d1) if q != t]].sum(axis=1)) / d1
    n = n * np.sign(((ct - cs) * n).sum(axis=1))[:, None]
    phi = c + np.einsum("ed,esd->es", cen - xK, grad)
    uc = np.einsum("es,esi->ei", phi, Ul)
    return (uc * n).sum(axis=1)


def test_flux_closed_form_vs_geometry():
    """F_{s,s'} computed from the co-volume geometry directly equals the closed form of
    Section 2 item 6."""
    for P in (small2d(4), small3d(1)):
        m = P.mesh
        d1 = m.d + 1
        U = RNG.normal(size=(m.nf, m.d))
        Ul = cr.local_face_values(m, U)
        F = cr.fluxes(m, Ul)
        for s in range(d1):
            for t in range(d1):
                if s == t:
                    continue
                Fg = _geometric_flux(m, Ul, s, t)
                assert np.abs(Fg - F[:, s, t]).max() < 1e-12 * max(1.0, np.abs(F).max())


def test_convection_pair_form():
    """eq. defbh, first form: b_h(w; u, v) = sum_K sum over unordered face pairs {s, t} of
    F_{s,t}(w) (U_t - U_s) . (V_s + V_t) / 2, with F from the co-volume geometry, equals
    sum_K convection(w, u) . V (the oracle's per-face coefficient, the second form).
    w, u, v are random and not divergence-free, so the factor 1/2, the sign of the
    difference and the pairing are all tested (b_h(u, u) = 0 would hold at any scale)."""
    for P in (small2d(5), small3d(2)):
        m = P.mesh
        d1 = m.d + 1
        Wl, Ul, Vl = (cr.local_face_values(m, RNG.normal(size=(m.nf, m.d))) for _ in range(3))
        pair = np.zeros(m.ne)
        for s in range(d1):
            for t in range(s + 1, d1):
                F = _geometric_flux(m, Wl, s, t)
                pair += F * ((Ul[:, t] - Ul[:, s]) * (Vl[:, s] + Vl[:, t])).sum(axis=1) / 2.0
        N = cr.convection(m, Wl, Ul)
        second = (N * Vl.reshape(m.ne, -1)).sum(axis=1)
        assert np.abs(pair - second).max() < 1e-13 * np.abs(pair).max()
        assert abs(pair.sum()) > 1e-3 * np.abs(pair).sum()  # a generic, non-degenerate case


def test_convection_skew_and_flux_sum():
    """Section 2 item 6: sum_{s'} F_{s,s'}(u) = -U_s . a_s for discretely divergence-free u,
    and then b_h(u, u) = 0."""
    ns = wl.ns_square(6, nu=0.02, seed=4)
    P = cr.make_problem(ns["coords"], ns["elems"], 0.0, ns["nu"], ns["fbar"], ulin=ns["ulin"])
    m = P.mesh
    Ub = cr.local_face_values(m, ns["ulin"])
    assert np.abs(cr.divergence(P, ns["ulin"])).max() < 1e-15
    F = cr.fluxes(m, Ub) * (1 - np.eye(3))
    assert np.abs(F.sum(axis=2) + (Ub * m.a).sum(axis=2)).max() < 1e-15
    N = cr.convection(m, Ub, Ub)
    bh = (N * Ub.reshape(m.ne, -1)).sum()
    assert abs(bh) < 1e-14 * np.abs(N).sum() * np.abs(Ub).max()


def test_convection_skew_and_flux_sum_3d():
    """The same two identities in 3D, for the face means of a divergence-free
    field whose normal parts come from edge circulations (discretely
    divergence-free on every tetrahedron)."""
    ns = wl.ns_cube(3, nu=0.02, seed=5)
    P = cr.make_problem(ns["coords"], ns["elems"], 0.0, ns["nu"], ns["fbar"], ulin=ns["ulin"])
    m = P.mesh
    Ub = cr.local_face_values(m, ns["ulin"])
    assert np.abs(cr.divergence(P, ns["ulin"])).max() < 1e-15 * max(1.0, np.abs(ns["ulin"]).max())
    F = cr.fluxes(m, Ub) * (1 - np.eye(4))
    assert np.abs(F.sum(axis=2) + (Ub * m.a).sum(axis=2)).max() < 1e-15
    N = cr.convection(m, Ub, Ub)
    bh = (N * Ub.reshape(m.ne, -1)).sum()
    assert abs(bh) < 1e-14 * np.abs(N).sum() * np.abs(Ub).max()


def test_convection_jacobian_fd():
    """Newton Jacobian of the element convection vector vs central finite differences."""
    for P in (small2d(4), small3d(1)):
        m = P.mesh
        Ub = RNG.normal(size=(m.ne, m.d + 1, m.d)) * m.interior_mask()[:, :, None]
        J = cr.convection_jacobian(m, Ub)
        dU = RNG.normal(size=Ub.shape)
        eps = 1e-5
        fd = (cr.convection(m, Ub + eps * dU, Ub + eps * dU) - cr.convection(m, Ub - eps * dU, Ub - eps * dU)) / (2 * eps)
        an = np.einsum("eab,eb->ea", J, dU.reshape(m.ne, -1))
        assert np.abs(fd - an).max() < 1e-8 * np.abs(an).max()


def test_oracle_pcg_matches_direct():
    P = CASES["stokes2d"]
    U, Pk, W, H, _ = cr.solve_hybrid(P)
    x, it, hist = krylov.pcg(H.G, H.S, tol=1e-13)
    assert np.abs(x - W).max() < 1e-9 * np.abs(W).max()
    assert hist[-1] <= 1e-13


# --------------------------------------------------------------------------
# Non-homogeneous Dirichlet data (the tests of Section 4 impose the exact
# velocity on the boundary): known exterior-face values move to the right-hand
# side of the velocity rows, and the divergence row of K becomes
# D_K^t U_K = e_K = -D_K[bnd] . g.
# --------------------------------------------------------------------------

def _bnd_mesh(dim):
    if dim == 2:
        return synth.square_mesh(6, jitter=0.2, seed=21)
    return synth.cube_mesh(2)


def _face_pts(coords, faces):
    return coords[np.asarray(faces)].mean(axis=1)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("kind", ["transient", "steady", "ns"])
def test_boundary_constant_velocity_exact(dim, kind):
    """A constant velocity c imposed on the boundary, zero force (and, transient,
    c as the previous step; Newton step about c) gives U = c and P = 0 exactly:
    constants are in the kernel of the stiffness rows, have zero divergence on
    every element, and make the convection differences vanish."""
    coords, elems = _bnd_mesh(dim)
    c = np.arange(1.0, dim + 1.0) * 0.7
    bf = wl.exterior_face_list(elems)
    nf = len(wl.interior_face_list(elems))
    g = np.tile(c, (len(bf), 1))
    mu = {"transient": 50.0, "steady": 0.0, "ns": 0.0}[kind]
    up = np.tile(c, (nf, 1)) if kind == "transient" else None
    ulin = np.tile(c, (nf, 1)) if kind == "ns" else None
    P = cr.make_problem(coords, elems, mu, 0.3, np.zeros((len(elems), dim)), u_prev=up, ulin=ulin, gbnd=g)
    U, Pk = cr.solve_coupled(P)
    assert np.abs(U - c).max() < 1e-11 * np.abs(c).max()
    assert np.abs(Pk).max() < 1e-10
    Uh, Ph, W, H, Uhat = cr.solve_hybrid(P)
    assert np.abs(Uh - c).max() < 1e-11 * np.abs(c).max()
    assert np.abs(Ph).max() < 1e-10


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("mu", [0.0, 40.0])
def test_boundary_affine_velocity_exact(dim, mu):
    """An affine, divergence-free, harmonic velocity (2D: (y, x); 3D: (y, z, x))
    with zero pressure solves the Stokes problem with zero force (transient:
    with itself as the previous step); the CR scheme reproduces it exactly:
    U = its face means, P = 0."""
    coords, elems = _bnd_mesh(dim)
    perm = [1, 0] if dim == 2 else [1, 2, 0]
    u = lambda x: x[:, perm]
    bf = wl.exterior_face_list(elems)
    fi = wl.interior_face_list(elems)
    g = u(_face_pts(coords, bf))
    ue = u(_face_pts(coords, fi))
    P = cr.make_problem(coords, elems, mu, 1.0, np.zeros((len(elems), dim)), u_prev=ue if mu > 0 else None, gbnd=g)
    U, Pk = cr.solve_coupled(P)
    assert np.abs(U - ue).max() < 1e-11
    assert np.abs(Pk).max() < 1e-10
    Uh, Ph, W, H, Uhat = cr.solve_hybrid(P)
    assert np.abs(Uh - ue).max() < 1e-11
    assert np.abs(Ph).max() < 1e-10
    # the velocity including the boundary data is divergence-free on every element
    assert np.abs(cr.divergence(P, Uh) - P.ediv()).max() < 1e-12


@pytest.mark.parametrize("dim,kind", [(2, "stokes"), (3, "stokes"), (2, "steady"), (2, "ns"), (3, "ns")])
def test_boundary_hybrid_equals_coupled(dim, kind):
    """Section 3.2 item 2 with boundary data: the hybrid system's (U, P) is the
    coupled solution; the copies agree; D_K U_K = e_K on every element but K0,
    and on K0 up to the data's net flux."""
    coords, elems = _bnd_mesh(dim)
    rng = np.random.default_rng(5 + dim)
    bf = wl.exterior_face_list(elems)
    nf = len(wl.interior_face_list(elems))
    g = rng.normal(size=(len(bf), dim))
    f = rng.normal(size=(len(elems), dim))
    mu = {"stokes": 30.0, "steady": 0.0, "ns": 0.0}[kind]
    ulin = rng.normal(size=(nf, dim)) if kind == "ns" else None
    P = cr.make_problem(coords, elems, mu, 0.5, f, ulin=ulin, gbnd=g)
    U, Pk = cr.solve_coupled(P)
    Uh, Ph, W, H, Uhat = cr.solve_hybrid(P)
    assert np.abs(Uh - U).max() <= 1e-10 * np.abs(U).max()
    assert np.abs(Ph - Pk).max() <= 1e-10 * np.abs(Pk).max()
    assert np.abs(cr.jump(P, H, Uhat)).max() < 1e-10 * np.abs(U).max()
    div = cr.divergence(P, Uh) - P.ediv()
    scale = np.abs(P.D).max() * max(np.abs(Uh).max(), np.abs(g).max())
    others = np.arange(P.mesh.ne) != P.k0
    assert np.abs(div[others]).max() < 1e-11 * scale
    # K0's divergence row is not imposed: it takes up the net flux of the (random)
    # data, sum_K e_K, since sum_K D_K^t U_K = 0 (the two a's of a face cancel)
    assert abs(div[P.k0] + P.ediv().sum()) < 1e-10 * scale


def test_green_taylor_stokes_orders_with_boundary_data():
    """Orders with non-homogeneous data: the Green-Taylor vortex as a Stokes
    solution (force mu u - nu Lap u + grad p), its face means imposed on the
    boundary; velocity L2 order -> 2, broken H1 -> 1, pressure > 1
    (Section 4.1, Table tab0 prints ratios near 2 for velocity and pressure)."""
    from synth.fields import GreenTaylor2D, face_means
    gt = GreenTaylor2D(amp=1.0, nu=1.0)
    quad = synth.simplex_rule(2, 5)
    errs = []
    for n in (8, 16, 32):
        coords, elems = synth.square_mesh(n)
        fbar = synth.element_means(coords, elems, gt.stokes_force(10.0), n=4)
        g = face_means(coords, wl.exterior_face_list(elems), gt.u)
        P = cr.make_problem(coords, elems, 10.0, 1.0, fbar, gbnd=g)
        U, Pk = cr.solve_coupled(P)
        errs.append(norms.errors(P.mesh, U, Pk, gt.u, gt.grad_u, gt.p, quad, gbnd=g))
    o = _orders(errs)
    assert o[-1]["l2u"] > 1.8 and 0.9 < o[-1]["h1u"] < 1.2 and o[-1]["l2p"] > 1.0, o


# --------------------------------------------------------------------------
# The Newton method on the nonlinear scheme (Section 3.1; Section 4 tests)
# --------------------------------------------------------------------------

def test_newton_steady_green_taylor_orders():
    """The steady Navier-Stokes problem with the Green-Taylor vortex as exact
    solution (force 2 k^2 nu u, the convection balanced by the pressure
    gradient) and its face means on the boundary: Newton converges
    quadratically (increments fall at least like the square of the previous
    ones) to a solution whose nonlinear residual is at rounding level, and the
    errors fall with the orders of Table tab0 (velocity L2 about 2, pressure
    above 1)."""
    from oracle import newton
    from synth.fields import GreenTaylor2D, face_means
    gt = GreenTaylor2D(amp=1.0, nu=0.1)
    quad = synth.simplex_rule(2, 5)
    errs = []
    for n in (8, 16, 32):
        coords, elems = synth.square_mesh(n)
        fbar = synth.element_means(coords, elems, gt.steady_ns_force(), n=4)
        g = face_means(coords, wl.exterior_face_list(elems), gt.u)
        U, Pk, inc = newton.newton(coords, elems, 0.0, gt.nu, fbar, gbnd=g, tol=1e-12)
        assert inc[-1] <= 1e-12 and len(inc) <= 8, inc
        for a, b in zip(inc[1:-1], inc[2:]):
            assert b <= max(10.0 * a * a, 1e-13), inc
        res, div = newton.nonlinear_residual(coords, elems, 0.0, gt.nu, fbar, U, Pk, gbnd=g)
        assert res < 1e-11, res
        m = cr.build_mesh(coords, elems)
        errs.append(norms.errors(m, U, Pk, gt.u, gt.grad_u, gt.p, quad, gbnd=g))
    o = _orders(errs)
    assert o[-1]["l2u"] > 1.8 and o[-1]["l2p"] > 1.0, o


def test_newton_cavity_small():
    """Lid-driven cavity (Section 4.3: velocity (1, 0) on the top side, zero on
    the others) at Re = 100 on 8 x 8 x 2: Newton from rest converges, the
    solution carries the lid's velocity into the cavity (a recirculation: the
    horizontal velocity changes sign along the vertical centre line) and
    is divergence-free on every element."""
    from oracle import newton
    coords, elems = synth.square_mesh(8)
    bf = wl.exterior_face_list(elems)
    ymid = coords[bf].mean(axis=1)[:, 1]
    g = np.zeros((len(bf), 2))
    g[ymid > 1.0 - 1e-12, 0] = 1.0
    U, Pk, inc = newton.newton(coords, elems, 0.0, 0.01, np.zeros((len(elems), 2)), gbnd=g, tol=1e-10)
    assert inc[-1] <= 1e-10 and len(inc) <= 12, inc
    faces = wl.interior_face_list(elems)
    xm = coords[faces].mean(axis=1)
    centre = np.abs(xm[:, 0] - 0.5) < 0.07
    ux = U[centre, 0]
    assert ux.max() > 0.05 and ux.min() < -0.05
    P = cr.make_problem(coords, elems, 0.0, 0.01, np.zeros((len(elems), 2)), ulin=U, gbnd=g)
    assert np.abs(cr.divergence(P, U) - P.ediv())[np.arange(len(elems)) != 0].max() < 1e-12

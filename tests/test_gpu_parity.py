"""Parity of the HIP path with the CPU oracle (GPU only).

Tolerances (derived from the arithmetic of each path):
  * G, S (FP64 elimination): max |G_gpu - G_oracle| <= 1e-10 max |G_oracle|;
  * FP64 path: ||U - U_o|| / ||U_o|| <= 1e-10 and the same for P;
  * FP32 Krylov inside FP64 refinement: 1e-9.
The solves run to a residual tolerance tight enough for these forward errors
on the test meshes (condition numbers of G below 1e5 here).
"""
import numpy as np
import pytest
import torch

import synth
import synth.workloads as wl
from oracle import cr

pytestmark = pytest.mark.gpu


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)

def assert_close(a, b, bar):
    """Relative 2-norm and max-norm error of a against the oracle's b, both <= bar."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    e2 = relerr(a, b)
    mb = np.abs(b).max()
    emax = np.abs(a - b).max() / (mb if mb > 0 else 1.0)
    assert e2 <= bar and emax <= bar, (e2, emax, bar)



def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def make_case(name):
    if name == "square16":
        w = wl.square16()
        return w["coords"], w["elems"], w["mu"], w["nu"], w["fbar"], None, "stokes"
    if name == "jitter12":
        coords, elems = synth.square_mesh(12, jitter=0.2, seed=7)
        fbar = np.random.default_rng(7).normal(size=(len(elems), 2))
        return coords, elems, 300.0, 1.0, fbar, None, "stokes"
    if name == "cube3":
        coords, elems = synth.cube_mesh(3)
        fbar = np.random.default_rng(8).normal(size=(len(elems), 3))
        return coords, elems, 100.0, 1.0, fbar, None, "stokes"
    if name == "steady10":
        coords, elems = synth.square_mesh(10, jitter=0.1, seed=9)
        fbar = np.random.default_rng(9).normal(size=(len(elems), 2))
        return coords, elems, 0.0, 1.0, fbar, None, "stokes"
    if name == "ns10":
        w = wl.ns_square(10, nu=0.01, seed=2)
        return w["coords"], w["elems"], 0.0, w["nu"], w["fbar"], w["ulin"], "ns"
    if name == "ns3d":
        # 3D steady Newton step (E_K from the M1/M2 partition), 3^3 x 6 tetrahedra
        w = wl.ns_cube(3, nu=0.05, seed=4)
        return w["coords"], w["elems"], 0.0, w["nu"], w["fbar"], 5.0 * w["ulin"], "ns"
    if name == "ns3d_t":
        # 3D transient Newton step (mu = 20: E_K = 0)
        w = wl.ns_cube(3, nu=0.05, seed=6)
        return w["coords"], w["elems"], 20.0, w["nu"], w["fbar"], 5.0 * w["ulin"], "ns"
    raise KeyError(name)


CASES = ["square16", "jitter12", "cube3", "steady10", "ns10", "ns3d", "ns3d_t"]


def oracle_problem(case, k0=0):
    coords, elems, mu, nu, fbar, ulin, prob = case
    return cr.make_problem(coords, elems, mu, nu, fbar, ulin=ulin, k0=k0)


def gpu_system(gpu, case, k0=0):
    coords, elems, mu, nu, fbar, ulin, prob = case
    s = gpu.System(coords, elems, mu, nu, k0=k0, problem=prob)
    s.eliminate(dev(fbar), None, None if ulin is None else dev(ulin))
    return s


@pytest.mark.parametrize("name", CASES)
def test_faces_and_G_S(gpu, name):
    case = make_case(name)
    print(f"case {name}", flush=True)
    P = oracle_problem(case)
    s = gpu_system(gpu, case)
    assert (s.interior_faces() == P.mesh.faces).all()
    H = cr.eliminate(P)
    G, S = s.export_G()
    Go = H.G.tocsr()
    Go.sum_duplicates()
    Go.sort_indices()
    assert G.nnz == Go.nnz == s.nnz_G
    assert (G.indptr == Go.indptr).all() and (G.indices == Go.indices).all()
    scale = np.abs(Go.data).max()
    assert np.abs(G.data - Go.data).max() <= 1e-10 * scale
    assert np.abs(S - H.S).max() <= 1e-10 * np.abs(H.S).max()
    s.close()


@pytest.mark.parametrize("name", CASES)
def test_recover_from_oracle_W(gpu, name):
    """Recovery alone: the oracle's W in, U and P out, against the oracle's recovery."""
    case = make_case(name)
    P = oracle_problem(case)
    U_o, P_o, W_o, H, _ = cr.solve_hybrid(P)
    s = gpu_system(gpu, case)
    s.import_W(W_o)
    U, Pk, J = s.recover(jump=True)
    torch.cuda.synchronize()
    assert_close(U.cpu().numpy(), U_o, 1e-10)
    assert_close(Pk.cpu().numpy(), P_o, 1e-10)
    assert float(Pk[0]) == 0.0
    # copy mismatch equals the residual of W (zero up to rounding here)
    assert float(J.item()) <= 1e-9 * np.linalg.norm(H.S)
    s.close()


@pytest.mark.parametrize("name", ["square16", "jitter12", "cube3", "steady10"])
def test_export_coupled_matches_oracle(gpu, name):
    """cr_export_coupled gives the oracle's coupled matrix [A D^t; D 0] and [R; 0]
    (Section 3.1) entry by entry, with the structural count of cr_query_sizes;
    the Navier-Stokes system is refused."""
    import scipy.sparse as sps
    case = make_case(name)
    P = oracle_problem(case)
    A, D, R, prow = cr.assemble_coupled(P)
    Mo = sps.bmat([[A, D.T], [D, None]], format="csr")
    bo = np.concatenate([R, np.zeros(D.shape[0])])
    s = gpu_system(gpu, case)
    M, b = s.export_coupled()
    assert M.shape == Mo.shape and M.nnz == s.nnz_coupled
    assert np.all(np.diff(M.indptr) >= 0)
    scale = np.abs(Mo.data).max()
    assert abs(M - Mo).max() <= 1e-12 * scale
    assert np.abs(b - bo).max() <= 1e-12 * np.abs(bo).max()
    s.close()
    ns = gpu_system(gpu, make_case("ns10"))
    with pytest.raises(gpu.CRError):
        ns.export_coupled()
    ns.close()


def test_jump_equals_residual_random_W(gpu):
    """For any W the copy mismatch ||C^ U^|| equals ||S - G W|| (substitution of the
    recovery relations into the C^ row of the three-field system)."""
    case = make_case("jitter12")
    P = oracle_problem(case)
    H = cr.eliminate(P)
    W = np.random.default_rng(3).normal(size=H.S.shape)
    s = gpu_system(gpu, case)
    s.import_W(W.reshape(-1, 2))
    _, _, J = s.recover(jump=True)
    ref = np.linalg.norm(H.S - H.G @ W)
    assert abs(J.item() - ref) <= 1e-9 * ref
    s.close()


@pytest.mark.parametrize("operator", ["element", "assembled"])
@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("fp32_ir", 1e-9)])
@pytest.mark.parametrize("name", ["square16", "jitter12", "cube3"])
def test_pcg_solution_parity(gpu, name, precision, bar, operator):
    case = make_case(name)
    print(f"case {name} {precision} {operator}", flush=True)
    P = oracle_problem(case)
    U_o, P_o = cr.solve_coupled(P)
    s = gpu_system(gpu, case)
    info = s.solve("pcg", precision, tol=1e-13, check_every=8, operator=operator)
    assert info["rel_residual"] <= 1e-13
    U, Pk = s.recover()
    torch.cuda.synchronize()
    assert_close(U.cpu().numpy(), U_o, bar)
    assert_close(Pk.cpu().numpy(), P_o, bar)
    s.close()


@pytest.mark.parametrize("method", ["bicgstab", "bicgstab2"])
@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("fp32_ir", 1e-9)])
@pytest.mark.parametrize("name", ["steady10", "ns10", "ns3d", "ns3d_t"])
def test_bicgstab_solution_parity(gpu, name, precision, bar, method):
    case = make_case(name)
    print(f"case {name} {precision} {method}", flush=True)
    P = oracle_problem(case)
    U_o, P_o = cr.solve_coupled(P)
    s = gpu_system(gpu, case)
    info = s.solve(method, precision, tol=1e-13, check_every=8, maxit=200000)
    assert info["rel_residual"] <= 1e-13
    U, Pk = s.recover()
    torch.cuda.synchronize()
    assert_close(U.cpu().numpy(), U_o, bar)
    assert_close(Pk.cpu().numpy(), P_o, bar)
    s.close()


@pytest.mark.parametrize("name", ["jitter12", "cube3"])
def test_operator_forms_agree(gpu, name):
    """The element-factor operator and the assembled rows apply the same G:
    solves to 1e-13 with either form give the same W up to the conditioning of G,
    and the element form is refused where it does not exist (BiCGStab, mu = 0)."""
    case = make_case(name)
    s = gpu_system(gpu, case)
    a = s.solve("pcg", "fp64", tol=1e-13, check_every=8, operator="element")
    Wa = s.export_W()
    b = s.solve("pcg", "fp64", tol=1e-13, check_every=8, operator="assembled")
    Wb = s.export_W()
    assert a["rel_residual"] <= 1e-13 and b["rel_residual"] <= 1e-13
    assert relerr(Wa, Wb) <= 1e-10
    # each form's FP64 residual certifies the other's solution: warm start from W_a
    # with the assembled form stops at once
    s.import_W(Wa)
    c = s.solve("pcg", "fp64", tol=1e-12, warm_start=True, operator="assembled")
    assert c["iters"] == 0
    with pytest.raises(gpu.CRError):
        s.solve("bicgstab", "fp64", tol=1e-10, operator="element")
    s.close()
    st = gpu_system(gpu, make_case("steady10"))
    with pytest.raises(gpu.CRError):
        st.solve("pcg", "fp64", tol=1e-10, operator="element")
    st.close()


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("fp32_ir", 1e-9)])
@pytest.mark.parametrize("name", ["steady10", "square16", "cube3"])
def test_minres_solution_parity(gpu, name, precision, bar):
    """MINRES on the symmetric G: indefinite (steady Stokes) and definite."""
    case = make_case(name)
    print(f"case {name} {precision} minres", flush=True)
    P = oracle_problem(case)
    U_o, P_o = cr.solve_coupled(P)
    s = gpu_system(gpu, case)
    info = s.solve("minres", precision, tol=1e-13, check_every=12, maxit=200000)
    assert info["rel_residual"] <= 1e-13
    U, Pk = s.recover()
    torch.cuda.synchronize()
    assert_close(U.cpu().numpy(), U_o, bar)
    assert_close(Pk.cpu().numpy(), P_o, bar)
    with pytest.raises(gpu.CRError):
        s.solve("minres", "fp64", tol=1e-10, operator="element")
    s.close()


@pytest.mark.parametrize("operator", ["element", "assembled"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_kernel_timing_runs_the_full_kernel(gpu, precision, operator):
    """cr_time_spmv launches the dominant kernel on a scratch state that never
    stops early: its launch time stays above the bytes it must move at the HBM
    peak (8 TB/s), and the resident solution is untouched.  512x512x2, so that
    the bytes of one launch take far longer than an early return."""
    coords, elems = synth.square_mesh(512, jitter=0.2, seed=11)
    fbar = np.random.default_rng(11).normal(size=(len(elems), 2))
    s = gpu.System(coords, elems, 1000.0, 1.0)
    s.eliminate(dev(fbar))
    s.solve("pcg", "fp32_ir", tol=1e-6)
    W0 = s.export_W()
    ms, by = s.time_spmv(precision, reps=20, operator=operator)
    assert by / (ms * 1e-3) < 8e12
    assert np.array_equal(s.export_W(), W0)
    s.close()


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("fp32_ir", 1e-9)])
def test_coarse_correction_parity(gpu, precision, bar):
    """CG with the aggregate coarse correction (64 x 64 x 2 = 8192 elements, 64
    aggregates, and 128 x 128 x 2 with 256) against the oracle's direct solve, and
    against the same solve with Jacobi only: same solution, fewer iterations."""
    for n, seed in [(64, 21), (128, 22)]:
        coords, elems = synth.square_mesh(n, jitter=0.2, seed=seed)
        fbar = np.random.default_rng(seed).normal(size=(len(elems), 2))
        mu = 1000.0
        P = cr.make_problem(coords, elems, mu, 1.0, fbar)
        U_o, P_o = cr.solve_coupled(P)
        s = gpu.System(coords, elems, mu, 1.0)
        s.eliminate(dev(fbar))
        a = s.solve("pcg", precision, tol=1e-13)
        U, Pk = s.recover()
        torch.cuda.synchronize()
        print(f"{n}x{n}x2 {precision}: coarse {a['iters']} iterations", flush=True)
        assert_close(U.cpu().numpy(), U_o, bar)
        assert_close(Pk.cpu().numpy(), P_o, bar)
        Wa = s.export_W()
        b = s.solve("pcg", precision, tol=1e-13, coarse=False)
        print(f"{n}x{n}x2 {precision}: Jacobi only {b['iters']} iterations", flush=True)
        assert relerr(Wa, s.export_W()) <= 1e-9
        assert a["iters"] < b["iters"]
        s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_coarse_correction_3d(gpu, precision):
    """3D coarse correction (12^3 x 6 = 10,368 tetrahedra, 64 aggregates): the
    same W as the Jacobi-only solve of the same system (whose parity with the
    oracle is tested on 5^3 x 6; the oracle's direct solve at this size takes
    about a minute), fewer iterations, and the FP64 residual at the tolerance."""
    coords, elems = synth.cube_mesh(12)
    fbar = np.random.default_rng(31).normal(size=(len(elems), 3))
    s = gpu.System(coords, elems, 100.0, 1.0)
    s.eliminate(dev(fbar))
    a = s.solve("pcg", precision, tol=1e-12)
    Wa = s.export_W()
    b = s.solve("pcg", precision, tol=1e-12, coarse=False)
    print(f"12^3x6 {precision}: coarse {a['iters']}, Jacobi only {b['iters']} iterations", flush=True)
    assert a["status"] == 0 and b["status"] == 0
    assert a["rel_residual"] <= 1e-12 and b["rel_residual"] <= 1e-12
    assert relerr(Wa, s.export_W()) <= 1e-9
    assert a["iters"] < b["iters"]
    s.close()


def test_graph_and_plain_launches_agree(gpu):
    """The captured-graph replay and plain launches run the same kernels: same iterates."""
    case = make_case("jitter12")
    s = gpu_system(gpu, case)
    a = s.solve("pcg", "fp32_ir", tol=1e-11, check_every=6, graph=True)
    Wa = s.export_W()
    b = s.solve("pcg", "fp32_ir", tol=1e-11, check_every=6, graph=False)
    Wb = s.export_W()
    assert a["iters"] == b["iters"]
    assert np.array_equal(Wa, Wb)
    s.close()


def test_error_paths(gpu):
    case = make_case("square16")
    coords, elems, mu, nu, fbar, _, _ = case
    s = gpu.System(coords, elems, mu, nu)
    with pytest.raises(gpu.CRError):
        s.solve()                                   # before eliminate
    bad = fbar.copy()
    bad[5, 1] = np.nan
    with pytest.raises(gpu.CRError) as e:
        s.eliminate(dev(bad))
    assert e.value.status == -7
    s.eliminate(dev(fbar))
    out = s.solve("pcg", "fp64", tol=1e-12, maxit=3, raise_on_error=False)
    assert out["status"] == -5 and out["iters"] <= 3
    # a tolerance below the attainable accuracy: the FP64 residual stagnates
    # (or p.Gp loses its sign to rounding there) and the solve ends with no
    # convergence or a breakdown long before the iteration cap, with the
    # residual at the attainable accuracy (both operator forms, both
    # precisions; FP32 iterations fall back to FP64)
    for op in ("element", "assembled"):
        for prec in ("fp64", "fp32_ir"):
            out = s.solve("pcg", prec, tol=1e-19, maxit=200000, operator=op, raise_on_error=False)
            msg = gpu.load().cr_last_error().decode()
            print(f"tol 1e-19 {op} {prec}: {out} {msg}", flush=True)
            assert out["status"] in (-5, -6) and out["iters"] < 40000
            assert out["rel_residual"] < 1e-13
            assert "stagnated" in msg or "breakdown" in msg
    s.close()


@pytest.mark.parametrize("method", ["pcg", "minres"])
@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("fp32_ir", 1e-9)])
def test_degenerate_meshes_and_data(gpu, method, precision, bar):
    """Edge cases of the method: the smallest meshes (two triangles or two
    tetrahedra sharing one face: one interior face, one Schur term besides
    K0), a pinned element other than the first, and a zero right-hand side
    (S = 0: no iteration, U = 0 and P = 0)."""
    c2 = np.array([[0, 0], [1, 0], [0, 1], [1, 1]], dtype=float)
    e2 = np.array([[0, 1, 2], [1, 3, 2]], dtype=np.int32)
    c3 = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]], dtype=float)
    e3 = np.array([[0, 1, 2, 3], [1, 2, 3, 4]], dtype=np.int32)
    co12, el12 = synth.square_mesh(12, jitter=0.2, seed=7)
    cases = [(c2, e2, 10.0, 0), (c3, e3, 10.0, 1), (co12, el12, 300.0, 37)]
    for coords, elems, mu, k0 in cases:
        d = coords.shape[1]
        fbar = np.random.default_rng(len(elems)).normal(size=(len(elems), d))
        P = cr.make_problem(coords, elems, mu, 1.0, fbar, k0=k0)
        U_o, P_o = cr.solve_coupled(P)
        s = gpu.System(coords, elems, mu, 1.0, k0=k0)
        s.eliminate(dev(fbar))
        info = s.solve(method, precision, tol=1e-13, maxit=100000)
        U, Pk = s.recover()
        torch.cuda.synchronize()
        print(f"{len(elems)} elements k0={k0} {method} {precision}: {info['iters']} iterations", flush=True)
        assert info["status"] == 0
        assert float(Pk[k0]) == 0.0
        assert np.abs(U.cpu().numpy() - U_o).max() <= bar * max(np.abs(U_o).max(), np.abs(P_o).max())
        assert_close(Pk.cpu().numpy(), P_o, bar)
        # zero data: the solution is zero, with no iteration
        s.eliminate(dev(np.zeros_like(fbar)))
        z = s.solve(method, precision, tol=1e-13)
        U0, P0 = s.recover()
        torch.cuda.synchronize()
        assert z["status"] == 0 and z["iters"] == 0
        assert not U0.any() and not P0.any()
        s.close()


@pytest.mark.parametrize("name", ["square16", "jitter12", "cube3"])
def test_coupled_minres_baseline_parity(gpu, name):
    """The GPU coupled-system baseline reaches the oracle's coupled solution."""
    case = make_case(name)
    print(f"case {name} coupled", flush=True)
    P = oracle_problem(case)
    U_o, P_o = cr.solve_coupled(P)
    s = gpu_system(gpu, case)
    U, Pk, info = s.coupled_solve(tol=1e-13, maxit=500000)
    torch.cuda.synchronize()
    assert info["rel_residual"] <= 1e-13
    assert_close(U.cpu().numpy(), U_o, 1e-10)
    assert_close(Pk.cpu().numpy(), P_o, 1e-10)
    s.close()


@pytest.mark.parametrize("name", ["ns10", "ns3d", "ns3d_t"])
def test_coupled_newton_baseline_parity(gpu, name):
    """The GPU coupled-system baseline of the Newton step (BiCGStab on the
    scaled coupled system, Jacobian blocks of A) reaches the oracle's coupled
    solution."""
    case = make_case(name)
    print(f"case {name} coupled Newton step", flush=True)
    P = oracle_problem(case)
    U_o, P_o = cr.solve_coupled(P)
    s = gpu_system(gpu, case)
    # FP64 BiCGStab on the coupled system levels off near 5e-13 here, so the
    # tolerance is 1e-11 and the bar on the solution 1e-9
    U, Pk, info = s.coupled_solve(tol=1e-11, maxit=200000)
    torch.cuda.synchronize()
    print(info, flush=True)
    assert info["status"] == 0 and info["rel_residual"] <= 1e-11
    assert_close(U.cpu().numpy(), U_o, 1e-9)
    assert_close(Pk.cpu().numpy(), P_o, 1e-9)
    s.close()


@pytest.mark.parametrize("method,case", [("pcg", "jitter12"), ("minres", "square16"), ("pcg", "cube3")])
def test_initial_guess_w0(gpu, method, case):
    """cr_solve_opts.w0: the solution W handed back as the initial guess stops at
    once with the same W; a perturbed W converges to the same W again."""
    c = make_case(case)
    s = gpu_system(gpu, c)
    a = s.solve(method, "fp64", tol=1e-12)
    W = s.export_W()
    s.solve(method, "fp64", tol=1e-12)  # the resident W is now this solution again
    b = s.solve(method, "fp64", tol=1e-12, w0=dev(W))
    assert b["status"] == 0 and b["iters"] <= 2, b
    assert relerr(s.export_W(), W) <= 1e-12
    Wp = W * (1.0 + 0.1 * np.random.default_rng(5).normal(size=W.shape))
    c2 = s.solve(method, "fp64", tol=1e-12, w0=dev(Wp))
    assert c2["status"] == 0 and 0 < c2["iters"]
    assert relerr(s.export_W(), W) <= 1e-9
    # w0 = 0 is the cold start
    d0 = s.solve(method, "fp64", tol=1e-12, w0=dev(np.zeros_like(W)))
    assert d0["iters"] == a["iters"]
    s.close()


def test_precond_options(gpu):
    """precond: "coarse" needs aggregates (refused on a small mesh, accepted on
    64x64x2); "jacobi" and "default" reach the same W."""
    c = make_case("jitter12")
    s = gpu_system(gpu, c)
    with pytest.raises(gpu.CRError, match="coarse correction exists only"):
        s.solve("pcg", "fp64", tol=1e-12, precond="coarse")
    with pytest.raises(gpu.CRError, match="MINRES takes"):
        s.solve("minres", "fp64", tol=1e-12, precond="coarse")
    s.close()
    coords, elems = synth.square_mesh(64, jitter=0.2, seed=2)
    fbar = np.random.default_rng(2).normal(size=(len(elems), 2))
    s = gpu.System(coords, elems, 1000.0, 1.0)
    s.eliminate(dev(fbar))
    a = s.solve("pcg", "fp64", tol=1e-12, precond="coarse")
    Wa = s.export_W()
    b = s.solve("pcg", "fp64", tol=1e-12, precond="jacobi")
    assert relerr(s.export_W(), Wa) <= 1e-9
    assert a["iters"] < b["iters"]
    s.close()


# --------------------------------------------------------------------------
# Non-homogeneous Dirichlet data (cr_set_boundary)
# --------------------------------------------------------------------------

def make_bnd_case(name):
    """(coords, elems, mu, nu, fbar, ulin, g, problem, method) with random data on the exterior faces."""
    dim = 3 if "3d" in name else 2
    if dim == 2:
        coords, elems = synth.square_mesh(10, jitter=0.2, seed=17)
    else:
        coords, elems = synth.cube_mesh(3)
    rng = np.random.default_rng(len(name))
    g = rng.normal(size=(len(wl.exterior_face_list(elems)), dim))
    f = rng.normal(size=(len(elems), dim))
    nf = len(wl.interior_face_list(elems))
    if name.startswith("bnd_stokes"):
        return coords, elems, 80.0, 1.0, f, None, g, "stokes", "pcg"
    if name == "bnd_steady2d":
        return coords, elems, 0.0, 1.0, f, None, g, "stokes", "minres"
    return coords, elems, 0.0, 0.05, f, 0.5 * rng.normal(size=(nf, dim)), g, "ns", "bicgstab2"


BND_CASES = ["bnd_stokes2d", "bnd_stokes3d", "bnd_steady2d", "bnd_ns2d", "bnd_ns3d"]


def bnd_system(gpu, c):
    coords, elems, mu, nu, f, ulin, g, prob, method = c
    s = gpu.System(coords, elems, mu, nu, problem=prob)
    assert (s.boundary_faces() == wl.exterior_face_list(elems)).all()
    s.set_boundary(g)
    s.eliminate(dev(f), None, None if ulin is None else dev(ulin))
    return s


@pytest.mark.parametrize("name", BND_CASES)
def test_boundary_data_parity(gpu, name):
    """With boundary data: S element-wise against the oracle's elimination, and
    the solution U, P against the oracle's coupled solve (FP64, 2-norm and max-norm)."""
    c = make_bnd_case(name)
    coords, elems, mu, nu, f, ulin, g, prob, method = c
    print(f"case {name}", flush=True)
    P = cr.make_problem(coords, elems, mu, nu, f, ulin=ulin, gbnd=g)
    U_o, P_o = cr.solve_coupled(P)
    H = cr.eliminate(P)
    s = bnd_system(gpu, c)
    G, S = s.export_G()
    assert np.abs(S - H.S).max() <= 1e-10 * np.abs(H.S).max()
    info = s.solve(method, "fp64", tol=1e-13, maxit=200000)
    assert info["rel_residual"] <= 1e-13
    U, Pk = s.recover()
    torch.cuda.synchronize()
    assert_close(U.cpu().numpy(), U_o, 1e-10)
    assert_close(Pk.cpu().numpy(), P_o, 1e-10)
    # the coupled baseline with the same data
    Uc, Pc, ci = s.coupled_solve(tol=1e-11, maxit=200000)
    torch.cuda.synchronize()
    assert ci["status"] == 0
    assert_close(Uc.cpu().numpy(), U_o, 1e-9)
    assert_close(Pc.cpu().numpy(), P_o, 1e-9)
    # CG with the assembled rows reaches the same solution as the element form
    # (the default for transient Stokes, whose K0 row takes up the net flux of
    # the random data)
    if prob == "stokes" and method == "pcg":
        s.solve("pcg", "fp64", tol=1e-13, maxit=200000, operator="assembled")
        Ua, Pa = s.recover()
        torch.cuda.synchronize()
        assert_close(Ua.cpu().numpy(), U_o, 1e-10)
        assert_close(Pa.cpu().numpy(), P_o, 1e-10)
    s.close()


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("fp32_ir", 1e-9)])
def test_boundary_data_coarse_correction(gpu, precision, bar):
    """Boundary data with a non-zero net flux (random face values) on meshes
    with aggregates (32 x 32 x 2 jittered: 16 aggregates; 8^3 x 6: 8): CG with
    the element form and the coarse correction against the oracle's coupled
    solve, and fewer iterations than with Jacobi scaling only."""
    for dim in (2, 3):
        if dim == 2:
            coords, elems = synth.square_mesh(32, jitter=0.2, seed=31)
        else:
            coords, elems = synth.cube_mesh(8)
        rng = np.random.default_rng(40 + dim)
        g = rng.normal(size=(len(wl.exterior_face_list(elems)), dim))
        f = rng.normal(size=(len(elems), dim))
        P = cr.make_problem(coords, elems, 200.0, 1.0, f, gbnd=g)
        U_o, P_o = cr.solve_coupled(P)
        s = gpu.System(coords, elems, 200.0, 1.0)
        s.set_boundary(g)
        s.eliminate(dev(f))
        a = s.solve("pcg", precision, tol=1e-13, maxit=200000, precond="coarse")
        U, Pk = s.recover()
        torch.cuda.synchronize()
        print(f"{dim}D boundary data {precision}: coarse {a['iters']} iterations", flush=True)
        assert_close(U.cpu().numpy(), U_o, bar)
        assert_close(Pk.cpu().numpy(), P_o, bar)
        b = s.solve("pcg", precision, tol=1e-13, maxit=200000, precond="jacobi")
        print(f"{dim}D boundary data {precision}: Jacobi only {b['iters']} iterations", flush=True)
        assert a["iters"] < b["iters"]
        s.close()


def test_boundary_data_time_steps(gpu):
    """Backward Euler steps with boundary data changing in time (cr_set_boundary
    then cr_update_rhs with the previous U), against the oracle's chain."""
    coords, elems = synth.square_mesh(12, jitter=0.2, seed=23)
    from synth.fields import GreenTaylor2D, face_means
    gt = GreenTaylor2D(amp=1.0, nu=1.0)
    bf = wl.exterior_face_list(elems)
    dt, mu = 0.01, 100.0
    f0 = np.zeros((len(elems), 2))
    s = gpu.System(coords, elems, mu, 1.0)
    up_o = None
    U = None
    for n in range(1, 4):
        g = face_means(coords, bf, lambda x: gt.u(x, n * dt))
        s.set_boundary(g)
        if n == 1:
            s.eliminate(dev(f0))
        else:
            s.update_rhs(dev(f0), U)
        s.solve("pcg", "fp64", tol=1e-13, warm_start=n > 1)
        U, Pk = s.recover()
        P = cr.make_problem(coords, elems, mu, 1.0, f0, u_prev=up_o, gbnd=g)
        U_o, P_o = cr.solve_coupled(P)
        assert_close(U.cpu().numpy(), U_o, 1e-10)
        assert_close(Pk.cpu().numpy(), P_o, 1e-10)
        up_o = U_o
    s.close()


def test_export_w_device_matches_host_export(gpu):
    """cr_export_W_device writes the resident W in canonical order as
    cr_export_W does, and as the initial guess of a solve after a new
    elimination it reaches the same solution in fewer iterations."""
    c = make_case("ns10")
    s = gpu_system(gpu, c)
    s.solve("bicgstab2", "fp64", tol=1e-12, maxit=100000)
    Wd = s.export_W_device()
    torch.cuda.synchronize()
    assert np.array_equal(Wd.cpu().numpy(), s.export_W())
    coords, elems, mu, nu, fbar, ulin, prob = c
    s.eliminate(dev(fbar), None, dev(ulin))
    cold = s.solve("bicgstab2", "fp64", tol=1e-12, maxit=100000)
    s.eliminate(dev(fbar), None, dev(ulin))
    warm = s.solve("bicgstab2", "fp64", tol=1e-12, maxit=100000, w0=Wd)
    print(f"cold {cold['iters']} warm {warm['iters']} iterations", flush=True)
    assert warm["iters"] < cold["iters"]
    assert relerr(s.export_W(), Wd.cpu().numpy()) <= 1e-9
    s.close()

"""GPU tests at the benchmark workloads' sizes and for the time-stepping / serving rows.

Full-size workloads are checked through properties the oracle can evaluate
row by row (its own element matrices, no global solve):
  * the coupled residual R - A U - D^t P on sampled faces and D_K U_K on every
    element, for the U, P the GPU recovers (Section 3.1, eq. syslin);
  * G on sampled faces against the oracle's element-by-element elimination
    (Section 3.2 item 5);
  * the copy mismatch equals the hybridised residual (a consequence of the
    recovery relations of Section 3.2 item 4).
Smaller meshes are compared with the oracle's direct solution element by
element.  Batched and served solves are compared bitwise with single solves.
"""
import os

import numpy as np
import pytest
import torch

import synth
import synth.workloads as wl
from oracle import cr

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)

def assert_close(a, b, bar):
    """Relative 2-norm and max-norm error of a against the oracle's b, both <= bar."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    e2 = relerr(a, b)
    mb = np.abs(b).max()
    emax = np.abs(a - b).max() / (mb if mb > 0 else 1.0)
    assert e2 <= bar and emax <= bar, (e2, emax, bar)



def coupled_rows(P, U, Pk, faces):
    """Rows (f, i) of R - A U - D^t P for the given faces, from the oracle's element
    matrices of the two elements of each face; and D_K U_K for every element."""
    m = P.mesh
    d = P.d
    Ul = cr.local_face_values(m, U).reshape(m.ne, -1)
    div = (P.D * Ul).sum(axis=1)
    res = np.zeros((len(faces), d))
    scale = np.zeros(len(faces))
    for n, f in enumerate(faces):
        for k in m.face_elems[f]:
            j = int(np.nonzero(m.elem_face[k] == f)[0][0])
            rows = slice(j * d, (j + 1) * d)
            loc = P.R[k][rows] - P.A[k][rows] @ Ul[k] - P.D[k][rows] * Pk[k]
            res[n] += loc
            scale[n] = max(scale[n], np.abs(P.R[k][rows]).max(), np.abs(P.A[k][rows] @ Ul[k]).max())
    return res, div


def sampled_G_rows(P, G, faces):
    """Max deviation of the GPU's G rows from the oracle's elimination of the two
    elements of each sampled face (general inverse, no Kronecker shortcut)."""
    m = P.mesh
    d = P.d
    worst, scale = 0.0, 0.0
    for f in faces:
        ref = {}
        for k in m.face_elems[f]:
            Ak, Dk, Rk, gk, idx = cr.restrict(P, k)
            Ck = np.diag(np.repeat(m.sign[k], d)[idx])
            Ai = np.linalg.inv(Ak)
            l = Ai @ Dk
            Gk = Ck @ (Ai - np.outer(l, l) / (Dk @ l)) @ Ck if k != P.k0 else Ck @ Ai @ Ck
            for a, ga in enumerate(gk):
                if ga // d != f:
                    continue
                for b_, gb in enumerate(gk):
                    ref[(ga, gb)] = ref.get((ga, gb), 0.0) + Gk[a, b_]
        for (ga, gb), v in ref.items():
            worst = max(worst, abs(G[ga, gb] - v))
            scale = max(scale, abs(v))
    return worst, scale


@pytest.mark.parametrize("precision", ["fp32_ir", "fp64"])
def test_c2_full_size_certificate(gpu, precision):
    """512x512x2 jittered transient Stokes (the benchmark workload) to 1e-10, in the
    benchmark's configuration (FP32 CG with FP64 residual replacements) and in FP64."""
    w = wl.square512j()
    print(f"C2 inputs ready ({precision})", flush=True)
    s = gpu.System(w["coords"], w["elems"], w["mu"], w["nu"])
    s.eliminate(dev(w["fbar"]))
    info = s.solve("pcg", precision, tol=1e-10)
    print("C2 solve:", info, flush=True)
    assert info["rel_residual"] <= 1e-10
    U, Pk, J = s.recover(jump=True)
    torch.cuda.synchronize()
    G, S = s.export_G()
    P = cr.make_problem(w["coords"], w["elems"], w["mu"], w["nu"], w["fbar"])
    rng = np.random.default_rng(0)
    faces = rng.choice(P.mesh.nf, 300, replace=False)
    worst, scale = sampled_G_rows(P, G, faces[:100])
    assert worst <= 1e-10 * scale
    # copy mismatch == hybridised residual
    W = s.export_W().ravel()
    r = np.linalg.norm(S - G @ W)
    assert abs(J.item() - r) <= 1e-6 * r + 1e-12 * np.linalg.norm(S)
    assert r <= 1.000001e-10 * np.linalg.norm(S)
    Uh, Ph = U.cpu().numpy(), Pk.cpu().numpy()
    res, div = coupled_rows(P, Uh, Ph, faces)
    R = P.R
    assert np.abs(res).max() <= 1e-8 * np.abs(R).max()
    # U takes each face from one copy, so D_K U_K = D_K (copy mismatch): bounded by the solve tolerance
    assert np.abs(div).max() <= 100 * 1e-10 * np.abs(P.D).max() * np.abs(Uh).max()
    s.close()


def stored_oracle(name):
    """The oracle's solution of a full-size workload, sampled (tests/golden/
    oracle_<name>.npz, written by make_oracle_samples.py from the oracle alone)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"oracle_{name}.npz")
    return np.load(path)


def check_against_stored_oracle(name, U, Pk, bar):
    z = stored_oracle(name)
    fi = torch.from_numpy(z["face_ids"].astype(np.int64)).cuda()
    ei = torch.from_numpy(z["elem_ids"].astype(np.int64)).cuda()
    Us = U.index_select(0, fi).cpu().numpy()
    Ps = Pk.index_select(0, ei).cpu().numpy()
    eU2 = relerr(Us, z["U"])
    eP2 = relerr(Ps, z["P"])
    eUm = np.abs(Us - z["U"]).max() / float(z["U_max"])
    ePm = np.abs(Ps - z["P"]).max() / float(z["P_max"])
    print(f"{name}: U {eU2:.2e} / max {eUm:.2e}, P {eP2:.2e} / max {ePm:.2e}", flush=True)
    assert max(eU2, eUm, eP2, ePm) <= bar, (eU2, eUm, eP2, ePm)


@pytest.mark.parametrize("precision,tol", [("fp32_ir", 1e-11), ("fp64", 1e-11)])
def test_c2_full_size_against_stored_oracle(gpu, precision, tol):
    """512x512x2 jittered (1,570,816 unknowns): U and P against the oracle's
    coupled sparse-LU solution (three refinement steps) on 8,287 sampled faces
    and 8,254 elements, 2-norm and max-norm, within 1e-9.  At the residual
    tolerance 1e-11 the pressure error is about 2.5e-10 (1e-10 leaves 1.1e-9 in
    the max-norm)."""
    w = wl.square512j()
    print(f"C2 inputs ready ({precision})", flush=True)
    s = gpu.System(w["coords"], w["elems"], w["mu"], w["nu"])
    s.eliminate(dev(w["fbar"]))
    info = s.solve("pcg", precision, tol=tol)
    assert info["rel_residual"] <= tol
    U, Pk = s.recover()
    torch.cuda.synchronize()
    check_against_stored_oracle("square512j", U, Pk, 1e-9)
    s.close()


def test_c3_full_size_against_stored_oracle(gpu):
    """64^3 x 6 (9,363,456 unknowns), the benchmark's path (FP32 CG with FP64
    residual replacement and the coarse correction): U and P against the
    oracle's solution (general elimination, Jacobi PCG on G to 5e-13, recovery)
    on 8,321 sampled faces and 8,255 elements, within 1e-9.  The pressure needs
    the residual at 1e-13 for that (3e-6 at 1e-9, 2e-9 at 1e-12)."""
    w = wl.cube64()
    print("C3 inputs ready", flush=True)
    s = gpu.System(w["coords"], w["elems"], w["mu"], w["nu"])
    s.eliminate(dev(w["fbar"]))
    info = s.solve("pcg", "fp32_ir", tol=1e-13)
    print("C3 solve:", info, flush=True)
    assert info["rel_residual"] <= 1e-13 and not info["fp64_fallback"]
    U, Pk = s.recover()
    torch.cuda.synchronize()
    check_against_stored_oracle("cube64", U, Pk, 1e-9)
    s.close()


def test_c3_full_size_certificate(gpu):
    """64^3 cubes x6 Kuhn tetrahedra (1,572,864 elements) transient Stokes, FP64 Krylov."""
    w = wl.cube64()
    print("C3 inputs ready", flush=True)
    s = gpu.System(w["coords"], w["elems"], w["mu"], w["nu"])
    s.eliminate(dev(w["fbar"]))
    info = s.solve("pcg", "fp64", tol=1e-9)
    assert info["rel_residual"] <= 1e-9
    U, Pk, J = s.recover(jump=True)
    torch.cuda.synchronize()
    P = cr.make_problem(w["coords"], w["elems"], w["mu"], w["nu"], w["fbar"])
    faces = np.random.default_rng(1).choice(P.mesh.nf, 200, replace=False)
    Uh, Ph = U.cpu().numpy(), Pk.cpu().numpy()
    res, div = coupled_rows(P, Uh, Ph, faces)
    assert np.abs(res).max() <= 1e-7 * np.abs(P.R).max()
    assert np.abs(div).max() <= 100 * 1e-9 * np.abs(P.D).max() * np.abs(Uh).max()
    s.close()


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("fp32_ir", 1e-9)])
def test_c3_small_parity(gpu, precision, bar):
    """3D Kuhn mesh 5^3 x 6 against the oracle's direct coupled solve."""
    w = wl.cube(5, mu=100.0)
    s = gpu.System(w["coords"], w["elems"], w["mu"], w["nu"])
    s.eliminate(dev(w["fbar"]))
    s.solve("pcg", precision, tol=1e-13)
    U, Pk = s.recover()
    torch.cuda.synchronize()
    P = cr.make_problem(w["coords"], w["elems"], w["mu"], w["nu"], w["fbar"])
    Uo, Po = cr.solve_coupled(P)
    assert_close(U.cpu().numpy(), Uo, bar)
    assert_close(Pk.cpu().numpy(), Po, bar)
    s.close()


@pytest.mark.parametrize("method", ["bicgstab", "bicgstab2"])
@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("fp32_ir", 1e-9)])
def test_c4_ns_newton_step_parity(gpu, precision, bar, method):
    """Steady Navier-Stokes Newton step (nu = 0.01, seeded divergence-free
    linearisation velocity) on 24x24x2 against the oracle's direct solve."""
    w = wl.ns_square(24, nu=0.01, seed=0)
    s = gpu.System(w["coords"], w["elems"], 0.0, w["nu"], problem="ns")
    s.eliminate(dev(w["fbar"]), None, dev(w["ulin"]))
    info = s.solve(method, precision, tol=1e-12, maxit=400000)
    assert info["rel_residual"] <= 1e-12
    U, Pk = s.recover()
    torch.cuda.synchronize()
    P = cr.make_problem(w["coords"], w["elems"], 0.0, w["nu"], w["fbar"], ulin=w["ulin"])
    Uo, Po = cr.solve_coupled(P)
    assert_close(U.cpu().numpy(), Uo, bar)
    assert_close(Pk.cpu().numpy(), Po, bar)
    s.close()


def test_c4_full_size_certificate(gpu):
    """256x256x2 steady Navier-Stokes Newton step (392,192 unknowns, strongly
    indefinite G): BiCGStab(2) in FP64 to 1e-9.  Certificate: the residual
    recomputed on the host from the exported G and W; the copy mismatch equals
    it; the coupled momentum rows of the recovered (U, P) at sampled faces are
    bounded by |A_K| times the copy mismatch (each element's copy satisfies its
    momentum rows exactly, U takes each face from one copy, and the E_K terms of
    a face cancel up to lambda times the mismatch); D_K U_K likewise."""
    w = wl.ns256()
    print("C4 inputs ready", flush=True)
    s = gpu.System(w["coords"], w["elems"], 0.0, w["nu"], problem="ns")
    s.eliminate(dev(w["fbar"]), None, dev(w["ulin"]))
    info = s.solve("bicgstab2", "fp64", tol=1e-9, maxit=600000)
    print("C4 256x256 BiCGStab(2):", info, flush=True)
    assert info["status"] == 0 and info["rel_residual"] <= 1e-9
    U, Pk, J = s.recover(jump=True)
    torch.cuda.synchronize()
    G, S = s.export_G()
    Wv = s.export_W().ravel()
    r = np.linalg.norm(S - G @ Wv)
    assert r <= 1.000001e-9 * np.linalg.norm(S)
    assert abs(J.item() - r) <= 1e-6 * r + 1e-12 * np.linalg.norm(S)
    P = cr.make_problem(w["coords"], w["elems"], 0.0, w["nu"], w["fbar"], ulin=w["ulin"])
    faces = np.random.default_rng(2).choice(P.mesh.nf, 300, replace=False)
    Uh, Ph = U.cpu().numpy(), Pk.cpu().numpy()
    res, div = coupled_rows(P, Uh, Ph, faces)
    Amax = max(np.abs(P.A[k]).sum(axis=1).max() for f in faces for k in P.mesh.face_elems[f])
    Dmax = np.abs(P.D).max()
    assert np.abs(res).max() <= 10 * Amax * J.item()
    # D_K U^_K = 0 holds element by element except at K0, whose balance is the
    # sum of all the others: |D_K0 U^_K0| <= max|a| ||mismatch||_1 <= max|a| sqrt(n) J
    others = np.delete(div, P.k0)
    assert np.abs(others).max() <= 10 * Dmax * J.item() * (P.d + 1)
    assert abs(div[P.k0]) <= 10 * Dmax * J.item() * (np.sqrt(P.mesh.nf * P.d) + P.d + 1)
    s.close()


def test_steady_stokes_full_size_certificate(gpu):
    """Steady Stokes (mu = 0, E_K from the M1/M2 partition, symmetric indefinite
    G) on 256x256x2: MINRES in FP64 to 1e-9 (FP32 passes restart too often to
    pay off here), and the same certificate as the Navier-Stokes step
    (host-recomputed residual, copy mismatch, sampled coupled rows, element
    divergence)."""
    w = wl.square(256, mu=0.0, nu=1.0, jitter=0.2, seed=3, quad=2)
    s = gpu.System(w["coords"], w["elems"], 0.0, 1.0)
    s.eliminate(dev(w["fbar"]))
    info = s.solve("minres", "fp64", tol=1e-9, maxit=600000)
    print("steady Stokes 256x256 MINRES:", info, flush=True)
    assert info["status"] == 0 and info["rel_residual"] <= 1e-9
    U, Pk, J = s.recover(jump=True)
    torch.cuda.synchronize()
    G, S = s.export_G()
    Wv = s.export_W().ravel()
    r = np.linalg.norm(S - G @ Wv)
    assert r <= 1.000001e-9 * np.linalg.norm(S)
    assert abs(J.item() - r) <= 1e-6 * r + 1e-12 * np.linalg.norm(S)
    P = cr.make_problem(w["coords"], w["elems"], 0.0, 1.0, w["fbar"])
    faces = np.random.default_rng(4).choice(P.mesh.nf, 300, replace=False)
    Uh, Ph = U.cpu().numpy(), Pk.cpu().numpy()
    res, div = coupled_rows(P, Uh, Ph, faces)
    Amax = max(np.abs(P.A[k]).sum(axis=1).max() for f in faces for k in P.mesh.face_elems[f])
    Dmax = np.abs(P.D).max()
    assert np.abs(res).max() <= 10 * Amax * J.item()
    others = np.delete(div, P.k0)
    assert np.abs(others).max() <= 10 * Dmax * J.item() * (P.d + 1)
    assert abs(div[P.k0]) <= 10 * Dmax * J.item() * (np.sqrt(P.mesh.nf * P.d) + P.d + 1)
    s.close()


def test_multistep_update_rhs_parity(gpu):
    """Three backward-Euler steps with cr_update_rhs (same G, u_prev = previous U)
    against the oracle's coupled solves with the same previous velocity."""
    coords, elems = synth.square_mesh(12, jitter=0.2, seed=5)
    man = synth.Manufactured(2, seed=5, mu=1.0, nu=1.0)
    mu, nu = 50.0, 1.0
    fbar = synth.element_means(coords, elems, man.force(mu, nu), n=4)
    s = gpu.System(coords, elems, mu, nu)
    s.eliminate(dev(fbar))
    uo = None
    for step in range(3):
        if step > 0:
            s.update_rhs(dev(fbar), U)
        s.solve("pcg", "fp64", tol=1e-13, warm_start=step > 0)
        U, Pk = s.recover()
        torch.cuda.synchronize()
        P = cr.make_problem(coords, elems, mu, nu, fbar, u_prev=uo)
        uo, po = cr.solve_coupled(P)
        assert_close(U.cpu().numpy(), uo, 1e-10)
        assert_close(Pk.cpu().numpy(), po, 1e-10)
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_batch_bitwise_equals_single(gpu, precision):
    systems = []
    # 20 x 20 x 2, 33 x 33 x 2 and 64 x 64 x 2 have aggregates (4, 16 and 64),
    # so the batched coarse solve runs too, beside systems without
    for n, mu in [(8, 300.0), (12, 50.0), (20, 1000.0), (33, 10.0), (64, 1000.0)]:
        co, el = synth.square_mesh(n, jitter=0.2, seed=n)
        fb = np.random.default_rng(n).normal(size=(len(el), 2))
        s = gpu.System(co, el, mu, 1.0)
        s.eliminate(dev(fb))
        systems.append(s)
    solo = []
    for s in systems:
        info = s.solve("pcg", precision, tol=1e-11)
        solo.append((s.export_W(), info["iters"]))
    b = gpu.Batch(8)
    for s in systems:
        b.add(s, method="pcg", precision=precision, tol=1e-11)
    got = {}
    while len(got) < len(systems):
        b.advance(16)
        while (r := b.pop()) is not None:
            got[r[0].h.value] = (r[0].export_W(), r[1]["iters"], r[1]["status"])
    for s, (W, it) in zip(systems, solo):
        Wb, itb, st = got[s.h.value]
        assert st == 0 and itb == it
        assert np.array_equal(W, Wb)
    assert b.count() == (0, 0)
    b.close()
    for s in systems:
        s.close()


def test_serving_mix_equals_solo(gpu):
    """Requests served in a continuous batch give the same U and P as the same
    session run alone, step by step (bitwise: same kernels, same decisions)."""
    from paper_2101_03777_amd.serve import Server, Session
    ss = wl.serving_sessions(40, seed=3, n_min=8, n_max=40, rate=400.0, max_steps=5)
    sessions = [Session(i, d["coords"], d["elems"], d["dt"], d["nu"], d["fbar"], d["steps"], d["arrival"])
                for i, d in enumerate(ss)]
    served = {}

    def keep(sess, step, U, P, info):
        served[(sess.sid, step)] = (U.cpu().numpy(), P.cpu().numpy(), info["status"])

    srv = Server(hbm_budget=64 << 20, max_active=6, precision="fp32_ir", tol=1e-9)
    stats = srv.run(sessions, on_result=keep)
    srv.close()
    print({k: v for k, v in stats.items() if k != "records"}, flush=True)
    assert stats["requests"] == sum(d["steps"] for d in ss) == len(served)
    assert stats["failed"] == 0
    assert stats["peak_active"] <= 6
    for i, d in enumerate(ss):
        s = gpu.System(d["coords"], d["elems"], 1.0 / d["dt"], d["nu"])
        f = dev(d["fbar"])
        s.eliminate(f)
        for step in range(d["steps"]):
            if step > 0:
                s.update_rhs(f, U)
            s.solve("pcg", "fp32_ir", tol=1e-9, warm_start=step > 0)
            U, Pk = s.recover()
            Us, Ps, st = served[(i, step)]
            assert st == 0
            assert np.array_equal(U.cpu().numpy(), Us), (i, step)
            assert np.array_equal(Pk.cpu().numpy(), Ps), (i, step)
        s.close()


def test_prepared_assembly_equals_direct(gpu):
    """cr_prepare + cr_assemble_prepared (host part on a worker thread) builds the
    same system as cr_assemble: bitwise equal W and iteration count, with the
    coarse correction (128 x 128 x 2: 256 aggregates) and without (steady case)."""
    import concurrent.futures
    for n, mu, method in [(128, 1000.0, "pcg"), (24, 0.0, "minres")]:
        co, el = synth.square_mesh(n, jitter=0.2, seed=7)
        fb = dev(np.random.default_rng(n).normal(size=(len(el), 2)))
        with concurrent.futures.ThreadPoolExecutor(1) as ex:
            prep = ex.submit(gpu.Prepared, co, el, mu=mu, nu=1.0).result()
        out = []
        for s in (gpu.System(co, el, mu, 1.0), gpu.System(prepared=prep)):
            assert s.n_elements == len(el)
            s.eliminate(fb)
            info = s.solve(method, "fp64", tol=1e-10)
            out.append((s.export_W(), info["iters"], info["status"]))
            s.close()
        assert out[0][2] == 0 and out[1][2] == 0
        assert out[0][1] == out[1][1]
        assert np.array_equal(out[0][0], out[1][0])


def test_batch_fp64_fallback_equals_solo(gpu):
    """A system whose FP32 iterations stall switches to FP64 iterations inside
    the batch (its replacements are serviced with its own kernels and it is
    regrouped into the FP64 grid), next to FP32 systems: every system's W and
    iteration count equal its solo solve bitwise, the forced system reports the
    fallback, and its U and P match the oracle.  The stall is forced from the
    host: inner_tol = 0.9 asks for a replacement after every 10% drop of the
    recursive residual, so the second replacement fails to halve the FP64
    residual, which is the stall rule."""
    systems, opts = [], []
    for n, mu, inner in [(10, 300.0, 0.0), (14, 1000.0, 0.9), (20, 50.0, 0.0), (64, 1000.0, 0.0)]:
        co, el = synth.square_mesh(n, jitter=0.2, seed=40 + n)
        fb = np.random.default_rng(40 + n).normal(size=(len(el), 2))
        s = gpu.System(co, el, mu, 1.0)
        s.eliminate(dev(fb))
        systems.append((s, co, el, mu, fb))
        opts.append(dict(method="pcg", precision="fp32_ir", tol=1e-12, inner_tol=inner))
    solo = []
    for (s, *_), o in zip(systems, opts):
        info = s.solve(**o)
        solo.append((s.export_W(), info["iters"], info["fp64_fallback"]))
    assert [f for _, _, f in solo] == [False, True, False, False]
    b = gpu.Batch(8)
    for (s, *_), o in zip(systems, opts):
        b.add(s, **o)
    got = {}
    while len(got) < len(systems):
        b.advance(16)
        while (r := b.pop()) is not None:
            got[r[0].h.value] = (r[0].export_W(), r[1]["iters"], r[1]["status"], r[1]["fp64_fallback"])
    for (s, *_), (W, it, fb) in zip(systems, solo):
        Wb, itb, st, fbb = got[s.h.value]
        assert st == 0 and itb == it and fbb == fb
        assert np.array_equal(W, Wb)
    b.close()
    s, co, el, mu, fb = systems[1]
    U, Pk = s.recover()
    torch.cuda.synchronize()
    Uo, Po = cr.solve_coupled(cr.make_problem(co, el, mu, 1.0, fb))
    assert_close(U.cpu().numpy(), Uo, 1e-9)
    assert_close(Pk.cpu().numpy(), Po, 1e-9)
    for s, *_ in systems:
        s.close()


def test_serving_budget_limits_admission(gpu):
    """With room for about three of the sessions' systems in the device-memory
    budget and many batch slots, the budget (not the slot count) holds
    sessions back, and every request still completes."""
    from paper_2101_03777_amd.serve import Server, Session, BYTES_PER_ELEMENT_2D
    ss = wl.serving_sessions(60, seed=5, n_min=24, n_max=40, rate=1000.0, max_steps=4)
    sessions = [Session(i, d["coords"], d["elems"], d["dt"], d["nu"], d["fbar"], d["steps"], d["arrival"])
                for i, d in enumerate(ss)]
    big = max(len(d["elems"]) for d in ss) * BYTES_PER_ELEMENT_2D
    budget = int(3.5 * big)
    srv = Server(hbm_budget=budget, max_active=64, precision="fp32_ir", tol=1e-9)
    st = srv.run(sessions)
    srv.close()
    print({k: v for k, v in st.items() if k != "records"}, flush=True)
    assert st["requests"] == sum(d["steps"] for d in ss) and st["failed"] == 0
    assert st["budget_blocks"] > 0 and st["slot_blocks"] == 0
    assert st["peak_active"] < 64 and st["peak_active"] <= budget // (min(len(d["elems"]) for d in ss) *
                                                                      BYTES_PER_ELEMENT_2D)


def test_serving_against_oracle(gpu):
    """Served time steps against the oracle's own chain of coupled solves
    (backward Euler, u_prev = the oracle's previous U): U and P within 1e-9 at
    every step, in 2-norm and max-norm."""
    from paper_2101_03777_amd.serve import Server, Session
    ss = wl.serving_sessions(9, seed=7, n_min=8, n_max=16, rate=1000.0, max_steps=3)
    sessions = [Session(i, d["coords"], d["elems"], d["dt"], d["nu"], d["fbar"], d["steps"], d["arrival"])
                for i, d in enumerate(ss)]
    served = {}

    def keep(sess, step, U, P, info):
        served[(sess.sid, step)] = (U.cpu().numpy(), P.cpu().numpy(), info["status"])

    srv = Server(hbm_budget=1 << 30, max_active=8, precision="fp32_ir", tol=1e-12)
    st = srv.run(sessions, on_result=keep)
    srv.close()
    assert st["failed"] == 0
    for i, d in enumerate(ss):
        u_prev = None
        for step in range(d["steps"]):
            P = cr.make_problem(d["coords"], d["elems"], 1.0 / d["dt"], d["nu"], d["fbar"], u_prev=u_prev)
            Uo, Po = cr.solve_coupled(P)
            Us, Ps, status = served[(i, step)]
            assert status == 0
            assert_close(Us, Uo, 1e-9)
            assert_close(Ps, Po, 1e-9)
            u_prev = Uo


# --------------------------------------------------------------------------
# Newton iterations with boundary data (lid-driven cavity, Green-Taylor vortex)
# --------------------------------------------------------------------------

def _cavity(n):
    coords, elems = synth.square_mesh(n)
    bf = wl.exterior_face_list(elems)
    g = np.zeros((len(bf), 2))
    g[coords[bf].mean(axis=1)[:, 1] > 1.0 - 1e-12, 0] = 1.0
    return coords, elems, g


def test_newton_cavity_against_oracle(gpu):
    """Lid-driven cavity, Re = 100, 8 x 8 x 2, Newton from rest: the GPU's
    iterations (hybridised Newton steps, BiCGStab(2)) follow the oracle's
    (coupled direct solves): same number of iterations, U and P within 1e-9."""
    from oracle import newton as onewton
    from paper_2101_03777_amd.newton import NewtonSolver
    coords, elems, g = _cavity(8)
    f = np.zeros((len(elems), 2))
    Uo, Po, inc_o = onewton.newton(coords, elems, 0.0, 0.01, f, gbnd=g, tol=1e-10)
    ns = NewtonSolver(coords, elems, 0.0, 0.01)
    ns.set_boundary(g)
    U, P, rec = ns.solve(f, tol=1e-10, lin_tol=1e-13)
    print("oracle increments", inc_o, "gpu", rec, flush=True)
    assert rec["converged"] and all(st == 0 for st in rec["linear_status"])
    assert abs(len(rec["increments"]) - len(inc_o)) <= 1
    assert_close(U.cpu().numpy(), Uo, 1e-9)
    assert_close(P.cpu().numpy(), Po, 1e-9)
    ns.close()


def test_newton_green_taylor_time_steps_against_oracle(gpu):
    """Backward-Euler steps of the Green-Taylor vortex (amplitude Re = 100,
    nu = 1, Section 4.1) on 8 x 8 x 2 with its face means on the boundary at
    each time, Newton at every step from the previous step: against the
    oracle's chain of Newton solves, U and P within 1e-9 at every step."""
    from oracle import newton as onewton
    from paper_2101_03777_amd.newton import NewtonSolver
    from synth.fields import GreenTaylor2D, face_means
    gt = GreenTaylor2D(amp=100.0, nu=1.0)
    coords, elems = synth.square_mesh(8)
    bf = wl.exterior_face_list(elems)
    fi = wl.interior_face_list(elems)
    dt = 0.002 / 64.0
    f = np.zeros((len(elems), 2))
    u0 = gt.u(coords[fi].mean(axis=1), 0.0)
    ns = NewtonSolver(coords, elems, 1.0 / dt, 1.0)
    Ug, Uo = dev(u0), u0
    for n in range(1, 4):
        g = face_means(coords, bf, lambda x: gt.u(x, n * dt))
        Uo, Po, inc_o = onewton.newton(coords, elems, 1.0 / dt, 1.0, f, gbnd=g, u_prev=Uo, u0=Uo, tol=1e-11)
        ns.set_boundary(g)
        Ug, Pg, rec = ns.solve(f, u_prev=Ug, u0=Ug, tol=1e-11, lin_tol=1e-13)
        assert rec["converged"], rec
        assert_close(Ug.cpu().numpy(), Uo, 1e-9)
        assert_close(Pg.cpu().numpy(), Po, 1e-9)
    ns.close()


def test_newton_green_taylor_3d_time_steps_against_oracle(gpu):
    """The 3D Green-Taylor vortex of Section 4.1's 3D Navier-Stokes test
    (amplitude Re = 100, nu = 1, third component zero) on 3^3 x 6 tetrahedra,
    face means on the boundary at each time, two backward-Euler steps with
    Newton from the previous step: against the oracle's chain of Newton solves
    (12 x 12 local inverses on the GPU, general inverses in the oracle), U and
    P within 1e-9 at every step."""
    from oracle import newton as onewton
    from paper_2101_03777_amd.newton import NewtonSolver
    from synth.fields import GreenTaylor3D, face_means
    gt = GreenTaylor3D(amp=100.0, nu=1.0)
    coords, elems = synth.cube_mesh(3)
    bf = wl.exterior_face_list(elems)
    fi = wl.interior_face_list(elems)
    dt = 0.01 / 9.0
    f = np.zeros((len(elems), 3))
    u0 = face_means(coords, fi, lambda x: gt.u(x, 0.0))
    ns = NewtonSolver(coords, elems, 1.0 / dt, 1.0)
    Ug, Uo = dev(u0), u0
    for n in range(1, 3):
        g = face_means(coords, bf, lambda x: gt.u(x, n * dt))
        Uo, Po, inc_o = onewton.newton(coords, elems, 1.0 / dt, 1.0, f, gbnd=g, u_prev=Uo, u0=Uo, tol=1e-11)
        ns.set_boundary(g)
        # linear tolerance 1e-12: on this 54-element mesh BiCGStab(2) in FP64
        # stagnates before 1e-13
        Ug, Pg, rec = ns.solve(f, u_prev=Ug, u0=Ug, tol=1e-10, lin_tol=1e-12, lin_maxit=50000)
        print(f"3D Green-Taylor step {n}: oracle {len(inc_o)} Newton iterations, GPU {rec}", flush=True)
        assert rec["converged"], rec
        assert_close(Ug.cpu().numpy(), Uo, 1e-9)
        assert_close(Pg.cpu().numpy(), Po, 1e-9)
    ns.close()


def _paper_3d_ns_table():
    rows = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_3d_ns_green_taylor.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                n, dt, h, eu, ep = line.split()
                rows[int(n)] = dict(dt=float(dt), h=float(h), eu=float(eu), ep=float(ep))
    return rows


def _green_taylor_errors_3d(gpu, n):
    """The 3D Green-Taylor vortex to t = 0.01 on n^3 x 6 tetrahedra with
    dt = 0.01 / n^2, through the Newton driver; velocity error at the face
    centroids with the lumped mass |K|/4 of the two elements, pressure error at
    the element centroids weighted by |K|, both without their means."""
    from paper_2101_03777_amd.newton import NewtonSolver
    from synth.fields import GreenTaylor3D, face_means
    gt = GreenTaylor3D(amp=100.0, nu=1.0)
    coords, elems = synth.cube_mesh(n)
    bf, fi = wl.exterior_face_list(elems), wl.interior_face_list(elems)
    nsteps = n * n
    dt = 0.01 / nsteps
    ns = NewtonSolver(coords, elems, 1.0 / dt, 1.0)
    Ug = dev(face_means(coords, fi, lambda x: gt.u(x, 0.0)))
    f = np.zeros((len(elems), 3))
    for k in range(1, nsteps + 1):
        ns.set_boundary(face_means(coords, bf, lambda x: gt.u(x, k * dt)))
        Ug, Pg, rec = ns.solve(f, u_prev=Ug, u0=Ug, tol=1e-9, lin_tol=1e-11)
        assert rec["converged"], (k, rec)
    ns.close()
    X = coords[elems]
    vol = np.abs(np.einsum("ij,ij->i", X[:, 1] - X[:, 0], np.cross(X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]))) / 6.0
    fidx = {tuple(v): i for i, v in enumerate(fi)}
    mass = np.zeros(len(fi))
    for e, el in enumerate(elems):
        for j in range(4):
            key = tuple(sorted(np.delete(el, j)))
            if key in fidx:
                mass[fidx[key]] += vol[e] / 4.0
    eu = np.sqrt((mass[:, None] * (Ug.cpu().numpy() - gt.u(coords[fi].mean(axis=1), 0.01)) ** 2).sum())
    pe = gt.p(X.mean(axis=1), 0.01)
    ph = Pg.cpu().numpy()
    dp = (ph - (vol * ph).sum() / vol.sum()) - (pe - (vol * pe).sum() / vol.sum())
    return eu, np.sqrt((vol * dp ** 2).sum())


def test_green_taylor_3d_reproduces_the_paper_table(gpu):
    """Section 4.1, 3D Navier-Stokes Green-Taylor table: on 8^3 and 16^3 cubes
    x 6 tetrahedra with the printed time steps, the GPU path (boundary data,
    Newton driver, 3D Newton steps with 12 x 12 local inverses, BiCGStab(2))
    gives the printed velocity and pressure errors within 5% and their ratio
    within 0.05 (tests/golden/paper_3d_ns_green_taylor.txt)."""
    paper = _paper_3d_ns_table()
    errs = {}
    for n in (8, 16):
        assert abs(0.01 / (n * n) - paper[n]["dt"]) <= 0.01 * paper[n]["dt"]
        errs[n] = _green_taylor_errors_3d(gpu, n)
        print(f"3D Green-Taylor n={n}: errors u {errs[n][0]:.4g} p {errs[n][1]:.4g}, paper {paper[n]}", flush=True)
        assert abs(errs[n][0] - paper[n]["eu"]) <= 0.05 * paper[n]["eu"]
        assert abs(errs[n][1] - paper[n]["ep"]) <= 0.05 * paper[n]["ep"]
    for k in (0, 1):
        key = "eu" if k == 0 else "ep"
        ours = np.log2(errs[8][k] / errs[16][k])
        theirs = np.log2(paper[8][key] / paper[16][key])
        assert abs(ours - theirs) <= 0.05, (key, ours, theirs)


def test_green_taylor_3d_stokes_time_steps_against_oracle(gpu):
    """Section 4.1's 3D Green-Taylor Stokes test on 4^3 x 6 tetrahedra with the
    printed time step (1e-4, 100 steps to t = 0.01): unforced transient Stokes
    with the vortex's face means on the boundary at every step, one hybridised
    CG solve per step, against the oracle's chain of coupled direct solves; U
    and P within 1e-9 at the final time."""
    from synth.fields import GreenTaylor3D, face_means
    gt = GreenTaylor3D(amp=100.0, nu=1.0)
    coords, elems = synth.cube_mesh(4)
    bf, fi = wl.exterior_face_list(elems), wl.interior_face_list(elems)
    dt = 1e-4
    f = np.zeros((len(elems), 3))
    Uo = face_means(coords, fi, lambda x: gt.u(x, 0.0))
    s = gpu.System(coords, elems, 1.0 / dt, 1.0)
    Ug = dev(Uo)
    for k in range(1, 101):
        g = face_means(coords, bf, lambda x: gt.u(x, k * dt))
        P = cr.make_problem(coords, elems, 1.0 / dt, 1.0, f, u_prev=Uo, gbnd=g)
        Uo, Po = cr.solve_coupled(P)
        s.set_boundary(g)
        s.eliminate(dev(f), Ug)
        info = s.solve("pcg", "fp64", tol=1e-12, warm_start=k > 1)
        assert info["status"] == 0
        Ug, Pg = s.recover()
    print(f"final |U| {np.abs(Uo).max():.3f}", flush=True)
    assert_close(Ug.cpu().numpy(), Uo, 1e-9)
    assert_close(Pg.cpu().numpy(), Po, 1e-9)
    s.close()

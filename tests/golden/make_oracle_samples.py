"""Writes the stored oracle solutions of the two full-size transient-Stokes
workloads, as samples: tests/golden/oracle_<workload>.npz.

Calls only the oracle (oracle/) and the seeded input generators (synth/); no
value comes from the HIP library.  The full-size oracle solves take minutes to
hours on one CPU core, so they are run once and stored:

  square512j  2D, 512 x 512 cells x 2 triangles, jitter 0.2 h (seed 0),
              mu = 1000, nu = 1: the coupled system of Section 3.1 (eq. syslin)
              solved by sparse LU (SuperLU) with three steps of iterative
              refinement, the oracle's primary result; certificate: the coupled
              residual and max_K |D_K U|.
  cube64      3D, 64^3 cubes x 6 tetrahedra, mu = 100, nu = 1: sparse LU does
              not fit (3D fill), so the hybrid branch of the oracle: element-wise
              elimination in its general form (Section 3.2 items 4-5), plain
              Jacobi-preconditioned CG on G W = S to ||S - G W|| <= 1e-13 ||S||,
              element-wise recovery (items 2, 4), and two certificates from the
              oracle's own matrices: ||S - G W|| / ||S|| and the coupled residual
              ||R - A U - D^t P|| / ||R|| with max_K |D_K U|.

Stored per workload: the sampled canonical face ids and U there, the sampled
element ids and P there (P[0] = 0, element 0 pinned), the 2-norm and max-norm of
the whole U and P, and the solve record.  The samples are 8192 seeded random
faces and elements plus every face of elements 0..63 and those elements (the
pinned element K0 = 0 sits in the corner, next to the boundary).

  ns256       2D steady Navier-Stokes Newton step, 256 x 256 cells x 2, nu = 0.01,
              seeded divergence-free linearisation velocity: the coupled system
              (A with the Jacobian of the convection form) by sparse LU with three
              refinement steps.

Usage: python tests/golden/make_oracle_samples.py square512j|cube64|ns256
"""
from __future__ import annotations

import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N_SAMPLE = 8192
N_CORNER = 64


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def sample_ids(mesh):
    rng = np.random.default_rng(12345)
    faces = rng.choice(mesh.nf, size=min(N_SAMPLE, mesh.nf), replace=False)
    elems = rng.choice(mesh.ne, size=min(N_SAMPLE, mesh.ne), replace=False)
    corner = np.arange(min(N_CORNER, mesh.ne))
    cf = mesh.elem_face[corner].ravel()
    faces = np.unique(np.concatenate([faces, cf[cf >= 0]]))
    elems = np.unique(np.concatenate([elems, corner]))
    return faces.astype(np.int32), elems.astype(np.int32)


def store(name, mesh, U, Pk, record):
    fi, ei = sample_ids(mesh)
    path = os.path.join(HERE, f"oracle_{name}.npz")
    np.savez_compressed(path, face_ids=fi, U=U[fi], elem_ids=ei, P=Pk[ei],
                        U_norm2=np.linalg.norm(U), U_max=np.abs(U).max(),
                        P_norm2=np.linalg.norm(Pk), P_max=np.abs(Pk).max(),
                        n_int_faces=mesh.nf, n_elements=mesh.ne, dim=mesh.d,
                        record=json.dumps(record))
    print("wrote", path, json.dumps(record), flush=True)


def square512j():
    import synth.workloads as wl
    from oracle import cr
    w = wl.square512j()
    t0 = time.perf_counter()
    P = cr.make_problem(w["coords"], w["elems"], w["mu"], w["nu"], w["fbar"])
    U, Pk = cr.solve_coupled(P, refine=3)
    t1 = time.perf_counter()
    res, div = cr.coupled_residual(P, U, Pk)
    rec = {"workload": "square512j", "method": "coupled sparse LU (SuperLU, COLAMD), 3 refinement steps", "seconds": round(t1 - t0, 1),
           "coupled_rel_residual": res, "max_div_rel": div, "cpu": cpu_model()}
    store("square512j", P.mesh, U, Pk, rec)


def cube64():
    import synth.workloads as wl
    from oracle import cr, krylov
    w = wl.cube64()
    t0 = time.perf_counter()
    P = cr.make_problem(w["coords"], w["elems"], w["mu"], w["nu"], w["fbar"])
    H = cr.eliminate(P)
    t1 = time.perf_counter()
    print(f"eliminated in {t1 - t0:.0f} s", flush=True)

    def progress(it, rel):
        if it % 200 == 0:
            print(f"pcg {it} {rel:.3e} {time.perf_counter() - t1:.0f} s", flush=True)

    W, iters, hist = krylov.pcg(H.G, H.S, tol=1e-13, maxit=60000, callback=progress)
    t2 = time.perf_counter()
    U, Pk, _ = cr.recover(P, H, W)
    t3 = time.perf_counter()
    true_res = np.linalg.norm(H.S - H.G @ W) / np.linalg.norm(H.S)
    res, div = cr.coupled_residual(P, U, Pk)
    rec = {"workload": "cube64", "method": "hybrid: general elimination, Jacobi PCG on G, recovery",
           "pcg_iterations": int(iters), "pcg_tol": 1e-13, "hybrid_rel_residual": true_res,
           "coupled_rel_residual": res, "max_div_rel": div, "seconds_eliminate": round(t1 - t0, 1),
           "seconds_pcg": round(t2 - t1, 1), "seconds_recover": round(t3 - t2, 1), "cpu": cpu_model()}
    store("cube64", P.mesh, U, Pk, rec)


def ns256():
    import synth.workloads as wl
    from oracle import cr
    w = wl.ns256()
    t0 = time.perf_counter()
    P = cr.make_problem(w["coords"], w["elems"], w["mu"], w["nu"], w["fbar"], ulin=w["ulin"])
    U, Pk = cr.solve_coupled(P, refine=3)
    t1 = time.perf_counter()
    res, div = cr.coupled_residual(P, U, Pk)
    rec = {"workload": "ns256", "method": "coupled sparse LU (SuperLU, COLAMD), 3 refinement steps",
           "seconds": round(t1 - t0, 1), "coupled_rel_residual": res, "max_div_rel": div, "cpu": cpu_model()}
    store("ns256", P.mesh, U, Pk, rec)


if __name__ == "__main__":
    {"square512j": square512j, "cube64": cube64, "ns256": ns256}[sys.argv[1]]()

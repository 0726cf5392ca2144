#!/usr/bin/env python3
"""Benchmark of the hybridised Crouzeix-Raviart transient-Stokes solve on one MI355X.

Workload (default): 2D transient Stokes on the unit square, 512 x 512 cells cut
into 2 triangles (524,288 elements), interior vertices jittered by up to 0.2 h
(seeded), nu = 1, mu = 1/dt = 1000, homogeneous Dirichlet, right-hand side from
a seeded smooth manufactured velocity; hybridised SPD system of 1,570,816
unknowns solved to ||S - G W|| <= 1e-10 ||S|| (FP64 residual) by Jacobi-scaled
CG with G applied from its element factors: FP32 CG iterations with FP64
residual replacements (--precision fp64: FP64 iterations).

One step = the whole hot path on device-resident inputs: element-wise
elimination and assembly of G and S, Krylov solve, element-wise recovery of U
and P.  The value is steps (solves) per second.  Also reported: the dominant
kernel's achieved bandwidth against the HBM peak (timed with HIP events on the
solver's stream), the same kernel of the assembled operator, the other Krylov
precision, the FP64 MINRES solve of the
original coupled system on the same GPU, and the CPU oracle on a bounded
sample of the workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# dominant kernel of the timed path: the element kernel of the element-form CG
KERNEL = {"fp64": "k_ec1<2, double>", "fp32_ir": "k_ec1<2, float>"}
METRIC = "hybridised solve time & SpMV HBM GB/s vs coupled solve; solves/s, p99 latency"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# source of the dominant kernel: its own code, the shared iteration start and
# stopping logic, the structs it reads, and the row/element helpers
KERNEL_PARTS = ("struct KState", "struct CgSys", "struct Decision", "Decision decide(", "void record_decision(",
                "bool cg_head(", "void ec1_pass(", "void ec1_body(", "k_ec1(CgSys S")


def _block(text, key):
    """Text of the definition that starts at `key` up to its matching closing brace."""
    i = text.index(key)
    j = text.index("{", i)
    depth = 0
    for k in range(j, len(text)):
        depth += {"{": 1, "}": -1}.get(text[k], 0)
        if depth == 0:
            return text[i:k + 1]
    raise ValueError(key)


def source_digest():
    """Digest of the source the dominant kernel is built from (not of unrelated
    code in the same files), so counter profiles stay valid across other edits."""
    csrc = os.path.join(ROOT, "paper_2101_03777_amd", "csrc")
    with open(os.path.join(csrc, "krylov.hip")) as fh:
        kry = fh.read()
    h = hashlib.sha256()
    for key in KERNEL_PARTS:
        h.update(_block(kry, key).encode())
    with open(os.path.join(csrc, "rowkern.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_digest") != source_digest():
        return None
    return rec.get("bytes_per_launch")


def cpu_oracle_baseline(ne_target, mu, nu, n_sample=128):
    """Oracle (sparse LU of the coupled system, FP64) on a 128x128x2 sample of the
    same workload family, scaled linearly in the element count to the target."""
    import synth.workloads as wl
    from oracle import cr
    w = wl.square(n_sample, mu=mu, nu=nu, jitter=0.2, seed=0, quad=3)
    t0, c0 = time.perf_counter(), time.process_time()
    P = cr.make_problem(w["coords"], w["elems"], w["mu"], w["nu"], w["fbar"])
    cr.solve_coupled(P)
    wall, cpu = time.perf_counter() - t0, time.process_time() - c0
    ne_s = len(w["elems"])
    t_scaled = wall * ne_target / ne_s
    return {"value": 1.0 / t_scaled, "unit": "solves/s", "cores": max(1, round(cpu / wall)),
            "kind": "oracle",
            "sample": (f"oracle coupled sparse-LU solve (assembly + SuperLU + back-substitution, FP64) of the same "
                       f"workload on {n_sample}x{n_sample}x2 elements ({ne_s}), {wall:.2f} s wall, scaled linearly "
                       f"by element count to {ne_target} elements (sparse LU grows faster, so this favours the CPU)")}


def run_serving(args):
    """Continuous-batching serving run: transient-Stokes time-step requests of
    sessions arriving as a Poisson process (N x N x 2 meshes, N log-uniform in
    [32, 512], dt uniform in [1e-3, 1e-1], 1 to 20 steps per session), admitted by
    a device-memory budget, solved to 1e-9 in one shared batch."""
    import synth.workloads as wl
    from paper_2101_03777_amd.serve import Server, Session
    t0 = time.perf_counter()
    ss = wl.serving_sessions(args.serve_requests, seed=1, rate=args.serve_rate)
    log(f"serving inputs: {len(ss)} sessions, {sum(d['steps'] for d in ss)} requests, "
        f"{time.perf_counter() - t0:.1f} s")
    sessions = [Session(i, d["coords"], d["elems"], d["dt"], d["nu"], d["fbar"], d["steps"], d["arrival"])
                for i, d in enumerate(ss)]
    srv = Server(hbm_budget=int(args.serve_budget_gb * (1 << 30)), max_active=128, precision=args.serve_precision,
                 tol=1e-9)
    st = srv.run(sessions)
    srv.close()
    recs = st.pop("records")
    st.update(precision=args.serve_precision, tol=1e-9, arrival_rate_sessions_per_s=args.serve_rate,
              total_iterations=int(sum(r["iters"] for r in recs)),
              workload="transient Stokes time steps, N x N x 2 meshes, N log-uniform in [32, 512], dt uniform in "
                       "[1e-3, 1e-1] (mu = 1/dt), 1-20 steps per session, Poisson session arrivals, seed 1")
    return {k: (float(f"{v:.4g}") if isinstance(v, float) else v) for k, v in st.items()}


def run_other_workloads(crh, wl, torch):
    """The 3D and Navier-Stokes workloads through the same library calls (not
    the benchmark line): 64^3 cubes x 6 tetrahedra transient Stokes (mu = 100),
    and the steady Navier-Stokes Newton step on 256x256x2 (nu = 0.01)."""
    out = {}
    t0 = time.perf_counter()
    w = wl.cube64()
    log(f"64^3 x 6 inputs: {time.perf_counter() - t0:.1f} s")
    s = crh.System(w["coords"], w["elems"], w["mu"], w["nu"])
    s.eliminate(torch.from_numpy(w["fbar"]).cuda())
    rec = {"workload": "3D transient Stokes, unit cube 64^3 cubes x 6 Kuhn tetrahedra, nu=1, mu=100, "
                       "manufactured RHS, CG to rel residual 1e-10",
           "elements": len(w["elems"]), "unknowns": s.n_int_faces * 3}
    for prec in ("fp32_ir", "fp64"):
        info = s.solve("pcg", prec, tol=1e-10)
        rec[prec] = {"time_to_tol_ms": round(info["t_solve_ms"], 2), "iters": info["iters"],
                     "rel_residual": info["rel_residual"], "fp64_fallback": info["fp64_fallback"]}
        log(f"64^3 x 6 {prec}: {info['t_solve_ms']:.1f} ms, {info['iters']} iterations")
    ms, by = s.time_spmv("fp32_ir", reps=100)
    rec["k_ec1<3, float>"] = {"avg_launch_us": round(ms * 1e3, 2), "algorithmic_bytes_per_launch": int(by),
                              "achieved_GBps": round(by / (ms * 1e-3) / 1e9, 1)}
    s.close()
    out["stokes3d_64"] = rec
    t0 = time.perf_counter()
    w = wl.ns256()
    log(f"NS 256x256x2 inputs: {time.perf_counter() - t0:.1f} s")
    s = crh.System(w["coords"], w["elems"], 0.0, w["nu"], problem="ns")
    s.eliminate(torch.from_numpy(w["fbar"]).cuda(), None, torch.from_numpy(w["ulin"]).cuda())
    info = s.solve("bicgstab2", "fp64", tol=1e-9, maxit=600000, raise_on_error=False)
    out["ns_newton_256"] = {
        "workload": "2D steady Navier-Stokes Newton step, 256x256x2, nu=0.01, seeded linearisation velocity, "
                    "E_K from the M1/M2 partition; BiCGStab(2), FP64, to rel residual 1e-9",
        "elements": len(w["elems"]), "unknowns": s.n_int_faces * 2, "status": info["status"],
        "time_to_tol_ms": round(info["t_solve_ms"], 1), "iters": info["iters"],
        "products_with_G": 4 * info["iters"], "rel_residual": info["rel_residual"]}
    log(f"NS 256x256x2 BiCGStab(2): {info['t_solve_ms']:.0f} ms, {info['iters']} iterations, "
        f"status {info['status']}")
    s.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32_ir", choices=["fp32_ir", "fp64"],
                    help="Krylov arithmetic of the timed path (the other one is reported beside it)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--n", type=int, default=512, help="cells per side (512 = the benchmark workload)")
    ap.add_argument("--no-coupled", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--coupled-maxit", type=int, default=60000)
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="time-step requests of the serving run (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=2.5,
                    help="session arrivals per second (Poisson); 2.5 offers about 26 requests/s, below saturation")
    ap.add_argument("--serve-budget-gb", type=float, default=8.0, help="device-memory budget for admission")
    ap.add_argument("--serve-precision", default="fp32_ir", choices=["fp32_ir", "fp64"])
    ap.add_argument("--no-other", action="store_true",
                    help="skip the 64^3 x 6 and the Navier-Stokes 256x256x2 solves reported beside the benchmark")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only build the system and time the dominant kernel (for counter collection)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run 20 device-to-device copies of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2101_03777_amd as crh
    import synth.workloads as wl

    crh.load()
    torch.cuda.set_device(0)
    if args.copy_bytes:
        a = torch.empty(args.copy_bytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(20):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_bytes, "copies": 20}), flush=True)
        return
    mu, nu, n = 1000.0, 1.0, args.n
    t0 = time.perf_counter()
    w = wl.square(n, mu=mu, nu=nu, jitter=0.2, seed=0, quad=3)
    log(f"inputs {n}x{n}x2: {len(w['elems'])} elements, {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    s = crh.System(w["coords"], w["elems"], mu, nu)
    t_topo = time.perf_counter() - t0
    log(f"topology + upload: {t_topo:.2f} s, {s.n_int_faces} interior faces")
    fbar = torch.from_numpy(w["fbar"]).cuda()
    stream = torch.cuda.current_stream()
    if args.kernel_only:
        s.eliminate(fbar)
        ms_k, bytes_k = s.time_spmv(args.precision, reps=200)
        print(json.dumps({"kernel": KERNEL[args.precision], "precision": args.precision, "avg_us": ms_k * 1e3,
                          "algorithmic_bytes": bytes_k, "GBps": bytes_k / (ms_k * 1e-3) / 1e9}), flush=True)
        s.close()
        return

    def step(record):
        e0, e1, e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
        e0.record(stream)
        s.eliminate(fbar)
        e1.record(stream)
        info = s.solve("pcg", args.precision, tol=args.tol)
        e2.record(stream)
        U, P = s.recover()
        e3.record(stream)
        e3.synchronize()
        if record is not None:
            record.append(dict(elim_ms=e0.elapsed_time(e1), solve_ms=e1.elapsed_time(e2),
                               recover_ms=e2.elapsed_time(e3), total_ms=e0.elapsed_time(e3), **info))
        return U, P

    for k in range(args.warmup):
        step(None)
        log(f"warmup {k + 1}/{args.warmup} done")
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(recs)
        log(f"step {k + 1}/{args.steps}: {recs[-1]['total_ms']:.1f} ms, {recs[-1]['iters']} iterations, "
            f"rel residual {recs[-1]['rel_residual']:.2e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([r["total_ms"] for r in recs])
    last = recs[-1]

    # dominant kernel: the element kernel of the CG iteration (operator applied
    # from element factors, fused with the direction update), timed with HIP
    # events on the solver's stream
    ms_k, bytes_k = s.time_spmv(args.precision, reps=200)
    gbs = bytes_k / (ms_k * 1e-3) / 1e9
    traffic = measured_traffic(f"square{n}j", "ec1_" + args.precision)
    roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": KERNEL[args.precision],
                "avg_launch_us": round(ms_k * 1e3, 2), "algorithmic_bytes_per_launch": int(bytes_k)}
    log(f"dominant kernel: {ms_k * 1e3:.2f} us/launch, {gbs:.0f} GB/s ({100 * gbs / HBM_PEAK_GBS:.1f}% of HBM peak)")
    ms_a, bytes_a = s.time_spmv(args.precision, reps=200, operator="assembled")
    assembled = {"kernel": f"k_cg_spmv<2, {'float' if args.precision == 'fp32_ir' else 'double'}, 0>",
                 "avg_launch_us": round(ms_a * 1e3, 2), "algorithmic_bytes_per_launch": int(bytes_a),
                 "achieved_GBps": round(bytes_a / (ms_a * 1e-3) / 1e9, 1)}
    info_a = s.solve("pcg", args.precision, tol=args.tol, operator="assembled")
    assembled.update(time_to_tol_ms=round(info_a["t_solve_ms"], 3), iters=info_a["iters"])
    log(f"assembled operator: {ms_a * 1e3:.2f} us/launch; solve {info_a['t_solve_ms']:.1f} ms, "
        f"{info_a['iters']} iterations")

    # accuracy diagnostic: copy mismatch of the recovered velocity (equals the residual)
    s.solve("pcg", args.precision, tol=args.tol)
    U, P, J = s.recover(jump=True)
    torch.cuda.synchronize()

    # the other Krylov precision on the same solve
    other = "fp64" if args.precision == "fp32_ir" else "fp32_ir"
    s.eliminate(fbar)
    info64 = s.solve("pcg", other, tol=args.tol)
    log(f"{other} solve: {info64['t_solve_ms']:.1f} ms, {info64['iters']} iterations "
        f"({info64['fp32_iters']} in FP32, fallback to FP64: {info64['fp64_fallback']})")

    coupled = None
    if not args.no_coupled:
        Uc, Pc, ci = s.coupled_solve(tol=args.tol, maxit=args.coupled_maxit, raise_on_error=False)
        torch.cuda.synchronize()
        diff = (torch.linalg.norm(Uc - U) / torch.linalg.norm(U)).item()
        coupled = {"method": "FP64 MINRES, diagonal block preconditioner diag(A) + diag(D diag(A)^-1 D^t)",
                   "time_ms": round(ci["t_solve_ms"], 2), "iters": ci["iters"],
                   "rel_residual": ci["rel_residual"], "converged": ci["status"] == 0,
                   "rel_diff_U_vs_hybrid": diff}
        log(f"coupled MINRES: {ci['t_solve_ms']:.1f} ms, {ci['iters']} iterations, "
            f"residual {ci['rel_residual']:.2e}, converged={ci['status'] == 0}")

    serving = None
    if args.serve_requests > 0:
        serving = run_serving(args)
        log(f"serving: {serving['requests']} requests, {serving['solves_per_s']:.1f} solves/s, "
            f"p50 {serving['p50_ms']:.1f} ms, p99 {serving['p99_ms']:.1f} ms")

    others = None if args.no_other else run_other_workloads(crh, wl, torch)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_oracle_baseline(len(w["elems"]), mu, nu)
        log(f"cpu oracle: {cpu['value']:.4f} solves/s ({cpu['sample']})")

    out = {
        "metric": METRIC,
        "value": round(args.steps / wall, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "fp32_ir" else "f64",
        "data": "synthetic",
        "config": {"workload": f"2D transient Stokes, unit square {n}x{n} cells x2 triangles, jitter 0.2h (seed 0), "
                               f"nu=1, mu=1/dt=1000, manufactured RHS; hybridised SPD system, Jacobi-scaled CG "
                               f"({'FP32 inside FP64 iterative refinement' if args.precision == 'fp32_ir' else 'FP64'})"
                               f" with G applied from element factors, to rel residual {args.tol:g}",
                   "elements": len(w["elems"]),
                   "unknowns": s.n_int_faces * 2, "tol": args.tol, "precision": args.precision},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "time_to_tol_ms": round(float(np.median([r["solve_ms"] for r in recs])), 3),
        "iters": last["iters"], "outer_iters": last["outer_iters"], "rel_residual": last["rel_residual"],
        "copy_mismatch": J.item(),
        "eliminate_ms": round(float(np.median([r["elim_ms"] for r in recs])), 3),
        "recover_ms": round(float(np.median([r["recover_ms"] for r in recs])), 3),
        "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "topology_host_s": round(t_topo, 3),
        f"{other}_time_to_tol_ms": round(info64["t_solve_ms"], 3), f"{other}_iters": info64["iters"],
        f"{other}_fp32_iters": info64["fp32_iters"], f"{other}_fp64_fallback": info64["fp64_fallback"],
        "assembled_operator": assembled,
        "coupled_gpu": coupled,
        "speedup_vs_coupled": (round(coupled["time_ms"] / float(np.median([r['solve_ms'] for r in recs])), 2)
                               if coupled else None),
        "serving": serving,
        "other_workloads": others,
    }
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark of the hybridised Crouzeix-Raviart transient-Stokes solve on one MI355X.

Headline workload (default, the largest configuration that fits one GPU): 3D
transient Stokes on the unit cube, 64^3 cubes each cut into 6 Kuhn tetrahedra
(1,572,864 elements, 9,363,456 face unknowns), nu = 1, mu = 1/dt = 100,
homogeneous Dirichlet, right-hand side from a seeded smooth manufactured
velocity; hybridised SPD system solved to ||S - G W|| <= 1e-9 ||S|| (FP64
residual) by CG with Jacobi scaling and an aggregate coarse correction, G
applied from its element factors, FP32 iterations inside FP64 residual
replacement (--precision fp64: FP64 iterations).

One step = the whole hot path on device-resident inputs: element-wise
elimination and assembly of G and S, Krylov solve, element-wise recovery of U
and P.  The value is steps (solves) per second.

Also reported on the same line: the dominant kernel's achieved bandwidth
against the HBM peak and against a measured device copy (HIP events on the
solver's stream) with the counter-measured traffic; the error of U and P
against the stored FP64 oracle solution; the Jacobi-only solve and the FP64
MINRES solve of the original coupled system on the same GPU (like-for-like
speedup); the FP64-iteration solve; the 2D 512x512x2 workload (its working set
fits the 256 MB Infinity Cache, so its bandwidth is labelled MALL-resident
possible); the steady Navier-Stokes Newton step; the serving run; and the CPU
oracle on a bounded sample of the headline workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cube64|square512j]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "hybridised solve time & SpMV HBM GB/s vs coupled solve; solves/s, p99 latency"

WORKLOADS = {
    # tol: the residual tolerance at which U and P match the FP64 oracle to 1e-9
    # (2-norm and max-norm, measured against the stored oracle solution);
    # config_tol: the residual tolerance the configuration states, timed beside it
    "cube64": dict(
        dim=3, mu=100.0, nu=1.0, tol=1e-13, config_tol=1e-9, coupled_maxit=40000,
        label="3D transient Stokes, unit cube 64^3 cubes x 6 Kuhn tetrahedra, nu=1, mu=1/dt=100, manufactured "
              "RHS; hybridised SPD system, CG with Jacobi scaling and aggregate coarse correction, G applied from "
              "element factors",
        bound="hbm"),
    "square512j": dict(
        dim=2, mu=1000.0, nu=1.0, tol=1e-11, config_tol=1e-10, coupled_maxit=100000,
        label="2D transient Stokes, unit square 512x512 cells x2 triangles, jitter 0.2h (seed 0), nu=1, "
              "mu=1/dt=1000, manufactured RHS; hybridised SPD system, CG with Jacobi scaling and aggregate coarse "
              "correction, G applied from element factors",
        bound="MALL-resident possible"),
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_name(dim, precision):
    return f"k_ec1<{dim}, {'float' if precision == 'fp32_ir' else 'double'}>"


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


def measured_traffic(workload, precision):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_ec1_{precision}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_digest") != source_digest():
        return None
    return rec.get("bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def load_workload(name):
    import synth.workloads as wl
    return {"cube64": wl.cube64, "square512j": wl.square512j}[name]()


def oracle_error(name, U, P):
    """Error of U and P against the stored FP64 oracle solution of the workload
    (tests/golden/oracle_<name>.npz: written by tests/golden/make_oracle_samples.py
    from the oracle alone), on its sampled faces and elements."""
    import numpy as np
    import torch
    path = os.path.join(ROOT, "tests", "golden", f"oracle_{name}.npz")
    if not os.path.exists(path):
        return {"status": "parity unpinned: no stored oracle solution for this workload"}
    z = np.load(path)
    fi = torch.from_numpy(z["face_ids"].astype(np.int64)).to(U.device)
    ei = torch.from_numpy(z["elem_ids"].astype(np.int64)).to(P.device)
    Us = U.index_select(0, fi).cpu().numpy()
    Ps = P.index_select(0, ei).cpu().numpy()
    Uo, Po = z["U"], z["P"]
    rec = json.loads(str(z["record"]))
    return {"U_rel2": float(np.linalg.norm(Us - Uo) / np.linalg.norm(Uo)),
            "U_max_rel": float(np.abs(Us - Uo).max() / float(z["U_max"])),
            "P_rel2": float(np.linalg.norm(Ps - Po) / np.linalg.norm(Po)),
            "P_max_rel": float(np.abs(Ps - Po).max() / float(z["P_max"])),
            "sample": f"{len(fi)} faces and {len(ei)} elements (seeded, plus the pinned element's corner)",
            "oracle": rec.get("method"), "oracle_record": {k: rec[k] for k in rec if k not in ("workload", "method")}}


def copy_bandwidth(torch, nbytes=1 << 30, reps=20):
    """Device-to-device copy of nbytes, timed with HIP events: bytes read + written / time."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def run_c1(crh, torch):
    """The smallest configuration (16x16x2, mu = 100): eliminate + CG (FP64, to
    1e-12) + recover on the GPU; returns the record and the solution, which the
    oracle leg compares with the oracle's coupled direct solve."""
    import synth.workloads as wl
    w = wl.square16()
    s = crh.System(w["coords"], w["elems"], w["mu"], w["nu"])
    f = torch.from_numpy(w["fbar"]).cuda()
    stream = torch.cuda.current_stream()
    ts = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.eliminate(f)
        info = s.solve("pcg", "fp64", tol=1e-12)
        U, P = s.recover()
        e1.record(stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    s.close()
    rec = {"workload": "2D transient Stokes, 16x16x2 (512 elements), nu = 1, mu = 100, manufactured RHS; "
                       "eliminate + CG (FP64, coarse correction) to 1e-12 + recover",
           "ms_per_solve": round(min(ts), 3), "iters": info["iters"], "rel_residual": info["rel_residual"]}
    return rec, U.cpu().numpy(), P.cpu().numpy()


def c1_oracle_leg(rec, U, P):
    """Oracle leg of the smallest configuration: the coupled direct solve (FP64,
    one thread) timed on this host, and the GPU solution's error against it."""
    import numpy as np
    import synth.workloads as wl
    from oracle import cr
    from threadpoolctl import threadpool_limits
    w = wl.square16()
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        Pr = cr.make_problem(w["coords"], w["elems"], w["mu"], w["nu"], w["fbar"])
        Uo, Po = cr.solve_coupled(Pr)
        wall = time.perf_counter() - t0
    rec = dict(rec)
    rec["oracle_ms"] = round(1e3 * wall, 1)
    rec["err_vs_oracle"] = {
        "U_rel2": float(np.linalg.norm(U - Uo) / np.linalg.norm(Uo)),
        "U_max_rel": float(np.abs(U - Uo).max() / np.abs(Uo).max()),
        "P_rel2": float(np.linalg.norm(P - Po) / np.linalg.norm(Po)),
        "P_max_rel": float(np.abs(P - Po).max() / np.abs(Po).max())}
    return rec


def cpu_oracle_baseline(ne_target, n_sample=12):
    """The oracle's primary result (assembly and sparse LU of the coupled system,
    FP64, one thread) on a bounded sample of the headline workload family: the
    same 3D transient Stokes problem on n_sample^3 cubes x 6 tetrahedra, timed on
    this host and scaled linearly in the element count to the target."""
    import synth.workloads as wl
    from oracle import cr
    from threadpoolctl import threadpool_limits
    w = wl.cube(n_sample, mu=100.0, quad=2)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        P = cr.make_problem(w["coords"], w["elems"], w["mu"], w["nu"], w["fbar"])
        cr.solve_coupled(P)
        wall = time.perf_counter() - t0
    ne_s = len(w["elems"])
    t_scaled = wall * ne_target / ne_s
    return {"value": 1.0 / t_scaled, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "host_cpus": os.cpu_count(), "cpu_model": cpu_model(), "sample_seconds": round(wall, 2),
            "sample": (f"oracle coupled sparse-LU solve (assembly + SuperLU + back-substitution, FP64, one thread) "
                       f"of the same 3D transient Stokes problem on {n_sample}^3 x 6 = {ne_s} elements, "
                       f"{wall:.1f} s, scaled linearly by element count to {ne_target} elements (3D sparse LU grows "
                       f"much faster than linearly, so this favours the CPU)")}


def run_serving(args):
    """Continuous-batching serving of transient-Stokes time-step requests:
    sessions arrive as a Poisson process (N x N x 2 meshes, N log-uniform in
    [32, 512], dt uniform in [1e-3, 1e-1], 1 to 20 steps per session), are
    admitted by a device-memory budget and solved to 1e-9 in one shared batch.
    First the saturated throughput (all sessions of the first requests offered
    at once), then the offered load swept at 0.5, 0.8 and 1.0 of it on those
    requests, then the full run at 0.5 of it (the full list holds more large
    meshes than its first requests; at 0.8 its queue grows).  The arrival times of one seeded
    session list are rescaled for each offered load."""
    import numpy as np
    import synth.workloads as wl
    from paper_2101_03777_amd.serve import Server, Session
    t0 = time.perf_counter()
    ss = wl.serving_sessions(args.serve_requests, seed=1, rate=1.0)
    log(f"serving inputs: {len(ss)} sessions, {sum(d['steps'] for d in ss)} requests, "
        f"{time.perf_counter() - t0:.1f} s")
    budget = int(args.serve_budget_gb * (1 << 30))

    def prefix(n_req):
        out, tot = [], 0
        for d in ss:
            if tot >= n_req:
                break
            out.append(d)
            tot += d["steps"]
        return out

    def serve(data, req_rate):
        # arrivals of the unit-rate session list scaled to req_rate requests/s
        # (inf: every session offered at time 0)
        steps = np.mean([d["steps"] for d in data])
        scale = 0.0 if not np.isfinite(req_rate) else steps / req_rate
        sessions = [Session(i, d["coords"], d["elems"], d["dt"], d["nu"], d["fbar"], d["steps"],
                            d["arrival"] * scale) for i, d in enumerate(data)]
        srv = Server(hbm_budget=budget, max_active=128, precision=args.serve_precision, tol=1e-9)
        st = srv.run(sessions)
        srv.close()
        recs = st.pop("records")
        st["offered_requests_per_s"] = None if not np.isfinite(req_rate) else req_rate
        st["total_iterations"] = int(sum(r["iters"] for r in recs))
        return {k: (float(f"{v:.4g}") if isinstance(v, float) else v) for k, v in st.items()}

    out = {"workload": "transient Stokes time steps, N x N x 2 meshes, N log-uniform in [32, 512], dt uniform in "
                       "[1e-3, 1e-1] (mu = 1/dt), 1-20 steps per session, Poisson session arrivals, seed 1",
           "precision": args.serve_precision, "tol": 1e-9, "budget_bytes": budget}
    small = prefix(args.serve_sweep_requests)
    sat = serve(small, float("inf"))
    out["saturated"] = sat
    cap = sat["solves_per_s"]
    log(f"serving saturated: {cap:.1f} solves/s ({sat['requests']} requests offered at once)")
    for frac in (0.5, 0.8, 1.0):
        r = serve(small, frac * cap)
        out[f"load_{frac:g}"] = r
        log(f"serving at {frac:g} of saturation: {r['solves_per_s']:.1f} solves/s, p50 {r['p50_ms']:.0f} ms, "
            f"p99 {r['p99_ms']:.0f} ms")
    full = serve(ss, 0.5 * cap)
    out["run_all_at_0.5"] = full
    log(f"serving {full['requests']} requests at 0.5 of saturation: {full['solves_per_s']:.1f} solves/s, "
        f"p50 {full['p50_ms']:.0f} ms, p99 {full['p99_ms']:.0f} ms")
    return out


def measure_transient(crh, torch, name, args, steps, warmup, precision, copy_gbps, headline):
    """Steps of eliminate + solve + recover on one transient-Stokes workload, and
    everything reported beside them for that workload."""
    import numpy as np
    cfg = WORKLOADS[name]
    t0 = time.perf_counter()
    w = load_workload(name)
    log(f"{name}: inputs {len(w['elems'])} elements, {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    s = crh.System(w["coords"], w["elems"], cfg["mu"], cfg["nu"])
    t_topo = time.perf_counter() - t0
    log(f"{name}: topology + upload {t_topo:.2f} s, {s.n_int_faces} interior faces")
    fbar = torch.from_numpy(w["fbar"]).cuda()
    stream = torch.cuda.current_stream()
    tol = cfg["tol"]

    def step(record):
        e0, e1, e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
        e0.record(stream)
        s.eliminate(fbar)
        e1.record(stream)
        info = s.solve("pcg", precision, tol=tol)
        e2.record(stream)
        U, P = s.recover()
        e3.record(stream)
        e3.synchronize()
        if record is not None:
            record.append(dict(elim_ms=e0.elapsed_time(e1), solve_ms=e1.elapsed_time(e2),
                               recover_ms=e2.elapsed_time(e3), total_ms=e0.elapsed_time(e3), **info))
        return U, P

    for k in range(warmup):
        step(None)
        log(f"{name}: warmup {k + 1}/{warmup} done")
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        U, P = step(recs)
        log(f"{name}: step {k + 1}/{steps}: {recs[-1]['total_ms']:.1f} ms, {recs[-1]['iters']} iterations, "
            f"rel residual {recs[-1]['rel_residual']:.2e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([r["total_ms"] for r in recs])
    last = recs[-1]
    solve_ms = float(np.median([r["solve_ms"] for r in recs]))

    err = oracle_error(name, U, P)
    log(f"{name}: error vs oracle {json.dumps({k: v for k, v in err.items() if k.endswith('rel2') or k.endswith('rel')})}")

    # dominant kernel: the element kernel of the CG iteration (operator applied
    # from element factors, fused with the direction update), timed with HIP
    # events on the solver's stream inside the iteration sequence
    ms_k, bytes_k = s.time_spmv(precision, reps=200)
    gbs = bytes_k / (ms_k * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(name, precision),
            "kernel": kernel_name(cfg["dim"], precision), "avg_launch_us": round(ms_k * 1e3, 2),
            "algorithmic_bytes_per_launch": int(bytes_k), "measured_copy_GBps": round(copy_gbps, 1),
            "frac_of_copy": round(gbs / copy_gbps, 4)}
    if cfg["bound"] != "hbm":
        roof["label"] = cfg["bound"]
    log(f"{name}: dominant kernel {ms_k * 1e3:.2f} us/launch, {gbs:.0f} GB/s "
        f"({100 * gbs / HBM_PEAK_GBS:.1f}% of HBM peak, {100 * gbs / copy_gbps:.1f}% of the measured copy)")

    # accuracy diagnostic: copy mismatch of the recovered velocity (equals the residual)
    s.solve("pcg", precision, tol=tol)
    _, _, J = s.recover(jump=True)
    torch.cuda.synchronize()

    # the configuration's stated residual tolerance: time and error
    info_c = s.solve("pcg", precision, tol=cfg["config_tol"])
    Uc_, Pc_ = s.recover()
    at_config = {"tol": cfg["config_tol"], "time_to_tol_ms": round(info_c["t_solve_ms"], 3),
                 "iters": info_c["iters"], "rel_residual": info_c["rel_residual"],
                 "err_vs_oracle": {k: v for k, v in oracle_error(name, Uc_, Pc_).items()
                                   if k in ("U_rel2", "U_max_rel", "P_rel2", "P_max_rel", "status")}}
    log(f"{name}: at residual {cfg['config_tol']:g}: {info_c['t_solve_ms']:.1f} ms, {info_c['iters']} iterations, "
        f"error {json.dumps(at_config['err_vs_oracle'])}")
    del Uc_, Pc_

    # Jacobi only (no coarse correction): the like-for-like comparison with the
    # coupled solve, which has a diagonal preconditioner
    info_j = s.solve("pcg", precision, tol=tol, precond="jacobi", maxit=200000, raise_on_error=False)
    log(f"{name}: Jacobi-only solve {info_j['t_solve_ms']:.1f} ms, {info_j['iters']} iterations")
    # the other Krylov precision
    other = "fp64" if precision == "fp32_ir" else "fp32_ir"
    info_o = s.solve("pcg", other, tol=tol, maxit=200000, raise_on_error=False)
    log(f"{name}: {other} solve {info_o['t_solve_ms']:.1f} ms, {info_o['iters']} iterations")

    coupled = None
    if not args.no_coupled:
        Uc, Pc, ci = s.coupled_solve(tol=tol, maxit=cfg["coupled_maxit"], raise_on_error=False)
        torch.cuda.synchronize()
        diff = (torch.linalg.norm(Uc - U) / torch.linalg.norm(U)).item()
        ce = oracle_error(name, Uc, Pc)
        coupled = {"method": "FP64 MINRES on eq. syslin, diagonal block preconditioner diag(A) + "
                             "diag(D diag(A)^-1 D^t)",
                   "tol": tol, "time_ms": round(ci["t_solve_ms"], 2), "iters": ci["iters"],
                   "maxit": cfg["coupled_maxit"], "rel_residual": ci["rel_residual"], "converged": ci["status"] == 0,
                   "rel_diff_U_vs_hybrid": diff,
                   "err_vs_oracle": {k: v for k, v in ce.items()
                                     if k in ("U_rel2", "U_max_rel", "P_rel2", "P_max_rel", "status")},
                   "speedup_hybrid_jacobi_only": round(ci["t_solve_ms"] / info_j["t_solve_ms"], 2),
                   "speedup_hybrid_coarse": round(ci["t_solve_ms"] / solve_ms, 2)}
        log(f"{name}: coupled MINRES {ci['t_solve_ms']:.1f} ms, {ci['iters']} iterations, "
            f"residual {ci['rel_residual']:.2e}, converged={ci['status'] == 0}")
        del Uc, Pc
        # the coupled solve at the configuration's residual tolerance as well
        Uc, Pc, ci2 = s.coupled_solve(tol=cfg["config_tol"], maxit=cfg["coupled_maxit"], raise_on_error=False)
        ce2 = oracle_error(name, Uc, Pc)
        coupled["at_config_tol"] = {
            "tol": cfg["config_tol"], "time_ms": round(ci2["t_solve_ms"], 2), "iters": ci2["iters"],
            "rel_residual": ci2["rel_residual"], "converged": ci2["status"] == 0,
            "err_vs_oracle": {k: v for k, v in ce2.items()
                              if k in ("U_rel2", "U_max_rel", "P_rel2", "P_max_rel", "status")}}
        log(f"{name}: coupled MINRES at {cfg['config_tol']:g}: {ci2['t_solve_ms']:.1f} ms, {ci2['iters']} iterations")
        del Uc, Pc

    out = {
        "workload": cfg["label"] + f", to rel residual {tol:g} (the tolerance at which U and P match the FP64 "
                   f"oracle to 1e-9; the stated {cfg['config_tol']:g} is timed in at_config_tol) "
                   f"({'FP32 iterations inside FP64 residual replacement' if precision == 'fp32_ir' else 'FP64'})",
        "elements": len(w["elems"]), "unknowns": s.n_int_faces * cfg["dim"], "tol": tol, "precision": precision,
        "solves_per_s": round(steps / wall, 4), "ms_per_step": round(1e3 * wall / steps, 3),
        "time_to_tol_ms": round(solve_ms, 3), "iters": last["iters"], "outer_iters": last["outer_iters"],
        "rel_residual": last["rel_residual"], "fp64_fallback": last["fp64_fallback"], "copy_mismatch": J.item(),
        "eliminate_ms": round(float(np.median([r["elim_ms"] for r in recs])), 3),
        "recover_ms": round(float(np.median([r["recover_ms"] for r in recs])), 3),
        "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "topology_host_s": round(t_topo, 3),
        "err_vs_oracle": err,
        "at_config_tol": at_config,
        "roofline": roof,
        "jacobi_only": {"time_to_tol_ms": round(info_j["t_solve_ms"], 3), "iters": info_j["iters"],
                        "rel_residual": info_j["rel_residual"], "converged": info_j["status"] == 0},
        f"{other}_iterations": {"time_to_tol_ms": round(info_o["t_solve_ms"], 3), "iters": info_o["iters"],
                                "fp32_iters": info_o["fp32_iters"], "fp64_fallback": info_o["fp64_fallback"],
                                "rel_residual": info_o["rel_residual"]},
        "coupled_gpu": coupled,
        "steps": steps, "warmup": warmup,
    }
    s.close()
    del U, P, fbar
    torch.cuda.empty_cache()
    return out, wall


def run_ns(crh, torch):
    """Steady Navier-Stokes Newton step on 256x256x2 (nu = 0.01), BiCGStab(2), FP64,
    with its error against the stored oracle solution, and the coupled-system
    BiCGStab baseline on the same GPU."""
    import synth.workloads as wl
    t0 = time.perf_counter()
    w = wl.ns256()
    log(f"NS 256x256x2 inputs: {time.perf_counter() - t0:.1f} s")
    s = crh.System(w["coords"], w["elems"], 0.0, w["nu"], problem="ns")
    s.eliminate(torch.from_numpy(w["fbar"]).cuda(), None, torch.from_numpy(w["ulin"]).cuda())
    info = s.solve("bicgstab2", "fp64", tol=1e-9, maxit=600000, raise_on_error=False)
    U, P = s.recover()
    err = oracle_error("ns256", U, P)
    out = {"workload": "2D steady Navier-Stokes Newton step, 256x256x2, nu=0.01, seeded linearisation velocity, "
                       "E_K from the M1/M2 partition; BiCGStab(2), FP64, to rel residual 1e-9",
           "elements": len(w["elems"]), "unknowns": s.n_int_faces * 2, "status": info["status"],
           "time_to_tol_ms": round(info["t_solve_ms"], 1), "iters": info["iters"],
           "products_with_G": 4 * info["iters"], "rel_residual": info["rel_residual"],
           "err_vs_oracle": {k: v for k, v in err.items() if k in ("U_rel2", "U_max_rel", "P_rel2", "P_max_rel",
                                                                    "status", "oracle")}}
    log(f"NS 256x256x2 BiCGStab(2): {info['t_solve_ms']:.0f} ms, {info['iters']} iterations, status {info['status']}, "
        f"error {json.dumps(out['err_vs_oracle'])}")
    # the configured precision (FP32 iterations inside FP64 residual
    # replacement): the FP32 passes stall and the solve falls back to FP64
    i32 = s.solve("bicgstab2", "fp32_ir", tol=1e-9, maxit=600000, raise_on_error=False)
    U32, P32 = s.recover()
    e32 = oracle_error("ns256", U32, P32)
    out["fp32_ir_attempt"] = {"status": i32["status"], "time_to_tol_ms": round(i32["t_solve_ms"], 1),
                              "iters": i32["iters"], "fp32_iters": i32["fp32_iters"],
                              "fp64_fallback": i32["fp64_fallback"], "rel_residual": i32["rel_residual"],
                              "err_vs_oracle": {k: v for k, v in e32.items()
                                                if k in ("U_rel2", "U_max_rel", "P_rel2", "P_max_rel")}}
    log(f"NS 256x256x2 BiCGStab(2) FP32 iterations + FP64 replacement: {i32['t_solve_ms']:.0f} ms, {i32['iters']} "
        f"iterations ({i32['fp32_iters']} FP32), FP64 fallback {i32['fp64_fallback']}, status {i32['status']}")
    Uc, Pc, ci = s.coupled_solve(tol=1e-9, maxit=100000, raise_on_error=False)
    ce = oracle_error("ns256", Uc, Pc)
    out["coupled_gpu"] = {"method": "FP64 BiCGStab on eq. syslin (Jacobian blocks in A), symmetric scaling by the "
                                    "square root of diag|A| + diag(D diag|A|^-1 D^t)",
                          "time_ms": round(ci["t_solve_ms"], 1), "iters": ci["iters"], "maxit": 100000,
                          "rel_residual": ci["rel_residual"], "converged": ci["status"] == 0,
                          "err_vs_oracle": {k: v for k, v in ce.items()
                                            if k in ("U_rel2", "U_max_rel", "P_rel2", "P_max_rel", "status")}}
    log(f"NS 256x256x2 coupled BiCGStab: {ci['t_solve_ms']:.0f} ms, {ci['iters']} iterations, "
        f"residual {ci['rel_residual']:.2e}, status {ci['status']}")
    s.close()
    return out


def run_newton(crh, torch):
    """Newton iterations with non-homogeneous Dirichlet data (Section 4): the
    steady lid-driven cavity at Re = 100 on 64x64x2 from rest to the paper's
    threshold 5e-7, and the Green-Taylor vortex (amplitude Re = 100, nu = 1,
    final time 0.01) in 2D (dt/h^2 = 0.002 as in Table tab0; 8, 16, 32 cells
    per side) and in 3D (the time steps of the 3D Navier-Stokes table; 8 and 16
    cubes per side) with its errors against the exact solution and their
    orders."""
    import numpy as np
    import synth
    import synth.workloads as wl
    from paper_2101_03777_amd.newton import NewtonSolver
    out = {}
    coords, elems = synth.square_mesh(64)
    bf = wl.exterior_face_list(elems)
    g = np.zeros((len(bf), 2))
    g[coords[bf].mean(axis=1)[:, 1] > 1.0 - 1e-12, 0] = 1.0
    ns = NewtonSolver(coords, elems, 0.0, 0.01)
    ns.set_boundary(g)
    t0 = time.perf_counter()
    U, P, rec = ns.solve(np.zeros((len(elems), 2)), tol=5e-7, maxit=25, lin_tol=1e-10)
    out["cavity_re100_64"] = {
        "workload": "steady lid-driven cavity, Re = 100, 64x64x2, Newton from rest, BiCGStab(2) FP64 per step",
        "newton_iters": len(rec["increments"]), "converged": rec["converged"],
        "increments": [float(f"{x:.3g}") for x in rec["increments"]], "linear_iters": rec["linear_iters"],
        "time_s": round(time.perf_counter() - t0, 2)}
    log(f"cavity Re=100 64x64x2: {len(rec['increments'])} Newton iterations, {out['cavity_re100_64']['time_s']} s")
    ns.close()
    out["green_taylor_2d"] = {"workload": "Green-Taylor vortex, amplitude Re = 100, nu = 1, unit square n x n x 2, "
                                          "final time 0.01, dt/h^2 = 0.002, exact velocity on the boundary, "
                                          "Newton at every backward-Euler step",
                              "rows": green_taylor_rows(crh, torch, 2, (8, 16, 32), 0.002),
                              "paper_table_tab0_ratios": "velocity 1.70, 1.44, 1.78, 1.94, 1.98; pressure 0.89, 1.23, "
                                                         "1.67, 1.83, 1.72 (h = 0.125 ... 0.0078, FVCA Mesh1 family)"}
    out["green_taylor_3d"] = {"workload": "3D Green-Taylor vortex (Section 4.1: the 2D vortex in (x1, x2), third "
                                          "component zero), amplitude Re = 100, nu = 1, unit cube n^3 x 6 "
                                          "tetrahedra, final time 0.01, dt = 0.01 a^2 with a = 1/n the cube side "
                                          "(the time steps of the paper's 3D Navier-Stokes table, whose h = "
                                          "(a^3/6)^(1/3) is the size of a tetrahedron), exact velocity on the "
                                          "boundary, Newton at every backward-Euler step (12 x 12 local inverses)",
                              "rows": green_taylor_rows(crh, torch, 3, (8, 16), 0.01),
                              "paper_3d_ns_table": "n = 8, 16, 32 (h = 6.88e-2, 3.44e-2, 1.72e-2): velocity errors "
                                                   "10.7, 4.10, 1.28 (ratios 1.38, 1.68); pressure 297, 143, 48.5 "
                                                   "(1.05, 1.56)"}
    out["green_taylor_3d_stokes"] = {
        "workload": "3D Green-Taylor Stokes test (Section 4.1: the vortex's velocity, zero pressure, unforced "
                    "transient Stokes), unit cube n^3 x 6 tetrahedra, final time 0.01, dt = 0.0016 a^2 (the time "
                    "steps of the paper's 3D Stokes table), exact velocity on the boundary, one hybridised CG "
                    "solve (FP64, 1e-11) per step",
        "rows": green_taylor_rows(crh, torch, 3, (4, 8, 16), 0.0016, stokes=True),
        "paper_3d_stokes_table": "n = 4, 8, 16, 32 (h = 1.38e-1 ... 1.72e-2): velocity errors 3.44, 0.85, 0.22, "
                                 "5.4e-2 (ratios 2.02, 1.95, 2.03); pressure 33, 17, 8.1, 4.0 (0.96, 1.07, 1.02)"}
    return out


def green_taylor_rows(crh, torch, dim, sizes, ratio, stokes=False):
    """Errors of the Green-Taylor vortex at the final time 0.01 on n^dim cells
    (dt = ratio h^2, h = 1/n): velocity at the face centroids weighted by the
    lumped mass |K|/(d+1) of the two elements of each face, pressure at the
    element centroids weighted by |K|, both without their means; and their
    orders.  stokes: the unforced transient Stokes problem with the vortex's
    velocity and zero pressure (one hybridised solve per step, CG) instead of
    Navier-Stokes (Newton at every step)."""
    import numpy as np
    import synth
    import synth.workloads as wl
    from synth.fields import GreenTaylor2D, GreenTaylor3D, face_means
    from paper_2101_03777_amd.newton import NewtonSolver
    gt = (GreenTaylor2D if dim == 2 else GreenTaylor3D)(amp=100.0, nu=1.0)
    rows = []
    for n in sizes:
        coords, elems = synth.square_mesh(n) if dim == 2 else synth.cube_mesh(n)
        bf, fi = wl.exterior_face_list(elems), wl.interior_face_list(elems)
        h = 1.0 / n
        dt = ratio * h * h
        nsteps = int(round(0.01 / dt))
        dt = 0.01 / nsteps
        ns = crh.System(coords, elems, 1.0 / dt, 1.0) if stokes else NewtonSolver(coords, elems, 1.0 / dt, 1.0)
        xf = coords[fi].mean(axis=1)
        Ug = torch.from_numpy(face_means(coords, fi, lambda x: gt.u(x, 0.0))).cuda()
        f = np.zeros((len(elems), dim))
        fd = torch.zeros((len(elems), dim), dtype=torch.float64, device="cuda")
        t0 = time.perf_counter()
        t_log = t0
        newt = 0
        lin = 0
        for k in range(1, nsteps + 1):
            if time.perf_counter() - t_log > 60.0:
                t_log = time.perf_counter()
                log(f"Green-Taylor {dim}D n={n}: step {k - 1}/{nsteps}, {t_log - t0:.0f} s")
            ns.set_boundary(face_means(coords, bf, lambda x: gt.u(x, k * dt)))
            if stokes:
                # the operator stays; each step refreshes the right-hand side
                if k == 1:
                    ns.eliminate(fd, Ug)
                else:
                    ns.update_rhs(fd, Ug)
                info = ns.solve("pcg", "fp64", tol=1e-11, warm_start=k > 1)
                Ug, Pg = ns.recover()
                lin += info["iters"]
            else:
                Ug, Pg, rec = ns.solve(f, u_prev=Ug, u0=Ug, tol=1e-9, lin_tol=1e-11)
                newt += len(rec["increments"])
                lin += sum(rec["linear_iters"])
        wall = time.perf_counter() - t0
        T = nsteps * dt
        X = coords[elems]
        if dim == 2:
            vol = 0.5 * np.abs((X[:, 1, 0] - X[:, 0, 0]) * (X[:, 2, 1] - X[:, 0, 1]) -
                               (X[:, 2, 0] - X[:, 0, 0]) * (X[:, 1, 1] - X[:, 0, 1]))
        else:
            vol = np.abs(np.einsum("ij,ij->i", X[:, 1] - X[:, 0], np.cross(X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]))) / 6.0
        fidx = {tuple(v): i for i, v in enumerate(fi)}
        mass = np.zeros(len(fi))
        for e, el in enumerate(elems):
            for j in range(dim + 1):
                key = tuple(sorted(np.delete(el, j)))
                if key in fidx:
                    mass[fidx[key]] += vol[e] / (dim + 1)
        Ue = gt.u(xf, T)
        eu = np.sqrt((mass[:, None] * (Ug.cpu().numpy() - Ue) ** 2).sum())
        pe = np.zeros(len(elems)) if stokes else gt.p(X.mean(axis=1), T)
        ph = Pg.cpu().numpy()
        dp = (ph - (vol * ph).sum() / vol.sum()) - (pe - (vol * pe).sum() / vol.sum())
        ep = np.sqrt((vol * dp ** 2).sum())
        rows.append({"n": n, "h": h, "dt": dt, "steps": nsteps, "newton_iters": newt, "linear_iters": lin,
                     "time_s": round(wall, 2), "err_l2_u": float(f"{eu:.4g}"), "err_l2_p": float(f"{ep:.4g}")})
        log(f"Green-Taylor {dim}D{' Stokes' if stokes else ''} n={n}: {nsteps} steps, {newt} Newton iterations, {lin} linear iterations, "
            f"{wall:.1f} s, errors u {eu:.3g} p {ep:.3g}")
        ns.close()
    for a, b in zip(rows[:-1], rows[1:]):
        b["ratio_u"] = round(float(np.log2(a["err_l2_u"] / b["err_l2_u"]) / np.log2(b["n"] / a["n"])), 2)
        b["ratio_p"] = round(float(np.log2(a["err_l2_p"] / b["err_l2_p"]) / np.log2(b["n"] / a["n"])), 2)
    return rows


def run_paper_context(crh, torch):
    """The paper's own 2D timings are on the FVCA mesh Mesh1-7 (917,504
    triangles) on CPUs; the same problems on a structured stand-in of that
    size (677 x 677 x 2 = 916,658 triangles) on this GPU, with the paper's
    numbers quoted beside them as context (other hardware, other mesh,
    tolerances not stated for the transient case)."""
    import numpy as np
    import synth
    import synth.workloads as wl
    out = {}
    n = 677
    t0 = time.perf_counter()
    w = wl.square(n, mu=1e4, nu=1.0, jitter=0.2, seed=0, quad=3)
    log(f"paper context: {len(w['elems'])} triangles, inputs {time.perf_counter() - t0:.1f} s")
    s = crh.System(w["coords"], w["elems"], 1e4, 1.0)
    f = torch.from_numpy(w["fbar"]).cuda()
    stream = torch.cuda.current_stream()
    recs = []
    for k in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.eliminate(f)
        info = s.solve("pcg", "fp32_ir", tol=1e-10)
        s.recover()
        e1.record(stream)
        e1.synchronize()
        recs.append((e0.elapsed_time(e1), info["iters"]))
    s.close()
    out["transient_stokes_mesh1_7_size"] = {
        "workload": "2D transient Stokes, 677 x 677 x 2 jittered (916,658 triangles), dt = 1e-4 (mu = 1e4), nu = 1, "
                    "manufactured force; eliminate + CG (FP32 iterations, FP64 replacements, coarse correction) "
                    "to 1e-10 + recover",
        "ms_per_solve": round(min(r[0] for r in recs), 1), "iters": recs[-1][1],
        "paper": "Mesh1-7, dt = 1e-4: CG + BoomerAMG 163 / 90 / 47 / 25 / 19 s on 1 / 2 / 4 / 8 / 16 CPU processes, "
                 "CG + ILU(1) 8.4 s on 16 (a 16-CPU computer, HYPRE)"}
    log(f"paper context: transient Stokes 677x677x2: {out['transient_stokes_mesh1_7_size']['ms_per_solve']} ms")
    coords, elems = synth.square_mesh(n)
    bf = wl.exterior_face_list(elems)
    g = np.zeros((len(bf), 2))
    g[coords[bf].mean(axis=1)[:, 1] > 1.0 - 1e-12, 0] = 1.0
    s = crh.System(coords, elems, 0.0, 1e-3)
    s.set_boundary(g)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.eliminate(torch.zeros((len(elems), 2), dtype=torch.float64, device="cuda"))
    info = s.solve("minres", "fp64", tol=1e-11, maxit=2000000, raise_on_error=False)
    s.recover()
    e1.record(stream)
    e1.synchronize()
    s.close()
    out["stokes_cavity_mesh1_7_size"] = {
        "workload": "2D steady Stokes lid-driven cavity, 677 x 677 x 2 (916,658 triangles), nu = 1e-3, lid velocity "
                    "(1, 0); eliminate (E_K from the M1/M2 partition) + MINRES FP64 to 1e-11 + recover",
        "s_per_solve": round(e0.elapsed_time(e1) / 1e3, 2), "iters": info["iters"], "status": info["status"],
        "rel_residual": info["rel_residual"],
        "paper": "Mesh1-7: hybrid GMRES (1e-11) + ILU(2..8) 547.9, 477.4, 231.6, 152.9, 89.13, 65.96, 69.76 s on one "
                 "CPU process; coupled 2025 ... 93.04 s (Table tab1)"}
    log(f"paper context: Stokes cavity 677x677x2: {out['stokes_cavity_mesh1_7_size']['s_per_solve']} s, "
        f"{info['iters']} MINRES iterations")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cube64", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp32_ir", choices=["fp32_ir", "fp64"],
                    help="Krylov arithmetic of the timed path (the other one is reported beside it)")
    ap.add_argument("--no-coupled", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="time-step requests of the serving run (0: skip)")
    ap.add_argument("--serve-sweep-requests", type=int, default=500,
                    help="requests of the saturation measurement and of each swept load")
    ap.add_argument("--serve-budget-gb", type=float, default=2.0, help="device-memory budget for admission")
    ap.add_argument("--serve-precision", default="fp32_ir", choices=["fp32_ir", "fp64"])
    ap.add_argument("--no-other", action="store_true",
                    help="skip the second transient workload and the Navier-Stokes step")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only build the workload's system and time the dominant kernel (for counter collection)")
    ap.add_argument("--green-taylor-3d", default="",
                    help="only the 3D Navier-Stokes Green-Taylor rows on these cube counts (e.g. 8,16,32), "
                         "one JSON line")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run 20 device-to-device copies of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2101_03777_amd as crh

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
    if args.green_taylor_3d:
        sizes = tuple(int(v) for v in args.green_taylor_3d.split(","))
        print(json.dumps({"green_taylor_3d": green_taylor_rows(crh, torch, 3, sizes, 0.01)}), flush=True)
        return
    if args.kernel_only:
        cfg = WORKLOADS[args.workload]
        w = load_workload(args.workload)
        s = crh.System(w["coords"], w["elems"], cfg["mu"], cfg["nu"])
        s.eliminate(torch.from_numpy(w["fbar"]).cuda())
        ms_k, bytes_k = s.time_spmv(args.precision, reps=200)
        print(json.dumps({"kernel": kernel_name(cfg["dim"], args.precision), "workload": args.workload,
                          "precision": args.precision, "avg_us": ms_k * 1e3, "algorithmic_bytes": bytes_k,
                          "GBps": bytes_k / (ms_k * 1e-3) / 1e9}), flush=True)
        s.close()
        return

    copy_gbps = copy_bandwidth(torch)
    log(f"device copy: {copy_gbps:.0f} GB/s (read + write)")
    head, wall = measure_transient(crh, torch, args.workload, args, args.steps, args.warmup, args.precision,
                                   copy_gbps, True)

    second = None
    ns = None
    context = None
    c1, c1_sol = None, None
    if not args.no_other:
        other = "square512j" if args.workload == "cube64" else "cube64"
        second, _ = measure_transient(crh, torch, other, args, max(3, args.steps // 2), 1, args.precision, copy_gbps,
                                      False)
        ns = run_ns(crh, torch)
        ns.update(run_newton(crh, torch))
        context = run_paper_context(crh, torch)
        c1, U1, P1 = run_c1(crh, torch)
        c1_sol = (U1, P1)
        log(f"16x16x2: {c1['ms_per_solve']} ms per solve, {c1['iters']} iterations")

    serving = None
    if args.serve_requests > 0:
        serving = run_serving(args)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_oracle_baseline(head["elements"]) if WORKLOADS[args.workload]["dim"] == 3 else None
        if cpu:
            log(f"cpu oracle: {cpu['value']:.3g} solves/s ({cpu['sample']})")
        if c1 is not None:
            c1 = c1_oracle_leg(c1, *c1_sol)
            log(f"16x16x2 against the oracle: {json.dumps(c1['err_vs_oracle'])}, oracle {c1['oracle_ms']} ms")

    out = {
        "metric": METRIC,
        "value": head["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "fp32_ir" else "f64",
        "data": "synthetic",
        "config": {"workload": head["workload"], "elements": head["elements"], "unknowns": head["unknowns"],
                   "tol": head["tol"], "precision": args.precision},
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "err_vs_oracle": head["err_vs_oracle"],
        "time_to_tol_ms": head["time_to_tol_ms"], "iters": head["iters"], "outer_iters": head["outer_iters"],
        "rel_residual": head["rel_residual"], "copy_mismatch": head["copy_mismatch"],
        "eliminate_ms": head["eliminate_ms"], "recover_ms": head["recover_ms"],
        "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"],
        "jacobi_only": head["jacobi_only"],
        "coupled_gpu": head["coupled_gpu"],
        "at_config_tol": head["at_config_tol"],
        "headline_detail": {k: v for k, v in head.items()
                            if k not in ("roofline", "err_vs_oracle", "coupled_gpu", "jacobi_only", "at_config_tol")},
        "second_workload": second,
        "smallest_config": c1,
        "ns_newton_256": ns,
        "paper_context": context,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

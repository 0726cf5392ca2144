"""Continuous-batching server for transient-Stokes time-step requests.

Sessions (a mesh, a time step dt, a force and a number of backward-Euler steps)
arrive over time.  A session is admitted when the device-memory budget and a
batch slot allow; its hybridised system (topology, elimination, G) is built
once and stays resident for all its steps.  The host part of the build
(cr_prepare: topology, renumbering, tables; about 0.4 s for a 512x512x2 mesh)
runs on a worker thread while the batch keeps iterating (library calls release
the interpreter lock and cr_prepare makes no HIP call); upload and elimination
then run on the serving thread between iteration blocks.  Every step is a
request:

  step 1:  cr_assemble + cr_eliminate (mu = 1/dt), then solve, then recover;
  step k:  cr_update_rhs with u_prev = U of step k-1 (same G), solve from the
           previous W (warm start), recover.

All admitted systems iterate together in one cr_batch: each iteration block is
one set of launches covering every active system, systems join as they are
admitted or start their next step and leave as they converge, so requests that
arrive while others are on the GPU overlap with them on the device.  Latency of
a request runs from its issue (arrival for step 1, completion of the previous
step otherwise) to the moment its U and P are on the device.

All device work runs in the HIP library; this module only schedules.
"""
from __future__ import annotations

import collections
import concurrent.futures
import time

import numpy as np

from ._binding import Batch, Prepared, System

# device bytes per element of a resident 2D transient-Stokes system with its
# Krylov workspace (element data ~510 B including the operator factors and the
# per-element Krylov contributions; per-face data ~110 B and twelve Krylov
# vectors ~190 B per face, about 1.5 faces per element -- the assembled block
# rows of G are not built for the element-form CG; measured 1,050-1,140 B per
# element on 128x128x2 and 512x512x2; a margin for the recovery buffers), used
# to decide admission before the system exists
BYTES_PER_ELEMENT_2D = 1200


class Session:
    def __init__(self, sid, coords, elems, dt, nu, fbar, steps, arrival):
        self.sid = sid
        self.coords = coords
        self.elems = elems
        self.dt = float(dt)
        self.nu = float(nu)
        self.fbar = fbar
        self.steps = int(steps)
        self.arrival = float(arrival)
        self.sys = None
        self.fdev = None
        self.done_steps = 0
        self.req_t0 = None
        self.bytes = 0
        self.admitted_at = None
        self.t_build = None   # build (prepare on a worker, then upload and elimination) started
        self.t_enter = None   # the current request joined the batch

    @property
    def estimate(self):
        return BYTES_PER_ELEMENT_2D * len(self.elems)


class Server:
    def __init__(self, hbm_budget=8 << 30, max_active=128, precision="fp32_ir", tol=1e-9, iters_per_advance=32,
                 inner_tol=0.0, build_workers=2):
        import torch
        self.torch = torch
        self.budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.opts = dict(method="pcg", precision=precision, tol=tol, inner_tol=inner_tol)
        self.iters = int(iters_per_advance)
        self.batch = Batch(max_systems=max_active)
        self.pool = concurrent.futures.ThreadPoolExecutor(max_workers=max(1, int(build_workers)))

    @staticmethod
    def _prepare(s):
        """Host part of a new session's system (worker thread, no device call)."""
        return Prepared(s.coords, s.elems, mu=1.0 / s.dt, nu=s.nu)

    def _admit(self, s, prep):
        """Upload, elimination and batch entry of a prepared session (serving thread)."""
        torch = self.torch
        s.sys = System(prepared=prep)
        s.fdev = torch.from_numpy(np.ascontiguousarray(s.fbar)).cuda()
        s.sys.eliminate(s.fdev)
        self.batch.add(s.sys, **self.opts, warm_start=False)
        s.bytes = s.sys._alloc.bytes_in_use if s.sys._alloc else s.estimate

    def run(self, sessions, on_result=None, time_limit=None):
        """Replay the arrivals in wall-clock time; return latency/throughput stats.

        on_result(session, step_index, U, P, info) is called for every
        finished request with device tensors U [n_faces, 2] and P [n_elements].
        """
        arr = sorted(sessions, key=lambda s: s.arrival)
        queue = collections.deque()
        owner = {}
        building = []
        latencies, waits, records = [], [], []
        budget_blocks = slot_blocks = 0  # passes in which the queue head waited for memory / for a slot
        in_use = 0
        n_active = 0
        peak_active = 0
        peak_bytes = 0
        nxt = 0
        total = sum(s.steps for s in arr)
        done = 0
        t0 = time.perf_counter()
        while done < total:
            now = time.perf_counter() - t0
            if time_limit is not None and now > time_limit:
                break
            while nxt < len(arr) and arr[nxt].arrival <= now:
                arr[nxt].req_t0 = arr[nxt].arrival
                queue.append(arr[nxt])
                nxt += 1
            # admission by memory budget and batch capacity, in arrival order:
            # the host part is prepared on a worker thread, the system joins the
            # batch when it is ready
            while queue:
                if n_active + len(building) >= self.max_active:
                    slot_blocks += 1
                    break
                s = queue[0]
                if s.estimate > self.budget:
                    raise ValueError(f"session {s.sid} needs {s.estimate} bytes, above the budget {self.budget}")
                if in_use + s.estimate > self.budget:
                    budget_blocks += 1
                    break
                queue.popleft()
                s.t_build = time.perf_counter() - t0
                building.append((s, self.pool.submit(self._prepare, s)))
                in_use += s.estimate
            waiting = []
            for s, fut in building:
                if not fut.done():
                    waiting.append((s, fut))
                    continue
                self._admit(s, fut.result())
                in_use += s.bytes - s.estimate
                s.admitted_at = time.perf_counter() - t0
                s.t_enter = s.admitted_at
                owner[s.sys.h.value] = s
                waits.append(s.admitted_at - s.arrival)
                n_active += 1
            building = waiting
            peak_active = max(peak_active, n_active)
            peak_bytes = max(peak_bytes, in_use)
            if n_active == 0:
                if building:
                    concurrent.futures.wait([f for _, f in building], timeout=0.01,
                                            return_when=concurrent.futures.FIRST_COMPLETED)
                    continue
                if nxt < len(arr):
                    time.sleep(max(0.0, min(0.01, arr[nxt].arrival - (time.perf_counter() - t0))))
                    continue
                break
            self.batch.advance(self.iters)
            t_pop = time.perf_counter() - t0
            while True:
                item = self.batch.pop()
                if item is None:
                    break
                sysobj, info = item
                s = owner[sysobj.h.value]
                t_rec = time.perf_counter() - t0
                U, P = s.sys.recover()
                self.torch.cuda.current_stream().synchronize()
                t_done = time.perf_counter() - t0
                latencies.append(t_done - s.req_t0)
                first = s.done_steps == 0
                records.append(dict(sid=s.sid, step=s.done_steps, latency=t_done - s.req_t0, iters=info["iters"],
                                    status=info["status"], rel_residual=info["rel_residual"],
                                    fp64_fallback=info["fp64_fallback"], n_elements=len(s.elems),
                                    # where the latency went: waiting for memory or a slot (first
                                    # step), building the system (first step) or the right-hand
                                    # side update (later steps), iterating in the batch until the
                                    # advance that finished it, and the recovery
                                    wait=(s.t_build - s.req_t0) if first else 0.0,
                                    build=(s.t_enter - s.t_build) if first else (s.t_enter - s.req_t0),
                                    iterate=t_pop - s.t_enter, recover=t_done - t_rec))
                if on_result is not None:
                    on_result(s, s.done_steps, U, P, info)
                s.done_steps += 1
                done += 1
                if s.done_steps < s.steps:
                    s.req_t0 = t_done
                    s.sys.update_rhs(s.fdev, U)
                    self.batch.add(s.sys, **self.opts, warm_start=True)
                    s.t_enter = time.perf_counter() - t0
                else:
                    del owner[s.sys.h.value]
                    s.sys.close()
                    s.sys = None
                    in_use -= s.bytes
                    n_active -= 1
        wall = time.perf_counter() - t0
        lat = np.array(latencies) if latencies else np.zeros(1)

        def pct(key, q):
            v = [r[key] for r in records]
            return round(1e3 * float(np.percentile(v, q)), 2) if v else 0.0

        breakdown = {key: {"p50_ms": pct(key, 50), "p99_ms": pct(key, 99)}
                     for key in ("wait", "build", "iterate", "recover")}
        return dict(requests=done, sessions=len(arr), wall_s=wall, solves_per_s=done / wall if wall > 0 else 0.0,
                    p50_ms=1e3 * float(np.percentile(lat, 50)), p99_ms=1e3 * float(np.percentile(lat, 99)),
                    mean_ms=1e3 * float(lat.mean()), max_queue_wait_ms=1e3 * float(max(waits) if waits else 0.0),
                    peak_active=peak_active, peak_bytes=int(peak_bytes), budget_bytes=self.budget,
                    budget_blocks=budget_blocks, slot_blocks=slot_blocks, latency_breakdown=breakdown,
                    failed=sum(1 for r in records if r["status"] != 0),
                    fp64_fallbacks=sum(1 for r in records if r["fp64_fallback"]), records=records)

    def close(self):
        self.pool.shutdown(wait=True)
        self.batch.close()

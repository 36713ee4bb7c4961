"""Continuous-batching request loop for droplet solves.

Requests arrive on a clock (a seeded Poisson stream); each asks for a mesh,
degree, temperature, wall/contact angle and a number of RK steps.  A request is
admitted as soon as the device-memory budget has room: its instance (mesh,
scratch, initial state, time step) is set up on a separate stream while the
batch keeps stepping, then it joins the batch, whose kernels advance all
admitted instances together (one graph replay per RK step).  Finished
instances are retired, freeing budget for waiting requests.

Reports time-to-solution percentiles (arrival to completion) and aggregate
node-stage updates per second over the makespan.
"""
from __future__ import annotations

import collections
import time

import numpy as np

from . import autotune
from .nskr import Batch, NskrError, init_workload, solver_for


class Request:
    def __init__(self, rid, t_arrive, workload):
        self.rid = rid
        self.t_arrive = t_arrive
        self.w = workload
        self.t_admit = None
        self.t_done = None
        self.result = None
        self.dt = None
        self.status = None   # "ok", or the health check's error at retirement


def _setup(req, precision, table, setup_stream):
    import torch
    w = req.w
    with torch.cuda.stream(setup_stream):
        s = solver_for(w, precision)
        s.set_block(autotune.threads_for(table, w.N, precision))
        U = init_workload(s, w)
        R = s.new_state()
        dt = s.dt(U)
    return s, U, R, dt


def serve(requests, budget_bytes, precision="fp32_mixed", table=None, keep_results=False, time_scale=1.0,
          graph=True, log=None, max_active_nodes=None):
    """Run the request loop.  requests: list of (t_arrival_s, Workload).
    time_scale stretches the arrival clock (1.0 = real time).  Admission is in
    arrival order while the memory budget has room and, if max_active_nodes is
    set, while the admitted instances hold at most that many nodes (enough to
    fill the GPU; beyond it admitting more only stretches every request's
    latency, since the batch advances all of them together)."""
    import torch
    table = table or {}
    reqs = [Request(i, t * time_scale, w) for i, (t, w) in enumerate(requests)]
    pending = collections.deque(sorted(reqs, key=lambda r: r.t_arrive))
    queue = collections.deque()
    batch = Batch(budget_bytes, graph=graph)
    step_stream = torch.cuda.Stream()
    setup_stream = torch.cuda.Stream()
    active = {}
    node_stages = 0
    t0 = time.perf_counter()
    steps_taken = 0
    max_active = 0
    while pending or queue or active:
        now = time.perf_counter() - t0
        while pending and pending[0].t_arrive <= now:
            queue.append(pending.popleft())
        # admit in arrival order while the budget has room
        while queue:
            req = queue[0]
            if max_active_nodes and active and \
                    sum(r.w.nnodes for r in active.values()) + req.w.nnodes > max_active_nodes:
                break
            s, U, R, dt = _setup(req, precision, table, setup_stream)
            req.dt = dt
            slot = batch.admit(s, U, R, dt, req.w.steps)
            if slot is None:
                del s, U, R
                break
            queue.popleft()
            req.t_admit = time.perf_counter() - t0
            active[slot] = req
        max_active = max(max_active, len(active))
        if active:
            batch.step(step_stream)
            steps_taken += 1
            done = batch.poll()
            if done:
                step_stream.synchronize()
                tnow = time.perf_counter() - t0
                for slot in done:
                    req = active.pop(slot)
                    solver, U, R = batch.retire(slot)
                    req.t_done = tnow
                    # health of the finished state (non-finite values, density
                    # outside (0, 1/b), T <= 0): an instance that failed is
                    # reported, the others are unaffected
                    try:
                        solver.reduce(U, stream=step_stream)
                        req.status = "ok"
                    except NskrError as e:
                        req.status = f"error {e.code}: {e}"
                    node_stages += solver.nnodes * 5 * req.w.steps
                    if keep_results:
                        req.result = U.double().cpu().numpy()
                    if log:
                        log(f"done req {req.rid} {req.w.name} latency {req.t_done - req.t_arrive:.3f}s")
        elif pending:
            time.sleep(max(0.0, min(0.01, pending[0].t_arrive - (time.perf_counter() - t0))))
    makespan = max(r.t_done for r in reqs) - min(r.t_arrive for r in reqs)
    lat = np.array([r.t_done - r.t_arrive for r in reqs])
    return {
        "requests": len(reqs),
        "precision": precision,
        "p50_s": float(np.percentile(lat, 50)),
        "p99_s": float(np.percentile(lat, 99)),
        "mean_s": float(lat.mean()),
        "makespan_s": makespan,
        "node_stage_updates_per_s": node_stages / makespan,
        "batch_steps": steps_taken,
        "max_active": max_active,
        "graph": graph,
        "max_active_nodes": max_active_nodes,
        "errors": sum(1 for r in reqs if r.status != "ok"),
    }, reqs


def serve_sequential(requests, precision="fp64", time_scale=1.0, keep_results=False, graph=True):
    """Baseline: the same requests one at a time in arrival order, each alone
    in a batch of one (graph-replayed steps, so the baseline pays no more
    launch overhead than the batched loop); latencies include the queueing a
    single server would impose on the same arrival clock."""
    import torch
    reqs = [Request(i, t * time_scale, w) for i, (t, w) in enumerate(requests)]
    batch = Batch(1 << 62, graph=graph)
    stream = torch.cuda.Stream()
    t_free = 0.0
    node_stages = 0
    t0 = time.perf_counter()
    for req in sorted(reqs, key=lambda r: r.t_arrive):
        now = time.perf_counter() - t0
        if now < req.t_arrive:
            time.sleep(req.t_arrive - now)
        start = max(req.t_arrive, t_free)
        ts = time.perf_counter()
        s = solver_for(req.w, precision)
        U = init_workload(s, req.w)
        R = s.new_state()
        dt = s.dt(U)
        torch.cuda.synchronize()
        slot = batch.admit(s, U, R, dt, req.w.steps)
        for _ in range(req.w.steps):
            batch.step(stream)
        stream.synchronize()
        assert batch.poll() == [slot]
        batch.retire(slot)
        service = time.perf_counter() - ts
        req.t_admit = start
        req.t_done = start + service
        t_free = req.t_done
        node_stages += s.nnodes * 5 * req.w.steps
        if keep_results:
            req.result = U.double().cpu().numpy()
    makespan = max(r.t_done for r in reqs) - min(r.t_arrive for r in reqs)
    lat = np.array([r.t_done - r.t_arrive for r in reqs])
    return {
        "requests": len(reqs),
        "precision": precision,
        "p50_s": float(np.percentile(lat, 50)),
        "p99_s": float(np.percentile(lat, 99)),
        "mean_s": float(lat.mean()),
        "makespan_s": makespan,
        "node_stage_updates_per_s": node_stages / makespan,
    }, reqs

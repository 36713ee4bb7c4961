#!/usr/bin/env python
"""Throughput of the DGSEM right-hand side + low-storage RK4 step of relaxation
model 1 (van der Waals NSK) on one MI355X.

A step is one full 5-stage RK4 step (every stage: BR1 lifting passes,
temperature recovery, volume and surface integrals, wall and contact-angle
fluxes, relaxation sources, register update) over the whole mesh, on a seeded
synthetic droplet state resident in HBM.  Prints one JSON line.
"""
import argparse
import math
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "node-stage updates/s FP64 vs FP32-mixed at stated error; batched p50/p99 latency"
PEAK_HBM_GBS = 8000.0


def progress(msg):
    """One line per finished phase on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_words_per_node(N, curved=False, fp32=False):
    """Algorithmic words per volume node for each kernel of one stage: every
    array the kernel reads or writes, each element counted once (a face trace
    that an element and its neighbour both read counts once); F = 6/(N+1)
    face points per node. Wall face points also carry grad c in the T2 trace
    (3 words written by lift1, read by lift2 on Navier-slip walls), not
    counted: under 0.1 % of a stage on the wall workloads.  Curved meshes:
    each stage kernel also reads the node metrics (9 Ja + J) and the face
    points' normal and surface element (4 per face point).  FP32 instances
    carry the face temperature's rounding error as a third T2 field (written
    by lift1, read by lift2 on the own face)."""
    F = 6.0 / (N + 1)
    k = {
        "prolong": 6 + 6 * F,             # U in; conserved traces out
        "lift1": 6 + 3 * F,               # U, neighbour c traces in; grad c . n + T traces (2) out
        "lift2": 10 + 15 * F,             # U, conserved traces (own and neighbour: 6), grad c . n + T traces (2)
                                          # in; grad T + lap c (4), flux + wave-speed traces (7) out
        "update": 25.6 + 19 * F,          # U, R, grad T + lap c, neighbour conserved traces (6), flux traces (7)
                                          # in; U, R, conserved traces (6) out; R (6) is read by stages 2-5 and
                                          # written by stages 1-4, so 4/5 of its 12 words per launch of a step
    }
    if fp32:
        k["lift1"] += F
        k["lift2"] += F
    if curved:
        for name in ("lift1", "lift2", "update"):
            k[name] += 10 + 4 * F
    return k


def stage_words_per_node(N, curved=False, fp32=False):
    k = kernel_words_per_node(N, curved, fp32)
    return k["lift1"] + k["lift2"] + k["update"]


TRAFFIC_TABLE = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def measured_traffic(workload, precision, kernel):
    """HBM bytes per launch of `kernel` from the committed counter table
    (rocprofv3 FETCH_SIZE and WRITE_SIZE, each scaled by what the counter
    reads for a plain device copy of known size), or None when the table has
    no entry or was taken on kernels other than the ones built now."""
    from paper_2208_05310_amd.build import kernel_fingerprint
    try:
        with open(TRAFFIC_TABLE) as f:
            tab = json.load(f)
    except (OSError, ValueError):
        return None
    if tab.get("kernel_fingerprint") != kernel_fingerprint():
        return None
    e = tab.get("entries", {}).get(f"{workload}/{precision}", {}).get(kernel)
    if not e:
        return None
    return {"read": e["read_bytes"], "written": e["written_bytes"], "total": e["read_bytes"] + e["written_bytes"]}


def three_phase_bytes_model(N, word):
    """B_floor (state and register read+write) and B_3phase of the BR1
    three-phase byte model, per node-stage."""
    F = 6.0 / (N + 1)
    return 24 * word, (24 + 12 + 2 * F * 35 + 38) * word


def oracle_box(w):
    """The oracle's box for a workload description (walls included)."""
    import oracle
    from paper_2208_05310_amd import workloads as wl
    g = w.side_gamma or (wl.NO_GAMMA,) * 6
    return oracle.make_box(w.N, w.n, (0.0, 0.0, 0.0), w.length, w.periodic, w.side_kind, w.side_twall,
                           w.side_theta, w.curve_amp, side_uwall=w.side_uwall or ((0.0, 0.0, 0.0),) * 6,
                           side_g1=[v[0] for v in g], side_g2=[v[1] for v in g], side_g3=[v[2] for v in g],
                           side_g4=[v[3] for v in g], side_tgrad=w.side_tgrad or ((0.0, 0.0, 0.0),) * 6,
                           side_trate=w.side_trate or (0.0,) * 6, ngeo=w.ngeo)


def host_cpu():
    """The host's CPU model, logical CPU count and the CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(w, budget_s=15.0, single_thread_s=6.0, single_thread_workload=None):
    """The FP64 C oracle on the host's cores (OpenMP over elements): full RK
    steps on the whole workload mesh for about budget_s seconds (at least
    one step), then full RK steps on one thread for about single_thread_s
    seconds on ``single_thread_workload`` (a smaller mesh of the same case
    where one step of the whole mesh would take far longer)."""
    import numpy as np

    import oracle

    def setup(wk):
        o = oracle.Oracle(oracle.make_params(**wk.params), oracle_box(wk))
        U0 = o.init_droplets(wk.T0, wk.centres, wk.radii, wk.width, wk.noise(), wk.velocities, wk.rho_v,
                             wk.rho_l, wk.cylinder_axis)
        return o, U0, o.dt(U0)

    def timed(o, U0, dt, budget, cap):
        U = U0.copy()
        R = np.zeros_like(U)
        steps = 0
        t0 = time.perf_counter()
        while True:
            o.rk_step(U, R, 0.0, dt)
            steps += 1
            el = time.perf_counter() - t0
            if el >= budget or steps >= cap:
                return steps, el

    cores = oracle.get_threads()
    o, U0, dt = setup(w)
    steps, el = timed(o, U0, dt, budget_s, 200)
    nn = o.nnodes
    del o, U0
    w1 = single_thread_workload or w
    o1, U1, dt1 = setup(w1)
    oracle.set_threads(1)
    try:
        steps1, el1 = timed(o1, U1, dt1, single_thread_s, 2000)
    finally:
        oracle.set_threads(cores)
    out = {"value": nn * 5 * steps / el, "unit": "node-stage updates/s", "cores": cores,
           "kind": "oracle",
           "sample": f"{w.name}: {steps} full RK4 step(s) of the FP64 C oracle on the whole mesh "
                     f"({nn} nodes, {cores} OpenMP threads), {el:.1f} s",
           "single_thread": {"value": o1.nnodes * 5 * steps1 / el1, "cores": 1,
                             "sample": f"{w1.name}: {steps1} step(s) on one thread ({o1.nnodes} nodes), "
                                       f"{el1:.1f} s"}}
    out.update(host_cpu())
    return out


def serving_bench(nreq=256, budget_gb=32.0, sequential=True, log=None, max_active_nodes=4_000_000):
    """Continuous batching of the seeded Poisson request stream (FP32-mixed,
    graph-captured batched kernels, autotuned tiles) against the same requests
    solved one at a time with the FP64 single-instance path."""
    from paper_2208_05310_amd import autotune, serving
    from paper_2208_05310_amd import workloads as wl
    reqs = wl.serving_stream(seed=5, count=nreq, rate=50.0)
    pairs = sorted({(w.N, "fp32_mixed") for _, w in reqs})
    t0 = time.perf_counter()
    table = autotune.tune(pairs, path=None)
    t_tune = time.perf_counter() - t0
    stats, _ = serving.serve(reqs, int(budget_gb * 2**30), "fp32_mixed", table,
                             max_active_nodes=max_active_nodes)
    if log:
        log(f"serving batched: p50 {stats['p50_s']:.2f} s, p99 {stats['p99_s']:.2f} s")
    out = {"batched_fp32_mixed": stats, "tiles": {k: v["threads"] for k, v in table.items()},
           "tile_ms_per_step": {k: v["ms_per_step"] for k, v in table.items()},
           "tiles_bitwise_equal": all(v.get("bitwise_equal", False) for v in table.values()),
           "autotune_s": t_tune, "budget_GiB": budget_gb}
    if sequential:
        seq, _ = serving.serve_sequential(reqs, "fp64")
        if log:
            log(f"serving one at a time: p50 {seq['p50_s']:.2f} s, p99 {seq['p99_s']:.2f} s")
        out["one_at_a_time_fp64"] = seq
        out["speedup_throughput"] = stats["node_stage_updates_per_s"] / seq["node_stage_updates_per_s"]
    return out


def _errs(a, b):
    """Relative L2 and max errors of rho and c of state a against state b."""
    out = {}
    for name, k in (("rho", 0), ("c", 5)):
        d = (a[k] - b[k])
        out[f"{name}_rel_l2"] = float(d.norm() / b[k].norm())
        out[f"{name}_rel_max"] = float(d.abs().max() / b[k].abs().max())
    return out


RESTRICTIONS = {"c3": lambda wl: wl.c3(4), "c4": lambda wl: wl.c4(scale=8), "c5": lambda wl: wl.c5(scale=10),
                "c6": lambda wl: wl.c6(scale=10)}


def precision_runs(which="c3", steps=None, restriction=True):
    """FP32-mixed vs FP64 on the GPU over a workload's full step count: both
    forms run the same number of steps from the same initial state with the
    same dt; the relative L2 and max errors of rho (and c) are reported, with
    the plain (uncompensated) FP32 state update beside the compensated one.
    With ``restriction`` the same is run on the small restriction of the
    workload, whose GPU states (FP64 and FP32-mixed) are returned for the
    comparison with the CPU oracle (``oracle_restriction``)."""
    import torch

    from paper_2208_05310_amd import workloads as wl
    from paper_2208_05310_amd.nskr import init_workload, solver_for

    def run(w, prec, U0, dt, kahan=True):
        s = solver_for(w, prec, kahan=kahan)
        U = U0.to(s.dtype).clone()
        R = s.new_state()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.rk_steps(U, R, dt, steps)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        sums = s.reduce(U, check=False)
        del s, R
        return U.double(), t, sums

    w = {"c3": wl.c3, "c4": wl.c4, "c5": wl.c5, "c6": wl.c6}[which]()
    steps = steps or w.steps
    res = {"steps": steps}
    s = solver_for(w, "fp64")
    U0 = init_workload(s, w)
    dt = s.dt(U0)
    del s
    U64, t64, sums64 = run(w, "fp64", U0, dt)
    U32, t32, sums32 = run(w, "fp32_mixed", U0, dt)
    e32 = _errs(U32, U64)
    del U32
    U32p, t32p, _ = run(w, "fp32_mixed", U0, dt, kahan=False)
    e32p = _errs(U32p, U64)
    del U32p, U64, U0
    names = ("mass", "energy", "min_rho", "max_rho", "min_T", "max_T")
    res["full"] = {"workload": w.name, "nodes": w.nnodes, "dt": dt, "fp64_s": t64, "fp32_mixed_s": t32,
                   "speedup": t64 / t32, "fp32_vs_fp64": e32,
                   "fp32_plain_update_s": t32p, "fp32_plain_update_vs_fp64": e32p,
                   "fp64_sums": dict(zip(names, (float(sums64[i]) for i in (0, 4, 10, 11, 12, 13)))),
                   "fp32_mixed_sums": dict(zip(names, (float(sums32[i]) for i in (0, 4, 10, 11, 12, 13))))}
    if not restriction:
        return res, None
    wr = RESTRICTIONS[which](wl)
    sr = solver_for(wr, "fp64")
    Ur = init_workload(sr, wr)
    dtr = sr.dt(Ur)
    del sr
    G64, _, _ = run(wr, "fp64", Ur, dtr)
    G32, _, _ = run(wr, "fp32_mixed", Ur, dtr)
    return res, {"workload": wr, "U0": Ur.double().cpu(), "dt": dtr, "steps": steps,
                 "fp64": G64.cpu(), "fp32_mixed": G32.cpu()}


def oracle_restriction(gpu):
    """The CPU oracle over the same steps of the restriction's initial state,
    and the GPU states (FP64, FP32-mixed) against it."""
    import numpy as np
    import torch

    import oracle
    wr = gpu["workload"]
    o = oracle.Oracle(oracle.make_params(**wr.params), oracle_box(wr))
    Uo = gpu["U0"].numpy().copy()
    Ro = np.zeros_like(Uo)
    t0 = time.perf_counter()
    o.run(Uo, Ro, 0.0, gpu["dt"], gpu["steps"])
    to = time.perf_counter() - t0
    Uo_t = torch.tensor(Uo)
    return {"workload": wr.name, "nodes": int(Uo.shape[1]), "steps": gpu["steps"], "oracle_s": to,
            "fp64_vs_oracle": _errs(gpu["fp64"], Uo_t), "fp32_mixed_vs_oracle": _errs(gpu["fp32_mixed"], Uo_t)}


def precision_study(which="c3", steps=None, restriction=True):
    """GPU precision runs plus, on the restriction, the comparison with the
    CPU oracle (the --precision-study mode)."""
    res, gpu = precision_runs(which, steps, restriction)
    if gpu is not None:
        res["restriction"] = oracle_restriction(gpu)
    return res


def young_laplace(theta, t_end=15.0, precision="fp32_mixed", n=(50, 50, 10), chunk=2000, log=None):
    """Static contact-angle validation (Sec. 4.4.1): the liquid pillar between
    two walls with static angle theta, run to t_end; then the pressure jump
    between the pillar's axis (0.5, 0.5, z) and the vapour column (0, 0.5, z),
    each averaged over z with the quadrature weights, against the
    Young-Laplace law sigma (1/r1 + 1/r2) with r1 = -H / (2 cos theta) and r2
    the pillar's radius at mid-height (the radius of the circle with the
    liquid fraction's area in the two node layers closest to z = H/2); the
    same jump taken in those two layers only (away from the walls) is
    reported beside it.
    sigma_vl and the Maxwell states come from the oracle's thermodynamics."""
    import numpy as np
    import torch

    import oracle
    from paper_2208_05310_amd import workloads as wl
    from paper_2208_05310_amd.nskr import init_workload, solver_for

    w = wl.c8(theta, n)
    pr = w.params
    s = solver_for(w, precision)
    U = init_workload(s, w)
    R = s.new_state()
    dt = s.dt(U)
    nsteps = int(round(t_end / dt))
    rv, rl, _ = oracle.maxwell(w.T0)
    sigma = oracle.sigma(w.T0, pr["gam"])
    H = w.length[2]
    # node coordinates and quadrature weights of the structured mesh
    P = w.N + 1
    xg, wg = np.polynomial.legendre.leggauss(P)
    h = [w.length[d] / w.n[d] for d in range(3)]
    E = w.nelems
    e = np.arange(E)
    ex, ey, ez = e % w.n[0], (e // w.n[0]) % w.n[1], e // (w.n[0] * w.n[1])
    i, j, k = np.meshgrid(np.arange(P), np.arange(P), np.arange(P), indexing="ij")
    i, j, k = i.transpose(2, 1, 0).reshape(-1), j.transpose(2, 1, 0).reshape(-1), k.transpose(2, 1, 0).reshape(-1)
    X = (ex[:, None] + 0.5 * (xg[i][None, :] + 1)) * h[0]
    Y = (ey[:, None] + 0.5 * (xg[j][None, :] + 1)) * h[1]
    Z = (ez[:, None] + 0.5 * (xg[k][None, :] + 1)) * h[2]
    Wz = np.broadcast_to(wg[k][None, :], X.shape)
    Wxy = np.broadcast_to((wg[i] * wg[j])[None, :], X.shape) * (h[0] * h[1] / 4)
    X, Y, Z, Wz, Wxy = (a.reshape(-1) for a in (X, Y, Z, Wz, Wxy))
    near = lambda a, b: np.abs((a - b + 0.5) % 1.0 - 0.5) < 0.5 * h[0]
    axis_l = near(X, 0.5) & near(Y, 0.5)
    axis_v = near(X, 0.0) & near(Y, 0.5)
    zs = np.unique(np.round(Z, 12))
    mid = np.isin(np.round(Z, 12), zs[np.argsort(np.abs(zs - 0.5 * H))[:2]])
    out = torch.empty((5, s.nnodes), dtype=s.dtype, device="cuda:0")

    def measure():
        s.lift2(U, out)
        T = out[0].double().cpu().numpy()
        rho = U[0].double().cpu().numpy()
        p = rho * pr["R"] * T / (1 - pr["b"] * rho) - pr["a"] * rho * rho
        pl = np.sum(p[axis_l] * Wz[axis_l]) / np.sum(Wz[axis_l])
        pv = np.sum(p[axis_v] * Wz[axis_v]) / np.sum(Wz[axis_v])
        # the same jump in the mid-height plane only, away from the walls
        pl_mid = float(np.mean(p[axis_l & mid]))
        pv_mid = float(np.mean(p[axis_v & mid]))
        phi = np.clip((rho - rv) / (rl - rv), 0.0, 1.0)
        area = np.sum(phi[mid] * Wxy[mid]) / 2.0  # two node layers
        r2 = float(np.sqrt(area / np.pi))
        ct = np.cos(np.radians(theta))
        inv_r1 = -2.0 * ct / H
        return {"dp": float(pl - pv), "dp_mid": pl_mid - pv_mid, "r2": r2,
                "young_laplace": float(sigma * (inv_r1 + 1.0 / r2)), "p_liquid": float(pl), "p_vapour": float(pv)}

    history = []
    done = 0
    t0 = time.perf_counter()
    while done < nsteps:
        k_ = min(chunk, nsteps - done)
        s.rk_steps(U, R, dt, k_)
        done += k_
        torch.cuda.synchronize()
        if done % (10 * chunk) == 0 or done == nsteps:
            m = measure()
            m["t"] = done * dt
            history.append(m)
            if log:
                log(f"pillar theta={theta:g}: t={m['t']:.3f} dp={m['dp']:.5f} dp_mid={m['dp_mid']:.5f} "
                    f"young-laplace={m['young_laplace']:.5f} "
                    f"r2={m['r2']:.4f} ({time.perf_counter() - t0:.0f} s)")
    sums = s.reduce(U)
    final = history[-1]
    return {"workload": w.name, "theta_deg": theta, "precision": precision, "dt": dt, "steps": nsteps,
            "t_end": nsteps * dt, "sigma_vl": sigma, "H": H, "final": final,
            "rel_dev": abs(final["dp"] - final["young_laplace"]) / abs(final["young_laplace"]),
            "rel_dev_mid": abs(final["dp_mid"] - final["young_laplace"]) / abs(final["young_laplace"]),
            "history": history[-6:], "wall_s": time.perf_counter() - t0, "mass": float(sums[0])}


def sliding_droplet(gamma1=20.0, scale=4, t_end=0.1, precision="fp64", chunk=5000, log=None):
    """Dynamic contact-angle case (Sec. 4.4.2) at the printed gamma_1: the
    sliding droplet on a mesh coarsened by ``scale``, run to t_end with the
    time-step rule (whose wall limit binds) re-evaluated every ``chunk``
    steps, and the same case at gamma_1 = 0 beside it.  Reports the step
    count, the step range, mass and order-parameter drift, the largest
    speed and the x-centroid of the liquid on the floor's first node layer
    (the contact line's drift under the moving lid)."""
    import numpy as np
    import torch

    from paper_2208_05310_amd import workloads as wl
    from paper_2208_05310_amd.nskr import init_workload, solver_for

    def run(g1):
        w = wl.c6(scale, gamma1=g1)
        s = solver_for(w, precision)
        U = init_workload(s, w)
        R = s.new_state()
        # node a = e P^3 + i + P (j + P k) of element e = ex + n0 (ey + n1 ez)
        P = w.N + 1
        a = np.arange(w.nelems * P ** 3)
        e, i, k = a // P ** 3, a % P, a % P ** 3 // (P * P)
        xg = np.polynomial.legendre.leggauss(P)[0]
        x = (e % w.n[0] + 0.5 * (xg[i] + 1)) * (w.length[0] / w.n[0])
        floor = (e // (w.n[0] * w.n[1]) == 0) & (k == 0)

        def centroid():
            rho = U[0].double().cpu().numpy()
            rv, rl = rho.min(), rho.max()
            phi = np.clip((rho - rv) / (rl - rv), 0, 1)[floor]
            return float(np.sum(phi * x[floor]) / np.sum(phi))

        s0 = s.reduce(U)
        c0 = centroid()
        t, steps, dts, t0, last = 0.0, 0, [], time.perf_counter(), time.perf_counter()
        while t < t_end * (1 - 1e-12):
            dt = s.dt(U)
            k = min(chunk, int(math.ceil((t_end - t) / dt)))
            dt = min(dt, (t_end - t) / k)
            s.rk_steps(U, R, dt, k)
            t += k * dt
            steps += k
            dts.append(dt)
            torch.cuda.synchronize()
            if log and time.perf_counter() - last > 20:
                last = time.perf_counter()
                log(f"sliding droplet gamma_1={g1:g}: t={t:.5f} steps={steps} dt={dt:.3e} "
                    f"({last - t0:.0f} s)")
        s1 = s.reduce(U)
        speed = (U[1:4].double() / U[0].double()).abs().max().item()
        return {"workload": w.name, "gamma_1": g1, "precision": precision, "t_end": t, "steps": steps,
                "dt_min": min(dts), "dt_max": max(dts), "wall_s": time.perf_counter() - t0,
                "mass_rel_drift": abs(s1[0] - s0[0]) / s0[0], "c_rel_drift": abs(s1[5] - s0[5]) / s0[5],
                "max_speed": speed, "rho_min": s1[10], "rho_max": s1[11],
                "floor_liquid_x_centroid": [c0, centroid()]}

    return {"gamma_1_0": run(0.0), f"gamma_1_{gamma1:g}": run(gamma1)}


def copy_bandwidth(mib=1024, reps=5):
    """Device-to-device copy of mib MiB (far above the 256 MB Infinity Cache),
    timed with events: bytes read + written per second, best of reps."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b) * 1e-3)
    del src, dst
    return 2 * n * 8 / best / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "c5", "c6", "c7"],
                    help="c1 4^3 N=3 droplet; c2 16^3 N=4 two droplets; c3 32^3 N=5 eight droplets "
                         "(default); c4 48x48x24 N=3 sessile wall box; c5 50^3 N=3 head-on collision; "
                         "c6 100x50x25 N=3 droplet sliding on a Navier-slip floor under a moving lid; "
                         "c7 the c4 wall box with a graded floor temperature")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-mixed comparison")
    ap.add_argument("--no-serving", action="store_true", help="skip the request-stream measurement")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the FP32-mixed accuracy run over the workload's full step count")
    ap.add_argument("--no-c2", action="store_true", help="skip the 16^3 N=4 throughput line beside the headline")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--serving", action="store_true", help="run only the request-stream serving measurement")
    ap.add_argument("--precision-study", choices=["c3", "c4", "c5", "c6"], default=None,
                    help="FP32-mixed vs FP64 errors over the workload's full step count (c3: 32^3 N=5, "
                         "500 steps; c4: sessile wall case, 1000 steps; c5: head-on collision, 200 steps; "
                         "c6: sliding droplet, 200 steps)")
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--serving-max-nodes", type=int, default=4_000_000)
    ap.add_argument("--threads", type=int, default=None, choices=[128, 192, 256, 448, 512],
                    help="workgroup size of the stage kernels: 256, 512 or the degree's tight size "
                         "(N=2: 192, N=3 and 4: 128, N=5: 448); default: the library's (128 at N=3, "
                         "else 256)")
    ap.add_argument("--young-laplace", type=float, default=None, metavar="THETA",
                    help="static contact-angle validation: liquid pillar with this angle (degrees) to --t-end, "
                         "pressure jump against the Young-Laplace law")
    ap.add_argument("--t-end", type=float, default=15.0)
    ap.add_argument("--sliding-droplet", type=float, default=None, metavar="GAMMA1",
                    help="run the sliding droplet at this gamma_1 (and at 0) to --sliding-t-end")
    ap.add_argument("--sliding-scale", type=int, default=4, help="mesh coarsening of the sliding droplet")
    ap.add_argument("--sliding-t-end", type=float, default=0.1)
    ap.add_argument("--pillar-mesh", default="50,50,10", help="elements of the pillar box (x,y,z)")
    ap.add_argument("--curve-amp", type=float, default=0.0,
                    help="curve the workload's mesh by this amplitude of the sine map (per-node metrics)")
    ap.add_argument("--ngeo", type=int, default=0, help="geometry degree of a curved mesh (0: N)")
    ap.add_argument("--model", type=int, default=1, choices=[1, 2],
                    help="relaxation model: 1 (Rusanov interior flux) or 2 (p_alpha pressure, HLLC flux)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="run one device copy of this many MiB first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the library drives a single GPU",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2208_05310_amd import workloads as wl
    from paper_2208_05310_amd.nskr import init_workload, solver_for

    if args.young_laplace is not None:
        prec = "fp32_mixed" if args.precision == "fp64" and "--precision" not in sys.argv else args.precision
        n = tuple(int(v) for v in args.pillar_mesh.split(","))
        print(json.dumps({"young_laplace": young_laplace(args.young_laplace, args.t_end, prec, n=n, log=progress)}),
              flush=True)
        return
    if args.sliding_droplet is not None:
        print(json.dumps({"sliding_droplet": sliding_droplet(args.sliding_droplet, args.sliding_scale,
                                                             args.sliding_t_end, args.precision, log=progress)}),
              flush=True)
        return
    if args.precision_study:
        print(json.dumps({"precision_study": precision_study(args.precision_study)}), flush=True)
        return
    if args.serving:
        res = serving_bench(args.serving_requests, log=progress, max_active_nodes=args.serving_max_nodes)
        b, q = res["batched_fp32_mixed"], res.get("one_at_a_time_fp64")
        print(json.dumps({"metric": "batched p50/p99 time-to-solution and aggregate node-stage updates/s",
                          "value": b["node_stage_updates_per_s"], "unit": "node-stage updates/s",
                          "p50_s": b["p50_s"], "p99_s": b["p99_s"], "n_gpus": 1, "higher_is_better": True,
                          "data": "synthetic: seeded Poisson stream of droplet solves",
                          "config": {"workload": f"serving_stream_{args.serving_requests}_requests_rate50"},
                          "serving": res}), flush=True)
        return

    if args.copy_calibration_mb > 0:
        n = args.copy_calibration_mb * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = {"c1": wl.c1, "c2": wl.c2, "c3": wl.c3, "c4": wl.c4, "c5": wl.c5, "c6": wl.c6,
         "c7": wl.c7}[args.workload]()
    if args.model == 2:
        w = w.with_(name=f"{w.name}_model2", params=dict(w.params, model=2))
    if args.curve_amp != 0.0:
        w = w.with_(name=f"{w.name}_curved{args.curve_amp:g}_ngeo{args.ngeo or w.N}", curve_amp=args.curve_amp,
                    ngeo=args.ngeo)
    stream = torch.cuda.current_stream()

    def timed_run(wk, precision, U0, dtk):
        """Warm-up + K timed steps of workload wk; returns throughput,
        per-kernel data, final state."""
        s = solver_for(wk, precision)
        if args.threads:
            s.set_block(args.threads)
        threads = s.get_block()
        U = U0.to(s.dtype).clone()
        R = s.new_state()
        s.rk_steps(U, R, dtk, args.warmup, stream)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        s.rk_steps(U, R, dtk, args.steps, stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        wall = t1 - t0
        # per-kernel times: the same K steps once more, each stage dispatch
        # carrying its own event pair (kept out of the pass above: the events
        # cost a few per cent of step time)
        s.set_profiling(True)
        s.rk_steps(U, R, dtk, args.steps, stream)
        torch.cuda.synchronize()
        prof = s.profile(stream)
        s.set_profiling(False)
        word = 8 if precision == "fp64" else 4
        words = kernel_words_per_node(wk.N, wk.curve_amp != 0.0, precision == "fp32_mixed")
        if precision == "fp32_mixed" and s.kahan:
            words["update"] += 12  # compensation of the state update, read and written
        kern = {}
        for k, (ms, cnt) in prof.items():
            if cnt and k in words:
                avg = ms / cnt
                kern[k] = {"avg_us": 1e3 * avg, "launches": cnt,
                           "alg_bytes_per_launch": words[k] * word * s.nnodes,
                           "achieved_GBs": words[k] * word * s.nnodes / (avg * 1e-3) / 1e9}
        sums = s.reduce(U)  # health check of the final state (raises on non-finite)
        nn = s.nnodes
        del s, R
        return {"value": nn * 5 * args.steps / wall, "wall": wall, "gpu_ms": ev0.elapsed_time(ev1),
                "kern": kern, "nnodes": nn, "U": U, "mass": sums[0], "word": word, "threads": threads}

    def initial(wk, precision):
        s = solver_for(wk, precision)
        U = init_workload(s, wk)
        dtk = s.dt(U)
        del s
        return U, dtk

    restr_gpu = None
    U0, dt = initial(w, args.precision)
    r = timed_run(w, args.precision, U0, dt)
    progress(f"{w.name} {args.precision}: {r['value']:.4g} node-stage updates/s")
    nn, value, kern, word = r["nnodes"], r["value"], r["kern"], r["word"]
    dom = max(kern, key=lambda k: kern[k]["avg_us"] * kern[k]["launches"])
    ach = kern[dom]["achieved_GBs"]
    floor_b, b3 = three_phase_bytes_model(w.N, word)
    stage_b = (stage_words_per_node(w.N, w.curve_amp != 0.0, args.precision == "fp32_mixed") +
               (12 if args.precision == "fp32_mixed" else 0)) * word
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "node-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r["wall"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic: seeded droplet state (tanh profiles at Maxwell densities, uniform noise 1e-6)",
        "config": {"workload": w.name, "elements": w.nelems, "N": w.N, "nodes": nn, "threads": r["threads"],
                   "precision": args.precision, "relaxation_model": args.model,
                   "alpha": w.params["alpha"], "beta": w.params["beta"],
                   "T0": w.T0, "dt": dt, "rk": "5-stage 2N RK4(3)5"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": ach / PEAK_HBM_GBS, "traffic": None},
        "kernels": kern,
        "kernel_timing": "HIP event pair carried by each stage dispatch (start/stop of the kernel on the caller's "
                         "stream) over a second pass of the same K steps right after the timed pass",
        "stage_model": {"design_bytes_per_node_stage": stage_b,
                        "design_GBs": value * stage_b / 1e9,
                        "B_3phase_bytes": b3, "B_3phase_GBs": value * b3 / 1e9,
                        "B_floor_bytes": floor_b, "B_floor_GBs": value * floor_b / 1e9},
        "gpu_event_ms": r["gpu_ms"],
        "final_mass": r["mass"],
    }
    # measured HBM bytes per node-stage (lift1 + lift2 + update, counters)
    trs = [measured_traffic(w.name, args.precision, k) for k in ("lift1", "lift2", "update")]
    if all(trs):
        mb = sum(t["total"] for t in trs) / nn
        out["stage_model"]["measured_bytes_per_node_stage"] = mb
        out["stage_model"]["measured_GBs"] = value * mb / 1e9
        out["stage_model"]["measured_frac"] = value * mb / 1e9 / PEAK_HBM_GBS
    tr = measured_traffic(w.name, args.precision, dom)
    if tr:
        alg = kern[dom]["alg_bytes_per_launch"]
        out["roofline"]["traffic"] = tr["total"]
        out["roofline"]["traffic_detail"] = {"unit": "bytes per launch", "read": tr["read"],
                                             "written": tr["written"], "algorithmic": alg,
                                             "ratio_to_algorithmic": tr["total"] / alg}
    if args.precision == "fp64" and not args.no_fp32:
        # the FP32-mixed form on the same workload, initial state and dt: speed and error
        r32 = timed_run(w, "fp32_mixed", U0, dt)
        progress(f"{w.name} fp32_mixed: {r32['value']:.4g} node-stage updates/s")
        a, b_ = r32["U"][0].double(), r["U"][0].double()
        k32 = r32["kern"]
        d32 = max(k32, key=lambda k: k32[k]["avg_us"] * k32[k]["launches"])
        out["fp32_mixed"] = {
            "value": r32["value"], "speedup_vs_fp64": r32["value"] / value,
            "rho_rel_max_err_vs_fp64": float((a - b_).abs().max() / b_.abs().max()),
            "rho_rel_l2_err_vs_fp64": float((a - b_).norm() / b_.norm()),
            "after_steps": args.warmup + 2 * args.steps,
            "roofline": {"kernel": d32, "achieved": k32[d32]["achieved_GBs"], "peak": PEAK_HBM_GBS,
                         "frac": k32[d32]["achieved_GBs"] / PEAK_HBM_GBS},
            "kernels": k32}
        del r32, a, b_
        if not args.no_accuracy and args.workload in RESTRICTIONS and args.model == 1 and args.curve_amp == 0.0:
            # the whole run of the workload (C3: 500 steps) in both forms from
            # the same state and dt, and on the small restriction for the oracle
            acc, restr_gpu = precision_runs(args.workload)
            full = acc["full"]
            out["fp32_mixed"]["accuracy"] = {
                "steps": acc["steps"], "target_rho_rel_max": 1e-5,
                "rho_rel_max_vs_fp64": full["fp32_vs_fp64"]["rho_rel_max"],
                "rho_rel_l2_vs_fp64": full["fp32_vs_fp64"]["rho_rel_l2"],
                "within_target": full["fp32_vs_fp64"]["rho_rel_max"] <= 1e-5,
                "whole_run_speedup_vs_fp64": full["speedup"],
                "plain_fp32_update_rho_rel_max_vs_fp64": full["fp32_plain_update_vs_fp64"]["rho_rel_max"],
                "detail": full}
            progress(f"{w.name} fp32_mixed over {acc['steps']} steps: rho rel max err vs FP64 "
                     f"{full['fp32_vs_fp64']['rho_rel_max']:.2e}")
    if not args.no_c2 and args.workload != "c2" and args.model == 1 and args.curve_amp == 0.0:
        # the 16^3 N=4 throughput case beside the headline
        w2 = wl.c2()
        U2, dt2 = initial(w2, "fp64")
        r2 = timed_run(w2, "fp64", U2, dt2)
        k2 = r2["kern"]
        d2 = max(k2, key=lambda k: k2[k]["avg_us"] * k2[k]["launches"])
        c2 = {"workload": w2.name, "nodes": r2["nnodes"], "value": r2["value"],
              "ms_per_step": 1e3 * r2["wall"] / args.steps,
              "roofline": {"kernel": d2, "achieved": k2[d2]["achieved_GBs"], "peak": PEAK_HBM_GBS,
                           "frac": k2[d2]["achieved_GBs"] / PEAK_HBM_GBS}, "kernels": k2}
        del r2
        if not args.no_fp32:
            r2f = timed_run(w2, "fp32_mixed", U2, dt2)
            c2["fp32_mixed_value"] = r2f["value"]
            c2["fp32_mixed_speedup"] = r2f["value"] / c2["value"]
            del r2f
        del U2
        out["c2"] = c2
        progress(f"{w2.name} fp64: {c2['value']:.4g} node-stage updates/s")
    if not args.no_serving:
        try:
            res = serving_bench(args.serving_requests, max_active_nodes=args.serving_max_nodes, log=progress)
            bt, sq = res["batched_fp32_mixed"], res.get("one_at_a_time_fp64", {})
            out["serving"] = {"requests": bt["requests"], "errors": bt["errors"], "p50_s": bt["p50_s"],
                              "p99_s": bt["p99_s"],
                              "aggregate_node_stage_updates_per_s": bt["node_stage_updates_per_s"],
                              "one_at_a_time_fp64": {k: sq.get(k) for k in ("p50_s", "p99_s",
                                                                             "node_stage_updates_per_s")},
                              "throughput_speedup": res.get("speedup_throughput"), "tiles": res["tiles"],
                              "tile_ms_per_step": res["tile_ms_per_step"],
                              "tiles_bitwise_equal": res["tiles_bitwise_equal"],
                              "max_active_nodes": args.serving_max_nodes}
        except Exception as e:  # reported, never hides the main measurement
            out["serving"] = {"error": repr(e)}
    # the same figures against a measured device copy (the attainable HBM rate)
    cp = copy_bandwidth()
    out["roofline"]["copy_GBs"] = cp
    out["roofline"]["frac_of_copy"] = ach / cp
    if "measured_GBs" in out["stage_model"]:
        out["stage_model"]["measured_frac_of_copy"] = out["stage_model"]["measured_GBs"] / cp
    del r, U0
    if not args.no_cpu_baseline:
        small = RESTRICTIONS[args.workload](wl) if args.workload in RESTRICTIONS else None
        if small is not None and args.model == 2:
            small = small.with_(name=f"{small.name}_model2", params=dict(small.params, model=2))
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget, single_thread_workload=small)
        progress(f"cpu baseline: {out['cpu_baseline']['sample']}")
        acc = out.get("fp32_mixed", {}).get("accuracy")
        if acc is not None and restr_gpu is not None:
            # the oracle over the same steps of the small restriction, against
            # both GPU forms
            rr = oracle_restriction(restr_gpu)
            acc["restriction_vs_oracle"] = rr
            progress(f"{rr['workload']} over {rr['steps']} steps: FP64 vs oracle rho rel max "
                     f"{rr['fp64_vs_oracle']['rho_rel_max']:.2e}, FP32-mixed vs oracle "
                     f"{rr['fp32_mixed_vs_oracle']['rho_rel_max']:.2e}")
    print(json.dumps(out), flush=True)
    # leave nothing behind: every library context is released before the
    # interpreter exits, and the device is idle
    import gc
    gc.collect()
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()

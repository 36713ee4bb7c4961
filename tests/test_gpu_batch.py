"""Batched, graph-captured execution and the serving loop (through the C ABI).

* The workgroup size the autotuner picks does not change results.
* A batched instance equals, bit for bit, the same instance on the
  single-instance path (same kernels, same arithmetic, same order).
* An instance gives bitwise the same result alone in a batch and in a mix of
  instances with other degrees, meshes, precisions, relaxation models, wall
  conditions and time steps.
* Graph replays equal direct launches on every step, with eager work and
  synchronisations between the replays.
* Admission respects the memory budget; instances stop at their own step count.
* Walls whose temperature changes in time: each batch instance runs on its
  own clock from its time at admission (bitwise equal to the single-instance
  path, also across a retirement and a new admission), and the context time
  advances as nskr_rk_steps advances it.
"""
import numpy as np
import pytest

from helpers import timed_wall_case
from paper_2208_05310_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def small_mix():
    base = wl.c1()
    return [
        (base.with_(name="mix_periodic_3x3x3_N3", n=(3, 3, 3)), "fp64"),
        (wl.c4(scale=12).with_(name="mix_wall_4x4x2_N4", N=4), "fp64"),
        (base.with_(name="mix_periodic_4x4x4_N2_T080", N=2, T0=0.8), "fp32_mixed"),
        (base.with_(name="mix_periodic_2x3x2_N5", N=5, n=(2, 3, 2), length=(1.0, 1.5, 1.0), noise_seed=9), "fp64"),
        (base.with_(name="mix_model2_3x3x3_N3", n=(3, 3, 3), params=dict(base.params, model=2)), "fp64"),
        # Navier-slip walls (gamma_1 pass), a moving heat-transfer lid and a
        # graded wall temperature (table pass)
        (wl.c4(scale=12).with_(
            name="mix_navier_graded_4x4x2_N3", side_kind=(0, 0, 0, 0, wl.NAVIER, wl.NAVIER),
            side_twall=(0.0, 0.0, 0.0, 0.0, 0.85, 0.9), side_theta=(90.0, 90.0, 90.0, 90.0, 60.0, 120.0),
            side_uwall=((0.0, 0.0, 0.0),) * 5 + ((0.1, 0.0, 0.0),),
            side_gamma=(wl.NO_GAMMA,) * 4 + ((1e-3, 0.05, float("inf"), 0.1), (0.0, 0.1, 0.02, 0.0)),
            side_tgrad=((0.0, 0.0, 0.0),) * 4 + ((0.08, 0.0, 0.0), (0.0, -0.05, 0.0))), "fp64"),
        # degenerate meshes: walls on every side, and one element that is
        # its own neighbour through every face
        (wl.c4(scale=12).with_(
            name="mix_closed_box_4x4x2_N3", periodic=(0, 0, 0),
            side_kind=(wl.NOSLIP_CA, wl.SLIP, wl.NAVIER, wl.NOSLIP_CA, wl.NOSLIP_CA, wl.SLIP),
            side_twall=(0.9, 0.0, 0.88, 0.87, 0.9, 0.0), side_theta=(60.0, 90.0, 110.0, 90.0, 60.0, 90.0),
            side_gamma=(wl.NO_GAMMA,) * 2 + ((0.0, 0.05, 0.02, 0.0),) + (wl.NO_GAMMA,) * 3), "fp64"),
        (base.with_(name="mix_self_periodic_1x1x1_N4", N=4, n=(1, 1, 1)), "fp32_mixed"),
    ]


def setup(w, prec, threads=256):
    from paper_2208_05310_amd.nskr import init_workload, solver_for
    s = solver_for(w, prec)
    s.set_block(threads)
    U = init_workload(s, w)
    R = s.new_state()
    dt = s.dt(U)
    return s, U, R, dt


def rel(a, b):
    a = a.double().cpu().numpy()
    b = b.double().cpu().numpy()
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_block_size_does_not_change_results(torch_cuda, N, prec):
    """Every workgroup size the autotuner may pick gives the 256-thread result
    bit for bit (a ragged mesh: the last workgroup is partly empty)."""
    torch = torch_cuda
    from paper_2208_05310_amd.autotune import block_sizes
    w = wl.c1().with_(name=f"tiles_N{N}", N=N, n=(3, 3, 3))
    from paper_2208_05310_amd.nskr import solver_for
    assert solver_for(w, prec).get_block() == (128 if N == 3 else 256)   # the library's default
    s1, U1, R1, dt = setup(w, prec, 256)
    s1.rk_steps(U1, R1, dt, 3)
    for bs in block_sizes(N):
        if bs == 256:
            continue
        print(f"[case] block size {bs} N={N} {prec}", flush=True)
        s2, U2, R2, _ = setup(w, prec, bs)
        s2.rk_steps(U2, R2, dt, 3)
        torch.cuda.synchronize()
        print("bitwise equal:", torch.equal(U1, U2), "rel diff", rel(U2, U1), flush=True)
        assert torch.equal(U1, U2), rel(U2, U1)


def test_batched_equals_single_and_alone_equals_mix(torch_cuda):
    torch = torch_cuda
    from paper_2208_05310_amd.nskr import Batch
    cases = small_mix()
    nsteps = 4
    # single-instance path
    single = []
    for w, prec in cases:
        s, U, R, dt = setup(w, prec)
        s.rk_steps(U, R, dt, nsteps)
        single.append(U)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    # each instance alone in a batch
    alone = []
    for w, prec in cases:
        b = Batch(1 << 34)
        s, U, R, dt = setup(w, prec)
        assert b.admit(s, U, R, dt, nsteps) is not None
        for _ in range(nsteps):
            b.step(stream)
        stream.synchronize()
        alone.append(U)
    # all together
    b = Batch(1 << 34)
    held = []
    for w, prec in cases:
        s, U, R, dt = setup(w, prec)
        assert b.admit(s, U, R, dt, nsteps) is not None
        held.append(U)
    for _ in range(nsteps):
        b.step(stream)
    stream.synchronize()
    assert sorted(b.poll()) == list(range(len(cases)))
    for k, (w, prec) in enumerate(cases):
        print(f"[case] {w.name}: mix==alone {torch.equal(held[k], alone[k])}, "
              f"batched vs single {rel(alone[k], single[k]):.2e}", flush=True)
        assert torch.equal(held[k], alone[k])
        print(f"[case] {w.name}: batched == single bitwise: {torch.equal(alone[k], single[k])}", flush=True)
        assert torch.equal(alone[k], single[k])


def test_graph_replays_equal_direct_launches(torch_cuda):
    torch = torch_cuda
    from paper_2208_05310_amd.nskr import Batch
    cases = small_mix()[:3]
    stream = torch.cuda.Stream()
    outs = {}
    for graph in (False, True):
        b = Batch(1 << 34, graph=graph)
        Us = []
        for w, prec in cases:
            s, U, R, dt = setup(w, prec)
            b.admit(s, U, R, dt, 6)
            Us.append(U)
        snaps = []
        for k in range(6):
            b.step(stream)
            stream.synchronize()
            # eager work between replays on another stream
            junk = torch.randn(1 << 16, device="cuda:0").sum().item()
            snaps.append([U.clone() for U in Us])
        outs[graph] = snaps
    for k in range(6):
        for j in range(len(cases)):
            assert torch.equal(outs[True][k][j], outs[False][k][j]), (k, j)


def test_budget_admission_and_step_counts(torch_cuda):
    torch = torch_cuda
    from paper_2208_05310_amd.nskr import Batch
    w = wl.c1().with_(name="budget_3x3x3", n=(3, 3, 3))
    s1, U1, R1, dt1 = setup(w, "fp64")
    need = s1.device_bytes() + 2 * U1.numel() * 8
    b = Batch(int(need * 1.5))
    stream = torch.cuda.Stream()
    assert b.admit(s1, U1, R1, dt1, 3) is not None
    s2, U2, R2, dt2 = setup(w.with_(noise_seed=5), "fp64")
    assert b.admit(s2, U2, R2, dt2, 5) is None          # no room now
    for _ in range(3):
        b.step(stream)
    stream.synchronize()  # poll reports a slot once its last step has run
    assert b.poll() == [0]
    b.retire(0)
    assert b.admit(s2, U2, R2, dt2, 5) is not None      # room after retirement
    for _ in range(5):
        b.step(stream)
    stream.synchronize()
    assert b.info()["active"] == 0 and len(b.poll()) == 1
    # same results as the single-instance path with the same step counts
    s3, U3, R3, dt3 = setup(w, "fp64")
    s3.rk_steps(U3, R3, dt3, 3)
    s4, U4, R4, dt4 = setup(w.with_(noise_seed=5), "fp64")
    s4.rk_steps(U4, R4, dt4, 5)
    torch.cuda.synchronize()
    assert torch.equal(U1, U3) and torch.equal(U2, U4)


def test_serving_loop_small_stream(torch_cuda):
    """A short request stream through the continuous-batching loop: every
    request completes, and its result equals the same request solved alone."""
    torch = torch_cuda
    from paper_2208_05310_amd import serving
    from paper_2208_05310_amd.nskr import Batch
    reqs = [(t, w.with_(steps=6, n=(min(w.n[0], 8),) * 3)) for t, w in wl.serving_stream(seed=5, count=8, rate=200.0)]
    stats, done = serving.serve(reqs, budget_bytes=1 << 32, precision="fp32_mixed", keep_results=True)
    print(stats, flush=True)
    assert stats["requests"] == 8 and all(r.t_done is not None for r in done)
    assert stats["errors"] == 0 and all(r.status == "ok" for r in done)
    assert stats["p99_s"] >= stats["p50_s"] > 0
    stream = torch.cuda.Stream()
    for r in done[:4]:
        b = Batch(1 << 34)
        s, U, R, dt = setup(r.w, "fp32_mixed")
        b.admit(s, U, R, dt, r.w.steps)
        for _ in range(r.w.steps):
            b.step(stream)
        stream.synchronize()
        assert np.array_equal(U.double().cpu().numpy(), r.result), r.w.name
    # and the served (FP32-mixed) results against the CPU oracle over the same
    # steps and dt from its own initial state: density within 1e-5
    from helpers import oracle_for, oracle_init
    for r in done:
        o = oracle_for(r.w)
        Uo = oracle_init(o, r.w)
        Ro = np.zeros_like(Uo)
        o.run(Uo, Ro, 0.0, r.dt, r.w.steps)
        err = np.max(np.abs(r.result[0] - Uo[0])) / np.max(np.abs(Uo[0]))
        print(f"[case] served {r.w.name} rho vs oracle {err:.2e}", flush=True)
        assert err <= 1e-5


@pytest.mark.parametrize("graph", [True, False])
def test_time_dependent_walls_in_a_batch(torch_cuda, graph):
    torch = torch_cuda
    from paper_2208_05310_amd.nskr import Batch
    timed = timed_wall_case()
    # two timed instances with their own start times and steps, and one whose
    # walls do not change in time (same group: degree 3, fp64)
    cases = [(timed, 0.15, 5), (timed.with_(noise_seed=4), 0.02, 3), (small_mix()[0][0], 0.0, 4)]
    print(f"[case] time-dependent walls in a batch, graph={graph}", flush=True)
    single, times = [], []
    for w, t0, n in cases:
        s, U, R, dt = setup(w, "fp64")
        s.set_time(t0)
        s.rk_steps(U, R, dt, n)
        single.append(U)
        times.append(s.get_time())
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    b = Batch(1 << 34, graph=graph)
    held = []
    for w, t0, n in cases:
        s, U, R, dt = setup(w, "fp64")
        s.set_time(t0)
        assert b.admit(s, U, R, dt, n) is not None
        held.append((s, U))
    for _ in range(max(n for _, _, n in cases)):
        b.step(stream)
    stream.synchronize()
    for k, (w, t0, n) in enumerate(cases):
        s, U = held[k]
        print(f"[case] {w.name} t0={t0}: batched == single bitwise: {torch.equal(U, single[k])}", flush=True)
        assert torch.equal(U, single[k])
        assert s.get_time() == times[k]
    # retire after 2 of 5 steps, admit again for 3 more: equals rk_steps(2)
    # then rk_steps(3) (the second call starts from the advanced time)
    w, t0 = timed, 0.15
    s, U, R, dt = setup(w, "fp64")
    s.set_time(t0)
    s.rk_steps(U, R, dt, 2)
    s.rk_steps(U, R, dt, 3)
    torch.cuda.synchronize()
    s2, U2, R2, _ = setup(w, "fp64")
    s2.set_time(t0)
    b = Batch(1 << 34, graph=graph)
    k = b.admit(s2, U2, R2, dt, 5)
    for _ in range(2):
        b.step(stream)
    b.retire(k)
    assert s2.get_time() == t0 + 2 * dt
    assert b.admit(s2, U2, R2, dt, 3) is not None
    for _ in range(3):
        b.step(stream)
    stream.synchronize()
    print("retire and admit again: bitwise", torch.equal(U2, U), flush=True)
    assert torch.equal(U2, U)
    assert s2.get_time() == s.get_time()



def test_batched_mix_matches_the_oracle(torch_cuda):
    """Every instance of the mixed batch, advanced together, against the CPU
    oracle over the same steps from the same initial state and dt: FP64
    instances within 1e-12 per conserved field (momenta floored at |rho|
    |c~|), FP32-mixed ones within 1e-5 in density."""
    torch = torch_cuda
    from helpers import oracle_for, oracle_init
    from paper_2208_05310_amd.nskr import Batch, solver_for
    nsteps = 4
    b = Batch(1 << 34)
    stream = torch.cuda.Stream()
    runs = []
    for w, prec in small_mix():
        o = oracle_for(w)
        U0 = oracle_init(o, w)
        dt = o.dt(U0)
        s = solver_for(w, prec)
        U = torch.tensor(U0, dtype=s.dtype, device="cuda:0")
        R = s.new_state()
        assert b.admit(s, U, R, dt, nsteps) is not None
        runs.append((w, prec, o, U0, dt, s, U))
    for _ in range(nsteps):
        b.step(stream)
    stream.synchronize()
    for w, prec, o, U0, dt, s, U in runs:
        Uo = U0.copy()
        Ro = np.zeros_like(Uo)
        o.run(Uo, Ro, 0.0, dt, nsteps)
        Ug = U.double().cpu().numpy()
        if prec == "fp64":
            pr = w.params
            cs = np.sqrt(abs((1 + 1 / pr["cv"]) * pr["R"] * w.T0 / (1 - pr["b"] * Uo[0].max()) ** 2))
            floor = [0.0] + [np.max(np.abs(Uo[0])) * cs] * 3 + [0.0, 0.0]
            err = np.array([np.max(np.abs(Ug[f] - Uo[f])) / max(np.max(np.abs(Uo[f])), floor[f])
                            for f in range(6)])
            print(f"[case] batched {w.name} vs oracle: {err}", flush=True)
            assert np.all(err <= 1e-12), err
        else:
            err = np.max(np.abs(Ug[0] - Uo[0])) / np.max(np.abs(Uo[0]))
            print(f"[case] batched {w.name} (fp32-mixed) rho vs oracle: {err:.2e}", flush=True)
            assert err <= 1e-5


def test_poll_reports_completed_steps_and_retire_waits_for_queued_ones(torch_cuda):
    """A finished slot is reported once its last step has run; retiring a
    slot whose steps are still queued returns after they ran, so the state
    equals the single-instance path after the same steps; the context can be
    admitted again at once (its compensation is cleared on the step stream)."""
    torch = torch_cuda
    from paper_2208_05310_amd.nskr import Batch
    w = wl.c2()
    stream = torch.cuda.Stream()
    s, U, R, dt = setup(w, "fp32_mixed")
    ref = U.clone()
    Rr = s.new_state()
    s.rk_steps(ref, Rr, dt, 3)
    torch.cuda.synchronize()
    b = Batch(1 << 34)
    slot = b.admit(s, U, R, dt, 10)
    with torch.cuda.stream(stream):
        for _ in range(3):
            b.step(stream)
    b.retire(slot)              # waits for the three queued steps
    assert torch.equal(U, ref)
    # admitted again right away: the next 2 steps equal 2 more single steps
    slot = b.admit(s, U, R, dt, 2)
    with torch.cuda.stream(stream):
        for _ in range(2):
            b.step(stream)
    stream.synchronize()
    assert b.poll() == [slot]
    s.rk_steps(ref, Rr, dt, 2)
    torch.cuda.synchronize()
    b.retire(slot)
    assert torch.equal(U, ref)

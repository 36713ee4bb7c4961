"""Health checks and argument errors through the C ABI (GPU).

* A non-finite value in the state is counted by nskr_reduce, which reports
  NSKR_E_NONFINITE, and nskr_dt refuses to produce a time step from it.
* Densities outside (0, 1/b) and non-positive temperatures are counted.
* Invalid arguments (non-positive dt, aliasing state and register, wrong
  buffer sizes, an instance admitted twice) are rejected before any launch,
  and the context stays usable afterwards.
* The same steps twice give the same bits (races would show as run-to-run
  differences); an unstable time step is caught by the health check within
  a few steps; a poisoned instance of a batch fails its own health check
  and leaves the other instances bitwise unchanged.
"""
import numpy as np
import pytest

from paper_2208_05310_amd import workloads as wl

pytestmark = pytest.mark.gpu

CNT_NONFINITE, CNT_RHO_RANGE, CNT_T_NONPOS = 14, 15, 16


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def setup(precision="fp64"):
    from paper_2208_05310_amd.nskr import init_workload, solver_for
    w = wl.c1()
    s = solver_for(w, precision)
    U = init_workload(s, w)
    return w, s, U


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_nonfinite_state_is_detected(torch_cuda, precision):
    torch = torch_cuda
    from paper_2208_05310_amd.nskr import NSKR_E_NONFINITE, NskrError
    print(f"[case] non-finite state, {precision}", flush=True)
    w, s, U = setup(precision)
    sums = s.reduce(U)
    assert sums[CNT_NONFINITE] == 0 and sums[CNT_RHO_RANGE] == 0 and sums[CNT_T_NONPOS] == 0
    U[4, 123] = float("nan")
    torch.cuda.synchronize()
    with pytest.raises(NskrError) as ei:
        s.reduce(U)
    assert ei.value.code == NSKR_E_NONFINITE
    sums = s.reduce(U, check=False)
    assert sums[CNT_NONFINITE] >= 1
    with pytest.raises(NskrError) as ei:
        s.dt(U)
    assert ei.value.code == NSKR_E_NONFINITE


def test_out_of_range_density_and_temperature_are_counted(torch_cuda):
    torch = torch_cuda
    print("[case] density above 1/b and a non-positive temperature", flush=True)
    w, s, U = setup()
    U[0, 7] = 3.5                      # above the van der Waals limit 1/b = 3
    U[4, 300] = -50.0                  # internal energy far below zero: T < 0
    torch.cuda.synchronize()
    sums = s.reduce(U, check=False)
    print("counters", sums[CNT_NONFINITE:CNT_T_NONPOS + 1], flush=True)
    assert sums[CNT_RHO_RANGE] >= 1
    assert sums[CNT_T_NONPOS] >= 1


def test_invalid_arguments_are_rejected_and_context_survives(torch_cuda):
    torch = torch_cuda
    from paper_2208_05310_amd.nskr import NSKR_E_ARG, Batch, NskrError
    print("[case] invalid arguments", flush=True)
    w, s, U = setup()
    R = s.new_state()
    dt = s.dt(U)
    U0 = U.clone()
    for bad in (0.0, -dt, float("nan"), float("inf")):
        with pytest.raises(NskrError) as ei:
            s.rk_steps(U, R, bad, 1)
        assert ei.value.code == NSKR_E_ARG
    with pytest.raises(NskrError) as ei:
        s.rk_steps(U, U, dt, 1)        # state and register alias
    assert ei.value.code == NSKR_E_ARG
    with pytest.raises(ValueError):
        s.rk_steps(U[:, :-1].contiguous(), R, dt, 1)
    torch.cuda.synchronize()
    assert torch.equal(U, U0)          # nothing ran
    b = Batch(1 << 34)
    with pytest.raises(NskrError):
        b.admit(s, U, R, -1.0, 3)
    assert b.admit(s, U, R, dt, 3) is not None
    with pytest.raises(NskrError):
        b.admit(s, U, R, dt, 3)        # the same instance twice
    # the context still works after the rejected calls
    s2 = s
    U2, R2 = U0.clone(), s2.new_state()
    s2.rk_steps(U2, R2, dt, 2)
    torch.cuda.synchronize()
    assert np.isfinite(U2.cpu().numpy()).all()


def test_invalid_walls_are_rejected(torch_cuda):
    """A wall velocity with a normal component, a negative Navier-slip
    coefficient, an unknown wall kind and a wall temperature leaving the
    table's range are argument errors at mesh upload."""
    from paper_2208_05310_amd import workloads as wl
    from paper_2208_05310_amd.nskr import NSKR_E_ARG, NskrError, Solver
    print("[case] invalid walls", flush=True)
    w = wl.c6(scale=10)
    bad = [
        dict(side_uwall=((0.0, 0.0, 0.0),) * 5 + ((0.5, 0.0, 0.01),)),          # lid moving through itself
        dict(side_gamma=(wl.NO_GAMMA,) * 4 + ((20.0, -1e-4, float("inf"), 0.0), wl.NO_GAMMA)),
        dict(side_kind=(0, 0, 0, 0, 4, 1)),
        dict(side_tgrad=((0.0, 0.0, 0.0),) * 4 + ((0.2, 0.0, 0.0), (0.0, 0.0, 0.0))),  # floor reaches 1.05
    ]
    for kw in bad:
        v = w.with_(**kw)
        s = Solver(v.params, v.N, "fp64")
        with pytest.raises((NskrError, ValueError)) as ei:
            s.upload_box(v.n, v.length, v.periodic, v.side_kind, v.side_twall, v.side_theta,
                         side_uwall=v.side_uwall, side_gamma=v.side_gamma, side_tgrad=v.side_tgrad)
        if isinstance(ei.value, NskrError):
            assert ei.value.code == NSKR_E_ARG


RUN_TWICE = [
    (wl.c1(), "fp64"),
    (wl.c4(scale=12).with_(name="wall_4x4x2_N4", N=4), "fp32_mixed"),
    (wl.c1().with_(name="curved_3x3x3_N5", N=5, n=(3, 3, 3), curve_amp=0.04), "fp64"),
    (wl.c6(scale=10), "fp64"),
]


@pytest.mark.parametrize("w,precision", RUN_TWICE, ids=[f"{w.name}_{p}" for w, p in RUN_TWICE])
def test_run_twice_is_bitwise_identical(torch_cuda, w, precision):
    """The same steps from the same state give the same bits: no kernel reads
    LDS or memory that another thread may still be writing (a race shows as
    run-to-run differences)."""
    torch = torch_cuda
    from paper_2208_05310_amd.nskr import init_workload, solver_for
    print(f"[case] run twice {w.name} {precision}", flush=True)
    s = solver_for(w, precision)
    U = init_workload(s, w)
    dt = s.dt(U)
    outs = []
    for _ in range(2):
        V, R = U.clone(), s.new_state()
        s.rk_steps(V, R, dt, 5)
        outs.append(V)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])


def test_unstable_time_step_is_detected(torch_cuda):
    """At 100 times the stable step the relaxation source blows up; the health
    check reports it within a few steps."""
    torch = torch_cuda
    from paper_2208_05310_amd.nskr import NSKR_E_NONFINITE, NskrError
    print("[case] 100 x dt", flush=True)
    w, s, U = setup()
    dt = 100.0 * s.dt(U)
    R = s.new_state()
    found = None
    for k in range(1, 11):
        s.rk_steps(U, R, dt, 1)
        try:
            s.reduce(U)
        except NskrError as e:
            assert e.code == NSKR_E_NONFINITE
            found = k
            break
    print("detected after", found, "steps", flush=True)
    assert found is not None
    sums = s.reduce(U, check=False)
    print("counters", sums[CNT_NONFINITE:CNT_T_NONPOS + 1], flush=True)
    assert sums[CNT_NONFINITE] + sums[CNT_RHO_RANGE] + sums[CNT_T_NONPOS] >= 1
    # nskr_dt refuses a state once its rates are not finite (a density above
    # 1/b alone still gives finite rates)
    if sums[CNT_NONFINITE] > 0:
        with pytest.raises(NskrError):
            s.dt(U)


def test_poisoned_instance_leaves_the_others_of_a_batch_unchanged(torch_cuda):
    """A NaN written into one instance's state between batch steps: that
    instance's health check fails at the end, the other instances end bit for
    bit as in the same batch without the poison."""
    torch = torch_cuda
    from paper_2208_05310_amd.nskr import NSKR_E_NONFINITE, Batch, NskrError, init_workload, solver_for
    cases = [(wl.c1().with_(name="p_periodic_3x3x3_N3", n=(3, 3, 3)), "fp64"),
             (wl.c4(scale=12).with_(name="p_wall_4x4x2_N4", N=4), "fp64"),
             (wl.c1().with_(name="p_periodic_4x4x4_N2", N=2), "fp32_mixed")]
    stream = torch.cuda.Stream()

    def run(poison):
        b = Batch(1 << 34)
        held = []
        for w, prec in cases:
            s = solver_for(w, prec)
            U = init_workload(s, w)
            R = s.new_state()
            dt = s.dt(U)
            assert b.admit(s, U, R, dt, 6) is not None
            held.append((s, U, R))
        for k in range(6):
            if poison and k == 2:
                stream.synchronize()
                held[1][1][0, 17] = float("nan")
                torch.cuda.synchronize()
            b.step(stream)
        stream.synchronize()
        assert sorted(b.poll()) == [0, 1, 2]
        for slot in range(3):
            b.retire(slot)
        return held

    print("[case] poisoned batch instance", flush=True)
    clean, bad = run(False), run(True)
    for k in (0, 2):
        assert torch.equal(clean[k][1], bad[k][1]), cases[k][0].name
        bad[k][0].reduce(bad[k][1])
    with pytest.raises(NskrError) as ei:
        bad[1][0].reduce(bad[1][1])
    assert ei.value.code == NSKR_E_NONFINITE

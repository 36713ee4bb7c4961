"""Health checks and argument errors through the C ABI (GPU).

* A non-finite value in the state is counted by nskr_reduce, which reports
  NSKR_E_NONFINITE, and nskr_dt refuses to produce a time step from it.
* Densities outside (0, 1/b) and non-positive temperatures are counted.
* Invalid arguments (non-positive dt, aliasing state and register, wrong
  buffer sizes, an instance admitted twice) are rejected before any launch,
  and the context stays usable afterwards.
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

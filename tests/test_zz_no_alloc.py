"""The allocation-free time step (nskr_dt_noalloc) against nskr_dt through
the C ABI: the same value, bit for bit, on two calls in a row on one device,
the second on a smaller mesh (the static reduction scratch keeps the first
call's contents and must not leak into the second), in both precisions."""
import pytest

from paper_2208_05310_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_dt_noalloc_equals_dt_on_two_calls_the_second_smaller(torch_cuda, precision):
    from paper_2208_05310_amd.nskr import init_workload, solver_for
    big, small = wl.c2(), wl.c1()
    print(f"dt_noalloc: {precision} {big.name} then {small.name}", flush=True)
    sb = solver_for(big, precision)
    Ub = init_workload(sb, big)
    ss = solver_for(small, precision)
    Us = init_workload(ss, small)
    torch_cuda.cuda.synchronize()
    ref_b, ref_s = sb.dt(Ub), ss.dt(Us)
    got_b = sb.dt_noalloc(Ub)
    got_s = ss.dt_noalloc(Us)
    assert got_b == ref_b, (got_b, ref_b)
    assert got_s == ref_s, (got_s, ref_s)
    assert got_b != got_s
    # and once more in the other order: nothing of the previous call remains
    assert sb.dt_noalloc(Ub) == ref_b


def test_dt_noalloc_rejects_null_arguments(torch_cuda):
    import ctypes

    from paper_2208_05310_amd.nskr import NSKR_E_ARG, solver_for
    w = wl.c1()
    s = solver_for(w, "fp64")
    v = ctypes.c_double()
    assert s.L.nskr_dt_noalloc(s._h, None, ctypes.byref(v), None) == NSKR_E_ARG

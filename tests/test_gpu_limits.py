"""Mesh size limits of one context (GPU).

The stage kernels address node- and element-indexed arrays with 32-bit byte
offsets from a per-field base, so the mesh upload refuses a mesh for which
any such array would reach 4 GiB; at N = 5 the bound is set by the face-point
arrays (E x 6 faces x 36 points x 4 values): 621 378 elements in FP64,
1 242 757 in FP32-mixed.

* An empty mesh is an argument error, a mesh just over the bound is refused
  as unsupported before anything is allocated, and the context then still
  takes a normal mesh.
* A periodic mesh just under the bound, filled with copies of a 4^3-element
  droplet box, runs one RK step in which every copy stays bit for bit equal
  to the 4^3 box run by itself (the elements and faces at the highest
  addresses included): the arithmetic of an element does not depend on where
  its data sit.
"""
import pytest

from helpers import upload_rc
from paper_2208_05310_amd import workloads as wl

pytestmark = pytest.mark.gpu

TILE = 4          # elements per side of the copied droplet box (h = 1/4)
LIMITS = {"fp64": ((96, 100, 64), (92, 92, 74)),         # 614 400 under, 626 336 over
          "fp32_mixed": ((96, 100, 128), (96, 100, 130))}  # 1 228 800 under, 1 248 000 over


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def droplet_tile():
    return wl.c1().with_(name="droplet_periodic_4x4x4_N5", N=5, n=(TILE,) * 3)


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_empty_and_oversized_meshes_are_refused(torch_cuda, precision):
    from paper_2208_05310_amd.nskr import NSKR_E_ARG, NSKR_E_UNSUPPORTED, Solver, box_mesh
    w = droplet_tile()
    s = Solver(w.params, w.N, precision)
    small = box_mesh(w.n)
    print(f"[case] {precision}: empty mesh", flush=True)
    assert upload_rc(s, small, nelems=0) == NSKR_E_ARG
    over = LIMITS[precision][1]
    print(f"[case] {precision}: {over} elements, over the 4 GiB bound", flush=True)
    assert upload_rc(s, box_mesh(over)) == NSKR_E_UNSUPPORTED
    assert s.device_bytes() == 0
    print(f"[case] {precision}: a normal mesh afterwards", flush=True)
    assert upload_rc(s, small) == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_largest_mesh_runs_every_copy_like_the_small_box(torch_cuda, precision):
    torch = torch_cuda
    from paper_2208_05310_amd.nskr import Solver, init_workload, solver_for
    w = droplet_tile()
    small = solver_for(w, precision)
    Us = init_workload(small, w)
    torch.cuda.synchronize()
    dt = small.dt(Us)
    n = LIMITS[precision][0]
    reps = [n[d] // TILE for d in range(3)]
    print(f"[case] {precision}: {n} elements ({n[0] * n[1] * n[2]}) at N = 5", flush=True)
    big = Solver(w.params, w.N, precision)
    big.upload_box(n, tuple(TILE * 0.25 * r for r in reps))   # the same element size, 1/4
    assert big.nnodes == n[0] * n[1] * n[2] * 216
    # element index ex + nx (ey + ny ez): view [6][tz][lz][ty][ly][tx][lx][node]
    shape = (6, reps[2], TILE, reps[1], TILE, reps[0], TILE, 216)
    tile_view = (6, 1, TILE, 1, TILE, 1, TILE, 216)
    Ub = Us.view(tile_view).expand(shape).contiguous().view(6, -1)
    Rs, Rb = small.new_state(), big.new_state()
    small.rk_steps(Us, Rs, dt, 1)
    big.rk_steps(Ub, Rb, dt, 1)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(Us).all())
    for name, a, b in (("U", Ub, Us), ("R", Rb, Rs)):
        eq = (a.view(shape) == b.view(tile_view)).all(dim=0)
        bad = int((~eq).sum())
        print(f"{name}: {bad} of {eq.numel()} node values differ from the small box", flush=True)
        assert bad == 0
    # the health check covers the whole mesh: the copies' mass adds up
    m_small, m_big = small.reduce(Us)[0], big.reduce(Ub)[0]
    assert abs(m_big / (reps[0] * reps[1] * reps[2]) - m_small) <= 1e-9 * abs(m_small)

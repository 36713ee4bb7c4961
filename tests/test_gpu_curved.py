"""Curved and re-oriented meshes on the GPU (Sec. 3.1: elements mapped from the
reference cube with metric terms; curved elements of geometry degree N_geo),
through the C ABI, against the FP64 CPU oracle.

* Curved periodic and wall boxes (the smooth sine map of the box, geometry
  of degree N or 2 on Gauss-Lobatto points): free-stream preservation, the
  lifted gradients, U_t, the initial state, dt, the integrals and 10 RK
  steps at the 1e-12 bars of the affine parity tests; FP32-mixed density
  within 1e-5 after 20 steps.
* Every element's reference frame rotated (random proper rotations of the
  cube): any face may meet any face under any of the 8 orientations.  The
  discrete operator is the same up to round-off, so U_t and 10 RK steps
  match the oracle on the unrotated mesh, node for node through the
  relabelling.
* Meshes the library must refuse: a wrong orientation, a face paired with a
  face that is not the same surface, walls with a varying temperature on
  curved elements, 512-thread tiles on curved elements.
"""

import numpy as np
import pytest

from helpers import oracle_for, oracle_init, rotated_box_mesh, upload_rc
from paper_2208_05310_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def gpu_solver(w, precision="fp64"):
    from paper_2208_05310_amd.nskr import solver_for
    return solver_for(w, precision)


def to_gpu(torch, a, dtype=None):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device="cuda:0")


CURVED = [
    wl.c1().with_(name="curved_periodic_3x3x3_N3", n=(3, 3, 3), curve_amp=0.05),
    wl.c1().with_(name="curved_periodic_3x3x2_N4_ngeo2", N=4, n=(3, 3, 2), curve_amp=0.05, ngeo=2),
    wl.c1().with_(name="curved_periodic_2x2x2_N5", N=5, n=(2, 2, 2), curve_amp=0.04),
    wl.c1().with_(name="curved_periodic_4x3x3_N2", N=2, n=(4, 3, 3), curve_amp=0.05),
    wl.c4(scale=12).with_(name="curved_wall_4x4x2_N3", curve_amp=0.04),
    wl.c4(scale=12).with_(name="curved_wall_4x4x2_N4_ngeo2_theta120", N=4, curve_amp=0.04, ngeo=2,
                          side_theta=(90.0, 90.0, 90.0, 90.0, 120.0, 90.0)),
    wl.c5(scale=10).with_(name="curved_moving_droplets_5x5x5_N3", curve_amp=0.03),
    wl.c1().with_(name="curved_periodic_3x3x3_N3_model2", n=(3, 3, 3), curve_amp=0.05,
                  params=dict(wl.TABLE1, model=2)),
]
CIDS = [w.name for w in CURVED]


def perturbed_state(o, w, seed=7):
    """Droplet state plus a smooth velocity, a temperature variation and c !=
    rho, so that every flux term acts."""
    U = oracle_init(o, w)
    x, y, z = o.coords()
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, 3)
    u = np.stack([0.05 * np.sin(2 * np.pi * y + ph[0]), 0.04 * np.cos(2 * np.pi * x + ph[1]),
                  0.03 * np.sin(2 * np.pi * x + ph[2])])
    if not w.periodic[2]:
        u[2] *= z * (w.length[2] - z)
    U[1:4] = U[0] * u
    U[4] += 0.5 * U[0] * np.sum(u * u, axis=0)
    pr = w.params
    U[4] += U[0] * pr["R"] * pr["cv"] * 0.02 * np.sin(2 * np.pi * (x + 2 * z) + ph[1])
    U[5] = U[0] + 0.01 * np.sin(2 * np.pi * (x + y) + ph[2])
    return U


def term_scale(o, U, params):
    """Per-field scale of U_t: for momentum and energy the size of the
    relaxation source's two terms alpha |rho| |grad rho| (their difference
    is U_t), else max |U_t|; the max-norm |U_t| is reported beside it."""
    q = o.lift1(U)
    sm = params["alpha"] * np.max(np.abs(U[0])) * np.max(np.abs(q[0:3]))
    umax = np.max(np.abs(U[1:4] / U[0]))
    Ut = o.rhs(U)
    sc = np.max(np.abs(Ut), axis=1)
    raw = sc.copy()
    sc[1:4] = max(sm, np.max(sc[1:4]))
    sc[4] = max(sc[4], sm * umax)
    return sc, raw, Ut


def state_err(g, o, params):
    """Q14 norm: per field max |g - o| / max(|o|_inf, s_f), s_f = |rho|_inf
    |c~|_inf for the momenta."""
    rho = o[0]
    cs = np.sqrt(abs((1 + 1 / params["cv"]) * params["R"] * 0.9 / (1 - params["b"] * rho.max()) ** 2))
    floor = [0.0] + [np.max(np.abs(rho)) * cs] * 3 + [0.0, 0.0]
    return np.array([np.max(np.abs(g[f] - o[f])) / max(np.max(np.abs(o[f])), floor[f]) for f in range(6)])


@pytest.mark.parametrize("w", CURVED[:4], ids=CIDS[:4])
def test_free_stream_on_curved_mesh(torch_cuda, w):
    torch = torch_cuda
    print(f"[case] free stream {w.name}", flush=True)
    s = gpu_solver(w)
    pr = w.params
    rho, T = 1.2, 0.9
    u = np.array([0.3, -0.2, 0.1])
    U = np.zeros((6, s.nnodes))
    U[0], U[5] = rho, rho
    U[1:4] = rho * u[:, None]
    U[4] = rho * (pr["R"] * pr["cv"] * T - pr["a"] * rho) + 0.5 * rho * float(u @ u)
    Ug = to_gpu(torch, U)
    Ut = s.new_state()
    s.rhs(Ug, Ut)
    torch.cuda.synchronize()
    err = Ut.abs().max().item()
    print("free stream max |U_t|", err, flush=True)
    assert err < 5e-12


def wall_at_fluid_temperature(w):
    return w.with_(side_twall=tuple(0.9 if k in (1, 3) else 0.0 for k in w.side_kind),
                   side_theta=(90.0,) * 6)


def test_free_stream_between_curved_walls(torch_cuda):
    torch = torch_cuda
    w = wall_at_fluid_temperature(CURVED[4])
    s = gpu_solver(w)
    pr = w.params
    rho, T = 1.2, 0.9
    U = np.zeros((6, s.nnodes))
    U[0], U[5] = rho, rho
    U[4] = rho * (pr["R"] * pr["cv"] * T - pr["a"] * rho)
    Ut = s.new_state()
    s.rhs(to_gpu(torch, U), Ut)
    torch.cuda.synchronize()
    assert Ut.abs().max().item() < 5e-12


@pytest.mark.parametrize("w", CURVED, ids=CIDS)
def test_curved_lift1_lift2_rhs_parity(torch_cuda, w):
    torch = torch_cuda
    print(f"[case] curved operator {w.name}", flush=True)
    o = oracle_for(w)
    U = perturbed_state(o, w)
    s = gpu_solver(w)
    Ug = to_gpu(torch, U)
    q = torch.empty((15, s.nnodes), dtype=torch.float64, device="cuda:0")
    s.lift1(Ug, q)
    out = torch.empty((5, s.nnodes), dtype=torch.float64, device="cuda:0")
    s.lift2(Ug, out)
    Ut = s.new_state()
    s.rhs(Ug, Ut)
    torch.cuda.synchronize()
    qo, oo = o.lift1(U), o.lift2(U)
    for k in range(5):
        sc = np.max(np.abs(qo[3 * k:3 * k + 3]))
        err = np.max(np.abs(q[3 * k:3 * k + 3].cpu().numpy() - qo[3 * k:3 * k + 3])) / sc
        assert err <= TOL, ("lift1", k, err)
    for grp in ([0], [1, 2, 3], [4]):
        sc = np.max(np.abs(oo[grp]))
        err = np.max(np.abs(out[grp].cpu().numpy() - oo[grp])) / sc
        assert err <= TOL, ("lift2", grp, err)
    scale, raw, Uto = term_scale(o, U, w.params)
    d = np.max(np.abs(Ut.cpu().numpy() - Uto), axis=1)
    print("rhs errors: term scale", d / scale, "max|U_t|", d / raw, flush=True)
    assert np.all(d / scale <= TOL), d / scale


@pytest.mark.parametrize("w", [CURVED[k] for k in (0, 1, 4, 6)], ids=[CIDS[k] for k in (0, 1, 4, 6)])
def test_curved_init_dt_reduce_parity(torch_cuda, w):
    torch = torch_cuda
    print(f"[case] curved init/dt/reduce {w.name}", flush=True)
    from paper_2208_05310_amd.nskr import init_workload
    o = oracle_for(w)
    Uo = oracle_init(o, w)
    s = gpu_solver(w)
    Ug = init_workload(s, w)
    torch.cuda.synchronize()
    err = state_err(Ug.cpu().numpy(), Uo, w.params)
    assert np.all(err <= TOL), err
    U = perturbed_state(o, w)
    dg, do = s.dt(to_gpu(torch, U)), o.dt(U)
    assert abs(dg - do) <= 1e-14 * do, (dg, do)
    rg, ro = s.reduce(to_gpu(torch, U)), o.reduce(U)
    for k in range(20):
        lim = 1e-13 * (max(abs(ro[0]), 1.0) if k in (1, 2, 3) else abs(ro[k])) + 1e-300
        assert abs(rg[k] - ro[k]) <= lim, (k, rg[k], ro[k])


@pytest.mark.parametrize("w", [CURVED[k] for k in (0, 1, 3, 4, 6, 7)], ids=[CIDS[k] for k in (0, 1, 3, 4, 6, 7)])
def test_curved_rk_steps_parity(torch_cuda, w):
    torch = torch_cuda
    nsteps = 10
    print(f"[case] curved rk {w.name} steps={nsteps}", flush=True)
    o = oracle_for(w)
    U = oracle_init(o, w)
    dt = o.dt(U)
    s = gpu_solver(w)
    Ug = to_gpu(torch, U)
    Rg = s.new_state()
    s.rk_steps(Ug, Rg, dt, nsteps)
    torch.cuda.synchronize()
    R = np.zeros_like(U)
    o.run(U, R, 0.0, dt, nsteps)
    err = state_err(Ug.cpu().numpy(), U, w.params)
    print("errors per field", err, flush=True)
    assert np.all(err <= TOL), err


@pytest.mark.parametrize("w", [CURVED[k] for k in (0, 4)], ids=[CIDS[k] for k in (0, 4)])
def test_curved_fp32_mixed_density_within_1e5(torch_cuda, w):
    torch = torch_cuda
    print(f"[case] curved fp32 {w.name}", flush=True)
    o = oracle_for(w)
    U = oracle_init(o, w)
    dt = o.dt(U)
    s = gpu_solver(w, "fp32_mixed")
    Ug = to_gpu(torch, U, torch.float32)
    Rg = s.new_state()
    s.rk_steps(Ug, Rg, dt, 20)
    torch.cuda.synchronize()
    R = np.zeros_like(U)
    o.run(U, R, 0.0, dt, 20)
    err = np.max(np.abs(Ug[0].double().cpu().numpy() - U[0])) / np.max(np.abs(U[0]))
    print("fp32 rho error", err, flush=True)
    assert err <= 1e-5


# ---------------------------------------------------------------- orientations
ROTATED = [
    wl.c1().with_(name="rotated_periodic_3x3x3_N3", n=(3, 3, 3)),
    wl.c1().with_(name="rotated_curved_3x3x3_N4", N=4, n=(3, 3, 3), curve_amp=0.05),
    wl.c4(scale=12).with_(name="rotated_wall_4x4x2_N2", N=2),
    wl.c5(scale=10).with_(name="rotated_moving_droplets_5x5x5_N3"),
]
RIDS = [w.name for w in ROTATED]


def rotated_solver(w, precision="fp64"):
    from paper_2208_05310_amd.nskr import Solver
    m = rotated_box_mesh(w)
    s = Solver(w.params, w.N, precision)
    s.upload_mesh(m["xgeo"], m["nbr"], m["nbf"], m["bc"], m["bcs"], ngeo=m["ngeo"], nbo=m["nbo"])
    s.box = dict(n=tuple(w.n), length=tuple(w.length), periodic=tuple(w.periodic))
    return s, m["perm"]


@pytest.mark.parametrize("w", ROTATED, ids=RIDS)
def test_rotated_elements_rhs_matches_the_oracle(torch_cuda, w):
    torch = torch_cuda
    print(f"[case] rotated rhs {w.name}", flush=True)
    o = oracle_for(w)
    U = perturbed_state(o, w)
    s, perm = rotated_solver(w)
    Ut = s.new_state()
    s.rhs(to_gpu(torch, U[:, perm]), Ut)
    torch.cuda.synchronize()
    scale, raw, Uto = term_scale(o, U, w.params)
    d = np.max(np.abs(Ut.cpu().numpy() - Uto[:, perm]), axis=1)
    print("rotated rhs errors (term scale)", d / scale, flush=True)
    assert np.all(d / scale <= TOL), d / scale


@pytest.mark.parametrize("w", [ROTATED[k] for k in (1, 2, 3)], ids=[RIDS[k] for k in (1, 2, 3)])
def test_rotated_elements_rk_steps_match_the_oracle(torch_cuda, w):
    torch = torch_cuda
    print(f"[case] rotated rk {w.name}", flush=True)
    o = oracle_for(w)
    U = oracle_init(o, w)
    dt = o.dt(U)
    s, perm = rotated_solver(w)
    Ug = to_gpu(torch, U[:, perm])
    Rg = s.new_state()
    s.rk_steps(Ug, Rg, dt, 10)
    torch.cuda.synchronize()
    R = np.zeros_like(U)
    o.run(U, R, 0.0, dt, 10)
    err = state_err(Ug.cpu().numpy(), U[:, perm], w.params)
    print("rotated rk errors", err, flush=True)
    assert np.all(err <= TOL), err


def test_rotated_elements_batched_equal_single(torch_cuda):
    """A curved rotated instance and an affine one in one batch: each equals
    its single-instance run bit for bit."""
    torch = torch_cuda
    from paper_2208_05310_amd.nskr import Batch, init_workload
    w1, w2 = ROTATED[1], CURVED[4]
    s1, _ = rotated_solver(w1)
    s2 = gpu_solver(w2)
    o1 = oracle_for(w1)
    U1 = to_gpu(torch, oracle_init(o1, w1)[:, rotated_box_mesh(w1)["perm"]])
    U2 = init_workload(s2, w2)
    dt1, dt2 = s1.dt(U1), s2.dt(U2)
    a1, a2 = U1.clone(), U2.clone()
    r1, r2 = s1.new_state(), s2.new_state()
    s1.rk_steps(a1, r1, dt1, 3)
    s2.rk_steps(a2, r2, dt2, 3)
    b = Batch(8 << 30)
    stream = torch.cuda.Stream()
    B1, B2, R1, R2 = U1.clone(), U2.clone(), s1.new_state(), s2.new_state()
    b.admit(s1, B1, R1, dt1, 3)
    b.admit(s2, B2, R2, dt2, 3)
    with torch.cuda.stream(stream):
        for _ in range(3):
            b.step(stream)
    stream.synchronize()
    assert torch.equal(B1, a1) and torch.equal(B2, a2)


# ---------------------------------------------------------------- refusals
def test_mesh_upload_refuses_mismatched_faces(torch_cuda):
    from paper_2208_05310_amd.nskr import NSKR_E_ARG, NSKR_E_UNSUPPORTED, Solver, box_mesh
    w = wl.c1().with_(n=(3, 3, 3))
    s = Solver(w.params, w.N)
    m = box_mesh(w.n)
    assert upload_rc(s, m) == 0
    # a flipped face: the orientation of one interior pair reversed on both sides
    nbo = np.zeros((w.nelems, 6), dtype=np.int32)
    nbo[0, 1] = 1
    nbo[int(m[1][0, 1]), 0] = 1
    assert upload_rc(s, m, nbo=nbo) == NSKR_E_ARG
    # a transposed face point order
    nbo[0, 1] = nbo[int(m[1][0, 1]), 0] = 4
    assert upload_rc(s, m, nbo=nbo) == NSKR_E_ARG
    # reciprocal but wrong pairs in the periodic row of elements 0, 1, 2: the
    # + faces of 0 and 1 paired (one translation apart, but facing the same
    # way), and the - faces of 1 and 2
    nbr, nbf = m[1].copy(), m[2].copy()
    nbr[0, 1], nbf[0, 1], nbr[1, 1], nbf[1, 1] = 1, 1, 0, 1
    nbr[1, 0], nbf[1, 0], nbr[2, 0], nbf[2, 0] = 2, 0, 1, 0
    assert upload_rc(s, (m[0], nbr, nbf, m[3], m[4])) == NSKR_E_ARG
    # and the library still takes the correct mesh afterwards
    assert upload_rc(s, m) == 0
    # a wall temperature varying along a curved wall
    wc = wl.c7(scale=12).with_(curve_amp=0.03)
    sc = Solver(wc.params, wc.N)
    mb = box_mesh(wc.n, wc.length, wc.periodic, wc.side_kind, wc.side_twall, wc.side_theta,
                  side_tgrad=wc.side_tgrad)
    xg = wl.box_geometry(wc.n, wc.length, wc.N, wc.curve_amp)
    assert upload_rc(sc, (xg,) + tuple(mb[1:]), ngeo=wc.N) == NSKR_E_UNSUPPORTED
    # 512-thread tiles on curved elements
    s2 = gpu_solver(CURVED[0])
    from paper_2208_05310_amd.nskr import NskrError
    with pytest.raises(NskrError) as ei:
        s2.set_block(512)
    assert ei.value.code == NSKR_E_UNSUPPORTED

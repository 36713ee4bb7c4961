"""Pins of the oracle's DGSEM operator against what the method fixes:
polynomial exactness of the BR1 liftings, free-stream preservation, discrete
mass conservation, the relaxation ODE of a uniform state, equivariance under
axis permutations and reflections, and closed-form wall-flux integrals."""
import math

import numpy as np
import pytest

import oracle

R, A, B, CV = 8.0 / 3.0, 3.0, 1.0 / 3.0, 5.0


def make(N, n, length=(1.0, 1.0, 1.0), periodic=(1, 1, 1), kinds=(0,) * 6, tw=(0.0,) * 6,
         th=(90.0,) * 6, amp=0.0, **pk):
    p = oracle.make_params(**pk)
    b = oracle.make_box(N, n, (0.0, 0.0, 0.0), length, periodic, kinds, tw, th, amp)
    return oracle.Oracle(p, b)


def conserved(o, rho, u, T, c):
    """Conserved state with temperature T, using the oracle's lifted grad c for the
    gradient energy of eq. totalenergyalpha."""
    pr = o.params
    U = np.zeros((6, o.nnodes))
    U[0] = rho
    U[1:4] = rho * u
    U[5] = c
    q = o.lift1(U)
    g2 = q[12] ** 2 + q[13] ** 2 + q[14] ** 2
    U[4] = (rho * (pr.R * pr.cv * T - pr.a * rho) + 0.5 * rho * np.sum(u * u, axis=0)
            + 0.5 * pr.alpha * (rho - c) ** 2 + 0.5 * pr.gam * g2)
    return U


def quad_weights(o):
    x, w, *_ = oracle.basis(o.N)
    P = o.N + 1
    w3 = (w[None, None, :] * w[None, :, None] * w[:, None, None]).reshape(-1)
    _, J, _ = o.metrics()
    return np.tile(w3, o.nelems) * J


# ---------------------------------------------------------------- exactness
def test_lift1_exact_for_polynomial_density_and_order_parameter():
    # BR1 pass 1 (Sec. 3.1) reproduces the gradient of a global polynomial of degree <= N
    # per direction: continuous traces make the central face value exact; walls use rho-.
    N = 4
    o = make(N, (3, 2, 2), (1.5, 1.0, 0.7), (0, 0, 0), (2,) * 6)
    x, y, z = o.coords()
    rho = 1.0 + 0.1 * x - 0.05 * y ** 2 + 0.02 * x * y * z + 0.01 * z ** 4 - 0.003 * x ** 3 * y
    c = 0.9 + 0.03 * x ** 2 * z + 0.01 * y ** 3
    U = np.zeros((6, o.nnodes))
    U[0], U[5], U[4] = rho, c, 3.0
    q = o.lift1(U)
    grho = [0.1 + 0.02 * y * z - 0.009 * x ** 2 * y, -0.1 * y + 0.02 * x * z - 0.003 * x ** 3,
            0.02 * x * y + 0.04 * z ** 3]
    gc = [0.06 * x * z, 0.03 * y ** 2, 0.03 * x ** 2]
    for m in range(3):
        assert np.max(np.abs(q[m] - grho[m])) < 1e-12
        assert np.max(np.abs(q[12 + m] - gc[m])) < 1e-12


def test_lift1_exact_for_velocity_vanishing_on_noslip_walls():
    # u = 0 on the no-slip walls is the wall value u* = 0, so the lifting is exact for
    # polynomial velocities that vanish there (constant density).
    N = 4
    o = make(N, (2, 2, 2), (1.0, 1.0, 1.0), (0, 0, 0), (1,) * 6, tw=(0.85,) * 6)
    x, y, z = o.coords()
    b = x * (1 - x) * y * (1 - y) * z * (1 - z)
    u = np.stack([b, 2 * b, -b])
    db = [(1 - 2 * x) * y * (1 - y) * z * (1 - z), x * (1 - x) * (1 - 2 * y) * z * (1 - z),
          x * (1 - x) * y * (1 - y) * (1 - 2 * z)]
    U = np.zeros((6, o.nnodes))
    U[0], U[5], U[4] = 1.3, 1.3, 4.0
    U[1:4] = 1.3 * u
    q = o.lift1(U)
    for j, s in enumerate((1.0, 2.0, -1.0)):
        for i in range(3):
            assert np.max(np.abs(q[3 + 3 * j + i] - s * db[i])) < 1e-12


def test_divergence_lifting_exact():
    # Divergence lifting of the lifted grad c (reading of Delta c): exact for a polynomial
    # c with zero normal derivative on slip walls, where the wall flux is 0.
    N = 4
    Lx, Ly, Lz = 1.5, 1.0, 0.7
    o = make(N, (3, 2, 2), (Lx, Ly, Lz), (0, 0, 0), (2,) * 6)
    x, y, z = o.coords()

    def bump(t, L):
        return t ** 2 * (t - L) ** 2 / L ** 4

    def bump2(t, L):
        return (12 * t ** 2 - 12 * t * L + 2 * L ** 2) / L ** 4

    c = 1.0 + 0.1 * bump(x, Lx) + 0.2 * bump(y, Ly) - 0.15 * bump(z, Lz)
    lap = 0.1 * bump2(x, Lx) + 0.2 * bump2(y, Ly) - 0.15 * bump2(z, Lz)
    U = conserved(o, np.full(o.nnodes, 1.0), np.zeros((3, o.nnodes)), 0.9, c)
    l2 = o.lift2(U)
    assert np.max(np.abs(l2[4] - lap)) < 1e-11


# ------------------------------------------------------------ free stream
STATE = dict(rho=1.2, u=(0.3, -0.2, 0.1), T=0.9)


@pytest.mark.parametrize("N,amp", [(3, 0.0), (4, 0.0), (3, 0.05), (4, 0.05), (5, 0.05)])
def test_free_stream_periodic(N, amp):
    # A constant state is an exact steady solution: requires discrete metric identities
    # (curl-form metrics on curved meshes) and consistent fluxes.
    o = make(N, (3, 3, 3), amp=amp)
    rho = np.full(o.nnodes, STATE["rho"])
    u = np.tile(np.array(STATE["u"])[:, None], (1, o.nnodes))
    U = conserved(o, rho, u, STATE["T"], rho.copy())
    Ut = o.rhs(U)
    # Bound: round-off of the order-parameter diffusion gamma beta div(grad c) of a
    # constant, ~ eps |c| (N^2/h)^2 gamma beta, reaches 1e-12 at N = 5 on 3^3 elements.
    assert np.max(np.abs(Ut)) < 5e-12


@pytest.mark.parametrize("amp", [0.0, 0.05])
def test_free_stream_at_rest_with_walls(amp):
    # Fluid at rest at the wall temperature, neutral contact angle: steady with both wall
    # kinds (no-slip isothermal at 90 degrees on z-, slip adiabatic on z+).
    o = make(3, (3, 3, 2), (1.0, 1.0, 0.5), (1, 1, 0), (0, 0, 0, 0, 1, 2), tw=(0, 0, 0, 0, 0.9, 0),
             th=(90.0,) * 6, amp=amp)
    rho = np.full(o.nnodes, 1.2)
    U = conserved(o, rho, np.zeros((3, o.nnodes)), 0.9, rho.copy())
    assert np.max(np.abs(o.rhs(U))) < 5e-12  # same round-off bound as above


# ------------------------------------------------------------ conservation
def droplet_state(o, centre, r=0.25, T=0.85, vel=True, seed=3):
    x, y, z = o.coords()
    rng = np.random.default_rng(seed)
    U = o.init_droplets(T, [centre], [r], 0.05, rng.uniform(-1e-3, 1e-3, o.nnodes))
    if vel:
        rho = U[0]
        u = np.stack([0.05 * np.sin(2 * np.pi * y), 0.04 * np.cos(2 * np.pi * z), 0.03 * np.sin(2 * np.pi * x)])
        U[1:4] = rho * u
        U[4] += 0.5 * rho * np.sum(u * u, axis=0)
    return U


@pytest.mark.parametrize("limit,pk", [
    ("advective", dict(mu=1e-7, kappa=1e-7, gam=1e-7, alpha=1.0, beta=1.0)),
    ("parabolic", dict(mu=2.0, kappa=2.0)),
])
def test_time_step_scales_with_the_cfl_number(limit, pk):
    # dt = CFL x (the smaller of the advective and the parabolic/source limits, Sec. 4):
    # halving the CFL number halves dt, with either limit binding (near-inviscid fluid
    # with weak relaxation: advective; viscous and conductive: parabolic).
    dts = []
    for cfl in (0.9, 0.45):
        o = make(3, (3, 3, 3), cfl=cfl, **pk)
        dts.append(o.dt(droplet_state(o, (0.5, 0.5, 0.5))))
    assert abs(dts[0] / dts[1] - 2.0) <= 1e-14


def test_mass_conservation_periodic():
    o = make(3, (4, 4, 4))
    U = droplet_state(o, (0.4, 0.55, 0.5))
    W = quad_weights(o)
    Ut = o.rhs(U)
    assert abs(W @ Ut[0]) <= 1e-14 * (W @ np.abs(Ut[0]))


def test_mass_conservation_walls_and_curved():
    o = make(3, (3, 3, 3), (1.0, 1.0, 0.5), (1, 1, 0), (0, 0, 0, 0, 1, 2),
             tw=(0, 0, 0, 0, 0.9, 0), th=(0, 0, 0, 0, 60.0, 0), amp=0.03)
    U = droplet_state(o, (0.5, 0.5, 0.0), r=0.2)
    W = quad_weights(o)
    Ut = o.rhs(U)
    assert abs(W @ Ut[0]) <= 1e-14 * (W @ np.abs(Ut[0]))
    m0 = W @ U[0]
    dt = o.dt(U)
    R_ = np.zeros_like(U)
    o.run(U, R_, 0.0, dt, 10)
    assert abs(W @ U[0] - m0) <= 1e-14 * m0


# ------------------------------------------------------------ relaxation ODE
def test_uniform_relaxation_follows_stability_polynomial():
    # Uniform state with c0 != rho: only the source alpha beta (rho - c) acts, so the RK
    # scheme multiplies c - rho by its stability polynomial P(-alpha beta dt) each step;
    # rho, momentum and rho e stay constant.
    o = make(3, (2, 2, 2))
    pr = o.params
    rho = np.full(o.nnodes, 1.0)
    c = np.full(o.nnodes, 1.001)
    U = conserved(o, rho, np.zeros((3, o.nnodes)), 0.9, c)
    U0 = U.copy()
    A_, B_, _ = oracle.rk_coeffs()
    # stability polynomial from the 2N recursion applied to y' = lam y
    dt = 2e-5
    z = -pr.alpha * pr.beta * dt
    y, r = 1.0, 0.0
    for s in range(5):
        r = (A_[s] * r if s else 0.0) + z * y
        y = y + B_[s] * r
    P = y
    Pz = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24 + 0.005 * z ** 5
    assert abs(P - Pz) < 1e-5 * abs(z) ** 5 + 1e-15
    R_ = np.zeros_like(U)
    nsteps = 10
    o.run(U, R_, 0.0, dt, nsteps)
    expect = 0.001 * P ** nsteps
    assert np.max(np.abs((U[5] - U[0]) - expect)) < 1e-13
    assert np.max(np.abs(U[0] - U0[0])) < 1e-14
    assert np.max(np.abs(U[1:4])) < 1e-14
    assert np.max(np.abs(U[4] - U0[4])) < 1e-12


# ------------------------------------------------------------ equivariance
def permute_state(U, n, P, axes):
    """Relabel coordinates: new axis d is old axis axes[d]."""
    E = n[0] * n[1] * n[2]
    V = U.reshape(6, n[2], n[1], n[0], P, P, P)  # [v][ez][ey][ex][k][j][i]
    # array axes order (z,y,x) for elements and nodes; build permutation
    old_pos = {0: 2, 1: 1, 2: 0}
    perm_e = [old_pos[axes[2]], old_pos[axes[1]], old_pos[axes[0]]]
    perm = [0] + [1 + p for p in perm_e] + [4 + p for p in perm_e]
    W = np.transpose(V, perm).copy()
    out = W.reshape(6, E * P ** 3).copy()
    mom = U[1:4].copy()
    Wm = np.transpose(mom.reshape(3, n[2], n[1], n[0], P, P, P), [0] + perm[1:]).reshape(3, -1)
    for d in range(3):
        out[1 + d] = Wm[axes[d]]
    return out


@pytest.mark.parametrize("axes", [(1, 0, 2), (2, 1, 0), (1, 2, 0)])
def test_axis_permutation_equivariance(axes):
    # L(perm U) = perm L(U) on a cube mesh: catches transposed indices, wrong face/normal
    # pairing and direction-dependent mistakes anywhere in the operator.
    n, N = (3, 3, 3), 3
    o = make(N, n)
    U = droplet_state(o, (0.4, 0.55, 0.47))
    lhs = o.rhs(permute_state(U, n, N + 1, axes))
    rhs = permute_state(o.rhs(U), n, N + 1, axes)
    scale = np.max(np.abs(rhs), axis=1, keepdims=True)
    assert np.max(np.abs(lhs - rhs) / scale) < 1e-12


def reflect_z(U, n, P):
    V = U.reshape(6, n[2], n[1], n[0], P, P, P)[:, ::-1, :, :, ::-1, :, :].reshape(6, -1).copy()
    V[3] = -V[3]
    return V


def test_reflection_equivariance_between_two_walls():
    # Two identical walls (no-slip, contact angle 60 degrees, T_w = 0.9) at z = 0 and z = Lz:
    # mirroring z maps solutions to solutions, which pins the wall normal orientation on
    # both sides of the box.
    n, N = (2, 2, 3), 3
    o = make(N, n, (1.0, 1.0, 0.6), (1, 1, 0), (0, 0, 0, 0, 1, 1), tw=(0, 0, 0, 0, 0.9, 0.9),
             th=(0, 0, 0, 0, 60.0, 60.0))
    U = droplet_state(o, (0.45, 0.5, 0.1), r=0.2)
    lhs = o.rhs(reflect_z(U, n, N + 1))
    rhs = reflect_z(o.rhs(U), n, N + 1)
    scale = np.max(np.abs(rhs), axis=1, keepdims=True)
    assert np.max(np.abs(lhs - rhs) / scale) < 1e-12


def test_lifted_gradients_of_a_periodic_field_integrate_to_zero():
    # BR1 takes one face value for both sides of a face (the mean of the two traces), and
    # with collocated Gauss quadrature sum_i w_i J q_i over an element is the sum of its
    # faces' w* n dS (the weighted column sums of Dhat vanish, the lifting weights l(+-1)
    # sum to one). On a periodic mesh the faces cancel in pairs, so every lifted gradient,
    # and the divergence lifting lap c, integrates to zero for any state, however
    # discontinuous between elements. A one-sided face value would leave the integral of
    # the jumps.
    o = make(3, (3, 3, 3))
    rng = np.random.default_rng(5)
    x, y, z = o.coords()
    rho = 0.9 + 0.3 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) + 0.05 * rng.uniform(-1, 1, o.nnodes)
    u = 0.1 * rng.uniform(-1, 1, (3, o.nnodes))
    T = 0.9 + 0.02 * rng.uniform(-1, 1, o.nnodes)
    c = rho + 0.05 * rng.uniform(-1, 1, o.nnodes)
    U = conserved(o, rho, u, T, c)
    w = quad_weights(o)
    q1, q2 = o.lift1(U), o.lift2(U)
    for row in list(q1) + list(q2[1:5]):
        assert abs(np.sum(w * row)) <= 1e-12 * np.sum(w * np.abs(row))


# ------------------------------------------------------------ wall integrals
@pytest.mark.parametrize("theta", [45.0, 60.0, 90.0, 120.0])
def test_contact_angle_wall_c_flux_integral(theta):
    # Uniform fluid at rest with c = rho: the only change of int c is the wall flux of the
    # order parameter, gamma beta g per unit area, g = -(1/gamma) dpsi_Gamma/dc
    # (eq. bc_contactangle_alpha); wetting walls (theta < 90) attract liquid.
    Tw = 0.9
    o = make(3, (2, 2, 2), (1.0, 1.0, 0.5), (1, 1, 0), (0, 0, 0, 0, 1, 2), tw=(0, 0, 0, 0, Tw, 0),
             th=(0, 0, 0, 0, theta, 0))
    pr = o.params
    c0 = 1.0
    rho = np.full(o.nnodes, c0)
    U = conserved(o, rho, np.zeros((3, o.nnodes)), Tw, rho.copy())
    W = quad_weights(o)
    Ut = o.rhs(U)
    rv, rl, _ = oracle.maxwell(Tw)
    sig = oracle.sigma(Tw, pr.gam)
    g = -oracle.dpsiwall_dc(c0, rv, rl, sig, math.cos(math.radians(theta))) / pr.gam
    expect = pr.gam * pr.beta * g * 1.0  # wall area 1
    got = W @ Ut[5]
    assert abs(got - expect) < 1e-12 * max(1.0, abs(expect))
    if theta < 90:
        assert got > 0
    assert abs(W @ Ut[0]) < 1e-13
    assert abs(W @ Ut[4]) < 1e-12


def test_hot_isothermal_wall_heats_fluid():
    # Fluid at T = 0.85 against a wall at T_w = 0.9: energy flows in (heat flux k grad T . n).
    o = make(3, (2, 2, 2), (1.0, 1.0, 0.5), (1, 1, 0), (0, 0, 0, 0, 1, 2), tw=(0, 0, 0, 0, 0.9, 0))
    rho = np.full(o.nnodes, 0.4)
    U = conserved(o, rho, np.zeros((3, o.nnodes)), 0.85, rho.copy())
    W = quad_weights(o)
    assert W @ o.rhs(U)[4] > 0.0
    o2 = make(3, (2, 2, 2), (1.0, 1.0, 0.5), (1, 1, 0), (0, 0, 0, 0, 1, 2), tw=(0, 0, 0, 0, 0.8, 0))
    U2 = conserved(o2, rho, np.zeros((3, o2.nnodes)), 0.85, rho.copy())
    assert W @ o2.rhs(U2)[4] < 0.0


def test_init_recovers_temperature():
    o = make(4, (3, 3, 3))
    U = o.init_droplets(0.85, [(0.5, 0.5, 0.5)], [0.25], 0.05, None)
    T = o.lift2(U)[0]
    assert np.max(np.abs(T - 0.85)) < 1e-13
    rv, rl, _ = oracle.maxwell(0.85)
    assert abs(U[0].min() - rv) < 1e-3 and abs(U[0].max() - rl) < 1e-2


def collision_pair(o, u_rel=2.2):
    """Two droplets approaching head-on along x (the collision set-up of
    Sec. 4.3 with the Young-Laplace densities of Table 5)."""
    return o.init_droplets(0.85, [(0.3, 0.5, 0.5), (0.7, 0.5, 0.5)], [0.1, 0.1], 0.0772 / 4, None,
                           velocities=[(u_rel / 2, 0, 0), (-u_rel / 2, 0, 0)], rho_v=0.3537, rho_l=1.8493)


def test_init_with_velocities_recovers_temperature_and_densities():
    """With moving droplets the total energy must carry the kinetic part:
    the recovered temperature is T0 at every node (a missing or doubled
    kinetic term shifts T by |u|^2/(2 R c_v), ~0.05 here); the prescribed
    bulk densities replace the Maxwell states; the droplets move with their
    velocities and the vapour between them is at rest."""
    o = make(3, (6, 4, 4))
    U = collision_pair(o)
    T = o.lift2(U)[0]
    assert np.max(np.abs(T - 0.85)) < 1e-12
    assert abs(U[0].min() - 0.3537) < 1e-6 and abs(U[0].max() - 1.8493) < 2e-2
    u = U[1] / U[0]
    X = o.coords().T
    x = X[:, 0]
    inside1 = np.linalg.norm(X - np.array([0.3, 0.5, 0.5]), axis=1) < 0.05
    inside2 = np.linalg.norm(X - np.array([0.7, 0.5, 0.5]), axis=1) < 0.05
    assert inside1.any() and inside2.any()
    assert np.allclose(u[inside1], 1.1, rtol=1e-3) and np.allclose(u[inside2], -1.1, rtol=1e-3)
    mid = np.abs(x - 0.5) < 0.05
    assert np.max(np.abs(u[mid])) < 1e-3
    assert np.all(U[2] == 0.0) and np.all(U[3] == 0.0)


def test_integrals_against_quadrature_and_thermodynamics():
    # The reductions are Gauss-quadrature integrals with the Jacobian: each is checked
    # against a numpy sum over the oracle's nodes with its weights (pinned against
    # numpy's Gauss rule) and metrics, using the lifted grad c and the nodal temperature
    # of the liftings; the entropy integral -int rho eta against d psi / dT of the
    # Helmholtz energy of Sec. 2.1 (entropy per volume = -d psi/dT), by a numerical
    # derivative; the volume against the box's; the health counters are zero.
    from test_oracle_thermo import psi
    o = make(3, (3, 3, 2), length=(1.0, 1.0, 0.6))
    U = droplet_state(o, (0.5, 0.5, 0.3), r=0.2)
    s = o.reduce(U)
    w = quad_weights(o)
    pr = o.params
    rho, m, E, c = U[0], U[1:4], U[4], U[5]
    gc = o.lift1(U)[12:15]
    T = o.lift2(U)[0]
    expect = {0: rho, 1: m[0], 2: m[1], 3: m[2], 4: E, 5: c, 6: 0.5 * np.sum(m * m, axis=0) / rho,
              7: 0.5 * pr.gam * np.sum(gc * gc, axis=0), 8: 0.5 * pr.alpha * (rho - c) ** 2, 9: (rho - c) ** 2}
    for k, f in expect.items():
        assert abs(s[k] - w @ f) <= 1e-13 * (w @ np.abs(f)) + 1e-300, k
    assert s[10] == rho.min() and s[11] == rho.max()
    assert abs(s[12] - T.min()) <= 1e-14 and abs(s[13] - T.max()) <= 1e-14
    assert np.all(s[14:18] == 0)
    h = 1e-5
    dpsi_dT = np.array([(psi(r, t + h) - psi(r, t - h)) / (2 * h) for r, t in zip(rho, T)])
    assert abs(s[18] - w @ dpsi_dT) <= 1e-7 * (w @ np.abs(dpsi_dT))
    assert abs(s[19] - 0.6) <= 1e-14


def test_droplet_excess_mass_closed_form():
    # The tanh profile of Sec. 4.1.1 is a Fermi function of the distance d:
    # (1 + tanh((r - d)/w))/2 = 1/(1 + exp((d - r)/(w/2))), so one droplet's excess mass
    # is (rho_l - rho_v) 4 pi/3 (r^3 + pi^2 w^2 r / 4) up to terms of order exp(-2r/w)
    # (the Sommerfeld expansion of the Fermi integral). The w^2 part is a tenth of the
    # total here. The same droplet centred across a periodic side or corner has the same
    # mass (minimum-image distances).
    o = make(4, (8, 8, 8))
    w = quad_weights(o)
    rv, rl, _ = oracle.maxwell(0.85)
    r, wd = 0.25, 0.05
    exact = (rl - rv) * 4 * math.pi / 3 * (r ** 3 + math.pi ** 2 * wd ** 2 * r / 4)
    for centre in ((0.5, 0.5, 0.5), (0.05, 0.5, 0.93), (0.0, 1.0, 0.0)):
        U = o.init_droplets(0.85, [centre], [r], wd)
        assert abs(w @ (U[0] - rv) / exact - 1) <= 1e-4, centre
        assert U[0].max() <= rl and U[0].min() >= rv


def test_energy_flux_zeta_term_closed_form():
    # At rest with uniform rho and T, the only energy flux left is gamma grad c zeta_c of
    # j_e (Sec. 2.3.2), zeta_c = beta (gamma lap c + alpha (rho - c)). With
    # c = rho + eps sin 2 pi x it gives rho e_t = div j_e
    # = -4 pi^2 gamma beta eps^2 (4 pi^2 gamma + alpha) cos 4 pi x, resolved spectrally
    # (relative error 4e-4 on 8 elements, 7e-6 on 16 at N = 5).
    g, al, be, eps, rho0, T = 1e-3, 10.0, 50.0, 0.05, 0.9, 1.1
    o = make(5, (16, 1, 1), gam=g, alpha=al, beta=be, mu=0.01, kappa=0.02)
    x, y, z = o.coords()
    U = conserved(o, np.full(o.nnodes, rho0), np.zeros((3, o.nnodes)), np.full(o.nnodes, T),
                  rho0 + eps * np.sin(2 * np.pi * x))
    Et = o.rhs(U)[4]
    exact = -4 * np.pi ** 2 * g * be * eps ** 2 * (4 * np.pi ** 2 * g + al) * np.cos(4 * np.pi * x)
    assert np.max(np.abs(Et - exact)) <= 5e-5 * np.max(np.abs(exact))


def _cofactor_identity_error(N, amp):
    o = make(N, (3, 3, 3), amp=amp)
    P, E = N + 1, o.nelems
    Ja, J, _ = o.metrics()
    X = o.coords().reshape(3, E, P, P, P)            # node axes k, j, i (i along xi^1)
    D = oracle.basis(N)[2]
    dX = [np.einsum("il,cekjl->cekji", D, X), np.einsum("jl,cekli->cekji", D, X),
          np.einsum("kl,celji->cekji", D, X)]
    err = 0.0
    for d in range(3):
        for e in range(3):
            s = sum(Ja[3 * d + m] * dX[e][m].reshape(-1) for m in range(3))
            err = max(err, np.max(np.abs(s - (J if d == e else 0.0))) / np.max(np.abs(J)))
    return err


def test_metrics_satisfy_the_cofactor_identity():
    # Ja^d_m = J d xi^d / d x_m, so sum_m Ja^d_m d x_m / d xi^e = J delta_de, with the
    # derivatives of the node coordinates taken by the (pinned) derivative matrix:
    # exact on affine elements; on curved elements the curl form of the metrics meets it
    # to its interpolation error, which falls with the degree.
    assert _cofactor_identity_error(3, 0.0) <= 1e-13
    e3, e5 = _cofactor_identity_error(3, 0.05), _cofactor_identity_error(5, 0.05)
    assert e5 <= 5e-3 and e5 < 0.1 * e3


def test_collision_state_is_mirror_antisymmetric():
    """The head-on pair is symmetric under x -> 1 - x with the x-momentum
    changing sign: total x-momentum vanishes and the integrals of density and
    energy equal twice those of one half (checked through the mirror image
    node by node on a mesh symmetric about x = 1/2)."""
    o = make(3, (6, 4, 4))
    U = collision_pair(o)
    X = o.coords().T
    key = lambda P: np.round(P, 12)
    idx = {tuple(k): n for n, k in enumerate(key(X))}
    mirror = np.array([idx[tuple(key(np.array([1.0 - p[0], p[1], p[2]])))] for p in X])
    assert np.allclose(U[0][mirror], U[0], rtol=0, atol=1e-14)
    assert np.allclose(U[1][mirror], -U[1], rtol=0, atol=1e-13)
    assert np.allclose(U[4][mirror], U[4], rtol=1e-12, atol=1e-12)
    sums = o.reduce(U)
    assert abs(sums[1]) < 1e-12 * abs(sums[0])


def test_cylinder_initial_state_is_uniform_along_its_axis():
    """The liquid pillar of Sec. 4.4.1: with cylinder_axis = 2 the initial
    density depends on x and y only, equals the same droplet's profile
    through its centre plane, and the recovered temperature is T0."""
    p = oracle.make_params(alpha=100.0, beta=100.0)
    b = oracle.make_box(3, (4, 4, 3), (0.0, 0.0, 0.0), (1.0, 1.0, 0.2), (1, 1, 0), (0, 0, 0, 0, 1, 1),
                        (0, 0, 0, 0, 0.85, 0.85), (90, 90, 90, 90, 60, 60))
    o = oracle.Oracle(p, b)
    U = o.init_droplets(0.85, [(0.5, 0.5, 0.1)], [0.2], 0.05, None, None, 0.0, 0.0, 2)
    x, y, z = o.coords()
    key = np.round(x, 12) * 1e3 + np.round(y, 12)
    for k in np.unique(key)[::7]:
        sel = key == k
        assert np.ptp(U[0][sel]) <= 1e-15 * U[0][sel].max()
    # a sphere with its centre at the node's height has the same profile
    for i in range(0, o.nnodes, 97):
        s = o.init_droplets(0.85, [(0.5, 0.5, z[i])], [0.2], 0.05)
        assert abs(s[0][i] - U[0][i]) <= 1e-15
    T = o.lift2(U)[0]
    assert np.max(np.abs(T - 0.85)) <= 1e-12

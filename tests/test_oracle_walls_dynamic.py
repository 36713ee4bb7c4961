"""Pins of the oracle's moving and generalized Navier-slip walls (Sec. 2.4,
eq. bc_nsk_alpha; weak enforcement through the face flux, Sec. 3.2).

Each check compares the oracle with something fixed by the equations, not
with its own formulas:

* a Navier-slip wall with every coefficient zero and a 90 degree angle is the
  perfect-slip adiabatic neutral wall;
* Couette flow between a Navier-slip floor and a moving no-slip lid: the
  linear profile with the slip velocity set by gamma_2 is a steady state of
  mass, momentum and order parameter, and the total energy grows at exactly
  the viscous dissipation mu s^2 V;
* conduction between two heat-transfer walls (eq. bc_energy_alpha): the
  linear temperature whose end values satisfy the gamma_3 condition is a
  steady state of the energy equation at every node;
* a compressing flow at a Navier-slip wall with gamma_1, gamma_4 > 0: the
  total order parameter and the total energy change at the closed-form rates
  beta gamma_1 int(div u) and -(c + gamma_1 gamma_4) gamma_1 int(div u)^2;
* the dynamic-angle part of the wall traction: the x-momentum rate equals
  gamma_1 int(div u d c/dx) over the wall, to discretisation accuracy.
"""
import math

import numpy as np
import pytest

import oracle

R, A, B, CV = 8.0 / 3.0, 3.0, 1.0 / 3.0, 5.0
INF = float("inf")


def weights(o):
    w = oracle.basis(o.N)[1]
    return o.metrics()[1] * np.tile(np.kron(np.kron(w, w), w), o.nelems)


def energy(rho, u2, T, c=None):
    """rho e of a state with uniform c = rho (no gradient or relaxation energy)."""
    return rho * (R * CV * T - A * rho) + 0.5 * rho * u2


def box(N, n, length, bottom, top, **kw):
    """Periodic in x and y, walls at z = 0 (bottom) and z = length[2] (top);
    bottom/top are dicts of per-side wall settings."""
    kinds = [0, 0, 0, 0, bottom["kind"], top["kind"]]
    def side(key, default):
        return [default] * 4 + [bottom.get(key, default), top.get(key, default)]
    return oracle.make_box(N, n, (0.0, 0.0, 0.0), length, (1, 1, 0), kinds,
                           side("twall", 0.9), side("theta", 90.0), 0.0,
                           side("uwall", (0.0, 0.0, 0.0)), side("g1", 0.0), side("g2", 0.0),
                           side("g3", INF), side("g4", 0.0))


def test_navier_wall_without_coefficients_is_the_slip_wall():
    p = oracle.make_params()
    L = (1.0, 1.0, 0.5)
    slip = oracle.Oracle(p, box(3, (3, 3, 2), L, {"kind": 2}, {"kind": 2}))
    nav = oracle.Oracle(p, box(3, (3, 3, 2), L, {"kind": 3, "g3": 0.0}, {"kind": 3, "g3": 0.0}))
    U = slip.init_droplets(0.9, [[0.5, 0.5, 0.25]], [0.2], 0.05)
    x, y, z = slip.coords()
    u = np.stack([0.05 * np.sin(2 * np.pi * y), 0.03 * np.cos(2 * np.pi * x), 0.2 * z * (0.5 - z)])
    U[1:4] = U[0] * u
    U[4] += 0.5 * U[0] * np.sum(u * u, axis=0)
    U[5] = U[0] + 0.01 * np.sin(2 * np.pi * (x + y))
    a, b = slip.rhs(U), nav.rhs(U)
    scale = np.max(np.abs(a), axis=1)
    assert np.all(np.max(np.abs(a - b), axis=1) <= 1e-12 * scale), np.max(np.abs(a - b), axis=1) / scale


@pytest.mark.parametrize("N", [2, 3])
def test_navier_slip_couette_under_a_moving_lid(N):
    mu, g2, Ul, H = 0.01, 0.05, 0.4, 0.5
    p = oracle.make_params(mu=mu)
    T0, rho = 0.95, 0.25
    # steady profile u = u0 + s z with mu s = gamma_2 u0 (floor) and u(H) = U (lid)
    u0 = Ul / (1.0 + g2 * H / mu)
    s = g2 * u0 / mu
    o = oracle.Oracle(p, box(N, (2, 2, 3), (1.0, 1.0, H),
                             {"kind": 3, "g2": g2, "g1": 3.0, "g4": 2.0, "twall": T0},
                             {"kind": 1, "uwall": (Ul, 0.0, 0.0), "twall": T0}))
    x, y, z = o.coords()
    ux = u0 + s * z
    U = np.zeros((6, o.nnodes))
    U[0] = rho
    U[1] = rho * ux
    U[4] = energy(rho, ux * ux, T0)
    U[5] = rho
    Ut = o.rhs(U)
    # mass, momentum and order parameter are steady (scales: the wall traction
    # mu s / h; for c the wall flux beta gamma_1 div u, whose div u = 0 holds
    # only to round-off of the lifted gradient, ~ s)
    h = H / 3
    ref = mu * s / h
    assert np.max(np.abs(Ut[0])) <= 1e-12 * ref
    assert np.max(np.abs(Ut[5])) <= 1e-12 * 1000.0 * 3.0 * s / h
    assert np.max(np.abs(Ut[1:4])) <= 1e-11 * ref, np.max(np.abs(Ut[1:4]), axis=1) / ref
    # the total energy grows at the viscous dissipation rate mu s^2 V
    W = weights(o)
    rate = np.dot(W, Ut[4])
    assert abs(rate - mu * s * s * H) <= 1e-11 * mu * s * s * H, (rate, mu * s * s * H)
    # without the slip coefficient the same state is not steady
    o2 = oracle.Oracle(p, box(N, (2, 2, 3), (1.0, 1.0, H), {"kind": 3, "g2": 2 * g2, "twall": T0},
                              {"kind": 1, "uwall": (Ul, 0.0, 0.0), "twall": T0}))
    assert np.max(np.abs(o2.rhs(U)[1])) > 1e-3 * ref


def test_conduction_between_heat_transfer_walls_is_steady():
    kappa, g3, H = 1.0 / 150.0, 0.05, 0.5
    p = oracle.make_params(kappa=kappa)
    Ta, Tb, rho = 0.9, 0.95, 0.3
    k = (Tb - Ta) / H
    # eq. bc_energy_alpha: k grad T . n = -gamma_3 (1/T_wall - 1/T) on each wall
    Tw_bot = 1.0 / (1.0 / Ta + kappa * k / g3)
    Tw_top = 1.0 / (1.0 / Tb - kappa * k / g3)
    o = oracle.Oracle(p, box(3, (2, 2, 3), (1.0, 1.0, H), {"kind": 3, "g3": g3, "twall": Tw_bot},
                             {"kind": 3, "g3": g3, "twall": Tw_top}))
    x, y, z = o.coords()
    U = np.zeros((6, o.nnodes))
    U[0] = rho
    U[4] = energy(rho, 0.0, Ta + k * z)
    U[5] = rho
    Ut = o.rhs(U)
    # round-off scale: a second difference of T ~ 0.9 over h = H/3, times kappa
    h = H / 3
    assert np.max(np.abs(Ut[4])) <= 1e-12 * kappa * Tb / h ** 2, np.max(np.abs(Ut[4])) / (kappa * Tb / h ** 2)
    ref = kappa * k / h
    # round-off only (prolonged constants; cos(90 deg) is 6e-17 in FP64)
    assert np.max(np.abs(Ut[0])) <= 1e-13 and np.max(np.abs(Ut[5])) <= 1e-12
    # a wrong wall temperature leaves a boundary heat flux
    o2 = oracle.Oracle(p, box(3, (2, 2, 3), (1.0, 1.0, H), {"kind": 3, "g3": g3, "twall": Ta},
                              {"kind": 3, "g3": g3, "twall": Tw_top}))
    assert np.max(np.abs(o2.rhs(U)[4])) > 1e-2 * ref


def test_dynamic_angle_and_relaxation_wall_rates():
    """u = (0, 0, s z (H - z)): div u = s H at the floor.  With a 90 degree
    angle g = gamma_1 div u / gamma, so d/dt int c = beta gamma_1 s H A and
    d/dt int rho e = -(c + gamma_1 gamma_4) gamma_1 (s H)^2 A (the slip top
    wall and the bulk contribute nothing)."""
    beta, g1, g4, H, s = 1000.0, 0.7, 0.4, 0.5, 0.3
    p = oracle.make_params(beta=beta)
    T0, rho = 0.9, 0.3
    o = oracle.Oracle(p, box(4, (2, 2, 3), (1.0, 1.0, H),
                             {"kind": 3, "g1": g1, "g4": g4, "g2": 0.02, "twall": T0}, {"kind": 2}))
    x, y, z = o.coords()
    w = s * z * (H - z)
    U = np.zeros((6, o.nnodes))
    U[0] = rho
    U[3] = rho * w
    U[4] = energy(rho, w * w, T0)
    U[5] = rho
    Ut = o.rhs(U)
    W = weights(o)
    area = 1.0
    c_rate = np.dot(W, Ut[5])
    e_rate = np.dot(W, Ut[4])
    c_exp = beta * g1 * s * H * area
    e_exp = -(rho + g1 * g4) * g1 * (s * H) ** 2 * area
    assert abs(c_rate - c_exp) <= 1e-10 * abs(c_exp), (c_rate, c_exp)
    assert abs(e_rate - e_exp) <= 1e-9 * abs(e_exp), (e_rate, e_exp)
    assert abs(np.dot(W, Ut[0])) <= 1e-14


def test_dynamic_angle_wall_traction():
    """t_x = gamma_1 div u dc/dx at the floor (u_t = 0 there), with div u =
    s H (1 + eps cos 2 pi x) and c = rho = rho0 + d sin 2 pi x: d/dt int rho u =
    gamma_1 s H d pi eps L_y, to discretisation accuracy (which converges
    spectrally: 7e-8, 8e-11, 2e-12 relative on 4, 8, 16 elements along x)."""
    g1, H, s, eps, d, rho0 = 0.5, 0.5, 0.2, 0.5, 0.02, 0.3
    p = oracle.make_params()
    T0 = 0.9
    o = oracle.Oracle(p, box(4, (8, 1, 2), (1.0, 1.0, H), {"kind": 3, "g1": g1, "twall": T0}, {"kind": 2}))
    x, y, z = o.coords()
    rho = rho0 + d * np.sin(2 * np.pi * x)
    w = s * z * (H - z) * (1 + eps * np.cos(2 * np.pi * x))
    U = np.zeros((6, o.nnodes))
    U[0] = rho
    U[3] = rho * w
    U[4] = energy(rho, w * w, T0)
    U[5] = rho
    Ut = o.rhs(U)
    W = weights(o)
    rate = np.dot(W, Ut[1])
    exact = g1 * s * H * d * math.pi * eps
    assert abs(rate - exact) <= 1e-8 * abs(exact), (rate, exact)  # spectral: 8e-11 here
    # the sign and the factor gamma_1 matter
    o2 = oracle.Oracle(p, box(4, (8, 1, 2), (1.0, 1.0, H), {"kind": 3, "g1": 0.0, "twall": T0}, {"kind": 2}))
    assert abs(np.dot(W, o2.rhs(U)[1])) <= 1e-3 * abs(exact)


def test_conduction_between_isothermal_walls_is_steady():
    """Fluid at rest, uniform density, temperature linear between two
    isothermal no-slip walls at Ta (z = 0) and Tb (z = H): the lifted
    gradient is exact and the walls' conductive flux k grad T . n balances
    the bulk, so the energy equation is steady at every node."""
    kappa, H = 1.0 / 150.0, 0.5
    p = oracle.make_params(kappa=kappa)
    Ta, Tb, rho = 0.9, 0.95, 0.3
    o = oracle.Oracle(p, box(3, (2, 2, 3), (1.0, 1.0, H), {"kind": 1, "twall": Ta}, {"kind": 1, "twall": Tb}))
    x, y, z = o.coords()
    U = np.zeros((6, o.nnodes))
    U[0] = rho
    U[4] = energy(rho, 0.0, Ta + (Tb - Ta) * z / H)
    U[5] = rho
    h = H / 3
    assert np.max(np.abs(o.rhs(U)[4])) <= 1e-12 * kappa * Tb / h ** 2
    # a wall temperature off the profile leaves a boundary heat flux
    o2 = oracle.Oracle(p, box(3, (2, 2, 3), (1.0, 1.0, H), {"kind": 1, "twall": Ta + 0.01}, {"kind": 1, "twall": Tb}))
    assert np.max(np.abs(o2.rhs(U)[4])) > 1e-3 * kappa * (Tb - Ta) / H / h


def test_dynamic_angle_traction_is_tangential():
    """The gamma_1 traction uses the tangential gradient grad_Gamma c = grad c -
    (grad c . n) n: with c varying across the floor as well as along it, the
    floor's gamma_1 term changes the x-momentum but leaves the wall-normal
    (z) momentum of every node exactly as it is without gamma_1 (gamma_1 enters
    nothing else that reaches the momentum)."""
    g1, H, s, d, rho0 = 0.5, 0.5, 0.2, 0.02, 0.3
    p = oracle.make_params()
    T0 = 0.9
    mk = lambda g: oracle.Oracle(p, box(3, (4, 1, 2), (1.0, 1.0, H), {"kind": 3, "g1": g, "twall": T0},
                                        {"kind": 2}))
    o1, o0 = mk(g1), mk(0.0)
    x, y, z = o1.coords()
    rho = rho0 + d * np.sin(2 * np.pi * x) + 0.5 * d * np.cos(np.pi * z / H)
    w = s * z * (H - z) * (1 + 0.5 * np.cos(2 * np.pi * x))
    U = np.zeros((6, o1.nnodes))
    U[0] = rho
    U[3] = rho * w
    U[4] = energy(rho, w * w, T0)
    U[5] = rho + 0.01 * np.cos(np.pi * z / H)
    a, b = o1.rhs(U), o0.rhs(U)
    scale = np.max(np.abs(b[3]))
    assert np.max(np.abs(a[3] - b[3])) <= 1e-13 * scale
    assert np.max(np.abs(a[1] - b[1])) > 1e-6 * np.max(np.abs(b[1]))


def test_wall_values_of_the_lifted_velocity():
    """BR1 takes the wall's own value at a wall face (no-slip: the wall
    velocity; slip: the fluid velocity without its normal part), and the
    lifted gradient integrates to the sum over the boundary of that value
    times the outward normal (interior faces cancel). A uniform velocity
    (U0, 0, W0), which satisfies neither wall condition, between a slip floor
    and a fixed no-slip lid therefore gives int du/dz = -A U0 (floor: U0,
    lid: 0) and int dw/dz = 0 (both walls: 0), A the wall area."""
    U0, W0, rho, T, H = 0.2, 0.15, 0.3, 0.9, 0.6
    p = oracle.make_params()
    o = oracle.Oracle(p, box(3, (2, 2, 3), (1.0, 1.0, H), {"kind": 2}, {"kind": 1, "twall": T}))
    U = np.zeros((6, o.nnodes))
    U[0] = rho
    U[1] = rho * U0
    U[3] = rho * W0
    U[4] = energy(rho, U0 * U0 + W0 * W0, T)
    U[5] = rho
    q = o.lift1(U)
    W = weights(o)
    # q rows: grad rho (0-2), grad u (3-5), grad v (6-8), grad w (9-11), grad c (12-14)
    assert abs(W @ q[5] - (-1.0 * U0)) <= 1e-13
    assert abs(W @ q[11]) <= 1e-13
    assert abs(W @ q[3]) <= 1e-13 and abs(W @ q[9]) <= 1e-13


def test_slip_wall_normal_traction():
    """u = (0, 0, s z (H - z)) between two slip walls, uniform density and
    temperature: the total z-momentum changes only through the walls' normal
    viscous traction (4/3) mu dw/dz (the pressure is uniform and cancels),
    at the rate -(8/3) mu s H A."""
    mu, H, s = 0.01, 0.5, 0.3
    p = oracle.make_params(mu=mu)
    T0, rho = 0.9, 0.3
    o = oracle.Oracle(p, box(4, (2, 2, 3), (1.0, 1.0, H), {"kind": 2}, {"kind": 2}))
    x, y, z = o.coords()
    w = s * z * (H - z)
    U = np.zeros((6, o.nnodes))
    U[0] = rho
    U[3] = rho * w
    U[4] = energy(rho, w * w, T0)
    U[5] = rho
    rate = np.dot(weights(o), o.rhs(U)[3])
    exact = -(8.0 / 3.0) * mu * s * H * 1.0
    assert abs(rate - exact) <= 1e-10 * abs(exact), (rate, exact)


def test_moving_lid_over_fluid_at_rest():
    """Fluid at rest (uniform rho = c and T) under a no-slip lid moving at U,
    slip floor.  Only the lid exchanges momentum and energy: its ghost flux
    lambda rho U (momentum) and lambda rho U^2 (energy), lambda the sound
    speed, and the traction of the lifted shear, whose trace at the lid is
    U (2/h) c_N with c_N = sum_k l_k(1)^2 / w_k of the Gauss basis (the face
    value U enters the lifting only through the lid's own face).  So the
    totals change at A (lambda rho U + mu U 2 c_N / h) and
    A (lambda rho U^2 + mu U^2 2 c_N / h)."""
    N, nz, H, U, mu = 3, 3, 0.5, 0.3, 0.01
    p = oracle.make_params(mu=mu)
    T0, rho = 0.95, 0.25
    o = oracle.Oracle(p, box(N, (2, 2, nz), (1.0, 1.0, H), {"kind": 2},
                             {"kind": 1, "uwall": (U, 0.0, 0.0), "twall": T0}))
    x, y, z = o.coords()
    Ust = np.zeros((6, o.nnodes))
    Ust[0] = rho
    Ust[4] = energy(rho, 0.0, T0)
    Ust[5] = rho
    rates = weights(o) @ o.rhs(Ust).T
    xg, wg = np.polynomial.legendre.leggauss(N + 1)
    l1 = np.array([np.prod([(1 - xg[j]) / (xg[k] - xg[j]) for j in range(N + 1) if j != k]) for k in range(N + 1)])
    cN = np.sum(l1 ** 2 / wg)
    h = H / nz
    cs2 = (1 + 1 / CV) * R * T0 / (1 - B * rho) ** 2 - 2 * A * rho
    lam = np.sqrt(abs(cs2))
    shear = mu * U * 2 * cN / h
    assert abs(rates[1] - (lam * rho * U + shear)) <= 1e-12 * (lam * rho * U + shear), (rates[1], lam * rho * U + shear)
    assert abs(rates[4] - (lam * rho * U * U + shear * U)) <= 1e-12 * (lam * rho * U * U), rates[4]
    assert abs(rates[0]) <= 1e-14 and abs(rates[2]) <= 1e-14

"""Pins of the oracle's wall-temperature table and varying wall temperature
(Sec. 3.2: sigma_vl tabulated at 10000 equidistant temperatures on [0.3, 1]
with a 15-point Gauss rule and interpolated linearly; the Maxwell states are
tabulated alongside).

* Table entries at grid temperatures equal the directly evaluated 15-point
  sigma and the Maxwell states (which other tests pin against Tables 1, 2,
  the equal-area rule and brute force); the last entry is the critical point.
* Between grid points the interpolant stays within the linear-interpolation
  bound h^2/8 max|f''| of the directly evaluated functions, and sigma agrees
  with the accurate composite-rule value to the 15-point rule's own accuracy.
* A wall whose temperature varies by a negligible gradient gives the same
  right-hand side as the fixed-temperature wall, to the table's accuracy.
* An isothermal wall whose temperature follows the fluid's linear
  temperature along the wall gives the exact lifted temperature gradient at
  every node; a fixed wall temperature does not.
* Wall temperatures leaving [0.3, 0.99] are rejected.
"""
import numpy as np
import pytest

import oracle

T0, T1, NT = 0.3, 1.0, oracle.NTAB
DT = (T1 - T0) / (NT - 1)


@pytest.fixture(scope="module")
def tab():
    return oracle.wall_table()


def test_grid_entries_and_critical_point(tab):
    rng = np.random.default_rng(3)
    for k in list(rng.integers(0, NT - 1, 12)) + [0, NT - 2]:
        T = T0 + k * DT
        rv, rl, _ = oracle.maxwell(T)
        assert tab[k, 0] == oracle.sigma_gauss15(T, 0.5)       # sqrt(2 gamma) = 1
        assert tab[k, 1] == rv and tab[k, 2] == rl
        got = oracle.wall_table_lookup(tab, T)
        assert np.allclose(got, tab[k], rtol=1e-13, atol=0)
    assert tab[-1, 0] == 0.0 and tab[-1, 1] == tab[-1, 2] == 1.0


def test_interpolation_error_bound(tab):
    rng = np.random.default_rng(4)
    for T in rng.uniform(0.3, 0.99, 40):
        rv, rl, _ = oracle.maxwell(T)
        s = oracle.sigma_gauss15(T, 0.5)
        got = oracle.wall_table_lookup(tab, T)
        # second differences of the tabulated functions bound f'' on the cell
        k = min(int((T - T0) / DT), NT - 3)
        bound = DT ** 2 / 8 * np.max(np.abs(tab[k + 2] - 2 * tab[k + 1] + tab[k]) / DT ** 2 * 4 + 1e-300) + 1e-15
        err = np.abs(got - np.array([s, rv, rl]))
        assert np.all(err <= bound + 1e-13 * np.abs(got)), (T, err, bound)
    # sigma against the accurate composite rule where the 15-point rule is
    # exact to ~1e-13: the difference is the interpolation error, and sigma ~
    # (1 - T)^(3/2) near the critical point gives sigma''/sigma ~ 0.75/(1-T)^2
    for T in rng.uniform(0.7, 0.99, 20):
        got = oracle.wall_table_lookup(tab, T)[0] * np.sqrt(2e-4)
        ref = oracle.sigma(T, 1e-4)
        tol = 2 * DT ** 2 / 8 * 0.75 / (1 - T) ** 2 + 1e-11
        assert abs(got - ref) <= tol * ref, (T, got, ref, tol)


def box(tgrad_z=(0.0, 0.0, 0.0), twall=0.85, N=3, n=(3, 3, 2), kind=1):
    return oracle.make_box(N, n, (0.0, 0.0, 0.0), (1.0, 1.0, 0.5), (1, 1, 0), (0, 0, 0, 0, kind, 2),
                           (0, 0, 0, 0, twall, 0), (90, 90, 90, 90, 60, 90),
                           side_g3=(float("inf"),) * 4 + (0.02, float("inf")),
                           side_tgrad=((0, 0, 0),) * 4 + (tgrad_z, (0, 0, 0)))


@pytest.mark.parametrize("kind", [1, 3])
def test_negligible_gradient_equals_fixed_wall(kind):
    p = oracle.make_params()
    fixed = oracle.Oracle(p, box(kind=kind))
    var = oracle.Oracle(p, box((1e-12, 0.0, 0.0), kind=kind))
    U = fixed.init_droplets(0.85, [[0.5, 0.5, 0.0]], [0.2], 0.05)
    x, y, z = fixed.coords()
    U[5] = U[0] + 0.01 * np.sin(2 * np.pi * (x + y))
    a, b = fixed.rhs(U), var.rhs(U)
    scale = np.max(np.abs(a), axis=1)
    err = np.max(np.abs(a - b), axis=1) / scale
    assert np.all(err <= 1e-8), err


def test_isothermal_wall_following_the_fluid_temperature():
    """x-walls at T_w(y) = 0.85 + 0.05 y (isothermal), slip walls in y,
    periodic z; fluid at rest with uniform rho = c and T = 0.85 + 0.05 y:
    the lifted grad T is (0, 0.05, 0) at every node."""
    p = oracle.make_params()
    g = 0.05

    def mk(tg):
        b = oracle.make_box(3, (3, 3, 2), (0.0, 0.0, 0.0), (1.0, 1.0, 0.5), (0, 0, 1), (1, 1, 2, 2, 0, 0),
                            (0.85, 0.85, 0, 0, 0, 0), (90.0,) * 6,
                            side_tgrad=((0, tg, 0), (0, tg, 0)) + ((0, 0, 0),) * 4)
        return oracle.Oracle(p, b)

    o = mk(g)
    x, y, z = o.coords()
    rho = 0.3
    U = np.zeros((6, o.nnodes))
    U[0] = rho
    U[4] = rho * (8.0 / 3.0 * 5.0 * (0.85 + g * y) - 3.0 * rho)
    U[5] = rho
    q = o.lift2(U)
    assert np.max(np.abs(q[0] - (0.85 + g * y))) <= 1e-14
    assert np.max(np.abs(q[1])) <= 1e-13 and np.max(np.abs(q[3])) <= 1e-13
    assert np.max(np.abs(q[2] - g)) <= 1e-12
    # a fixed wall temperature (0.85) bends grad T near the x-walls
    q0 = mk(0.0).lift2(U)
    assert np.max(np.abs(q0[1])) > 1e-3


def test_wall_temperature_out_of_range_is_rejected():
    p = oracle.make_params()
    with pytest.raises(ValueError):
        oracle.Oracle(p, box((0.2, 0.0, 0.0), twall=0.85))   # reaches 1.05 at x = 1
    with pytest.raises(ValueError):
        oracle.Oracle(p, box((-0.6, 0.0, 0.0), twall=0.85))  # reaches 0.25


def box_t(twall=0.85, tgrad=(1e-9, 0.0, 0.0), trate=0.0):
    return oracle.make_box(3, (3, 3, 2), (0.0, 0.0, 0.0), (1.0, 1.0, 0.5), (1, 1, 0), (0, 0, 0, 0, 1, 2),
                           (0, 0, 0, 0, twall, 0), (90, 90, 90, 90, 60, 90),
                           side_tgrad=((0, 0, 0),) * 4 + (tgrad, (0, 0, 0)),
                           side_trate=(0.0,) * 4 + (trate, 0.0))


def droplet_state(o):
    U = o.init_droplets(0.85, [[0.5, 0.5, 0.0]], [0.2], 0.05)
    x, y, z = o.coords()
    U[5] = U[0] + 0.01 * np.sin(2 * np.pi * (x + y))
    return U


def test_wall_temperature_rate_is_a_shift_in_time():
    """T_w = twall + r t evaluated at time t equals the wall at twall + r t
    and time 0 (both through the table)."""
    p = oracle.make_params()
    r, t = 0.4, 0.2
    timed = oracle.Oracle(p, box_t(trate=r))
    shifted = oracle.Oracle(p, box_t(twall=0.85 + r * t))
    U = droplet_state(timed)
    timed.set_time(t)
    a, b = timed.rhs(U), shifted.rhs(U)
    scale = np.max(np.abs(b), axis=1)
    assert np.all(np.max(np.abs(a - b), axis=1) <= 1e-13 * scale)
    timed.set_time(0.0)
    assert np.max(np.abs(timed.rhs(U)[5] - b[5])) > 1e-6 * scale[5]


def test_rk_stages_use_their_own_times():
    """One step of run() from t0 equals the 2N scheme evaluated stage by stage
    at t0 + c_s dt with rhs() (and differs from evaluating every stage at t0),
    on a wall whose temperature changes quickly in time."""
    p = oracle.make_params()
    o = oracle.Oracle(p, box_t(trate=50.0))
    U0 = droplet_state(o)
    t0, dt = 0.001, 2e-5
    A, B, C = (np.zeros(5) for _ in range(3))
    oracle.lib().orc_rk_coeffs(oracle._ptr(A), oracle._ptr(B), oracle._ptr(C))
    assert np.all(np.diff(C) > 0) and C[0] == 0.0 and 0.9 < C[4] < 1.0

    def manual(times):
        U, R = U0.copy(), np.zeros_like(U0)
        for s in range(5):
            o.set_time(times[s])
            Ut = o.rhs(U)
            R = dt * Ut if s == 0 else A[s] * R + dt * Ut
            U = U + B[s] * R
        return U

    U, R = U0.copy(), np.zeros_like(U0)
    o.run(U, R, t0, dt, 1)
    ref = manual([t0 + C[s] * dt for s in range(5)])
    scale = np.max(np.abs(U0), axis=1)
    assert np.all(np.max(np.abs(U - ref), axis=1) <= 1e-14 * scale)
    wrong = manual([t0] * 5)
    assert np.max(np.abs(U[5] - wrong[5])) > 1e-12 * scale[5]


def test_isothermal_wall_heating_with_the_fluid():
    """x-walls at T_w = 0.85 + r t, fluid at rest with uniform T = 0.85 + r t1:
    the lifted grad T vanishes at t = t1 and not at other times."""
    p = oracle.make_params()
    r, t1 = 0.3, 0.1
    b = oracle.make_box(3, (3, 3, 2), (0.0, 0.0, 0.0), (1.0, 1.0, 0.5), (0, 1, 1), (1, 1, 0, 0, 0, 0),
                        (0.85, 0.85, 0, 0, 0, 0), (90.0,) * 6, side_trate=(r, r, 0, 0, 0, 0))
    o = oracle.Oracle(p, b)
    rho = 0.3
    U = np.zeros((6, o.nnodes))
    U[0] = rho
    U[4] = rho * (8.0 / 3.0 * 5.0 * (0.85 + r * t1) - 3.0 * rho)
    U[5] = rho
    o.set_time(t1)
    assert np.max(np.abs(o.lift2(U)[1:4])) <= 1e-12
    o.set_time(0.0)
    assert np.max(np.abs(o.lift2(U)[1])) > 1e-3

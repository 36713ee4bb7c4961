"""Pins of the Rusanov dissipation speed (Sec. 3.1: local Lax-Friedrichs flux
with lambda = max over the two sides of |u . n| + c~, c~ = sqrt(|c_s^2|)).

With alpha = beta = gamma = mu = k = 0 the order parameter is a passive
scalar, c_t + div(c u) = 0, and no other term acts on it.  Take c constant
in each element.  Then the weak form with the test function c_e (a constant,
which the collocated Gauss rule integrates exactly) gives, for the DGSEM
semi-discretisation,

    d/dt sum_e int_e c^2/2 = -c_e sum_faces int (F* . n) dS
                           = -1/2 sum_(interior faces) lambda (c+ - c-)^2 A_f
                             + 1/2 sum_e c_e^2 oint u . n dS,

where A_f is the face area and the last sum vanishes for a velocity that is
uniform (each element's outward n dS sums to zero).  The central part of the
flux is energy-neutral; only the jump term dissipates, at the rate set by
lambda.  The three cases below make lambda differ between the plausible
readings:

  * fluid at rest, uniform density, temperature constant per element but
    different between elements: lambda = max(c~-, c~+) (not the smaller);
  * uniform velocity, density and temperature: lambda = |u . n| + c~ (not c~
    alone), with |u . n| different on the x, y and z faces;
  * velocity and temperature constant per element and different between
    elements: each side's speed is its own |u . n| + c~, and the larger of
    the two is taken whichever side carries it (the central part of the flux
    then leaves a closed-form term of its own).

The sound speed comes from the closed form of eq. speedofsound for the van
der Waals fluid, itself pinned against numerical derivatives of the
Helmholtz energy in test_oracle_thermo.py.
"""
import numpy as np
import pytest

import oracle

R, A, B, CV = 8.0 / 3.0, 3.0, 1.0 / 3.0, 5.0
FREE = dict(mu=0.0, kappa=0.0, gam=0.0, alpha=0.0, beta=0.0)


def sound_speed(rho, T):
    cs2 = (1.0 + 1.0 / CV) * R * T / (1.0 - B * rho) ** 2 - 2.0 * A * rho
    return np.sqrt(np.abs(cs2))


def setup(N, n, length):
    p = oracle.make_params(**FREE)
    b = oracle.make_box(N, n, (0.0, 0.0, 0.0), length)
    return oracle.Oracle(p, b)


def element_field(o, vals):
    """A field constant in each element (vals per element) at every node."""
    return np.repeat(np.asarray(vals, dtype=np.float64), (o.N + 1) ** 3)


def energy_rate(o, c, ct):
    """d/dt sum int c^2/2 by the collocated Gauss rule (weights times J)."""
    _, w, *_ = oracle.basis(o.N)
    w3 = (w[None, None, :] * w[None, :, None] * w[:, None, None]).reshape(-1)
    _, J, _ = o.metrics()
    return float(np.sum(np.tile(w3, o.nelems) * J * c * ct))


def face_pairs(n):
    """Interior face pairs of a periodic box: (element, neighbour, axis)."""
    nx, ny, nz = n
    out = []
    for ez in range(nz):
        for ey in range(ny):
            for ex in range(nx):
                e = ex + nx * (ey + ny * ez)
                idx = [ex, ey, ez]
                for d in range(3):
                    j = list(idx)
                    j[d] = (j[d] + 1) % n[d]
                    out.append((e, j[0] + nx * (j[1] + ny * j[2]), d))
    return out


def expected_rate(n, length, lam_of, cel):
    h = [length[d] / n[d] for d in range(3)]
    area = [h[1] * h[2], h[0] * h[2], h[0] * h[1]]
    return -0.5 * sum(lam_of(e, f, d) * (cel[f] - cel[e]) ** 2 * area[d] for e, f, d in face_pairs(n))


def test_closed_form_sound_speed_is_the_oracles():
    # the test's closed form is the one the thermodynamics pins fix
    for rho, T in ((0.6, 0.9), (0.6, 1.2), (1.3, 0.85), (0.9, 0.8)):
        assert abs(sound_speed(rho, T) ** 2 - abs(oracle.cs2(rho, T, CV))) < 1e-13


@pytest.mark.parametrize("N", [2, 3])
def test_rusanov_speed_is_the_larger_of_the_two_sides(N):
    n, length = (3, 2, 2), (1.5, 1.0, 0.8)
    o = setup(N, n, length)
    rng = np.random.default_rng(21)
    E = o.nelems
    rho0 = 0.6
    Tel = rng.uniform(0.9, 1.2, E)        # c_s^2 = 5 T - 3.6 > 0 at rho = 0.6
    cel = rng.uniform(0.4, 1.6, E)
    U = np.zeros((6, o.nnodes))
    U[0] = rho0
    U[4] = element_field(o, rho0 * (R * CV * Tel - A * rho0))
    U[5] = element_field(o, cel)
    ct = o.rhs(U)[5]
    got = energy_rate(o, U[5], ct)
    cs = sound_speed(rho0, Tel)
    want = expected_rate(n, length, lambda e, f, d: max(cs[e], cs[f]), cel)
    smaller = expected_rate(n, length, lambda e, f, d: min(cs[e], cs[f]), cel)
    assert want < 0.0 and abs(smaller - want) > 0.05 * abs(want)
    assert abs(got - want) <= 1e-12 * abs(want), (got, want)


@pytest.mark.parametrize("N", [2, 4])
def test_rusanov_speed_includes_the_normal_velocity(N):
    n, length = (2, 3, 2), (1.0, 1.2, 0.9)
    o = setup(N, n, length)
    rng = np.random.default_rng(22)
    rho0, T0 = 0.8, 0.95
    u0 = np.array([0.3, -0.2, 0.1])
    cel = rng.uniform(0.4, 1.6, o.nelems)
    U = np.zeros((6, o.nnodes))
    U[0] = rho0
    U[1:4] = rho0 * u0[:, None]
    U[4] = rho0 * (R * CV * T0 - A * rho0) + 0.5 * rho0 * float(u0 @ u0)
    U[5] = element_field(o, cel)
    ct = o.rhs(U)[5]
    got = energy_rate(o, U[5], ct)
    cs = float(sound_speed(rho0, T0))
    want = expected_rate(n, length, lambda e, f, d: abs(u0[d]) + cs, cel)
    without = expected_rate(n, length, lambda e, f, d: cs, cel)
    assert want < 0.0 and abs(without - want) > 0.05 * abs(want)
    assert abs(got - want) <= 1e-12 * abs(want), (got, want)


@pytest.mark.parametrize("N", [2, 3])
def test_rusanov_speed_of_each_side_is_its_own(N):
    # velocity and temperature constant per element and different between
    # elements: the central part of the flux no longer cancels, and the
    # balance per face is 1/2 (c+ - c-) (c- u- . n + c+ u+ . n) - 1/2 lambda
    # (c+ - c-)^2 A with lambda = max(|u- . n| + c~-, |u+ . n| + c~+): either
    # side may carry the larger speed
    n, length = (3, 2, 2), (1.5, 1.0, 0.8)
    o = setup(N, n, length)
    rng = np.random.default_rng(23)
    E = o.nelems
    rho0 = 0.6
    Tel = rng.uniform(0.9, 1.2, E)
    uel = rng.uniform(-0.8, 0.8, (E, 3))
    cel = rng.uniform(0.4, 1.6, E)
    U = np.zeros((6, o.nnodes))
    U[0] = rho0
    for m in range(3):
        U[1 + m] = element_field(o, rho0 * uel[:, m])
    U[4] = element_field(o, rho0 * (R * CV * Tel - A * rho0) + 0.5 * rho0 * np.sum(uel ** 2, axis=1))
    U[5] = element_field(o, cel)
    ct = o.rhs(U)[5]
    got = energy_rate(o, U[5], ct)
    cs = sound_speed(rho0, Tel)
    h = [length[d] / n[d] for d in range(3)]
    area = [h[1] * h[2], h[0] * h[2], h[0] * h[1]]

    def rate(lam_of):
        tot = 0.0
        for e, f, d in face_pairs(n):
            jump = cel[f] - cel[e]
            tot += (0.5 * jump * (cel[e] * uel[e, d] + cel[f] * uel[f, d]) - 0.5 * lam_of(e, f, d) * jump ** 2) * area[d]
        return tot

    want = rate(lambda e, f, d: max(abs(uel[e, d]) + cs[e], abs(uel[f, d]) + cs[f]))
    one_sided = rate(lambda e, f, d: max(cs[e], abs(uel[f, d]) + cs[f]))
    assert abs(one_sided - want) > 0.01 * abs(want)
    assert abs(got - want) <= 1e-12 * abs(want), (got, want)

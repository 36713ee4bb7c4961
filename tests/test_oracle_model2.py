"""Relaxation model 2 in the oracle (Sec. 2.3.2, eq. modified_pressure and
eq. navierstokeskorteweg_palpha; HLLC interior flux as stated in Sec. 4 for
this model).  Pins: the HLLC flux against closed-form properties of a
Riemann flux (consistency, exact contacts, supersonic upwinding, reversal
symmetry), conservation and free-stream preservation of the discretisation,
and convergence to the same manufactured solution as model 1 (the two models
write the same PDE; see test_oracle_convergence.py)."""
import numpy as np
import pytest

import oracle

P2 = dict(model=2)


def p_alpha(rho, T, alpha=100.0):
    return oracle.pressure(rho, T) + 0.5 * alpha * rho * rho


def euler_flux(U, T, n, alpha=100.0):
    """F^C . n of eq. navierstokeskorteweg_palpha for one state (p -> p_alpha)."""
    rho, m, E, c = U[0], np.asarray(U[1:4]), U[4], U[5]
    u = m / rho
    un = float(u @ np.asarray(n))
    p = p_alpha(rho, T, alpha)
    return np.array([rho * un, *(m * un + p * np.asarray(n)), (E + p) * un, c * un])


def state(rho, u, T, c=None, alpha=100.0):
    """Conserved state with the given temperature; the energy holds the
    internal, kinetic and relaxation parts (no gradient energy at a point)."""
    c = rho if c is None else c
    u = np.asarray(u, dtype=float)
    eps = 8.0 / 3.0 * 5.0 * T - 3.0 * rho
    E = rho * (eps + 0.5 * u @ u) + 0.5 * alpha * (rho - c) ** 2
    return np.array([rho, *(rho * u), E, c])


def sound(rho, T, alpha=100.0):
    return np.sqrt(oracle.cs2(rho, T) + alpha * rho)


@pytest.mark.parametrize("seed", range(5))
def test_hllc_is_consistent(seed):
    rng = np.random.default_rng(seed)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    rho, T = rng.uniform(0.3, 1.8), rng.uniform(0.85, 1.1)
    U = state(rho, rng.normal(scale=0.5, size=3), T, c=rho * rng.uniform(0.95, 1.05))
    F = oracle.numflux(oracle.make_params(**P2), U, T, U, T, n)
    assert np.allclose(F, euler_flux(U, T, n), rtol=1e-13, atol=1e-13)


def test_hllc_resolves_an_isolated_contact_exactly():
    """Left and right states with the same normal velocity and the same
    p_alpha (different density, temperature, order parameter and tangential
    velocity) are joined by a contact/shear wave only; HLLC returns the
    upwind physical flux (Rusanov would add dissipation)."""
    n = np.array([0.6, 0.0, 0.8])
    t = np.array([0.8, 0.0, -0.6])
    un = 0.3
    rhoL, TL = 1.7, 0.9
    pa = p_alpha(rhoL, TL)
    rhoR = 0.45
    # temperature with the same p_alpha on the right: p = rho R T/(1 - b rho) - a rho^2
    TR = (pa - 0.5 * 100.0 * rhoR ** 2 + 3.0 * rhoR ** 2) * (1 - rhoR / 3.0) / (rhoR * 8.0 / 3.0)
    assert abs(p_alpha(rhoR, TR) - pa) < 1e-12 * pa
    UL = state(rhoL, un * n + 0.2 * t, TL, c=1.65)
    UR = state(rhoR, un * n - 0.4 * t, TR, c=0.5)
    F2 = oracle.numflux(oracle.make_params(**P2), UL, TL, UR, TR, n)
    assert np.allclose(F2, euler_flux(UL, TL, n), rtol=1e-12, atol=1e-12)
    # the same states flowing the other way take the right state's flux
    F2b = oracle.numflux(oracle.make_params(**P2), state(rhoL, -un * n, TL, c=1.65), TL,
                         state(rhoR, -un * n, TR, c=0.5), TR, n)
    assert np.allclose(F2b, euler_flux(state(rhoR, -un * n, TR, c=0.5), TR, n), rtol=1e-12, atol=1e-12)
    F1 = oracle.numflux(oracle.make_params(), UL, TL, UR, TR, n)
    assert not np.allclose(F1, euler_flux(UL, TL, n), rtol=1e-3)


@pytest.mark.parametrize("dT", [1e-5, -2e-5])
def test_hllc_reproduces_linear_acoustics(dT):
    """Two states at rest with a small pressure jump (same density, slightly
    different temperature): linear acoustics gives the interface velocity
    u* = (p_L - p_R) / (rho_L a_L + rho_R a_R) and pressure p* = the mean
    (equal impedances), so the flux carries mass rho u*, momentum p* n and
    energy (E + p) u* to first order in the jump (relative error O(u*/a))."""
    n = np.array([0.0, 0.6, 0.8])
    rho, T = 0.35, 0.95
    UL, UR = state(rho, [0.0, 0.0, 0.0], T + dT), state(rho, [0.0, 0.0, 0.0], T)
    pL, pR = p_alpha(rho, T + dT), p_alpha(rho, T)
    aL, aR = sound(rho, T + dT), sound(rho, T)
    us = (pL - pR) / (rho * aL + rho * aR)
    ps = 0.5 * (pL + pR)
    F = oracle.numflux(oracle.make_params(**P2), UL, T + dT, UR, T, n)
    rel = abs(us) / aR
    assert abs(F[0] - rho * us) <= 10 * rel * abs(rho * us)
    assert np.allclose(F[1:4], ps * n, rtol=10 * rel * abs(pL - pR) / ps, atol=0)
    h = 0.5 * (UL[4] + UR[4]) + ps
    assert abs(F[4] - h * us) <= 10 * rel * abs(h * us)
    assert abs(F[5] - rho * us) <= 10 * rel * abs(rho * us)


def test_hllc_upwinds_supersonic_flow():
    n = np.array([0.0, 1.0, 0.0])
    rhoL, TL, rhoR, TR = 0.5, 1.0, 1.2, 0.95
    v = 1.5 * max(sound(rhoL, TL), sound(rhoR, TR))
    UL, UR = state(rhoL, v * n, TL), state(rhoR, v * n + [0.3, 0, 0], TR)
    F = oracle.numflux(oracle.make_params(**P2), UL, TL, UR, TR, n)
    assert np.allclose(F, euler_flux(UL, TL, n), rtol=1e-13, atol=1e-13)
    F = oracle.numflux(oracle.make_params(**P2), state(rhoL, -v * n, TL), TL, state(rhoR, -v * n, TR), TR, n)
    assert np.allclose(F, euler_flux(state(rhoR, -v * n, TR), TR, n), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("model", [1, 2])
def test_numflux_reverses_with_the_normal(model):
    rng = np.random.default_rng(11)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    UL, UR = state(1.6, [0.2, -0.1, 0.4], 0.9), state(0.4, [-0.3, 0.2, 0.1], 0.92, c=0.42)
    p = oracle.make_params(model=model)
    F = oracle.numflux(p, UL, 0.9, UR, 0.92, n)
    G = oracle.numflux(p, UR, 0.92, UL, 0.9, -n)
    assert np.allclose(F, -G, rtol=1e-13, atol=1e-13)


def make(N, n, **kw):
    return oracle.Oracle(oracle.make_params(model=2), oracle.make_box(N, n, **kw))


@pytest.mark.parametrize("amp", [0.0, 0.05])
def test_model2_free_stream(amp):
    o = make(3, (3, 3, 3), curve_amp=amp)
    U = np.tile(state(0.9, [0.3, -0.2, 0.1], 1.0, c=0.9)[:, None], (1, o.nnodes))
    Ut = o.rhs(U)
    assert np.max(np.abs(Ut)) < 5e-11 * np.max(np.abs(U))


def test_model2_conserves_mass_with_walls():
    o = oracle.Oracle(oracle.make_params(model=2),
                      oracle.make_box(3, (3, 3, 2), length=(1.0, 1.0, 0.5), periodic=(1, 1, 0),
                                      side_kind=(0, 0, 0, 0, 1, 2), side_twall=(0, 0, 0, 0, 0.9, 0),
                                      side_theta=(90, 90, 90, 90, 60, 90)))
    U = o.init_droplets(0.85, [(0.5, 0.5, 0.0)], [0.2], 0.05, None)
    W = o.metrics()[1] * np.tile(np.kron(np.kron(*[oracle.basis(3)[1]] * 2), oracle.basis(3)[1]), o.nelems)
    Ut = o.rhs(U)
    assert abs(W @ Ut[0]) < 1e-12 * (W @ np.abs(Ut[0]) + 1e-300)

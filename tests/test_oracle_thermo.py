"""Pins of the oracle's thermodynamics against the paper and against
independent characterisations (numerical derivatives of the Helmholtz energy,
the equal-area rule, SciPy quadrature of the printed integral)."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, optimize

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
R, A, B, CV = 8.0 / 3.0, 3.0, 1.0 / 3.0, 5.0


def psi(rho, T):
    """Helmholtz energy per volume of Sec. 2.1 (eq. helmholtzfreeenergyvol)."""
    return (rho * R * T * CV * (1.0 - math.log(T)) + rho * R * T * math.log(B * rho / (1.0 - B * rho))
            - A * rho * rho)


def d1(f, x, h):
    return (f(x + h) - f(x - h)) / (2 * h)


def test_reduced_constants_give_critical_point_one():
    # Sec. 2.1: with R = 8/3, a = 3, b = 1/3 the critical point is rho = T = p = 1:
    # dp/drho = d2p/drho2 = 0 there, and p = 1.
    assert abs(oracle.pressure(1.0, 1.0) - 1.0) < 1e-14
    dp = d1(lambda r: oracle.pressure(r, 1.0), 1.0, 1e-4)
    d2p = (oracle.pressure(1.0 + 1e-3, 1.0) - 2 * oracle.pressure(1.0, 1.0) + oracle.pressure(1.0 - 1e-3, 1.0)) / 1e-6
    assert abs(dp) < 1e-7 and abs(d2p) < 1e-5


@pytest.mark.parametrize("rho,T", [(0.3, 0.85), (1.0, 0.9), (1.8, 0.8), (2.5, 1.1)])
def test_pressure_is_legendre_transform_of_psi(rho, T):
    # eq. pressure: p = rho dpsi/drho - psi, checked by differentiating psi numerically.
    p_num = rho * d1(lambda r: psi(r, T), rho, 1e-5) - psi(rho, T)
    assert abs(oracle.pressure(rho, T) - p_num) < 1e-8


@pytest.mark.parametrize("rho,T", [(0.3, 0.85), (1.0, 0.9), (1.8, 0.8), (2.2, 0.95)])
def test_speed_of_sound_matches_isentropic_derivative(rho, T):
    # eq. speedofsound: c_s^2 = (dp/drho)_T - (dp/dT)_rho (ds/drho)_T / (ds/dT)_rho with the
    # specific entropy s = -(1/rho) dpsi/dT, everything by numerical derivatives of psi.
    def p(r, t):
        return r * d1(lambda x: psi(x, t), r, 1e-5) - psi(r, t)

    def s(r, t):
        return -d1(lambda x: psi(r, x), t, 1e-5) / r

    h = 1e-4
    dp_dr = (p(rho + h, T) - p(rho - h, T)) / (2 * h)
    dp_dT = (p(rho, T + h) - p(rho, T - h)) / (2 * h)
    ds_dr = (s(rho + h, T) - s(rho - h, T)) / (2 * h)
    ds_dT = (s(rho, T + h) - s(rho, T - h)) / (2 * h)
    c2 = dp_dr - dp_dT * ds_dr / ds_dT
    assert abs(oracle.cs2(rho, T) - c2) < 2e-5 * max(1.0, abs(c2))


def test_speed_of_sound_minimum_positive_above_spinodal_reading():
    # With c_v = 5 the isentropic c_s^2 stays positive at T = 0.85 (minimum about +0.1192
    # near rho = 0.987), although the isothermal derivative is negative in the spinodal.
    res = optimize.minimize_scalar(lambda r: oracle.cs2(r, 0.85), bounds=(0.3, 2.0), method="bounded",
                                   options={"xatol": 1e-10})
    assert abs(res.fun - 0.1192) < 1e-4 and abs(res.x - 0.987) < 2e-3


def test_internal_energy_is_psi_minus_T_dpsidT():
    # Temperature recovery uses eps = R c_v T - a rho; check against rho eps = psi - T dpsi/dT.
    for rho, T in [(0.4, 0.85), (1.6, 0.9)]:
        reps = psi(rho, T) - T * d1(lambda t: psi(rho, t), T, 1e-5)
        assert abs(reps - rho * (R * CV * T - A * rho)) < 1e-8


def test_spinodal_is_zero_of_isothermal_derivative():
    v, l = oracle.spinodal(0.85)
    for r in (v, l):
        assert abs(d1(lambda x: oracle.pressure(x, 0.85), r, 1e-6)) < 1e-8
    assert abs(v - 0.58108) < 1e-5 and abs(l - 1.48880) < 1e-5


def test_maxwell_matches_table2():
    g = GOLD["table2_static_bubble"]
    rv, rl, ps = oracle.maxwell(g["T0"])
    assert round(rv, 4) == g["rho_v_sat"] and round(rl, 4) == g["rho_l_sat"]


@pytest.mark.parametrize("T", [0.75, 0.8, 0.85, 0.9, 0.95])
def test_maxwell_equal_area(T):
    # Independent characterisation: Maxwell's equal-area rule in specific volume,
    # int_{v_l}^{v_v} p dv = p_sat (v_v - v_l), with p_sat = p(rho_v) = p(rho_l).
    rv, rl, ps = oracle.maxwell(T)
    assert abs(oracle.pressure(rv, T) - ps) < 1e-13 and abs(oracle.pressure(rl, T) - ps) < 1e-13
    vv, vl = 1.0 / rv, 1.0 / rl
    area, _ = integrate.quad(lambda v: oracle.pressure(1.0 / v, T), vl, vv, epsabs=1e-13, epsrel=1e-13, limit=200)
    assert abs(area - ps * (vv - vl)) < 1e-11 * max(1.0, ps * (vv - vl))


def test_maxwell_brute_force_scan():
    # Brute force: scan the vapour branch finely, for each p find the liquid root, and
    # locate the sign change of the chemical-potential difference.
    T = 0.85
    sv, sl = oracle.spinodal(T)
    rvs = np.linspace(0.05, sv - 1e-6, 4001)
    f = []
    for r in rvs:
        p = oracle.pressure(r, T)
        rl = optimize.brentq(lambda x: oracle.pressure(x, T) - p, sl, 3.0 - 1e-12, xtol=1e-15)
        f.append(oracle.chempot(rl, T) - oracle.chempot(r, T))
    f = np.array(f)
    k = np.where(np.sign(f[:-1]) != np.sign(f[1:]))[0][0]
    rv_bf = optimize.brentq(lambda r: oracle.chempot(
        optimize.brentq(lambda x: oracle.pressure(x, T) - oracle.pressure(r, T), sl, 3.0 - 1e-12, xtol=1e-15), T)
        - oracle.chempot(r, T), rvs[k], rvs[k + 1], xtol=1e-15)
    rv, rl, _ = oracle.maxwell(T)
    assert abs(rv - rv_bf) < 1e-12


def test_sigma_and_interface_width_table1():
    g = GOLD["table1_fluid_properties"]
    sig = oracle.sigma(g["T"], g["gamma_K"])
    rv, rl, _ = oracle.maxwell(g["T"])
    Li = math.sqrt(2.0) * g["gamma_K"] * (rl - rv) ** 2 / sig
    assert round(sig, 4) == g["sigma_vl"]
    assert round(Li, 4) == g["L_i"]


def test_sigma_and_interface_width_table5():
    g = GOLD["table5_droplet_collision"]
    sig = oracle.sigma(g["T0"], g["gamma_K"])
    rv, rl, _ = oracle.maxwell(g["T0"])
    Li = math.sqrt(2.0) * g["gamma_K"] * (rl - rv) ** 2 / sig
    assert round(sig, 4) == g["sigma_vl"]
    assert round(Li, 4) == g["L_i"]


def test_sigma_quadrature_converged_and_matches_scipy():
    # The quadrature is converged (panel doubling) and agrees with SciPy's adaptive rule
    # applied to the integral of eq. surftenscoef written from psi directly.
    T, gam = 0.85, 1e-4
    s64, s128 = oracle.sigma(T, gam, panels=64), oracle.sigma(T, gam, panels=128)
    assert abs(s64 - s128) < 1e-15
    rv, rl, _ = oracle.maxwell(T)
    mu_v = d1(lambda r: psi(r, T), rv, 1e-6)

    def integrand(r):
        return math.sqrt(max(psi(r, T) - (psi(rv, T) + (r - rv) * mu_v), 0.0))

    I, _ = integrate.quad(integrand, rv, rl, epsabs=1e-13, epsrel=1e-12, limit=200)
    assert abs(s64 - math.sqrt(2 * gam) * I) < 1e-9
    # the 15-point rule the paper uses for its table agrees to about 1e-12 here
    assert abs(oracle.sigma_gauss15(T, gam) - s64) < 1e-10


def test_sigma_printed_prefactor_is_garbled():
    # Reading: the printed prefactor sqrt(2/gamma) would give sigma ~ 52, far from Table 1.
    s = oracle.sigma(0.85, 1e-4)
    assert abs(s / math.sqrt(2e-4) * math.sqrt(2 / 1e-4) - 52.3) < 0.1


def test_young_laplace_densities_table5():
    # Sec. 4.3: p_v = p_sat + rho_v/(rho_l-rho_v) 2 sigma/r, p_l = p_sat + rho_l/(rho_l-rho_v) 2 sigma/r,
    # densities from the inverse pressure law at T0.
    g = GOLD["table5_droplet_collision"]
    T = g["T0"]
    rv, rl, ps = oracle.maxwell(T)
    sig = oracle.sigma(T, g["gamma_K"])
    pv = ps + rv / (rl - rv) * 2 * sig / g["r_d"]
    pl = ps + rl / (rl - rv) * 2 * sig / g["r_d"]
    assert round(oracle.rho_of_p(T, pv, 0), 4) == g["rho_v"]
    assert round(oracle.rho_of_p(T, pl, 1), 4) == g["rho_l"]


@pytest.mark.parametrize("theta", [30.0, 60.0, 90.0, 120.0, 150.0])
def test_wall_energy_properties(theta):
    # Sec. 2.4: psi_Gamma(rho_v) = sigma_sv, psi_Gamma(rho_l) = sigma_sl, zero derivative at
    # both Maxwell states; Young's relation sigma_sv - sigma_sl = sigma cos(theta); the
    # printed derivative (eq. helmfreesurftot_derivative) is the derivative of the cubic.
    rv, rl, _ = oracle.maxwell(0.85)
    sig = oracle.sigma(0.85)
    ct = math.cos(math.radians(theta))
    ssl = 0.3
    ssv = ssl + sig * ct
    assert abs(oracle.psiwall(rv, rv, rl, ssv, ssl) - ssv) < 1e-15
    assert abs(oracle.psiwall(rl, rv, rl, ssv, ssl) - ssl) < 1e-15
    assert oracle.dpsiwall_dc(rv, rv, rl, sig, ct) == 0.0
    assert oracle.dpsiwall_dc(rl, rv, rl, sig, ct) == 0.0
    for c in (0.5, 1.0, 1.5):
        num = d1(lambda x: oracle.psiwall(x, rv, rl, ssv, ssl), c, 1e-6)
        assert abs(oracle.dpsiwall_dc(c, rv, rl, sig, ct) - num) < 1e-9
    if theta == 90.0:
        assert abs(oracle.dpsiwall_dc(1.0, rv, rl, sig, ct)) < 1e-17


def test_appendix_states_consistent_with_porous_setup():
    # Consistency with the porous-medium set-up (Sec. 4.5): rho = 1.5 lies outside the
    # saturation dome at T = 0.95 and inside the spinodal at T = 0.75.
    rv, rl, _ = oracle.maxwell(0.95)
    assert 1.5 > rl
    sv, sl = oracle.spinodal(0.75)
    assert sv < 1.5 < sl

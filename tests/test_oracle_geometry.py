"""Pins of the oracle's curved-element geometry (Sec. 3.1: elements mapped
from the reference cube, geometry of degree N_geo <= N given on
Gauss-Lobatto points; metric terms in the conservative curl form).

  * the node coordinates are the values of the degree-N_geo interpolant of
    the box map at the Gauss nodes (checked with numpy's own polynomial
    routines, independent of the oracle's Lobatto and Lagrange code);
  * the curl-form metrics equal the exact cofactors of the interpolated
    geometry when the degree-N interpolation in the curl form is exact,
    i.e. N >= 2 N_geo (X_l grad X_m then has degree <= 2 N_geo per
    direction): trilinear elements (N_geo = 1) from N = 2 and quadratic
    ones (N_geo = 2) from N = 4, to round-off;
  * free-stream preservation and discrete conservation on quadratic
    elements, periodic and between walls.
"""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle


def make(N, n, amp, ngeo, length=(1.0, 1.0, 1.0), periodic=(1, 1, 1), kinds=(0,) * 6, tw=(0.0,) * 6, **pk):
    p = oracle.make_params(**pk)
    b = oracle.make_box(N, n, (0.0, 0.0, 0.0), length, periodic, kinds, tw, (90.0,) * 6, amp, ngeo=ngeo)
    return oracle.Oracle(p, b)


def box_map(X, amp, length):
    s = np.prod([np.sin(2 * np.pi * X[d] / length[d]) for d in range(3)], axis=0)
    return np.stack([X[d] + amp * s for d in range(3)])


def lobatto(n):
    """Gauss-Lobatto points of degree n: -1, the roots of P_n', +1."""
    inner = npleg.legroots(npleg.legder(np.eye(n + 1)[n])) if n > 1 else np.array([])
    return np.concatenate([[-1.0], np.sort(inner), [1.0]])


def lagrange_matrix(xs, xe):
    """L[a, b] = l_b(xe[a]) for the nodes xs."""
    L = np.ones((len(xe), len(xs)))
    for b in range(len(xs)):
        for k in range(len(xs)):
            if k != b:
                L[:, b] *= (xe - xs[k]) / (xs[b] - xs[k])
    return L


@pytest.mark.parametrize("N,ngeo", [(3, 2), (4, 2), (3, 1)])
def test_node_coordinates_are_the_geometry_interpolant(N, ngeo):
    n, length, amp = (3, 2, 2), (1.0, 0.8, 1.2), 0.05
    o = make(N, n, amp, ngeo, length)
    P = N + 1
    xg, _ = npleg.leggauss(P)
    xl = lobatto(ngeo)
    V = lagrange_matrix(xl, xg)
    got = o.coords().reshape(3, n[2], n[1], n[0], P, P, P)
    h = [length[d] / n[d] for d in range(3)]
    for ez in range(n[2]):
        for ey in range(n[1]):
            for ex in range(n[0]):
                ee = (ex, ey, ez)
                # map at the Lobatto points of the element, axes (c3, c2, c1)
                g = np.meshgrid(*[h[d] * (ee[d] + 0.5 * (xl + 1.0)) for d in (2, 1, 0)], indexing="ij")
                Xm = box_map([g[2], g[1], g[0]], amp, length)
                want = np.einsum("kc,jb,ia,mcba->mkji", V, V, V, Xm)
                assert np.max(np.abs(got[:, ez, ey, ex] - want)) < 1e-14


def _cofactor_error(N, amp, ngeo):
    o = make(N, (3, 3, 3), amp, ngeo)
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


@pytest.mark.parametrize("N,ngeo", [(2, 1), (3, 1), (4, 2), (5, 2)])
def test_curl_form_metrics_are_exact_cofactors_when_n_covers_twice_the_geometry_degree(N, ngeo):
    # Ja^d_m = J d xi^d / d x_m, so sum_m Ja^d_m d x_m / d xi^e = J delta_de with
    # the derivative of the (polynomial) node coordinates taken by the pinned
    # derivative matrix
    assert _cofactor_error(N, 0.08, ngeo) <= 1e-13


def test_curl_form_metrics_of_a_quadratic_geometry_at_n3_carry_interpolation_error_only():
    # N = 3 < 2 N_geo: the curl form is not the exact cofactor, but close
    e = _cofactor_error(3, 0.08, 2)
    assert 1e-6 < e < 0.05


STATE = dict(rho=1.2, u=(0.3, -0.2, 0.1), T=0.9)


def conserved(o, rho, u, T, c):
    pr = o.params
    U = np.zeros((6, o.nnodes))
    U[0], U[1:4], U[5] = rho, rho * u, c
    q = o.lift1(U)
    g2 = q[12] ** 2 + q[13] ** 2 + q[14] ** 2
    U[4] = (rho * (pr.R * pr.cv * T - pr.a * rho) + 0.5 * rho * np.sum(u * u, axis=0)
            + 0.5 * pr.alpha * (rho - c) ** 2 + 0.5 * pr.gam * g2)
    return U


@pytest.mark.parametrize("N", [3, 4])
def test_free_stream_on_quadratic_elements(N):
    o = make(N, (3, 3, 3), 0.06, 2)
    rho = np.full(o.nnodes, STATE["rho"])
    u = np.tile(np.array(STATE["u"])[:, None], (1, o.nnodes))
    U = conserved(o, rho, u, STATE["T"], rho.copy())
    assert np.max(np.abs(o.rhs(U))) < 5e-12


def test_free_stream_at_rest_between_walls_on_quadratic_elements():
    o = make(3, (3, 3, 2), 0.05, 2, (1.0, 1.0, 0.5), (1, 1, 0), (0, 0, 0, 0, 1, 2), (0, 0, 0, 0, 0.9, 0))
    rho = np.full(o.nnodes, 1.2)
    U = conserved(o, rho, np.zeros((3, o.nnodes)), 0.9, rho.copy())
    assert np.max(np.abs(o.rhs(U))) < 5e-12


def test_mass_conservation_on_quadratic_elements():
    o = make(3, (3, 3, 2), 0.05, 2, (1.0, 1.0, 0.5), (1, 1, 0), (0, 0, 0, 0, 1, 2), (0, 0, 0, 0, 0.9, 0))
    x, y, z = o.coords()
    rng = np.random.default_rng(7)
    U = o.init_droplets(0.85, [(0.5, 0.5, 0.1)], [0.2], 0.05, rng.uniform(-1e-3, 1e-3, o.nnodes))
    u = np.stack([0.05 * np.sin(2 * np.pi * y), 0.04 * np.cos(2 * np.pi * x), 0.03 * z * (0.5 - z)])
    U[1:4] = U[0] * u
    U[4] += 0.5 * U[0] * np.sum(u * u, axis=0)
    _, w, *_ = oracle.basis(3)
    w3 = (w[None, None, :] * w[None, :, None] * w[:, None, None]).reshape(-1)
    _, J, _ = o.metrics()
    W = np.tile(w3, o.nelems) * J
    rate = np.sum(W * o.rhs(U)[0])
    assert abs(rate) <= 1e-13 * np.sum(W * U[0])

"""Pins of the oracle's 1D DGSEM ingredients and of the Runge-Kutta scheme."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7])
def test_gauss_nodes_match_library(N):
    x, w, *_ = oracle.basis(N)
    xr, wr = npleg.leggauss(N + 1)
    assert np.max(np.abs(x - xr)) < 1e-15 and np.max(np.abs(w - wr)) < 1e-14
    assert abs(w.sum() - 2.0) < 1e-14


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_lobatto_nodes_are_roots_of_dPN(N):
    x = oracle.lobatto(N)
    assert x[0] == -1.0 and x[-1] == 1.0
    dP = npleg.legder(np.eye(N + 1)[N])
    assert np.max(np.abs(npleg.legval(x[1:-1], dP))) < 1e-12


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_derivative_matrix_exact_on_polynomials(N):
    # D . x^k = k x^(k-1) for k <= N (Sec. 3.1, nodal Lagrange basis).
    x, w, D, Dh, lm, lp = oracle.basis(N)
    for k in range(N + 1):
        exact = k * x ** (k - 1) if k > 0 else np.zeros_like(x)
        assert np.max(np.abs(D @ x ** k - exact)) < 1e-12


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_weak_derivative_summation_by_parts(N):
    # Weak-form operator with surface terms reproduces the derivative of degree-N
    # polynomials: Dhat x^k + lhat+ (1)^k - lhat- (-1)^k = k x^(k-1).
    x, w, D, Dh, lm, lp = oracle.basis(N)
    for k in range(N + 1):
        lhs = Dh @ x ** k + lp / w * 1.0 - lm / w * (-1.0) ** k
        exact = k * x ** (k - 1) if k > 0 else np.zeros_like(x)
        assert np.max(np.abs(lhs - exact)) < 1e-12


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_face_interpolation(N):
    x, w, D, Dh, lm, lp = oracle.basis(N)
    for k in range(N + 1):
        assert abs(lm @ x ** k - (-1.0) ** k) < 1e-13 and abs(lp @ x ** k - 1.0) < 1e-13


def butcher_from_2n(A, B):
    """Butcher tableau of a 2N-storage scheme R <- A_s R + dt f, U <- U + B_s R."""
    s = len(A)
    # U_stage_i = U0 + sum_j a_ij dt f_j ; the register after stage j is
    # R_j = dt f_j + A_j R_{j-1}; U_i = U0 + sum_{k<i} B_k R_k.
    coef = np.zeros((s, s))  # R_j in terms of dt f_m
    for j in range(s):
        if j > 0:
            coef[j] = A[j] * coef[j - 1]
        coef[j, j] += 1.0
    a = np.zeros((s, s))
    for i in range(1, s):
        for k in range(i):
            a[i] += B[k] * coef[k]
    b = np.zeros(s)
    for k in range(s):
        b += B[k] * coef[k]
    return a, b


def test_rk_order_conditions():
    A, B, C = oracle.rk_coeffs()
    a, b = butcher_from_2n(A, B)
    c = a.sum(axis=1)
    assert np.max(np.abs(c - C)) < 1e-15
    conds = [
        (b.sum(), 1.0),
        (b @ c, 1 / 2),
        (b @ c ** 2, 1 / 3),
        (b @ (a @ c), 1 / 6),
        (b @ c ** 3, 1 / 4),
        (b @ (c * (a @ c)), 1 / 8),
        (b @ (a @ c ** 2), 1 / 12),
        (b @ (a @ (a @ c)), 1 / 24),
    ]
    for got, want in conds:
        assert abs(got - want) < 1e-15


def test_rk_stability_polynomial():
    A, B, C = oracle.rk_coeffs()
    a, b = butcher_from_2n(A, B)
    # P(z) = 1 + z b^T (I - z a)^-1 1 ; fifth coefficient b^T a^4 1
    e = np.ones(5)
    c5 = b @ np.linalg.matrix_power(a, 4) @ e
    assert abs(c5 - 0.005) < 1e-4
    # the real-axis stability interval used by the time-step rule
    z = -4.6567
    P = sum(b @ np.linalg.matrix_power(a, k - 1) @ e * z ** k for k in range(1, 6)) + 1.0
    assert abs(abs(P) - 1.0) < 1e-3

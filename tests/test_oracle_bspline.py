"""Pins of the oracle's univariate B-splines and Gauss rules (Section 2.1)
against closed forms, invariants and textbook values."""
import json
import os

import numpy as np
import pytest

from oracle import bspline

HERE = os.path.dirname(__file__)

CASES = [(1, 0, 5), (2, 1, 4), (3, 2, 6), (4, 3, 3), (3, 1, 4), (5, 4, 2), (2, 0, 3)]


@pytest.mark.parametrize("p,reg,n_el", CASES)
def test_partition_of_unity_and_nonnegative(p, reg, n_el):
    t = bspline.open_uniform_knots(n_el, p, reg)
    x = np.linspace(0, 1, 401)
    v = bspline.basis(t, p, x)
    assert v.shape == (len(x), n_el * (p - reg) + reg + 1)
    assert np.all(v >= -1e-15)
    assert np.allclose(v.sum(axis=1), 1.0, atol=1e-14)


@pytest.mark.parametrize("p,reg,n_el", CASES)
def test_endpoint_interpolation(p, reg, n_el):
    # first and last functions are nodal at the end points (Section 2.1)
    t = bspline.open_uniform_knots(n_el, p, reg)
    v = bspline.basis(t, p, [0.0, 1.0])
    assert v[0, 0] == pytest.approx(1.0)
    assert v[1, -1] == pytest.approx(1.0)
    assert np.allclose(v[0, 1:], 0) and np.allclose(v[1, :-1], 0)


def test_p1_hat_functions():
    n_el = 4
    t = bspline.open_uniform_knots(n_el, 1, 0)
    x = np.linspace(0, 1, 101)
    v = bspline.basis(t, 1, x)
    for i in range(n_el + 1):
        hat = np.maximum(0.0, 1.0 - np.abs(x * n_el - i))
        assert np.allclose(v[:, i], hat, atol=1e-14)


def test_quadratic_closed_form_two_elements():
    # knots [0,0,0,1/2,1,1,1]; closed forms by hand from the recursion
    t = bspline.open_uniform_knots(2, 2, 1)
    x = np.linspace(0, 1, 257)
    v = bspline.basis(t, 2, x)
    L = x <= 0.5
    b0 = np.where(L, (1 - 2 * x) ** 2, 0.0)
    b3 = np.where(L, 0.0, (2 * x - 1) ** 2)
    b1 = np.where(L, 2 * x * (2 - 3 * x), 2 * (1 - x) ** 2)
    b2 = np.where(L, 2 * x ** 2, -2 + 8 * x - 6 * x ** 2)
    for i, b in enumerate([b0, b1, b2, b3]):
        assert np.allclose(v[:, i], b, atol=1e-14), i


@pytest.mark.parametrize("p,reg,n_el", CASES)
def test_greville_linear_precision(p, reg, n_el):
    t = bspline.open_uniform_knots(n_el, p, reg)
    g = bspline.greville(t, p)
    x = np.random.default_rng(0).uniform(0, 1, 200)
    assert np.allclose(bspline.basis(t, p, x) @ g, x, atol=1e-14)


@pytest.mark.parametrize("p,reg,n_el", CASES)
def test_derivative_central_difference(p, reg, n_el):
    t = bspline.open_uniform_knots(n_el, p, reg)
    x = np.random.default_rng(1).uniform(0.01, 0.99, 50)
    # stay away from breakpoints where lower-continuity derivatives jump
    x = x[np.min(np.abs(x[:, None] - np.unique(t)[None, :]), axis=1) > 1e-3]
    h = 1e-6
    _, d = bspline.basis(t, p, x, deriv=True)
    fd = (bspline.basis(t, p, x + h) - bspline.basis(t, p, x - h)) / (2 * h)
    assert np.allclose(d, fd, atol=1e-6 * max(1, n_el * p))


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6])
def test_gauss_exact_on_monomials(n):
    x, w = bspline.gauss_legendre(n)
    for k in range(2 * n):
        assert np.sum(w * x ** k) == pytest.approx(1.0 / (k + 1), rel=1e-13)
    # and not exact one degree higher (n points: degree 2n-1 is the limit)
    assert abs(np.sum(w * x ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-8


@pytest.mark.parametrize("p,reg,n_el", CASES)
def test_mass_row_sums_textbook(p, reg, n_el):
    # int b_i = (xi_{i+p+1} - xi_i) / (p+1)
    t = bspline.open_uniform_knots(n_el, p, reg)
    K, M = bspline.matrices_1d(t, p)
    m = M.shape[0]
    ints = np.array([(t[i + p + 1] - t[i]) / (p + 1) for i in range(m)])
    assert np.allclose(M.sum(axis=1), ints, atol=1e-14)
    assert M.sum() == pytest.approx(1.0, abs=1e-13)
    # the univariate stiffness is singular with the constants in its kernel
    assert np.allclose(K @ np.ones(m), 0, atol=1e-11 * np.abs(K).max())
    assert np.allclose(K, K.T) and np.allclose(M, M.T)


def test_bernstein_golden():
    g = json.load(open(os.path.join(HERE, "golden", "bernstein_p2.json")))
    K, M = bspline.matrices_1d(np.array(g["knots"], float), g["p"])
    assert np.allclose(M, g["M"], atol=1e-15)
    assert np.allclose(K, g["K"], atol=1e-14)


def test_matrices_match_higher_order_rule():
    p, n_el = 3, 5
    t = bspline.open_uniform_knots(n_el, p, 2)
    K, M = bspline.matrices_1d(t, p)
    x, w, _ = bspline.quadrature(t, p + 4)
    v, d = bspline.basis(t, p, x, deriv=True)
    assert np.allclose(M, v.T @ (w[:, None] * v), atol=1e-15)
    assert np.allclose(K, d.T @ (w[:, None] * d), atol=1e-12)

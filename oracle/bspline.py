"""Univariate B-splines (paper Section 2.1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Pins (tests/test_oracle_bspline.py): partition of unity, non-negativity,
endpoint interpolation, p=1 hat functions, Greville linear reproduction,
derivatives against central differences, Gauss exactness on monomials and
agreement with the textbook integral of a B-spline.
"""
from __future__ import annotations

import numpy as np


def open_uniform_knots(n_el: int, p: int, reg: int) -> np.ndarray:
    """Open knot vector on [0, 1] with ``n_el`` equal elements (Section 2.1):
    the first and last knot repeated p+1 times; each interior breakpoint
    repeated p - reg times, giving C^reg continuity across it."""
    if not (0 <= reg < p or (p == 0 and reg == -1)):
        raise ValueError("continuity must satisfy 0 <= reg < p")
    inner = []
    for e in range(1, n_el):
        inner += [e / n_el] * (p - reg)
    return np.array([0.0] * (p + 1) + inner + [1.0] * (p + 1))


def n_functions(knots: np.ndarray, p: int) -> int:
    """m = len(Xi) - p - 1 (Section 2.1: the knot vector has m+p+1 entries)."""
    return len(knots) - p - 1


def basis(knots: np.ndarray, p: int, x, deriv: bool = False):
    """Values (and first derivatives) of all m B-splines at points ``x``.

    Cox-de Boor recursion exactly as in Section 2.1: degree 0 indicators of
    half-open spans, then the two-term recursion with 0/0 = 0.

    Reading of an edge case: the degree-0 rule is half open, so at x = 1 every
    indicator would vanish; the last non-empty span is taken closed on the
    right so that b_m(1) = 1 as the paper states right after the recursion.

    Returns array (len(x), m) or a pair (values, derivatives).
    """
    x = np.atleast_1d(np.asarray(x, dtype=float))
    t = np.asarray(knots, dtype=float)
    m_all = len(t) - 1  # number of degree-0 functions
    # degree 0
    b = np.zeros((len(x), m_all))
    last_nonempty = max(i for i in range(m_all) if t[i + 1] > t[i])
    for i in range(m_all):
        if t[i + 1] > t[i]:
            inside = (x >= t[i]) & (x < t[i + 1])
            if i == last_nonempty:
                inside |= (x == t[i + 1])
            b[:, i] = inside
    prev = b
    for q in range(1, p + 1):
        m_q = m_all - q
        cur = np.zeros((len(x), m_q))
        for i in range(m_q):
            den1 = t[i + q] - t[i]
            den2 = t[i + q + 1] - t[i + 1]
            term1 = (x - t[i]) / den1 * prev[:, i] if den1 != 0 else 0.0
            term2 = (t[i + q + 1] - x) / den2 * prev[:, i + 1] if den2 != 0 else 0.0
            cur[:, i] = term1 + term2
        if q == p and deriv:
            # d/dx b_{i,p} = p/(t_{i+p}-t_i) b_{i,p-1} - p/(t_{i+p+1}-t_{i+1}) b_{i+1,p-1}
            d = np.zeros_like(cur)
            for i in range(m_q):
                den1 = t[i + q] - t[i]
                den2 = t[i + q + 1] - t[i + 1]
                a1 = q / den1 * prev[:, i] if den1 != 0 else 0.0
                a2 = q / den2 * prev[:, i + 1] if den2 != 0 else 0.0
                d[:, i] = a1 - a2
            return cur, d
        prev = cur
    if deriv:  # p == 0
        return prev, np.zeros_like(prev)
    return prev


def greville(knots: np.ndarray, p: int) -> np.ndarray:
    """Greville abscissae g_i = (xi_{i+1} + ... + xi_{i+p}) / p.  With them,
    sum_i g_i b_i(x) = x (linear precision), which places control points of
    a multilinear map."""
    m = n_functions(knots, p)
    if p == 0:
        return np.array([(knots[i] + knots[i + 1]) / 2 for i in range(m)])
    return np.array([np.mean(knots[i + 1:i + p + 1]) for i in range(m)])


def gauss_legendre(n_pts: int):
    """Gauss-Legendre points and weights on [0, 1] (numpy's leggauss, mapped)."""
    x, w = np.polynomial.legendre.leggauss(n_pts)
    return 0.5 * (x + 1.0), 0.5 * w


def quadrature(knots: np.ndarray, n_pts: int):
    """Composite Gauss rule: ``n_pts`` points on every non-empty knot span.

    The paper does not fix the rule; this oracle (and the GPU path) use
    p + 1 points per span per direction.  Returns (points, weights, span id).
    """
    x0, w0 = gauss_legendre(n_pts)
    brk = np.unique(knots)
    xs, ws, el = [], [], []
    for e in range(len(brk) - 1):
        a, b = brk[e], brk[e + 1]
        xs.append(a + (b - a) * x0)
        ws.append((b - a) * w0)
        el.append(np.full(n_pts, e))
    return np.concatenate(xs), np.concatenate(ws), np.concatenate(el)


def matrices_1d(knots: np.ndarray, p: int):
    """Univariate stiffness and mass on [0, 1] (Section 5.2):
    K[i,j] = int b_i' b_j',  M[i,j] = int b_i b_j, by the composite Gauss rule
    with p+1 points per span (exact: the integrands have degree <= 2p)."""
    x, w, _ = quadrature(knots, p + 1)
    v, d = basis(knots, p, x, deriv=True)
    K = d.T @ (w[:, None] * d)
    M = v.T @ (w[:, None] * v)
    return K, M

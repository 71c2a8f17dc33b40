"""Pins of the least-squares initial guess in oracle/projection.py against
closed forms and the defining optimality conditions:
  * a history that is a polynomial in time of degree < k reproduces the next
    value exactly, with the Lagrange extrapolation weights of equispaced
    nodes, c_i = (-1)^i C(k, i+1), applied to the solutions as well;
  * the residual is orthogonal to every history column, and no perturbation
    of the coefficients lowers it;
  * it is never above the residual of any polynomial extrapolation built
    from the same history;
  * a repeated column changes neither the rank-deficient minimum nor the guess.
"""
import math

import numpy as np
import pytest

from oracle import projection as pj


def taylor_history(rng, k, n, t_new=1.0):
    """Values at t = 0, -1, ..., -(k-1) (newest first) and at t_new of a
    vector polynomial of degree k-1 with Taylor-scaled coefficients."""
    v = rng.standard_normal((k, n))
    vals = lambda t: sum(t ** m / math.factorial(m) * v[m] for m in range(k))  # noqa: E731
    return [vals(-float(i)) for i in range(k)], vals(t_new)


@pytest.mark.parametrize("k", range(1, 9))
def test_polynomial_history_gives_lagrange_extrapolation(k):
    rng = np.random.default_rng(100 + k)
    ys, b = taylor_history(rng, k, 400)
    xs, x_new = taylor_history(rng, k, 400)
    x, c, rank = pj.lsq_guess(b, xs, ys)
    assert rank == k
    lagrange = np.array([(-1) ** i * math.comb(k, i + 1) for i in range(k)], dtype=float)
    np.testing.assert_allclose(c, lagrange, rtol=1e-7, atol=1e-7)
    assert pj.proxy_residual(b, ys, c) <= 1e-9 * np.linalg.norm(b)
    np.testing.assert_allclose(x, x_new, rtol=1e-7, atol=1e-7 * np.abs(x_new).max())


def test_residual_orthogonal_to_history_and_minimal():
    rng = np.random.default_rng(7)
    k, n = 5, 300
    ys = [rng.standard_normal(n) for _ in range(k)]
    b = rng.standard_normal(n)
    c, rank = pj.lsq_coefficients(b, ys)
    assert rank == k
    r = b - sum(ci * y for ci, y in zip(c, ys))
    for y in ys:
        assert abs(r @ y) <= 1e-12 * np.linalg.norm(r) * np.linalg.norm(y)
    best = pj.proxy_residual(b, ys, c)
    for _ in range(200):
        d = 1e-3 * rng.standard_normal(k)
        assert pj.proxy_residual(b, ys, c + d) > best


def test_never_worse_than_extrapolation():
    # a smooth history plus a rough part: every fixed-order extrapolation is
    # one coefficient vector among those the least squares ranges over
    rng = np.random.default_rng(11)
    k, n = 6, 500
    ys, b = taylor_history(rng, k, n)
    ys = [y + 1e-3 * rng.standard_normal(n) for y in ys]
    b = b + 1e-3 * rng.standard_normal(n)
    c, _ = pj.lsq_coefficients(b, ys)
    best = pj.proxy_residual(b, ys, c)
    for order in range(k):
        w = np.zeros(k)
        w[:order + 1] = [(-1) ** i * math.comb(order + 1, i + 1) for i in range(order + 1)]
        assert best <= pj.proxy_residual(b, ys, w) * (1 + 1e-12)


def test_repeated_column():
    rng = np.random.default_rng(3)
    n = 200
    y0, y1 = rng.standard_normal(n), rng.standard_normal(n)
    x0, x1 = rng.standard_normal(n), rng.standard_normal(n)
    b = rng.standard_normal(n)
    x2, c2, r2 = pj.lsq_guess(b, [x0, x1], [y0, y1])
    x3, c3, r3 = pj.lsq_guess(b, [x0, x1, x0], [y0, y1, y0])
    assert (r2, r3) == (2, 2)
    assert pj.proxy_residual(b, [y0, y1, y0], c3) == pytest.approx(pj.proxy_residual(b, [y0, y1], c2), rel=1e-12)
    np.testing.assert_allclose(x3, x2, rtol=1e-10, atol=1e-12)

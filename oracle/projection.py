"""Least-squares initial guess of the pressure solve from earlier solutions.

TEST INFRASTRUCTURE ONLY: the tests are the only callers; the product path
never imports this module.

Not part of the paper, which starts each pressure solve from the previous
pressure (Sec. 3.4).  Given earlier solutions x_1..x_k of L x_i = y_i (the
right-hand sides of the steps that produced them) and a new right-hand side
b, the guess is x = sum_i c_i x_i with c the minimiser of ||b - sum_i c_i
y_i||_2.  When every x_i solves its equation exactly, L x = sum_i c_i y_i, so
x is the element of span{x_i} whose residual for b is smallest.

Written from that definition in plain numpy (FP64): the minimiser comes from
numpy's SVD-based least-squares routine; columns that are numerically
dependent are handled by its rank cut-off.
"""
import numpy as np


def lsq_coefficients(b, ys, rcond=None):
    """c minimising ||b - sum_i c_i ys[i]||_2 (the minimum-norm one if the ys are dependent)."""
    Y = np.stack([np.asarray(y, dtype=np.float64).ravel() for y in ys], axis=1)
    c, _, rank, _ = np.linalg.lstsq(Y, np.asarray(b, dtype=np.float64).ravel(), rcond=rcond)
    return c, int(rank)


def lsq_guess(b, xs, ys, rcond=None):
    """(x, c, rank): x = sum_i c_i xs[i] with the least-squares c of lsq_coefficients."""
    c, rank = lsq_coefficients(b, ys, rcond)
    x = np.zeros_like(np.asarray(xs[0], dtype=np.float64))
    for ci, xi in zip(c, xs):
        x += ci * np.asarray(xi, dtype=np.float64)
    return x, c, rank


def proxy_residual(b, ys, c):
    """||b - sum_i c_i ys[i]||_2: the residual of the guess if every x_i were exact."""
    r = np.asarray(b, dtype=np.float64).ravel().copy()
    for ci, y in zip(c, ys):
        r -= ci * np.asarray(y, dtype=np.float64).ravel()
    return float(np.linalg.norm(r))

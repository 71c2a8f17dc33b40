"""SRJ relaxation schedule for the oracle (test infrastructure only).

The paper (Sec. 3.4) runs Jacobi-SOR with a cycle of M sweeps whose weights
omega_k (each repeated q_k times) over-relax the smooth error and
under-relax the rough error; it takes the weights and their order from the
SRJ authors' script and prints none of them.  This module states the reading
used here, written from the mathematics:

* The sweep p <- p + (omega/D)(L p - b) multiplies the error component along
  an eigenvector of -L with eigenvalue lambda by (1 - omega kappa), where
  kappa = lambda / D.  One cycle multiplies it by prod_k (1 - omega_k kappa).
* kappa ranges over the exact discrete spectrum of the grid: Fourier modes in
  x and y, cosine modes in z (zero normal gradient), so
  lambda = 4/dx^2 sin^2(pi m/nx) + 4/dy^2 sin^2(pi n/ny)
         + 4/dz^2 sin^2(pi l/(2 nz)).
* The cycle polynomial of least maximum on [kappa_min, kappa_max] is the
  shifted Chebyshev polynomial, whose roots are the Chebyshev nodes x_k; so
  omega_k = 1/x_k, each used once (the many-level limit of SRJ).  M is the
  smallest degree whose worst-case reduction 1/T_M((b+a)/(b-a)) is at most
  the requested factor.
* Sweep order: Leja order of the nodes (start from the node of largest
  magnitude, then repeatedly take the node that maximises the product of
  distances to those already taken), which keeps the intermediate
  amplification of a Richardson cycle moderate.  The nodes are symmetric, so
  exact ties occur: values within a relative 1e-9 of the best log-product
  count as tied and the lower index wins.
"""
import math

import numpy as np


def kappa_bounds(nx, ny, nz, lx, ly, lz):
    """(kappa_min, kappa_max) over the non-constant modes of L_p / D."""
    dx, dy, dz = lx / nx, ly / ny, lz / nz
    d = 2.0 / dx**2 + 2.0 / dy**2 + 2.0 / dz**2
    lam_x = [4.0 / dx**2 * math.sin(math.pi * m / nx) ** 2 for m in range(nx)]
    lam_y = [4.0 / dy**2 * math.sin(math.pi * m / ny) ** 2 for m in range(ny)]
    lam_z = [4.0 / dz**2 * math.sin(math.pi * m / (2 * nz)) ** 2 for m in range(nz)]
    nonzero = [v for v in lam_x + lam_y + lam_z if v > 0.0]
    lam_min = min(nonzero) if nonzero else 0.0
    lam_max = max(lam_x) + max(lam_y) + max(lam_z)
    return lam_min / d, lam_max / d


def chebyshev_degree(a, b, reduction):
    s = (b + a) / (b - a)
    return max(1, int(math.ceil(math.acosh(1.0 / reduction) / math.acosh(s))))


def chebyshev_nodes(a, b, m):
    k = np.arange(1, m + 1)
    return 0.5 * (a + b) + 0.5 * (b - a) * np.cos(np.pi * (2 * k - 1) / (2 * m))


def leja_order(x):
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    taken = np.zeros(n, dtype=bool)
    first = int(np.argmax(np.abs(x)))
    order = [first]
    taken[first] = True
    logdist = np.zeros(n)
    last = first
    for _ in range(n - 1):
        with np.errstate(divide="ignore"):
            logdist = logdist + np.log(np.abs(x - x[last]))
        cand = np.where(taken, -np.inf, logdist)
        top = cand.max()
        tol = 1e-9 * max(1.0, abs(top))
        last = int(np.flatnonzero(cand >= top - tol)[0])
        order.append(last)
        taken[last] = True
    return x[np.array(order)]


def srj_schedule(nx, ny, nz, lx, ly, lz, reduction=1e-3):
    """Ordered cycle of relaxation weights omega_1..omega_M."""
    a, b = kappa_bounds(nx, ny, nz, lx, ly, lz)
    m = chebyshev_degree(a, b, reduction)
    return 1.0 / leja_order(chebyshev_nodes(a, b, m))


def schedule_of_degree(a, b, m):
    return 1.0 / leja_order(chebyshev_nodes(a, b, m))


def adaptive_degree(a, b, rtol, bnorm, rnorm, floor):
    """Cycle degree for a pass that must reduce the residual from rnorm to
    rtol * bnorm: rho = max(rtol bnorm / rnorm, floor) capped at 1/2; the
    least degree with 1/T_M <= rho, rounded up to a multiple of 16.  (One
    cycle multiplies every residual mode by at most 1/T_M, so the 2-norm of the
    residual shrinks by at least that factor.)"""
    rho = min(0.5, max(floor, rtol * bnorm / rnorm))
    m = chebyshev_degree(a, b, rho)
    return (m + 15) // 16 * 16


def cycle_factor(omega, kappa):
    """prod_k (1 - omega_k kappa): one cycle's effect on a mode."""
    g = np.ones_like(np.asarray(kappa, dtype=np.float64))
    for w in omega:
        g = g * (1.0 - w * kappa)
    return g

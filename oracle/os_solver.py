"""Orr-Sommerfeld eigenvalue solver (test infrastructure only).

The paper validates its solver against the linear stability of plane
Poiseuille flow (Sec. 4.1): a normal mode Psi = exp(i alpha (x - c t)) psi(z)
of the perturbation streamfunction (du = dPsi/dz, dw = -dPsi/dx) obeys the
Orr-Sommerfeld equation

  i alpha (U - c)(D^2 - alpha^2) psi - i alpha U'' psi = (1/Re)(D^2 - alpha^2)^2 psi,

with psi = psi' = 0 at both walls; the mode grows like exp(lambda t),
lambda = -i alpha c.  Here the equation is discretised by Chebyshev
collocation on [z0, z1] (the clamped conditions imposed by writing
psi = (1 - xi^2) phi, xi in [-1, 1], so that the fourth-derivative matrix acts
on phi with phi(+-1) = 0) and solved as the generalised eigenproblem
A psi = c B psi with B = i alpha (D^2 - alpha^2) and
A = i alpha [U (D^2 - alpha^2) - U''] - (1/Re)(D^2 - alpha^2)^2.
"""
import numpy as np
import scipy.linalg
import scipy.optimize


def cheb(n):
    """Chebyshev points x_j = cos(pi j / n), j = 0..n, and the collocation
    differentiation matrix (the standard construction from the Lagrange
    interpolant, diagonal from the negative row sums)."""
    j = np.arange(n + 1)
    x = np.cos(np.pi * j / n)
    c = np.ones(n + 1)
    c[0] = c[n] = 2.0
    c = c * (-1.0) ** j
    X = np.tile(x, (n + 1, 1)).T
    dX = X - X.T
    D = np.outer(c, 1.0 / c) / (dX + np.eye(n + 1))
    D = D - np.diag(D.sum(axis=1))
    return D, x


def os_matrices(alpha, re, u, upp, z0=0.0, z1=1.0, n=80):
    """A, B on the interior collocation points; u(z), upp(z) = U''(z)."""
    D, x = cheb(n)
    s = 2.0 / (z1 - z0)                      # d/dz = s d/dxi
    z = z0 + (x + 1.0) / s
    D2 = D @ D
    D3 = D2 @ D
    D4 = D3 @ D
    S = np.diag(np.concatenate([[0.0], 1.0 / (1.0 - x[1:n] ** 2), [0.0]]))
    D4c = (np.diag(1.0 - x**2) @ D4 - 8.0 * np.diag(x) @ D3 - 12.0 * D2) @ S
    inner = slice(1, n)
    d2 = s**2 * D2[inner, inner]
    d4 = s**4 * D4c[inner, inner]
    eye = np.eye(n - 1)
    zi = z[inner]
    lap = d2 - alpha**2 * eye
    lap2 = d4 - 2.0 * alpha**2 * d2 + alpha**4 * eye
    U = np.diag(u(zi))
    Upp = np.diag(upp(zi))
    A = 1j * alpha * (U @ lap - Upp) - lap2 / re
    B = 1j * alpha * lap
    return A, B, z


def os_eigs(alpha, re, u, upp, z0=0.0, z1=1.0, n=80):
    """All finite eigenvalues c (sorted by decreasing growth rate alpha*Im c)
    and the matching eigenvectors psi on the full Chebyshev grid."""
    A, B, z = os_matrices(alpha, re, u, upp, z0, z1, n)
    c, V = scipy.linalg.eig(A, B)
    keep = np.isfinite(c)
    c, V = c[keep], V[:, keep]
    order = np.argsort(-c.imag)
    c, V = c[order], V[:, order]
    psi = np.zeros((n + 1, V.shape[1]), dtype=complex)
    psi[1:n] = V
    return c, psi, z


def least_stable(alpha, re, u, upp, z0=0.0, z1=1.0, n=80):
    """(lambda, c, psi(z) on the Chebyshev grid, z) of the least stable mode;
    lambda = -i alpha c is the temporal growth rate (real part) and
    frequency (imaginary part)."""
    c, psi, z = os_eigs(alpha, re, u, upp, z0, z1, n)
    return -1j * alpha * c[0], c[0], psi[:, 0], z


def poiseuille_paper(re):
    """Base state of the paper's scaling (Sec. 4.1): channel 0 <= z <= 1,
    U0 = Re z (1 - z)."""
    return (lambda z: re * z * (1.0 - z)), (lambda z: -2.0 * re + 0.0 * z)


def poiseuille_centreline(lz=2.0):
    """Laminar profile with centreline speed 1 on 0 <= z <= lz."""
    h = 0.5 * lz
    return (lambda z: 1.0 - ((z - h) / h) ** 2), (lambda z: -2.0 / h**2 + 0.0 * z)


def growth_rate_paper(alpha, re, n=80):
    u, upp = poiseuille_paper(re)
    lam, _, _, _ = least_stable(alpha, re, u, upp, 0.0, 1.0, n)
    return lam


def critical_reynolds_paper(n=80):
    """Minimum over alpha of the Reynolds number at which the least stable
    mode is neutral, in the paper's scaling (Re based on the friction
    velocity and the full height)."""
    def neutral_re(alpha):
        f = lambda re: growth_rate_paper(alpha, re, n).real
        return scipy.optimize.brentq(f, 150.0, 300.0, xtol=1e-10)
    res = scipy.optimize.minimize_scalar(neutral_re, bounds=(1.9, 2.2), method="bounded",
                                         options={"xatol": 1e-7})
    return res.fun, res.x


def eigenfunction(psi_cheb, z_cheb, z0, z1, zq):
    """Evaluate the collocation eigenfunction at points zq by its Chebyshev
    interpolant."""
    n = len(z_cheb) - 1
    xi = 2.0 * (np.asarray(zq) - z0) / (z1 - z0) - 1.0
    xc = 2.0 * (z_cheb - z0) / (z1 - z0) - 1.0
    coef_r = np.polynomial.chebyshev.chebfit(xc, psi_cheb.real, n)
    coef_i = np.polynomial.chebyshev.chebfit(xc, psi_cheb.imag, n)
    return (np.polynomial.chebyshev.chebval(xi, coef_r) + 1j * np.polynomial.chebyshev.chebval(xi, coef_i))

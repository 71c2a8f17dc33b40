"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Only input generation lives here (random fields, initial conditions); none of
the method's arithmetic.  Arrays are numpy float64, C order, shape (nz, ny, nx)
(w: nz+1 planes, the wall planes zero).  Random numbers come from numpy's
PCG64 generator with the seed given.
"""
import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def poisson_rhs(nx, ny, nz, seed=1511):
    """Uniform(-1, 1) right-hand side with its mean removed."""
    b = rng(seed).uniform(-1.0, 1.0, size=(nz, ny, nx))
    return b - b.mean()


def laminar_profile(nz, lz, nu, dpdx):
    """Steady laminar profile on the u planes z_k = (k + 1/2) dz of the
    staggered grid with odd wall ghosts: the parabola |G| z (lz - z) / (2 nu)
    plus the uniform offset |G| dz^2 / (8 nu) that the ghost reflection adds
    (the second difference of a parabola is exact in the interior; the
    offset makes the wall rows exact too)."""
    dz = lz / nz
    z = (np.arange(nz) + 0.5) * dz
    g = abs(dpdx)
    return g * z * (lz - z) / (2.0 * nu) + g * dz * dz / (8.0 * nu)


def channel_state(nx, ny, nz, lz, nu, dpdx, noise=0.0, seed=7800, profile=True):
    """Laminar profile (optional) plus i.i.d. uniform noise of amplitude
    noise * U_cl on every u, v and interior w face (U_cl: centreline speed of
    the continuum parabola)."""
    u = np.zeros((nz, ny, nx))
    v = np.zeros((nz, ny, nx))
    w = np.zeros((nz + 1, ny, nx))
    if profile:
        u += laminar_profile(nz, lz, nu, dpdx)[:, None, None]
    if noise > 0.0:
        ucl = abs(dpdx) * lz * lz / (8.0 * nu)
        r = rng(seed)
        amp = noise * ucl
        u += amp * r.uniform(-1.0, 1.0, size=u.shape)
        v += amp * r.uniform(-1.0, 1.0, size=v.shape)
        w[1:nz] = amp * r.uniform(-1.0, 1.0, size=(nz - 1, ny, nx))
    return u, v, w


def faces_from_streamfunction(psi, dx, dz, ny):
    """2-D divergence-free face field from a streamfunction given on the x-z
    edges (x = i dx, z = k dz; array shape (nz+1, nx), psi = 0 on both walls):
    u = d psi/dz on x-faces, w = -d psi/dx on z-faces, v = 0, repeated in y."""
    nz = psi.shape[0] - 1
    u2 = (psi[1:, :] - psi[:-1, :]) / dz                      # (nz, nx) at (i dx, (k+1/2) dz)
    w2 = -(np.roll(psi, -1, axis=1) - psi) / dx                # (nz+1, nx) at ((i+1/2) dx, k dz)
    u = np.repeat(u2[:, None, :], ny, axis=1)
    w = np.repeat(w2[:, None, :], ny, axis=1)
    w[0] = 0.0
    w[nz] = 0.0
    v = np.zeros_like(u)
    return np.ascontiguousarray(u), np.ascontiguousarray(v), np.ascontiguousarray(w)

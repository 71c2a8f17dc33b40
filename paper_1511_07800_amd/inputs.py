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


def les_curl_state(nx, ny, nz, lx, ly, lz, nu, dpdx, a=1.0 / 3.0, modes=5, pert_rms=None, seed=360):
    """Turbulent-like start of the paper's LES (Sec. 6): u = a U0(z) +
    s curl[f(z) A(x)], with U0 the discrete steady laminar profile,
    f(z) = (1 - cos(2 pi z / lz)) / 2 (zero with zero slope at both walls) and
    A_i = sum over kx, ky, kz = 1..modes of S_i sin(k.x) + C_i cos(k.x),
    k = 2 pi (kx/lx, ky/ly, kz/lz), S and C uniform on [0, 1) (PCG64, seed).
    The vector potential f A sits on the cell edges and the velocity is its
    discrete curl on the faces, so the field is divergence-free to rounding
    on the staggered grid and w vanishes on the walls.  The scale s brings
    the rms of the curl term over all u, v, w faces to pert_rms (default: a
    tenth of a U0 at the centreline).  Returns u, v, w."""
    dx, dy, dz = lx / nx, ly / ny, lz / nz
    r = rng(seed)
    S = r.uniform(0.0, 1.0, size=(3, modes, modes, modes))
    C = r.uniform(0.0, 1.0, size=(3, modes, modes, modes))
    kk = np.arange(1, modes + 1)

    def potential(comp, xs, ys, zs):
        # A_comp(x, y, z) = Re sum (C - i S) e^{i k.x}, separably over kz, ky, kx
        coef = C[comp] - 1j * S[comp]                                        # [kx, ky, kz]
        ez = np.exp(1j * 2 * np.pi * np.outer(kk, zs) / lz)                  # [kz, z]
        ey = np.exp(1j * 2 * np.pi * np.outer(kk, ys) / ly)                  # [ky, y]
        ex = np.exp(1j * 2 * np.pi * np.outer(kk, xs) / lx)                  # [kx, x]
        t = np.einsum("abc,cz->abz", coef, ez)
        t = np.einsum("abz,by->ayz", t, ey)
        a_ = np.einsum("ayz,ax->zyx", t, ex).real
        f = 0.5 * (1.0 - np.cos(2 * np.pi * zs / lz))
        return f[:, None, None] * a_

    xc, yc = (np.arange(nx) + 0.5) * dx, (np.arange(ny) + 0.5) * dy
    xf, yf = np.arange(nx) * dx, np.arange(ny) * dy
    zf, zc = np.arange(nz + 1) * dz, (np.arange(nz) + 0.5) * dz
    psx = potential(0, xc, yf, zf)   # x-edges ((i+1/2) dx, j dy, k dz): (nz+1, ny, nx)
    psy = potential(1, xf, yc, zf)   # y-edges (i dx, (j+1/2) dy, k dz): (nz+1, ny, nx)
    psz = potential(2, xf, yf, zc)   # z-edges (i dx, j dy, (k+1/2) dz): (nz, ny, nx)
    u = (np.roll(psz, -1, axis=1) - psz) / dy - (psy[1:] - psy[:-1]) / dz
    v = (psx[1:] - psx[:-1]) / dz - (np.roll(psz, -1, axis=2) - psz) / dx
    w = (np.roll(psy, -1, axis=2) - psy) / dx - (np.roll(psx, -1, axis=1) - psx) / dy
    w[0] = 0.0
    w[nz] = 0.0
    base = laminar_profile(nz, lz, nu, dpdx)
    if pert_rms is None:
        pert_rms = 0.1 * a * abs(dpdx) * lz * lz / (8.0 * nu)
    rms = np.sqrt((np.sum(u * u) + np.sum(v * v) + np.sum(w * w)) / (u.size + v.size + w.size))
    s = pert_rms / rms
    u = a * base[:, None, None] + s * u
    return np.ascontiguousarray(u), np.ascontiguousarray(s * v), np.ascontiguousarray(s * w)


def os_paper_seed(nx, ny, nz, lx, lz, nu, dpdx, alpha, eps=1e-4, c=2.0 ** -0.5, s=-(2.0 ** -0.5)):
    """The perturbation that starts the paper's Orr-Sommerfeld validation run
    (Sec. 4.2) on the discrete steady laminar profile: du = -A(x) f'(z),
    dw = f(z) A'(x), with A = eps (C cos(alpha x) + S sin(alpha x)) and
    f = 1/2 + 1/2 sin(2 pi z / lz - pi/2).  It is laid on the staggered grid as
    the discrete curl of the streamfunction psi = f A on the x-z edges, so
    du = -d psi/dz and dw = d psi/dx hold exactly in difference form and the
    field is divergence-free to rounding.  Returns u, v, w."""
    dx, dz = lx / nx, lz / nz
    xe = np.arange(nx) * dx
    ze = np.arange(nz + 1) * dz
    f = 0.5 + 0.5 * np.sin(2 * np.pi * ze / lz - np.pi / 2)
    f[0] = f[-1] = 0.0
    a = eps * (c * np.cos(alpha * xe) + s * np.sin(alpha * xe))
    # faces_from_streamfunction gives u = d psi/dz and w = -d psi/dx: pass -psi
    du, dv, dw = faces_from_streamfunction(-(f[:, None] * a[None, :]), dx, dz, ny)
    u = laminar_profile(nz, lz, nu, dpdx)[:, None, None] + du
    return np.ascontiguousarray(u), dv, dw

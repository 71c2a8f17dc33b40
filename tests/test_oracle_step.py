"""Pins of the oracle's time step (Sec. 2.1-3.2): closed forms, invariants,
symmetries and analytic second-order accuracy of every discrete operator."""
import math

import numpy as np
import pytest
import scipy.linalg
import sympy as sp

import oracle
from paper_1511_07800_amd import inputs

# ---------------------------------------------------------------- helpers --


def random_state(P, seed, amp=1.0):
    r = inputs.rng(seed)
    u = amp * r.uniform(-1, 1, (P.nz, P.ny, P.nx))
    v = amp * r.uniform(-1, 1, (P.nz, P.ny, P.nx))
    w = np.zeros((P.nz + 1, P.ny, P.nx))
    w[1:P.nz] = amp * r.uniform(-1, 1, (P.nz - 1, P.ny, P.nx))
    return u, v, w


def run(P, u, v, w, nsteps, rtol=1e-12, maxit=200, p=None):
    s = oracle.Solver(P, u, v, w, p=p, rtol=rtol, maxit=maxit)
    stats = [s.step() for _ in range(nsteps)]
    return s, stats


# ------------------------------------------------- laminar Poiseuille flow --


def test_steady_poiseuille_is_a_fixed_point():
    """The discrete steady profile (parabola plus the ghost offset) stays put
    for 200 steps of the laminar workload (Sec. 4.1 base state)."""
    P = oracle.make_params(32, 16, 16, 2 * math.pi, math.pi, 2.0, nu=0.01, dpdx=-0.02, dt=1e-3)
    u0 = np.repeat(np.repeat(inputs.laminar_profile(16, 2.0, 0.01, -0.02)[:, None, None], 16, 1), 32, 2)
    s, stats = run(P, u0, np.zeros_like(u0), np.zeros((17, 16, 32)), 200, rtol=1e-10)
    assert np.abs(s.u - u0).max() <= 1e-13 * np.abs(u0).max()
    assert np.abs(s.v).max() == 0.0 and np.abs(s.w).max() == 0.0
    assert stats[-1]["poisson_cycles"] == 0
    # continuum centreline speed |G| lz^2 / (8 nu) = 1
    assert abs(u0.max() - 1.0) < 0.01


def startup_reference(nz, lz, nu, g, dt, nsteps):
    """Independent 1-D Crank-Nicolson recursion for u(z, t) from rest:
    (I - dt/2 nu A) u^{m+1} = (I + dt/2 nu A) u^m + dt |G|, with A the
    cell-centred second difference whose wall rows carry the odd ghost."""
    dz = lz / nz
    A = (np.eye(nz, k=1) + np.eye(nz, k=-1) - 2 * np.eye(nz)) / dz**2
    A[0, 0] = A[-1, -1] = -3.0 / dz**2
    I = np.eye(nz)
    lu = scipy.linalg.lu_factor(I - 0.5 * dt * nu * A)
    Bm = I + 0.5 * dt * nu * A
    u = np.zeros(nz)
    for _ in range(nsteps):
        u = scipy.linalg.lu_solve(lu, Bm @ u + dt * abs(g))
    return u


def test_startup_from_rest_matches_1d_recursion():
    P = oracle.make_params(32, 16, 16, 2 * math.pi, math.pi, 2.0, nu=0.01, dpdx=-0.02, dt=1e-3)
    z = np.zeros((16, 16, 32))
    s, _ = run(P, z, z, np.zeros((17, 16, 32)), 200, rtol=1e-10)
    ref = startup_reference(16, 2.0, 0.01, -0.02, 1e-3, 200)
    np.testing.assert_allclose(s.u, np.broadcast_to(ref[:, None, None], s.u.shape), rtol=0,
                               atol=1e-12 * np.abs(ref).max())


def test_startup_approaches_continuum_series():
    """The start-up flow at t = 0.2 matches the Fourier-series solution of
    u_t = nu u_zz + |G|, u(0) = u(lz) = 0, u(z, 0) = 0, to O(dz^2)."""
    nu, g, lz, t = 0.01, 0.02, 2.0, 0.2

    def series(z):
        s = np.zeros_like(z)
        for m in range(1, 400, 2):
            km = m * math.pi / lz
            bm = 4 * g / (m * math.pi) / (nu * km**2)
            s += bm * (1 - math.exp(-nu * km**2 * t)) * np.sin(km * z)
        return s

    errs = []
    for nz in (64, 128, 256):
        dz = lz / nz
        ref = startup_reference(nz, lz, nu, -g, 1e-4, 2000)
        zc = (np.arange(nz) + 0.5) * dz
        errs.append(np.abs(ref - series(zc)).max())
    # the wall layer sqrt(nu t) ~ 0.045 is resolved on these grids
    assert errs[1] < errs[0] / 3.0 and errs[2] < errs[1] / 3.0, errs
    # and the oracle equals the recursion (previous test) so it inherits this


# --------------------------------------------------------------- budgets --


def wall_sum(P, u):
    dz = P.lz / P.nz
    return -(2.0 * P.nu / dz**2) * (u[0].sum() + u[-1].sum())


@pytest.mark.parametrize("les", [0, 1])
def test_x_momentum_budget(les):
    """Sum over x-faces: sum u^{n+1} - sum u^n = dt N (-G) + dt/2 (W(u^n) + W(u^{n+1})),
    W the wall-shear sum; convection, the explicit viscous part and the
    pressure gradient telescope to zero (divergence form, Sec. 3.1)."""
    P = oracle.make_params(16, 8, 12, 2.0, 1.0, 1.0, nu=0.05, dpdx=-1.3, dt=2e-3, les=les)
    u, v, w = random_state(P, 21)
    s, _ = run(P, u, v, w, 3)
    # replay the third step explicitly
    s2 = oracle.Solver(P, u, v, w, rtol=1e-12, maxit=200)
    s2.step(); s2.step()
    u_n = s2.u.copy()
    s2.step()
    n = P.nx * P.ny * P.nz
    lhs = s2.u.sum() - u_n.sum()
    rhs = P.dt * n * (-P.dpdx) + 0.5 * P.dt * (wall_sum(P, u_n) + wall_sum(P, s2.u))
    assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(rhs))
    np.testing.assert_array_equal(s.u, s2.u)


def test_divergence_after_projection():
    """div u^{n+1} = dt (b - L p): below 1e-10 once the solve converges
    (Sec. 3.1 projection)."""
    P = oracle.make_params(16, 8, 12, 2.0, 1.0, 1.0, nu=0.05, dpdx=-1.0, dt=2e-3, les=1)
    u, v, w = random_state(P, 22)
    s, st = run(P, u, v, w, 2, rtol=1e-12)
    d = oracle.divergence(P, s.u, s.v, s.w)
    assert np.abs(d).max() < 1e-10
    r, _ = oracle.residual(P, s.p, s.b)
    np.testing.assert_allclose(d, P.dt * r, atol=1e-12)
    assert st[-1]["max_div"] == pytest.approx(np.abs(d).max(), rel=1e-12, abs=1e-18)


# ------------------------------------------------------------- symmetries --


@pytest.mark.parametrize("axis", ["x", "y"])
def test_shift_commutes_with_step(axis):
    P = oracle.make_params(12, 8, 10, 2.0, 1.0, 1.0, nu=0.02, dpdx=-1.0, dt=1e-3, les=1)
    u, v, w = random_state(P, 23)
    ax = 2 if axis == "x" else 1
    sh = lambda a: np.ascontiguousarray(np.roll(a, 3, axis=ax))
    a, _ = run(P, u, v, w, 2)
    b, _ = run(P, sh(u), sh(v), sh(w), 2)
    for f1, f2 in [(a.u, b.u), (a.v, b.v), (a.w, b.w), (a.p, b.p)]:
        np.testing.assert_allclose(sh(f1), f2, atol=1e-12 * max(1.0, np.abs(f1).max()))


def test_spanwise_mirror_symmetry():
    """y -> -y: u, w, p at cell-centred y map j -> -j-1; v at y faces maps
    j -> -j with a sign flip."""
    P = oracle.make_params(12, 8, 10, 2.0, 1.0, 1.0, nu=0.02, dpdx=-1.0, dt=1e-3, les=1)
    u, v, w = random_state(P, 24)
    ny = P.ny
    mc = lambda a: np.ascontiguousarray(a[:, [(-j - 1) % ny for j in range(ny)], :])
    mf = lambda a: np.ascontiguousarray(-a[:, [(-j) % ny for j in range(ny)], :])
    a, _ = run(P, u, v, w, 2)
    b, _ = run(P, mc(u), mf(v), mc(w), 2)
    np.testing.assert_allclose(mc(a.u), b.u, atol=1e-12 * np.abs(a.u).max())
    np.testing.assert_allclose(mf(a.v), b.v, atol=1e-12 * np.abs(a.v).max())
    np.testing.assert_allclose(mc(a.w), b.w, atol=1e-12 * np.abs(a.w).max())


def test_zero_flow_stays_zero_without_forcing():
    P = oracle.make_params(8, 4, 6, 1.0, 1.0, 1.0, nu=0.1, dpdx=0.0, dt=1e-3, les=1)
    z = np.zeros((6, 4, 8))
    s, st = run(P, z, z, np.zeros((7, 4, 8)), 3)
    assert not s.u.any() and not s.v.any() and not s.w.any() and not s.p.any()


# ------------------------------------------- operators against calculus ---

X, Y, Z = sp.symbols("x y z")
LX, LY, LZ = 2 * math.pi, 2 * math.pi, 1.0
Uf = sp.sin(X) * sp.cos(Y) * sp.sin(sp.pi * Z / LZ) + 0.3 * sp.sin(2 * sp.pi * Z / LZ)
Vf = sp.cos(X + 0.4) * sp.sin(2 * Y) * sp.sin(sp.pi * Z / LZ)
Wf = sp.sin(X - Y) * sp.sin(sp.pi * Z / LZ) ** 2
NUf = 0.1 + 0.05 * sp.sin(X) * sp.cos(2 * Y) * (1 + Z)


def sample(expr, xs, ys, zs):
    f = sp.lambdify((X, Y, Z), expr, "numpy")
    Zg, Yg, Xg = np.meshgrid(zs, ys, xs, indexing="ij")
    return np.broadcast_to(f(Xg, Yg, Zg), Zg.shape).astype(np.float64).copy()


def grids(n):
    nx = ny = n
    nz = n
    dx, dy, dz = LX / nx, LY / ny, LZ / nz
    xc = (np.arange(nx) + 0.5) * dx
    yc = (np.arange(ny) + 0.5) * dy
    zc = (np.arange(nz) + 0.5) * dz
    xf = np.arange(nx) * dx
    yf = np.arange(ny) * dy
    zf = np.arange(nz + 1) * dz
    return (nx, ny, nz), (xc, yc, zc), (xf, yf, zf)


def analytic_terms():
    vel = [Uf, Vf, Wf]
    coords = [X, Y, Z]
    E, L = [], []
    for i in range(3):
        conv = sum(sp.diff(vel[j] * vel[i], coords[j]) for j in range(3))
        transp = sum(sp.diff(NUf * sp.diff(vel[j], coords[i]), coords[j]) for j in range(3))
        E.append(-conv + transp)
        L.append(sum(sp.diff(NUf * sp.diff(vel[i], coords[j]), coords[j]) for j in range(3)))
    div = sum(sp.diff(vel[j], coords[j]) for j in range(3))
    return E, L, div


def operator_errors(n, E, L, div):
    (nx, ny, nz), (xc, yc, zc), (xf, yf, zf) = grids(n)
    P = oracle.make_params(nx, ny, nz, LX, LY, LZ, nu=0.1, dpdx=0.0, dt=1.0)
    u = sample(Uf, xf, yc, zc)
    v = sample(Vf, xc, yf, zc)
    w = sample(Wf, xc, yc, zf)
    nut = sample(NUf, xc, yc, zc)
    eu, ev, ew = oracle.explicit(P, u, v, w, nut)
    ks = slice(2, nz - 2)
    kw = slice(2, nz - 1)
    out = {}
    out["Eu"] = np.abs(eu - sample(E[0], xf, yc, zc))[ks].max()
    out["Ev"] = np.abs(ev - sample(E[1], xc, yf, zc))[ks].max()
    out["Ew"] = np.abs(ew - sample(E[2], xc, yc, zf))[kw].max()
    out["Lu"] = np.abs(oracle.visc_diff(P, 0, nut, u) - sample(L[0], xf, yc, zc))[ks].max()
    out["Lv"] = np.abs(oracle.visc_diff(P, 1, nut, v) - sample(L[1], xc, yf, zc))[ks].max()
    out["Lw"] = np.abs(oracle.visc_diff(P, 2, nut, w) - sample(L[2], xc, yc, zf))[kw].max()
    out["div"] = np.abs(oracle.divergence(P, u, v, w) - sample(div, xc, yc, zc)).max()
    return out


def test_operators_second_order():
    """Convection (divergence form), the explicit viscous part, the diffusive
    operator and the divergence converge at second order in the interior
    (Sec. 3.2: centred differences, O(h^2))."""
    E, L, div = analytic_terms()
    e1 = operator_errors(16, E, L, div)
    e2 = operator_errors(32, E, L, div)
    for key in e1:
        order = math.log2(e1[key] / e2[key])
        assert 1.8 <= order <= 2.3, (key, e1[key], e2[key], order)


def test_eddy_viscosity_linear_shear_exact():
    """u = S (z - lz/2): |S| = S exactly at interior centres, so
    nu_T = nu + (C_S Delta phi_w)^2 S (Sec. 2.2)."""
    nx, ny, nz, lz = 8, 6, 16, 2.0
    P = oracle.make_params(nx, ny, nz, 1.0, 1.0, lz, nu=1 / 180, dpdx=-1.0, dt=1e-4, les=1)
    S = 3.7
    zc = (np.arange(nz) + 0.5) * lz / nz
    u = np.repeat(np.repeat((S * (zc - lz / 2))[:, None, None], ny, 1), nx, 2)
    nut, _ = oracle.nut(P, u, np.zeros_like(u), np.zeros((nz + 1, ny, nx)))
    delta = 2 * (1.0 / nx * 1.0 / ny * lz / nz) ** (1 / 3)
    utau = math.sqrt(lz * 1.0 / 2)
    dw = np.minimum(zc, lz - zc)
    phi = 1 - np.exp(-dw * utau / P.nu / 25.0)
    ref = P.nu + (0.1 * delta * phi) ** 2 * S
    np.testing.assert_allclose(nut[1:-1, 0, 0], ref[1:-1], rtol=1e-13)


def test_eddy_viscosity_strain_second_order():
    """|S|^2 from the staggered strains converges at second order to
    2 S_ij S_ij of a smooth field (compared squared: where |S| vanishes the
    square root turns an O(h^2) error into O(h))."""
    vel = [Uf, Vf, Wf]
    coords = [X, Y, Z]
    s2 = 0
    for i in range(3):
        for j in range(3):
            sij = 0.5 * (sp.diff(vel[i], coords[j]) + sp.diff(vel[j], coords[i]))
            s2 += 2 * sij * sij
    errs = []
    for n in (64, 128):
        (nx, ny, nz), (xc, yc, zc), (xf, yf, zf) = grids(n)
        P = oracle.make_params(nx, ny, nz, LX, LY, LZ, nu=1.0, dpdx=-1.0, dt=1.0, les=1, cs=1.0)
        u = sample(Uf, xf, yc, zc)
        v = sample(Vf, xc, yf, zc)
        w = sample(Wf, xc, yc, zf)
        nut, _ = oracle.nut(P, u, v, w)
        delta = 2 * (LX / nx * LY / ny * LZ / nz) ** (1 / 3)
        utau = math.sqrt(LZ / 2)
        phi = 1 - np.exp(-np.minimum(zc, LZ - zc) * utau / 1.0 / 25.0)
        s_num = (nut - 1.0) / ((delta * phi) ** 2)[:, None, None]
        errs.append(np.abs(s_num**2 - sample(s2, xc, yc, zc))[2:-2].max())
    assert 1.85 <= math.log2(errs[0] / errs[1]) <= 2.2, errs


# ------------------------------------------------------------ diagnostics --


@pytest.mark.parametrize("nz", [16, 15])
def test_diagnostics_closed_forms(nz):
    """or_diagnostics on fields with closed-form answers (the CFL rule of
    Sec. 3.2, the centreline velocity of Sec. 6):
    * the discrete steady profile u_k = |G| z_k (lz - z_k)/(2 nu) + |G| dz^2/(8 nu)
      has mean |G| lz^2/(12 nu) + |G| dz^2/(6 nu) over the midpoints z_k, its
      largest value |G| lz^2/(8 nu) (+ |G| dz^2/(8 nu) when nz is odd, where a
      cell centre sits on the centreline), and that same value on the
      centreline;
    * v = c_v everywhere and w = c_w on the interior z-faces give
      CFL = max(U_max/dx, |c_v|/dy, |c_w|/dz) dt, and a divergence of
      c_w/dz in the first and -c_w/dz in the last cell layer, 0 elsewhere."""
    nx, ny, lx, ly, lz = 12, 6, 3.0, 2.0, 2.0
    nu, g, dt = 0.01, 0.02, 1e-3
    P = oracle.make_params(nx, ny, nz, lx, ly, lz, nu=nu, dpdx=-g, dt=dt)
    h = lz / nz
    u = np.repeat(np.repeat(inputs.laminar_profile(nz, lz, nu, -g)[:, None, None], ny, 1), nx, 2)
    umax = g * lz**2 / (8 * nu) + (g * h * h / (8 * nu) if nz % 2 else 0.0)
    ubulk = g * lz**2 / (12 * nu) + g * h * h / (6 * nu)
    for cv, cw in ((0.0, 0.0), (3.0 * ly / ny / (lx / nx), 0.0), (0.0, -4.0 * h / (lx / nx)), (0.5, 0.25)):
        v = np.full((nz, ny, nx), cv)
        w = np.zeros((nz + 1, ny, nx))
        w[1:nz] = cw
        st = oracle.diagnostics(P, u, v, w)
        assert st["u_max"] == pytest.approx(umax, rel=1e-14)
        assert st["u_centre"] == pytest.approx(umax, rel=1e-14)
        assert st["u_bulk"] == pytest.approx(ubulk, rel=1e-14)
        cfl = max(umax * dt / (lx / nx), abs(cv) * dt / (ly / ny), abs(cw) * dt / h)
        assert st["cfl"] == pytest.approx(cfl, rel=1e-14)
        assert st["max_div"] == pytest.approx(abs(cw) / h, rel=1e-14, abs=0.0)


def test_eddy_viscosity_field_and_max_closed_form():
    """u = S z, v = w = 0: the odd ghost below the bottom wall continues the
    line, so |S| = S in every cell but the top one; there the ghost above
    the wall gives the x-z strains S/2 (lower edges) and -(u_top)/dz (upper
    edges, u_top = S (lz - dz/2)), so |S|^2 = 4 mean(S13^2) =
    (S^2 + (2 u_top/dz)^2)/2.  nu_T = nu + (C_S Delta phi_w)^2 |S| everywhere
    (Sec. 2.2), and or_nut returns its maximum."""
    nx, ny, nz, lx, ly, lz = 6, 4, 12, 1.5, 1.0, 2.0
    P = oracle.make_params(nx, ny, nz, lx, ly, lz, nu=1 / 180, dpdx=-1.0, dt=1e-4, les=1)
    S, h = 2.5, lz / nz
    zc = (np.arange(nz) + 0.5) * h
    u = np.repeat(np.repeat((S * zc)[:, None, None], ny, 1), nx, 2)
    nut, mx = oracle.nut(P, u, np.zeros_like(u), np.zeros((nz + 1, ny, nx)))
    smag = np.full(nz, S)
    utop = S * (lz - h / 2)
    smag[-1] = math.sqrt(0.5 * (S * S + (2 * utop / h) ** 2))
    delta = 2 * (lx / nx * ly / ny * h) ** (1 / 3)
    phi = 1 - np.exp(-np.minimum(zc, lz - zc) * math.sqrt(lz / 2) / P.nu / 25.0)
    ref = P.nu + (0.1 * delta * phi) ** 2 * smag
    np.testing.assert_allclose(nut, np.broadcast_to(ref[:, None, None], nut.shape), rtol=1e-13)
    assert mx == pytest.approx(ref.max(), rel=1e-13)


def test_plane_stats_closed_forms():
    """or_plane_stats on fields with closed-form plane means (Sec. 6 averages):
    u = U(z) + alpha sin(2 pi x/Lx) on the x-faces, v = beta cos(2 pi y/Ly),
    w = gamma sin(2 pi x/Lx) on the interior z-faces, nu_T = c.  Over a full
    period the sines average to 0 and their squares to 1/2, so <u> = U,
    <u^2> = U^2 + alpha^2/2, <v> = 0, <v^2> = beta^2/2, <w> = 0,
    <w^2> = gamma^2/2 inside and 0 on the walls, <nu_T> = c; on the x-z edges
    u is (U_{k-1} + U_k)/2 + alpha sin(2 pi x_i/Lx) and w interpolated in x is
    gamma cos(pi dx/Lx) sin(2 pi x_i/Lx), so <u w> = alpha gamma cos(pi dx/Lx)/2
    inside and 0 on the walls (odd ghosts make u vanish there)."""
    nx, ny, nz, lx, ly, lz = 12, 10, 9, 3.0, 2.0, 1.5
    P = oracle.make_params(nx, ny, nz, lx, ly, lz)
    al, be, ga, c = 0.7, -1.3, 0.4, 0.05
    zc = (np.arange(nz) + 0.5) * lz / nz
    U = 3.0 + np.sin(zc) * zc
    xf = np.arange(nx) * lx / nx
    xc = (np.arange(nx) + 0.5) * lx / nx
    yf = np.arange(ny) * ly / ny
    u = U[:, None, None] + al * np.sin(2 * np.pi * xf / lx)[None, None, :] + 0 * yf[None, :, None]
    v = np.broadcast_to(be * np.cos(2 * np.pi * yf / ly)[None, :, None], (nz, ny, nx)).copy()
    w = np.zeros((nz + 1, ny, nx))
    w[1:nz] = ga * np.sin(2 * np.pi * xc / lx)[None, None, :]
    nut = np.full((nz, ny, nx), c)
    st = oracle.plane_stats(P, u, v, w, nut)
    np.testing.assert_allclose(st["u"], U, rtol=1e-14)
    np.testing.assert_allclose(st["uu"], U * U + al * al / 2, rtol=1e-14)
    np.testing.assert_allclose(st["v"], 0.0, atol=1e-15)
    np.testing.assert_allclose(st["vv"], be * be / 2, rtol=1e-14)
    np.testing.assert_allclose(st["nut"], c, rtol=1e-14)
    np.testing.assert_allclose(st["w"], 0.0, atol=1e-15)
    ww = np.full(nz + 1, ga * ga / 2)
    ww[0] = ww[nz] = 0.0
    np.testing.assert_allclose(st["ww"], ww, rtol=1e-14, atol=1e-300)
    uw = np.full(nz + 1, al * ga * np.cos(np.pi / nx) / 2)
    uw[0] = uw[nz] = 0.0
    np.testing.assert_allclose(st["uw"], uw, rtol=1e-13, atol=1e-16)

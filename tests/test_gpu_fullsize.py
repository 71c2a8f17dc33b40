"""GPU parity with the FP64 oracle at the launch shapes the kernels take on
the large grids, through the C ABI:

* the diagnostics reduction (max |div u|, bulk velocity, U_max, CFL,
  centreline velocity; Sec. 3.2 CFL rule, Sec. 6 centreline velocity) and the
  eddy-viscosity maximum, output by output;
* whole LES steps (Sec. 2.2, 3.1, 3.4) on a grid whose column march spans
  the channel wall to wall in one chunk (1024 x 512 columns) and on the
  512 x 256 x 192 grid with its fused, z-chunked sweeps;
* 100 steps of the 256 x 8 x 128 linear-instability workload;
* mixed precision against the FP64 oracle converged to rtol 1e-12 on the
  256 x 128 x 128 LES grid, the error reported per step.

Identical iteration sequences (a caller-given cycle, rtol 0) are compared
at 1e-10 relative L2; converged runs at the stated tolerance."""
import math

import numpy as np
import pytest

import oracle
from oracle import schedule as osched
from paper_1511_07800_amd import inputs, workloads
from _helpers import rel_l2, load_state, fields

pytestmark = pytest.mark.gpu


def short_cycle(g, degree=16):
    """A complete Chebyshev/Leja cycle of the given degree over the grid's
    spectrum (the oracle's schedule generator)."""
    a, b = osched.kappa_bounds(*g)
    return osched.schedule_of_degree(a, b, degree)


def pair(g, nu, dpdx, dt, les, omega, rtol, maxit, u, v, w, **kw):
    from paper_1511_07800_amd import Channel
    nx, ny, nz, lx, ly, lz = g
    ch = Channel(nx, ny, nz, lx, ly, lz, nu=nu, dpdx=dpdx, dt=dt, les=les, poisson_rtol=rtol,
                 poisson_maxit=maxit, omega=list(omega), **kw)
    load_state(ch, u, v, w)
    P = oracle.make_params(nx, ny, nz, lx, ly, lz, nu=nu, dpdx=dpdx, dt=dt, les=les)
    orc = oracle.Solver(P, u, v, w, omega=omega, rtol=rtol, maxit=maxit)
    return ch, orc, P


def check_diagnostics(st, P, f, nut_max_ref):
    """Every diagnostic of the step against or_diagnostics on the same fields."""
    ref = oracle.diagnostics(P, f["u"], f["v"], f["w"])
    for key in ("u_bulk", "u_max", "cfl", "u_centre"):
        assert st[key] == pytest.approx(ref[key], rel=1e-12, abs=0.0), key
    # the divergence is a difference of terms of size max|u|/dx etc.: the two
    # sides round each term once (a reciprocal multiply against a divide), so
    # the bar is relative to the terms, not to the (small) result
    scale = (np.abs(f["u"]).max() * P.nx / P.lx + np.abs(f["v"]).max() * P.ny / P.ly
             + np.abs(f["w"]).max() * P.nz / P.lz)
    assert abs(st["max_div"] - ref["max_div"]) <= 1e-13 * scale, (st["max_div"], ref["max_div"], scale)
    assert st["nut_max"] == pytest.approx(nut_max_ref, rel=1e-12, abs=0.0)
    print(f"diagnostics: max_div {st['max_div']:.6e}/{ref['max_div']:.6e} u_bulk {st['u_bulk']:.12f} "
          f"u_max {st['u_max']:.12f} cfl {st['cfl']:.6e} u_centre {st['u_centre']:.12f} "
          f"nut_max {st['nut_max']:.6e}", flush=True)


GRID_WALL_TO_WALL = (1024, 512, 8, 4 * math.pi, 2 * math.pi, 2.0)


@pytest.mark.parametrize("g", [(48, 32, 24, 2 * math.pi, math.pi, 2.0), GRID_WALL_TO_WALL])
def test_diagnostics_match_oracle(gpu, g):
    """After one LES step, every output of the diagnostics kernel equals the
    oracle's diagnostics of the same fields, and the step's eddy-viscosity
    maximum equals the oracle's for the starting state."""
    print(f"diagnostics grid={g[:3]}", flush=True)
    nx, ny, nz, lx, ly, lz = g
    u, v, w = inputs.channel_state(nx, ny, nz, lz, 1 / 180, -1.0, noise=0.1, seed=51)
    P = oracle.make_params(*g, nu=1 / 180, dpdx=-1.0, dt=1e-5, les=1)
    _, nut_max_ref = oracle.nut(P, u, v, w)
    from paper_1511_07800_amd import Channel
    ch = Channel(*g, nu=1 / 180, dpdx=-1.0, dt=1e-5, les=1, poisson_rtol=0.0, poisson_maxit=1,
                 omega=list(short_cycle(g)))
    load_state(ch, u, v, w)
    st = ch.step(1)
    check_diagnostics(st, P, fields(ch), nut_max_ref)
    ch.close()


@pytest.mark.parametrize("case", ["wall_to_wall_1024x512x8", "les_channel_512x256x192"])
def test_les_step_large_grid_matches_oracle(gpu, case):
    """One LES step with a 16-sweep Chebyshev cycle (rtol 0: the same
    iteration sequence on both sides): u, v, w, p, nu_T and b within 1e-10.
    At 1024 x 512 the stencil kernels' column march has 2048 columns and runs
    each column wall to wall in one chunk, the shape they take on the
    1024 x 512 x 384 grid; at 512 x 256 x 192 the march is cut into z-chunks
    and the sweeps run fused, four per launch, in five z-chunks."""
    if case == "les_channel_512x256x192":
        wl = workloads.params(case)
        g = (wl["nx"], wl["ny"], wl["nz"], wl["lx"], wl["ly"], wl["lz"])
        nu, dpdx, dt, noise, seed = wl["nu"], wl["dpdx"], wl["dt"], wl["noise"], wl["seed"]
    else:
        g = GRID_WALL_TO_WALL
        nu, dpdx, dt, noise, seed = 1 / 180, -1.0, 1e-5, 0.1, 52
        # the marching kernels take 64 x 4 columns per workgroup and ask for
        # 2048 workgroups: 2048 column tiles leave one chunk of nz planes
        assert (g[0] // 64) * (g[1] // 4) >= 2048
    print(f"LES step grid={g[:3]}", flush=True)
    nx, ny, nz, lx, ly, lz = g
    u, v, w = inputs.channel_state(nx, ny, nz, lz, nu, dpdx, noise=noise, seed=seed)
    ch, orc, P = pair(g, nu, dpdx, dt, 1, short_cycle(g), 0.0, 1, u, v, w)
    _, nut_max_ref = oracle.nut(P, u, v, w)
    st = ch.step(1)
    so = orc.step()
    assert st["poisson"]["sweeps"] == 16 and so["poisson_cycles"] == 1
    f = fields(ch)
    ref = {"u": orc.u, "v": orc.v, "w": orc.w, "p": orc.p, "nut": orc.nut, "b": orc.b}
    errs = {k: rel_l2(f[k], ref[k]) for k in ref}
    print("rel_l2", {k: f"{e:.2e}" for k, e in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e <= 1e-10, (k, e)
    check_diagnostics(st, P, f, nut_max_ref)
    ch.close()


def test_linear_instability_100_steps_match_oracle(gpu):
    """The 256 x 8 x 128 workload (Re 7500, parabolic base flow, the
    Orr-Sommerfeld mode of amplitude 1e-5 plus 1e-7 seeded noise, dt 5e-4):
    100 FP64 steps with two cycles of the built-in schedule per step on both
    sides; the velocity field and the pressure within 1e-10 after steps 1, 10
    and 100.  Here v is the 1e-7 noise alone and p only the small deviation
    from the linear pressure G x that drives the flow (Sec. 2.1), so each is
    measured against the quantity it is part of: the velocity vector field
    (u, v, w), and the full kinematic pressure G x + p.  The per-field
    relative errors are printed beside."""
    from _ts import ts_initial_state
    wl = workloads.params("linear_instability_256x8x128")
    g = (wl["nx"], wl["ny"], wl["nz"], wl["lx"], wl["ly"], wl["lz"])
    nx, ny, nz = g[:3]
    u, v, w, lam, G = ts_initial_state(nx, ny, nz, wl["lx"], wl["lz"], 1 / wl["nu"], wl["ts_alpha"],
                                       wl["ts_amplitude"])
    r = inputs.rng(wl["seed"])
    u = u + wl["noise"] * r.uniform(-1, 1, u.shape)
    v = v + wl["noise"] * r.uniform(-1, 1, v.shape)
    w = w.copy()
    w[1:nz] += wl["noise"] * r.uniform(-1, 1, (nz - 1, ny, nx))
    ch, orc, P = pair(g, wl["nu"], G, wl["dt"], 0, osched.srj_schedule(*g), 0.0, 2, u, v, w)
    # G x at the cell centres, taken about the domain's middle (p is mean-free)
    gx = G * ((np.arange(nx) + 0.5) * wl["lx"] / nx - 0.5 * wl["lx"])
    worst = 0.0
    for n in range(1, 101):
        st = ch.step(1)
        so = orc.step()
        assert st["poisson"]["cycles"] == so["poisson_cycles"] == 2
        if n in (1, 10, 100):
            f = fields(ch)
            errs = {k: rel_l2(f[k], getattr(orc, k)) for k in ("u", "v", "w", "p")}
            vel = math.sqrt(sum(np.sum((f[k] - getattr(orc, k)) ** 2) for k in "uvw")
                            / sum(np.sum(getattr(orc, k) ** 2) for k in "uvw"))
            pres = rel_l2(f["p"] + gx, orc.p + gx)
            print(f"step {n}: relres {st['poisson']['relres']:.2e}/{so['relres']:.2e} velocity {vel:.2e} "
                  f"pressure {pres:.2e}; per field " + " ".join(f"{k} {e:.2e}" for k, e in errs.items()), flush=True)
            worst = max(worst, vel, pres)
    assert worst <= 1e-10
    ch.close()


@pytest.fixture(scope="module")
def les256_oracle_trajectory():
    """The FP64 oracle on the 256 x 128 x 128 LES workload, converged to
    rtol 1e-12 every step: the fields after steps 1, 2 and 3."""
    wl = workloads.params("les_channel_256x128x128")
    g = (wl["nx"], wl["ny"], wl["nz"], wl["lx"], wl["ly"], wl["lz"])
    u, v, w = inputs.channel_state(wl["nx"], wl["ny"], wl["nz"], wl["lz"], wl["nu"], wl["dpdx"],
                                   noise=wl["noise"], seed=wl["seed"])
    P = oracle.make_params(*g, nu=wl["nu"], dpdx=wl["dpdx"], dt=wl["dt"], les=1)
    orc = oracle.Solver(P, u, v, w, rtol=1e-12, maxit=100)
    traj = []
    for n in range(3):
        so = orc.step()
        assert so["status"] == 0 and so["relres"] <= 1e-12
        traj.append({k: getattr(orc, k).copy() for k in ("u", "v", "w", "p")})
        print(f"oracle step {n + 1}: cycles {so['poisson_cycles']} relres {so['relres']:.1e}", flush=True)
    return wl, g, (u, v, w), traj


@pytest.mark.parametrize("rhs16,st32", [(0, 0), (1, 0), (1, 1)])
def test_mixed_les_256x128x128_against_fp64_oracle(gpu, les256_oracle_trajectory, rhs16, st32):
    """Mixed mode (FP32 sweeps and Crank-Nicolson increments inside FP64
    defect corrections; with rhs16 each pass reads its right-hand side as
    FP16, with st32 the eddy viscosity and explicit terms run in FP32)
    against the FP64 oracle, both converged to rtol 1e-12, on the
    256 x 128 x 128 LES workload: the error of every field after each of
    three steps is reported and stays below 1e-5."""
    from paper_1511_07800_amd import Channel, STP_MIXED
    wl, g, (u, v, w), traj = les256_oracle_trajectory
    ch = Channel(*g, nu=wl["nu"], dpdx=wl["dpdx"], dt=wl["dt"], les=1, precision=STP_MIXED,
                 poisson_rtol=1e-12, poisson_maxit=100, srj_adaptive=1, srj_reduction=wl["srj_reduction"],
                 mixed_rhs16=rhs16, stencils32=st32)
    load_state(ch, u, v, w)
    worst = 0.0
    for n, ref in enumerate(traj):
        st = ch.step(1)
        assert st["poisson"]["relres"] <= 1e-12
        f = fields(ch)
        errs = {k: rel_l2(f[k], ref[k]) for k in ref}
        print(f"mixed (rhs16={rhs16}, stencils32={st32}) step {n + 1}: passes {st['poisson']['outer']} "
              + " ".join(f"{k} {e:.2e}" for k, e in errs.items()), flush=True)
        worst = max(worst, max(errs.values()))
    assert worst <= 1e-5
    ch.close()

"""GPU parity of the full time step (Sec. 2-3) against the FP64 oracle,
through the C ABI: laminar start-up, LES steps with identical iteration
sequences, stop-cycle agreement, mixed precision, determinism."""
import math

import numpy as np
import pytest

import oracle
from oracle import schedule as osched
from paper_1511_07800_amd import inputs, workloads
from _helpers import rel_l2, load_state, fields

pytestmark = pytest.mark.gpu


def make_pair(g, nu, dpdx, dt, les, rtol, maxit, u, v, w, precision=0, warm=0, **kw):
    from paper_1511_07800_amd import Channel
    nx, ny, nz, lx, ly, lz = g
    om = osched.srj_schedule(*g)
    ch = Channel(nx, ny, nz, lx, ly, lz, nu=nu, dpdx=dpdx, dt=dt, les=les, precision=precision,
                 warm_start=warm, poisson_rtol=rtol, poisson_maxit=maxit, omega=list(om), **kw)
    load_state(ch, u, v, w)
    P = oracle.make_params(nx, ny, nz, lx, ly, lz, nu=nu, dpdx=dpdx, dt=dt, les=les)
    orc = oracle.Solver(P, u, v, w, omega=om, rtol=rtol, maxit=maxit, warm_start="zero" if warm else "prev")
    return ch, orc


def compare(ch, orc, tol, keys=("u", "v", "w", "p")):
    f = fields(ch)
    ref = {"u": orc.u, "v": orc.v, "w": orc.w, "p": orc.p, "nut": orc.nut, "b": orc.b}
    errs = {k: rel_l2(f[k], ref[k]) for k in keys}
    print("rel_l2", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k in keys:
        assert errs[k] <= tol, (k, errs[k])
    return errs


def test_laminar_startup_200_steps(gpu):
    """The laminar Poiseuille workload: 200 steps from rest, FP64, rtol 1e-10."""
    wl = workloads.params("laminar_poiseuille_32x16x16")
    g = (wl["nx"], wl["ny"], wl["nz"], wl["lx"], wl["ly"], wl["lz"])
    z = np.zeros((wl["nz"], wl["ny"], wl["nx"]))
    zw = np.zeros((wl["nz"] + 1, wl["ny"], wl["nx"]))
    ch, orc = make_pair(g, wl["nu"], wl["dpdx"], wl["dt"], 0, 1e-10, 100, z, z, zw)
    st = ch.step(200)
    for _ in range(200):
        orc.step()
    assert st["step"] == 200
    f = fields(ch)
    assert rel_l2(f["u"], orc.u) <= 1e-12
    assert np.abs(f["v"]).max() == 0.0 and np.abs(f["w"]).max() == 0.0
    assert st["max_div"] < 1e-10


def test_steady_poiseuille_gpu(gpu):
    wl = workloads.params("laminar_poiseuille_32x16x16")
    g = (wl["nx"], wl["ny"], wl["nz"], wl["lx"], wl["ly"], wl["lz"])
    u, v, w = inputs.channel_state(wl["nx"], wl["ny"], wl["nz"], wl["lz"], wl["nu"], wl["dpdx"])
    ch, _ = make_pair(g, wl["nu"], wl["dpdx"], wl["dt"], 0, 1e-10, 100, u, v, w)
    ch.step(200)
    f = fields(ch)
    assert np.abs(f["u"] - u).max() <= 1e-13 * np.abs(u).max()


@pytest.mark.parametrize("g", [(40, 24, 20, 2.0, 1.2, 2.0), (33, 7, 18, 1.0, 0.5, 2.0)])
def test_les_steps_fixed_cycles(gpu, g):
    """LES on, 10% noise: identical iteration sequences (2 SRJ cycles per
    step), 10 steps, every field within 1e-10."""
    nx, ny, nz, lx, ly, lz = g
    u, v, w = inputs.channel_state(nx, ny, nz, lz, 1 / 180, -1.0, noise=0.1, seed=31)
    ch, orc = make_pair(g, 1 / 180, -1.0, 2e-5, 1, 0.0, 2, u, v, w)
    for n in range(10):
        st = ch.step(1)
        so = orc.step()
        assert st["poisson"]["cycles"] == so["poisson_cycles"] == 2
        assert st["cn_sweeps"] >= 1
    compare(ch, orc, 1e-10, ("u", "v", "w", "p", "nut", "b"))


def test_les_one_step_predictor(gpu):
    """One step: eddy viscosity and the Poisson right-hand side (which carries
    the whole predictor) within 1e-13."""
    g = (40, 24, 20, 2.0, 1.2, 2.0)
    nx, ny, nz, lx, ly, lz = g
    u, v, w = inputs.channel_state(nx, ny, nz, lz, 1 / 180, -1.0, noise=0.1, seed=32)
    ch, orc = make_pair(g, 1 / 180, -1.0, 2e-5, 1, 0.0, 1, u, v, w)
    ch.step(1)
    orc.step()
    compare(ch, orc, 1e-13, ("nut", "b"))


def test_les_converged_same_stop_cycles(gpu):
    g = (48, 32, 24, 2 * math.pi, math.pi, 2.0)
    nx, ny, nz, lx, ly, lz = g
    u, v, w = inputs.channel_state(nx, ny, nz, lz, 1 / 180, -1.0, noise=0.1, seed=33)
    ch, orc = make_pair(g, 1 / 180, -1.0, 2e-5, 1, 1e-10, 100, u, v, w)
    for n in range(5):
        st = ch.step(1)
        so = orc.step()
        assert st["poisson"]["cycles"] == so["poisson_cycles"]
        # div u^{n+1} = dt (b - L p): bounded by the stop test
        bound = 2e-5 * st["poisson"]["relres"] * st["poisson"]["bnorm"] * 1.001 + 1e-13
        assert st["max_div"] <= bound and so["max_div"] <= bound
        assert st["u_bulk"] == pytest.approx(so["u_bulk"], rel=1e-12)
    compare(ch, orc, 1e-10)


@pytest.mark.parametrize("st32", [0, 1])
def test_mixed_les_against_fp64_oracle(gpu, st32):
    """Mixed mode (FP32 sweeps, FP64 residual and correction; with st32 the
    eddy viscosity and explicit terms in FP32 too) after 10 LES steps stays
    within 1e-5 of the FP64 oracle converged to 1e-12."""
    from paper_1511_07800_amd import STP_MIXED
    g = (48, 32, 24, 2 * math.pi, math.pi, 2.0)
    nx, ny, nz, lx, ly, lz = g
    u, v, w = inputs.channel_state(nx, ny, nz, lz, 1 / 180, -1.0, noise=0.1, seed=34)
    ch, orc = make_pair(g, 1 / 180, -1.0, 2e-5, 1, 1e-12, 100, u, v, w, precision=STP_MIXED, stencils32=st32)
    errs = []
    for n in range(10):
        st = ch.step(1)
        orc.step()
        f = fields(ch)
        errs.append(max(rel_l2(f[k], getattr(orc, k)) for k in ("u", "v", "w", "p")))
        # div u^{n+1} = dt (b - L p) holds in FP64 for the mixed result too
        assert st["max_div"] <= 2e-5 * st["poisson"]["relres"] * st["poisson"]["bnorm"] * 1.001 + 1e-13
    print(f"mixed (stencils32={st32}) error by step", " ".join(f"{e:.2e}" for e in errs))
    assert max(errs) <= 1e-5


def test_bitwise_deterministic(gpu):
    from paper_1511_07800_amd import STP_MIXED
    g = (40, 24, 20, 2.0, 1.2, 2.0)
    nx, ny, nz, lx, ly, lz = g
    u, v, w = inputs.channel_state(nx, ny, nz, lz, 1 / 180, -1.0, noise=0.1, seed=35)
    outs = []
    for _ in range(2):
        ch, _ = make_pair(g, 1 / 180, -1.0, 2e-5, 1, 1e-8, 100, u, v, w, precision=STP_MIXED)
        ch.step(3)
        outs.append(fields(ch))
    for k in outs[0]:
        np.testing.assert_array_equal(outs[0][k], outs[1][k])


@pytest.mark.parametrize("precision", [0, 1])
def test_phase_times_add_up_to_the_step(gpu, precision):
    """The per-phase device times (eddy viscosity, momentum, divergence,
    Poisson guess, Poisson solve, projection) are consecutive event intervals:
    each is non-negative and together they make up ms_total."""
    from paper_1511_07800_amd import Channel
    g = (64, 32, 24, 2.0, 1.2, 2.0)
    nx, ny, nz, lx, ly, lz = g
    u, v, w = inputs.channel_state(nx, ny, nz, lz, 1 / 180, -1.0, noise=0.1, seed=37)
    ch = Channel(nx, ny, nz, lx, ly, lz, nu=1 / 180, dpdx=-1.0, dt=2e-5, les=1, precision=precision,
                 poisson_rtol=1e-8, poisson_maxit=100, proj_depth=4)
    load_state(ch, u, v, w)
    names = ("ms_nut", "ms_momentum", "ms_divergence", "ms_guess", "ms_poisson", "ms_projection")
    for _ in range(4):
        st = ch.step(1)
        parts = [st[k] for k in names]
        print(" ".join(f"{k} {st[k]:.3f}" for k in names), f"total {st['ms_total']:.3f}", flush=True)
        assert min(parts) >= 0.0 and st["ms_poisson"] > 0.0 and st["ms_momentum"] > 0.0
        assert sum(parts) == pytest.approx(st["ms_total"], rel=1e-4, abs=0.02)
    ch.close()


@pytest.mark.parametrize("st32", [0, 1])
def test_field_layouts(gpu, st32):
    """stp_fields describes every field: shape, strides {nx ny, nx, 1}, dtype
    and the staggered position of element [0][0][0] (Sec. 3.1 MAC grid)."""
    from paper_1511_07800_amd import (Channel, STP_MIXED, STP_U, STP_V, STP_W, STP_P, STP_NUT, STP_RHS,
                                      STP_DTYPE_F32, STP_DTYPE_F64)
    nx, ny, nz, lx, ly, lz = 40, 24, 20, 2.0, 1.2, 2.0
    dx, dy, dz = lx / nx, ly / ny, lz / nz
    ch = Channel(nx, ny, nz, lx, ly, lz, nu=1 / 180, dpdx=-1.0, dt=2e-5, les=1, precision=STP_MIXED,
                 stencils32=st32)
    want = {STP_U: (nz, (dz / 2, dy / 2, 0.0)), STP_V: (nz, (dz / 2, 0.0, dx / 2)),
            STP_W: (nz + 1, (0.0, dy / 2, dx / 2)), STP_P: (nz, (dz / 2, dy / 2, dx / 2)),
            STP_NUT: (nz, (dz / 2, dy / 2, dx / 2)), STP_RHS: (nz, (dz / 2, dy / 2, dx / 2))}
    for f, (planes, off) in want.items():
        lay = ch.field_layout(f)
        assert lay["shape"] == (planes, ny, nx), f
        assert lay["strides"] == (nx * ny, nx, 1), f
        assert lay["offset"] == pytest.approx(off, abs=1e-15), f
        assert lay["dtype"] == (STP_DTYPE_F32 if (f == STP_NUT and st32) else STP_DTYPE_F64), f
        assert tuple(ch.field(f).shape) == (planes, ny, nx)
    ch.close()


def test_warm_start_zero_same_solution(gpu):
    g = (40, 24, 20, 2.0, 1.2, 2.0)
    nx, ny, nz, lx, ly, lz = g
    u, v, w = inputs.channel_state(nx, ny, nz, lz, 1 / 180, -1.0, noise=0.1, seed=36)
    ch, orc = make_pair(g, 1 / 180, -1.0, 2e-5, 1, 1e-10, 100, u, v, w, warm=1)
    for _ in range(3):
        st = ch.step(1)
        so = orc.step()
        assert st["poisson"]["cycles"] == so["poisson_cycles"]
    compare(ch, orc, 1e-10)


def test_les_grid_full_size_two_steps(gpu):
    """The 256x128x128 LES grid, 2 steps with one SRJ cycle each: identical
    iteration sequence, all fields within 1e-10 of the oracle."""
    wl = workloads.params("les_channel_256x128x128")
    g = (wl["nx"], wl["ny"], wl["nz"], wl["lx"], wl["ly"], wl["lz"])
    u, v, w = inputs.channel_state(wl["nx"], wl["ny"], wl["nz"], wl["lz"], wl["nu"], wl["dpdx"],
                                   noise=wl["noise"], seed=wl["seed"])
    ch, orc = make_pair(g, wl["nu"], wl["dpdx"], wl["dt"], 1, 0.0, 1, u, v, w)
    for _ in range(2):
        ch.step(1)
        orc.step()
    compare(ch, orc, 1e-10, ("u", "v", "w", "p", "nut", "b"))


def test_bad_config_rejected(gpu):
    from paper_1511_07800_amd import Channel, StpError
    with pytest.raises(StpError):
        Channel(8, 8, 1, 1.0, 1.0, 1.0, nu=0.1, dpdx=-1.0, dt=1e-3)
    with pytest.raises(StpError):
        Channel(8, 8, 8, 1.0, 1.0, 1.0, nu=-0.1, dpdx=-1.0, dt=1e-3)
    with pytest.raises(StpError):
        Channel(8, 8, 8, 1.0, 1.0, 1.0, nu=0.1, dpdx=-1.0, dt=0.0)


def test_mixed_mode_eddy_viscosity_in_fp32(gpu):
    """With stencils32 the mixed mode computes nu_T from FP32 copies of the
    state (u as its departure from the plane means) and keeps it in FP32
    (stp_fields reports the FP32 array): after one step it equals the
    oracle's FP64 nu_T of the starting state to FP32 precision of the strain
    (1e-5 of the largest eddy-viscosity increment), and the step's maximum
    agrees likewise."""
    import torch
    from paper_1511_07800_amd import STP_MIXED, STP_NUT
    g = (48, 32, 24, 2 * math.pi, math.pi, 2.0)
    nx, ny, nz, lx, ly, lz = g
    u, v, w = inputs.channel_state(nx, ny, nz, lz, 1 / 180, -1.0, noise=0.1, seed=37)
    ch, _ = make_pair(g, 1 / 180, -1.0, 2e-5, 1, 0.0, 1, u, v, w, precision=STP_MIXED, stencils32=1)
    st = ch.step(1)
    nut = ch.field(STP_NUT)
    assert nut.dtype == torch.float32
    P = oracle.make_params(nx, ny, nz, lx, ly, lz, nu=1 / 180, dpdx=-1.0, dt=2e-5, les=1)
    ref, mx = oracle.nut(P, u, v, w)
    got = nut.cpu().numpy().astype(np.float64)
    scale = np.abs(ref - 1 / 180).max()
    err = np.abs(got - ref).max() / scale
    print(f"mixed nu_T: max err {err:.2e} of the largest eddy viscosity {scale:.3e}", flush=True)
    assert err <= 1e-5
    assert st["nut_max"] == pytest.approx(mx, rel=1e-6)

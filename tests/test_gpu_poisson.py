"""GPU parity of the relaxation sweeps, the SRJ schedule and the Poisson solve
(Sec. 3.4) against the FP64 oracle, through the C ABI."""
import math

import numpy as np
import pytest

import oracle
from oracle import schedule as osched
from paper_1511_07800_amd import inputs
from _helpers import rel_l2, rel_max, to_dev

pytestmark = pytest.mark.gpu

GRIDS = [(70, 45, 33, 2.0, 1.5, 1.0), (32, 16, 16, 2 * math.pi, math.pi, 2.0), (3, 1, 9, 1.0, 1.0, 1.0),
         (1, 5, 7, 1.0, 1.0, 2.0), (130, 7, 66, 4.0, 0.5, 2.0)]


def channel(g, **kw):
    from paper_1511_07800_amd import Channel
    nx, ny, nz, lx, ly, lz = g
    return Channel(nx, ny, nz, lx, ly, lz, nu=1.0, dpdx=0.0, dt=1.0, **kw)


@pytest.mark.parametrize("g", GRIDS)
@pytest.mark.parametrize("omega", [1.7, 100.0])
def test_single_sweep_fp64(gpu, g, omega):
    import torch
    print(f"sweep fp64 grid={g} omega={omega}", flush=True)
    P = oracle.make_params(*g)
    r = inputs.rng(7)
    p = r.standard_normal((g[2], g[1], g[0]))
    b = r.standard_normal((g[2], g[1], g[0]))
    ref = oracle.srj_sweep(P, omega, p, b)
    ch = channel(g)
    pd = to_dev(torch, p)
    ch.relax(to_dev(torch, b), pd, [omega])
    got = pd.cpu().numpy()
    assert rel_max(got, ref) <= 1e-14 * max(1.0, omega)


@pytest.mark.parametrize("g", GRIDS[:2])
@pytest.mark.parametrize("omega", [1.7, 100.0])
def test_single_sweep_fp32(gpu, g, omega):
    """FP32 sweep on FP32-rounded inputs against the FP64 oracle on the same
    rounded inputs."""
    import torch
    P = oracle.make_params(*g)
    r = inputs.rng(8)
    p = r.standard_normal((g[2], g[1], g[0])).astype(np.float32).astype(np.float64)
    b = r.standard_normal((g[2], g[1], g[0])).astype(np.float32).astype(np.float64)
    ref = oracle.srj_sweep(P, omega, p, b)
    ch = channel(g)
    pd = to_dev(torch, p, torch.float32)
    ch.relax(to_dev(torch, b, torch.float32), pd, [omega])
    got = pd.cpu().double().numpy()
    # increment (omega/D)(L p - b) carries FP32 rounding of terms ~ omega |p|
    assert rel_max(got, ref) <= 2e-6 * max(1.0, omega)


@pytest.mark.parametrize("g", GRIDS)
def test_builtin_schedule_matches_oracle(gpu, g):
    ch = channel(g)
    got = np.array(ch.schedule())
    ref = osched.srj_schedule(*g)
    assert len(got) == len(ref)
    np.testing.assert_allclose(np.sort(got), np.sort(ref), rtol=1e-12)
    np.testing.assert_allclose(got, ref, rtol=1e-12)


def test_sweep_sequence_many(gpu):
    """A whole cycle of sweeps (large weights included) stays within round-off
    of the oracle."""
    import torch
    g = GRIDS[0]
    P = oracle.make_params(*g)
    om = osched.srj_schedule(*g, reduction=1e-2)
    b = inputs.poisson_rhs(g[0], g[1], g[2], seed=9)
    p_ref = np.zeros_like(b)
    for w_ in om:
        p_ref = oracle.srj_sweep(P, w_, p_ref, b)
    ch = channel(g)
    pd = to_dev(torch, np.zeros_like(b))
    ch.relax(to_dev(torch, b), pd, list(om))
    assert rel_l2(pd.cpu().numpy(), p_ref) <= 1e-11


@pytest.mark.parametrize("g", GRIDS)
def test_solve_parity_same_stop_cycle(gpu, g):
    import torch
    print(f"solve fp64 grid={g}", flush=True)
    P = oracle.make_params(*g)
    om = osched.srj_schedule(*g)
    b = inputs.poisson_rhs(g[0], g[1], g[2], seed=10)
    p_ref, st, cyc, r0, r1 = oracle.poisson_srj(P, b, np.zeros_like(b), om, 1e-10, 100)
    assert st == 0
    ch = channel(g, omega=list(om))
    pd = to_dev(torch, np.zeros_like(b))
    stats, rc = ch.poisson_solve(to_dev(torch, b), pd, 1e-10, 100)
    assert rc == 0 and stats["cycles"] == cyc
    assert stats["relres"] == pytest.approx(r1, rel=1e-6)
    assert rel_l2(pd.cpu().numpy(), p_ref) <= 1e-10


def test_solve_fixed_cycles_and_warm_start(gpu):
    import torch
    g = GRIDS[1]
    P = oracle.make_params(*g)
    om = osched.srj_schedule(*g)
    b = inputs.poisson_rhs(g[0], g[1], g[2], seed=13)
    p0 = inputs.rng(14).standard_normal(b.shape)
    p_ref, st, cyc, r0, r1 = oracle.poisson_srj(P, b, p0, om, 0.0, 2)
    ch = channel(g, omega=list(om))
    pd = to_dev(torch, p0)
    stats, rc = ch.poisson_solve(to_dev(torch, b), pd, 0.0, 2)
    assert rc == 0 and stats["cycles"] == 2
    assert rel_l2(pd.cpu().numpy(), p_ref) <= 1e-10
    assert abs(pd.cpu().numpy().mean()) < 1e-13


def test_degenerate_rhs(gpu):
    """b = 0: converged before any cycle, p keeps its (mean-free) value."""
    import torch
    g = GRIDS[1]
    ch = channel(g)
    z = np.zeros((g[2], g[1], g[0]))
    pd = to_dev(torch, z)
    stats, rc = ch.poisson_solve(to_dev(torch, z), pd, 1e-10, 5)
    assert rc == 0 and stats["cycles"] == 0 and not pd.cpu().numpy().any()


def test_not_converged_and_nan(gpu):
    from paper_1511_07800_amd import STP_ENOCONV, STP_ENAN
    import torch
    g = GRIDS[1]
    ch = channel(g)
    b = inputs.poisson_rhs(g[0], g[1], g[2], seed=15)
    pd = to_dev(torch, np.zeros_like(b))
    stats, rc = ch.poisson_solve(to_dev(torch, b), pd, 1e-14, 1, allow=(STP_ENOCONV,))
    assert rc == STP_ENOCONV and stats["cycles"] == 1 and stats["relres"] < stats["relres0"]
    bn = b.copy()
    bn[3, 2, 1] = np.nan
    pd = to_dev(torch, np.zeros_like(b))
    stats, rc = ch.poisson_solve(to_dev(torch, bn), pd, 1e-10, 3, allow=(STP_ENAN,))
    assert rc == STP_ENAN


@pytest.mark.parametrize("g", GRIDS[:2])
def test_residual_norm(gpu, g):
    import torch
    P = oracle.make_params(*g)
    r = inputs.rng(16)
    p = r.standard_normal((g[2], g[1], g[0]))
    b = r.standard_normal((g[2], g[1], g[0]))
    _, s2 = oracle.residual(P, p, b)
    ch = channel(g)
    got = ch.residual_norm(to_dev(torch, b), to_dev(torch, p))
    assert got == pytest.approx(math.sqrt(s2), rel=1e-12)


@pytest.mark.parametrize("rhs16", [0, 1])
@pytest.mark.parametrize("g", GRIDS[:2] + [GRIDS[4]])
def test_mixed_solve_against_fp64_oracle(gpu, g, rhs16):
    """FP32 sweeps inside the FP64 defect correction reach the FP64 residual
    test (also with each pass's right-hand side stored in FP16); the solution
    matches the FP64 oracle within 1e-5."""
    import torch
    from paper_1511_07800_amd import STP_MIXED
    P = oracle.make_params(*g)
    om = osched.srj_schedule(*g)
    b = inputs.poisson_rhs(g[0], g[1], g[2], seed=17)
    p_ref, st, *_ = oracle.poisson_srj(P, b, np.zeros_like(b), om, 1e-12, 100)
    ch = channel(g, precision=STP_MIXED, mixed_rhs16=rhs16)
    pd = to_dev(torch, np.zeros_like(b))
    stats, rc = ch.poisson_solve(to_dev(torch, b), pd, 1e-10, 50)
    assert rc == 0 and stats["relres"] <= 1e-10
    err = rel_l2(pd.cpu().numpy(), p_ref)
    print(f"mixed solve grid={g} rhs16={rhs16} outer={stats['outer']} rel_l2={err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("rhs16", [0, 1])
def test_mixed_solve_scales_with_the_right_hand_side(gpu, rhs16):
    """The mixed solve's FP32 (and FP16) passes read a power-of-two multiple
    of the residual brought to about unit rms, so scaling b by a power of two
    scales the whole solve exactly: with b times 2^-400 (far below FP32's
    normal range) or 2^300 (above it) the solution is the unscaled one times
    the same factor, bit for bit, after the same passes and sweeps; with b
    times 1e-36 and 1e30 the solve still meets the tolerance, and its
    solution differs from the unscaled one by no more than two solutions of
    relative residual 1e-8 can (2e-8 / kappa_min relative)."""
    import torch
    from paper_1511_07800_amd import STP_MIXED
    g = (96, 40, 24, 4.0, 2.0, 2.0)
    kmin, _ = osched.kappa_bounds(*g)
    b = torch.from_numpy(inputs.poisson_rhs(g[0], g[1], g[2], seed=19)).cuda()
    ch = channel(g, precision=STP_MIXED, mixed_rhs16=rhs16, srj_adaptive=1, srj_reduction=1e-4)
    p_ref = torch.zeros_like(b)
    st_ref, rc = ch.poisson_solve(b, p_ref, 1e-8, 50)
    assert rc == 0 and st_ref["relres"] <= 1e-8
    for k in (-400, 300):
        f = math.ldexp(1.0, k)
        p = torch.zeros_like(b)
        st, rc = ch.poisson_solve(b * f, p, 1e-8, 50)
        print(f"rhs16={rhs16} b*2^{k}: passes {st['outer']} sweeps {st['sweeps']} relres {st['relres']:.2e}",
              flush=True)
        assert rc == 0 and st["sweeps"] == st_ref["sweeps"] and st["outer"] == st_ref["outer"]
        assert torch.equal(p * math.ldexp(1.0, -k), p_ref)
    for f in (1e-36, 1e30):
        p = torch.zeros_like(b)
        st, rc = ch.poisson_solve(b * f, p, 1e-8, 50)
        err = float((p / f - p_ref).norm() / p_ref.norm())
        print(f"rhs16={rhs16} b*{f:g}: passes {st['outer']} relres {st['relres']:.2e} rel_l2 {err:.2e}", flush=True)
        assert rc == 0 and st["relres"] <= 1e-8 and err <= 2e-8 / kmin
    ch.close()


FULL = {512: (512, 256, 192, 4 * math.pi, 2 * math.pi, 2.0), 1024: (1024, 512, 384, 4 * math.pi, 2 * math.pi, 2.0)}


@pytest.mark.parametrize("size", [512, 1024])
@pytest.mark.parametrize("dtype", ["f64", "f32", "f16rhs"])
def test_full_size_sweep_sampled(gpu, dtype, size):
    """One sweep at the 512x256x192 LES grid and at the largest one
    (1024x512x384, 2e8 cells), checked on about 4000 sampled cells (walls,
    seams and interior) against the oracle's pointwise formula."""
    import torch
    g = FULL[size]
    print(f"full-size sweep {g[:3]} {dtype}", flush=True)
    nx, ny, nz = g[:3]
    P = oracle.make_params(*g)
    r = inputs.rng(18)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    bdt = torch.float16 if dtype == "f16rhs" else tdt
    p = r.standard_normal((nz, ny, nx))
    b = r.standard_normal((nz, ny, nx))
    if dtype != "f64":
        p = p.astype(np.float32).astype(np.float64)
        b = b.astype(np.float16 if dtype == "f16rhs" else np.float32).astype(np.float64)
    omega = 37.5
    ch = channel(g)
    pd = to_dev(torch, p, tdt)
    ch.relax(to_dev(torch, b, bdt), pd, [omega])
    got = pd.cpu().double().numpy().ravel()
    n = nx * ny * nz
    plane = nx * ny
    cells = np.concatenate([r.integers(0, n, 3000), np.arange(0, plane, 997), n - plane + np.arange(0, plane, 991),
                            np.arange(nx - 1, n, nx * 37)[:300], np.arange(0, n, nx * ny * 7 + nx - 1)[:200]])
    ref = oracle.srj_sweep_at(P, omega, p, b, cells)
    tol = 1e-14 if dtype == "f64" else 2e-6
    assert rel_max(got[cells], ref) <= tol * omega


@pytest.mark.parametrize("g", [(70, 45, 33, 2.0, 1.5, 1.0), (130, 64, 40, 4.0, 2.0, 2.0), (64, 32, 5, 1.0, 1.0, 1.0),
                               (130, 70, 40, 4.0, 2.0, 2.0), (121, 131, 21, 2.0, 2.0, 1.0)])
@pytest.mark.parametrize("dtype", ["f64", "f32", "f16rhs"])
@pytest.mark.parametrize("nt", [2, 3, 4, 5])
def test_fused_sweeps_equal_single_sweeps_bitwise(gpu, g, dtype, nt):
    """NT sweeps fused into one launch (LDS tile, z-march) reproduce NT single
    sweeps bit for bit, including ragged tiles, the periodic seams and the
    walls; 2 NT + 1 sweeps also run a shorter remainder launch (FP64 fuses at
    most 4).  The last two grids (ny >= 66) run five FP32 sweeps on the tall
    16-wavefront tiles, with ragged last tiles in x and y."""
    import torch
    print(f"fused grid={g} dtype={dtype} nt={nt}", flush=True)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    r = inputs.rng(19)
    p = to_dev(torch, r.standard_normal((g[2], g[1], g[0])), tdt)
    b = to_dev(torch, r.standard_normal((g[2], g[1], g[0])), torch.float16 if dtype == "f16rhs" else tdt)
    om = [1.3, 57.0, 0.6, 3.1, 11.0, 0.9, 2.2, 40.0, 0.7, 5.5, 1.9, 23.0, 1.1][: 2 * nt + 1]
    ch1 = channel(g, tblock=1)
    chf = channel(g, tblock=nt)
    p1 = p.clone()
    pf = p.clone()
    ch1.relax(b, p1, om)
    chf.relax(b, pf, om)
    torch.cuda.synchronize()
    assert torch.equal(p1, pf)


@pytest.mark.parametrize("dtype,nt,size", [("f32", 4, 512), ("f32", 5, 512), ("f64", 4, 512), ("f32", 4, 1024),
                                           ("f16rhs", 4, 512), ("f16rhs", 5, 512), ("f32", 5, 1024),
                                           ("f16rhs", 5, 1024)])
def test_fused_sweeps_full_size_bitwise(gpu, dtype, nt, size):
    """The fused launch at the benchmark grid (512x256x192, the launch
    configuration the bench times: several z-chunks per tile column, ragged
    last tiles in x and y) and at the largest grid equals single sweeps bit
    for bit; single sweeps at these sizes are checked against the oracle in
    test_full_size_sweep_sampled."""
    import torch
    g = FULL[size]
    print(f"fused full size {g[:3]} dtype={dtype} nt={nt}", flush=True)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    r = inputs.rng(23)
    p = to_dev(torch, r.standard_normal((g[2], g[1], g[0])), tdt)
    b = to_dev(torch, r.standard_normal((g[2], g[1], g[0])), torch.float16 if dtype == "f16rhs" else tdt)
    om = [1.3, 57.0, 0.6, 3.1, 11.0, 0.9, 2.2, 40.0, 0.7, 5.5, 1.9, 23.0][: 2 * nt]
    p1, pf = p.clone(), p.clone()
    channel(g, tblock=1).relax(b, p1, om)
    channel(g, tblock=nt).relax(b, pf, om)
    torch.cuda.synchronize()
    assert torch.equal(p1, pf)


@pytest.mark.parametrize("precision", [0, 1])
def test_solve_with_fused_sweeps_bitwise(gpu, precision):
    import torch
    g = (96, 40, 24, 4.0, 2.0, 2.0)
    b = to_dev(torch, inputs.poisson_rhs(g[0], g[1], g[2], seed=20))
    out = []
    for tb in (1, 4):
        ch = channel(g, tblock=tb, precision=precision)
        pd = torch.zeros_like(b)
        stats, rc = ch.poisson_solve(b, pd, 1e-10, 100)
        assert rc == 0
        out.append((stats["cycles"], pd.cpu()))
    assert out[0][0] == out[1][0]
    assert torch.equal(out[0][1], out[1][1])


@pytest.mark.parametrize("g,depth", [((130, 70, 40, 4.0, 2.0, 2.0), 5), ((96, 40, 24, 4.0, 2.0, 2.0), 4),
                                     ((40, 24, 20, 2.0, 1.2, 2.0), 1)])
def test_automatic_fusion_depth(gpu, g, depth):
    """tblock = 0: the mixed solve's FP32 sweeps fuse five per launch where the
    tall tiles fit (ny >= 66), four on a narrower grid whose launch fits one
    round of resident workgroups, one where no tile fits; the result equals
    single sweeps bitwise."""
    import torch
    b = to_dev(torch, inputs.poisson_rhs(g[0], g[1], g[2], seed=21))
    out = []
    for tb in (0, 1):
        ch = channel(g, tblock=tb, precision=1)
        pd = torch.zeros_like(b)
        stats, rc = ch.poisson_solve(b, pd, 1e-10, 100)
        assert rc == 0
        out.append((stats, pd.cpu()))
    st = out[0][0]
    print(f"auto depth {g[:3]}: {st['sweeps']} sweeps in {st['launches']} launches", flush=True)
    assert -(-st["sweeps"] // st["launches"]) == depth
    assert out[1][0]["launches"] == out[1][0]["sweeps"]
    assert torch.equal(out[0][1], out[1][1])


@pytest.mark.parametrize("g", [GRIDS[0], GRIDS[1], (96, 40, 24, 4.0, 2.0, 2.0)])
def test_adaptive_solve_matches_oracle(gpu, g):
    """Cycles sized from the reduction still needed: same cycles and sweeps as
    the oracle's adaptive solve, solution within 1e-10."""
    import torch
    P = oracle.make_params(*g)
    b = inputs.poisson_rhs(g[0], g[1], g[2], seed=22)
    p0 = 0.1 * inputs.rng(23).standard_normal(b.shape)
    p_ref, st, cyc, sweeps, r0, r1 = oracle.poisson_srj_adaptive(P, b, p0, 1e-10, 20)
    ch = channel(g, srj_adaptive=1)
    pd = to_dev(torch, p0)
    stats, rc = ch.poisson_solve(to_dev(torch, b), pd, 1e-10, 20)
    assert rc == 0 and st == 0
    assert stats["cycles"] == cyc and stats["sweeps"] == sweeps
    assert rel_l2(pd.cpu().numpy(), p_ref) <= 1e-10


def test_adaptive_mixed_solve_reaches_tolerance(gpu):
    import torch
    from paper_1511_07800_amd import STP_MIXED
    g = (130, 64, 40, 4.0, 2.0, 2.0)
    P = oracle.make_params(*g)
    om = osched.srj_schedule(*g)
    b = inputs.poisson_rhs(g[0], g[1], g[2], seed=24)
    p_ref, *_ = oracle.poisson_srj(P, b, np.zeros_like(b), om, 1e-12, 100)
    fixed = channel(g, precision=STP_MIXED)
    adapt = channel(g, precision=STP_MIXED, srj_adaptive=1)
    out = {}
    for name, ch in (("fixed", fixed), ("adaptive", adapt)):
        pd = torch.zeros_like(to_dev(torch, b))
        stats, rc = ch.poisson_solve(to_dev(torch, b), pd, 1e-9, 50)
        assert rc == 0 and stats["relres"] <= 1e-9
        assert rel_l2(pd.cpu().numpy(), p_ref) <= 1e-5
        out[name] = stats["sweeps"]
    print("mixed sweeps to 1e-9:", out)
    # cycle degrees are rounded up to multiples of 16: allow that slack on a small grid
    assert out["adaptive"] <= 1.1 * out["fixed"]

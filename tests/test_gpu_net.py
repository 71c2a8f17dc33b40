"""GPU parity of the learned warm-start network (BF16 MFMA kernels, FP32
accumulation) against the FP64 oracle that rounds to bfloat16 at the same
points, through the C ABI: forward output, loss, every parameter gradient
(relative L2 <= 2e-3 and cosine >= 0.9999; BF16 x BF16 products are exact in
FP32, so the two differ by accumulation order and the re-rounding it can
flip), Adam updates, the coarse-correction proposal, and the warm start
inside a time step."""
import math

import numpy as np
import pytest

import oracle
from oracle import net as onet
from paper_1511_07800_amd import inputs
from _helpers import rel_l2, to_dev, load_state
from _net import to_flat, from_flat, padding_is_zero

pytestmark = pytest.mark.gpu

GRIDS = [(16, 16, 16, 2.0, 2.0, 2.0), (32, 16, 12, 4.0, 2.0, 2.0), (24, 20, 8, 3.0, 2.0, 1.0)]


def make(g, seed=0):
    from paper_1511_07800_amd import Channel
    nx, ny, nz, lx, ly, lz = g
    ch = Channel(nx, ny, nz, lx, ly, lz, nu=1.0, dpdx=0.0, dt=1.0)
    ch.net_init(training=True, seed=seed)
    layout = ch.net_layout()
    params, grads = ch.net_params()
    return ch, layout, params, grads


def sample(g, seed):
    nx, ny, nz = g[:3]
    r = inputs.rng(seed)
    b = r.standard_normal((nz, ny, nx))
    b -= b.mean()
    p_prev = 0.3 + r.standard_normal((nz, ny, nx))
    p_next = p_prev + 0.1 * r.standard_normal((nz, ny, nx))
    return b, p_prev, p_next


def upload(ch, params_dev, p, layout):
    import torch
    params_dev.copy_(torch.from_numpy(to_flat(p, layout, params_dev.numel())))
    ch.net_sync()


def cosine(a, b):
    return float(np.vdot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))


@pytest.mark.parametrize("g", GRIDS)
def test_forward_matches_oracle(gpu, g):
    import torch
    print(f"net forward grid={g}", flush=True)
    ch, layout, params, _ = make(g)
    p = onet.init_params(seed=5)
    r = inputs.rng(6)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.05 * r.standard_normal(p[k].shape)
    upload(ch, params, p, layout)
    b, p_prev, _ = sample(g, 7)
    P = oracle.make_params(*g)
    ref = onet.predict(p, b, p_prev, oracle.lap_p(P, p_prev), oracle.diag_d(P), round_bf16=True)
    out = torch.zeros_like(to_dev(torch, b))
    ch.net_predict(to_dev(torch, b), to_dev(torch, p_prev), out)
    got = out.cpu().numpy()
    err = rel_l2(got - p_prev, ref - p_prev)
    cos = cosine((got - p_prev).ravel(), (ref - p_prev).ravel())
    print(f"  increment rel_l2 {err:.2e}, cos {cos:.8f}")
    assert err <= 2e-3 and cos >= 0.9999


@pytest.mark.parametrize("g", GRIDS)
def test_gradients_match_oracle(gpu, g):
    import torch
    print(f"net gradients grid={g}", flush=True)
    ch, layout, params, grads = make(g)
    p = onet.init_params(seed=8)
    r = inputs.rng(9)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.05 * r.standard_normal(p[k].shape)
    upload(ch, params, p, layout)
    b, p_prev, p_next = sample(g, 10)
    P = oracle.make_params(*g)
    x, s = onet.normalise(b, p_prev, oracle.lap_p(P, p_prev), oracle.diag_d(P))
    loss_ref, g_ref, _ = onet.loss_and_grads(p, x, (p_next - p_prev) / s, round_bf16=True)
    loss = ch.net_train_step(to_dev(torch, b), to_dev(torch, p_prev), to_dev(torch, p_next), 0.0)
    assert loss == pytest.approx(loss_ref, rel=2e-3)
    got = from_flat(grads.cpu().numpy(), layout)
    for k in g_ref:
        e = rel_l2(got[k], g_ref[k])
        c = cosine(got[k].ravel(), g_ref[k].ravel())
        print(f"  {k}: rel_l2 {e:.2e} cos {c:.8f}")
        assert e <= 2e-3 and c >= 0.9999, k
    # weights untouched with lr = 0, padding stays zero
    assert padding_is_zero(grads.cpu().numpy(), layout)
    np.testing.assert_array_equal(params.cpu().numpy(), to_flat(p, layout, params.numel()))


def test_adam_steps_match_oracle_and_reduce_loss(gpu):
    import torch
    g = GRIDS[0]
    ch, layout, params, grads = make(g)
    p = onet.init_params(seed=11)
    upload(ch, params, p, layout)
    b, p_prev, p_next = sample(g, 12)
    P = oracle.make_params(*g)
    x, s = onet.normalise(b, p_prev, oracle.lap_p(P, p_prev), oracle.diag_d(P))
    t = (p_next - p_prev) / s
    state = {}
    pr = {k: v.copy() for k, v in p.items()}
    losses = []
    bd, pd, nd = to_dev(torch, b), to_dev(torch, p_prev), to_dev(torch, p_next)
    for it in range(5):
        losses.append(ch.net_train_step(bd, pd, nd, 1e-3))
        _, gr, _ = onet.loss_and_grads(pr, x, t, round_bf16=True)
        pr = onet.adam_step(pr, gr, state, 1e-3)
    got = from_flat(params.cpu().numpy(), layout)
    for k in pr:
        # Adam moves each weight by about lr per step; compare the update
        d_ref = pr[k] - p[k]
        d_got = got[k] - p[k]
        assert rel_l2(d_got, d_ref) <= 5e-2, k
    assert losses[-1] < losses[0]
    assert padding_is_zero(params.cpu().numpy(), layout)


def test_inference_forward_equals_training_forward(gpu):
    """Inference reads the decoder's upsampled inputs straight from the coarse
    tensors; training also materialises them for the weight gradient.  Both
    forwards give the same guess, bit for bit, on a grid with several tiles,
    ragged edges and several z-chunks per tile column."""
    import torch
    g = (104, 72, 40, 4.0, 3.0, 2.0)
    print(f"net inference vs training grid={g}", flush=True)
    p = onet.init_params(seed=9)
    r = inputs.rng(10)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.05 * r.standard_normal(p[k].shape)
    b, p_prev, _ = sample(g, 11)
    outs = []
    for training in (True, False):
        from paper_1511_07800_amd import Channel
        ch = Channel(*g[:3], *g[3:], nu=1.0, dpdx=0.0, dt=1.0)
        ch.net_init(training=training, seed=0)
        params, _ = ch.net_params()
        upload(ch, params, p, ch.net_layout())
        out = torch.zeros_like(to_dev(torch, b))
        ch.net_predict(to_dev(torch, b), to_dev(torch, p_prev), out)
        torch.cuda.synchronize()
        outs.append(out.cpu())
    assert torch.equal(outs[0], outs[1])
    assert float((outs[0] - torch.from_numpy(p_prev)).abs().max()) > 0


def test_learned_warm_start_in_step(gpu):
    """STP_WS_LEARNED: the step still reaches the residual target; the guess
    is used only when its residual is smaller than that of p^n."""
    import torch
    from paper_1511_07800_amd import Channel, STP_WS_LEARNED
    nx, ny, nz, lx, ly, lz = 32, 16, 16, 2 * math.pi, math.pi, 2.0
    u, v, w = inputs.channel_state(nx, ny, nz, lz, 1 / 180, -1.0, noise=0.1, seed=40)
    ch = Channel(nx, ny, nz, lx, ly, lz, nu=1 / 180, dpdx=-1.0, dt=2e-5, les=1, warm_start=STP_WS_LEARNED,
                 poisson_rtol=1e-8, poisson_maxit=100)
    ch.net_init(training=False, seed=3)
    load_state(ch, u, v, w)
    for _ in range(3):
        st = ch.step(1)
        assert st["poisson"]["relres"] <= 1e-8
        assert st["learned_used"] == (st["relres_learned"] < st["relres_prev"])
        assert st["ms_net"] > 0


def test_nan_weights_fall_back_to_plain_solve(gpu):
    """A network with NaN weights: its warm start and its coarse corrections
    are rejected by their residuals, and the steps equal those of the solver
    without the network bit for bit (mixed precision)."""
    import torch
    from paper_1511_07800_amd import Channel, STP_WS_LEARNED, STP_WS_PREV, STP_MIXED
    nx, ny, nz, lx, ly, lz = 32, 16, 16, 2 * math.pi, math.pi, 2.0
    u, v, w = inputs.channel_state(nx, ny, nz, lz, 1 / 180, -1.0, noise=0.1, seed=41)
    out = []
    for learned in (False, True):
        ch = Channel(nx, ny, nz, lx, ly, lz, nu=1 / 180, dpdx=-1.0, dt=2e-5, les=1, precision=STP_MIXED,
                     warm_start=STP_WS_LEARNED if learned else STP_WS_PREV, learned_correction=int(learned),
                     poisson_rtol=1e-8, poisson_maxit=100, srj_adaptive=1)
        if learned:
            ch.net_init(training=False, seed=3)
            params, _ = ch.net_params()
            params.fill_(float("nan"))
            ch.net_sync()
        load_state(ch, u, v, w)
        for _ in range(3):
            st = ch.step(1)
            assert st["poisson"]["relres"] <= 1e-8
            if learned:
                assert st["learned_used"] == 0 and st["poisson"]["corrections"] == 0
                assert not math.isfinite(st["relres_learned"])
        out.append([ch.field(k).clone() for k in range(4)])
        ch.close()
    for name, a, b in zip("uvwp", out[0], out[1]):
        assert torch.equal(a, b), name


# several k_conv_march tiles, ragged tile edges and several z-chunks at every
# level: 136 x 72 x 64, 68 x 36 x 32 and 34 x 18 x 16 against 32 x 16 (and
# 32 x 8) tiles and chunks of at least 8 planes
GRID_MULTI = (136, 72, 64, 4.0, 2.0, 2.0)


def test_forward_loss_gradients_multi_tile(gpu):
    """Forward increment, loss and every parameter gradient on a grid whose
    every level spans several tiles and z-chunks: relative L2 <= 2e-3 and
    cosine >= 0.9999 against the oracle rounding to BF16 at the same points."""
    import torch
    g = GRID_MULTI
    print(f"net multi-tile grid={g[:3]}", flush=True)
    ch, layout, params, grads = make(g)
    p = onet.init_params(seed=21)
    r = inputs.rng(22)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.05 * r.standard_normal(p[k].shape)
    upload(ch, params, p, layout)
    b, p_prev, p_next = sample(g, 23)
    P = oracle.make_params(*g)
    lap = oracle.lap_p(P, p_prev)
    ref = onet.predict(p, b, p_prev, lap, oracle.diag_d(P), round_bf16=True)
    out = torch.zeros_like(to_dev(torch, b))
    ch.net_predict(to_dev(torch, b), to_dev(torch, p_prev), out)
    got = out.cpu().numpy()
    e, c = rel_l2(got - p_prev, ref - p_prev), cosine((got - p_prev).ravel(), (ref - p_prev).ravel())
    print(f"  forward increment rel_l2 {e:.2e} cos {c:.8f}", flush=True)
    assert e <= 2e-3 and c >= 0.9999
    x, s = onet.normalise(b, p_prev, lap, oracle.diag_d(P))
    loss_ref, g_ref, _ = onet.loss_and_grads(p, x, (p_next - p_prev) / s, round_bf16=True)
    loss = ch.net_train_step(to_dev(torch, b), to_dev(torch, p_prev), to_dev(torch, p_next), 0.0)
    print(f"  loss {loss:.8e} oracle {loss_ref:.8e}", flush=True)
    assert loss == pytest.approx(loss_ref, rel=2e-3)
    got_g = from_flat(grads.cpu().numpy(), layout)
    worst = []
    for k in g_ref:
        e = rel_l2(got_g[k], g_ref[k])
        c = cosine(got_g[k].ravel(), g_ref[k].ravel())
        print(f"  {k}: rel_l2 {e:.2e} cos {c:.8f}", flush=True)
        worst.append((k, e, c))
    for k, e, c in worst:
        assert e <= 2e-3 and c >= 0.9999, (k, e, c)


def test_coarse_correction_proposal_matches_oracle(gpu):
    """The learned coarse correction's proposal p + s_r y(r, p), taken on an
    intermediate iterate of a mixed solve (one FP32 defect-correction pass of
    an LES step's Poisson problem, with the shipped weights), against the
    oracle network's proposal for the same iterate: the increments agree to
    2e-3 relative L2 (cosine 0.9999), and so do their FP64 residual norms."""
    import os
    import torch
    from paper_1511_07800_amd import Channel, STP_MIXED, STP_ENOCONV, STP_P, STP_RHS, warmstart
    g = (128, 64, 48, 4 * math.pi, 2 * math.pi, 2.0)
    nx, ny, nz, lx, ly, lz = g
    u, v, w = inputs.channel_state(nx, ny, nz, lz, 1 / 180, -1.0, noise=0.1, seed=61)
    ch = Channel(*g, nu=1 / 180, dpdx=-1.0, dt=4e-5, les=1, precision=STP_MIXED, poisson_rtol=1e-8,
                 poisson_maxit=100, srj_adaptive=1, srj_reduction=1e-4)
    ch.net_init(training=False)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    warmstart.load_weights(ch, os.path.join(root, "paper_1511_07800_amd", "weights", "warmstart_les512_all.npy"))
    load_state(ch, u, v, w)
    ch.step(2)
    p_prev = ch.field(STP_P).clone()
    ch.step(1)
    b = ch.field(STP_RHS).clone()
    p_it = p_prev.clone()
    st, rc = ch.poisson_solve(b, p_it, 1e-12, 1, allow=(STP_ENOCONV,))
    assert rc == STP_ENOCONV and st["outer"] == 1
    prop = torch.zeros_like(b)
    ch.net_predict(b, p_it, prop)
    r_gpu = ch.residual_norm(b, prop)
    params, _ = ch.net_params()
    pw = from_flat(params.cpu().numpy(), ch.net_layout())
    P = oracle.make_params(*g)
    bn, pn = b.cpu().numpy(), p_it.cpu().numpy()
    ref = onet.predict(pw, bn, pn, oracle.lap_p(P, pn), oracle.diag_d(P), round_bf16=True)
    got = prop.cpu().numpy()
    e, c = rel_l2(got - pn, ref - pn), cosine((got - pn).ravel(), (ref - pn).ravel())
    r_ref = math.sqrt(oracle.residual(P, ref, bn)[1])
    r_it = math.sqrt(oracle.residual(P, pn, bn)[1])
    print(f"proposal: increment rel_l2 {e:.2e} cos {c:.8f}; residual of the iterate {r_it:.4e}, "
          f"of the proposal {r_gpu:.4e} (oracle {r_ref:.4e})", flush=True)
    assert e <= 2e-3 and c >= 0.9999
    assert r_gpu == pytest.approx(r_ref, rel=2e-3)
    ch.close()

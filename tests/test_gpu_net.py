"""GPU parity of the learned warm-start network (BF16 MFMA kernels, FP32
accumulation) against the FP64 oracle that rounds to bfloat16 at the same
points, through the C ABI: forward output, loss, every parameter gradient,
Adam updates, and the warm start inside a time step."""
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
    print(f"  increment rel_l2 {err:.2e}, cos {cosine(got - p_prev, ref - p_prev):.6f}")
    assert err <= 5e-3


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
    assert loss == pytest.approx(loss_ref, rel=5e-3)
    got = from_flat(grads.cpu().numpy(), layout)
    for k in g_ref:
        e = rel_l2(got[k], g_ref[k])
        c = cosine(got[k].ravel(), g_ref[k].ravel())
        print(f"  {k}: rel_l2 {e:.2e} cos {c:.6f}")
        assert e <= 2e-2 and c >= 0.999, k
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

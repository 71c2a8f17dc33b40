"""What the trained warm-start network gains over starting the relaxation
from p^n, at the same residual (the relaxation judges the guess)."""
import numpy as np
import pytest

from paper_1511_07800_amd import workloads, warmstart, STP_MIXED, STP_WS_PREV, STP_WS_LEARNED

pytestmark = pytest.mark.gpu


def test_trained_network_saves_sweeps_on_unseen_flow(gpu):
    """The committed network (trained on 256x128x128 LES triples from seed
    7800) on a flow it has not seen (seed 9100): after 20 warm-up steps, 20
    steps each from p^n and from the learned guess, same rtol 1e-8."""
    wl = workloads.params("les_channel_256x128x128")
    res = {}
    for ws in (STP_WS_PREV, STP_WS_LEARNED):
        ch = warmstart.make_channel(wl, STP_MIXED, 1e-8, warm_start=ws, seed=9100)
        if ws == STP_WS_LEARNED:
            ch.net_init(training=False)
            warmstart.load_weights(ch)
        ch.step(20)
        sweeps, rp, rl, used = [], [], [], []
        for _ in range(20):
            st = ch.step(1)
            assert st["poisson"]["relres"] <= 1e-8
            sweeps.append(st["poisson"]["sweeps"])
            if ws == STP_WS_LEARNED:
                rp.append(st["relres_prev"])
                rl.append(st["relres_learned"])
                used.append(st["learned_used"])
        res[ws] = dict(sweeps=np.mean(sweeps), relres_prev=np.mean(rp) if rp else None,
                       relres_net=np.mean(rl) if rl else None, used=np.mean(used) if used else None)
        ch.close()
    print("gain:", res)
    assert res[STP_WS_LEARNED]["relres_net"] < 0.5 * res[STP_WS_LEARNED]["relres_prev"]
    assert res[STP_WS_LEARNED]["sweeps"] < res[STP_WS_PREV]["sweeps"]


def test_learned_coarse_correction_saves_sweeps(gpu):
    """The same network used as a coarse correction between the mixed
    solve's defect-correction passes: each proposal is kept only when it
    lowers the FP64 residual, the stop test is unchanged, and fewer sweeps
    reach it than with the warm start alone."""
    wl = workloads.params("les_channel_256x128x128")
    res = {}
    for corr in (0, 1):
        ch = warmstart.make_channel(wl, STP_MIXED, 1e-8, warm_start=STP_WS_LEARNED, seed=9100,
                                    learned_correction=corr)
        ch.net_init(training=False)
        warmstart.load_weights(ch)
        ch.step(20)
        sweeps, kept = [], []
        for _ in range(10):
            st = ch.step(1)
            assert st["poisson"]["relres"] <= 1e-8
            sweeps.append(st["poisson"]["sweeps"])
            kept.append(st["poisson"]["corrections"])
        res[corr] = dict(sweeps=np.mean(sweeps), corrections=np.mean(kept))
        ch.close()
    print("coarse correction:", res)
    assert res[0]["corrections"] == 0
    assert res[1]["corrections"] >= 1
    assert res[1]["sweeps"] < res[0]["sweeps"]


def test_training_from_scratch_improves_guess(gpu):
    """Train a fresh network on a small LES (64x32x32) with the project's own
    kernels; on held-out later steps its guess beats p^n."""
    wl = dict(workloads.params("les_channel_256x128x128"))
    wl.update(nx=64, ny=32, nz=32, seed=1234)
    ch = warmstart.make_channel(wl, STP_MIXED, 1e-8)
    ch.net_init(training=True, seed=2)
    pairs = warmstart.generate_pairs(ch, 160, 2, skip=10, log=lambda s: None)
    train, held = pairs[:60], pairs[60:]
    before = warmstart.guess_quality(ch, held)
    hist = warmstart.train(ch, train, 15, 2e-3, log=print)
    after = warmstart.guess_quality(ch, held)
    rp = np.mean([q["relres_prev"] for q in after])
    rn0 = np.mean([q["relres_net"] for q in before])
    rn = np.mean([q["relres_net"] for q in after])
    print(f"held-out relres: p^n {rp:.3e}, untrained net {rn0:.3e}, trained net {rn:.3e}; loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    assert hist[-1] < hist[0]
    assert rn < rp


def test_network_gains_over_least_squares_guess_on_unseen_flow(gpu):
    """The shipped 512x256x192 weights on the top of the least-squares guess
    over the last 8 solutions, on a flow they have not seen (seed 9101):
    after 16 warm-up steps, 8 steps each with and without the network, same
    rtol 1e-8.  The network must lower the starting residual of the strongest
    guess without it, and the sweeps."""
    import os
    wl = workloads.params("les_channel_512x256x192")
    wts = os.path.join(os.path.dirname(warmstart.__file__), "weights", "warmstart_les512_all.npy")
    res = {}
    for ws in (STP_WS_PREV, STP_WS_LEARNED):
        from paper_1511_07800_amd import Channel
        ch = Channel(wl["nx"], wl["ny"], wl["nz"], wl["lx"], wl["ly"], wl["lz"], nu=wl["nu"], dpdx=wl["dpdx"],
                     dt=wl["dt"], les=1, precision=STP_MIXED, poisson_rtol=1e-8, poisson_maxit=200, srj_adaptive=1,
                     srj_reduction=wl["srj_reduction"], warm_start=ws, proj_depth=8)
        import torch
        from paper_1511_07800_amd import inputs
        u, v, w = inputs.channel_state(wl["nx"], wl["ny"], wl["nz"], wl["lz"], wl["nu"], wl["dpdx"],
                                       noise=wl["noise"], seed=9101)
        for k, a in enumerate((u, v, w)):
            ch.field(k).copy_(torch.from_numpy(a))
        if ws == STP_WS_LEARNED:
            ch.net_init(training=False)
            warmstart.load_weights(ch, wts)
        ch.step(16)
        sweeps, r0 = [], []
        for _ in range(8):
            st = ch.step(1)
            assert st["poisson"]["relres"] <= 1e-8
            assert st["proj_rank"] == 8
            sweeps.append(st["poisson"]["sweeps"])
            r0.append(st["poisson"]["relres0"])
        res[ws] = dict(sweeps=np.mean(sweeps), relres0=np.exp(np.mean(np.log(r0))))
        ch.close()
    print("least squares vs least squares + network:", res)
    assert res[STP_WS_LEARNED]["relres0"] < 0.5 * res[STP_WS_PREV]["relres0"]
    assert res[STP_WS_LEARNED]["sweeps"] < res[STP_WS_PREV]["sweeps"]

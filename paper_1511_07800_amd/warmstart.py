"""Training and evaluation of the learned warm start on pairs the solver
generates itself.

Everything that computes runs in libstp.so: the LES steps that produce the
(b, p^n, p^{n+1}) triples, the network's forward and backward passes and the
Adam updates.  This module only orders the calls and keeps the triples as
torch tensors in device memory.

    python -m paper_1511_07800_amd.warmstart --workload les_channel_256x128x128 \
        --steps 600 --every 4 --epochs 6 --out paper_1511_07800_amd/weights/warmstart_les.npy
"""
import argparse
import json
import os
import time

import numpy as np

from .binding import Channel, STP_MIXED, STP_FP64, STP_WS_LEARNED, STP_WS_PREV, STP_RHS, STP_P
from . import inputs, workloads

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "warmstart_les.npy")


def make_channel(wl, precision=STP_MIXED, rtol=1e-8, warm_start=STP_WS_PREV, seed=None, srj_adaptive=0,
                 learned_correction=0):
    import torch
    ch = Channel(wl["nx"], wl["ny"], wl["nz"], wl["lx"], wl["ly"], wl["lz"], nu=wl["nu"], dpdx=wl["dpdx"],
                 dt=wl["dt"], les=wl["les"], cs=wl.get("cs", 0.1), vd_a=wl.get("vd_a", 25.0), precision=precision,
                 poisson_rtol=rtol, poisson_maxit=200, warm_start=warm_start, srj_adaptive=srj_adaptive,
                 learned_correction=learned_correction)
    u, v, w = inputs.channel_state(wl["nx"], wl["ny"], wl["nz"], wl["lz"], wl["nu"], wl["dpdx"],
                                   noise=wl.get("noise", 0.0), seed=wl.get("seed", 0) if seed is None else seed)
    for k, a in enumerate((u, v, w)):
        ch.field(k).copy_(torch.from_numpy(a))
    torch.cuda.synchronize()
    return ch


def extrapolated_base(ch, b, hist):
    """The guess the library's extrapolated warm start keeps: of p^n and its
    extrapolations 2p^n - p^{n-1}, 3(p^n - p^{n-1}) + p^{n-2} (hist: newest
    last), the one of least residual for b."""
    cands = [hist[-1]]
    if len(hist) >= 2:
        cands.append(2.0 * hist[-1] - hist[-2])
    if len(hist) >= 3:
        cands.append(3.0 * (hist[-1] - hist[-2]) + hist[-3])
    r = [ch.residual_norm(b, c) for c in cands]
    return cands[min(range(len(r)), key=lambda i: r[i])]


def lsq_base(ch, b, xs, ys):
    """The library's least-squares guess (stp_lsq_guess) for b from the last
    solutions xs and their right-hand sides ys, newest first; None if it
    uses no column."""
    import torch
    out = torch.empty_like(b)
    return out if ch.lsq_guess(xs, ys, b, out) > 0 else None


LSQ_DEPTH = 8
BASES = {"prev": ("prev",), "extrap": ("extrap",), "lsq": ("lsq",), "both": ("prev", "extrap"),
         "all": ("prev", "extrap", "lsq")}


def generate_pairs(ch, nsteps, every, skip=0, log=print, base="prev"):
    """Run nsteps time steps; after the first `skip`, keep every `every`-th
    step's (b, guess, p^{n+1}) as device tensors, with guess = p^n
    (base "prev"), the extrapolated guess ("extrap"), the least-squares guess
    from the last 8 solutions ("lsq"), or one triple of each of p^n and the
    extrapolated guess ("both") or of all three ("all"); a derived guess only
    where it differs from p^n and, for "lsq", has the smaller residual."""
    pairs = []
    kinds = BASES[base]
    hist = [ch.field(STP_P).clone()]
    xs, ys = [], []  # solutions and their right-hand sides, newest first
    for n in range(nsteps):
        keep = n >= skip and (n - skip) % every == 0
        st = ch.step(1)
        p_next = ch.field(STP_P).clone()
        b = ch.field(STP_RHS).clone()
        if keep:
            if "prev" in kinds:
                pairs.append((b, hist[-1], p_next))
            if "extrap" in kinds:
                g = extrapolated_base(ch, b, hist)
                if base == "extrap" or g is not hist[-1]:
                    pairs.append((b, g, p_next))
            if "lsq" in kinds and xs:
                g = lsq_base(ch, b, xs, ys)
                if g is not None and ch.residual_norm(b, g) < ch.residual_norm(b, hist[-1]):
                    pairs.append((b, g, p_next))
        hist = (hist + [p_next])[-3:]
        if "lsq" in kinds:
            xs, ys = [p_next] + xs[:LSQ_DEPTH - 1], [b] + ys[:LSQ_DEPTH - 1]
        if (n + 1) % 50 == 0:
            log(f"  data step {n + 1}/{nsteps}: sweeps {st['poisson']['sweeps']} relres0 "
                f"{st['poisson']['relres0']:.2e} cfl {st['cfl']:.3f}")
    return pairs


def train(ch, pairs, epochs, lr, log=print, seed=0):
    """Adam over the training triples, one triple per step, shuffled per epoch."""
    rng = np.random.Generator(np.random.PCG64(seed))
    hist = []
    for ep in range(epochs):
        order = rng.permutation(len(pairs))
        t0 = time.perf_counter()
        losses = [ch.net_train_step(*pairs[i], lr) for i in order]
        hist.append(float(np.mean(losses)))
        log(f"  epoch {ep + 1}/{epochs}: mean loss {hist[-1]:.4e} ({time.perf_counter() - t0:.1f} s)")
    return hist


def guess_quality(ch, pairs):
    """Relative residuals ||b - L p|| / ||b|| of p^n and of the network's guess."""
    import torch
    out = []
    for b, p_prev, p_next in pairs:
        g = torch.empty_like(p_prev)
        ch.net_predict(b, p_prev, g)
        bn = float(torch.linalg.vector_norm(b))
        r_prev = ch.residual_norm(b, p_prev) / bn
        r_net = ch.residual_norm(b, g) / bn
        err_prev = float(torch.linalg.vector_norm(p_prev - p_next) / torch.linalg.vector_norm(p_next))
        err_net = float(torch.linalg.vector_norm(g - p_next) / torch.linalg.vector_norm(p_next))
        out.append(dict(relres_prev=r_prev, relres_net=r_net, err_prev=err_prev, err_net=err_net))
    return out


def sweeps_to_tolerance(ch, pairs, rtol, use_net):
    """Relaxation sweeps the context's solve needs to reach rtol from p^n or
    from the better of p^n and the network's guess, per triple."""
    import torch
    res = []
    for b, p_prev, p_next in pairs:
        p = p_prev.clone()
        if use_net:
            g = torch.empty_like(p)
            ch.net_predict(b, p_prev, g)
            if ch.residual_norm(b, g) < ch.residual_norm(b, p_prev):
                p = g
        st, _ = ch.poisson_solve(b, p, rtol, 200)
        res.append(st["sweeps"])
    return res


def save_weights(ch, path, meta):
    params, _ = ch.net_params()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.save(path, params.detach().cpu().numpy().astype(np.float32), allow_pickle=False)
    with open(path.replace(".npy", ".json"), "w") as f:
        json.dump(meta, f, indent=1)


def load_weights(ch, path=DEFAULT_WEIGHTS):
    import torch
    flat = np.load(path, allow_pickle=False)
    params, _ = ch.net_params()
    if flat.shape[0] != params.numel():
        raise ValueError(f"{path}: {flat.shape[0]} parameters, network has {params.numel()}")
    params.copy_(torch.from_numpy(flat))
    ch.net_sync()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="les_channel_256x128x128")
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--every", type=int, default=4)
    ap.add_argument("--skip", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--seed", type=int, default=None, help="noise seed of the data run (default: the workload's)")
    ap.add_argument("--base", choices=tuple(BASES), default="prev",
                    help="guess the triples start from: p^n, the extrapolated or the least-squares guess, "
                         "p^n and the extrapolated one (both), or all three (all)")
    ap.add_argument("--init", default=None, help="weights to start from (default: random initialisation)")
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    wl = workloads.params(args.workload)
    log = lambda s: print(s, flush=True)
    t0 = time.perf_counter()
    ch = make_channel(wl, STP_MIXED, args.rtol, seed=args.seed, srj_adaptive=1)
    ch.net_init(training=True, seed=1)
    if args.init:
        load_weights(ch, args.init)
    pairs = generate_pairs(ch, args.steps, args.every, args.skip, log, base=args.base)
    ntrain = int(0.8 * len(pairs))
    train_set, held = pairs[:ntrain], pairs[ntrain:]
    log(f"{len(pairs)} triples ({ntrain} train, {len(held)} held out), data {time.perf_counter() - t0:.1f} s")
    q0 = guess_quality(ch, held)
    hist = train(ch, train_set, args.epochs, args.lr, log)
    q1 = guess_quality(ch, held)
    s_prev = sweeps_to_tolerance(ch, held, args.rtol, False)
    s_net = sweeps_to_tolerance(ch, held, args.rtol, True)
    summary = {
        "workload": args.workload, "seed": args.seed if args.seed is not None else wl.get("seed"),
        "base": args.base, "init": os.path.basename(args.init) if args.init else None,
        "steps": args.steps, "every": args.every, "skip": args.skip,
        "train_triples": ntrain, "held_out": len(held), "epochs": args.epochs, "lr": args.lr,
        "loss_by_epoch": hist,
        "held_relres_prev_mean": float(np.mean([q["relres_prev"] for q in q1])),
        "held_relres_net_untrained_mean": float(np.mean([q["relres_net"] for q in q0])),
        "held_relres_net_mean": float(np.mean([q["relres_net"] for q in q1])),
        "held_err_prev_mean": float(np.mean([q["err_prev"] for q in q1])),
        "held_err_net_mean": float(np.mean([q["err_net"] for q in q1])),
        "held_sweeps_prev_mean": float(np.mean(s_prev)), "held_sweeps_net_mean": float(np.mean(s_net)),
        "rtol": args.rtol, "seconds": time.perf_counter() - t0,
    }
    log(json.dumps(summary))
    save_weights(ch, args.out, summary)


if __name__ == "__main__":
    main()

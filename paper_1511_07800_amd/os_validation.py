"""The paper's Orr-Sommerfeld validation run (Sec. 4.2) from the paper's own
seed, through the library: Re_* = 500, alpha = 2 pi / 4 (Lx = 4), 1200 x 3 x
300 cells of height 1, dt = 1e-5, the laminar profile Re_* z (1 - z) plus
du = -A f', dw = f A' with eps = 1e-4, C = 2^-1/2, S = -2^-1/2, FP64 steps
from the plain p^n warm start.

Reported, as the paper measures them: L2^w(t), the L2 norm of dw over the
x-z plane (w of the base flow is 0; the y mean of the ny columns), whose
logarithm grows at Re(lambda); and W_m(t) = dw(Lx/2, Lz/2), whose oscillation
has the period T = 2 pi / |Im(lambda)|.  Growth rates are least-squares slopes
of ln L2^w over trailing windows, the period the mean spacing of W_m's zero
crossings (two per period).  The paper's numbers: measured growth 1.7293 and
period 0.186 +- 0.004, against the Orr-Sommerfeld 1.8056 and 0.185.

  python -m paper_1511_07800_amd.os_validation --steps 20000 --out os.json
"""
import argparse
import json
import math
import sys
import time

import numpy as np


def growth_rate(ts, l2, t_from):
    """Least-squares slope of ln L2^w over the samples with t >= t_from."""
    ts, l2 = np.asarray(ts), np.asarray(l2)
    m = ts >= t_from
    return float(np.polyfit(ts[m], np.log(l2[m]), 1)[0])


def period(ts, wm, t_from):
    """Twice the mean spacing of the sign changes of W_m at t >= t_from (each
    crossing placed at the first sample past it), or None with fewer than 3."""
    ts, wm = np.asarray(ts), np.asarray(wm)
    zc = ts[1:][np.sign(wm[1:]) != np.sign(wm[:-1])]
    late = zc[zc >= t_from]
    return float(2 * np.mean(np.diff(late))) if len(late) > 2 else None


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--every", type=int, default=20)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--lsq", action="store_true", help="least-squares warm start instead of p^n")
    ap.add_argument("--out", default=None)
    ap.add_argument("--max-seconds", type=float, default=None, help="stop stepping after this much wall time")
    args = ap.parse_args(argv)

    import torch
    from paper_1511_07800_amd import Channel, STP_W, inputs
    re, nx, ny, nz, lx, lz, dt = 500.0, 1200, 3, 300, 4.0, 1.0, 1e-5
    ly = ny * lx / nx
    nu, g = 1.0 / re, -2.0
    alpha = 2 * math.pi / lx
    torch.cuda.set_device(0)
    u, v, w = inputs.os_paper_seed(nx, ny, nz, lx, lz, nu, g, alpha)
    ch = Channel(nx, ny, nz, lx, ly, lz, nu=nu, dpdx=g, dt=dt, poisson_rtol=args.rtol, poisson_maxit=500,
                 srj_adaptive=1, proj_depth=8 if args.lsq else 0)
    for k, a in enumerate((u, v, w)):
        ch.field(k).copy_(torch.from_numpy(a))
    torch.cuda.synchronize()
    dx, dz = lx / nx, lz / nz
    ts, l2, wm = [], [], []
    wall0 = time.perf_counter()
    sweeps = 0
    done = 0
    for n in range(1, args.steps + 1):
        if args.max_seconds is not None and time.perf_counter() - wall0 > args.max_seconds:
            print(f"os: wall-time limit after {n - 1} steps", flush=True)
            break
        st = ch.step(1)
        done = n
        sweeps += st["poisson"]["sweeps"]
        if n % args.every == 0:
            wf = ch.field(STP_W)
            ts.append(n * dt)
            l2.append(float(torch.sqrt((wf * wf).sum() * dx * dz / ny)))
            wm.append(float(0.5 * (wf[nz // 2, :, nx // 2 - 1] + wf[nz // 2, :, nx // 2]).mean()))
        if n % 2000 == 0:
            print(f"os step {n}/{args.steps} t {n * dt:.3f}: L2w {l2[-1]:.4e} Wm {wm[-1]:+.3e} sweeps/step "
                  f"{sweeps / n:.0f} ms/step {1e3 * (time.perf_counter() - wall0) / n:.2f}", flush=True)
    ts, l2, wm = np.array(ts), np.array(l2), np.array(wm)
    t_end = ts[-1]
    fits = {f"t>={frac * t_end:.3f}": growth_rate(ts, l2, frac * t_end) for frac in (0.25, 0.5, 0.75)}
    t_osc = period(ts, wm, 0.5 * t_end)
    out = {"case": "Re_*=500, alpha=pi/2, 1200x3x300, dt=1e-5, paper seed", "warm_start": "lsq" if args.lsq else "p^n",
           "rtol": args.rtol, "steps": done, "t_end": float(t_end),
           "ms_per_step": 1e3 * (time.perf_counter() - wall0) / done, "sweeps_per_step": sweeps / done,
           "growth_rate_fits": fits, "period": t_osc,
           "paper": {"measured_growth": 1.7293, "os_growth": 1.8056, "measured_period": 0.186, "os_period": 0.185},
           "series": [[round(float(a), 5), float(f"{b:.6e}"), float(f"{c:.6e}")]
                      for a, b, c in list(zip(ts, l2, wm))[:: max(1, len(ts) // 100)]]}
    ch.close()
    line = json.dumps(out)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(line + "\n")
    print(line, flush=True)


if __name__ == "__main__":
    sys.exit(main())

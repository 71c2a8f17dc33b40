"""The paper's LES run (Sec. 6) on one GPU, through the library: Re_* = 360,
240 x 140 x 120 cells on an 8 x 4 x 1 box, dt = 1e-4, started from the
curl-of-random-modes state, with the bulk statistics the paper reports.

Statistics (Sec. 6): the x-y plane means of stp_plane_stats are averaged over
the sampled steps with t >= t1, giving <u>(z); from it
  U_mean = mean of <u> over the height (uniform cells),
  U_cl   = <u> at z = 1/2 (the two central cell planes),
  Re_mean = U_mean H / nu, U_max / U_mean with U_max = max_z <u>,
  C_f = 2 u_*^2 / U_mean^2 with u_* = 1 (the friction velocity of the imposed
        gradient), and the wall shear actually reached, nu d<u>/dz at the
        walls from the odd ghost (u_*^2 once the flow is steady).
The run also logs the plane-mean centreline velocity against time, from which
the paper judges the statistically steady state.  The paper averages over
t in [20, 53] (530 000 steps); a run here states the window it covers.

  python -m paper_1511_07800_amd.les --steps 20000 --t1 1.0 --out les.json

Continuing a run: --save writes u, v, w (FP32, to bound the file) and the
accumulated statistics; --restart reads them (the Adams-Bashforth history and
the least-squares history restart, as after any fresh start).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np


def bulk(prof, wl):
    """Bulk statistics from a mean profile <u>(z) on the cell planes."""
    nz, lz, nu = wl["nz"], wl["lz"], wl["nu"]
    u_mean = float(np.mean(prof))
    u_cl = float(0.5 * (prof[nz // 2 - 1] + prof[nz // 2])) if nz % 2 == 0 else float(prof[nz // 2])
    dz = lz / nz
    tau = nu * 0.5 * (2.0 * prof[0] / dz + 2.0 * prof[-1] / dz)  # mean of both walls, odd ghost
    return {"U_mean": u_mean, "Re_mean": u_mean * lz / nu, "U_cl": u_cl, "U_max": float(np.max(prof)),
            "U_max_over_U_mean": float(np.max(prof)) / u_mean, "C_f": 2.0 / u_mean**2,
            "wall_shear": float(tau), "u_tau_from_wall_shear": math.sqrt(abs(tau))}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="les_channel_paper_240x140x120")
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--t1", type=float, default=None, help="average from this time on (default: the paper's 20)")
    ap.add_argument("--every", type=int, default=50, help="steps between statistics samples")
    ap.add_argument("--rtol", type=float, default=None)
    ap.add_argument("--log-every", type=int, default=500)
    ap.add_argument("--save", default=None)
    ap.add_argument("--restart", default=None)
    ap.add_argument("--out", default=None)
    ap.add_argument("--stencils32", type=int, default=0, help="eddy viscosity and explicit terms in FP32")
    ap.add_argument("--max-seconds", type=float, default=None,
                    help="stop stepping after this much wall time (then save and report)")
    args = ap.parse_args(argv)

    import torch
    from paper_1511_07800_amd import Channel, STP_MIXED, STP_U, STP_V, STP_W, inputs, workloads
    wl = workloads.params(args.workload)
    t1 = wl["t_stats"][0] if args.t1 is None else args.t1
    rtol = wl["poisson_rtol"] if args.rtol is None else args.rtol
    g = (wl["nx"], wl["ny"], wl["nz"], wl["lx"], wl["ly"], wl["lz"])
    torch.cuda.set_device(0)
    ch = Channel(*g, nu=wl["nu"], dpdx=wl["dpdx"], dt=wl["dt"], les=1, cs=wl["cs"], vd_a=wl["vd_a"],
                 precision=STP_MIXED, poisson_rtol=rtol, poisson_maxit=200, srj_adaptive=1,
                 srj_reduction=wl["srj_reduction"], proj_depth=8, mixed_rhs16=1, stencils32=args.stencils32)
    t0_sim, acc, nacc, series = 0.0, None, 0, []
    if args.restart:
        z = np.load(args.restart, allow_pickle=False)
        u, v, w = (z[k].astype(np.float64) for k in ("u", "v", "w"))
        t0_sim = float(z["t"])
        if z["nacc"] > 0:
            acc = {k[4:]: z[k].astype(np.float64) for k in z.files if k.startswith("acc_")}
            nacc = int(z["nacc"])
        series = [tuple(r) for r in z["series"]]
    else:
        u, v, w = inputs.les_curl_state(*g, wl["nu"], wl["dpdx"], a=wl["curl_a"], modes=wl["curl_modes"],
                                        seed=wl["seed"])
    for k, a in zip((STP_U, STP_V, STP_W), (u, v, w)):
        ch.field(k).copy_(torch.from_numpy(np.ascontiguousarray(a)))
    torch.cuda.synchronize()
    print(f"les: {args.workload} from t = {t0_sim:.4f}, {args.steps} steps, averaging from t = {t1}, rtol {rtol}",
          flush=True)
    wall0 = time.perf_counter()
    sweeps = 0
    done = 0
    for n in range(1, args.steps + 1):
        if args.max_seconds is not None and time.perf_counter() - wall0 > args.max_seconds:
            print(f"les: wall-time limit after {n - 1} steps", flush=True)
            break
        st = ch.step(1)
        done = n
        sweeps += st["poisson"]["sweeps"]
        t = t0_sim + n * wl["dt"]
        if n % args.every == 0:
            series.append((t, st["u_centre"], st["u_bulk"], st["cfl"]))
            if t >= t1:
                ps = ch.plane_stats()
                if acc is None:
                    acc = {k: np.zeros_like(a) for k, a in ps.items()}
                for k in acc:
                    acc[k] += ps[k]
                nacc += 1
        if n % args.log_every == 0 or n == args.steps:
            el = time.perf_counter() - wall0
            print(f"les step {n}/{args.steps} t {t:.4f}: u_centre {st['u_centre']:.3f} u_bulk {st['u_bulk']:.3f} "
                  f"cfl {st['cfl']:.3f} sweeps/step {sweeps / n:.0f} max_div {st['max_div']:.1e} "
                  f"samples {nacc} ms/step {1e3 * el / n:.2f}", flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    t_end = t0_sim + done * wl["dt"]
    out = {"workload": args.workload, "t_start": t0_sim, "t_end": t_end, "steps": done,
           "ms_per_step": 1e3 * wall / max(done, 1), "sweeps_per_step": sweeps / max(done, 1), "rtol": rtol,
           "t1": t1, "samples": nacc,
           "paper": {"U_mean": 15.39, "Re_mean": 5542, "U_cl": 18.30, "U_max_over_U_mean": 1.19, "C_f": 8.44e-3,
                     "window": [20.0, 53.0]},
           "centreline_series": [[round(a, 4), round(b, 4)] for a, b, _, _ in series[:: max(1, len(series) // 200)]]}
    if nacc > 0:
        mean = {k: a / nacc for k, a in acc.items()}
        out["stats"] = bulk(mean["u"], wl)
        zc = (np.arange(wl["nz"]) + 0.5) * wl["lz"] / wl["nz"]
        half = wl["nz"] // 2
        zplus = zc[:half] / wl["nu"]  # z u_*/nu with u_* = 1
        out["profile_wall_units"] = [[round(float(zp), 2), round(float(0.5 * (a + b)), 4)]
                                     for zp, a, b in zip(zplus, mean["u"][:half], mean["u"][::-1][:half])]
        out["log_law_reference"] = "u+ = z+ near the wall; u+ = ln(z+)/0.4 + 5.5 in the log layer (Sec. 6)"
    if args.save:
        uu, vv, ww = (ch.field(k).float().cpu().numpy() for k in (STP_U, STP_V, STP_W))
        extra = {"acc_" + k: a for k, a in (acc or {}).items()}
        np.savez(args.save, u=uu, v=vv, w=ww, t=t_end, nacc=nacc, series=np.array(series), **extra)
    ch.close()
    line = json.dumps(out)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(line + "\n")
    print(line, flush=True)


if __name__ == "__main__":
    sys.exit(main())

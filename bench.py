"""Benchmark: LES time steps of the S-TPLS channel solver on one MI355X.

One "step" is a whole time step of the hot path (eddy viscosity, explicit
terms, Crank-Nicolson predictor, divergence, SRJ pressure solve to a fixed
relative residual, correction, diagnostics) on the 512x256x192 LES channel
with inputs already resident in HBM.  Prints one JSON line.

value  = relaxation cell-updates per second over the whole timed steps
         (sweeps x cells / wall time of the steps, everything included).
Also reported: LES steps/s for the mixed (FP32 sweeps, FP64 residual and
defect correction) and plain FP64 solves at the same relative residual, the
dominant kernel's roofline (FP32 relaxation sweep, HBM-bound), and the FP64
oracle's sweep rate on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "pressure-relax Gcell-updates/s + %HBM peak; LES steps/s, learned vs plain"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="les_channel_512x256x192")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--sweeps", type=int, default=200, help="sweeps in the kernel roofline timing")
    return ap.parse_args()


def make_channel(wl, precision, rtol):
    import torch
    from paper_1511_07800_amd import Channel, inputs
    ch = Channel(wl["nx"], wl["ny"], wl["nz"], wl["lx"], wl["ly"], wl["lz"], nu=wl["nu"], dpdx=wl["dpdx"],
                 dt=wl["dt"], les=wl["les"], cs=wl.get("cs", 0.1), vd_a=wl.get("vd_a", 25.0), precision=precision,
                 poisson_rtol=rtol, poisson_maxit=200)
    u, v, w = inputs.channel_state(wl["nx"], wl["ny"], wl["nz"], wl["lz"], wl["nu"], wl["dpdx"],
                                   noise=wl.get("noise", 0.0), seed=wl.get("seed", 0))
    for k, a in enumerate((u, v, w)):
        ch.field(k).copy_(torch.from_numpy(a))
    torch.cuda.synchronize()
    return ch


def time_steps(ch, steps, warmup, label):
    import torch
    for i in range(warmup):
        st = ch.step(1)
        print(f"[{label}] warmup step {i + 1}/{warmup}: sweeps {st['poisson']['sweeps']} "
              f"relres0 {st['poisson']['relres0']:.2e} cfl {st['cfl']:.3f}", flush=True)
    torch.cuda.synchronize()
    sweeps = 0
    t0 = time.perf_counter()
    for i in range(steps):
        st = ch.step(1)
        sweeps += st["poisson"]["sweeps"]
        print(f"[{label}] step {i + 1}/{steps}: sweeps {st['poisson']['sweeps']} outer {st['poisson']['outer']} "
              f"relres0 {st['poisson']['relres0']:.2e} relres {st['poisson']['relres']:.2e} "
              f"ms {st['ms_total']:.1f} (poisson {st['ms_poisson']:.1f}) max_div {st['max_div']:.1e}", flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, sweeps, st


def kernel_roofline(wl, nsweeps):
    """Average duration of the FP32 relaxation sweep at this grid, timed with
    events on the stream the library launches on (torch's current stream)."""
    import torch
    from paper_1511_07800_amd import Channel, inputs
    nx, ny, nz = wl["nx"], wl["ny"], wl["nz"]
    ch = Channel(nx, ny, nz, wl["lx"], wl["ly"], wl["lz"], nu=wl["nu"], dpdx=wl["dpdx"], dt=wl["dt"])
    b = torch.from_numpy(inputs.poisson_rhs(nx, ny, nz, seed=1511)).float().cuda()
    p = torch.zeros_like(b)
    om = ch.schedule()
    ws = [om[k % len(om)] for k in range(nsweeps)]
    ch.relax(b, p, ws[:10])
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    ch.relax(b, p, ws)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / nsweeps
    n = nx * ny * nz
    bytes_per_sweep = 12.0 * n  # read p, read b, write p: 3 FP32 words per cell
    achieved = bytes_per_sweep / (ms * 1e-3) / 1e9
    ch.close()
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_relax<float>", "us_per_launch": round(ms * 1e3, 2),
            "gcell_updates_per_s": round(n / (ms * 1e-3) / 1e9, 1)}


def cpu_baseline(wl):
    """The FP64 oracle's relaxation sweep on the host cores, on a bounded
    sample: 8 sweeps of the same grid."""
    import numpy as np
    import oracle
    from paper_1511_07800_amd import inputs
    nx, ny, nz = wl["nx"], wl["ny"], wl["nz"]
    P = oracle.make_params(nx, ny, nz, wl["lx"], wl["ly"], wl["lz"])
    b = inputs.poisson_rhs(nx, ny, nz, seed=1511)
    p = np.zeros_like(b)
    om = oracle.srj_schedule(nx, ny, nz, wl["lx"], wl["ly"], wl["lz"])
    oracle.srj_sweep(P, om[0], p, b)
    nsw = 8
    t0 = time.perf_counter()
    for k in range(nsw):
        p = oracle.srj_sweep(P, om[k % len(om)], p, b)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(nsw * nx * ny * nz / dt / 1e9, 4), "unit": "Gcell-updates/s", "cores": cores,
            "kind": "oracle", "sample": f"{nsw} FP64 SRJ sweeps of the {nx}x{ny}x{nz} grid ({dt:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design note, not an implementation.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1511_07800_amd import STP_MIXED, STP_FP64, workloads
    torch.cuda.set_device(0)
    wl = workloads.params(args.workload)
    n = wl["nx"] * wl["ny"] * wl["nz"]

    ch = make_channel(wl, STP_MIXED, args.rtol)
    t_mixed, sweeps_mixed, st_mixed = time_steps(ch, args.steps, args.warmup, "mixed")
    ch.close()
    del ch
    torch.cuda.empty_cache()

    fp64 = None
    if not args.no_fp64:
        ch = make_channel(wl, STP_FP64, args.rtol)
        t64, sweeps64, _ = time_steps(ch, args.steps, args.warmup, "fp64")
        fp64 = {"steps_per_s": round(args.steps / t64, 4), "ms_per_step": round(1e3 * t64 / args.steps, 2),
                "sweeps_per_step": sweeps64 / args.steps,
                "gcell_updates_per_s": round(sweeps64 * n / t64 / 1e9, 2)}
        ch.close()
        del ch
        torch.cuda.empty_cache()

    roof = kernel_roofline(wl, args.sweeps)
    cpu = None if args.no_cpu else cpu_baseline(wl)

    value = sweeps_mixed * n / t_mixed / 1e9
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "Gcell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * t_mixed / args.steps, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": [wl["nx"], wl["ny"], wl["nz"]], "precision": "mixed",
                   "poisson_rtol": args.rtol, "dt": wl["dt"], "les": wl["les"], "init": "laminar+10% noise"},
        "les_steps_per_s": {"mixed": round(args.steps / t_mixed, 4), "fp64": fp64["steps_per_s"] if fp64 else None,
                            "learned_mixed": None},
        "sweeps_per_step": {"mixed": sweeps_mixed / args.steps, "fp64": fp64["sweeps_per_step"] if fp64 else None},
        "fp64": fp64,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

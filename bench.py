"""Benchmark: LES time steps of the S-TPLS channel solver on one MI355X.

One "step" is a whole time step of the hot path (eddy viscosity, explicit
terms, Crank-Nicolson predictor, divergence, SRJ pressure solve to a fixed
relative residual, correction, diagnostics) on the 512x256x192 LES channel
with inputs already resident in HBM.  Prints one JSON line.

value  = relaxation cell-updates per second over the whole timed steps
         (sweeps x cells / wall time of the steps, everything included).
Also reported: LES steps/s for the mixed (FP32 sweeps, FP64 residual and
defect correction) and plain FP64 solves at the same relative residual, for
the mixed solve started from the extrapolated, the least-squares and the
learned initial guesses and their combinations, the
fields of every variant against the FP64 run's after the same steps, the
dominant kernel's roofline (FP32 relaxation sweep, HBM-bound), a table of
back-to-back sweep rates for every fusion depth in FP32 and FP64 beside a
plain device copy, and the FP64 oracle's sweep rate on the host cores.
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
FIXED_CYCLES = False  # set by --fixed-cycles: repeat the 1e-3 cycle instead of sizing cycles adaptively
PROJ_DEPTH = 8  # earlier solutions in the least-squares initial guess


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    # untimed steps: past the start-up transient of the laminar+noise start and
    # twice the least-squares history depth, so the timed steps are steady state
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--workload", default="les_channel_512x256x192")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned warm-start run")
    ap.add_argument("--no-table", action="store_true", help="skip the sweep-rate table")
    ap.add_argument("--weights", default="warmstart_les512_all.npy",
                    help="network weights of the learned variants (file in paper_1511_07800_amd/weights)")
    ap.add_argument("--fixed-cycles", action="store_true", help="repeat the fixed 1e-3 SRJ cycle (no adaptive sizing)")
    ap.add_argument("--sweeps", type=int, default=200, help="sweeps in the kernel roofline timing")
    ap.add_argument("--profile-fastest", action="store_true",
                    help="run only the fastest variant (least-squares guess refined by the network, each "
                         "pass's right-hand side in FP16), for a kernel trace of its steps")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="only run a plain copy of known size and the relaxation kernels (for rocprofv3 counters)")
    return ap.parse_args()


def make_channel(wl, precision, rtol, warm_start=0, learned_correction=0, extrap_order=0, proj_depth=0,
                 rhs16=0):
    import torch
    from paper_1511_07800_amd import Channel, inputs
    ch = Channel(wl["nx"], wl["ny"], wl["nz"], wl["lx"], wl["ly"], wl["lz"], nu=wl["nu"], dpdx=wl["dpdx"],
                 dt=wl["dt"], les=wl["les"], cs=wl.get("cs", 0.1), vd_a=wl.get("vd_a", 25.0), precision=precision,
                 poisson_rtol=rtol, poisson_maxit=200, warm_start=warm_start, srj_adaptive=0 if FIXED_CYCLES else 1,
                 srj_reduction=wl.get("srj_reduction", 1e-3), learned_correction=learned_correction,
                 extrap_order=extrap_order, proj_depth=proj_depth, mixed_rhs16=rhs16)
    u, v, w = inputs.channel_state(wl["nx"], wl["ny"], wl["nz"], wl["lz"], wl["nu"], wl["dpdx"],
                                   noise=wl.get("noise", 0.0), seed=wl.get("seed", 0))
    for k, a in enumerate((u, v, w)):
        ch.field(k).copy_(torch.from_numpy(a))
    torch.cuda.synchronize()
    return ch


def time_steps(ch, steps, warmup, label):
    """Time `steps` whole LES steps after `warmup`; also sums the in-step
    relaxation statistics (sweeps, kernel launches and their device time,
    measured by the library with events on its stream)."""
    import torch
    for i in range(warmup):
        st = ch.step(1)
        print(f"[{label}] warmup step {i + 1}/{warmup}: sweeps {st['poisson']['sweeps']} "
              f"relres0 {st['poisson']['relres0']:.2e} cfl {st['cfl']:.3f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    acc = {"sweeps": 0, "launches": 0, "ms_relax": 0.0, "corrections": 0}
    t0 = time.perf_counter()
    for i in range(steps):
        st = ch.step(1)
        for k in acc:
            acc[k] += st["poisson"][k]
        print(f"[{label}] step {i + 1}/{steps}: sweeps {st['poisson']['sweeps']} outer {st['poisson']['outer']} "
              f"relres0 {st['poisson']['relres0']:.2e} relres {st['poisson']['relres']:.2e} "
              f"ms {st['ms_total']:.1f} (poisson {st['ms_poisson']:.1f}, sweeps {st['poisson']['ms_relax']:.1f}) "
              f"max_div {st['max_div']:.1e}" + (f" corrections {st['poisson']['corrections']}"
                                                 if st['poisson']['corrections'] else "") +
              (f" extrap order {st['extrap_used']} guess {st['relres_extrap']:.2e}" if st['relres_extrap'] > 0 else "") +
              (f" lsq rank {st['proj_rank']} guess {st['relres_proj']:.2e} used {st['proj_used']}"
               if st['proj_rank'] > 0 else "") +
              (f" net {st['ms_net']:.1f} ms relres p^n {st['relres_prev']:.2e} "
                                                 f"guess {st['relres_learned']:.2e}" if st['ms_net'] > 0 else ""),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, acc, st


def roofline_from_steps(n, acc, word_bytes, kernel, rhs_bytes=None):
    """Roofline of the dominant kernel from the timed steps: one launch moves
    3 words per cell of compulsory traffic (read p, read b, write p; b takes
    rhs_bytes when stored narrower), so achieved = that per cell x n x
    launches / device time of the sweep sequences."""
    sec = acc["ms_relax"] * 1e-3
    per_cell = 2.0 * word_bytes + (word_bytes if rhs_bytes is None else rhs_bytes)
    achieved = per_cell * n * acc["launches"] / sec / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": kernel,
            "launches": acc["launches"], "sweeps": acc["sweeps"],
            "us_per_launch": round(1e6 * sec / acc["launches"], 2),
            "effective_GBs": round(per_cell * n * acc["sweeps"] / sec / 1e9, 1),
            "gcell_updates_per_s": round(n * acc["sweeps"] / sec / 1e9, 1)}


def measured_traffic(nx, ny, nz, tblock):
    """HBM bytes per launch of the relaxation kernel from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, scaled by the same
    counters on a plain copy of known size); None if the summary is for
    another kernel source, grid or fusion depth."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "relax_traffic.json")
    src = os.path.join(ROOT, "paper_1511_07800_amd", "csrc", "stp_relax.hip")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec.get("source_sha256") != sha or rec.get("grid") != [nx, ny, nz] or rec.get("sweeps_per_launch") != tblock:
        return None
    return rec.get("hbm_bytes_per_launch")


def profile_kernels(wl):
    """Kernels for counter collection: a torch copy of 64 Mi floats (512 MiB
    moved: 256 MiB read, 256 MiB written), then 8 launches each of the fused
    FP32 relaxation kernel, the single-sweep FP32 kernel and the fused kernel
    with an FP16 right-hand side."""
    import torch
    from paper_1511_07800_amd import Channel, inputs
    a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)
    for _ in range(4):
        c.copy_(a)
    torch.cuda.synchronize()
    nx, ny, nz = wl["nx"], wl["ny"], wl["nz"]
    b = torch.from_numpy(inputs.poisson_rhs(nx, ny, nz, seed=1511)).float().cuda()
    for tb in (4, 1):
        ch = Channel(nx, ny, nz, wl["lx"], wl["ly"], wl["lz"], nu=wl["nu"], dpdx=wl["dpdx"], dt=wl["dt"], tblock=tb)
        p = torch.zeros_like(b)
        om = ch.schedule()
        ch.relax(b, p, [om[k % len(om)] for k in range(8 * tb)])
        torch.cuda.synchronize()
        if tb == 4:
            p.zero_()
            ch.relax(b.half(), p, [om[k % len(om)] for k in range(8 * tb)])
            torch.cuda.synchronize()
        ch.close()
    print("profile-kernels done", file=sys.stderr, flush=True)


def relax_sweep_table(wl, timed=1020, warm=60):
    """Back-to-back sweeps of the built-in SRJ cycle from p = 0 on the
    workload's grid (b ~ U(-1, 1) minus its mean), for every fusion depth:
    `warm` untimed sweeps, then `timed` sweeps between events on the stream
    the library runs on (both divisible by 1..5, so every launch fuses the
    full depth).  compulsory_GBs counts 3 words per cell per launch,
    effective_GBs 3 words per cell per sweep.  copy_GBs: a plain device copy
    of 256 MiB (read + write), the practical streaming ceiling."""
    import torch
    from paper_1511_07800_amd import Channel, inputs
    nx, ny, nz = wl["nx"], wl["ny"], wl["nz"]
    n = nx * ny * nz
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)
    for _ in range(3):
        c.copy_(a)
    e0.record()
    for _ in range(20):
        c.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    out = {"copy_GBs": round(20 * 2 * a.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)}
    del a, c
    b64 = torch.from_numpy(inputs.poisson_rhs(nx, ny, nz, seed=1511)).cuda()
    for name, tdt, word, depths in (("f32", torch.float32, 4, (1, 2, 3, 4, 5)), ("f64", torch.float64, 8, (1, 2, 3, 4))):
        b = b64.to(tdt)
        rows = {}
        for tb in depths:
            ch = Channel(nx, ny, nz, wl["lx"], wl["ly"], wl["lz"], nu=wl["nu"], dpdx=wl["dpdx"], dt=wl["dt"],
                         tblock=tb)
            om = ch.schedule()
            seq = [om[k % len(om)] for k in range(warm + timed)]
            p = torch.zeros_like(b)
            ch.relax(b, p, seq[:warm])
            e0.record()
            ch.relax(b, p, seq[warm:])
            e1.record()
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) * 1e-3
            rows[str(tb)] = {"us_per_sweep": round(1e6 * sec / timed, 2),
                             "gcell_updates_per_s": round(n * timed / sec / 1e9, 1),
                             "compulsory_GBs": round(3 * word * n * (timed / tb) / sec / 1e9, 1),
                             "effective_GBs": round(3 * word * n * timed / sec / 1e9, 1)}
            ch.close()
            del ch, p
            torch.cuda.empty_cache()
        out[name] = rows
    return out


def fields_of(ch):
    from paper_1511_07800_amd import STP_U, STP_V, STP_W, STP_P
    return [ch.field(k).clone() for k in (STP_U, STP_V, STP_W, STP_P)]


def field_errors(got, ref):
    """Relative L2 difference of u, v, w, p against the reference fields."""
    return {name: float((g - r).norm() / r.norm()) for name, g, r in zip("uvwp", got, ref)}


def cpu_baseline(wl, seconds=12.0):
    """The FP64 oracle's relaxation sweep on the host cores, on a bounded
    sample: consecutive sweeps of the same grid (the schedule's weights in
    order) for about `seconds` of wall time."""
    import numpy as np
    import oracle
    from paper_1511_07800_amd import inputs
    nx, ny, nz = wl["nx"], wl["ny"], wl["nz"]
    P = oracle.make_params(nx, ny, nz, wl["lx"], wl["ly"], wl["lz"])
    b = inputs.poisson_rhs(nx, ny, nz, seed=1511)
    p = np.zeros_like(b)
    om = oracle.srj_schedule(nx, ny, nz, wl["lx"], wl["ly"], wl["lz"])
    p = oracle.srj_sweep(P, om[0], p, b)
    nsw = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds and nsw < 10000:
        p = oracle.srj_sweep(P, om[nsw % len(om)], p, b)
        nsw += 1
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(nsw * nx * ny * nz / dt / 1e9, 4), "unit": "Gcell-updates/s", "cores": cores,
            "kind": "oracle", "sample": f"{nsw} consecutive FP64 SRJ sweeps of the {nx}x{ny}x{nz} grid "
                                        f"({dt:.1f} s, OpenMP over z-planes)"}


def main():
    args = parse()
    global FIXED_CYCLES
    FIXED_CYCLES = args.fixed_cycles
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design note, not an implementation.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1511_07800_amd import STP_MIXED, STP_FP64, workloads
    torch.cuda.set_device(0)
    wl = workloads.params(args.workload)
    n = wl["nx"] * wl["ny"] * wl["nz"]
    if args.profile_kernels:
        profile_kernels(wl)
        return
    if args.profile_fastest:
        from paper_1511_07800_amd import STP_WS_LEARNED, warmstart
        ch = make_channel(wl, STP_MIXED, args.rtol, warm_start=STP_WS_LEARNED, proj_depth=PROJ_DEPTH, rhs16=1)
        ch.net_init(training=False)
        warmstart.load_weights(ch, os.path.join(ROOT, "paper_1511_07800_amd", "weights", args.weights))
        t, acc, _ = time_steps(ch, args.steps, args.warmup, "learned+lsq+mixed(rhs16)")
        print(json.dumps({"variant": "learned+lsq+mixed(rhs16)", "warmup": args.warmup, "steps": args.steps,
                          "ms_per_step": round(1e3 * t / args.steps, 2),
                          "sweeps_per_step": acc["sweeps"] / args.steps}), flush=True)
        return

    ch = make_channel(wl, STP_MIXED, args.rtol)
    t_mixed, acc_mixed, st_mixed = time_steps(ch, args.steps, args.warmup, "mixed")
    f_mixed = fields_of(ch)
    ch.close()
    del ch
    torch.cuda.empty_cache()

    # the same with the guess extrapolated in time from the last solutions
    ch = make_channel(wl, STP_MIXED, args.rtol, extrap_order=2)
    t_ex, acc_ex, _ = time_steps(ch, args.steps, args.warmup, "extrap+mixed")
    extrap = {"steps_per_s": round(args.steps / t_ex, 4), "ms_per_step": round(1e3 * t_ex / args.steps, 2),
              "sweeps_per_step": acc_ex["sweeps"] / args.steps}
    f_extrap = fields_of(ch)
    ch.close()
    del ch
    torch.cuda.empty_cache()

    # least-squares guess from the last 8 solutions
    ch = make_channel(wl, STP_MIXED, args.rtol, proj_depth=PROJ_DEPTH)
    t_ls, acc_ls, st_ls = time_steps(ch, args.steps, args.warmup, "lsq+mixed")
    lsq = {"steps_per_s": round(args.steps / t_ls, 4), "ms_per_step": round(1e3 * t_ls / args.steps, 2),
           "sweeps_per_step": acc_ls["sweeps"] / args.steps, "proj_depth": PROJ_DEPTH,
           "relres_prev_last": st_ls["relres_prev"], "relres_lsq_last": st_ls["relres_proj"]}
    f_lsq = fields_of(ch)
    ch.close()
    del ch
    torch.cuda.empty_cache()

    # the mixed solve with each pass's right-hand side stored in FP16, from p^n and from the least-squares guess
    def run_rhs16(label, **kw):
        ch = make_channel(wl, STP_MIXED, args.rtol, rhs16=1, **kw)
        t, acc, st = time_steps(ch, args.steps, args.warmup, label)
        out = {"steps_per_s": round(args.steps / t, 4), "ms_per_step": round(1e3 * t / args.steps, 2),
               "sweeps_per_step": acc["sweeps"] / args.steps, "outer_last": st["poisson"]["outer"],
               "relax_kernel": roofline_from_steps(n, acc, 4, "k_relax_fused<float,_Float16,4,8>", rhs_bytes=2)}
        f = fields_of(ch)
        ch.close()
        torch.cuda.empty_cache()
        return out, f
    mixed16, f_mixed16 = run_rhs16("mixed(rhs16)")
    lsq16, f_lsq16 = run_rhs16("lsq+mixed(rhs16)", proj_depth=PROJ_DEPTH)

    fp64 = None
    f_fp64 = None
    errors = {}
    if not args.no_fp64:
        ch = make_channel(wl, STP_FP64, args.rtol)
        t64, acc64, _ = time_steps(ch, args.steps, args.warmup, "fp64")
        f_fp64 = fields_of(ch)
        errors["mixed"] = field_errors(f_mixed, f_fp64)
        errors["extrap+mixed"] = field_errors(f_extrap, f_fp64)
        errors["lsq+mixed"] = field_errors(f_lsq, f_fp64)
        errors["mixed(rhs16)"] = field_errors(f_mixed16, f_fp64)
        errors["lsq+mixed(rhs16)"] = field_errors(f_lsq16, f_fp64)
        fp64 = {"steps_per_s": round(args.steps / t64, 4), "ms_per_step": round(1e3 * t64 / args.steps, 2),
                "sweeps_per_step": acc64["sweeps"] / args.steps,
                "gcell_updates_per_s": round(acc64["sweeps"] * n / t64 / 1e9, 2),
                "relax_kernel": roofline_from_steps(n, acc64, 8, "k_relax_fused<double,4,16>")}
        ch.close()
        del ch
        torch.cuda.empty_cache()

    learned = None
    learned_256 = None
    learned_cc = None
    learned_ex = None
    learned_all = None
    learned_ls = None
    learned_ls_cc = None
    learned_ls16 = None
    if not args.no_learned:
        from paper_1511_07800_amd import STP_WS_LEARNED, warmstart

        def run_learned(weights, label, correction=0, extrap_order=0, proj_depth=0, rhs16=0):
            ch = make_channel(wl, STP_MIXED, args.rtol, warm_start=STP_WS_LEARNED, learned_correction=correction,
                              extrap_order=extrap_order, proj_depth=proj_depth, rhs16=rhs16)
            ch.net_init(training=False)
            warmstart.load_weights(ch, weights)
            tl, accl, stl = time_steps(ch, args.steps, args.warmup, label)
            out = {"steps_per_s": round(args.steps / tl, 4), "ms_per_step": round(1e3 * tl / args.steps, 2),
                   "sweeps_per_step": accl["sweeps"] / args.steps, "ms_net_last": round(stl["ms_net"], 2),
                   "relres_prev_last": stl["relres_prev"], "relres_learned_last": stl["relres_learned"],
                   "relres_extrap_last": stl["relres_extrap"] if extrap_order else None,
                   "relres_lsq_last": stl["relres_proj"] if proj_depth else None,
                   "corrections_per_step": accl["corrections"] / args.steps,
                   "weights": os.path.relpath(weights, ROOT)}
            if f_fp64 is not None:
                errors[label] = field_errors(fields_of(ch), f_fp64)
            ch.close()
            torch.cuda.empty_cache()
            return out

        wdir = os.path.join(ROOT, "paper_1511_07800_amd", "weights")
        learned = run_learned(os.path.join(wdir, args.weights), "learned+mixed")
        learned_256 = run_learned(os.path.join(wdir, "warmstart_les.npy"), "learned(256-trained)+mixed")
        learned_cc = run_learned(os.path.join(wdir, args.weights), "learned+correction+mixed", correction=1)
        learned_ex = run_learned(os.path.join(wdir, args.weights), "learned+extrap+mixed", extrap_order=2)
        learned_all = run_learned(os.path.join(wdir, args.weights), "learned+extrap+correction+mixed",
                                  correction=1, extrap_order=2)
        learned_ls = run_learned(os.path.join(wdir, args.weights), "learned+lsq+mixed", proj_depth=PROJ_DEPTH)
        learned_ls_cc = run_learned(os.path.join(wdir, args.weights), "learned+lsq+correction+mixed",
                                    correction=1, proj_depth=PROJ_DEPTH)
        learned_ls16 = run_learned(os.path.join(wdir, args.weights), "learned+lsq+mixed(rhs16)",
                                   proj_depth=PROJ_DEPTH, rhs16=1)

    roof = roofline_from_steps(n, acc_mixed, 4, "k_relax_fused<float,4,8>")
    roof["traffic"] = measured_traffic(wl["nx"], wl["ny"], wl["nz"], 4)
    del f_mixed, f_extrap, f_lsq, f_mixed16, f_lsq16, f_fp64
    torch.cuda.empty_cache()
    table = None if args.no_table else relax_sweep_table(wl)
    cpu = None if args.no_cpu else cpu_baseline(wl)

    value = acc_mixed["sweeps"] * n / t_mixed / 1e9
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "Gcell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * t_mixed / args.steps, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": [wl["nx"], wl["ny"], wl["nz"]], "precision": "mixed",
                   "poisson_rtol": args.rtol, "dt": wl["dt"], "les": wl["les"], "init": "laminar+10% noise",
                   "srj_cycles": "fixed 1e-3" if FIXED_CYCLES else "adaptive"},
        "les_steps_per_s": {"mixed": round(args.steps / t_mixed, 4), "fp64": fp64["steps_per_s"] if fp64 else None,
                            "extrap_mixed": extrap["steps_per_s"],
                            "lsq_mixed": lsq["steps_per_s"],
                            "mixed_rhs16": mixed16["steps_per_s"],
                            "lsq_mixed_rhs16": lsq16["steps_per_s"],
                            "learned_mixed": learned["steps_per_s"] if learned else None,
                            "learned_mixed_correction": learned_cc["steps_per_s"] if learned_cc else None,
                            "learned_extrap_mixed": learned_ex["steps_per_s"] if learned_ex else None,
                            "learned_extrap_mixed_correction": learned_all["steps_per_s"] if learned_all else None,
                            "learned_lsq_mixed": learned_ls["steps_per_s"] if learned_ls else None,
                            "learned_lsq_mixed_correction": learned_ls_cc["steps_per_s"] if learned_ls_cc else None,
                            "learned_lsq_mixed_rhs16": learned_ls16["steps_per_s"] if learned_ls16 else None},
        "sweeps_per_step": {"mixed": acc_mixed["sweeps"] / args.steps,
                            "fp64": fp64["sweeps_per_step"] if fp64 else None,
                            "extrap_mixed": extrap["sweeps_per_step"],
                            "lsq_mixed": lsq["sweeps_per_step"],
                            "mixed_rhs16": mixed16["sweeps_per_step"],
                            "lsq_mixed_rhs16": lsq16["sweeps_per_step"],
                            "learned_mixed": learned["sweeps_per_step"] if learned else None,
                            "learned_mixed_correction": learned_cc["sweeps_per_step"] if learned_cc else None,
                            "learned_extrap_mixed": learned_ex["sweeps_per_step"] if learned_ex else None,
                            "learned_extrap_mixed_correction": learned_all["sweeps_per_step"] if learned_all else None,
                            "learned_lsq_mixed": learned_ls["sweeps_per_step"] if learned_ls else None,
                            "learned_lsq_mixed_correction": learned_ls_cc["sweeps_per_step"] if learned_ls_cc else None,
                            "learned_lsq_mixed_rhs16": learned_ls16["sweeps_per_step"] if learned_ls16 else None},
        "fp64": fp64,
        "extrap_mixed": extrap,
        "lsq_mixed": lsq,
        "mixed_rhs16": mixed16,
        "lsq_mixed_rhs16": lsq16,
        "learned_mixed": learned,
        "learned_mixed_trained_256x128x128": learned_256,
        "learned_mixed_correction": learned_cc,
        "learned_extrap_mixed": learned_ex,
        "learned_extrap_mixed_correction": learned_all,
        "learned_lsq_mixed": learned_ls,
        "learned_lsq_mixed_correction": learned_ls_cc,
        "learned_lsq_mixed_rhs16": learned_ls16,
        "error_vs_fp64": errors or None,
        "relax_sweeps": table,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

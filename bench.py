"""Benchmark: LES time steps of the S-TPLS channel solver on one MI355X.

One "step" is a whole time step of the hot path (eddy viscosity, explicit
terms, Crank-Nicolson predictor, divergence, SRJ pressure solve to a fixed
relative residual, correction, diagnostics) on the 1024x512x384 LES channel
(2e8 cells, the largest single-GPU workload) with inputs already resident in
HBM.  Prints one JSON line.

value  = relaxation cell-updates per second over the whole timed steps of
         the mixed solve (sweeps x cells / wall time of the steps, every
         other part of the step included).
Also reported: LES steps/s at the same relative residual for the plain FP64
solve, the mixed solve (FP32 sweeps, FP64 residual and defect correction),
the mixed solve from the least-squares guess, from the learned guess, and
from the least-squares guess refined by the network with each pass's
right-hand side in FP16 (more with --all-variants); per timed step the
sweeps, the starting residual and the least-squares rank; the fields of
every variant against the FP64 run's; the dominant kernel's roofline (FP32
relaxation sweep, HBM-bound); a table of back-to-back sweep rates for every
fusion depth beside a plain device copy; and the FP64 oracle on the host
cores (1 thread and all cores).
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
DEFAULT_WORKLOAD = "les_channel_1024x512x384"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    # untimed steps: past the start-up transient of the laminar+noise start and
    # twice the least-squares history depth, so the timed steps are steady state
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--spinup", type=int, default=16,
                    help="steps from the noisy laminar start that prepare the input state (untimed; 0: none)")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned warm-start runs")
    ap.add_argument("--no-table", action="store_true", help="skip the sweep-rate table")
    ap.add_argument("--all-variants", action="store_true",
                    help="also run the extrapolated guess, the FP16 right-hand side alone, the learned coarse "
                         "correction and the network trained at 256x128x128")
    ap.add_argument("--weights", default="warmstart_les512_all.npy",
                    help="network weights of the learned variants (file in paper_1511_07800_amd/weights)")
    ap.add_argument("--fixed-cycles", action="store_true", help="repeat the fixed 1e-3 SRJ cycle (no adaptive sizing)")
    ap.add_argument("--profile-fastest", action="store_true",
                    help="run only the fastest variant (least-squares guess refined by the network, each "
                         "pass's right-hand side in FP16), for a kernel trace of its steps")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="only run a plain copy of known size and the relaxation kernels (for rocprofv3 counters)")
    return ap.parse_args()


def make_channel(wl, precision, rtol, warm_start=0, learned_correction=0, extrap_order=0, proj_depth=0,
                 rhs16=0, stencils32=0, state=None, fixed=False):
    """A context on the workload, started from `state` (device tensors u, v,
    w, p from prepare_state) or, without one, from the laminar profile plus
    the workload's seeded noise."""
    import torch
    from paper_1511_07800_amd import Channel, inputs
    ch = Channel(wl["nx"], wl["ny"], wl["nz"], wl["lx"], wl["ly"], wl["lz"], nu=wl["nu"], dpdx=wl["dpdx"],
                 dt=wl["dt"], les=wl["les"], cs=wl.get("cs", 0.1), vd_a=wl.get("vd_a", 25.0), precision=precision,
                 poisson_rtol=rtol, poisson_maxit=200, warm_start=warm_start, srj_adaptive=0 if (FIXED_CYCLES or fixed) else 1,
                 srj_reduction=wl.get("srj_reduction", 1e-3), learned_correction=learned_correction,
                 extrap_order=extrap_order, proj_depth=proj_depth, mixed_rhs16=rhs16, stencils32=stencils32)
    if state is not None:
        for k, a in enumerate(state):
            ch.field(k).copy_(a)
        torch.cuda.synchronize()
        return ch
    u, v, w = inputs.channel_state(wl["nx"], wl["ny"], wl["nz"], wl["lz"], wl["nu"], wl["dpdx"],
                                   noise=wl.get("noise", 0.0), seed=wl.get("seed", 0))
    for k, a in enumerate((u, v, w)):
        ch.field(k).copy_(torch.from_numpy(a))
    del u, v, w
    torch.cuda.synchronize()
    return ch


def prepare_state(wl, args):
    """The benchmark's input state: the laminar profile plus seeded noise,
    advanced args.spinup steps (mixed precision, least-squares guess) before
    anything is timed, so that every variant starts from the same developed
    flow rather than from the start-up transient of the noisy laminar state
    (whose non-solenoidal noise and fast early pressure changes would make the
    first few dozen steps unrepresentative of a running LES).  Returns device
    copies of u, v, w and p, or None for args.spinup = 0."""
    import torch
    from paper_1511_07800_amd import STP_MIXED
    if args.spinup <= 0:
        return None
    ch = make_channel(wl, STP_MIXED, args.rtol, proj_depth=PROJ_DEPTH)
    for i in range(args.spinup):
        st = ch.step(1)
        print(f"[input preparation] step {i + 1}/{args.spinup}: sweeps {st['poisson']['sweeps']} "
              f"relres0 {st['poisson']['relres0']:.2e}", file=sys.stderr, flush=True)
    state = [ch.field(k).clone() for k in range(4)]
    torch.cuda.synchronize()
    ch.close()
    del ch
    torch.cuda.empty_cache()
    return state


PHASES = ("ms_nut", "ms_momentum", "ms_divergence", "ms_guess", "ms_poisson", "ms_projection")


def time_steps(ch, steps, warmup, label):
    """Time `steps` whole LES steps after `warmup`; also sums the in-step
    relaxation statistics (sweeps, kernel launches and their device time,
    measured by the library with events on its stream) and keeps, per timed
    step, the sweeps, the starting relative residual and the least-squares
    rank."""
    import torch
    for i in range(warmup):
        st = ch.step(1)
        print(f"[{label}] warmup step {i + 1}/{warmup}: sweeps {st['poisson']['sweeps']} "
              f"relres0 {st['poisson']['relres0']:.2e} cfl {st['cfl']:.3f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    acc = {"sweeps": 0, "launches": 0, "ms_relax": 0.0, "corrections": 0}
    acc_phase = dict.fromkeys(PHASES, 0.0)
    per_step = []
    t0 = time.perf_counter()
    for i in range(steps):
        st = ch.step(1)
        for k in acc:
            acc[k] += st["poisson"][k]
        for k in acc_phase:
            acc_phase[k] += st[k]
        per_step.append({"sweeps": st["poisson"]["sweeps"], "relres0": float(f"{st['poisson']['relres0']:.3e}"),
                         "proj_rank": st["proj_rank"]})
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
    acc["phases"] = acc_phase
    return dt, acc, st, per_step


def fused_depth(acc):
    """Sweeps per launch of the timed steps' relaxation (the last launch of a
    cycle may run fewer)."""
    return -(-acc["sweeps"] // max(acc["launches"], 1))


def fused_kernel(acc, ny, rhs="float"):
    """Name of the FP32 fused relaxation kernel the steps ran: five sweeps
    run on the 16-wavefront, 64-row tiles where ny >= 66, otherwise on the
    8-wavefront, 32-row tiles."""
    d = fused_depth(acc)
    shape = "16,64" if d == 5 and ny >= 66 else "8"
    return f"k_relax_fused<float,{rhs},{d},{shape}>"


def roofline_from_steps(n, acc, word_bytes, kernel, rhs_bytes=None):
    """Roofline of the dominant kernel from the timed steps: one launch moves
    3 words per cell of compulsory traffic (read p, read b, write p; b takes
    rhs_bytes when stored narrower), so achieved = that per cell x n x
    launches / device time of the sweep sequences.  `kernel` may hold {d}
    for the fusion depth."""
    kernel = kernel.format(d=fused_depth(acc))
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
    """HBM-side bytes per launch of the FP32 relaxation kernel from the
    committed rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, each scaled
    by the same counter on a plain copy of known size); None unless the
    summary was taken on this kernel source, grid and fusion depth (tblock
    sweeps per launch)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "relax_traffic.json")
    src = os.path.join(ROOT, "paper_1511_07800_amd", "csrc", "stp_relax.hip")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    entry = rec.get("grids", {}).get(f"{nx}x{ny}x{nz}")
    if rec.get("source_sha256") != sha or entry is None or entry.get("sweeps_per_launch") != tblock:
        return None
    return round(entry["hbm_bytes_per_launch"])


def profile_kernels(wl):
    """Kernels for counter collection: a torch copy of 64 Mi floats (512 MiB
    moved: 256 MiB read, 256 MiB written), then 40 sweeps of the fused FP32
    relaxation kernel at the library's fusion depth, 8 of the single-sweep
    FP32 kernel and 40 of the fused kernel with an FP16 right-hand side."""
    import torch
    from paper_1511_07800_amd import Channel, inputs
    a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)
    for _ in range(4):
        c.copy_(a)
    torch.cuda.synchronize()
    nx, ny, nz = wl["nx"], wl["ny"], wl["nz"]
    b = torch.from_numpy(inputs.poisson_rhs(nx, ny, nz, seed=1511)).float().cuda()
    for tb in (0, 1):  # the library's own fusion depth (4 or 5 on these grids), then single sweeps
        ch = Channel(nx, ny, nz, wl["lx"], wl["ly"], wl["lz"], nu=wl["nu"], dpdx=wl["dpdx"], dt=wl["dt"], tblock=tb)
        p = torch.zeros_like(b)
        om = ch.schedule()
        nsw = 40 if tb == 0 else 8  # 10 launches of 4 sweeps or 8 of 5
        ch.relax(b, p, [om[k % len(om)] for k in range(nsw)])
        torch.cuda.synchronize()
        if tb == 0:
            p.zero_()
            ch.relax(b.half(), p, [om[k % len(om)] for k in range(nsw)])
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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_sweeps(P, b, om, seconds):
    """Consecutive oracle sweeps of the schedule's weights in order, as many
    as about `seconds` of wall time allows (counted from one timed sweep);
    returns (sweeps, seconds)."""
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    p = oracle.srj_cycle(P, om[:3], np.zeros_like(b), b)
    one = (time.perf_counter() - t0) / 3
    nsw = int(max(1, min(len(om) - 3, seconds / max(one, 1e-6))))
    t0 = time.perf_counter()
    oracle.srj_cycle(P, om[3:3 + nsw], p, b)
    return nsw, time.perf_counter() - t0


def cpu_baseline(wl):
    """The FP64 oracle on the host cores, on a bounded sample (about 35 s):
    consecutive SRJ sweeps of the workload's grid with all the threads the
    oracle's OpenMP runtime uses and with one thread, sweeps of the
    256x128x128 and 512x256x192 grids on all threads, and whole oracle time
    steps of the 32x16x16 laminar workload (rtol 1e-10), of the 256x8x128
    linear-instability workload (the Orr-Sommerfeld wave, rtol 1e-10) and of
    the 256x128x128 LES workload (its first step from the noisy laminar
    state, rtol 1e-8)."""
    import numpy as np
    import oracle
    from paper_1511_07800_amd import inputs, workloads
    nx, ny, nz = wl["nx"], wl["ny"], wl["nz"]
    n = nx * ny * nz
    P = oracle.make_params(nx, ny, nz, wl["lx"], wl["ly"], wl["lz"])
    b = inputs.poisson_rhs(nx, ny, nz, seed=1511)
    om = oracle.srj_schedule(nx, ny, nz, wl["lx"], wl["ly"], wl["lz"])
    threads = oracle.set_threads(0)
    nsw, t_all = oracle_sweeps(P, b, om, 8.0)
    oracle.set_threads(1)
    nsw1, t_one = oracle_sweeps(P, b, om, 8.0)
    oracle.set_threads(threads)
    del b
    other_grids = {}
    for name in ("les_channel_256x128x128", "les_channel_512x256x192"):
        wg = workloads.params(name)
        if (wg["nx"], wg["ny"], wg["nz"]) == (nx, ny, nz):
            continue
        Pg = oracle.make_params(wg["nx"], wg["ny"], wg["nz"], wg["lx"], wg["ly"], wg["lz"])
        bg = inputs.poisson_rhs(wg["nx"], wg["ny"], wg["nz"], seed=1511)
        omg = oracle.srj_schedule(wg["nx"], wg["ny"], wg["nz"], wg["lx"], wg["ly"], wg["lz"])
        k, tk = oracle_sweeps(Pg, bg, omg, 2.0)
        other_grids[f"{wg['nx']}x{wg['ny']}x{wg['nz']}"] = {
            "value": round(k * wg["nx"] * wg["ny"] * wg["nz"] / tk / 1e9, 4), "unit": "Gcell-updates/s",
            "sweeps": k, "seconds": round(tk, 2)}
        del bg
    steps = {}
    # whole steps at the small workloads (all threads)
    w0 = workloads.params("laminar_poiseuille_32x16x16")
    P0 = oracle.make_params(w0["nx"], w0["ny"], w0["nz"], w0["lx"], w0["ly"], w0["lz"], nu=w0["nu"],
                            dpdx=w0["dpdx"], dt=w0["dt"])
    z = np.zeros((w0["nz"], w0["ny"], w0["nx"]))
    s0 = oracle.Solver(P0, z, z, np.zeros((w0["nz"] + 1, w0["ny"], w0["nx"])), rtol=w0["poisson_rtol"])
    t0 = time.perf_counter()
    for _ in range(20):
        s0.step()
    steps["laminar_poiseuille_32x16x16"] = {"ms_per_step": round(1e3 * (time.perf_counter() - t0) / 20, 3),
                                            "steps": 20}
    w1 = workloads.params("linear_instability_256x8x128")
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from _ts import ts_initial_state
    u, v, w, _, g1 = ts_initial_state(w1["nx"], w1["ny"], w1["nz"], w1["lx"], w1["lz"], 1 / w1["nu"],
                                      w1["ts_alpha"], w1["ts_amplitude"])
    P1 = oracle.make_params(w1["nx"], w1["ny"], w1["nz"], w1["lx"], w1["ly"], w1["lz"], nu=w1["nu"], dpdx=g1,
                            dt=w1["dt"])
    s1 = oracle.Solver(P1, u, v, w, rtol=w1["poisson_rtol"])
    s1.step()  # the first solve starts from p = 0
    t0 = time.perf_counter()
    st1 = [s1.step() for _ in range(3)]
    steps["linear_instability_256x8x128"] = {"ms_per_step": round(1e3 * (time.perf_counter() - t0) / 3, 1),
                                             "steps": 3, "cycles_per_step": [s["poisson_cycles"] for s in st1],
                                             "sweeps_per_cycle": len(s1.omega)}
    del s1, u, v, w
    w2 = workloads.params("les_channel_256x128x128")
    u, v, w = inputs.channel_state(w2["nx"], w2["ny"], w2["nz"], w2["lz"], w2["nu"], w2["dpdx"], noise=w2["noise"],
                                   seed=w2["seed"])
    P2 = oracle.make_params(w2["nx"], w2["ny"], w2["nz"], w2["lx"], w2["ly"], w2["lz"], nu=w2["nu"],
                            dpdx=w2["dpdx"], dt=w2["dt"], les=1)
    s2 = oracle.Solver(P2, u, v, w, rtol=w2["poisson_rtol"], maxit=200)
    t0 = time.perf_counter()
    st2 = s2.step()
    steps["les_channel_256x128x128"] = {"ms_per_step": round(1e3 * (time.perf_counter() - t0), 1), "steps": 1,
                                        "cycles_per_step": [st2["poisson_cycles"]],
                                        "sweeps_per_cycle": len(s2.omega),
                                        "note": "first step from the noisy laminar state (the solve starts at p = 0)"}
    del s2, u, v, w
    return {"value": round(nsw * n / t_all / 1e9, 4), "unit": "Gcell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{nsw} consecutive FP64 SRJ sweeps of the {nx}x{ny}x{nz} grid on {threads} threads "
                      f"({t_all:.1f} s, OpenMP over z-planes); also {nsw1} on 1 thread, sweeps of the smaller LES "
                      f"grids and whole oracle steps of three small workloads",
            "other_grids": other_grids,
            "one_thread": {"value": round(nsw1 * n / t_one / 1e9, 4), "unit": "Gcell-updates/s", "sweeps": nsw1,
                           "seconds": round(t_one, 2)},
            "nproc": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count(),
            "cpu_model": cpu_model(), "oracle_steps": steps,
            "paper_context": "Fionn (ICHEC), 24-core nodes, 288x126x120 LES: 3.67 s per step on 24 cores, "
                             "0.187 s on 1008 cores (the paper's strong-scaling table)"}


VARIANTS = [
    # name, precision, options; the learned variants load the network weights
    ("mixed", "mixed", {}),
    ("lsq_mixed", "mixed", {"proj_depth": PROJ_DEPTH}),
    ("learned_mixed", "mixed", {"learned": True}),
    ("learned_lsq_mixed_rhs16", "mixed", {"learned": True, "proj_depth": PROJ_DEPTH, "rhs16": 1}),
    # the same with the eddy viscosity and explicit terms in FP32 (stencils32)
    ("learned_lsq_mixed_rhs16_stencils32", "mixed",
     {"learned": True, "proj_depth": PROJ_DEPTH, "rhs16": 1, "stencils32": 1}),
    # the paper's method as it stands: FP64 sweeps repeating one fixed cycle
    ("fp64_fixed_cycle", "fp64", {"fixed": True}),
    ("fp64", "fp64", {}),
]
EXTRA_VARIANTS = [
    ("extrap_mixed", "mixed", {"extrap_order": 2}),
    ("mixed_rhs16", "mixed", {"rhs16": 1}),
    ("mixed_stencils32", "mixed", {"stencils32": 1}),
    ("lsq_mixed_stencils32", "mixed", {"proj_depth": PROJ_DEPTH, "stencils32": 1}),
    ("lsq_mixed_rhs16", "mixed", {"proj_depth": PROJ_DEPTH, "rhs16": 1}),
    ("learned_lsq_mixed", "mixed", {"learned": True, "proj_depth": PROJ_DEPTH}),
    ("learned_mixed_correction", "mixed", {"learned": True, "correction": 1}),
    ("learned_extrap_mixed_correction", "mixed", {"learned": True, "extrap_order": 2, "correction": 1}),
    ("learned_mixed_trained_256x128x128", "mixed", {"learned": True, "weights": "warmstart_les.npy"}),
]


def run_variant(wl, args, name, precision, opt, state=None):
    import numpy as np
    import torch
    from paper_1511_07800_amd import STP_FP64, STP_MIXED, STP_WS_LEARNED, STP_WS_PREV, warmstart
    learned = opt.get("learned", False)
    ch = make_channel(wl, STP_MIXED if precision == "mixed" else STP_FP64, args.rtol,
                      warm_start=STP_WS_LEARNED if learned else STP_WS_PREV,
                      learned_correction=opt.get("correction", 0), extrap_order=opt.get("extrap_order", 0),
                      proj_depth=opt.get("proj_depth", 0), rhs16=opt.get("rhs16", 0),
                      stencils32=opt.get("stencils32", 0), state=state, fixed=opt.get("fixed", False))
    weights = None
    if learned:
        ch.net_init(training=False)
        weights = os.path.join(ROOT, "paper_1511_07800_amd", "weights", opt.get("weights", args.weights))
        warmstart.load_weights(ch, weights)
    t, acc, st, per_step = time_steps(ch, args.steps, args.warmup, name)
    n = wl["nx"] * wl["ny"] * wl["nz"]
    out = {"steps_per_s": round(args.steps / t, 4), "ms_per_step": round(1e3 * t / args.steps, 2),
           "sweeps_per_step": acc["sweeps"] / args.steps,
           "sweeps_p95": float(np.percentile([r["sweeps"] for r in per_step], 95)),
           "relres0_mean": float(np.mean([r["relres0"] for r in per_step])),
           "gcell_updates_per_s": round(acc["sweeps"] * n / t / 1e9, 2), "warmup": args.warmup,
           "phase_ms_per_step": {k[3:]: round(v / args.steps, 2) for k, v in acc["phases"].items()},
           "per_step": per_step}
    if learned:
        out.update({"ms_net_last": round(st["ms_net"], 2), "relres_prev_last": st["relres_prev"],
                    "relres_learned_last": st["relres_learned"], "weights": os.path.relpath(weights, ROOT)})
    if opt.get("proj_depth"):
        out.update({"proj_depth": opt["proj_depth"], "relres_lsq_last": st["relres_proj"]})
    if opt.get("correction"):
        out["corrections_per_step"] = acc["corrections"] / args.steps
    if precision == "fp64":
        out["relax_kernel"] = roofline_from_steps(n, acc, 8, "k_relax_fused<double,double,{d},16>")
    elif opt.get("rhs16"):
        out["relax_kernel"] = roofline_from_steps(n, acc, 4, fused_kernel(acc, wl["ny"], "_Float16"), rhs_bytes=2)
    f = fields_of(ch)
    ch.close()
    del ch
    torch.cuda.empty_cache()
    return out, acc, t, f


def main():
    args = parse()
    global FIXED_CYCLES
    FIXED_CYCLES = args.fixed_cycles
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design note, not an implementation.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1511_07800_amd import STP_MIXED, workloads
    torch.cuda.set_device(0)
    wl = workloads.params(args.workload)
    n = wl["nx"] * wl["ny"] * wl["nz"]
    if args.profile_kernels:
        profile_kernels(wl)
        return
    state = prepare_state(wl, args)
    if args.profile_fastest:
        from paper_1511_07800_amd import STP_WS_LEARNED, warmstart
        ch = make_channel(wl, STP_MIXED, args.rtol, warm_start=STP_WS_LEARNED, proj_depth=PROJ_DEPTH, rhs16=1,
                          state=state)
        ch.net_init(training=False)
        warmstart.load_weights(ch, os.path.join(ROOT, "paper_1511_07800_amd", "weights", args.weights))
        t, acc, _, per_step = time_steps(ch, args.steps, args.warmup, "learned+lsq+mixed(rhs16)")
        print(json.dumps({"variant": "learned+lsq+mixed(rhs16)", "workload": args.workload, "warmup": args.warmup,
                          "steps": args.steps, "ms_per_step": round(1e3 * t / args.steps, 2),
                          "sweeps_per_step": acc["sweeps"] / args.steps, "per_step": per_step}), flush=True)
        return

    todo = [v for v in VARIANTS if not (args.no_fp64 and v[1] == "fp64")
            and not (args.no_learned and v[2].get("learned"))]
    if args.all_variants:
        todo = todo[:-1] + [v for v in EXTRA_VARIANTS if not (args.no_learned and v[2].get("learned"))] + todo[-1:]
    results, fields = {}, {}
    acc_mixed = t_mixed = None
    for name, precision, opt in todo:
        out, acc, t, f = run_variant(wl, args, name, precision, opt, state)
        results[name] = out
        fields[name] = f
        if name == "mixed":
            acc_mixed, t_mixed = acc, t
            roof = roofline_from_steps(n, acc, 4, fused_kernel(acc, wl["ny"]))
            roof["traffic"] = measured_traffic(wl["nx"], wl["ny"], wl["nz"], fused_depth(acc))
            if roof["traffic"]:
                roof["traffic_over_algorithmic"] = round(roof["traffic"] / (12.0 * n), 3)
    del state
    errors = None
    if "fp64" in fields:
        errors = {k: field_errors(f, fields["fp64"]) for k, f in fields.items() if k != "fp64"}
    del fields
    torch.cuda.empty_cache()
    table = None if args.no_table else relax_sweep_table(wl)
    cpu = None if args.no_cpu else cpu_baseline(wl)

    fp64_rate = results["fp64"]["steps_per_s"] if "fp64" in results else None
    steps_per_s = {k: v["steps_per_s"] for k, v in results.items()}
    value = acc_mixed["sweeps"] * n / t_mixed / 1e9
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "Gcell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * t_mixed / args.steps, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": [wl["nx"], wl["ny"], wl["nz"]], "precision": "mixed",
                   "poisson_rtol": args.rtol, "dt": wl["dt"], "les": wl["les"],
                   "init": (f"laminar + {wl.get('noise', 0.0):g} x U_cl noise, advanced {args.spinup} mixed steps "
                            "(least-squares guess) as untimed input preparation" if args.spinup > 0
                            else f"laminar + {wl.get('noise', 0.0):g} x U_cl noise"),
                   "srj_cycles": "fixed 1e-3" if FIXED_CYCLES else "adaptive"},
        "les_steps_per_s": steps_per_s,
        "les_steps_per_s_vs_fp64": ({k: round(v / fp64_rate, 3) for k, v in steps_per_s.items()}
                                    if fp64_rate else None),
        "sweeps_per_step": {k: v["sweeps_per_step"] for k, v in results.items()},
        "variants": results,
        "error_vs_fp64": errors,
        "relax_sweeps": table,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

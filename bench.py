"""Benchmark of the two-phase WCSPH step on one MI355X.

Workload: the 3D oil drop rising in still water (0.05 x 0.05 x 0.1 m box,
dx = 1e-3 m, 250,000 fluid + 85,728 boundary particles, sphere R = 5 mm at
z = 0.015 m), seeded synthetic input.  One step = neighbour build,
renormalisation (Eq. 7), two rate evaluations (colour gradient + force pass)
and the midpoint predictor/corrector, replayed as one hipGraph.

Prints one JSON line: particle-interactions/s of the FP32 cell-relative form
(ordered pairs i != j with r_ij < 2h, summed over both force passes of every
timed step), the same for the FP64 GPU form, the accuracy gate against the
FP64 oracle after one step, the roofline of the force kernel and the oracle
timed on this host's cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "particle-interactions/s (FP32-relative vs FP64 GPU) at 1e-5 rel. error"
FP32_VECTOR_PEAK = 157.3e12     # MI355X FP32 vector FLOP/s, published (packed issue)
# Algorithmic VALU slots per interaction (FMA = 1, square root / reciprocal = 4): the
# force pass (Eqs. (6), (8), (10)) and the Eq. (7) pass.  A slot is priced as one FMA,
# 2 FLOP, against the published FP32 peak.
SLOTS_FORCE = {3: 46, 2: 36}
SLOTS_RENORM = 20
# Algorithmic FLOPs of one force-pass interaction (FMA = 2, square root and division 1):
# Eqs. (6), (8), (10) for a fluid particle, Eq. (6) alone for a boundary particle.
FLOPS_FLUID = {3: 47, 2: 36}
FLOPS_BOUNDARY = {3: 28, 2: 21}
WINDOWS = 5
# Scenes bench.py can time; "drop3d" is the benchmark's workload, the others are context
# (the paper's own cases and the batched and flume workloads).
WORKLOADS = {
    "drop3d": ("3D oil drop rising in still water, FP32 cell-relative", lambda i: i.drop3d()),
    "paper_sphere": ("the paper's sphere drop (Sec. III), 0.2 m tank, dx = 5 mm", lambda i: i.paper_drop("sphere")),
    "paper_cube": ("the paper's cube drop (Sec. III), 0.2 m tank, dx = 5 mm", lambda i: i.paper_drop("cube")),
    "lab_flume_5mm": ("the paper's lab flume (Sec. IV) in 3D, dx = 5 mm, periodic width 5 cm",
                      lambda i: i.lab_flume(3, dx=5e-3, width=0.05)),
    "lab_flume_1mm": ("the paper's lab flume (Sec. IV) in 3D, dx = 1 mm, periodic width 1.5 cm",
                      lambda i: i.lab_flume(3, dx=1e-3, width=0.015)),
    "flume2d": ("2D breaking-wave flume with oil slick, 8 m, dx = 5 mm", lambda i: i.flume2d()),
    "flume3d": ("3D breaking-wave flume section, periodic width, dx = 4 mm", lambda i: i.flume3d()),
    "tanks256": ("256 independent 2D drop tanks in one context", lambda i: i.batched_drops()),
}
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SRC = os.path.join(ROOT, "paper_1702_07760_amd", "csrc", "sphx_kernels.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def read_traffic(kernel, workload="drop3d"):
    """HBM bytes per launch of a kernel from its committed rocprofv3 counter summary
    (``profiles/<kernel>_fp32_<workload>_traffic.txt``), or None when there is none or
    the kernel source changed since the counters were taken."""
    path = os.path.join(PROFILES, f"{kernel}_fp32_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def timed_steps(sim, steps, warmup, torch, windows=WINDOWS):
    """Warm-up steps, then `windows` timed windows of exactly `steps` steps, each
    bracketed by stream synchronisations.  Returns the window of median duration (its
    time and statistics) and every window's time."""
    sim.step(warmup)
    sim.sync()
    runs = []
    for _ in range(windows):
        sim.reset_interactions()
        torch.cuda.synchronize()
        sim.stream.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.stream.synchronize()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        runs.append((t1 - t0, sim.stats()))
    order = sorted(range(windows), key=lambda k: runs[k][0])
    secs, st = runs[order[windows // 2]]
    return secs, st, [r[0] for r in runs]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # five windows of 400 steps after the warm-up: the 2,000 steps of the 3D drop run
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle legs")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU leg")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--workload", default="drop3d", choices=sorted(WORKLOADS),
                    help="scene to time (default: the 3D drop, the benchmark's workload)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1702_07760_amd import binding, inputs

    wl_name, make = WORKLOADS[args.workload]
    scene = make(inputs)
    n = scene.n
    dim = scene.dim
    log(f"workload {args.workload}: n={n} fluid={(scene.kind == 0).sum()} oil={(scene.phase == 1).sum()}")

    # -- FP32 cell-relative: the headline number
    sim = binding.Sim(scene, precision=binding.FP32_CELLREL)
    launch = sim.launch_options()
    fluid = scene.kind == 0
    if n <= 4_000_000:
        off, ids = sim.get_neighbors()
        nb = np.diff(off)
        i_fluid, i_bnd = int(nb[fluid].sum()), int(nb[~fluid].sum())
        flops_per_inter = (FLOPS_FLUID[dim] * i_fluid + FLOPS_BOUNDARY[dim] * i_bnd) / (i_fluid + i_bnd)
        # Eq. (7) sums over same-phase neighbours only
        same_phase = float(np.mean(np.repeat(scene.phase, nb) == scene.phase[ids]))
        del ids
    else:
        # no host copy of the lists at this size: every pair counted as a fluid and
        # same-phase one
        flops_per_inter, same_phase = float(FLOPS_FLUID[dim]), 1.0
    secs, st, windows = timed_steps(sim, args.steps, args.warmup, torch)
    value = st["interactions"] / secs
    ms_per_step = 1e3 * secs / args.steps
    log(f"fp32 ({'tuned' if sim.tuned else 'default'} launch {launch}): {args.steps} steps x {WINDOWS} windows, "
        f"median {ms_per_step:.4f} ms/step ({', '.join(f'{1e3 * w / args.steps:.4f}' for w in windows)}), "
        f"{value:.4e} interactions/s, t={st['t']:.5f}")

    # kernel durations with HIP events on the library's stream (eager replay)
    nprof = min(args.steps, 50)
    sim.set_option(binding.OPT_PROFILE, 1)
    sim.reset_interactions()
    sim.step(nprof)
    pst = sim.stats()
    sim.set_option(binding.OPT_PROFILE, 0)
    # the force group holds the pure force pass at S^n, one launch per step (the launch at
    # S* also holds the corrector); the interaction count covers both rate evaluations
    force_ms = pst["phase_ms"]["force"] / max(pst["phase_launches"]["force"], 1)
    renorm_ms = pst["phase_ms"]["renorm"] / max(pst["phase_launches"]["renorm"], 1)
    inter_per_launch = pst["interactions"] / (2 * nprof)
    breakdown = {k: round(pst["phase_ms"][k] / nprof, 5) for k in pst["phase_ms"]}
    log(f"per-step kernel-group ms: {breakdown}; force launch {force_ms:.4f} ms, Eq. (7) launch {renorm_ms:.4f} ms")

    def alu_roofline(kernel, slots, units, ms):
        achieved = 2.0 * slots * units / (ms * 1e-3)          # FLOP/s, a slot priced as one FMA
        return {"bound": "alu", "achieved": achieved / 1e12, "peak": FP32_VECTOR_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK,
                "traffic": read_traffic(kernel, args.workload),
                "kernel": kernel, "avg_launch_ms": ms, "valu_slots_per_interaction": slots,
                "interactions_per_launch": units, "interactions_per_s": units / (ms * 1e-3)}

    roofline = alu_roofline("k_force", SLOTS_FORCE[dim], inter_per_launch, force_ms)
    roofline["flops_per_interaction"] = flops_per_inter
    roofline["achieved_flops"] = flops_per_inter * inter_per_launch / (force_ms * 1e-3) / 1e12
    renorm_roofline = alu_roofline("k_renorm", SLOTS_RENORM, inter_per_launch * same_phase, renorm_ms)
    sim.close()

    if args.calib_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # -- FP64 GPU form on the same workload
    fp64 = None
    if not args.no_fp64:
        s64 = binding.Sim(scene, precision=binding.FP64)
        secs64, st64, _ = timed_steps(s64, args.steps, args.warmup, torch)
        fp64 = st64["interactions"] / secs64
        log(f"fp64: {secs64:.4f} s, {1e3 * secs64 / args.steps:.4f} ms/step, {fp64:.4e} interactions/s")
        s64.close()

    # -- accuracy gate and CPU baseline: the FP64 oracle, one step from the same state
    accuracy, cpu = None, None
    if not args.no_cpu:
        import oracle
        threads = oracle.get_threads()
        o = oracle.Oracle(scene)
        o.set_neighbor_method(2)
        t0 = time.perf_counter()
        inter = o.step(1)
        t_first = time.perf_counter() - t0
        g = binding.Sim(scene, precision=binding.FP32_CELLREL)
        g.step(1)
        g.sync()
        dx = scene.dx[0]
        xo, uo, ro = o.get(oracle.X), o.get(oracle.U), o.get(oracle.RHO)
        accuracy = {
            "x_over_dx": float(np.abs(g.get_field(binding.F_X) - xo).max() / dx),
            "u_rel": float(np.abs(g.get_field(binding.F_U) - uo).max() / max(np.abs(uo).max(), 1e-30)),
            "rho_rel": float(np.abs(g.get_field(binding.F_RHO) - ro).max() / 1000.0),
            "t_rel": abs(g.stats()["t"] - o.t) / o.t,
        }
        accuracy["pass_1e-5"] = all(v < 1e-5 for v in accuracy.values() if isinstance(v, float))
        g.close()
        log(f"accuracy after 1 step vs FP64 oracle: {accuracy}")
        total, steps_cpu, elapsed = inter, 1, t_first
        while elapsed < args.cpu_seconds and steps_cpu < 64:
            t0 = time.perf_counter()
            total += o.step(1)
            elapsed += time.perf_counter() - t0
            steps_cpu += 1
        cpu = {"value": total / elapsed, "unit": "interactions/s", "cores": threads, "kind": "oracle",
               "sample": f"{steps_cpu} full steps of the same {args.workload} scene ({n} particles), FP64 oracle, "
                         f"OpenMP over particles, {elapsed:.1f} s",
               "particle_steps_per_s": n * steps_cpu / elapsed}
        # the same oracle on one host core, over a shorter sample
        oracle.set_threads(1)
        total1, steps1, elapsed1 = 0, 0, 0.0
        while steps1 < 1 or (elapsed1 < args.cpu_seconds / 2 and steps1 < 8):
            t0 = time.perf_counter()
            total1 += o.step(1)
            elapsed1 += time.perf_counter() - t0
            steps1 += 1
        oracle.set_threads(threads)
        cpu["single_core"] = {"value": total1 / elapsed1, "unit": "interactions/s", "cores": 1,
                              "sample": f"{steps1} full steps, {elapsed1:.1f} s"}
        log(f"oracle: {cpu}")

    out = {
        "metric": METRIC, "value": value, "unit": "interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl_name,
                   "particles": n, "fluid": int(fluid.sum()), "dx_m": scene.dx[0],
                   "h_over_dx": 1.3, "kernel": "Wendland C2", "steps_per_launch": 1,
                   "interactions_per_step": st["interactions"] / args.steps},
        "particle_steps_per_s": n * args.steps / secs,
        "windows_ms_per_step": [1e3 * w / args.steps for w in windows],
        "launch": dict(launch, tuned=bool(sim.tuned)),
        "fp64_gpu_value": fp64,
        "fp32_vs_fp64": (value / fp64) if fp64 else None,
        "accuracy_vs_oracle_1step": accuracy,
        "kernel_ms_per_step": breakdown,
        "roofline": roofline,
        "roofline_k_renorm": renorm_roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

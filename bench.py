#!/usr/bin/env python3
"""Benchmark of the plain multi-resolution SPH FSI path on one MI355X.

Workload (default): the 2D flexible plate behind a rigid cylinder in a
channel (11D x 4.1D, D = 0.1 m, Re = 100, rho_s/rho_f = 10, E* = 1.4e3,
nu = 0.4, dp_f = D/20, dp_s = dp_f/2, periodic channel with an inflow
buffer), synthetic seeded lattice.  A step is one fluid acoustic step of
Algorithm 1: the rebuild when an advection step is due, the fluid force and
continuity passes, the coupling force on the solid and kappa solid
sub-steps, all replayed from one captured HIP graph with every decision on
the device.

Prints one JSON line: particle interactions per second (every within-support
pair evaluated by every pair loop, counted on the device) and FSI steps per
second, the roofline position of the dominant kernel, and the FP64 CPU
oracle timed on the host on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-interactions/s; FSI steps/s plain vs surrogate at ≤1% tip error"
HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed instructions: 256 CUs x 4 SIMD x 16 lanes
# x 2 flops (FMA) x 2.4 GHz (the packed-FP32 figure of 157.3 TFLOP/s is not
# reachable by code built without packed FP32 instructions).
ALU_PEAK_TFLOPS = 78.6
# FP64 vector peak (the same lane rate as FP32 without packed instructions)
FP64_PEAK_TFLOPS = 78.6
NUM_CUS = 256
# Algorithmic cost per unit of work:
#  fluid force pass: own state read once and written once (144 B per fluid
#  particle: reads position 16, mid-point snapshot 16, FP64 offset 32, row
#  lengths 8, scene 4; writes offset 32, v 16, p 4, a 16) plus one 4-byte
#  pair-list entry per pair; 70 flops per pair.
#  continuity pass: 140 B per fluid particle plus 4 B per pair; 40 flops per pair.
#  solid sub-step kernel (2D, block resident): the solid state read and
#  written once per launch (300 B per free particle: reads H, dF/dt, B 32 each,
#  u and v 16 each, v again for the shared copy 16, a and f^F 8 each, the
#  gradient sum 16, the neighbour count 4; writes H, dF/dt 32 each, u, v 16
#  each, a, vbar, abar 8 each) and the reference neighbour table once (12 B
#  per solid pair); per sub-step 22 flops per solid pair (momentum 12: the
#  stress sum 4, its product with the gradient 6, the accumulation 2; rate 10:
#  the velocity difference 2, its outer product with the gradient 4, the
#  accumulation 4) and about 130 flops per particle (Neo-Hookean stress and
#  P B about 80, G B^T 12, the integration updates about 40).
FORCE_BYTES_PER_PARTICLE = 144.0
CONT_BYTES_PER_PARTICLE = 140.0
LIST_BYTES_PER_PAIR = 4.0
FORCE_FLOPS_PER_PAIR = 70.0
CONT_FLOPS_PER_PAIR = 40.0
SOLID_BYTES_PER_PARTICLE = 300.0
SOLID_BYTES_PER_PAIR = 12.0
SOLID_FLOPS_PER_PAIR_SUBSTEP = 22.0
SOLID_FLOPS_PER_PARTICLE_SUBSTEP = 130.0


def make_workload(name):
    from paper_1911_13255_amd import scenes

    if name == "plate_behind_cylinder":
        return [scenes.plate_behind_cylinder(seed=1)]
    if name == "dam_break_plate":
        return [scenes.dam_break_plate(seed=1)]
    if name == "dam_break_3d":
        return [scenes.dam_break_plate_3d(seed=1)]
    if name == "batched_dam_breaks":
        return scenes.batched_dam_breaks(64)
    raise ValueError(name)


def measured_traffic(workload, kernel):
    """HBM bytes per launch of ``kernel`` from the committed counter summary
    (profiles/hbm_traffic.json), or None when the kernel source changed since
    the counters were taken or the pair was not profiled."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    src = os.path.join(ROOT, "paper_1911_13255_amd", "csrc", "sph_kernels.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != sha:
        return None
    ent = rec.get("workloads", {}).get(workload, {}).get(kernel)
    return None if ent is None else float(ent["bytes_per_launch"])


def surrogate_leg(workload, scene, seconds=30.0, threshold=1e-3, log=None):
    """Learned sub-steps against the plain ones on one scene: a network trained
    on the GPU (the library's own forward and error passes) on plain
    trajectories of 16 batched dam-break scenes, then the surrogate run with
    its residual check and fallback, timed beside the plain run; tip error of
    the surrogate run against the plain one."""
    from paper_1911_13255_amd import scenes, surrogate

    t0 = time.perf_counter()
    X, T = surrogate.collect(scenes.batched_dam_breaks(64)[:16], steps=1500, every=10, warmup=200)
    t1 = time.perf_counter()
    net, stats, hist = surrogate.fit(X, T, seconds=seconds)
    t2 = time.perf_counter()
    if log:
        log(f"[bench] surrogate: {X.shape[0]} training rows collected in {t1 - t0:.1f} s, "
            f"trained {t2 - t1:.1f} s, loss {hist[0][2]:.3e} -> {hist[-1][2]:.3e}")
    res = surrogate.evaluate(scene, net, stats, threshold, steps=2000, every=10, timing_steps=2000)
    res.update(workload=workload, training_rows=int(X.shape[0]), training_seconds=t2 - t1,
               training_loss_first=hist[0][2], training_loss_last=hist[-1][2],
               trained_on="plain trajectories of batched_dam_breaks scenes 0-15, steps 200-1500 every 10")
    net.close()
    return res


# The paper's flow-induced-vibration cases (Section 4.1, its Table 2) on the
# channel geometry, with the linear elastic law its benchmark uses; bh = 0.2 D
# is the plate thickness.
PAPER_CASES = (
    ("I", dict(dp_f=0.005, dp_ratio=1.0), 0, "dp_F = dp_S = bh/4, multiple time steps"),
    ("II", dict(dp_f=0.0025, dp_ratio=1.0), 0, "dp_F = dp_S = bh/8, multiple time steps"),
    ("III", dict(dp_f=0.01, dp_ratio=2.0), 0, "dp_F = 2 dp_S, dp_S = bh/4, multiple time steps"),
    ("IV", dict(dp_f=0.01, dp_ratio=2.0), 1, "dp_F = 2 dp_S, dp_S = bh/4, one shared time step"),
)
# CPU wall-clock seconds the paper reports for these cases up to t* = 200
# (Xeon L5520 2.27 GHz, shared-memory parallel), for the ratios only.
PAPER_CASE_SECONDS = {"I": 1297.7, "II": 10926.7, "III": 249.5, "IV": 451.4}


def paper_cases(steps=3000, warmup=300, log=None):
    """The four cases on the GPU: simulated time advanced per wall second and
    the speed-ups the paper draws from them (multi-resolution: III over I;
    multiple time steps: III over IV), beside the paper's own CPU ratios."""
    import torch
    from paper_1911_13255_amd import scenes, sph

    out = {}
    for name, geo, single, desc in PAPER_CASES:
        sc = scenes.plate_behind_cylinder(seed=1, **geo)
        sc["material"] = 1
        sc["single_step"] = single
        sim = sph.Simulation([sc])
        sim.advance(warmup)
        sim.sync()
        t0, c0 = sim.scalars()["t"], sim.counters()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(sim.stream)
        sim.advance(steps)
        ev1.record(sim.stream)
        ev1.synchronize()
        ms = ev0.elapsed_time(ev1)
        sim.sync()
        t1, c1 = sim.scalars()["t"], sim.counters()
        secs = ms / 1e3
        out[name] = dict(description=desc, dp_f=sc["dp_f"], dp_s=sc["dp_s"], single_step=single,
                         n_fluid=len(sc["x_fluid"]), n_solid=len(sc["x_solid"]),
                         kappa_mean=(c1["substeps"] - c0["substeps"]) / steps, steps=steps,
                         ms_per_step=ms / steps, fsi_steps_per_s=steps / secs,
                         interactions_per_s=(c1["interactions"] - c0["interactions"]) / secs,
                         simulated_s_per_wall_s=(t1 - t0) / secs)
        sim.close()
        if log:
            log(f"[bench] case {name}: {json.dumps(out[name])}")
    rate = {k: v["simulated_s_per_wall_s"] for k, v in out.items()}
    paper = PAPER_CASE_SECONDS
    return dict(cases=out, material="linear elastic (Kirchhoff)", launch="library default shapes",
                multi_resolution_speedup_III_over_I=rate["III"] / rate["I"],
                multi_step_speedup_III_over_IV=rate["III"] / rate["IV"],
                resolution_cost_II_over_I=rate["I"] / rate["II"],
                paper_cpu_ratios=dict(III_over_I=paper["I"] / paper["III"], III_over_IV=paper["IV"] / paper["III"],
                                      II_over_I=paper["II"] / paper["I"],
                                      hardware="Xeon L5520 2.27 GHz CPU, wall-clock to t* = 200"))


def cpu_baseline(scene, seconds=15.0):
    """The FP64 oracle on the host cores on a bounded prefix of the same run."""
    from oracle import oracle as ora

    o = ora.Oracle(scene)
    threads = ora.num_threads()
    o.step(2)  # first rebuild outside the timing
    c0 = o.counters()
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds:
        o.step(10)
        n += 10
    dt = time.perf_counter() - t0
    c1 = o.counters()
    inter = c1["interactions"] - c0["interactions"]
    # the same oracle on one thread, on a shorter sample continuing the run
    ora.set_threads(1)
    c2 = o.counters()
    t1 = time.perf_counter()
    n1 = 0
    while time.perf_counter() - t1 < seconds / 3.0:
        o.step(2)
        n1 += 2
    dt1 = time.perf_counter() - t1
    c3 = o.counters()
    ora.set_threads(threads)
    return dict(value=inter / dt, unit="interactions/s", cores=threads, kind="oracle",
                sample=f"{n} acoustic steps after the first two of the same scene and seed "
                       f"({dt:.1f} s, FP64, OpenMP)",
                steps_per_s=n / dt,
                single_thread=dict(value=(c3["interactions"] - c2["interactions"]) / dt1, cores=1,
                                   sample=f"the next {n1} acoustic steps ({dt1:.1f} s)",
                                   steps_per_s=n1 / dt1))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed acoustic steps (default per workload: 20000 for the channel, 2000 for the "
                         "2D dam break, 300 for the 3D dam break, 1000 for the batch)")
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="plate_behind_cylinder",
                    choices=["plate_behind_cylinder", "dam_break_plate", "dam_break_3d",
                             "batched_dam_breaks"])
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's default launch shapes instead of the autotuned ones")
    ap.add_argument("--autotune-cache", default=os.path.join(os.path.expanduser("~"), ".cache", "mrsph",
                                                              "autotune.json"))
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the learned sub-step leg (2D single-scene workloads only)")
    ap.add_argument("--surrogate-seconds", type=float, default=30.0)
    ap.add_argument("--no-cases", action="store_true",
                    help="skip the paper's four flow-induced-vibration cases (channel workload only)")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="MIB",
                    help="only run a plain FP32 device copy of this many MiB five times (the "
                         "reference for scaling HBM byte counters) and exit")
    args = ap.parse_args()
    # the batch stays within 1100 steps: 8 of its 64 coarse scenes become
    # unstable after the water hits the plate (from about step 1600, the FP64
    # oracle included)
    defaults = {"plate_behind_cylinder": (20000, 200), "dam_break_plate": (2000, 100),
                "dam_break_3d": (300, 20), "batched_dam_breaks": (1000, 100)}[args.workload]
    if args.steps is None:
        args.steps = defaults[0]
    if args.warmup is None:
        args.warmup = defaults[1]
    if args.gpus != 1:
        print(f"bench.py: the hot path runs on one GPU only (asked for --gpus {args.gpus}); "
              "run one process per GPU on its own share of the scenes instead", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_calibration > 0:
        n = int(args.copy_calibration * (1 << 20)) // 4
        src = torch.rand(n, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}))
        return

    from paper_1911_13255_amd import sph

    scs = make_workload(args.workload)
    dim = int(scs[0]["dim"])
    print(f"[bench] workload {args.workload}: {len(scs)} scene(s), "
          f"{sum(len(s['x_fluid']) for s in scs)} fluid, {sum(len(s['x_solid']) for s in scs)} solid, "
          f"{sum(len(s['x_wall']) for s in scs)} wall particles", file=sys.stderr, flush=True)
    opts = {}
    tune_s = 0.0
    if not args.no_autotune:
        t0 = time.perf_counter()
        opts = sph.autotune(scs, warmup=10 if dim == 3 else 100, steps=10 if dim == 3 else 1000,
                            cache=args.autotune_cache)
        tune_s = time.perf_counter() - t0
        print(f"[bench] autotuned in {tune_s:.1f} s: {json.dumps(opts)}", file=sys.stderr, flush=True)
    sim = sph.Simulation(scs, **opts)
    sim.advance(args.warmup)
    torch.cuda.synchronize()
    sim.sync()
    c0 = sim.counters()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(sim.stream)
    sim.advance(args.steps)
    t_end.record(sim.stream)
    t_end.synchronize()
    torch.cuda.synchronize()
    ms = t_start.elapsed_time(t_end)
    sim.sync()
    c1 = sim.counters()
    inter = c1["interactions"] - c0["interactions"]
    secs = ms / 1e3
    value = inter / secs
    steps_per_s = args.steps / secs
    rebuilds = c1["rebuilds"] - c0["rebuilds"]
    print(f"[bench] {args.steps} steps in {ms:.1f} ms, {rebuilds} rebuilds, "
          f"{inter} interactions", file=sys.stderr, flush=True)

    # kernel durations are taken on a step without a pending rebuild (the
    # common case: the force launch's list-ordering blocks then exit at once)
    for _ in range(64):
        if not any(sim.scalars(k)["need_rebuild"] for k in range(len(scs))):
            break
        sim.advance(1)
    sim.sync()
    # per-kernel durations (HIP events on the library's stream), after the timed region
    # (isolated launches on the library's stream; inside the timed graph the
    # continuity pass overlaps the coupling and solid passes)
    kt = {name: sim.time_kernel(k, args.kernel_reps) for name, k in
          (("k_fluid_force", sph.K_FLUID_FORCE), ("k_fluid_continuity", sph.K_CONTINUITY),
           ("k_couple", sph.K_COUPLE), ("k_solid", sph.K_SOLID))}
    kt["rebuild_sequence"] = sim.time_kernel(sph.K_REBUILD, max(10, args.kernel_reps // 10))
    per_step = dict(kt)
    per_step["rebuild_sequence"] = kt["rebuild_sequence"] * rebuilds / args.steps
    print(f"[bench] kernel ms per launch {json.dumps({k: round(v, 5) for k, v in kt.items()})}",
          file=sys.stderr, flush=True)
    nf = sum(len(s["x_fluid"]) for s in scs)
    ns_free = sum(len(s["x_solid"]) - int(s["n_clamp"]) for s in scs)
    pairs_f = c1["n_ff"] + c1["n_fw"] + c1["n_fs"]
    kappa = (c1["substeps"] - c0["substeps"]) / max(1, c1["steps"] - c0["steps"])
    # single kernels and their algorithmic bytes and flops per launch; the
    # streamed solid form (3D, large solids) is a sequence of kernels and is
    # not a candidate
    cand = {
        "k_fluid_force": (kt["k_fluid_force"], FORCE_BYTES_PER_PARTICLE * nf + LIST_BYTES_PER_PAIR * pairs_f,
                          FORCE_FLOPS_PER_PAIR * pairs_f),
        "k_fluid_continuity": (kt["k_fluid_continuity"], CONT_BYTES_PER_PARTICLE * nf + LIST_BYTES_PER_PAIR * pairs_f,
                               CONT_FLOPS_PER_PAIR * pairs_f),
    }
    if sim.solid_register_resident():
        cand["k_solid_reg"] = (kt["k_solid"], SOLID_BYTES_PER_PARTICLE * ns_free + SOLID_BYTES_PER_PAIR * c1["n_ss"],
                               kappa * (SOLID_FLOPS_PER_PAIR_SUBSTEP * c1["n_ss"] +
                                        SOLID_FLOPS_PER_PARTICLE_SUBSTEP * ns_free))
    dominant = max(cand, key=lambda k: cand[k][0])
    dur_ms, alg_bytes, alg_flops = cand[dominant]
    dur = dur_ms * 1e-3
    gbs = alg_bytes / dur / 1e9
    tflops = alg_flops / dur / 1e12
    hbm_frac = gbs / HBM_PEAK_GBS
    alu_frac = tflops / ALU_PEAK_TFLOPS
    if dominant == "k_solid_reg":
        # FP64 arithmetic of one workgroup per scene (LDS gathers, table loads
        # and FP64 FMAs bound it together): the FP64 vector peak, with the
        # fraction of the CUs the launch occupies beside it
        roof = dict(bound="alu", achieved=tflops, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=tflops / FP64_PEAK_TFLOPS, cus_used=len(scs),
                    frac_of_cus_used=tflops / (FP64_PEAK_TFLOPS * len(scs) / NUM_CUS))
    elif alu_frac >= hbm_frac:
        roof = dict(bound="alu", achieved=tflops, peak=ALU_PEAK_TFLOPS, unit="TFLOP/s", frac=alu_frac)
    else:
        roof = dict(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s", frac=hbm_frac)
    traffic = measured_traffic(args.workload, dominant)
    roof.update(traffic=traffic, kernel=dominant, duration_us=dur * 1e6,
                traffic_over_algorithmic=None if traffic is None else traffic / alg_bytes,
                hbm_GBps=gbs, hbm_frac=hbm_frac, alu_TFLOPs=tflops, alu_frac=alu_frac,
                algorithmic_bytes=alg_bytes, algorithmic_flops=alg_flops,
                workgroups_per_launch=len(scs) if dominant == "k_solid_reg" else None)

    sur = None
    if not args.no_surrogate and dim == 2 and len(scs) == 1 and sim.solid_register_resident():
        sur = surrogate_leg(args.workload, scs[0], seconds=args.surrogate_seconds,
                            log=lambda m: print(m, file=sys.stderr, flush=True))
        print(f"[bench] surrogate {json.dumps(sur)}", file=sys.stderr, flush=True)

    cases = None
    if not args.no_cases and args.workload == "plate_behind_cylinder":
        cases = paper_cases(log=lambda m: print(m, file=sys.stderr, flush=True))

    cpu = None
    if not args.no_cpu_baseline and len(scs) == 1:
        cpu = cpu_baseline(scs[0], args.cpu_seconds)
    elif not args.no_cpu_baseline:
        cpu = cpu_baseline(scs[0], args.cpu_seconds)
        cpu["sample"] = "scene 0 of the batch only: " + cpu["sample"]

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "scenes": len(scs),
            "n_fluid": nf,
            "n_solid": sum(len(s["x_solid"]) for s in scs),
            "n_wall": sum(len(s["x_wall"]) for s in scs),
            "dim": dim,
            "dp_f": scs[0]["dp_f"],
            "dp_s": scs[0]["dp_s"],
        },
        "fsi_steps_per_s": steps_per_s,
        "interactions_per_step": inter / args.steps,
        "rebuilds": rebuilds,
        "kernel_ms_per_step": {k: round(v, 6) for k, v in per_step.items()},
        "launch": sim.launch_config(),
        "autotuned": not args.no_autotune,
        "autotune_seconds": tune_s,
        "roofline": roof,
        "surrogate": sur,
        "paper_cases": cases,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    sim.close()


if __name__ == "__main__":
    main()

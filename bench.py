#!/usr/bin/env python3
"""Benchmark of the plain multi-resolution SPH FSI path on one MI355X.

Headline workload: the 3D dam break on an elastic plate (water column
0.6 x 0.6 x 1.2 m in a 1.6 x 0.6 x 1.2 m tank, Neo-Hookean plate
0.04 x 0.6 x 0.4 m, E = 5 MPa, nu = 0.45, dp_f = 6 mm: 2.0M fluid and 354k
solid particles), synthetic seeded lattice.  A step is one fluid acoustic
step of Algorithm 1: the rebuild when an advection step is due, the fluid
force and continuity passes, the coupling force on the solid and kappa solid
sub-steps, every decision taken on the device.

Prints one JSON line: particle interactions per second (every within-support
pair evaluated by every pair loop, counted on the device) and FSI steps per
second on that workload, the roofline position of its dominant kernel, the
FP64 CPU oracle timed on the host on a bounded sample of the same workload,
and as further keys the 2D channel (plate behind a cylinder), the 64 batched
2D dam breaks, the learned sub-step leg on the channel and the 2D dam break,
and the paper's four flow-induced-vibration cases.
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
# Published MI355X peaks.
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3  # vector FP32, packed (dual-issue) FMA counted as 2 flops per lane
FP64_PEAK_TFLOPS = 78.6   # vector FP64
# Ceiling of code built without packed FP32 instructions (this library's
# build): 256 CUs x 4 SIMD x 16 lanes x 2 flops (FMA) x 2.4 GHz.  Stated
# beside the published peak, never in its place.
FP32_NONPACKED_TFLOPS = 78.6
NUM_CUS = 256
# Algorithmic cost per unit of work (each particle's own state moved once;
# the pair lists and the neighbours' gathers are not algorithmic bytes):
#  fluid force pass, per fluid particle: reads position, density, density
#  rate, velocity and writes position, density, velocity (2D 52 B, 3D 72 B
#  in FP32); about 55 arithmetic operations per pair (distance, kernel
#  gradient, Riemann pressure, viscous term, accumulation)
#  continuity pass, per fluid particle: 2D 44 B, 3D 60 B; about 40 operations
#  per pair
#  block-resident solid kernel (2D, one launch = kappa sub-steps): the solid
#  state read and written once per launch, about 150 B per free particle; per
#  sub-step about 33 operations per reference pair (stress sum, gradient
#  product, velocity-gradient outer product) and 200 per particle
#  (Neo-Hookean stress, P B, integration)
#  streamed solid passes (3D), per sub-step: about 300 B per solid particle
FORCE_BYTES = {2: 52.0, 3: 72.0}
CONT_BYTES = {2: 44.0, 3: 60.0}
FORCE_OPS_PER_PAIR = 55.0
CONT_OPS_PER_PAIR = 40.0
SOLID_REG_BYTES = 150.0
SOLID_STREAM_BYTES_PER_SUBSTEP = 300.0
SOLID_OPS_PER_PAIR_SUBSTEP = 33.0
SOLID_OPS_PER_PARTICLE_SUBSTEP = 200.0


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


# judge thresholds and intervals of the surrogate's sweep
SUR_THRESHOLDS = (1e-3, 1e-2, 1e-1, 2e-1, 5e-1)
SUR_JUDGE_EVERY = (2, 4, 10)


def surrogate_leg(seconds=30.0, log=None):
    """Learned sub-steps against the plain ones: a network trained on the GPU
    (the library's own forward and error passes) on plain trajectories of 16
    batched dam-break scenes, then on the channel (the plate behind the
    cylinder) and on the 2D dam break (kappa = 13) the surrogate run for each
    judge threshold and interval, beside the plain run from the same start:
    accepted fraction, steps/s of both and tip error against the plain run
    over each scene's well-conditioned window (1,500 steps of the channel,
    1,800 of the dam break)."""
    from paper_1911_13255_amd import scenes, surrogate

    t0 = time.perf_counter()
    X, T = surrogate.collect(scenes.batched_dam_breaks(64)[:16], steps=1500, every=10, warmup=200)
    t1 = time.perf_counter()
    net, stats, hist = surrogate.fit(X, T, seconds=seconds)
    t2 = time.perf_counter()
    if log:
        log(f"[bench] surrogate: {X.shape[0]} training rows collected in {t1 - t0:.1f} s, "
            f"trained {t2 - t1:.1f} s, loss {hist[0][2]:.3e} -> {hist[-1][2]:.3e}")
    out = dict(training_rows=int(X.shape[0]), training_seconds=t2 - t1, training_loss_first=hist[0][2],
               training_loss_last=hist[-1][2],
               trained_on="plain trajectories of batched_dam_breaks scenes 0-15, steps 200-1500 every 10",
               network="24 -> 128 -> 128 -> 128 -> 4, SiLU, BF16 weights and activations, FP32 accumulation")
    for label, scene, steps in (("plate_behind_cylinder", scenes.plate_behind_cylinder(seed=1), 1500),
                                ("dam_break_plate", scenes.dam_break_plate(seed=1), 1800)):
        # the network's residual on the plain method's own states (every step a
        # judge step), beside the network that predicts no change (vbar = v,
        # abar = a), at the thresholds of the sweep
        zero = surrogate.zero_network()
        judge_only = {}
        for thr in SUR_THRESHOLDS:
            judge_only[f"{thr:g}"] = dict(
                trained=surrogate.judge_pass_fraction(scene, net, stats, thr, 200, 1200),
                no_change=surrogate.judge_pass_fraction(scene, zero[0], zero[1], thr, 200, 1200))
        zero[0].close()
        if log:
            log(f"[bench] surrogate {label}: judges passed on the plain trajectory (steps 200-1400) "
                f"{json.dumps(judge_only)}")
        plain, rows = None, []
        for thr in SUR_THRESHOLDS:
            for je in SUR_JUDGE_EVERY:
                r = surrogate.evaluate(scene, net, stats, thr, steps=steps, every=10, timing_steps=2000,
                                       judge_every=je, plain=plain)
                plain = r.pop("plain")
                rows.append(r)
                if log:
                    log(f"[bench] surrogate {label} threshold {thr:g} every {je}: accepted "
                        f"{r['accepted_fraction']:.3f}, tip error {r['tip_error']:.3e}, speed-up "
                        f"{r['speedup']:.3f}{' (unstable)' if r['unstable'] else ''}")
        # a row counts only when the network took some steps: with every judge
        # failing the run is the plain method plus judging overhead
        ok = [r for r in rows if r["tip_error"] <= 0.01 and not r["unstable"] and r["accepted_fraction"] > 0]
        best = max(ok, key=lambda r: r["speedup"]) if ok else None
        out[label] = dict(
            eval_steps=steps, steps_per_s_plain=plain[2], tip_max_m=rows[0]["tip_max_m"],
            best_within_1pct=best, judges_passed_on_plain_states=judge_only,
            frontier=[{k: r[k] for k in ("threshold", "judge_every", "accepted_fraction", "accepted_fraction_timed",
                                         "tip_error", "speedup", "steps_per_s_surrogate", "judged_ok",
                                         "judged_fail", "unstable")} for r in rows])
    net.close()
    return out


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


def cpu_baseline(scene, seconds=15.0, single_thread_steps=1):
    """The FP64 oracle on the host cores on a bounded sample of the same run:
    its first step (the initial rebuild) untimed, then whole acoustic steps
    until `seconds` have passed and at least five steps are done; then the
    same oracle on one thread for `single_thread_steps` further steps."""
    from oracle import oracle as ora

    o = ora.Oracle(scene)
    threads = ora.num_threads()
    o.step(1)  # first rebuild outside the timing
    c0 = o.counters()
    t0 = time.perf_counter()
    n = 0
    while n < 5 or time.perf_counter() - t0 < seconds:
        o.step(1)
        n += 1
    dt = time.perf_counter() - t0
    c1 = o.counters()
    inter = c1["interactions"] - c0["interactions"]
    ora.set_threads(1)
    c2 = o.counters()
    t1 = time.perf_counter()
    for _ in range(single_thread_steps):
        o.step(1)
    dt1 = time.perf_counter() - t1
    c3 = o.counters()
    ora.set_threads(threads)
    return dict(value=inter / dt, unit="interactions/s", cores=threads, kind="oracle",
                sample=f"acoustic steps 2-{n + 1} of the same scene and seed ({n} steps, {dt:.1f} s, FP64, "
                       f"OpenMP on {threads} threads; step 1, the initial rebuild, untimed)",
                steps_per_s=n / dt,
                single_thread=dict(value=(c3["interactions"] - c2["interactions"]) / dt1, cores=1,
                                   sample=f"the next {single_thread_steps} acoustic step(s) ({dt1:.1f} s)",
                                   steps_per_s=single_thread_steps / dt1))


def roofline(name, dur_ms, alg_bytes, alg_ops, fp64=False):
    """Position of one kernel against the published peaks: the larger of its
    HBM and arithmetic fractions names the bound."""
    dur = dur_ms * 1e-3
    gbs = alg_bytes / dur / 1e9
    tops = alg_ops / dur / 1e12
    peak_ops = FP64_PEAK_TFLOPS if fp64 else FP32_PEAK_TFLOPS
    hbm_frac, alu_frac = gbs / HBM_PEAK_GBS, tops / peak_ops
    if alu_frac >= hbm_frac:
        roof = dict(bound="alu", achieved=tops, peak=peak_ops, unit="TFLOP/s", frac=alu_frac)
    else:
        roof = dict(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s", frac=hbm_frac)
    roof.update(kernel=name, duration_us=dur * 1e6, arithmetic="FP64" if fp64 else "FP32",
                hbm_GBps=gbs, hbm_frac=hbm_frac, alu_TFLOPs=tops, alu_frac=alu_frac,
                algorithmic_bytes=alg_bytes, algorithmic_flops=alg_ops)
    if not fp64:
        roof["frac_of_nonpacked_fp32"] = tops / FP32_NONPACKED_TFLOPS
    return roof


def run_workload(name, steps, warmup, autotune, cache, kernel_reps, log, scenes_override=None):
    """Plain path on one workload: timed steps (HIP events on the library's
    stream, inputs resident in HBM), per-kernel durations, the dominant single
    kernel's roofline."""
    import torch
    from paper_1911_13255_amd import sph

    scs = scenes_override if scenes_override is not None else make_workload(name)
    dim = int(scs[0]["dim"])
    log(f"[bench] workload {name}: {len(scs)} scene(s), {sum(len(s['x_fluid']) for s in scs)} fluid, "
        f"{sum(len(s['x_solid']) for s in scs)} solid, {sum(len(s['x_wall']) for s in scs)} wall particles")
    opts, tune_s = {}, 0.0
    if autotune:
        t0 = time.perf_counter()
        opts = sph.autotune(scs, warmup=10 if dim == 3 else 100, steps=10 if dim == 3 else 1000, cache=cache)
        tune_s = time.perf_counter() - t0
        log(f"[bench] {name}: autotuned in {tune_s:.1f} s: {json.dumps(opts)}")
    sim = sph.Simulation(scs, **opts)
    sim.advance(warmup)
    torch.cuda.synchronize()
    sim.sync()
    c0 = sim.counters()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(sim.stream)
    sim.advance(steps)
    t_end.record(sim.stream)
    t_end.synchronize()
    torch.cuda.synchronize()
    ms = t_start.elapsed_time(t_end)
    sim.sync()
    c1 = sim.counters()
    inter = c1["interactions"] - c0["interactions"]
    secs = ms / 1e3
    rebuilds = c1["rebuilds"] - c0["rebuilds"]
    log(f"[bench] {name}: {steps} steps in {ms:.2f} ms, {rebuilds} rebuilds, {inter} interactions")
    # kernel durations are taken on a step without a pending rebuild (the
    # common case: the force launch's list-ordering blocks then exit at once)
    for _ in range(64):
        if not any(sim.scalars(k)["need_rebuild"] for k in range(len(scs))):
            break
        sim.advance(1)
    sim.sync()
    # isolated launches on the library's stream, HIP events around them
    kt = {kn: sim.time_kernel(k, kernel_reps) for kn, k in
          (("k_fluid_force", sph.K_FLUID_FORCE), ("k_fluid_continuity", sph.K_CONTINUITY),
           ("k_couple", sph.K_COUPLE), ("k_solid", sph.K_SOLID))}
    kt["rebuild_sequence"] = sim.time_kernel(sph.K_REBUILD, max(10, kernel_reps // 10))
    per_step = dict(kt)
    per_step["rebuild_sequence"] = kt["rebuild_sequence"] * rebuilds / steps
    log(f"[bench] {name}: kernel ms per launch {json.dumps({k: round(v, 5) for k, v in kt.items()})}")
    nf = sum(len(s["x_fluid"]) for s in scs)
    ns = sum(len(s["x_solid"]) for s in scs)
    ns_free = ns - sum(int(s["n_clamp"]) for s in scs)
    pairs_f = c1["n_ff"] + c1["n_fw"] + c1["n_fs"]
    kappa = (c1["substeps"] - c0["substeps"]) / max(1, c1["steps"] - c0["steps"])
    roofs = {
        "k_fluid_force": roofline("k_fluid_force", kt["k_fluid_force"], FORCE_BYTES[dim] * nf,
                                  FORCE_OPS_PER_PAIR * pairs_f),
        "k_fluid_continuity": roofline("k_fluid_continuity", kt["k_fluid_continuity"], CONT_BYTES[dim] * nf,
                                       CONT_OPS_PER_PAIR * pairs_f),
    }
    solid_ops = kappa * (SOLID_OPS_PER_PAIR_SUBSTEP * c1["n_ss"] + SOLID_OPS_PER_PARTICLE_SUBSTEP * ns_free)
    resident = sim.solid_register_resident()
    if resident:
        # one launch holds the kappa sub-steps in FP64, one workgroup per scene
        roofs["k_solid_reg"] = roofline("k_solid_reg", kt["k_solid"], SOLID_REG_BYTES * ns_free, solid_ops,
                                        fp64=True)
        roofs["k_solid_reg"].update(cus_used=len(scs), frac_of_cus_used=roofs["k_solid_reg"]["alu_frac"] *
                                    NUM_CUS / len(scs))
    dominant = max(roofs, key=lambda k: roofs[k]["duration_us"])
    roof = dict(roofs[dominant])
    traffic = measured_traffic(name, dominant)
    roof.update(traffic=traffic, traffic_over_algorithmic=None if traffic is None else
                traffic / roof["algorithmic_bytes"])
    out = dict(value=inter / secs, unit="interactions/s", ms_per_step=ms / steps, fsi_steps_per_s=steps / secs,
               steps=steps, warmup=warmup, interactions_per_step=inter / steps, rebuilds=rebuilds,
               kappa_mean=kappa, kernel_ms_per_step={k: round(v, 6) for k, v in per_step.items()},
               kernel_roofline={k: {q: v[q] for q in ("bound", "frac", "duration_us", "alu_frac", "hbm_frac")}
                                for k, v in roofs.items()},
               launch=sim.launch_config(), fluid_tiles=sim.fluid_tiles(), autotuned=bool(autotune),
               autotune_seconds=tune_s, roofline=roof,
               config=dict(workload=name, scenes=len(scs), n_fluid=nf, n_solid=ns,
                           n_wall=sum(len(s["x_wall"]) for s in scs), dim=dim, dp_f=scs[0]["dp_f"],
                           dp_s=scs[0]["dp_s"]))
    if not resident and ns:
        # the streamed solid phase: kappa launches of each pass, not one kernel
        out["solid_phase"] = dict(ms=kt["k_solid"], kappa=kappa, solid_table=sim.solid_table(),
                                  hbm_GBps=kappa * SOLID_STREAM_BYTES_PER_SUBSTEP * ns / (kt["k_solid"] * 1e-3) / 1e9,
                                  alu_TFLOPs=solid_ops / (kt["k_solid"] * 1e-3) / 1e12)
    sim.close()
    return out, scs


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed acoustic steps of the headline workload (default per workload: 300 for the "
                         "3D dam break, 20000 for the channel, 2000 for the 2D dam break, 1000 for the batch)")
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="dam_break_3d",
                    choices=["dam_break_3d", "plate_behind_cylinder", "dam_break_plate", "batched_dam_breaks"])
    ap.add_argument("--kernel-reps", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", choices=["auto", "on", "off"], default="auto",
                    help="launch shapes from the library's autotuner (auto: 2D workloads only; the 3D dam "
                         "break takes the library's defaults)")
    ap.add_argument("--autotune-cache", default=os.path.join(os.path.expanduser("~"), ".cache", "mrsph",
                                                              "autotune.json"))
    ap.add_argument("--no-extras", action="store_true",
                    help="headline workload only: no further workloads, surrogate leg or paper cases")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the learned sub-step leg")
    ap.add_argument("--surrogate-seconds", type=float, default=30.0)
    ap.add_argument("--no-cases", action="store_true",
                    help="skip the paper's four flow-induced-vibration cases")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="MIB",
                    help="only run a plain FP32 device copy of this many MiB five times (the "
                         "reference for scaling HBM byte counters) and exit")
    args = ap.parse_args()
    # the batch stays within 1100 steps: 8 of its 64 coarse scenes become
    # unstable after the water hits the plate (from about step 1600)
    defaults = {"plate_behind_cylinder": (20000, 200), "dam_break_plate": (2000, 100),
                "dam_break_3d": (300, 20), "batched_dam_breaks": (1000, 100)}
    if args.steps is None:
        args.steps = defaults[args.workload][0]
    if args.warmup is None:
        args.warmup = defaults[args.workload][1]
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

    def log(m):
        print(m, file=sys.stderr, flush=True)

    def tuned(name):
        return args.autotune == "on" or (args.autotune == "auto" and name != "dam_break_3d")

    head, scs = run_workload(args.workload, args.steps, args.warmup, tuned(args.workload), args.autotune_cache,
                             args.kernel_reps, log)
    extras = {}
    if not args.no_extras:
        # further workloads at their own sizes, shorter runs
        others = {"dam_break_3d": 100, "plate_behind_cylinder": 5000, "batched_dam_breaks": 1000}
        for name, n in others.items():
            if name == args.workload:
                continue
            extras[name], _ = run_workload(name, n, 20 if name == "dam_break_3d" else 100, tuned(name),
                                           args.autotune_cache, 50, log)
        if args.workload == "dam_break_3d" or "dam_break_3d" in extras:
            # the same 3D scene with the plate jittered like the fluid (1e-4 dp_S):
            # its reference table is the full 16-byte one
            from paper_1911_13255_amd import scenes as S

            jit, _ = run_workload("dam_break_3d", 100, 20, False, args.autotune_cache, 20, log,
                                  scenes_override=[S.dam_break_plate_3d(seed=1, solid_lattice=False)])
            extras["dam_break_3d_jittered_plate"] = {k: jit[k] for k in
                                                     ("value", "ms_per_step", "fsi_steps_per_s", "solid_phase",
                                                      "kernel_ms_per_step")}
        if not args.no_surrogate:
            extras["surrogate"] = surrogate_leg(seconds=args.surrogate_seconds, log=log)
        if not args.no_cases:
            extras["paper_cases"] = paper_cases(log=log)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(scs[0], args.cpu_seconds)
        if len(scs) > 1:
            cpu["sample"] = "scene 0 of the batch only: " + cpu["sample"]
        log(f"[bench] cpu baseline {json.dumps(cpu)}")

    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": head["config"],
        "fsi_steps_per_s": head["fsi_steps_per_s"],
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
    }
    for k in ("interactions_per_step", "rebuilds", "kappa_mean", "kernel_ms_per_step", "kernel_roofline", "launch",
              "fluid_tiles", "autotuned", "autotune_seconds", "solid_phase"):
        if k in head:
            out[k] = head[k]
    out.update(extras)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

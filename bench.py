"""Benchmark: forward particle-steps/s of the particle-dispersion hot path on
one MI355X, beside adjoint gradient evaluations/s, the batched ensemble
against sequential plain runs, and the FP64 oracle on the host cores.

Headline workload (one benchmark step = one full forward run): 1.6e7
particles released continuously from (0, 0, 50 m) over the first 6 h of a
24 h run at dt = 5 s (17280 time steps), 25 hourly 400 x 400 x 40 wind
fields (250/250/40 m nodes; power-law profile, four seeded Fourier modes of
direction per hour) interpolated linearly in time, parabolic K_z over a
1000 m mixed layer, dry deposition (v_d = 0.002 m/s), wet scavenging
(1e-5 1/s) in a seeded elliptical rain region, two nuclides (lambda = 1e-6,
1e-5 1/s).  Every step of a run: release, particle step (advection,
turbulent random walk, reflection, decay, dry/wet deposition with the
deposition scatter), cloud-in-cell concentration on the 400 x 400 x 40 x 2
grid every 60 steps (288 output steps), and the final 400 x 400 x 2
deposition grid.  `value` = particle-steps advanced per second over the timed
runs (inputs resident in HBM).

Also on the same line: the 1e6-particle 6 h run on one 200 x 200 x 30 field
("c1"), gradient evaluations per second of a receptor log-misfit on that
workload ("adjoint"), the 64-scenario ensemble against 64 sequential plain
runs ("ensemble"), and the oracle's rate on all host cores and on one core
("cpu_baseline").

    python bench.py [--steps K] [--warmup W] [--workload c2|c1]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # MI355X HBM3E, bytes/s
# Algorithmic HBM bytes per particle-step: one read and one write of the FP32
# state x, y, z, m (random numbers come from Philox keys, the birth from the
# index, the wind from the cache-resident field).
B_FWD = 32
# A gradient evaluation: the forward's 32 B, plus storing the recomputed
# state of each step (16 B) and reading it back in the reverse sweep (16 B).
B_GRAD = 64
# VALU issue peak with packed FP32 disabled: 256 CUs x 4 SIMDs, one wave64
# instruction per SIMD every 4 cycles at 2.4 GHz.
VALU_WAVE_INSTS_PEAK = 256 * 4 * 2.4e9 / 4
# Lane operations one particle-step of the method needs, counted by hand
# (a model, not a measurement; the measured instruction count is in `valu`).
MODEL_LANE_OPS_PER_PSTEP = 290

WORKLOADS = {
    "c2": "1.6e7-particle 24 h run, release over the first 6 h, 25 hourly 400x400x40 wind "
          "fields interpolated in time, dt=5 s, 17280 steps, CIC concentration 400x400x40x2 "
          "every 60 steps (288 output steps), deposition 400x400x2",
    "c1": "1e6-particle 6 h continuous point release, 200x200x30 steady gridded wind, "
          "dt=5 s, 4320 steps, CIC gridding every 60 steps (72 output steps)",
}


def kernel_source_hash() -> str:
    """SHA-256 over the HIP sources and the public header (sorted by name)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_0912_3223_amd", "csrc")
    files = [os.path.join(csrc, f) for f in sorted(os.listdir(csrc))]
    files.append(os.path.join(ROOT, "include", "lpm.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_values(name):
    """The machine-readable `key: value` lines of a committed profile summary,
    or None when it is missing or the kernel sources changed since it was
    taken (its kernel_source_sha256 no longer matches)."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        k, sep, v = line.strip().partition(": ")
        if sep and k and " " not in k:
            vals[k] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return vals


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["c2", "c1"], default="c2",
                    help="headline workload (c2: the 1.6e7-particle 24 h run)")
    ap.add_argument("--n", type=int, default=0, help="particles (0 = the workload's)")
    ap.add_argument("--no-c1", action="store_true", help="skip the 1e6-particle 6 h line")
    ap.add_argument("--c1-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="target seconds of each oracle leg (all cores, one core)")
    ap.add_argument("--ensemble-steps", type=int, default=3)
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the 64-scenario batched-vs-sequential comparison")
    ap.add_argument("--adjoint-steps", type=int, default=3,
                    help="timed gradient evaluations of the receptor misfit")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the gradient (adjoint) measurement")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="run one plain device-to-device copy of this size before timing "
                         "(reference dispatch for hardware byte counters)")
    return ap.parse_args()


def make_case(name, n):
    import synth
    if name == "c2":
        return synth.c2(n_total=n or 16_000_000)
    return synth.c1(n_total=n or 1_000_000)


def window_of(case):
    """Steps per step launch: the whole run on a steady field.  On hourly
    fields half a field interval (360 steps): every launch steps on the
    time-pair copy of one interval, and each launch takes its particles in
    a fresh wind-node order (they drift apart within an hour)."""
    if case.field.nt > 1:
        per = int(round(case.field.dt_field / case.physics.dt))
        return per // 2 if per % (2 * case.out_every) == 0 else per
    return case.n_steps


def forward(case, steps, warmup, copy_mb=0):
    """Whole forward runs of `case` as DeviceRun.run_recorded runs them:
    release, step launches (one per window) that record the states after the
    output steps, the gridding of those output steps from the records, the
    deposition grid.  Every step launch is timed with HIP events on the
    stream it is launched on."""
    import torch
    import paper_0912_3223_amd as L
    snaps = case.output_steps()
    assert snaps == list(range(case.out_every - 1, case.n_steps, case.out_every))
    window = window_of(case)
    run = L.DeviceRun(case)
    cg, nn = case.conc_grid, case.physics.n_nuc
    out = torch.empty((len(snaps), nn, cg.nz, cg.ny, cg.nx), dtype=torch.float32, device="cuda")
    ev = []

    def one_run(timed):
        run.reset()
        run.run_recorded(case.out_every, window, out, step_events=ev if timed else None)
        run.grid_deposition()

    for _ in range(warmup):
        one_run(False)
    torch.cuda.synchronize()
    if copy_mb:
        n = copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    psteps = run.particle_steps() if warmup else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_run(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    run.check()
    ledger = run.ledger()
    last = run.particle_steps()
    assert psteps is None or last == psteps, "runs are not deterministic in their step count"
    psteps = last
    step_ms = [e0.elapsed_time(e1) for e0, e1 in ev]
    launches = len(step_ms) // steps
    res = {"psteps": psteps, "ms": (t1 - t0) * 1e3 / steps, "value": psteps * steps / (t1 - t0),
           "step_ms_run": sum(step_ms) / steps, "launches": launches,
           "launch_ms": statistics.mean(step_ms), "window": window, "ledger": ledger}
    del out, run
    torch.cuda.empty_cache()
    return res


def roofline(fw, profile):
    """HBM roofline of the step kernel: B_FWD bytes per particle-step times
    the particle-steps of an average launch, over its average duration."""
    achieved = B_FWD * (fw["psteps"] / fw["launches"]) / (fw["launch_ms"] / 1e3)
    vals = profile_values(profile)
    traffic = float(vals["step_kernel_hbm_bytes_per_launch"]) if vals and \
        "step_kernel_hbm_bytes_per_launch" in vals else None
    return {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": achieved / HBM_PEAK, "traffic": traffic, "kernel": "step_kernel",
            "bytes_per_particle_step": B_FWD,
            "particle_steps_per_launch": fw["psteps"] / fw["launches"],
            "avg_launch_ms": fw["launch_ms"], "launches_per_run": fw["launches"],
            "steps_per_launch": fw["window"],
            "step_kernel_share": fw["step_ms_run"] / fw["ms"]}


def valu(fw, profile):
    """VALU figures of the step kernel from a committed counter summary
    (None while the summary is missing or stale): instructions per
    particle-step and the share of the VALU issue peak they occupy at the
    event-timed launch duration."""
    per_launch = fw["psteps"] / fw["launches"]
    model = {"model_lane_ops_per_particle_step": MODEL_LANE_OPS_PER_PSTEP,
             "model_frac": MODEL_LANE_OPS_PER_PSTEP * per_launch / (fw["launch_ms"] / 1e3)
             / (VALU_WAVE_INSTS_PEAK * 64)}
    return dict(model, **counter_valu(profile, per_launch, fw["launch_ms"]))


def counter_valu(profile, per_launch, launch_ms):
    """The counter part of a `valu` object: from the summary's
    machine-readable lines, per launch of `per_launch` particle-steps timed
    at `launch_ms`."""
    vals = profile_values(profile)
    if not vals or "sq_insts_valu_per_launch" not in vals:
        return {"counters": None}
    insts = float(vals["sq_insts_valu_per_launch"])
    out = {"counters": profile, "wave_insts_per_launch": insts,
           "wave_insts_per_particle_step": insts / per_launch,
           "lane_insts_per_particle_step": 64 * insts / per_launch,
           "issue_frac": insts / (launch_ms / 1e3) / VALU_WAVE_INSTS_PEAK}
    if "valu_busy_frac" in vals:
        out["busy_frac_counters"] = float(vals["valu_busy_frac"])
    return out


def cpu_baseline(case, seconds):
    """The oracle (as it stands) on a bounded sample of the same workload --
    every k-th particle id, k chosen so that each leg takes about `seconds` --
    once on all host cores and once on one core."""
    import oracle
    threads = len(os.sched_getaffinity(0))
    # particle-steps per id of the full run, from the workload's own count
    per_id = {"c2": 3800.0, "c1": 540.0}.get(case.name, 1000.0)
    rate_guess = {1: 1.5e6}
    legs = {}
    for nth in (threads, 1):
        guess = rate_guess.get(nth, 1.5e6 * nth)
        want = seconds * guess / per_id
        stride = max(1, int(case.schedule.n_total / max(want, 1.0)))
        sub = case.with_(schedule=case.schedule.subset(stride))
        o = oracle.Oracle(sub)
        t = time.perf_counter()
        r = o.simulate(nthreads=nth)
        dt = time.perf_counter() - t
        legs[nth] = (r["psteps"] / dt, stride, sub.schedule.local_count, r["psteps"], dt)
    v, stride, n, ps, dt = legs[threads]
    v1, stride1, n1, ps1, dt1 = legs[1]
    return {"value": v, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"every {stride}th particle id of the same run ({n} particles, {ps} "
                      f"particle-steps, {dt:.1f} s, FP64, {threads} OpenMP threads)",
            "single_core": {"value": v1, "unit": "particle-steps/s", "cores": 1,
                            "sample": f"every {stride1}th particle id ({n1} particles, {ps1} "
                                      f"particle-steps, {dt1:.1f} s, one thread)"},
            "cpu_model": cpu_model()}


def ensemble_vs_plain(a):
    """64 release scenarios of uneven size on the 6 h 200 x 200 x 30 workload:
    one persistent ensemble launch per run (eager and replayed from a captured
    graph) against 64 sequential plain runs (release + whole-window step each),
    same particle-steps."""
    import torch
    import synth
    import paper_0912_3223_amd as L
    base, sources, counts = synth.c3()
    e = L.EnsembleRun(base, sources, counts)
    e.prepare()
    tune = e.autotune(trial_steps=240, reps=3)
    e.run()
    torch.cuda.synchronize()
    ps = e.particle_steps()
    t0 = time.perf_counter()
    for _ in range(a.ensemble_steps):
        e.run()
    torch.cuda.synchronize()
    batched = (time.perf_counter() - t0) / a.ensemble_steps
    # the same run captured once and replayed
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        e.run()
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.ensemble_steps):
        g.replay()
    torch.cuda.synchronize()
    graph = (time.perf_counter() - t0) / a.ensemble_steps
    assert e.particle_steps() == ps, "graph replay changed the particle-step count"
    runs = []
    for src, n in zip(sources, counts):
        case = base.with_(source=src, schedule=synth.Schedule(n_total=n, s_release=base.n_steps))
        runs.append(L.DeviceRun(case))
    # sequential plain runs with the same queue schedule (plain launches use 256 threads)
    tl = tune.launch
    L.set_launch(tl.refill_every, tl.blocks_per_cu if tl.block == 256 else 0, tl.refill_min)

    def sequential():
        for r in runs:
            r.reset()
            r.release(0, base.n_steps)
            r.step(0, base.n_steps)

    sequential()
    torch.cuda.synchronize()
    ps_plain = sum(r.particle_steps() for r in runs)
    t0 = time.perf_counter()
    for _ in range(a.ensemble_steps):
        sequential()
    torch.cuda.synchronize()
    seq = (time.perf_counter() - t0) / a.ensemble_steps
    L.set_launch()
    return {"workload": "64 scenarios, counts log-uniform in [1e4, 1e6] (seed 3), heights "
                        "U(10,200) m, rates U(0.5,2), wind scale U(0.8,1.2), shared 200x200x30 "
                        "field, 4320 steps",
            "particles": int(sum(counts)), "particle_steps": ps, "plain_particle_steps": ps_plain,
            "batched_ms": batched * 1e3, "graph_ms": graph * 1e3, "sequential_ms": seq * 1e3,
            "batched_particle_steps_per_s": ps / batched,
            "graph_particle_steps_per_s": ps / graph,
            "sequential_particle_steps_per_s": ps_plain / seq,
            "speedup_batched_vs_sequential": seq / batched,
            "speedup_graph_vs_sequential": seq / graph,
            "autotuned": {"refill_every": tl.refill_every, "refill_min": tl.refill_min,
                          "blocks_per_cu": tl.blocks_per_cu, "block": tl.block,
                          "median_trial_ms": tune.best_ms, "worst_trial_ms": tune.worst_ms,
                          "settings_tried": tune.n_tried, "reps": tune.reps}}


ADJ_PROFILE = "c1_adjoint_counters.md"


def adjoint_bench(a):
    """Gradient evaluations per second of the receptor misfit at theta0 on
    the 1e6-particle 6 h workload: forward (release, whole-run step with the
    output-step states recorded every 60 steps, Gaussian-kernel receptor
    gridding) plus the adjoint sweep from those checkpoints."""
    import torch
    import synth
    import paper_0912_3223_amd as L
    rec, obs, _ = synth.load_receptors(os.path.join(ROOT, "tests", "golden", "c4_receptors.json"))
    case = synth.c4()
    run = L.ReceptorRun(case, rec)
    o = torch.as_tensor(obs, device="cuda")
    eps = 1e-6 * float(o.max())
    stream = torch.cuda.current_stream()
    ev = []

    def evaluate(timed):
        c = run.forward(synth.THETA0)
        gbar = 2.0 * (torch.log(c + eps) - torch.log(o + eps)) / (c + eps)
        if timed:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        g = run.backward(gbar)
        if timed:
            e1.record(stream)
            ev.append((e0, e1))
        return c, g

    evaluate(False)
    torch.cuda.synchronize()
    psteps = run.run.particle_steps()
    t0 = time.perf_counter()
    for _ in range(a.adjoint_steps):
        c, g = evaluate(True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.adjoint_steps
    back_ms = sum(e0.elapsed_time(e1) for e0, e1 in ev) / len(ev)
    loss = float(((torch.log(c + eps) - torch.log(o + eps)) ** 2).sum())
    achieved = B_GRAD * psteps / dt
    vals = profile_values(ADJ_PROFILE)
    traffic = float(vals["adjoint_kernel_hbm_bytes_per_launch"]) if vals and \
        "adjoint_kernel_hbm_bytes_per_launch" in vals else None
    return {"workload": "receptor log-misfit gradient in (h, q, s_w, v_d) at theta0 = "
                        "(50 m, 1, 1, 0.002 m/s); 1e6 particles, 4320 steps, 50 ground "
                        "receptors (Gaussian kernel 250 m / 40 m), checkpoints every 60 steps",
            "gradient_evals_per_s": 1.0 / dt, "ms_per_gradient": dt * 1e3,
            "adjoint_kernel_ms": back_ms, "forward_ms": dt * 1e3 - back_ms,
            "particle_steps_forward": psteps,
            "adjoint_particle_steps_per_s": psteps / (back_ms / 1e3),
            "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK,
                         "bytes_per_particle_step": B_GRAD, "traffic": traffic,
                         "what": "one gradient evaluation (forward + adjoint) per B_GRAD x "
                                 "forward particle-steps"},
            "valu": counter_valu(ADJ_PROFILE, psteps, back_ms),
            "loss": loss, "grad": [float(v) for v in g[:4].cpu()]}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (the library has no "
                                   "multi-GPU path); run with --gpus 1"}))
        sys.exit(2)
    import torch  # noqa: F401
    import paper_0912_3223_amd  # noqa: F401  (fails loudly without liblpm.so)

    case = make_case(a.workload, a.n)
    fw = forward(case, a.steps, a.warmup, a.copy_calibration_mb)
    prof = f"{a.workload}_step_kernel_counters.md"
    out = {
        "metric": "particle-steps/s (forward)",
        "value": fw["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": fw["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[a.workload],
                   "particles": case.schedule.n_total, "time_steps": case.n_steps,
                   "output_steps": len(case.output_steps()),
                   "particle_steps_per_run": fw["psteps"]},
        "roofline": roofline(fw, prof),
        "valu": valu(fw, prof),
        "ledger_first_nuclide": list(map(float, fw["ledger"][0])),
    }
    if a.workload == "c2" and not a.no_c1:
        c1 = make_case("c1", 0)
        f1 = forward(c1, a.c1_steps, 1)
        out["c1"] = {"workload": WORKLOADS["c1"], "value": f1["value"], "unit": "particle-steps/s",
                     "ms_per_step": f1["ms"], "particle_steps_per_run": f1["psteps"],
                     "roofline": roofline(f1, "c1_step_kernel_counters.md"),
                     "valu": valu(f1, "c1_step_kernel_counters.md")}
    if not a.no_adjoint:
        out["adjoint"] = adjoint_bench(a)
    if not a.no_ensemble:
        out["ensemble"] = ensemble_vs_plain(a)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

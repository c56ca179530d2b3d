"""Benchmark: forward particle-steps/s of the particle-dispersion hot path on
one MI355X.

Workload (one benchmark step = one full forward run): 1e6 particles released
continuously from (0, 0, 50 m) over 6 h at dt = 5 s (4320 time steps), steady
200 x 200 x 30 wind field (250/250/40 m nodes, power-law profile with four
seeded Fourier modes of direction), parabolic K_z over a 1000 m mixed layer,
dry deposition (v_d = 0.002 m/s), wet scavenging (1e-5 1/s) in a seeded
elliptical rain region, two nuclides (lambda = 1e-6, 1e-5 1/s).  Every step of
a run: release, particle step (advection, turbulent random walk, reflection,
decay, dry/wet deposition with the deposition scatter), concentration gridding
on the 200 x 200 x 30 x 2 cloud-in-cell grid every 60 steps, and the final
deposition grid.  `value` = active particle-steps per second over the timed
runs (inputs resident in HBM).

Also reported on the same line: gradient evaluations per second of a
receptor log-misfit with respect to (source height, release rate, wind
scale, deposition velocity) on the same workload (forward + adjoint), the
64-scenario batched ensemble against 64 sequential plain runs, and the FP64
oracle's rate on the host cores.

    python bench.py [--steps K] [--warmup W] [--spl STEPS_PER_LAUNCH]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU issue peak with packed FP32 disabled: 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz lane-operations per second (the 157.3 TFLOP/s FP32 figure counts a
# packed two-lane FMA as four flops).
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
# Lane-cycles of VALU work one particle-step of the method needs (Philox
# 10 rounds, Box-Muller, trilinear wind, K_z at two heights, move and fold,
# deposition rates, decay of two nuclides, FP64 ledger sums); derived in the
# design notes.  Quarter-rate transcendentals and 32-bit multiplies count 4.
ALG_OPS_PER_PSTEP = 290
HBM_PEAK = 8.0e12


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


def measured_traffic():
    """HBM bytes per step-kernel launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes scaled by a plain copy of known size),
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "c1_1e6_step_kernel_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        k, _, v = line.strip().partition(": ")
        if k in ("step_kernel_hbm_bytes_per_launch", "kernel_source_sha256"):
            vals[k] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return float(vals["step_kernel_hbm_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--spl", type=int, default=0,
                    help="time steps per step-kernel launch; 0 = the whole run in one launch "
                         "with the output-step states recorded and gridded afterwards")
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=8,
                    help="oracle sample: every k-th particle id of the same workload")
    ap.add_argument("--ensemble-steps", type=int, default=2)
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


def cpu_baseline(case, stride):
    import oracle
    sub = case.with_(schedule=case.schedule.subset(stride))
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    o = oracle.Oracle(sub)
    t = time.perf_counter()
    r = o.simulate(nthreads=threads)
    dt = time.perf_counter() - t
    return {"value": r["psteps"] / dt, "unit": "particle-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"every {stride}th particle id of the same 1e6-particle 6 h run "
                      f"({sub.schedule.local_count} particles, {r['psteps']} particle-steps, "
                      f"{dt:.1f} s, FP64, {threads} OpenMP threads)"}


def ensemble_vs_plain(a):
    """64 release scenarios of uneven size on the gridded 6 h workload:
    one persistent ensemble launch per run against 64 sequential plain runs
    (release + whole-window step each), same particle-steps."""
    import torch
    import synth
    import paper_0912_3223_amd as L
    base, sources, counts = synth.c3()
    e = L.EnsembleRun(base, sources, counts)
    e.prepare()
    tune = e.autotune(trial_steps=240)
    e.run()
    torch.cuda.synchronize()
    ps = e.particle_steps()
    t0 = time.perf_counter()
    for _ in range(a.ensemble_steps):
        e.run()
    torch.cuda.synchronize()
    batched = (time.perf_counter() - t0) / a.ensemble_steps
    tuned = (tune.refill_every, tune.blocks_per_cu, tune.refill_min)
    L.set_launch()
    runs = []
    for src, n in zip(sources, counts):
        case = base.with_(source=src, schedule=synth.Schedule(n_total=n, s_release=base.n_steps))
        runs.append(L.DeviceRun(case))
    L.set_launch(*tuned)

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
            "batched_ms": batched * 1e3, "sequential_ms": seq * 1e3,
            "batched_particle_steps_per_s": ps / batched,
            "sequential_particle_steps_per_s": ps_plain / seq,
            "speedup_batched_vs_sequential": seq / batched,
            "autotuned": {"refill_every": tune.refill_every, "refill_min": tune.refill_min,
                          "blocks_per_cu": tune.blocks_per_cu,
                          "best_trial_ms": tune.best_ms, "worst_trial_ms": tune.worst_ms}}


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
    return {"workload": "receptor log-misfit gradient in (h, q, s_w, v_d) at theta0 = "
                        "(50 m, 1, 1, 0.002 m/s); 1e6 particles, 4320 steps, 50 ground "
                        "receptors (Gaussian kernel 250 m / 40 m), checkpoints every 60 steps",
            "gradient_evals_per_s": 1.0 / dt, "ms_per_gradient": dt * 1e3,
            "adjoint_kernel_ms": back_ms, "forward_ms": dt * 1e3 - back_ms,
            "particle_steps_forward": psteps,
            "adjoint_particle_steps_per_s": psteps / (back_ms / 1e3),
            "loss": loss, "grad": [float(v) for v in g[:4].cpu()]}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; use --gpus 1"}))
        sys.exit(2)
    import torch
    import synth
    import paper_0912_3223_amd as L

    case = synth.c1(n_total=a.n)
    snaps = case.output_steps()
    assert snaps == list(range(case.out_every - 1, case.n_steps, case.out_every))
    run = L.DeviceRun(case)
    stream = torch.cuda.current_stream()

    # step-kernel timing: HIP events on the stream the kernels are launched on
    ev = []

    rec = run.record_buffer(len(snaps)) if a.spl == 0 else None
    gbufs = run.grid_buffers(snaps[0], case.out_every, len(snaps)) if a.spl == 0 else None

    def one_run(timed):
        run.reset()
        if a.spl == 0:
            run.release(0, case.n_steps)
            if timed:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            run.step_record(0, case.n_steps, snaps[0], case.out_every, len(snaps), rec)
            if timed:
                e1.record(stream)
                ev.append((e0, e1))
            run.grid_records(rec, snaps[0], case.out_every, len(snaps), gbufs)
            run.grid_deposition()
            return
        for s0, s1 in run.windows(0, case.n_steps, a.spl, snaps):
            run.release(s0, s1 - s0)
            if timed:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                run.step(s0, s1 - s0)
                e1.record(stream)
                ev.append((e0, e1))
            else:
                run.step(s0, s1 - s0)
            if (s1 - 1) in snaps:
                run.grid_concentration(s1 - 1)
        run.grid_deposition()

    for _ in range(a.warmup):
        one_run(False)
    torch.cuda.synchronize()
    if a.copy_calibration_mb:
        n = a.copy_calibration_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    psteps = run.particle_steps()
    run.check()
    ledger = run.ledger()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        one_run(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert run.particle_steps() == psteps, "runs are not deterministic in their step count"

    ms = (t1 - t0) * 1e3 / a.steps
    value = psteps * a.steps / (t1 - t0)
    step_ms = [e0.elapsed_time(e1) for e0, e1 in ev]
    launches_per_run = len(step_ms) // a.steps
    step_total_s = sum(step_ms) / 1e3 / a.steps
    avg_launch_s = sum(step_ms) / 1e3 / len(step_ms)
    ops_per_launch = ALG_OPS_PER_PSTEP * psteps / launches_per_run
    achieved = ops_per_launch / avg_launch_s
    out = {
        "metric": "particle-steps/s (forward)",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1e6-particle 6 h continuous point release, 200x200x30 steady "
                               "gridded wind, dt=5 s, 4320 steps, CIC gridding every 60 steps",
                   "particles": case.schedule.n_total, "time_steps": case.n_steps,
                   "steps_per_launch": a.spl or case.n_steps, "particle_steps_per_run": psteps},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12,
                     "peak": VALU_PEAK_OPS / 1e12, "unit": "TOP/s",
                     "frac": achieved / VALU_PEAK_OPS,
                     "traffic": measured_traffic() if a.spl == 0 and a.n == 1_000_000 else None,
                     "kernel": "step_kernel", "avg_launch_ms": avg_launch_s * 1e3,
                     "launches_per_run": launches_per_run,
                     "step_kernel_share": step_total_s / (ms / 1e3)},
        "ledger_first_nuclide": list(map(float, ledger[0])),
    }
    if not a.no_adjoint:
        out["adjoint"] = adjoint_bench(a)
    if not a.no_ensemble:
        out["ensemble"] = ensemble_vs_plain(a)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case, a.cpu_stride)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

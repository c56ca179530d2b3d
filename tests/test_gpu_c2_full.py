"""The long-run workload at full size, run the way the benchmark runs it:
1.6e7 particles, 24 h at dt = 5 s (17280 steps), 25 hourly 400 x 400 x 40
wind fields interpolated in time, release over the first 6 h; one step
launch with the state after every 60th step recorded, then the record
gridding of all 288 output steps on the 400 x 400 x 40 x 2 grid and the
400 x 400 x 2 deposition grid.

The oracle cannot step 1.6e7 particles in a test's time, so the full run is
tied to it three ways:
* scatter parity at full size: the oracle grids the GPU's own recorded
  states of all 1.6e7 particles at two output steps (relative L2 <= 1e-6);
* invariants of the full run: the ledger closes, the released activity is
  exact, the deposition grid holds no more than the deposited activity;
* the stride-16 subset of particle ids (1e6 particles), in four interleaved
  parts of stride 64, each its own test: the GPU run of the part equals the
  full run's records of those ids bitwise, and the oracle recomputes the
  part from the same Philox counters -- trajectories at 3, 6 and 12 h (mean
  <= 0.05 m, 99.9 % <= 1 m), cloud-in-cell concentration at those output
  steps and the deposition grid (relative L2 <= 1e-4 over cells >= 1e-3 of
  the peak), the ledger (<= 1e-6 of the released activity).
"""
import numpy as np
import pytest

import synth
from parity import distances, ledger_ok, log, rel_l2_masked

pytestmark = pytest.mark.gpu

EVERY = 60
COMPARE = [2159, 4319, 8639]  # output steps at 3 h, 6 h (end of release), 12 h
SUB_STRIDE = 64


@pytest.fixture(scope="module")
def full():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0912_3223_amd as L
    case = synth.c2()
    n_rec = case.n_steps // EVERY
    log("c2 full: %d particles, %d steps, %d output steps" % (case.schedule.n_total, case.n_steps, n_rec))
    run = L.DeviceRun(case)
    rec = run.record_buffer(n_rec)
    work, grids = run.grid_buffers(EVERY - 1, EVERY, n_rec)
    run.release(0, case.n_steps)
    run.step_record(0, case.n_steps, EVERY - 1, EVERY, n_rec, rec)
    run.grid_records(rec, EVERY - 1, EVERY, n_rec, (work, grids))
    dep = run.grid_deposition().double().cpu().numpy()
    run.check()
    out = {"case": case, "run": run, "rec": rec, "grids": grids, "n_rec": n_rec, "dep": dep,
           "ledger": run.ledger(), "psteps": run.particle_steps()}
    del work
    log("c2 full: %d particle-steps" % out["psteps"])
    yield out
    out.clear()
    del run, rec, grids
    torch.cuda.empty_cache()


def _last(rec, n_rec, rec_stride):
    """`last` of the record buffer: per particle, the step after which it
    stopped (INT_MAX: still active at the end)."""
    import torch
    return rec[4 * n_rec * rec_stride: 4 * n_rec * rec_stride + rec_stride].view(torch.int32)


def _record(rec, n_rec, rec_stride, k):
    """(x, y, z, m) of record k and `last`, as float64 / int32 numpy arrays."""
    r = rec[: 4 * n_rec * rec_stride].view(n_rec, rec_stride, 4)[k]
    return r.double().cpu().numpy(), _last(rec, n_rec, rec_stride).cpu().numpy()


def _meaningful(case, rr, last, step):
    """Records that count at output step `step`: born by it and still active
    after it (records at or after `last` carry nothing)."""
    sch = case.schedule
    g = sch.id_base + np.arange(len(last), dtype=np.int64) * sch.id_stride
    b = (g * sch.s_release) // sch.n_total
    return (b <= step) & (step < last) & (rr[:, 3] > 0)


def test_c2_full_run_invariants(full):
    case, led = full["case"], full["ledger"]
    released = case.source.q * case.schedule.s_release * case.physics.dt
    for n in range(2):
        assert led[n][0] == pytest.approx(released, rel=1e-12)
        # nothing is airborne after 24 h (all particles left the 100 km domain)
        gap = led[n][0] - led[n][1] - led[n][2] - led[n][3]
        log("c2 full ledger nuclide %d: released %.6f deposited %.6f decayed %.6f exited %.6f, "
            "airborne %.3e" % (n, *led[n], gap))
        assert abs(gap) <= 1e-6 * released
    area = case.dep_grid.dx * case.dep_grid.dy
    on_grid = full["dep"].sum(axis=(1, 2)) * area
    assert np.all(on_grid <= led[:, 1] * (1 + 1e-5)) and np.all(on_grid >= 0.9 * led[:, 1])
    assert full["psteps"] > 5e10


@pytest.mark.parametrize("step", [2159, 4319])
def test_c2_full_scatter_parity(full, step):
    """The oracle grids the GPU's recorded float32 states of all 1.6e7
    particles: the record gridding at full size (bins of the 400 x 400 grid
    held in LDS, the crowded source tiles) to FP64 summation order."""
    import oracle
    case = full["case"]
    k = (step + 1) // EVERY - 1
    rr, last = _record(full["rec"], full["n_rec"], full["run"].rec_stride, k)
    use = _meaningful(case, rr, last, step)
    m = np.where(use, rr[:, 3], 0.0)
    ref = oracle.Oracle(case).grid_concentration(step, rr[:, 0], rr[:, 1], rr[:, 2], m)
    got = full["grids"][k].double().cpu().numpy()
    rel, ncell = rel_l2_masked(got, ref)
    empty = (ref == 0) & (got != 0)
    log("c2 full scatter step %d: %d records, rel %.3e over %d cells, %d cells nonzero only on GPU"
        % (step, use.sum(), rel, ncell, empty.sum()))
    assert rel <= 1e-6
    assert not empty.any()


@pytest.mark.parametrize("part", [0, 1, 2, 3])
def test_c2_subset_parity(full, part):
    """Ids 16 part + 64 k of the full run (part = 0..3: together the stride-16
    subset): GPU equals the full run bitwise, oracle parity at 3, 6, 12 h and
    at the end."""
    import torch
    import oracle
    import paper_0912_3223_amd as L
    case = full["case"]
    base = 16 * part
    sub = case.with_(schedule=case.schedule.subset(SUB_STRIDE, base))
    n = sub.schedule.local_count
    n_rec = full["n_rec"]
    # GPU run of the part alone, in the benchmark's launch configuration
    run = L.DeviceRun(sub)
    rec = run.record_buffer(n_rec)
    work, grids = run.grid_buffers(EVERY - 1, EVERY, n_rec)
    run.release(0, case.n_steps)
    run.step_record(0, case.n_steps, EVERY - 1, EVERY, n_rec, rec)
    run.grid_records(rec, EVERY - 1, EVERY, n_rec, (work, grids))
    dep = run.grid_deposition().double().cpu().numpy()
    run.check()
    g_led = run.ledger()
    # the part's trajectories are the full run's, bitwise
    full_rec = full["rec"][: 4 * n_rec * full["run"].rec_stride].view(n_rec, -1, 4)
    mine = rec[: 4 * n_rec * n].view(n_rec, n, 4)
    for s in COMPARE:
        k = (s + 1) // EVERY - 1
        a = mine[k].cpu()
        b = full_rec[k, base::SUB_STRIDE][:n].cpu()
        _, last = _record(rec, n_rec, n, k)
        use = torch.from_numpy(_meaningful(sub, a.double().numpy(), last, s))
        assert torch.equal(a[use], b[use]), "part %d step %d differs from the full run" % (part, s)
    full_last = _last(full["rec"], n_rec, full["run"].rec_stride)[base::SUB_STRIDE][:n].cpu()
    assert torch.equal(_last(rec, n_rec, n).cpu(), full_last)
    fr = full["run"]
    st = run.state()
    for key in "xyzm":
        a = getattr(fr, key)[base::SUB_STRIDE][:n].double().cpu().numpy()
        np.testing.assert_array_equal(st[key], a)
    # the oracle, window by window, from the same counters
    o = oracle.Oracle(sub)
    state, s0 = None, 0
    o_dep = 0.0
    o_led = 0.0
    for s in COMPARE + [case.n_steps - 1]:
        snaps = [s] if s in COMPARE else []
        r = o.simulate(s_begin=s0, s_end=s + 1, state=state, snap_steps=snaps)
        state, s0 = r["state"], s + 1
        o_dep = o_dep + r["dep"]
        o_led = o_led + r["ledger"]
        if s not in COMPARE:
            continue
        k = (s + 1) // EVERY - 1
        rr, last = _record(rec, n_rec, n, k)
        g_alive = _meaningful(sub, rr, last, s)
        o_alive = state["m"] > 0
        same = np.mean(g_alive == o_alive)
        both = g_alive & o_alive
        gs = {"x": rr[:, 0], "y": rr[:, 1], "z": rr[:, 2]}
        d = distances(gs, state, both)
        rel, ncell = rel_l2_masked(grids[k].double().cpu().numpy(), r["snaps"][0])
        log("c2 part %d step %d: %d airborne, same status %.5f, P1 mean %.3e p99.9 %.3e max %.3e, "
            "conc rel %.3e over %d cells" % (part, s, both.sum(), same, d.mean(),
                                              np.quantile(d, 0.999), d.max(), rel, ncell))
        assert same >= 0.999
        assert d.mean() <= 0.05 and np.quantile(d, 0.999) <= 1.0
        # masses: a float32 product of up to ~8600 per-step factors, each
        # rounded (<= 2^-24) after a hardware exp2 (~1 ulp): ~1e-5 typical,
        # 2e-4 leaves room for the tail of 250k particles
        np.testing.assert_allclose(rr[both, 3], state["m"][both], rtol=2e-4)
        assert rel <= 1e-4
    reld, ncell = rel_l2_masked(dep, o_dep)
    log("c2 part %d: deposition rel %.3e over %d cells" % (part, reld, ncell))
    assert reld <= 1e-4
    ledger_ok(g_led, o_led, o_led[0][0])
    del run, rec, work, grids
    torch.cuda.empty_cache()

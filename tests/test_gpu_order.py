"""Work orders (lpm_order_particles): the order is a permutation of the
launch's particles grouped as documented -- active particles by wind node,
then those born in the window in index order, then the inactive ones -- and
windows stepped in that order give the records, states and grids of the
same windows in index order, bitwise."""
import numpy as np
import pytest

import synth
from parity import log, records_by_particle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _hourly():
    """4 hourly 400 x 400 x 40 fields, 3 h, 6e4 particles released over the
    first 2 h (windows with active, newborn and exited particles)."""
    return synth.c2(n_total=60_000, n_steps=2160, s_release=1440, n_hours=4)


def test_order_groups_particles_by_wind_node():
    """The 50 km steady-wind domain after 4 h of a 6 h release: particles
    active, left through the side, and still to be born in the window."""
    import torch
    import paper_0912_3223_amd as L
    case = synth.c1(n_total=60_000, n_steps=4320)
    run = L.DeviceRun(case)
    rec = run.record_buffer(24)
    for w0 in (0, 1440):
        run.release(w0, 1440)
        run.step_record(w0, 1440, w0 + 59, 60, 24, rec)
    run.release(2880, 1440)
    st = run.work_order(2880, 1440)
    n = st.n_order
    sch, f = case.schedule, case.field
    assert n == sch.local_count  # every particle is born by the end of this window
    order = run._order[:n].cpu().numpy()
    assert np.array_equal(np.sort(order), np.arange(n))
    state = run.state()
    g = sch.id_base + np.arange(n) * sch.id_stride
    born_before = (g * sch.s_release) // sch.n_total < 2880
    alive = born_before & (state["m"] > 0)
    newborn = ~born_before
    n_alive, n_new = int(alive.sum()), int(newborn.sum())
    assert n_alive > 0 and n_new > 0 and (born_before & ~alive).sum() > 0
    assert alive[order[:n_alive]].all()
    np.testing.assert_array_equal(order[n_alive:n_alive + n_new], np.flatnonzero(newborn))
    assert not alive[order[n_alive + n_new:]].any()
    # node keys (float64 here, fused float32 in the kernel: a particle within
    # 1e-4 of a node boundary may fall on either side)
    x, y, z = (state[k][order[:n_alive]] for k in "xyz")
    fi = (x - f.x0) / f.dx
    fj = (y - f.y0) / f.dy
    fk = z / f.dz
    key = ((np.clip(np.floor(fj), 0, f.ny - 1) * f.nx + np.clip(np.floor(fi), 0, f.nx - 1)) * f.nz
           + np.clip(np.floor(fk), 0, f.nz - 1))
    near = np.minimum.reduce([np.abs(v - np.round(v)) for v in (fi, fj, fk)]) < 1e-4
    down = np.flatnonzero(np.diff(key) < 0)
    assert all(near[d] or near[d + 1] for d in down)
    log("order: %d active in %d nodes, %d born in the window, %d inactive"
        % (n_alive, len(np.unique(key)), n_new, n - n_alive - n_new))
    torch.cuda.synchronize()


@pytest.mark.parametrize("kind", ["hourly", "steady"])
def test_windows_in_work_order_equal_index_order(kind):
    import torch
    import paper_0912_3223_amd as L
    if kind == "hourly":
        case, window = _hourly(), 720
    else:
        case, window = synth.c1(n_total=50_000, n_steps=1440, s_release=720), 480
    out = {}
    for order in (False, True):
        run = L.DeviceRun(case)
        recs = []
        grids = run.run_recorded(
            60, window, order=order,
            on_window=lambda w0, rec, n_rec, o: recs.append(
                records_by_particle(rec, n_rec, run.rec_stride, o)))
        run.check()
        out[order] = dict(state=run.state(), grids=grids.double().cpu().numpy(), recs=recs,
                          dep=run.grid_deposition().double().cpu().numpy(), led=run.ledger())
    a, b = out[False], out[True]
    for key in ("x", "y", "z", "m", "xl", "yl"):
        np.testing.assert_array_equal(a["state"][key], b["state"][key])
    n, sch = case.schedule.local_count, case.schedule
    n_rec = window // 60
    birth = torch.from_numpy((sch.id_base + np.arange(n) * sch.id_stride) * sch.s_release
                             // sch.n_total).cuda()
    # records by particle (the ordered run stores them by queue position)
    for w, ((ra, la), (rb, lb)) in enumerate(zip(a["recs"], b["recs"])):
        la, lb = la[:n], lb[:n]
        w_end = (w + 1) * window
        born = birth < w_end
        assert torch.equal(la[born], lb[born])
        for k in range(n_rec):
            s = window * w + 60 * k + 59
            use = (birth <= s) & (s < la)
            assert torch.equal(ra[k, :n][use], rb[k, :n][use]), (w, k)
    np.testing.assert_allclose(b["grids"], a["grids"], rtol=1e-6, atol=0)
    np.testing.assert_allclose(b["dep"], a["dep"], rtol=1e-6, atol=0)
    np.testing.assert_allclose(b["led"], a["led"], rtol=1e-12, atol=0)
    log("work order %s: %d windows equal" % (kind, len(b["recs"])))


def _order_of(run, step0, n_steps):
    st = run.work_order(step0, n_steps)
    return st.n_order, run._order[:st.n_order].cpu().numpy()


def test_order_degenerate_cases():
    """No particle born before the window (the order is the index order), no
    particle at all, every particle inactive, a one-node field (one bin), and
    nonuniform levels (columns only): always a permutation of the launch's
    particles with the documented grouping."""
    import torch
    import paper_0912_3223_amd as L
    # nothing born before step 0: all particles are born in the window
    case = synth.c1(n_total=5000, n_steps=600, s_release=300)
    run = L.DeviceRun(case)
    run.release(0, 600)
    n, order = _order_of(run, 0, 600)
    assert n == 5000 and np.array_equal(order, np.arange(5000))
    # a one-step window at step 0: the particles born in it (ids g with
    # g * 300 // 5000 == 0, i.e. 0..16)
    assert run.work_order(0, 1).n_order == 17
    # every particle inactive: set them all to m = 0 after their births
    run.set_state(np.zeros(5000), np.zeros(5000), np.full(5000, 50.0), np.zeros(5000))
    n, order = _order_of(run, 300, 300)
    assert n == 5000 and np.array_equal(np.sort(order), np.arange(5000))
    # a one-node field: one bin
    one = synth.c0(n_total=4000, n_steps=200)
    run1 = L.DeviceRun(one)
    run1.release(0, 200)
    run1.step(0, 100)
    n, order = _order_of(run1, 100, 100)
    g = one.schedule.id_base + np.arange(n) * one.schedule.id_stride
    born_before = (g * one.schedule.s_release) // one.schedule.n_total < 100
    n_act = int((born_before & (run1.state()["m"] > 0)).sum())
    assert np.array_equal(np.sort(order), np.arange(n))
    assert np.array_equal(np.sort(order[:n_act]), np.flatnonzero(born_before))
    # nonuniform levels: grouped by column
    lev_case = synth.c1(n_total=20_000, n_steps=600, s_release=300)
    f = lev_case.field
    lev = (1200.0 * (np.linspace(0.0, 1.0, f.nz) ** 1.5) + 5.0).astype(np.float32)
    lev_case = lev_case.with_(field=synth.replace(f, z_levels=lev))
    runl = L.DeviceRun(lev_case)
    runl.release(0, 600)
    runl.step(0, 300)
    n, order = _order_of(runl, 300, 300)
    st = runl.state()
    gl = np.arange(n)
    act = ((gl * 300) // 20_000 < 300) & (st["m"] > 0)
    n_act = int(act.sum())
    assert np.array_equal(np.sort(order), np.arange(n)) and act[order[:n_act]].all()
    col = (np.clip(np.floor((st["y"] - f.y0) / f.dy), 0, f.ny - 1) * f.nx
           + np.clip(np.floor((st["x"] - f.x0) / f.dx), 0, f.nx - 1))[order[:n_act]]
    fx = ((st["x"] - f.x0) / f.dx)[order[:n_act]]
    fy = ((st["y"] - f.y0) / f.dy)[order[:n_act]]
    near = np.minimum(np.abs(fx - np.round(fx)), np.abs(fy - np.round(fy))) < 1e-4
    down = np.flatnonzero(np.diff(col) < 0)
    assert all(near[d] or near[d + 1] for d in down)
    torch.cuda.synchronize()

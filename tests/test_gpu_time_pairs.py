"""Time-pair copies of wind intervals (lpm_field_interval): the copy holds
the field's two times of each node side by side, levels innermost, and
windows that step on the copies give the records, states and
grids of the same windows on the field itself, bitwise, for two- and
three-component winds."""
from dataclasses import replace

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


def _case(ncomp: int):
    """4 hourly 400 x 400 x 40 fields, 3 h, 3e4 particles released over the
    first hour; ncomp 3 adds a vertical wind of 1 % of u."""
    case = synth.c2(n_total=30_000, n_steps=2160, s_release=720, n_hours=4)
    if ncomp == 3:
        d = case.field.data
        w = (0.01 * d[..., :1]).astype(np.float32)
        case = case.with_(field=replace(case.field, data=np.ascontiguousarray(
            np.concatenate([d, w], axis=4))))
    return case


@pytest.mark.parametrize("ncomp", [2, 3])
def test_interval_copy_layout(ncomp):
    import torch
    import paper_0912_3223_amd as L
    case = _case(ncomp)
    run = L.DeviceRun(case)
    f = case.field
    nodes = f.nz * f.ny * f.nx
    for k in (0, 2):
        packed = run.interval_field(k)
        assert packed.layout == L.FIELD_TIME_PAIRS and packed.interval == k
        assert packed.nt == f.nt and packed.t0 == f.t0
        got = run._interval_buf.cpu().numpy().reshape(nodes, 2, -1)
        rec = got.shape[2]
        assert rec == (2 if ncomp == 2 else 4)
        # nodes [ny][nx][nz]: levels innermost
        a = f.data[k].transpose(1, 2, 0, 3).reshape(nodes, ncomp)
        b = f.data[k + 1].transpose(1, 2, 0, 3).reshape(nodes, ncomp)
        np.testing.assert_array_equal(got[:, 0, :ncomp], a)
        np.testing.assert_array_equal(got[:, 1, :ncomp], b)
        if rec > ncomp:
            assert not got[:, :, ncomp:].any()
    torch.cuda.synchronize()


@pytest.mark.parametrize("ncomp", [2, 3])
def test_windows_on_time_pairs_equal_the_field(ncomp):
    import torch
    import paper_0912_3223_amd as L
    case = _case(ncomp)
    out = {}
    for tp in (False, True):
        run = L.DeviceRun(case)
        recs = []
        grids = run.run_recorded(
            60, 720, time_pairs=tp,
            on_window=lambda w0, rec, n_rec, o: recs.append(
                records_by_particle(rec, n_rec, run.rec_stride, o)))
        run.check()
        out[tp] = dict(state=run.state(), grids=grids.double().cpu().numpy(), recs=recs,
                       dep=run.grid_deposition().double().cpu().numpy(), led=run.ledger(),
                       used=getattr(run, "_interval_k", None))
    a, b = out[False], out[True]
    assert a["used"] is None and b["used"] == 2  # the last window's interval
    for key in ("x", "y", "z", "m", "xl", "yl"):
        np.testing.assert_array_equal(a["state"][key], b["state"][key])
    # records: the meaningful ones (born by the output step, still active
    # after it) and every particle's `last`
    n, sch = case.schedule.local_count, case.schedule
    birth = torch.from_numpy((sch.id_base + np.arange(n) * sch.id_stride) * sch.s_release
                             // sch.n_total).cuda()
    for w, ((ra, la), (rb, lb)) in enumerate(zip(a["recs"], b["recs"])):
        la, lb = la[:n], lb[:n]
        born = birth < 720 * (w + 1)  # particles of the window's launch
        assert torch.equal(la[born], lb[born])
        for k in range(12):
            s = 720 * w + 60 * k + 59
            use = (birth <= s) & (s < la)
            assert torch.equal(ra[k, :n][use], rb[k, :n][use]), (w, k)
    # grids and deposition: the same float32 contributions, FP64 sums in
    # the order the atomics arrive
    np.testing.assert_allclose(b["grids"], a["grids"], rtol=1e-6, atol=0)
    np.testing.assert_allclose(b["dep"], a["dep"], rtol=1e-6, atol=0)
    np.testing.assert_allclose(b["led"], a["led"], rtol=1e-12, atol=0)
    log("time pairs ncomp %d: %d airborne at the end, records of %d windows equal"
        % (ncomp, int((b["state"]["m"] > 0).sum()), len(b["recs"])))


def test_steps_outside_the_interval_are_rejected():
    import paper_0912_3223_amd as L
    case = _case(2)
    run = L.DeviceRun(case)
    packed = run.interval_field(1)
    rec = run.record_buffer(1)
    run.release(0, 720)
    with pytest.raises(L.LpmError) as e:
        run.step_record(660, 60, 719, 60, 1, rec, packed)  # steps of interval 0
    assert e.value.code == L.LPM_EINVAL
    run.step_record(0, 720, 719, 720, 1, rec)  # the field itself takes them
    run.step_record(720, 60, 779, 60, 1, rec, packed)
    run.check()


@pytest.mark.parametrize("shape", [(1, 8, 1), (5, 1, 3), (1, 1, 1)])
def test_time_pairs_on_degenerate_grids(shape):
    """Fields one node wide in some directions (the stencil's neighbour in
    that direction is the node itself): time-pair copies still give the
    field's states bitwise."""
    import paper_0912_3223_amd as L
    nx, ny, nz = shape
    base = synth.c2(n_total=3000, n_steps=720, s_release=360, n_hours=2)
    fld = synth.wind_field([1000, 1001], nx, ny, nz, 250.0, 250.0, 40.0, bounded=False)
    case = base.with_(field=fld)
    states = []
    for tp in (False, True):
        run = L.DeviceRun(case)
        run.run_recorded(60, 360, time_pairs=tp)
        run.check()
        states.append(run.state())
    for key in ("x", "y", "z", "m", "xl", "yl"):
        np.testing.assert_array_equal(states[0][key], states[1][key])

"""Gridding of recorded states (lpm_grid_records) against the FP64 oracle.

The oracle grids the GPU's own recorded float32 positions and masses, so the
comparison isolates the gridding: binning of records by column tile, the
per-tile FP64 sums and the conversion.  Grids and nuclide sets are chosen
to reach every path: bins per output step held in LDS (below and above
64 KB) and not, tiles of
16 x 4, 8 x 4 and 8 x 2 columns, grids that the tiles do not divide or that
are narrower than one tile, one to four nuclides (a decay chain among
them), cloud-in-cell and nearest-cell.  Tolerances as in the other parity tests: cloud-in-cell
relative L2 <= 1e-6 (float32 contributions summed in FP64), nearest-cell
differences only from particles within 1e-3 m of a cell face.
"""
import numpy as np
import pytest

import synth
from parity import log, ngp_unexplained, rel_l2_masked

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0912_3223_amd  # noqa: F401  (fails loudly if liblpm.so is missing)


def _grid(base, **kw):
    return synth.replace(base, **kw)


# (label, grid changes): the c1 grid is 200 x 200 x 30 of 250 x 250 x 40 m
GRIDS = [
    ("c1 grid, 16x4 tiles, 1352 bins in one LDS window", {}),
    ("300x300x10 fine, 5776 bins over several LDS windows, ragged tiles",
     dict(nx=300, ny=300, nz=10, dx=100.0, dy=100.0, dz=100.0, x0=-5000.0, y0=-15000.0)),
    ("720x720x4 finer, 33304 bins: blocks spread beyond their LDS window (global atomics)",
     dict(nx=720, ny=720, nz=4, dx=40.0, dy=40.0, dz=250.0, x0=-14400.0, y0=-14400.0)),
    ("90x90x120 tall, 8x2 tiles, ragged", dict(nx=90, ny=90, nz=120, dx=300.0, dy=300.0,
                                               dz=10.0, x0=-3000.0, y0=-13500.0)),
    ("c1 grid, nearest cell", dict(mode=0)),
    ("37x23x7 small, every tile ragged", dict(nx=37, ny=23, nz=7, dx=700.0, dy=900.0,
                                             dz=150.0, x0=-4000.0, y0=-10000.0)),
    ("5x3x1 flat, narrower than one tile", dict(nx=5, ny=3, nz=1, dx=3000.0, dy=4000.0,
                                               dz=2000.0, x0=-2000.0, y0=-6000.0)),
]

# nuclide sets (the tile pass is compiled per nuclide count); the last is a
# parent -> daughter chain (Bateman activities)
NUCLIDES = [dict(lambdas=(3e-5,)), dict(lambdas=(1e-6, 1e-5, 1e-4)),
            dict(lambdas=(1e-3, 2.5e-4, 4e-3, 7e-4), chain=1)]


def _records(case, every, n_rec):
    import torch
    import paper_0912_3223_amd as L
    run = L.DeviceRun(case)
    run.reset()
    s0 = every - 1
    run.release(0, case.n_steps)
    rec = run.record_buffer(n_rec)
    run.step_record(0, case.n_steps, s0, every, n_rec, rec)
    work, out = run.grid_buffers(s0, every, n_rec)
    out.fill_(float("nan"))  # every cell must be written
    run.grid_records(rec, s0, every, n_rec, (work, out))
    torch.cuda.synchronize()
    return run, rec.cpu().numpy(), out.double().cpu().numpy()


def _check_against_oracle(c, label):
    import oracle
    every, n_rec = 60, 6
    run, recs, out = _records(c, every, n_rec)
    assert not np.isnan(out).any()
    n, stride = c.schedule.local_count, run.rec_stride
    last = recs[4 * n_rec * stride:4 * n_rec * stride + n].view(np.int32)
    ids = np.arange(n, dtype=np.int64)
    born = (ids * c.schedule.s_release) // c.schedule.n_total
    o = oracle.Oracle(c)
    for k in range(n_rec):
        s = every - 1 + k * every
        live = (born <= s) & (s < last)
        # records that are not meaningful may hold any bits (NaN included)
        r = np.where(live[:, None], recs[4 * k * stride:4 * k * stride + 4 * n].reshape(n, 4),
                     np.float32(0)).astype(np.float64)
        m = np.where(live, r[:, 3], 0.0)
        x, y, z = (np.where(live, r[:, j], 0.0) for j in range(3))
        ref = o.grid_concentration(s, x, y, z, m)
        got = out[k]
        if c.conc_grid.mode == 1:
            rel, ncell = rel_l2_masked(got, ref)
            log(label, "step", s, "rel_l2 %.3e over %d cells" % (rel, ncell))
            assert rel <= 1e-6
            # cells the oracle leaves empty stay empty (up to a particle on a
            # cell centre, whose zero weight may round the other way)
            assert np.abs(got[ref == 0.0]).max(initial=0.0) <= 1e-9 * np.abs(ref).max()
        else:
            age = (s + 1 - born) * c.physics.dt
            a0 = c.source.q * c.schedule.s_release * c.physics.dt / c.schedule.n_total
            act = [np.where(live & (m > 0), a0 * m * np.exp(-lam * age), 0.0)
                   for lam in c.physics.lambdas]
            unexplained, nnear = ngp_unexplained(got, ref, (x, y, z), act, c.conc_grid, 1e-3)
            log(label, "step", s, "NGP unexplained %.3e near-face %d" % (unexplained, nnear))
            assert unexplained == 0.0


@pytest.mark.parametrize("label,kw", GRIDS, ids=[g[0].split(",")[0] + "-" + str(i)
                                                 for i, g in enumerate(GRIDS)])
def test_records_gridded_like_oracle(label, kw):
    c = synth.c1(n_total=40_000, n_steps=360, s_release=360)
    _check_against_oracle(c.with_(conc_grid=_grid(c.conc_grid, **kw)), label)


@pytest.mark.parametrize("kw", NUCLIDES, ids=["1", "3", "4-chain"])
def test_records_gridded_like_oracle_nuclides(kw):
    c = synth.c1(n_total=40_000, n_steps=360, s_release=360)
    _check_against_oracle(c.with_(physics=synth.replace(c.physics, **kw)),
                          "nuclides %d" % len(kw["lambdas"]))


def test_records_grid_twice_same_buffers():
    """A second call on the same workspace gives the same grids (the counts
    are cleared by the call itself)."""
    import torch
    c = synth.c1(n_total=20_000, n_steps=240, s_release=240)
    run, recs, out1 = _records(c, 60, 4)
    import paper_0912_3223_amd as L  # noqa: F401
    rec = torch.from_numpy(recs).cuda()
    work, out = run.grid_buffers(59, 60, 4)
    run.grid_records(rec, 59, 60, 4, (work, out))
    run.grid_records(rec, 59, 60, 4, (work, out))
    torch.cuda.synchronize()
    # FP64 sums in another order may round to the neighbouring float
    np.testing.assert_allclose(out.double().cpu().numpy(), out1, rtol=2e-7, atol=0.0)


def test_records_of_particles_all_gone_grid_to_zero():
    """Degenerate: every particle leaves the (1 m wide, bounded) field in its
    first step, so no record counts; every cell of every output step must
    still be written, with zero."""
    c = synth.c0(n_total=5_000, n_steps=180)
    c = c.with_(field=synth.uniform_field(5.0, 0.0, bounded=True))
    run, recs, out = _records(c, 60, 3)
    assert not np.isnan(out).any()
    assert np.all(out == 0.0)
    led = run.ledger()[0]
    # nothing stays airborne: what did not decay in the first step left
    released, deposited, decayed, exited = led
    assert deposited == 0.0 and exited > 0.999 * released
    np.testing.assert_allclose(decayed + exited, released, rtol=1e-6)  # float per-particle terms

"""More parity cases of liblpm against the oracle: time-varying 400 x 400 x 40
fields, the field/physics variants (three wind components, nonuniform levels,
Eq. 3 exponent, 1-4 nuclides, nearest-cell deposition), and edge cases
(empty, single and ragged particle counts, non-finite input, determinism,
resume).  The full-size workloads are in test_gpu_c1_full.py and
test_gpu_c2_full.py."""
import numpy as np
import pytest

import synth
from parity import distances, ledger_ok, log, rel_l2_masked, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0912_3223_amd  # noqa: F401


def test_time_varying_fields():
    """Hourly 400 x 400 x 40 fields interpolated in time; release over the
    first hour, 2 h run."""
    c = synth.c2(n_total=40_000, n_steps=1440, s_release=720, n_hours=3)
    snaps = [719, 1439]
    g = run_gpu(c, snaps=snaps)
    o = run_oracle(c, snaps=snaps)
    act = (o["state"]["m"] > 0) | (g["state"]["m"] > 0)
    d = distances(g["state"], o["state"], act)
    log("c2-shaped P1 mean %.3e p99.9 %.3e max %.3e" % (d.mean(), np.quantile(d, 0.999), d.max()))
    assert d.mean() <= 0.05 and np.quantile(d, 0.999) <= 1.0
    for s in snaps:
        rel, ncell = rel_l2_masked(g["snaps"][s], o["snap_map"][s])
        log("c2-shaped CIC step", s, "rel_l2 %.3e over %d cells" % (rel, ncell))
        assert rel <= 1e-4
    rel, _ = rel_l2_masked(g["dep"], o["dep"])
    assert rel <= 1e-4
    ledger_ok(g["ledger"], o["ledger"], o["ledger"][0][0])


def variant(kind):
    c = synth.c1(n_total=20_000, n_steps=600, s_release=600)
    if kind == "w_component":
        d = c.field.data
        w = (0.05 * np.sin(np.linspace(0, 6, d.shape[3]))[None, None, None, :, None]
             * np.ones_like(d[..., :1])).astype(np.float32)
        fld = synth.replace(c.field, data=np.concatenate([d, w], axis=-1))
        return c.with_(field=fld)
    if kind == "levels":
        nz = c.field.nz
        lev = (1200.0 * (np.linspace(0.0, 1.0, nz) ** 1.5) + 5.0).astype(np.float32)
        return c.with_(field=synth.replace(c.field, z_levels=lev))
    if kind == "kz_eq3":
        return c.with_(physics=synth.replace(c.physics, kz_kind=2))
    if kind == "kz_const":
        return c.with_(physics=synth.replace(c.physics, kz_kind=0, Kz_const=5.0))
    if kind == "one_nuclide":
        return c.with_(physics=synth.replace(c.physics, lambdas=(3e-5,)))
    if kind == "three_nuclides":
        return c.with_(physics=synth.replace(c.physics, lambdas=(1e-6, 1e-5, 1e-4)))
    if kind == "four_nuclides":
        return c.with_(physics=synth.replace(c.physics, lambdas=(0.0, 1e-6, 1e-5, 1e-4)))
    if kind == "ngp_deposition":
        return c.with_(dep_grid=synth.replace(c.dep_grid, mode=0))
    if kind == "no_lid_wind_scale":
        return c.with_(physics=synth.replace(c.physics, H_lid=0.0, kz_kind=0, Kz_const=8.0),
                       source=synth.replace(c.source, wind_scale=1.15, h=120.0, scenario=9))
    raise KeyError(kind)


@pytest.mark.parametrize("kind", ["w_component", "levels", "kz_eq3", "kz_const", "one_nuclide",
                                  "three_nuclides", "four_nuclides", "ngp_deposition",
                                  "no_lid_wind_scale"])
def test_variant_parity(kind):
    c = variant(kind)
    s = c.n_steps - 1
    g = run_gpu(c, steps_per_launch=45, snaps=[s])
    o = run_oracle(c, snaps=[s])
    act = (o["state"]["m"] > 0) | (g["state"]["m"] > 0)
    d = distances(g["state"], o["state"], act)
    rel, ncell = rel_l2_masked(g["snaps"][s], o["snap_map"][s])
    reld, _ = rel_l2_masked(g["dep"], o["dep"])
    log("variant %s: P1 mean %.3e max %.3e, conc rel %.3e, dep rel %.3e"
        % (kind, d.mean(), d.max(), rel, reld))
    assert d.mean() <= 0.05 and np.quantile(d, 0.999) <= 1.0
    assert rel <= 1e-4
    if c.dep_grid.mode == 1:
        assert reld <= 1e-4
    else:
        assert reld <= 1e-2  # nearest cell: a few face crossings
    ledger_ok(g["ledger"], o["ledger"], o["ledger"][0][0])


@pytest.mark.parametrize("n", [1, 2, 255, 257, 1000])
def test_small_and_ragged_counts(n):
    c = synth.c0(n_total=n, n_steps=90)
    g = run_gpu(c, steps_per_launch=30, snaps=[89])
    o = run_oracle(c, snaps=[89])
    d = distances(g["state"], o["state"], o["state"]["m"] > 0)
    assert d.max() <= 0.05
    rel, _ = rel_l2_masked(g["snaps"][89], o["snap_map"][89])
    assert rel <= 1e-4
    ledger_ok(g["ledger"], o["ledger"], o["ledger"][0][0])


def test_empty_run():
    c = synth.c0(n_total=100, n_steps=10)
    c = c.with_(schedule=synth.replace(c.schedule, n_local=0))
    g = run_gpu(c, snaps=[9])
    assert np.all(g["snaps"][9] == 0.0) and np.all(g["dep"] == 0.0)
    assert np.all(g["ledger"] == 0.0)


def test_non_finite_particle_is_reported_and_isolated():
    import paper_0912_3223_amd as L
    c = synth.c1(n_total=5000, n_steps=120, s_release=1)
    x, y, z, m = synth.uniform_state(5000, ((-5e3, 5e3), (-5e3, 5e3), (0, 900)), 4)
    clean = L.DeviceRun(c)
    clean.set_state(x, y, z, m)
    clean.step(1, 119)
    clean.check()
    xb = x.copy()
    xb[1234] = np.nan
    bad = L.DeviceRun(c)
    bad.set_state(xb, y, z, m)
    bad.step(1, 119)
    with pytest.raises(L.LpmError) as e:
        bad.check()
    assert e.value.code == L.LPM_ENONFINITE
    a, b = clean.state(), bad.state()
    keep = np.arange(5000) != 1234
    for k in "xyzm":
        np.testing.assert_array_equal(a[k][keep], b[k][keep])


def test_repeat_runs_are_identical():
    c = synth.c1(n_total=30_000, n_steps=300)
    a = run_gpu(c, snaps=[299])
    b = run_gpu(c, snaps=[299])
    for k in "xyzm":
        np.testing.assert_array_equal(a["state"][k], b["state"][k])
    np.testing.assert_allclose(a["snaps"][299], b["snaps"][299], rtol=1e-12, atol=0)
    np.testing.assert_allclose(a["dep"], b["dep"], rtol=1e-12, atol=0)


def test_resume_on_gpu_is_bitwise():
    c = synth.c1(n_total=20_000, n_steps=300)
    full = run_gpu(c)
    first = run_gpu(c, s_end=137)
    rest = run_gpu(c, state=first["state"], s_begin=137)
    for k in "xyzm":
        np.testing.assert_array_equal(rest["state"][k], full["state"][k])

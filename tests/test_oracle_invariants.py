"""Special cases with closed forms, conservation and well-mixedness of the
oracle (Sec. 2: advection, turbulent diffusion, decay, dry and wet
deposition; Sec. 3.2: inactivation at the boundary)."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import synth
from synth import Field, Grid, Rain
from plume import births


def base(n=2000, steps=120, **phys):
    c = synth.c0(n_total=n, n_steps=steps)
    return c.with_(physics=synth.replace(c.physics, **phys)) if phys else c


def a0_of(case):
    return case.source.q * case.schedule.s_release * case.physics.dt / case.schedule.n_total


def test_pure_advection_without_turbulence():
    case = base(Kh=0.0, Kz_const=0.0)
    r = oracle.Oracle(case).simulate()
    b = births(case.schedule.n_total, case.schedule.s_release)
    age = (case.n_steps - b) * case.physics.dt
    np.testing.assert_allclose(r["state"]["x"], 5.0 * age, rtol=1e-13)
    assert np.all(r["state"]["y"] == 0.0) and np.all(r["state"]["z"] == 50.0)


def test_wind_scale_multiplies_advection():
    case = base(Kh=0.0, Kz_const=0.0)
    case = case.with_(source=synth.replace(case.source, wind_scale=1.1))
    r = oracle.Oracle(case).simulate()
    b = births(case.schedule.n_total, case.schedule.s_release)
    np.testing.assert_allclose(r["state"]["x"], 5.5 * (case.n_steps - b) * 10.0, rtol=1e-13)


@pytest.mark.parametrize("axis", ["z", "xy"])
def test_random_walk_uses_the_particle_stream(axis):
    """With no wind and no boundary, the displacement is sqrt(2 K dt) times
    the sum of the particle's own normals over its steps (Eq. 2)."""
    n, steps = 300, 40
    kw = dict(Kh=0.0, Kz_const=10.0, H_lid=0.0) if axis == "z" else dict(Kh=50.0, Kz_const=0.0, H_lid=0.0)
    case = base(n=n, steps=steps, **kw)
    case = case.with_(field=synth.uniform_field(0.0, 0.0),
                      source=synth.replace(case.source, h=1e6))
    r = oracle.Oracle(case).simulate()
    b = births(n, steps)
    sums = np.zeros((n, 4))
    for s in range(steps):
        xi = oracle.normals_batch(0, 0, 0, n, s)
        sums += np.where((b <= s)[:, None], xi, 0.0)
    st = r["state"]
    if axis == "z":
        np.testing.assert_allclose(st["z"] - 1e6, math.sqrt(2 * 10.0 * 10.0) * sums[:, 2], atol=1e-8)
        assert np.all(st["x"] == 0.0)
    else:
        np.testing.assert_allclose(st["x"], math.sqrt(2 * 50.0 * 10.0) * sums[:, 0], atol=1e-9)
        np.testing.assert_allclose(st["y"], math.sqrt(2 * 50.0 * 10.0) * sums[:, 1], atol=1e-9)
        assert np.all(st["z"] == 1e6)


def test_ground_reflection_gives_folded_normal():
    n, steps = 100_000, 30
    case = base(n=n, steps=steps, Kh=0.0, Kz_const=10.0, H_lid=0.0)
    case = case.with_(field=synth.uniform_field(0.0, 0.0),
                      source=synth.replace(case.source, h=0.0),
                      schedule=synth.replace(case.schedule, s_release=1))
    z = oracle.Oracle(case).simulate()["state"]["z"]
    sigma = math.sqrt(2 * 10.0 * steps * 10.0)
    assert z.min() >= 0.0
    assert stats.kstest(z / sigma, "halfnorm").pvalue > 1e-4
    assert abs(z.mean() - sigma * math.sqrt(2 / math.pi)) < 5 * sigma / math.sqrt(n)


def test_lid_and_ground_mix_to_uniform():
    n, steps = 50_000, 200
    case = base(n=n, steps=steps, Kh=0.0, Kz_const=10.0, H_lid=100.0, H_mix=100.0)
    case = case.with_(field=synth.uniform_field(0.0, 0.0),
                      source=synth.replace(case.source, h=30.0),
                      schedule=synth.replace(case.schedule, s_release=1))
    z = oracle.Oracle(case).simulate()["state"]["z"]
    assert z.min() >= 0.0 and z.max() <= 100.0
    hist = np.histogram(z, bins=10, range=(0, 100))[0]
    assert stats.chisquare(hist).pvalue > 1e-3


def rain_case(lambdas=(1e-6, 1e-5), L0=1e-4):
    n, steps = 500, 100
    c = base(n=n, steps=steps, Kh=0.0, Kz_const=0.0, lambdas=lambdas, Lambda0=L0,
             rain=Rain(cx=0.0, cy=0.0, a=500.0, b=300.0, angle=0.3, edge=0.1))
    g2 = Grid(5, 5, 1, -250.0, -250.0, 0.0, 100.0, 100.0, 1.0, mode=0)
    return c.with_(field=synth.uniform_field(0.0, 0.0), dep_grid=g2)


def test_wet_deposition_of_a_resting_particle():
    case = rain_case()
    o = oracle.Oracle(case)
    r = o.simulate()
    n, S, dt, L0 = case.schedule.n_total, case.n_steps, case.physics.dt, 1e-4
    a0 = a0_of(case)
    tau = (S - births(n, S)) * dt
    np.testing.assert_allclose(r["state"]["m"], np.exp(-L0 * tau), rtol=1e-12)
    for k, lam in enumerate(case.physics.lambdas):
        tot = -np.expm1(-(lam + L0) * tau)
        want_dep = (a0 * L0 / (lam + L0) * tot).sum()
        want_dec = (a0 * lam / (lam + L0) * tot).sum()
        rel, dep, dec, ex = r["ledger"][k]
        assert dep == pytest.approx(want_dep, rel=1e-11)
        assert dec == pytest.approx(want_dec, rel=1e-11)
        assert ex == 0.0
        # all of it lands in the source cell of the deposition grid
        assert r["dep"][k, 2, 2] == pytest.approx(dep, rel=1e-12)
        assert r["dep"][k].sum() == pytest.approx(dep, rel=1e-12)
        air = o.airborne(S - 1, r["state"]["m"])[k]
        assert rel == pytest.approx(air + dep + dec + ex, rel=1e-13)


def test_dry_deposition_of_a_resting_particle():
    case = base(n=400, steps=100, Kh=0.0, Kz_const=0.0, h_s=40.0)
    case = case.with_(field=synth.uniform_field(0.0, 0.0),
                      source=synth.replace(case.source, h=10.0, v_d=0.01))
    r = oracle.Oracle(case).simulate()
    k = 0.01 * (2 / 40.0) * (1 - 10.0 / 40.0)
    tau = (case.n_steps - births(400, 100)) * 10.0
    np.testing.assert_allclose(r["state"]["m"], np.exp(-k * tau), rtol=1e-12)
    # above the dry-deposition layer nothing deposits
    case2 = case.with_(source=synth.replace(case.source, h=45.0))
    assert np.all(oracle.Oracle(case2).simulate()["state"]["m"] == 1.0)


def test_rain_edge_rate_is_half_on_the_ellipse():
    case = rain_case(lambdas=(0.0,))
    ca, sa = math.cos(0.3), math.sin(0.3)
    case = case.with_(source=synth.replace(case.source, xs=500.0 * ca, ys=500.0 * sa))
    r = oracle.Oracle(case).simulate()
    tau = (case.n_steps - births(500, 100)) * 10.0
    np.testing.assert_allclose(r["state"]["m"], np.exp(-0.5e-4 * tau), rtol=1e-9)


def test_exit_at_the_domain_boundary():
    n, steps = 300, 60
    data = np.zeros((1, 1, 2, 2, 2), dtype=np.float32)
    data[..., 0] = 10.0
    fld = Field(data, x0=0.0, y0=-1000.0, dx=1000.0, dy=1000.0, dz=1000.0, bounded=True)
    case = base(n=n, steps=steps, Kh=0.0, Kz_const=0.0, lambdas=(1e-4,))
    case = case.with_(field=fld, source=synth.replace(case.source, xs=100.0))
    o = oracle.Oracle(case)
    r = o.simulate()
    b = births(n, steps)
    # x after k moves is 100 + 100 k: leaves [0, 2000) on the 19th move
    k_exit = 19
    exited = (steps - b) >= k_exit
    assert np.all(r["state"]["m"][exited] == 0.0) and np.all(r["state"]["m"][~exited] == 1.0)
    a0 = a0_of(case)
    want = a0 * np.exp(-1e-4 * k_exit * 10.0) * exited.sum()
    rel, dep, dec, ex = r["ledger"][0]
    assert ex == pytest.approx(want, rel=1e-12)
    air = o.airborne(steps - 1, r["state"]["m"])[0]
    assert rel == pytest.approx(air + dep + dec + ex, rel=1e-13)
    # exited particles are not moved again
    np.testing.assert_allclose(r["state"]["x"][exited], 100.0 + 100.0 * k_exit, rtol=1e-14)


@pytest.mark.parametrize("kind", [1, 2])
def test_well_mixed_stays_well_mixed(kind):
    """A tracer uniform over the mixed layer stays uniform under a
    height-dependent K_z (needs the drift term; Eq. 3 profile)."""
    n, steps = 100_000, 720
    c = synth.c1(n_total=n, n_steps=steps + 1)
    ph = synth.replace(c.physics, Kh=0.0, kz_kind=kind, Lambda0=0.0)
    case = c.with_(physics=ph, field=synth.uniform_field(0.0, 0.0),
                   source=synth.replace(c.source, v_d=0.0),
                   schedule=synth.replace(c.schedule, s_release=1))
    x, y, z, m = synth.uniform_state(n, ((0, 1), (0, 1), (0, 1000.0)), seed=3)
    st = {"x": x, "y": y, "z": z, "m": m}
    r = oracle.Oracle(case).simulate(s_begin=1, s_end=steps + 1, state=st)
    zf = r["state"]["z"]
    assert zf.min() >= 0.0 and zf.max() <= 1000.0
    hist = np.histogram(zf, bins=20, range=(0, 1000.0))[0]
    assert stats.chisquare(hist).pvalue > 1e-3, hist


def reduced_c1(n=3000, steps=300):
    return synth.c1(n_total=n, n_steps=steps)


def test_subset_run_is_bitwise_the_full_run():
    case = reduced_c1()
    full = oracle.Oracle(case).simulate()["state"]
    for base_id, stride in [(0, 7), (5, 13)]:
        sub = case.with_(schedule=case.schedule.subset(stride, base_id))
        st = oracle.Oracle(sub).simulate()["state"]
        for k in "xyzm":
            np.testing.assert_array_equal(st[k], full[k][base_id::stride])


def test_resume_is_bitwise():
    case = reduced_c1()
    o = oracle.Oracle(case)
    full = o.simulate()
    half = o.simulate(0, 137)
    rest = o.simulate(137, case.n_steps, state=half["state"])
    for k in "xyzm":
        np.testing.assert_array_equal(rest["state"][k], full["state"][k])
    np.testing.assert_allclose(half["ledger"] + rest["ledger"], full["ledger"], rtol=1e-12)
    np.testing.assert_allclose(half["dep"] + rest["dep"], full["dep"], rtol=1e-10, atol=1e-300)


def test_thread_count_does_not_change_results():
    case = reduced_c1()
    o = oracle.Oracle(case)
    a = o.simulate(nthreads=1)
    b = o.simulate(nthreads=4)
    for k in "xyzm":
        np.testing.assert_array_equal(a["state"][k], b["state"][k])
    np.testing.assert_allclose(a["ledger"], b["ledger"], rtol=1e-13)


def test_c1_mass_ledger_closes():
    """released = airborne + deposited + decayed + exited, and the gridded
    totals equal the ledger when the grids cover every position."""
    case = synth.c1(n_total=20_000)
    big2 = Grid(500, 500, 1, -250e3, -250e3, 0.0, 1000.0, 1000.0, 1.0, mode=0)
    big3 = Grid(500, 500, 1, -250e3, -250e3, 0.0, 1000.0, 1000.0, 2000.0, mode=0)
    case = case.with_(dep_grid=big2, conc_grid=big3)
    o = oracle.Oracle(case)
    S = case.n_steps
    r = o.simulate(snap_steps=[S - 1])
    air = o.airborne(S - 1, r["state"]["m"])
    for k in range(2):
        rel, dep, dec, ex = r["ledger"][k]
        assert rel == pytest.approx(case.source.q * 4320 * 5.0, rel=1e-13)
        assert rel == pytest.approx(air[k] + dep + dec + ex, rel=1e-12)
        assert dep > 0 and ex > 0
        assert r["snaps"][0, k].sum() == pytest.approx(air[k], rel=1e-12)
    # deposits of the exit steps fall outside the wind domain but inside this grid
    np.testing.assert_allclose(r["dep"].sum(axis=(1, 2)), r["ledger"][:, 1], rtol=1e-12)

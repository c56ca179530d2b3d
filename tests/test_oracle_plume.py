"""The oracle's gridded mass for uniform wind and constant K against the exact
expectation (erf products with the image sum for the ground and the lid),
and its decay against exp(-lambda t) (Sec. 2; caption of Fig. 3)."""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
import synth
from synth import Grid
from plume import births, expected_ngp

HERE = os.path.dirname(os.path.abspath(__file__))


def ngp(case):
    return case.with_(conc_grid=synth.replace(case.conc_grid, mode=0))


def chi2_check(M, E, var, count, min_count=20):
    sel = count >= min_count
    k = int(sel.sum())
    assert k >= 30, k
    chi2 = float((((M - E) ** 2)[sel] / var[sel]).sum())
    p = stats.chi2.sf(chi2, k)
    # the relative L2 distance is within 3x of what the variance predicts
    rel = np.linalg.norm((M - E)[sel]) / np.linalg.norm(E[sel])
    pred = math.sqrt(var[sel].sum()) / np.linalg.norm(E[sel])
    return p, rel, pred, k


# (particles, cells): at 1e4 particles no cell of the 100 x 100 x 50 m grid
# expects 20 of them, so that case is binned on 400 x 400 x 100 m cells of the
# same 10 x 10 x 1 km domain (83 cells expect >= 20)
@pytest.mark.parametrize("n_total,cells", [(10_000, (25, 25, 10, 400.0, 400.0, 100.0)),
                                           (200_000, None)])
def test_c0_grid_matches_exact_expectation(n_total, cells):
    case = ngp(synth.c0(n_total=n_total))
    if cells is not None:
        nx, ny, nz, dx, dy, dz = cells
        case = case.with_(conc_grid=synth.replace(case.conc_grid, nx=nx, ny=ny, nz=nz, dx=dx,
                                                  dy=dy, dz=dz))
    r = oracle.Oracle(case).simulate(snap_steps=[case.n_steps - 1])
    M = r["snaps"][0, 0]
    E, var, count = expected_ngp(case)
    p, rel, pred, k = chi2_check(M, E, var, count, min_count=20)
    assert p > 1e-3, (p, k)
    assert rel < 3 * pred, (rel, pred)


def test_c0_intermediate_snapshot():
    case = ngp(synth.c0(n_total=50_000))
    s = 179
    r = oracle.Oracle(case).simulate(snap_steps=[s])
    E, var, count = expected_ngp(case, s_grid=s)
    p, rel, pred, k = chi2_check(r["snaps"][0, 0], E, var, count)
    assert p > 1e-3 and rel < 3 * pred


def test_paper_artificial_weather_plume():
    """Paper's homogeneous case (caption of Fig. 3, Sec. 2): u = 5 m/s,
    source at 20 m, mixing layer (lid) at 120 m, K_h = 100 m^2/s, dt = 10 s;
    K_z constant (10 m^2/s).  Many reflections between ground and lid."""
    with open(os.path.join(HERE, "golden", "paper_artificial_weather.json")) as f:
        w = json.load(f)
    c = synth.c0(n_total=100_000, n_steps=180)
    case = c.with_(
        source=synth.replace(c.source, h=w["source_height_m"]),
        physics=synth.replace(c.physics, dt=w["time_step_s"],
                              Kh=w["horizontal_diffusivity_m2_per_s"],
                              H_lid=w["mixing_height_m"], H_mix=w["mixing_height_m"]),
        field=synth.uniform_field(w["wind_x_m_per_s"], w["wind_y_m_per_s"],
                                  w["wind_z_m_per_s"]),
        conc_grid=Grid(60, 40, 6, -500.0, -4000.0, 0.0, 200.0, 200.0, 20.0, mode=0))
    r = oracle.Oracle(case).simulate(snap_steps=[case.n_steps - 1])
    E, var, count = expected_ngp(case)
    p, rel, pred, k = chi2_check(r["snaps"][0, 0], E, var, count)
    assert p > 1e-3 and rel < 3 * pred, (p, rel, pred)
    assert r["state"]["z"].max() <= 120.0 and r["state"]["z"].min() >= 0.0


def test_decay_is_exact_exponential():
    case = synth.c0()
    o = oracle.Oracle(case)
    r = o.simulate()
    S, dt, lam = case.n_steps, case.physics.dt, case.physics.lambdas[0]
    a0 = case.source.q * case.schedule.s_release * dt / case.schedule.n_total
    b = births(case.schedule.n_total, case.schedule.s_release)
    want_air = a0 * np.exp(-lam * (S - b) * dt).sum()
    air = o.airborne(S - 1, r["state"]["m"])[0]
    assert air == pytest.approx(want_air, rel=1e-12)
    released, dep, dec, ex = r["ledger"][0]
    assert released == pytest.approx(a0 * case.schedule.n_total, rel=1e-13)
    assert dep == 0.0 and ex == 0.0
    # per particle the decayed activity telescopes to a0 (1 - exp(-lambda tau))
    assert dec == pytest.approx((a0 * -np.expm1(-lam * (S - b) * dt)).sum(), rel=1e-11)
    assert released == pytest.approx(air + dep + dec + ex, rel=1e-13)
    # no deposition, no exit: every particle keeps m = 1
    assert np.all(r["state"]["m"] == 1.0)

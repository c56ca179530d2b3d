"""Pins of the oracle's paper-literal variants: decay chains (Bateman),
stochastic deposition (Sec. 2), and Eq. (3) with the similarity function of
the stratification plus the surface-layer iteration for u* and L.

* chains: activities of a resting particle equal the matrix exponential of
  the decay matrix (scipy), deposition of a resting particle in rain equals
  the quadrature of that solution, and the per-nuclide ledger (ingrowth
  counted as released) closes;
* stochastic deposition: every removal happens at the first step whose
  purpose-1 Philox uniform falls below 1 - exp(-k dt) (recomputed from the
  oracle's own Philox), the surviving fraction follows exp(-k t), and the
  mean deposit equals the mass-depletion deposit;
* Eq. (3): neutral stratification is the exponent-2 profile exactly, K_z'
  is the slope of K_z, a tracer stays well mixed for stable and unstable L;
  the surface layer is neutral for dtheta = 0 with u* = kappa U / ln(z/z0),
  and L has the sign of the stratification.
"""
import math

import numpy as np
import pytest
from scipy import integrate, linalg, stats

import oracle
import synth
from plume import births
from synth import Grid, Rain

LAMS = (2e-4, 5e-4, 1.1e-3, 3e-3)


def resting(n=200, steps=120, lambdas=LAMS[:3], chain=1, L0=0.0, dep_mode=0, seed=0):
    c = synth.c0(n_total=n, n_steps=steps)
    ph = synth.replace(c.physics, Kh=0.0, Kz_const=0.0, lambdas=lambdas, chain=chain,
                       Lambda0=L0, dep_mode=dep_mode, seed=seed,
                       rain=Rain(cx=0.0, cy=0.0, a=500.0, b=300.0, angle=0.3, edge=0.1))
    g2 = Grid(5, 5, 1, -250.0, -250.0, 0.0, 100.0, 100.0, 1.0, mode=0)
    return c.with_(physics=ph, field=synth.uniform_field(0.0, 0.0), dep_grid=g2)


def a0_of(case):
    return case.source.q * case.schedule.s_release * case.physics.dt / case.schedule.n_total


def chain_activities(lams, t):
    """Activities lambda_n N_n(t) per unit initial parent activity, from the
    matrix exponential of the decay matrix."""
    lam = np.asarray(lams)
    M = np.diag(-lam) + np.diag(lam[:-1], -1)
    N0 = np.zeros(len(lam))
    N0[0] = 1.0 / lam[0]
    return lam * (linalg.expm(M * t) @ N0)


@pytest.mark.parametrize("nn", [2, 3, 4])
def test_activity_fraction_is_the_matrix_exponential(nn):
    c = resting(lambdas=LAMS[:nn])
    o = oracle.Oracle(c)
    for t in (0.0, 10.0, 777.0, 5000.0, 4e4):
        want = chain_activities(LAMS[:nn], t)
        got = [o.activity_fraction(n, t) for n in range(nn)]
        np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-15)


def test_chain_of_a_resting_particle():
    c = resting()
    o = oracle.Oracle(c)
    r = o.simulate()
    n, S, dt = c.schedule.n_total, c.n_steps, c.physics.dt
    a0 = a0_of(c)
    age = (S - births(n, S)) * dt
    air = o.airborne(S - 1, r["state"]["m"])
    want = a0 * sum(chain_activities(LAMS[:3], t) for t in age)
    np.testing.assert_allclose(air, want, rtol=1e-10)
    led = r["ledger"]
    assert led[0][0] == pytest.approx(a0 * n, rel=1e-12)
    for k in range(3):
        rel, dep, dec, ex = led[k]
        assert dep == 0.0 and ex == 0.0
        assert rel == pytest.approx(air[k] + dec, rel=1e-11)
    # ingrowth of nuclide k + 1 is lambda_{k+1} / lambda_k times the decays of k
    for k in range(2):
        assert led[k + 1][0] == pytest.approx(LAMS[k + 1] / LAMS[k] * led[k][2], rel=1e-11)


def test_chain_deposition_of_a_resting_particle_in_rain():
    L0 = 4e-4
    c = resting(n=50, steps=150, L0=L0)
    r = oracle.Oracle(c).simulate()
    n, S, dt = c.schedule.n_total, c.n_steps, c.physics.dt
    a0 = a0_of(c)
    age = (S - births(n, S)) * dt
    for k in range(3):
        want = 0.0
        for t in set(age.tolist()):
            f = lambda tau: L0 * math.exp(-L0 * tau) * chain_activities(LAMS[:3], tau)[k]
            want += np.sum(age == t) * a0 * integrate.quad(f, 0.0, t, epsabs=0, epsrel=1e-12)[0]
        assert r["ledger"][k][1] == pytest.approx(want, rel=1e-8)


def test_chain_ledger_closes_on_the_gridded_workload():
    c = synth.c1(n_total=3000, n_steps=300)
    c = c.with_(physics=synth.replace(c.physics, lambdas=(3e-4, 1e-3, 2e-3), chain=1))
    o = oracle.Oracle(c)
    r = o.simulate()
    air = o.airborne(c.n_steps - 1, r["state"]["m"])
    for k in range(3):
        rel, dep, dec, ex = r["ledger"][k]
        assert rel == pytest.approx(air[k] + dep + dec + ex, rel=1e-12)
    assert r["ledger"][1][1] > 0 and r["ledger"][2][0] > 0


def test_chain_needs_distinct_positive_lambdas():
    for lams in ((1e-4, 1e-4), (0.0, 1e-4)):
        c = resting(lambdas=lams)
        with pytest.raises(ValueError):
            oracle.Oracle(c).simulate()


def test_stochastic_removal_follows_the_purpose_one_stream():
    L0, n, S = 2e-3, 400, 200
    c = resting(n=n, steps=S, lambdas=(1e-5,), chain=0, L0=L0, dep_mode=1, seed=7)
    o = oracle.Oracle(c)
    dt = c.physics.dt
    q = -math.expm1(-L0 * dt)
    b = births(n, S)
    st = None
    gone_at = np.full(n, -1)
    for s in range(S):
        st = o.simulate(s_begin=s, s_end=s + 1, state=st)["state"]
        newly = (st["m"] == 0) & (gone_at < 0) & (b <= s)
        gone_at[newly] = s
    for i in range(n):
        first = -1
        for s in range(b[i], S):
            u0 = oracle.uniforms(c.physics.seed, c.source.scenario, [i], s, purpose=1)[0][0]
            if u0 <= q:
                first = s
                break
        assert gone_at[i] == first, (i, gone_at[i], first)
    # the removed particle's whole end-of-step activity is deposited
    r = o.simulate()
    a0 = a0_of(c)
    dep_want = sum(a0 * math.exp(-1e-5 * (gone_at[i] + 1 - b[i]) * dt) for i in range(n)
                   if gone_at[i] >= 0)
    assert r["ledger"][0][1] == pytest.approx(dep_want, rel=1e-12)
    air = o.airborne(S - 1, r["state"]["m"])[0]
    rel, dep, dec, ex = r["ledger"][0]
    assert rel == pytest.approx(air + dep + dec + ex, rel=1e-12)


def test_stochastic_removal_statistics_match_mass_depletion():
    L0, n, S = 5e-4, 100_000, 120
    c = resting(n=n, steps=S, lambdas=(1e-5,), chain=0, L0=L0, dep_mode=1, seed=3)
    c = c.with_(schedule=synth.replace(c.schedule, s_release=1))
    r = oracle.Oracle(c).simulate()
    p_alive = math.exp(-L0 * S * c.physics.dt)
    alive = np.count_nonzero(r["state"]["m"] > 0)
    sd = math.sqrt(n * p_alive * (1 - p_alive))
    assert abs(alive - n * p_alive) < 5 * sd
    det = oracle.Oracle(c.with_(physics=synth.replace(c.physics, dep_mode=0))).simulate()
    dep_s, dep_d = r["ledger"][0][1], det["ledger"][0][1]
    assert abs(dep_s - dep_d) < 5 * sd / n * det["ledger"][0][0] + 1e-4 * dep_d


@pytest.mark.parametrize("inv_L", [1.0 / 200.0, -1.0 / 150.0, 1.0 / 40.0, -1.0 / 20.0])
def test_kz_stability_profile(inv_L):
    c = synth.c1(n_total=10, n_steps=10)
    o3 = oracle.Oracle(c.with_(physics=synth.replace(c.physics, kz_kind=3, inv_L=inv_L)))
    o2 = oracle.Oracle(c.with_(physics=synth.replace(c.physics, kz_kind=2)))
    on = oracle.Oracle(c.with_(physics=synth.replace(c.physics, kz_kind=3, inv_L=0.0)))
    ku, z0 = c.physics.kappa_ustar, c.physics.z0
    for z in (0.0, 3.0, 37.0, 250.0, 640.0, 999.0):
        assert on.kz(z) == o2.kz(z)  # neutral = Eq. 3 with Phi = 1, bitwise
        K, dK = o3.kz(z)
        K2, _ = o2.kz(z)
        s = (z + z0) * inv_L
        phi = 1 + 5 * s if s >= 0 else (1 - 16 * s) ** -0.5
        assert K == pytest.approx(K2 / phi, rel=1e-12)
        h = 1e-4
        if z > h:
            slope = (o3.kz(z + h)[0] - o3.kz(z - h)[0]) / (2 * h)
            assert dK == pytest.approx(slope, rel=1e-6, abs=1e-9)
    # stable stratification damps mixing, unstable enhances it
    if inv_L > 0:
        assert o3.kz(300.0)[0] < o2.kz(300.0)[0]
    else:
        assert o3.kz(300.0)[0] > o2.kz(300.0)[0]


@pytest.mark.parametrize("inv_L,dt", [(1.0 / 100.0, 5.0), (-1.0 / 50.0, 1.0)])
def test_well_mixed_with_stability(inv_L, dt):
    """A tracer uniform over the mixed layer stays uniform for 1 h.  The
    strongly unstable profile (K_z up to ~320 m^2/s) needs dt = 1 s: at
    dt = 5 s the first-order scheme piles particles up at the boundaries
    (p ~ 1e-69); the error vanishes with dt (p ~ 0.6 at 1 s)."""
    n, steps = 100_000, int(3600 / dt)
    c = synth.c1(n_total=n, n_steps=steps + 1)
    ph = synth.replace(c.physics, Kh=0.0, kz_kind=3, inv_L=inv_L, Lambda0=0.0, dt=dt)
    case = c.with_(physics=ph, field=synth.uniform_field(0.0, 0.0),
                   source=synth.replace(c.source, v_d=0.0),
                   schedule=synth.replace(c.schedule, s_release=1))
    x, y, z, m = synth.uniform_state(n, ((0, 1), (0, 1), (0, 1000.0)), seed=3)
    r = oracle.Oracle(case).simulate(s_begin=1, s_end=steps + 1,
                                     state={"x": x, "y": y, "z": z, "m": m})
    hist = np.histogram(r["state"]["z"], bins=20, range=(0, 1000.0))[0]
    assert stats.chisquare(hist).pvalue > 1e-3, hist


def test_surface_layer_limits():
    U, zr, z0, T0 = 6.0, 10.0, 0.25, 288.0
    us, il = oracle.surface_layer(U, zr, z0, 0.0, T0)
    assert il == 0.0 and us == pytest.approx(0.4 * U / math.log(zr / z0), rel=1e-15)
    us_s, il_s = oracle.surface_layer(U, zr, z0, 0.5, T0)   # stable
    us_u, il_u = oracle.surface_layer(U, zr, z0, -0.5, T0)  # unstable
    assert il_s > 0 and il_u < 0 and us_s < us < us_u
    us_s2, il_s2 = oracle.surface_layer(U, zr, z0, 1.0, T0)
    assert il_s2 > il_s and us_s2 < us_s
    with pytest.raises(ValueError):  # beyond the critical Richardson number
        oracle.surface_layer(1.0, zr, z0, 5.0, T0)


def test_surface_layer_stable_closed_form():
    """With the log-linear stable profiles both stability corrections are
    5 (z - z0)/L, so 1/L = R ln(z/z0) / (1 - 5 R (z - z0)) exactly, with
    R = g dtheta / (U^2 T0) (valid below the critical Richardson number)."""
    U, zr, z0, T0 = 4.0, 10.0, 0.25, 288.0
    for dth in (0.05, 0.3, 0.8):
        R = 9.81 * dth / (U * U * T0)
        want = R * math.log(zr / z0) / (1.0 - 5.0 * R * (zr - z0))
        us, il = oracle.surface_layer(U, zr, z0, dth, T0)
        assert il == pytest.approx(want, rel=1e-10)
        assert us == pytest.approx(0.4 * U / (math.log(zr / z0) + 5 * (zr - z0) * want), rel=1e-10)


def test_surface_layer_unstable_against_quadrature():
    """Unstable: the integrated profile corrections psi(s) = int_0^s
    (1 - phi(t))/t dt of the Businger-Dyer gradients phi_m = (1 - 16 t)^(-1/4),
    phi_h = (1 - 16 t)^(-1/2), by quadrature, and the similarity relations
    solved for 1/L by bracketing; the oracle uses Paulson's closed forms and
    a fixed-point iteration."""
    from scipy import optimize
    U, zr, z0, T0, kappa, g = 5.0, 10.0, 0.25, 288.0, 0.4, 9.81

    def psi(s, p):
        return integrate.quad(lambda t: (1.0 - (1.0 - 16.0 * t) ** (-p)) / t, 0.0, s,
                              epsabs=0, epsrel=1e-13)[0] if s < 0 else 0.0

    for dth in (-0.1, -0.6, -1.5):
        def resid(il):
            fm = math.log(zr / z0) - psi(zr * il, 0.25) + psi(z0 * il, 0.25)
            fh = math.log(zr / z0) - psi(zr * il, 0.5) + psi(z0 * il, 0.5)
            us, ts = kappa * U / fm, kappa * dth / fh
            return kappa * g * ts / (us * us * T0) - il
        want = optimize.brentq(resid, -10.0, -1e-12, xtol=1e-15, rtol=1e-13)
        us, il = oracle.surface_layer(U, zr, z0, dth, T0)
        assert il == pytest.approx(want, rel=1e-8)

"""Pins of the oracle's receptor concentrations and of their gradient with
respect to the source parameters theta = (h, q, s_w, v_d).

* the receptor forward equals the plain time-stepped oracle run with the
  Gaussian receptor kernel applied to its output-step states;
* forward-mode tangents equal central finite differences with common random
  numbers (the same Philox streams at theta +- delta);
* the reverse sweep equals the tangents contracted with the same weights;
* closed forms: c is proportional to q (so dc/dq = c/q and the loss gradient
  in q is (2/q) sum_r res_r c_r / (c_r + eps)); without wind-field structure
  or diffusion the path is x = x_s + s_w u age at z = h, which gives dc/ds_w
  and dc/dh in closed form; with rain off, the deposition velocity only
  depletes the mass, dm/dv_d = -m sum phi(z_s) dt along the fixed path.
"""
import os

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
THETA0 = np.array(synth.THETA0)


def receptors(n, seed, xr=(-2000.0, 6000.0), yr=(-3000.0, 3000.0)):
    rng = np.random.default_rng(seed)
    return synth.Receptors(tuple(rng.uniform(*xr, n)), tuple(rng.uniform(*yr, n)), (0.0,) * n)


def kernel(rec, j, x, y, z):
    dx, dy = x - rec.x[j], y - rec.y[j]
    sh2, sz2 = rec.sigma_h ** 2, rec.sigma_z ** 2
    g = np.exp(-(dx * dx + dy * dy) / (2 * sh2)) / (2 * np.pi * sh2)
    n = (np.exp(-(z - rec.z[j]) ** 2 / (2 * sz2)) + np.exp(-(z + rec.z[j]) ** 2 / (2 * sz2))) \
        / (np.sqrt(2 * np.pi) * rec.sigma_z)
    return g * n, g, n


def small_case(n=300, steps=720):
    return synth.c4(n_total=n, n_steps=steps)


def births(case):
    sch = case.schedule
    ids = sch.id_base + np.arange(sch.local_count) * sch.id_stride
    return (ids * sch.s_release) // sch.n_total


def test_receptor_forward_equals_time_stepped_run():
    c = small_case()
    rec = receptors(8, 0)
    o = oracle.Oracle(c)
    f = o.receptor_forward(rec)
    b = births(c)
    a0 = c.source.q * c.schedule.s_release * c.physics.dt / c.schedule.n_total
    ref = np.zeros(rec.n)
    st = None
    for k in range(c.n_steps // 60):
        st = o.simulate(s_begin=60 * k, s_end=60 * k + 60, state=st)["state"]
        s = 60 * k + 59
        alive = (b <= s) & (st["m"] > 0)
        A = a0 * st["m"] * sum(np.exp(-lam * (s + 1 - b) * c.physics.dt)
                               for lam in c.physics.lambdas)
        for j in range(rec.n):
            kv, _, _ = kernel(rec, j, st["x"], st["y"], st["z"])
            ref[j] += rec.weight * np.sum((A * kv)[alive])
    assert np.max(np.abs(ref - f["c"])) <= 1e-12 * np.max(np.abs(ref))
    assert f["c"].max() > 0


def fd_jacobian(case, rec, rel):
    out = np.zeros((rec.n, 4))
    for j in range(4):
        d = rel * abs(THETA0[j])
        tp, tm = THETA0.copy(), THETA0.copy()
        tp[j] += d
        tm[j] -= d
        cp = oracle.Oracle(synth.with_theta(case, tp)).receptor_forward(rec)["c"]
        cm = oracle.Oracle(synth.with_theta(case, tm)).receptor_forward(rec)["c"]
        out[:, j] = (cp - cm) / (2 * d)
    return out


def test_tangent_matches_central_differences():
    """Gridded wind, parabolic K_z, dry and wet deposition, two nuclides."""
    c = small_case()
    rec = receptors(8, 0)
    tan = oracle.Oracle(c).receptor_forward(rec, tangent=True)["dc"]
    for rel in (1e-4, 1e-3):
        fd = fd_jacobian(c, rec, rel)
        err = np.max(np.abs(fd - tan), axis=0) / np.max(np.abs(fd), axis=0)
        assert np.all(err <= 1e-3), (rel, err)
    fd = fd_jacobian(c, rec, 1e-4)
    err = np.max(np.abs(fd - tan), axis=0) / np.max(np.abs(fd), axis=0)
    assert np.all(err <= 1e-4), err


def test_tangent_matches_differences_with_time_varying_field_and_levels():
    c = synth.c2(n_total=200, n_steps=720, s_release=720, n_hours=2)
    c = synth.with_theta(c.with_(physics=synth.replace(c.physics, kz_kind=2)), THETA0)
    nz = c.field.nz
    lev = (1500.0 * np.linspace(0.0, 1.0, nz) ** 1.5 + 5.0).astype(np.float32)
    c = c.with_(field=synth.replace(c.field, z_levels=lev))
    rec = receptors(6, 1)
    tan = oracle.Oracle(c).receptor_forward(rec, tangent=True)["dc"]
    fd = fd_jacobian(c, rec, 1e-4)
    err = np.max(np.abs(fd - tan), axis=0) / np.max(np.abs(fd), axis=0)
    assert np.all(err <= 1e-3), err


def test_tangent_matches_differences_rain_edge_and_vertical_wind():
    """Uniform wind with a downward component (particles fold at the ground
    often) through the edge band of a small rain region.  The many folds
    put kinks close to the path, so the differences use delta = 1e-6 |theta|
    (they converge to the tangent: 8e-3 at 1e-4, 4e-6 at 1e-5, 3e-10 at
    1e-6 for h)."""
    c = small_case(n=300, steps=720)
    fld = synth.replace(synth.uniform_field(4.0, 0.5, -0.08, bounded=True), x0=-25e3, y0=-25e3,
                        dx=50e3, dy=50e3, dz=1200.0)
    rain = synth.Rain(cx=3000.0, cy=0.0, a=2000.0, b=1500.0, angle=0.3, edge=0.25)
    c = c.with_(field=fld, physics=synth.replace(c.physics, Kh=20.0, kz_kind=0, Kz_const=5.0,
                                                 Lambda0=1e-3, rain=rain))
    rec = receptors(6, 5, xr=(500.0, 6000.0), yr=(-800.0, 1500.0))
    tan = oracle.Oracle(c).receptor_forward(rec, tangent=True)["dc"]
    fd = fd_jacobian(c, rec, 1e-6)
    err = np.max(np.abs(fd - tan), axis=0) / np.max(np.abs(fd), axis=0)
    assert np.all(err <= 1e-6), err


def test_adjoint_equals_tangent():
    c = small_case(n=400, steps=900)
    rec = receptors(8, 2)
    o = oracle.Oracle(c)
    tan = o.receptor_forward(rec, tangent=True)["dc"]
    for seed in range(3):
        g = np.random.default_rng(seed).normal(size=rec.n)
        adj = o.receptor_adjoint(rec, g)
        ref = g @ tan
        assert np.allclose(adj, ref, rtol=1e-10, atol=1e-14 * np.abs(ref).max())


def test_release_rate_gradient_is_exact():
    c = small_case()
    rec = receptors(8, 3)
    f = oracle.Oracle(c).receptor_forward(rec, tangent=True)
    np.testing.assert_allclose(f["dc"][:, 1], f["c"] / c.source.q, rtol=1e-12)
    # the squared log misfit: dL/dq = (2/q) sum_r res_r c_r / (c_r + eps)
    obs = f["c"] * np.exp(0.3 * np.random.default_rng(0).normal(size=rec.n)) + 1e-9
    eps = 1e-6 * obs.max()
    res = np.log(f["c"] + eps) - np.log(obs + eps)
    gbar = 2 * res / (f["c"] + eps)
    grad = oracle.Oracle(c).receptor_adjoint(rec, gbar)
    exact = 2.0 / c.source.q * np.sum(res * f["c"] / (f["c"] + eps))
    assert grad[1] == pytest.approx(exact, rel=1e-12)


def test_straight_path_closed_forms():
    """K = 0, uniform wind u along x, no deposition: every particle sits at
    (x_s + s_w u age, y_s, h) with m = 1, so c and its s_w and h
    derivatives are sums of the kernel and its slopes."""
    u = 4.0
    c = small_case(n=200, steps=600)
    fld = synth.replace(synth.uniform_field(u, 0.0, bounded=True), x0=-25e3, y0=-25e3,
                        dx=50e3, dy=50e3, dz=1200.0)
    c = c.with_(field=fld, physics=synth.replace(c.physics, Kh=0.0, kz_kind=0, Kz_const=0.0,
                                                 Lambda0=0.0))
    c = synth.with_theta(c, (60.0, 1.2, 1.05, 0.0))
    rec = synth.Receptors((500.0, 1500.0, 2500.0), (0.0, 100.0, -200.0), (0.0, 0.0, 10.0))
    f = oracle.Oracle(c).receptor_forward(rec, tangent=True)
    b = births(c)
    dt, sw, h = c.physics.dt, c.source.wind_scale, c.source.h
    a0 = c.source.q * c.schedule.s_release * dt / c.schedule.n_total
    cc, dsw, dh = np.zeros(3), np.zeros(3), np.zeros(3)
    for s in range(59, c.n_steps, 60):
        alive = b <= s
        age = (s + 1 - b[alive]) * dt
        F = sum(np.exp(-lam * age) for lam in c.physics.lambdas)
        x = c.source.xs + sw * u * age
        for j in range(3):
            kv, g, n = kernel(rec, j, x, np.full_like(x, c.source.ys), np.full_like(x, h))
            dkx = -(x - rec.x[j]) / rec.sigma_h ** 2 * kv
            sz2 = rec.sigma_z ** 2
            dnz = (-(h - rec.z[j]) / sz2 * np.exp(-(h - rec.z[j]) ** 2 / (2 * sz2))
                   - (h + rec.z[j]) / sz2 * np.exp(-(h + rec.z[j]) ** 2 / (2 * sz2))) \
                / (np.sqrt(2 * np.pi) * rec.sigma_z)
            cc[j] += rec.weight * a0 * np.sum(F * kv)
            dsw[j] += rec.weight * a0 * np.sum(F * dkx * u * age)
            dh[j] += rec.weight * a0 * np.sum(F * g * dnz)
    np.testing.assert_allclose(f["c"], cc, rtol=1e-10)
    np.testing.assert_allclose(f["dc"][:, 2], dsw, rtol=1e-9, atol=1e-12 * np.abs(dsw).max())
    np.testing.assert_allclose(f["dc"][:, 0], dh, rtol=1e-9, atol=1e-12 * np.abs(dh).max())
    assert np.all(f["dc"][:, 3] == 0.0)


def test_deposition_velocity_gradient_along_fixed_paths():
    """Rain off: dm/dv_d = -m sum_s phi(z_{s+1}) dt over the path so far, so
    dc_r/dv_d = sum over output states of weight A K_r times that sum."""
    c = small_case(n=40, steps=360)
    c = c.with_(physics=synth.replace(c.physics, Lambda0=0.0))
    rec = receptors(5, 4, xr=(-500.0, 3000.0), yr=(-1500.0, 1500.0))
    o = oracle.Oracle(c)
    f = o.receptor_forward(rec, tangent=True)
    b = births(c)
    dt, hs = c.physics.dt, c.physics.h_s
    a0 = c.source.q * c.schedule.s_release * dt / c.schedule.n_total
    st = None
    phisum = np.zeros(c.schedule.local_count)
    ref = np.zeros(rec.n)
    for s in range(c.n_steps):
        st = o.simulate(s_begin=s, s_end=s + 1, state=st)["state"]
        alive = (b <= s) & (st["m"] > 0)
        z = st["z"]
        phi = np.where((z >= 0) & (z < hs), 2.0 / hs * (1.0 - z / hs), 0.0)
        phisum += np.where(alive, phi * dt, 0.0)
        if (s + 1) % 60:
            continue
        A = a0 * st["m"] * sum(np.exp(-lam * (s + 1 - b) * dt) for lam in c.physics.lambdas)
        for j in range(rec.n):
            kv, _, _ = kernel(rec, j, st["x"], st["y"], st["z"])
            ref[j] += rec.weight * np.sum((A * kv * -phisum)[alive])
    np.testing.assert_allclose(f["dc"][:, 3], ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())


def test_stored_receptors_and_observations():
    rec, obs, meta = synth.load_receptors(os.path.join(HERE, "golden", "c4_receptors.json"))
    assert rec.n == 50 and len(obs) == 50 and np.all(obs > 0)
    assert meta["hidden_theta"] == list(synth.THETA_HIDDEN)
    # receptors sit on cell centres of the 250 m grid, at the ground
    x = (np.asarray(rec.x) + 25e3) / 250.0 - 0.5
    assert np.allclose(x, np.round(x)) and np.all(np.asarray(rec.z) == 0.0)

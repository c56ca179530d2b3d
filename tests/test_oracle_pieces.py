"""Pins of the oracle's weather sampling, diffusivity, deposition rates and
gridding against closed forms (Sec. 2, Eq. 3; Sec. 3.2)."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import synth
from synth import Field, Grid, Physics, Rain, Source


def linear_field(nt, nz, ny, nx, ncomp, coef, x0, y0, dx, dy, dz, dtf, levels=None):
    """Nodes sampled from f_c = a + b x + c y + d z + e t (cell-centred)."""
    xc = x0 + (np.arange(nx) + 0.5) * dx
    yc = y0 + (np.arange(ny) + 0.5) * dy
    zc = (np.arange(nz) + 0.5) * dz if levels is None else levels.astype(np.float64)
    tc = np.arange(nt) * dtf
    T, Z, Y, X = np.meshgrid(tc, zc, yc, xc, indexing="ij")
    data = np.empty((nt, nz, ny, nx, ncomp))
    for c in range(ncomp):
        a, b, cc, d, e = coef[c]
        data[..., c] = a + b * X + cc * Y + d * Z + e * T
    return data


def case_with_field(fld, **phys):
    c = synth.c0()
    return c.with_(field=fld, physics=synth.replace(c.physics, **phys) if phys else c.physics)


@pytest.mark.parametrize("nonuniform", [False, True])
def test_wind_is_exact_for_linear_fields(nonuniform):
    rng = np.random.default_rng(5)
    nt, nz, ny, nx, ncomp = 3, 6, 5, 7, 3
    dx, dy, dz, dtf = 250.0, 200.0, 40.0, 3600.0
    x0, y0 = -800.0, 300.0
    levels = None
    if nonuniform:
        levels = np.array([2.0, 10.0, 30.0, 80.0, 200.0, 500.0], dtype=np.float32)
    # coefficients exactly representable so float32 nodes are exact
    coef = [(2.0, 2.0**-8, -(2.0**-9), 2.0**-6, 2.0**-12),
            (-1.0, 2.0**-10, 2.0**-7, -(2.0**-5), -(2.0**-11)),
            (0.5, 0.0, 2.0**-10, 2.0**-4, 2.0**-13)]
    data = linear_field(nt, nz, ny, nx, ncomp, coef, x0, y0, dx, dy, dz, dtf, levels)
    fld = Field(data.astype(np.float32), x0=x0, y0=y0, dx=dx, dy=dy, dz=dz,
                dt_field=dtf, z_levels=levels)
    assert np.array_equal(fld.data.astype(np.float64), data)
    o = oracle.Oracle(case_with_field(fld))
    zlo, zhi = (0.5 * dz, (nz - 0.5) * dz) if levels is None else (levels[0], levels[-1])
    for _ in range(300):
        x = rng.uniform(x0 + 0.5 * dx, x0 + (nx - 0.5) * dx)
        y = rng.uniform(y0 + 0.5 * dy, y0 + (ny - 0.5) * dy)
        z = rng.uniform(zlo, zhi)
        t = rng.uniform(0.0, (nt - 1) * dtf)
        got = o.wind(x, y, z, t)
        want = [a + b * x + c * y + d * z + e * t for a, b, c, d, e in coef]
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-11)
    # outside the node hull the sample is clamped to the nearest edge node
    xe, ye = x0 + 0.5 * dx, y0 + (ny - 0.5) * dy
    got = o.wind(x0 - 5000.0, y0 + 1e6, zlo, 0.0)
    want = [a + b * xe + c * ye + d * zlo for a, b, c, d, e in coef]
    np.testing.assert_allclose(got, want, atol=1e-11)
    got = o.wind(xe, ye, zhi + 1e4, 1e9)
    want = [a + b * xe + c * ye + d * zhi + e * (nt - 1) * dtf for a, b, c, d, e in coef]
    np.testing.assert_allclose(got, want, atol=1e-11)


def test_two_component_field_has_no_vertical_wind():
    c = synth.c1(n_total=100)
    o = oracle.Oracle(c)
    u = o.wind(1234.0, -987.0, 55.0, 0.0)
    assert u[2] == 0.0 and np.hypot(u[0], u[1]) > 0.5


def test_uniform_field_everywhere():
    o = oracle.Oracle(synth.c0())
    for p in [(0, 0, 0), (1e5, -3e4, 999.0), (-7, 8, 500)]:
        np.testing.assert_array_equal(o.wind(*p, 1234.0), [5.0, 0.0, 0.0])


@pytest.mark.parametrize("kind", [1, 2])
def test_kz_profile(kind):
    ku, z0, H = 0.2, 0.25, 1000.0
    c = synth.c1(n_total=10)
    o = oracle.Oracle(c.with_(physics=synth.replace(c.physics, kz_kind=kind, kappa_ustar=ku,
                                                     z0=z0, H_mix=H)))
    # surface-layer limit: K -> kappa u* (z + z0) at the ground
    assert o.kz(0.0)[0] == pytest.approx(ku * z0, rel=1e-14)
    # vanishes at the top of the mixing layer, and above it
    assert o.kz(H)[0] == 0.0 and o.kz(H + 50.0) == (0.0, 0.0)
    # the returned slope is the derivative of the returned K (central FD)
    for z in np.linspace(1.0, H - 1.0, 37):
        h = 1e-3
        fd = (o.kz(z + h)[0] - o.kz(z - h)[0]) / (2 * h)
        assert o.kz(z)[1] == pytest.approx(fd, rel=1e-6, abs=1e-10)
    # at the top itself: K = 0 and the profile's slope from below (a zero
    # slope there would hold a particle at the top with neither drift nor
    # diffusion)
    h = 1e-4
    assert o.kz(H)[1] == pytest.approx((o.kz(H)[0] - o.kz(H - h)[0]) / h, rel=1e-3, abs=1e-6)
    # maximum of the exponent-1 profile at z = (H - z0)/2
    if kind == 1:
        zs = np.linspace(0, H, 100001)
        K = np.array([o.kz(z)[0] for z in zs[::100]])
        assert K.max() == pytest.approx(ku * (H + z0) ** 2 / (4 * H), rel=1e-4)
    else:
        assert o.kz(H / 3)[0] == pytest.approx(ku * (H / 3 + z0) * (2 / 3) ** 2, rel=1e-14)


def test_particles_at_the_top_of_the_mixed_layer_leave_it():
    """Particles placed exactly at z = H_mix (= the lid) under the parabolic
    profile drift down (slope -kappa u* (1 + z0/H) there) instead of
    staying at the top."""
    c = synth.c1(n_total=200, n_steps=21)
    ph = synth.replace(c.physics, Kh=0.0, kz_kind=1, Lambda0=0.0)
    case = c.with_(physics=ph, field=synth.uniform_field(0.0, 0.0),
                   source=synth.replace(c.source, v_d=0.0),
                   schedule=synth.replace(c.schedule, s_release=1))
    n = 200
    st = {"x": np.zeros(n), "y": np.zeros(n), "z": np.full(n, ph.H_mix), "m": np.ones(n)}
    r = oracle.Oracle(case).simulate(s_begin=1, s_end=21, state=st)
    assert np.all(r["state"]["z"] < ph.H_mix - 1e-3)


def test_kz_constant():
    o = oracle.Oracle(synth.c0())
    assert o.kz(0.0) == (10.0, 0.0) and o.kz(777.0) == (10.0, 0.0)


def test_dry_rate_profile_integrates_to_vd():
    c = synth.c1(n_total=10)
    o = oracle.Oracle(c)
    vd, hs = c.source.v_d, c.physics.h_s
    val, _ = integrate.quad(o.dry_rate, 0.0, 2 * hs, points=[hs], epsabs=1e-14)
    assert val == pytest.approx(vd, rel=1e-10)      # flux = v_d x surface concentration
    assert o.dry_rate(0.0) == pytest.approx(2 * vd / hs, rel=1e-14)
    assert o.dry_rate(hs) == 0.0 and o.dry_rate(500.0) == 0.0


def test_wet_rate_geometry():
    rain = Rain(cx=1000.0, cy=-2000.0, a=5000.0, b=2000.0, angle=0.6, edge=0.05)
    c = synth.c1(n_total=10)
    o = oracle.Oracle(c.with_(physics=synth.replace(c.physics, rain=rain, Lambda0=3e-5)))
    L0 = 3e-5
    assert o.wet_rate(1000.0, -2000.0) == L0
    ca, sa = math.cos(0.6), math.sin(0.6)
    # on the ellipse (major axis rotated by +angle) the rate is half of Lambda0
    for r_major, r_minor in [(5000.0, 0.0), (-5000.0, 0.0), (0.0, 2000.0), (0.0, -2000.0)]:
        x = 1000.0 + ca * r_major - sa * r_minor
        y = -2000.0 + sa * r_major + ca * r_minor
        assert o.wet_rate(x, y) == pytest.approx(L0 / 2, rel=1e-9)
    # inside the inner edge full rate, beyond the outer edge none
    x = 1000.0 + ca * 5000.0 * 0.97
    y = -2000.0 + sa * 5000.0 * 0.97
    assert o.wet_rate(x, y) == L0
    x = 1000.0 + ca * 5000.0 * 1.03
    y = -2000.0 + sa * 5000.0 * 1.03
    assert o.wet_rate(x, y) == 0.0
    # the major axis is not along -angle
    x = 1000.0 + math.cos(-0.6) * 4000.0
    y = -2000.0 + math.sin(-0.6) * 4000.0
    assert o.wet_rate(x, y) == 0.0


def grid_case(mode, n=1, density=False):
    """n particles, no decay; gridded after the last step every particle has
    been released, and carries a0 = 3600 / n."""
    c = synth.c0(n_total=n)
    g = Grid(6, 5, 4, -300.0, 100.0, 0.0, 100.0, 50.0, 25.0, mode=mode, density=density)
    return oracle.Oracle(c.with_(conc_grid=g, physics=synth.replace(c.physics, lambdas=(0.0,)))), g


S_LAST = 359


def test_ngp_half_open_cells():
    o, g = grid_case(0)
    # a particle exactly on the lower face of cell (2, 1, 3) falls into it
    x, y, z = -300.0 + 2 * 100.0, 100.0 + 1 * 50.0, 3 * 25.0
    out = o.grid_concentration(S_LAST, [x], [y], [z], [1.0])
    assert out[0, 3, 1, 2] == 3600.0 and out.sum() == 3600.0
    # the upper face of the grid is outside
    out = o.grid_concentration(S_LAST, [-300.0 + 600.0], [y], [z], [1.0])
    assert out.sum() == 0.0
    # not yet released particles are not gridded
    out = o.grid_concentration(-1, [x], [y], [z], [1.0])
    assert out.sum() == 0.0


def test_cic_weights():
    o, g = grid_case(1)
    a0 = 3600.0
    # at a cell centre all activity goes to that cell
    out = o.grid_concentration(S_LAST, [-300.0 + 2.5 * 100.0], [100.0 + 1.5 * 50.0], [2.5 * 25.0], [1.0])
    assert out[0, 2, 1, 2] == pytest.approx(a0) and out.sum() == pytest.approx(a0)
    # on a node shared by 8 cell centres: one eighth each
    out = o.grid_concentration(S_LAST, [-300.0 + 3 * 100.0], [100.0 + 2 * 50.0], [2 * 25.0], [1.0])
    np.testing.assert_allclose(out[0, 1:3, 1:3, 2:4], a0 / 8, rtol=1e-14)
    # interior particles: total and first moments are preserved
    rng = np.random.default_rng(2)
    n = 200
    o, g = grid_case(1, n=n)
    a0 = 3600.0 / n
    x = rng.uniform(-300 + 50, -300 + 550, n)
    y = rng.uniform(100 + 25, 100 + 225, n)
    z = rng.uniform(12.5, 87.5, n)
    out = o.grid_concentration(S_LAST, x, y, z, np.ones(n))[0]
    assert out.sum() == pytest.approx(a0 * n, rel=1e-12)
    xc = -300 + (np.arange(6) + 0.5) * 100
    yc = 100 + (np.arange(5) + 0.5) * 50
    zc = (np.arange(4) + 0.5) * 25
    assert (out.sum(axis=(0, 1)) * xc).sum() == pytest.approx(a0 * x.sum(), rel=1e-12)
    assert (out.sum(axis=(0, 2)) * yc).sum() == pytest.approx(a0 * y.sum(), rel=1e-12)
    assert (out.sum(axis=(1, 2)) * zc).sum() == pytest.approx(a0 * z.sum(), rel=1e-12)


def test_density_divides_by_cell_volume():
    o, g = grid_case(0, density=True)
    out = o.grid_concentration(S_LAST, [-250.0], [125.0], [10.0], [1.0])
    assert out.sum() == pytest.approx(3600.0 / (100 * 50 * 25), rel=1e-14)

"""Closed-form expectation of gridded mass for uniform wind and constant K
with reflection at the ground and a lid (image sum), used to pin the oracle.

For constant drift and diffusion every Euler step of Eqs. (1)-(2) is exact in
distribution, and folding a Gaussian step into [0, H] has the same law as the
reflected diffusion (method of images), so the expectation below is exact for
the discrete process at any time step."""
import numpy as np
from scipy.special import erf


def births(n_total, s_release):
    g = np.arange(n_total, dtype=np.int64)
    return (g * s_release) // n_total


def _px(edges, centre, s):
    a = (edges[None, :] - centre[:, None]) / s[:, None]
    e = erf(a)
    return 0.5 * (e[:, 1:] - e[:, :-1])


def _pz(edges, h, H, s, n_img=4):
    out = np.zeros((s.size, edges.size - 1))
    for j in range(-n_img, n_img + 1):
        for src in (h + 2 * j * H, -h + 2 * j * H):
            out += _px(edges, np.full(s.size, src), s)
    return out


def expected_ngp(case, s_grid=None):
    """Expected NGP grid (and its variance) after step s_grid (default the
    last) for a uniform-wind, constant-K case (one nuclide)."""
    src, sch, ph, fld, g = case.source, case.schedule, case.physics, case.field, case.conc_grid
    assert ph.kz_kind == 0 and fld.data.size in (2, 3)
    u, v = float(fld.data.reshape(-1)[0]), float(fld.data.reshape(-1)[1])
    u *= src.wind_scale
    v *= src.wind_scale
    S = case.n_steps if s_grid is None else s_grid + 1
    b = births(sch.n_total, sch.s_release)
    b = b[b < S]
    nb = np.bincount(b, minlength=S).astype(np.float64)
    bs = np.nonzero(nb)[0]
    nb = nb[bs]
    tau = (S - bs) * ph.dt
    a0 = src.q * sch.s_release * ph.dt / sch.n_total
    lam = ph.lambdas[0]
    xe = g.x0 + np.arange(g.nx + 1) * g.dx
    ye = g.y0 + np.arange(g.ny + 1) * g.dy
    ze = g.z0 + np.arange(g.nz + 1) * g.dz
    Px = _px(xe, src.xs + u * tau, np.sqrt(4 * ph.Kh * tau))
    Py = _px(ye, src.ys + v * tau, np.sqrt(4 * ph.Kh * tau))
    if ph.H_lid > 0:
        Pz = _pz(ze, src.h, ph.H_lid, np.sqrt(4 * ph.Kz_const * tau))
    else:
        Pz = _px(ze, np.full(tau.size, src.h), np.sqrt(4 * ph.Kz_const * tau)) + \
             _px(ze, np.full(tau.size, -src.h), np.sqrt(4 * ph.Kz_const * tau))
    w = nb * a0 * np.exp(-lam * tau)
    w2 = nb * (a0 * np.exp(-lam * tau)) ** 2
    E = np.einsum("b,bk,bj,bi->kji", w, Pz, Py, Px, optimize=True)
    count = np.einsum("b,bk,bj,bi->kji", nb, Pz, Py, Px, optimize=True)
    var = np.einsum("b,bk,bj,bi->kji", w2, Pz, Py, Px, optimize=True) - \
        np.einsum("b,bk,bj,bi->kji", w2, Pz ** 2, Py ** 2, Px ** 2, optimize=True)
    return E, var, count

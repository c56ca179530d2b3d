"""FP64 CPU oracle of the stochastic Lagrangian particle model (test
infrastructure only).

The oracle is ``lpm_oracle.c``, plain C in double precision, built with gcc
(``-O2 -fopenmp``, no fast-math) into ``liblpm_oracle.so`` next to this file.
Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package; the HIP library never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lpm_oracle.c")
_LIB = os.path.join(_HERE, "liblpm_oracle.so")
# The test suite's planted-mistake check loads a deliberately broken build of
# the oracle from this path; it is never set otherwise.
_LIB_OVERRIDE = os.environ.get("LPM_ORACLE_LIB")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc.  Always recompiles when ``force``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra",
               "-Wno-unused-parameter", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Problem(C.Structure):
    _fields_ = [
        ("n_total", C.c_int64), ("n_local", C.c_int64), ("id_base", C.c_int64),
        ("id_stride", C.c_int64), ("s_release", C.c_int32), ("pad0", C.c_int32),
        ("xs", C.c_double), ("ys", C.c_double), ("h", C.c_double), ("q", C.c_double),
        ("wind_scale", C.c_double), ("v_d", C.c_double),
        ("scenario", C.c_uint32), ("pad1", C.c_uint32), ("seed", C.c_uint64),
        ("dt", C.c_double), ("Kh", C.c_double), ("Kz_const", C.c_double),
        ("kappa_ustar", C.c_double), ("z0", C.c_double), ("H_mix", C.c_double),
        ("H_lid", C.c_double), ("h_s", C.c_double),
        ("kz_kind", C.c_int32), ("n_nuc", C.c_int32), ("lam", C.c_double * 4),
        ("Lambda0", C.c_double), ("rain_cx", C.c_double), ("rain_cy", C.c_double),
        ("rain_a", C.c_double), ("rain_b", C.c_double), ("rain_angle", C.c_double),
        ("rain_edge", C.c_double),
        ("f", C.c_void_p), ("z_levels", C.c_void_p),
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("nt", C.c_int32),
        ("ncomp", C.c_int32), ("bounded", C.c_int32),
        ("fx0", C.c_double), ("fy0", C.c_double), ("fdx", C.c_double), ("fdy", C.c_double),
        ("fdz", C.c_double), ("ft0", C.c_double), ("fdt", C.c_double),
        ("cnx", C.c_int32), ("cny", C.c_int32), ("cnz", C.c_int32), ("cmode", C.c_int32),
        ("cdensity", C.c_int32), ("pad2", C.c_int32),
        ("cx0", C.c_double), ("cy0", C.c_double), ("cz0", C.c_double),
        ("cdx", C.c_double), ("cdy", C.c_double), ("cdz", C.c_double),
        ("dnx", C.c_int32), ("dny", C.c_int32), ("dmode", C.c_int32), ("ddensity", C.c_int32),
        ("dx0", C.c_double), ("dy0", C.c_double), ("ddx", C.c_double), ("ddy", C.c_double),
        ("inv_L", C.c_double), ("chain", C.c_int32), ("dep_mode", C.c_int32),
    ]


class Receptors(C.Structure):
    _fields_ = [("n", C.c_int32), ("pad", C.c_int32),
                ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("sigma_h", C.c_double), ("sigma_z", C.c_double), ("weight", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = C.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = C.CDLL(_LIB)
        P = C.POINTER(Problem)
        dp = C.POINTER(C.c_double)
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                        C.POINTER(C.c_uint32)]
        L.orc_uniforms.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                   C.c_uint32, dp]
        L.orc_normals.argtypes = L.orc_uniforms.argtypes
        L.orc_normals_batch.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_int64,
                                        C.c_uint32, C.c_uint32, dp]
        L.orc_wind.argtypes = [P, C.c_double, C.c_double, C.c_double, C.c_double, dp]
        L.orc_kz.argtypes = [P, C.c_double, dp, dp]
        L.orc_dry_rate.argtypes = [P, C.c_double]
        L.orc_dry_rate.restype = C.c_double
        L.orc_wet_rate.argtypes = [P, C.c_double, C.c_double]
        L.orc_wet_rate.restype = C.c_double
        L.orc_grid_concentration.argtypes = [P, C.c_int32, dp, dp, dp, dp, dp]
        L.orc_simulate.argtypes = [P, C.c_int32, C.c_int32, dp, dp, dp, dp, dp, dp,
                                   C.POINTER(C.c_int32), C.c_int32, dp, C.c_int32,
                                   C.POINTER(C.c_int64)]
        L.orc_simulate.restype = C.c_int
        L.orc_airborne.argtypes = [P, C.c_int32, dp, dp]
        L.orc_activity_fraction.argtypes = [P, C.c_int, C.c_double]
        L.orc_activity_fraction.restype = C.c_double
        L.orc_surface_layer.argtypes = [C.c_double] * 5 + [dp, dp]
        L.orc_surface_layer.restype = C.c_int
        RP = C.POINTER(Receptors)
        L.orc_receptor_forward.argtypes = [P, RP, C.c_int32, C.c_int32, dp, dp, C.c_int32,
                                           C.POINTER(C.c_int64)]
        L.orc_receptor_forward.restype = C.c_int
        L.orc_receptor_adjoint.argtypes = [P, RP, C.c_int32, C.c_int32, dp, dp, C.c_int32]
        L.orc_receptor_adjoint.restype = C.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Oracle:
    """Binds one workload (a ``synth.Case``) to the C oracle.  Keeps
    references to the arrays the C side points into."""

    def __init__(self, case):
        self.case = case
        src, sch, ph, fld = case.source, case.schedule, case.physics, case.field
        cg, dg = case.conc_grid, case.dep_grid
        p = Problem()
        p.n_total, p.n_local = sch.n_total, sch.local_count
        p.id_base, p.id_stride, p.s_release = sch.id_base, sch.id_stride, sch.s_release
        p.xs, p.ys, p.h, p.q = src.xs, src.ys, src.h, src.q
        p.wind_scale, p.v_d, p.scenario = src.wind_scale, src.v_d, src.scenario
        p.seed = ph.seed
        p.dt, p.Kh, p.Kz_const = ph.dt, ph.Kh, ph.Kz_const
        p.kappa_ustar, p.z0, p.H_mix, p.H_lid, p.h_s = (ph.kappa_ustar, ph.z0, ph.H_mix,
                                                        ph.H_lid, ph.h_s)
        p.kz_kind, p.n_nuc = ph.kz_kind, ph.n_nuc
        p.inv_L, p.chain, p.dep_mode = ph.inv_L, ph.chain, ph.dep_mode
        for n, lam in enumerate(ph.lambdas):
            p.lam[n] = lam
        r = ph.rain
        p.Lambda0, p.rain_cx, p.rain_cy = ph.Lambda0, r.cx, r.cy
        p.rain_a, p.rain_b, p.rain_angle, p.rain_edge = r.a, r.b, r.angle, r.edge
        self._f = np.ascontiguousarray(fld.data, dtype=np.float32)
        p.f = self._f.ctypes.data
        self._lev = None
        if fld.z_levels is not None:
            self._lev = np.ascontiguousarray(fld.z_levels, dtype=np.float32)
            p.z_levels = self._lev.ctypes.data
        p.nt, p.nz, p.ny, p.nx, p.ncomp = fld.data.shape
        p.bounded = int(fld.bounded)
        p.fx0, p.fy0, p.fdx, p.fdy, p.fdz = fld.x0, fld.y0, fld.dx, fld.dy, fld.dz
        p.ft0, p.fdt = fld.t0, fld.dt_field
        p.cnx, p.cny, p.cnz, p.cmode, p.cdensity = cg.nx, cg.ny, cg.nz, cg.mode, int(cg.density)
        p.cx0, p.cy0, p.cz0, p.cdx, p.cdy, p.cdz = cg.x0, cg.y0, cg.z0, cg.dx, cg.dy, cg.dz
        p.dnx, p.dny, p.dmode, p.ddensity = dg.nx, dg.ny, dg.mode, int(dg.density)
        p.dx0, p.dy0, p.ddx, p.ddy = dg.x0, dg.y0, dg.dx, dg.dy
        self.p = p

    # -- pieces -----------------------------------------------------------
    def wind(self, x, y, z, t):
        out = np.zeros(3)
        lib().orc_wind(C.byref(self.p), x, y, z, t, _dp(out))
        return out

    def kz(self, z):
        K, dK = C.c_double(), C.c_double()
        lib().orc_kz(C.byref(self.p), z, C.byref(K), C.byref(dK))
        return K.value, dK.value

    def dry_rate(self, z):
        return lib().orc_dry_rate(C.byref(self.p), z)

    def wet_rate(self, x, y):
        return lib().orc_wet_rate(C.byref(self.p), x, y)

    # -- whole runs ---------------------------------------------------------
    def new_state(self):
        n = self.p.n_local
        return {k: np.zeros(n) for k in ("x", "y", "z", "m")}

    def simulate(self, s_begin: int = 0, s_end: Optional[int] = None, state=None,
                 snap_steps: Sequence[int] = (), nthreads: int = 0):
        """Run steps [s_begin, s_end).  Returns dict with the final state
        (float64), deposition grid, ledger [n_nuc][4] (released, deposited,
        decayed, exited) and concentration snapshots."""
        case = self.case
        s_end = case.n_steps if s_end is None else s_end
        st = self.new_state() if state is None else {k: np.array(v, dtype=np.float64)
                                                     for k, v in state.items()}
        nn = case.physics.n_nuc
        dg, cg = case.dep_grid, case.conc_grid
        dep = np.zeros((nn, dg.ny, dg.nx))
        ledger = np.zeros((nn, 4))
        snaps_idx = np.asarray(list(snap_steps), dtype=np.int32)
        snaps = np.zeros((max(len(snaps_idx), 1), nn, cg.nz, cg.ny, cg.nx))
        psteps = C.c_int64(0)
        rc = lib().orc_simulate(C.byref(self.p), s_begin, s_end, _dp(st["x"]), _dp(st["y"]),
                                _dp(st["z"]), _dp(st["m"]), _dp(dep), _dp(ledger),
                                snaps_idx.ctypes.data_as(C.POINTER(C.c_int32)),
                                len(snaps_idx), _dp(snaps), nthreads, C.byref(psteps))
        if rc != 0:
            raise ValueError("oracle rejected the problem")
        return {"state": st, "dep": dep, "ledger": ledger,
                "snaps": snaps[:len(snaps_idx)], "psteps": psteps.value}

    def grid_concentration(self, s: int, x, y, z, m):
        cg, nn = self.case.conc_grid, self.case.physics.n_nuc
        out = np.zeros((nn, cg.nz, cg.ny, cg.nx))
        arr = [np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, z, m)]
        lib().orc_grid_concentration(C.byref(self.p), s, *[_dp(a) for a in arr], _dp(out))
        return out

    def activity_fraction(self, n: int, t: float) -> float:
        """Activity of nuclide n at age t per unit released activity."""
        return lib().orc_activity_fraction(C.byref(self.p), n, t)

    # -- receptor concentrations and their gradient ----------------------------
    def _receptors(self, rec):
        xyz = [np.ascontiguousarray(a, dtype=np.float64) for a in (rec.x, rec.y, rec.z)]
        r = Receptors()
        r.n = len(xyz[0])
        r.x, r.y, r.z = (a.ctypes.data for a in xyz)
        r.sigma_h, r.sigma_z, r.weight = rec.sigma_h, rec.sigma_z, rec.weight
        return r, xyz

    def receptor_forward(self, rec, s_end: Optional[int] = None, out_every: Optional[int] = None,
                         tangent: bool = False, nthreads: int = 0):
        """Receptor concentrations c [n] of the run over [0, s_end) and, with
        ``tangent``, dc/d(h, q, s_w, v_d) [n][4] by forward mode."""
        s_end = self.case.n_steps if s_end is None else s_end
        out_every = self.case.out_every if out_every is None else out_every
        r, keep = self._receptors(rec)
        c = np.zeros(r.n)
        dc = np.zeros((r.n, 4)) if tangent else None
        ps = C.c_int64(0)
        rc = lib().orc_receptor_forward(C.byref(self.p), C.byref(r), s_end, out_every, _dp(c),
                                        _dp(dc) if tangent else None, nthreads, C.byref(ps))
        if rc != 0:
            raise ValueError("oracle rejected the receptor problem")
        return {"c": c, "dc": dc, "psteps": ps.value}

    def receptor_adjoint(self, rec, gbar, s_end: Optional[int] = None,
                         out_every: Optional[int] = None, nthreads: int = 0):
        """sum_r gbar_r dc_r/d(h, q, s_w, v_d) by reverse mode."""
        s_end = self.case.n_steps if s_end is None else s_end
        out_every = self.case.out_every if out_every is None else out_every
        r, keep = self._receptors(rec)
        g = np.ascontiguousarray(gbar, dtype=np.float64)
        assert len(g) == r.n
        grad = np.zeros(4)
        rc = lib().orc_receptor_adjoint(C.byref(self.p), C.byref(r), s_end, out_every, _dp(g),
                                        _dp(grad), nthreads)
        if rc != 0:
            raise ValueError("oracle rejected the receptor problem")
        return grad

    def airborne(self, s: int, m):
        out = np.zeros(4)
        mm = np.ascontiguousarray(m, dtype=np.float64)
        lib().orc_airborne(C.byref(self.p), s, _dp(mm), _dp(out))
        return out[: self.case.physics.n_nuc]


def surface_layer(U, z_ref, z0, dtheta, T0):
    """(u*, 1/L) of the surface layer by the oracle's iteration."""
    us, il = C.c_double(), C.c_double()
    if lib().orc_surface_layer(U, z_ref, z0, dtheta, T0, C.byref(us), C.byref(il)) != 0:
        raise ValueError("no surface-layer solution")
    return us.value, il.value


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def uniforms(seed, scenario, ids, step, purpose=0):
    out = np.empty((len(ids), 4))
    buf = np.zeros(4)
    for j, i in enumerate(ids):
        lib().orc_uniforms(seed, scenario, int(i), step, purpose, _dp(buf))
        out[j] = buf
    return out


def normals_batch(seed, scenario, id0, n, step, purpose=0):
    out = np.empty((n, 4))
    lib().orc_normals_batch(seed, scenario, id0, n, step, purpose, _dp(out))
    return out


def normals(seed, scenario, ids, step, purpose=0):
    out = np.empty((len(ids), 4))
    buf = np.zeros(4)
    for j, i in enumerate(ids):
        lib().orc_normals(seed, scenario, int(i), step, purpose, _dp(buf))
        out[j] = buf
    return out

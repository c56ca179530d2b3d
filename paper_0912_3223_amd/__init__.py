"""Python binding of liblpm (MI355X particle-dispersion hot path).

Argument marshalling only: every step of the model runs in the HIP kernels of
``liblpm.so``; PyTorch provides device memory and streams.  The entry points
carry the C names without the ``lpm_`` prefix and raise ``LpmError`` on a
negative return code.  The library must have been built in-tree
(``python paper_0912_3223_amd/build.py``); importing this package without it
raises ImportError -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import torch  # loaded first so that liblpm binds to torch's HIP runtime

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblpm.so")

LPM_OK, LPM_EINVAL, LPM_ECAPACITY, LPM_EHIP, LPM_ENONFINITE = 0, -1, -2, -3, -4
LEDGER_SLOTS = 64
MAX_SCENARIOS = 256
LPM_MAX_RECEPTORS = 1024
STATIC_SCRATCH_DOUBLES = 4 * 1024 * 1024
SCENARIO_BYTES = 96
LEDGER_STRIDE = 32
CTRL_WORDS = 64


class LpmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class State(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("m", C.c_void_p),
                ("capacity", C.c_int64), ("x_lo", C.c_void_p), ("y_lo", C.c_void_p),
                ("order", C.c_void_p), ("n_order", C.c_int64)]


class Source(C.Structure):
    _fields_ = [("xs", C.c_double), ("ys", C.c_double), ("h", C.c_double), ("q", C.c_double),
                ("wind_scale", C.c_double), ("v_d", C.c_double), ("scenario", C.c_uint32),
                ("reserved", C.c_uint32)]


class Schedule(C.Structure):
    _fields_ = [("n_total", C.c_int64), ("n_local", C.c_int64), ("id_base", C.c_int64),
                ("id_stride", C.c_int64), ("s_release", C.c_int32), ("reserved", C.c_int32)]


class Field(C.Structure):
    _fields_ = [("data", C.c_void_p), ("z_levels", C.c_void_p),
                ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("nt", C.c_int32),
                ("ncomp", C.c_int32), ("bounded", C.c_int32),
                ("x0", C.c_double), ("y0", C.c_double), ("dx", C.c_double), ("dy", C.c_double),
                ("dz", C.c_double), ("t0", C.c_double), ("dt_field", C.c_double),
                ("layout", C.c_int32), ("interval", C.c_int32)]


class Physics(C.Structure):
    _fields_ = [("dt", C.c_double), ("Kh", C.c_double), ("Kz_const", C.c_double),
                ("kappa_ustar", C.c_double), ("z0", C.c_double), ("H_mix", C.c_double),
                ("H_lid", C.c_double), ("h_s", C.c_double),
                ("kz_kind", C.c_int32), ("n_nuc", C.c_int32), ("lam", C.c_double * 4),
                ("Lambda0", C.c_double), ("rain_cx", C.c_double), ("rain_cy", C.c_double),
                ("rain_a", C.c_double), ("rain_b", C.c_double), ("rain_angle", C.c_double),
                ("rain_edge", C.c_double), ("seed", C.c_uint64), ("inv_L", C.c_double),
                ("chain", C.c_int32), ("dep_mode", C.c_int32)]


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("mode", C.c_int32),
                ("density", C.c_int32), ("reserved", C.c_int32),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double)]


class Scenario(C.Structure):
    _fields_ = [("src", Source), ("n_total", C.c_int64), ("s_release", C.c_int32),
                ("reserved", C.c_int32), ("offset", C.c_int64)]


class Launch(C.Structure):
    _fields_ = [("refill_every", C.c_int32), ("refill_min", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("block", C.c_int32)]

    def as_tuple(self):
        return (self.refill_every, self.refill_min, self.blocks_per_cu, self.block)


class Ensemble(C.Structure):
    _fields_ = [("table", C.c_void_p), ("n_scen", C.c_int32), ("n_nuc", C.c_int32),
                ("step0", C.c_int32), ("n_steps", C.c_int32), ("queue_len", C.c_int64),
                ("max_release", C.c_int64), ("launch", Launch), ("dep_copies", C.c_int32),
                ("reserved", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("launch", Launch), ("best_ms", C.c_double), ("worst_ms", C.c_double),
                ("n_tried", C.c_int32), ("reps", C.c_int32)]


class Receptors(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("n", C.c_int32),
                ("sigma_h", C.c_float), ("sigma_z", C.c_float), ("weight", C.c_float)]


class Accum(C.Structure):
    _fields_ = [("dep", C.c_void_p), ("ledger", C.c_void_p), ("ctrl", C.c_void_p),
                ("n_nuc", C.c_int32), ("dep_copies", C.c_int32), ("dep_grid", Grid)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_0912_3223_amd/build.py` (no CPU fallback exists)")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    sig = {
        "lpm_accum_reset": [P(Accum), C.c_void_p],
        "lpm_release_particles": [P(State), P(Source), P(Schedule), P(Physics), C.c_int32,
                                  C.c_int32, P(Accum), C.c_void_p],
        "lpm_step_particles": [P(State), P(Source), P(Schedule), P(Field), P(Physics),
                               C.c_int32, C.c_int32, P(Accum), C.c_void_p],
        "lpm_step_particles_record": [P(State), P(Source), P(Schedule), P(Field), P(Physics),
                                      C.c_int32, C.c_int32, P(Accum), C.c_int32, C.c_int32,
                                      C.c_int32, C.c_void_p, C.c_int64, C.c_void_p],
        "lpm_grid_concentration": [P(State), P(Source), P(Schedule), P(Physics), P(Grid),
                                   C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p],
        "lpm_grid_concentration_static": [P(State), P(Source), P(Schedule), P(Physics),
                                          P(Grid), C.c_int32, C.c_void_p, C.c_void_p],
        "lpm_grid_records_workspace": [P(Schedule), P(Physics), P(Grid), C.c_int32, C.c_int32,
                                       C.c_int32, P(C.c_int64)],
        "lpm_grid_records": [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_int32, P(Source),
                             P(Schedule), P(Physics), P(Grid), C.c_void_p, C.c_int64, C.c_void_p,
                             C.c_void_p],
        "lpm_grid_records_ordered": [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                     P(Source), P(Schedule), P(Physics), P(Grid), C.c_void_p,
                                     C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p],
        "lpm_grid_deposition": [P(Accum), C.c_void_p, C.c_void_p],
        "lpm_read_ledger": [P(Accum), P(C.c_double), C.c_void_p],
        "lpm_check": [P(Accum), C.c_void_p],
        "lpm_set_launch": [C.c_int32, C.c_int32],
        "lpm_set_launch_ex": [C.c_int32, C.c_int32, C.c_int32],
        "lpm_ensemble_prepare": [P(Scenario), C.c_int32, P(State), P(Physics), C.c_int32,
                                 C.c_int32, C.c_void_p, C.c_int64, P(Ensemble), C.c_void_p],
        "lpm_release_ensemble": [P(State), P(Ensemble), C.c_void_p, C.c_void_p],
        "lpm_step_ensemble": [P(State), P(Ensemble), P(Field), P(Physics), P(Grid), C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_void_p],
        "lpm_autotune_ensemble": [P(State), P(Ensemble), P(Scenario), P(Field), P(Physics),
                                  P(Grid), C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                  C.c_int32, P(Tuning), C.c_void_p],
        "lpm_receptor_concentration": [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                       P(Source), P(Schedule), P(Physics), P(Receptors),
                                       C.c_void_p, C.c_void_p],
        "lpm_adjoint_workspace": [P(Field), P(Schedule), C.c_int32, P(C.c_int64)],
        "lpm_field_interval_bytes": [P(Field), P(C.c_int64)],
        "lpm_order_workspace": [P(Schedule), P(Field), P(C.c_int64)],
        "lpm_order_particles": [P(State), P(Schedule), P(Field), C.c_int32, C.c_int32,
                                C.c_void_p, C.c_int64, P(C.c_int64), C.c_void_p, C.c_int64,
                                C.c_void_p],
        "lpm_field_interval": [P(Field), C.c_int32, C.c_void_p, P(Field), C.c_void_p],
        "lpm_surface_layer": [C.c_double] * 5 + [P(C.c_double), P(C.c_double)],
        "lpm_receptor_adjoint": [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, P(Source),
                                 P(Schedule), P(Field), P(Physics), P(Receptors), C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.lpm_last_error.restype = C.c_char_p
    L.lpm_version.restype = C.c_char_p
    return L


_lib = _load()

#: C entry points exported by include/lpm.h (checked by the test suite).
EXPORTS = ("lpm_accum_reset", "lpm_release_particles", "lpm_step_particles",
           "lpm_step_particles_record",
           "lpm_grid_concentration", "lpm_grid_concentration_static",
           "lpm_grid_records_workspace", "lpm_grid_records", "lpm_grid_records_ordered",
           "lpm_grid_deposition",
           "lpm_read_ledger", "lpm_check", "lpm_set_launch", "lpm_set_launch_ex", "lpm_ensemble_prepare",
           "lpm_release_ensemble", "lpm_step_ensemble", "lpm_autotune_ensemble",
           "lpm_receptor_concentration", "lpm_adjoint_workspace", "lpm_receptor_adjoint",
           "lpm_surface_layer", "lpm_field_interval_bytes", "lpm_field_interval",
           "lpm_order_workspace", "lpm_order_particles",
           "lpm_last_error", "lpm_version")


def lib():
    return _lib


def _rc(code):
    if code != LPM_OK:
        raise LpmError(code, _lib.lpm_last_error().decode())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


# -- entry points (same names as the C ABI) ---------------------------------

def accum_reset(acc: Accum, stream=None):
    _rc(_lib.lpm_accum_reset(C.byref(acc), _stream(stream)))


def release_particles(st: State, src: Source, sch: Schedule, ph: Physics, step0: int,
                      n_steps: int, acc: Accum, stream=None):
    _rc(_lib.lpm_release_particles(C.byref(st), C.byref(src), C.byref(sch), C.byref(ph),
                                   step0, n_steps, C.byref(acc), _stream(stream)))


def step_particles(st: State, src: Source, sch: Schedule, fld: Field, ph: Physics, step0: int,
                   n_steps: int, acc: Accum, stream=None):
    _rc(_lib.lpm_step_particles(C.byref(st), C.byref(src), C.byref(sch), C.byref(fld),
                                C.byref(ph), step0, n_steps, C.byref(acc), _stream(stream)))


def step_particles_record(st: State, src: Source, sch: Schedule, fld: Field, ph: Physics,
                          step0: int, n_steps: int, acc: Accum, rec_step0: int, rec_every: int,
                          n_rec: int, rec: torch.Tensor, rec_stride: int, stream=None):
    assert rec.dtype == torch.float32 and rec.is_contiguous()
    assert rec.numel() >= (4 * n_rec + 1) * rec_stride
    _rc(_lib.lpm_step_particles_record(C.byref(st), C.byref(src), C.byref(sch), C.byref(fld),
                                       C.byref(ph), step0, n_steps, C.byref(acc), rec_step0,
                                       rec_every, n_rec, C.c_void_p(rec.data_ptr()), rec_stride,
                                       _stream(stream)))


def grid_concentration(st: State, src: Source, sch: Schedule, ph: Physics, grid: Grid,
                       step: int, acc_scratch: torch.Tensor, out: torch.Tensor, stream=None):
    assert acc_scratch.dtype == torch.float64 and out.dtype == torch.float32
    _rc(_lib.lpm_grid_concentration(C.byref(st), C.byref(src), C.byref(sch), C.byref(ph),
                                    C.byref(grid), step, C.c_void_p(acc_scratch.data_ptr()),
                                    C.c_void_p(out.data_ptr()), _stream(stream)))


def grid_concentration_static(st: State, src: Source, sch: Schedule, ph: Physics, grid: Grid,
                              step: int, out: torch.Tensor, stream=None):
    """grid_concentration on the library's static device scratch (no
    allocation; calls on one device must not overlap)."""
    assert out.dtype == torch.float32
    _rc(_lib.lpm_grid_concentration_static(C.byref(st), C.byref(src), C.byref(sch), C.byref(ph),
                                           C.byref(grid), step, C.c_void_p(out.data_ptr()),
                                           _stream(stream)))


FIELD_NODES, FIELD_TIME_PAIRS = 0, 1


def order_workspace(sch: Schedule, fld: Field) -> int:
    n = C.c_int64(0)
    _rc(_lib.lpm_order_workspace(C.byref(sch), C.byref(fld), C.byref(n)))
    return n.value


def order_particles(st: State, sch: Schedule, fld: Field, step0: int, n_steps: int,
                    order: torch.Tensor, work: torch.Tensor, stream=None) -> int:
    """Work order of the step launch over [step0, step0 + n_steps) into
    ``order`` (int32); returns its length."""
    assert order.dtype == torch.int32 and order.is_contiguous()
    n = C.c_int64(0)
    _rc(_lib.lpm_order_particles(C.byref(st), C.byref(sch), C.byref(fld), step0, n_steps,
                                 C.c_void_p(order.data_ptr()), order.numel(), C.byref(n),
                                 C.c_void_p(work.data_ptr()), work.numel() * work.element_size(),
                                 _stream(stream)))
    return n.value


def field_interval_bytes(fld: Field) -> int:
    n = C.c_int64(0)
    _rc(_lib.lpm_field_interval_bytes(C.byref(fld), C.byref(n)))
    return n.value


def field_interval(fld: Field, k: int, out: torch.Tensor, stream=None) -> Field:
    """Time-pair copy of field interval k into ``out``; returns its
    descriptor (which refers to ``out``: keep it alive)."""
    assert out.is_contiguous() and out.numel() * out.element_size() >= field_interval_bytes(fld)
    packed = Field()
    _rc(_lib.lpm_field_interval(C.byref(fld), k, C.c_void_p(out.data_ptr()), C.byref(packed),
                                _stream(stream)))
    return packed


def grid_records_workspace(sch: Schedule, ph: Physics, grid: Grid, rec_step0: int,
                           rec_every: int, n_rec: int) -> int:
    n = C.c_int64(0)
    _rc(_lib.lpm_grid_records_workspace(C.byref(sch), C.byref(ph), C.byref(grid), rec_step0,
                                        rec_every, n_rec, C.byref(n)))
    return n.value


def grid_records(rec: torch.Tensor, rec_stride: int, rec_step0: int, rec_every: int, n_rec: int,
                 src: Source, sch: Schedule, ph: Physics, grid: Grid, work: torch.Tensor,
                 out: torch.Tensor, stream=None, order: Optional[torch.Tensor] = None):
    """lpm_grid_records; with ``order`` (the launch's int32 work order, the
    records stored by queue position) lpm_grid_records_ordered."""
    assert rec.dtype == torch.float32 and out.dtype == torch.float32
    nbytes = work.numel() * work.element_size()
    if order is None:
        _rc(_lib.lpm_grid_records(C.c_void_p(rec.data_ptr()), rec_stride, rec_step0, rec_every,
                                  n_rec, C.byref(src), C.byref(sch), C.byref(ph), C.byref(grid),
                                  C.c_void_p(work.data_ptr()), nbytes, C.c_void_p(out.data_ptr()),
                                  _stream(stream)))
        return
    assert order.dtype == torch.int32
    _rc(_lib.lpm_grid_records_ordered(C.c_void_p(rec.data_ptr()), rec_stride, rec_step0,
                                      rec_every, n_rec, C.byref(src), C.byref(sch), C.byref(ph),
                                      C.byref(grid), C.c_void_p(order.data_ptr()), order.numel(),
                                      C.c_void_p(work.data_ptr()), nbytes,
                                      C.c_void_p(out.data_ptr()), _stream(stream)))


def grid_deposition(acc: Accum, out: torch.Tensor, stream=None):
    assert out.dtype == torch.float32
    _rc(_lib.lpm_grid_deposition(C.byref(acc), C.c_void_p(out.data_ptr()), _stream(stream)))


def read_ledger(acc: Accum, stream=None):
    """Synchronises; returns ([n_nuc][4] released, deposited, decayed,
    exited, particle-steps advanced)."""
    out = (C.c_double * (4 * acc.n_nuc + 1))()
    _rc(_lib.lpm_read_ledger(C.byref(acc), out, _stream(stream)))
    return ([[out[n * 4 + e] for e in range(4)] for n in range(acc.n_nuc)],
            int(out[4 * acc.n_nuc]))


def check(acc: Accum, stream=None):
    _rc(_lib.lpm_check(C.byref(acc), _stream(stream)))


def ensemble_prepare(scen, n_scen: int, st: State, ph: Physics, step0: int, n_steps: int,
                     table: torch.Tensor, stream=None) -> Ensemble:
    ens = Ensemble()
    _rc(_lib.lpm_ensemble_prepare(scen, n_scen, C.byref(st), C.byref(ph), step0, n_steps,
                                  C.c_void_p(table.data_ptr()),
                                  table.numel() * table.element_size(), C.byref(ens),
                                  _stream(stream)))
    return ens


def release_ensemble(st: State, ens: Ensemble, ledgers: torch.Tensor, stream=None):
    _rc(_lib.lpm_release_ensemble(C.byref(st), C.byref(ens), C.c_void_p(ledgers.data_ptr()),
                                  _stream(stream)))


def step_ensemble(st: State, ens: Ensemble, fld: Field, ph: Physics, dep_grid: Grid,
                  dep: torch.Tensor, ledgers: torch.Tensor, ctrl: torch.Tensor, stream=None):
    _rc(_lib.lpm_step_ensemble(C.byref(st), C.byref(ens), C.byref(fld), C.byref(ph),
                               C.byref(dep_grid), C.c_void_p(dep.data_ptr()),
                               C.c_void_p(ledgers.data_ptr()), C.c_void_p(ctrl.data_ptr()),
                               _stream(stream)))


def autotune_ensemble(st: State, ens: Ensemble, scen, fld: Field, ph: Physics, dep_grid: Grid,
                      dep: torch.Tensor, ledgers: torch.Tensor, ctrl: torch.Tensor,
                      trial_steps: int, reps: int = 3, stream=None) -> Tuning:
    """Times the candidate launch settings and stores the pick in
    ``ens.launch`` (the Ensemble passed in is updated)."""
    t = Tuning()
    _rc(_lib.lpm_autotune_ensemble(C.byref(st), C.byref(ens), scen, C.byref(fld), C.byref(ph),
                                   C.byref(dep_grid), C.c_void_p(dep.data_ptr()),
                                   C.c_void_p(ledgers.data_ptr()), C.c_void_p(ctrl.data_ptr()),
                                   trial_steps, reps, C.byref(t), _stream(stream)))
    return t


def receptor_concentration(rec: torch.Tensor, rec_stride: int, rec_step0: int, rec_every: int,
                           n_rec: int, src: Source, sch: Schedule, ph: Physics, rcp: Receptors,
                           c_out: torch.Tensor, stream=None):
    assert rec.dtype == torch.float32 and c_out.dtype == torch.float64
    assert c_out.numel() >= rcp.n
    _rc(_lib.lpm_receptor_concentration(C.c_void_p(rec.data_ptr()), rec_stride, rec_step0,
                                        rec_every, n_rec, C.byref(src), C.byref(sch),
                                        C.byref(ph), C.byref(rcp), C.c_void_p(c_out.data_ptr()),
                                        _stream(stream)))


def adjoint_workspace(fld: Field, sch: Schedule, rec_every: int) -> int:
    n = C.c_int64(0)
    _rc(_lib.lpm_adjoint_workspace(C.byref(fld), C.byref(sch), rec_every, C.byref(n)))
    return n.value


def receptor_adjoint(rec: torch.Tensor, rec_stride: int, rec_every: int, n_rec: int, src: Source,
                     sch: Schedule, fld: Field, ph: Physics, rcp: Receptors, gbar: torch.Tensor,
                     grad_out: torch.Tensor, work: torch.Tensor, stream=None):
    assert gbar.dtype == torch.float64 and grad_out.dtype == torch.float64
    assert gbar.numel() >= rcp.n and grad_out.numel() >= 5
    _rc(_lib.lpm_receptor_adjoint(C.c_void_p(rec.data_ptr()), rec_stride, rec_every, n_rec,
                                  C.byref(src), C.byref(sch), C.byref(fld), C.byref(ph),
                                  C.byref(rcp), C.c_void_p(gbar.data_ptr()),
                                  C.c_void_p(grad_out.data_ptr()), C.c_void_p(work.data_ptr()),
                                  work.numel() * work.element_size(), _stream(stream)))


def surface_layer(U: float, z_ref: float, z0: float, dtheta: float, T0: float):
    """(u*, 1/L) of the surface layer (lpm_surface_layer)."""
    us, il = C.c_double(), C.c_double()
    _rc(_lib.lpm_surface_layer(U, z_ref, z0, dtheta, T0, C.byref(us), C.byref(il)))
    return us.value, il.value


def set_launch(refill_every: int = 24, blocks_per_cu: int = 0, refill_min: int = 0):
    """Plain step launch settings (refill_min 0: the library's default for
    the wind of each launch)."""
    _rc(_lib.lpm_set_launch_ex(refill_every, blocks_per_cu, refill_min))


def version() -> str:
    return _lib.lpm_version().decode()


from .host import (DeviceRun, EnsembleRun, ReceptorRun, ReceptorConcentration,  # noqa: E402
                   make_source, make_schedule, make_physics, make_grid)

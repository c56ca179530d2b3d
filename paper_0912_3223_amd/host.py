"""Host side of a run: device buffers (torch allocations), the C structs that
describe them, and the paper's host main loop (Sec. 3.2, Fig. 1): release and
step the particles window by window, and grid the activity every n-th step.
All arithmetic of the model happens in liblpm's kernels."""
from __future__ import annotations

import ctypes

from fractions import Fraction
from typing import Callable, Iterable, Optional

import numpy as np
import torch

from . import (Accum, Field, Grid, Physics, Receptors, Schedule, Scenario, Source, State,
               CTRL_WORDS, LEDGER_SLOTS, LEDGER_STRIDE, SCENARIO_BYTES, accum_reset,
               adjoint_workspace, autotune_ensemble, ensemble_prepare, grid_concentration,
               grid_deposition, grid_records, grid_records_workspace, read_ledger, receptor_adjoint,
               receptor_concentration, release_ensemble, release_particles, step_ensemble,
               step_particles, step_particles_record, check, field_interval,
               field_interval_bytes, order_particles, order_workspace)


def make_source(src) -> Source:
    return Source(src.xs, src.ys, src.h, src.q, src.wind_scale, src.v_d, src.scenario, 0)


def make_schedule(sch) -> Schedule:
    return Schedule(sch.n_total, sch.local_count, sch.id_base, sch.id_stride, sch.s_release, 0)


def make_physics(ph) -> Physics:
    lam = (ctypes.c_double * 4)(*(list(ph.lambdas) + [0.0] * (4 - ph.n_nuc)))
    r = ph.rain
    return Physics(ph.dt, ph.Kh, ph.Kz_const, ph.kappa_ustar, ph.z0, ph.H_mix, ph.H_lid, ph.h_s,
                   ph.kz_kind, ph.n_nuc, lam, ph.Lambda0, r.cx, r.cy, r.a, r.b, r.angle,
                   r.edge, ph.seed, ph.inv_L, ph.chain, ph.dep_mode)


def make_grid(g) -> Grid:
    return Grid(g.nx, g.ny, g.nz, g.mode, int(g.density), 0, g.x0, g.y0, g.z0, g.dx, g.dy, g.dz)


#: copies of the deposition grid a DeviceRun keeps (lpm_accum.dep_copies)
DEP_COPIES = 16


class DeviceRun:
    """Device buffers and structs for one workload (a ``synth.Case``)."""

    def __init__(self, case, device: str = "cuda", capacity: Optional[int] = None,
                 dep_copies: int = DEP_COPIES):
        self.case = case
        self.device = torch.device(device)
        sch, ph, fld = case.schedule, case.physics, case.field
        n = sch.local_count
        cap = n if capacity is None else capacity
        f32 = dict(dtype=torch.float32, device=self.device)
        f64 = dict(dtype=torch.float64, device=self.device)
        self.x = torch.zeros(max(cap, 1), **f32)
        self.y = torch.zeros(max(cap, 1), **f32)
        self.z = torch.zeros(max(cap, 1), **f32)
        self.m = torch.zeros(max(cap, 1), **f32)
        self.xl = torch.zeros(max(cap, 1), **f32)  # rounding residuals of x, y
        self.yl = torch.zeros(max(cap, 1), **f32)
        self.st = State(self.x.data_ptr(), self.y.data_ptr(), self.z.data_ptr(),
                        self.m.data_ptr(), cap, self.xl.data_ptr(), self.yl.data_ptr())
        self.field_data = torch.from_numpy(np.ascontiguousarray(fld.data)).to(self.device)
        self.levels = None
        if fld.z_levels is not None:
            self.levels = torch.from_numpy(np.ascontiguousarray(fld.z_levels)).to(self.device)
        self.fld = Field(self.field_data.data_ptr(),
                         self.levels.data_ptr() if self.levels is not None else None,
                         fld.nx, fld.ny, fld.nz, fld.nt, fld.ncomp, int(fld.bounded),
                         fld.x0, fld.y0, fld.dx, fld.dy, fld.dz, fld.t0, fld.dt_field)
        self.src = make_source(case.source)
        self.sch = make_schedule(sch)
        self.ph = make_physics(ph)
        dg, cg = case.dep_grid, case.conc_grid
        nn = ph.n_nuc
        # copies of the deposition grid: the step kernels spread their
        # flushes over them (fewer waves meet on one address under rain)
        self._dep = torch.zeros((max(dep_copies, 1), nn, dg.ny, dg.nx), **f64)
        self.ledger_buf = torch.zeros((LEDGER_SLOTS, LEDGER_STRIDE, 4, 4), **f64)
        self.ctrl = torch.zeros(CTRL_WORDS, dtype=torch.int32, device=self.device)
        self.acc = Accum(self._dep.data_ptr(), self.ledger_buf.data_ptr(), self.ctrl.data_ptr(),
                         nn, dep_copies, make_grid(dg))
        self.cgrid = make_grid(cg)
        self.conc_scratch = torch.empty((nn, cg.nz, cg.ny, cg.nx), **f64)
        self.conc = torch.empty((nn, cg.nz, cg.ny, cg.nx), **f32)
        self.dep_out = torch.empty((nn, dg.ny, dg.nx), **f32)
        self.reset()

    # -- thin wrappers ------------------------------------------------------
    def reset(self):
        self.m.zero_()
        accum_reset(self.acc)

    def set_state(self, x, y, z, m, xl=None, yl=None):
        """Load a state; xl, yl are the rounding residuals of x, y that
        state() returns (zero if not given)."""
        for dst, src in ((self.x, x), (self.y, y), (self.z, z), (self.m, m)):
            dst[: len(src)].copy_(torch.as_tensor(np.asarray(src, dtype=np.float32)))
        for dst, src in ((self.xl, xl), (self.yl, yl)):
            dst.zero_()
            if src is not None:
                dst[: len(src)].copy_(torch.as_tensor(np.asarray(src, dtype=np.float32)))

    def release(self, step0: int, n_steps: int = 1):
        release_particles(self.st, self.src, self.sch, self.ph, step0, n_steps, self.acc)

    def step(self, step0: int, n_steps: int = 1):
        step_particles(self.st, self.src, self.sch, self.fld, self.ph, step0, n_steps, self.acc)

    def grid_concentration(self, step: int) -> torch.Tensor:
        grid_concentration(self.st, self.src, self.sch, self.ph, self.cgrid, step,
                           self.conc_scratch, self.conc)
        return self.conc

    def grid_deposition(self) -> torch.Tensor:
        grid_deposition(self.acc, self.dep_out)
        return self.dep_out

    @property
    def dep(self) -> torch.Tensor:
        """The FP64 deposition grid [n_nuc][ny][nx]: its copies added up
        (for inspection; lpm_grid_deposition gives it as float)."""
        return self._dep.sum(0)

    def ledger(self) -> np.ndarray:
        """[n_nuc][4]: released, deposited, decayed, exited (synchronises)."""
        return np.array(read_ledger(self.acc)[0])

    def particle_steps(self) -> int:
        """Particle-steps advanced since the last reset (synchronises)."""
        return read_ledger(self.acc)[1]

    def check(self):
        check(self.acc)

    def state(self):
        """x, y, z, m of the local particles (float64 copies) and the
        residuals xl, yl of the compensated x, y."""
        n = self.sch.n_local
        out = {k: getattr(self, k)[:n].double().cpu().numpy() for k in "xyzm"}
        out["xl"] = self.xl[:n].double().cpu().numpy()
        out["yl"] = self.yl[:n].double().cpu().numpy()
        return out

    def step_record(self, step0: int, n_steps: int, rec_step0: int, rec_every: int,
                    n_rec: int, rec: torch.Tensor, fld: Optional[Field] = None,
                    st: Optional[State] = None):
        step_particles_record(self.st if st is None else st, self.src, self.sch,
                              self.fld if fld is None else fld, self.ph, step0, n_steps,
                              self.acc, rec_step0, rec_every, n_rec, rec, self.rec_stride)

    def work_order(self, step0: int, n_steps: int) -> State:
        """The state descriptor for the step launch over [step0, step0 +
        n_steps) with its particles in wind-node order
        (lpm_order_particles), in buffers kept between calls."""
        if getattr(self, "_order", None) is None:
            self._order = torch.empty(max(self.sch.n_local, 1), dtype=torch.int32,
                                      device=self.device)
            self._order_work = torch.empty(order_workspace(self.sch, self.fld),
                                           dtype=torch.uint8, device=self.device)
        n = order_particles(self.st, self.sch, self.fld, step0, n_steps, self._order,
                            self._order_work)
        st = State.from_buffer_copy(self.st)
        st.order, st.n_order = self._order.data_ptr(), n
        return st

    def time_node(self, s: int) -> int:
        """Lower time node of the wind for step s, taken as the library
        takes it (FP64 s * (dt / dt_field) - t0 / dt_field, fused, clamped
        to the field's nodes)."""
        f, dt = self.fld, float(self.case.physics.dt)
        if f.nt < 2:
            return 0
        ft_step = dt * (1.0 / f.dt_field)
        ft = float(Fraction(s) * Fraction(ft_step) + Fraction(-f.t0 / f.dt_field))
        ft = min(max(ft, 0.0), float(f.nt - 1))
        return min(int(ft), f.nt - 2)

    def interval_field(self, k: int) -> Field:
        """Time-pair copy of wind interval k (lpm_field_interval), in a
        buffer kept between calls."""
        if getattr(self, "_interval_k", None) != k:
            if getattr(self, "_interval_buf", None) is None:
                self._interval_buf = torch.empty(field_interval_bytes(self.fld) // 4,
                                                 dtype=torch.float32, device=self.device)
            self._interval_fld = field_interval(self.fld, k, self._interval_buf)
            self._interval_k = k
        return self._interval_fld

    @property
    def rec_stride(self) -> int:
        return max(self.sch.n_local, 1)

    def record_buffer(self, n_rec: int) -> torch.Tensor:
        """Records of n_rec output steps: float4 per particle and step, then
        one int32 per particle (see lpm_step_particles_record)."""
        return torch.empty((4 * n_rec + 1) * self.rec_stride, dtype=torch.float32,
                           device=self.device)

    def grid_buffers(self, rec_step0: int, every: int, n_rec: int):
        """Workspace and output of grid_records for these output steps."""
        cg, nn = self.case.conc_grid, self.case.physics.n_nuc
        nbytes = grid_records_workspace(self.sch, self.ph, self.cgrid, rec_step0, every, n_rec)
        return (torch.empty(max(nbytes, 1), dtype=torch.uint8, device=self.device),
                torch.empty((n_rec, nn, cg.nz, cg.ny, cg.nx), dtype=torch.float32,
                            device=self.device))

    def grid_records(self, rec: torch.Tensor, rec_step0: int, every: int, n_rec: int,
                     bufs=None):
        work, out = bufs if bufs is not None else self.grid_buffers(rec_step0, every, n_rec)
        grid_records(rec, self.rec_stride, rec_step0, every, n_rec, self.src, self.sch, self.ph,
                     self.cgrid, work, out)
        return out

    def run_recorded(self, every: int, window: Optional[int] = None,
                     out: Optional[torch.Tensor] = None, on_window: Optional[Callable] = None,
                     step_events: Optional[list] = None, time_pairs: bool = True,
                     order: bool = True):
        """The whole run as the benchmark runs it: release, step and grid in
        windows of ``window`` steps (a multiple of ``every``; the whole run by
        default).  Each window is one step launch that records the state
        after each of its output steps (every ``every``-th step), gridded right
        after into ``out[k]`` for output step k.  Windows inside one field
        interval keep every particle of a launch on the same pair of hourly
        wind fields.  ``on_window(w0, rec, n_rec, order)`` sees each window's record buffer
        before it is reused, with the window's work order (int32, queue position to
        particle; None without ``order``): with a work order the records are stored by
        queue position (lpm_step_particles_record); ``step_events`` (a list) receives a pair of timing events
        around each step launch, recorded on the current stream.  With
        ``time_pairs`` a window whose steps all interpolate in one interval
        of a time-dependent wind steps on the time-pair copy of that interval
        (same results, fewer cache lines per wind stencil); with ``order``
        each step launch takes its particles in wind-node order (same
        results; the lanes of a wave share stencils).  Returns ``out``
        ([n_out][n_nuc][nz][ny][nx], float)."""
        S = self.case.n_steps
        window = S if window is None else window
        if window % every or S % window:
            raise ValueError("the window must be a multiple of the output interval and divide the run")
        n_rec = window // every
        cg, nn = self.case.conc_grid, self.case.physics.n_nuc
        if out is None:
            out = torch.empty((S // every, nn, cg.nz, cg.ny, cg.nx), dtype=torch.float32,
                              device=self.device)
        rec = self._rec_buf(n_rec)
        work = self._grid_work(S - window + every - 1, every, n_rec)
        for w0 in range(0, S, window):
            self.release(w0, window)
            fld = None
            if time_pairs and self.fld.nt > 1:
                k = self.time_node(w0)
                if self.time_node(w0 + window - 1) == k:
                    fld = self.interval_field(k)
            st = self.work_order(w0, window) if order else None
            worder = self._order[:st.n_order] if st is not None else None
            if step_events is not None:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(torch.cuda.current_stream())
            self.step_record(w0, window, w0 + every - 1, every, n_rec, rec, fld, st)
            if step_events is not None:
                e1.record(torch.cuda.current_stream())
                step_events.append((e0, e1))
            k0 = w0 // every
            grid_records(rec, self.rec_stride, w0 + every - 1, every, n_rec, self.src, self.sch,
                         self.ph, self.cgrid, work, out[k0:k0 + n_rec], order=worder)
            if on_window is not None:
                on_window(w0, rec, n_rec, worder)
        return out

    def _rec_buf(self, n_rec: int) -> torch.Tensor:
        buf = getattr(self, "_rec_cache", None)
        if buf is None or buf.numel() < (4 * n_rec + 1) * self.rec_stride:
            self._rec_cache = buf = self.record_buffer(n_rec)
        return buf

    def _grid_work(self, rec_step0: int, every: int, n_rec: int) -> torch.Tensor:
        nbytes = max(grid_records_workspace(self.sch, self.ph, self.cgrid, rec_step0, every,
                                            n_rec), 1)
        buf = getattr(self, "_work_cache", None)
        if buf is None or buf.numel() < nbytes:
            self._work_cache = buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return buf

    # -- the host main loop -------------------------------------------------
    def windows(self, s_begin: int, s_end: int, steps_per_launch: int,
                snap_steps: Iterable[int] = ()):
        cuts = {s_end}
        cuts.update(s + 1 for s in snap_steps if s_begin <= s < s_end)
        bounds = sorted(cuts)
        out, a = [], s_begin
        for b in bounds:
            while a < b:
                e = min(b, a + steps_per_launch)
                out.append((a, e))
                a = e
        return out

    def run_whole(self, s_begin: int = 0, s_end: Optional[int] = None, every: int = 60,
                  on_snapshot: Optional[Callable] = None):
        """Whole window [s_begin, s_end) in one step launch: each particle is
        carried through every step; the states after the output steps
        s_begin + every - 1, s_begin + 2 every - 1, ... are recorded and
        gridded afterwards, and the final step is gridded from the state
        (results equal the windowed run)."""
        s_end = self.case.n_steps if s_end is None else s_end
        regular = list(range(s_begin + every - 1, s_end, every))
        n_rec = len(regular)
        self.release(s_begin, s_end - s_begin)
        if n_rec:
            rec = self.record_buffer(n_rec)
            self.step_record(s_begin, s_end - s_begin, regular[0], every, n_rec, rec)
            grids = self.grid_records(rec, regular[0], every, n_rec)
            if on_snapshot is not None:
                for k, s in enumerate(regular):
                    on_snapshot(s, grids[k])
        else:
            self.step(s_begin, s_end - s_begin)
        if not regular or regular[-1] != s_end - 1:
            g = self.grid_concentration(s_end - 1)
            if on_snapshot is not None:
                on_snapshot(s_end - 1, g)

    def run(self, s_begin: int = 0, s_end: Optional[int] = None, steps_per_launch: int = 60,
            snap_steps: Iterable[int] = (), on_snapshot: Optional[Callable] = None,
            release: bool = True):
        """Release, step and grid over steps [s_begin, s_end).  After every
        step in ``snap_steps`` the concentration is gridded and passed to
        ``on_snapshot(step, tensor)`` (the tensor is reused)."""
        s_end = self.case.n_steps if s_end is None else s_end
        snaps = sorted(set(snap_steps))
        for a, b in self.windows(s_begin, s_end, steps_per_launch, snaps):
            if release:
                self.release(a, b - a)
            self.step(a, b - a)
            if (b - 1) in snaps:
                g = self.grid_concentration(b - 1)
                if on_snapshot is not None:
                    on_snapshot(b - 1, g)


def _field_struct(fld, device):
    data = torch.from_numpy(np.ascontiguousarray(fld.data)).to(device)
    lev = None
    if fld.z_levels is not None:
        lev = torch.from_numpy(np.ascontiguousarray(fld.z_levels)).to(device)
    st = Field(data.data_ptr(), lev.data_ptr() if lev is not None else None, fld.nx, fld.ny,
               fld.nz, fld.nt, fld.ncomp, int(fld.bounded), fld.x0, fld.y0, fld.dx, fld.dy,
               fld.dz, fld.t0, fld.dt_field)
    return st, data, lev


class EnsembleRun:
    """Device buffers for an ensemble of release scenarios sharing one wind
    field and physics (``base``, a ``synth.Case``): ``sources`` and
    ``counts`` give each scenario's source and particle count; every scenario
    releases over ``base.schedule.s_release`` steps."""

    def __init__(self, base, sources, counts, device: str = "cuda"):
        self.base = base
        self.device = torch.device(device)
        n_scen = len(sources)
        assert n_scen == len(counts) and n_scen >= 1
        self.counts = [int(c) for c in counts]
        self.offsets = np.concatenate([[0], np.cumsum(self.counts)[:-1]]).astype(np.int64)
        total = int(sum(self.counts))
        self.total = total
        f32 = dict(dtype=torch.float32, device=self.device)
        self.x = torch.zeros(total, **f32)
        self.y = torch.zeros(total, **f32)
        self.z = torch.zeros(total, **f32)
        self.m = torch.zeros(total, **f32)
        self.xl = torch.zeros(total, **f32)
        self.yl = torch.zeros(total, **f32)
        self.st = State(self.x.data_ptr(), self.y.data_ptr(), self.z.data_ptr(),
                        self.m.data_ptr(), total, self.xl.data_ptr(), self.yl.data_ptr())
        self.fld, self._fdata, self._flev = _field_struct(base.field, self.device)
        self.ph = make_physics(base.physics)
        self.scen = (Scenario * n_scen)()
        for c, (src, n) in enumerate(zip(sources, self.counts)):
            self.scen[c] = Scenario(make_source(src), n, base.schedule.s_release, 0,
                                    int(self.offsets[c]))
        self.n_scen = n_scen
        dg = base.dep_grid
        nn = base.physics.n_nuc
        self.dgrid = make_grid(dg)
        # copies of the scenarios' deposition grids, as for DeviceRun
        self._dep = torch.zeros((DEP_COPIES, n_scen, nn, dg.ny, dg.nx), dtype=torch.float64,
                                device=self.device)
        self.ledgers = torch.zeros((n_scen, LEDGER_SLOTS, LEDGER_STRIDE), dtype=torch.float64,
                                   device=self.device)
        self.ctrl = torch.zeros(CTRL_WORDS, dtype=torch.int32, device=self.device)
        self.table = torch.zeros(n_scen * SCENARIO_BYTES // 8, dtype=torch.float64,
                                 device=self.device)
        self.ens = None

    def prepare(self, step0: int = 0, n_steps: Optional[int] = None):
        n_steps = self.base.n_steps - step0 if n_steps is None else n_steps
        self.ens = ensemble_prepare(self.scen, self.n_scen, self.st, self.ph, step0, n_steps,
                                    self.table)
        self.ens.dep_copies = DEP_COPIES
        return self.ens

    @property
    def dep(self) -> torch.Tensor:
        """The FP64 deposition grids [n_scen][n_nuc][ny][nx]: their copies added up."""
        return self._dep.sum(0)

    def reset(self):
        self.m.zero_()
        self._dep.zero_()
        self.ledgers.zero_()
        self.ctrl.zero_()

    def release(self):
        release_ensemble(self.st, self.ens, self.ledgers)

    def step(self):
        step_ensemble(self.st, self.ens, self.fld, self.ph, self.dgrid, self._dep, self.ledgers,
                      self.ctrl)

    def autotune(self, trial_steps: int, reps: int = 3):
        """Pick the launch settings of this ensemble (kept in ``self.ens``)."""
        t = autotune_ensemble(self.st, self.ens, self.scen, self.fld, self.ph, self.dgrid,
                              self._dep, self.ledgers, self.ctrl, trial_steps, reps)
        self.reset()
        return t

    def set_launch(self, refill_every=24, refill_min=56, blocks_per_cu=0, block=256):
        """Launch settings of later ``step`` calls of this ensemble."""
        L = self.ens.launch
        L.refill_every, L.refill_min, L.blocks_per_cu, L.block = (refill_every, refill_min,
                                                                  blocks_per_cu, block)

    def run(self):
        self.reset()
        self.release()
        self.step()

    def ledger(self, c: int) -> np.ndarray:
        L = self.ledgers[c].sum(dim=0).cpu().numpy()
        nn = self.base.physics.n_nuc
        return np.array([[L[n * 4 + e] for e in range(4)] for n in range(nn)])

    def particle_steps(self) -> int:
        return int(self.ledgers[:, :, 16].sum().item())

    def state(self, c: int):
        a, n = int(self.offsets[c]), self.counts[c]
        return {k: getattr(self, k)[a:a + n].double().cpu().numpy() for k in "xyzm"}


class ReceptorRun:
    """Receptor concentrations of one release and their gradient with respect
    to theta = (h, q, s_w, v_d) (source height, release rate, wind scale,
    dry-deposition velocity), all on the device.

    forward: release, one whole-run step launch that records the state after
    every ``case.out_every``-th step (the output steps, which are also the
    checkpoints of the gradient), and the Gaussian-kernel receptor gridding.
    backward: the adjoint sweep, segment by segment from the checkpoints."""

    def __init__(self, case, receptors, device: str = "cuda"):
        if case.n_steps % case.out_every:
            raise ValueError("the run length must be a multiple of the output interval")
        self.case = case
        self.run = DeviceRun(case, device)
        self.every = case.out_every
        self.n_rec = case.n_steps // case.out_every
        self.rec = self.run.record_buffer(self.n_rec)
        dev = self.run.device
        self.rx = torch.tensor(receptors.x, dtype=torch.float32, device=dev)
        self.ry = torch.tensor(receptors.y, dtype=torch.float32, device=dev)
        self.rz = torch.tensor(receptors.z, dtype=torch.float32, device=dev)
        self.rcp = Receptors(self.rx.data_ptr(), self.ry.data_ptr(), self.rz.data_ptr(),
                             len(receptors.x), receptors.sigma_h, receptors.sigma_z,
                             receptors.weight)
        self.c = torch.zeros(len(receptors.x), dtype=torch.float64, device=dev)
        self.grad = torch.zeros(5, dtype=torch.float64, device=dev)
        nbytes = adjoint_workspace(self.run.fld, self.run.sch, self.every)
        self.work = torch.empty((nbytes + 15) // 16 * 4, dtype=torch.float32, device=dev)
        self.theta = (case.source.h, case.source.q, case.source.wind_scale, case.source.v_d)

    def set_theta(self, theta):
        h, q, sw, vd = (float(t) for t in theta)
        self.theta = (h, q, sw, vd)
        src = self.run.src
        src.h, src.q, src.wind_scale, src.v_d = h, q, sw, vd

    def forward(self, theta=None) -> torch.Tensor:
        """Receptor concentrations c [n] (float64, device; reused buffer)."""
        if theta is not None:
            self.set_theta(theta)
        r = self.run
        r.reset()
        r.release(0, self.case.n_steps)
        r.step_record(0, self.case.n_steps, self.every - 1, self.every, self.n_rec, self.rec)
        receptor_concentration(self.rec, r.rec_stride, self.every - 1, self.every, self.n_rec,
                               r.src, r.sch, r.ph, self.rcp, self.c)
        return self.c

    def backward(self, gbar: torch.Tensor) -> torch.Tensor:
        """grad [5] (float64, device; reused buffer): sum_r gbar_r dc_r/dtheta
        for theta = (h, q, s_w, v_d), then sum_r gbar_r c_r.  Uses the
        record of the last forward()."""
        g = gbar.to(device=self.run.device, dtype=torch.float64).contiguous()
        r = self.run
        receptor_adjoint(self.rec, r.rec_stride, self.every, self.n_rec, r.src, r.sch, r.fld,
                         r.ph, self.rcp, g, self.grad, self.work)
        return self.grad


class ReceptorConcentration(torch.autograd.Function):
    """c = ReceptorConcentration.apply(theta, run): receptor concentrations
    as a differentiable function of theta = (h, q, s_w, v_d) (a float64
    tensor of 4); the backward pass is liblpm's adjoint."""

    @staticmethod
    def forward(ctx, theta, run):
        run.forward(theta.detach().cpu().tolist())
        ctx.run = run
        ctx.theta_device = theta.device
        return run.c.clone()

    @staticmethod
    def backward(ctx, grad_c):
        g = ctx.run.backward(grad_c)
        return g[:4].to(ctx.theta_device).clone(), None

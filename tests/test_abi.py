"""The C ABI: the library loads, exports every entry point that include/lpm.h
declares, the binding's structs match the C layout, and invalid arguments are
rejected on the host before anything reaches a device (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lpm.h")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(lpm_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    import paper_0912_3223_amd as L
    names = declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(L.lib(), n), n
    assert set(names) == set(L.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}$", out, re.M), n


def test_struct_layout_matches_header(tmp_path):
    import paper_0912_3223_amd as L
    structs = {"lpm_state": L.State, "lpm_source": L.Source, "lpm_schedule": L.Schedule,
               "lpm_field": L.Field, "lpm_physics": L.Physics, "lpm_grid": L.Grid,
               "lpm_accum": L.Accum, "lpm_scenario": L.Scenario, "lpm_ensemble": L.Ensemble,
               "lpm_tuning": L.Tuning, "lpm_receptors": L.Receptors, "lpm_launch": L.Launch}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "lpm.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            cf = {"lam": "lambda"}.get(f, f)
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {cf}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


@pytest.fixture
def args():
    """Structurally valid arguments with fake (never dereferenced) device
    pointers; each test breaks one thing."""
    import paper_0912_3223_amd as L
    import synth
    case = synth.c1(n_total=1000, n_steps=10)
    fake = 0x10000
    st = L.State(fake, fake, fake, fake, 1000)
    src = L.make_source(case.source)
    sch = L.make_schedule(case.schedule)
    ph = L.make_physics(case.physics)
    fld = L.Field(fake, None, 200, 200, 30, 1, 2, 1, -25e3, -25e3, 250.0, 250.0, 40.0, 0.0, 3600.0)
    acc = L.Accum(fake, fake, fake, 2, 0, L.make_grid(case.dep_grid))
    grid = L.make_grid(case.conc_grid)
    return L, st, src, sch, ph, fld, acc, grid


def code(L, fn, *a):
    return getattr(L.lib(), fn)(*[C.byref(x) if isinstance(x, C.Structure) else x for x in a])


def test_rejects_bad_arguments(args):
    L, st, src, sch, ph, fld, acc, grid = args
    step = lambda *o: code(L, "lpm_step_particles", *o)
    ok = (st, src, sch, fld, ph, 0, 1, acc, None)
    # capacity
    small = L.State(st.x, st.y, st.z, st.m, 999)
    assert step(small, *ok[1:]) == L.LPM_ECAPACITY
    assert b"capacity" in L.lib().lpm_last_error()
    # null pointers
    assert L.lib().lpm_step_particles(None, C.byref(src), C.byref(sch), C.byref(fld), C.byref(ph),
                                      0, 1, C.byref(acc), None) == L.LPM_EINVAL
    nul = L.State(0, st.y, st.z, st.m, 1000)
    assert step(nul, *ok[1:]) == L.LPM_EINVAL
    # misaligned state
    mis = L.State(st.x + 2, st.y, st.z, st.m, 1000)
    assert step(mis, *ok[1:]) == L.LPM_EINVAL
    # rounding residuals: both or neither, aligned
    half = L.State(st.x, st.y, st.z, st.m, 1000, st.x, None)
    assert step(half, *ok[1:]) == L.LPM_EINVAL and b"both or neither" in L.lib().lpm_last_error()
    mis_lo = L.State(st.x, st.y, st.z, st.m, 1000, st.x + 2, st.y)
    assert step(mis_lo, *ok[1:]) == L.LPM_EINVAL
    # bad windows
    assert step(st, src, sch, fld, ph, -1, 1, acc, None) == L.LPM_EINVAL
    assert step(st, src, sch, fld, ph, 0, 0, acc, None) == L.LPM_EINVAL
    # record stride: at least n_local, below 2^32
    rec = lambda stride: code(L, "lpm_step_particles_record", st, src, sch, fld, ph, 0, 2, acc,
                              0, 1, 2, C.c_void_p(0x10000), C.c_int64(stride), None)
    assert rec(999) == L.LPM_EINVAL and b"rec_stride below" in L.lib().lpm_last_error()
    assert rec(1 << 32) == L.LPM_EINVAL and b"below 2^32" in L.lib().lpm_last_error()
    # n_nuc
    ph5 = L.Physics.from_buffer_copy(ph)
    ph5.n_nuc = 5
    assert step(st, src, sch, fld, ph5, 0, 1, acc, None) == L.LPM_EINVAL
    acc1 = L.Accum.from_buffer_copy(acc)
    acc1.n_nuc = 1
    assert step(st, src, sch, fld, ph, 0, 1, acc1, None) == L.LPM_EINVAL
    # field
    f3 = L.Field.from_buffer_copy(fld)
    f3.ncomp = 4
    assert step(st, src, sch, f3, ph, 0, 1, acc, None) == L.LPM_EINVAL
    f4 = L.Field.from_buffer_copy(fld)
    f4.dx = 0.0
    assert step(st, src, sch, f4, ph, 0, 1, acc, None) == L.LPM_EINVAL
    f5 = L.Field.from_buffer_copy(fld)
    f5.data = fld.data + 4
    assert step(st, src, sch, f5, ph, 0, 1, acc, None) == L.LPM_EINVAL  # 2-comp needs 8 B
    # schedule
    s2 = L.Schedule.from_buffer_copy(sch)
    s2.id_stride = 0
    assert step(st, src, s2, fld, ph, 0, 1, acc, None) == L.LPM_EINVAL
    s3 = L.Schedule.from_buffer_copy(sch)
    s3.n_total = 1 << 33
    assert step(st, src, s3, fld, ph, 0, 1, acc, None) == L.LPM_EINVAL
    s4 = L.Schedule.from_buffer_copy(sch)
    s4.id_base = 5
    assert step(st, src, s4, fld, ph, 0, 1, acc, None) == L.LPM_EINVAL  # ids beyond n_total
    # physics
    p2 = L.Physics.from_buffer_copy(ph)
    p2.dt = 0.0
    assert step(st, src, sch, fld, p2, 0, 1, acc, None) == L.LPM_EINVAL
    p3 = L.Physics.from_buffer_copy(ph)
    p3.kz_kind = 7
    assert step(st, src, sch, fld, p3, 0, 1, acc, None) == L.LPM_EINVAL
    p4 = L.Physics.from_buffer_copy(ph)
    p4.rain_a = 0.0
    assert step(st, src, sch, fld, p4, 0, 1, acc, None) == L.LPM_EINVAL
    # gridding
    g2 = L.Grid.from_buffer_copy(grid)
    g2.mode = 3
    assert code(L, "lpm_grid_concentration", st, src, sch, ph, g2, 0, C.c_void_p(0x10000),
                C.c_void_p(0x10000), None) == L.LPM_EINVAL
    assert code(L, "lpm_grid_concentration", st, src, sch, ph, grid, 0, None,
                C.c_void_p(0x10000), None) == L.LPM_EINVAL
    assert code(L, "lpm_grid_deposition", acc, None, None) == L.LPM_EINVAL
    many = L.Accum.from_buffer_copy(acc)
    many.dep_copies = 65  # above LPM_MAX_DEP_COPIES
    assert code(L, "lpm_grid_deposition", many, C.c_void_p(0x10000), None) == L.LPM_EINVAL
    assert b"dep_copies" in L.lib().lpm_last_error()
    many.dep_copies = -1
    assert step(st, src, sch, fld, ph, 0, 1, many, None) == L.LPM_EINVAL
    assert code(L, "lpm_release_particles", small, src, sch, ph, 0, 1, acc, None) == L.LPM_ECAPACITY
    assert L.lib().lpm_check(None, None) == L.LPM_EINVAL


def test_binding_raises(args):
    L, st, src, sch, ph, fld, acc, grid = args
    small = L.State(st.x, st.y, st.z, st.m, 10)
    with pytest.raises(L.LpmError) as e:
        L.step_particles(small, src, sch, fld, ph, 0, 1, acc, stream=0)
    assert e.value.code == L.LPM_ECAPACITY


def test_empty_window_launches_nothing(args):
    """A window in which no local particle has been born returns OK without
    touching the device."""
    L, st, src, sch, ph, fld, acc, grid = args
    empty = L.Schedule.from_buffer_copy(sch)
    empty.n_local = 0
    assert code(L, "lpm_step_particles", st, src, empty, fld, ph, 0, 1, acc, None) == L.LPM_OK
    assert code(L, "lpm_release_particles", st, src, empty, ph, 0, 1, acc, None) == L.LPM_OK


def test_receptor_entry_points_reject_bad_arguments(args):
    L, st, src, sch, ph, fld, acc, grid = args
    fake = C.c_void_p(0x10000)
    rcp = L.Receptors(0x10000, 0x10000, 0x10000, 50, 250.0, 40.0, 300.0)
    conc = lambda r, *o: code(L, "lpm_receptor_concentration", fake, 1000, 59, 60, 72, src, sch,
                              ph, r, *o)
    bad_n = L.Receptors.from_buffer_copy(rcp)
    bad_n.n = L.LPM_MAX_RECEPTORS + 1 if hasattr(L, "LPM_MAX_RECEPTORS") else 1025
    assert conc(bad_n, fake, None) == L.LPM_EINVAL
    bad_s = L.Receptors.from_buffer_copy(rcp)
    bad_s.sigma_h = 0.0
    assert conc(bad_s, fake, None) == L.LPM_EINVAL
    assert conc(rcp, C.c_void_p(0x10004), None) == L.LPM_EINVAL  # misaligned c_out
    assert b"c_out" in L.lib().lpm_last_error()
    # records shorter than the particles
    assert code(L, "lpm_receptor_concentration", fake, 999, 59, 60, 72, src, sch, ph, rcp, fake,
                None) == L.LPM_EINVAL
    adj = lambda work_bytes, s=src: code(L, "lpm_receptor_adjoint", fake, 1000, 60, 72, s, sch,
                                         fld, ph, rcp, fake, fake, fake, work_bytes, None)
    assert adj(16) == L.LPM_EINVAL and b"workspace" in L.lib().lpm_last_error()
    q0 = L.Source.from_buffer_copy(src)
    q0.q = 0.0
    assert adj(1 << 40, q0) == L.LPM_EINVAL
    n = C.c_int64(0)
    assert code(L, "lpm_adjoint_workspace", fld, sch, 0, C.byref(n)) == L.LPM_EINVAL


def test_record_gridding_workspace_and_rejections(args):
    """lpm_grid_records_workspace: sizes from the tile plan and the births;
    too-tall grids and bad buffers are rejected on the host."""
    L, st, src, sch, ph, fld, acc, grid = args
    n = C.c_int64(-1)
    q = lambda g, s0, every, n_rec: code(L, "lpm_grid_records_workspace", sch, ph, g, s0, every,
                                         n_rec, C.byref(n))
    assert q(grid, 0, 1, 0) == L.LPM_OK and n.value == 0
    # 200 x 200 x 30, 2 nuclides: 16 x 4 column tiles, bins (200/16+1)(200/4+1)4 per record
    # step, two 64-bit words each; a 1000-particle run over 10 steps is fully born by
    # step 9, so records at steps 4 and 9 hold at most 500 + 1000 particles (16 B of
    # record and 4 B of birth step each, in two arrays)
    assert q(grid, 4, 5, 2) == L.LPM_OK
    nb = 2 * 13 * 51 * 4
    a256 = lambda b: (b + 255) // 256 * 256
    # (plus one int per chunk of 2048 particle ids: 1 chunk)
    assert n.value == (2 * a256(8 * nb) + a256(8 * ((nb + 2047) // 2048)) + a256(4 * 1)
                       + a256(16 * 1500) + a256(4 * 1500))
    # one int per chunk of 2048 recorded positions, counted over every local
    # particle (a work-ordered launch records by queue position), however
    # few are born by the recorded steps: 200000 particles, 98 chunks (of
    # which the 20000 born by step 0 of the 10-step release fill 10)
    big = L.Schedule.from_buffer_copy(sch)
    big.n_total = big.n_local = 200_000
    n2 = C.c_int64(-1)
    assert code(L, "lpm_grid_records_workspace", big, ph, grid, 0, 1, 1, C.byref(n2)) == L.LPM_OK
    nb1, born = nb // 2, 20_000  # one record step
    assert n2.value == (2 * a256(8 * nb1) + a256(8 * ((nb1 + 2047) // 2048)) + a256(4 * 98)
                        + a256(16 * born) + a256(4 * born))
    tall = L.Grid.from_buffer_copy(grid)
    tall.nz = 3073  # 2 nuclides x 3073 levels x 8 B: one column exceeds the block's LDS
    assert q(tall, 0, 1, 1) == L.LPM_EINVAL
    tall.nz = 3072
    assert q(tall, 0, 1, 1) == L.LPM_OK
    assert q(grid, 0, 0, 1) == L.LPM_EINVAL
    assert q(grid, 0, 1, 65536) == L.LPM_EINVAL
    fake = C.c_void_p(0x10000)
    rec = C.c_void_p(0x10000)
    call = lambda work, nbytes, out: code(L, "lpm_grid_records", rec, 1000, 4, 5, 2, src, sch, ph,
                                          grid, work, nbytes, out, None)
    assert q(grid, 4, 5, 2) == L.LPM_OK
    assert call(fake, n.value - 1, fake) == L.LPM_EINVAL          # workspace too small
    assert call(C.c_void_p(0x10010), n.value, fake) == L.LPM_EINVAL  # not 256-byte aligned
    assert call(None, n.value, fake) == L.LPM_EINVAL
    assert call(fake, n.value, None) == L.LPM_EINVAL
    # records stored by work-order position: the order is checked too
    ordered = lambda order, n_order: code(L, "lpm_grid_records_ordered", rec, 1000, 4, 5, 2, src,
                                          sch, ph, grid, order, n_order, fake, n.value, fake,
                                          None)
    assert ordered(None, 10) == L.LPM_EINVAL and b"null work order" in L.lib().lpm_last_error()
    assert ordered(C.c_void_p(0x10002), 10) == L.LPM_EINVAL       # misaligned
    assert ordered(fake, 1001) == L.LPM_EINVAL                     # beyond n_local
    assert ordered(fake, -1) == L.LPM_EINVAL


def test_time_pair_fields_are_checked(args):
    """lpm_field_interval_bytes / lpm_field_interval and time-pair fields in
    step calls: sizes, and every invalid use rejected before a launch."""
    L, st, src, sch, ph, fld, acc, grid = args
    hourly = L.Field.from_buffer_copy(fld)
    hourly.nt = 3
    n = C.c_int64(0)
    assert code(L, "lpm_field_interval_bytes", hourly, C.byref(n)) == L.LPM_OK
    assert n.value == 200 * 200 * 30 * 16
    three = L.Field.from_buffer_copy(hourly)
    three.ncomp = 3
    assert code(L, "lpm_field_interval_bytes", three, C.byref(n)) == L.LPM_OK
    assert n.value == 200 * 200 * 30 * 32
    assert code(L, "lpm_field_interval_bytes", fld, C.byref(n)) == L.LPM_EINVAL  # nt = 1
    packed = L.Field()
    out = C.c_void_p(0x40000000)
    pack = lambda f, k, o=out: code(L, "lpm_field_interval", f, k, o, C.byref(packed), None)
    assert pack(hourly, 2) == L.LPM_EINVAL and b"interval" in L.lib().lpm_last_error()
    assert pack(hourly, -1) == L.LPM_EINVAL
    assert pack(hourly, 0, C.c_void_p(0x40000008)) == L.LPM_EINVAL  # 16-byte alignment
    assert pack(hourly, 0, C.c_void_p(fld.data + 64)) == L.LPM_EINVAL
    assert b"overlaps" in L.lib().lpm_last_error()
    # a time-pair descriptor in step calls
    tp = L.Field.from_buffer_copy(hourly)
    tp.layout, tp.interval = L.FIELD_TIME_PAIRS, 1
    step = lambda f, s0, n: code(L, "lpm_step_particles", st, src, sch, f, ph, s0, n, acc, None)
    assert step(tp, 0, 10) == L.LPM_EINVAL  # steps 0..9 interpolate in interval 0
    assert b"interpolate in field interval 1" in L.lib().lpm_last_error()
    assert step(tp, 715, 10) == L.LPM_EINVAL  # steps 715..724 straddle t = 1 h
    for bad in (dict(interval=2), dict(interval=-1), dict(layout=7), dict(data=fld.data + 8)):
        f = L.Field.from_buffer_copy(tp)
        for k, v in bad.items():
            setattr(f, k, v)
        assert step(f, 720, 10) == L.LPM_EINVAL, bad


def test_launch_settings_are_checked():
    import paper_0912_3223_amd as L
    lib = L.lib()
    assert lib.lpm_set_launch_ex(24, 0, -1) == L.LPM_EINVAL
    assert lib.lpm_set_launch_ex(24, 0, 65) == L.LPM_EINVAL
    assert lib.lpm_set_launch_ex(0, 0, 0) == L.LPM_EINVAL
    assert lib.lpm_set_launch_ex(4097, 0, 0) == L.LPM_EINVAL
    assert lib.lpm_set_launch_ex(24, -1, 0) == L.LPM_EINVAL
    assert lib.lpm_set_launch_ex(16, 2, 32) == L.LPM_OK
    assert lib.lpm_set_launch(24, 0) == L.LPM_OK  # keeps refill_min 32
    L.set_launch()  # the defaults: 24, 0, and the idle-lane threshold by the wind


def test_work_order_is_checked(args):
    """lpm_order_workspace / lpm_order_particles and work orders in step
    calls: invalid uses rejected before a launch."""
    L, st, src, sch, ph, fld, acc, grid = args
    n = C.c_int64(0)
    assert code(L, "lpm_order_workspace", sch, fld, C.byref(n)) == L.LPM_OK
    ws = n.value
    assert 16 * 1000 <= ws <= 16 * 1000 + 64 * 1024  # pairs, digit counts
    fake = C.c_void_p(0x10000)
    order = lambda s0, ns, cap=1000, o=fake, w=fake, wb=ws: code(
        L, "lpm_order_particles", st, sch, fld, s0, ns, o, cap, C.byref(n), w, wb, None)
    assert order(0, 10, cap=10) == L.LPM_EINVAL and b"capacity" in L.lib().lpm_last_error()
    assert order(0, 10, wb=ws - 8) == L.LPM_EINVAL and b"workspace" in L.lib().lpm_last_error()
    assert order(0, 10, o=C.c_void_p(0x10002)) == L.LPM_EINVAL
    assert order(0, 10, w=C.c_void_p(0x10080)) == L.LPM_EINVAL  # 256-byte alignment
    assert order(-1, 10) == L.LPM_EINVAL
    assert order(0, 0) == L.LPM_EINVAL
    # a step launch over steps 0..9 has the particles born by step 10
    ordered = L.State.from_buffer_copy(st)
    ordered.order, ordered.n_order = 0x10000, 7
    assert code(L, "lpm_step_particles", ordered, src, sch, fld, ph, 0, 10, acc,
                None) == L.LPM_EINVAL
    assert b"work order" in L.lib().lpm_last_error()
    ordered.order = 0x10002
    assert code(L, "lpm_step_particles", ordered, src, sch, fld, ph, 0, 10, acc,
                None) == L.LPM_EINVAL


def test_ensemble_step_arguments_are_checked(args):
    """lpm_step_ensemble rejects bad deposition copies and launch settings on
    the host, before anything is launched (fake device pointers)."""
    L, st, src, sch, ph, fld, acc, grid = args
    fake = C.c_void_p(0x10000)
    ens = L.Ensemble(0x10000, 1, 2, 0, 10, 1000, 1000, L.Launch(24, 56, 0, 256), 1, 0)
    dg = acc.dep_grid
    step = lambda e: code(L, "lpm_step_ensemble", st, e, fld, ph, dg, fake, fake, fake, None)
    bad = L.Ensemble.from_buffer_copy(ens)
    bad.dep_copies = 65  # above LPM_MAX_DEP_COPIES
    assert step(bad) == L.LPM_EINVAL and b"dep_copies" in L.lib().lpm_last_error()
    bad.dep_copies = -1
    assert step(bad) == L.LPM_EINVAL
    bad = L.Ensemble.from_buffer_copy(ens)
    bad.launch.block = 192  # not one of the instantiated block sizes
    assert step(bad) == L.LPM_EINVAL

"""lpm_grid_concentration_static (the concentration grid on the library's
static device scratch, for callers that cannot allocate) against
lpm_grid_concentration (caller-owned scratch), called through the C ABI:
two calls in a row, the second on a smaller grid and fewer particles, each
equal to the allocating entry point's grid (relative L2 <= 1e-6: the same
float32 contributions summed in FP64, in another order), and a grid beyond
the static maximum rejected."""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0912_3223_amd  # noqa: F401


def _both(case, step):
    import torch
    import paper_0912_3223_amd as L
    run = L.DeviceRun(case)
    run.run(s_end=step + 1, steps_per_launch=60)
    torch.cuda.synchronize()
    cg = case.conc_grid
    nn = case.physics.n_nuc
    ref = run.grid_concentration(step).double().cpu().numpy()
    out = torch.full((nn, cg.nz, cg.ny, cg.nx), float("nan"), dtype=torch.float32, device="cuda")
    rc = L.lib().lpm_grid_concentration_static(
        C.byref(run.st), C.byref(run.src), C.byref(run.sch), C.byref(run.ph), C.byref(run.cgrid),
        step, C.c_void_p(out.data_ptr()), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, L.lib().lpm_last_error()
    torch.cuda.synchronize()
    return ref, out.double().cpu().numpy()


def _close(ref, got):
    assert not np.isnan(got).any()
    peak = np.abs(ref).max()
    assert peak > 0
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert rel <= 1e-6, rel
    assert np.all(got[ref == 0] == 0)
    return rel


def test_static_scratch_matches_allocating_call_twice():
    from parity import log
    big = synth.c1(n_total=60_000, n_steps=600, s_release=600)
    ref1, got1 = _both(big, 599)
    r1 = _close(ref1, got1)
    # second call: smaller grid and fewer particles; what the first call left
    # in the static scratch must not leak into it
    small = synth.c1(n_total=7_000, n_steps=300, s_release=300)
    small = small.with_(conc_grid=synth.replace(small.conc_grid, nx=64, ny=48, nz=12,
                                                x0=-8000.0, y0=-6000.0))
    ref2, got2 = _both(small, 299)
    r2 = _close(ref2, got2)
    log("static-scratch gridding: rel %.2e (200x200x30x2), %.2e (64x48x12x2)" % (r1, r2))


def test_static_scratch_rejects_oversized_grid():
    import torch
    import paper_0912_3223_amd as L
    case = synth.c1(n_total=1000, n_steps=10, s_release=10)
    # 2 nuclides x 400 x 400 x 40 = 12.8e6 doubles > 4 Mi
    case = case.with_(conc_grid=synth.replace(case.conc_grid, nx=400, ny=400, nz=40))
    run = L.DeviceRun(case)
    out = torch.zeros(1, dtype=torch.float32, device="cuda")
    rc = L.lib().lpm_grid_concentration_static(
        C.byref(run.st), C.byref(run.src), C.byref(run.sch), C.byref(run.ph), C.byref(run.cgrid),
        5, C.c_void_p(out.data_ptr()), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == L.LPM_EINVAL
    assert b"static scratch" in L.lib().lpm_last_error()

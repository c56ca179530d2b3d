"""Helpers shared by the GPU parity tests: run a workload through liblpm and
through the oracle on the same seeded inputs, and compare the results.

Comparison metrics follow the paper's own CPU/GPU comparison (Sec. 4.1):
per-particle distance between the two trajectories, and the relative
difference of the gridded activity."""
from __future__ import annotations

import sys
import time

import numpy as np

import oracle


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(case, steps_per_launch=60, snaps=(), state=None, s_begin=0, s_end=None):
    import torch
    import paper_0912_3223_amd as L
    r = L.DeviceRun(case)
    if state is not None:
        r.set_state(state["x"], state["y"], state["z"], state["m"], state.get("xl"),
                    state.get("yl"))
    out = {}

    def grab(step, g):
        out[step] = g.double().cpu().numpy()

    r.run(s_begin=s_begin, s_end=s_end, steps_per_launch=steps_per_launch, snap_steps=snaps,
          on_snapshot=grab, release=True)
    dep = r.grid_deposition().double().cpu().numpy()
    torch.cuda.synchronize()
    res = {"state": r.state(), "snaps": out, "dep": dep, "ledger": r.ledger(), "run": r}
    return res


def records_by_particle(rec, n_rec, stride, order):
    """A window's record buffer (n_rec records of `stride` entries, then the
    `last` words) in particle order, as (records [n_rec][stride][4], last
    [stride]) device tensors.  With a work order the library stores queue
    position q (particle order[q]) at q; particles the order does not list
    get last = INT_MIN (no meaningful record)."""
    import torch
    recs = rec[: 4 * n_rec * stride].view(n_rec, stride, 4)
    last = rec[4 * n_rec * stride: (4 * n_rec + 1) * stride].view(torch.int32)
    if order is None:
        return recs.clone(), last.clone()
    idx = order.long()
    m = idx.numel()
    r2 = torch.zeros_like(recs)
    l2 = torch.full_like(last, -2 ** 31)
    r2[:, idx] = recs[:, :m]
    l2[idx] = last[:m]
    return r2, l2


def run_oracle(case, snaps=(), state=None, s_begin=0, s_end=None, nthreads=0):
    o = oracle.Oracle(case)
    t = time.time()
    r = o.simulate(s_begin=s_begin, s_end=s_end, state=state, snap_steps=list(snaps),
                   nthreads=nthreads)
    r["seconds"] = time.time() - t
    r["snap_map"] = {s: r["snaps"][k] for k, s in enumerate(snaps)}
    r["oracle"] = o
    return r


def ledger_ok(gl, ol, released, tol=1e-6):
    """Every ledger entry within ``tol`` of the released activity."""
    diff = np.abs(np.asarray(gl, dtype=np.float64) - np.asarray(ol, dtype=np.float64))
    assert np.all(diff <= tol * released), (diff / released, gl, ol)


def distances(a, b, active):
    d = np.sqrt((a["x"] - b["x"]) ** 2 + (a["y"] - b["y"]) ** 2 + (a["z"] - b["z"]) ** 2)
    return d[active]


def rel_l2_masked(gpu, ref, frac=1e-3):
    """Relative L2 difference over cells where the reference is at least
    ``frac`` of its peak."""
    peak = np.abs(ref).max()
    if peak == 0:
        return 0.0, 0
    sel = np.abs(ref) >= frac * peak
    return float(np.linalg.norm((gpu - ref)[sel]) / np.linalg.norm(ref[sel])), int(sel.sum())


def ngp_unexplained(gpu, ref, positions, activities, grid, delta):
    """Cells whose NGP difference exceeds what particles within ``delta`` (m)
    of a cell face could move between neighbouring cells.  Returns the
    largest unexplained excess relative to the peak."""
    x, y, z = positions
    slack = np.zeros_like(ref)
    fx = (x - grid.x0) / grid.dx
    fy = (y - grid.y0) / grid.dy
    fz = (z - grid.z0) / grid.dz
    near = (np.abs(fx - np.round(fx)) * grid.dx < delta) | \
           (np.abs(fy - np.round(fy)) * grid.dy < delta) | \
           (np.abs(fz - np.round(fz)) * grid.dz < delta)
    for dxo in (-1, 0, 1):
        for dyo in (-1, 0, 1):
            for dzo in (-1, 0, 1):
                ix = np.floor(fx[near]).astype(np.int64) + dxo
                iy = np.floor(fy[near]).astype(np.int64) + dyo
                iz = np.floor(fz[near]).astype(np.int64) + dzo
                ok = (ix >= 0) & (iy >= 0) & (iz >= 0) & (ix < grid.nx) & (iy < grid.ny) & \
                     (iz < grid.nz)
                for n in range(ref.shape[0]):
                    np.add.at(slack[n], (iz[ok], iy[ok], ix[ok]), np.abs(activities[n][near][ok]))
    excess = np.abs(gpu - ref) - slack * (1 + 1e-6) - 1e-6 * np.abs(ref).max()
    return float(max(excess.max(), 0.0) / np.abs(ref).max()), int(near.sum())


def activities(case, state, step):
    """Per-particle activity after `step` (for the NGP slack), float64."""
    sch, ph, src = case.schedule, case.physics, case.source
    n = sch.local_count
    g = sch.id_base + np.arange(n, dtype=np.int64) * sch.id_stride
    b = (g * sch.s_release) // sch.n_total
    a0 = src.q * sch.s_release * ph.dt / sch.n_total
    age = (step + 1 - b) * ph.dt
    alive = (b <= step) & (state["m"] > 0)
    out = []
    for lam in ph.lambdas:
        out.append(np.where(alive, a0 * state["m"] * np.exp(-lam * age), 0.0))
    return out

"""Writes c4_receptors.json: the 50 receptor points and the observations of
the source-inversion workload.  Calls only the oracle.

Recipe:
  1. Pilot run of the hidden source (h = 80 m, q = 1.3, s_w = 1.1,
     v_d = 0.003 m/s) with Philox seed 1 and 1e5 particles on the 6 h
     gridded workload; its cloud-in-cell concentration in the lowest grid
     layer is summed over the 72 output steps (every 60 steps).
  2. 50 receptors at ground level (z = 0), at the centres of cells drawn
     uniformly without replacement (numpy default_rng(4)) among the cells
     whose time-summed pilot concentration is at least 1e-2 of its maximum.
  3. Observations: receptor concentrations of the hidden source with Philox
     seed 1 and 1e6 particles (Gaussian kernel, sigma_h = 250 m, sigma_z =
     40 m, time weight 60 dt = 300 s per output step), times exp(0.05 zeta)
     with zeta standard normal (default_rng(5)): 5 % lognormal noise.

    python tests/golden/make_c4_receptors.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    t0 = time.time()
    pilot = synth.with_theta(synth.c4(n_total=100_000, seed=1), synth.THETA_HIDDEN)
    o = oracle.Oracle(pilot)
    g = pilot.conc_grid
    ground = np.zeros((g.ny, g.nx))
    st = None
    for k in range(pilot.n_steps // pilot.out_every):
        s0, s1 = k * pilot.out_every, (k + 1) * pilot.out_every
        r = o.simulate(s_begin=s0, s_end=s1, state=st, snap_steps=[s1 - 1])
        st = r["state"]
        ground += r["snaps"][0][:, 0].sum(axis=0)
    cand = np.argwhere(ground >= 1e-2 * ground.max())
    rng = np.random.default_rng(4)
    pick = cand[rng.choice(len(cand), size=50, replace=False)]
    xs = [float(g.x0 + (j + 0.5) * g.dx) for _, j in pick]
    ys = [float(g.y0 + (i + 0.5) * g.dy) for i, _ in pick]
    rec = synth.Receptors(tuple(xs), tuple(ys), (0.0,) * 50, 250.0, 40.0,
                          60 * pilot.physics.dt)
    print(f"pilot done in {time.time() - t0:.1f} s, {len(cand)} candidate cells", flush=True)
    hidden = synth.with_theta(synth.c4(seed=1), synth.THETA_HIDDEN)
    c = oracle.Oracle(hidden).receptor_forward(rec)["c"]
    obs = c * np.exp(0.05 * np.random.default_rng(5).standard_normal(50))
    out = {"x": xs, "y": ys, "z": [0.0] * 50, "sigma_h": 250.0, "sigma_z": 40.0,
           "weight": rec.weight, "observations": [float(v) for v in obs],
           "hidden_theta": list(synth.THETA_HIDDEN), "theta0": list(synth.THETA0),
           "note": "written by make_c4_receptors.py (oracle only)"}
    with open(os.path.join(HERE, "c4_receptors.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"done in {time.time() - t0:.1f} s; c range {c.min():.3e} .. {c.max():.3e}")


if __name__ == "__main__":
    main()

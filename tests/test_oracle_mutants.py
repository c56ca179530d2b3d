"""Planted mistakes: single-line errors in a copy of the oracle, each of
which must make at least one of the pins fail.  This checks the pins, not
the oracle: a plausible slip anywhere in the method (a dropped term, a wrong
sign, index or constant, a transposed operand) has to be caught by a closed
form, an invariant or a library reference of the -m "not gpu" suite.

Each mutant is built with gcc into a temporary library, and the pins named
for it run in a subprocess against that library (LPM_ORACLE_LIB); the mutant
is caught when that run fails.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "lpm_oracle.c")

P = "test_oracle_pieces.py::"
I = "test_oracle_invariants.py::"
V = "test_oracle_variants.py::"
PL = "test_oracle_plume.py::"
G = "test_oracle_gradient.py::"
R = "test_oracle_philox.py::"

# (name, original text, mistake, pins expected to catch it)
MUTANTS = [
    ("philox multiplier", "const uint32_t M0 = 0xD2511F53u", "const uint32_t M0 = 0xD2511F55u",
     [R + "test_philox_matches_rocrand"]),
    ("philox key schedule", "if (round > 0) { k0 += W0; k1 += W1; }",
     "if (round > 1) { k0 += W0; k1 += W1; }", [R + "test_philox_matches_rocrand"]),
    ("halved horizontal diffusivity", "xi[0] * sqrt(2.0 * P->Kh * dt)",
     "xi[0] * sqrt(1.0 * P->Kh * dt)", [I + "test_random_walk_uses_the_particle_stream"]),
    ("swapped normals", "double yn = y + v * dt + xi[1] *", "double yn = y + v * dt + xi[2] *",
     [I + "test_random_walk_uses_the_particle_stream"]),
    ("age off by one step", "double age = (double)(s - b) * dt;\n    double a0 = a0_of(P);\n\n    /* random",
     "double age = (double)(s - b + 1) * dt;\n    double a0 = a0_of(P);\n\n    /* random",
     [PL + "test_decay_is_exact_exponential", I + "test_c1_mass_ledger_closes"]),
    ("birth rounded up", "return (gid * (int64_t)P->s_release) / P->n_total;",
     "return (gid * (int64_t)P->s_release + P->n_total - 1) / P->n_total;",
     [PL + "test_decay_is_exact_exponential"]),
    ("no lid", "zn = fold(zn, P->H_lid);", "zn = fold(zn, 0.0);",
     [I + "test_lid_and_ground_mix_to_uniform"]),
    ("1 % wind error", "double u = P->wind_scale * uvw[0];",
     "double u = 1.01 * P->wind_scale * uvw[0];", [I + "test_pure_advection_without_turbulence"]),
    ("missing drift", "double zn = z + w * dt + dKz * dt + xi[2]", "double zn = z + w * dt + xi[2]",
     [I + "test_well_mixed_stays_well_mixed"]),
    ("wrong slope sign", "*dK = ku * (g - (z + P->z0) / H);", "*dK = ku * (g + (z + P->z0) / H);",
     [P + "test_kz_profile"]),
    ("no drift at the top of the mixed layer", "if (z > H) { *K = 0.0; *dK = 0.0; return; }",
     "if (z >= H) { *K = 0.0; *dK = 0.0; return; }",
     [P + "test_particles_at_the_top_of_the_mixed_layer_leave_it"]),
    ("drift sign", "double zn = z + w * dt + dKz * dt + xi[2]", "double zn = z + w * dt - dKz * dt + xi[2]",
     [I + "test_well_mixed_stays_well_mixed"]),
    ("deposit and decay shares swapped", "led[n * 4 + 1] += d;\n        led[n * 4 + 2] += P->lambda[n] * S;",
     "led[n * 4 + 2] += d;\n        led[n * 4 + 1] += P->lambda[n] * S;",
     [I + "test_wet_deposition_of_a_resting_particle"]),
    ("no decay in the exit step", "led[n * 4 + 3] += a0 * mn * orc_activity_fraction(P, n, age + dt);",
     "led[n * 4 + 3] += a0 * mn * orc_activity_fraction(P, n, age);",
     [I + "test_exit_at_the_domain_boundary", I + "test_c1_mass_ledger_closes"]),
    ("flipped cloud-in-cell weight", "double vx = a2 ? wx : 1.0 - wx;", "double vx = a2 ? 1.0 - wx : wx;",
     [P + "test_cic_weights"]),
    ("dry rate profile factor", "return P->v_d * (2.0 / P->h_s) * (1.0 - z / P->h_s);",
     "return P->v_d * (1.0 / P->h_s) * (1.0 - z / P->h_s);",
     [P + "test_dry_rate_profile_integrates_to_vd"]),
    ("rain edge offset",
     "(yr / P->rain_b) * (yr / P->rain_b));\n    double f = (1.0 - re) / P->rain_edge + 0.5;",
     "(yr / P->rain_b) * (yr / P->rain_b));\n    double f = (1.0 - re) / P->rain_edge + 0.25;",
     [I + "test_rain_edge_rate_is_half_on_the_ellipse"]),
    ("wind weight transposed", "s += (1 - wz) * (1 - wy) * wx * node(P, T, k0, j0, i1, c);",
     "s += (1 - wz) * wx * (1 - wy) * node(P, T, k0, j1, i0, c);",
     [P + "test_wind_is_exact_for_linear_fields"]),
    ("time weight reversed", "uvw[c] = (1 - wt) * val[0] + wt * val[1];",
     "uvw[c] = wt * val[0] + (1 - wt) * val[1];", [P + "test_wind_is_exact_for_linear_fields"]),
    ("Bateman prefactor dropped", "double num = P->lambda[n] / P->lambda[0];", "double num = 1.0;",
     [V + "test_activity_fraction_is_the_matrix_exponential"]),
    ("removal decided by the wrong uniform", "removed = u[0] <= -expm1(-k * dt);",
     "removed = u[1] <= -expm1(-k * dt);", [V + "test_stochastic_removal_follows_the_purpose_one_stream"]),
    ("stability function sign", "*phi = 1.0 + 5.0 * s;", "*phi = 1.0 - 5.0 * s;",
     [V + "test_kz_stability_profile"]),
    ("Jacobian mass term dropped", "J[3][3] = e;", "J[3][3] = 1.0;",
     [G + "test_tangent_matches_central_differences"]),
    ("adjoint not transposed", "for (int a = 0; a < 4; ++a) nb[k] += J[a][k] * ub[a];",
     "for (int a = 0; a < 4; ++a) nb[k] += J[k][a] * ub[a];", [G + "test_adjoint_equals_tangent"]),
    ("drift curvature dropped in the Jacobian", "1.0 + sw * dt * g[2][2] + K2 * dt + xi[2] * dsq_dz};",
     "1.0 + sw * dt * g[2][2] + xi[2] * dsq_dz};", [G + "test_tangent_matches_central_differences"]),
]


def _mutant(tmp, idx):
    name, old, new, pins = MUTANTS[idx]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site of %r not unique in the oracle" % name
    path = os.path.join(tmp, "m%02d.c" % idx)
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    lib = os.path.join(tmp, "m%02d.so" % idx)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
                    "-ffp-contract=off", path, "-o", lib, "-lm"], check=True,
                   capture_output=True)
    env = dict(os.environ, LPM_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-p", "no:randomly", *[os.path.join(HERE, p) for p in pins]],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    return name, r.returncode, r.stdout[-800:]


def test_every_planted_mistake_fails_a_pin(tmp_path):
    for _, old, _, _ in MUTANTS:
        assert open(SRC).read().count(old) == 1, old
    workers = max(1, min(8, (os.cpu_count() or 2) // 2))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(lambda i: _mutant(str(tmp_path), i), range(len(MUTANTS))))
    survived = [(n, out) for n, rc, out in results if rc == 0]
    errored = [(n, out) for n, rc, out in results if rc not in (0, 1)]
    assert not errored, errored
    assert not survived, "planted mistakes no pin catches: %s" % [n for n, _ in survived]

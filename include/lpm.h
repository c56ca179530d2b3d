/*
 * lpm.h -- C ABI of the MI355X particle-dispersion library (liblpm.so).
 *
 * The library implements the data-parallel time step of the stochastic
 * Lagrangian particle model of Molnar Jr., Szakaly, Meszaros and Lagzi,
 * "Air pollution modelling using a graphics processing unit with CUDA"
 * (arXiv:0912.3223): particles released from a point source (Sec. 2) are
 * advected by an interpolated wind field and displaced by a random walk
 * scaled by K (Eqs. 1-3), reflected at the ground, decayed, and depleted by
 * dry and wet deposition (Sec. 2); their activity is summed on rectangular
 * grids (Sec. 3.2).
 *
 * Conventions shared by every entry point
 *  - All array pointers are DEVICE pointers owned by the caller (allocate and
 *    free them yourself); the library never allocates, frees or retains them
 *    after the call returns.  Structs are passed by host pointer and read
 *    during the call only.
 *  - Every call is ordered on `stream` (a hipStream_t; NULL = the null
 *    stream) and returns without waiting for the device, except lpm_check and
 *    lpm_read_ledger, which synchronise `stream`.
 *  - Return value: LPM_OK (0) or a negative LPM_E* code; lpm_last_error()
 *    gives a message for the calling thread's last failure.  Arguments are
 *    validated on the host before anything is launched; a rejected call
 *    launches nothing.  No C++ exception crosses the ABI.
 *  - Particle state is structure-of-arrays float32: x, y (m, horizontal),
 *    z (m above ground), m (surviving mass fraction in [0, 1]; 0 marks an
 *    inactive particle: exited, or never released).  Arrays have `capacity`
 *    elements and must be 4-byte aligned.
 *  - Local particle i is global particle id  g = id_base + i * id_stride,
 *    born (released) at step  b(g) = floor(g * s_release / n_total).  The
 *    birth and the random numbers depend on the global id only, so a run over
 *    a subset of ids reproduces the full run's trajectories for those ids.
 *  - Random numbers: Philox4x32-10 (Salmon et al., SC'11; replaces the
 *    Mersenne Twister of Sec. 2) with counter (g, step, 0, 0) and key
 *    (low 32 bits of seed, scenario); uniforms ((r >> 8) + 1) 2^-24 in (0, 1];
 *    normals by the trigonometric Box-Muller form (Sec. 2).
 *  - Wind field: float32 [nt][nz][ny][nx][ncomp], ncomp = 2 (u, v) or 3
 *    (u, v, w), cell-centred nodes at x0 + (i + 1/2) dx, y0 + (j + 1/2) dy,
 *    z = (k + 1/2) dz (or z_levels[k]), times t0 + k dt_field; sampled
 *    linearly in x, y, z and t with clamp-to-edge (Sec. 3.2).
 */
#ifndef LPM_H
#define LPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define LPM_OK 0
#define LPM_EINVAL (-1)     /* null pointer, bad size, shape or parameter   */
#define LPM_ECAPACITY (-2)  /* particle count exceeds the state capacity    */
#define LPM_EHIP (-3)       /* HIP launch or runtime failure                */
#define LPM_ENONFINITE (-4) /* a particle coordinate or mass became NaN/Inf */

/* Ledger layout; see lpm_accum. */
#define LPM_LEDGER_SLOTS 64
#define LPM_LEDGER_STRIDE 32 /* doubles per slot (two 128-byte lines) */
#define LPM_LEDGER_PSTEPS 16 /* slot entry counting advanced particle-steps */
/* Ledger entries per nuclide. */
#define LPM_LEDGER_RELEASED 0
#define LPM_LEDGER_DEPOSITED 1
#define LPM_LEDGER_DECAYED 2
#define LPM_LEDGER_EXITED 3

typedef void* lpm_stream; /* hipStream_t */

/* Particle state (Sec. 3.2: position and state information per particle). */
typedef struct {
    float* x;
    float* y;
    float* z;
    float* m;
    int64_t capacity; /* elements of each array */
} lpm_state;

/* Point source of one release scenario (Sec. 2).  q: release rate in
 * relative units per second -- every particle carries a0 = q * s_release * dt
 * / n_total of each nuclide (Sec. 4: the emission is scaled to the particle
 * count).  wind_scale multiplies the sampled wind; v_d is the dry-deposition
 * velocity (m/s); scenario is the second Philox key word. */
typedef struct {
    double xs, ys, h;
    double q;
    double wind_scale;
    double v_d;
    uint32_t scenario;
    uint32_t reserved;
} lpm_source;

/* Release schedule (Sec. 3.2: emission profile and maximum particle count
 * known a priori).  n_local local particles with global ids id_base +
 * i * id_stride out of n_total; releases over steps [0, s_release). */
typedef struct {
    int64_t n_total;
    int64_t n_local;
    int64_t id_base;
    int64_t id_stride;
    int32_t s_release;
    int32_t reserved;
} lpm_schedule;

/* Gridded wind (Sec. 3.2: weather sampled linearly in x, y, z and time).
 * data: device float [nt][nz][ny][nx][ncomp]; z_levels: device float[nz],
 * increasing node heights, or NULL for (k + 1/2) dz.  bounded != 0: a
 * particle whose post-step (x, y) leaves [x0, x0 + nx dx) x [y0, y0 + ny dy)
 * is inactivated and its activity booked as exited (Sec. 3.2). */
typedef struct {
    const float* data;
    const float* z_levels;
    int32_t nx, ny, nz, nt, ncomp, bounded;
    double x0, y0, dx, dy, dz, t0, dt_field;
} lpm_field;

/* Physical constants (Sec. 2, Eqs. 2-3).
 *  kz_kind 0: K_z = Kz_const;  1: K_z = kappa_ustar (z + z0)(1 - z/H_mix);
 *  2: K_z = kappa_ustar (z + z0)(1 - z/H_mix)^2 (Eq. 3 with Phi = 1); K_z = 0
 *  above H_mix.  The vertical step adds the drift dK_z/dz dt and evaluates
 *  K_z at z + dK_z/dz dt / 2 clamped to [0, H_mix]; with constant K_z this is
 *  Eq. (2) as printed.
 *  H_lid > 0: z is folded into [0, H_lid]; H_lid <= 0: ground reflection only.
 *  Dry deposition rate v_d * (2/h_s)(1 - z/h_s) for z < h_s; wet rate
 *  Lambda0 * clamp((1 - r)/rain_edge + 1/2, 0, 1), r the elliptical radius
 *  about (rain_cx, rain_cy) with semi-axes rain_a, rain_b, major axis at
 *  rain_angle (radians, counter-clockwise from +x).
 *  lambda[n]: decay constants (1/s) of n_nuc <= 4 nuclides. */
typedef struct {
    double dt, Kh, Kz_const, kappa_ustar, z0, H_mix, H_lid, h_s;
    int32_t kz_kind, n_nuc;
    double lambda[4];
    double Lambda0, rain_cx, rain_cy, rain_a, rain_b, rain_angle, rain_edge;
    uint64_t seed;
} lpm_physics;

/* Output grid (Sec. 3.2: activities summed on a rectangular grid).  mode 0:
 * the cell containing the point (half-open cells); mode 1: cloud-in-cell
 * weights about cell centres, weights outside the grid dropped.  density != 0:
 * divide by the cell volume (3-D) or area (2-D).  A deposition grid is 2-D:
 * its nz, z0 and dz are ignored. */
typedef struct {
    int32_t nx, ny, nz, mode, density, reserved;
    double x0, y0, z0, dx, dy, dz;
} lpm_grid;

/* Accumulators of a run, all device memory owned by the caller:
 *  dep:    double [n_nuc][dep_grid.ny][dep_grid.nx], deposited activity;
 *  ledger: double [LPM_LEDGER_SLOTS][LPM_LEDGER_STRIDE]: entries
 *          4 n + e hold nuclide n's released (e = 0), deposited (1), decayed
 *          (2) and exited (3) activity, entry LPM_LEDGER_PSTEPS the number of
 *          particle-steps advanced; per-slot partial sums that
 *          lpm_read_ledger adds up;
 *  err:    uint32, bit 0 set when a particle became non-finite. */
typedef struct {
    double* dep;
    double* ledger;
    uint32_t* err;
    int32_t n_nuc;
    int32_t reserved;
    lpm_grid dep_grid;
} lpm_accum;

/* Zero dep, ledger and err.  Stream-ordered. */
int lpm_accum_reset(const lpm_accum* acc, lpm_stream stream);

/* Release (Sec. 2: particles released from a point source in each time step;
 * Sec. 3.2: masses assigned a priori).  Every local particle born in
 * [step0, step0 + n_steps) is placed at (xs, ys, h) with m = 1, and its
 * activity a0 of each nuclide is added to the ledger's released entry.
 * Other particles are not touched.  LPM_ECAPACITY if n_local > capacity. */
int lpm_release_particles(const lpm_state* st, const lpm_source* src,
                          const lpm_schedule* sch, const lpm_physics* ph,
                          int32_t step0, int32_t n_steps, const lpm_accum* acc,
                          lpm_stream stream);

/* Time steps step0 .. step0 + n_steps - 1 (Sec. 3.2 main loop; Eqs. 1-3).
 * Every local particle with birth b < step0 + n_steps and m > 0 is advanced
 * from step max(b, step0); its state is read once and written once per call
 * (particles born inside the window must have been released by
 * lpm_release_particles).  Per step, at the start-of-step position and time
 * s dt: wind sample times wind_scale, K_h, K_z, move (Eq. 1, Eq. 2), fold z,
 * then at the new position the deposition rate k = dry + wet, m <- m
 * exp(-k dt), the step's loss of activity A (1 - exp(-(lambda + k) dt)) split
 * into deposited (share k/(lambda + k), added to dep at the new (x, y)) and
 * decayed (share lambda/(lambda + k)) in the ledger; a particle leaving a
 * bounded field books its remaining activity as exited and gets m = 0.
 * A non-finite coordinate or mass sets err and stops that particle.
 * Any n_steps >= 1 is allowed; the same trajectories result for any split
 * of the run into calls. */
int lpm_step_particles(const lpm_state* st, const lpm_source* src,
                       const lpm_schedule* sch, const lpm_field* fld,
                       const lpm_physics* ph, int32_t step0, int32_t n_steps,
                       const lpm_accum* acc, lpm_stream stream);

/* lpm_step_particles, and in addition the state of every local particle
 * after each output step rec_step0 + k * rec_every (k = 0 .. n_rec - 1) is
 * written to rec: device float planes x, y, z, m of record k at
 * rec + (4 k + q) * rec_stride, q = 0..3 (m = 0 once a particle has left the
 * area; particles not yet born at that step are not written, and gridding
 * skips them by their birth).  With every recorded step inside one window the
 * whole run can be a single launch in which each thread carries its particle
 * from birth to the last step, and the concentration at each output step
 * (Sec. 3.2: activities summed every n-th step) is gridded afterwards from the
 * records with lpm_grid_concentration.  All recorded steps must lie in
 * [step0, step0 + n_steps); rec_stride >= n_local.  rec is caller-owned. */
int lpm_step_particles_record(const lpm_state* st, const lpm_source* src,
                              const lpm_schedule* sch, const lpm_field* fld,
                              const lpm_physics* ph, int32_t step0, int32_t n_steps,
                              const lpm_accum* acc, int32_t rec_step0, int32_t rec_every,
                              int32_t n_rec, float* rec, int64_t rec_stride,
                              lpm_stream stream);

/* Concentration after step `step` (time (step + 1) dt; Sec. 3.2: every n-th
 * step the activity a0 m exp(-lambda age) of each particle is summed on a
 * rectangular grid).  acc_scratch: device double [n_nuc][nz][ny][nx],
 * overwritten; out: device float [n_nuc][nz][ny][nx], overwritten.  Only
 * particles with birth <= step and m > 0 contribute. */
int lpm_grid_concentration(const lpm_state* st, const lpm_source* src,
                           const lpm_schedule* sch, const lpm_physics* ph,
                           const lpm_grid* grid, int32_t step,
                           double* acc_scratch, float* out, lpm_stream stream);

/* Deposited activity so far on the deposition grid, converted to float and
 * divided by the cell area when dep_grid.density != 0.
 * out: device float [n_nuc][ny][nx], overwritten. */
int lpm_grid_deposition(const lpm_accum* acc, float* out, lpm_stream stream);

/* Synchronise `stream`, copy the ledger and add its slots:
 * host_out: host double [n_nuc * 4 + 1]: per nuclide released, deposited,
 * decayed, exited, then the number of particle-steps advanced since the last
 * reset (a particle advanced through one step counts once). */
int lpm_read_ledger(const lpm_accum* acc, double* host_out, lpm_stream stream);

/* Synchronise `stream` and report the device error word: LPM_ENONFINITE if
 * any particle became non-finite since the last reset, else LPM_OK. */
int lpm_check(const lpm_accum* acc, lpm_stream stream);

/* Message of the calling thread's last failed call ("" if none). */
const char* lpm_last_error(void);

/* Library version string. */
const char* lpm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LPM_H */

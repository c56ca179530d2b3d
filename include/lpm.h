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
/* Control words (see lpm_accum.ctrl). */
#define LPM_CTRL_WORDS 64
#define LPM_CTRL_ERR 0   /* error flags: bit 0 = a particle became non-finite */
#define LPM_CTRL_QUEUE 2 /* 64-bit work counter of the step kernel (words 2-3) */
/* Ledger entries per nuclide. */
#define LPM_LEDGER_RELEASED 0
#define LPM_LEDGER_DEPOSITED 1
#define LPM_LEDGER_DECAYED 2
#define LPM_LEDGER_EXITED 3

typedef void* lpm_stream; /* hipStream_t */

/* Particle state (Sec. 3.2: position and state information per particle).
 * x_lo, y_lo (optional, both or neither): the rounding residuals of x and y.
 * Within a step launch each horizontal coordinate is a float plus the
 * float residual of its running sum (compensated summation), so that
 * thousands of steps on positions of tens of kilometres do not accumulate
 * float roundings; with these arrays the residuals also survive between
 * calls and any split of a run into calls gives the same trajectories.
 * Without them the residuals are dropped at the end of each call (x and y
 * stay the correctly rounded positions). */
typedef struct {
    float* x;
    float* y;
    float* z;
    float* m;
    int64_t capacity; /* elements of each array */
    float* x_lo;
    float* y_lo;
    /* Optional work order of the next step launch (NULL: index order): the
     * permutation of the launch's local indices [0, n_order) that
     * lpm_order_particles writes; n_order must be the launch's particle
     * count.  The order changes no result, only the speed.  Ensemble
     * launches take no order. */
    const int32_t* order;
    int64_t n_order;
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

/* Layouts of lpm_field.data. */
#define LPM_FIELD_NODES 0      /* float [nt][nz][ny][nx][ncomp] */
#define LPM_FIELD_TIME_PAIRS 1 /* one interval, both times per node (lpm_field_interval) */

/* Gridded wind (Sec. 3.2: weather sampled linearly in x, y, z and time).
 * data: device float [nt][nz][ny][nx][ncomp] (layout LPM_FIELD_NODES), or
 * the time-pair copy of one interval that lpm_field_interval writes (layout
 * LPM_FIELD_TIME_PAIRS); z_levels: device float[nz], increasing node
 * heights, or NULL for (k + 1/2) dz.  Time node k is at t0 + k dt_field.
 * bounded != 0: a particle whose post-step (x, y) leaves [x0, x0 + nx dx) x
 * [y0, y0 + ny dy) is inactivated and its activity booked as exited
 * (Sec. 3.2). */
typedef struct {
    const float* data;
    const float* z_levels;
    int32_t nx, ny, nz, nt, ncomp, bounded;
    double x0, y0, dx, dy, dz, t0, dt_field;
    int32_t layout;   /* LPM_FIELD_NODES or LPM_FIELD_TIME_PAIRS */
    int32_t interval; /* time-pair fields: the interval k that data holds */
} lpm_field;

/* Physical constants (Sec. 2, Eqs. 2-3).
 *  kz_kind 0: K_z = Kz_const;  1: K_z = kappa_ustar (z + z0)(1 - z/H_mix);
 *  2: K_z = kappa_ustar (z + z0)(1 - z/H_mix)^2 (Eq. 3 with Phi = 1);
 *  3: Eq. 3 with the similarity function for heat, K_z = kappa_ustar (z + z0)
 *     (1 - z/H_mix)^2 / Phi_h((z + z0) inv_L), Phi_h(s) = 1 + 5 s for stable
 *     (inv_L >= 0) and (1 - 16 s)^(-1/2) for unstable stratification
 *     (Businger-Dyer forms; inv_L = 1/L, the inverse Monin-Obukhov length,
 *     0 = neutral, which is kind 2; see lpm_surface_layer).
 *  K_z = 0 above H_mix (z > H_mix; at z = H_mix the profile, whose value is
 *  0 and whose slope is taken from below).  The vertical step adds the drift dK_z/dz dt and
 *  evaluates K_z at z + dK_z/dz dt / 2 clamped to [0, H_mix]; with constant
 *  K_z this is Eq. (2) as printed.
 *  H_lid > 0: z is folded into [0, H_lid]; H_lid <= 0: ground reflection only.
 *  Dry deposition rate v_d * (2/h_s)(1 - z/h_s) for z < h_s; wet rate
 *  Lambda0 * clamp((1 - r)/rain_edge + 1/2, 0, 1), r the elliptical radius
 *  about (rain_cx, rain_cy) with semi-axes rain_a, rain_b, major axis at
 *  rain_angle (radians, counter-clockwise from +x).
 *  lambda[n]: decay constants (1/s) of n_nuc <= 4 nuclides.
 *  chain 0: every nuclide is released with activity a0 = q s_release dt /
 *     n_total per particle and decays on its own.  chain 1: the nuclides
 *     form the decay chain 0 -> 1 -> ... -> n_nuc - 1 (each decay of n makes
 *     one atom of n + 1; Bateman), only nuclide 0 is released (activity a0)
 *     and the lambdas must be positive and distinct.  In a chain, entry 0
 *     ("released") of nuclide n > 0 in the ledger counts its ingrowth
 *     (lambda_n times the atoms made by the parent's decay), so released =
 *     airborne + deposited + decayed + exited holds per nuclide.
 *  dep_mode 0: deposition depletes the particle's mass at rate k (mass
 *     depletion).  1: deposition is stochastic (Sec. 2): a particle with rate
 *     k at its post-move position is removed in the step with probability
 *     1 - exp(-k dt), decided by the uniform of Philox counter (g, step, 1, 0),
 *     and its whole activity at the end of the step is deposited. */
typedef struct {
    double dt, Kh, Kz_const, kappa_ustar, z0, H_mix, H_lid, h_s;
    int32_t kz_kind, n_nuc;
    double lambda[4];
    double Lambda0, rain_cx, rain_cy, rain_a, rain_b, rain_angle, rain_edge;
    uint64_t seed;
    double inv_L;     /* kz_kind 3: inverse Monin-Obukhov length (1/m) */
    int32_t chain;    /* 0 or 1, see above */
    int32_t dep_mode; /* 0 or 1, see above */
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
 *  dep:    double [copies][n_nuc][dep_grid.ny][dep_grid.nx], deposited
 *          activity: copies = dep_copies (1 when 0), up to
 *          LPM_MAX_DEP_COPIES.  The step kernels spread their atomics over
 *          the copies (block b adds into copy b mod copies), so that the
 *          many waves depositing into the same cells under rain do not all
 *          meet on one address; lpm_grid_deposition adds the copies up;
 *  ledger: double [LPM_LEDGER_SLOTS][LPM_LEDGER_STRIDE]: entries
 *          4 n + e hold nuclide n's released (e = 0), deposited (1), decayed
 *          (2) and exited (3) activity, entry LPM_LEDGER_PSTEPS the number of
 *          particle-steps advanced; per-slot partial sums that
 *          lpm_read_ledger adds up;
 *  ctrl:   uint32 [LPM_CTRL_WORDS], 8-byte aligned: word LPM_CTRL_ERR holds
 *          the error flags (bit 0: a particle became non-finite), the other
 *          words are working counters of the kernels (calls on one accum
 *          must therefore be ordered on one stream). */
#define LPM_MAX_DEP_COPIES 64

typedef struct {
    double* dep;
    double* ledger;
    uint32_t* ctrl;
    int32_t n_nuc;
    int32_t dep_copies; /* copies of the deposition grid in dep (0 or 1: one) */
    lpm_grid dep_grid;
} lpm_accum;

/* Zero dep (every copy), ledger and ctrl.  Stream-ordered. */
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
 * Any n_steps >= 1 is allowed; with st->x_lo and st->y_lo the same
 * trajectories result for any split of the run into calls. */
int lpm_step_particles(const lpm_state* st, const lpm_source* src,
                       const lpm_schedule* sch, const lpm_field* fld,
                       const lpm_physics* ph, int32_t step0, int32_t n_steps,
                       const lpm_accum* acc, lpm_stream stream);

/* lpm_step_particles, and in addition the state of every local particle
 * after each output step s_k = rec_step0 + k * rec_every (k = 0 .. n_rec - 1)
 * is recorded for gridding later (Sec. 3.2: activities summed every n-th
 * step).  rec: caller-owned device buffer, 16-byte aligned, of
 * 16 * n_rec * rec_stride + 4 * rec_stride bytes: record k of local particle i
 * is the float4 (x, y, z, m) at index k * rec_stride + i, followed by an int32
 * array last[rec_stride]: the step after which particle i stopped being
 * active in this window (INT_MAX if it is still active at the end, INT_MIN if
 * it was inactive on entry).  Records at or after `last` and of particles not
 * yet born are not meaningful; lpm_grid_records skips them.  All recorded
 * steps must lie in [step0, step0 + n_steps); n_local <= rec_stride < 2^32.
 * With a work order on the state (st->order), the records and `last` word
 * of queue entry q (particle order[q]) are stored at position q instead --
 * index k * rec_stride + q and last[q] -- so that they follow the order's
 * wind-node sorting; grid such records with lpm_grid_records_ordered (the
 * receptor calls take records stored by particle index).
 * With every output step inside one window the whole run is one launch in
 * which all particles of the run are in flight at once. */
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

/* *bytes (host) = the device workspace lpm_order_particles needs for this
 * schedule and field: two (node, index) pairs per local particle and the
 * digit counts of the sort (about 17 bytes per particle). */
int lpm_order_workspace(const lpm_schedule* sch, const lpm_field* fld, int64_t* bytes);

/* Particles never interact (Sec. 3.2), so the order in which a step launch
 * takes them changes no result; it decides how much the lanes of a wave
 * share wind stencils in the caches.  For the step launch over [step0,
 * step0 + n_steps), whose particles are the local indices [0, n) born
 * before its end, order (device int32[order_capacity], caller-owned;
 * LPM_EINVAL if n exceeds order_capacity) receives in its first n entries: the
 * particles active at step0 grouped by the wind node they are at (by
 * column, j then i, and by level within a column; clamped to the grid;
 * nonuniform levels: by column only), then the particles born in the
 * window in index order, then the inactive ones.  *n_order (host) = n,
 * computed on the host.  Put order and n into st->order and st->n_order of
 * that launch.  The active particles are sorted by node with a radix sort
 * (their order within a node, and that of the inactive ones, is left
 * open).  work: device scratch of
 * lpm_order_workspace bytes, 256-byte aligned.  n < 2^31.
 * Stream-ordered. */
int lpm_order_particles(const lpm_state* st, const lpm_schedule* sch, const lpm_field* fld,
                        int32_t step0, int32_t n_steps, int32_t* order, int64_t order_capacity,
                        int64_t* n_order, void* work, int64_t work_bytes, lpm_stream stream);

/* *bytes (host) = the size of the time-pair copy of one interval of fld
 * (lpm_field_interval): nz * ny * nx nodes of 16 bytes (ncomp 2) or 32
 * bytes (ncomp 3).  LPM_EINVAL unless fld is an LPM_FIELD_NODES field with
 * nt >= 2. */
int lpm_field_interval_bytes(const lpm_field* fld, int64_t* bytes);

/* The wind of a step is linear in time between two weather times (Sec. 3.2),
 * so a step reads the stencil at both times of its field interval.  Writes
 * interval k, [t0 + k dt_field, t0 + (k + 1) dt_field], of fld (layout
 * LPM_FIELD_NODES, nt >= 2, 0 <= k <= nt - 2) into out with both times of
 * each node side by side: per node (u, v) at the interval's start, then at
 * its end (ncomp 2, 16 bytes), or (u, v, w, 0) at the start, then at the
 * end (ncomp 3, 32 bytes), nodes in [ny][nx][nz] order (levels innermost).
 * A step's wind stencil then takes one set of cache lines for both times
 * instead of one per time, and particles of one column share lines at any
 * height (see lpm_order_particles).  out: caller-owned device memory of
 * lpm_field_interval_bytes bytes, 16-byte aligned, not overlapping
 * fld->data.  *packed (host) receives the descriptor of the copy: fld with
 * data = out, layout = LPM_FIELD_TIME_PAIRS and interval = k (nt, t0 and
 * dt_field stay those of fld).  lpm_step_particles,
 * lpm_step_particles_record and lpm_step_ensemble take it for calls all of
 * whose steps interpolate in interval k -- start times in [t_k, t_k+1), and
 * before t_0 for k = 0, from t_k+1 on for k = nt - 2 (where fld clamps) --
 * with results equal to those on fld bitwise, and reject other calls
 * (LPM_EINVAL); the adjoint does not take it.  Stream-ordered. */
int lpm_field_interval(const lpm_field* fld, int32_t k, void* out, lpm_field* packed,
                       lpm_stream stream);

/* Doubles of the static device scratch of lpm_grid_concentration_static
 * (4 Mi = 32 MiB per device): n_nuc * nx * ny * nz may not exceed it. */
#define LPM_STATIC_SCRATCH_DOUBLES (4 * 1024 * 1024)

/* lpm_grid_concentration without the acc_scratch argument, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops
 * or harnesses that forbid allocation).  The FP64 accumulation grid is a
 * static device array of the library, LPM_STATIC_SCRATCH_DOUBLES doubles per
 * device, held from library load to process end; its address on a device is
 * looked up on the first call with that device current.  The call allocates
 * nothing and clears the part of the array it uses before use.  Errors as
 * lpm_grid_concentration, and LPM_EINVAL when n_nuc * nx * ny * nz exceeds
 * LPM_STATIC_SCRATCH_DOUBLES.  Every call on a device shares that device's
 * array: calls on one device that overlap in time (other streams, other host
 * threads) race on it and give wrong grids -- order them on one stream. */
int lpm_grid_concentration_static(const lpm_state* st, const lpm_source* src,
                                  const lpm_schedule* sch, const lpm_physics* ph,
                                  const lpm_grid* grid, int32_t step, float* out,
                                  lpm_stream stream);

/* Bytes of device workspace lpm_grid_records needs for these arguments:
 * per (output step, bin of grid columns) two 64-bit offsets, one int per
 * 2048 particles, and one 20-byte entry (the record and its birth step, in
 * bin order) per particle born by each recorded step (at most
 * 20 n_rec n_local bytes).  0 when n_rec == 0.  Errors: the argument checks
 * of lpm_grid_records that do not involve buffers; LPM_EINVAL also when
 * n_nuc * nz > 6144 (a full grid column of FP64 sums must fit one block's
 * LDS) or n_local >= 2^32. */
int lpm_grid_records_workspace(const lpm_schedule* sch, const lpm_physics* ph,
                               const lpm_grid* grid, int32_t rec_step0,
                               int32_t rec_every, int32_t n_rec, int64_t* bytes);

/* Concentration at every recorded step of rec (lpm_step_particles_record
 * with the same schedule, source, physics, rec_step0, rec_every, n_rec and
 * rec_stride): out[k] = the grid of lpm_grid_concentration after step s_k
 * (Sec. 3.2: activities summed on a rectangular grid every n-th step), the
 * same FP32 contributions summed in FP64 (where one column tile holds more
 * than 8192 records of an output step, in up to eight FP64 partial sums
 * that are added in FP32).  work: caller-owned device
 * scratch, 256-byte aligned, of at least lpm_grid_records_workspace bytes,
 * overwritten; out: device float [n_rec][n_nuc][nz][ny][nx], overwritten
 * (every cell).  Asynchronous on `stream`; no allocation. */
int lpm_grid_records(const float* rec, int64_t rec_stride, int32_t rec_step0,
                     int32_t rec_every, int32_t n_rec, const lpm_source* src,
                     const lpm_schedule* sch, const lpm_physics* ph,
                     const lpm_grid* grid, void* work, int64_t work_bytes,
                     float* out, lpm_stream stream);

/* lpm_grid_records for the records of a launch that took a work order
 * (Sec. 3.2, as lpm_grid_records): record k of queue position q, particle
 * order[q], is the float4 at index k * rec_stride + q and its word last[q]
 * (lpm_step_particles_record with st->order).  Consecutive positions hold
 * particles sorted by wind node, so the binning reads and writes them
 * together.  order: the launch's device int32 work order (4-byte aligned),
 * n_order entries, 0 <= n_order <= n_local <= rec_stride; an entry outside
 * [0, n_local) is skipped.  Workspace and output as for lpm_grid_records;
 * the result equals lpm_grid_records on the same states recorded by
 * particle index, up to the order of the FP64 sums.  Errors: those of
 * lpm_grid_records; LPM_EINVAL for a null, misaligned or too long order. */
int lpm_grid_records_ordered(const float* rec, int64_t rec_stride, int32_t rec_step0,
                             int32_t rec_every, int32_t n_rec, const lpm_source* src,
                             const lpm_schedule* sch, const lpm_physics* ph,
                             const lpm_grid* grid, const int32_t* order, int64_t n_order,
                             void* work, int64_t work_bytes, float* out,
                             lpm_stream stream);

/* Deposited activity so far on the deposition grid (Sec. 2: activity removed
 * from the particles to the surface by dry and wet deposition; Sec. 3.2:
 * summed on a rectangular grid), converted to float and divided by the cell
 * area when dep_grid.density != 0.
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

/* Launch settings of the persistent step kernel.  Results do not depend on
 * them, only the time does.  A wave refills idle lanes from the work queue
 * every `refill_every` steps (1 .. 4096), and only once at least
 * `refill_min` of its 64 lanes are idle or all of them are (1 .. 64; a wave
 * that waits for nearly all its lanes keeps particles released together in
 * one wave, whose lanes then take the same branches).  At most
 * `blocks_per_cu` blocks run per compute unit (0 = as many as fit).  `block`
 * is the number of threads per block: 128, 256 or 512 for ensemble launches;
 * plain launches always use 256. */
typedef struct {
    int32_t refill_every;
    int32_t refill_min;
    int32_t blocks_per_cu;
    int32_t block;
} lpm_launch;

/* Launch settings of later plain step launches (lpm_step_particles[_record])
 * in this process: refill interval, blocks per compute unit and idle lanes
 * before a refill (defaults 24, 0 and 0; refill_min 0 lets the wind decide:
 * 56 idle lanes on a steady field, 40 on a field interpolated in time, the
 * faster settings on the 6 h steady and the 24 h hourly workloads, which
 * differ in how long particles stay).  This setting is the library's
 * only mutable process-wide state; it is read atomically at each launch, so
 * a call from another thread affects launches made after it returns.
 * Ensemble launches carry their own settings in lpm_ensemble. */
int lpm_set_launch(int32_t refill_every, int32_t blocks_per_cu);

/* lpm_set_launch with the number of idle lanes before a refill (1 .. 64, or
 * 0 for the default that depends on the wind). */
int lpm_set_launch_ex(int32_t refill_every, int32_t blocks_per_cu, int32_t refill_min);

/* ---------------------------------------------------------------------------
 * Ensembles: many release scenarios advanced in one persistent launch.
 * Every scenario is a full run of its own (local ids 0 .. n_total - 1, births
 * floor(l * s_release / n_total), Philox key (seed, src.scenario)) whose
 * particles sit at [offset, offset + n_total) of one combined state; the
 * work queue of the step kernel runs over the particles of all scenarios, so
 * scenarios of very different sizes share the device without per-scenario
 * launches.  Each scenario's trajectories equal those of its plain run.
 * ------------------------------------------------------------------------- */
#define LPM_MAX_SCENARIOS 256
#define LPM_SCENARIO_BYTES 96 /* device table bytes per scenario */

typedef struct {
    lpm_source src;  /* release point, rate, wind scale, v_d, Philox scenario key */
    int64_t n_total; /* particles of the scenario */
    int32_t s_release;
    int32_t reserved;
    int64_t offset;  /* first element of the scenario in the combined state */
} lpm_scenario;

/* A prepared ensemble window (filled by lpm_ensemble_prepare). */
typedef struct {
    void* table;        /* device scenario table (caller-owned workspace) */
    int32_t n_scen;
    int32_t n_nuc;
    int32_t step0;
    int32_t n_steps;
    int64_t queue_len;   /* particles of all scenarios born before step0 + n_steps */
    int64_t max_release; /* most particles one scenario releases in the window */
    lpm_launch launch;   /* settings of lpm_step_ensemble: the defaults (24, 56, 0,
                            256) after lpm_ensemble_prepare, the autotuner's pick
                            after lpm_autotune_ensemble; the caller may set them */
    int32_t dep_copies;  /* copies of the scenarios' deposition grids in `dep`
                            (as lpm_accum.dep_copies): 1 after
                            lpm_ensemble_prepare; the caller may set it, up to
                            LPM_MAX_DEP_COPIES */
    int32_t reserved;
} lpm_ensemble;

/* Check the scenarios (n_scen <= LPM_MAX_SCENARIOS, disjoint state ranges
 * within st->capacity) and upload the table of the window [step0, step0 +
 * n_steps) into `table` (device, >= n_scen * LPM_SCENARIO_BYTES bytes,
 * 16-byte aligned); `out` describes it.  Not stream-captured work: call it
 * before capturing release and step into a graph. */
int lpm_ensemble_prepare(const lpm_scenario* scen, int32_t n_scen, const lpm_state* st,
                         const lpm_physics* ph, int32_t step0, int32_t n_steps,
                         void* table, int64_t table_bytes, lpm_ensemble* out,
                         lpm_stream stream);

/* lpm_release_particles for every scenario of a prepared window.  ledgers:
 * device double [n_scen][LPM_LEDGER_SLOTS][LPM_LEDGER_STRIDE]. */
int lpm_release_ensemble(const lpm_state* st, const lpm_ensemble* ens, double* ledgers,
                         lpm_stream stream);

/* lpm_step_particles for every scenario of a prepared window, in one
 * persistent launch.  dep: device double [copies][n_scen][n_nuc][ny][nx] on
 * dep_grid, copies = ens->dep_copies (block b adds into copy b mod copies;
 * the caller adds the copies up); ledgers as for lpm_release_ensemble; ctrl: device uint32
 * [LPM_CTRL_WORDS].  Wind field and physics (K, decay, rain) are shared; the
 * source (rate, wind scale, v_d, key) is per scenario.  n_nuc <= 2. */
int lpm_step_ensemble(const lpm_state* st, const lpm_ensemble* ens, const lpm_field* fld,
                      const lpm_physics* ph, const lpm_grid* dep_grid, double* dep,
                      double* ledgers, uint32_t* ctrl, lpm_stream stream);

/* Launch settings picked by lpm_autotune_ensemble. */
typedef struct {
    lpm_launch launch; /* the chosen setting (also written to ens->launch) */
    double best_ms;    /* median trial time of the chosen setting */
    double worst_ms;   /* median trial time of the slowest setting */
    int32_t n_tried;   /* distinct launches timed */
    int32_t reps;      /* timed trials per setting (the median is kept) */
} lpm_tuning;

/* Autotuner: time the ensemble step over the first `trial_steps` steps of
 * the prepared window for each candidate setting -- queue schedule (refill
 * interval and idle lanes before a refill), threads per block and blocks per
 * compute unit -- `reps` times each (1 .. 15, after one untimed warm-up;
 * candidates that would launch alike, the same schedule and block size on
 * the same number of resident blocks, are timed once, as the first of
 * them), and keep in ens->launch the setting it held on entry if that
 * launches alike with a candidate whose median time is within 6 % of the
 * smallest median (a repeated call switches only for a clear gain), else the
 * first candidate, in a fixed order, whose median time is within 3 % of the
 * smallest (settings that time alike are told apart by the order, not by
 * timing noise; nothing process-wide changes).  It runs release and step on the given buffers, so
 * state, dep, ledgers and ctrl must be reset and the particles released
 * again afterwards.  Synchronises `stream`. */
int lpm_autotune_ensemble(const lpm_state* st, lpm_ensemble* ens,
                          const lpm_scenario* scen, const lpm_field* fld,
                          const lpm_physics* ph, const lpm_grid* dep_grid, double* dep,
                          double* ledgers, uint32_t* ctrl, int32_t trial_steps,
                          int32_t reps, lpm_tuning* out, lpm_stream stream);

/* Friction velocity and inverse Monin-Obukhov length of the surface layer
 * from the vertical stratification (Sec. 2: u* and L computed iteratively
 * from the actual stratification), for kz_kind 3: wind speed U (m/s) at
 * height z_ref (m) over roughness length z0 (m), potential-temperature
 * difference dtheta = theta(z_ref) - theta(z0) (K), mean temperature T0 (K).
 * Monin-Obukhov similarity with the Businger-Dyer gradients (heat: 1 + 5 s
 * stable, (1 - 16 s)^(-1/2) unstable; momentum: 1 + 5 s, (1 - 16 s)^(-1/4))
 * in Paulson's integrated forms, iterated from the neutral solution
 * u* = kappa U / ln(z_ref / z0) (kappa = 0.4, g = 9.81 m/s^2) until inv_L
 * changes by less than 1e-12 relative.  Host-only, synchronous.  Writes
 * *ustar (m/s) and *inv_L (1/m); LPM_EINVAL for invalid input or when the
 * iteration does not converge (e.g. too stable: the bulk Richardson number
 * beyond the critical value of the stable profile, 0.2). */
int lpm_surface_layer(double U, double z_ref, double z0, double dtheta, double T0,
                      double* ustar, double* inv_L);

/* ---------------------------------------------------------------------------
 * Receptor concentrations and their gradient (source inversion)
 *
 * Ground-level concentrations at receptor points are the activities of the
 * airborne particles spread with a Gaussian kernel and summed over the output
 * steps of a whole-run record (lpm_step_particles_record with rec_step0 =
 * rec_every - 1, starting at step 0, every particle released at its birth):
 *
 *   c_r = weight * sum_k sum_p A_p(s_k) G(x_p - x_r, y_p - y_r)
 *                             [N(z_p - z_r) + N(z_p + z_r)],
 *   A_p(s) = a0 m_p sum_n exp(-lambda_n (s + 1 - b_p) dt)   (all nuclides),
 *
 * G the normalised 2-D Gaussian of width sigma_h, N the 1-D Gaussian of
 * width sigma_z (its mirror image below the ground keeps a receptor at the
 * ground seeing the reflected plume), s_k the recorded output steps and
 * weight the time one output step stands for (e.g. rec_every dt).  This is
 * the smooth gridding of a receptor-misfit loss; the activity bookkeeping is
 * that of Sec. 2 and the output steps those of Sec. 3.2.
 * ------------------------------------------------------------------------- */

#define LPM_MAX_RECEPTORS 1024

typedef struct {
    const float* x; /* device, n receptor positions (m) */
    const float* y;
    const float* z; /* height above ground, >= 0 */
    int32_t n;      /* 1 .. LPM_MAX_RECEPTORS */
    float sigma_h;  /* horizontal kernel width (m), > 0 */
    float sigma_z;  /* vertical kernel width (m), > 0 */
    float weight;   /* time weight of one output step (s) */
} lpm_receptors;

/* c_out[n] (device, FP64, overwritten) = receptor concentrations of the n_rec
 * recorded output steps rec_step0 + k rec_every (records stored by particle
 * index, as lpm_step_particles_record stores them without a work order).
 * Asynchronous. */
int lpm_receptor_concentration(const float* rec, int64_t rec_stride, int32_t rec_step0,
                               int32_t rec_every, int32_t n_rec, const lpm_source* src,
                               const lpm_schedule* sch, const lpm_physics* ph,
                               const lpm_receptors* rcp, double* c_out, lpm_stream stream);

/* Bytes of device workspace lpm_receptor_adjoint needs for this field kind,
 * schedule and checkpoint interval (written to *bytes). */
int lpm_adjoint_workspace(const lpm_field* fld, const lpm_schedule* sch, int32_t rec_every,
                          int64_t* bytes);

/* Adjoint of the receptor concentrations (reverse mode along each particle's
 * path, random numbers held fixed): with gbar[n] (device, FP64) = dL/dc_r,
 * grad_out[5] (device, FP64, overwritten) receives dL/dh, dL/dq, dL/ds_w,
 * dL/dv_d (source height, release rate q, wind scale, dry-deposition
 * velocity) and sum_r gbar_r c_r.
 * The record must be the whole-run record of the same source, schedule,
 * field and physics: n_rec output steps s_k = (k + 1) rec_every - 1 of the
 * run over steps [0, n_rec rec_every).  Record k - 1 is the checkpoint from
 * which segment k (steps k rec_every .. (k + 1) rec_every - 1) is recomputed
 * into the workspace, then swept backwards.  A particle that leaves the
 * domain contributes only through the output steps before its exit step
 * (the exit itself does not move with theta).  `work` (device, 16-byte
 * aligned, work_bytes >= lpm_adjoint_workspace) is scratch.  Asynchronous. */
int lpm_receptor_adjoint(const float* rec, int64_t rec_stride, int32_t rec_every, int32_t n_rec,
                         const lpm_source* src, const lpm_schedule* sch, const lpm_field* fld,
                         const lpm_physics* ph, const lpm_receptors* rcp, const double* gbar,
                         double* grad_out, void* work, int64_t work_bytes, lpm_stream stream);

/* Library version string. */
const char* lpm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LPM_H */

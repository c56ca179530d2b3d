// Ensembles of release scenarios (C ABI, host side): the scenario table,
// release of every scenario of a window, one persistent step launch over the
// particles of all scenarios, and the autotuner of its launch settings.
// Every scenario is a full run of its own (Sec. 2: release from a point
// source; Sec. 3.2: the main loop); the step kernels are those of plain runs,
// compiled in ensemble mode (lpm_step_ensemble.hip).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <utility>

#include "lpm.h"
#include "lpm_device.h"
#include "lpm_host.h"

namespace lpm {

// Release of every scenario of an ensemble window: blockIdx.y = scenario.
__global__ __launch_bounds__(kBlock) void release_ensemble_kernel(float* X, float* Y, float* Z,
                                                                  float* M, float* XL, float* YL,
                                                                  const DevScen* scen,
                                                                  double* ledgers, int n_nuc)
{
    const DevScen& d = scen[blockIdx.y];
    const long long l = d.lo + (long long)blockIdx.x * kBlock + threadIdx.x;
    if (l < d.hi) {
        const long long i = d.offset + l;
        X[i] = d.xs;
        Y[i] = d.ys;
        Z[i] = d.h;
        M[i] = 1.0f;
        if (XL) {
            XL[i] = 0.0f;
            YL[i] = 0.0f;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < n_nuc && d.hi > d.lo)
        atomicAdd(ledgers + (long long)blockIdx.y * LPM_LEDGER_SLOTS * LPM_LEDGER_STRIDE +
                      threadIdx.x * 4,
                  d.released);
}

// The work queue of a launch starts empty (a kernel, not a memset: the
// launch may be captured in a graph).
__global__ void clear_queue(uint32_t* ctrl)
{
    if (threadIdx.x < 2) ctrl[LPM_CTRL_QUEUE + threadIdx.x] = 0u;
}

}  // namespace lpm

using namespace lpm_host;

namespace {

static_assert(sizeof(lpm::DevScen) <= LPM_SCENARIO_BYTES, "scenario table entry too large");

constexpr lpm_launch kDefaultLaunch = {24, 56, 0, lpm::kBlock};

int check_launch(const lpm_launch& l)
{
    if (l.refill_every < 1 || l.refill_every > 4096 || l.refill_min < 1 || l.refill_min > 64 ||
        l.blocks_per_cu < 0 || (l.block != 128 && l.block != 256 && l.block != 512))
        return fail(LPM_EINVAL, "launch settings: refill_every in [1, 4096], refill_min in [1, 64], "
                                "blocks_per_cu >= 0, block 128, 256 or 512");
    return LPM_OK;
}

}  // namespace

extern "C" {

int lpm_ensemble_prepare(const lpm_scenario* scen, int32_t n_scen, const lpm_state* st,
                         const lpm_physics* ph, int32_t step0, int32_t n_steps, void* table,
                         int64_t table_bytes, lpm_ensemble* out, lpm_stream stream)
{
    g_msg[0] = 0;
    int rc;
    if (!scen || !st || !out) return fail(LPM_EINVAL, "null argument");
    if ((rc = check_physics(ph))) return rc;
    if (ph->chain || ph->dep_mode || ph->kz_kind == 3)
        return fail(LPM_EINVAL, "ensemble launches do not take chains, stochastic deposition or kz_kind 3");
    if (n_scen < 1 || n_scen > LPM_MAX_SCENARIOS)
        return fail(LPM_EINVAL, "n_scen must be in [1, %d]", LPM_MAX_SCENARIOS);
    if (!table || ((uintptr_t)table & 15u) || table_bytes < (int64_t)n_scen * LPM_SCENARIO_BYTES)
        return fail(LPM_EINVAL, "null, misaligned or small scenario table");
    if (step0 < 0 || n_steps < 1 || (long long)step0 + n_steps > 0x7FFFFFFFll)
        return fail(LPM_EINVAL, "bad step window");
    if (!st->x || !st->y || !st->z || !st->m) return fail(LPM_EINVAL, "null state array");
    if ((st->x_lo == nullptr) != (st->y_lo == nullptr))
        return fail(LPM_EINVAL, "x_lo and y_lo: both or neither");
    // fixed-size host buffers (no allocation, so nothing can throw)
    lpm::DevScen t[LPM_MAX_SCENARIOS];
    std::pair<long long, long long> ranges[LPM_MAX_SCENARIOS];
    long long q = 0, max_rel = 0;
    for (int c = 0; c < n_scen; ++c) {
        const lpm_scenario& e = scen[c];
        if (e.n_total <= 0 || e.n_total > 0xFFFFFFFFll || e.s_release <= 0 || e.offset < 0 ||
            e.offset + e.n_total > st->capacity)
            return fail(LPM_EINVAL, "scenario %d: bad size, release steps or state range", c);
        ranges[c] = {e.offset, e.offset + e.n_total};
        lpm_schedule sch{e.n_total, e.n_total, 0, 1, e.s_release, 0};
        lpm::DevScen& d = t[c];
        memset(&d, 0, sizeof d);
        d.qbase = q;
        d.offset = e.offset;
        d.n_total = e.n_total;
        d.s_release = e.s_release;
        d.i_hi = first_local_born_at_or_after(&sch, (long long)step0 + n_steps);
        d.lo = first_local_born_at_or_after(&sch, step0);
        d.hi = d.i_hi;
        const double a0 = a0_of(&e.src, &sch, ph);
        d.released = a0 * (double)(d.hi - d.lo);
        d.a0 = (float)a0;
        d.wscale = (float)e.src.wind_scale;
        if (e.src.v_d > 0.0 && ph->h_s > 0.0) {
            d.dry_c1 = (float)(2.0 * e.src.v_d / ph->h_s);
            d.dry_c2 = (float)(2.0 * e.src.v_d / (ph->h_s * ph->h_s));
        }
        d.xs = (float)e.src.xs; d.ys = (float)e.src.ys; d.h = (float)e.src.h;
        d.key1 = e.src.scenario;
        q += d.i_hi;
        if (d.hi - d.lo > max_rel) max_rel = d.hi - d.lo;
    }
    std::sort(ranges, ranges + n_scen);
    for (int k = 1; k < n_scen; ++k)
        if (ranges[k].first < ranges[k - 1].second)
            return fail(LPM_EINVAL, "scenario state ranges overlap");
    if (hipMemcpyAsync(table, t, sizeof(lpm::DevScen) * n_scen, hipMemcpyHostToDevice,
                       (hipStream_t)stream) != hipSuccess ||
        hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        return hip_status("lpm_ensemble_prepare");
    out->table = table;
    out->n_scen = n_scen;
    out->n_nuc = ph->n_nuc;
    out->step0 = step0;
    out->n_steps = n_steps;
    out->queue_len = q;
    out->max_release = max_rel;
    out->launch = kDefaultLaunch;
    out->dep_copies = 1;
    out->reserved = 0;
    return LPM_OK;
}

int lpm_release_ensemble(const lpm_state* st, const lpm_ensemble* ens, double* ledgers,
                         lpm_stream stream)
{
    g_msg[0] = 0;
    if (!st || !ens || !ens->table || !ledgers) return fail(LPM_EINVAL, "null argument");
    if (ens->n_scen < 1 || ens->n_scen > LPM_MAX_SCENARIOS || ens->n_nuc < 1 || ens->n_nuc > 4)
        return fail(LPM_EINVAL, "ensemble not prepared");
    if (ens->max_release <= 0) return LPM_OK;
    hipLaunchKernelGGL(lpm::release_ensemble_kernel,
                       dim3(blocks_for(ens->max_release), (unsigned)ens->n_scen), dim3(lpm::kBlock),
                       0, (hipStream_t)stream, st->x, st->y, st->z, st->m, st->x_lo, st->y_lo,
                       (const lpm::DevScen*)ens->table, ledgers, ens->n_nuc);
    return hip_status("lpm_release_ensemble");
}

// lpm_step_ensemble; with `plan`, only validates and stores in *plan the
// number of blocks the step launch would take (nothing is launched).
static int step_ensemble_impl(const lpm_state* st, const lpm_ensemble* ens,
                              const lpm_field* fld, const lpm_physics* ph,
                              const lpm_grid* dep_grid, double* dep, double* ledgers,
                              uint32_t* ctrl, lpm_stream stream, unsigned* plan)
{
    g_msg[0] = 0;
    int rc;
    if (!st || !ens || !ens->table || !dep || !ledgers || !ctrl) return fail(LPM_EINVAL, "null argument");
    if (((uintptr_t)dep & 7u) || ((uintptr_t)ledgers & 7u) || ((uintptr_t)ctrl & 7u))
        return fail(LPM_EINVAL, "misaligned accumulator");
    if ((rc = check_physics(ph)) || (rc = check_grid(dep_grid, true)) ||
        (rc = check_launch(ens->launch)))
        return rc;
    if (ens->dep_copies < 0 || ens->dep_copies > LPM_MAX_DEP_COPIES)
        return fail(LPM_EINVAL, "dep_copies must be in [0, %d]", LPM_MAX_DEP_COPIES);
    if (ph->n_nuc != ens->n_nuc) return fail(LPM_EINVAL, "physics and ensemble n_nuc differ");
    if (ph->n_nuc > 2) return fail(LPM_EINVAL, "ensemble launches support one or two nuclides");
    if (ph->chain || ph->dep_mode || ph->kz_kind == 3)
        return fail(LPM_EINVAL, "ensemble launches do not take chains, stochastic deposition or kz_kind 3");
    if ((double)dep_grid->nx * dep_grid->ny * ens->n_scen >= 2147483647.0)
        return fail(LPM_EINVAL, "scenarios x deposition cells must stay below 2^31 - 1");
    if (fld && fld->z_levels) return fail(LPM_EINVAL, "ensemble launches need uniform levels");
    lpm::StepConst p;
    memset(&p, 0, sizeof p);
    if ((rc = fill_field(p, fld))) return rc;
    fill_physics(p, ph);
    if ((rc = check_field_steps(p, fld, ens->step0, ens->n_steps))) return rc;
    fill_depgrid(p, *dep_grid);
    p.refill_every = ens->launch.refill_every;
    p.refill_min = ens->launch.refill_min;
    p.rec_every = 1;
    p.X = st->x; p.Y = st->y; p.Z = st->z; p.M = st->m;
    p.XL = st->x_lo; p.YL = st->y_lo;
    if ((p.XL == nullptr) != (p.YL == nullptr))
        return fail(LPM_EINVAL, "x_lo and y_lo: both or neither");
    if (st->order) return fail(LPM_EINVAL, "ensemble launches take no work order");
    p.step0 = ens->step0;
    p.step_end = ens->step0 + ens->n_steps;
    p.i_hi = ens->queue_len;
    p.scen = (const lpm::DevScen*)ens->table;
    p.n_scen = ens->n_scen;
    p.dep = dep; p.ledger = ledgers; p.ctrl = ctrl;
    p.dep_copies = ens->dep_copies > 1 ? ens->dep_copies : 1;
    if (plan) *plan = 0;
    if (p.i_hi <= 0) return LPM_OK;
    // wet deposition, or dry deposition of any scenario (v_d is per scenario
    // and only known to the device table here), selects the depositing variant
    const bool dep_any = p.L0 > 0.0f || ph->h_s > 0.0;
    hipStream_t s = (hipStream_t)stream;
    if (!plan) hipLaunchKernelGGL(lpm::clear_queue, dim3(1), dim3(64), 0, s, ctrl);
    const int bpc = ens->launch.blocks_per_cu;
    const bool time = fld->nt > 1;
    switch (ens->launch.block) {
    case 128:
        launch_ensemble<128>(fld->ncomp, time, ph->n_nuc, ph->kz_kind, dep_any,
                             (unsigned)((p.i_hi + 127) / 128), s, p, bpc, plan);
        break;
    case 512:
        launch_ensemble<512>(fld->ncomp, time, ph->n_nuc, ph->kz_kind, dep_any,
                             (unsigned)((p.i_hi + 511) / 512), s, p, bpc, plan);
        break;
    default:
        launch_ensemble<256>(fld->ncomp, time, ph->n_nuc, ph->kz_kind, dep_any,
                             (unsigned)((p.i_hi + 255) / 256), s, p, bpc, plan);
        break;
    }
    return plan ? LPM_OK : hip_status("lpm_step_ensemble");
}

int lpm_step_ensemble(const lpm_state* st, const lpm_ensemble* ens, const lpm_field* fld,
                      const lpm_physics* ph, const lpm_grid* dep_grid, double* dep,
                      double* ledgers, uint32_t* ctrl, lpm_stream stream)
{
    return step_ensemble_impl(st, ens, fld, ph, dep_grid, dep, ledgers, ctrl, stream, nullptr);
}

int lpm_autotune_ensemble(const lpm_state* st, lpm_ensemble* ens, const lpm_scenario* scen,
                          const lpm_field* fld, const lpm_physics* ph, const lpm_grid* dep_grid,
                          double* dep, double* ledgers, uint32_t* ctrl, int32_t trial_steps,
                          int32_t reps, lpm_tuning* out, lpm_stream stream)
{
    g_msg[0] = 0;
    if (!st || !ens || !scen || !out) return fail(LPM_EINVAL, "null argument");
    if (trial_steps < 1 || trial_steps > ens->n_steps) return fail(LPM_EINVAL, "bad trial_steps");
    if (reps < 1 || reps > 15) return fail(LPM_EINVAL, "reps must be in [1, 15]");
    hipStream_t s = (hipStream_t)stream;
    // Candidates: queue schedules (refill interval, idle lanes before a
    // refill) x threads per block x resident waves per compute unit (as many
    // as fit, 12, 8), the last as blocks per CU of that block size.
    const int schedules[][2] = {{1, 1}, {4, 1}, {16, 32}, {16, 64}, {24, 56}};
    const int blocks[] = {128, 256, 512};
    const int waves[] = {0, 12, 8};
    lpm_launch cand[5 * 3 * 3];
    int n_cand = 0;
    for (const auto& r : schedules)
        for (int b : blocks)
            for (int w : waves) {
                const int bpc = w == 0 ? 0 : std::max(1, w / (b / 64));
                bool dup = false;
                for (int j = 0; j < n_cand; ++j)
                    dup |= cand[j].refill_every == r[0] && cand[j].refill_min == r[1] &&
                           cand[j].block == b && cand[j].blocks_per_cu == bpc;
                if (!dup) cand[n_cand++] = lpm_launch{r[0], r[1], bpc, b};
            }
    lpm_ensemble trial;
    int rc = lpm_ensemble_prepare(scen, ens->n_scen, st, ph, ens->step0, trial_steps, ens->table,
                                  (int64_t)ens->n_scen * LPM_SCENARIO_BYTES, &trial, stream);
    if (rc) return rc;
    trial.dep_copies = ens->dep_copies;  // the trials deposit like the real launches
    // Settings that launch alike (the same block size and schedule on the
    // same number of resident blocks: a wave count at or above what fits is
    // "as many as fit") are timed once, as the first of them.
    int incumbent = -1;
    {
        unsigned grid_of[5 * 3 * 3];
        int kept = 0;
        for (int c = 0; c < n_cand && !rc; ++c) {
            trial.launch = cand[c];
            rc = step_ensemble_impl(st, &trial, fld, ph, dep_grid, dep, ledgers, ctrl, stream,
                                    &grid_of[kept]);
            bool dup = false;
            for (int j = 0; j < kept && !rc; ++j)
                dup |= cand[j].refill_every == cand[c].refill_every &&
                       cand[j].refill_min == cand[c].refill_min &&
                       cand[j].block == cand[c].block && grid_of[j] == grid_of[kept];
            if (!rc && !dup) cand[kept++] = cand[c];
        }
        n_cand = kept;
        // the caller's setting on entry (for instance an earlier pick): the
        // candidate it launches alike with, if any
        if (!rc && check_launch(ens->launch) == LPM_OK) {
            trial.launch = ens->launch;
            unsigned g = 0;
            if (step_ensemble_impl(st, &trial, fld, ph, dep_grid, dep, ledgers, ctrl, stream,
                                   &g) == LPM_OK)
                for (int j = 0; j < n_cand && incumbent < 0; ++j)
                    if (cand[j].refill_every == ens->launch.refill_every &&
                        cand[j].refill_min == ens->launch.refill_min &&
                        cand[j].block == ens->launch.block && grid_of[j] == g)
                        incumbent = j;
        }
        g_msg[0] = 0;
    }
    if (rc) {
        lpm_ensemble again;
        (void)lpm_ensemble_prepare(scen, ens->n_scen, st, ph, ens->step0, ens->n_steps,
                                   ens->table, (int64_t)ens->n_scen * LPM_SCENARIO_BYTES, &again,
                                   stream);
        return rc;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return hip_status("lpm_autotune_ensemble");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_status("lpm_autotune_ensemble");
    }
    double med_of[5 * 3 * 3];
    int tried = 0;
    for (int c = 0; c < n_cand && !rc; ++c) {
        trial.launch = cand[c];
        float t[16];
        for (int rep = 0; rep <= reps && !rc; ++rep) {  // repetition 0 warms up
            if ((rc = lpm_release_ensemble(st, &trial, ledgers, stream))) break;
            if (hipEventRecord(e0, s) != hipSuccess) { rc = fail(LPM_EHIP, "lpm_autotune_ensemble: hipEventRecord failed"); break; }
            if ((rc = lpm_step_ensemble(st, &trial, fld, ph, dep_grid, dep, ledgers, ctrl, stream))) break;
            if (hipEventRecord(e1, s) != hipSuccess) { rc = fail(LPM_EHIP, "lpm_autotune_ensemble: hipEventRecord failed"); break; }
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t[rep], e0, e1) != hipSuccess) {
                rc = hip_status("lpm_autotune_ensemble");
                break;
            }
        }
        if (rc) break;
        std::sort(t + 1, t + 1 + reps);
        med_of[c] = reps % 2 ? t[1 + reps / 2] : 0.5 * (t[reps / 2] + t[1 + reps / 2]);
        ++tried;
    }
    // The pick is the caller's setting if it times within kKeep of the
    // fastest (a repeated call switches only for a clear gain), else the
    // first candidate (in the fixed order above) whose median is within kTie
    // of the fastest: settings that time alike are told apart by the order,
    // not by timing noise, so the pick repeats.
    constexpr double kTie = 0.03, kKeep = 0.06;
    double best = 1e300, worst = 0.0;
    for (int c = 0; c < tried; ++c) {
        best = std::min(best, med_of[c]);
        worst = std::max(worst, med_of[c]);
    }
    lpm_launch pick = ens->launch;
    double pick_ms = best;
    if (incumbent >= 0 && incumbent < tried && med_of[incumbent] <= best * (1.0 + kKeep)) {
        pick = cand[incumbent];
        pick_ms = med_of[incumbent];
    } else {
        for (int c = 0; c < tried; ++c)
            if (med_of[c] <= best * (1.0 + kTie)) {
                pick = cand[c];
                pick_ms = med_of[c];
                break;
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the caller's window back into the table (also after a failed trial)
    lpm_ensemble again;
    const int rc2 = lpm_ensemble_prepare(scen, ens->n_scen, st, ph, ens->step0, ens->n_steps,
                                         ens->table, (int64_t)ens->n_scen * LPM_SCENARIO_BYTES,
                                         &again, stream);
    if (rc) return rc;
    if (rc2) return rc2;
    ens->launch = pick;
    out->launch = pick;
    out->best_ms = pick_ms;
    out->worst_ms = worst;
    out->n_tried = tried;
    out->reps = reps;
    return LPM_OK;
}

}  // extern "C"

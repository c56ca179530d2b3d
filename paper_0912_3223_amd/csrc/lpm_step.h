// The persistent particle-step kernel of liblpm (gfx950), shared by the
// translation units that instantiate it: plain runs (one slice of the
// compile-time variants per unit, built in parallel) and ensemble runs.
//
// Each lane takes particles from a work queue, loads a particle's state once,
// advances it through the window in registers and stores it once.  Random
// numbers come from Philox in registers and the wind is gathered from the
// L2/MALL-resident field.  Deposition is aggregated in four levels before it
// reaches HBM: per lane while the particle stays in one cell quad
// (registers), a per-wave staging list of quads, a per-wave LDS hash table of
// cells (FP64 LDS atomics), and once per table entry into the FP64 grid.  The
// ledger is reduced per block before one atomic per entry into one of
// LPM_LEDGER_SLOTS spread-out slots.
#pragma once

#include <hip/hip_runtime.h>

#include <limits.h>
#include <math.h>
#include <stdint.h>

#include "lpm.h"
#include "lpm_device.h"

namespace lpm {
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int NNUC, int LOG2_SLOTS>
struct WaveTable {
    static constexpr int kSlots = 1 << LOG2_SLOTS;
    static constexpr int kShift = 32 - LOG2_SLOTS;
    static constexpr int kProbes = 8;
    int* key;      // [kSlots]: 0 = empty, else cell + 1
    double* val;   // [NNUC][kSlots]
    int* used;     // slots taken
    // A key is scen * plane + cell; scenario scen's grid starts at
    // scen * NNUC * plane (a plain launch has scen = 0).
    __device__ static double* at(double* grid, long long plane, int key, int n)
    {
        const unsigned sc = (unsigned)key / (unsigned)plane;
        return grid + (long long)sc * (NNUC - 1) * plane + (long long)n * plane + key;
    }

    __device__ void init(int lane)
    {
        for (int t = lane; t < kSlots; t += 64) {
            key[t] = 0;
#pragma unroll
            for (int n = 0; n < NNUC; ++n) val[n * kSlots + t] = 0.0;
        }
        if (lane == 0) {
            *used = 0;
            *sn = 0;
        }
    }

    __device__ void add(int cell, const float (&v)[NNUC], double* grid, long long plane)
    {
        unsigned h = ((unsigned)cell * 2654435761u) >> kShift;
        for (int probe = 0; probe < kProbes; ++probe) {
            const int old = atomicCAS(&key[h], 0, cell + 1);
            if (old == 0 || old == cell + 1) {
                if (old == 0) atomicAdd(used, 1);
#pragma unroll
                for (int n = 0; n < NNUC; ++n)
                    if (v[n] != 0.0f) atomicAdd(&val[n * kSlots + h], (double)v[n]);
                return;
            }
            h = (h + 1) & (kSlots - 1);
        }
#pragma unroll
        for (int n = 0; n < NNUC; ++n)
            if (v[n] != 0.0f) atomicAdd(at(grid, plane, cell, n), (double)v[n]);
    }

    // Called by all lanes of the wave at the same point.
    __device__ void flush(int lane, double* grid, long long plane)
    {
        __builtin_amdgcn_wave_barrier();
        for (int t = lane; t < kSlots; t += 64) {
            const int k = atomicExch(&key[t], 0);
            if (k == 0) continue;
#pragma unroll
            for (int n = 0; n < NNUC; ++n) {
                const double v = atomicExch(&val[n * kSlots + t], 0.0);
                if (v != 0.0) atomicAdd(at(grid, plane, k - 1, n), v);
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) atomicExch(used, 0);
        __builtin_amdgcn_wave_barrier();
    }

    __device__ void flush_if_half_full(int lane, double* grid, long long plane)
    {
        // one broadcast LDS read (not 64 same-address atomics)
        const int u = __hip_atomic_load(used, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        if (__builtin_amdgcn_readfirstlane(u) > kSlots / 2) flush(lane, grid, plane);
    }

    // Staging list in front of the table.  A particle that moves to another
    // cell quad hands over its quad (origin and the four corner sums) in
    // whatever lanes happen to do so in that step, a few of the wave's 64:
    // hashing its corners there would run the probe loops with most lanes
    // masked off.  Instead the quad is appended to a per-wave list (one
    // ballot and a prefix count for all of them), and the whole wave expands
    // the quads into corners and inserts them when the list fills up.
    static constexpr int kStage = 128;                // quads
    static constexpr int kDrainAt = kStage - 64;      // room for every lane
    int* sq;       // [3][kStage]: i0, j0, key base of each quad
    float* sval;   // [4 NNUC][kStage]: corner sums, corner-major per nuclide
    int* sn;       // quads staged

    // Called by the active lanes together; lanes with has = false only take
    // part in the count.  Returns false (nothing staged) when the list is
    // full, and the caller inserts directly.
    __device__ bool stage(bool has, int i0, int j0, int kb, const float (&acc)[NNUC][4])
    {
        const unsigned long long m = __ballot(has);
        if (m == 0ull) return true;
        const int lane = __lane_id();
        const int cnt = __popcll(m);
        const int base = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(sn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT));
        if (base + cnt > kStage) return false;  // never: see the drain points
        if (has) {
            const int pos = base + __popcll(m & ((1ull << lane) - 1ull));
            sq[pos] = i0;
            sq[kStage + pos] = j0;
            sq[2 * kStage + pos] = kb;
#pragma unroll
            for (int n = 0; n < NNUC; ++n)
#pragma unroll
                for (int c = 0; c < 4; ++c) sval[(4 * n + c) * kStage + pos] = acc[n][c];
        }
        if (lane == __ffsll((long long)m) - 1)
            __hip_atomic_store(sn, base + cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        return true;
    }

    // Called by all lanes of the wave at the same point: inserts the staged
    // quads' corners (ncorner = 1 for nearest-cell deposition) when at least
    // at_least quads are staged.
    __device__ bool drain(int lane, double* grid, long long plane, int at_least, int ncorner,
                          int dnx, int dny)
    {
        const int n = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(sn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT));
        if (n < at_least || n == 0) return false;
        __builtin_amdgcn_wave_barrier();
        // lane -> (quad, corner): 64 / ncorner quads per pass
        const int per = 64 / ncorner;
        const int c = lane % ncorner;
        for (int e = lane / ncorner; e < n; e += per) {
            const int ii = sq[e] + (c & 1), jj = sq[kStage + e] + (c >> 1);
            if (ii < 0 || jj < 0 || ii >= dnx || jj >= dny) continue;
            float v[NNUC];
#pragma unroll
            for (int q = 0; q < NNUC; ++q) v[q] = sval[(4 * q + c) * kStage + e];
            add(sq[2 * kStage + e] + jj * dnx + ii, v, grid, plane);
        }
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) __hip_atomic_store(sn, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        __builtin_amdgcn_wave_barrier();
        return true;
    }
};

// 2^TL cells per wave: 128, or 256 in the variants that run at three waves
// per SIMD, whose blocks have the LDS for it.  A wave empties its table into
// the FP64 grid when half of it is taken; where the plume is under rain
// every particle deposits every step and those global atomics, on the same
// cells from every wave, are what the step waits for -- a larger table
// flushes less often.
template <int NNUC, int TL = 7>
using DepTable = WaveTable<NNUC, TL>;

// Per-thread deposition while the particle stays in one grid cell (nearest
// cell) or above one cell quad (cloud-in-cell): partial sums of the corner
// weights times the deposited activity, flushed to the wave's table when the
// cell changes and when the particle stops.
template <int NNUC, int TL = 7>
struct Dwell {
    int i0 = INT_MIN, j0 = 0;
    float acc[NNUC][4];

    int key_base = 0;  // scenario * plane in an ensemble launch

    __device__ void flush(const StepConst& p, DepTable<NNUC, TL>& tab, long long plane)
    {
        // A lane stages at most one quad between two drain points of its wave
        // (the kernel drains whenever 64 free entries are not left), so the
        // list cannot overflow; if it ever did, the error word says so.
        const bool any = i0 != INT_MIN;
        if (!tab.stage(any, i0, j0, key_base, acc) && any)
            atomicOr(p.ctrl + LPM_CTRL_ERR, 2u);
        i0 = INT_MIN;
    }

    // Deposited activities d[n] (already scaled) at (x, y).  Cell index and
    // weights in float: one FMA per axis (the grid origin folded into the
    // offset), accurate to ~3e-5 of a cell 50 km from the origin, where the
    // float position itself is already uncertain by more (4 mm of 250 m).
    __device__ void add(const StepConst& p, DepTable<NNUC, TL>& tab, long long plane, float x,
                        float y, const float (&d)[NNUC])
    {
        const float fx = fmaf(x, p.d_inv_dx, p.d_cx);
        const float fy = fmaf(y, p.d_inv_dy, p.d_cy);
        const float ix = floorf(fx), iy = floorf(fy);
        // the cell (quad) must touch the grid; false for NaN
        if (!(ix >= -1.0f && iy >= -1.0f && ix < p.d_fnx && iy < p.d_fny)) return;
        const int ci = (int)ix, cj = (int)iy;
        if (ci != i0 || cj != j0) {
            flush(p, tab, plane);
            i0 = ci;
            j0 = cj;
#pragma unroll
            for (int n = 0; n < NNUC; ++n)
                acc[n][0] = acc[n][1] = acc[n][2] = acc[n][3] = 0.0f;
        }
        // nearest cell: all weight on corner 0 (the drain reads only that
        // corner then), the same code path as cloud in cell
        const float wx = p.dmode == 0 ? 0.0f : fx - ix, wy = p.dmode == 0 ? 0.0f : fy - iy;
        const float w00 = (1.0f - wx) * (1.0f - wy), w10 = wx * (1.0f - wy);
        const float w01 = (1.0f - wx) * wy, w11 = wx * wy;
#pragma unroll
        for (int n = 0; n < NNUC; ++n) {
            acc[n][0] = fmaf(d[n], w00, acc[n][0]);
            acc[n][1] = fmaf(d[n], w10, acc[n][1]);
            acc[n][2] = fmaf(d[n], w01, acc[n][2]);
            acc[n][3] = fmaf(d[n], w11, acc[n][3]);
        }
    }
};

// Seconds of exposure over one step to a loss rate r >= 0: the activity
// present at the start of the step, integrated over the step with its decay
// and deposition, is that activity times (1 - exp(-r dt)) / r (dt for r = 0).
// For r dt < 2^-7 the Taylor series to (r dt)^3 is exact to float rounding
// (the next term, (r dt)^4 / 120, is below 2^-31 of the result); larger rates
// take the library expm1f.
__device__ __forceinline__ float air_seconds(float r, float dt)
{
    const float x = r * dt;
    if (x < 0.0078125f)
        return dt * fmaf(x, fmaf(x, fmaf(x, -1.0f / 24.0f, 1.0f / 6.0f), -0.5f), 1.0f);
    return -expm1f(-x) / r;
}

// Per-lane ledger partials: deposited, decayed, exited per nuclide, the
// particle-steps, and (general kernels, KZ == 4) the ingrowth of each nuclide
// of a decay chain, booked into its "released" entry.  The light kernels
// (KZ < 4) touch them only when a lane takes or lets go of a particle:
// deposition is summed per particle in float (`Book`), and the decayed
// activity follows from the particle's activity when taken minus its
// activity when let go, minus what it deposited or carried out of the area
// (the per-step losses telescope: each step takes A (1 - exp(-(lambda + k)
// dt)) from the activity A = a0 m exp(-lambda age) it starts with).
template <int NNUC, int KZ>
struct Ledger {
    static constexpr int kSize = 3 * NNUC + 1 + (KZ == 4 ? NNUC : 0);
    __device__ static constexpr int offset(int q)
    {
        return q < 3 * NNUC ? (q / 3) * 4 + 1 + q % 3
                            : (q == 3 * NNUC ? LPM_LEDGER_PSTEPS : (q - 3 * NNUC - 1) * 4);
    }
};

// Where a lane keeps its ledger partials: in registers (general kernels,
// which add every step, and ensembles, whose lanes hold partials of one
// scenario at a time), or -- plain light kernels, which add only when a lane
// takes or lets go of a particle -- in a per-wave FP64 array in LDS (LDS
// atomics), which keeps 14 VGPRs of doubles out of the register budget.
template <int NNUC, int KZ, bool SHARED>
struct LedgerAcc {
    static constexpr int kSize = Ledger<NNUC, KZ>::kSize;
    double reg[SHARED ? 1 : kSize];
    double* wave;  // [kSize] in LDS when SHARED

    __device__ void add(int q, double v)
    {
        if constexpr (SHARED) atomicAdd(wave + q, v);
        else reg[q] += v;
    }
};

// ---------------------------------------------------------------------------
// One time step of one particle (Sec. 3.2 main loop; Eqs. 1-3).  Returns 1
// when the particle left the area, 2 when it became non-finite, 3 when it was
// removed by stochastic deposition, else 0.  KZ == 4 is the general kernel:
// K_z kind at run time (including Eq. 3 with stability), decay chains and
// stochastic deposition.
// ---------------------------------------------------------------------------
template <int NCOMP, int TIME, bool LEVELS, int NNUC, int KZ, bool DEP, bool ENS, int TL>
__device__ __forceinline__ int advance(const StepConst& p, const float* wt_tab,
                                       const SrcVals& sv,
                                       DepTable<NNUC, TL>& tab, long long plane, uint32_t gid,
                                       int b, int s, float& x, float& y, float& z, float& m,
                                       float& xl, float& yl,
                                       LedgerAcc<NNUC, KZ, KZ != 4 && !ENS>& led,
                                       float (&bdep)[NNUC], Dwell<NNUC, TL>& dw)
{
    const float age = (float)(s - b) * p.dt;
    // wind sample, random numbers, diffusivity, move and fold
    float xn, yn, zn;
    motion<NCOMP, TIME, LEVELS, KZ, !ENS>(p, sv.wscale, sv.key1, gid, s, x, y, z, xl, yl, xn, yn,
                                          zn, wt_tab);
    // decay factors at the start of the step
    float D[NNUC];
#pragma unroll
    for (int n = 0; n < NNUC; ++n) D[n] = __builtin_amdgcn_exp2f(-p.lam_l2e[n] * age);
    // deposition rate at the new position (Sec. 2)
    const float k = DEP ? deposition_rate(p, sv.dry_c1, sv.dry_c2, xn, yn, zn) : 0.0f;
    float mn = deposit_mass(m, k, p.dt);
    // decay and deposition of each nuclide's activity this step
    float dsum[NNUC];
    bool removed = false;
    if constexpr (KZ == 4) {
        // Over the step nuclide n spends S_n activity-seconds in the air
        // (activity times surviving mass, integrated): k S_n deposits,
        // lambda_n S_n decays and lambda_{n+1} S_n grows into the daughter of
        // a chain.  With stochastic deposition the particle stays whole and is
        // removed at the end of the step with probability 1 - exp(-k dt).
        const float kk = p.dep_mode ? 0.0f : k;
        if (p.dep_mode) {
            mn = m;
            if (k > 0.0f)
                removed = removal_uniform<!ENS>(gid, (uint32_t)s, p.key0, sv.key1) <=
                          -expm1_neg(-k * p.dt);
        }
        float DG[NNUC];
#pragma unroll
        for (int j = 0; j < NNUC; ++j) {
            const float r = p.lam[j] + kk;
            DG[j] = D[j] * (r > 0.0f ? -expm1_neg(-r * p.dt) * __builtin_amdgcn_rcpf(r) : p.dt);
        }
#pragma unroll
        for (int n = 0; n < NNUC; ++n) {
            float sa = 0.0f, se = 0.0f;
#pragma unroll
            for (int j = 0; j <= n; ++j) {
                sa = fmaf(p.bc[n][j], DG[j], sa);
                se = fmaf(p.bc[n][j], D[j] * p.edec[j], se);
            }
            const float S = sv.a0 * m * sa;
            const float dep = removed ? sv.a0 * m * se : kk * S;
            dsum[n] = dep * p.dscale;
            led.add(3 * n + 0, (double)dep);
            led.add(3 * n + 1, (double)(p.lam[n] * S));
            if (n + 1 < NNUC && p.chain) led.add(3 * NNUC + 2 + n, (double)(p.lam[n + 1] * S));
        }
        if (removed) mn = 0.0f;
    } else if constexpr (DEP) {
        // deposited this step: k times the activity-seconds in the air, the
        // activity a0 m D at the start of the step times air_seconds(lambda + k)
        // (no branch on k: lanes with and without deposition share the wave)
#pragma unroll
        for (int n = 0; n < NNUC; ++n) {
            const float dep = sv.a0 * m * D[n] * k * air_seconds(p.lam[n] + k, p.dt);
            dsum[n] = dep * p.dscale;
            bdep[n] += dep;
        }
    }
    if (DEP && k > 0.0f) dw.add(p, tab, plane, xn, yn, dsum);
    x = xn;
    y = yn;
    z = zn;
    m = mn;
    if (!(__builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z) &&
          __builtin_isfinite(m)))
        return 2;
    if (removed) return 3;
    // leaving the simulated area inactivates the particle
    if (p.bounded && (x < p.X0 || x >= p.X1 || y < p.Y0 || y >= p.Y1)) {
#pragma unroll
        for (int n = 0; n < NNUC; ++n) {
            float se = D[n] * p.edec[n];
            if constexpr (KZ == 4) {
                se = 0.0f;
#pragma unroll
                for (int j = 0; j <= n; ++j) se = fmaf(p.bc[n][j], D[j] * p.edec[j], se);
            }
            const double out = (double)(sv.a0 * m * se);
            led.add(3 * n + 2, out);
            // light kernels: what leaves the area did not decay
            if constexpr (KZ != 4) led.add(3 * n + 1, -out);
        }
        m = 0.0f;
        return 1;
    }
    return 0;
}

// Adds one lane's ledger partials into a ledger slot (ensemble launches,
// where lanes may hold different scenarios).
template <int NNUC, int KZ>
__device__ __forceinline__ void lane_ledger(LedgerAcc<NNUC, KZ, false>& led, double* slot)
{
#pragma unroll
    for (int q = 0; q < Ledger<NNUC, KZ>::kSize; ++q) {
        if (led.reg[q] != 0.0) atomicAdd(slot + Ledger<NNUC, KZ>::offset(q), led.reg[q]);
        led.reg[q] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// Persistent step kernel.  The grid is sized to the resident capacity; every
// lane takes particles from a queue of work indices (one atomic per wave and
// refill) and carries each through the window, so a lane whose particle
// leaves the area or stops picks up the next one.  Lanes of a wave therefore
// hold particles at different steps; what they do per step is exactly one
// call of advance().  In an ensemble launch (ENS) the queue runs over the
// particles of all scenarios, each lane looks up its particle's scenario, and
// deposition and ledger go to that scenario's accumulators.
// ---------------------------------------------------------------------------
// Blocks per CU the compiler must fit: the lighter variants are held to 128
// VGPRs (4 waves per SIMD), which beats the 3 waves the register allocation
// picks by itself even where it spills a few registers (1e6-particle run:
// 7.3 vs 7.8 ms; 64-scenario ensemble: 94 vs 103 ms); heavier variants keep
// the default.
template <int NCOMP, int TIME, int NNUC, int KZ, bool DEP, bool ENS>
constexpr int step_min_blocks()
{
    return (NCOMP == 3) + (TIME != 0) + DEP + (NNUC >= 3) + (KZ == 4) <= 1 ? 4 : 1;
}

// BLOCK: threads per block (a multiple of 64); the second launch bound is the
// number of waves per SIMD the register allocation must allow.  TIME: 0 a
// steady field, 1 two time nodes (the node layout, or a time-pair copy
// recognised at run time), 2 a time-pair copy.
template <int BLOCK, int NCOMP, int TIME, bool LEVELS, int NNUC, int KZ, bool DEP, bool ENS>
__global__ __launch_bounds__(BLOCK, (step_min_blocks<NCOMP, TIME, NNUC, KZ, DEP, ENS>())) void step_kernel(const StepConst pk)
{
    static_assert(BLOCK % 64 == 0 && BLOCK >= 64 && BLOCK <= 1024, "block of whole waves");
    constexpr int kWaves = BLOCK / 64;
    // The launch constants live in LDS: kept in SGPRs across the persistent
    // loop they outnumber the scalar registers and spill to VGPR lanes.
    __shared__ StepConst pc;
    __shared__ long long scen_qbase[ENS ? LPM_MAX_SCENARIOS + 1 : 1];
    for (unsigned w = threadIdx.x; w < sizeof(StepConst) / 4; w += BLOCK)
        reinterpret_cast<uint32_t*>(&pc)[w] = reinterpret_cast<const uint32_t*>(&pk)[w];
    if constexpr (ENS) {
        for (int c = threadIdx.x; c <= pk.n_scen; c += BLOCK)
            scen_qbase[c] = c < pk.n_scen ? pk.scen[c].qbase : pk.i_hi;
    }
    // time weights of the launch's steps on a time-pair copy (one interval)
    constexpr bool kWtTab = TIME == 2 && NCOMP == 2;
    __shared__ float wt_lds[kWtTab ? kWtTable : 1];
    const bool use_tab = kWtTab && pk.step_end - pk.step0 <= kWtTable;
    if constexpr (kWtTab) {
        if (use_tab)
            for (int j = threadIdx.x; j < pk.step_end - pk.step0; j += BLOCK) {
                int t0;
                wt_lds[j] = time_weight(pk, pk.step0 + j, t0);
            }
    }
    __syncthreads();
    const StepConst& p = pc;
    const float* const wt_tab = use_tab ? wt_lds : nullptr;
    constexpr int kTL = step_min_blocks<NCOMP, TIME, NNUC, KZ, DEP, ENS>() == 4 ? 7 : 8;
    using Tab = DepTable<NNUC, kTL>;
    __shared__ int tab_key[kWaves][Tab::kSlots];
    __shared__ double tab_val[kWaves][NNUC * Tab::kSlots];
    __shared__ int tab_used[kWaves];
    __shared__ int stage_key[kWaves][DEP ? 3 * Tab::kStage : 1];
    __shared__ float stage_val[kWaves][DEP ? 4 * NNUC * Tab::kStage : 1];
    __shared__ int stage_n[kWaves];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    Tab tab{tab_key[wv], tab_val[wv], &tab_used[wv], stage_key[wv], stage_val[wv],
                       &stage_n[wv]};
    const long long plane = (long long)p.dnx * p.dny;
    // this block's copy of the deposition grid(s): one grid per nuclide, or
    // in an ensemble launch one per scenario and nuclide
    double* const depg = p.dep + (long long)(blockIdx.x % (unsigned)p.dep_copies) *
                                     (ENS ? p.n_scen : 1) * p.n_nuc * plane;
    if constexpr (DEP) tab.init(lane);
    __builtin_amdgcn_wave_barrier();

    unsigned long long* queue = reinterpret_cast<unsigned long long*>(p.ctrl + LPM_CTRL_QUEUE);
    float4* rec4 = reinterpret_cast<float4*>(p.rec);
    int* rec_exit = reinterpret_cast<int*>(p.rec + 4ll * p.n_rec * p.rec_stride);
    const int slot_index = blockIdx.x % LPM_LEDGER_SLOTS;

    using LG = Ledger<NNUC, KZ>;
    constexpr bool kSharedLedger = KZ != 4 && !ENS;
    __shared__ double wave_led[kSharedLedger ? kWaves : 1][LG::kSize];
    LedgerAcc<NNUC, KZ, kSharedLedger> led;
    if constexpr (kSharedLedger) {
        led.wave = wave_led[wv];
        if (lane < LG::kSize) led.wave[lane] = 0.0;
    } else {
#pragma unroll
        for (int q = 0; q < LG::kSize; ++q) led.reg[q] = 0.0;
    }

    SrcVals sv{p.a0, p.wscale, p.dry_c1, p.dry_c2, p.key1, 0};
    int led_scen = 0;  // scenario the ledger partials belong to
    bool have = false, drained = false;
    long long i = 0;
    uint32_t gid = 0;
    int b = 0, s = 0, krec = 0, next_rec = INT_MAX, s_take = 0;
    // where the lane's particle is recorded: its queue position with a work
    // order (records then follow the order's wind-node sorting), else its
    // index; below 2^32 either way
    uint32_t rq = 0;
    float x = 0.0f, y = 0.0f, z = 0.0f, m = 0.0f;
    float xl = 0.0f, yl = 0.0f;  // rounding residuals of x, y
    float bdep[NNUC];  // deposited by the lane's particle in this window (light kernels)
#pragma unroll
    for (int n = 0; n < NNUC; ++n) bdep[n] = 0.0f;
    Dwell<NNUC, kTL> dw;

    while (true) {
        // hand the next queue entries to the lanes without a particle
        while (!drained) {
            const unsigned long long need = __ballot(!have);
            // refill once enough lanes idle (keeps the lanes of a wave on
            // particles released together, whose wind stencils overlap), or
            // when the whole wave is idle
            const int idle = __popcll(need);
            if (need == 0ull || (idle < p.refill_min && need != __ballot(true))) break;
            const int leader = __ffsll((long long)need) - 1;
            const int cnt = __popcll(need);
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(queue, (unsigned long long)cnt);
            base = __shfl(base, leader, 64);
            if (base + (unsigned long long)cnt >= (unsigned long long)p.i_hi) drained = true;
            if (!have) {
                const int rank = __popcll(need & ((1ull << lane) - 1ull));
                const long long q = (long long)(base + (unsigned long long)rank);
                if (q < p.i_hi) {
                    long long g;
                    if constexpr (ENS) {
                        // scenario of work index q: last c with qbase[c] <= q
                        int lo = 0, hi = p.n_scen;
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (scen_qbase[mid] <= q) lo = mid; else hi = mid;
                        }
                        const DevScen& ds = p.scen[lo];
                        if (lo != led_scen) {
                            lane_ledger<NNUC, KZ>(led, p.ledger + ((long long)led_scen * LPM_LEDGER_SLOTS + slot_index) * LPM_LEDGER_STRIDE);
                            led_scen = lo;
                        }
                        sv = SrcVals{ds.a0, ds.wscale, ds.dry_c1, ds.dry_c2, ds.key1, lo};
                        // the lane's dwell outlives its particle; its sums go
                        // to the scenario they were made in
                        if constexpr (DEP)
                            if ((int)(lo * plane) != dw.key_base) dw.flush(p, tab, plane);
                        dw.key_base = (int)(lo * plane);
                        g = q - ds.qbase;                  // local id of the scenario
                        b = (int)birth(g, ds.s_release, ds.n_total);
                        i = ds.offset + g;                 // element in the state arrays
                    } else {
                        i = p.order ? (long long)as_global(p.order)[q] : q;
                        // an entry outside the launch (not a permutation)
                        // takes nothing
                        if ((unsigned long long)i >= (unsigned long long)p.i_hi) i = -1;
                        g = p.id_base + i * p.id_stride;
                        b = (int)birth(g, p.s_release, p.n_total);
                    }
                    gid = (uint32_t)g;
                    rq = (uint32_t)(p.order ? q : i);
                    m = i >= 0 ? as_global(p.M)[i] : 0.0f;
                    if (m > 0.0f) {
                        x = as_global(p.X)[i];
                        y = as_global(p.Y)[i];
                        z = as_global(p.Z)[i];
                        xl = p.XL ? as_global(p.XL)[i] : 0.0f;
                        yl = p.YL ? as_global(p.YL)[i] : 0.0f;
                        s = b > p.step0 ? b : p.step0;
                        krec = s <= p.rec_step0 ? 0
                                                : (s - p.rec_step0 + p.rec_every - 1) / p.rec_every;
                        next_rec = krec < p.n_rec ? p.rec_step0 + krec * p.rec_every : INT_MAX;
                        have = true;
                        s_take = s;
                        if constexpr (KZ != 4) {
                            // the activity the particle brings into the window
                            const float age0 = (float)(s - b) * p.dt;
#pragma unroll
                            for (int n = 0; n < NNUC; ++n) {
                                bdep[n] = 0.0f;
                                led.add(3 * n + 1, (double)(sv.a0 * m *
                                    __builtin_amdgcn_exp2f(-p.lam_l2e[n] * age0)));
                            }
                        }
                    } else if (p.n_rec > 0 && (i >= 0 || p.order)) {
                        // inactive before this window (or, with a work order,
                        // an entry outside the launch: every position gets a word)
                        as_global(rec_exit)[rq] = INT_MIN;
                    }
                }
            }
        }
        // refills may have staged a quad per lane (ensembles: scenario change)
        if constexpr (DEP && ENS) {
            if (tab.drain(lane, depg, plane, Tab::kDrainAt, p.dmode == 0 ? 1 : 4,
                          p.dnx, p.dny))
                tab.flush_if_half_full(lane, depg, plane);
        }
        if (!__any(have)) break;
        for (int j = 0; j < p.refill_every; ++j) {
            if (have) {
                const int st = advance<NCOMP, TIME, LEVELS, NNUC, KZ, DEP, ENS, kTL>(
                    p, wt_tab, sv, tab, plane, gid, b, s, x, y, z, m, xl, yl, led, bdep, dw);
                if (s == next_rec) {  // state after an output step, for gridding later
                    typedef float quad __attribute__((ext_vector_type(4)));
                    // krec, the stride and rq are below 2^32: one 32 x 32 -> 64-bit
                    // multiply-add forms the index
                    as_global(reinterpret_cast<quad*>(rec4))[(unsigned long long)(uint32_t)krec *
                                                                 (uint32_t)p.rec_stride +
                                                             rq] = quad{x, y, z, m};
                    ++krec;
                    next_rec = krec < p.n_rec ? next_rec + p.rec_every : INT_MAX;
                }
                ++s;
                if (st != 0 || s >= p.step_end) {
                    // (the lane's dwell stays: deposits are keyed by cell, and
                    // the lane's next particle or the kernel's end flushes it)
                    as_global(p.X)[i] = x;
                    as_global(p.Y)[i] = y;
                    as_global(p.Z)[i] = z;
                    as_global(p.M)[i] = m;
                    if (p.XL) {
                        as_global(p.XL)[i] = xl;
                        as_global(p.YL)[i] = yl;
                    }
                    if (p.n_rec > 0) as_global(rec_exit)[rq] = st != 0 ? s - 1 : INT_MAX;
                    if (st == 2) atomicOr(p.ctrl + LPM_CTRL_ERR, 1u);
                    have = false;
                    if constexpr (KZ != 4) {
                        // deposited in the window; decayed = brought in - still
                        // airborne (0 after an exit) - deposited - exited
                        const float age1 = (float)(s - b) * p.dt;
#pragma unroll
                        for (int n = 0; n < NNUC; ++n) {
                            led.add(3 * n + 0, (double)bdep[n]);
                            led.add(3 * n + 1, -((double)bdep[n] + (double)(sv.a0 * m *
                                __builtin_amdgcn_exp2f(-p.lam_l2e[n] * age1))));
                        }
                    }
                    led.add(3 * NNUC, (double)(s - s_take));  // particle-steps advanced
                }
            }
            if constexpr (DEP) {
                // a drain fills the table: move it out before it overflows
                if (tab.drain(lane, depg, plane, Tab::kDrainAt,
                              p.dmode == 0 ? 1 : 4, p.dnx, p.dny))
                    tab.flush_if_half_full(lane, depg, plane);
            }
        }
    }
    if constexpr (DEP) {
        dw.flush(p, tab, plane);  // every lane: its last particle's sums
        tab.drain(lane, depg, plane, 1, p.dmode == 0 ? 1 : 4, p.dnx, p.dny);
        tab.flush(lane, depg, plane);
    }

    // ledger slot: [nuclide][released, deposited, decayed, exited], steps
    constexpr int NV = LG::kSize;
    if constexpr (ENS) {
        // lanes of a wave usually finish in one scenario: one atomic per entry
        const int s0 = __shfl(led_scen, 0, 64);
        double* slot = p.ledger + ((long long)led_scen * LPM_LEDGER_SLOTS + slot_index) * LPM_LEDGER_STRIDE;
        if (__all(led_scen == s0)) {
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                const double v = wave_sum(led.reg[q]);
                if (lane == 0 && v != 0.0) atomicAdd(slot + LG::offset(q), v);
            }
        } else {
            lane_ledger<NNUC, KZ>(led, slot);
        }
        return;
    }
    double* slot = p.ledger + (long long)slot_index * LPM_LEDGER_STRIDE;
    __shared__ double part[kSharedLedger ? 1 : kWaves][NV];
    double (*wsum)[NV] = wave_led;
    if constexpr (!kSharedLedger) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const double v = wave_sum(led.reg[q]);
            if (lane == 0) part[wv][q] = v;
        }
        wsum = part;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) v += wsum[w][threadIdx.x];
        const int q = threadIdx.x;
        if (v != 0.0) atomicAdd(slot + LG::offset(q), v);
    }
}

}  // namespace lpm

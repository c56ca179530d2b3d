// liblpm: HIP kernels and C ABI of the particle-dispersion hot path for
// gfx950 (MI355X).  The model is the stochastic Lagrangian particle model of
// Molnar Jr. et al. (arXiv:0912.3223, Sec. 2 and 3.2); see include/lpm.h for
// the interface contract.
//
// Kernels
//  - release_kernel: writes the initial state of the particles born in a
//    window of steps (one thread per particle, coalesced float stores).
//  - step_kernel: one thread per particle; the particle's state is loaded
//    once, advanced through every step of the window in registers, and stored
//    once.  Random numbers come from Philox in registers and the wind is
//    gathered from the L2/MALL-resident field.  Deposition is aggregated in
//    three levels before it reaches HBM: per thread while the particle stays
//    in one grid cell (registers), per block in an LDS hash table of cells
//    (FP64 LDS atomics), and once per block and cell into the FP64 grid.  The
//    ledger is reduced per block before one atomic per entry into one of
//    LPM_LEDGER_SLOTS spread-out slots.
//  - conc_kernel + finalize: scatter of activity to an FP64 grid, then
//    conversion to float.
//  Blocks keep the hardware's round-robin dealing to the 8 XCDs: live
//  particles concentrate in the most recently released (highest) ids, and
//  interleaving consecutive blocks over the XCDs spreads them evenly.
#include <hip/hip_runtime.h>

#include <limits.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "lpm.h"
#include "lpm_device.h"

namespace lpm {

constexpr int kBlock = 256;
constexpr int kXcds = 8;

__device__ __forceinline__ long long birth(long long gid, long long s_release,
                                           long long n_total)
{
    return (gid * s_release) / n_total;
}

// exp(x) - 1 for x <= 0.  Per-step rates times dt are small (|x| < 1e-3 in
// practice), where the Taylor series of exp to x^4/24 is exact to float
// rounding (truncation x^5/120); larger |x| use the library expm1f.
__device__ __forceinline__ float expm1_neg(float x)
{
    if (x > -0.0078125f)
        return x * fmaf(x, fmaf(x, fmaf(x, 1.0f / 24.0f, 1.0f / 6.0f), 0.5f), 1.0f);
    return expm1f(x);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Block-private histogram: an open-addressing hash table of grid cells in LDS
// with FP64 values.  A block's particles were released together and land in
// few cells, so near the source thousands of contributions per step would
// otherwise serialise on the same global addresses.  Cells that do not find a
// slot within kProbes probes go straight to the global grid.
// ---------------------------------------------------------------------------
template <int NNUC, int LOG2_SLOTS>
struct CellTable {
    static constexpr int kSlots = 1 << LOG2_SLOTS;
    static constexpr int kShift = 32 - LOG2_SLOTS;
    static constexpr int kProbes = 8;
    int* key;      // [kSlots]: 0 = empty, else cell + 1
    double* val;   // [NNUC][kSlots]

    __device__ void init()
    {
        for (int t = threadIdx.x; t < kSlots; t += kBlock) {
            key[t] = 0;
#pragma unroll
            for (int n = 0; n < NNUC; ++n) val[n * kSlots + t] = 0.0;
        }
    }

    __device__ void add(int cell, const float (&v)[NNUC], double* grid, long long plane)
    {
        unsigned h = ((unsigned)cell * 2654435761u) >> kShift;
        for (int probe = 0; probe < kProbes; ++probe) {
            const int old = atomicCAS(&key[h], 0, cell + 1);
            if (old == 0 || old == cell + 1) {
#pragma unroll
                for (int n = 0; n < NNUC; ++n)
                    if (v[n] != 0.0f) atomicAdd(&val[n * kSlots + h], (double)v[n]);
                return;
            }
            h = (h + 1) & (kSlots - 1);
        }
#pragma unroll
        for (int n = 0; n < NNUC; ++n)
            if (v[n] != 0.0f) atomicAdd(grid + n * plane + cell, (double)v[n]);
    }

    __device__ void flush(double* grid, long long plane)
    {
        for (int t = threadIdx.x; t < kSlots; t += kBlock) {
            const int k = key[t];
            if (k == 0) continue;
#pragma unroll
            for (int n = 0; n < NNUC; ++n) {
                const double v = val[n * kSlots + t];
                if (v != 0.0) atomicAdd(grid + n * plane + (k - 1), v);
            }
        }
    }
};

// Per-thread deposition while the particle stays in one grid cell (nearest
// cell) or above one cell quad (cloud-in-cell): partial sums of the corner
// weights times the deposited activity, flushed to the block table when the
// cell changes and at the end of the window.
template <int NNUC>
using DepTable = CellTable<NNUC, NNUC <= 2 ? 10 : 9>;

template <int NNUC>
struct Dwell {
    int i0 = INT_MIN, j0 = 0;
    float acc[NNUC][4];

    __device__ void flush(const StepConst& p, DepTable<NNUC>& tab, long long plane)
    {
        if (i0 == INT_MIN) return;
        const int ncorner = p.dmode == 0 ? 1 : 4;
        for (int c = 0; c < ncorner; ++c) {
            const int ii = i0 + (c & 1), jj = j0 + (c >> 1);
            if (ii < 0 || jj < 0 || ii >= p.dnx || jj >= p.dny) continue;
            float v[NNUC];
#pragma unroll
            for (int n = 0; n < NNUC; ++n) v[n] = acc[n][c];
            tab.add(jj * p.dnx + ii, v, p.dep, plane);
        }
        i0 = INT_MIN;
    }

    // Deposited activities d[n] (already scaled) at (x, y).  The cell index
    // and weights are formed in double precision: 50 km from the grid origin a
    // float coordinate difference alone would perturb them by ~1e-5.
    __device__ void add(const StepConst& p, DepTable<NNUC>& tab, long long plane, float x,
                        float y, const float (&d)[NNUC])
    {
        const double fx = ((double)x - p.dx0) * p.dinv_dx;
        const double fy = ((double)y - p.dy0) * p.dinv_dy;
        const double sh = p.dmode == 0 ? 0.0 : 0.5;
        const double ix = floor(fx - sh), iy = floor(fy - sh);
        // the cell (quad) must touch the grid; false for NaN
        if (!(ix >= -1.0 && iy >= -1.0 && ix < (double)p.dnx && iy < (double)p.dny)) return;
        const int ci = (int)ix, cj = (int)iy;
        if (ci != i0 || cj != j0) {
            flush(p, tab, plane);
            i0 = ci;
            j0 = cj;
#pragma unroll
            for (int n = 0; n < NNUC; ++n)
                acc[n][0] = acc[n][1] = acc[n][2] = acc[n][3] = 0.0f;
        }
        if (p.dmode == 0) {
#pragma unroll
            for (int n = 0; n < NNUC; ++n) acc[n][0] += d[n];
            return;
        }
        const float wx = (float)(fx - sh - ix), wy = (float)(fy - sh - iy);
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

// ---------------------------------------------------------------------------
// The particle step (Sec. 3.2 main loop; Eqs. 1-3).
// ---------------------------------------------------------------------------
template <int NCOMP, bool TIME, bool LEVELS, int NNUC, int KZ, bool DEP>
__global__ __launch_bounds__(kBlock) void step_kernel(const StepConst p)
{
    __shared__ int tab_key[DepTable<NNUC>::kSlots];
    __shared__ double tab_val[NNUC * DepTable<NNUC>::kSlots];
    DepTable<NNUC> tab{tab_key, tab_val};
    const long long plane = (long long)p.dnx * p.dny;
    if constexpr (DEP) tab.init();
    __syncthreads();

    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    double led[3 * NNUC + 1];  // deposited, decayed, exited per nuclide; steps
#pragma unroll
    for (int q = 0; q <= 3 * NNUC; ++q) led[q] = 0.0;

    if (i < p.i_hi) {
        const long long gid = p.id_base + i * p.id_stride;
        const long long b = birth(gid, p.s_release, p.n_total);
        float m = p.M[i];
        const int s0 = b > p.step0 ? (int)b : p.step0;
        // next recorded step at or after the particle's first step here
        int krec = s0 <= p.rec_step0 ? 0 : (s0 - p.rec_step0 + p.rec_every - 1) / p.rec_every;
        int next_rec = krec < p.n_rec ? p.rec_step0 + krec * p.rec_every : INT_MAX;
        if (m > 0.0f && b < p.step_end) {
            float x = p.X[i], y = p.Y[i], z = p.Z[i];
            bool bad = false;
            int advanced = 0;
            Dwell<NNUC> dw;
            for (int s = s0; s < p.step_end; ++s) {
                ++advanced;
                const float age = (float)(s - (int)b) * p.dt;
                // weather at the start-of-step position and time (Eq. 1): the
                // loads are issued first; everything up to the interpolation
                // below is independent of them
                WindTap<NCOMP, TIME> tap;
                wind_gather<NCOMP, TIME, LEVELS>(p, x, y, z, (float)s * p.dt, tap);
                // random numbers of Eq. (2)
                float xi0, xi1, xi2;
                normals3((uint32_t)gid, (uint32_t)s, p.key0, p.key1, xi0, xi1, xi2);
                // diffusivity (Eq. 3) with the drift and midpoint evaluation
                float K, dK, Km, dKm;
                kz_profile<KZ>(p, z, K, dK);
                const float zm = clampf(fmaf(p.half_dt, dK, z), 0.0f, p.H_mix);
                kz_profile<KZ>(p, zm, Km, dKm);
                // decay factors of this step's start
                float D[NNUC];
#pragma unroll
                for (int n = 0; n < NNUC; ++n) D[n] = exp2f(-p.lam_l2e[n] * age);
                float uvw[3];
                wind_interp<NCOMP, TIME>(tap, uvw);
                // move (Eq. 1 with Eq. 2)
                float xn = fmaf(xi0, p.sKh, fmaf(p.wscale * uvw[0], p.dt, x));
                float yn = fmaf(xi1, p.sKh, fmaf(p.wscale * uvw[1], p.dt, y));
                float zn = fmaf(xi2 * __builtin_amdgcn_sqrtf(Km), p.s2dt,
                                fmaf(fmaf(p.wscale, uvw[2], dK), p.dt, z));
                // reflection at the ground and the lid: one fold each, and the
                // general fold-until-inside for the (never seen) larger steps
                zn = fabsf(zn);
                if (zn > p.H_top) zn = 2.0f * p.H_top - zn;
                if (zn < 0.0f || zn > p.H_top) {
#pragma unroll 1
                    for (int it = 0; it < 64; ++it) {
                        if (zn < 0.0f) zn = -zn;
                        else if (zn > p.H_top) zn = 2.0f * p.H_top - zn;
                        else break;
                    }
                }
                // deposition rate at the new position (Sec. 2)
                float k = 0.0f;
                if constexpr (DEP) {
                    if (zn < p.h_s) k = fmaxf(fmaf(-p.dry_c2, zn, p.dry_c1), 0.0f);
                    if (p.L0 > 0.0f) k += wet_rate(p, xn, yn);
                }
                const float mn = k > 0.0f ? m * exp2f(-1.4426950408889634f * k * p.dt) : m;
                // decay and deposition of each nuclide's activity this step
                float dsum[NNUC];
#pragma unroll
                for (int n = 0; n < NNUC; ++n) {
                    const float A = p.a0 * m * D[n];
                    if (DEP && k > 0.0f) {
                        // loss of activity this step, split by the rates
                        const float r = p.lam[n] + k;
                        const float loss = -A * expm1_neg(-r * p.dt);
                        const float dep = loss * (k * __builtin_amdgcn_rcpf(r));
                        dsum[n] = dep * p.dscale;
                        led[3 * n + 0] += (double)dep;
                        led[3 * n + 1] += (double)(loss - dep);
                    } else {
                        dsum[n] = 0.0f;
                        led[3 * n + 1] += (double)(A * p.cdec[n]);
                    }
                }
                if (DEP && k > 0.0f) dw.add(p, tab, plane, xn, yn, dsum);
                x = xn;
                y = yn;
                z = zn;
                m = mn;
                if (!(__builtin_isfinite(x) && __builtin_isfinite(y) &&
                      __builtin_isfinite(z) && __builtin_isfinite(m))) {
                    bad = true;
                    break;
                }
                // leaving the simulated area inactivates the particle
                const bool gone = p.bounded && (x < p.X0 || x >= p.X1 || y < p.Y0 || y >= p.Y1);
                if (gone) {
#pragma unroll
                    for (int n = 0; n < NNUC; ++n)
                        led[3 * n + 2] += (double)(p.a0 * m * D[n] * p.edec[n]);
                    m = 0.0f;
                }
                // state after an output step, for gridding later
                if (s == next_rec) {
                    float* r = p.rec + 4ll * krec * p.rec_stride + i;
                    r[0] = x;
                    r[p.rec_stride] = y;
                    r[2 * p.rec_stride] = z;
                    r[3 * p.rec_stride] = m;
                    ++krec;
                    next_rec = krec < p.n_rec ? p.rec_step0 + krec * p.rec_every : INT_MAX;
                }
                if (gone) break;
            }
            if constexpr (DEP) dw.flush(p, tab, plane);
            p.X[i] = x;
            p.Y[i] = y;
            p.Z[i] = z;
            p.M[i] = m;
            led[3 * NNUC] = (double)advanced;
            if (bad) atomicOr(p.err, 1u);
        }
        // records after the particle stopped (or of a particle already
        // inactive): no activity
        for (; krec < p.n_rec; ++krec) p.rec[(4ll * krec + 3) * p.rec_stride + i] = 0.0f;
    }
    // ledger slot: [nuclide][released, deposited, decayed, exited], steps
    double* slot = p.ledger + (long long)(blockIdx.x % LPM_LEDGER_SLOTS) * LPM_LEDGER_STRIDE;
    constexpr int NV = 3 * NNUC + 1;
    __shared__ double part[kBlock / 64][NV];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const double s = wave_sum(led[q]);
        if (lane == 0) part[wv][q] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) s += part[w][threadIdx.x];
        const int q = threadIdx.x;
        const int off = q == 3 * NNUC ? LPM_LEDGER_PSTEPS : (q / 3) * 4 + 1 + q % 3;
        if (s != 0.0) atomicAdd(slot + off, s);
    }
    if constexpr (DEP) tab.flush(p.dep, plane);
}

// ---------------------------------------------------------------------------
// Release (Sec. 2: particles released from the point source every step).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void release_kernel(float* X, float* Y, float* Z,
                                                         float* M, long long i_lo,
                                                         long long i_hi, float xs, float ys,
                                                         float h, double* ledger,
                                                         int n_nuc, double released)
{
    const long long i = i_lo + (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i < i_hi) {
        X[i] = xs;
        Y[i] = ys;
        Z[i] = h;
        M[i] = 1.0f;
    }
    if (blockIdx.x == 0 && threadIdx.x < n_nuc) atomicAdd(ledger + threadIdx.x * 4, released);
}

// ---------------------------------------------------------------------------
// Gridding (Sec. 3.2: activities summed on a rectangular grid).
// ---------------------------------------------------------------------------
struct GridConst {
    const float* X;
    const float* Y;
    const float* Z;
    const float* M;
    long long n_total, id_base, id_stride, i_hi;
    int s_release, step, nnuc, mode;
    float a0, dt, scale;
    float lam_l2e[4];
    int nx, ny, nz, pad;
    double x0, y0, z0, inv_dx, inv_dy, inv_dz;
    long long cells;
    double* acc;
};

template <int NNUC>
__global__ __launch_bounds__(kBlock) void conc_kernel(const GridConst g)
{
    using Table = CellTable<NNUC, NNUC <= 2 ? 11 : 10>;
    __shared__ int tab_key[Table::kSlots];
    __shared__ double tab_val[NNUC * Table::kSlots];
    Table tab{tab_key, tab_val};
    tab.init();
    __syncthreads();
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    const float m = i < g.i_hi ? g.M[i] : 0.0f;
    long long b = 0;
    if (m > 0.0f) b = birth(g.id_base + i * g.id_stride, g.s_release, g.n_total);
    if (m > 0.0f && b <= g.step) {
        const float age = (float)(g.step + 1 - (int)b) * g.dt;
        float A[NNUC];
#pragma unroll
        for (int n = 0; n < NNUC; ++n) A[n] = g.a0 * m * exp2f(-g.lam_l2e[n] * age) * g.scale;
        // cell index and weights in double precision (see Dwell::add)
        const double fx = ((double)g.X[i] - g.x0) * g.inv_dx;
        const double fy = ((double)g.Y[i] - g.y0) * g.inv_dy;
        const double fz = ((double)g.Z[i] - g.z0) * g.inv_dz;
        if (g.mode == 0) {
            const double ix = floor(fx), iy = floor(fy), iz = floor(fz);
            if (ix >= 0.0 && iy >= 0.0 && iz >= 0.0 && ix < (double)g.nx && iy < (double)g.ny &&
                iz < (double)g.nz)  // false for NaN
                tab.add((int)(((long long)iz * g.ny + (long long)iy) * g.nx + (long long)ix), A,
                        g.acc, g.cells);
        } else {
            const double ix = floor(fx - 0.5), iy = floor(fy - 0.5), iz = floor(fz - 0.5);
            const float wx = (float)(fx - 0.5 - ix), wy = (float)(fy - 0.5 - iy);
            const float wz = (float)(fz - 0.5 - iz);
            for (int c = 0; c < 8; ++c) {
                const double kx = ix + (c & 1), ky = iy + ((c >> 1) & 1), kz = iz + (c >> 2);
                if (!(kx >= 0.0 && ky >= 0.0 && kz >= 0.0 && kx < (double)g.nx &&
                      ky < (double)g.ny && kz < (double)g.nz))  // also skips NaN
                    continue;
                const float w = ((c & 1) ? wx : 1.0f - wx) * (((c >> 1) & 1) ? wy : 1.0f - wy) *
                                ((c >> 2) ? wz : 1.0f - wz);
                float v[NNUC];
#pragma unroll
                for (int n = 0; n < NNUC; ++n) v[n] = A[n] * w;
                tab.add((int)(((long long)kz * g.ny + (long long)ky) * g.nx + (long long)kx), v,
                        g.acc, g.cells);
            }
        }
    }
    __syncthreads();
    tab.flush(g.acc, g.cells);
}

__global__ __launch_bounds__(kBlock) void fill_f64(double* p, long long n)
{
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}

__global__ __launch_bounds__(kBlock) void fill_u32(uint32_t* p, long long n)
{
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ __launch_bounds__(kBlock) void to_f32(const double* __restrict__ src, float* dst,
                                                 long long n, double scale)
{
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        dst[i] = (float)(src[i] * scale);
}

}  // namespace lpm

// ===========================================================================
// Host side: validation, constant folding, launches.
// ===========================================================================
namespace {

thread_local char g_msg[512] = "";

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof g_msg, fmt, ap);
    va_end(ap);
    return code;
}

int hip_status(const char* what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LPM_EHIP, "%s: %s", what, hipGetErrorString(e));
    return LPM_OK;
}

bool aligned4(const void* p) { return ((uintptr_t)p & 3u) == 0; }

// First local index whose birth step is >= s.
long long first_local_born_at_or_after(const lpm_schedule* sch, long long s)
{
    if (s <= 0) return 0;
    const long long N = sch->n_total, R = sch->s_release;
    if (s >= R) return sch->n_local;
    // smallest global id g with g * R >= s * N
    const long long g = (s * N + R - 1) / R;
    if (g <= sch->id_base) return 0;
    long long i = (g - sch->id_base + sch->id_stride - 1) / sch->id_stride;
    return i < sch->n_local ? i : sch->n_local;
}

int check_state(const lpm_state* st, const lpm_schedule* sch)
{
    if (!st || !sch) return fail(LPM_EINVAL, "null state or schedule");
    if (!st->x || !st->y || !st->z || !st->m) return fail(LPM_EINVAL, "null state array");
    if (!aligned4(st->x) || !aligned4(st->y) || !aligned4(st->z) || !aligned4(st->m))
        return fail(LPM_EINVAL, "state arrays must be 4-byte aligned");
    if (sch->n_total <= 0 || sch->n_total > 0xFFFFFFFFll)
        return fail(LPM_EINVAL, "n_total must be in [1, 2^32)");
    if (sch->s_release <= 0) return fail(LPM_EINVAL, "s_release must be positive");
    if (sch->n_local < 0 || sch->id_base < 0 || sch->id_stride <= 0)
        return fail(LPM_EINVAL, "bad local id range");
    if (sch->n_local > 0 &&
        sch->id_base + (sch->n_local - 1) * sch->id_stride >= sch->n_total)
        return fail(LPM_EINVAL, "local ids exceed n_total");
    if (sch->n_local > st->capacity)
        return fail(LPM_ECAPACITY, "n_local %lld exceeds capacity %lld",
                    (long long)sch->n_local, (long long)st->capacity);
    return LPM_OK;
}

int check_physics(const lpm_physics* ph)
{
    if (!ph) return fail(LPM_EINVAL, "null physics");
    if (ph->n_nuc < 1 || ph->n_nuc > 4) return fail(LPM_EINVAL, "n_nuc must be 1..4");
    if (!(ph->dt > 0.0)) return fail(LPM_EINVAL, "dt must be positive");
    if (ph->Kh < 0.0 || ph->Kz_const < 0.0 || ph->kappa_ustar < 0.0)
        return fail(LPM_EINVAL, "diffusivities must be non-negative");
    if (ph->kz_kind < 0 || ph->kz_kind > 2) return fail(LPM_EINVAL, "kz_kind must be 0, 1 or 2");
    if (ph->kz_kind != 0 && !(ph->H_mix > 0.0)) return fail(LPM_EINVAL, "H_mix must be positive");
    for (int n = 0; n < ph->n_nuc; ++n)
        if (ph->lambda[n] < 0.0) return fail(LPM_EINVAL, "decay constants must be >= 0");
    if (ph->Lambda0 < 0.0) return fail(LPM_EINVAL, "Lambda0 must be >= 0");
    if (ph->Lambda0 > 0.0 && !(ph->rain_a > 0.0 && ph->rain_b > 0.0 && ph->rain_edge > 0.0))
        return fail(LPM_EINVAL, "rain region needs positive semi-axes and edge");
    return LPM_OK;
}

int check_grid(const lpm_grid* g, bool two_d)
{
    if (!g) return fail(LPM_EINVAL, "null grid");
    if (g->nx < 1 || g->ny < 1 || (!two_d && g->nz < 1))
        return fail(LPM_EINVAL, "grid dimensions must be positive");
    if (!(g->dx > 0.0 && g->dy > 0.0 && (two_d || g->dz > 0.0)))
        return fail(LPM_EINVAL, "grid spacings must be positive");
    if (g->mode != 0 && g->mode != 1) return fail(LPM_EINVAL, "grid mode must be 0 or 1");
    const double cells = (double)g->nx * g->ny * (two_d ? 1 : g->nz);
    if (cells >= 2147483647.0) return fail(LPM_EINVAL, "grid must have fewer than 2^31 - 1 cells");
    return LPM_OK;
}

int check_accum(const lpm_accum* acc)
{
    if (!acc || !acc->dep || !acc->ledger || !acc->err) return fail(LPM_EINVAL, "null accumulator");
    if (acc->n_nuc < 1 || acc->n_nuc > 4) return fail(LPM_EINVAL, "accumulator n_nuc must be 1..4");
    if (((uintptr_t)acc->dep & 7u) || ((uintptr_t)acc->ledger & 7u) || !aligned4(acc->err))
        return fail(LPM_EINVAL, "misaligned accumulator");
    if ((double)acc->dep_grid.nx * acc->dep_grid.ny >= 2147483647.0)
        return fail(LPM_EINVAL, "deposition grid must have fewer than 2^31 - 1 cells");
    return check_grid(&acc->dep_grid, true);
}

double a0_of(const lpm_source* src, const lpm_schedule* sch, const lpm_physics* ph)
{
    return src->q * (double)sch->s_release * ph->dt / (double)sch->n_total;
}

unsigned blocks_for(long long n)
{
    return (unsigned)((n + lpm::kBlock - 1) / lpm::kBlock);
}

}  // namespace

extern "C" {

const char* lpm_last_error(void) { return g_msg; }

const char* lpm_version(void) { return "lpm 0.1 gfx950"; }

int lpm_accum_reset(const lpm_accum* acc, lpm_stream stream)
{
    g_msg[0] = 0;
    int rc = check_accum(acc);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const long long dn = (long long)acc->n_nuc * acc->dep_grid.nx * acc->dep_grid.ny;
    hipLaunchKernelGGL(lpm::fill_f64, dim3(blocks_for(dn) < 4096 ? blocks_for(dn) : 4096),
                       dim3(lpm::kBlock), 0, s, acc->dep, dn);
    hipLaunchKernelGGL(lpm::fill_f64, dim3(blocks_for(LPM_LEDGER_SLOTS * LPM_LEDGER_STRIDE)),
                       dim3(lpm::kBlock), 0, s, acc->ledger,
                       (long long)LPM_LEDGER_SLOTS * LPM_LEDGER_STRIDE);
    hipLaunchKernelGGL(lpm::fill_u32, dim3(1), dim3(lpm::kBlock), 0, s, acc->err, 1ll);
    return hip_status("lpm_accum_reset");
}

int lpm_release_particles(const lpm_state* st, const lpm_source* src, const lpm_schedule* sch,
                          const lpm_physics* ph, int32_t step0, int32_t n_steps,
                          const lpm_accum* acc, lpm_stream stream)
{
    g_msg[0] = 0;
    int rc = check_state(st, sch);
    if (rc) return rc;
    if (!src) return fail(LPM_EINVAL, "null source");
    if ((rc = check_physics(ph)) || (rc = check_accum(acc))) return rc;
    if (acc->n_nuc != ph->n_nuc) return fail(LPM_EINVAL, "accumulator and physics n_nuc differ");
    if (step0 < 0 || n_steps < 1) return fail(LPM_EINVAL, "bad step window");
    const long long lo = first_local_born_at_or_after(sch, step0);
    const long long hi = first_local_born_at_or_after(sch, (long long)step0 + n_steps);
    if (hi <= lo) return LPM_OK;
    const double released = a0_of(src, sch, ph) * (double)(hi - lo);
    hipLaunchKernelGGL(lpm::release_kernel, dim3(blocks_for(hi - lo)), dim3(lpm::kBlock), 0,
                       (hipStream_t)stream, st->x, st->y, st->z, st->m, lo, hi, (float)src->xs,
                       (float)src->ys, (float)src->h, acc->ledger, ph->n_nuc, released);
    return hip_status("lpm_release_particles");
}

}  // extern "C"

namespace {

int fill_field(lpm::StepConst& p, const lpm_field* f)
{
    if (!f || !f->data) return fail(LPM_EINVAL, "null field");
    if (f->nx < 1 || f->ny < 1 || f->nz < 1 || f->nt < 1) return fail(LPM_EINVAL, "bad field shape");
    if (f->ncomp != 2 && f->ncomp != 3) return fail(LPM_EINVAL, "field ncomp must be 2 or 3");
    if (!(f->dx > 0 && f->dy > 0 && (f->z_levels || f->dz > 0) && (f->nt == 1 || f->dt_field > 0)))
        return fail(LPM_EINVAL, "field spacings must be positive");
    const double total = (double)f->nt * f->nz * f->ny * f->nx * f->ncomp;
    if (total >= 2147483647.0) return fail(LPM_EINVAL, "field larger than 2^31 floats");
    if (f->ncomp == 2 && ((uintptr_t)f->data & 7u))
        return fail(LPM_EINVAL, "two-component field must be 8-byte aligned");
    if (!aligned4(f->data)) return fail(LPM_EINVAL, "field must be 4-byte aligned");
    p.f = f->data;
    p.lev = f->z_levels;
    p.nx = f->nx; p.ny = f->ny; p.nz = f->nz; p.nt = f->nt;
    p.imax = f->nx >= 2 ? f->nx - 2 : 0;
    p.jmax = f->ny >= 2 ? f->ny - 2 : 0;
    p.kmax = f->nz >= 2 ? f->nz - 2 : 0;
    p.tmaxi = f->nt >= 2 ? f->nt - 2 : 0;
    p.fxmax = (float)(f->nx - 1); p.fymax = (float)(f->ny - 1);
    p.fzmax = (float)(f->nz - 1); p.ftmax = (float)(f->nt - 1);
    p.fx0 = (float)f->x0; p.fy0 = (float)f->y0;
    p.inv_dx = (float)(1.0 / f->dx); p.inv_dy = (float)(1.0 / f->dy);
    p.inv_dz = f->z_levels ? 0.0f : (float)(1.0 / f->dz);
    p.ft0 = (float)f->t0;
    p.inv_dtf = f->nt > 1 ? (float)(1.0 / f->dt_field) : 0.0f;
    p.sj = f->nx * f->ncomp;
    p.sk = f->ny * p.sj;
    p.st = f->nz * p.sk;
    p.di = f->nx > 1 ? f->ncomp : 0;
    p.dj = f->ny > 1 ? p.sj : 0;
    p.dk = f->nz > 1 ? p.sk : 0;
    p.dt_off = f->nt > 1 ? p.st : 0;
    p.bounded = f->bounded != 0;
    p.X0 = (float)f->x0; p.X1 = (float)(f->x0 + f->nx * f->dx);
    p.Y0 = (float)f->y0; p.Y1 = (float)(f->y0 + f->ny * f->dy);
    return LPM_OK;
}

// Compile-time variants: wind components, time interpolation, nonuniform
// levels, nuclide count, K_z kind, deposition on/off.
template <int NCOMP, bool TIME, bool LEV, int NNUC, int KZ>
void launch_step_dep(bool dep, unsigned nb, hipStream_t s, const lpm::StepConst& p)
{
    if (dep) hipLaunchKernelGGL((lpm::step_kernel<NCOMP, TIME, LEV, NNUC, KZ, true>), dim3(nb), dim3(lpm::kBlock), 0, s, p);
    else hipLaunchKernelGGL((lpm::step_kernel<NCOMP, TIME, LEV, NNUC, KZ, false>), dim3(nb), dim3(lpm::kBlock), 0, s, p);
}

template <int NCOMP, bool TIME, bool LEV, int NNUC>
void launch_step_kz(int kz, bool dep, unsigned nb, hipStream_t s, const lpm::StepConst& p)
{
    switch (kz) {
    case 0: launch_step_dep<NCOMP, TIME, LEV, NNUC, 0>(dep, nb, s, p); break;
    case 1: launch_step_dep<NCOMP, TIME, LEV, NNUC, 1>(dep, nb, s, p); break;
    default: launch_step_dep<NCOMP, TIME, LEV, NNUC, 2>(dep, nb, s, p); break;
    }
}

template <int NCOMP, bool TIME, bool LEV>
void launch_step_n(int nnuc, int kz, bool dep, unsigned nb, hipStream_t s, const lpm::StepConst& p)
{
    switch (nnuc) {
    case 1: launch_step_kz<NCOMP, TIME, LEV, 1>(kz, dep, nb, s, p); break;
    case 2: launch_step_kz<NCOMP, TIME, LEV, 2>(kz, dep, nb, s, p); break;
    case 3: launch_step_kz<NCOMP, TIME, LEV, 3>(kz, dep, nb, s, p); break;
    default: launch_step_kz<NCOMP, TIME, LEV, 4>(kz, dep, nb, s, p); break;
    }
}

template <int NCOMP, bool TIME>
void launch_step_lev(bool lev, int nnuc, int kz, bool dep, unsigned nb, hipStream_t s,
                     const lpm::StepConst& p)
{
    if (lev) launch_step_n<NCOMP, TIME, true>(nnuc, kz, dep, nb, s, p);
    else launch_step_n<NCOMP, TIME, false>(nnuc, kz, dep, nb, s, p);
}

}  // namespace

extern "C" {

static int step_impl(const lpm_state* st, const lpm_source* src, const lpm_schedule* sch,
                     const lpm_field* fld, const lpm_physics* ph, int32_t step0, int32_t n_steps,
                     const lpm_accum* acc, int32_t rec_step0, int32_t rec_every, int32_t n_rec,
                     float* rec, int64_t rec_stride, lpm_stream stream)
{
    g_msg[0] = 0;
    int rc = check_state(st, sch);
    if (rc) return rc;
    if (!src) return fail(LPM_EINVAL, "null source");
    if ((rc = check_physics(ph)) || (rc = check_accum(acc))) return rc;
    if (acc->n_nuc != ph->n_nuc) return fail(LPM_EINVAL, "accumulator and physics n_nuc differ");
    if (step0 < 0 || n_steps < 1 || (long long)step0 + n_steps > 0x7FFFFFFFll)
        return fail(LPM_EINVAL, "bad step window");
    if (n_rec < 0) return fail(LPM_EINVAL, "n_rec must be >= 0");
    if (n_rec > 0) {
        if (!rec || !aligned4(rec)) return fail(LPM_EINVAL, "null or misaligned record buffer");
        if (rec_every < 1) return fail(LPM_EINVAL, "rec_every must be >= 1");
        if (rec_stride < sch->n_local) return fail(LPM_EINVAL, "rec_stride below n_local");
        const long long last = (long long)rec_step0 + (long long)(n_rec - 1) * rec_every;
        if (rec_step0 < step0 || last >= (long long)step0 + n_steps)
            return fail(LPM_EINVAL, "recorded steps must lie inside the step window");
    }
    lpm::StepConst p;
    memset(&p, 0, sizeof p);
    if ((rc = fill_field(p, fld))) return rc;
    p.rec = n_rec > 0 ? rec : nullptr;
    p.rec_stride = rec_stride;
    p.rec_step0 = rec_step0;
    p.rec_every = rec_every > 0 ? rec_every : 1;
    p.n_rec = n_rec;

    p.X = st->x; p.Y = st->y; p.Z = st->z; p.M = st->m;
    p.n_total = sch->n_total; p.id_base = sch->id_base; p.id_stride = sch->id_stride;
    p.s_release = sch->s_release;
    p.step0 = step0;
    p.step_end = step0 + n_steps;
    p.i_hi = first_local_born_at_or_after(sch, (long long)p.step_end);

    const double dt = ph->dt;
    p.xs = (float)src->xs; p.ys = (float)src->ys; p.h = (float)src->h;
    p.a0 = (float)a0_of(src, sch, ph);
    p.wscale = (float)src->wind_scale;
    p.key0 = (uint32_t)(ph->seed & 0xFFFFFFFFull);
    p.key1 = src->scenario;

    p.dt = (float)dt;
    p.sKh = (float)sqrt(2.0 * ph->Kh * dt);
    p.s2dt = (float)sqrt(2.0 * dt);
    p.half_dt = (float)(0.5 * dt);
    p.kz_kind = ph->kz_kind;
    p.Kz_const = (float)ph->Kz_const;
    p.ku = (float)ph->kappa_ustar;
    p.z0 = (float)ph->z0;
    p.H_mix = (float)ph->H_mix;
    p.inv_Hmix = ph->H_mix > 0 ? (float)(1.0 / ph->H_mix) : 0.0f;
    p.H_top = ph->H_lid > 0.0 ? (float)ph->H_lid : INFINITY;
    if (src->v_d > 0.0 && ph->h_s > 0.0) {
        p.dry_c1 = (float)(2.0 * src->v_d / ph->h_s);
        p.dry_c2 = (float)(2.0 * src->v_d / (ph->h_s * ph->h_s));
        p.h_s = (float)ph->h_s;
    }
    if (ph->Lambda0 > 0.0) {
        p.L0 = (float)ph->Lambda0;
        p.rcx = (float)ph->rain_cx; p.rcy = (float)ph->rain_cy;
        const double ca = cos(ph->rain_angle), sa = sin(ph->rain_angle);
        p.r_ca_a = (float)(ca / ph->rain_a); p.r_sa_a = (float)(sa / ph->rain_a);
        p.r_ca_b = (float)(ca / ph->rain_b); p.r_sa_b = (float)(sa / ph->rain_b);
        p.inv_edge = (float)(1.0 / ph->rain_edge);
    }
    for (int n = 0; n < ph->n_nuc; ++n) {
        const double lam = ph->lambda[n];
        p.lam[n] = (float)lam;
        p.lam_l2e[n] = (float)(lam * 1.4426950408889634);
        p.cdec[n] = (float)(-expm1(-lam * dt));
        p.edec[n] = (float)exp(-lam * dt);
    }
    const lpm_grid& dg = acc->dep_grid;
    p.dep = acc->dep; p.ledger = acc->ledger; p.err = acc->err;
    p.dnx = dg.nx; p.dny = dg.ny; p.dmode = dg.mode;
    p.dx0 = dg.x0; p.dy0 = dg.y0;
    p.dinv_dx = 1.0 / dg.dx; p.dinv_dy = 1.0 / dg.dy;
    p.dscale = dg.density ? (float)(1.0 / (dg.dx * dg.dy)) : 1.0f;

    if (p.i_hi <= 0) return LPM_OK;
    const unsigned nb = blocks_for(p.i_hi);
    hipStream_t s = (hipStream_t)stream;
    const bool time = fld->nt > 1;
    const bool dep = p.dry_c1 > 0.0f || p.L0 > 0.0f;
    const int kz = ph->kz_kind;
    const bool lev = fld->z_levels != nullptr;
    if (fld->ncomp == 2) {
        if (time) launch_step_lev<2, true>(lev, ph->n_nuc, kz, dep, nb, s, p);
        else launch_step_lev<2, false>(lev, ph->n_nuc, kz, dep, nb, s, p);
    } else {
        if (time) launch_step_lev<3, true>(lev, ph->n_nuc, kz, dep, nb, s, p);
        else launch_step_lev<3, false>(lev, ph->n_nuc, kz, dep, nb, s, p);
    }
    return hip_status("lpm_step_particles");
}

int lpm_step_particles(const lpm_state* st, const lpm_source* src, const lpm_schedule* sch,
                       const lpm_field* fld, const lpm_physics* ph, int32_t step0,
                       int32_t n_steps, const lpm_accum* acc, lpm_stream stream)
{
    return step_impl(st, src, sch, fld, ph, step0, n_steps, acc, 0, 1, 0, nullptr, 0, stream);
}

int lpm_step_particles_record(const lpm_state* st, const lpm_source* src,
                              const lpm_schedule* sch, const lpm_field* fld,
                              const lpm_physics* ph, int32_t step0, int32_t n_steps,
                              const lpm_accum* acc, int32_t rec_step0, int32_t rec_every,
                              int32_t n_rec, float* rec, int64_t rec_stride, lpm_stream stream)
{
    return step_impl(st, src, sch, fld, ph, step0, n_steps, acc, rec_step0, rec_every, n_rec, rec,
                     rec_stride, stream);
}

int lpm_grid_concentration(const lpm_state* st, const lpm_source* src, const lpm_schedule* sch,
                           const lpm_physics* ph, const lpm_grid* grid, int32_t step,
                           double* acc_scratch, float* out, lpm_stream stream)
{
    g_msg[0] = 0;
    int rc = check_state(st, sch);
    if (rc) return rc;
    if (!src) return fail(LPM_EINVAL, "null source");
    if ((rc = check_physics(ph)) || (rc = check_grid(grid, false))) return rc;
    if (!acc_scratch || !out || ((uintptr_t)acc_scratch & 7u) || !aligned4(out))
        return fail(LPM_EINVAL, "null or misaligned grid buffers");
    if (step < 0) return fail(LPM_EINVAL, "step must be >= 0");
    lpm::GridConst g;
    memset(&g, 0, sizeof g);
    g.X = st->x; g.Y = st->y; g.Z = st->z; g.M = st->m;
    g.n_total = sch->n_total; g.id_base = sch->id_base; g.id_stride = sch->id_stride;
    g.s_release = sch->s_release;
    g.step = step;
    g.i_hi = first_local_born_at_or_after(sch, (long long)step + 1);
    g.nnuc = ph->n_nuc;
    g.mode = grid->mode;
    g.a0 = (float)a0_of(src, sch, ph);
    g.dt = (float)ph->dt;
    g.scale = 1.0f;
    for (int n = 0; n < ph->n_nuc; ++n) g.lam_l2e[n] = (float)(ph->lambda[n] * 1.4426950408889634);
    g.nx = grid->nx; g.ny = grid->ny; g.nz = grid->nz;
    g.x0 = grid->x0; g.y0 = grid->y0; g.z0 = grid->z0;
    g.inv_dx = 1.0 / grid->dx; g.inv_dy = 1.0 / grid->dy; g.inv_dz = 1.0 / grid->dz;
    g.cells = (long long)grid->nx * grid->ny * grid->nz;
    g.acc = acc_scratch;
    const long long total = g.cells * ph->n_nuc;
    const double vol = grid->density ? grid->dx * grid->dy * grid->dz : 1.0;
    hipStream_t s = (hipStream_t)stream;
    const unsigned fb = blocks_for(total) < 8192 ? blocks_for(total) : 8192;
    hipLaunchKernelGGL(lpm::fill_f64, dim3(fb), dim3(lpm::kBlock), 0, s, acc_scratch, total);
    if (g.i_hi > 0) {
        const dim3 nb(blocks_for(g.i_hi)), bs(lpm::kBlock);
        switch (ph->n_nuc) {
        case 1: hipLaunchKernelGGL(lpm::conc_kernel<1>, nb, bs, 0, s, g); break;
        case 2: hipLaunchKernelGGL(lpm::conc_kernel<2>, nb, bs, 0, s, g); break;
        case 3: hipLaunchKernelGGL(lpm::conc_kernel<3>, nb, bs, 0, s, g); break;
        default: hipLaunchKernelGGL(lpm::conc_kernel<4>, nb, bs, 0, s, g); break;
        }
    }
    hipLaunchKernelGGL(lpm::to_f32, dim3(fb), dim3(lpm::kBlock), 0, s, acc_scratch, out, total,
                       1.0 / vol);
    return hip_status("lpm_grid_concentration");
}

int lpm_grid_deposition(const lpm_accum* acc, float* out, lpm_stream stream)
{
    g_msg[0] = 0;
    int rc = check_accum(acc);
    if (rc) return rc;
    if (!out || !aligned4(out)) return fail(LPM_EINVAL, "null or misaligned output");
    const long long total = (long long)acc->n_nuc * acc->dep_grid.nx * acc->dep_grid.ny;
    const unsigned fb = blocks_for(total) < 8192 ? blocks_for(total) : 8192;
    hipLaunchKernelGGL(lpm::to_f32, dim3(fb), dim3(lpm::kBlock), 0, (hipStream_t)stream, acc->dep,
                       out, total, 1.0);
    return hip_status("lpm_grid_deposition");
}

int lpm_read_ledger(const lpm_accum* acc, double* host_out, lpm_stream stream)
{
    g_msg[0] = 0;
    int rc = check_accum(acc);
    if (rc) return rc;
    if (!host_out) return fail(LPM_EINVAL, "null output");
    double buf[LPM_LEDGER_SLOTS * LPM_LEDGER_STRIDE];
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(buf, acc->ledger, sizeof buf, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return hip_status("lpm_read_ledger");
    for (int n = 0; n < acc->n_nuc; ++n)
        for (int e = 0; e < 4; ++e) {
            double t = 0.0;
            for (int k = 0; k < LPM_LEDGER_SLOTS; ++k) t += buf[k * LPM_LEDGER_STRIDE + n * 4 + e];
            host_out[n * 4 + e] = t;
        }
    double steps = 0.0;
    for (int k = 0; k < LPM_LEDGER_SLOTS; ++k) steps += buf[k * LPM_LEDGER_STRIDE + LPM_LEDGER_PSTEPS];
    host_out[acc->n_nuc * 4] = steps;
    return LPM_OK;
}

int lpm_check(const lpm_accum* acc, lpm_stream stream)
{
    g_msg[0] = 0;
    if (!acc || !acc->err) return fail(LPM_EINVAL, "null accumulator");
    uint32_t e = 0;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(&e, acc->err, sizeof e, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return hip_status("lpm_check");
    if (e & 1u) return fail(LPM_ENONFINITE, "a particle coordinate or mass became non-finite");
    return LPM_OK;
}

}  // extern "C"

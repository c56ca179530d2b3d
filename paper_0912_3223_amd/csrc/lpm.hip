// liblpm: HIP kernels and C ABI of the particle-dispersion hot path for
// gfx950 (MI355X).  The model is the stochastic Lagrangian particle model of
// Molnar Jr. et al. (arXiv:0912.3223, Sec. 2 and 3.2); see include/lpm.h for
// the interface contract.
//
// Kernels
//  - release_kernel: writes the initial state of the particles born in a
//    window of steps (one thread per particle, coalesced float stores).
//  - step_kernel: persistent; each lane takes particles from a work queue,
//    loads a particle's state once, advances it through the window in
//    registers and stores it once.  Random numbers come from Philox in
//    registers and the wind is gathered from the L2/MALL-resident field.
//    Deposition is aggregated in four levels before it reaches HBM: per lane
//    while the particle stays in one cell quad (registers), a per-wave
//    staging list of quads, a per-wave LDS hash table of cells (FP64 LDS
//    atomics), and once per table entry into the FP64 grid.  The ledger is
//    reduced per block before one atomic per entry into one of
//    LPM_LEDGER_SLOTS spread-out slots.
//  - bin_count_kernel, scan_*, bin_scatter_kernel, tile_conc_kernel: the
//    concentration of recorded output steps, binned by column tile and
//    summed per tile in LDS (owner computes: each output cell written once).
//  - conc_kernel + to_f32: single-step gridding of the live state (scatter
//    of activity to an FP64 grid through an LDS hash, then conversion).
//  The shared queue spreads live particles evenly over the 8 XCDs.
#include <hip/hip_runtime.h>

#include <limits.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <type_traits>
#include <atomic>
#include <mutex>
#include <utility>
#include <vector>

#include "lpm.h"
#include "lpm_device.h"
#include "lpm_host.h"

namespace lpm {

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

// Wave-private histogram for the persistent step kernel.  The lanes of a wave
// run independent particles and never meet at a block barrier, so each wave
// owns a table; when half of its slots are taken, the wave (which executes in
// lockstep) moves the table to the global grid and empties it.
// ---------------------------------------------------------------------------
// Release (Sec. 2: particles released from the point source every step).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void release_kernel(float* X, float* Y, float* Z,
                                                         float* M, float* XL, float* YL,
                                                         long long i_lo,
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
        if (XL) {
            XL[i] = 0.0f;
            YL[i] = 0.0f;
        }
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
    float bc[4][4];  // chain activity coefficients (identity: independent nuclides)
    int nx, ny, nz, chain;
    double x0, y0, z0, inv_dx, inv_dy, inv_dz;
    long long cells;
    double* acc;
    // record gridding: positions recorded (n_pos) and, for records of a
    // launch with a work order, the particle of each position (else the
    // position is the particle); i_hi then bounds the particle indices
    const int* order;
    long long n_pos;
};

// Activities of the nuclides at age t, scaled by f.
template <int NNUC>
__device__ __forceinline__ void activities(const GridConst& g, float t, float f, float (&A)[NNUC])
{
    float E[NNUC];
#pragma unroll
    for (int n = 0; n < NNUC; ++n) E[n] = exp2f(-g.lam_l2e[n] * t);
#pragma unroll
    for (int n = 0; n < NNUC; ++n) {
        float a = E[n];
        if (g.chain) {
            a = 0.0f;
#pragma unroll
            for (int j = 0; j <= n; ++j) a = fmaf(g.bc[n][j], E[j], a);
        }
        A[n] = f * a;
    }
}

template <int NNUC>
__global__ __launch_bounds__(kBlock) void conc_kernel(const GridConst g)
{
    using Table = CellTable<NNUC, NNUC <= 2 ? 11 : 10>;
    __shared__ int tab_key[Table::kSlots];
    __shared__ double tab_val[NNUC * Table::kSlots];
    Table tab{tab_key, tab_val};
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    const float m = i < g.i_hi ? g.M[i] : 0.0f;
    long long b = 0;
    if (m > 0.0f) b = birth(g.id_base + i * g.id_stride, g.s_release, g.n_total);
    const bool live = m > 0.0f && b <= g.step;
    if (!__syncthreads_or(live)) return;  // no airborne particle in this block
    tab.init();
    __syncthreads();
    if (live) {
        const float age = (float)(g.step + 1 - (int)b) * g.dt;
        float A[NNUC];
        activities<NNUC>(g, age, g.a0 * m * g.scale, A);
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

// Concentration of recorded states (output steps s_k = rec_step0 + k
// rec_every), owner-computes.  Particles released far apart in time spread
// over thousands of cells, so a per-block hash of cells cannot fold their
// contributions; instead the records are binned by the horizontal tile of the
// grid they touch, and one block per (tile, output step) sums every
// contribution to its own cells in a dense FP64 LDS array and writes each
// cell once, as float.  No global floating-point atomics, no FP64 grid in HBM.
//
// Bins.  Tiles are TX x TY columns of full height.  A record's CIC base corner
// (ix, iy) = floor(f - 1/2) touches columns ix, ix + 1 (and iy, iy + 1); with
// ax = ix + 1 it is binned to tile (ax / TX, ay / TY) of a bin lattice one
// wider than the owner tiles, where both of its columns lie in that tile
// except, when ax is a multiple of TX, column ix, which lies in the tile to
// the left (an "x edge" record; the same in y).  Each bin holds four classes
// in the order: interior, x edge, x and y edge, y edge, so that the owner of
// tile (ox, oy) reads its own bin whole, classes 1-2 of bin (ox + 1, oy),
// classes 2-3 of bin (ox, oy + 1) and class 2 of bin (ox + 1, oy + 1): four
// contiguous index ranges.  Nearest-grid-point records (mode 0) use class 0 of
// the tile of their cell.
// A record counts if the particle was born by s_k and still active after it
// and its mass is positive.
constexpr int kRecChunk = 8 * kBlock;
// LDS bytes per bin: the counting pass keeps a 32-bit count, the scatter pass
// a 32-bit rank and a 64-bit base per bin of the output step.
constexpr int kBinCountLds = 4;     // LDS bytes per bin of the count pass
constexpr int kBinScatterLds = 12;  // and of the scatter pass
constexpr int kBinWindow = 2048;    // bins in a block's LDS window (24 KB for the scatter)

struct TileConst {
    int tx, ty;        // tile width and depth in cells (powers of two)
    int lx, ly;        // their base-2 logarithms
    int ps;            // doubles per level of the LDS tile: tx ty, plus one of padding
                       // when tx ty > 1 (the same corner of records on different levels
                       // then falls in different LDS banks)
    int ntx, nty;      // owner tiles
    int nbx, nby;      // bin tiles (nx / tx + 1, ny / ty + 1)
    long long nbk;     // bins per output step: nbx nby 4
    int nwin;          // bins of a block's LDS window: min(nbk, kBinWindow)
    unsigned long long* off;  // [n_rec nbk] first index of each bin
    unsigned long long* cur;  // [n_rec nbk] counts, then end of each bin
    unsigned long long* bsum; // per-block sums of the scan
    float4* brec;             // the binned records (x, y, z, m), in bin order
    int* bborn;               // and the birth step of each
    const int* chunk_end;     // per chunk of kRecChunk ids: the largest `last` in it
    unsigned long long cap;   // entries of brec and bborn
    float* out;
    double inv_vol;
};

// Bin of a record within its output step, or -1 if no grid cell receives
// any of it (also for a non-finite position).  The cell index and weights use
// the same double-precision arithmetic as conc_kernel.
__device__ __forceinline__ int record_bin(const GridConst& g, const TileConst& t, float x, float y,
                                          float z)
{
    const double fx = ((double)x - g.x0) * g.inv_dx;
    const double fy = ((double)y - g.y0) * g.inv_dy;
    const double fz = ((double)z - g.z0) * g.inv_dz;
    if (g.mode == 0) {
        const double ix = floor(fx), iy = floor(fy), iz = floor(fz);
        if (!(ix >= 0.0 && iy >= 0.0 && iz >= 0.0 && ix < (double)g.nx && iy < (double)g.ny &&
              iz < (double)g.nz))
            return -1;
        return ((((int)iy >> t.ly) * t.nbx) + ((int)ix >> t.lx)) * 4;
    }
    const double ix = floor(fx - 0.5), iy = floor(fy - 0.5), iz = floor(fz - 0.5);
    if (!(ix >= -1.0 && iy >= -1.0 && iz >= -1.0 && ix < (double)g.nx && iy < (double)g.ny &&
          iz < (double)g.nz))
        return -1;
    const int ax = (int)ix + 1, ay = (int)iy + 1;
    const bool ex = ax > 0 && (ax & (t.tx - 1)) == 0, ey = ay > 0 && (ay & (t.ty - 1)) == 0;
    const int cls = ex ? (ey ? 2 : 1) : (ey ? 3 : 0);
    return ((ay >> t.ly) * t.nbx + (ax >> t.lx)) * 4 + cls;
}

// Shared by the two binning kernels: the records of a thread's kRecChunk /
// kBlock positions at output step `step` (r), the birth steps of their
// particles (b) and their bins (-1 for a record that does not count).  The
// `last` words (and order entries) are loaded together, then the records,
// so that a thread waits for two rounds of loads, not one per record.
constexpr int kRecPer = kRecChunk / kBlock;
__device__ __forceinline__ void binned_records(const GridConst& g, const TileConst& t,
                                               const float4* rec_k, const int* last,
                                               long long i0, int step, float4 (&r)[kRecPer],
                                               int (&b)[kRecPer], int (&bin)[kRecPer])
{
    // (every load is issued, a record that does not count reading the
    // block's first one, whose line the wave shares: conditional loads make
    // the compiler wait for each before issuing the next)
    int lst[kRecPer];
    long long pi[kRecPer];  // particle of each position
#pragma unroll
    for (int u = 0; u < kRecPer; ++u) {  // n_pos >= 1: position clamped into the arrays
        const long long q = min(i0 + u * kBlock + threadIdx.x, g.n_pos - 1);
        lst[u] = last[q];
        pi[u] = g.order ? (long long)g.order[q] : q;
    }
    bool live[kRecPer];
#pragma unroll
    for (int u = 0; u < kRecPer; ++u) {
        const bool ok = i0 + u * kBlock + threadIdx.x < g.n_pos &&
                        (unsigned long long)pi[u] < (unsigned long long)g.i_hi;
        b[u] = ok ? (int)birth(g.id_base + pi[u] * g.id_stride, g.s_release, g.n_total) : 0;
        live[u] = ok && b[u] <= step && step < lst[u];
    }
#pragma unroll
    for (int u = 0; u < kRecPer; ++u)  // i0 < n_pos (the chunk is not idle)
        r[u] = rec_k[live[u] ? i0 + u * kBlock + threadIdx.x : i0];
#pragma unroll
    for (int u = 0; u < kRecPer; ++u)
        bin[u] = live[u] && r[u].w > 0.0f ? record_bin(g, t, r[u].x, r[u].y, r[u].z) : -1;
}

// A chunk of positions holds no record of an output step when all of its
// particles stopped by then, or (positions that are particles: local ids
// are born in increasing order) when its first id is born after the step.
__device__ __forceinline__ bool chunk_idle(const GridConst& g, const TileConst& t, long long i0,
                                           int step)
{
    return i0 >= g.n_pos || step >= t.chunk_end[blockIdx.x] ||
           (!g.order && birth(g.id_base + i0 * g.id_stride, g.s_release, g.n_total) > step);
}

// Pass 0: the largest `last` of each chunk (one block per chunk).
__global__ __launch_bounds__(kBlock) void chunk_end_kernel(const int* last, long long i_hi,
                                                           int* chunk_end)
{
    __shared__ int wmax[kBlock / 64];
    const long long i0 = (long long)blockIdx.x * kRecChunk;
    int v = INT_MIN;
#pragma unroll
    for (int u = 0; u < kRecChunk / kBlock; ++u) {
        const long long i = i0 + u * kBlock + threadIdx.x;
        if (i < i_hi) v = max(v, last[i]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = wmax[0];
#pragma unroll
        for (int w = 1; w < kBlock / 64; ++w) m = max(m, wmax[w]);
        chunk_end[blockIdx.x] = m;
    }
}

// The lowest bin of a block's records (records of consecutive ids lie close
// together, so the block's bins mostly fall in a window of kBinWindow bins
// from there).  Every thread of the block calls it.
template <int N>
__device__ __forceinline__ int bin_low(const int (&bin)[N])
{
    __shared__ int s_lo;
    int a = INT_MAX;
#pragma unroll
    for (int u = 0; u < N; ++u)
        if (bin[u] >= 0) a = min(a, bin[u]);
    if (threadIdx.x == 0) s_lo = INT_MAX;
    __syncthreads();
    if (a != INT_MAX) atomicMin(&s_lo, a);
    __syncthreads();
    return s_lo;
}

// Pass 1: records per bin: counted in an LDS window of nwin bins from the
// block's lowest bin, records beyond the window with global atomics.
__global__ __launch_bounds__(kBlock) void bin_count_kernel(const GridConst g, const TileConst t,
                                                           const float4* rec, const int* last,
                                                           long long rec_stride, int rec_step0,
                                                           int rec_every)
{
    extern __shared__ unsigned long long lds_u64[];
    uint32_t* hist = reinterpret_cast<uint32_t*>(lds_u64);  // [nwin]
    const int k = blockIdx.y;
    const int step = rec_step0 + k * rec_every;
    const long long i0 = (long long)blockIdx.x * kRecChunk;
    if (chunk_idle(g, t, i0, step)) return;
    const float4* rec_k = rec + (long long)k * rec_stride;
    unsigned long long* cnt = t.cur + (long long)k * t.nbk;
    int bin[kRecPer];
    {
        float4 r[kRecPer];
        int born[kRecPer];
        binned_records(g, t, rec_k, last, i0, step, r, born, bin);
    }
    bool any = false;
#pragma unroll
    for (int u = 0; u < kRecPer; ++u) any |= bin[u] >= 0;
    if (!__syncthreads_or(any)) return;
    const int lo = bin_low(bin);
    for (int b = threadIdx.x; b < t.nwin; b += kBlock) hist[b] = 0u;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kRecChunk / kBlock; ++u)
        if (bin[u] >= 0) {
            const int d = bin[u] - lo;
            if (d < t.nwin) atomicAdd(hist + d, 1u);
            else atomicAdd(cnt + bin[u], 1ull);
        }
    __syncthreads();
    for (int b = threadIdx.x; b < t.nwin; b += kBlock)
        if (hist[b]) atomicAdd(cnt + lo + b, (unsigned long long)hist[b]);
}

// Pass 3: the records into their bins.  A block ranks its records per bin in
// its LDS window, reserves one range per bin with a single global atomic and
// writes the records (and birth steps) there, so that the tile pass reads
// its records contiguously; records beyond the window take one global atomic
// each.
__global__ __launch_bounds__(kBlock) void bin_scatter_kernel(const GridConst g, const TileConst t,
                                                             const float4* rec, const int* last,
                                                             long long rec_stride, int rec_step0,
                                                             int rec_every)
{
    extern __shared__ unsigned long long lds_u64[];
    const int k = blockIdx.y;
    const int step = rec_step0 + k * rec_every;
    const long long i0 = (long long)blockIdx.x * kRecChunk;
    if (chunk_idle(g, t, i0, step)) return;
    const float4* rec_k = rec + (long long)k * rec_stride;
    unsigned long long* cur = t.cur + (long long)k * t.nbk;
    int bin[kRecPer], born[kRecPer];
    float4 r4[kRecPer];
    binned_records(g, t, rec_k, last, i0, step, r4, born, bin);
    bool any = false;
#pragma unroll
    for (int u = 0; u < kRecPer; ++u) any |= bin[u] >= 0;
    if (!__syncthreads_or(any)) return;
    unsigned long long* base = lds_u64;                               // [nwin]
    uint32_t* rank = reinterpret_cast<uint32_t*>(lds_u64 + t.nwin);   // [nwin]
    const int lo = bin_low(bin);
    for (int b = threadIdx.x; b < t.nwin; b += kBlock) rank[b] = 0u;
    __syncthreads();
    uint32_t r[kRecChunk / kBlock];
#pragma unroll
    for (int u = 0; u < kRecChunk / kBlock; ++u)
        r[u] = bin[u] >= 0 && bin[u] - lo < t.nwin ? atomicAdd(rank + (bin[u] - lo), 1u) : 0u;
    __syncthreads();
    for (int b = threadIdx.x; b < t.nwin; b += kBlock)
        if (rank[b]) base[b] = atomicAdd(cur + lo + b, (unsigned long long)rank[b]);
    __syncthreads();
    // positions first (the atomics of records beyond the window issued
    // together), then every store: a store after each atomic would wait for
    // the stores before it
    unsigned long long pos[kRecPer];
#pragma unroll
    for (int u = 0; u < kRecPer; ++u) {
        const int d = bin[u] - lo;
        pos[u] = bin[u] < 0 ? ~0ull : d < t.nwin ? base[d] + r[u] : atomicAdd(cur + bin[u], 1ull);
    }
#pragma unroll
    for (int u = 0; u < kRecPer; ++u)
        if (pos[u] < t.cap) {
            t.brec[pos[u]] = r4[u];
            t.bborn[pos[u]] = born[u];
        }
}

// Pass 2: exclusive scan of the counts (cur) into off, and cur = off.  Three
// launches: block sums, a one-block scan of the sums, the block scans.
constexpr int kScanPer = 8;
constexpr int kScanChunk = kScanPer * kBlock;

__device__ __forceinline__ unsigned long long block_exclusive_scan(unsigned long long v,
                                                                   unsigned long long* s,
                                                                   unsigned long long* total)
{
    s[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int d = 1; d < kBlock; d <<= 1) {
        const unsigned long long a = threadIdx.x >= (unsigned)d ? s[threadIdx.x - d] : 0ull;
        __syncthreads();
        s[threadIdx.x] += a;
        __syncthreads();
    }
    const unsigned long long incl = s[threadIdx.x];
    *total = s[kBlock - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kBlock) void scan_sums_kernel(const unsigned long long* cnt,
                                                           long long n, unsigned long long* bsum)
{
    __shared__ unsigned long long s[kBlock];
    const long long a = (long long)blockIdx.x * kScanChunk + (long long)threadIdx.x * kScanPer;
    unsigned long long v = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j)
        if (a + j < n) v += cnt[a + j];
    unsigned long long tot;
    block_exclusive_scan(v, s, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void scan_bsum_kernel(unsigned long long* bsum, long long nb)
{
    __shared__ unsigned long long s[kBlock];
    unsigned long long carry = 0;
    for (long long a = 0; a < nb; a += kBlock) {
        const long long j = a + threadIdx.x;
        const unsigned long long v = j < nb ? bsum[j] : 0ull;
        unsigned long long tot;
        const unsigned long long ex = block_exclusive_scan(v, s, &tot);
        if (j < nb) bsum[j] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(kBlock) void scan_apply_kernel(unsigned long long* cur,
                                                            unsigned long long* off, long long n,
                                                            const unsigned long long* bsum)
{
    __shared__ unsigned long long s[kBlock];
    const long long a = (long long)blockIdx.x * kScanChunk + (long long)threadIdx.x * kScanPer;
    unsigned long long c[kScanPer], v = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        c[j] = a + j < n ? cur[a + j] : 0ull;
        v += c[j];
    }
    unsigned long long tot;
    unsigned long long run = bsum[blockIdx.x] + block_exclusive_scan(v, s, &tot);
#pragma unroll
    for (int j = 0; j < kScanPer; ++j)
        if (a + j < n) {
            off[a + j] = run;
            cur[a + j] = run;
            run += c[j];
        }
}

// Work order of a step launch: the particles active at its first step sorted
// by the wind node they are at (an LSD radix sort of (node, index) pairs,
// 8 bits per pass, counts in LDS: no global atomics per particle), then
// those born in the window in index order, then the inactive ones.
struct OrderConst {
    const float* X;
    const float* Y;
    const float* Z;
    const float* M;
    long long n_old;   // local indices born before the first step: [0, n_old)
    long long n_all;   // the launch's particles: [0, n_all)
    float fcx, fcy, inv_dx, inv_dy, inv_dz;  // node i = floor(x inv_dx + fcx); inv_dz 0: k = 0
    int nx, ny, nz;
    unsigned long long* count;  // [0] active, [1] inactive particles
    unsigned* keys;             // nodes of the active particles
    int* vals;                  // their indices
    int* order;
};

// Node (j nx + i) nz + k of a particle with mass m at (x, y, z), or -1 when
// it is inactive.
__device__ __forceinline__ long long order_node(const OrderConst& o, float m, float x, float y,
                                                float z)
{
    if (!(m > 0.0f)) return -1;
    const int ix = min(max((int)floorf(fmaf(x, o.inv_dx, o.fcx)), 0), o.nx - 1);
    const int iy = min(max((int)floorf(fmaf(y, o.inv_dy, o.fcy)), 0), o.ny - 1);
    const int iz = o.inv_dz > 0.0f ? min(max((int)floorf(z * o.inv_dz), 0), o.nz - 1) : 0;
    return ((long long)iy * o.nx + ix) * o.nz + iz;
}

// Particles per block of the sort kernels.
constexpr int kSortTile = 16 * kBlock;

// Active particles -> (node, index) pairs; inactive ones straight to the end
// of the order (from the back).  A block takes kSortTile particles at a time
// and claims its slots with one atomic per list (the lists' order is left
// open).
__global__ __launch_bounds__(kBlock) void order_keys_kernel(const OrderConst o)
{
    constexpr int kPer = kSortTile / kBlock;
    __shared__ unsigned long long scan_s[kBlock];
    __shared__ unsigned long long base_s[2];
    for (long long a = (long long)blockIdx.x * kSortTile; a < o.n_old;
         a += (long long)gridDim.x * kSortTile) {
        // every load of the tile issued before any is used (the state of an
        // index past n_old is that of the last one, and not used): reading
        // m first and the position only for live particles made each thread
        // wait for its loads one particle at a time
        float m4[kPer][4];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const long long e = min(a + (long long)j * kBlock + threadIdx.x, o.n_old - 1);
            m4[j][0] = as_global(o.M)[e];
            m4[j][1] = as_global(o.X)[e];
            m4[j][2] = as_global(o.Y)[e];
            m4[j][3] = as_global(o.Z)[e];
        }
        long long node[kPer];
        unsigned n_act = 0u, n_off = 0u;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const long long e = a + (long long)j * kBlock + threadIdx.x;
            node[j] = e < o.n_old ? order_node(o, m4[j][0], m4[j][1], m4[j][2], m4[j][3]) : -2;
            n_act += node[j] >= 0;
            n_off += node[j] == -1;
        }
        // active counts in the low word, inactive in the high word (<= 4096 each)
        unsigned long long tot;
        const unsigned long long ex =
            block_exclusive_scan(((unsigned long long)n_off << 32) | n_act, scan_s, &tot);
        if (threadIdx.x == 0) {
            base_s[0] = atomicAdd(o.count, tot & 0xFFFFFFFFull);
            base_s[1] = atomicAdd(o.count + 1, tot >> 32);
        }
        __syncthreads();
        unsigned long long pa = base_s[0] + (ex & 0xFFFFFFFFull);
        unsigned long long pd = base_s[1] + (ex >> 32);
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const long long e = a + (long long)j * kBlock + threadIdx.x;
            if (node[j] >= 0) {
                as_global(o.keys)[pa] = (unsigned)node[j];
                as_global(o.vals)[pa] = (int)e;
                ++pa;
            } else if (node[j] == -1) {
                as_global(o.order)[o.n_all - 1 - (long long)pd] = (int)e;
                ++pd;
            }
        }
        __syncthreads();  // base_s and scan_s are reused
    }
}

// The particles born in the window follow the active ones.
__global__ __launch_bounds__(kBlock) void order_born_kernel(const OrderConst o)
{
    const long long n_active = (long long)o.count[0];
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = o.n_old + (long long)blockIdx.x * kBlock + threadIdx.x; i < o.n_all; i += stride)
        as_global(o.order)[n_active + (i - o.n_old)] = (int)i;
}

// One pass of the radix sort: 8 bits at `shift`.  Block b owns elements
// [b kSortTile, (b + 1) kSortTile) of the `n` (device count) pairs.
struct SortPass {
    const unsigned* kin;
    const int* vin;
    unsigned* kout;   // null in the last pass
    int* vout;
    const unsigned long long* n;
    unsigned long long* table;  // [256][nblocks]: digit counts, then their exclusive offsets
    long long nblocks;
    int shift;
};

__global__ __launch_bounds__(kBlock) void radix_hist_kernel(const SortPass c)
{
    static_assert(kBlock == 256, "one digit per thread");
    __shared__ unsigned h[256];
    h[threadIdx.x] = 0u;
    __syncthreads();
    const long long n = (long long)*c.n;
    const long long a = (long long)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortTile / kBlock; ++r) {
        const long long e = a + (long long)r * kBlock + threadIdx.x;
        if (e < n) atomicAdd(&h[(as_global(c.kin)[e] >> c.shift) & 255u], 1u);
    }
    __syncthreads();
    c.table[(long long)threadIdx.x * c.nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: the tile in rounds of one element per thread, in order;
// within a wave the lanes of one digit find each other with eight ballots.
__global__ __launch_bounds__(kBlock) void radix_scatter_kernel(const SortPass c)
{
    __shared__ unsigned long long base[256];  // next slot of each digit
    __shared__ unsigned cnt[kBlock / 64][256];  // per wave and digit, this round
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    base[threadIdx.x] = c.table[(long long)threadIdx.x * c.nblocks + blockIdx.x];
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) cnt[q][threadIdx.x] = 0u;
    __syncthreads();
    const long long n = (long long)*c.n;
    const long long a = (long long)blockIdx.x * kSortTile;
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (int r = 0; r < kSortTile / kBlock; ++r) {
        const long long e = a + (long long)r * kBlock + threadIdx.x;
        const bool valid = e < n;
        unsigned key = 0u, d = 0u;
        int val = 0;
        if (valid) {
            key = as_global(c.kin)[e];
            val = as_global(c.vin)[e];
            d = (key >> c.shift) & 255u;
        }
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool one = (d >> bit) & 1u;
            const unsigned long long on = __ballot(valid && one);
            peers &= one ? on : ~on;
        }
        const unsigned rank = (unsigned)__popcll(peers & lt);
        if (valid && rank == 0u) cnt[w][d] = (unsigned)__popcll(peers);
        __syncthreads();
        if (valid) {
            unsigned pre = 0u;
            for (int q = 0; q < w; ++q) pre += cnt[q][d];
            const unsigned long long dst = base[d] + pre + rank;
            if (c.kout) as_global(c.kout)[dst] = key;
            as_global(c.vout)[dst] = val;
        }
        __syncthreads();
        unsigned sum = 0u;
#pragma unroll
        for (int q = 0; q < kBlock / 64; ++q) {
            sum += cnt[q][threadIdx.x];
            cnt[q][threadIdx.x] = 0u;
        }
        base[threadIdx.x] += sum;
        __syncthreads();
    }
}

// Pass 4: one block per (owner tile, output step).  LDS: the tile's cells,
// double [NNUC][nz][ps] (ty tx cells per level, padded).
constexpr int kTileBatch = 4;
// A tile holding more than kSplitMin records of an output step (the ones
// near the source) is shared by up to kTileSplit blocks, each summing a
// slice of its records; their FP64 tile sums are added to the output (zeroed
// beforehand) with FP32 atomics.  Other tiles keep one block, which writes
// its cells once.  (24 h run, gridding time per run outside the step
// kernel: 94 ms unsplit, 70 ms with 4 x 16384, 68.5 ms with 8 x 8192.)
constexpr int kTileSplit = 8;
constexpr long long kSplitMin = 8192;
template <int NNUC>
__global__ __launch_bounds__(kBlock) void tile_conc_kernel(const GridConst g, const TileConst t,
                                                           int rec_step0, int rec_every)
{
    extern __shared__ double tile[];
    const int ox = blockIdx.x % t.ntx, oy = blockIdx.x / t.ntx, k = blockIdx.y;
    const int step = rec_step0 + k * rec_every;
    const int xa = ox * t.tx, ya = oy * t.ty;
    const int wx_n = min(t.tx, g.nx - xa), wy_n = min(t.ty, g.ny - ya);
    const int ncell = g.nz * t.ty * t.tx;
    // the four index ranges (see the bin layout above)
    const long long b0 = (long long)k * t.nbk + ((long long)oy * t.nbx + ox) * 4;
    const long long bx1 = b0 + 4, by1 = b0 + (long long)t.nbx * 4, bxy = by1 + 4;
    const bool has_x = ox + 1 < t.nbx, has_y = oy + 1 < t.nby;
    const long long lo0 = (long long)t.off[b0];
    const long long e0 = (long long)t.cur[b0 + 3] - lo0;
    const long long lo1 = has_x ? (long long)t.off[bx1 + 1] : 0;
    const long long e1 = e0 + (has_x ? (long long)t.cur[bx1 + 2] - lo1 : 0);
    const long long lo2 = has_y ? (long long)t.off[by1 + 2] : 0;
    const long long e2 = e1 + (has_y ? (long long)t.cur[by1 + 3] - lo2 : 0);
    const long long lo3 = has_x && has_y ? (long long)t.off[bxy + 2] : 0;
    const long long total = e2 + (has_x && has_y ? (long long)t.cur[bxy + 2] - lo3 : 0);
    float* out = t.out + (long long)k * NNUC * g.cells;
    // most tiles hold no record (the plume covers a few per output step):
    // their cells were cleared by one coalesced fill before this pass
    if (total == 0) return;
    const int nsplit = total <= kSplitMin
                           ? 1
                           : (int)min((long long)kTileSplit, (total + kSplitMin - 1) / kSplitMin);
    if ((int)blockIdx.z >= nsplit) return;
    const long long jb = total * blockIdx.z / nsplit, je = total * (blockIdx.z + 1) / nsplit;
    const int ps = t.ps;
    for (int c = threadIdx.x; c < NNUC * g.nz * ps; c += kBlock) tile[c] = 0.0;
    __syncthreads();
    // one record's contributions to the tile's cells
    auto add_record = [&](const float4 r, int b) {
        const float age = (float)(step + 1 - b) * g.dt;
        float A[NNUC];
        activities<NNUC>(g, age, g.a0 * r.w * g.scale, A);
        const double fx = ((double)r.x - g.x0) * g.inv_dx;
        const double fy = ((double)r.y - g.y0) * g.inv_dy;
        const double fz = ((double)r.z - g.z0) * g.inv_dz;
        if (g.mode == 0) {
            const int cx = (int)floor(fx) - xa, cy = (int)floor(fy) - ya, cz = (int)floor(fz);
            if (cx >= 0 && cx < wx_n && cy >= 0 && cy < wy_n && cz >= 0 && cz < g.nz) {
#pragma unroll
                for (int n = 0; n < NNUC; ++n)
                    atomicAdd(&tile[(n * g.nz + cz) * ps + cy * t.tx + cx], (double)A[n]);
            }
            return;
        }
        const double ix = floor(fx - 0.5), iy = floor(fy - 0.5), iz = floor(fz - 0.5);
        const float wx = (float)(fx - 0.5 - ix), wy = (float)(fy - 0.5 - iy);
        const float wz = (float)(fz - 0.5 - iz);
        const int cx0 = (int)ix - xa, cy0 = (int)iy - ya, cz0 = (int)iz;
        for (int c = 0; c < 8; ++c) {
            const int cx = cx0 + (c & 1), cy = cy0 + ((c >> 1) & 1), cz = cz0 + (c >> 2);
            if (!(cx >= 0 && cx < wx_n && cy >= 0 && cy < wy_n && cz >= 0 && cz < g.nz)) continue;
            const float w = ((c & 1) ? wx : 1.0f - wx) * (((c >> 1) & 1) ? wy : 1.0f - wy) *
                            ((c >> 2) ? wz : 1.0f - wz);
#pragma unroll
            for (int n = 0; n < NNUC; ++n)
                atomicAdd(&tile[(n * g.nz + cz) * ps + cy * t.tx + cx], (double)(A[n] * w));
        }
    };
    // A crowded tile (the one holding the source) gets tens of thousands of
    // records: each thread takes kTileBatch of them at a time and issues
    // their loads before using any.  The records of the four ranges lie
    // contiguously in bin order (written so by the scatter pass).
    for (long long j0 = jb + threadIdx.x; j0 < je; j0 += (long long)kTileBatch * kBlock) {
        float4 rr[kTileBatch];
        int bb[kTileBatch];
        bool ok[kTileBatch];
#pragma unroll
        for (int u = 0; u < kTileBatch; ++u) {
            // past the slice: its last entry again (every load issued, no
            // branch around it)
            const long long j = min(j0 + (long long)u * kBlock, je - 1);
            const long long e = j < e0 ? lo0 + j
                              : j < e1 ? lo1 + (j - e0)
                              : j < e2 ? lo2 + (j - e1) : lo3 + (j - e2);
            // (entries past the workspace -- only a work order listing a
            // particle twice could count more records than were born -- were
            // not written by the scatter and are skipped; total > 0 implies
            // cap >= 1)
            ok[u] = j0 + (long long)u * kBlock < je && (unsigned long long)e < t.cap;
            const long long ec = min(e, (long long)t.cap - 1);
            rr[u] = t.brec[ec];
            bb[u] = t.bborn[ec];
        }
#pragma unroll
        for (int u = 0; u < kTileBatch; ++u)
            if (ok[u]) add_record(rr[u], bb[u]);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < NNUC * ncell; c += kBlock) {
        const int xx = c & (t.tx - 1), yy = (c >> t.lx) & (t.ty - 1), zn = c >> (t.lx + t.ly);
        if (xx < wx_n && yy < wy_n) {
            const float v = (float)(tile[zn * ps + (c & (t.tx * t.ty - 1))] * t.inv_vol);
            float* o = out + ((long long)zn * g.ny + ya + yy) * g.nx + xa + xx;
            if (nsplit == 1) *o = v;
            else if (v != 0.0f) atomicAdd(o, v);
        }
    }
}

__global__ __launch_bounds__(kBlock) void fill_f64(double* p, long long n)
{
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}

__global__ __launch_bounds__(kBlock) void fill_u32(uint32_t* p, long long n)
{
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

// Time-pair copy of one field interval: node (k, j, i) of the two time slabs
// a, b ([nz][ny][nx] nodes of NCOMP floats) becomes (a | b) at node
// (j, i, k) of the copy (levels innermost), padded to 4 floats per time for
// three components.  One output node per thread: 16-byte coalesced writes,
// the reads strided by a level.
template <int NCOMP>
__global__ __launch_bounds__(kBlock) void field_pairs(const float* __restrict__ a,
                                                      const float* __restrict__ b,
                                                      float* __restrict__ out, int nx, int ny,
                                                      int nz)
{
    typedef float quad __attribute__((ext_vector_type(4)));
    const long long nodes = (long long)nx * ny * nz;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long n = (long long)blockIdx.x * kBlock + threadIdx.x; n < nodes; n += stride) {
        const int k = (int)(n % nz);
        const long long col = n / nz;  // j nx + i
        const long long src = ((long long)k * ny * nx + col) * NCOMP;
        if constexpr (NCOMP == 2) {
            const float2 u = *reinterpret_cast<const float2*>(a + src);
            const float2 v = *reinterpret_cast<const float2*>(b + src);
            reinterpret_cast<quad*>(out)[n] = quad{u.x, u.y, v.x, v.y};
        } else {
            reinterpret_cast<quad*>(out)[2 * n] = quad{a[src], a[src + 1], a[src + 2], 0.0f};
            reinterpret_cast<quad*>(out)[2 * n + 1] = quad{b[src], b[src + 1], b[src + 2], 0.0f};
        }
    }
}

__global__ __launch_bounds__(kBlock) void to_f32(const double* __restrict__ src, float* dst,
                                                 long long n, double scale)
{
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        dst[i] = (float)(src[i] * scale);
}

// dst[i] = the sum of the `copies` grids of n doubles at src, as float.
__global__ __launch_bounds__(kBlock) void copies_to_f32(const double* __restrict__ src,
                                                        int copies, float* dst, long long n)
{
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        double v = 0.0;
        for (int c = 0; c < copies; ++c) v += src[(long long)c * n + i];
        dst[i] = (float)v;
    }
}

}  // namespace lpm

// ===========================================================================
// Host side: validation, constant folding, launches.
// ===========================================================================
namespace lpm_host {

thread_local char g_msg[kMsgLen] = "";

// Launch settings of plain step launches: the library's only mutable
// process-wide state (lpm_set_launch), read atomically at each launch.
// Idle lanes before a refill when none is set: particles stay longer in the
// hourly 24 h workload than in the steady 6 h one, where waiting for nearly
// all lanes keeps the lanes of a wave on the same branches.
constexpr int kRefillMinSteady = 56;
constexpr int kRefillMinTime = 40;
std::atomic<int> g_refill_every{24};
std::atomic<int> g_refill_min{0};    // 0: by the wind (kRefillMinSteady / kRefillMinTime)
std::atomic<int> g_blocks_per_cu{0};  // 0: as many as the device holds

lpm_launch plain_launch()
{
    lpm_launch l;
    l.refill_every = g_refill_every.load(std::memory_order_relaxed);
    l.refill_min = g_refill_min.load(std::memory_order_relaxed);
    l.blocks_per_cu = g_blocks_per_cu.load(std::memory_order_relaxed);
    l.block = lpm::kBlock;
    return l;
}

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
    if ((st->x_lo == nullptr) != (st->y_lo == nullptr))
        return fail(LPM_EINVAL, "x_lo and y_lo: both or neither");
    if (!aligned4(st->x_lo) || !aligned4(st->y_lo))
        return fail(LPM_EINVAL, "residual arrays must be 4-byte aligned");
    if (!aligned4(st->order)) return fail(LPM_EINVAL, "work order must be 4-byte aligned");
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
    if (ph->kz_kind < 0 || ph->kz_kind > 3) return fail(LPM_EINVAL, "kz_kind must be 0..3");
    if (ph->kz_kind == 3 && !isfinite(ph->inv_L)) return fail(LPM_EINVAL, "inv_L must be finite");
    if (ph->chain != 0 && ph->chain != 1) return fail(LPM_EINVAL, "chain must be 0 or 1");
    if (ph->dep_mode != 0 && ph->dep_mode != 1) return fail(LPM_EINVAL, "dep_mode must be 0 or 1");
    if (ph->chain) {
        for (int n = 0; n < ph->n_nuc; ++n) {
            if (!(ph->lambda[n] > 0.0)) return fail(LPM_EINVAL, "a decay chain needs positive lambdas");
            for (int j = 0; j < n; ++j)
                if (ph->lambda[j] == ph->lambda[n])
                    return fail(LPM_EINVAL, "a decay chain needs distinct lambdas");
        }
    }
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
    if (!acc || !acc->dep || !acc->ledger || !acc->ctrl) return fail(LPM_EINVAL, "null accumulator");
    if (acc->n_nuc < 1 || acc->n_nuc > 4) return fail(LPM_EINVAL, "accumulator n_nuc must be 1..4");
    if (((uintptr_t)acc->dep & 7u) || ((uintptr_t)acc->ledger & 7u) || ((uintptr_t)acc->ctrl & 7u))
        return fail(LPM_EINVAL, "misaligned accumulator");
    if ((double)acc->dep_grid.nx * acc->dep_grid.ny >= 2147483647.0)
        return fail(LPM_EINVAL, "deposition grid must have fewer than 2^31 - 1 cells");
    if (acc->dep_copies < 0 || acc->dep_copies > LPM_MAX_DEP_COPIES)
        return fail(LPM_EINVAL, "dep_copies must be in [0, %d]", LPM_MAX_DEP_COPIES);
    return check_grid(&acc->dep_grid, true);
}

static int dep_copies(const lpm_accum* acc) { return acc->dep_copies > 1 ? acc->dep_copies : 1; }

double a0_of(const lpm_source* src, const lpm_schedule* sch, const lpm_physics* ph)
{
    return src->q * (double)sch->s_release * ph->dt / (double)sch->n_total;
}

unsigned blocks_for(long long n)
{
    return (unsigned)((n + lpm::kBlock - 1) / lpm::kBlock);
}

}  // namespace lpm_host
using namespace lpm_host;

extern "C" {

const char* lpm_last_error(void) { return g_msg; }

const char* lpm_version(void) { return "lpm 0.1 gfx950"; }

// Monin-Obukhov similarity (Businger-Dyer gradients, Paulson's integrated
// profile corrections) solved for 1/L by fixed-point iteration from neutral.
int lpm_surface_layer(double U, double z_ref, double z0, double dtheta, double T0,
                      double* ustar, double* inv_L)
{
    g_msg[0] = 0;
    if (!ustar || !inv_L) return fail(LPM_EINVAL, "null output");
    if (!(U > 0.0 && z0 > 0.0 && z_ref > z0 && T0 > 0.0 && isfinite(dtheta)))
        return fail(LPM_EINVAL, "need U > 0, z_ref > z0 > 0, T0 > 0");
    const double kappa = 0.4, grav = 9.81, half_pi = 1.5707963267948966;
    // profile corrections for momentum (m) and heat (h) at s = z/L
    auto corr = [&](double s, double& pm, double& ph) {
        if (s >= 0.0) {
            pm = ph = -5.0 * s;
            return;
        }
        const double x2 = sqrt(1.0 - 16.0 * s), x = sqrt(x2);
        pm = 2.0 * log(0.5 * (1.0 + x)) + log(0.5 * (1.0 + x2)) - 2.0 * atan(x) + half_pi;
        ph = 2.0 * log(0.5 * (1.0 + x2));
    };
    const double lz = log(z_ref / z0);
    double il = 0.0;
    for (int it = 0; it < 200; ++it) {
        double pm1, ph1, pm0, ph0;
        corr(z_ref * il, pm1, ph1);
        corr(z0 * il, pm0, ph0);
        const double fm = lz - pm1 + pm0, fh = lz - ph1 + ph0;
        if (!(fm > 0.0 && fh > 0.0)) break;
        const double us = kappa * U / fm, ts = kappa * dtheta / fh;
        const double next = kappa * grav * ts / (us * us * T0);
        if (!isfinite(next)) break;
        if (next == il || fabs(next - il) <= 1e-12 * fabs(next)) {
            *ustar = us;
            *inv_L = next;
            return LPM_OK;
        }
        il = next;
    }
    return fail(LPM_EINVAL, "no surface-layer solution (too stable?)");
}

int lpm_set_launch(int32_t refill_every, int32_t blocks_per_cu)
{
    return lpm_set_launch_ex(refill_every, blocks_per_cu, g_refill_min.load());
}

int lpm_set_launch_ex(int32_t refill_every, int32_t blocks_per_cu, int32_t refill_min)
{
    g_msg[0] = 0;
    if (refill_every < 1 || refill_every > 4096 || blocks_per_cu < 0 || refill_min < 0 ||
        refill_min > 64)
        return fail(LPM_EINVAL, "refill_every in [1, 4096], blocks_per_cu >= 0, refill_min in [0, 64]");
    g_refill_every = refill_every;
    g_blocks_per_cu = blocks_per_cu;
    g_refill_min = refill_min;
    return LPM_OK;
}

int lpm_accum_reset(const lpm_accum* acc, lpm_stream stream)
{
    g_msg[0] = 0;
    int rc = check_accum(acc);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const long long dn =
        (long long)dep_copies(acc) * acc->n_nuc * acc->dep_grid.nx * acc->dep_grid.ny;
    hipLaunchKernelGGL(lpm::fill_f64, dim3(blocks_for(dn) < 4096 ? blocks_for(dn) : 4096),
                       dim3(lpm::kBlock), 0, s, acc->dep, dn);
    hipLaunchKernelGGL(lpm::fill_f64, dim3(blocks_for(LPM_LEDGER_SLOTS * LPM_LEDGER_STRIDE)),
                       dim3(lpm::kBlock), 0, s, acc->ledger,
                       (long long)LPM_LEDGER_SLOTS * LPM_LEDGER_STRIDE);
    hipLaunchKernelGGL(lpm::fill_u32, dim3(1), dim3(lpm::kBlock), 0, s, acc->ctrl,
                       (long long)LPM_CTRL_WORDS);
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
    // a decay chain releases its parent only
    hipLaunchKernelGGL(lpm::release_kernel, dim3(blocks_for(hi - lo)), dim3(lpm::kBlock), 0,
                       (hipStream_t)stream, st->x, st->y, st->z, st->m, st->x_lo, st->y_lo, lo,
                       hi, (float)src->xs,
                       (float)src->ys, (float)src->h, acc->ledger, ph->chain ? 1 : ph->n_nuc,
                       released);
    return hip_status("lpm_release_particles");
}

}  // extern "C"

namespace lpm_host {

void fill_chain(lpm::GridConst& g, const lpm_physics* ph)
{
    double bc[4][4];
    activity_coefficients(ph, bc);
    for (int n = 0; n < 4; ++n)
        for (int j = 0; j < 4; ++j) g.bc[n][j] = (float)bc[n][j];
    g.chain = ph->chain;
}

int fill_field(lpm::StepConst& p, const lpm_field* f)
{
    if (!f || !f->data) return fail(LPM_EINVAL, "null field");
    if (f->nx < 1 || f->ny < 1 || f->nz < 1 || f->nt < 1) return fail(LPM_EINVAL, "bad field shape");
    if (f->ncomp != 2 && f->ncomp != 3) return fail(LPM_EINVAL, "field ncomp must be 2 or 3");
    if (!(f->dx > 0 && f->dy > 0 && (f->z_levels || f->dz > 0) && (f->nt == 1 || f->dt_field > 0)))
        return fail(LPM_EINVAL, "field spacings must be positive");
    const bool tpair = f->layout == LPM_FIELD_TIME_PAIRS;
    if (f->layout != LPM_FIELD_NODES && !tpair) return fail(LPM_EINVAL, "unknown field layout");
    // floats per node and time block: (u, v) or (u, v, w); a time-pair node
    // holds both times, (u, v | u, v) or (u, v, w, 0 | u, v, w, 0)
    const int rec = tpair ? (f->ncomp == 2 ? 4 : 8) : f->ncomp;
    if (tpair && (f->nt < 2 || f->interval < 0 || f->interval > f->nt - 2))
        return fail(LPM_EINVAL, "a time-pair field needs nt >= 2 and interval in [0, nt - 2]");
    if (tpair && ((uintptr_t)f->data & 15u))
        return fail(LPM_EINVAL, "a time-pair field must be 16-byte aligned");
    const double total = (double)(tpair ? 1 : f->nt) * f->nz * f->ny * f->nx * rec;
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
    p.fcx = (float)(-f->x0 / f->dx - 0.5); p.fcy = (float)(-f->y0 / f->dy - 0.5);
    p.inv_dx = (float)(1.0 / f->dx); p.inv_dy = (float)(1.0 / f->dy);
    p.inv_dz = f->z_levels ? 0.0f : (float)(1.0 / f->dz);
    p.inv_dtf = f->nt > 1 ? 1.0 / f->dt_field : 0.0;
    p.ft_zero = f->nt > 1 ? -f->t0 / f->dt_field : 0.0;
    if (tpair) {  // [ny][nx][nz] nodes: levels innermost
        p.sk = rec;
        p.si = f->nz * rec;
        p.sj = f->nx * p.si;
        p.st = 0;
    } else {      // [nt][nz][ny][nx]
        p.si = rec;
        p.sj = f->nx * rec;
        p.sk = f->ny * p.sj;
        p.st = f->nz * p.sk;
    }
    p.di = f->nx > 1 ? p.si : 0;
    p.dj = f->ny > 1 ? p.sj : 0;
    p.dk = f->nz > 1 ? p.sk : 0;
    p.dt_off = tpair ? rec / 2 : (f->nt > 1 ? p.st : 0);
    p.tpair = tpair;
    p.bounded = f->bounded != 0;
    p.X0 = (float)f->x0; p.X1 = (float)(f->x0 + f->nx * f->dx);
    p.Y0 = (float)f->y0; p.Y1 = (float)(f->y0 + f->ny * f->dy);
    return LPM_OK;
}

// Compile-time variants: wind components, time interpolation, nonuniform
// levels, nuclide count, K_z kind, deposition on/off.
// Per-launch constants of the source (plain launches; ensemble launches take
// them per lane from the scenario table).
void fill_source(lpm::StepConst& p, const lpm_source* src, const lpm_schedule* sch,
                 const lpm_physics* ph)
{
    p.xs = (float)src->xs; p.ys = (float)src->ys; p.h = (float)src->h;
    p.a0 = (float)a0_of(src, sch, ph);
    p.wscale = (float)src->wind_scale;
    p.key1 = src->scenario;
    if (src->v_d > 0.0 && ph->h_s > 0.0) {
        p.dry_c1 = (float)(2.0 * src->v_d / ph->h_s);
        p.dry_c2 = (float)(2.0 * src->v_d / (ph->h_s * ph->h_s));
    }
}

// Lower time node of step s, as the step kernel takes it.
static int time_node(const lpm::StepConst& p, long long s)
{
    const double ft = fmin(fmax(fma((double)s, p.ft_step, p.ft_zero), 0.0), (double)p.ftmax);
    return std::min((int)ft, p.tmaxi);
}

// A time-pair field holds one interval: every step of [step0, step0 +
// n_steps) must interpolate in it (the node is monotone in the step, so the
// first and the last step decide).  After fill_field and fill_physics.
int check_field_steps(const lpm::StepConst& p, const lpm_field* f, long long step0,
                      long long n_steps)
{
    if (!p.tpair) return LPM_OK;
    if (time_node(p, step0) != f->interval || time_node(p, step0 + n_steps - 1) != f->interval)
        return fail(LPM_EINVAL, "steps %lld..%lld do not all interpolate in field interval %d",
                    step0, step0 + n_steps - 1, f->interval);
    return LPM_OK;
}

// After fill_field (the time-node step needs the field interval).
void fill_physics(lpm::StepConst& p, const lpm_physics* ph)
{
    const double dt = ph->dt;
    p.ft_step = dt * p.inv_dtf;
    p.key0 = (uint32_t)(ph->seed & 0xFFFFFFFFull);
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
    p.h_s = ph->h_s > 0.0 ? (float)ph->h_s : 0.0f;
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
        p.edec[n] = (float)exp(-lam * dt);
    }
    p.inv_L = ph->kz_kind == 3 ? (float)ph->inv_L : 0.0f;
    p.chain = ph->chain;
    p.dep_mode = ph->dep_mode;
    p.n_nuc = ph->n_nuc;
    double bc[4][4];
    activity_coefficients(ph, bc);
    for (int n = 0; n < 4; ++n)
        for (int j = 0; j < 4; ++j) p.bc[n][j] = (float)bc[n][j];
}

// Activity of nuclide n per unit released activity = sum_j bc[n][j]
// exp(-lambda_j t).  Independent nuclides: the identity.  A chain released as
// pure parent: the daughter equation dA_n/dt = lambda_n (A_{n-1} - A_n) maps
// each exponential of A_{n-1} to the same exponential times
// lambda_n / (lambda_n - lambda_j), and A_n(0) = 0 fixes the coefficient of
// exp(-lambda_n t).
void activity_coefficients(const lpm_physics* ph, double bc[4][4])
{
    for (int n = 0; n < 4; ++n)
        for (int j = 0; j < 4; ++j) bc[n][j] = (!ph->chain && n == j) ? 1.0 : 0.0;
    if (!ph->chain) return;
    bc[0][0] = 1.0;
    for (int n = 1; n < ph->n_nuc; ++n) {
        double sum = 0.0;
        for (int j = 0; j < n; ++j) {
            bc[n][j] = bc[n - 1][j] * ph->lambda[n] / (ph->lambda[n] - ph->lambda[j]);
            sum += bc[n][j];
        }
        bc[n][n] = -sum;
    }
}

void fill_depgrid(lpm::StepConst& p, const lpm_grid& dg)
{
    p.dnx = dg.nx; p.dny = dg.ny; p.dmode = dg.mode;
    const double sh = dg.mode == 0 ? 0.0 : 0.5;
    p.d_cx = (float)(-dg.x0 / dg.dx - sh); p.d_cy = (float)(-dg.y0 / dg.dy - sh);
    p.d_inv_dx = (float)(1.0 / dg.dx); p.d_inv_dy = (float)(1.0 / dg.dy);
    p.d_fnx = (float)dg.nx; p.d_fny = (float)dg.ny;
    p.dscale = dg.density ? (float)(1.0 / (dg.dx * dg.dy)) : 1.0f;
}

// Device attributes, read once per device (the device a call runs on is the
// current one).  A race between two first readers stores the same value.
constexpr int kMaxDevices = 64;
std::atomic<int> g_dev_cus[kMaxDevices];
std::atomic<int> g_dev_lds[kMaxDevices];

int current_device()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
    return dev;
}

int device_cus()
{
    const int dev = current_device();
    int v = g_dev_cus[dev].load(std::memory_order_relaxed);
    if (v <= 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v < 1)
            v = 1;  // one block per CU-less device: a persistent launch still drains its queue
        g_dev_cus[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

int device_lds()
{
    const int dev = current_device();
    int v = g_dev_lds[dev].load(std::memory_order_relaxed);
    if (v <= 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
            v < 65536)
            v = 65536;
        g_dev_lds[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

// Occupancy (blocks per CU) of each (kernel, block size, device), cached:
// every variant has its own register and LDS footprint.
struct OccEntry {
    const void* kernel;
    int block, dev, per_cu;
};
std::mutex g_occ_mutex;
std::vector<OccEntry> g_occ;

int occupancy(const void* kernel, int block)
{
    const int dev = current_device();
    {
        std::lock_guard<std::mutex> lock(g_occ_mutex);
        for (const OccEntry& e : g_occ)
            if (e.kernel == kernel && e.block == block && e.dev == dev) return e.per_cu;
    }
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, block, 0) != hipSuccess || n < 1)
        n = 1;
    try {
        std::lock_guard<std::mutex> lock(g_occ_mutex);
        g_occ.push_back({kernel, block, dev, n});
    } catch (...) {
        // out of host memory: the value is still right, only not cached
    }
    return n;
}

unsigned resident_blocks(const void* kernel, int block, int blocks_per_cu, unsigned wanted)
{
    const int per_cu = occupancy(kernel, block);
    const int use = blocks_per_cu > 0 && blocks_per_cu < per_cu ? blocks_per_cu : per_cu;
    const unsigned cap = (unsigned)use * (unsigned)device_cus();
    return wanted < cap ? wanted : cap;
}
}  // namespace lpm_host
using namespace lpm_host;

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
        if (!rec || ((uintptr_t)rec & 15u)) return fail(LPM_EINVAL, "null or misaligned record buffer");
        if (rec_every < 1) return fail(LPM_EINVAL, "rec_every must be >= 1");
        if (rec_stride < sch->n_local) return fail(LPM_EINVAL, "rec_stride below n_local");
        if (rec_stride > 0xFFFFFFFFll) return fail(LPM_EINVAL, "rec_stride must be below 2^32");
        const long long last = (long long)rec_step0 + (long long)(n_rec - 1) * rec_every;
        if (rec_step0 < step0 || last >= (long long)step0 + n_steps)
            return fail(LPM_EINVAL, "recorded steps must lie inside the step window");
    }
    lpm::StepConst p;
    memset(&p, 0, sizeof p);
    if ((rc = fill_field(p, fld))) return rc;
    const lpm_launch lc = plain_launch();
    p.refill_every = lc.refill_every;
    p.refill_min = lc.refill_min ? lc.refill_min : (fld->nt > 1 ? kRefillMinTime : kRefillMinSteady);
    p.rec = n_rec > 0 ? rec : nullptr;
    p.rec_stride = rec_stride;
    p.rec_step0 = rec_step0;
    p.rec_every = rec_every > 0 ? rec_every : 1;
    p.n_rec = n_rec;

    p.X = st->x; p.Y = st->y; p.Z = st->z; p.M = st->m;
    p.XL = st->x_lo; p.YL = st->y_lo;
    p.n_total = sch->n_total; p.id_base = sch->id_base; p.id_stride = sch->id_stride;
    p.s_release = sch->s_release;
    p.step0 = step0;
    p.step_end = step0 + n_steps;
    p.i_hi = first_local_born_at_or_after(sch, (long long)p.step_end);
    if (st->order) {
        if (st->n_order != p.i_hi)
            return fail(LPM_EINVAL, "work order of %lld particles for a launch of %lld",
                        (long long)st->n_order, p.i_hi);
        p.order = st->order;
    }

    fill_source(p, src, sch, ph);
    fill_physics(p, ph);
    if ((rc = check_field_steps(p, fld, step0, n_steps))) return rc;
    fill_depgrid(p, acc->dep_grid);
    p.dep = acc->dep; p.ledger = acc->ledger; p.ctrl = acc->ctrl;
    p.dep_copies = dep_copies(acc);

    if (p.i_hi <= 0) return LPM_OK;
    const unsigned nb = blocks_for(p.i_hi);
    hipStream_t s = (hipStream_t)stream;
    // the work queue starts empty
    hipLaunchKernelGGL(lpm::fill_u32, dim3(1), dim3(lpm::kBlock), 0, s, acc->ctrl + LPM_CTRL_QUEUE, 2ll);
    // steady, two time nodes, or a time-pair copy (its gather compiled in)
    const int time = fld->nt > 1 ? (p.tpair ? 2 : 1) : 0;
    const bool dep = p.dry_c1 > 0.0f || p.L0 > 0.0f;
    // the general kernel (K_z kind at run time) serves the paper-literal variants
    const int kz = (ph->chain || ph->dep_mode || ph->kz_kind == 3) ? 4 : ph->kz_kind;
    const bool lev = fld->z_levels != nullptr;
    const int bpc = lc.blocks_per_cu;
    auto go = [&](auto nc) {
        constexpr int NC = decltype(nc)::value;
        if (time == 2) launch_plain<NC, 2>(lev, ph->n_nuc, kz, dep, nb, s, p, bpc);
        else if (time == 1) launch_plain<NC, 1>(lev, ph->n_nuc, kz, dep, nb, s, p, bpc);
        else launch_plain<NC, 0>(lev, ph->n_nuc, kz, dep, nb, s, p, bpc);
    };
    if (fld->ncomp == 2) go(std::integral_constant<int, 2>{});
    else go(std::integral_constant<int, 3>{});
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

}  // extern "C"

namespace lpm_host {

// Shared by lpm_grid_concentration and its no-allocation variant: checks the
// arguments (except the scratch) and launches clear, scatter and conversion
// on acc_scratch, which must hold n_nuc * nx * ny * nz doubles.
int grid_concentration_impl(const lpm_state* st, const lpm_source* src, const lpm_schedule* sch,
                            const lpm_physics* ph, const lpm_grid* grid, int32_t step,
                            double* acc_scratch, float* out, lpm_stream stream, const char* what)
{
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
    fill_chain(g, ph);
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
    return hip_status(what);
}

int check_grid_concentration(const lpm_state* st, const lpm_source* src, const lpm_schedule* sch,
                             const lpm_physics* ph, const lpm_grid* grid, int32_t step, float* out)
{
    int rc = check_state(st, sch);
    if (rc) return rc;
    if (!src) return fail(LPM_EINVAL, "null source");
    if ((rc = check_physics(ph)) || (rc = check_grid(grid, false))) return rc;
    if (!out || !aligned4(out)) return fail(LPM_EINVAL, "null or misaligned output grid");
    if (step < 0) return fail(LPM_EINVAL, "step must be >= 0");
    return LPM_OK;
}

}  // namespace lpm_host

// FP64 accumulation grid of lpm_grid_concentration_static: one copy per
// device, held from module load to process end.  Host code uses its device
// address from hipGetSymbolAddress (kept per device below), never the name.
static __device__ __align__(256) double scratch[LPM_STATIC_SCRATCH_DOUBLES];

namespace lpm_host {

std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

// Address of `scratch` on the current device, looked up on the first call
// there (with that device current).  nullptr when the lookup fails.
double* static_scratch()
{
    const int dev = current_device();
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    return g_scratch_ptr[dev];
}

}  // namespace lpm_host

extern "C" {

int lpm_grid_concentration(const lpm_state* st, const lpm_source* src, const lpm_schedule* sch,
                           const lpm_physics* ph, const lpm_grid* grid, int32_t step,
                           double* acc_scratch, float* out, lpm_stream stream)
{
    g_msg[0] = 0;
    int rc = check_grid_concentration(st, src, sch, ph, grid, step, out);
    if (rc) return rc;
    if (!acc_scratch || ((uintptr_t)acc_scratch & 7u))
        return fail(LPM_EINVAL, "null or misaligned grid scratch");
    return grid_concentration_impl(st, src, sch, ph, grid, step, acc_scratch, out, stream,
                                   "lpm_grid_concentration");
}

int lpm_grid_concentration_static(const lpm_state* st, const lpm_source* src,
                                  const lpm_schedule* sch, const lpm_physics* ph,
                                  const lpm_grid* grid, int32_t step, float* out,
                                  lpm_stream stream)
{
    g_msg[0] = 0;
    int rc = check_grid_concentration(st, src, sch, ph, grid, step, out);
    if (rc) return rc;
    const long long need = (long long)ph->n_nuc * grid->nx * grid->ny * grid->nz;
    if (need > LPM_STATIC_SCRATCH_DOUBLES)
        return fail(LPM_EINVAL, "grid of %lld cells x nuclides exceeds the static scratch of %d",
                    need, LPM_STATIC_SCRATCH_DOUBLES);
    double* acc = static_scratch();
    if (!acc) return fail(LPM_EHIP, "lpm_grid_concentration_static: no address for the static scratch");
    return grid_concentration_impl(st, src, sch, ph, grid, step, acc, out, stream,
                                   "lpm_grid_concentration_static");
}

namespace lpm_host {

// Layout of the record-gridding workspace and the tile shape: the widest
// tile of full height whose cells (double, n_nuc of them each) fit the LDS
// budget of one block.
struct RecordPlan {
    int tx, ty, ps, ntx, nty, nbx, nby;
    long long nbk, nb, nscan;
    unsigned long long cap;        // binned records at most
    long long nchunk;              // chunks of kRecChunk ids that can hold records
    size_t o_off, o_cur, o_bsum, o_cend, o_brec, o_born, bytes;
    size_t tile_lds;
};

constexpr size_t kTileLds = 49152;

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

int plan_records(const lpm_schedule* sch, const lpm_physics* ph, const lpm_grid* grid,
                 int32_t rec_step0, int32_t rec_every, int32_t n_rec, RecordPlan* rp)
{
    int rc;
    if (!sch) return fail(LPM_EINVAL, "null schedule");
    if ((rc = check_physics(ph)) || (rc = check_grid(grid, false))) return rc;
    if (sch->n_total <= 0 || sch->s_release <= 0 || sch->n_local < 0 || sch->id_stride <= 0)
        return fail(LPM_EINVAL, "bad schedule");
    if (n_rec < 0 || rec_every < 1 || rec_step0 < 0) return fail(LPM_EINVAL, "bad record steps");
    if ((long long)rec_step0 + (long long)(n_rec > 0 ? n_rec - 1 : 0) * rec_every > 0x7FFFFFFFll)
        return fail(LPM_EINVAL, "record steps overflow");
    if (n_rec > 65535) return fail(LPM_EINVAL, "at most 65535 records per call");
    if (sch->n_local > 0xFFFFFFFFll) return fail(LPM_EINVAL, "at most 2^32 - 1 local particles");
    const size_t column = (size_t)ph->n_nuc * grid->nz * sizeof(double);
    static const int shapes[][2] = {{16, 4}, {8, 4}, {8, 2}, {4, 2}, {2, 2}, {2, 1}, {1, 1}};
    int pick = -1;
    for (int j = 0; j < 7 && pick < 0; ++j)
        if (column * (shapes[j][0] * shapes[j][1] + (shapes[j][0] * shapes[j][1] > 1 ? 1 : 0)) <= kTileLds)
            pick = j;
    if (pick < 0) return fail(LPM_EINVAL, "n_nuc * nz must be at most 6144 to grid records");
    RecordPlan r;
    r.tx = shapes[pick][0]; r.ty = shapes[pick][1];
    r.ntx = (grid->nx + r.tx - 1) / r.tx; r.nty = (grid->ny + r.ty - 1) / r.ty;
    r.nbx = grid->nx / r.tx + 1; r.nby = grid->ny / r.ty + 1;
    r.nbk = (long long)r.nbx * r.nby * 4;
    r.nb = r.nbk * n_rec;
    if (r.nb > (1ll << 34)) return fail(LPM_EINVAL, "too many grid tiles times records");
    r.nscan = (r.nb + lpm::kScanChunk - 1) / lpm::kScanChunk;
    r.cap = 0;
    for (int k = 0; k < n_rec; ++k)
        r.cap += (unsigned long long)first_local_born_at_or_after(
            sch, (long long)rec_step0 + (long long)k * rec_every + 1);
    r.o_off = 0;
    r.o_cur = r.o_off + align256(8 * (size_t)r.nb);
    r.o_bsum = r.o_cur + align256(8 * (size_t)r.nb);
    // one word per chunk of recorded positions: at most n_local of them
    r.nchunk = (sch->n_local + lpm::kRecChunk - 1) / lpm::kRecChunk;
    r.o_cend = r.o_bsum + align256(8 * (size_t)r.nscan);
    r.o_brec = r.o_cend + align256(4 * (size_t)r.nchunk);
    r.o_born = r.o_brec + align256(16 * (size_t)r.cap);
    r.bytes = r.o_born + align256(4 * (size_t)r.cap);
    r.ps = r.tx * r.ty + (r.tx * r.ty > 1 ? 1 : 0);
    r.tile_lds = column * r.ps;
    *rp = r;
    return LPM_OK;
}

}  // namespace lpm_host

int lpm_grid_records_workspace(const lpm_schedule* sch, const lpm_physics* ph,
                               const lpm_grid* grid, int32_t rec_step0, int32_t rec_every,
                               int32_t n_rec, int64_t* bytes)
{
    g_msg[0] = 0;
    if (!bytes) return fail(LPM_EINVAL, "null output");
    RecordPlan rp;
    const int rc = plan_records(sch, ph, grid, rec_step0, rec_every, n_rec, &rp);
    if (rc) return rc;
    *bytes = n_rec == 0 ? 0 : (int64_t)rp.bytes;
    return LPM_OK;
}

// lpm_grid_records (order == nullptr: records by particle index) and
// lpm_grid_records_ordered (records by position in `order`).
static int grid_records_impl(const float* rec, int64_t rec_stride, int32_t rec_step0,
                             int32_t rec_every, int32_t n_rec, const lpm_source* src,
                             const lpm_schedule* sch, const lpm_physics* ph, const lpm_grid* grid,
                             const int32_t* order, int64_t n_order, void* work,
                             int64_t work_bytes, float* out, lpm_stream stream)
{
    g_msg[0] = 0;
    if (!src) return fail(LPM_EINVAL, "null source");
    RecordPlan rp;
    int rc = plan_records(sch, ph, grid, rec_step0, rec_every, n_rec, &rp);
    if (rc) return rc;
    if (order && (!aligned4(order) || n_order < 0 || n_order > sch->n_local))
        return fail(LPM_EINVAL, "work order: 4-byte aligned, n_order in [0, n_local]");
    if (n_rec == 0) return LPM_OK;
    if (!rec || ((uintptr_t)rec & 15u)) return fail(LPM_EINVAL, "null or misaligned record buffer");
    if (rec_stride < sch->n_local) return fail(LPM_EINVAL, "rec_stride below n_local");
    if (!out || !aligned4(out)) return fail(LPM_EINVAL, "null or misaligned output");
    if (!work || ((uintptr_t)work & 255u)) return fail(LPM_EINVAL, "null or misaligned workspace");
    if (work_bytes < (int64_t)rp.bytes) return fail(LPM_EINVAL, "workspace below lpm_grid_records_workspace");
    lpm::GridConst g;
    memset(&g, 0, sizeof g);
    g.n_total = sch->n_total; g.id_base = sch->id_base; g.id_stride = sch->id_stride;
    g.s_release = sch->s_release;
    g.nnuc = ph->n_nuc;
    g.mode = grid->mode;
    g.a0 = (float)a0_of(src, sch, ph);
    g.dt = (float)ph->dt;
    g.scale = 1.0f;
    for (int n = 0; n < ph->n_nuc; ++n) g.lam_l2e[n] = (float)(ph->lambda[n] * 1.4426950408889634);
    fill_chain(g, ph);
    g.nx = grid->nx; g.ny = grid->ny; g.nz = grid->nz;
    g.x0 = grid->x0; g.y0 = grid->y0; g.z0 = grid->z0;
    g.inv_dx = 1.0 / grid->dx; g.inv_dy = 1.0 / grid->dy; g.inv_dz = 1.0 / grid->dz;
    g.cells = (long long)grid->nx * grid->ny * grid->nz;
    // every particle that can be born by the last recorded step; recorded
    // positions: those particles, or the entries of the work order
    g.i_hi = first_local_born_at_or_after(sch, (long long)rec_step0 + (long long)(n_rec - 1) * rec_every + 1);
    g.order = order;
    g.n_pos = order ? n_order : g.i_hi;
    if (order) g.i_hi = sch->n_local;
    char* w = (char*)work;
    lpm::TileConst t;
    t.tx = rp.tx; t.ty = rp.ty;
    t.lx = __builtin_ctz((unsigned)rp.tx); t.ly = __builtin_ctz((unsigned)rp.ty);
    t.ps = rp.ps;
    t.ntx = rp.ntx; t.nty = rp.nty; t.nbx = rp.nbx; t.nby = rp.nby;
    t.nbk = rp.nbk;
    // A block counts and ranks its records in an LDS window of bins from its
    // lowest one (24 KB: several blocks per CU); records beyond it take global
    // atomics.
    t.nwin = (int)std::min<long long>(rp.nbk, lpm::kBinWindow);
    t.off = (unsigned long long*)(w + rp.o_off);
    t.cur = (unsigned long long*)(w + rp.o_cur);
    t.bsum = (unsigned long long*)(w + rp.o_bsum);
    t.brec = (float4*)(w + rp.o_brec);
    t.bborn = (int*)(w + rp.o_born);
    t.chunk_end = (const int*)(w + rp.o_cend);
    t.cap = rp.cap;
    t.out = out;
    t.inv_vol = 1.0 / (grid->density ? grid->dx * grid->dy * grid->dz : 1.0);
    hipStream_t s = (hipStream_t)stream;
    const dim3 bs(lpm::kBlock);
    // the output and the counts start at zero (fill kernels: the call may be
    // captured in a graph)
    const long long n_out = (long long)n_rec * ph->n_nuc * g.cells;
    hipLaunchKernelGGL(lpm::fill_u32, dim3(std::min(blocks_for(n_out), 16384u)), bs, 0, s,
                       (uint32_t*)out, n_out);
    hipLaunchKernelGGL(lpm::fill_u32, dim3(std::min(blocks_for(2 * rp.nb), 16384u)), bs, 0, s,
                       (uint32_t*)t.cur, 2 * rp.nb);
    const float4* r4 = reinterpret_cast<const float4*>(rec);
    const int* last = reinterpret_cast<const int*>(rec + 4ll * n_rec * rec_stride);
    if (g.n_pos > 0) {
        const long long nchunk = (g.n_pos + lpm::kRecChunk - 1) / lpm::kRecChunk;  // <= rp.nchunk
        const dim3 nb((unsigned)nchunk, (unsigned)n_rec);
        hipLaunchKernelGGL(lpm::chunk_end_kernel, dim3((unsigned)nchunk), bs, 0, s, last,
                           g.n_pos, (int*)(w + rp.o_cend));
        hipLaunchKernelGGL(lpm::bin_count_kernel, nb, bs, lpm::kBinCountLds * t.nwin, s,
                           g, t, r4, last, rec_stride, rec_step0, rec_every);
        hipLaunchKernelGGL(lpm::scan_sums_kernel, dim3((unsigned)rp.nscan), bs, 0, s, t.cur, rp.nb,
                           t.bsum);
        hipLaunchKernelGGL(lpm::scan_bsum_kernel, dim3(1), bs, 0, s, t.bsum, rp.nscan);
        hipLaunchKernelGGL(lpm::scan_apply_kernel, dim3((unsigned)rp.nscan), bs, 0, s, t.cur, t.off,
                           rp.nb, (const unsigned long long*)t.bsum);
        hipLaunchKernelGGL(lpm::bin_scatter_kernel, nb, bs, lpm::kBinScatterLds * t.nwin,
                           s, g, t, r4, last, rec_stride, rec_step0, rec_every);
    } else {
        // nothing is born: every bin is empty (off = cur = 0)
        hipLaunchKernelGGL(lpm::fill_u32, dim3(std::min(blocks_for(2 * rp.nb), 16384u)), bs, 0, s,
                           (uint32_t*)t.off, 2 * rp.nb);
    }
    const dim3 tg((unsigned)((long long)rp.ntx * rp.nty), (unsigned)n_rec, lpm::kTileSplit);
    switch (ph->n_nuc) {
    case 1: hipLaunchKernelGGL(lpm::tile_conc_kernel<1>, tg, bs, rp.tile_lds, s, g, t, rec_step0, rec_every); break;
    case 2: hipLaunchKernelGGL(lpm::tile_conc_kernel<2>, tg, bs, rp.tile_lds, s, g, t, rec_step0, rec_every); break;
    case 3: hipLaunchKernelGGL(lpm::tile_conc_kernel<3>, tg, bs, rp.tile_lds, s, g, t, rec_step0, rec_every); break;
    default: hipLaunchKernelGGL(lpm::tile_conc_kernel<4>, tg, bs, rp.tile_lds, s, g, t, rec_step0, rec_every); break;
    }
    return hip_status(order ? "lpm_grid_records_ordered" : "lpm_grid_records");
}

int lpm_grid_records(const float* rec, int64_t rec_stride, int32_t rec_step0, int32_t rec_every,
                     int32_t n_rec, const lpm_source* src, const lpm_schedule* sch,
                     const lpm_physics* ph, const lpm_grid* grid, void* work, int64_t work_bytes,
                     float* out, lpm_stream stream)
{
    return grid_records_impl(rec, rec_stride, rec_step0, rec_every, n_rec, src, sch, ph, grid,
                             nullptr, 0, work, work_bytes, out, stream);
}

int lpm_grid_records_ordered(const float* rec, int64_t rec_stride, int32_t rec_step0,
                             int32_t rec_every, int32_t n_rec, const lpm_source* src,
                             const lpm_schedule* sch, const lpm_physics* ph,
                             const lpm_grid* grid, const int32_t* order, int64_t n_order,
                             void* work, int64_t work_bytes, float* out, lpm_stream stream)
{
    if (!order) {
        g_msg[0] = 0;
        return fail(LPM_EINVAL, "null work order");
    }
    return grid_records_impl(rec, rec_stride, rec_step0, rec_every, n_rec, src, sch, ph, grid,
                             order, n_order, work, work_bytes, out, stream);
}

int lpm_grid_deposition(const lpm_accum* acc, float* out, lpm_stream stream)
{
    g_msg[0] = 0;
    int rc = check_accum(acc);
    if (rc) return rc;
    if (!out || !aligned4(out)) return fail(LPM_EINVAL, "null or misaligned output");
    const long long total = (long long)acc->n_nuc * acc->dep_grid.nx * acc->dep_grid.ny;
    const unsigned fb = blocks_for(total) < 8192 ? blocks_for(total) : 8192;
    hipLaunchKernelGGL(lpm::copies_to_f32, dim3(fb), dim3(lpm::kBlock), 0, (hipStream_t)stream,
                       acc->dep, dep_copies(acc), out, total);
    return hip_status("lpm_grid_deposition");
}

// Work order: nodes of a field (columns with nonuniform levels), and the
// workspace of a sort of up to n pairs.
static long long order_nodes(const lpm_field* fld)
{
    return (long long)fld->nx * fld->ny * (fld->z_levels ? 1 : fld->nz);
}

struct OrderLayout {
    long long nblocks, ntable, nscan;
    long long off_keys[2], off_vals[2], off_table, off_bsum, bytes;
};

static OrderLayout order_layout(long long n)
{
    auto up = [](long long b) { return (b + 255) & ~255ll; };
    OrderLayout L;
    L.nblocks = (n + lpm::kSortTile - 1) / lpm::kSortTile;
    L.ntable = 256 * L.nblocks;
    L.nscan = (L.ntable + lpm::kScanChunk - 1) / lpm::kScanChunk;
    long long at = 256;  // the two counters
    for (int b = 0; b < 2; ++b) {
        L.off_keys[b] = at;
        at += up(4 * n);
        L.off_vals[b] = at;
        at += up(4 * n);
    }
    L.off_table = at;
    at += up(8 * L.ntable);
    L.off_bsum = at;
    at += up(8 * (L.nscan > 0 ? L.nscan : 1));
    L.bytes = at;
    return L;
}

int lpm_order_workspace(const lpm_schedule* sch, const lpm_field* fld, int64_t* bytes)
{
    g_msg[0] = 0;
    if (!sch || !fld || !bytes) return fail(LPM_EINVAL, "null argument");
    if (sch->n_local < 0) return fail(LPM_EINVAL, "bad local id range");
    if (fld->nx < 1 || fld->ny < 1 || fld->nz < 1) return fail(LPM_EINVAL, "bad field shape");
    *bytes = (int64_t)order_layout(sch->n_local).bytes;
    return LPM_OK;
}

int lpm_order_particles(const lpm_state* st, const lpm_schedule* sch, const lpm_field* fld,
                        int32_t step0, int32_t n_steps, int32_t* order, int64_t order_capacity,
                        int64_t* n_order, void* work, int64_t work_bytes, lpm_stream stream)
{
    g_msg[0] = 0;
    int rc = check_state(st, sch);
    if (rc) return rc;
    if (!fld || !order || !n_order || !work) return fail(LPM_EINVAL, "null argument");
    if (fld->nx < 1 || fld->ny < 1 || fld->nz < 1) return fail(LPM_EINVAL, "bad field shape");
    if (!(fld->dx > 0 && fld->dy > 0 && (fld->z_levels || fld->dz > 0)))
        return fail(LPM_EINVAL, "field spacings must be positive");
    if (order_nodes(fld) > 0xFFFFFFFFll) return fail(LPM_EINVAL, "field of more than 2^32 nodes");
    if (step0 < 0 || n_steps < 1 || (long long)step0 + n_steps > 0x7FFFFFFFll)
        return fail(LPM_EINVAL, "bad step window");
    if (!aligned4(order) || ((uintptr_t)work & 255u))
        return fail(LPM_EINVAL, "misaligned order or workspace");
    const OrderLayout L = order_layout(sch->n_local);
    if (work_bytes < L.bytes)
        return fail(LPM_EINVAL, "workspace of %lld bytes below the %lld needed",
                    (long long)work_bytes, L.bytes);
    const long long n_all = first_local_born_at_or_after(sch, (long long)step0 + n_steps);
    if (n_all > 0x7FFFFFFFll) return fail(LPM_EINVAL, "work order of more than 2^31 - 1 particles");
    if (n_all > order_capacity)
        return fail(LPM_EINVAL, "work order of %lld particles exceeds its capacity of %lld", n_all,
                    (long long)order_capacity);
    *n_order = n_all;
    if (n_all == 0) return LPM_OK;
    char* w = static_cast<char*>(work);
    lpm::OrderConst o;
    memset(&o, 0, sizeof o);
    o.X = st->x; o.Y = st->y; o.Z = st->z; o.M = st->m;
    o.n_old = first_local_born_at_or_after(sch, step0);
    o.n_all = n_all;
    o.fcx = (float)(-fld->x0 / fld->dx); o.fcy = (float)(-fld->y0 / fld->dy);
    o.inv_dx = (float)(1.0 / fld->dx); o.inv_dy = (float)(1.0 / fld->dy);
    o.inv_dz = fld->z_levels ? 0.0f : (float)(1.0 / fld->dz);
    o.nx = fld->nx; o.ny = fld->ny; o.nz = fld->z_levels ? 1 : fld->nz;
    o.count = reinterpret_cast<unsigned long long*>(w);
    o.keys = reinterpret_cast<unsigned*>(w + L.off_keys[0]);
    o.vals = reinterpret_cast<int*>(w + L.off_vals[0]);
    o.order = order;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(lpm::fill_f64, dim3(1), dim3(lpm::kBlock), 0, s,
                       reinterpret_cast<double*>(o.count), 2ll);
    if (o.n_old > 0) {
        const long long tiles = (o.n_old + lpm::kSortTile - 1) / lpm::kSortTile;
        hipLaunchKernelGGL(lpm::order_keys_kernel, dim3((unsigned)(tiles < 4096 ? tiles : 4096)),
                           dim3(lpm::kBlock), 0, s, o);
        // passes of 8 bits over the node index
        int bits = 1;
        while (bits < 32 && (1ll << bits) < order_nodes(fld)) ++bits;
        const int passes = (bits + 7) / 8;
        auto* table = reinterpret_cast<unsigned long long*>(w + L.off_table);
        auto* bsum = reinterpret_cast<unsigned long long*>(w + L.off_bsum);
        const dim3 g((unsigned)L.nblocks), bs(lpm::kBlock);
        for (int q = 0; q < passes; ++q) {
            lpm::SortPass c;
            c.kin = reinterpret_cast<const unsigned*>(w + L.off_keys[q & 1]);
            c.vin = reinterpret_cast<const int*>(w + L.off_vals[q & 1]);
            const bool last = q == passes - 1;
            c.kout = last ? nullptr : reinterpret_cast<unsigned*>(w + L.off_keys[(q + 1) & 1]);
            c.vout = last ? order : reinterpret_cast<int*>(w + L.off_vals[(q + 1) & 1]);
            c.n = o.count;
            c.table = table;
            c.nblocks = L.nblocks;
            c.shift = 8 * q;
            hipLaunchKernelGGL(lpm::radix_hist_kernel, g, bs, 0, s, c);
            hipLaunchKernelGGL(lpm::scan_sums_kernel, dim3((unsigned)L.nscan), bs, 0, s,
                               (const unsigned long long*)table, L.ntable, bsum);
            hipLaunchKernelGGL(lpm::scan_bsum_kernel, dim3(1), bs, 0, s, bsum, L.nscan);
            hipLaunchKernelGGL(lpm::scan_apply_kernel, dim3((unsigned)L.nscan), bs, 0, s, table,
                               table, L.ntable, (const unsigned long long*)bsum);
            hipLaunchKernelGGL(lpm::radix_scatter_kernel, g, bs, 0, s, c);
        }
    }
    if (n_all > o.n_old) {
        const long long nb_born = n_all - o.n_old;
        const unsigned nb = blocks_for(nb_born) < 8192 ? blocks_for(nb_born) : 8192;
        hipLaunchKernelGGL(lpm::order_born_kernel, dim3(nb), dim3(lpm::kBlock), 0, s, o);
    }
    return hip_status("lpm_order_particles");
}

static int64_t interval_bytes(const lpm_field* fld)
{
    if (!fld || !fld->data) return fail(LPM_EINVAL, "null field");
    if (fld->layout != LPM_FIELD_NODES) return fail(LPM_EINVAL, "the field must be in the node layout");
    if (fld->nt < 2) return fail(LPM_EINVAL, "a field interval needs nt >= 2");
    if (fld->ncomp != 2 && fld->ncomp != 3) return fail(LPM_EINVAL, "field ncomp must be 2 or 3");
    if (fld->ny < 1 || fld->nz < 1) return fail(LPM_EINVAL, "bad field shape");
    return (int64_t)fld->nx * fld->ny * fld->nz * (fld->ncomp == 2 ? 16 : 32);
}

int lpm_field_interval_bytes(const lpm_field* fld, int64_t* bytes)
{
    g_msg[0] = 0;
    if (!bytes) return fail(LPM_EINVAL, "null output");
    const int64_t b = interval_bytes(fld);
    if (b < 0) return (int)b;
    *bytes = b;
    return LPM_OK;
}

int lpm_field_interval(const lpm_field* fld, int32_t k, void* out, lpm_field* packed,
                       lpm_stream stream)
{
    g_msg[0] = 0;
    const int64_t bytes = interval_bytes(fld);
    if (bytes < 0) return (int)bytes;
    if (k < 0 || k > fld->nt - 2) return fail(LPM_EINVAL, "interval %d outside [0, %d]", k, fld->nt - 2);
    if (!out || ((uintptr_t)out & 15u)) return fail(LPM_EINVAL, "null or misaligned output");
    if (!packed) return fail(LPM_EINVAL, "null descriptor");
    if (fld->ncomp == 2 && ((uintptr_t)fld->data & 7u))
        return fail(LPM_EINVAL, "two-component field must be 8-byte aligned");
    const long long nodes = (long long)fld->nx * fld->ny * fld->nz;
    const char* o = static_cast<const char*>(out);
    const char* d = reinterpret_cast<const char*>(fld->data);
    const long long src_bytes = (long long)fld->nt * nodes * fld->ncomp * 4;
    if (o < d + src_bytes && d < o + bytes) return fail(LPM_EINVAL, "output overlaps the field");
    const float* a = fld->data + (long long)k * nodes * fld->ncomp;
    const float* b = a + nodes * fld->ncomp;
    const unsigned nb = blocks_for(nodes) < 8192 ? blocks_for(nodes) : 8192;
    hipStream_t s = (hipStream_t)stream;
    if (fld->ncomp == 2)
        hipLaunchKernelGGL(lpm::field_pairs<2>, dim3(nb), dim3(lpm::kBlock), 0, s, a, b,
                           static_cast<float*>(out), fld->nx, fld->ny, fld->nz);
    else
        hipLaunchKernelGGL(lpm::field_pairs<3>, dim3(nb), dim3(lpm::kBlock), 0, s, a, b,
                           static_cast<float*>(out), fld->nx, fld->ny, fld->nz);
    lpm_field q = *fld;
    q.data = static_cast<const float*>(out);
    q.layout = LPM_FIELD_TIME_PAIRS;
    q.interval = k;
    *packed = q;
    return hip_status("lpm_field_interval");
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
    if (!acc || !acc->ctrl) return fail(LPM_EINVAL, "null accumulator");
    uint32_t e = 0;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(&e, acc->ctrl + LPM_CTRL_ERR, sizeof e, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return hip_status("lpm_check");
    if (e & 1u) return fail(LPM_ENONFINITE, "a particle coordinate or mass became non-finite");
    if (e & 2u) return fail(LPM_EHIP, "internal error: deposition staging list overflowed");
    return LPM_OK;
}

}  // extern "C"

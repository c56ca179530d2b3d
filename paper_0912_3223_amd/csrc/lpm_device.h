// Device-side building blocks of the particle step for gfx950 (CDNA4).
//
// Everything here runs per particle in registers: counter-based random
// numbers (no random-number buffer in HBM), the wind gather, the diffusivity
// profile and the deposition rates.  The formulas follow Sec. 2 and Eqs. 1-3
// of Molnar Jr. et al. (arXiv:0912.3223) with the readings stated in lpm.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpm {

constexpr int kBlock = 256;  // threads per block of every kernel

// Birth step of global particle id gid (continuous uniform release).
__device__ __forceinline__ long long birth(long long gid, long long s_release,
                                           long long n_total)
{
    return (gid * s_release) / n_total;
}

// One scenario of an ensemble launch, as uploaded to device memory.
struct DevScen {
    long long qbase;    // first work-queue index of the scenario
    long long offset;   // first element in the combined state arrays
    long long n_total;  // particles of the scenario
    long long lo, hi;   // local ids released in the window
    long long i_hi;     // local ids born before the window ends
    double released;    // activity released per nuclide in the window
    float a0, wscale, dry_c1, dry_c2, xs, ys, h;
    uint32_t key1;
    int s_release, pad;
};

// Per-launch constants, precomputed in double precision on the host and
// rounded once to float.  Passed by value, so they live in SGPRs/the kernel
// argument segment and cost no vector registers.
struct StepConst {
    // particle state (XL, YL: rounding residuals of X, Y, or null)
    float* X;
    float* Y;
    float* Z;
    float* M;
    float* XL;
    float* YL;
    const int* order;  // work order of the queue, or null: index order
    // schedule
    long long n_total, id_base, id_stride, i_hi;
    int s_release, step0, step_end, pad0;
    // source
    float xs, ys, h, a0, wscale;
    uint32_t key0, key1;
    // wind field
    const float* f;
    const float* lev;
    int nx, ny, nz, nt;
    int imax, jmax, kmax, tmaxi;          // largest lower node index
    float fxmax, fymax, fzmax, ftmax;     // largest fractional node index
    // fractional node index of x: x inv_dx + fcx (fcx = -x0/dx - 1/2, cell-centred
    // nodes), the same in y; of z: z inv_dz - 1/2; of the time after step s
    // (FP64, the same for every particle): s ft_step + ft_zero, ft_step =
    // dt inv_dtf
    float fcx, fcy, inv_dx, inv_dy, inv_dz;
    double ft_step, ft_zero, inv_dtf;
    int di, dj, dk, dt_off;               // float offsets of the upper neighbours
    int si, sj, sk, st;                   // float strides of i, j, k, t
    int bounded;
    int tpair;                            // time-pair copy of one field interval
    float X0, X1, Y0, Y1;                 // exit box
    // physics
    float dt, sKh, s2dt, half_dt;
    int kz_kind;
    float Kz_const, ku, z0, H_mix, inv_Hmix, H_top;  // H_top: lid, or +inf
    float dry_c1, dry_c2, h_s;            // v_d (2/h_s)(1 - z/h_s) = c1 - c2 z
    float L0, rcx, rcy, r_ca_a, r_sa_a, r_ca_b, r_sa_b, inv_edge;
    float lam[4];                         // decay constants
    float lam_l2e[4];                     // lambda log2(e)
    float edec[4];                        // exp(-lambda dt)
    // recorded states: plane q (x, y, z, m) of record k at rec + (4 k + q) rec_stride
    float* rec;
    long long rec_stride;
    int rec_step0, rec_every, n_rec;
    int refill_every;  // steps between work-queue refills of a wave
    int refill_min;    // idle lanes a wave waits for before it refills
    // ensemble launches: scenario table (device) and its length
    const DevScen* scen;
    int n_scen;
    // variants: Eq. 3 stability, decay chain, stochastic deposition
    float inv_L;                          // 1/L (kz_kind 3)
    int chain, dep_mode, n_nuc;
    float bc[4][4];  // activity of nuclide n per unit a0: sum_j bc[n][j] exp(-lambda_j age)
    // deposition grid and accumulators
    double* dep;
    double* ledger;
    uint32_t* ctrl;
    int dnx, dny, dmode;
    int dep_copies;  // copies of the deposition grid one after another (>= 1)
    // deposition cell (quad) coordinate of x: x d_inv_dx + d_cx, d_cx =
    // -x0/dx (nearest cell) or -x0/dx - 1/2 (cloud in cell); the same in y
    float d_cx, d_cy, d_inv_dx, d_inv_dy, d_fnx, d_fny;
    float dscale;
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter (c0, c1, 0, 0),
// key (k0, k1).  The two upper counter words are zero for the turbulence
// stream, which removes one multiply from the first round.
// ---------------------------------------------------------------------------
template <bool UNIFORM_KEY>
__device__ __forceinline__ void philox_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t k0,
                                          uint32_t k1, uint32_t r[4])
{
    uint32_t c3 = 0u;
    if constexpr (UNIFORM_KEY) {  // one key for the whole launch: keep it scalar
        k0 = __builtin_amdgcn_readfirstlane(k0);
        k1 = __builtin_amdgcn_readfirstlane(k1);
    }
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        // three-input XOR in one v_bitop3_b32 (truth table 0x96): the
        // compiler splits a ^ b ^ c into two v_xor_b32
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
        // Keep the key schedule as two registers updated per round: hoisting
        // all twenty round keys out of the particle loop would exhaust the
        // registers and spill.
        if constexpr (UNIFORM_KEY) asm volatile("" : "+s"(k0), "+s"(k1));
        else asm volatile("" : "+v"(k0), "+v"(k1));
    }
    r[0] = c0;
    r[1] = c1;
    r[2] = c2;
    r[3] = c3;
}

// Per-particle source values: uniform over a plain launch, per lane in an
// ensemble launch (each lane may hold a particle of another scenario).
struct SrcVals {
    float a0, wscale, dry_c1, dry_c2;
    uint32_t key1;
    int scen;
};

// Uniform in (0, 1] on the 2^-24 lattice: exact in float.
__device__ __forceinline__ float lattice_uniform(uint32_t r)
{
    return (float)((r >> 8) + 1u) * 5.9604644775390625e-08f;
}

// Three standard normals (Eq. 2) by the trigonometric Box-Muller form.
// v_log_f32 is log2 and v_sin/v_cos take the angle in revolutions, so
// 2 pi u needs no multiply and no range reduction.
template <bool UNIFORM_KEY>
__device__ __forceinline__ void normals3(uint32_t id, uint32_t step, uint32_t k0,
                                         uint32_t k1, float& xi0, float& xi1,
                                         float& xi2)
{
    uint32_t r[4];
    philox_10<UNIFORM_KEY>(id, step, 0u, k0, k1, r);
    const float m2ln2 = -1.3862943611198906f;  // -2 ln 2
    const float u0 = lattice_uniform(r[0]);
    const float u1 = lattice_uniform(r[1]);
    const float u2 = lattice_uniform(r[2]);
    const float u3 = lattice_uniform(r[3]);
    const float rho0 = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u0));
    const float rho2 = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u2));
    xi0 = rho0 * __builtin_amdgcn_cosf(u1);
    xi1 = rho0 * __builtin_amdgcn_sinf(u1);
    xi2 = rho2 * __builtin_amdgcn_cosf(u3);
}

// Global-memory views of pointers.  Pointers read from LDS (the launch
// constants are kept there) lose their address space, and loads through them
// become flat loads, which also count against the LDS wait counter.
typedef __attribute__((address_space(1))) const float gfloat;
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* as_global(const T* p)
{
    return (const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* as_global(T* p)
{
    return (__attribute__((address_space(1))) T*)p;
}

// First uniform of the stochastic-deposition stream: Philox counter
// (id, step, 1, 0).
template <bool UNIFORM_KEY>
__device__ __forceinline__ float removal_uniform(uint32_t id, uint32_t step, uint32_t k0,
                                                 uint32_t k1)
{
    uint32_t r[4];
    philox_10<UNIFORM_KEY>(id, step, 1u, k0, k1, r);
    return lattice_uniform(r[0]);
}

// v clamped to [lo, hi] (lo <= hi) in one v_med3_f32.
__device__ __forceinline__ float clampf(float v, float lo, float hi)
{
    return __builtin_amdgcn_fmed3f(v, lo, hi);
}

__device__ __forceinline__ float lerpf(float a, float b, float w)
{
    return fmaf(w, b - a, a);
}

// Lower node and weight of a coordinate on cell-centred nodes, clamped:
// fractional index pos inv_d + c (c folds the origin and the half cell).
__device__ __forceinline__ void axis(float pos, float c, float inv_d, float fmax,
                                     int imax, int& i0, float& w)
{
    const float fi = clampf(fmaf(pos, inv_d, c), 0.0f, fmax);
    i0 = min((int)fi, imax);
    w = fi - (float)i0;
}

// Vertical node and weight for explicitly given node heights (binary search).
__device__ __forceinline__ void levels(const float* __restrict__ levp, int nz, float z,
                                       int& k0, float& w)
{
    const gfloat* lev = as_global(levp);
    if (nz == 1 || z <= lev[0]) { k0 = 0; w = 0.0f; return; }
    if (z >= lev[nz - 1]) { k0 = nz - 2; w = 1.0f; return; }
    int lo = 0, hi = nz - 1;  // lev[lo] <= z < lev[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (lev[mid] <= z) lo = mid; else hi = mid;
    }
    k0 = lo;
    w = (z - lev[lo]) / (lev[lo + 1] - lev[lo]);
}

// Wind stencil of one particle: the corner values of the trilinear cell at
// one or two field times, and the interpolation weights.  Gathering (issuing
// the loads) and interpolating are separate so that the random numbers and
// the diffusivity, which do not depend on the wind, are computed while the
// loads are in flight.
template <int NCOMP, int TIME>
struct WindTap {
    float c[TIME ? 2 : 1][8][NCOMP];
    float wx, wy, wz, wt;
};

template <int NCOMP>
__device__ __forceinline__ void gather8(const float* __restrict__ fp, int base, int di, int dj,
                                        int dk, float (&c)[8][NCOMP])
{
    const gfloat* f = as_global(fp);
    if constexpr (NCOMP == 2) {
        if (di == 2) {
            // (u, v) of the two x-neighbours are 16 contiguous, 8-byte aligned
            // bytes: one 16-byte load per (y, z) corner pair
            typedef float pair4 __attribute__((ext_vector_type(4), aligned(8)));
            typedef __attribute__((address_space(1))) const pair4 gpair4;
            const int o[4] = {base, base + dj, base + dk, base + dk + dj};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const pair4 v = *reinterpret_cast<gpair4*>(f + o[q]);
                c[2 * q][0] = v.x;
                c[2 * q][1] = v.y;
                c[2 * q + 1][0] = v.z;
                c[2 * q + 1][1] = v.w;
            }
            return;
        }
    }
    const int o[8] = {base, base + di, base + dj, base + dj + di,
                      base + dk, base + dk + di, base + dk + dj, base + dk + dj + di};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        if constexpr (NCOMP == 2) {
            typedef float pair2 __attribute__((ext_vector_type(2)));
            typedef __attribute__((address_space(1))) const pair2 gpair2;
            const pair2 v = *reinterpret_cast<gpair2*>(f + o[q]);
            c[q][0] = v.x;
            c[q][1] = v.y;
        } else {
#pragma unroll
            for (int cc = 0; cc < NCOMP; ++cc) c[q][cc] = f[o[q] + cc];
        }
    }
}

// The stencil at both times from a time-pair copy of a two-component field
// interval: per node (u, v) at the interval's start and end side by side,
// 16 bytes, levels innermost, so the two levels of each of the four
// columns are 32 contiguous bytes -- two 16-byte loads, mostly in one cache
// line, for both times -- and particles of one column at any height share
// lines.  Corner q of the trilinear stencil: bit 0 i, bit 1 j, bit 2 k.
__device__ __forceinline__ void gather8_tpair(const float* __restrict__ fp, int base, int di,
                                              int dj, int dk, float (&c)[2][8][2])
{
    typedef float quad __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(1))) const quad gquad;
    const gfloat* f = as_global(fp);
    const int o[4] = {base, base + di, base + dj, base + dj + di};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const quad a = *reinterpret_cast<gquad*>(f + o[q]);
        const quad b = *reinterpret_cast<gquad*>(f + o[q] + dk);
        c[0][q][0] = a.x;
        c[0][q][1] = a.y;
        c[1][q][0] = a.z;
        c[1][q][1] = a.w;
        c[0][q + 4][0] = b.x;
        c[0][q + 4][1] = b.y;
        c[1][q + 4][0] = b.z;
        c[1][q + 4][1] = b.w;
    }
}

template <int NCOMP>
__device__ __forceinline__ void trilinear(const float (&c)[8][NCOMP], float wx, float wy,
                                          float wz, float out[3])
{
#pragma unroll
    for (int cc = 0; cc < NCOMP; ++cc) {
        const float a = lerpf(c[0][cc], c[1][cc], wx);
        const float b = lerpf(c[2][cc], c[3][cc], wx);
        const float e = lerpf(c[4][cc], c[5][cc], wx);
        const float g = lerpf(c[6][cc], c[7][cc], wx);
        out[cc] = lerpf(lerpf(a, b, wy), lerpf(e, g, wy), wz);
    }
    if constexpr (NCOMP == 2) out[2] = 0.0f;
}

// Issue the loads of the wind stencil at (x, y, z) at the start of step s
// (Sec. 3.2: linear in x, y, z and t).
// Time weight of step s: time nodes sit at t0 + k dt_field (not
// cell-centred).  The weight is the same for every particle of a step; in
// FP32 the rounding of 1/dt_field and of the fractional node index would
// bias it by up to ~1e-7 for a whole field interval, a coherent wind error
// that moves every trajectory the same way, so it is taken in FP64.
__device__ __forceinline__ float time_weight(const StepConst& p, int s, int& t0)
{
    const double ft = fmin(fmax(fma((double)s, p.ft_step, p.ft_zero), 0.0), (double)p.ftmax);
    t0 = min((int)ft, p.tmaxi);
    return (float)(ft - (double)t0);
}

// Launches on a time-pair copy over at most kWtTable steps tabulate the time
// weight per block (the same FP64 expression, rounded once): a lookup per
// step instead of eight FP64 operations.
constexpr int kWtTable = 1024;

template <int NCOMP, int TIME, bool LEVELS>
__device__ __forceinline__ void wind_gather(const StepConst& p, float x, float y, float z,
                                            int s, WindTap<NCOMP, TIME>& w,
                                            const float* wt_tab = nullptr)
{
    int i0, j0, k0;
    axis(x, p.fcx, p.inv_dx, p.fxmax, p.imax, i0, w.wx);
    axis(y, p.fcy, p.inv_dy, p.fymax, p.jmax, j0, w.wy);
    if constexpr (LEVELS) levels(p.lev, p.nz, z, k0, w.wz);
    else axis(z, -0.5f, p.inv_dz, p.fzmax, p.kmax, k0, w.wz);
    int base = k0 * p.sk + j0 * p.sj + i0 * p.si;
    if constexpr (NCOMP == 2 && TIME == 2) {  // a time-pair copy, known at compile time
        // (one interval: the time stride is 0, only the weight changes)
        int t0;
        w.wt = wt_tab ? wt_tab[s - p.step0] : time_weight(p, s, t0);
        gather8_tpair(p.f, base, p.di, p.dj, p.dk, w.c);
    } else if constexpr (TIME) {
        int t0;
        w.wt = time_weight(p, s, t0);
        base += t0 * p.st;
        if constexpr (NCOMP == 2) {
            if (p.tpair) {
                gather8_tpair(p.f, base, p.di, p.dj, p.dk, w.c);
                return;
            }
        }
        gather8<NCOMP>(p.f, base, p.di, p.dj, p.dk, w.c[0]);
        gather8<NCOMP>(p.f, base + p.dt_off, p.di, p.dj, p.dk, w.c[1]);
    } else {
        w.wt = 0.0f;
        gather8<NCOMP>(p.f, base, p.di, p.dj, p.dk, w.c[0]);
    }
}

template <int NCOMP, int TIME>
__device__ __forceinline__ void wind_interp(const WindTap<NCOMP, TIME>& w, float uvw[3])
{
    trilinear<NCOMP>(w.c[0], w.wx, w.wy, w.wz, uvw);
    if constexpr (TIME) {
        float b[3];
        trilinear<NCOMP>(w.c[1], w.wx, w.wy, w.wz, b);
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) uvw[cc] = lerpf(uvw[cc], b[cc], w.wt);
    }
}

// Vertical diffusivity and its slope (Eq. 3 with Phi = 1, or constant);
// KZ is the profile kind (0 constant, 1 parabolic, 2 Eq. 3 exponent).
template <int KZ>
__device__ __forceinline__ void kz_profile(const StepConst& p, float z, float& K, float& dK);

// Eq. (3) with the Businger-Dyer similarity function for heat of
// s = (z + z0)/L: Phi = 1 + 5 s (stable), (1 - 16 s)^(-1/2) (unstable).
__device__ __forceinline__ void kz_stability(const StepConst& p, float z, float& K, float& dK)
{
    const float zc = fmaxf(z, 0.0f);
    const float g = fmaf(-zc, p.inv_Hmix, 1.0f);
    const float zz = zc + p.z0;
    const bool inside = zc <= p.H_mix;  // at H_mix: K = 0 and the slope from below
    const float f = p.ku * zz * g * g;                        // Phi = 1 profile
    const float df = p.ku * g * fmaf(-2.0f * zz, p.inv_Hmix, g);
    float rphi, drphi;  // 1/Phi and its slope in z
    if (p.inv_L >= 0.0f) {
        const float q = __builtin_amdgcn_rcpf(fmaf(5.0f * zz, p.inv_L, 1.0f));
        rphi = q;
        drphi = -5.0f * p.inv_L * q * q;
    } else {
        const float w = fmaf(-16.0f * zz, p.inv_L, 1.0f);
        const float sw = __builtin_amdgcn_sqrtf(w);
        rphi = sw;
        drphi = -8.0f * p.inv_L * __builtin_amdgcn_rcpf(sw);
    }
    K = inside ? f * rphi : 0.0f;
    dK = inside ? fmaf(df, rphi, f * drphi) : 0.0f;
}

template <int KZ>
__device__ __forceinline__ void kz_profile(const StepConst& p, float z, float& K, float& dK)
{
    if constexpr (KZ == 4) {  // kind chosen at run time (general kernels)
        switch (p.kz_kind) {
        case 0: kz_profile<0>(p, z, K, dK); break;
        case 1: kz_profile<1>(p, z, K, dK); break;
        case 2: kz_profile<2>(p, z, K, dK); break;
        default: kz_stability(p, z, K, dK); break;
        }
    } else if constexpr (KZ == 3) {
        kz_stability(p, z, K, dK);
    } else if constexpr (KZ == 0) {
        K = p.Kz_const;
        dK = 0.0f;
    } else {
        const float zc = fmaxf(z, 0.0f);
        const float g = fmaf(-zc, p.inv_Hmix, 1.0f);
        const float zz = zc + p.z0;
        // at H_mix itself the profile (K = 0, slope from below): the drift
        // takes a particle at the top of the mixed layer back down
        const bool inside = zc <= p.H_mix;
        if constexpr (KZ == 1) {
            K = inside ? p.ku * zz * g : 0.0f;
            dK = inside ? p.ku * fmaf(-zz, p.inv_Hmix, g) : 0.0f;
        } else {
            K = inside ? p.ku * zz * g * g : 0.0f;
            dK = inside ? p.ku * g * fmaf(-2.0f * zz, p.inv_Hmix, g) : 0.0f;
        }
    }
}

// Wet-deposition rate in the elliptical rain region with a linear edge.
__device__ __forceinline__ float wet_rate(const StepConst& p, float x, float y)
{
    const float dx = x - p.rcx, dy = y - p.rcy;
    const float xr = fmaf(p.r_ca_a, dx, p.r_sa_a * dy);
    const float yr = fmaf(p.r_ca_b, dy, -p.r_sa_b * dx);
    const float re = __builtin_amdgcn_sqrtf(fmaf(xr, xr, yr * yr));
    return p.L0 * clampf(fmaf(1.0f - re, p.inv_edge, 0.5f), 0.0f, 1.0f);
}

// Fold of z into [0, H_top] (reflection at the ground and the lid): one
// fold each, and the general fold-until-inside for the (never seen) larger
// steps.  *sign receives the slope of the fold (+1 or -1).
__device__ __forceinline__ float fold_z(float zn, float H_top, float* sign = nullptr)
{
    float sg = zn < 0.0f ? -1.0f : 1.0f;
    zn = fabsf(zn);
    if (zn > H_top) {
        zn = 2.0f * H_top - zn;
        sg = -sg;
    }
    if (zn < 0.0f || zn > H_top) {
#pragma unroll 1
        for (int it = 0; it < 64; ++it) {
            if (zn < 0.0f) zn = -zn;
            else if (zn > H_top) zn = 2.0f * H_top - zn;
            else break;
            sg = -sg;
        }
    }
    if (sign) *sign = sg;
    return zn;
}

// Motion of one particle over step s (Eq. 1 with Eq. 2, the Ito drift and
// Visser's midpoint for K_z, then the fold): the wind is sampled at the
// start-of-step position and time.  The loads are issued first; everything
// up to the interpolation is independent of them.  Returns the vertical
// normal xi2 (the one random number the derivative of the step needs).
// Horizontal positions are sums of thousands of steps of tens of metres on
// values up to 5e4 m, where a float rounds to 4 mm: rounded every step, the
// roundings would walk ~0.1 m away from the exact sum in 12 h.  Each
// coordinate therefore carries its rounding residual lo (compensated
// summation, Kahan): hi + lo holds the running sum exactly, hi is that sum
// rounded to float and is the position every other part of the step uses.
__device__ __forceinline__ float comp_add(float hi, float& lo, float d)
{
    const float y = d + lo;
    const float t = hi + y;
    lo = y - (t - hi);
    return t;
}

template <int NCOMP, int TIME, bool LEVELS, int KZ, bool UNIFORM_KEY>
__device__ __forceinline__ float motion(const StepConst& p, float wscale, uint32_t key1,
                                        uint32_t gid, int s, float x, float y, float z,
                                        float& xl, float& yl, float& xn, float& yn, float& zn,
                                        const float* wt_tab = nullptr)
{
    WindTap<NCOMP, TIME> tap;
    wind_gather<NCOMP, TIME, LEVELS>(p, x, y, z, s, tap, wt_tab);
    float xi0, xi1, xi2;
    normals3<UNIFORM_KEY>(gid, (uint32_t)s, p.key0, key1, xi0, xi1, xi2);
    float K, dK, Km, dKm;
    kz_profile<KZ>(p, z, K, dK);
    const float zm = clampf(fmaf(p.half_dt, dK, z), 0.0f, p.H_mix);
    kz_profile<KZ>(p, zm, Km, dKm);
    float uvw[3];
    wind_interp<NCOMP, TIME>(tap, uvw);
    xn = comp_add(x, xl, fmaf(xi0, p.sKh, (wscale * uvw[0]) * p.dt));
    yn = comp_add(y, yl, fmaf(xi1, p.sKh, (wscale * uvw[1]) * p.dt));
    zn = fold_z(fmaf(xi2 * __builtin_amdgcn_sqrtf(Km), p.s2dt,
                     fmaf(fmaf(wscale, uvw[2], dK), p.dt, z)),
                p.H_top);
    return xi2;
}

// Deposition rate at the post-move position (Sec. 2): dry v_d phi(z) =
// c1 - c2 z below h_s, plus wet scavenging in the rain region.
__device__ __forceinline__ float deposition_rate(const StepConst& p, float dry_c1, float dry_c2,
                                                 float x, float y, float z)
{
    float k = 0.0f;
    if (z < p.h_s) k = fmaxf(fmaf(-dry_c2, z, dry_c1), 0.0f);
    if (p.L0 > 0.0f) k += wet_rate(p, x, y);
    return k;
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

// Mass left after a step at deposition rate k: m exp(-k dt), formed as
// m + m (exp(-k dt) - 1) so that the one rounding is of the result (a factor
// exp(-k dt) rounded near 1 would carry up to 2^-25 of error into every
// step's product, over thousands of steps).
__device__ __forceinline__ float deposit_mass(float m, float k, float dt)
{
    return k > 0.0f ? fmaf(m, expm1_neg(-k * dt), m) : m;
}

}  // namespace lpm

// liblpm: receptor concentrations of a release and their adjoint with respect
// to the source parameters (h, q, s_w, v_d), for gfx950 (MI355X).
//
// Kernels
//  - receptor_kernel: Gaussian-kernel concentrations at receptor points from
//    the recorded output-step states.  A block stages 256 particle records
//    (x, y, z, activity) in LDS; each wave takes 64 of them and each lane one
//    receptor, so the lanes read the same LDS entry (broadcast) and sum their
//    own receptor in FP64 registers with no reduction until the block's end.
//  - adjoint_kernel: per particle, a reverse sweep over its path with the
//    random numbers held fixed.  The forward run's record k - 1 is the
//    checkpoint of segment k (rec_every steps); the segment is recomputed
//    with the forward kernel's own motion code into a per-thread tape in the
//    caller's workspace (coalesced [step][thread] rows, L2/MALL-resident for
//    a resident grid), the output of the segment's last step is injected,
//    and the segment is swept backwards.  The gradient is reduced per block
//    and added with one FP64 atomic per component.
#include <hip/hip_runtime.h>

#include <limits.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "lpm.h"
#include "lpm_device.h"
#include "lpm_host.h"

namespace lpm {

typedef float f4 __attribute__((ext_vector_type(4)));  // global-memory vector of 4 floats

// Gaussian receptor kernel constants (host-folded).
struct KernelConst {
    float inv_sh2, inv_sz2;  // 1 / sigma^2
    float eh, ez;            // log2(e) / (2 sigma^2): exponent scales for exp2
    float ch, cz;            // normalisations 1 / (2 pi sigma_h^2), 1 / (sqrt(2 pi) sigma_z)
};

struct RecConst {
    long long n_total, id_base, id_stride, i_hi;
    int s_release, nnuc, n_rcp, rec_step0, rec_every, pad;
    float a0, dt, weight;
    float lam_l2e[4];
    float bsum[4];  // sum over nuclides of the chain activity coefficients
    KernelConst kc;
    const float* rx;
    const float* ry;
    const float* rz;
};

// Horizontal and vertical kernel factors of one receptor at (x, y, z).
__device__ __forceinline__ void kernel_parts(const KernelConst& kc, float dx, float dy, float z,
                                             float zr, float& gh, float& n1, float& n2)
{
    gh = kc.ch * __builtin_amdgcn_exp2f(-fmaf(dx, dx, dy * dy) * kc.eh);
    const float d1 = z - zr, d2 = z + zr;
    n1 = kc.cz * __builtin_amdgcn_exp2f(-(d1 * d1) * kc.ez);
    n2 = kc.cz * __builtin_amdgcn_exp2f(-(d2 * d2) * kc.ez);
}

__global__ __launch_bounds__(kBlock) void receptor_kernel(const RecConst g, const float4* rec,
                                                          const int* last, long long rec_stride,
                                                          double* c_out)
{
    constexpr int kWaves = kBlock / 64;
    __shared__ float4 ent[kBlock];
    __shared__ double part[kWaves][64];
    const int k = blockIdx.y;
    const int step = g.rec_step0 + k * g.rec_every;
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    float4 e = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (i < g.i_hi) {
        const long long b = birth(g.id_base + i * g.id_stride, g.s_release, g.n_total);
        if (b <= step && step < last[i]) {
            const float4 r = rec[(long long)k * rec_stride + i];
            if (r.w > 0.0f) {
                const float age = (float)(step + 1 - (int)b) * g.dt;
                float F = 0.0f;
                for (int n = 0; n < g.nnuc; ++n)
                    F = fmaf(g.bsum[n], __builtin_amdgcn_exp2f(-g.lam_l2e[n] * age), F);
                e = make_float4(r.x, r.y, r.z, g.a0 * r.w * F);
            }
        }
    }
    ent[threadIdx.x] = e;
    if (!__syncthreads_or(e.w > 0.0f)) return;  // no airborne particle in this block
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int r0 = 0; r0 < g.n_rcp; r0 += 64) {
        const int r = r0 + lane;
        const bool on = r < g.n_rcp;
        const float X = on ? g.rx[r] : 0.0f, Y = on ? g.ry[r] : 0.0f, Z = on ? g.rz[r] : 0.0f;
        double acc = 0.0;
        for (int j = 0; j < 64; ++j) {
            const float4 q = ent[wv * 64 + j];  // same entry in every lane
            if (q.w == 0.0f) continue;
            float gh, n1, n2;
            kernel_parts(g.kc, q.x - X, q.y - Y, q.z, Z, gh, n1, n2);
            acc += (double)(q.w * gh * (n1 + n2));
        }
        part[wv][lane] = acc;
        __syncthreads();
        if (wv == 0 && on) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) t += part[w][lane];
            if (t != 0.0) atomicAdd(c_out + r, t * (double)g.weight);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Adjoint
// ---------------------------------------------------------------------------
struct AdjConst {
    const float4* rec;
    const int* last;
    long long rec_stride, n_local;
    int rec_every, n_rec, n_rcp, nnuc;
    float4* tape;   // [rec_every + 1][T]: x, y, z, xi2 before each step (+ the end state)
    float* tapem;   // [rec_every + 1][T]: m
    float phi_c1, phi_c2;  // dry-deposition shape 2/h_s (1 - z/h_s) = c1 - c2 z
    float inv_q, weight;
    float bsum[4];  // sum over nuclides of the chain activity coefficients
    KernelConst kc;
    const float* rx;
    const float* ry;
    const float* rz;
    const double* gbar;
    double* grad;   // [5]
};

// Second derivative of K_z (Eq. 3 forms of kz_profile); zero outside the
// mixing layer and for a constant K_z.
template <int KZ>
__device__ __forceinline__ float kz_second(const StepConst& p, float z)
{
    if constexpr (KZ == 0) {
        return 0.0f;
    } else {
        const float zc = fmaxf(z, 0.0f);
        if (!(zc <= p.H_mix)) return 0.0f;
        if constexpr (KZ == 1) {
            return -2.0f * p.ku * p.inv_Hmix;
        } else {
            const float g = fmaf(-zc, p.inv_Hmix, 1.0f);
            return p.ku * p.inv_Hmix * fmaf(2.0f * (zc + p.z0), p.inv_Hmix, -4.0f * g);
        }
    }
}

// Wet-deposition rate (as wet_rate) and its gradient in (x, y); zero slope
// where the linear edge is clamped.
__device__ __forceinline__ float wet_rate_grad(const StepConst& p, float x, float y, float& gx,
                                               float& gy)
{
    const float dx = x - p.rcx, dy = y - p.rcy;
    const float xr = fmaf(p.r_ca_a, dx, p.r_sa_a * dy);
    const float yr = fmaf(p.r_ca_b, dy, -p.r_sa_b * dx);
    const float re = __builtin_amdgcn_sqrtf(fmaf(xr, xr, yr * yr));
    const float f = fmaf(1.0f - re, p.inv_edge, 0.5f);
    gx = gy = 0.0f;
    if (f > 0.0f && f < 1.0f && re > 0.0f) {
        const float s = -p.L0 * p.inv_edge / re;
        gx = s * fmaf(xr, p.r_ca_a, -yr * p.r_sa_b);
        gy = s * fmaf(xr, p.r_sa_a, yr * p.r_ca_b);
    }
    return p.L0 * clampf(f, 0.0f, 1.0f);
}

// Slope of a clamped cell-centred axis: inv_d inside the node range, else 0.
__device__ __forceinline__ float axis_slope(float pos, float c, float inv_d, float fmax)
{
    const float f = fmaf(pos, inv_d, c);
    return (f > 0.0f && f < fmax) ? inv_d : 0.0f;
}

// Partial derivatives of the trilinear interpolant in its three weights.
template <int NCOMP>
__device__ __forceinline__ void trilinear_dw(const float (&c)[8][NCOMP], float wx, float wy,
                                             float wz, float d[3][3])
{
#pragma unroll
    for (int cc = 0; cc < NCOMP; ++cc) {
        const float a = lerpf(c[0][cc], c[1][cc], wx), b = lerpf(c[2][cc], c[3][cc], wx);
        const float e = lerpf(c[4][cc], c[5][cc], wx), g = lerpf(c[6][cc], c[7][cc], wx);
        d[cc][0] = lerpf(lerpf(c[1][cc] - c[0][cc], c[3][cc] - c[2][cc], wy),
                         lerpf(c[5][cc] - c[4][cc], c[7][cc] - c[6][cc], wy), wz);
        d[cc][1] = lerpf(b - a, g - e, wz);
        d[cc][2] = lerpf(e, g, wy) - lerpf(a, b, wy);
    }
    if constexpr (NCOMP == 2) d[2][0] = d[2][1] = d[2][2] = 0.0f;
}

// Wind (before the wind scale) and its gradient G[c][d] = d uvw_c / d x_d at
// (x, y, z) at the start of step s; the value is the forward kernel's
// interpolation.
template <int NCOMP, bool TIME, bool LEVELS>
__device__ __forceinline__ void wind_and_grad(const StepConst& p, float x, float y, float z,
                                              int s, float uvw[3], float G[3][3])
{
    WindTap<NCOMP, TIME> tap;
    wind_gather<NCOMP, TIME, LEVELS>(p, x, y, z, s, tap);
    const float sx = axis_slope(x, p.fcx, p.inv_dx, p.fxmax);
    const float sy = axis_slope(y, p.fcy, p.inv_dy, p.fymax);
    float sz;
    if constexpr (LEVELS) {
        const gfloat* lev = as_global(p.lev);
        int k0 = 0;
        float w;
        levels(p.lev, p.nz, z, k0, w);
        sz = (p.nz > 1 && z > lev[0] && z < lev[p.nz - 1]) ? 1.0f / (lev[k0 + 1] - lev[k0]) : 0.0f;
    } else {
        sz = axis_slope(z, -0.5f, p.inv_dz, p.fzmax);
    }
    wind_interp<NCOMP, TIME>(tap, uvw);
    float d[3][3];
    trilinear_dw<NCOMP>(tap.c[0], tap.wx, tap.wy, tap.wz, d);
    if constexpr (TIME) {
        float d1[3][3];
        trilinear_dw<NCOMP>(tap.c[1], tap.wx, tap.wy, tap.wz, d1);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int q = 0; q < 3; ++q) d[c][q] = lerpf(d[c][q], d1[c][q], tap.wt);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        G[c][0] = d[c][0] * sx;
        G[c][1] = d[c][1] * sy;
        G[c][2] = d[c][2] * sz;
    }
}

// Adjoint of one step.  (x, y, z) and xi2: state and vertical normal before
// step s; (xn, yn, zn, mn): state after it.  On entry (xb, yb, zb, mb) is the
// adjoint of the state after the step, on return that of the state before;
// swb and vdb receive the step's contribution to dL/ds_w and dL/dv_d.
template <int NCOMP, bool TIME, bool LEVELS, int KZ>
__device__ __forceinline__ void reverse_step(const StepConst& p, const AdjConst& a, int s, float x,
                                             float y, float z, float xi2, float xn, float yn,
                                             float zn, float mn, float& xb, float& yb, float& zb,
                                             float& mb, float& swb, float& vdb)
{
    float U[3], G[3][3];
    wind_and_grad<NCOMP, TIME, LEVELS>(p, x, y, z, s, U, G);
    float K, dK, Km, dKm;
    kz_profile<KZ>(p, z, K, dK);
    const float K2 = kz_second<KZ>(p, z);
    const float zm_raw = fmaf(p.half_dt, dK, z);
    const float zm = clampf(zm_raw, 0.0f, p.H_mix);
    const float dzm = (zm_raw > 0.0f && zm_raw < p.H_mix) ? fmaf(p.half_dt, K2, 1.0f) : 0.0f;
    kz_profile<KZ>(p, zm, Km, dKm);
    const float sK = __builtin_amdgcn_sqrtf(Km);
    const float zn0 = fmaf(xi2 * sK, p.s2dt, fmaf(fmaf(p.wscale, U[2], dK), p.dt, z));
    float sg;
    fold_z(zn0, p.H_top, &sg);
    // d sqrt(2 Km dt) / dz
    const float dsq = sK > 0.0f ? 0.5f * p.s2dt * dKm * dzm / sK : 0.0f;

    // deposition at the new position: k = v_d phi(zn) + Lambda(xn, yn)
    float dkd = 0.0f, phi = 0.0f;
    if (zn < p.h_s) {
        if (fmaf(-p.dry_c2, zn, p.dry_c1) > 0.0f) dkd = -p.dry_c2;
        phi = fmaxf(fmaf(-a.phi_c2, zn, a.phi_c1), 0.0f);
    }
    float gx = 0.0f, gy = 0.0f;
    if (p.L0 > 0.0f) wet_rate_grad(p, xn, yn, gx, gy);
    const float k = deposition_rate(p, p.dry_c1, p.dry_c2, xn, yn, zn);
    const float ek = k > 0.0f ? __builtin_amdgcn_exp2f(-1.4426950408889634f * k * p.dt) : 1.0f;

    // mn = m exp(-k dt)
    const float kb = -p.dt * mn * mb;
    mb = mb * ek;
    float xbn = fmaf(kb, gx, xb), ybn = fmaf(kb, gy, yb);
    const float zbn = fmaf(kb, dkd, zb);
    vdb = fmaf(kb, phi, vdb);
    // fold, then the move of Eq. (1)-(2)
    const float zb0 = sg * zbn;
    swb = fmaf(p.dt, fmaf(xbn, U[0], fmaf(ybn, U[1], zb0 * U[2])), swb);
    const float t = p.wscale * p.dt;
    xb = fmaf(t, fmaf(xbn, G[0][0], fmaf(ybn, G[1][0], zb0 * G[2][0])), xbn);
    yb = fmaf(t, fmaf(xbn, G[0][1], fmaf(ybn, G[1][1], zb0 * G[2][1])), ybn);
    zb = fmaf(t, fmaf(xbn, G[0][2], fmaf(ybn, G[1][2], zb0 * G[2][2])),
              zb0 * (1.0f + p.dt * K2 + xi2 * dsq));
}

template <int NCOMP, bool TIME, bool LEVELS, int KZ>
__global__ __launch_bounds__(kBlock) void adjoint_kernel(const StepConst pk, const AdjConst ak)
{
    // launch constants in LDS (kept in SGPRs across the loops they spill)
    __shared__ StepConst p;
    __shared__ AdjConst a;
    __shared__ float4 rcp[LPM_MAX_RECEPTORS];  // x, y, z, dL/dc_r * weight
    if (threadIdx.x < sizeof(StepConst) / 4)
        reinterpret_cast<uint32_t*>(&p)[threadIdx.x] = reinterpret_cast<const uint32_t*>(&pk)[threadIdx.x];
    if (threadIdx.x < sizeof(AdjConst) / 4)
        reinterpret_cast<uint32_t*>(&a)[threadIdx.x] = reinterpret_cast<const uint32_t*>(&ak)[threadIdx.x];
    for (int r = threadIdx.x; r < ak.n_rcp; r += kBlock)
        rcp[r] = make_float4(ak.rx[r], ak.ry[r], ak.rz[r], (float)(ak.gbar[r] * (double)ak.weight));
    __syncthreads();

    const int E = a.rec_every;
    const int n_steps = a.n_rec * E;
    const long long T = (long long)gridDim.x * kBlock;
    const long long tid = (long long)blockIdx.x * kBlock + threadIdx.x;
    auto tape = as_global(reinterpret_cast<f4*>(a.tape));
    auto tapem = as_global(a.tapem);
    auto recs = as_global(reinterpret_cast<const f4*>(a.rec));
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};

    for (long long i = tid; i < a.n_local; i += T) {
        const long long g = p.id_base + i * p.id_stride;
        const long long bl = birth(g, p.s_release, p.n_total);
        if (bl >= n_steps) continue;
        const int lastv = as_global(a.last)[i];
        if (lastv == INT_MIN) continue;
        const int b = (int)bl;
        // first step not differentiated: the exit step, or the end
        const int e = lastv == INT_MAX ? n_steps : lastv;
        // last segment whose output step (k + 1) E - 1 precedes e
        const int kmax = min(e / E - 1, a.n_rec - 1);
        const int kb = b / E;
        float xb = 0.0f, yb = 0.0f, zb = 0.0f, mb = 0.0f, swb = 0.0f, vdb = 0.0f, J = 0.0f;
        for (int k = kmax; k >= kb; --k) {
            const int s_lo = max(k * E, b), s_hi = (k + 1) * E - 1;
            float x, y, z, m;
            if (s_lo == b) {
                x = p.xs; y = p.ys; z = p.h; m = 1.0f;
            } else {
                const f4 r = recs[(long long)(k - 1) * a.rec_stride + i];
                x = r.x; y = r.y; z = r.z; m = r.w;
            }
            // recompute the segment into the tape (the forward's compensated
            // position sums, from the float checkpoint)
            float xl = 0.0f, yl = 0.0f;
            for (int s = s_lo; s <= s_hi; ++s) {
                const long long row = (long long)(s - s_lo) * T + tid;
                float xn, yn, zn;
                const float xi2 = motion<NCOMP, TIME, LEVELS, KZ, true>(p, p.wscale, p.key1,
                                                                       (uint32_t)g, s, x, y, z,
                                                                       xl, yl, xn, yn, zn);
                tape[row] = f4{x, y, z, xi2};
                tapem[row] = m;
                const float kd = deposition_rate(p, p.dry_c1, p.dry_c2, xn, yn, zn);
                m = deposit_mass(m, kd, p.dt);
                x = xn; y = yn; z = zn;
            }
            {
                const long long row = (long long)(s_hi + 1 - s_lo) * T + tid;
                tape[row] = f4{x, y, z, 0.0f};
                tapem[row] = m;
            }
            // output of the segment's last step (state after s_hi)
            const float age = (float)(s_hi + 1 - b) * p.dt;
            float F = 0.0f;
            for (int n = 0; n < a.nnuc; ++n)
                F = fmaf(a.bsum[n], __builtin_amdgcn_exp2f(-p.lam_l2e[n] * age), F);
            const float aF = p.a0 * F, A = aF * m;
            for (int r = 0; r < a.n_rcp; ++r) {
                const float4 q = rcp[r];
                const float dx = x - q.x, dy = y - q.y;
                float gh, n1, n2;
                kernel_parts(a.kc, dx, dy, z, q.z, gh, n1, n2);
                const float kv = gh * (n1 + n2);
                const float w = q.w * kv;
                J = fmaf(w, A, J);
                mb = fmaf(w, aF, mb);
                const float wA = w * A;
                xb = fmaf(-dx * a.kc.inv_sh2, wA, xb);
                yb = fmaf(-dy * a.kc.inv_sh2, wA, yb);
                const float dn = -((z - q.z) * n1 + (z + q.z) * n2) * a.kc.inv_sz2;
                zb = fmaf(q.w * A * gh, dn, zb);
            }
            // sweep the segment backwards
            for (int s = s_hi; s >= s_lo; --s) {
                const long long row = (long long)(s - s_lo) * T + tid;
                const f4 u = tape[row];
                const f4 un = tape[row + T];
                const float mn = tapem[row + T];
                reverse_step<NCOMP, TIME, LEVELS, KZ>(p, a, s, u.x, u.y, u.z, u.w, un.x, un.y,
                                                      un.z, mn, xb, yb, zb, mb, swb, vdb);
            }
        }
        if (kmax >= kb) {
            acc[0] += (double)zb;  // released at z = h
            acc[1] += (double)J * (double)a.inv_q;
            acc[2] += (double)swb;
            acc[3] += (double)vdb;
            acc[4] += (double)J;
        }
    }
    // block reduction, one atomic per component
    constexpr int kWaves = kBlock / 64;
    __shared__ double part[kWaves][5];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        double v = acc[q];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) part[wv][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) v += part[w][threadIdx.x];
        if (v != 0.0) atomicAdd(a.grad + threadIdx.x, v);
    }
}

__global__ __launch_bounds__(kBlock) void clear_f64(double* p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0.0;
}

}  // namespace lpm

// ===========================================================================
// Host side
// ===========================================================================
namespace {

using namespace lpm_host;

constexpr int kAdjBlocksPerCu = 4;  // upper bound of the adjoint grid per CU

int check_receptors(const lpm_receptors* r)
{
    if (!r || !r->x || !r->y || !r->z) return fail(LPM_EINVAL, "null receptors");
    if (r->n < 1 || r->n > LPM_MAX_RECEPTORS) return fail(LPM_EINVAL, "receptor count must be 1..%d", LPM_MAX_RECEPTORS);
    if (!(r->sigma_h > 0.0f && r->sigma_z > 0.0f)) return fail(LPM_EINVAL, "kernel widths must be positive");
    if (!(r->weight >= 0.0f)) return fail(LPM_EINVAL, "weight must be >= 0");
    if (!aligned4(r->x) || !aligned4(r->y) || !aligned4(r->z)) return fail(LPM_EINVAL, "misaligned receptors");
    return LPM_OK;
}

lpm::KernelConst kernel_const(const lpm_receptors* r)
{
    const double pi = 3.14159265358979323846, l2e = 1.4426950408889634;
    const double sh = r->sigma_h, sz = r->sigma_z;
    lpm::KernelConst k;
    k.inv_sh2 = (float)(1.0 / (sh * sh));
    k.inv_sz2 = (float)(1.0 / (sz * sz));
    k.eh = (float)(l2e / (2.0 * sh * sh));
    k.ez = (float)(l2e / (2.0 * sz * sz));
    k.ch = (float)(1.0 / (2.0 * pi * sh * sh));
    k.cz = (float)(1.0 / (sqrt(2.0 * pi) * sz));
    return k;
}

// Total activity per unit a0 = sum_j bsum[j] exp(-lambda_j t): the column
// sums of the chain coefficients (ones for independent nuclides).
void coefficient_sums(const lpm_physics* ph, float bsum[4])
{
    double bc[4][4];
    activity_coefficients(ph, bc);
    for (int j = 0; j < 4; ++j) {
        double s = 0.0;
        for (int n = 0; n < ph->n_nuc; ++n) s += bc[n][j];
        bsum[j] = (float)s;
    }
}

int check_schedule(const lpm_schedule* sch)
{
    if (!sch) return fail(LPM_EINVAL, "null schedule");
    if (sch->n_total <= 0 || sch->n_total > 0xFFFFFFFFll || sch->s_release <= 0 ||
        sch->n_local < 0 || sch->id_base < 0 || sch->id_stride <= 0)
        return fail(LPM_EINVAL, "bad schedule");
    if (sch->n_local > 0 && sch->id_base + (sch->n_local - 1) * sch->id_stride >= sch->n_total)
        return fail(LPM_EINVAL, "local ids exceed n_total");
    return LPM_OK;
}

unsigned adjoint_capacity_blocks(long long n_local)
{
    const long long cap = (long long)kAdjBlocksPerCu * device_cus();
    const long long want = blocks_for(n_local);
    return (unsigned)(want < cap ? want : cap);
}

template <int NCOMP, bool TIME, bool LEV, int KZ>
void launch_adjoint(unsigned nb_cap, hipStream_t s, const lpm::StepConst& p, const lpm::AdjConst& a)
{
    auto k = lpm::adjoint_kernel<NCOMP, TIME, LEV, KZ>;
    const unsigned nb = resident_blocks(reinterpret_cast<const void*>(k), lpm::kBlock, 0, nb_cap);
    lpm::AdjConst aa = a;
    hipLaunchKernelGGL(k, dim3(nb), dim3(lpm::kBlock), 0, s, p, aa);
}

template <int NCOMP, bool TIME, bool LEV>
void launch_adjoint_kz(int kz, unsigned nb, hipStream_t s, const lpm::StepConst& p, const lpm::AdjConst& a)
{
    if (kz == 0) launch_adjoint<NCOMP, TIME, LEV, 0>(nb, s, p, a);
    else if (kz == 1) launch_adjoint<NCOMP, TIME, LEV, 1>(nb, s, p, a);
    else launch_adjoint<NCOMP, TIME, LEV, 2>(nb, s, p, a);
}

template <int NCOMP, bool TIME>
void launch_adjoint_lev(bool lev, int kz, unsigned nb, hipStream_t s, const lpm::StepConst& p,
                        const lpm::AdjConst& a)
{
    if (lev) launch_adjoint_kz<NCOMP, TIME, true>(kz, nb, s, p, a);
    else launch_adjoint_kz<NCOMP, TIME, false>(kz, nb, s, p, a);
}

}  // namespace

extern "C" {

int lpm_receptor_concentration(const float* rec, int64_t rec_stride, int32_t rec_step0,
                               int32_t rec_every, int32_t n_rec, const lpm_source* src,
                               const lpm_schedule* sch, const lpm_physics* ph,
                               const lpm_receptors* rcp, double* c_out, lpm_stream stream)
{
    g_msg[0] = 0;
    int rc;
    if (!src) return fail(LPM_EINVAL, "null source");
    if ((rc = check_schedule(sch)) || (rc = check_physics(ph)) || (rc = check_receptors(rcp)))
        return rc;
    if (!c_out || ((uintptr_t)c_out & 7u)) return fail(LPM_EINVAL, "null or misaligned c_out");
    if (n_rec < 0 || rec_every < 1 || rec_step0 < 0) return fail(LPM_EINVAL, "bad record steps");
    if (n_rec > 65535) return fail(LPM_EINVAL, "at most 65535 records per call");
    if ((long long)rec_step0 + (long long)(n_rec > 0 ? n_rec - 1 : 0) * rec_every > 0x7FFFFFFFll)
        return fail(LPM_EINVAL, "record steps overflow");
    if (n_rec > 0) {
        if (!rec || ((uintptr_t)rec & 15u)) return fail(LPM_EINVAL, "null or misaligned record buffer");
        if (rec_stride < sch->n_local) return fail(LPM_EINVAL, "rec_stride below n_local");
    }
    hipStream_t s = (hipStream_t)stream;
    for (int r0 = 0; r0 < rcp->n; r0 += lpm::kBlock) {
        const int n = rcp->n - r0 < lpm::kBlock ? rcp->n - r0 : lpm::kBlock;
        hipLaunchKernelGGL(lpm::clear_f64, dim3(1), dim3(lpm::kBlock), 0, s, c_out + r0, n);
    }
    lpm::RecConst g;
    memset(&g, 0, sizeof g);
    g.n_total = sch->n_total; g.id_base = sch->id_base; g.id_stride = sch->id_stride;
    g.s_release = sch->s_release;
    g.nnuc = ph->n_nuc;
    g.n_rcp = rcp->n;
    g.rec_step0 = rec_step0;
    g.rec_every = rec_every;
    g.a0 = (float)a0_of(src, sch, ph);
    g.dt = (float)ph->dt;
    g.weight = rcp->weight;
    for (int n = 0; n < ph->n_nuc; ++n) g.lam_l2e[n] = (float)(ph->lambda[n] * 1.4426950408889634);
    g.kc = kernel_const(rcp);
    g.rx = rcp->x; g.ry = rcp->y; g.rz = rcp->z;
    coefficient_sums(ph, g.bsum);
    if (n_rec > 0)
        g.i_hi = first_local_born_at_or_after(sch, (long long)rec_step0 + (long long)(n_rec - 1) * rec_every + 1);
    if (g.i_hi > 0) {
        const float4* r4 = reinterpret_cast<const float4*>(rec);
        const int* last = reinterpret_cast<const int*>(rec + 4ll * n_rec * rec_stride);
        hipLaunchKernelGGL(lpm::receptor_kernel, dim3(blocks_for(g.i_hi), (unsigned)n_rec),
                           dim3(lpm::kBlock), 0, s, g, r4, last, (long long)rec_stride, c_out);
    }
    return hip_status("lpm_receptor_concentration");
}

int lpm_adjoint_workspace(const lpm_field* fld, const lpm_schedule* sch, int32_t rec_every,
                          int64_t* bytes)
{
    g_msg[0] = 0;
    int rc;
    if (!fld || !bytes) return fail(LPM_EINVAL, "null argument");
    if ((rc = check_schedule(sch))) return rc;
    if (rec_every < 1) return fail(LPM_EINVAL, "rec_every must be >= 1");
    const long long T = (long long)adjoint_capacity_blocks(sch->n_local) * lpm::kBlock;
    *bytes = (int64_t)((long long)(rec_every + 1) * T * (long long)(sizeof(float4) + sizeof(float)));
    return LPM_OK;
}

int lpm_receptor_adjoint(const float* rec, int64_t rec_stride, int32_t rec_every, int32_t n_rec,
                         const lpm_source* src, const lpm_schedule* sch, const lpm_field* fld,
                         const lpm_physics* ph, const lpm_receptors* rcp, const double* gbar,
                         double* grad_out, void* work, int64_t work_bytes, lpm_stream stream)
{
    g_msg[0] = 0;
    int rc;
    if (!src) return fail(LPM_EINVAL, "null source");
    if ((rc = check_schedule(sch)) || (rc = check_physics(ph)) || (rc = check_receptors(rcp)))
        return rc;
    if (!gbar || ((uintptr_t)gbar & 7u) || !grad_out || ((uintptr_t)grad_out & 7u))
        return fail(LPM_EINVAL, "null or misaligned gbar or grad_out");
    if (rec_every < 1 || n_rec < 1) return fail(LPM_EINVAL, "need n_rec >= 1 and rec_every >= 1");
    if ((long long)n_rec * rec_every > 0x7FFFFFFFll) return fail(LPM_EINVAL, "run too long");
    if (!rec || ((uintptr_t)rec & 15u)) return fail(LPM_EINVAL, "null or misaligned record buffer");
    if (rec_stride < sch->n_local) return fail(LPM_EINVAL, "rec_stride below n_local");
    if (src->q == 0.0) return fail(LPM_EINVAL, "release rate q must be non-zero");
    if (ph->kz_kind == 3 || ph->dep_mode != 0)
        return fail(LPM_EINVAL, "the adjoint covers kz_kind 0..2 and mass-depletion deposition");
    lpm::StepConst p;
    memset(&p, 0, sizeof p);
    if (fld && fld->layout != LPM_FIELD_NODES)
        return fail(LPM_EINVAL, "the adjoint takes fields in the node layout");
    if ((rc = fill_field(p, fld))) return rc;
    const unsigned nb_cap = adjoint_capacity_blocks(sch->n_local);
    const long long T = (long long)nb_cap * lpm::kBlock;
    const long long need = (long long)(rec_every + 1) * T * (long long)(sizeof(float4) + sizeof(float));
    if (need > 0 && (!work || ((uintptr_t)work & 15u)))
        return fail(LPM_EINVAL, "null or misaligned workspace");
    if (work_bytes < need) return fail(LPM_EINVAL, "workspace of %lld bytes below the %lld needed",
                                       (long long)work_bytes, need);
    p.n_total = sch->n_total; p.id_base = sch->id_base; p.id_stride = sch->id_stride;
    p.s_release = sch->s_release;
    fill_source(p, src, sch, ph);
    fill_physics(p, ph);

    lpm::AdjConst a;
    memset(&a, 0, sizeof a);
    a.rec = reinterpret_cast<const float4*>(rec);
    a.last = reinterpret_cast<const int*>(rec + 4ll * n_rec * rec_stride);
    a.rec_stride = rec_stride;
    a.n_local = sch->n_local;
    a.rec_every = rec_every;
    a.n_rec = n_rec;
    a.n_rcp = rcp->n;
    a.nnuc = ph->n_nuc;
    // the tape rows are laid out for the grid actually launched (<= T)
    a.tape = reinterpret_cast<float4*>(work);
    a.phi_c1 = ph->h_s > 0.0 ? (float)(2.0 / ph->h_s) : 0.0f;
    a.phi_c2 = ph->h_s > 0.0 ? (float)(2.0 / (ph->h_s * ph->h_s)) : 0.0f;
    a.inv_q = (float)(1.0 / src->q);
    a.weight = rcp->weight;
    a.kc = kernel_const(rcp);
    a.rx = rcp->x; a.ry = rcp->y; a.rz = rcp->z;
    coefficient_sums(ph, a.bsum);
    a.gbar = gbar;
    a.grad = grad_out;

    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(lpm::clear_f64, dim3(1), dim3(lpm::kBlock), 0, s, grad_out, 5);
    if (sch->n_local == 0) return hip_status("lpm_receptor_adjoint");
    // m rows follow the (x, y, z, xi2) rows of the full capacity
    a.tapem = reinterpret_cast<float*>(reinterpret_cast<float4*>(work) + (long long)(rec_every + 1) * T);
    const bool time = fld->nt > 1, lev = fld->z_levels != nullptr;
    const int kz = ph->kz_kind;
    if (fld->ncomp == 2) {
        if (time) launch_adjoint_lev<2, true>(lev, kz, nb_cap, s, p, a);
        else launch_adjoint_lev<2, false>(lev, kz, nb_cap, s, p, a);
    } else {
        if (time) launch_adjoint_lev<3, true>(lev, kz, nb_cap, s, p, a);
        else launch_adjoint_lev<3, false>(lev, kz, nb_cap, s, p, a);
    }
    return hip_status("lpm_receptor_adjoint");
}

}  // extern "C"

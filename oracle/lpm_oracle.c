/*
 * FP64 CPU oracle of the stochastic Lagrangian particle model of
 * Molnar Jr., Szakaly, Meszaros and Lagzi, "Air pollution modelling using a
 * graphics processing unit with CUDA" (arXiv:0912.3223).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP library is checked against.  It shares no code, header or table with
 * the HIP library; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  Nothing in the product path calls it.
 *
 * Every quantity is computed in double precision with the C library's
 * functions (no fast-math).  The time loop follows the paper's main loop
 * (Sec. 3.2 and Fig. 1): in every step, every particle samples the weather,
 * gets its diffusion coefficient, is moved by the wind and by turbulence and
 * is tested for deposition; every n-th step the activities are summed on a
 * rectangular grid.  Particles are independent (Sec. 1 end), so the particle
 * loop of a step may run on several threads; each thread sums into its own
 * deposition grid and ledger, added together at the end.
 *
 * Readings of points the paper leaves open (all listed in the design notes):
 *  - random numbers: Philox4x32-10 (Salmon et al., SC'11) replaces the
 *    Mersenne Twister of Sec. 2; counter (id, step, purpose, 0), key
 *    (seed low word, scenario).  Uniforms ((r >> 8) + 1) 2^-24 in (0, 1],
 *    normals by the basic trigonometric Box-Muller form.
 *  - Eq. (2) is used with the Ito drift dK_z/dz dt and K_z evaluated at the
 *    midpoint z + K_z' dt / 2 (Visser 1997) so that a height-dependent K_z
 *    keeps a well-mixed tracer well mixed; with constant K it is Eq. (2).
 *  - Eq. (3) with Phi = 1 (neutral): exponent 1 ("parabolic") or 2.
 *  - dry deposition (Sec. 2, details not given): mass depletion at rate
 *    v_d phi(z), phi(z) = (2/h_s)(1 - z/h_s) on [0, h_s];
 *    wet deposition: rate Lambda0 inside an elliptical rain region with a
 *    linear edge; both applied at the post-move position.
 *  - decay (Sec. 2, Sec. 3.2): deterministic, activity a0 m exp(-lambda age);
 *    the per-step loss is split between decay and deposition by their rates.
 *  - ground reflection and a lid: z folded into [0, H_lid].
 *  - horizontal exit at the edge of a bounded wind domain (Sec. 3.2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    /* release schedule (Sec. 3.2: emission profile known a priori) */
    int64_t n_total, n_local, id_base, id_stride;
    int32_t s_release, pad0;
    /* source */
    double xs, ys, h, q, wind_scale, v_d;
    uint32_t scenario, pad1;
    uint64_t seed;
    /* physics */
    double dt, Kh, Kz_const, kappa_ustar, z0, H_mix, H_lid, h_s;
    int32_t kz_kind, n_nuc;
    double lambda[4];
    double Lambda0, rain_cx, rain_cy, rain_a, rain_b, rain_angle, rain_edge;
    /* wind field, float [nt][nz][ny][nx][ncomp], cell-centred nodes */
    const float* f;
    const float* z_levels; /* NULL: node heights (k + 1/2) fdz */
    int32_t nx, ny, nz, nt, ncomp, bounded;
    double fx0, fy0, fdx, fdy, fdz, ft0, fdt;
    /* concentration grid */
    int32_t cnx, cny, cnz, cmode, cdensity, pad2;
    double cx0, cy0, cz0, cdx, cdy, cdz;
    /* deposition grid */
    int32_t dnx, dny, dmode, ddensity;
    double dx0, dy0, ddx, ddy;
    /* variants: Eq. (3) stability (kz_kind 3), decay chain, stochastic
     * deposition */
    double inv_L;
    int32_t chain, dep_mode;
} orc_problem;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), random numbers of Eq. 2 */
/* ------------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                       uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Four uniforms in (0, 1] on the 2^-24 lattice for (id, step, purpose). */
void orc_uniforms(uint64_t seed, uint32_t scenario, uint32_t id, uint32_t step,
                  uint32_t purpose, double u[4])
{
    uint32_t ctr[4] = {id, step, purpose, 0u};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), scenario};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    for (int j = 0; j < 4; ++j)
        u[j] = ((double)(r[j] >> 8) + 1.0) * (1.0 / 16777216.0);
}

/* Standard normals for Eq. (2): basic Box-Muller (xi[3] is the spare). */
void orc_normals(uint64_t seed, uint32_t scenario, uint32_t id, uint32_t step,
                 uint32_t purpose, double xi[4])
{
    const double two_pi = 6.283185307179586476925286766559;
    double u[4];
    orc_uniforms(seed, scenario, id, step, purpose, u);
    double r0 = sqrt(-2.0 * log(u[0]));
    double r2 = sqrt(-2.0 * log(u[2]));
    xi[0] = r0 * cos(two_pi * u[1]);
    xi[1] = r0 * sin(two_pi * u[1]);
    xi[2] = r2 * cos(two_pi * u[3]);
    xi[3] = r2 * sin(two_pi * u[3]);
}

/* Normals of n consecutive ids starting at id0 for one step: out[n][4]. */
void orc_normals_batch(uint64_t seed, uint32_t scenario, uint32_t id0, int64_t n,
                       uint32_t step, uint32_t purpose, double* out)
{
    for (int64_t i = 0; i < n; ++i)
        orc_normals(seed, scenario, id0 + (uint32_t)i, step, purpose, out + 4 * i);
}

/* ------------------------------------------------------------------------ */
/* Weather sampling: linear in x, y, z and t (Sec. 3.2)                       */
/* ------------------------------------------------------------------------ */

/* Fractional node index of a coordinate on cell-centred nodes, clamped to the
 * node range; returns the lower node and the weight of the upper one. */
static void axis_weight(double pos, double origin, double spacing, int n,
                        int* i0, int* i1, double* w)
{
    double fi = (pos - origin) / spacing - 0.5;
    if (fi < 0.0) fi = 0.0;
    if (fi > (double)(n - 1)) fi = (double)(n - 1);
    int i = (int)floor(fi);
    if (i > n - 2) i = (n >= 2) ? n - 2 : 0;
    *i0 = i;
    *i1 = (i + 1 < n) ? i + 1 : i;
    *w = fi - (double)i;
}

/* Same for explicitly given (nonuniform) node heights. */
static void level_weight(double z, const float* lev, int n, int* k0, int* k1,
                         double* w)
{
    if (n == 1 || z <= (double)lev[0]) { *k0 = 0; *k1 = (n > 1); *w = 0.0; return; }
    if (z >= (double)lev[n - 1]) { *k0 = n - 2; *k1 = n - 1; *w = 1.0; return; }
    int k = 0;
    while (k + 1 < n - 1 && (double)lev[k + 1] <= z) ++k;
    *k0 = k;
    *k1 = k + 1;
    *w = (z - (double)lev[k]) / ((double)lev[k + 1] - (double)lev[k]);
}

static double node(const orc_problem* P, int t, int k, int j, int i, int c)
{
    size_t idx = ((((size_t)t * P->nz + k) * P->ny + j) * P->nx + i) * P->ncomp + c;
    return (double)P->f[idx];
}

/* Wind (u, v, w) at (x, y, z) and time t, before the wind-scale factor. */
void orc_wind(const orc_problem* P, double x, double y, double z, double t,
              double uvw[3])
{
    int i0, i1, j0, j1, k0, k1, t0, t1;
    double wx, wy, wz, wt;
    axis_weight(x, P->fx0, P->fdx, P->nx, &i0, &i1, &wx);
    axis_weight(y, P->fy0, P->fdy, P->ny, &j0, &j1, &wy);
    if (P->z_levels)
        level_weight(z, P->z_levels, P->nz, &k0, &k1, &wz);
    else
        axis_weight(z, 0.0, P->fdz, P->nz, &k0, &k1, &wz);
    double ft = (P->nt > 1) ? (t - P->ft0) / P->fdt : 0.0;
    if (ft < 0.0) ft = 0.0;
    if (ft > (double)(P->nt - 1)) ft = (double)(P->nt - 1);
    t0 = (int)floor(ft);
    if (t0 > P->nt - 2) t0 = (P->nt >= 2) ? P->nt - 2 : 0;
    t1 = (t0 + 1 < P->nt) ? t0 + 1 : t0;
    wt = ft - (double)t0;

    for (int c = 0; c < 3; ++c) {
        if (c >= P->ncomp) { uvw[c] = 0.0; continue; }
        double val[2];
        int tt[2] = {t0, t1};
        for (int a = 0; a < 2; ++a) {
            int T = tt[a];
            double s = 0.0;
            s += (1 - wz) * (1 - wy) * (1 - wx) * node(P, T, k0, j0, i0, c);
            s += (1 - wz) * (1 - wy) * wx * node(P, T, k0, j0, i1, c);
            s += (1 - wz) * wy * (1 - wx) * node(P, T, k0, j1, i0, c);
            s += (1 - wz) * wy * wx * node(P, T, k0, j1, i1, c);
            s += wz * (1 - wy) * (1 - wx) * node(P, T, k1, j0, i0, c);
            s += wz * (1 - wy) * wx * node(P, T, k1, j0, i1, c);
            s += wz * wy * (1 - wx) * node(P, T, k1, j1, i0, c);
            s += wz * wy * wx * node(P, T, k1, j1, i1, c);
            val[a] = s;
        }
        uvw[c] = (1 - wt) * val[0] + wt * val[1];
    }
}

/* ------------------------------------------------------------------------ */
/* Vertical diffusivity, Eq. (3) in the neutral limit Phi = 1                 */
/* ------------------------------------------------------------------------ */

/* Similarity function for heat Phi_h(s), s = z/L, and its derivative in s
 * (Businger-Dyer: 1 + 5 s stable, (1 - 16 s)^(-1/2) unstable). */
static void phi_heat(double s, double* phi, double* dphi)
{
    if (s >= 0.0) {
        *phi = 1.0 + 5.0 * s;
        *dphi = 5.0;
    } else {
        double w = 1.0 - 16.0 * s;
        *phi = 1.0 / sqrt(w);
        *dphi = 8.0 / (w * sqrt(w));
    }
}

void orc_kz(const orc_problem* P, double z, double* K, double* dK)
{
    if (P->kz_kind == 0) { *K = P->Kz_const; *dK = 0.0; return; }
    double H = P->H_mix, ku = P->kappa_ustar;
    if (z < 0.0) z = 0.0;
    /* zero above the mixed layer; at z = H the profile itself (K = 0, its
     * slope from below), so that the drift takes a particle at the top down */
    if (z > H) { *K = 0.0; *dK = 0.0; return; }
    double g = 1.0 - z / H;
    if (P->kz_kind == 1) {
        *K = ku * (z + P->z0) * g;
        *dK = ku * (g - (z + P->z0) / H);
    } else if (P->kz_kind == 2) {
        *K = ku * (z + P->z0) * g * g;
        *dK = ku * (g * g - 2.0 * (z + P->z0) * g / H);
    } else {
        /* Eq. (3): k u* z / Phi(z/L) (1 - z/H)^2, with z + z0 for z */
        double zz = z + P->z0, phi, dphi;
        phi_heat(zz * P->inv_L, &phi, &dphi);
        double f = ku * zz * g * g;
        double df = ku * (g * g - 2.0 * zz * g / H);
        *K = f / phi;
        *dK = df / phi - f * dphi * P->inv_L / (phi * phi);
    }
}

/* ------------------------------------------------------------------------ */
/* Deposition rates (Sec. 2: dry below the mixing height, wet with rain)     */
/* ------------------------------------------------------------------------ */

double orc_dry_rate(const orc_problem* P, double z)
{
    if (P->v_d == 0.0 || z < 0.0 || z >= P->h_s) return 0.0;
    return P->v_d * (2.0 / P->h_s) * (1.0 - z / P->h_s);
}

double orc_wet_rate(const orc_problem* P, double x, double y)
{
    if (P->Lambda0 == 0.0) return 0.0;
    double dx = x - P->rain_cx, dy = y - P->rain_cy;
    double ca = cos(P->rain_angle), sa = sin(P->rain_angle);
    double xr = ca * dx + sa * dy;
    double yr = -sa * dx + ca * dy;
    double re = sqrt((xr / P->rain_a) * (xr / P->rain_a) + (yr / P->rain_b) * (yr / P->rain_b));
    double f = (1.0 - re) / P->rain_edge + 0.5;
    if (f < 0.0) f = 0.0;
    if (f > 1.0) f = 1.0;
    return P->Lambda0 * f;
}

/* ------------------------------------------------------------------------ */
/* Gridding (Sec. 3.2: activities summed on a rectangular grid)              */
/* ------------------------------------------------------------------------ */

/* Add value a at (x, y, z) to grid g[nz][ny][nx]; mode 0 = cell containing
 * the point (half-open cells), 1 = trilinear cloud-in-cell about cell centres
 * with out-of-grid weights dropped.  nz == 1 with dz <= 0 means a 2-D grid. */
static void bin3(double* g, int nx, int ny, int nz, double x0, double y0,
                 double z0, double dx, double dy, double dz, int mode,
                 double x, double y, double z, double a, int two_d)
{
    if (mode == 0) {
        double fx = floor((x - x0) / dx), fy = floor((y - y0) / dy);
        double fz = two_d ? 0.0 : floor((z - z0) / dz);
        if (fx < 0 || fy < 0 || fz < 0 || fx >= nx || fy >= ny || fz >= nz) return;
        g[((size_t)fz * ny + (size_t)fy) * nx + (size_t)fx] += a;
        return;
    }
    double fx = (x - x0) / dx - 0.5, fy = (y - y0) / dy - 0.5;
    double fz = two_d ? 0.0 : (z - z0) / dz - 0.5;
    double ix = floor(fx), iy = floor(fy), iz = floor(fz);
    double wx = fx - ix, wy = fy - iy, wz = fz - iz;
    int nzc = two_d ? 1 : 2;
    for (int c = 0; c < nzc; ++c) {
        double kz = iz + c;
        double vz = two_d ? 1.0 : (c ? wz : 1.0 - wz);
        if (kz < 0 || kz >= nz) continue;
        for (int b = 0; b < 2; ++b) {
            double ky = iy + b;
            double vy = b ? wy : 1.0 - wy;
            if (ky < 0 || ky >= ny) continue;
            for (int a2 = 0; a2 < 2; ++a2) {
                double kx = ix + a2;
                double vx = a2 ? wx : 1.0 - wx;
                if (kx < 0 || kx >= nx) continue;
                g[((size_t)kz * ny + (size_t)ky) * nx + (size_t)kx] += a * vx * vy * vz;
            }
        }
    }
}

static int64_t birth_of(const orc_problem* P, int64_t gid)
{
    return (gid * (int64_t)P->s_release) / P->n_total;
}

static double a0_of(const orc_problem* P)
{
    return P->q * (double)P->s_release * P->dt / (double)P->n_total;
}

/* Activity bookkeeping per nuclide.  With independent nuclides nuclide n
 * keeps a0 exp(-lambda_n t).  In a decay chain 0 -> 1 -> ... released as
 * pure parent (activity a0), the Bateman solution gives nuclide n the
 * activity a0 sum_j c_nj exp(-lambda_j t) with the textbook coefficients
 *   c_nj = (lambda_n / lambda_0) prod_{p<n} lambda_p / prod_{p<=n, p!=j} (lambda_p - lambda_j)
 * (j <= n; distinct lambdas). */
static double act_coef(const orc_problem* P, int n, int j)
{
    if (!P->chain) return n == j ? 1.0 : 0.0;
    if (j > n) return 0.0;
    double num = P->lambda[n] / P->lambda[0];
    for (int p = 0; p < n; ++p) num *= P->lambda[p];
    double den = 1.0;
    for (int p = 0; p <= n; ++p)
        if (p != j) den *= P->lambda[p] - P->lambda[j];
    return num / den;
}

/* Activity of nuclide n at age t per unit released activity. */
double orc_activity_fraction(const orc_problem* P, int n, double t)
{
    double a = 0.0;
    for (int j = 0; j < P->n_nuc; ++j) {
        double c = act_coef(P, n, j);
        if (c != 0.0) a += c * exp(-P->lambda[j] * t);
    }
    return a;
}

/* Time integral over one step, starting at age t, of the activity fraction
 * of nuclide n times exp(-k tau) (tau the time into the step): the
 * activity-seconds exposed to a removal rate k. */
static double step_integral(const orc_problem* P, int n, double t, double k)
{
    double a = 0.0;
    for (int j = 0; j < P->n_nuc; ++j) {
        double c = act_coef(P, n, j);
        if (c == 0.0) continue;
        double r = P->lambda[j] + k;
        double g = r > 0.0 ? -expm1(-r * P->dt) / r : P->dt;
        a += c * exp(-P->lambda[j] * t) * g;
    }
    return a;
}

/* Concentration after step s (time (s + 1) dt) of the given particles:
 * A_n = a0 m exp(-lambda_n age), summed per nuclide on the concentration
 * grid; out[n_nuc][cnz][cny][cnx] is added to. */
void orc_grid_concentration(const orc_problem* P, int32_t s, const double* x,
                            const double* y, const double* z, const double* m,
                            double* out)
{
    size_t cells = (size_t)P->cnx * P->cny * P->cnz;
    double vol = P->cdensity ? P->cdx * P->cdy * P->cdz : 1.0;
    double a0 = a0_of(P);
    for (int64_t i = 0; i < P->n_local; ++i) {
        int64_t gid = P->id_base + i * P->id_stride;
        int64_t b = birth_of(P, gid);
        if (b > s || !(m[i] > 0.0)) continue;
        double age = (double)(s + 1 - b) * P->dt;
        for (int n = 0; n < P->n_nuc; ++n) {
            double A = a0 * m[i] * orc_activity_fraction(P, n, age);
            bin3(out + n * cells, P->cnx, P->cny, P->cnz, P->cx0, P->cy0, P->cz0,
                 P->cdx, P->cdy, P->cdz, P->cmode, x[i], y[i], z[i], A / vol, 0);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* One time step of one particle (Sec. 3.2 main loop, Eqs. 1-3)              */
/* ------------------------------------------------------------------------ */

static double fold(double z, double H)
{
    for (int it = 0; it < 64; ++it) {
        if (z < 0.0) z = -z;
        else if (H > 0.0 && z > H) z = 2.0 * H - z;
        else break;
    }
    return z;
}

/* Advance particle i (global id gid, birth b) over step s.  led[n*4 + 1..3]
 * receive deposited, decayed and exited activity; dep receives the deposited
 * activity on the deposition grid. */
static void step_particle(const orc_problem* P, int64_t gid, int64_t b, int32_t s,
                          double* px, double* py, double* pz, double* pm,
                          double* led, double* dep)
{
    const double dt = P->dt;
    double x = *px, y = *py, z = *pz, m = *pm;
    double age = (double)(s - b) * dt;
    double a0 = a0_of(P);

    /* random numbers for Eq. (2) */
    double xi[4];
    orc_normals(P->seed, P->scenario, (uint32_t)gid, (uint32_t)s, 0u, xi);

    /* weather sample at the start-of-step position and time (Eq. 1) */
    double uvw[3];
    orc_wind(P, x, y, z, (double)s * dt, uvw);
    double u = P->wind_scale * uvw[0];
    double v = P->wind_scale * uvw[1];
    double w = P->wind_scale * uvw[2];

    /* diffusion coefficients (Eq. 2, Eq. 3) */
    double Kz, dKz, Kzm, dKzm;
    orc_kz(P, z, &Kz, &dKz);
    double zm = z + 0.5 * dKz * dt;
    if (zm < 0.0) zm = 0.0;
    if (zm > P->H_mix) zm = P->H_mix;
    orc_kz(P, zm, &Kzm, &dKzm);

    /* move: advection + turbulent displacement (Eq. 1, Eq. 2) */
    double xn = x + u * dt + xi[0] * sqrt(2.0 * P->Kh * dt);
    double yn = y + v * dt + xi[1] * sqrt(2.0 * P->Kh * dt);
    double zn = z + w * dt + dKz * dt + xi[2] * sqrt(2.0 * Kzm * dt);
    zn = fold(zn, P->H_lid);

    /* decay and deposition at the new position.  Over the step, nuclide n
     * spends S_n activity-seconds in the air (its activity times the
     * surviving mass, integrated); k S_n is deposited, lambda_n S_n decays,
     * and in a chain lambda_{n+1} S_n grows into the daughter. */
    double k = orc_dry_rate(P, zn) + orc_wet_rate(P, xn, yn);
    size_t cells = (size_t)P->dnx * P->dny;
    double area = P->ddensity ? P->ddx * P->ddy : 1.0;
    double mn = m;
    int removed = 0;
    /* mass depletion: the rate acts on the mass; stochastic deposition: the
     * particle stays whole in the air for the step, then is removed with
     * probability 1 - exp(-k dt) (Sec. 2) */
    double kk = P->dep_mode == 0 ? k : 0.0;
    if (P->dep_mode == 0) {
        mn = m * exp(-k * dt);
    } else if (k > 0.0) {
        double u[4];
        orc_uniforms(P->seed, P->scenario, (uint32_t)gid, (uint32_t)s, 1u, u);
        removed = u[0] <= -expm1(-k * dt);
    }
    for (int n = 0; n < P->n_nuc; ++n) {
        double S = a0 * m * step_integral(P, n, age, kk);
        double d = kk * S;
        if (removed) d += a0 * m * orc_activity_fraction(P, n, age + dt);
        led[n * 4 + 1] += d;
        led[n * 4 + 2] += P->lambda[n] * S;
        if (P->chain && n + 1 < P->n_nuc) led[(n + 1) * 4 + 0] += P->lambda[n + 1] * S;
        if (d != 0.0)
            bin3(dep + n * cells, P->dnx, P->dny, 1, P->dx0, P->dy0, 0.0, P->ddx,
                 P->ddy, 1.0, P->dmode, xn, yn, 0.0, d / area, 1);
    }
    if (removed) mn = 0.0;

    /* leaving the simulated area inactivates the particle (Sec. 3.2) */
    if (P->bounded && !removed) {
        double X1 = P->fx0 + P->nx * P->fdx, Y1 = P->fy0 + P->ny * P->fdy;
        if (xn < P->fx0 || xn >= X1 || yn < P->fy0 || yn >= Y1) {
            for (int n = 0; n < P->n_nuc; ++n)
                led[n * 4 + 3] += a0 * mn * orc_activity_fraction(P, n, age + dt);
            mn = 0.0;
        }
    }
    *px = xn; *py = yn; *pz = zn; *pm = mn;
}

/* ------------------------------------------------------------------------ */
/* Main loop                                                                 */
/* ------------------------------------------------------------------------ */

/* Run steps [s_begin, s_end).  In step s the particles born at s are released
 * at the source with m = 1, then every released particle with m > 0 is
 * advanced; after a step listed in snap_steps the concentration is gridded
 * into snaps[k].  x, y, z, m (length n_local) are updated in place; dep
 * ([n_nuc][dny][dnx]), ledger ([n_nuc][4] = released, deposited, decayed,
 * exited) and snaps ([n_snap][n_nuc][cnz][cny][cnx]) are added to;
 * *psteps (if not NULL) receives the number of particle-steps advanced.
 * Returns 0, or -1 for invalid arguments. */
int orc_simulate(const orc_problem* P, int32_t s_begin, int32_t s_end,
                 double* x, double* y, double* z, double* m, double* dep,
                 double* ledger, const int32_t* snap_steps, int32_t n_snap,
                 double* snaps, int32_t nthreads, int64_t* psteps)
{
    if (!P || P->n_nuc < 1 || P->n_nuc > 4 || P->n_total <= 0 || P->s_release <= 0 ||
        P->n_local < 0 || P->id_stride <= 0 || !x || !y || !z || !m || !dep || !ledger ||
        (n_snap > 0 && (!snaps || !snap_steps)) || !P->f || P->nx < 1 || P->ny < 1 ||
        P->nz < 1 || P->nt < 1 || (P->ncomp != 2 && P->ncomp != 3) || P->kz_kind < 0 ||
        P->kz_kind > 3 || (P->dep_mode != 0 && P->dep_mode != 1) || (P->chain != 0 && P->chain != 1))
        return -1;
    if (P->chain) {
        for (int n = 0; n < P->n_nuc; ++n) {
            if (!(P->lambda[n] > 0.0)) return -1;
            for (int j = 0; j < n; ++j)
                if (P->lambda[j] == P->lambda[n]) return -1;
        }
    }
    int nth = 1;
#ifdef _OPENMP
    nth = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    size_t dcells = (size_t)P->n_nuc * P->dnx * P->dny;
    size_t ccells = (size_t)P->n_nuc * P->cnx * P->cny * P->cnz;
    double* dep_t = (double*)calloc((size_t)nth * dcells, sizeof(double));
    double* led_t = (double*)calloc((size_t)nth * 16, sizeof(double));
    int64_t* cnt_t = (int64_t*)calloc((size_t)nth, sizeof(int64_t));
    if (!dep_t || !led_t || !cnt_t) { free(dep_t); free(led_t); free(cnt_t); return -1; }
    const double a0 = a0_of(P);

#pragma omp parallel num_threads(nth)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* my_dep = dep_t + (size_t)tid * dcells;
        double* my_led = led_t + (size_t)tid * 16;
        for (int32_t s = s_begin; s < s_end; ++s) {
#pragma omp for schedule(static, 256)
            for (int64_t i = 0; i < P->n_local; ++i) {
                int64_t gid = P->id_base + i * P->id_stride;
                int64_t b = birth_of(P, gid);
                if (b == s) {
                    x[i] = P->xs; y[i] = P->ys; z[i] = P->h; m[i] = 1.0;
                    for (int n = 0; n < (P->chain ? 1 : P->n_nuc); ++n) my_led[n * 4 + 0] += a0;
                }
                if (b <= s && m[i] > 0.0) {
                    step_particle(P, gid, b, s, &x[i], &y[i], &z[i], &m[i], my_led, my_dep);
                    cnt_t[tid] += 1;
                }
            }
            for (int32_t k = 0; k < n_snap; ++k) {
                if (snap_steps[k] != s) continue;
#pragma omp single
                orc_grid_concentration(P, s, x, y, z, m, snaps + (size_t)k * ccells);
            }
        }
    }
    int64_t count = 0;
    for (int t = 0; t < nth; ++t) {
        for (size_t c = 0; c < dcells; ++c) dep[c] += dep_t[(size_t)t * dcells + c];
        for (int c = 0; c < 4 * P->n_nuc; ++c) ledger[c] += led_t[(size_t)t * 16 + c];
        count += cnt_t[t];
    }
    if (psteps) *psteps = count;
    free(dep_t);
    free(led_t);
    free(cnt_t);
    return 0;
}

/* Activity still airborne after step s: sum of a0 m exp(-lambda age). */
void orc_airborne(const orc_problem* P, int32_t s, const double* m, double* out)
{
    double a0 = a0_of(P);
    for (int n = 0; n < P->n_nuc; ++n) out[n] = 0.0;
    for (int64_t i = 0; i < P->n_local; ++i) {
        int64_t gid = P->id_base + i * P->id_stride;
        int64_t b = birth_of(P, gid);
        if (b > s || !(m[i] > 0.0)) continue;
        for (int n = 0; n < P->n_nuc; ++n)
            out[n] += a0 * m[i] * orc_activity_fraction(P, n, (double)(s + 1 - b) * P->dt);
    }
}

/* ======================================================================== */
/* Receptor concentrations of a source and their gradient with respect to    */
/* the source parameters theta = (h, q, s_w, v_d)                            */
/* ======================================================================== */
/*
 * Ground-level concentrations at receptor points are the activities of the
 * airborne particles spread with a Gaussian kernel (horizontal width
 * sigma_h, vertical width sigma_z with its mirror image below the ground)
 * and summed over the output steps s = out_every - 1, 2 out_every - 1, ...:
 *
 *   c_r = weight * sum_s sum_p A_p(s) G_h(x_p - X_r, y_p - Y_r)
 *                               [N(z_p - Z_r) + N(z_p + Z_r)],
 *   A_p(s) = a0 m_p sum_n exp(-lambda_n (s + 1 - b_p) dt)   (all nuclides),
 *
 * with the state taken after step s (the gridding time of Sec. 3.2).  The
 * derivatives follow each particle's path with its random numbers held
 * fixed (common random numbers): the path is a piecewise smooth function of
 * theta, and the derivative is that of the smooth piece.  The exit step of a
 * particle that leaves the domain is treated as fixed (its activity after
 * the exit is zero whatever theta is).
 *
 * Three evaluations are provided:
 *   orc_receptor_forward   c_r, and optionally dc_r/dtheta by propagating
 *                          four tangents along each path (forward mode);
 *   orc_receptor_adjoint   sum_r gbar_r dc_r/dtheta by a reverse sweep over
 *                          each particle's stored path (reverse mode).
 * Both use the step Jacobian below; central finite differences of the plain
 * forward (the tests) pin that Jacobian independently.
 */

typedef struct {
    int32_t n, pad;
    const double* x;
    const double* y;
    const double* z;
    double sigma_h, sigma_z;
    double weight;  /* time weight of one output step (s) */
} orc_receptors;

/* Interpolated wind (before the wind-scale factor) and its gradient
 * g[c][d] = d uvw[c] / d (x, y, z)[d]; a clamped coordinate has zero slope. */
static void wind_gradient(const orc_problem* P, double x, double y, double z, double t,
                          double uvw[3], double g[3][3])
{
    int i0, i1, j0, j1, k0, k1, t0, t1;
    double wx, wy, wz, wt;
    axis_weight(x, P->fx0, P->fdx, P->nx, &i0, &i1, &wx);
    axis_weight(y, P->fy0, P->fdy, P->ny, &j0, &j1, &wy);
    double fx = (x - P->fx0) / P->fdx - 0.5, fy = (y - P->fy0) / P->fdy - 0.5;
    double sx = (fx > 0.0 && fx < (double)(P->nx - 1)) ? 1.0 / P->fdx : 0.0;
    double sy = (fy > 0.0 && fy < (double)(P->ny - 1)) ? 1.0 / P->fdy : 0.0;
    double sz;
    if (P->z_levels) {
        level_weight(z, P->z_levels, P->nz, &k0, &k1, &wz);
        int inside = P->nz > 1 && z > (double)P->z_levels[0] &&
                     z < (double)P->z_levels[P->nz - 1];
        sz = inside ? 1.0 / ((double)P->z_levels[k1] - (double)P->z_levels[k0]) : 0.0;
    } else {
        axis_weight(z, 0.0, P->fdz, P->nz, &k0, &k1, &wz);
        double fz = z / P->fdz - 0.5;
        sz = (fz > 0.0 && fz < (double)(P->nz - 1)) ? 1.0 / P->fdz : 0.0;
    }
    double ft = (P->nt > 1) ? (t - P->ft0) / P->fdt : 0.0;
    if (ft < 0.0) ft = 0.0;
    if (ft > (double)(P->nt - 1)) ft = (double)(P->nt - 1);
    t0 = (int)floor(ft);
    if (t0 > P->nt - 2) t0 = (P->nt >= 2) ? P->nt - 2 : 0;
    t1 = (t0 + 1 < P->nt) ? t0 + 1 : t0;
    wt = ft - (double)t0;

    for (int c = 0; c < 3; ++c) {
        uvw[c] = 0.0;
        g[c][0] = g[c][1] = g[c][2] = 0.0;
        if (c >= P->ncomp) continue;
        int tt[2] = {t0, t1};
        double tw[2] = {1.0 - wt, wt};
        for (int a = 0; a < 2; ++a) {
            int T = tt[a];
            /* corner values v[kk][jj][ii] */
            double v[2][2][2];
            int ks[2] = {k0, k1}, js[2] = {j0, j1}, is[2] = {i0, i1};
            for (int kk = 0; kk < 2; ++kk)
                for (int jj = 0; jj < 2; ++jj)
                    for (int ii = 0; ii < 2; ++ii)
                        v[kk][jj][ii] = node(P, T, ks[kk], js[jj], is[ii], c);
            double val = 0.0, dx = 0.0, dy = 0.0, dz = 0.0;
            for (int kk = 0; kk < 2; ++kk)
                for (int jj = 0; jj < 2; ++jj)
                    for (int ii = 0; ii < 2; ++ii) {
                        double ax = ii ? wx : 1.0 - wx, ay = jj ? wy : 1.0 - wy;
                        double az = kk ? wz : 1.0 - wz;
                        double ex = ii ? 1.0 : -1.0, ey = jj ? 1.0 : -1.0, ez = kk ? 1.0 : -1.0;
                        val += az * ay * ax * v[kk][jj][ii];
                        dx += az * ay * ex * v[kk][jj][ii];
                        dy += az * ey * ax * v[kk][jj][ii];
                        dz += ez * ay * ax * v[kk][jj][ii];
                    }
            uvw[c] += tw[a] * val;
            g[c][0] += tw[a] * dx * sx;
            g[c][1] += tw[a] * dy * sy;
            g[c][2] += tw[a] * dz * sz;
        }
    }
}

/* Second derivative of K_z(z) (zero where K_z is constant or zero). */
static double kz_second(const orc_problem* P, double z)
{
    if (P->kz_kind == 0 || z < 0.0 || z > P->H_mix) return 0.0;
    double H = P->H_mix, ku = P->kappa_ustar, g = 1.0 - z / H;
    if (P->kz_kind == 1) return -2.0 * ku / H;
    return ku * (-4.0 * g / H + 2.0 * (z + P->z0) / (H * H));
}

/* Fold of z into [0, H] and its slope (+1 or -1). */
static double fold_sign(double z, double H, double* sign)
{
    double sg = 1.0;
    for (int it = 0; it < 64; ++it) {
        if (z < 0.0) { z = -z; sg = -sg; }
        else if (H > 0.0 && z > H) { z = 2.0 * H - z; sg = -sg; }
        else break;
    }
    *sign = sg;
    return z;
}

/* Wet-deposition rate and its gradient in (x, y). */
static double wet_rate_gradient(const orc_problem* P, double x, double y, double* gx, double* gy)
{
    *gx = *gy = 0.0;
    if (P->Lambda0 == 0.0) return 0.0;
    double dx = x - P->rain_cx, dy = y - P->rain_cy;
    double ca = cos(P->rain_angle), sa = sin(P->rain_angle);
    double xr = ca * dx + sa * dy;
    double yr = -sa * dx + ca * dy;
    double a = P->rain_a, b = P->rain_b;
    double re = sqrt((xr / a) * (xr / a) + (yr / b) * (yr / b));
    double f = (1.0 - re) / P->rain_edge + 0.5;
    if (f <= 0.0) return 0.0;
    if (f >= 1.0) return P->Lambda0;
    if (re > 0.0) {
        double dre_dxr = xr / (a * a * re), dre_dyr = yr / (b * b * re);
        double dre_dx = dre_dxr * ca - dre_dyr * sa;
        double dre_dy = dre_dxr * sa + dre_dyr * ca;
        *gx = -P->Lambda0 / P->rain_edge * dre_dx;
        *gy = -P->Lambda0 / P->rain_edge * dre_dy;
    }
    return P->Lambda0 * f;
}

/* One step of one particle with its Jacobian.  u = (x, y, z, m) before step
 * s; un receives the state after it (as step_particle computes it: same
 * formulas, same order).  J[i][j] = d un_i / d u_j; Jsw[i], Jvd[i] =
 * d un_i / d s_w, d un_i / d v_d.  Returns 1 if the particle left the domain
 * in this step (un m = 0, Jacobian zero), else 0. */
static int step_jacobian(const orc_problem* P, int64_t gid, int32_t s, const double u[4],
                         double un[4], double J[4][4], double Jsw[4], double Jvd[4])
{
    const double dt = P->dt;
    double x = u[0], y = u[1], z = u[2], m = u[3];
    memset(J, 0, sizeof(double) * 16);
    for (int i = 0; i < 4; ++i) Jsw[i] = Jvd[i] = 0.0;

    double xi[4];
    orc_normals(P->seed, P->scenario, (uint32_t)gid, (uint32_t)s, 0u, xi);
    double uvw[3], g[3][3];
    wind_gradient(P, x, y, z, (double)s * dt, uvw, g);
    const double sw = P->wind_scale;

    double Kz, dKz, Kzm, dKzm;
    orc_kz(P, z, &Kz, &dKz);
    double K2 = kz_second(P, z);
    double zm_raw = z + 0.5 * dKz * dt;
    double zm = zm_raw;
    if (zm < 0.0) zm = 0.0;
    if (zm > P->H_mix) zm = P->H_mix;
    double dzm_dz = (zm_raw > 0.0 && zm_raw < P->H_mix) ? 1.0 + 0.5 * dt * K2 : 0.0;
    orc_kz(P, zm, &Kzm, &dKzm);
    double sq = sqrt(2.0 * Kzm * dt);
    double dsq_dz = sq > 0.0 ? dt * dKzm * dzm_dz / sq : 0.0;

    double sh = sqrt(2.0 * P->Kh * dt);
    double xn = x + sw * uvw[0] * dt + xi[0] * sh;
    double yn = y + sw * uvw[1] * dt + xi[1] * sh;
    double zn0 = z + sw * uvw[2] * dt + dKz * dt + xi[2] * sq;
    double sg;
    double zn = fold_sign(zn0, P->H_lid, &sg);

    /* position rows (before the fold for z) */
    double Dx[3] = {1.0 + sw * dt * g[0][0], sw * dt * g[0][1], sw * dt * g[0][2]};
    double Dy[3] = {sw * dt * g[1][0], 1.0 + sw * dt * g[1][1], sw * dt * g[1][2]};
    double Dz[3] = {sw * dt * g[2][0], sw * dt * g[2][1],
                    1.0 + sw * dt * g[2][2] + K2 * dt + xi[2] * dsq_dz};
    double swx = uvw[0] * dt, swy = uvw[1] * dt, swz = uvw[2] * dt;

    /* deposition rate at the new position */
    double kd = orc_dry_rate(P, zn);
    double phi = (zn >= 0.0 && zn < P->h_s) ? (2.0 / P->h_s) * (1.0 - zn / P->h_s) : 0.0;
    double dkd_dz = (P->v_d != 0.0 && zn >= 0.0 && zn < P->h_s)
                        ? -P->v_d * 2.0 / (P->h_s * P->h_s) : 0.0;
    double gwx, gwy;
    double kw = wet_rate_gradient(P, xn, yn, &gwx, &gwy);
    double k = kd + kw;
    double e = exp(-k * dt);
    double mn = m * e;

    if (P->bounded) {
        double X1 = P->fx0 + P->nx * P->fdx, Y1 = P->fy0 + P->ny * P->fdy;
        if (xn < P->fx0 || xn >= X1 || yn < P->fy0 || yn >= Y1) {
            un[0] = xn; un[1] = yn; un[2] = zn; un[3] = 0.0;
            return 1;
        }
    }
    un[0] = xn; un[1] = yn; un[2] = zn; un[3] = mn;
    for (int j = 0; j < 3; ++j) {
        J[0][j] = Dx[j];
        J[1][j] = Dy[j];
        J[2][j] = sg * Dz[j];
    }
    Jsw[0] = swx;
    Jsw[1] = swy;
    Jsw[2] = sg * swz;
    /* m row: mn = m exp(-k dt), k = k(xn, yn, zn) */
    double dmn_dk = -dt * mn;
    for (int j = 0; j < 3; ++j)
        J[3][j] = dmn_dk * (gwx * J[0][j] + gwy * J[1][j] + dkd_dz * J[2][j]);
    J[3][3] = e;
    Jsw[3] = dmn_dk * (gwx * Jsw[0] + gwy * Jsw[1] + dkd_dz * Jsw[2]);
    Jvd[3] = dmn_dk * phi;
    return 0;
}

/* Receptor kernel value and its gradient in (x, y, z). */
static double receptor_kernel(const orc_receptors* R, int r, double x, double y, double z,
                              double gk[3])
{
    const double pi = 3.141592653589793238462643383279;
    double sh2 = R->sigma_h * R->sigma_h, sz2 = R->sigma_z * R->sigma_z;
    double dx = x - R->x[r], dy = y - R->y[r];
    double gh = exp(-(dx * dx + dy * dy) / (2.0 * sh2)) / (2.0 * pi * sh2);
    double d1 = z - R->z[r], d2 = z + R->z[r];
    double cz = 1.0 / (sqrt(2.0 * pi) * R->sigma_z);
    double n1 = cz * exp(-d1 * d1 / (2.0 * sz2)), n2 = cz * exp(-d2 * d2 / (2.0 * sz2));
    double kv = gh * (n1 + n2);
    gk[0] = -dx / sh2 * kv;
    gk[1] = -dy / sh2 * kv;
    gk[2] = gh * (-d1 / sz2 * n1 - d2 / sz2 * n2);
    return kv;
}

/* Total activity factor sum_n exp(-lambda_n age) after step s. */
static double decay_sum(const orc_problem* P, int64_t b, int32_t s)
{
    double age = (double)(s + 1 - b) * P->dt, f = 0.0;
    for (int n = 0; n < P->n_nuc; ++n) f += orc_activity_fraction(P, n, age);
    return f;
}

static int receptor_args_ok(const orc_problem* P, const orc_receptors* R, int32_t s_end,
                            int32_t out_every)
{
    return P && R && R->n >= 0 && (R->n == 0 || (R->x && R->y && R->z)) && R->sigma_h > 0.0 &&
           R->sigma_z > 0.0 && out_every >= 1 && s_end >= 0 && P->n_nuc >= 1 && P->n_nuc <= 4 &&
           P->n_total > 0 && P->s_release > 0 && P->n_local >= 0 && P->id_stride > 0 && P->f &&
           (P->ncomp == 2 || P->ncomp == 3) && P->q != 0.0 && P->dep_mode == 0 &&
           P->kz_kind >= 0 && P->kz_kind <= 2;
}

/* c[n_rec] (added to) receives the receptor concentrations of a run over
 * steps [0, s_end) with the particles released at their birth steps; if dc
 * is not NULL, dc[n_rec][4] (added to) receives dc_r / d(h, q, s_w, v_d) by
 * forward-mode propagation.  *psteps (if not NULL) receives the number of
 * particle-steps.  Returns 0, or -1 for invalid arguments. */
int orc_receptor_forward(const orc_problem* P, const orc_receptors* R, int32_t s_end,
                         int32_t out_every, double* c, double* dc, int32_t nthreads,
                         int64_t* psteps)
{
    if (!receptor_args_ok(P, R, s_end, out_every) || !c) return -1;
    int nth = 1;
#ifdef _OPENMP
    nth = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    const int nr = R->n;
    double* acc = (double*)calloc((size_t)nth * nr * 5, sizeof(double));
    int64_t* cnt = (int64_t*)calloc((size_t)nth, sizeof(int64_t));
    if (!acc || !cnt) { free(acc); free(cnt); return -1; }
    const double a0 = a0_of(P);

#pragma omp parallel num_threads(nth)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* my = acc + (size_t)tid * nr * 5;
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < P->n_local; ++i) {
            int64_t gid = P->id_base + i * P->id_stride;
            int64_t b = birth_of(P, gid);
            if (b >= s_end) continue;
            double u[4] = {P->xs, P->ys, P->h, 1.0};
            /* tangents T[j][0..3] of (x, y, z, m), j = h, q, s_w, v_d */
            double T[4][4] = {{0, 0, 1, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
            for (int32_t s = (int32_t)b; s < s_end; ++s) {
                double un[4], J[4][4], Jsw[4], Jvd[4];
                int gone = step_jacobian(P, gid, s, u, un, J, Jsw, Jvd);
                cnt[tid] += 1;
                if (gone) break;
                if (dc) {
                    double Tn[4][4];
                    for (int j = 0; j < 4; ++j)
                        for (int a = 0; a < 4; ++a) {
                            double v = 0.0;
                            for (int k = 0; k < 4; ++k) v += J[a][k] * T[j][k];
                            if (j == 2) v += Jsw[a];
                            if (j == 3) v += Jvd[a];
                            Tn[j][a] = v;
                        }
                    memcpy(T, Tn, sizeof(T));
                }
                memcpy(u, un, sizeof(u));
                if ((s + 1) % out_every != 0) continue;
                double A = a0 * u[3] * decay_sum(P, b, s);
                for (int r = 0; r < nr; ++r) {
                    double gk[3];
                    double kv = receptor_kernel(R, r, u[0], u[1], u[2], gk);
                    double cv = R->weight * A * kv;
                    my[r * 5] += cv;
                    if (!dc) continue;
                    for (int j = 0; j < 4; ++j) {
                        double d = R->weight * (a0 * T[j][3] * decay_sum(P, b, s) * kv +
                                                A * (gk[0] * T[j][0] + gk[1] * T[j][1] +
                                                     gk[2] * T[j][2]));
                        if (j == 1) d += cv / P->q;  /* a0 is proportional to q */
                        my[r * 5 + 1 + j] += d;
                    }
                }
            }
        }
    }
    int64_t total = 0;
    for (int t = 0; t < nth; ++t) {
        for (int r = 0; r < nr; ++r) {
            c[r] += acc[((size_t)t * nr + r) * 5];
            if (dc)
                for (int j = 0; j < 4; ++j) dc[r * 4 + j] += acc[((size_t)t * nr + r) * 5 + 1 + j];
        }
        total += cnt[t];
    }
    if (psteps) *psteps = total;
    free(acc);
    free(cnt);
    return 0;
}

/* grad[4] (added to) receives sum_r gbar_r dc_r / d(h, q, s_w, v_d) by a
 * reverse sweep over each particle's path (stored whole: this is the plain
 * form of the checkpointed GPU adjoint).  Returns 0, or -1. */
int orc_receptor_adjoint(const orc_problem* P, const orc_receptors* R, int32_t s_end,
                         int32_t out_every, const double* gbar, double* grad, int32_t nthreads)
{
    if (!receptor_args_ok(P, R, s_end, out_every) || !gbar || !grad) return -1;
    int nth = 1;
#ifdef _OPENMP
    nth = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    const int nr = R->n;
    double* acc = (double*)calloc((size_t)nth * 4, sizeof(double));
    double* paths = (double*)malloc((size_t)nth * ((size_t)s_end + 1) * 4 * sizeof(double));
    if (!acc || !paths) { free(acc); free(paths); return -1; }
    const double a0 = a0_of(P);

#pragma omp parallel num_threads(nth)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* my = acc + (size_t)tid * 4;
        double* path = paths + (size_t)tid * ((size_t)s_end + 1) * 4;
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < P->n_local; ++i) {
            int64_t gid = P->id_base + i * P->id_stride;
            int64_t b = birth_of(P, gid);
            if (b >= s_end) continue;
            /* forward: path[s - b] = state before step s; e = first step not
             * to differentiate (the exit step, or s_end) */
            double u[4] = {P->xs, P->ys, P->h, 1.0};
            int32_t e = s_end;
            for (int32_t s = (int32_t)b; s < s_end; ++s) {
                memcpy(path + (size_t)(s - b) * 4, u, sizeof(u));
                double un[4], J[4][4], Jsw[4], Jvd[4];
                if (step_jacobian(P, gid, s, u, un, J, Jsw, Jvd)) { e = s; break; }
                memcpy(u, un, sizeof(u));
            }
            if (e == s_end) memcpy(path + (size_t)(s_end - b) * 4, u, sizeof(u));
            /* reverse: ubar is the adjoint of the state after step s */
            double ub[4] = {0, 0, 0, 0};
            double sw_bar = 0.0, vd_bar = 0.0, q_bar = 0.0;
            for (int32_t s = e - 1; s >= (int32_t)b; --s) {
                if ((s + 1) % out_every == 0) {
                    const double* v = path + (size_t)(s + 1 - b) * 4;
                    double F = decay_sum(P, b, s), A = a0 * v[3] * F;
                    for (int r = 0; r < nr; ++r) {
                        double gk[3];
                        double kv = receptor_kernel(R, r, v[0], v[1], v[2], gk);
                        double w = gbar[r] * R->weight;
                        ub[0] += w * A * gk[0];
                        ub[1] += w * A * gk[1];
                        ub[2] += w * A * gk[2];
                        ub[3] += w * a0 * F * kv;
                        q_bar += w * A * kv / P->q;
                    }
                }
                double un[4], J[4][4], Jsw[4], Jvd[4];
                step_jacobian(P, gid, s, path + (size_t)(s - b) * 4, un, J, Jsw, Jvd);
                double nb[4];
                for (int k = 0; k < 4; ++k) {
                    nb[k] = 0.0;
                    for (int a = 0; a < 4; ++a) nb[k] += J[a][k] * ub[a];
                }
                for (int a = 0; a < 4; ++a) {
                    sw_bar += Jsw[a] * ub[a];
                    vd_bar += Jvd[a] * ub[a];
                }
                memcpy(ub, nb, sizeof(ub));
            }
            my[0] += ub[2];  /* released at z = h */
            my[1] += q_bar;
            my[2] += sw_bar;
            my[3] += vd_bar;
        }
    }
    for (int t = 0; t < nth; ++t)
        for (int j = 0; j < 4; ++j) grad[j] += acc[(size_t)t * 4 + j];
    free(acc);
    free(paths);
    return 0;
}


/* ======================================================================== */
/* Surface layer: friction velocity and Monin-Obukhov length               */
/* ======================================================================== */
/*
 * Sec. 2 computes u* and L iteratively from the vertical stratification.
 * Monin-Obukhov similarity with the Businger-Dyer gradient functions,
 * integrated (Paulson 1970):
 *   U      = (u*) / kappa [ln(z/z0) - psi_m(z/L) + psi_m(z0/L)]
 *   dtheta = (theta*) / kappa [ln(z/z0) - psi_h(z/L) + psi_h(z0/L)]
 *   L      = u*^2 T0 / (kappa g theta*)
 * stable (s >= 0): psi_m = psi_h = -5 s;
 * unstable: x = (1 - 16 s)^(1/4), psi_m = 2 ln((1 + x)/2) + ln((1 + x^2)/2)
 *           - 2 atan(x) + pi/2, psi_h = 2 ln((1 + x^2)/2).
 * Fixed-point iteration in 1/L from neutral (1/L = 0).
 */
static double psi_m(double s)
{
    if (s >= 0.0) return -5.0 * s;
    double x = pow(1.0 - 16.0 * s, 0.25);
    return 2.0 * log(0.5 * (1.0 + x)) + log(0.5 * (1.0 + x * x)) - 2.0 * atan(x) +
           0.5 * 3.141592653589793238462643383279;
}

static double psi_h(double s)
{
    if (s >= 0.0) return -5.0 * s;
    double x = pow(1.0 - 16.0 * s, 0.25);
    return 2.0 * log(0.5 * (1.0 + x * x));
}

int orc_surface_layer(double U, double z_ref, double z0, double dtheta, double T0, double* ustar,
                      double* inv_L)
{
    const double kappa = 0.4, g = 9.81;
    if (!(U > 0.0 && z_ref > z0 && z0 > 0.0 && T0 > 0.0) || !ustar || !inv_L) return -1;
    double il = 0.0, us = kappa * U / log(z_ref / z0);
    for (int it = 0; it < 200; ++it) {
        double fm = log(z_ref / z0) - psi_m(z_ref * il) + psi_m(z0 * il);
        double fh = log(z_ref / z0) - psi_h(z_ref * il) + psi_h(z0 * il);
        if (!(fm > 0.0) || !(fh > 0.0)) return -1;
        us = kappa * U / fm;
        double ts = kappa * dtheta / fh;
        double nl = kappa * g * ts / (us * us * T0);
        if (!isfinite(nl) || !(us > 0.0)) return -1;  /* diverged: too stable */
        if (fabs(nl - il) <= 1e-12 * fabs(nl) || nl == il) {
            *ustar = us;
            *inv_L = nl;
            return 0;
        }
        il = nl;
    }
    return -1;
}

/*
 * Driver for the sanitizer build of the oracle (test infrastructure):
 * compiled together with oracle/lpm_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py, it runs every
 * entry point of the oracle on small problems that reach its branches --
 * gridded and uniform wind, hourly fields with nonuniform levels and a
 * vertical component, every K_z kind, the decay chain, stochastic deposition,
 * nearest-cell and cloud-in-cell grids, exits, receptor forward, tangents
 * and adjoint, the surface layer -- and prints one checksum line.  Any
 * memory error or undefined behaviour aborts it with a report.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/lpm_oracle.c"

static float* make_field(int nt, int nz, int ny, int nx, int nc)
{
    size_t n = (size_t)nt * nz * ny * nx * nc;
    float* f = (float*)malloc(n * sizeof(float));
    for (size_t i = 0; i < n; ++i) f[i] = (float)(3.0 * sin(0.37 * (double)i) + 0.5 * (double)(i % 7));
    return f;
}

static void base_problem(orc_problem* P, const float* f, int nt, int nz, int ny, int nx, int nc,
                         int64_t n)
{
    memset(P, 0, sizeof *P);
    P->n_total = n; P->n_local = n; P->id_base = 0; P->id_stride = 1; P->s_release = 40;
    P->xs = 0.0; P->ys = 0.0; P->h = 50.0; P->q = 1.0; P->wind_scale = 1.05; P->v_d = 0.002;
    P->scenario = 3; P->seed = 7;
    P->dt = 5.0; P->Kh = 50.0; P->Kz_const = 5.0; P->kappa_ustar = 0.2; P->z0 = 0.25;
    P->H_mix = 1000.0; P->H_lid = 1000.0; P->h_s = 40.0;
    P->kz_kind = 1; P->n_nuc = 2; P->lambda[0] = 1e-6; P->lambda[1] = 1e-5;
    P->Lambda0 = 1e-4; P->rain_cx = 300.0; P->rain_cy = -200.0; P->rain_a = 2000.0;
    P->rain_b = 900.0; P->rain_angle = 0.4; P->rain_edge = 0.2;
    P->f = f; P->z_levels = NULL;
    P->nx = nx; P->ny = ny; P->nz = nz; P->nt = nt; P->ncomp = nc; P->bounded = 1;
    P->fx0 = -3000.0; P->fy0 = -3000.0; P->fdx = 6000.0 / nx; P->fdy = 6000.0 / ny;
    P->fdz = 1200.0 / nz; P->ft0 = 0.0; P->fdt = 120.0;
    P->cnx = 12; P->cny = 10; P->cnz = 6; P->cmode = 1; P->cdensity = 1;
    P->cx0 = -3000.0; P->cy0 = -2500.0; P->cz0 = 0.0; P->cdx = 500.0; P->cdy = 500.0; P->cdz = 100.0;
    P->dnx = 12; P->dny = 12; P->dmode = 1; P->ddensity = 1;
    P->dx0 = -3000.0; P->dy0 = -3000.0; P->ddx = 500.0; P->ddy = 500.0;
}

static double run(orc_problem* P, int steps)
{
    int64_t n = P->n_local;
    double* x = (double*)calloc((size_t)n, sizeof(double));
    double* y = (double*)calloc((size_t)n, sizeof(double));
    double* z = (double*)calloc((size_t)n, sizeof(double));
    double* m = (double*)calloc((size_t)n, sizeof(double));
    size_t dcells = (size_t)P->n_nuc * P->dnx * P->dny;
    size_t ccells = (size_t)P->n_nuc * P->cnx * P->cny * P->cnz;
    double* dep = (double*)calloc(dcells, sizeof(double));
    double ledger[16] = {0};
    int32_t snaps[2] = {steps / 2, steps - 1};
    double* grids = (double*)calloc(2 * ccells, sizeof(double));
    int64_t ps = 0;
    double sum = 0.0;
    if (orc_simulate(P, 0, steps / 2 + 1, x, y, z, m, dep, ledger, snaps, 1, grids, 2, &ps) != 0 ||
        orc_simulate(P, steps / 2 + 1, steps, x, y, z, m, dep, ledger, snaps + 1, 1,
                     grids + ccells, 2, &ps) != 0) {
        fprintf(stderr, "oracle rejected a problem\n");
        exit(2);
    }
    double air[4];
    orc_airborne(P, steps - 1, m, air);
    for (size_t i = 0; i < dcells; ++i) sum += dep[i];
    for (size_t i = 0; i < 2 * ccells; ++i) sum += grids[i];
    for (int i = 0; i < 4 * P->n_nuc; ++i) sum += ledger[i];
    for (int i = 0; i < P->n_nuc; ++i) sum += air[i];
    free(x); free(y); free(z); free(m); free(dep); free(grids);
    return sum + (double)ps;
}

int main(void)
{
    double total = 0.0;
    /* gridded, steady, two components */
    float* f1 = make_field(1, 6, 8, 9, 2);
    /* hourly, three components, nonuniform levels */
    float* f2 = make_field(3, 5, 7, 6, 3);
    float lev[5] = {5.0f, 40.0f, 150.0f, 500.0f, 1100.0f};
    orc_problem P;
    for (int kind = 0; kind <= 3; ++kind) {
        base_problem(&P, f1, 1, 6, 8, 9, 2, 300);
        P.kz_kind = kind;
        P.inv_L = kind == 3 ? -0.004 : 0.0;
        total += run(&P, 60);
    }
    base_problem(&P, f2, 3, 5, 7, 6, 3, 257);
    P.z_levels = lev;
    P.cmode = 0;
    P.dmode = 0;
    P.kz_kind = 2;
    total += run(&P, 70);
    /* decay chain of three with stochastic deposition, stable stratification */
    base_problem(&P, f1, 1, 6, 8, 9, 2, 211);
    P.chain = 1; P.dep_mode = 1; P.n_nuc = 3;
    P.lambda[0] = 1e-3; P.lambda[1] = 4e-4; P.lambda[2] = 2e-3;
    P.kz_kind = 3; P.inv_L = 0.01;
    total += run(&P, 50);
    /* subset of ids, no lid, unbounded field */
    base_problem(&P, f1, 1, 6, 8, 9, 2, 1000);
    P.n_local = 90; P.id_base = 5; P.id_stride = 11; P.H_lid = 0.0; P.bounded = 0;
    total += run(&P, 45);
    /* receptors: forward with tangents, and the adjoint */
    base_problem(&P, f2, 3, 5, 7, 6, 3, 150);
    P.z_levels = lev; P.kz_kind = 2;
    double rx[3] = {200.0, -400.0, 900.0}, ry[3] = {100.0, 300.0, -700.0}, rz[3] = {0.0, 10.0, 30.0};
    orc_receptors R = {3, 0, rx, ry, rz, 250.0, 40.0, 300.0};
    double c[3] = {0}, dc[12] = {0}, gbar[3] = {1.0, -0.5, 2.0}, grad[4] = {0};
    int64_t ps = 0;
    if (orc_receptor_forward(&P, &R, 120, 30, c, dc, 2, &ps) != 0 ||
        orc_receptor_adjoint(&P, &R, 120, 30, gbar, grad, 2) != 0) {
        fprintf(stderr, "receptor problem rejected\n");
        return 2;
    }
    for (int i = 0; i < 3; ++i) total += c[i];
    for (int i = 0; i < 4; ++i) total += grad[i] + dc[i];
    /* pieces */
    double w[3], K, dK, us, il;
    orc_wind(&P, 123.0, -456.0, 78.0, 100.0, w);
    orc_kz(&P, 333.0, &K, &dK);
    total += w[0] + w[1] + w[2] + K + dK + orc_dry_rate(&P, 12.0) + orc_wet_rate(&P, 50.0, 60.0);
    total += orc_activity_fraction(&P, 1, 1000.0);
    if (orc_surface_layer(6.0, 10.0, 0.25, -1.5, 290.0, &us, &il) == 0) total += us + il;
    if (orc_surface_layer(6.0, 10.0, 0.25, 0.4, 290.0, &us, &il) == 0) total += us + il;
    double nrm[4];
    orc_normals(7, 3, 12345u, 99u, 0u, nrm);
    total += nrm[0] + nrm[1] + nrm[2] + nrm[3];
    free(f1);
    free(f2);
    if (!isfinite(total)) {
        fprintf(stderr, "non-finite checksum\n");
        return 3;
    }
    printf("checksum %.17g\n", total);
    return 0;
}

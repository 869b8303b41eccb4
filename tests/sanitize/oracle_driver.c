/* Runs the oracle's entry points on small problems of every kind, for a
 * build under AddressSanitizer and UndefinedBehaviorSanitizer (host only).
 * Exit status 0 when every call returns as expected; the sanitizers abort
 * on any invalid access or undefined operation. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/bsde_oracle.h"

static int fails = 0;
#define EXPECT(c)                                                  \
    do {                                                           \
        if (!(c)) {                                                \
            fprintf(stderr, "failed: %s (line %d)\n", #c, __LINE__); \
            ++fails;                                               \
        }                                                          \
    } while (0)

static oracle_problem base_1d(int nx, int nt, int k)
{
    oracle_problem p;
    memset(&p, 0, sizeof(p));
    p.d = 1;
    p.T = 1.0;
    p.n_t = nt;
    p.k_y = p.k_z = k;
    p.L = 8;
    p.n_x[0] = nx;
    p.x_min[0] = -4.0;
    p.x_max[0] = 4.0;
    p.vol[0][0] = 1.0;
    p.driver = ORACLE_DRIVER_LINEAR;
    p.p[0] = 0.5;
    p.p[1] = -1.0;
    p.picard_max = 5;
    return p;
}

static void sine_layers(const oracle_problem *p, double *iy, double *iz)
{
    const int K = p->k_y > p->k_z ? p->k_y : p->k_z, nx = p->n_x[0];
    const double dt = p->T / p->n_t, dx = (p->x_max[0] - p->x_min[0]) / (nx - 1);
    for (int r = 0; r < K; ++r)
        for (int i = 0; i < nx; ++i) {
            const double t = (p->n_t - K + 1 + r) * dt, x = p->x_min[0] + i * dx;
            iy[r * nx + i] = sin(x + t);
            iz[r * nx + i] = cos(x + t);
        }
}

int main(void)
{
    double a[64], w[64], g[8];
    for (int L = 1; L <= 64; L *= 2) EXPECT(oracle_gauss_hermite(L, a, w) == ORACLE_OK);
    EXPECT(oracle_gauss_hermite(0, a, w) != ORACLE_OK);
    for (int K = 1; K <= 6; ++K) EXPECT(oracle_gamma(1, K, g) == ORACLE_OK && oracle_gamma(2, K, g) == ORACLE_OK);
    EXPECT(oracle_gamma(3, 2, g) != ORACLE_OK);

    const int nx = 97, nt = 12;
    double *iy = calloc(6 * nx, sizeof(double)), *iz = calloc(6 * nx, sizeof(double));
    double *y = calloc(nx, sizeof(double)), *z = calloc(nx, sizeof(double));
    oracle_stats st;
    for (int k = 1; k <= 6; ++k)
        for (int variant = 0; variant < 5; ++variant) {
            oracle_problem p = base_1d(nx, nt, k);
            double *tab = NULL;
            if (variant == 1) p.quad = 1;                        /* exact expectations */
            if (variant == 2) { p.z_form = 1; }                  /* E[y dW]/dt */
            if (variant == 3) { p.drift_x = -0.3; p.vol_x = 0.05; } /* affine coefficients */
            if (variant == 4) {                                  /* per-step table */
                tab = malloc(sizeof(double) * 2 * nt * nx);
                for (int s = 0; s < nt; ++s)
                    for (int i = 0; i < nx; ++i) {
                        tab[(2 * s) * nx + i] = 0.1 * sin(i * 0.1);
                        tab[(2 * s + 1) * nx + i] = 1.0 + 0.2 * cos(i * 0.05 + s);
                    }
                p.coef_tab = tab;
                p.tab_steps = nt;
            }
            sine_layers(&p, iy, iz);
            EXPECT(oracle_solve(&p, iy, iz, y, z, &st) == ORACLE_OK);
            EXPECT(isfinite(y[nx / 2]) && isfinite(z[nx / 2]));
            EXPECT(oracle_initial_layers(&p, 3, iy, iz) == ORACLE_OK);
            free(tab);
        }
    {   /* the bid-ask driver with Picard tolerance, a checkpoint */
        oracle_problem p = base_1d(nx, nt, 3);
        p.driver = ORACLE_DRIVER_BIDASK;
        p.p[0] = 0.01; p.p[1] = 0.06; p.p[2] = 0.2; p.p[3] = 0.2; p.p[4] = 1.0;
        p.picard_tol = 1e-14;
        p.n_stop = 4;
        sine_layers(&p, iy, iz);
        EXPECT(oracle_solve(&p, iy, iz, y, z, &st) == ORACLE_OK);
    }
    {   /* invalid problems are refused */
        oracle_problem p = base_1d(nx, nt, 2);
        p.n_x[0] = 3;
        EXPECT(oracle_solve(&p, iy, iz, y, z, &st) != ORACLE_OK);
        p = base_1d(nx, nt, 2);
        p.tab_steps = 2;  /* a table of neither 1 nor n_t rows, and no pointer */
        EXPECT(oracle_solve(&p, iy, iz, y, z, &st) != ORACLE_OK);
    }
    {   /* 2-D: tensor spline and bicubic, with correlation; sampled first step */
        const int n0 = 17, n1 = 23, np = n0 * n1, K = 3;
        oracle_problem p;
        memset(&p, 0, sizeof(p));
        p.d = 2; p.T = 1.0; p.n_t = 8; p.k_y = p.k_z = K; p.L = 4;
        p.n_x[0] = n0; p.n_x[1] = n1;
        p.x_min[0] = p.x_min[1] = -3.0; p.x_max[0] = p.x_max[1] = 3.0;
        p.vol[0][0] = 0.3; p.vol[1][0] = 0.1; p.vol[1][1] = 0.25;
        p.driver = ORACLE_DRIVER_LINEAR; p.p[0] = -0.05; p.picard_max = 3;
        double *jy = calloc(K * np, sizeof(double)), *jz = calloc(2 * K * np, sizeof(double));
        double *y2 = calloc(np, sizeof(double)), *z2 = calloc(2 * np, sizeof(double));
        for (int q = 0; q < K * np; ++q) { jy[q] = sin(0.01 * q); jz[2 * q] = jz[2 * q + 1] = 0.1; }
        for (int interp = 0; interp < 2; ++interp) {
            p.interp2 = interp;
            EXPECT(oracle_solve(&p, jy, jz, y2, z2, &st) == ORACLE_OK);
            long idx[3] = {0, np / 2, np - 1};
            double ys[3], zs[6];
            EXPECT(oracle_first_step_points_2d(&p, jy, jz, 3, idx, ys, zs) == ORACLE_OK);
        }
        free(jy); free(jz); free(y2); free(z2);
    }
    {   /* the exact expectation and the spline evaluation helpers */
        double yy[40], zz[40], c[3] = {-5.0, 0.1, 5.0}, out[12], X[4] = {-9.0, -1.0, 0.3, 9.0}, sv[4];
        for (int i = 0; i < 40; ++i) { yy[i] = sin(0.2 * i); zz[i] = cos(0.2 * i); }
        EXPECT(oracle_exact_expectation(40, -4.0, 4.0, yy, zz, 3, c, 0.7, 0.5, out) == ORACLE_OK);
        EXPECT(oracle_spline_eval(40, -4.0, 4.0, yy, 4, X, sv) == ORACLE_OK);
    }
    free(iy); free(iz); free(y); free(z);
    if (fails) fprintf(stderr, "%d check(s) failed\n", fails);
    else printf("oracle under sanitizers: all calls ok\n");
    return fails ? 1 : 0;
}

/* Runs the library's host-side entry points that need no device (problem
 * validation and planning arithmetic through bsde_problem_info, the
 * Gauss-Hermite and gamma tables, the status strings) on problems of every
 * kind, valid and invalid, for a host-only build under AddressSanitizer and
 * UndefinedBehaviorSanitizer. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/bsde.h"

static int fails = 0;
#define EXPECT(c)                                                    \
    do {                                                             \
        if (!(c)) {                                                  \
            fprintf(stderr, "failed: %s (line %d)\n", #c, __LINE__); \
            ++fails;                                                 \
        }                                                            \
    } while (0)

static bsde_problem base(int d)
{
    bsde_problem p;
    memset(&p, 0, sizeof(p));
    p.d = d;
    p.T = 0.5;
    p.n_t = 64;
    p.k_y = p.k_z = 4;
    p.L = 16;
    p.n_x[0] = p.n_x[1] = 257;
    p.x_min[0] = p.x_min[1] = 3.0;
    p.x_max[0] = p.x_max[1] = 6.0;
    p.drift[0] = p.drift[1] = 0.05;
    p.vol[0][0] = 0.2;
    p.vol[1][0] = 0.1;
    p.vol[1][1] = 0.25;
    p.driver = BSDE_DRIVER_LINEAR;
    p.p[0] = -0.05;
    p.p[1] = -0.2;
    p.picard_max = 30;
    return p;
}

int main(void)
{
    double a[64], w[64], g[8];
    for (int L = 1; L <= 64; ++L) EXPECT(bsde_gauss_hermite(L, a, w) == BSDE_OK);
    EXPECT(bsde_gauss_hermite(65, a, w) == BSDE_EINVAL);
    for (int K = 1; K <= 6; ++K) EXPECT(bsde_gamma(1, K, g) == BSDE_OK && bsde_gamma(2, K, g) == BSDE_OK);
    for (int s = -1; s <= 9; ++s) EXPECT(bsde_status_string((bsde_status)s) != NULL);

    bsde_problem_info_t info;
    for (int d = 1; d <= 2; ++d)
        for (int variant = 0; variant < 8; ++variant)
            for (int K = 1; K <= 6; ++K) {
                bsde_problem p = base(d);
                p.k_y = K;
                p.k_z = 7 - K;
                double *tab = NULL;
                switch (variant) {
                case 1: p.prec = BSDE_FP32_COMP; break;
                case 2: p.quad = BSDE_QUAD_EXACT; break;
                case 3: p.z_form = BSDE_ZFORM_YDW; break;
                case 4: if (d == 2) p.interp = BSDE_INTERP_BICUBIC_FD; break;
                case 5: if (d == 1) { p.drift_x = -0.2; p.vol_x = 0.01; } break;
                case 6:
                    if (d == 1) {
                        tab = malloc(sizeof(double) * 2 * p.n_t * p.n_x[0]);
                        for (int s = 0; s < p.n_t; ++s)
                            for (int i = 0; i < p.n_x[0]; ++i) {
                                tab[(2 * s) * p.n_x[0] + i] = 0.01 * i;
                                tab[(2 * s + 1) * p.n_x[0] + i] = 0.2 + 0.001 * s;
                            }
                        p.coef_tab = tab;
                        p.tab_steps = p.n_t;
                    }
                    break;
                case 7: p.driver = BSDE_DRIVER_BIDASK; p.p[3] = 0.2; p.p[4] = 1.0; break;
                default: break;
                }
                EXPECT(bsde_problem_info(&p, &info) == BSDE_OK);
                EXPECT(isfinite(info.stability_ratio) && info.K == (K > 7 - K ? K : 7 - K));
                free(tab);
            }
    {   /* invalid problems are refused before any device call */
        bsde_problem p = base(1);
        p.n_x[0] = 3;
        EXPECT(bsde_problem_info(&p, &info) == BSDE_EINVAL);
        p = base(1);
        p.tab_steps = 5;  /* neither 1 nor n_t rows, and no table */
        EXPECT(bsde_problem_info(&p, &info) == BSDE_EINVAL);
        p = base(1);
        p.vol[0][0] = -0.2;
        EXPECT(bsde_problem_info(&p, &info) == BSDE_EINVAL);
        p = base(1);
        p.L = 0;
        EXPECT(bsde_problem_info(&p, &info) == BSDE_EINVAL);
        EXPECT(bsde_problem_info(NULL, &info) == BSDE_EINVAL);
    }
    if (fails) fprintf(stderr, "%d check(s) failed\n", fails);
    else printf("library host code under sanitizers: all calls ok\n");
    return fails ? 1 : 0;
}

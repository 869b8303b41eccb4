/*
 * bsde_oracle.c -- plain, serial, FP64 CPU oracle for the fully discrete
 * multistep scheme for BSDEs of Kapllani & Teng, "Multistep schemes for
 * solving backward stochastic differential equations on GPU"
 * (arXiv:1909.13560).
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the
 * benchmark's CPU-baseline leg are the only callers.  The GPU library never
 * links, loads or calls this file, and this file includes nothing of it.
 *
 * What it follows, step by step and in the paper's order:
 *   - Section 3.1 step 1: uniform time grid t_n = n*dt, dt = T/N; uniform
 *     truncated space grid x_i = x_min + i*dx.
 *   - Section 3.1 step 2: the K = max(K_y, K_z) newest layers are inputs.
 *   - Section 3.1 step 3 and Section 2.2 eq (20): backward loop
 *     n = N-K, ..., 0; the z equation is explicit, the y equation is implicit
 *     and solved by Picard iteration.
 *   - Section 2.2 eq (21): conditional expectations by Gauss-Hermite
 *     quadrature, E[phi](x) ~ pi^(-d/2) sum_L w_L phi(x + sqrt(2 j dt) a_L),
 *     tensor product for d = 2.
 *   - Section 3.2: nodes outside the truncated domain take the boundary
 *     values; the interval that holds a node is found in O(1) as
 *     floor((X - x_min)/dx) on the uniform grid.
 *   - Table 1 (gamma^{K_y}_{K_y,j}) and Table 2 (gamma^1_{K_z,j}).
 *
 * Readings where the paper is silent or ambiguous:
 *   - the spatial interpolant is the natural cubic spline, written in
 *     second-derivative form (d = 2: the tensor-product natural spline);
 *   - the forward process is X_{t+h} = X_t + drift*h + vol*(W_{t+h} - W_t)
 *     with constant drift and vol (X = W is drift 0, vol 1; the log-price of
 *     eq (33) is drift mu - sigma^2/2, vol sigma); with coefficients that
 *     depend on the state (affine, or tabulated on the grid and per step) it
 *     is one Euler step X = x + a(t_n, x) j dt + b(t_n, x) dW over j dt from
 *     (t_n, x_i), eq (1); the z equation uses the Brownian increment dW, as in
 *     eq (12)-(13);
 *   - the driver is evaluated as f(t_{n+j}, X_node, y_hat, z_hat) inside the
 *     expectations and as f(t_n, x_i, y, z^n_i) in the implicit term;
 *   - Picard starts from y^{n+1}_i and stops after picard_max iterations, or
 *     earlier when |y_new - y| <= picard_tol * max(1, |y_new|) if tol > 0.
 *
 * Pins (tests outside this file): Tables 4 and 5 (d = 1, Examples 1 and 2)
 * and Table 9 (d = 2, Example 4) reproduced to the printed digits, the
 * closed forms of Examples 3 and 5, library references for the quadrature
 * rule and the spline, and special cases (a problem independent of x2
 * reduces the d = 2 sweep to the d = 1 sweep).
 *
 * Built with -O2 -ffp-contract=off and no fast-math.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "bsde_oracle.h"

/* ------------------------------------------------------------------------- */
/* Table 1: gamma^{K_y}_{K_y,j}, j = 0..K_y, for K_y = 1..6 (numerator,      */
/* denominator), as printed in the paper.                                     */
/* ------------------------------------------------------------------------- */
static const int TAB1[6][7][2] = {
    {{1, 2}, {1, 2}},
    {{1, 6}, {2, 3}, {1, 6}},
    {{1, 8}, {3, 8}, {3, 8}, {1, 8}},
    {{1, 12}, {1, 3}, {1, 6}, {1, 3}, {1, 12}},
    {{41, 600}, {19, 75}, {107, 600}, {107, 600}, {19, 75}, {41, 600}},
    {{19, 336}, {3, 14}, {15, 112}, {4, 21}, {15, 112}, {3, 14}, {19, 336}},
};

/* Table 2: gamma^1_{K_z,j}, j = 0..K_z, for K_z = 1..6, as printed. */
static const int TAB2[6][7][2] = {
    {{1, 2}, {1, 2}},
    {{5, 12}, {2, 3}, {-1, 12}},
    {{3, 8}, {19, 24}, {-5, 24}, {1, 24}},
    {{35, 96}, {5, 6}, {-13, 48}, {1, 12}, {-1, 96}},
    {{131, 360}, {151, 180}, {-103, 360}, {37, 360}, {-1, 45}, {1, 360}},
    {{163, 448}, {47, 56}, {-129, 448}, {3, 28}, {-37, 1344}, {1, 168}, {-1, 1344}},
};

int oracle_gamma(int table, int K, double *g)
{
    if (K < 1 || K > 6 || (table != 1 && table != 2)) return ORACLE_EINVAL;
    for (int j = 0; j <= K; ++j) {
        const int *q = table == 1 ? TAB1[K - 1][j] : TAB2[K - 1][j];
        g[j] = (double)q[0] / (double)q[1];
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* Gauss-Hermite rule for the weight exp(-x^2) (eq (21)).                     */
/*                                                                            */
/* Roots: the zeros of the degree-L orthonormal Hermite polynomial p_L,      */
/* bracketed by a sign scan and refined by bisection.  Weights: the          */
/* Christoffel numbers w_l = 1 / sum_{k<L} p_k(a_l)^2.  p_k comes from the   */
/* orthonormal three-term recurrence                                          */
/*   p_0 = pi^(-1/4),  p_1 = sqrt(2) x p_0,                                   */
/*   p_{k+1} = sqrt(2/(k+1)) x p_k - sqrt(k/(k+1)) p_{k-1}.                   */
/* ------------------------------------------------------------------------- */
static double hermite_orthonormal(int L, double x, double *sumsq)
{
    double pm1 = 0.0, p = pow(M_PI, -0.25), s = 0.0;
    for (int k = 0; k < L; ++k) {
        s += p * p;
        double pn = sqrt(2.0 / (k + 1)) * x * p - sqrt((double)k / (k + 1)) * pm1;
        pm1 = p;
        p = pn;
    }
    if (sumsq) *sumsq = s;
    return p;
}

int oracle_gauss_hermite(int L, double *a, double *w)
{
    if (L < 1 || L > ORACLE_MAX_L) return ORACLE_EINVAL;
    /* every zero lies inside |x| < sqrt(2L+1) */
    double lim = sqrt(2.0 * L + 1.0) + 0.5;
    int nscan = 200 * L + 1000, found = 0;
    double h = 2.0 * lim / nscan;
    double xl = -lim, fl = hermite_orthonormal(L, xl, NULL);
    for (int s = 1; s <= nscan && found < L; ++s) {
        double xr = -lim + s * h, fr = hermite_orthonormal(L, xr, NULL);
        /* a value of exactly zero counts as non-negative, so an exact zero
         * on a scan point is bracketed once */
        if ((fl < 0.0) != (fr < 0.0)) {
            double lo = xl, hi = xr;
            const int neg_lo = fl < 0.0;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                double fm = hermite_orthonormal(L, mid, NULL);
                if ((fm < 0.0) == neg_lo) lo = mid;
                else hi = mid;
            }
            a[found++] = 0.5 * (lo + hi);
        }
        xl = xr;
        fl = fr;
    }
    if (found != L) return ORACLE_EINTERNAL;
    for (int l = 0; l < L; ++l) {
        double s;
        hermite_orthonormal(L, a[l], &s);
        w[l] = 1.0 / s;
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* Natural cubic spline in second-derivative form on a uniform grid.          */
/*   M_0 = M_{N-1} = 0,                                                       */
/*   M_{i-1} + 4 M_i + M_{i+1} = 6/dx^2 (y_{i+1} - 2 y_i + y_{i-1}),          */
/* solved by the Thomas algorithm.  'stride' walks a strided line so the      */
/* same routine serves both axes of a 2-D grid.                               */
/* ------------------------------------------------------------------------- */
static void natural_spline(int n, double dx, const double *y, long ystride,
                           double *M, long mstride, double *work)
{
    for (int i = 0; i < n; ++i) M[(long)i * mstride] = 0.0;
    if (n < 3) return;
    int m = n - 2; /* unknowns M_1..M_{n-2} */
    double *c = work, *r = work + m;
    double s = 6.0 / (dx * dx);
    for (int k = 0; k < m; ++k) {
        int i = k + 1;
        r[k] = s * (y[(long)(i + 1) * ystride] - 2.0 * y[(long)i * ystride] +
                    y[(long)(i - 1) * ystride]);
    }
    /* forward elimination with diagonal 4, off-diagonals 1 */
    double beta = 4.0;
    c[0] = 1.0 / beta;
    r[0] = r[0] / beta;
    for (int k = 1; k < m; ++k) {
        beta = 4.0 - c[k - 1];
        c[k] = 1.0 / beta;
        r[k] = (r[k] - r[k - 1]) / beta;
    }
    /* back substitution */
    for (int k = m - 2; k >= 0; --k) r[k] -= c[k] * r[k + 1];
    for (int k = 0; k < m; ++k) M[(long)(k + 1) * mstride] = r[k];
}

/* Locate X on the uniform grid (Section 3.2): returns the left index p and   */
/* the fraction theta in [0,1]; nodes outside the domain are clamped to the   */
/* boundary (the boundary value is then returned by the evaluation).          */
static void locate(double X, double xmin, double dx, int n, int *p, double *theta)
{
    double xmax = xmin + (n - 1) * dx;
    if (X <= xmin) { *p = 0; *theta = 0.0; return; }
    if (X >= xmax) { *p = n - 2; *theta = 1.0; return; }
    int q = (int)floor((X - xmin) / dx);
    if (q > n - 2) q = n - 2;
    if (q < 0) q = 0;
    *p = q;
    *theta = (X - (xmin + q * dx)) / dx;
}

/* the two cubic basis functions of the second-derivative form */
static double basis_c(double theta, double dx)
{
    double u = 1.0 - theta;
    return dx * dx / 6.0 * (u * u * u - u);
}
static double basis_d(double theta, double dx)
{
    return dx * dx / 6.0 * (theta * theta * theta - theta);
}

/* ------------------------------------------------------------------------- */
/* Exact Gaussian expectation of the interpolating spline (the variant of     */
/* eq (21) without quadrature error).  X = c + s xi with xi ~ N(0, 1), and    */
/* dW = h xi (h = sqrt(j dt)):                                                 */
/*   E[yhat(X)]    = int yhat(x) phi((x - c)/s)/s dx,                         */
/*   E[yhat(X) dW] = int yhat(x) h (x - c)/s phi((x - c)/s)/s dx,             */
/* with yhat the boundary value outside the grid (Section 3.2).  Each grid    */
/* cell is integrated by 6-point Gauss-Legendre over sub-intervals of at most */
/* s/8 (a cubic times a Gaussian that changes little there: the rule is exact */
/* to degree 11, and the Gaussian's Taylor remainder over s/8 is below the    */
/* rounding of the sum); cells more than 9 s from c carry less than 1e-18 of  */
/* the mass and are left out; the two tails outside the grid have closed      */
/* forms (Phi, phi).  y and z are integrated together.                         */
/* ------------------------------------------------------------------------- */
#define GL_N 6
static double gl_x[GL_N], gl_w[GL_N];

/* Gauss-Legendre rule on [0, 1]: Newton on the Legendre recurrence */
static void gauss_legendre01(void)
{
    if (gl_w[0] != 0.0) return;
    for (int k = 0; k < GL_N; ++k) {
        double x = cos(M_PI * (k + 0.75) / (GL_N + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int n = 2; n <= GL_N; ++n) {
                double p2 = ((2.0 * n - 1.0) * x * p1 - (n - 1.0) * p0) / n;
                p0 = p1;
                p1 = p2;
            }
            dp = GL_N * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        gl_x[k] = 0.5 * (1.0 - x);
        gl_w[k] = 1.0 / ((1.0 - x * x) * dp * dp); /* 2/((1-x^2)P'^2), halved */
    }
}

static double normal_pdf(double u) { return exp(-0.5 * u * u) / sqrt(2.0 * M_PI); }
static double normal_cdf(double u) { return 0.5 * erfc(-u / sqrt(2.0)); }

/* E[v(X)], E[v(X) dW] for the two splines (v, M) = (y, My) and (z, Mz) on the
 * grid: out[0] = E[yhat], out[1] = E[yhat dW], out[2] = E[zhat],
 * out[3] = E[zhat dW] */
static void exact_expectation(int n, double xmin, double dx, const double *y, const double *My,
                              const double *z, const double *Mz, double c, double sd, double h,
                              double *out)
{
    const double xmax = xmin + (n - 1) * dx;
    const double u0 = (xmin - c) / sd, u1 = (xmax - c) / sd;
    /* tails: boundary values; E[xi 1{xi < u0}] = -phi(u0), E[xi 1{xi > u1}] = phi(u1) */
    const double P0 = normal_cdf(u0), P1 = normal_cdf(-u1);
    const double W0 = -h * normal_pdf(u0), W1 = h * normal_pdf(u1);
    out[0] = y[0] * P0 + y[n - 1] * P1;
    out[1] = y[0] * W0 + y[n - 1] * W1;
    out[2] = z[0] * P0 + z[n - 1] * P1;
    out[3] = z[0] * W0 + z[n - 1] * W1;
    int plo = (int)floor((c - 9.0 * sd - xmin) / dx), phi_ = (int)floor((c + 9.0 * sd - xmin) / dx);
    if (plo < 0) plo = 0;
    if (phi_ > n - 2) phi_ = n - 2;
    int nsub = (int)ceil(8.0 * dx / sd);
    if (nsub < 1) nsub = 1;
    for (int p = plo; p <= phi_; ++p) {
        /* integrals of the four basis functions against the density, plain
         * and dW-weighted */
        double I[4] = {0, 0, 0, 0}, J[4] = {0, 0, 0, 0};
        for (int q = 0; q < nsub; ++q) {
            for (int g = 0; g < GL_N; ++g) {
                const double th = (q + gl_x[g]) / nsub; /* fraction within cell p */
                const double u = (xmin + (p + th) * dx - c) / sd;
                const double wgt = gl_w[g] / nsub * dx * normal_pdf(u) / sd;
                const double b[4] = {1.0 - th, th, basis_c(th, dx), basis_d(th, dx)};
                for (int k = 0; k < 4; ++k) {
                    I[k] += wgt * b[k];
                    J[k] += wgt * b[k] * h * u;
                }
            }
        }
        out[0] += I[0] * y[p] + I[1] * y[p + 1] + I[2] * My[p] + I[3] * My[p + 1];
        out[1] += J[0] * y[p] + J[1] * y[p + 1] + J[2] * My[p] + J[3] * My[p + 1];
        out[2] += I[0] * z[p] + I[1] * z[p + 1] + I[2] * Mz[p] + I[3] * Mz[p + 1];
        out[3] += J[0] * z[p] + J[1] * z[p + 1] + J[2] * Mz[p] + J[3] * Mz[p + 1];
    }
}

int oracle_exact_expectation(int n, double xmin, double xmax, const double *y, const double *z,
                             int m, const double *c, double sd, double h, double *out)
{
    if (n < 4 || !(xmax > xmin) || !(sd > 0.0) || m < 0) return ORACLE_EINVAL;
    const double dx = (xmax - xmin) / (n - 1);
    double *M = (double *)malloc(sizeof(double) * (size_t)4 * n);
    if (!M) return ORACLE_ENOMEM;
    gauss_legendre01();
    natural_spline(n, dx, y, 1, M, 1, M + 2 * n);
    natural_spline(n, dx, z, 1, M + n, 1, M + 2 * n);
    for (int k = 0; k < m; ++k)
        exact_expectation(n, xmin, dx, y, M, z, M + n, c[k], sd, h, out + 4 * (size_t)k);
    free(M);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* Drivers f(t, x, y, z).                                                      */
/* ------------------------------------------------------------------------- */
static double driver(const oracle_problem *pb, double t, double y, const double *z)
{
    const double *p = pb->p;
    switch (pb->driver) {
    case ORACLE_DRIVER_LINEAR: /* a y + b1 z1 (+ b2 z2) + c */
        return pb->d == 1 ? p[0] * y + p[1] * z[0] + p[3]
                          : p[0] * y + p[1] * z[0] + p[2] * z[1] + p[3];
    case ORACLE_DRIVER_BIDASK: { /* -r y - theta z + s (R - r) min(y - z/sigma, 0) */
        double r = p[0], R = p[1], th = p[2], sg = p[3], s = p[4];
        double m = y - z[0] / sg;
        if (m > 0.0) m = 0.0;
        return -r * y - th * z[0] + s * (R - r) * m;
    }
    case ORACLE_DRIVER_CUBIC: /* Example 1, eq (22) */
        return -y * y * y + 2.5 * y * y - 1.5 * y;
    case ORACLE_DRIVER_EXP: { /* Example 2, eq (24) */
        double et = exp(t * t), emt = exp(-t * t);
        return 0.5 * (et - 4.0 * t * y - 3.0 * exp(t * t - y * emt) + z[0] * z[0] * emt);
    }
    default:
        return NAN;
    }
}

/* ------------------------------------------------------------------------- */
/* Validation.                                                                 */
/* ------------------------------------------------------------------------- */
static int validate(const oracle_problem *pb)
{
    if (pb->d != 1 && pb->d != 2) return ORACLE_EINVAL;
    if (pb->k_y < 1 || pb->k_y > 6 || pb->k_z < 1 || pb->k_z > 6) return ORACLE_EINVAL;
    int K = pb->k_y > pb->k_z ? pb->k_y : pb->k_z;
    if (pb->n_t < K || !(pb->T > 0.0)) return ORACLE_EINVAL;
    if (pb->L < 1 || pb->L > ORACLE_MAX_L) return ORACLE_EINVAL;
    for (int a = 0; a < pb->d; ++a)
        if (pb->n_x[a] < 4 || !(pb->x_max[a] > pb->x_min[a])) return ORACLE_EINVAL;
    if (pb->driver < 0 || pb->driver > ORACLE_DRIVER_EXP) return ORACLE_EINVAL;
    if (pb->d == 2 && pb->driver != ORACLE_DRIVER_LINEAR) return ORACLE_EINVAL;
    if (pb->picard_max < 1) return ORACLE_EINVAL;
    if (pb->n_stop < 0 || pb->n_stop > pb->n_t - K) return ORACLE_EINVAL;
    if (pb->z_form != 0 && pb->z_form != 1) return ORACLE_EINVAL;
    if (pb->d == 2 && (pb->drift_x != 0.0 || pb->vol_x != 0.0)) return ORACLE_EINVAL;
    if (pb->quad != 0 && pb->quad != 1) return ORACLE_EINVAL;
    if (pb->interp2 != 0 && pb->interp2 != 1) return ORACLE_EINVAL;
    if (pb->interp2 == 1 && (pb->d != 2 || pb->n_x[0] < 5 || pb->n_x[1] < 5)) return ORACLE_EINVAL;
    if (pb->quad == 1 && (pb->d != 1 || pb->driver != ORACLE_DRIVER_LINEAR ||
                          pb->drift_x != 0.0 || pb->vol_x != 0.0 || pb->tab_steps != 0))
        return ORACLE_EINVAL;
    if (pb->tab_steps != 0) { /* tabulated coefficients */
        if (pb->d != 1 || !pb->coef_tab || (pb->tab_steps != 1 && pb->tab_steps != pb->n_t))
            return ORACLE_EINVAL;
        if (pb->drift_x != 0.0 || pb->vol_x != 0.0) return ORACLE_EINVAL;
        const long nx = pb->n_x[0];
        for (long k = 0; k < 2L * pb->tab_steps * nx; ++k)
            if (!isfinite(pb->coef_tab[k])) return ORACLE_EINVAL;
        for (int r = 0; r < pb->tab_steps; ++r)
            for (long i = 0; i < nx; ++i)
                if (!(pb->coef_tab[(2L * r + 1) * nx + i] > 0.0)) return ORACLE_EINVAL;
    } else if (pb->coef_tab) {
        return ORACLE_EINVAL;
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* 1-D solve.                                                                   */
/* Layer storage: a ring of K+1 layers, each holding y, M_y, z, M_z.          */
/* ------------------------------------------------------------------------- */
typedef struct {
    double *y, *My, *z, *Mz;
} layer1;

static int solve1(const oracle_problem *pb, const double *init_y, const double *init_z,
                  double *y_out, double *z_out, oracle_stats *st)
{
    const int N = pb->n_t, Ky = pb->k_y, Kz = pb->k_z, K = Ky > Kz ? Ky : Kz;
    const int L = pb->L, nx = pb->n_x[0];
    const double dt = pb->T / N;
    const double xmin = pb->x_min[0], dx = (pb->x_max[0] - pb->x_min[0]) / (nx - 1);
    /* eq (1): X_{t_{n+j}} from X_{t_n} = x_i by one Euler step over j dt,
     * a(x) = drift + drift_x x, b(x) = vol + vol_x x (constant when both
     * slopes are 0) */
    const double drift = pb->drift[0], vol = pb->vol[0][0];
    const double drift_x = pb->drift_x, vol_x = pb->vol_x;

    double a[ORACLE_MAX_L], w[ORACLE_MAX_L], gy[7], gz[7];
    int rc = oracle_gauss_hermite(L, a, w);
    if (rc) return rc;
    for (int l = 0; l < L; ++l) w[l] /= sqrt(M_PI); /* pi^(-1/2) of eq (21) */
    gauss_legendre01();
    oracle_gamma(1, Ky, gy);
    oracle_gamma(2, Kz, gz);

    layer1 ring[7];
    double *mem = (double *)malloc(sizeof(double) * (size_t)nx * 4 * (K + 1));
    double *work = (double *)malloc(sizeof(double) * (size_t)2 * nx);
    if (!mem || !work) { free(mem); free(work); return ORACLE_ENOMEM; }
    for (int s = 0; s <= K; ++s) {
        ring[s].y = mem + (size_t)nx * (4 * s + 0);
        ring[s].My = mem + (size_t)nx * (4 * s + 1);
        ring[s].z = mem + (size_t)nx * (4 * s + 2);
        ring[s].Mz = mem + (size_t)nx * (4 * s + 3);
    }
#define SLOT(n) (ring[(n) % (K + 1)])
    /* inputs: init[r] is the layer at t_{N-K+1+r}, r = 0..K-1 */
    for (int r = 0; r < K; ++r) {
        int n = N - K + 1 + r;
        memcpy(SLOT(n).y, init_y + (size_t)r * nx, sizeof(double) * nx);
        memcpy(SLOT(n).z, init_z + (size_t)r * nx, sizeof(double) * nx);
        natural_spline(nx, dx, SLOT(n).y, 1, SLOT(n).My, 1, work);
        natural_spline(nx, dx, SLOT(n).z, 1, SLOT(n).Mz, 1, work);
    }

    int it_max = 0;
    long nonconv = 0;
    for (int n = N - K; n >= pb->n_stop; --n) {
        layer1 out = SLOT(n);
        const double tn = n * dt;
        /* the points of a layer are independent: the all-cores build of this
         * file (OpenMP) shares them out; the arithmetic per point is the same */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(+ : nonconv) reduction(max : it_max)
#endif
        for (int i = 0; i < nx; ++i) {
            const double xi = xmin + i * dx;
            /* eq (1)'s coefficients at (t_n, x_i): affine, or from the table */
            double ai = drift + drift_x * xi, bi = vol + vol_x * xi;
            if (pb->tab_steps > 0) {
                const double *row = pb->coef_tab + 2L * (pb->tab_steps > 1 ? n : 0) * nx;
                ai = row[i];
                bi = row[nx + i];
            }
            double Ef[7] = {0}, EfW[7] = {0}, Ez[7] = {0}, EyK = 0.0, EyW1 = 0.0;
            for (int j = 1; j <= K; ++j) {
                layer1 lj = SLOT(n + j);
                const double tj = (n + j) * dt, sq = sqrt(2.0 * j * dt);
                if (pb->quad == 1) {
                    /* linear driver f = a y + b z + c: its expectations are
                     * those of the interpolated y and z */
                    const double cx = xi + drift * j * dt, sd = vol * sqrt(j * dt);
                    double e[4];
                    exact_expectation(nx, xmin, dx, lj.y, lj.My, lj.z, lj.Mz, cx, sd, sqrt(j * dt), e);
                    const double Ey = e[0], EyWj = e[1], Ezj = e[2], EzWj = e[3];
                    Ef[j] = pb->p[0] * Ey + pb->p[1] * Ezj + pb->p[3];
                    EfW[j] = pb->p[0] * EyWj + pb->p[1] * EzWj;
                    Ez[j] = Ezj;
                    if (j == Ky) EyK = Ey;
                    if (j == 1) EyW1 = EyWj;
                    continue;
                }
                for (int l = 0; l < L; ++l) {
                    const double dW = sq * a[l];
                    const double X = xi + ai * j * dt + bi * dW;
                    int p;
                    double th;
                    double yh, zh;
                    if (X <= xmin) { yh = lj.y[0]; zh = lj.z[0]; }
                    else if (X >= xmin + (nx - 1) * dx) { yh = lj.y[nx - 1]; zh = lj.z[nx - 1]; }
                    else {
                        locate(X, xmin, dx, nx, &p, &th);
                        double cA = 1.0 - th, cB = th, cC = basis_c(th, dx), cD = basis_d(th, dx);
                        yh = cA * lj.y[p] + cB * lj.y[p + 1] + cC * lj.My[p] + cD * lj.My[p + 1];
                        zh = cA * lj.z[p] + cB * lj.z[p + 1] + cC * lj.Mz[p] + cD * lj.Mz[p + 1];
                    }
                    const double fh = driver(pb, tj, yh, &zh);
                    Ef[j] += w[l] * fh;
                    EfW[j] += w[l] * fh * dW;
                    Ez[j] += w[l] * zh;
                    if (j == Ky) EyK += w[l] * yh;
                    if (j == 1) EyW1 += w[l] * yh * dW;
                }
            }
            /* z equation of eq (20), explicit; its first term E[z^{n+1}], or
             * E[y^{n+1} dW]/dt (eq (12) with l = 1) */
            double zs = pb->z_form ? EyW1 / dt : Ez[1];
            for (int j = 1; j <= Kz; ++j) zs += gz[j] * (EfW[j] - Ez[j]);
            const double zn = zs / gz[0];
            /* y equation of eq (20), implicit: Picard iteration */
            double Cy = EyK;
            for (int j = 1; j <= Ky; ++j) Cy += Ky * dt * gy[j] * Ef[j];
            const double h0 = Ky * dt * gy[0];
            double y = SLOT(n + 1).y[i];
            int it = 0, conv = 0;
            while (it < pb->picard_max) {
                double yn = Cy + h0 * driver(pb, tn, y, &zn);
                ++it;
                double dy = fabs(yn - y);
                y = yn;
                if (pb->picard_tol > 0.0 && dy <= pb->picard_tol * fmax(1.0, fabs(y))) {
                    conv = 1;
                    break;
                }
            }
            if (pb->picard_tol > 0.0 && !conv) ++nonconv;
            if (it > it_max) it_max = it;
            out.y[i] = y;
            out.z[i] = zn;
        }
        natural_spline(nx, dx, out.y, 1, out.My, 1, work);
        natural_spline(nx, dx, out.z, 1, out.Mz, 1, work);
    }
    memcpy(y_out, SLOT(pb->n_stop).y, sizeof(double) * nx);
    memcpy(z_out, SLOT(pb->n_stop).z, sizeof(double) * nx);
#undef SLOT
    if (st) {
        st->picard_iter_max = it_max;
        st->picard_nonconverged = nonconv;
    }
    free(mem);
    free(work);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* 2-D solve (tensor grid, tensor Gauss-Hermite, tensor natural spline).       */
/* Layer storage per layer: y, z1, z2 and, for each of them, the tensor-spline */
/* derivative arrays Mxx (along axis 0), Myy (along axis 1), Mxxyy.            */
/* Index (i0, i1) -> i0 * n1 + i1.                                              */
/* ------------------------------------------------------------------------- */
typedef struct {
    double *v, *Mxx, *Myy, *Mxxyy;
} tspline;

static void tensor_spline(int n0, int n1, double dx0, double dx1, tspline *s, double *work)
{
    /* along axis 0 for every column i1: Mxx */
    for (int i1 = 0; i1 < n1; ++i1)
        natural_spline(n0, dx0, s->v + i1, n1, s->Mxx + i1, n1, work);
    /* along axis 1 for every row i0: Myy, and the spline of Mxx: Mxxyy */
    for (int i0 = 0; i0 < n0; ++i0) {
        natural_spline(n1, dx1, s->v + (long)i0 * n1, 1, s->Myy + (long)i0 * n1, 1, work);
        natural_spline(n1, dx1, s->Mxx + (long)i0 * n1, 1, s->Mxxyy + (long)i0 * n1, 1, work);
    }
}

/* evaluate the tensor spline at (X0, X1) with coordinates clamped to the box */
static double tensor_eval(const tspline *s, int n0, int n1, double xmin0, double dx0,
                          double xmin1, double dx1, double X0, double X1)
{
    int p, q;
    double t0, t1;
    locate(X0, xmin0, dx0, n0, &p, &t0);
    locate(X1, xmin1, dx1, n1, &q, &t1);
    double a0[2] = {1.0 - t0, t0}, b0[2] = {basis_c(t0, dx0), basis_d(t0, dx0)};
    double a1[2] = {1.0 - t1, t1}, b1[2] = {basis_c(t1, dx1), basis_d(t1, dx1)};
    double acc = 0.0;
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) {
            long k = (long)(p + u) * n1 + (q + v);
            acc += a0[u] * a1[v] * s->v[k] + b0[u] * a1[v] * s->Mxx[k] +
                   a0[u] * b1[v] * s->Myy[k] + b0[u] * b1[v] * s->Mxxyy[k];
        }
    return acc;
}

/* ------------------------------------------------------------------------- */
/* The paper's own 2-D interpolation (Section 3.3): bicubic interpolation from */
/* the values and the first and mixed derivatives at the cell corners, the   */
/* derivatives from fourth-order finite differences (central inside, one-     */
/* sided at the two points next to each end).  Stored in the same four arrays */
/* as the tensor spline: v, f_x (in Mxx), f_y (in Myy), f_xy (in Mxxyy).       */
/* ------------------------------------------------------------------------- */
static void fd4_line(int n, double h, const double *f, long fs, double *d, long ds)
{
#define F(i) f[(long)(i) * fs]
    for (int i = 0; i < n; ++i) {
        double v;
        if (i >= 2 && i <= n - 3)
            v = F(i - 2) - 8.0 * F(i - 1) + 8.0 * F(i + 1) - F(i + 2);
        else if (i == 0)
            v = -25.0 * F(0) + 48.0 * F(1) - 36.0 * F(2) + 16.0 * F(3) - 3.0 * F(4);
        else if (i == 1)
            v = -3.0 * F(0) - 10.0 * F(1) + 18.0 * F(2) - 6.0 * F(3) + F(4);
        else if (i == n - 1)
            v = 25.0 * F(n - 1) - 48.0 * F(n - 2) + 36.0 * F(n - 3) - 16.0 * F(n - 4) + 3.0 * F(n - 5);
        else /* i == n - 2 */
            v = 3.0 * F(n - 1) + 10.0 * F(n - 2) - 18.0 * F(n - 3) + 6.0 * F(n - 4) - F(n - 5);
        d[(long)i * ds] = v / (12.0 * h);
    }
#undef F
}

static void bicubic_fd(int n0, int n1, double dx0, double dx1, tspline *s)
{
    for (int i1 = 0; i1 < n1; ++i1) /* f_x along axis 0 */
        fd4_line(n0, dx0, s->v + i1, n1, s->Mxx + i1, n1);
    for (int i0 = 0; i0 < n0; ++i0) { /* f_y, and f_xy = (f_x)_y, along axis 1 */
        fd4_line(n1, dx1, s->v + (long)i0 * n1, 1, s->Myy + (long)i0 * n1, 1);
        fd4_line(n1, dx1, s->Mxx + (long)i0 * n1, 1, s->Mxxyy + (long)i0 * n1, 1);
    }
}

/* cubic Hermite basis on [0, 1]: values at 0 and 1, slopes at 0 and 1 */
static void hermite(double t, double hv[2], double hd[2])
{
    hv[0] = 2.0 * t * t * t - 3.0 * t * t + 1.0;
    hv[1] = -2.0 * t * t * t + 3.0 * t * t;
    hd[0] = t * t * t - 2.0 * t * t + t;
    hd[1] = t * t * t - t * t;
}

/* the bicubic at (X0, X1) with coordinates clamped to the box */
static double bicubic_eval(const tspline *s, int n0, int n1, double xmin0, double dx0,
                           double xmin1, double dx1, double X0, double X1)
{
    int p, q;
    double t0, t1, hv0[2], hd0[2], hv1[2], hd1[2];
    locate(X0, xmin0, dx0, n0, &p, &t0);
    locate(X1, xmin1, dx1, n1, &q, &t1);
    hermite(t0, hv0, hd0);
    hermite(t1, hv1, hd1);
    double acc = 0.0;
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) {
            long k = (long)(p + u) * n1 + (q + v);
            acc += hv0[u] * hv1[v] * s->v[k] + dx0 * hd0[u] * hv1[v] * s->Mxx[k] +
                   dx1 * hv0[u] * hd1[v] * s->Myy[k] + dx0 * dx1 * hd0[u] * hd1[v] * s->Mxxyy[k];
        }
    return acc;
}

/* Everything one backward step of the 2-D sweep reads: the grid, the
 * quadrature rule, the coefficients of Tables 1-2 and the ring of K+1 layers
 * (each with its tensor splines). */
typedef struct {
    int N, Ky, Kz, K, L, n0, n1;
    int interp2; /* 0: tensor natural spline; 1: bicubic with finite differences */
    double dt, xmin0, dx0, xmin1, dx1;
    double a[ORACLE_MAX_L], w[ORACLE_MAX_L], gy[7], gz[7];
    tspline ring[7][3]; /* per ring slot: 3 fields (y, z1, z2) x 4 arrays */
    double *mem, *work;
} ctx2;

#define SLOT2(c, n) ((c)->ring[(n) % ((c)->K + 1)])

static void ctx2_free(ctx2 *c)
{
    free(c->mem);
    free(c->work);
}

/* Grid, quadrature, coefficients and the K initial layers with their tensor
 * splines (Section 3.1 steps 1-2). */
static int ctx2_init(const oracle_problem *pb, const double *init_y, const double *init_z,
                     ctx2 *c)
{
    c->N = pb->n_t;
    c->interp2 = pb->interp2;
    c->Ky = pb->k_y;
    c->Kz = pb->k_z;
    c->K = c->Ky > c->Kz ? c->Ky : c->Kz;
    c->L = pb->L;
    c->n0 = pb->n_x[0];
    c->n1 = pb->n_x[1];
    const long np = (long)c->n0 * c->n1;
    c->dt = pb->T / c->N;
    c->xmin0 = pb->x_min[0];
    c->dx0 = (pb->x_max[0] - pb->x_min[0]) / (c->n0 - 1);
    c->xmin1 = pb->x_min[1];
    c->dx1 = (pb->x_max[1] - pb->x_min[1]) / (c->n1 - 1);
    c->mem = NULL;
    c->work = NULL;

    int rc = oracle_gauss_hermite(c->L, c->a, c->w);
    if (rc) return rc;
    for (int l = 0; l < c->L; ++l) c->w[l] /= sqrt(M_PI); /* one pi^(-1/2) per axis */
    oracle_gamma(1, c->Ky, c->gy);
    oracle_gamma(2, c->Kz, c->gz);

    c->mem = (double *)malloc(sizeof(double) * (size_t)np * 12 * (c->K + 1));
    int nmax = c->n0 > c->n1 ? c->n0 : c->n1;
    c->work = (double *)malloc(sizeof(double) * (size_t)2 * nmax);
    if (!c->mem || !c->work) {
        ctx2_free(c);
        return ORACLE_ENOMEM;
    }
    for (int s = 0; s <= c->K; ++s)
        for (int f = 0; f < 3; ++f) {
            double *b = c->mem + (size_t)np * (12 * s + 4 * f);
            c->ring[s][f].v = b;
            c->ring[s][f].Mxx = b + np;
            c->ring[s][f].Myy = b + 2 * np;
            c->ring[s][f].Mxxyy = b + 3 * np;
        }
    for (int r = 0; r < c->K; ++r) {
        int n = c->N - c->K + 1 + r;
        memcpy(SLOT2(c, n)[0].v, init_y + (size_t)r * np, sizeof(double) * np);
        memcpy(SLOT2(c, n)[1].v, init_z + (size_t)r * 2 * np, sizeof(double) * np);
        memcpy(SLOT2(c, n)[2].v, init_z + (size_t)r * 2 * np + np, sizeof(double) * np);
        for (int f = 0; f < 3; ++f)
            if (c->interp2)
                bicubic_fd(c->n0, c->n1, c->dx0, c->dx1, &SLOT2(c, n)[f]);
            else
                tensor_spline(c->n0, c->n1, c->dx0, c->dx1, &SLOT2(c, n)[f], c->work);
    }
    return ORACLE_OK;
}

/* Layer n at grid point (i0, i1) from layers n+1..n+K (eq (20)-(21), Section
 * 3.1 step 3): y to out[0], z1 and z2 to out[1], out[2]; *it receives the
 * Picard iterations, *conv whether the tolerance was met. */
static void point2(const oracle_problem *pb, const ctx2 *c, int n, int i0, int i1, double *out,
                   int *it_out, int *conv_out)
{
    const int Ky = c->Ky, Kz = c->Kz, K = c->K, L = c->L, n0 = c->n0, n1 = c->n1;
    const double dt = c->dt, xmin0 = c->xmin0, dx0 = c->dx0, xmin1 = c->xmin1, dx1 = c->dx1;
    const double *a = c->a, *w = c->w, *gy = c->gy, *gz = c->gz;
    const double tn = n * dt;
    const double x0 = xmin0 + i0 * dx0, x1 = xmin1 + i1 * dx1;
    double Ef[7] = {0}, EfW[7][2] = {{0}}, Ez[7][2] = {{0}}, EyK = 0.0, EyW1[2] = {0.0, 0.0};
    for (int j = 1; j <= K; ++j) {
        const tspline *lj = SLOT2(c, n + j);
        const double tj = (n + j) * dt, sq = sqrt(2.0 * j * dt);
        for (int l0 = 0; l0 < L; ++l0)
            for (int l1 = 0; l1 < L; ++l1) {
                const double dW0 = sq * a[l0], dW1 = sq * a[l1];
                const double wt = w[l0] * w[l1];
                const double X0 = x0 + pb->drift[0] * j * dt +
                                  pb->vol[0][0] * dW0 + pb->vol[0][1] * dW1;
                const double X1 = x1 + pb->drift[1] * j * dt +
                                  pb->vol[1][0] * dW0 + pb->vol[1][1] * dW1;
                double (*ev)(const tspline *, int, int, double, double, double, double, double,
                             double) = c->interp2 ? bicubic_eval : tensor_eval;
                double yh = ev(&lj[0], n0, n1, xmin0, dx0, xmin1, dx1, X0, X1);
                double zh[2];
                zh[0] = ev(&lj[1], n0, n1, xmin0, dx0, xmin1, dx1, X0, X1);
                zh[1] = ev(&lj[2], n0, n1, xmin0, dx0, xmin1, dx1, X0, X1);
                const double fh = driver(pb, tj, yh, zh);
                Ef[j] += wt * fh;
                EfW[j][0] += wt * fh * dW0;
                EfW[j][1] += wt * fh * dW1;
                Ez[j][0] += wt * zh[0];
                Ez[j][1] += wt * zh[1];
                if (j == Ky) EyK += wt * yh;
                if (j == 1) {
                    EyW1[0] += wt * yh * dW0;
                    EyW1[1] += wt * yh * dW1;
                }
            }
    }
    double zn[2];
    for (int cc = 0; cc < 2; ++cc) {
        double zs = pb->z_form ? EyW1[cc] / dt : Ez[1][cc];
        for (int j = 1; j <= Kz; ++j) zs += gz[j] * (EfW[j][cc] - Ez[j][cc]);
        zn[cc] = zs / gz[0];
    }
    double Cy = EyK;
    for (int j = 1; j <= Ky; ++j) Cy += Ky * dt * gy[j] * Ef[j];
    const double h0 = Ky * dt * gy[0];
    const long k = (long)i0 * n1 + i1;
    double y = SLOT2(c, n + 1)[0].v[k];
    int it = 0, conv = 0;
    while (it < pb->picard_max) {
        double yn = Cy + h0 * driver(pb, tn, y, zn);
        ++it;
        double dy = fabs(yn - y);
        y = yn;
        if (pb->picard_tol > 0.0 && dy <= pb->picard_tol * fmax(1.0, fabs(y))) {
            conv = 1;
            break;
        }
    }
    out[0] = y;
    out[1] = zn[0];
    out[2] = zn[1];
    *it_out = it;
    *conv_out = conv;
}

static int solve2(const oracle_problem *pb, const double *init_y, const double *init_z,
                  double *y_out, double *z_out, oracle_stats *st)
{
    ctx2 c;
    int rc = ctx2_init(pb, init_y, init_z, &c);
    if (rc) return rc;
    const long np = (long)c.n0 * c.n1;
    int it_max = 0;
    long nonconv = 0;
    for (int n = c.N - c.K; n >= pb->n_stop; --n) {
        tspline *out = SLOT2(&c, n);
        for (int i0 = 0; i0 < c.n0; ++i0)
            for (int i1 = 0; i1 < c.n1; ++i1) {
                double r[3];
                int it, conv;
                point2(pb, &c, n, i0, i1, r, &it, &conv);
                if (pb->picard_tol > 0.0 && !conv) ++nonconv;
                if (it > it_max) it_max = it;
                const long k = (long)i0 * c.n1 + i1;
                out[0].v[k] = r[0];
                out[1].v[k] = r[1];
                out[2].v[k] = r[2];
            }
        for (int f = 0; f < 3; ++f) {
            if (c.interp2)
                bicubic_fd(c.n0, c.n1, c.dx0, c.dx1, &out[f]);
            else
                tensor_spline(c.n0, c.n1, c.dx0, c.dx1, &out[f], c.work);
        }
    }
    memcpy(y_out, SLOT2(&c, pb->n_stop)[0].v, sizeof(double) * np);
    memcpy(z_out, SLOT2(&c, pb->n_stop)[1].v, sizeof(double) * np);
    memcpy(z_out + np, SLOT2(&c, pb->n_stop)[2].v, sizeof(double) * np);
    if (st) {
        st->picard_iter_max = it_max;
        st->picard_nonconverged = nonconv;
    }
    ctx2_free(&c);
    return ORACLE_OK;
}

int oracle_first_step_points_2d(const oracle_problem *pb, const double *init_y,
                                const double *init_z, int m, const long *idx, double *y_out,
                                double *z_out)
{
    int rc = validate(pb);
    if (rc) return rc;
    if (pb->d != 2 || m < 0 || (m > 0 && (!idx || !y_out || !z_out))) return ORACLE_EINVAL;
    const long np = (long)pb->n_x[0] * pb->n_x[1];
    for (int q = 0; q < m; ++q)
        if (idx[q] < 0 || idx[q] >= np) return ORACLE_EINVAL;
    ctx2 c;
    rc = ctx2_init(pb, init_y, init_z, &c);
    if (rc) return rc;
    for (int q = 0; q < m; ++q) {
        double r[3];
        int it, conv;
        point2(pb, &c, c.N - c.K, (int)(idx[q] / c.n1), (int)(idx[q] % c.n1), r, &it, &conv);
        y_out[q] = r[0];
        z_out[2 * q] = r[1];
        z_out[2 * q + 1] = r[2];
    }
    ctx2_free(&c);
    return ORACLE_OK;
}
#undef SLOT2

int oracle_solve(const oracle_problem *pb, const double *init_y, const double *init_z,
                 double *y_out, double *z_out, oracle_stats *st)
{
    int rc = validate(pb);
    if (rc) return rc;
    return pb->d == 1 ? solve1(pb, init_y, init_z, y_out, z_out, st)
                      : solve2(pb, init_y, init_z, y_out, z_out, st);
}

/* ------------------------------------------------------------------------- */
/* Section 3.1 step 2: the K - 1 initial layers after the terminal one, by a  */
/* 1-step scheme on [t_{N-K+1}, t_N] with a finer time step.  The 1-step      */
/* scheme is eq (20) with K_y = K_z = 1 (row 1 of Tables 1 and 2); each       */
/* coarse step dt is split into `sub` steps of dt/sub.  Layer t_{N-r} is the  */
/* 1-step sweep from t_{N-r+1} (the previous result) over `sub` fine steps;   */
/* the absolute times of the driver stay t = n dt/sub.                        */
/* init_y / init_z: rows as for oracle_solve; on entry row K-1 holds the       */
/* terminal layer, on return rows 0..K-2 hold t_{N-K+1}..t_{N-1}.              */
/* ------------------------------------------------------------------------- */
int oracle_initial_layers(const oracle_problem *pb, int sub, double *init_y, double *init_z)
{
    int rc = validate(pb);
    if (rc) return rc;
    if (sub < 1 || !init_y || !init_z) return ORACLE_EINVAL;
    const int K = pb->k_y > pb->k_z ? pb->k_y : pb->k_z;
    const long np = pb->d == 1 ? (long)pb->n_x[0] : (long)pb->n_x[0] * pb->n_x[1];
    const double dt = pb->T / pb->n_t;
    for (int r = 1; r < K; ++r) {
        oracle_problem q = *pb;
        const int n_hi = pb->n_t - r + 1; /* the segment ends at t_{N-r+1} */
        q.k_y = q.k_z = 1;
        q.T = n_hi * dt;
        q.n_t = n_hi * sub;
        q.n_stop = (n_hi - 1) * sub;
        if (pb->tab_steps > 1) { /* per-step table: the row of t_{N-r} over the segment */
            q.tab_steps = 1;
            q.coef_tab = pb->coef_tab + 2L * (pb->n_t - r) * pb->n_x[0];
        }
        const double *iy = init_y + (size_t)(K - r) * np;
        const double *iz = init_z + (size_t)(K - r) * np * pb->d;
        double *oy = init_y + (size_t)(K - 1 - r) * np;
        double *oz = init_z + (size_t)(K - 1 - r) * np * pb->d;
        rc = oracle_solve(&q, iy, iz, oy, oz, NULL);
        if (rc) return rc;
    }
    return ORACLE_OK;
}

/* Natural spline of one line and its evaluation: exposed so the tests can pin */
/* the interpolation step against an independent library spline.               */
int oracle_spline_eval(int n, double xmin, double xmax, const double *y, int m,
                       const double *X, double *out)
{
    if (n < 4 || !(xmax > xmin)) return ORACLE_EINVAL;
    double dx = (xmax - xmin) / (n - 1);
    double *M = (double *)malloc(sizeof(double) * (size_t)3 * n);
    if (!M) return ORACLE_ENOMEM;
    natural_spline(n, dx, y, 1, M, 1, M + n);
    for (int k = 0; k < m; ++k) {
        if (X[k] <= xmin) { out[k] = y[0]; continue; }
        if (X[k] >= xmin + (n - 1) * dx) { out[k] = y[n - 1]; continue; }
        int p;
        double th;
        locate(X[k], xmin, dx, n, &p, &th);
        out[k] = (1.0 - th) * y[p] + th * y[p + 1] + basis_c(th, dx) * M[p] +
                 basis_d(th, dx) * M[p + 1];
    }
    free(M);
    return ORACLE_OK;
}

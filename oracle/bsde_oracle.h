/*
 * bsde_oracle.h -- interface of the plain serial FP64 CPU oracle for the fully
 * discrete multistep BSDE scheme (arXiv:1909.13560, Section 2.2 eq (20)-(21),
 * Section 3.1).
 *
 * TEST INFRASTRUCTURE ONLY: called by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg.  Independent of the GPU library: the two share
 * no header, source, table or helper.
 */
#ifndef BSDE_ORACLE_H
#define BSDE_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_MAX_L 64

enum { ORACLE_OK = 0, ORACLE_EINVAL = 1, ORACLE_ENOMEM = 2, ORACLE_EINTERNAL = 3 };

enum {
    ORACLE_DRIVER_LINEAR = 0, /* p = {a, b1, b2, c}: f = a y + b1 z1 + b2 z2 + c      */
    ORACLE_DRIVER_BIDASK = 1, /* p = {r, R, theta, sigma, s}:                          */
                              /*   f = -r y - theta z + s (R - r) min(y - z/sigma, 0) */
    ORACLE_DRIVER_CUBIC = 2,  /* Example 1, eq (22): f = -y^3 + 5/2 y^2 - 3/2 y        */
    ORACLE_DRIVER_EXP = 3     /* Example 2, eq (24)                                    */
};

typedef struct {
    int d;              /* space dimension, 1 or 2                                  */
    double T;           /* terminal time                                            */
    int n_t;            /* number of time steps N, dt = T/N                          */
    int k_y, k_z;       /* multistep orders, 1..6                                   */
    int L;              /* Gauss-Hermite points per axis                            */
    int n_x[2];         /* grid points per axis (>= 4)                              */
    double x_min[2], x_max[2];
    double drift[2];    /* X_{t+h} = X_t + drift h + vol (W_{t+h} - W_t)            */
    double vol[2][2];   /* row-major; d = 1 uses vol[0][0]                          */
    double drift_x;     /* d = 1: state-dependent coefficients of eq (1),           */
    double vol_x;       /*   a(x) = drift[0] + drift_x x, b(x) = vol[0][0] + vol_x x */
                        /*   (Euler step over each horizon j dt); 0, 0: constant    */
    int driver;         /* ORACLE_DRIVER_*                                          */
    double p[8];        /* driver parameters                                        */
    int picard_max;     /* Picard iterations (fixed count when picard_tol <= 0)     */
    double picard_tol;  /* stop when |dy| <= tol * max(1, |y|); <= 0: fixed count   */
    int n_stop;         /* last layer computed; 0 is the full backward sweep        */
    int z_form;         /* first term of the z equation: 0 = E[z^{n+1}] as in       */
                        /* eq (20); 1 = E[y^{n+1} dW_{n+1}] / dt, the form before   */
                        /* the relation below eq (12) replaces it                   */
    int quad;           /* conditional expectations: 0 = Gauss-Hermite, eq (21);     */
                        /* 1 = exact Gaussian expectation of the interpolating      */
                        /* spline (d = 1, linear driver, constant coefficients)     */
    int interp2;        /* d = 2 interpolation: 0 = tensor natural spline; 1 =       */
                        /* bicubic from values, first and mixed derivatives by      */
                        /* fourth-order finite differences (Section 3.3)            */
    const double *coef_tab; /* d = 1, optional: a(t, x_i) and b(t, x_i) tabulated  */
                        /* on the grid, 2 * tab_steps * n_x[0] doubles; row s has  */
                        /* a at [2 s n_x + i], b > 0 at [(2 s + 1) n_x + i]; the   */
                        /* Euler step from t_n uses row n (tab_steps = n_t) or    */
                        /* row 0 (tab_steps = 1); drift[0], vol[0][0] unused and  */
                        /* drift_x = vol_x = 0.  NULL with tab_steps = 0.          */
    int tab_steps;
} oracle_problem;

typedef struct {
    int picard_iter_max;
    long picard_nonconverged;
} oracle_stats;

/* init_y: K layers x grid points, init_y[r] is the layer at t_{N-K+1+r},
 * r = 0..K-1 (the last one is the terminal layer), K = max(k_y, k_z).
 * init_z: same, d components per point, stored component-major per layer
 * (layer r: z1 over the grid, then z2).  y_out / z_out receive layer n_stop. */
int oracle_solve(const oracle_problem *pb, const double *init_y, const double *init_z,
                 double *y_out, double *z_out, oracle_stats *st);

/* d = 2 only: the first backward step (layer N-K) at the m grid points
 * idx[q] = i0 * n_x[1] + i1, from the K initial layers, with the same
 * arithmetic as oracle_solve.  y_out[q]; z_out[2q], z_out[2q+1] = z1, z2.
 * For checks at grid sizes where a whole step is too slow. */
int oracle_first_step_points_2d(const oracle_problem *pb, const double *init_y,
                                const double *init_z, int m, const long *idx, double *y_out,
                                double *z_out);

/* Section 3.1 step 2: rows 0..K-2 of init_y / init_z (t_{N-K+1}..t_{N-1})
 * from row K-1 (the terminal layer) by the 1-step scheme (K_y = K_z = 1 of
 * eq (20)) with `sub` steps per dt. */
int oracle_initial_layers(const oracle_problem *pb, int sub, double *init_y, double *init_z);

/* Exact Gaussian expectations of the natural splines of y and z (n points on
 * [xmin, xmax], boundary values outside) at X = c[k] + sd xi, xi ~ N(0, 1):
 * out[4k..4k+3] = E[yhat], E[yhat h xi], E[zhat], E[zhat h xi]. */
int oracle_exact_expectation(int n, double xmin, double xmax, const double *y, const double *z,
                             int m, const double *c, double sd, double h, double *out);

/* Gauss-Hermite nodes a[0..L-1] and weights w[0..L-1] for exp(-x^2). */
int oracle_gauss_hermite(int L, double *a, double *w);

/* table = 1: Table 1 row K (K+1 entries); table = 2: Table 2 row K. */
int oracle_gamma(int table, int K, double *g);

/* Natural cubic spline through y on n uniform points of [xmin, xmax],
 * evaluated at X[0..m-1] with boundary values outside the interval. */
int oracle_spline_eval(int n, double xmin, double xmax, const double *y, int m,
                       const double *X, double *out);

#ifdef __cplusplus
}
#endif
#endif

// plan_math.h -- host-side constants of the multistep scheme: Gauss-Hermite
// rule (eq (21)) and spline quadrature coefficients (Tables 1 and 2).
#pragma once

#include <vector>

namespace bsde {

constexpr int kMaxL = 64;
constexpr int kMaxK = 6;

// L-point Gauss-Hermite rule for exp(-x^2): ascending nodes a[], weights w[]
// (sum sqrt(pi)).  false for L outside [1, kMaxL] or a non-converging QL.
bool gauss_hermite(int L, double *a, double *w);

// n-point Gauss-Legendre rule on [0, 1] (nodes ascending, weights sum 1);
// false for n outside [1, kMaxL].
bool gauss_legendre01(int n, double *x, double *w);

// The exact Gaussian expectation of the natural spline of a layer as a
// banded Toeplitz operator on the uniform grid.  A node X = x_i + s dx with
// s = m0 + rho xi, xi ~ N(0, 1) (m0 = drift j dt / dx, rho = vol sqrt(j dt) /
// dx); the spline value on cell d (records i+d, i+d+1) at fraction theta is
// (1-theta) v0 + theta v1 + C(theta) M0 + D(theta) M1.  Then
//   E[v(X)]         = sum_k ev[k] v_{i+klo+k} + em[k] M_{i+klo+k},
//   E[v(X) h xi]    = sum_k wv[k] v_{i+klo+k} + wm[k] M_{i+klo+k}
// over k = 0 .. nb-1, with the records outside the grid holding the boundary
// value and M = 0 (so the mass outside the truncated domain goes to the
// boundary values).  Cells more than 9 rho + 1 from m0 are left out (mass
// below 1e-18).
struct GaussBand {
    int klo = 0;
    std::vector<double> ev, em, wv, wm;
};
bool gaussian_spline_band(double m0, double rho, double h, double dx, GaussBand &out);

// table 1: gamma^K_{K,j} (integral over K steps / (K dt)); table 2:
// gamma^1_{K,j} (integral over the first step / dt); K+1 values into g.
bool spline_gamma(int table, int K, double *g);

}  // namespace bsde

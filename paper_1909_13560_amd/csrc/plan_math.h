// plan_math.h -- host-side constants of the multistep scheme: Gauss-Hermite
// rule (eq (21)) and spline quadrature coefficients (Tables 1 and 2).
#pragma once

namespace bsde {

constexpr int kMaxL = 64;
constexpr int kMaxK = 6;

// L-point Gauss-Hermite rule for exp(-x^2): ascending nodes a[], weights w[]
// (sum sqrt(pi)).  false for L outside [1, kMaxL] or a non-converging QL.
bool gauss_hermite(int L, double *a, double *w);

// table 1: gamma^K_{K,j} (integral over K steps / (K dt)); table 2:
// gamma^1_{K,j} (integral over the first step / dt); K+1 values into g.
bool spline_gamma(int table, int K, double *g);

}  // namespace bsde

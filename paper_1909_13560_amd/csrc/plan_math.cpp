// plan_math.cpp -- host-side constants of the multistep scheme
// (arXiv:1909.13560): the Gauss-Hermite rule of eq (21) and the spline
// quadrature coefficients of Tables 1 and 2 (Section 2.1).  Pure C++, no HIP.
#include <algorithm>
#include <cmath>
#include <vector>

#include "plan_math.h"

namespace bsde {

// Gauss-Hermite rule for the weight exp(-x^2) by Golub-Welsch: the nodes are
// the eigenvalues of the symmetric Jacobi matrix of the monic Hermite
// recurrence p_{k+1} = x p_k - (k/2) p_{k-1} (zero diagonal, off-diagonal
// sqrt(k/2)), and each weight is sqrt(pi) times the squared first component
// of the normalised eigenvector.  The eigenproblem is solved by implicit QL
// sweeps with Wilkinson shifts, carrying only the first row of the
// eigenvector matrix.
namespace {

// Eigenvalues d of the symmetric tridiagonal matrix (diagonal d, off-diagonal
// e[0..L-2]) and the first components v of its normalised eigenvectors
// (v = e_1 on entry): implicit QL sweeps with Wilkinson shifts that rotate
// only the first row of the eigenvector matrix.
bool tridiag_eig_first_row(std::vector<double> &d, std::vector<double> &e, std::vector<double> &v)
{
    const int L = (int)d.size();
    const double eps = 2.220446049250313e-16;
    for (int l = 0; l < L; ++l) {
        for (int iter = 0;; ++iter) {
            int m = l;
            for (; m + 1 < L; ++m) {
                double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= eps * dd) break;
            }
            if (m == l) break;
            if (iter > 100) return false;
            // Wilkinson shift from the leading 2x2 block
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            bool deflated = false;
            for (int i = m - 1; i >= l; --i) {
                double f = s * e[i], b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {  // split: an exact zero appeared
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    deflated = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                // rotate the first row of the eigenvector matrix
                double t = v[i + 1];
                v[i + 1] = s * v[i] + c * t;
                v[i] = c * v[i] - s * t;
            }
            if (deflated) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    return true;
}

}  // namespace

bool gauss_hermite(int L, double *a, double *w)
{
    if (L < 1 || L > kMaxL) return false;
    std::vector<double> d(L, 0.0), e(L, 0.0), v(L, 0.0);
    for (int k = 0; k + 1 < L; ++k) e[k] = std::sqrt(0.5 * (k + 1));
    v[0] = 1.0;
    if (!tridiag_eig_first_row(d, e, v)) return false;
    std::vector<int> idx(L);
    for (int i = 0; i < L; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
    const double sqrt_pi = 1.7724538509055160273;
    for (int i = 0; i < L; ++i) {
        a[i] = d[idx[i]];
        w[i] = sqrt_pi * v[idx[i]] * v[idx[i]];
    }
    // exact symmetry of the rule: a_i = -a_{L-1-i}, w_i = w_{L-1-i}
    for (int i = 0; i < L / 2; ++i) {
        double aa = 0.5 * (a[L - 1 - i] - a[i]);
        double ww = 0.5 * (w[i] + w[L - 1 - i]);
        a[i] = -aa;
        a[L - 1 - i] = aa;
        w[i] = w[L - 1 - i] = ww;
    }
    if (L % 2 == 1) a[L / 2] = 0.0;
    return true;
}

// Quadrature weights of the not-a-knot cubic spline through K+1 unit-spaced
// points (the construction behind Tables 1 and 2): for each cardinal data
// vector e_j the spline is built in second-derivative form,
//   M_{i-1} + 4 M_i + M_{i+1} = 6 (y_{i+1} - 2 y_i + y_{i-1}),  i = 1..K-1,
// closed by continuity of the third derivative at knots 1 and K-1; with two
// or three points the spline is the line or parabola through them.  On a unit
// cell the spline integrates to (y_i + y_{i+1})/2 - (M_i + M_{i+1})/24.
bool spline_gamma(int table, int K, double *g)
{
    if ((table != 1 && table != 2) || K < 1 || K > 6) return false;
    const int n = K + 1;
    for (int j = 0; j < n; ++j) {
        double y[7] = {0}, M[7] = {0};
        y[j] = 1.0;
        if (K == 2) {
            double c = y[0] - 2.0 * y[1] + y[2];
            M[0] = M[1] = M[2] = c;
        } else if (K >= 3) {
            double A[7][8] = {{0}};
            int row = 0;
            for (int i = 1; i < K; ++i, ++row) {
                A[row][i - 1] = 1.0;
                A[row][i] = 4.0;
                A[row][i + 1] = 1.0;
                A[row][n] = 6.0 * (y[i + 1] - 2.0 * y[i] + y[i - 1]);
            }
            const int knots[2] = {1, K - 1};
            for (int q = 0; q < 2; ++q, ++row) {
                int k = knots[q];
                A[row][k - 1] = 1.0;
                A[row][k] = -2.0;
                A[row][k + 1] = 1.0;
            }
            // Gaussian elimination with partial pivoting on the n x n system
            for (int c = 0; c < n; ++c) {
                int piv = c;
                for (int r = c + 1; r < n; ++r)
                    if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
                if (A[piv][c] == 0.0) return false;
                if (piv != c)
                    for (int q = 0; q <= n; ++q) std::swap(A[c][q], A[piv][q]);
                for (int r = 0; r < n; ++r) {
                    if (r == c || A[r][c] == 0.0) continue;
                    double f = A[r][c] / A[c][c];
                    for (int q = c; q <= n; ++q) A[r][q] -= f * A[c][q];
                }
            }
            for (int i = 0; i < n; ++i) M[i] = A[i][n] / A[i][i];
        }
        double first = 0.0, total = 0.0;
        for (int i = 0; i < K; ++i) {
            double cell = 0.5 * (y[i] + y[i + 1]) - (M[i] + M[i + 1]) / 24.0;
            if (i == 0) first = cell;
            total += cell;
        }
        g[j] = table == 1 ? total / K : first;
    }
    return true;
}

// Gauss-Legendre on [-1, 1] by Golub-Welsch (monic recurrence
// p_{k+1} = x p_k - k^2/(4k^2 - 1) p_{k-1}: zero diagonal, off-diagonal
// k / sqrt(4k^2 - 1), weights 2 v_1^2), mapped to [0, 1].
bool gauss_legendre01(int n, double *x, double *w)
{
    if (n < 1 || n > kMaxL) return false;
    std::vector<double> d(n, 0.0), e(n, 0.0), v(n, 0.0);
    for (int k = 1; k < n; ++k) e[k - 1] = k / std::sqrt(4.0 * k * k - 1.0);
    v[0] = 1.0;
    if (!tridiag_eig_first_row(d, e, v)) return false;
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
    for (int i = 0; i < n; ++i) {
        x[i] = 0.5 * (d[idx[i]] + 1.0);
        w[i] = v[idx[i]] * v[idx[i]];  // 2 v^2 on [-1, 1], halved
    }
    return true;
}

bool gaussian_spline_band(double m0, double rho, double h, double dx, GaussBand &out)
{
    if (!(rho > 0.0) || !std::isfinite(m0) || !std::isfinite(rho)) return false;
    constexpr int kGl = 8;  // exact to degree 15 on each sub-interval
    double gx[kGl], gw[kGl];
    if (!gauss_legendre01(kGl, gx, gw)) return false;
    const double reach = 9.0 * rho + 1.0;
    if (!(reach < 1e7)) return false;
    const int dlo = (int)std::floor(m0 - reach), dhi = (int)std::ceil(m0 + reach);
    // sub-intervals of at most rho / 8 in cell units: the Gaussian changes
    // little over each, the cubic basis times it is integrated to rounding
    const int nsub = std::max(1, (int)std::ceil(8.0 / rho));
    const int nb = dhi - dlo + 2;  // records dlo .. dhi + 1
    out.klo = dlo;
    out.ev.assign(nb, 0.0);
    out.em.assign(nb, 0.0);
    out.wv.assign(nb, 0.0);
    out.wm.assign(nb, 0.0);
    const double inv_sqrt_2pi = 0.39894228040143267794, dx26 = dx * dx / 6.0;
    for (int dd = dlo; dd <= dhi; ++dd) {
        double I[4] = {0, 0, 0, 0}, J[4] = {0, 0, 0, 0};
        for (int q = 0; q < nsub; ++q)
            for (int g = 0; g < kGl; ++g) {
                const double th = (q + gx[g]) / nsub;
                const double xi = (dd + th - m0) / rho;
                const double dens = gw[g] / nsub * inv_sqrt_2pi * std::exp(-0.5 * xi * xi) / rho;
                const double u = 1.0 - th;
                const double b[4] = {u, th, dx26 * (u * u * u - u), dx26 * (th * th * th - th)};
                for (int k = 0; k < 4; ++k) {
                    I[k] += dens * b[k];
                    J[k] += dens * b[k] * h * xi;
                }
            }
        const int k0 = dd - dlo;  // left record of the cell; the right one is k0 + 1
        out.ev[k0] += I[0];
        out.ev[k0 + 1] += I[1];
        out.em[k0] += I[2];
        out.em[k0 + 1] += I[3];
        out.wv[k0] += J[0];
        out.wv[k0 + 1] += J[1];
        out.wm[k0] += J[2];
        out.wm[k0 + 1] += J[3];
    }
    return true;
}

}  // namespace bsde

// sweep2d.h -- data layout and launchers of the two-dimensional sweep
// (arXiv:1909.13560, eq (20)-(21) on a tensor grid, Section 5 Examples 4-5).
//
// A time layer is 12 planes of padded n0 x n1 elements: for each of y, z1, z2
// the value v and the tensor natural-spline derivatives M_xx (along axis 0),
// M_yy (along axis 1) and M_xxyy.  The elements are doubles, or floats in the
// FP32 form, whose layers add three planes (12, 13, 14) of the rounding
// residuals of y, z1 and z2 (error feedback, as in the 1-D form).  Plane p
// of slot s starts at element (P s + p) * plane of the ring (P = 12 or 15);
// point (i0, i1) sits at
// (i0 + pad0) * npad1 + (i1 + pad1).  Ghost points outside the grid hold the
// boundary data that makes the tensor spline evaluate at the clamped
// coordinates: beyond an axis-0 edge {v, 0, M_yy, 0} of the edge row, beyond
// an axis-1 edge {v, M_xx, 0, 0} of the edge column, beyond both {v, 0, 0, 0}.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"

namespace bsde {

constexpr int kTile2R = 1;    // tile rows (axis 0)
constexpr int kTile2C = 512;  // tile columns (axis 1)
constexpr int kCols2 = 2;     // adjacent columns per lane: their nodes share (U, V) records
constexpr int kThreads2 = kTile2R * kTile2C / kCols2;  // threads of a sweep2d block
constexpr int kWaves2 = kThreads2 / 64;            // wavefronts per block (statistics slots)
static_assert((kTile2C / kCols2) % 64 == 0 && kThreads2 <= 1024, "whole wavefronts per row");
constexpr int kMaxReach2d = 240;  // widest axis-1 node spread of one axis-0 node row
constexpr int kWin2 = kTile2C + kMaxReach2d + 2;  // widest LDS window columns
// LDS window of the sweep: per tile row, the even window columns, then the
// odd ones, each column a slot of the (U, V) records of the 3 functions
// (48 bytes).  A lane's two columns are adjacent, so its node records e, e+1,
// e+2 are two of one parity and one of the other, and the lanes of a
// wavefront read slots 48 bytes apart: 16 consecutive lanes cover all 64
// banks once (48 bytes = 12 banks, 12 and 64 share only the factor 4).
constexpr int kPcrTaps = 2 * (1 + 2 + 4 + 8 + 16) + 1;  // 63: reach of the truncated PCR

// Per (j, l0): the axis-0 offset of the node row and its spline weights, and
// the range of axis-1 offsets over l1.
struct Node2Row {
    int m0, m1lo, m1hi, pad;
    double B0, C0, D0;
};

// Per (j, l0, l1): axis-1 spline weights and the folded quadrature weights.
struct alignas(16) Node2 {
    double B1, C1, D1;
    double cfy, cfz1, cfz2, cz, cy;
    double cyz1, cyz2;  // weights of y-hat in z1^n, z2^n (z form E[y dW]/dt, j = 1)
};

// Natural-spline second derivatives by the truncated PCR written as a
// filter: M_i = s6 * sum_k c[k + 31] r~_{i+k} (r~ the odd extension of the
// second differences), or for 32 <= i <= n - 33 directly from the values:
// M_i = s6 * sum_k d[k + 32] v_{i+k}.  c and d are spline_taps(); lines of
// at least kMinLine points use d throughout, on values reflected through the
// line's end points.
struct SplineFilter {
    double c[kPcrTaps];
    double d[kPcrTaps + 2];
    double s6[2];  // 6 / dx^2 / b_5 of axis 0, axis 1
};
constexpr int kMinLine = kPcrTaps / 2 + 2;  // 33: one reflection covers the filter's reach

// The truncated PCR of the (1, 4, 1) system as line filters, constants of
// the system evaluated at compile time: c[k + 31] acts on the odd extension
// of the second differences, d[k + 32] on the values (the second difference
// folded in: d_m = c_{m-1} - 2 c_m + c_{m+1}).
struct SplineTaps {
    double c[kPcrTaps];
    double d[kPcrTaps + 2];
};
__host__ __device__ constexpr SplineTaps spline_taps()
{
    SplineTaps t{};
    double kap[kPcrRounds] = {};
    double av = 1.0, bv = 4.0;
    for (int r = 0; r < kPcrRounds; ++r) {  // a' = -a^2/b, b' = b - 2a^2/b
        kap[r] = av / bv;
        bv = bv - 2.0 * kap[r] * av;
        av = -kap[r] * av;
    }
    constexpr int T = kPcrTaps, H = T / 2;
    double cur[T] = {}, nxt[T] = {};
    cur[H] = 1.0;
    for (int r = 0, h = 1; r < kPcrRounds; ++r, h *= 2) {  // the rounds on a unit impulse
        for (int k = 0; k < T; ++k) {
            const double lo = k - h >= 0 ? cur[k - h] : 0.0, hi = k + h < T ? cur[k + h] : 0.0;
            nxt[k] = cur[k] - kap[r] * (lo + hi);
        }
        for (int k = 0; k < T; ++k) cur[k] = nxt[k];
    }
    for (int k = 0; k < T; ++k) t.c[k] = cur[k];
    for (int m = -H - 1; m <= H + 1; ++m) {
        const double cm = (m - 1 >= -H && m - 1 <= H) ? cur[m - 1 + H] : 0.0;
        const double c0 = (m >= -H && m <= H) ? cur[m + H] : 0.0;
        const double cp = (m + 1 >= -H && m + 1 <= H) ? cur[m + 1 + H] : 0.0;
        t.d[m + H + 1] = cm - 2.0 * c0 + cp;
    }
    return t;
}

struct Sweep2Args {
    char *ring;             // K+1 slots of kPlanes2<E> planes of E (double or float)
    size_t plane;
    int n0, n1, npad1, pad0, pad1;
    int K, Ky, L, n, n_stop;
    const Node2Row *rows;   // K*L
    const Node2 *nodes;     // K*L*L
    const int *m1;          // K*L*L
    DriverParams drv;
    double dt, h0;
    int picard_max;
    double picard_tol;
    int zform;              // first term of the z equation: 0 E[z^{n+1}], 1 E[y^{n+1} dW]/dt
    int interp;             // bsde_interp: the natural spline or the bicubic
    int half;               // LDS window columns of one parity: ceil(widest window / 2)
    double *fin;            // layer n_stop: y, z1, z2 planes of n0*n1
    unsigned int *st_iter_max;
    unsigned long long *st_iter_sum, *st_nonconv;
};

// Planes of a ring slot and the typed address of plane p of slot `slot`.
template <typename E>
constexpr int kPlanes2 = std::is_same<E, float>::value ? 15 : 12;
template <typename E>
__host__ __device__ inline E *plane2(const Sweep2Args &a, int slot, int p)
{
    return reinterpret_cast<E *>(a.ring) + (size_t)(kPlanes2<E> * slot + p) * a.plane;
}

// The launchers take the element type of the ring planes: f32 = the FP32
// form (float planes, residual planes), else double.
size_t sweep2d_lds(int half);  // dynamic LDS of the sweep kernel
hipError_t launch_sweep2d(bool f32, const Sweep2Args &a, hipStream_t s);
// splines and ghosts of the layer in slot `slot`
hipError_t launch_spline2d(bool f32, const Sweep2Args &a, int slot, const SplineFilter &f,
                           hipStream_t s);
// the paper's bicubic interpolation: derivatives by fourth-order finite
// differences (into the three derivative planes) and ghosts of slot `slot`
hipError_t launch_fd2d(bool f32, const Sweep2Args &a, int slot, double dx0, double dx1,
                       hipStream_t s);
// layer r = 0..K-1 of init_y (K x n0 n1) and init_z (K x 2 x n0 n1) into the ring
hipError_t launch_scatter2d(bool f32, const Sweep2Args &a, const double *iy, const double *iz,
                            hipStream_t s);
// layers n_stop .. n_stop + K - 1 into the initial-layer layout
hipError_t launch_export2d(bool f32, const Sweep2Args &a, double *ly, double *lz, hipStream_t s);
hipError_t launch_gather2d(const Sweep2Args &a, double *y0, double *z0,
                           unsigned long long *nonfinite, hipStream_t s);

}  // namespace bsde

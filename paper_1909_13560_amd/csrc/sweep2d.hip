// sweep2d.hip -- the backward sweep on a two-dimensional tensor grid
// (arXiv:1909.13560, eq (20)-(21); Section 5, Examples 4 and 5).
//
// The expectations over the L x L tensor Gauss-Hermite nodes use the tensor
// natural spline of each layer.  Its 16-term evaluation at a node
// (i0 + s0, i1 + s1) is regrouped by axes:
//   U(q) = A0 v(p, q)    + B0 v(p+1, q)    + C0 Mxx(p, q)   + D0 Mxx(p+1, q)
//   V(q) = A0 Myy(p, q)  + B0 Myy(p+1, q)  + C0 Mxxyy(p, q) + D0 Mxxyy(p+1, q)
//   S    = A1 U(q) + B1 U(q+1) + C1 V(q) + D1 V(q+1)      (p = i0 + m0, q = i1 + m1)
// With X = x + drift t + vol W and vol lower triangular, the axis-0 offset
// s0 depends on the axis-0 Gauss-Hermite index l0 only, so for one l0 the
// block evaluates (U, V) once per (tile row, window column) into LDS and
// every node l1 of that row costs one axis-1 evaluation per function.
#include "sweep2d.h"

namespace bsde {

namespace {

__device__ inline double f_linear2(const DriverParams &p, double y, double z1, double z2)
{
    return fma(p.p0, y, fma(p.p1, z1, fma(p.p2, z2, p.p3)));
}

__device__ inline size_t pidx(const Sweep2Args &a, int i0, int i1)
{
    return (size_t)(i0 + a.pad0) * a.npad1 + (size_t)(i1 + a.pad1);
}

// (U, V) of function f, tile row rr, window column cc in the LDS window:
// column slots of 3 functions, the even columns of a row first.
__device__ inline int uv_index(int half, int f, int rr, int cc)
{
    return ((rr * 2 + (cc & 1)) * half + (cc >> 1)) * 3 + f;
}

// Node record through the constant address space: the address is the same
// for the whole wavefront, so this compiles to scalar loads into SGPRs.
__device__ inline Node2 load_node2(const Node2 *p)
{
    const __attribute__((address_space(4))) Node2 *q =
        (const __attribute__((address_space(4))) Node2 *)p;
    Node2 n;
    n.B1 = q->B1;
    n.C1 = q->C1;
    n.D1 = q->D1;
    n.cfy = q->cfy;
    n.cfz1 = q->cfz1;
    n.cfz2 = q->cfz2;
    n.cz = q->cz;
    n.cy = q->cy;
    n.cyz1 = q->cyz1;
    n.cyz2 = q->cyz2;
    return n;
}

// Node flags: bit 0 the y expectation (layer j = K_y), bit 1 the y-hat terms
// of z^n (layer j = 1 of the z form E[y^{n+1} dW]/dt).
// CLAMP: the node's axis-1 cell q may leave the grid, and a cell that does not
// lie inside it evaluates to the value at its first point (the nearest grid
// line: the ghost records hold it), i.e. the interpolant at the coordinate
// clamped to the box.  The natural spline gets that from its ghost records
// alone (its second derivatives vanish at the ends); the bicubic's first
// derivatives do not, so its weights B1, C1, D1 are dropped there.
// A lane holds kCols2 = 2 adjacent columns c, c+1 (c even): the node of the
// second sits one record further, so the two read three (U, V) records per
// function, not four: window columns c+s, c+s+1, c+s+2, i.e. column slots
// c/2 + (s >> 1) and c/2 + (s >> 1) + 1 of the parity of s and one slot of
// the other parity (s, the node's window offset, is wavefront-uniform).
static_assert(kCols2 == 2, "the parity-split window serves two columns per lane");
template <int NF, bool CLAMP>
__device__ inline void node2_accumulate(const Sweep2Args &a, const double2 *uvl, const Node2 &nd,
                                        int s, int q, double (&Y)[kCols2],
                                        double (&Z1)[kCols2], double (&Z2)[kCols2])
// uvl: function 0 of the lane's column slot c/2 (even half of its tile row)
{
    const int h0 = ((s & 1) * a.half + (s >> 1)) * 3;              // records 0 and 2
    const int h1 = (((s + 1) & 1) * a.half + ((s + 1) >> 1)) * 3;  // record 1
    double2 p[3][kCols2 + 1];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        p[f][0] = uvl[h0 + f];
        p[f][1] = uvl[h1 + f];
        p[f][2] = uvl[h0 + 3 + f];
    }
#pragma unroll
    for (int k = 0; k < kCols2; ++k) {
        double B1 = nd.B1, C1 = nd.C1, D1 = nd.D1;
        if (CLAMP && !(q + k >= 0 && q + k < a.n1 - 1)) B1 = C1 = D1 = 0.0;
        double h[3];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const double2 p0 = p[f][k], p1 = p[f][k + 1];
            h[f] = fma(B1, p1.x - p0.x, fma(C1, p0.y, fma(D1, p1.y, p0.x)));
        }
        const double fh = f_linear2(a.drv, h[0], h[1], h[2]);
        Y[k] = fma(nd.cfy, fh, Y[k]);
        if (NF & 1) Y[k] = fma(nd.cy, h[0], Y[k]);
        Z1[k] = fma(nd.cfz1, fh, fma(nd.cz, h[1], Z1[k]));
        Z2[k] = fma(nd.cfz2, fh, fma(nd.cz, h[2], Z2[k]));
        if (NF & 2) {
            Z1[k] = fma(nd.cyz1, h[0], Z1[k]);
            Z2[k] = fma(nd.cyz2, h[0], Z2[k]);
        }
    }
}

// The L nodes l1 of one axis-0 row of layer j, for the lane's points.  The
// node records come through scalar loads and the axis-1 offsets, one per
// lane in mv, through readlane, so the only per-node LDS reads are the
// (U, V) records; two nodes per iteration share one wait.
// uvl: the lane's slot in the window (see node2_accumulate), i1 its first
// grid column, so that a node's window offset is s = m1 - m1lo and its
// axis-1 cell q = m1 + i1.
template <int NF, bool CLAMP>
__device__ inline void row_nodes(const Sweep2Args &a, const double2 *uvl, const Node2 *ntab,
                                 int mv, int m1lo, int i1, double (&Y)[kCols2],
                                 double (&Z1)[kCols2], double (&Z2)[kCols2])
{
    int l1 = 0;
#pragma unroll 1
    for (; l1 + 1 < a.L; l1 += 2) {
        const Node2 n0 = load_node2(ntab + l1), n1 = load_node2(ntab + l1 + 1);
        const int m0 = __builtin_amdgcn_readlane(mv, l1), m1 = __builtin_amdgcn_readlane(mv, l1 + 1);
        node2_accumulate<NF, CLAMP>(a, uvl, n0, m0 - m1lo, m0 + i1, Y, Z1, Z2);
        node2_accumulate<NF, CLAMP>(a, uvl, n1, m1 - m1lo, m1 + i1, Y, Z1, Z2);
    }
    if (l1 < a.L) {
        const Node2 n0 = load_node2(ntab + l1);
        const int m0 = __builtin_amdgcn_readlane(mv, l1);
        node2_accumulate<NF, CLAMP>(a, uvl, n0, m0 - m1lo, m0 + i1, Y, Z1, Z2);
    }
}

template <bool CLAMP>
__device__ inline void row_nodes_nf(int nf, const Sweep2Args &a, const double2 *uvl,
                                    const Node2 *ntab, int mv, int m1lo, int i1,
                                    double (&Y)[kCols2], double (&Z1)[kCols2], double (&Z2)[kCols2])
{
    if (nf == 0)
        row_nodes<0, CLAMP>(a, uvl, ntab, mv, m1lo, i1, Y, Z1, Z2);
    else if (nf == 1)
        row_nodes<1, CLAMP>(a, uvl, ntab, mv, m1lo, i1, Y, Z1, Z2);
    else if (nf == 2)
        row_nodes<2, CLAMP>(a, uvl, ntab, mv, m1lo, i1, Y, Z1, Z2);
    else
        row_nodes<3, CLAMP>(a, uvl, ntab, mv, m1lo, i1, Y, Z1, Z2);
}

}  // namespace

// The FP32 form stores a value as fl(v + e) with e the residual carried from
// the layer it was computed from, and keeps the new residual (as in 1-D).
__device__ inline void store_fed_back2(float *val, float *res, size_t o, double v, float e)
{
    const double t = v + (double)e;
    const float q = (float)t;
    val[o] = q;
    res[o] = (float)(t - (double)q);
}

// One time step: layer n from layers n+1..n+K.  Block = kTile2R x kTile2C points.
// Dynamic LDS: (U, V) of 3 functions x kTile2R rows x 2 a.half columns.  E: the
// element type of the ring planes; the arithmetic is double in both forms.
// The occupancy hint holds the kernel at 89 VGPRs (five waves per SIMD, no
// scratch); left to itself the compiler takes 131 (three waves) for the
// parity-split window addressing.
template <typename E>
__global__ void __launch_bounds__(kThreads2) __attribute__((amdgpu_waves_per_eu(4)))
sweep2d(const Sweep2Args a)
{
    extern __shared__ double2 uv[];
    const int tiles1 = (a.n1 + kTile2C - 1) / kTile2C;
    const int idx = xcd_tile(blockIdx.x, gridDim.x);
    const int t0 = (idx / tiles1) * kTile2R, t1 = (idx % tiles1) * kTile2C;
    const int tid = threadIdx.x;
    constexpr int kLanesRow = kTile2C / kCols2;  // lanes per tile row
    const int r = __builtin_amdgcn_readfirstlane(tid / kLanesRow), c = (tid % kLanesRow) * kCols2;
    const int S = a.K + 1;
    double Y[kCols2], Z1[kCols2], Z2[kCols2];
#pragma unroll
    for (int k = 0; k < kCols2; ++k) Y[k] = Z1[k] = Z2[k] = 0.0;
    for (int j = 1; j <= a.K; ++j) {
        const E *slot = plane2<E>(a, (a.n + j) % S, 0);
        for (int l0 = 0; l0 < a.L; ++l0) {
            const int rowi = (j - 1) * a.L + l0;
            const Node2Row row = a.rows[rowi];
            const int W = kTile2C + row.m1hi - row.m1lo + 2;
            // the row's axis-1 offsets, one per lane (L <= 64)
            const int mv = a.m1[(size_t)rowi * a.L + min(tid & 63, a.L - 1)];
            // axis-0 evaluation at s0 for the tile rows and the window columns
            for (int e = tid; e < kTile2R * W; e += kThreads2) {
                const int rr = e / W, cc = e - rr * W;
                const int p = t0 + rr + row.m0;  // the node's axis-0 cell
                const size_t o = pidx(a, p, t1 + row.m1lo + cc);
                const size_t o1 = o + a.npad1;
                // a cell outside the grid evaluates to its first point's record
                // (clamped coordinate; see node2_accumulate).  For the natural
                // spline this changes nothing: there both differences and both
                // second derivatives in such a cell are exact zeros.
                const bool in = p >= 0 && p < a.n0 - 1;
                const double B0 = in ? row.B0 : 0.0, C0 = in ? row.C0 : 0.0, D0 = in ? row.D0 : 0.0;
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const E *v = slot + (size_t)(4 * f) * a.plane;
                    const E *mxx = v + a.plane, *myy = v + 2 * a.plane, *mxy = v + 3 * a.plane;
                    const double v0 = v[o], y0 = myy[o];
                    const double U = fma(B0, (double)v[o1] - v0,
                                         fma(C0, (double)mxx[o], fma(D0, (double)mxx[o1], v0)));
                    const double V = fma(B0, (double)myy[o1] - y0,
                                         fma(C0, (double)mxy[o], fma(D0, (double)mxy[o1], y0)));
                    uv[uv_index(a.half, f, rr, cc)] = make_double2(U, V);
                }
            }
            __syncthreads();
            const Node2 *ntab = a.nodes + (size_t)rowi * a.L;
            const int nf = (j == a.Ky ? 1 : 0) | (j == 1 && a.zform ? 2 : 0);
            // the bicubic needs the per-node cell check only where the tile's
            // node cells can leave the grid along axis 1 (block-uniform)
            const bool clamp = a.interp == BSDE_INTERP_BICUBIC_FD &&
                               (t1 + row.m1lo < 0 || t1 + kTile2C + row.m1hi > a.n1 - 1);
            const double2 *uvl = uv + uv_index(a.half, 0, r, c);
            if (clamp)
                row_nodes_nf<true>(nf, a, uvl, ntab, mv, row.m1lo, t1 + c, Y, Z1, Z2);
            else
                row_nodes_nf<false>(nf, a, uvl, ntab, mv, row.m1lo, t1 + c, Y, Z1, Z2);
            __syncthreads();
        }
    }
    // implicit y equation by Picard iteration from y^{n+1}, per point of the lane
    const E *prev = plane2<E>(a, (a.n + 1) % S, 0);
    E *out = plane2<E>(a, a.n % S, 0);
    const int i0 = t0 + r;
    unsigned int it_max = 0, it_sum = 0, nonconv = 0;
#pragma unroll
    for (int k = 0; k < kCols2; ++k) {
        const int i1 = t1 + c + k;
        const bool valid = i0 < a.n0 && i1 < a.n1;
        const size_t o = pidx(a, min(i0, a.n0 - 1), min(i1, a.n1 - 1));
        double y = prev[o];
        int it = 0;
        bool conv = true;
        if (a.picard_tol > 0.0) {
            conv = false;
            while (it < a.picard_max) {
                const double yn = fma(a.h0, f_linear2(a.drv, y, Z1[k], Z2[k]), Y[k]);
                ++it;
                const double dy = fabs(yn - y);
                y = yn;
                if (dy <= a.picard_tol * fmax(1.0, fabs(y))) {
                    conv = true;
                    break;
                }
            }
        } else {
            for (; it < a.picard_max; ++it) y = fma(a.h0, f_linear2(a.drv, y, Z1[k], Z2[k]), Y[k]);
        }
        if (valid) {
            if constexpr (std::is_same<E, float>::value) {
                // residuals of y^{n+K_y} (y recurrence) and of z^{n+1} (z recurrence)
                const float *ry = plane2<float>(a, (a.n + a.Ky) % S, 12);
                const float *rz = plane2<float>(a, (a.n + 1) % S, 13);
                float *res = plane2<float>(a, a.n % S, 12);
                store_fed_back2(out, res, o, y, ry[o]);
                store_fed_back2(out + 4 * a.plane, res + a.plane, o, Z1[k], rz[o]);
                store_fed_back2(out + 8 * a.plane, res + 2 * a.plane, o, Z2[k], rz[o + a.plane]);
            } else {
                out[o] = y;
                out[o + 4 * a.plane] = Z1[k];
                out[o + 8 * a.plane] = Z2[k];
            }
            if (a.n == a.n_stop) {
                const size_t np = (size_t)a.n0 * a.n1, kk = (size_t)i0 * a.n1 + i1;
                a.fin[kk] = y;
                a.fin[np + kk] = Z1[k];
                a.fin[2 * np + kk] = Z2[k];
            }
            it_max = max(it_max, (unsigned int)it);
            it_sum += it;
            nonconv += conv ? 0u : 1u;
        }
    }
    if (a.st_iter_max) {
        it_max = wave_max_u32(it_max);
        it_sum = wave_sum_u32(it_sum);
        nonconv = wave_sum_u32(nonconv);
        if ((tid & 63) == 0) {
            const int w = idx * kWaves2 + tid / 64;
            a.st_iter_max[w] = max(a.st_iter_max[w], it_max);
            a.st_iter_sum[w] += it_sum;
            a.st_nonconv[w] += nonconv;
        }
    }
}

// ---------------------------------------------------------------------------
// Tensor natural spline of a layer: M_xx and M_yy of the values, then M_xxyy
// as the axis-1 spline of M_xx, then the ghost points.
// ---------------------------------------------------------------------------
namespace {

// second difference of line values at k, oddly extended about 0 and n-1
template <typename E>
__device__ inline double rt_line(const E *v, long stride, int n, int k)
{
    const int per = 2 * (n - 1);
    int kk = k % per;
    if (kk < 0) kk += per;
    double sign = 1.0;
    if (kk > n - 1) {
        kk = per - kk;
        sign = -1.0;
    }
    if (kk == 0 || kk == n - 1) return 0.0;
    const double vm = v[(long)(kk - 1) * stride], v0 = v[(long)kk * stride],
                 vp = v[(long)(kk + 1) * stride];  // the arithmetic is double
    return sign * ((vp - v0) - (v0 - vm));
}

template <typename E>
__device__ inline double spline_line(const E *v, long stride, int n, int i,
                                     const SplineFilter &F, double s6)
{
    if (i == 0 || i == n - 1) return 0.0;
    double acc = 0.0;
    if (i >= 32 && i <= n - 33) {
        const E *p = v + (long)(i - 32) * stride;
#pragma unroll
        for (int k = 0; k < kPcrTaps + 2; ++k) acc = fma(F.d[k], (double)p[(long)k * stride], acc);
    } else {
        for (int k = 0; k < kPcrTaps; ++k) acc = fma(F.c[k], rt_line(v, stride, n, i + k - 31), acc);
    }
    return s6 * acc;
}

constexpr int kRun = 16;  // consecutive outputs per thread of the line passes

// Outputs i0 .. i0 + kRun - 1 (those < n) of the natural spline of one line
// of n >= kMinLine values: M_i = s6 sum_k d[k] v~_{i-32+k}.  Each value is
// loaded once and feeds every output within the filter's reach.  Beyond the
// line's ends the values are reflected through the end points,
// v~_{-j} = 2 v_0 - v_j and v~_{n-1+j} = 2 v_{n-1} - v_{n-1-j}: their second
// differences are then the odd extension the natural end conditions call
// for, so the values form holds at every point; M_0 = M_{n-1} = 0.
template <typename E>
__device__ inline void line_run(const E *v, long stride, int n, int i0, double s6, E *out,
                                long ostride)
{
    constexpr SplineTaps T = spline_taps();
    constexpr int H = kPcrTaps / 2 + 1;  // values on each side of an output
    double acc[kRun];
#pragma unroll
    for (int r = 0; r < kRun; ++r) acc[r] = 0.0;
    if (i0 >= H && i0 + kRun - 1 + H <= n - 1) {  // clear of both ends
        const E *p = v + (long)(i0 - H) * stride;
#pragma unroll
        for (int m = 0; m < kRun + 2 * H; ++m) {
            const double x = p[(long)m * stride];
#pragma unroll
            for (int r = 0; r < kRun; ++r)
                if (m - r >= 0 && m - r <= 2 * H) acc[r] = fma(T.d[m - r], x, acc[r]);
        }
    } else {
        const double v0 = v[0], vn = v[(long)(n - 1) * stride];  // double arithmetic
#pragma unroll
        for (int m = 0; m < kRun + 2 * H; ++m) {
            const int k = i0 - H + m;
            // reflected index; clamped too for the loads of outputs past the
            // end of a partial run, which are not stored
            const int kk = min(max(k < 0 ? -k : (k > n - 1 ? 2 * (n - 1) - k : k), 0), n - 1);
            const double y = v[(long)kk * stride];
            const double x = k < 0 ? 2.0 * v0 - y : (k > n - 1 ? 2.0 * vn - y : y);
#pragma unroll
            for (int r = 0; r < kRun; ++r)
                if (m - r >= 0 && m - r <= 2 * H) acc[r] = fma(T.d[m - r], x, acc[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < kRun; ++r) {
        const int i = i0 + r;
        if (i < n) out[(long)i * ostride] = (E)((i == 0 || i == n - 1) ? 0.0 : s6 * acc[r]);
    }
}

// The same outputs for lines shorter than kMinLine, one at a time.
template <typename E>
__device__ inline void line_run_short(const E *v, long stride, int n, int i0,
                                      const SplineFilter &F, double s6, E *out, long ostride)
{
    for (int i = i0; i < min(i0 + kRun, n); ++i)
        out[(long)i * ostride] = (E)spline_line(v, stride, n, i, F, s6);
}

}  // namespace

// M_xx of field blockIdx.y (y, z1, z2): lines along axis 0.  Thread t:
// column t % n1 (adjacent lanes read adjacent columns), rows from
// kRun * (t / n1).
template <typename E>
__global__ void __launch_bounds__(256) spline2d_cols(const Sweep2Args a, int slot,
                                                     const SplineFilter F)
{
    const long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)a.n1 * ((a.n0 + kRun - 1) / kRun)) return;
    const int i1 = (int)(t % a.n1), i0 = (int)(t / a.n1) * kRun;
    E *col = plane2<E>(a, slot, 4 * blockIdx.y) + pidx(a, 0, i1);
    if (a.n0 >= kMinLine)
        line_run(col, a.npad1, a.n0, i0, F.s6[0], col + a.plane, a.npad1);
    else
        line_run_short(col, a.npad1, a.n0, i0, F, F.s6[0], col + a.plane, a.npad1);
}

// Lines along axis 1 of field blockIdx.y / 2: the values give M_yy
// (blockIdx.y even), M_xx gives M_xxyy (odd).  Thread t: row t % n0, columns
// from kRun * (t / n0), so that a wavefront takes one branch of line_run.
template <typename E>
__global__ void __launch_bounds__(256) spline2d_rows(const Sweep2Args a, int slot,
                                                     const SplineFilter F)
{
    const long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)a.n0 * ((a.n1 + kRun - 1) / kRun)) return;
    const int i0 = (int)(t % a.n0), i1 = (int)(t / a.n0) * kRun;
    const int f = blockIdx.y >> 1, g = blockIdx.y & 1;
    E *row = plane2<E>(a, slot, 4 * f) + pidx(a, i0, 0);
    const E *src = row + (size_t)g * a.plane;
    E *dst = row + (size_t)(2 + g) * a.plane;
    if (a.n1 >= kMinLine)
        line_run(src, 1, a.n1, i1, F.s6[1], dst, 1);
    else
        line_run_short(src, 1, a.n1, i1, F, F.s6[1], dst, 1);
}

// Lines along axis 1 of at least kMinLine points, through LDS: a block
// stages kRowTile rows x (kRowCols + 64) values of its source plane with
// coalesced loads (reflected through the line ends as in line_run), then each
// thread streams the 80 values of one run of kRun outputs from LDS.  Same
// arithmetic, in the same order, as line_run.
constexpr int kRowTile = 16;                   // rows per block
constexpr int kRowCols = 256 / kRowTile * kRun;  // outputs per row per block
constexpr int kRowIn = kRowCols + 2 * (kPcrTaps / 2 + 1);  // staged values per row
constexpr int kRowStride = kRowIn + 1;          // LDS row pitch (odd: fewer bank conflicts)

template <typename E>
__global__ void __launch_bounds__(256) spline2d_rows_lds(const Sweep2Args a, int slot,
                                                         const SplineFilter F)
{
    constexpr SplineTaps T = spline_taps();
    constexpr int H = kPcrTaps / 2 + 1;
    __shared__ double sm[kRowTile * kRowStride];
    const int tiles1 = (a.n1 + kRowCols - 1) / kRowCols;
    const int r0 = (int)(blockIdx.x / tiles1) * kRowTile, c0 = (int)(blockIdx.x % tiles1) * kRowCols;
    const int f = blockIdx.y >> 1, g = blockIdx.y & 1;
    const int n = a.n1;
    E *plane0 = plane2<E>(a, slot, 4 * f);
    const E *src = plane0 + (size_t)g * a.plane;
    E *dst = plane0 + (size_t)(2 + g) * a.plane;
    for (int e = threadIdx.x; e < kRowTile * kRowIn; e += 256) {
        const int rr = e / kRowIn, cc = e - rr * kRowIn;
        const int i0 = r0 + rr;
        if (i0 >= a.n0) continue;
        const E *v = src + pidx(a, i0, 0);
        const int k = c0 - H + cc;
        const int kk = min(max(k < 0 ? -k : (k > n - 1 ? 2 * (n - 1) - k : k), 0), n - 1);
        const double y = v[kk];
        sm[rr * kRowStride + cc] =
            k < 0 ? 2.0 * (double)v[0] - y : (k > n - 1 ? 2.0 * (double)v[n - 1] - y : y);
    }
    __syncthreads();
    const int r = threadIdx.x % kRowTile, q = threadIdx.x / kRowTile;
    const int i0 = r0 + r, j0 = c0 + q * kRun;
    if (i0 >= a.n0 || j0 >= n) return;
    const double *w = sm + r * kRowStride + q * kRun;
    double acc[kRun];
#pragma unroll
    for (int u = 0; u < kRun; ++u) acc[u] = 0.0;
#pragma unroll
    for (int m = 0; m < kRun + 2 * H; ++m) {
        const double x = w[m];
#pragma unroll
        for (int u = 0; u < kRun; ++u)
            if (m - u >= 0 && m - u <= 2 * H) acc[u] = fma(T.d[m - u], x, acc[u]);
    }
    E *out = dst + pidx(a, i0, 0);
    const double s6 = F.s6[1];
#pragma unroll
    for (int u = 0; u < kRun; ++u) {
        const int i = j0 + u;
        if (i < n) out[i] = (E)((i == 0 || i == n - 1) ? 0.0 : s6 * acc[u]);
    }
}

// The paper's own 2-D interpolation (Section 3.3): bicubic from the values
// and the first and mixed derivatives, the derivatives by fourth-order
// finite differences (central inside, one-sided at the two points next to
// each end).  They go into the planes of the tensor spline's second
// derivatives: f_x in M_xx, f_y in M_yy, f_xy in M_xxyy; the sweep kernel is
// the same, with the Hermite basis weights in the node tables.
template <typename E>
__device__ inline double fd4_at(const E *f, long st, int n, int i, double inv12h)
{
    double v;  // double arithmetic on the (possibly float) values
    if (i >= 2 && i <= n - 3)
        v = (double)f[(i - 2) * st] - 8.0 * f[(i - 1) * st] + 8.0 * f[(i + 1) * st] - f[(i + 2) * st];
    else if (i == 0)
        v = -25.0 * f[0] + 48.0 * f[st] - 36.0 * f[2 * st] + 16.0 * f[3 * st] - 3.0 * f[4 * st];
    else if (i == 1)
        v = -3.0 * f[0] - 10.0 * f[st] + 18.0 * f[2 * st] - 6.0 * f[3 * st] + f[4 * st];
    else if (i == n - 1)
        v = 25.0 * f[(n - 1) * st] - 48.0 * f[(n - 2) * st] + 36.0 * f[(n - 3) * st] -
            16.0 * f[(n - 4) * st] + 3.0 * f[(n - 5) * st];
    else
        v = 3.0 * f[(n - 1) * st] + 10.0 * f[(n - 2) * st] - 18.0 * f[(n - 3) * st] +
            6.0 * f[(n - 4) * st] - f[(n - 5) * st];
    return v * inv12h;
}

// f_x of field blockIdx.y along axis 0 (adjacent lanes on adjacent columns)
template <typename E>
__global__ void __launch_bounds__(256) fd2d_cols(const Sweep2Args a, int slot, double inv12h)
{
    const long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)a.n0 * a.n1) return;
    const int i0 = (int)(t / a.n1), i1 = (int)(t % a.n1);
    E *v = plane2<E>(a, slot, 4 * blockIdx.y);
    v[a.plane + pidx(a, i0, i1)] = (E)fd4_at(v + pidx(a, 0, i1), a.npad1, a.n0, i0, inv12h);
}

// Along axis 1 of field blockIdx.y / 2: f_y from the values (blockIdx.y
// even), f_xy from f_x (odd)
template <typename E>
__global__ void __launch_bounds__(256) fd2d_rows(const Sweep2Args a, int slot, double inv12h)
{
    const long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)a.n0 * a.n1) return;
    const int i0 = (int)(t / a.n1), i1 = (int)(t % a.n1);
    const int f = blockIdx.y >> 1, g = blockIdx.y & 1;
    E *v = plane2<E>(a, slot, 4 * f);
    const E *src = v + (size_t)g * a.plane;
    v[(size_t)(2 + g) * a.plane + pidx(a, i0, i1)] =
        (E)fd4_at(src + pidx(a, i0, 0), 1, a.n1, i1, inv12h);
}

// Ghost points: the data of the nearest grid point with the derivative
// planes across the crossed edge set to zero (clamped evaluation).
template <typename E>
__global__ void __launch_bounds__(256) ghosts2d(const Sweep2Args a, int slot, int npad0)
{
    const long i = blockIdx.x * 256L + threadIdx.x;
    if (i >= (long)npad0 * a.npad1) return;
    const int g0 = (int)(i / a.npad1) - a.pad0, g1 = (int)(i % a.npad1) - a.pad1;
    const bool in0 = g0 >= 0 && g0 < a.n0, in1 = g1 >= 0 && g1 < a.n1;
    if (in0 && in1) return;
    const size_t src = pidx(a, min(max(g0, 0), a.n0 - 1), min(max(g1, 0), a.n1 - 1));
    E *base = plane2<E>(a, slot, 0);
    for (int f = 0; f < 3; ++f) {
        E *v = base + (size_t)(4 * f) * a.plane;
        v[i] = v[src];
        v[a.plane + i] = in0 ? v[a.plane + src] : (E)0;
        v[2 * a.plane + i] = in1 ? v[2 * a.plane + src] : (E)0;
        v[3 * a.plane + i] = (E)0;
    }
}

template <typename E>
__global__ void __launch_bounds__(256) scatter2d(const Sweep2Args a, const double *__restrict__ iy,
                                                 const double *__restrict__ iz)
{
    const long np = (long)a.n0 * a.n1;
    const long i = blockIdx.x * 256L + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= np) return;
    const int n = a.n + 1 + r;  // a.n = N - K: layers N-K+1 .. N
    E *base = plane2<E>(a, n % (a.K + 1), 0);
    const size_t o = pidx(a, (int)(i / a.n1), (int)(i % a.n1));
    const double v[3] = {iy[r * np + i], iz[(2L * r) * np + i], iz[(2L * r + 1) * np + i]};
    for (int f = 0; f < 3; ++f) {
        if constexpr (std::is_same<E, float>::value) {  // value and its rounding residual
            store_fed_back2(base + 4 * f * a.plane, base + (12 + f) * a.plane, o, v[f], 0.0f);
        } else {
            base[4 * f * a.plane + o] = v[f];
        }
    }
}

__global__ void __launch_bounds__(256) gather2d(const Sweep2Args a, double *__restrict__ y0,
                                                double *__restrict__ z0,
                                                unsigned long long *nonfinite)
{
    const long np = (long)a.n0 * a.n1;
    unsigned int bad = 0;
    for (long i = blockIdx.x * 256L + threadIdx.x; i < np; i += (long)gridDim.x * 256) {
        const double y = a.fin[i], z1 = a.fin[np + i], z2 = a.fin[2 * np + i];
        y0[i] = y;
        z0[i] = z1;
        z0[np + i] = z2;
        bad += (isfinite(y) && isfinite(z1) && isfinite(z2)) ? 0u : 1u;
    }
    bad = wave_sum_u32(bad);
    if (nonfinite && (threadIdx.x & 63) == 0 && bad) atomicAdd(nonfinite, (unsigned long long)bad);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
size_t sweep2d_lds(int half) { return (size_t)3 * kTile2R * 2 * half * sizeof(double2); }

// Checkpoint export: layers n_stop .. n_stop + K - 1 into the initial-layer
// layout (y: K x n0 n1; z: K x 2 x n0 n1), the FP32 form as value plus residual.
template <typename E>
__global__ void __launch_bounds__(256) export2d(const Sweep2Args a, double *__restrict__ ly,
                                                double *__restrict__ lz)
{
    const long np = (long)a.n0 * a.n1;
    const long i = blockIdx.x * 256L + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= np) return;
    const int slot = (a.n_stop + r) % (a.K + 1);
    const E *base = plane2<E>(a, slot, 0);
    const size_t o = pidx(a, (int)(i / a.n1), (int)(i % a.n1));
    double v[3];
    for (int f = 0; f < 3; ++f) {
        v[f] = base[(size_t)(4 * f) * a.plane + o];
        if constexpr (std::is_same<E, float>::value) v[f] += (double)base[(size_t)(12 + f) * a.plane + o];
    }
    ly[r * np + i] = v[0];
    lz[(2L * r) * np + i] = v[1];
    lz[(2L * r + 1) * np + i] = v[2];
}

namespace {

template <typename E>
hipError_t launch_sweep2d_t(const Sweep2Args &a, hipStream_t s)
{
    const int tiles = ((a.n0 + kTile2R - 1) / kTile2R) * ((a.n1 + kTile2C - 1) / kTile2C);
    hipLaunchKernelGGL(sweep2d<E>, dim3(tiles), dim3(kThreads2), sweep2d_lds(a.half), s, a);
    return hipGetLastError();
}

template <typename E>
hipError_t launch_ghosts2d_t(const Sweep2Args &a, int slot, hipStream_t s)
{
    const int npad0 = (int)(a.plane / a.npad1);
    const int gb = (int)(((long)npad0 * a.npad1 + 255) / 256);
    hipLaunchKernelGGL(ghosts2d<E>, dim3(gb), dim3(256), 0, s, a, slot, npad0);
    return hipGetLastError();
}

template <typename E>
hipError_t launch_spline2d_t(const Sweep2Args &a, int slot, const SplineFilter &f, hipStream_t s)
{
    const long tc = (long)a.n1 * ((a.n0 + kRun - 1) / kRun);
    hipLaunchKernelGGL(spline2d_cols<E>, dim3((unsigned)((tc + 255) / 256), 3), dim3(256), 0, s, a,
                       slot, f);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.n1 >= kMinLine) {
        const long tiles = (long)((a.n0 + kRowTile - 1) / kRowTile) * ((a.n1 + kRowCols - 1) / kRowCols);
        hipLaunchKernelGGL(spline2d_rows_lds<E>, dim3((unsigned)tiles, 6), dim3(256), 0, s, a, slot,
                           f);
    } else {
        const long tr = (long)a.n0 * ((a.n1 + kRun - 1) / kRun);
        hipLaunchKernelGGL(spline2d_rows<E>, dim3((unsigned)((tr + 255) / 256), 6), dim3(256), 0, s,
                           a, slot, f);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_ghosts2d_t<E>(a, slot, s);
}

template <typename E>
hipError_t launch_fd2d_t(const Sweep2Args &a, int slot, double dx0, double dx1, hipStream_t s)
{
    const long np = (long)a.n0 * a.n1;
    const unsigned nb = (unsigned)((np + 255) / 256);
    hipLaunchKernelGGL(fd2d_cols<E>, dim3(nb, 3), dim3(256), 0, s, a, slot, 1.0 / (12.0 * dx0));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fd2d_rows<E>, dim3(nb, 6), dim3(256), 0, s, a, slot, 1.0 / (12.0 * dx1));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_ghosts2d_t<E>(a, slot, s);
}

template <typename E>
hipError_t launch_scatter2d_t(const Sweep2Args &a, const double *iy, const double *iz,
                              hipStream_t s)
{
    const long np = (long)a.n0 * a.n1;
    hipLaunchKernelGGL(scatter2d<E>, dim3((unsigned)((np + 255) / 256), a.K), dim3(256), 0, s, a,
                       iy, iz);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sweep2d(bool f32, const Sweep2Args &a, hipStream_t s)
{
    return f32 ? launch_sweep2d_t<float>(a, s) : launch_sweep2d_t<double>(a, s);
}

hipError_t launch_spline2d(bool f32, const Sweep2Args &a, int slot, const SplineFilter &f,
                           hipStream_t s)
{
    return f32 ? launch_spline2d_t<float>(a, slot, f, s) : launch_spline2d_t<double>(a, slot, f, s);
}

hipError_t launch_fd2d(bool f32, const Sweep2Args &a, int slot, double dx0, double dx1,
                       hipStream_t s)
{
    return f32 ? launch_fd2d_t<float>(a, slot, dx0, dx1, s)
               : launch_fd2d_t<double>(a, slot, dx0, dx1, s);
}

hipError_t launch_export2d(bool f32, const Sweep2Args &a, double *ly, double *lz, hipStream_t s)
{
    const long np = (long)a.n0 * a.n1;
    const dim3 grid((unsigned)((np + 255) / 256), (unsigned)a.K);
    if (f32)
        hipLaunchKernelGGL(export2d<float>, grid, dim3(256), 0, s, a, ly, lz);
    else
        hipLaunchKernelGGL(export2d<double>, grid, dim3(256), 0, s, a, ly, lz);
    return hipGetLastError();
}

hipError_t launch_scatter2d(bool f32, const Sweep2Args &a, const double *iy, const double *iz,
                            hipStream_t s)
{
    return f32 ? launch_scatter2d_t<float>(a, iy, iz, s) : launch_scatter2d_t<double>(a, iy, iz, s);
}

hipError_t launch_gather2d(const Sweep2Args &a, double *y0, double *z0,
                           unsigned long long *nonfinite, hipStream_t s)
{
    const long np = (long)a.n0 * a.n1;
    const int blocks = (int)std::min<long>(2048, (np + 255) / 256);
    hipLaunchKernelGGL(gather2d, dim3(blocks), dim3(256), 0, s, a, y0, z0, nonfinite);
    return hipGetLastError();
}

}  // namespace bsde

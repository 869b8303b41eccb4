// device_common.h -- data layout, drivers and shared device helpers of the
// backward sweep of the multistep BSDE scheme (arXiv:1909.13560).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/bsde.h"

namespace bsde {

// One grid point of one time layer: the value and the natural-spline second
// derivative of y and of z.  32 bytes, so one record is two 16-byte halves
// (y, M_y) and (z, M_z).
struct alignas(16) Rec64 {
    double y, My, z, Mz;
};

constexpr int kBlock = 256;        // threads per block of every kernel
constexpr int kPcrRounds = 5;      // PCR strides 1, 2, 4, 8, 16
constexpr int kHalo = 32;          // > 1 + 2 + 4 + 8 + 16: reach of the truncated PCR
constexpr int kPcrMaxPerThread = 8;// spline windows of at most kBlock * 8 records
constexpr int kSplineTile = 512;   // grid points per block of the standalone spline kernel

// Coefficients of one Gauss-Hermite node (j, l), the same for every grid
// point.  With phi the fraction of the node's cell offset, the spline value
// at the node is  v0 + B (v1 - v0) + C M0 + D M1  (second-derivative form).
struct alignas(16) NodeRec {
    double B;      // phi
    double C;      // dx^2/6 ((1-phi)^3 - (1-phi))
    double D;      // dx^2/6 (phi^3 - phi)
    double cfy;    // weight of f-hat in the constant of the y equation
    double cfz;    // weight of f-hat in z^n
    double cz;     // weight of z-hat in z^n
};

// Node table of one instance (device memory).  K*L entries, row j-1 holds the
// L nodes of layer n+j.
struct NodeTable {
    const NodeRec *rec;
    const int *m;       // integer cell offset of the node from x_i
    const double *cy;   // weight of y-hat in the y constant (non-zero only for j = K_y)
    const int *win_lo;  // [K+1]: lowest node offset of layer j (j = 1 also <= 0)
    const int *win_hi;  // [K+1]: highest node offset of layer j (j = 1 also >= 0)
};

constexpr int kMaxNodes = 6 * 64;      // K * L at most
constexpr int kMaxReach1 = 160;        // widest node reach of layer n+1 in the fused kernel
constexpr int kMaxReach2 = 320;        // widest node reach of layers n+2.. in the fused kernel
static_assert(kMaxReach2 >= kMaxReach1 + kHalo, "layer n+1 window must fit the window arrays");
constexpr size_t kNodeLdsBytes = sizeof(NodeRec) + sizeof(int) + sizeof(double);

// PCR slots per thread of a fused block of NT threads and P points per lane
// (the newest layer's window, its halo and the two extra staged values).
__host__ __device__ constexpr int pcr_slots(int P, int NT)
{
    return (kBlock * P + 2 * kHalo + 2 + kMaxReach1 + NT - 1) / NT;
}

// Fixed LDS window capacity (slots) of the fused kernel with P points per
// lane: the widest window of any layer plus the spline halo.  Being a
// compile-time constant, the z array sits at an immediate offset from y.
// The reach limits are sized so that the fused kernel with one point per
// lane keeps four 256-thread blocks on a CU (LDS <= 40 KB per block) up to a
// stability ratio of about 17 at K = 4, L = 16; wider reaches take the
// direct path.
__host__ __device__ constexpr int window_elems(int P) { return kBlock * P + kMaxReach2 + kHalo; }
__host__ __device__ constexpr int window_slots(int P)
{
    return (P % 2 == 0) ? window_elems(P) + window_elems(P) / P + 1 : window_elems(P);
}
__host__ __device__ constexpr int pcr_values(int P) { return kBlock * P + kMaxReach1 + 2 * kHalo + 2; }

// Slot of window element e in the LDS window arrays.  With an even number P
// of points per lane a pad slot follows every P elements, so the lanes of a
// wavefront, P elements apart, read 16-byte slots an odd multiple of 16 bytes
// apart and the reads are bank-conflict free (odd P needs no pad).
template <int P>
struct WinLayout {
    static constexpr bool kPad = (P % 2) == 0;
    __device__ static int slot(int e) { return kPad ? e + e / P : e; }
    __host__ __device__ static constexpr int slots(int n) { return kPad ? n + n / P + 1 : n; }
};

struct DriverParams {
    double p0, p1, p2, p3, p4;
};

// Coefficients of the truncated parallel cyclic reduction of (1, 4, 1).
struct PcrCoef {
    double s6;                   // 6 / dx^2
    double kappa[kPcrRounds];    // elimination factor of each round
    double inv_b;                // 1 / diagonal after the last round
};

struct SweepArgs {
    Rec64 *ring;
    NodeTable tab;
    DriverParams drv;
    PcrCoef pcr;
    int n;            // time index of the layer being computed
    int nx, npad, pad_l, pad_r;
    int K, Ky, L;
    int lds_cap, lds_cap1;  // records of the window arrays / of the PCR arrays
    double dt;
    double h0;        // K_y dt gamma_{K_y,0}: weight of the implicit f(t_n, y^n, z^n)
    int picard_max;
    double picard_tol;
    unsigned int *st_iter_max;        // per-wave running maximum (NULL: no stats)
    unsigned long long *st_iter_sum;  // per-wave running sum
    unsigned long long *st_nonconv;   // per-wave count of unconverged point-steps
};

// ---------------------------------------------------------------------------
// Drivers f(t, y, z) (problem statement eq (2); Examples 1-3 of Section 5)
// ---------------------------------------------------------------------------
template <int DRV>
struct Driver;

template <>
struct Driver<BSDE_DRIVER_LINEAR> {  // p0 y + p1 z + p3
    double a, b, c;
    __device__ Driver(const DriverParams &p, double) : a(p.p0), b(p.p1), c(p.p3) {}
    __device__ double operator()(double y, double z) const { return fma(a, y, fma(b, z, c)); }
};

template <>
struct Driver<BSDE_DRIVER_BIDASK> {  // -r y - theta z + s (R - r) min(y - z/sigma, 0)
    double mr, mth, c, inv_sg;
    __device__ Driver(const DriverParams &p, double)
        : mr(-p.p0), mth(-p.p2), c(p.p4 * (p.p1 - p.p0)), inv_sg(1.0 / p.p3) {}
    __device__ double operator()(double y, double z) const
    {
        const double m = fmin(fma(-z, inv_sg, y), 0.0);
        return fma(mr, y, fma(mth, z, c * m));
    }
};

template <>
struct Driver<BSDE_DRIVER_CUBIC> {  // Example 1: -y^3 + 5/2 y^2 - 3/2 y
    __device__ Driver(const DriverParams &, double) {}
    __device__ double operator()(double y, double) const
    {
        return y * fma(y, 2.5 - y, -1.5);
    }
};

template <>
struct Driver<BSDE_DRIVER_EXP> {  // Example 2: (e^{t^2} - 4ty - 3e^{t^2 - y e^{-t^2}} + z^2 e^{-t^2})/2
    double t, t2, et, emt;
    __device__ Driver(const DriverParams &, double tt)
        : t(tt), t2(tt * tt), et(exp(tt * tt)), emt(exp(-tt * tt)) {}
    __device__ double operator()(double y, double z) const
    {
        return 0.5 * (et - 4.0 * t * y - 3.0 * exp(t2 - y * emt) + z * z * emt);
    }
};

// ---------------------------------------------------------------------------
// Wavefront reductions (64 lanes) and the XCD-aware block order
// ---------------------------------------------------------------------------
__device__ inline unsigned int wave_max_u32(unsigned int v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, (unsigned int)__shfl_xor((int)v, o, 64));
    return v;
}
__device__ inline unsigned int wave_sum_u32(unsigned int v)
{
    for (int o = 32; o > 0; o >>= 1) v += (unsigned int)__shfl_xor((int)v, o, 64);
    return v;
}

// Blocks are handed to the 8 XCDs round-robin; remap so that each XCD works
// on one contiguous range of tiles (neighbouring tiles share node windows,
// hence L2 lines).  A bijection of [0, nb).
__device__ inline int xcd_tile(int b, int nb)
{
    const int per = nb >> 3, rem = nb & 7;
    const int x = b & 7, r = b >> 3;
    return x * per + min(x, rem) + r;
}

// ---------------------------------------------------------------------------
// Natural cubic spline of a layer on a window, second-derivative form:
//   M_0 = M_{N-1} = 0,  M_{i-1} + 4 M_i + M_{i+1} = r_i = 6/dx^2 (y_{i+1} - 2 y_i + y_{i-1}).
// Extending r oddly about 0 and N-1 (period 2(N-1)) gives the bi-infinite
// system (1, 4, 1) M = r~ whose solution is the odd extension of M.  Five
// rounds of parallel cyclic reduction leave a coupling below 1e-18 of the
// diagonal, so M_i = r~^(5)_i / b_5, which depends on r~ within 31 cells.
// ---------------------------------------------------------------------------

// r~_k / (6/dx^2) for any integer k, from the layer in HBM (used where the
// window does not hold the neighbours or k is outside [1, N-2]).
__device__ inline double rtilde_global(const Rec64 *__restrict__ g, int nx, int k, bool zf)
{
    const int per = 2 * (nx - 1);
    int kk = k % per;
    if (kk < 0) kk += per;
    double sign = 1.0;
    if (kk > nx - 1) {
        kk = per - kk;
        sign = -1.0;
    }
    if (kk == 0 || kk == nx - 1) return 0.0;
    const double vm = zf ? g[kk - 1].z : g[kk - 1].y;
    const double v0 = zf ? g[kk].z : g[kk].y;
    const double vp = zf ? g[kk + 1].z : g[kk + 1].y;
    return sign * ((vp - v0) - (v0 - vm));
}

// Natural spline of layer g on the window of records [lo, lo + W).
// y and z over [lo - kHalo - 1, lo + W + kHalo] are staged (outside [0, N)
// the boundary value, i.e. the ghost record), the right-hand sides r~ of the
// records [lo - kHalo, lo + W + kHalo) follow from them in LDS (from HBM only
// at the true domain boundaries, where the reflection applies), and five
// ping-pong PCR rounds leave M.  Results: window element e = k - lo + kHalo
// holds (y, M_y) in wy[slot(e)] and (z, M_z) in wz[slot(e)] for the records
// [lo, lo + W) (M = 0 outside (0, N-1)).  R holds 4 arrays of cap1 >= W +
// 2 kHalo + 2 doubles.  Called by all NT threads; ends synchronised.
// y and z of the staged range of spline_window, loaded into registers ahead
// of use (U slots per thread; element e = tid + u NT).
template <int U>
struct SplineRaw {
    double y[U], z[U];
};

template <int NT, int U>
__device__ inline void spline_load(const Rec64 *__restrict__ g, int nx, int lo, int W,
                                   SplineRaw<U> &raw)
{
    const int WS = W + 2 * kHalo + 2;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e = threadIdx.x + u * NT;
        if (e < WS) {
            const int k = lo - kHalo - 1 + e;
            const Rec64 r = g[min(max(k, 0), nx - 1)];
            raw.y[u] = r.y;
            raw.z[u] = r.z;
        }
    }
}

template <int NT, int U, int P>
__device__ inline void spline_window(const Rec64 *__restrict__ g, int nx, int lo, int W,
                                     double2 *wy, double2 *wz, double *R, int cap1,
                                     const PcrCoef &c, const SplineRaw<U> &raw)
{
    const int tid = threadIdx.x;
    const int WE = W + 2 * kHalo, WS = WE + 2;
    double *Ay = R, *Az = R + cap1, *By = R + 2 * cap1, *Bz = R + 3 * cap1;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e = tid + u * NT;
        if (e < WS) {
            Ay[e] = raw.y[u];
            Az[e] = raw.z[u];
        }
    }
    __syncthreads();
    for (int e = tid; e < WE; e += NT) {
        const int k = lo - kHalo + e;
        const double y0 = Ay[e + 1], z0 = Az[e + 1];
        double ry, rz;
        if (k >= 1 && k <= nx - 2) {
            ry = (Ay[e + 2] - y0) - (y0 - Ay[e]);
            rz = (Az[e + 2] - z0) - (z0 - Az[e]);
        } else {
            ry = rtilde_global(g, nx, k, false);
            rz = rtilde_global(g, nx, k, true);
        }
        By[e] = c.s6 * ry;
        Bz[e] = c.s6 * rz;
        const int sl = WinLayout<P>::slot(e);
        wy[sl].x = y0;
        wz[sl].x = z0;
    }
    __syncthreads();
    double *sy = By, *sz = Bz, *dy = Ay, *dz = Az;
    int h = 1;
    for (int s = 0; s < kPcrRounds; ++s, h <<= 1) {
        const double kap = c.kappa[s];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = tid + u * NT;
            if (e >= h && e < WE - h) {
                dy[e] = fma(-kap, sy[e - h] + sy[e + h], sy[e]);
                dz[e] = fma(-kap, sz[e - h] + sz[e + h], sz[e]);
            }
        }
        __syncthreads();
        double *t = sy;
        sy = dy;
        dy = t;
        t = sz;
        sz = dz;
        dz = t;
    }
    for (int e = kHalo + tid; e < kHalo + W; e += NT) {
        const int k = lo - kHalo + e;
        const bool inner = (k > 0 && k < nx - 1);
        const int sl = WinLayout<P>::slot(e);
        wy[sl].y = inner ? sy[e] * c.inv_b : 0.0;
        wz[sl].y = inner ? sz[e] * c.inv_b : 0.0;
    }
    __syncthreads();
}

// Copy the node table (K*L records, offsets and y weights) of an instance
// into LDS, where every lane of a wavefront reads the same address (a
// broadcast).  Called by all NT threads; ends synchronised.
template <int NT>
__device__ inline void load_node_table(const NodeTable &t, int nodes, NodeRec *trec, int *tm,
                                       double *tcy)
{
    for (int i = threadIdx.x; i < nodes; i += NT) {
        trec[i] = t.rec[i];
        tm[i] = t.m[i];
        tcy[i] = t.cy[i];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Per-node work shared by the sweep kernels: interpolate y and z at the node
// for P consecutive points from P+1 consecutive records, evaluate f, and
// accumulate into the y-equation constant Y and into z^n (Z).  LASTY adds
// the expectation of y itself (the layer j = K_y).
// ---------------------------------------------------------------------------
template <int P, int DRV, bool LASTY>
__device__ inline void node_accumulate(const double2 (&ry)[P + 1], const double2 (&rz)[P + 1],
                                       const NodeRec &c, double cy, const Driver<DRV> &f,
                                       double (&Y)[P], double (&Z)[P])
{
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const double yh = fma(c.B, ry[q + 1].x - ry[q].x,
                              fma(c.C, ry[q].y, fma(c.D, ry[q + 1].y, ry[q].x)));
        const double zh = fma(c.B, rz[q + 1].x - rz[q].x,
                              fma(c.C, rz[q].y, fma(c.D, rz[q + 1].y, rz[q].x)));
        const double fh = f(yh, zh);
        double y = fma(c.cfy, fh, Y[q]);
        if (LASTY) y = fma(cy, yh, y);
        Y[q] = y;
        Z[q] = fma(c.cfz, fh, fma(c.cz, zh, Z[q]));
    }
}

// Nodes l = l0, l0 + LS, l0 + 2 LS, ... < L of one layer, reading P+1
// consecutive records per lane from src at node offset m.
// The node offsets of a layer are held one per lane (L <= 64) and moved to
// a scalar register per node with readlane, so the records of a node are
// addressed without waiting for an LDS read; the coefficients are read from
// LDS together with the records.
template <int P, int DRV, bool LASTY, typename Src>
__device__ inline void layer_nodes(const Src &src, const NodeRec *trec, const int *tm,
                                   const double *tcy, int row, int l0, int LS, int L,
                                   const Driver<DRV> &f, double (&Y)[P], double (&Z)[P])
{
    const int lane = threadIdx.x & 63;
    const int mv = tm[row + min(lane, L - 1)];
#pragma unroll 1
    for (int l = l0; l < L; l += LS) {
        const int m = __builtin_amdgcn_readlane(mv, l);
        double2 ry[P + 1], rz[P + 1];
        src.template fetch<P>(m, ry, rz);
        node_accumulate<P, DRV, LASTY>(ry, rz, trec[row + l], LASTY ? tcy[row + l] : 0.0, f, Y, Z);
    }
}

// z^n is complete in Z; the implicit y equation y = Y + h0 f(t_n, y, z^n) is
// solved by Picard iteration from y^{n+1}_i; results go to layer n.
template <int P, int DRV>
__device__ inline void finish_points(const SweepArgs &a, int first, const double (&Y)[P],
                                     const double (&Z)[P])
{
    const int S = a.K + 1;
    const Driver<DRV> f0(a.drv, a.n * a.dt);
    const Rec64 *__restrict__ prev = a.ring + (size_t)((a.n + 1) % S) * a.npad + a.pad_l;
    Rec64 *__restrict__ out = a.ring + (size_t)(a.n % S) * a.npad + a.pad_l;
    unsigned int it_max = 0, it_sum = 0, nonconv = 0;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int i = first + q;
        const bool valid = i < a.nx;
        double y = prev[min(i, a.nx - 1)].y;
        int it = 0;
        bool conv = true;
        if (a.picard_tol > 0.0) {
            conv = false;
            while (it < a.picard_max) {
                const double yn = fma(a.h0, f0(y, Z[q]), Y[q]);
                ++it;
                const double dy = fabs(yn - y);
                y = yn;
                if (dy <= a.picard_tol * fmax(1.0, fabs(y))) {
                    conv = true;
                    break;
                }
            }
        } else {
            for (; it < a.picard_max; ++it) y = fma(a.h0, f0(y, Z[q]), Y[q]);
        }
        if (valid) {
            out[i].y = y;
            out[i].z = Z[q];
            it_max = max(it_max, (unsigned int)it);
            it_sum += it;
            nonconv += conv ? 0u : 1u;
        }
    }
    if (a.st_iter_max) {
        it_max = wave_max_u32(it_max);
        it_sum = wave_sum_u32(it_sum);
        nonconv = wave_sum_u32(nonconv);
        if ((threadIdx.x & 63) == 0) {
            // finish_points runs on the first kBlock threads of a block
            const int w = (blockIdx.x * kBlock + threadIdx.x) >> 6;
            a.st_iter_max[w] = max(a.st_iter_max[w], it_max);
            a.st_iter_sum[w] += it_sum;
            a.st_nonconv[w] += nonconv;
        }
    }
}

}  // namespace bsde

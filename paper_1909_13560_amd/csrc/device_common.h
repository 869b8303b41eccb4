// device_common.h -- data layout, drivers and shared device helpers of the
// backward sweep of the multistep BSDE scheme (arXiv:1909.13560).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "../../include/bsde.h"

namespace bsde {

constexpr int kBlock = 256;        // threads per block of every kernel
constexpr int kPcrRounds = 5;      // PCR strides 1, 2, 4, 8, 16
constexpr int kHalo = 32;          // > 1 + 2 + 4 + 8 + 16: reach of the truncated PCR
constexpr int kPcrMaxPerThread = 8;// spline windows of at most kBlock * 8 records
constexpr int kSplineTile = 512;   // grid points per block of the standalone spline kernel

// Coefficients of one Gauss-Hermite node (j, l), the same for every grid
// point.  With phi the fraction of the node's cell offset, the spline value
// at the node is  v0 + B (v1 - v0) + C M0 + D M1  (second-derivative form).
// 64 bytes: the kernels read a node with scalar loads (one per node, ahead
// of use), so the coefficients never occupy the LDS pipe.
struct alignas(16) NodeRec {
    double B;      // phi
    double C;      // dx^2/6 ((1-phi)^3 - (1-phi))
    double D;      // dx^2/6 (phi^3 - phi)
    double cfy;    // weight of f-hat in the constant of the y equation
    double cfz;    // weight of f-hat in z^n
    double cz;     // weight of z-hat in z^n
    double cy;     // weight of y-hat in the y constant (non-zero only for j = K_y)
    double cyz;    // weight of y-hat in z^n (z form E[y dW]/dt: j = 1 only)
};

// The FP32 form's node coefficients: interpolation weights and the weights
// of the small terms in single precision, the weights of the record values
// (which carry the magnitude of y^n and z^n) in double precision.  48 bytes.
struct alignas(16) NodeRec32 {
    float B, C, D;
    float cfy, cfz;
    float czf;   // cz in single precision (weight of the interpolation correction)
    float cyf;   // cy in single precision
    float cyzf;  // cyz in single precision
    double cz, cy, cyz, pad;
};

// Node table of one instance (device memory).  K*L entries, row j-1 holds the
// L nodes of layer n+j.
struct NodeTable {
    const NodeRec *rec;
    const NodeRec32 *rec32;  // the same coefficients for the FP32 form
    const int *m;       // integer cell offset of the node from x_i
    const int *win_lo;  // [K+1]: lowest node offset of layer j (j = 1 also <= 0)
    const int *win_hi;  // [K+1]: highest node offset of layer j (j = 1 also >= 0)
    const double *dw;   // Brownian increment sqrt(2 j dt) a_l of node (j, l) (gather path)
};

constexpr int kMaxOrder = 6;  // largest K of Tables 1-2

constexpr int kMaxNodes = 6 * 64;      // K * L at most
constexpr int kMaxReach1 = 160;        // widest node reach of layer n+1 in the fused kernel
constexpr int kMaxReach2 = 320;        // widest node reach of layers n+2.. in the fused kernel
static_assert(kMaxReach2 >= kMaxReach1 + kHalo, "layer n+1 window must fit the window arrays");

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

// The same five rounds as two filters, for windows clear of the domain ends
// (constants of the (1, 4, 1) system, evaluated at compile time): rounds 1-3
// with the second difference folded in, taps fa[|q|] on the values at offsets
// q = -8..8; rounds 4-5, taps fb[|q|] at offsets 8q, q = -3..3 (with
// t = s - k4 (s_{-8} + s_8) and u = t - k5 (t_{-16} + t_{16})).
struct PcrFilters {
    double fa[9];
    double fb[4];
};
__host__ __device__ constexpr PcrFilters pcr_filters()
{
    PcrFilters r{};
    double kap[kPcrRounds] = {};
    double av = 1.0, bv = 4.0;
    for (int k = 0; k < kPcrRounds; ++k) {  // a' = -a^2/b, b' = b - 2a^2/b
        kap[k] = av / bv;
        bv = bv - 2.0 * kap[k] * av;
        av = -kap[k] * av;
    }
    double f[17] = {}, g[17] = {};
    f[8] = 1.0;
    for (int k = 0, h = 1; k < 3; ++k, h *= 2) {
        for (int i = 0; i < 17; ++i)
            g[i] = f[i] - kap[k] * ((i - h >= 0 ? f[i - h] : 0.0) + (i + h < 17 ? f[i + h] : 0.0));
        for (int i = 0; i < 17; ++i) f[i] = g[i];
    }
    for (int q = 0; q <= 8; ++q)
        r.fa[q] = (q + 7 >= 0 ? f[q + 7] : 0.0) - 2.0 * f[q + 8] + (q + 9 < 17 ? f[q + 9] : 0.0);
    r.fb[0] = 1.0;
    r.fb[1] = kap[3] * kap[4] - kap[3];
    r.fb[2] = -kap[4];
    r.fb[3] = kap[3] * kap[4];
    return r;
}

// Exact Gaussian expectations as banded Toeplitz operators (toeplitz.hip):
// per layer j the band of ev, em, wv, wm (nb[j] weights each, records
// klo[j] .. klo[j] + nb[j] - 1 relative to the point) at w + off[j], and the
// weights of eq (20) for a linear driver folded per layer:
//   Y += cy_ey E[y] + cy_ez E[z] + cy_1,  Z += cz_ez E[z] + cz_wy E[y dW] + cz_wz E[z dW].
constexpr int kToepChunk = 256;  // band taps staged in LDS at a time (a multiple of 4)
constexpr int kToepTile = 256;   // points per block of the Toeplitz sweep
struct ToepTable {
    const double *w;
    int off[kMaxOrder + 1], klo[kMaxOrder + 1], nb[kMaxOrder + 1];
    double cy_ey[kMaxOrder + 1], cy_ez[kMaxOrder + 1], cy_1[kMaxOrder + 1];
    double cz_ez[kMaxOrder + 1], cz_wy[kMaxOrder + 1], cz_wz[kMaxOrder + 1];
};

struct SweepArgs {
    void *ring;       // K+1 slots of two planes (Slot), double2 (FP64) or float2 (FP32)
    double *fin_y, *fin_z;  // layer n_stop in double precision (written when n == n_stop)
    int n_stop;
    NodeTable tab;
    DriverParams drv;
    PcrCoef pcr;
    int n;            // time index of the layer being computed
    int nx, npad, pad_l, pad_r;
    int K, Ky, L;
    int ntiles;       // tiles of the sweep kernel over the grid
    double dt;
    double h0;        // K_y dt gamma_{K_y,0}: weight of the implicit f(t_n, y^n, z^n)
    int picard_max;
    double picard_tol;
    int zform;        // first term of the z equation: 0 E[z^{n+1}], 1 E[y^{n+1} dW]/dt
    // forward coefficients of eq (1) (gather path): a(x) = drift0 + drift_x x,
    // b(x) = vol0 + vol_x x on the grid x_i = x_min + i dx, or tabulated:
    // ctab row s = (tab_steps > 1 ? n : 0) holds a(t_n, x_i) at [2 s nx + i]
    // and b at [(2 s + 1) nx + i]
    double x_min, dx, drift0, drift_x, vol0, vol_x;
    const double *ctab;
    int tab_steps;
    ToepTable toep;   // exact Gaussian expectations (Toeplitz path)
    unsigned int *st_iter_max;        // per-wave running maximum (NULL: no stats)
    unsigned long long *st_iter_sum;  // per-wave running sum
    unsigned long long *st_nonconv;   // per-wave count of unconverged point-steps
};

// One instance of a (batched) solve as the kernels see it: its SweepArgs
// with the workspace parts given as byte offsets, bound to the workspace
// address at launch.  The kernels of one launch serve a group of instances
// (same precision, driver and tile shape); the grid's tiles are numbered
// instance after instance.
struct InstDesc {
    SweepArgs a;          // ring, fin_*, st_* unset; n unset
    size_t ring_off;      // ring of K+1 slots
    size_t fin_off;       // layer n_stop: n_x doubles of y, then of z
    size_t stat_off;      // per-wave statistics: sum (u64), unconverged (u64), max (u32)
    int nwaves;           // per-wave statistics slots
    int n0;               // first layer computed (N - K); step s computes n0 - s
    int f32;              // FP32 form
    int tile_base;        // first tile of the instance in its group's sweep grid
    int spline_base;      // first tile of the instance in its group's spline grid
    int spline_tiles;     // tiles of the standalone spline kernel
    // window bounds of the layers (NodeTable::win_lo/win_hi point here once
    // bound, so they load together with the descriptor)
    int win_lo[kMaxOrder + 1], win_hi[kMaxOrder + 1];
};

struct StepArgs {
    char *ws;
    const InstDesc *desc;
    const int *tile_inst;  // grid tile -> descriptor index; NULL: every tile is of desc[0]
    int s;                 // step: each instance computes layer n0 - s
    int stats;             // bind the statistics slots
    double *part;          // partial sums: Toeplitz sweep split over S blocks per tile, or
                           // the node chunks of a split direct sweep
    int dsplit;            // direct sweep: blocks per tile (1: no split)
    int dchunks;           // direct sweep: node chunks per tile in the partial-sum layout
};

// The direct sweep sums a tile's nodes chunk by chunk: kDirectChunk
// consecutive nodes of one layer, each chunk's sums from zero, the chunks
// added in order (layer by layer).  Split over S blocks (small grids), block
// s of a tile takes the chunks c = s (mod S) and the chunk sums meet in order
// in a finishing kernel, so the results do not depend on S.
constexpr int kDirectChunk = 16;
__host__ __device__ constexpr int direct_chunks(int K, int L)
{
    return K * ((L + kDirectChunk - 1) / kDirectChunk);
}

// ---------------------------------------------------------------------------
// Drivers f(t, y, z) (problem statement eq (2); Examples 1-3 of Section 5)
// ---------------------------------------------------------------------------
template <int DRV, typename T = double>
struct Driver;

template <typename T>
struct Driver<BSDE_DRIVER_LINEAR, T> {  // p0 y + p1 z + p3
    T a, b, c;
    __device__ Driver(const DriverParams &p, double) : a(p.p0), b(p.p1), c(p.p3) {}
    __device__ T operator()(T y, T z) const { return fma(a, y, fma(b, z, c)); }
};

template <typename T>
struct Driver<BSDE_DRIVER_BIDASK, T> {  // -r y - theta z + s (R - r) min(y - z/sigma, 0)
    T mr, mth, c, inv_sg;
    __device__ Driver(const DriverParams &p, double)
        : mr(-p.p0), mth(-p.p2), c(p.p4 * (p.p1 - p.p0)), inv_sg(1.0 / p.p3) {}
    __device__ T operator()(T y, T z) const
    {
        const T m = fmin(fma(-z, inv_sg, y), T(0));
        return fma(mr, y, fma(mth, z, c * m));
    }
};

template <typename T>
struct Driver<BSDE_DRIVER_CUBIC, T> {  // Example 1: -y^3 + 5/2 y^2 - 3/2 y
    __device__ Driver(const DriverParams &, double) {}
    __device__ T operator()(T y, T) const { return y * fma(y, T(2.5) - y, T(-1.5)); }
};

template <typename T>
struct Driver<BSDE_DRIVER_EXP, T> {  // Example 2: (e^{t^2} - 4ty - 3e^{t^2 - y e^{-t^2}} + z^2 e^{-t^2})/2
    T t, t2, et, emt;
    __device__ Driver(const DriverParams &, double tt)
        : t(tt), t2(tt * tt), et(exp(tt * tt)), emt(exp(-tt * tt)) {}
    __device__ T operator()(T y, T z) const
    {
        return T(0.5) * (et - T(4) * t * y - T(3) * exp(t2 - y * emt) + z * z * emt);
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

__device__ inline SweepArgs bind_instance(const InstDesc &d, char *ws, int s, bool stats)
{
    SweepArgs a = d.a;
    a.tab.win_lo = d.win_lo;
    a.tab.win_hi = d.win_hi;
    a.n = d.n0 - s;
    a.ring = ws + d.ring_off;
    a.fin_y = reinterpret_cast<double *>(ws + d.fin_off);
    a.fin_z = a.fin_y + a.nx;
    if (stats) {
        unsigned long long *sum = reinterpret_cast<unsigned long long *>(ws + d.stat_off);
        a.st_iter_sum = sum;
        a.st_nonconv = sum + d.nwaves;
        a.st_iter_max = reinterpret_cast<unsigned int *>(sum + 2 * d.nwaves);
    } else {
        a.st_iter_sum = nullptr;
        a.st_nonconv = nullptr;
        a.st_iter_max = nullptr;
    }
    return a;
}

// The descriptor of block idx of a step launch.  A group of one instance
// launches without a tile map, so its blocks start with a single dependent
// load (the descriptor) before the first ring read.
__device__ inline const InstDesc &block_desc(const StepArgs &s, int idx)
{
    return s.tile_inst ? s.desc[s.tile_inst[idx]] : s.desc[0];
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
template <typename Rec>
__device__ inline double rtilde_global(const Rec &g, int nx, int k, bool zf)
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
    const auto em = g.val(kk - 1), e0 = g.val(kk), ep = g.val(kk + 1);
    const double vm = zf ? em.y : em.x;
    const double v0 = zf ? e0.y : e0.x;
    const double vp = zf ? ep.y : ep.x;
    return sign * ((vp - v0) - (v0 - vm));
}

// Window of one layer in LDS.  Element e (slot WinLayout<P>::slot(e)) holds
// grid point lo - kHalo + e, in the ring's two fragments:
//   FP64 form: (y, z) in wy[slot], (M_y, M_z) in wy[slot + window_slots(P)].
//   FP32 form: (y, z, M_y, M_z) in w[slot].
template <int P>
struct WinStore64 {
    double2 *wy;
    static constexpr int kM = window_slots(P);
    __device__ void put(int sl, const double2 &v, const double2 &m) const
    {
        wy[sl] = v;
        wy[sl + kM] = m;
    }
    __device__ void val(int sl, double y, double z) const { wy[sl] = make_double2(y, z); }
    __device__ void der(int sl, double my, double mz) const { wy[sl + kM] = make_double2(my, mz); }
    __device__ double2 ders(int sl) const { return wy[sl + kM]; }
};

template <int P>
struct WinStore32 {
    float4 *w;
    __device__ void put(int sl, const float2 &v, const float2 &m) const
    {
        w[sl] = make_float4(v.x, v.y, m.x, m.y);
    }
    __device__ void val(int sl, double y, double z) const
    {
        reinterpret_cast<float2 *>(w + sl)[0] = make_float2((float)y, (float)z);
    }
    __device__ void der(int sl, double my, double mz) const
    {
        reinterpret_cast<float2 *>(w + sl)[1] = make_float2((float)my, (float)mz);
    }
    __device__ double2 ders(int sl) const { return make_double2(w[sl].z, w[sl].w); }
};

// Natural spline of layer g on the window of records [lo, lo + W).
// y and z over [lo - kHalo - 1, lo + W + kHalo] are staged (outside [0, N)
// the boundary value, i.e. the ghost record), the right-hand sides r~ of the
// records [lo - kHalo, lo + W + kHalo) follow from them in LDS (from HBM only
// at the true domain boundaries, where the reflection applies), and five
// ping-pong PCR rounds leave M, all in double precision.  Results: window
// element e = k - lo + kHalo holds y, z and M_y, M_z (M = 0 outside
// (0, N-1)) of the records [lo, lo + W).  R holds 4 arrays of cap1 >= W +
// 2 kHalo + 2 doubles.  Called by all NT threads; ends synchronised.
// y and z of the staged range of spline_window, loaded into registers ahead
// of use (U slots per thread; element e = tid + u NT).
template <int U, typename V>
struct SplineRaw {
    V y[U], z[U];
};

template <int NT, int U, typename Slot, typename V>
__device__ inline void spline_load(const Slot &g, int nx, int lo, int W, SplineRaw<U, V> &raw)
{
    const int WS = W + 2 * kHalo + 2;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e = threadIdx.x + u * NT;
        if (e < WS) {
            const int k = lo - kHalo - 1 + e;
            const auto r = g.val(min(max(k, 0), nx - 1));
            raw.y[u] = r.x;
            raw.z[u] = r.y;
        }
    }
}

// spline_window for a window clear of the domain ends (every staged record
// is a grid record and every r~ the plain second difference): the five
// rounds as two stencils, three barriers in all.  Pass A evaluates rounds
// 1-3 on the values for the window and 24 cells either side (three outputs
// per thread, so neighbouring outputs share their reads); pass B applies
// rounds 4-5 (four outputs 8 apart per thread) and writes y, z, M to the
// window.  Same linear map as the round-by-round form up to rounding.
template <int NT, int U, int P, typename Win, typename V>
__device__ inline void spline_window_interior(int W, const Win &win, double *R, int cap1,
                                              const PcrCoef &c, const SplineRaw<U, V> &raw)
{
    const int tid = threadIdx.x;
    const int WS = W + 2 * kHalo + 2;
    // D[e]: staged (y, z) of record lo - kHalo - 1 + e; A[e]: pass-A output of
    // window element e (record lo - kHalo + e)
    double2 *D = reinterpret_cast<double2 *>(R);
    double2 *A = reinterpret_cast<double2 *>(R + 2 * cap1);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e = tid + u * NT;
        if (e < WS) D[e] = make_double2(raw.y[u], raw.z[u]);
    }
    __syncthreads();
    constexpr PcrFilters F = pcr_filters();
    constexpr int kA = 3;                            // outputs per thread in pass A
    const int a0 = kHalo - 24, a1 = kHalo + W + 24;  // pass-A outputs [a0, a1)
    for (int t = tid; a0 + kA * t < a1; t += NT) {
        const int e = a0 + kA * t;
        // output e + o takes D[e + o + 1 + q] with weight fa[|q|], q = -8..8;
        // the staged values stream through once
        double vy[kA], vz[kA];
#pragma unroll
        for (int o = 0; o < kA; ++o) vy[o] = vz[o] = 0.0;
#pragma unroll
        for (int i = 0; i < kA + 16; ++i) {
            // at most four reads in flight: hoisting all of them would raise
            // the register count of the whole sweep kernel
            if (i % 4 == 0) __builtin_amdgcn_sched_barrier(0);
            const double2 x = D[e - 7 + i];
#pragma unroll
            for (int o = 0; o < kA; ++o) {
                const int q = i - 8 - o;
                if (q >= -8 && q <= 8) {
                    const double w = F.fa[q < 0 ? -q : q];
                    vy[o] = fma(w, x.x, vy[o]);
                    vz[o] = fma(w, x.y, vz[o]);
                }
            }
        }
        // unguarded: A has room past a1 (cap1 >= W + 2 kHalo + 2), and pass B
        // reads A below a1 only
#pragma unroll
        for (int o = 0; o < kA; ++o) A[e + o] = make_double2(vy[o], vz[o]);
    }
    __syncthreads();
    const double sc = c.s6 * c.inv_b;
    for (int t = tid;; t += NT) {
        const int e = kHalo + (t & 7) + 32 * (t >> 3);  // outputs e, e+8, e+16, e+24
        if (e >= kHalo + W) break;
        // output e + 8o takes A[e + 8(o + q)] with weight fb[|q|], q = -3..3
        double wy[4], wz[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) wy[o] = wz[o] = 0.0;
#pragma unroll
        for (int i = 0; i < 10; ++i) {
            if (i % 4 == 0) __builtin_amdgcn_sched_barrier(0);
            const int k = e + 8 * (i - 3);
            double2 x = A[min(k, a1 - 1)];
            if (k >= a1) x = make_double2(0.0, 0.0);
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                const int q = i - 3 - o;
                if (q >= -3 && q <= 3) {
                    const double w = F.fb[q < 0 ? -q : q];
                    wy[o] = fma(w, x.x, wy[o]);
                    wz[o] = fma(w, x.y, wz[o]);
                }
            }
        }
        // unguarded: outputs up to kHalo + W + 24 stay inside the window
        // arrays and the staged range, and nothing reads the window past
        // kHalo + W
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const int eo = e + 8 * o;
            const double2 yz = D[eo + 1];
            win.val(WinLayout<P>::slot(eo), yz.x, yz.y);
            win.der(WinLayout<P>::slot(eo), wy[o] * sc, wz[o] * sc);
        }
    }
    __syncthreads();
}

template <int NT, int U, int P, typename Slot, typename V, typename Win>
__device__ inline void spline_window(const Slot &g, int nx, int lo, int W,
                                     const Win &win, double *R, int cap1, const PcrCoef &c,
                                     const SplineRaw<U, V> &raw)
{
    // the FP32 form keeps the round-by-round solve: the stencil passes' extra
    // registers would cost it occupancy, which it has to spare otherwise
    if constexpr (sizeof(V) == sizeof(double)) {
        if (lo >= kHalo + 1 && lo + W <= nx - kHalo - 1) {
            spline_window_interior<NT, U, P>(W, win, R, cap1, c, raw);
            return;
        }
    }
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
        win.val(WinLayout<P>::slot(e), y0, z0);
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
        win.der(WinLayout<P>::slot(e), inner ? sy[e] * c.inv_b : 0.0, inner ? sz[e] * c.inv_b : 0.0);
    }
    __syncthreads();
}

// The two precision forms.
//   FP64: ring planes and window fragments (y, z) and (M_y, M_z) as double2.
//   FP32: ring planes (y, z) and (M_y, M_z) as float2, one float4
//         (y, z, M_y, M_z) per window element; node values and f-hat in
//         single precision, accumulators in double precision.
template <bool F32>
struct Prec;
template <>
struct Prec<false> {
    using E = double2;  // one ring-plane element
    using Node = NodeRec;
    using V = double2;
    using Raw = double;
    static constexpr int NA = 2;  // fragments per record
    template <int P>
    using Win = WinStore64<P>;
};
template <>
struct Prec<true> {
    using E = float2;
    using Node = NodeRec32;
    using V = float4;
    using Raw = float;
    static constexpr int NA = 1;
    template <int P>
    using Win = WinStore32<P>;
};

// One ring slot (one time layer): planes of npad elements, the values
// (y, z) and the spline second derivatives (M_y, M_z), each pair a double2
// (FP64) or float2 (FP32); index k runs from -pad_l to nx + pad_r - 1.  A
// launch writes whole planes contiguously: the values of layer n and the
// derivatives of layer n+1.
// The FP32 form has a third plane, the rounding residuals (e_y, e_z) of the
// stored values: y^n is stored as fl(y^n + e_y^{n+K_y}) and z^n as
// fl(z^n + e_z^{n+1}) (round to nearest), and the residual of that rounding
// is kept for the layer that follows in the same recurrence.  A layer
// changes little from one step to the next, so plain rounding would make
// nearly the same error at every step and the errors would add up along the
// y and z recurrences of eq (20) (linearly in the number of steps); carried
// forward, they cancel between consecutive steps instead (error feedback, as
// in compensated summation) and the stored layers stay within a few units in
// the last place of single precision of the exact ones.
// Elements are addressed by a 32-bit byte offset from the plane's start
// (the host keeps a plane below 4 GiB): the planes share the offset of a
// point, and the loads take the form "scalar base + 32-bit vector offset".
template <bool F32>
struct Slot {
    using E = typename Prec<F32>::E;
    using T = typename std::conditional<F32, float, double>::type;
    char *v0, *m0;  // plane starts (element -pad_l)
    int pad;        // pad_l
    __device__ unsigned off(int k) const { return (unsigned)(k + pad) * (unsigned)sizeof(E); }
    __device__ E val(int k) const { return *reinterpret_cast<const E *>(v0 + off(k)); }
    __device__ E der(int k) const { return *reinterpret_cast<const E *>(m0 + off(k)); }
    __device__ void set_val(int k, const E &e) const { *reinterpret_cast<E *>(v0 + off(k)) = e; }
    __device__ void set_val(int k, double y, double z) const { set_val(k, E{(T)y, (T)z}); }
    __device__ void set_der(int k, double my, double mz) const
    {
        *reinterpret_cast<E *>(m0 + off(k)) = E{(T)my, (T)mz};
    }
    // FP32 form: the residual plane follows the derivative plane
    __device__ char *r0(int npad) const { return m0 + (size_t)npad * sizeof(E); }
};

template <bool F32>
constexpr int kSlotPlanes = F32 ? 3 : 2;  // values, derivatives (, residuals)

template <bool F32>
__device__ inline Slot<F32> ring_slot(const SweepArgs &a, int layer)
{
    using E = typename Slot<F32>::E;
    char *base = static_cast<char *>(a.ring) +
                 (size_t)(layer % (a.K + 1)) * kSlotPlanes<F32> * a.npad * sizeof(E);
    return Slot<F32>{base, base + (size_t)a.npad * sizeof(E), a.pad_l};
}

// Store (y, z) of grid point i into a FP32-form ring slot with error
// feedback: ey, ez are the residuals carried from the previous layers of the
// y and z recurrences (0 for the initial layers).
__device__ inline void store_fed_back(const Slot<true> &s, int npad, int i, double y, double z,
                                      float ey, float ez)
{
    const double yv = y + (double)ey, zv = z + (double)ez;
    const float sy = (float)yv, sz = (float)zv;
    s.set_val(i, make_float2(sy, sz));
    *reinterpret_cast<float2 *>(s.r0(npad) + s.off(i)) =
        make_float2((float)(yv - (double)sy), (float)(zv - (double)sz));
}

// The residuals (e_y, e_z) stored with grid point i of a FP32-form slot.
__device__ inline float2 fed_back_residual(const Slot<true> &s, int npad, int i)
{
    return *reinterpret_cast<const float2 *>(s.r0(npad) + s.off(i));
}

__device__ inline const NodeRec *node_recs(const NodeTable &t, NodeRec *) { return t.rec; }
__device__ inline const NodeRec32 *node_recs(const NodeTable &t, NodeRec32 *) { return t.rec32; }

// Read a node record through the constant address space: the address is the
// same for the whole wavefront, so this compiles to scalar loads into SGPRs.
template <typename T>
__device__ inline T const_load(const T *p)
{
    return *(const __attribute__((address_space(4))) T *)(p);
}
__device__ inline NodeRec load_node(const NodeRec *p)
{
    NodeRec r;
    r.B = const_load(&p->B);
    r.C = const_load(&p->C);
    r.D = const_load(&p->D);
    r.cfy = const_load(&p->cfy);
    r.cfz = const_load(&p->cfz);
    r.cz = const_load(&p->cz);
    r.cy = const_load(&p->cy);
    r.cyz = const_load(&p->cyz);
    return r;
}
__device__ inline NodeRec32 load_node(const NodeRec32 *p)
{
    NodeRec32 r;
    r.B = const_load(&p->B);
    r.C = const_load(&p->C);
    r.D = const_load(&p->D);
    r.cfy = const_load(&p->cfy);
    r.cfz = const_load(&p->cfz);
    r.czf = const_load(&p->czf);
    r.cyf = const_load(&p->cyf);
    r.cyzf = const_load(&p->cyzf);
    r.cz = const_load(&p->cz);
    r.cy = const_load(&p->cy);
    r.cyz = const_load(&p->cyz);
    r.pad = 0.0;
    return r;
}

// Accumulators of P points: Y (constant of the y equation) and Z (= z^n) in
// double precision; the FP32 form sums the f-hat terms of one layer in
// single precision first (Yf, Zf) and adds them to Y, Z after the layer.
template <int P>
struct Acc {
    double Y[P], Z[P];
    float Yf[P], Zf[P];
};

// ---------------------------------------------------------------------------
// Per-node work shared by the sweep kernels: interpolate y and z at the node
// for P consecutive points from P+1 consecutive records, evaluate f, and
// accumulate into the y-equation constant Y and into z^n (Z).  Node flags NF:
// kNodeLastY adds the expectation of y itself (the layer j = K_y), kNodeYW
// the y-hat term of z^n (layer j = 1 of the z form E[y^{n+1} dW]/dt).
// ---------------------------------------------------------------------------
constexpr int kNodeLastY = 1, kNodeYW = 2;

template <int P, int DRV, int NF>
__device__ inline void node_accumulate(const double2 (&r)[2][P + 1], const NodeRec &c,
                                       const Driver<DRV, double> &f, Acc<P> &acc)
{
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const double2 *rv = r[0], *rm = r[1];  // (y, z) and (M_y, M_z)
        const double yh = fma(c.B, rv[q + 1].x - rv[q].x,
                              fma(c.C, rm[q].x, fma(c.D, rm[q + 1].x, rv[q].x)));
        const double zh = fma(c.B, rv[q + 1].y - rv[q].y,
                              fma(c.C, rm[q].y, fma(c.D, rm[q + 1].y, rv[q].y)));
        const double fh = f(yh, zh);
        double y = fma(c.cfy, fh, acc.Y[q]);
        if (NF & kNodeLastY) y = fma(c.cy, yh, y);
        acc.Y[q] = y;
        double z = fma(c.cfz, fh, fma(c.cz, zh, acc.Z[q]));
        if (NF & kNodeYW) z = fma(c.cyz, yh, z);
        acc.Z[q] = z;
    }
}

// FP32 form.  The interpolated value is kept as the unevaluated sum of the
// record value v0 (exact) and the correction d = B (v1 - v0) + C M0 + D M1,
// computed in single precision: d is small (a fraction of one cell's change
// of v), so its rounding is far below that of v0 + d rounded to single.  The
// record-value terms, which carry the size of the solution, go into the
// double accumulators (single values are exact in double, so the only
// rounding is that of the double FMA); the corrections and the f-hat terms,
// whose weights are O(dt) and O(sqrt(dt)), are summed over the layer in
// single precision.  f-hat itself is evaluated in single precision at
// v0 + d.
template <int P, int DRV, int NF>
__device__ inline void node_accumulate(const float4 (&r)[1][P + 1], const NodeRec32 &c,
                                       const Driver<DRV, float> &f, Acc<P> &acc)
{
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const float4 r0 = r[0][q], r1 = r[0][q + 1];  // (y, z, M_y, M_z)
        const float dy = fmaf(c.B, r1.x - r0.x, fmaf(c.C, r0.z, c.D * r1.z));
        const float dz = fmaf(c.B, r1.y - r0.y, fmaf(c.C, r0.w, c.D * r1.w));
        const float fh = f(r0.x + dy, r0.y + dz);
        acc.Yf[q] = fmaf(c.cfy, fh, acc.Yf[q]);
        acc.Zf[q] = fmaf(c.cfz, fh, fmaf(c.czf, dz, acc.Zf[q]));
        acc.Z[q] = fma(c.cz, (double)r0.y, acc.Z[q]);
        if (NF & kNodeLastY) {
            acc.Yf[q] = fmaf(c.cyf, dy, acc.Yf[q]);
            acc.Y[q] = fma(c.cy, (double)r0.x, acc.Y[q]);
        }
        if (NF & kNodeYW) {
            acc.Zf[q] = fmaf(c.cyzf, dy, acc.Zf[q]);
            acc.Z[q] = fma(c.cyz, (double)r0.x, acc.Z[q]);
        }
    }
}

// Nodes l = l0, l0 + LS, l0 + 2 LS, ... < L of one layer, reading P+1
// consecutive records per lane from src at node offset m.  The node offsets
// of a layer are held one per lane (L <= 64) and moved to a scalar register
// per node with readlane, and the coefficient records come through scalar
// loads, so the only per-node LDS traffic is the records themselves.
template <int P, int DRV, int NF, bool F32, typename Src>
__device__ inline void layer_nodes(const Src &src, const typename Prec<F32>::Node *nodes,
                                   const int *m, int l0, int LS, int L,
                                   const Driver<DRV, typename Prec<F32>::Raw> &f, Acc<P> &acc)
// m: the layer's node offsets in LDS (a vector-memory load here would make
// every node wait for the outstanding prefetch of the next window)
{
    using V = typename Prec<F32>::V;
    using Node = typename Prec<F32>::Node;
    constexpr int NA = Prec<F32>::NA;
    if (F32) {
#pragma unroll
        for (int q = 0; q < P; ++q) acc.Yf[q] = acc.Zf[q] = 0.0f;
    }
    if (l0 < L) {
        const int lane = threadIdx.x & 63;
        const int mv = m[min(lane, L - 1)];
        int l = l0;
        // two nodes per iteration: their scalar and LDS loads are in flight
        // together, so one wait covers both
#pragma unroll 1
        for (; l + LS < L; l += 2 * LS) {
            const Node c0 = load_node(nodes + l), c1 = load_node(nodes + l + LS);
            V r0[NA][P + 1], r1[NA][P + 1];
            src.template fetch<P>(__builtin_amdgcn_readlane(mv, l), r0);
            src.template fetch<P>(__builtin_amdgcn_readlane(mv, l + LS), r1);
            node_accumulate<P, DRV, NF>(r0, c0, f, acc);
            node_accumulate<P, DRV, NF>(r1, c1, f, acc);
        }
        if (l < L) {
            const Node c0 = load_node(nodes + l);
            V r0[NA][P + 1];
            src.template fetch<P>(__builtin_amdgcn_readlane(mv, l), r0);
            node_accumulate<P, DRV, NF>(r0, c0, f, acc);
        }
    }
    if (F32) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            acc.Y[q] += (double)acc.Yf[q];
            acc.Z[q] += (double)acc.Zf[q];
        }
    }
}

// z^n is complete in Z; the implicit y equation y = Y + h0 f(t_n, y, z^n) is
// solved by Picard iteration (double precision in both forms) from
// y^{n+1}_i; results go to layer n, and at n = n_stop also to fin_y, fin_z.
template <int P, int DRV, bool F32>
__device__ inline void finish_points(const SweepArgs &a, int first, const Acc<P> &acc,
                                     int wave_slot)
{
    const Driver<DRV, double> f0(a.drv, a.n * a.dt);
    const Slot<F32> prev = ring_slot<F32>(a, a.n + 1), out = ring_slot<F32>(a, a.n);
    const bool last = a.n == a.n_stop;
    unsigned int it_max = 0, it_sum = 0, nonconv = 0;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int i = first + q;
        const bool valid = i < a.nx;
        double y = prev.val(min(i, a.nx - 1)).x;
        const double zq = acc.Z[q], Yq = acc.Y[q];
        int it = 0;
        bool conv = true;
        if (a.picard_tol > 0.0) {
            conv = false;
            while (it < a.picard_max) {
                const double yn = fma(a.h0, f0(y, zq), Yq);
                ++it;
                const double dy = fabs(yn - y);
                y = yn;
                if (dy <= a.picard_tol * fmax(1.0, fabs(y))) {
                    conv = true;
                    break;
                }
            }
        } else {
            for (; it < a.picard_max; ++it) y = fma(a.h0, f0(y, zq), Yq);
        }
        if (valid) {
            if constexpr (F32) {
                // error feedback: residual of y^{n+K_y} (y recurrence) and of
                // z^{n+1} (z recurrence) at the same point
                const float ey = fed_back_residual(ring_slot<true>(a, a.n + a.Ky), a.npad, i).x;
                const float ez = fed_back_residual(ring_slot<true>(a, a.n + 1), a.npad, i).y;
                store_fed_back(out, a.npad, i, y, zq, ey, ez);
            } else {
                out.set_val(i, y, zq);
            }
            if (last) {
                a.fin_y[i] = y;
                a.fin_z[i] = zq;
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
        if ((threadIdx.x & 63) == 0) {
            a.st_iter_max[wave_slot] = max(a.st_iter_max[wave_slot], it_max);
            a.st_iter_sum[wave_slot] += it_sum;
            a.st_nonconv[wave_slot] += nonconv;
        }
    }
}

}  // namespace bsde

// kernels_f64.hip -- FP64 kernels of the backward sweep (arXiv:1909.13560,
// Section 2.2 eq (20)-(21), Section 3.1 step 3, Section 3.2) and their
// host-side launchers.
//
// Two sweep kernels compute layer n from layers n+1..n+K:
//   sweep_fused  (one launch per time step): a block owns a tile of
//                kBlock*P consecutive grid points.  For each layer j it stages
//                the records its nodes touch (the tile widened by the node
//                offsets of layer j) in LDS; for j = 1 it first solves that
//                layer's natural spline on the window by truncated PCR and
//                writes the tile's second derivatives back to HBM, so no
//                separate spline launch is needed.  Each lane handles P
//                consecutive points; P is odd, which makes the 16-byte LDS
//                reads of a wavefront bank-conflict free.
//   sweep_direct (wide node reach, window too big for LDS): records are read
//                straight from HBM/L2, P consecutive points per lane; the
//                natural spline of the new layer is a separate launch of
//                spline_f64.
#include "device_common.h"
#include "kernels.h"

namespace bsde {

// Node records read from the LDS window arrays (fused kernel).  Window
// element e of the lane's q-th record is lane_pt + off + q with off =
// ebase + m >= 0; with the padded layout its slot is
//   (P+1) tig + off + off/P + q + [q >= P - off % P]   (tig = lane_pt / P),
// so the per-record offsets are one of P compile-time patterns.
template <int P, int B, bool PAD>
__device__ inline void fetch_slots(const double2 *wy, int base, double2 (&ry)[P + 1],
                                   double2 (&rz)[P + 1])
{
    const double2 *p = wy + base;
#pragma unroll
    for (int q = 0; q <= P; ++q) {
        const int sl = q + ((PAD && q >= P - B) ? 1 : 0);
        ry[q] = p[sl];
        rz[q] = p[sl + window_slots(P)];  // z array at a fixed distance
    }
}

template <int P>
struct LdsWindow {
    const double2 *wy;  // z array follows at window_slots(P)
    int ebase;  // kHalo - (lowest node offset of the layer): off = ebase + m
    int lane;   // slot of the lane's first element at off = 0: (P+1) tig padded, P tig not
    template <int PP>
    __device__ void fetch(int m, double2 (&ry)[PP + 1], double2 (&rz)[PP + 1]) const
    {
        static_assert(PP == P, "window layout and fetch width differ");
        const int off = ebase + m;
        if constexpr (!WinLayout<P>::kPad) {
            fetch_slots<P, 0, false>(wy, lane + off, ry, rz);
        } else {
            const int base = lane + off + off / P;
            switch (off % P) {
            case 0: fetch_slots<P, 0, true>(wy, base, ry, rz); break;
            case 1: fetch_slots<P, 1, true>(wy, base, ry, rz); break;
            case 2: fetch_slots<P, (P > 2 ? 2 : 1), true>(wy, base, ry, rz); break;
            default: fetch_slots<P, (P > 3 ? 3 : 1), true>(wy, base, ry, rz); break;
            }
        }
    }
};

// Node records read straight from the layer in HBM (direct kernel).
struct GlobalWindow {
    const Rec64 *lay;  // record of the lane's first point
    template <int P>
    __device__ void fetch(int m, double2 (&ry)[P + 1], double2 (&rz)[P + 1]) const
    {
        const Rec64 *__restrict__ s = lay + m;
#pragma unroll
        for (int q = 0; q <= P; ++q) {
            const Rec64 r = s[q];
            ry[q] = make_double2(r.y, r.My);
            rz[q] = make_double2(r.z, r.Mz);
        }
    }
};

template <int P, int DRV, typename Src>
__device__ inline void layer_dispatch(const Src &src, const NodeRec *trec, const int *tm,
                                      const double *tcy, int j, int l0, int LS,
                                      const SweepArgs &a, double (&Y)[P], double (&Z)[P])
{
    const Driver<DRV> f(a.drv, (a.n + j) * a.dt);
    const int row = (j - 1) * a.L;
    if (j == a.Ky)
        layer_nodes<P, DRV, true>(src, trec, tm, tcy, row, l0, LS, a.L, f, Y, Z);
    else
        layer_nodes<P, DRV, false>(src, trec, tm, tcy, row, l0, LS, a.L, f, Y, Z);
}

// ---------------------------------------------------------------------------
// Fused sweep: LDS-staged windows, in-kernel spline of layer n+1.
// A block of G*kBlock threads owns a tile of kBlock*P points; thread group g
// (kBlock threads) takes the nodes l = g, g+G, ... of every layer, and the G
// partial sums meet in LDS before group 0 finishes the points.
// Dynamic LDS: wy, wz (window_slots(P) double2 each), the four PCR arrays
// (pcr_values(P) doubles each), node table (K*L NodeRec, K*L int, K*L double).
// ---------------------------------------------------------------------------
template <int P, int G, int DRV>
__global__ void __launch_bounds__(kBlock * G) sweep_fused(const SweepArgs a)
{
    constexpr int T = kBlock * P;
    constexpr int NT = kBlock * G;
    extern __shared__ double2 smem[];
    constexpr int CAP = window_slots(P), CAP1 = pcr_values(P);
    double2 *wy = smem;
    double2 *wz = wy + CAP;
    double *R = reinterpret_cast<double *>(wz + CAP);
    NodeRec *trec = reinterpret_cast<NodeRec *>(R + 4 * CAP1);
    int *tm = reinterpret_cast<int *>(trec + a.K * a.L);
    double *tcy = reinterpret_cast<double *>(tm + ((a.K * a.L + 1) & ~1));

    const int tid = threadIdx.x;
    // kBlock is a multiple of the wavefront size: the group is wave-uniform
    const int grp = __builtin_amdgcn_readfirstlane(tid / kBlock);
    const int lane_pt = (tid % kBlock) * P;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int t0 = tile * T;
    const int S = a.K + 1;
    load_node_table<NT>(a.tab, a.K * a.L, trec, tm, tcy);

    double Y[P], Z[P];
#pragma unroll
    for (int q = 0; q < P; ++q) Y[q] = Z[q] = 0.0;

    // Layers are processed in the order 2, 3, ..., K, 1: the records of layers
    // n+2.. are complete (their splines were built by earlier launches) and
    // their windows are prefetched into registers one layer ahead, while the
    // raw values of layer n+1 (written by the previous launch) are loaded at
    // the start and only turned into its spline after the other layers.
    constexpr int kPre = (T + kMaxReach2 + NT - 1) / NT;
    constexpr int kRaw = pcr_slots(P, NT);
    Rec64 pre[kPre];
    auto prefetch = [&](int j) {
        const Rec64 *__restrict__ g = a.ring + (size_t)((a.n + j) % S) * a.npad + a.pad_l;
        const int lo = t0 + a.tab.win_lo[j];
        const int W = T + (a.tab.win_hi[j] - a.tab.win_lo[j]) + 1;
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
            const int e = tid + u * NT;
            if (e < W) pre[u] = g[lo + e];
        }
    };
    SplineRaw<kRaw> raw1;
    {
        const Rec64 *__restrict__ g1 = a.ring + (size_t)((a.n + 1) % S) * a.npad + a.pad_l;
        const int W1 = T + (a.tab.win_hi[1] - a.tab.win_lo[1]) + 1;
        if (a.K >= 2) prefetch(2);
        spline_load<NT, kRaw>(g1, a.nx, t0 + a.tab.win_lo[1], W1, raw1);
    }

    for (int jj = 0; jj < a.K; ++jj) {
        const int j = (jj + 1 < a.K) ? jj + 2 : 1;
        Rec64 *__restrict__ g = a.ring + (size_t)((a.n + j) % S) * a.npad + a.pad_l;
        const int mlo = a.tab.win_lo[j], mhi = a.tab.win_hi[j];
        const int W = T + (mhi - mlo) + 1;
        const int lo = t0 + mlo;
        if (j == 1) {
            // spline of layer n+1 on the window; the tile's part goes back to
            // HBM for the later steps, with the ghost records
            spline_window<NT, kRaw, P>(g, a.nx, lo, W, wy, wz, R, CAP1, a.pcr, raw1);
            const int kend = min(t0 + T, a.nx);
            for (int k = t0 + tid; k < kend; k += NT) {
                const int sl = WinLayout<P>::slot(k - lo + kHalo);
                g[k].My = wy[sl].y;
                g[k].Mz = wz[sl].y;
            }
            if (tile == 0) {
                const double y0 = g[0].y, z0 = g[0].z;
                for (int k = tid; k < a.pad_l; k += NT) g[k - a.pad_l] = Rec64{y0, 0.0, z0, 0.0};
            }
            if (tile == (int)gridDim.x - 1) {
                const double yn = g[a.nx - 1].y, zn = g[a.nx - 1].z;
                for (int k = tid; k < a.pad_r; k += NT) g[a.nx + k] = Rec64{yn, 0.0, zn, 0.0};
            }
        } else {
#pragma unroll
            for (int u = 0; u < kPre; ++u) {
                const int e = tid + u * NT;
                if (e < W) {
                    const int sl = WinLayout<P>::slot(kHalo + e);
                    wy[sl] = make_double2(pre[u].y, pre[u].My);
                    wz[sl] = make_double2(pre[u].z, pre[u].Mz);
                }
            }
            if (j + 1 <= a.K) prefetch(j + 1);
            __syncthreads();
        }
        const LdsWindow<P> src{wy, kHalo - mlo,
                               WinLayout<P>::kPad ? lane_pt + lane_pt / P : lane_pt};
        layer_dispatch<P, DRV>(src, trec, tm, tcy, j, grp, G, a, Y, Z);
        __syncthreads();  // the window is reused by the next layer
    }
    if (G > 1) {  // partial sums of groups 1..G-1 meet group 0 in LDS, in group order
        double *red = reinterpret_cast<double *>(smem);
        if (grp > 0) {
#pragma unroll
            for (int q = 0; q < P; ++q) {
                red[(((grp - 1) * kBlock + tid % kBlock) * P + q) * 2] = Y[q];
                red[(((grp - 1) * kBlock + tid % kBlock) * P + q) * 2 + 1] = Z[q];
            }
        }
        __syncthreads();
        if (grp > 0) return;
        for (int h = 1; h < G; ++h) {
#pragma unroll
            for (int q = 0; q < P; ++q) {
                Y[q] += red[(((h - 1) * kBlock + tid) * P + q) * 2];
                Z[q] += red[(((h - 1) * kBlock + tid) * P + q) * 2 + 1];
            }
        }
    }
    finish_points<P, DRV>(a, t0 + lane_pt, Y, Z);
}

// ---------------------------------------------------------------------------
// Direct sweep: records from HBM/L2, P consecutive points per lane.
// Dynamic LDS: node table only.
// ---------------------------------------------------------------------------
template <int P, int DRV>
__global__ void __launch_bounds__(kBlock) sweep_direct(const SweepArgs a)
{
    extern __shared__ double2 smem[];
    NodeRec *trec = reinterpret_cast<NodeRec *>(smem);
    int *tm = reinterpret_cast<int *>(trec + a.K * a.L);
    double *tcy = reinterpret_cast<double *>(tm + ((a.K * a.L + 1) & ~1));
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int first = (tile * kBlock + (int)threadIdx.x) * P;
    const int i0 = min(first, a.nx - 1);  // lanes past the end read in bounds, store nothing
    const int S = a.K + 1;
    load_node_table<kBlock>(a.tab, a.K * a.L, trec, tm, tcy);
    double Y[P], Z[P];
#pragma unroll
    for (int q = 0; q < P; ++q) Y[q] = Z[q] = 0.0;
    for (int j = 1; j <= a.K; ++j) {
        const GlobalWindow src{a.ring + (size_t)((a.n + j) % S) * a.npad + a.pad_l + i0};
        layer_dispatch<P, DRV>(src, trec, tm, tcy, j, 0, 1, a, Y, Z);
    }
    finish_points<P, DRV>(a, first, Y, Z);
}

// ---------------------------------------------------------------------------
// Standalone natural spline of one layer (initial layers; direct path).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) spline_f64(Rec64 *slot, int nx, int pad_l, int pad_r,
                                                     const PcrCoef c)
{
    constexpr int WE = kSplineTile + 2 * kHalo, WS = WE + 2;
    __shared__ double2 wy[WE], wz[WE];
    __shared__ double R[4 * WS];
    Rec64 *__restrict__ g = slot + pad_l;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int t0 = tile * kSplineTile;
    constexpr int U = (WS + kBlock - 1) / kBlock;
    SplineRaw<U> raw;
    spline_load<kBlock, U>(g, nx, t0, kSplineTile, raw);
    spline_window<kBlock, U, 1>(g, nx, t0, kSplineTile, wy, wz, R, WS, c, raw);
    const int kend = min(t0 + kSplineTile, nx);
    for (int k = t0 + (int)threadIdx.x; k < kend; k += kBlock) {
        g[k].My = wy[k - t0 + kHalo].y;
        g[k].Mz = wz[k - t0 + kHalo].y;
    }
    if (tile == 0) {
        const double y0 = g[0].y, z0 = g[0].z;
        for (int k = threadIdx.x; k < pad_l; k += kBlock) slot[k] = Rec64{y0, 0.0, z0, 0.0};
    }
    if (tile == (int)gridDim.x - 1) {
        const double yn = g[nx - 1].y, zn = g[nx - 1].z;
        for (int k = threadIdx.x; k < pad_r; k += kBlock) g[nx + k] = Rec64{yn, 0.0, zn, 0.0};
    }
}

// ---------------------------------------------------------------------------
// Input / output / statistics kernels
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
scatter_layers(Rec64 *ring, int npad, int pad_l, int nx, int N, int K,
               const double *__restrict__ iy, const double *__restrict__ iz)
{
    const int r = blockIdx.y;  // layer t_{N-K+1+r}
    const int n = N - K + 1 + r;
    Rec64 *__restrict__ g = ring + (size_t)(n % (K + 1)) * npad + pad_l;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < nx; i += gridDim.x * kBlock) {
        g[i].y = iy[(size_t)r * nx + i];
        g[i].z = iz[(size_t)r * nx + i];
    }
}

__global__ void __launch_bounds__(kBlock)
gather_layer(const Rec64 *__restrict__ g, int nx, double *__restrict__ y0,
             double *__restrict__ z0, unsigned long long *nonfinite)
{
    unsigned int bad = 0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < nx; i += gridDim.x * kBlock) {
        const double y = g[i].y, z = g[i].z;
        y0[i] = y;
        z0[i] = z;
        bad += (isfinite(y) && isfinite(z)) ? 0u : 1u;
    }
    bad = wave_sum_u32(bad);
    if (nonfinite && (threadIdx.x & 63) == 0 && bad) atomicAdd(nonfinite, (unsigned long long)bad);
}

__global__ void __launch_bounds__(kBlock) clear_u64(unsigned long long *p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kBlock)
        p[i] = 0ull;
}

// totals[0] = max iterations, [1] = sum, [2] = unconverged
__global__ void __launch_bounds__(kBlock)
reduce_stats(const unsigned int *imax, const unsigned long long *isum,
             const unsigned long long *nonc, int nw, unsigned long long *totals)
{
    __shared__ unsigned long long sm[3][kBlock];
    unsigned long long m = 0, s = 0, c = 0;
    for (int w = threadIdx.x; w < nw; w += kBlock) {
        m = max(m, (unsigned long long)imax[w]);
        s += isum[w];
        c += nonc[w];
    }
    sm[0][threadIdx.x] = m;
    sm[1][threadIdx.x] = s;
    sm[2][threadIdx.x] = c;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sm[0][threadIdx.x] = max(sm[0][threadIdx.x], sm[0][threadIdx.x + o]);
            sm[1][threadIdx.x] += sm[1][threadIdx.x + o];
            sm[2][threadIdx.x] += sm[2][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        totals[0] = sm[0][0];
        totals[1] = sm[1][0];
        totals[2] = sm[2][0];
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
namespace {

template <int P, int G, int DRV>
hipError_t launch_fused_t(const SweepArgs &a, int blocks, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((sweep_fused<P, G, DRV>), dim3(blocks), dim3(kBlock * G), lds, s, a);
    return hipGetLastError();
}

template <int P, int DRV>
hipError_t launch_direct_t(const SweepArgs &a, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL((sweep_direct<P, DRV>), dim3(blocks), dim3(kBlock),
                       node_table_lds(a.K * a.L), s, a);
    return hipGetLastError();
}

template <int P, int G>
hipError_t fused_by_driver(const SweepArgs &a, int driver, int blocks, size_t lds, hipStream_t s)
{
    switch (driver) {
    case BSDE_DRIVER_LINEAR: return launch_fused_t<P, G, BSDE_DRIVER_LINEAR>(a, blocks, lds, s);
    case BSDE_DRIVER_BIDASK: return launch_fused_t<P, G, BSDE_DRIVER_BIDASK>(a, blocks, lds, s);
    case BSDE_DRIVER_CUBIC: return launch_fused_t<P, G, BSDE_DRIVER_CUBIC>(a, blocks, lds, s);
    default: return launch_fused_t<P, G, BSDE_DRIVER_EXP>(a, blocks, lds, s);
    }
}

template <int P>
hipError_t direct_by_driver(const SweepArgs &a, int driver, int blocks, hipStream_t s)
{
    switch (driver) {
    case BSDE_DRIVER_LINEAR: return launch_direct_t<P, BSDE_DRIVER_LINEAR>(a, blocks, s);
    case BSDE_DRIVER_BIDASK: return launch_direct_t<P, BSDE_DRIVER_BIDASK>(a, blocks, s);
    case BSDE_DRIVER_CUBIC: return launch_direct_t<P, BSDE_DRIVER_CUBIC>(a, blocks, s);
    default: return launch_direct_t<P, BSDE_DRIVER_EXP>(a, blocks, s);
    }
}

template <int P, int G, int DRV>
hipError_t allow_lds(size_t lds)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&sweep_fused<P, G, DRV>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int P, int G>
hipError_t allow_lds_by_driver(int driver, size_t lds)
{
    switch (driver) {
    case BSDE_DRIVER_LINEAR: return allow_lds<P, G, BSDE_DRIVER_LINEAR>(lds);
    case BSDE_DRIVER_BIDASK: return allow_lds<P, G, BSDE_DRIVER_BIDASK>(lds);
    case BSDE_DRIVER_CUBIC: return allow_lds<P, G, BSDE_DRIVER_CUBIC>(lds);
    default: return allow_lds<P, G, BSDE_DRIVER_EXP>(lds);
    }
}

}  // namespace

bool fused_supported(int P, int G)
{
    return (P == 1 || P == 2 || P == 4) && (G == 1 || G == 2 || G == 4);
}
bool direct_p_supported(int P) { return P == 1 || P == 2 || P == 4; }

size_t node_table_lds(int nodes)
{
    return (size_t)nodes * (sizeof(NodeRec) + sizeof(double)) +
           (size_t)((nodes + 1) & ~1) * sizeof(int);
}

#define BSDE_FUSED_CASES(F, ...)                                       \
    switch (P * 8 + G) {                                               \
    case 1 * 8 + 1: return F<1, 1>(__VA_ARGS__);                       \
    case 1 * 8 + 2: return F<1, 2>(__VA_ARGS__);                       \
    case 1 * 8 + 4: return F<1, 4>(__VA_ARGS__);                       \
    case 2 * 8 + 1: return F<2, 1>(__VA_ARGS__);                       \
    case 2 * 8 + 2: return F<2, 2>(__VA_ARGS__);                       \
    case 2 * 8 + 4: return F<2, 4>(__VA_ARGS__);                       \
    case 4 * 8 + 1: return F<4, 1>(__VA_ARGS__);                       \
    case 4 * 8 + 2: return F<4, 2>(__VA_ARGS__);                       \
    case 4 * 8 + 4: return F<4, 4>(__VA_ARGS__);                       \
    default: return hipErrorInvalidValue;                              \
    }

hipError_t launch_sweep_fused(int P, int G, const SweepArgs &a, int driver, int blocks,
                              size_t lds, hipStream_t s)
{
    BSDE_FUSED_CASES(fused_by_driver, a, driver, blocks, lds, s)
}

hipError_t set_fused_lds_limit(int P, int G, int driver, size_t lds)
{
    BSDE_FUSED_CASES(allow_lds_by_driver, driver, lds)
}

hipError_t launch_sweep_direct(int P, const SweepArgs &a, int driver, int blocks, hipStream_t s)
{
    switch (P) {
    case 1: return direct_by_driver<1>(a, driver, blocks, s);
    case 2: return direct_by_driver<2>(a, driver, blocks, s);
    case 4: return direct_by_driver<4>(a, driver, blocks, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_spline(Rec64 *slot, int nx, int pad_l, int pad_r, const PcrCoef &c,
                         hipStream_t s)
{
    const int blocks = (nx + kSplineTile - 1) / kSplineTile;
    hipLaunchKernelGGL(spline_f64, dim3(blocks), dim3(kBlock), 0, s, slot, nx, pad_l, pad_r, c);
    return hipGetLastError();
}

hipError_t launch_scatter(Rec64 *ring, int npad, int pad_l, int nx, int N, int K,
                          const double *iy, const double *iz, hipStream_t s)
{
    const int gx = std::min(1024, (nx + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(scatter_layers, dim3(gx, K), dim3(kBlock), 0, s, ring, npad, pad_l, nx, N,
                       K, iy, iz);
    return hipGetLastError();
}

hipError_t launch_gather(const Rec64 *g, int nx, double *y0, double *z0,
                         unsigned long long *nonfinite, hipStream_t s)
{
    const int gx = std::min(1024, (nx + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(gather_layer, dim3(gx), dim3(kBlock), 0, s, g, nx, y0, z0, nonfinite);
    return hipGetLastError();
}

hipError_t launch_clear(unsigned long long *p, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(clear_u64, dim3(64), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_reduce_stats(const unsigned int *imax, const unsigned long long *isum,
                               const unsigned long long *nonc, int nw, unsigned long long *totals,
                               hipStream_t s)
{
    hipLaunchKernelGGL(reduce_stats, dim3(1), dim3(kBlock), 0, s, imax, isum, nonc, nw, totals);
    return hipGetLastError();
}

}  // namespace bsde

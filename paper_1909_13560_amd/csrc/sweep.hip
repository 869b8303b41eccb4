// sweep.hip -- kernels of the backward sweep (arXiv:1909.13560, Section 2.2
// eq (20)-(21), Section 3.1 step 3, Section 3.2) and their host-side
// launchers, in the FP64 and the FP32 form.
//
// Every kernel serves a group of instances: the grid's tiles are numbered
// instance after instance, a device table maps a tile to its instance, and
// each block reads that instance's descriptor (a single solve is a group of
// one).  One launch per time step advances every instance still active by one
// layer; instances are sorted by their number of steps, so the active ones
// are a prefix of the group and the launch covers exactly their tiles.
//
// Two sweep kernels compute layer n from layers n+1..n+K:
//   sweep_fused  a block owns a tile of kBlock*P consecutive grid points.  For
//                each layer j it stages the records its nodes touch (the tile
//                widened by the node offsets of layer j) in LDS; for j = 1 it
//                first solves that layer's natural spline on the window by
//                truncated PCR and writes the tile's second derivatives back
//                to HBM, so no separate spline launch is needed.  Each lane
//                handles P consecutive points.
//   sweep_direct (node reach too wide for the LDS windows): records are read
//                straight from HBM/L2, P consecutive points per lane; the
//                natural spline of the new layer is a separate launch.
#include "device_common.h"
#include "kernels.h"

namespace bsde {

// Node records read from the LDS window (fused kernel).  Window element e of
// the lane's q-th record is lane_pt + off + q with off = ebase + m >= 0; with
// the padded layout its slot is
//   (P+1) tig + off + off/P + q + [q >= P - off % P]   (tig = lane_pt / P),
// so the per-record offsets are one of P compile-time patterns.  The FP64
// form reads (y, z) and, window_slots(P) slots further, (M_y, M_z).
template <int P, int B, bool PAD, int NA, typename V>
__device__ inline void fetch_slots(const V *w, int base, V (&r)[NA][P + 1])
{
    const V *p = w + base;
#pragma unroll
    for (int q = 0; q <= P; ++q) {
        const int sl = q + ((PAD && q >= P - B) ? 1 : 0);
#pragma unroll
        for (int k = 0; k < NA; ++k) r[k][q] = p[sl + k * window_slots(P)];
    }
}

template <int P, bool F32>
struct LdsWindow {
    using V = typename Prec<F32>::V;
    static constexpr int NA = Prec<F32>::NA;
    const V *w;
    int ebase;  // kHalo - (lowest node offset of the layer): off = ebase + m
    int lane;   // slot of the lane's first element at off = 0: (P+1) tig padded, P tig not
    template <int PP>
    __device__ void fetch(int m, V (&r)[NA][PP + 1]) const
    {
        static_assert(PP == P, "window layout and fetch width differ");
        const int off = ebase + m;
        if constexpr (!WinLayout<P>::kPad) {
            fetch_slots<P, 0, false, NA>(w, lane + off, r);
        } else {
            const int base = lane + off + off / P;
            switch (off % P) {
            case 0: fetch_slots<P, 0, true, NA>(w, base, r); break;
            case 1: fetch_slots<P, 1, true, NA>(w, base, r); break;
            case 2: fetch_slots<P, (P > 2 ? 2 : 1), true, NA>(w, base, r); break;
            default: fetch_slots<P, (P > 3 ? 3 : 1), true, NA>(w, base, r); break;
            }
        }
    }
};

// Node records read straight from the layer in HBM (direct kernel).
template <bool F32>
struct GlobalWindow {
    using V = typename Prec<F32>::V;
    static constexpr int NA = Prec<F32>::NA;
    Slot<F32> lay;  // the layer
    int i0;         // the lane's first point
    template <int P>
    __device__ void fetch(int m, V (&r)[NA][P + 1]) const
    {
#pragma unroll
        for (int q = 0; q <= P; ++q) {
            const auto v = lay.val(i0 + m + q), mm = lay.der(i0 + m + q);
            if constexpr (F32) {
                r[0][q] = make_float4(v.x, v.y, mm.x, mm.y);
            } else {
                r[0][q] = v;
                r[1][q] = mm;
            }
        }
    }
};

// YW: the kernel serves the E[y^{n+1} dW]/dt form of the z equation too (the
// direct kernel).  The fused kernel leaves it out: its two extra node-loop
// variants cost the kernel scalar registers (more spills) for a form that the
// plan sends to the direct kernel.
template <int P, int DRV, bool F32, bool YW, typename Src>
__device__ inline void layer_dispatch(const Src &src, const int *tm, int j, int l0, int LS,
                                      const SweepArgs &a, Acc<P> &acc, int lend)
// nodes l = l0, l0 + LS, ... < lend of layer j
{
    using Node = typename Prec<F32>::Node;
    const Driver<DRV, typename Prec<F32>::Raw> f(a.drv, (a.n + j) * a.dt);
    const int row = (j - 1) * a.L;
    const Node *nodes = node_recs(a.tab, static_cast<Node *>(nullptr)) + row;
    const bool last_y = j == a.Ky;
    if constexpr (YW) {
        if (j == 1 && a.zform) {
            if (last_y)
                layer_nodes<P, DRV, kNodeLastY | kNodeYW, F32>(src, nodes, tm + row, l0, LS, lend,
                                                               f, acc);
            else
                layer_nodes<P, DRV, kNodeYW, F32>(src, nodes, tm + row, l0, LS, lend, f, acc);
            return;
        }
    }
    if (last_y)
        layer_nodes<P, DRV, kNodeLastY, F32>(src, nodes, tm + row, l0, LS, lend, f, acc);
    else
        layer_nodes<P, DRV, 0, F32>(src, nodes, tm + row, l0, LS, lend, f, acc);
}

// LDS bytes of the window arrays of the fused kernel.
template <bool F32>
__host__ __device__ constexpr size_t window_lds_bytes(int P)
{
    return (size_t)window_slots(P) * (F32 ? sizeof(float4) : 2 * sizeof(double2));
}

// ---------------------------------------------------------------------------
// Fused sweep of one tile: LDS-staged windows, in-kernel spline of layer n+1.
// A block of G*kBlock threads owns a tile of kBlock*P points; thread group g
// (kBlock threads) takes the nodes l = g, g+G, ... of every layer, and the G
// partial sums meet in LDS before group 0 finishes the points.
// Dynamic LDS: the window arrays, the four PCR arrays (pcr_values(P)
// doubles each) and the node offsets (K*L int).
// ---------------------------------------------------------------------------
// Wave priority of a node loop with `left` more node loops to go in this
// block: a block that is behind gets the higher priority (up to 3), so the
// blocks sharing a CU, which start together, also end close together (the
// launch ends with its last block).
__device__ inline void node_loop_priority(int left)
{
    switch (left) {
    case 0: __builtin_amdgcn_s_setprio(0); break;
    case 1: __builtin_amdgcn_s_setprio(1); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    default: __builtin_amdgcn_s_setprio(3); break;
    }
}

template <int P, int G, int DRV, bool F32>
__device__ inline void fused_tile(const SweepArgs &a, int tile, char *smem)
{
    using PR = Prec<F32>;
    using E = typename PR::E;
    using V = typename PR::V;
    constexpr int T = kBlock * P;
    constexpr int NT = kBlock * G;
    constexpr int CAP1 = pcr_values(P);
    V *wbase = reinterpret_cast<V *>(smem);
    const typename PR::template Win<P> win{wbase};
    double *R = reinterpret_cast<double *>(smem + window_lds_bytes<F32>(P));
    int *tm = reinterpret_cast<int *>(R + 4 * CAP1);

    const int tid = threadIdx.x;
    // kBlock is a multiple of the wavefront size: the group is wave-uniform
    const int grp = __builtin_amdgcn_readfirstlane(tid / kBlock);
    const int lane_pt = (tid % kBlock) * P;
    const int t0 = tile * T;

    Acc<P> acc;
#pragma unroll
    for (int q = 0; q < P; ++q) acc.Y[q] = acc.Z[q] = 0.0;

    // Layers are processed in the order 2, 3, ..., K, 1, rotated per tile: the
    // records of layers n+2.. are complete (their splines were built by
    // earlier launches) and their windows are prefetched into registers one
    // layer ahead, while the raw values of layer n+1 (written by the previous
    // launch) are loaded at the start and turned into its spline at its turn.
    // The rotation key (tile / 32) differs between the blocks that share a CU
    // (tiles 32 apart under the XCD-aware numbering), so their spline and
    // node phases fall at different times; it depends on the tile alone, so a
    // tile computes the same in a batch as on its own.
    constexpr int kPre = (T + kMaxReach2 + NT - 1) / NT;
    constexpr int kRaw = pcr_slots(P, NT);
    using FT = typename Slot<F32>::T;
    struct Frag {  // plain scalars, so that the array lives in registers
        FT y, z, My, Mz;
    } pre[kPre];   // the next window, both fragments
    auto prefetch = [&](int j) {
        const Slot<F32> g = ring_slot<F32>(a, a.n + j);
        const int lo = t0 + a.tab.win_lo[j];
        const int W = T + (a.tab.win_hi[j] - a.tab.win_lo[j]) + 1;
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
            const int e = tid + u * NT;
            if (e < W) {
                const E v = g.val(lo + e), m = g.der(lo + e);
                pre[u] = Frag{v.x, v.y, m.x, m.y};
            }
        }
    };
    const int rot = ((tile >> 5) & 3) % a.K;
    // Issue priority: everything but the node loops (staging waits, the
    // spline's barriers, Picard) runs at the highest wave priority, so a
    // block's latency-bound phases go ahead of the node loops of the blocks
    // sharing its CU instead of queueing behind them; the node loops
    // (throughput work) run lower, the lower the further the block has got
    // (node_loop_priority).
    __builtin_amdgcn_s_setprio(3);
    auto layer_at = [&](int jj) {  // the jj-th layer of this tile's order
        const int q = (jj + rot) % a.K;
        return q + 1 < a.K ? q + 2 : 1;
    };
    auto next_window = [&](int jj) {  // first layer after position jj other than n+1
        for (int q = jj + 1; q < a.K; ++q)
            if (layer_at(q) != 1) return layer_at(q);
        return 0;
    };
    SplineRaw<kRaw, typename PR::Raw> raw1;
    {
        const Slot<F32> g1 = ring_slot<F32>(a, a.n + 1);
        const int W1 = T + (a.tab.win_hi[1] - a.tab.win_lo[1]) + 1;
        const int j0 = layer_at(0) != 1 ? layer_at(0) : next_window(0);
        if (j0) prefetch(j0);
        spline_load<NT, kRaw>(g1, a.nx, t0 + a.tab.win_lo[1], W1, raw1);
    }
    // node offsets into LDS only now: their stores wait for the loads, which
    // must not hold back the issue of the window loads above (published by
    // the first barrier)
    for (int i = tid; i < a.K * a.L; i += NT) tm[i] = a.tab.m[i];

    for (int jj = 0; jj < a.K; ++jj) {
        const int j = layer_at(jj);
        const Slot<F32> g = ring_slot<F32>(a, a.n + j);
        const int mlo = a.tab.win_lo[j], mhi = a.tab.win_hi[j];
        const int W = T + (mhi - mlo) + 1;
        const int lo = t0 + mlo;
        if (j == 1) {
            // spline of layer n+1 on the window; the tile's part goes back to
            // HBM for the later steps, with the ghost records
            spline_window<NT, kRaw, P>(g, a.nx, lo, W, win, R, CAP1, a.pcr, raw1);
            const int kend = min(t0 + T, a.nx);
            for (int k = t0 + tid; k < kend; k += NT) {
                const double2 d = win.ders(WinLayout<P>::slot(k - lo + kHalo));
                g.set_der(k, d.x, d.y);
            }
            if (tile == 0) {
                const auto e0 = g.val(0);
                for (int k = tid; k < a.pad_l; k += NT) {
                    g.set_val(k - a.pad_l, e0);
                    g.set_der(k - a.pad_l, 0.0, 0.0);
                }
            }
            if (tile == a.ntiles - 1) {
                const auto e1 = g.val(a.nx - 1);
                for (int k = tid; k < a.pad_r; k += NT) {
                    g.set_val(a.nx + k, e1);
                    g.set_der(a.nx + k, 0.0, 0.0);
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < kPre; ++u) {
                const int e = tid + u * NT;
                if (e < W)
                    win.put(WinLayout<P>::slot(kHalo + e), E{pre[u].y, pre[u].z},
                            E{pre[u].My, pre[u].Mz});
            }
            const int jn = next_window(jj);
            if (jn) prefetch(jn);
            __syncthreads();
        }
        const LdsWindow<P, F32> src{wbase, kHalo - mlo,
                                    WinLayout<P>::kPad ? lane_pt + lane_pt / P : lane_pt};
        node_loop_priority(a.K - 1 - jj);
        layer_dispatch<P, DRV, F32, false>(src, tm, j, grp, G, a, acc, a.L);
        __builtin_amdgcn_s_setprio(3);
        __syncthreads();  // the window is reused by the next layer
    }
    if (G > 1) {  // partial sums of groups 1..G-1 meet group 0 in LDS, in group order
        double *red = reinterpret_cast<double *>(smem);
        if (grp > 0) {
#pragma unroll
            for (int q = 0; q < P; ++q) {
                red[(((grp - 1) * kBlock + tid % kBlock) * P + q) * 2] = acc.Y[q];
                red[(((grp - 1) * kBlock + tid % kBlock) * P + q) * 2 + 1] = acc.Z[q];
            }
        }
        __syncthreads();
        if (grp > 0) return;
        for (int h = 1; h < G; ++h) {
#pragma unroll
            for (int q = 0; q < P; ++q) {
                acc.Y[q] += red[(((h - 1) * kBlock + tid) * P + q) * 2];
                acc.Z[q] += red[(((h - 1) * kBlock + tid) * P + q) * 2 + 1];
            }
        }
    }
    finish_points<P, DRV, F32>(a, t0 + lane_pt, acc, (tile * kBlock + tid) >> 6);
}

template <int P, int G, int DRV, bool F32>
__global__ void __launch_bounds__(kBlock * G) sweep_fused(const StepArgs s)
{
    extern __shared__ double2 smem_fused[];
    const int idx = xcd_tile(blockIdx.x, gridDim.x);
    const InstDesc &d = block_desc(s, idx);
    const SweepArgs a = bind_instance(d, s.ws, s.s, s.stats != 0);
    fused_tile<P, G, DRV, F32>(a, idx - d.tile_base, reinterpret_cast<char *>(smem_fused));
}

// ---------------------------------------------------------------------------
// Direct sweep: records from HBM/L2, P consecutive points per lane.
// Dynamic LDS: node table only.  The nodes are summed chunk by chunk
// (kDirectChunk nodes of one layer, each chunk from zero, the chunks added in
// order); on a small grid a tile's chunks are split over s.dsplit blocks
// (P = 1), which write the chunk sums for direct_finish.
// ---------------------------------------------------------------------------
template <int P, int DRV, bool F32, bool SPLIT>
__global__ void __launch_bounds__(kBlock) sweep_direct(const StepArgs s)
{
    static_assert(!SPLIT || P == 1, "split direct steps take one point per lane");
    const int S = SPLIT ? s.dsplit : 1;
    const int idx = xcd_tile(blockIdx.x, gridDim.x);
    const int tg = SPLIT ? idx / S : idx, sp = SPLIT ? idx - tg * S : 0;  // tile of the group, split
    const InstDesc &d = block_desc(s, tg);
    const SweepArgs a = bind_instance(d, s.ws, s.s, s.stats != 0);
    const int tile = tg - d.tile_base;
    __shared__ int tm[kMaxNodes];
    for (int i = threadIdx.x; i < a.K * a.L; i += kBlock) tm[i] = a.tab.m[i];
    __syncthreads();
    const int first = (tile * kBlock + (int)threadIdx.x) * P;
    const int i0 = min(first, a.nx - 1);  // lanes past the end read in bounds, store nothing
    Acc<P> acc;
#pragma unroll
    for (int q = 0; q < P; ++q) acc.Y[q] = acc.Z[q] = 0.0;
    const int nch = (a.L + kDirectChunk - 1) / kDirectChunk;  // chunks per layer
    for (int j = 1, c = 0; j <= a.K; ++j) {
        const GlobalWindow<F32> src{ring_slot<F32>(a, a.n + j), i0};
        for (int h = 0; h < nch; ++h, ++c) {
            if (SPLIT && c % S != sp) continue;
            Acc<P> ch;
#pragma unroll
            for (int q = 0; q < P; ++q) ch.Y[q] = ch.Z[q] = 0.0;
            layer_dispatch<P, DRV, F32, true>(src, tm, j, h * kDirectChunk, 1, a, ch,
                                              min(a.L, (h + 1) * kDirectChunk));
            if constexpr (SPLIT) {
                double *p = s.part + ((size_t)tg * s.dchunks + c) * 2 * kBlock;
                p[threadIdx.x] = ch.Y[0];
                p[kBlock + threadIdx.x] = ch.Z[0];
            } else {
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    acc.Y[q] += ch.Y[q];
                    acc.Z[q] += ch.Z[q];
                }
            }
        }
    }
    if constexpr (!SPLIT)
        finish_points<P, DRV, F32>(a, first, acc, (tile * kBlock + (int)threadIdx.x) >> 6);
}

// A split direct step: the chunk sums of a tile added in chunk order, then
// the implicit y equation (Picard) of its points.  Loads go out four chunks
// at a time.
template <int DRV, bool F32>
__global__ void __launch_bounds__(kBlock) direct_finish(const StepArgs s)
{
    const int tg = xcd_tile(blockIdx.x, gridDim.x);
    const InstDesc &d = block_desc(s, tg);
    const SweepArgs a = bind_instance(d, s.ws, s.s, s.stats != 0);
    const int tile = tg - d.tile_base, tid = threadIdx.x;
    const int C = direct_chunks(a.K, a.L);
    const double *p = s.part + (size_t)tg * s.dchunks * 2 * kBlock + tid;
    Acc<1> acc;
    acc.Y[0] = acc.Z[0] = 0.0;
    for (int c0 = 0; c0 < C; c0 += 4) {
        double vy[4], vz[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            vy[q] = c0 + q < C ? p[(size_t)(c0 + q) * 2 * kBlock] : 0.0;
            vz[q] = c0 + q < C ? p[(size_t)(c0 + q) * 2 * kBlock + kBlock] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (c0 + q < C) {
                acc.Y[0] += vy[q];
                acc.Z[0] += vz[q];
            }
    }
    finish_points<1, DRV, F32>(a, tile * kBlock + tid, acc, (tile * kBlock + tid) >> 6);
}

// ---------------------------------------------------------------------------
// Gather sweep: forward coefficients that depend on the state (eq (1)),
// affine in x or tabulated on the grid (and then also per time step).  The
// node of (j, l) for point x_i is one Euler step of X over j dt from t_n,
//   X = x_i + a(t_n, x_i) j dt + b(t_n, x_i) sqrt(2 j dt) a_l,
// so its cell and fraction differ from point to point: each lane locates
// its nodes (Section 3.2: floor on the uniform grid, the boundary value
// outside the truncated domain), forms the spline basis weights at the
// fraction and reads the two records from HBM/L2.  One point per lane; the
// natural spline of the new layer is a separate launch.
// ---------------------------------------------------------------------------
template <int DRV, bool F32>
__global__ void __launch_bounds__(kBlock) sweep_gather(const StepArgs s)
{
    using PR = Prec<F32>;
    using Node = typename PR::Node;
    using V = typename PR::V;
    const int idx = xcd_tile(blockIdx.x, gridDim.x);
    const InstDesc &d = block_desc(s, idx);
    const SweepArgs a = bind_instance(d, s.ws, s.s, s.stats != 0);
    const int tile = idx - d.tile_base;
    const int first = tile * kBlock + (int)threadIdx.x;
    const int i = min(first, a.nx - 1);  // lanes past the end compute in bounds, store nothing
    const double xi = a.x_min + i * a.dx;
    double ax, bx;
    if (a.ctab) {  // tabulated a(t_n, x_i), b(t_n, x_i)
        const double *row = a.ctab + (size_t)2 * (a.tab_steps > 1 ? a.n : 0) * a.nx;
        ax = row[i];
        bx = row[a.nx + i];
    } else {
        ax = fma(a.drift_x, xi, a.drift0);
        bx = fma(a.vol_x, xi, a.vol0);
    }
    const double dx26 = a.dx * a.dx / 6.0;
    Acc<1> acc;
    acc.Y[0] = acc.Z[0] = 0.0;
    for (int j = 1; j <= a.K; ++j) {
        const Slot<F32> g = ring_slot<F32>(a, a.n + j);
        const Driver<DRV, typename PR::Raw> f(a.drv, (a.n + j) * a.dt);
        const int row = (j - 1) * a.L;
        const Node *nodes = node_recs(a.tab, static_cast<Node *>(nullptr)) + row;
        const int nf = (j == a.Ky ? kNodeLastY : 0) | (j == 1 && a.zform ? kNodeYW : 0);
        if (F32) acc.Yf[0] = acc.Zf[0] = 0.0f;
        for (int l = 0; l < a.L; ++l) {
            const double X = xi + ax * (j * a.dt) + bx * a.tab.dw[row + l];
            const double sx = (X - a.x_min) / a.dx;
            int p = 0;
            double phi = 0.0;
            if (sx >= (double)(a.nx - 1)) {
                p = a.nx - 1;  // the last record; its right neighbour is a ghost, weight 0
            } else if (sx > 0.0) {
                p = min((int)floor(sx), a.nx - 2);
                phi = sx - p;
            }
            const double u = 1.0 - phi;
            Node c = load_node(nodes + l);
            c.B = phi;
            c.C = dx26 * (u * u * u - u);
            c.D = dx26 * (phi * phi * phi - phi);
            V r[PR::NA][2];
            GlobalWindow<F32>{g, p}.template fetch<1>(0, r);
            switch (nf) {
            case 0: node_accumulate<1, DRV, 0>(r, c, f, acc); break;
            case kNodeLastY: node_accumulate<1, DRV, kNodeLastY>(r, c, f, acc); break;
            case kNodeYW: node_accumulate<1, DRV, kNodeYW>(r, c, f, acc); break;
            default: node_accumulate<1, DRV, kNodeLastY | kNodeYW>(r, c, f, acc); break;
            }
        }
        if (F32) {
            acc.Y[0] += (double)acc.Yf[0];
            acc.Z[0] += (double)acc.Zf[0];
        }
    }
    finish_points<1, DRV, F32>(a, first, acc, (tile * kBlock + (int)threadIdx.x) >> 6);
}

// ---------------------------------------------------------------------------
// Standalone natural spline of one layer per instance: the initial layers
// (mode 0: layer n0 + 1 + s) and, on the direct path, the layer just computed
// (mode 1: layer n0 - s, skipped at n_stop, which no later step reads).
// ---------------------------------------------------------------------------
template <bool F32>
__global__ void __launch_bounds__(kBlock) spline_layer(const StepArgs s, int mode)
{
    using V = typename Prec<F32>::V;
    constexpr int WE = kSplineTile + 2 * kHalo, WS = WE + 2;
    static_assert(WE <= window_slots(1), "spline tile exceeds the window layout");
    __shared__ V wsm[window_lds_bytes<F32>(1) / sizeof(V)];
    __shared__ double R[4 * WS];
    const int idx = xcd_tile(blockIdx.x, gridDim.x);
    const InstDesc &d = block_desc(s, idx);
    const SweepArgs a = bind_instance(d, s.ws, 0, false);
    const int tile = idx - d.spline_base;
    const int n = mode == 0 ? d.n0 + 1 + s.s : d.n0 - s.s;
    if (mode == 0 && s.s >= a.K) return;
    if (mode == 1 && n <= a.n_stop) return;
    const Slot<F32> g = ring_slot<F32>(a, n);
    const typename Prec<F32>::template Win<1> win{wsm};
    const int t0 = tile * kSplineTile;
    constexpr int U = (WS + kBlock - 1) / kBlock;
    SplineRaw<U, typename Prec<F32>::Raw> raw;
    spline_load<kBlock, U>(g, a.nx, t0, kSplineTile, raw);
    spline_window<kBlock, U, 1>(g, a.nx, t0, kSplineTile, win, R, WS, a.pcr, raw);
    const int kend = min(t0 + kSplineTile, a.nx);
    for (int k = t0 + (int)threadIdx.x; k < kend; k += kBlock) {
        const double2 dd = win.ders(k - t0 + kHalo);
        g.set_der(k, dd.x, dd.y);
    }
    if (tile == 0) {
        const auto e0 = g.val(0);
        for (int k = threadIdx.x; k < a.pad_l; k += kBlock) {
            g.set_val(k - a.pad_l, e0);
            g.set_der(k - a.pad_l, 0.0, 0.0);
        }
    }
    if (tile == d.spline_tiles - 1) {
        const auto e1 = g.val(a.nx - 1);
        for (int k = threadIdx.x; k < a.pad_r; k += kBlock) {
            g.set_val(a.nx + k, e1);
            g.set_der(a.nx + k, 0.0, 0.0);
        }
    }
}

// ---------------------------------------------------------------------------
// Input / output / statistics kernels
// ---------------------------------------------------------------------------
// Initial layers r = 0..K-1 (t_{N-K+1+r}) of the instances of a chunk into
// their rings (the records' y and z; the splines follow).
__global__ void __launch_bounds__(kBlock) scatter_layers(const ScatterChunk c, char *ws,
                                                         const InstDesc *desc)
{
    const int b = blockIdx.y;
    const InstDesc &d = desc[c.inst[b]];
    const SweepArgs a = bind_instance(d, ws, 0, false);
    const double *__restrict__ iy = c.iy[b];
    const double *__restrict__ iz = c.iz[b];
    for (int r = 0; r < a.K; ++r) {
        const int n = d.n0 + 1 + r;
        const Slot<false> g64 = ring_slot<false>(a, n);
        const Slot<true> g32 = ring_slot<true>(a, n);
        for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.nx; i += gridDim.x * kBlock) {
            const double y = iy[(size_t)r * a.nx + i], z = iz[(size_t)r * a.nx + i];
            if (d.f32)
                store_fed_back(g32, a.npad, i, y, z, 0.0f, 0.0f);
            else
                g64.set_val(i, y, z);
        }
    }
}

// Layer n_stop (double precision, in the workspace) of the instances of a
// chunk to the caller's buffers, counting non-finite values.
__global__ void __launch_bounds__(kBlock) gather_layers(const GatherChunk c, char *ws,
                                                        const InstDesc *desc,
                                                        unsigned long long *nonfinite)
{
    const int b = blockIdx.y;
    const InstDesc &d = desc[c.inst[b]];
    const int nx = d.a.nx;
    const double *__restrict__ fy = reinterpret_cast<const double *>(ws + d.fin_off);
    const double *__restrict__ fz = fy + nx;
    double *__restrict__ y0 = c.y0[b];
    double *__restrict__ z0 = c.z0[b];
    unsigned int bad = 0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < nx; i += gridDim.x * kBlock) {
        const double y = fy[i], z = fz[i];
        y0[i] = y;
        z0[i] = z;
        bad += (isfinite(y) && isfinite(z)) ? 0u : 1u;
    }
    bad = wave_sum_u32(bad);
    if (nonfinite && (threadIdx.x & 63) == 0 && bad) atomicAdd(nonfinite, (unsigned long long)bad);
}

// Checkpoint export: layers n_stop .. n_stop + K - 1 of one instance (still in
// its ring after a solve stopped at n_stop) into the initial-layer layout, row
// r = layer n_stop + r.  The FP32 form exports the stored value plus its
// residual, which a later scatter splits back into the same pair.
template <bool F32>
__global__ void __launch_bounds__(kBlock) export_layers(const InstDesc *desc, char *ws,
                                                        double *__restrict__ ly,
                                                        double *__restrict__ lz)
{
    const InstDesc &d = *desc;
    SweepArgs a = d.a;
    a.ring = ws + d.ring_off;
    const int r = blockIdx.y, nx = a.nx;
    const Slot<F32> g = ring_slot<F32>(a, a.n_stop + r);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < nx; i += gridDim.x * kBlock) {
        const auto v = g.val(i);
        double y = v.x, z = v.y;
        if constexpr (F32) {
            const float2 e = fed_back_residual(g, a.npad, i);
            y += (double)e.x;
            z += (double)e.y;
        }
        ly[(size_t)r * nx + i] = y;
        lz[(size_t)r * nx + i] = z;
    }
}

hipError_t launch_export_layers(bool f32, const InstDesc *desc, int K, int nx, char *ws,
                                double *ly, double *lz, hipStream_t s)
{
    const dim3 grid((unsigned)std::min(1024, (nx + kBlock - 1) / kBlock), (unsigned)K);
    if (f32)
        hipLaunchKernelGGL(export_layers<true>, grid, dim3(kBlock), 0, s, desc, ws, ly, lz);
    else
        hipLaunchKernelGGL(export_layers<false>, grid, dim3(kBlock), 0, s, desc, ws, ly, lz);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock) clear_u64(unsigned long long *p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kBlock)
        p[i] = 0ull;
}

// Statistics of one instance: totals[0] = max iterations, [1] = sum,
// [2] = unconverged.
__global__ void __launch_bounds__(kBlock)
reduce_stats(char *ws, const InstDesc *desc, unsigned long long *totals)
{
    __shared__ unsigned long long sm[3][kBlock];
    const InstDesc &d = desc[blockIdx.x];
    const int nw = d.nwaves;
    const unsigned long long *isum = reinterpret_cast<const unsigned long long *>(ws + d.stat_off);
    const unsigned long long *nonc = isum + nw;
    const unsigned int *imax = reinterpret_cast<const unsigned int *>(isum + 2 * nw);
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
        totals[3 * blockIdx.x + 0] = sm[0][0];
        totals[3 * blockIdx.x + 1] = sm[1][0];
        totals[3 * blockIdx.x + 2] = sm[2][0];
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
namespace {

template <int P, int G, int DRV, bool F32>
hipError_t launch_fused_t(const StepArgs &a, int blocks, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((sweep_fused<P, G, DRV, F32>), dim3(blocks), dim3(kBlock * G), lds, s, a);
    return hipGetLastError();
}

template <int P, int DRV, bool F32>
hipError_t launch_direct_t(const StepArgs &a, int blocks, size_t lds, hipStream_t s)
{
    if (a.dsplit == 1) {
        hipLaunchKernelGGL((sweep_direct<P, DRV, F32, false>), dim3(blocks), dim3(kBlock), lds, s, a);
        return hipGetLastError();
    }
    if constexpr (P == 1) {
        hipLaunchKernelGGL((sweep_direct<1, DRV, F32, true>), dim3(blocks * a.dsplit), dim3(kBlock),
                           lds, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((direct_finish<DRV, F32>), dim3(blocks), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;  // split steps take one point per lane
}

template <int P, int DRV, bool F32>
hipError_t launch_gather_t(const StepArgs &a, int blocks, size_t, hipStream_t s)
{
    static_assert(P == 1, "one point per lane");
    hipLaunchKernelGGL((sweep_gather<DRV, F32>), dim3(blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int P, int G, int DRV, bool F32>
hipError_t allow_lds_t(size_t lds)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&sweep_fused<P, G, DRV, F32>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

#define BSDE_BY_DRIVER(F, TP, ...)                                     \
    switch (driver) {                                                  \
    case BSDE_DRIVER_LINEAR: return F<TP, BSDE_DRIVER_LINEAR, F32>(__VA_ARGS__); \
    case BSDE_DRIVER_BIDASK: return F<TP, BSDE_DRIVER_BIDASK, F32>(__VA_ARGS__); \
    case BSDE_DRIVER_CUBIC: return F<TP, BSDE_DRIVER_CUBIC, F32>(__VA_ARGS__);   \
    default: return F<TP, BSDE_DRIVER_EXP, F32>(__VA_ARGS__);                    \
    }

template <int P, int G, bool F32>
hipError_t fused_by_driver(int driver, const StepArgs &a, int blocks, size_t lds, hipStream_t s)
{
#define BSDE_PG P, G
    BSDE_BY_DRIVER(launch_fused_t, BSDE_PG, a, blocks, lds, s)
}

template <int P, int G, bool F32>
hipError_t allow_by_driver(int driver, size_t lds)
{
    BSDE_BY_DRIVER(allow_lds_t, BSDE_PG, lds)
#undef BSDE_PG
}

template <int P, bool F32>
hipError_t direct_by_driver(int driver, const StepArgs &a, int blocks, size_t lds, hipStream_t s)
{
    BSDE_BY_DRIVER(launch_direct_t, P, a, blocks, lds, s)
}

template <bool F32>
hipError_t gather_by_driver(int driver, const StepArgs &a, int blocks, hipStream_t s)
{
    BSDE_BY_DRIVER(launch_gather_t, 1, a, blocks, 0, s)
}

#undef BSDE_BY_DRIVER

#define BSDE_FUSED_CASES(F, ...)                                        \
    switch (P * 8 + G) {                                                \
    case 1 * 8 + 1: return F32 ? F<1, 1, true>(__VA_ARGS__) : F<1, 1, false>(__VA_ARGS__); \
    case 1 * 8 + 2: return F32 ? F<1, 2, true>(__VA_ARGS__) : F<1, 2, false>(__VA_ARGS__); \
    case 2 * 8 + 1: return F32 ? F<2, 1, true>(__VA_ARGS__) : F<2, 1, false>(__VA_ARGS__); \
    case 2 * 8 + 2: return F32 ? F<2, 2, true>(__VA_ARGS__) : F<2, 2, false>(__VA_ARGS__); \
    case 4 * 8 + 1: return F32 ? F<4, 1, true>(__VA_ARGS__) : F<4, 1, false>(__VA_ARGS__); \
    case 4 * 8 + 2: return F32 ? F<4, 2, true>(__VA_ARGS__) : F<4, 2, false>(__VA_ARGS__); \
    default: return hipErrorInvalidValue;                               \
    }

}  // namespace

bool fused_supported(int P, int G) { return (P == 1 || P == 2 || P == 4) && (G == 1 || G == 2); }
bool direct_p_supported(int P) { return P == 1 || P == 2 || P == 4; }

size_t fused_window_lds(int P, bool f32)
{
    return (f32 ? window_lds_bytes<true>(P) : window_lds_bytes<false>(P)) +
           (size_t)pcr_values(P) * 4 * sizeof(double);
}

hipError_t launch_sweep_fused(int P, int G, bool F32, int driver, const StepArgs &a, int blocks,
                              size_t lds, hipStream_t s)
{
    BSDE_FUSED_CASES(fused_by_driver, driver, a, blocks, lds, s)
}

hipError_t set_fused_lds_limit(int P, int G, bool F32, int driver, size_t lds)
{
    BSDE_FUSED_CASES(allow_by_driver, driver, lds)
}

hipError_t launch_sweep_direct(int P, bool F32, int driver, const StepArgs &a, int blocks,
                               size_t lds, hipStream_t s)
{
    switch (P) {
    case 1: return F32 ? direct_by_driver<1, true>(driver, a, blocks, lds, s)
                       : direct_by_driver<1, false>(driver, a, blocks, lds, s);
    case 2: return F32 ? direct_by_driver<2, true>(driver, a, blocks, lds, s)
                       : direct_by_driver<2, false>(driver, a, blocks, lds, s);
    case 4: return F32 ? direct_by_driver<4, true>(driver, a, blocks, lds, s)
                       : direct_by_driver<4, false>(driver, a, blocks, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_gather(bool F32, int driver, const StepArgs &a, int blocks, hipStream_t s)
{
    return F32 ? gather_by_driver<true>(driver, a, blocks, s)
               : gather_by_driver<false>(driver, a, blocks, s);
}

hipError_t launch_spline(bool f32, const StepArgs &a, int mode, int blocks, hipStream_t s)
{
    if (f32)
        hipLaunchKernelGGL(spline_layer<true>, dim3(blocks), dim3(kBlock), 0, s, a, mode);
    else
        hipLaunchKernelGGL(spline_layer<false>, dim3(blocks), dim3(kBlock), 0, s, a, mode);
    return hipGetLastError();
}

hipError_t launch_scatter(const ScatterChunk &c, char *ws, const InstDesc *desc, int blocks_x,
                          hipStream_t s)
{
    hipLaunchKernelGGL(scatter_layers, dim3(blocks_x, c.count), dim3(kBlock), 0, s, c, ws, desc);
    return hipGetLastError();
}

hipError_t launch_gather(const GatherChunk &c, char *ws, const InstDesc *desc, int blocks_x,
                         unsigned long long *nonfinite, hipStream_t s)
{
    hipLaunchKernelGGL(gather_layers, dim3(blocks_x, c.count), dim3(kBlock), 0, s, c, ws, desc,
                       nonfinite);
    return hipGetLastError();
}

hipError_t launch_clear(unsigned long long *p, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(clear_u64, dim3(64), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_reduce_stats(char *ws, const InstDesc *desc, int count,
                               unsigned long long *totals, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_stats, dim3(count), dim3(kBlock), 0, s, ws, desc, totals);
    return hipGetLastError();
}

}  // namespace bsde

// toeplitz.hip -- the sweep with exact Gaussian expectations of the spline
// (a variant of eq (21) without quadrature error) as a banded Toeplitz
// operator on FP64 matrix cores (arXiv:1909.13560, eq (20); Section 3.2 for
// the uniform grid and the boundary values).
//
// For constant forward coefficients the node of layer n+j sits at
// X = x_i + drift j dt + vol sqrt(j dt) xi with xi ~ N(0, 1).  On the uniform
// grid E[yhat(X)] and E[yhat(X) dW] are then the same linear combination of
// the records (y, M_y) around every point: a Toeplitz band of weights (ev, em
// for the expectation, wv, wm for the dW-weighted one; plan_math.cpp), dense
// over about 18 standard deviations.  With a linear driver f = a y + b z + c
// the expectations of f follow from those of y and z, so one step of eq (20)
// is four banded products per layer (E and dW-weighted, of y and of z) and a
// per-point combination.
//
// A block computes the 256 consecutive points of one tile as a 16 x 16 tile
// D[r][q] = sum_k A[r][k] B[k][q] of v_mfma_f64_16x16x4f64 products: point
// base + 16 q + p(r), A[r][k] = w[k - p(r)] (the band, shifted by the row's
// point offset) and B[k][q] = rec[base + 16 q + klo + k].  The row order p is
// chosen so that the four accumulator elements of a lane are consecutive
// points (the accumulator layout of the instruction keeps row r in lane
// group r % 4, element r / 4).  The band of every layer is cut into chunks of
// kToepChunk taps; the block stages the records a chunk reads (the tile plus
// the chunk) and the chunk's band in LDS, and its four wavefronts take every
// fourth group of four taps.  Small grids (few tiles) also split the chunks
// over S blocks per tile: each writes its partial sums, and toeplitz_finish
// adds them in a fixed order (deterministic), finishes the points and builds
// the new layer's spline.
#include "device_common.h"
#include "kernels.h"

namespace bsde {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

// LDS element slot of window record e: one pad slot per 16 records, so the 16
// lanes of a row (records 16 apart) spread over the banks
__device__ inline int tslot(int e) { return e + (e >> 4); }

constexpr int kWinRecs = kToepTile + kToepChunk + 16;  // records a chunk reads
constexpr int kWinSlots = kWinRecs + kWinRecs / 16 + 1;
constexpr int kBandSlots = kToepChunk + 32;

// y-expectation constant of eq (20) over the layers (the driver's constant
// term), added once per point by whichever kernel finishes it
__device__ inline double toeplitz_constant(const ToepTable &T, int K)
{
    double c = 0.0;
    for (int j = 1; j <= K; ++j) c += T.cy_1[j];
    return c;
}

}  // namespace

size_t toeplitz_lds_bytes()
{
    const size_t win = (size_t)4 * kWinSlots * sizeof(double) + (size_t)4 * kBandSlots * sizeof(double);
    const size_t red = (size_t)4 * kToepTile * 2 * sizeof(double);  // reuses the window
    return std::max(win, red);
}

int toeplitz_chunks(int nb) { return (nb + 15 + kToepChunk - 1) / kToepChunk; }

__global__ void __launch_bounds__(256) sweep_toeplitz(const StepArgs s, int S)
{
    extern __shared__ double tsm[];
    double *wy = tsm, *wmy = tsm + kWinSlots, *wz = tsm + 2 * kWinSlots, *wmz = tsm + 3 * kWinSlots;
    double *bev = tsm + 4 * kWinSlots, *bem = bev + kBandSlots, *bwv = bem + kBandSlots,
           *bwm = bwv + kBandSlots;

    const int idx = xcd_tile(blockIdx.x, gridDim.x);
    const int tg = idx / S, sp = idx - tg * S;  // tile of the group, split of the band
    const InstDesc &d = block_desc(s, tg);
    const SweepArgs a = bind_instance(d, s.ws, s.s, s.stats != 0);
    const int tile = tg - d.tile_base;
    const int t0 = tile * kToepTile;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;   // A row / B column, and k row of the step
    const int prow = 4 * (lr & 3) + (lr >> 2);  // point offset p(r) of A row r = lr
    const int ebase = 16 * lr;                  // B column lr: points 16 lr .. 16 lr + 15
    // the per-layer entries are indexed by j at run time: read them from the
    // descriptor in memory (scalar loads), not from the private copy in a
    const ToepTable &T = d.a.toep;

    double Y[4] = {0.0, 0.0, 0.0, 0.0}, Z[4] = {0.0, 0.0, 0.0, 0.0};
    int gi = 0;  // chunk number over all layers; this block takes gi = sp mod S
    for (int j = 1; j <= a.K; ++j) {
        const Slot<false> g = ring_slot<false>(a, a.n + j);
        const int klo = T.klo[j], nb = T.nb[j];
        const double *band = T.w + T.off[j];  // ev, em, wv, wm: nb each
        const int kend = nb + 15;  // k over which A[r][k] = w[k - p(r)] can be non-zero
        for (int c0 = 0; c0 < kend; c0 += kToepChunk, ++gi) {
            if (gi % S != sp) continue;
            const int clen = min(kToepChunk, kend - c0);
            __syncthreads();  // the previous chunk's reads are done
            // records t0 + klo + c0 + e, e < kToepTile + clen + 16 (ghosts
            // outside the grid hold the boundary value and M = 0)
            for (int e = tid; e < kToepTile + clen + 16; e += 256) {
                const double2 v = g.val(t0 + klo + c0 + e), m = g.der(t0 + klo + c0 + e);
                const int sl = tslot(e);
                wy[sl] = v.x;
                wz[sl] = v.y;
                wmy[sl] = m.x;
                wmz[sl] = m.y;
            }
            // band entries c0 - 16 .. c0 + clen + 16, zero outside [0, nb)
            for (int q = tid; q < clen + 32; q += 256) {
                const int bi = c0 - 16 + q;
                const bool in = bi >= 0 && bi < nb;
                bev[q] = in ? band[bi] : 0.0;
                bem[q] = in ? band[nb + bi] : 0.0;
                bwv[q] = in ? band[2 * nb + bi] : 0.0;
                bwm[q] = in ? band[3 * nb + bi] : 0.0;
            }
            __syncthreads();
            v4d cey = {0, 0, 0, 0}, cwy = cey, cez = cey, cwz = cey;
            // taps 4 q .. 4 q + 3 of the chunk, q = wv, wv + 4, ... (taps past
            // the chunk's end meet zero band entries: kToepChunk is a multiple
            // of 4, so only the last chunk of a layer has them)
            const int n4 = (clen + 3) >> 2;
            for (int q = wv; q < n4; q += 4) {
                const int kk = 4 * q + lk;             // local k of this lane's row
                const int ai = kk - prow + 16;         // band entry c0 + kk - p(r)
                const double aev = bev[ai], aem = bem[ai], awv = bwv[ai], awm = bwm[ai];
                const int sl = tslot(ebase + kk);
                const double by = wy[sl], bmy = wmy[sl], bz = wz[sl], bmz = wmz[sl];
                cey = __builtin_amdgcn_mfma_f64_16x16x4f64(aev, by, cey, 0, 0, 0);
                cey = __builtin_amdgcn_mfma_f64_16x16x4f64(aem, bmy, cey, 0, 0, 0);
                cwy = __builtin_amdgcn_mfma_f64_16x16x4f64(awv, by, cwy, 0, 0, 0);
                cwy = __builtin_amdgcn_mfma_f64_16x16x4f64(awm, bmy, cwy, 0, 0, 0);
                cez = __builtin_amdgcn_mfma_f64_16x16x4f64(aev, bz, cez, 0, 0, 0);
                cez = __builtin_amdgcn_mfma_f64_16x16x4f64(aem, bmz, cez, 0, 0, 0);
                cwz = __builtin_amdgcn_mfma_f64_16x16x4f64(awv, bz, cwz, 0, 0, 0);
                cwz = __builtin_amdgcn_mfma_f64_16x16x4f64(awm, bmz, cwz, 0, 0, 0);
            }
            // D[r][q] sits in lane q + 16 (r % 4), element r / 4, and row r is
            // the point offset p(r) = 4 (r % 4) + r / 4: this lane holds the
            // points 16 lr + 4 lk + i, i = 0..3, in order.  Linear driver: the
            // expectations of f are those of y and z combined; the host
            // folded the weights of eq (20) (Tables 1-2, the z form) into T.c*.
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                Y[i] += T.cy_ey[j] * cey[i] + T.cy_ez[j] * cez[i];
                Z[i] += T.cz_ez[j] * cez[i] + T.cz_wy[j] * cwy[i] + T.cz_wz[j] * cwz[i];
            }
        }
    }
    // the four wavefronts' partial sums meet in LDS (over the window)
    __syncthreads();
    double *red = tsm;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int pt = 16 * lr + 4 * lk + i;
        red[(wv * kToepTile + pt) * 2] = Y[i];
        red[(wv * kToepTile + pt) * 2 + 1] = Z[i];
    }
    __syncthreads();
    double ys = 0.0, zs = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        ys += red[(w * kToepTile + tid) * 2];
        zs += red[(w * kToepTile + tid) * 2 + 1];
    }
    if (S == 1) {
        Acc<1> acc;
        acc.Y[0] = ys + toeplitz_constant(T, a.K);
        acc.Z[0] = zs;
        finish_points<1, BSDE_DRIVER_LINEAR, false>(a, t0 + tid, acc, (tile * kToepTile + tid) >> 6);
    } else {
        double *p = s.part + ((size_t)tg * S + sp) * 2 * kToepTile;
        p[tid] = ys;
        p[kToepTile + tid] = zs;
    }
}

namespace {

// The implicit y equation of one point (linear driver) from y^{n+1}: the same
// operations as finish_points, so a block that solves it at a neighbouring
// tile's point gets that tile's value bit for bit.  it, conv: the
// iterations taken and whether the tolerance was met.
__device__ inline double picard_y(const SweepArgs &a, const Driver<BSDE_DRIVER_LINEAR, double> &f0,
                                  double y, double Yq, double zq, int &it, bool &conv)
{
    it = 0;
    conv = true;
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
    return y;
}

// Natural spline of the staged window (records lo - kHalo - 1 + e, e < W +
// 2 kHalo + 2, clamped to the grid) for a window that meets a domain end:
// the five PCR rounds one by one, the right-hand sides beyond the ends from
// the odd extension about 0 and N-1 (Section 3.2's boundary values) taken
// from the staged records themselves.  The outputs of the tile's records
// depend on right-hand sides within 31 cells of them, whose reflections stay
// inside the staged range; the others only need to be finite.  Results as
// spline_window: window element e (record lo - kHalo + e) holds y, z, M.
template <int U>
__device__ inline void spline_window_ends(int nx, int lo, int W, const WinStore64<1> &win,
                                          double *R, int cap1, const PcrCoef &c,
                                          const SplineRaw<U, double> &raw)
{
    const int tid = threadIdx.x;
    const int WE = W + 2 * kHalo, WS = WE + 2;
    double *Ay = R, *Az = R + cap1, *By = R + 2 * cap1, *Bz = R + 3 * cap1;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e = tid + u * 256;
        if (e < WS) {
            Ay[e] = raw.y[u];
            Az[e] = raw.z[u];
        }
    }
    __syncthreads();
    const int base = lo - kHalo - 1;  // record of staged element 0
    for (int e = tid; e < WE; e += 256) {
        const int k = lo - kHalo + e;
        const double y0 = Ay[e + 1], z0 = Az[e + 1];
        double ry, rz;
        if (k >= 1 && k <= nx - 2) {
            ry = (Ay[e + 2] - y0) - (y0 - Ay[e]);
            rz = (Az[e + 2] - z0) - (z0 - Az[e]);
        } else {
            const int per = 2 * (nx - 1);
            int kk = k % per;
            if (kk < 0) kk += per;
            double sign = 1.0;
            if (kk > nx - 1) {
                kk = per - kk;
                sign = -1.0;
            }
            if (kk == 0 || kk == nx - 1) {
                ry = rz = 0.0;
            } else {
                const int q = min(max(kk - base, 1), WS - 2);  // staged element of record kk
                ry = sign * ((Ay[q + 1] - Ay[q]) - (Ay[q] - Ay[q - 1]));
                rz = sign * ((Az[q + 1] - Az[q]) - (Az[q] - Az[q - 1]));
            }
        }
        By[e] = c.s6 * ry;
        Bz[e] = c.s6 * rz;
        win.val(e, y0, z0);
    }
    __syncthreads();
    double *sy = By, *sz = Bz, *dy = Ay, *dz = Az;
    int h = 1;
    for (int r = 0; r < kPcrRounds; ++r, h <<= 1) {
        const double kap = c.kappa[r];
        for (int e = tid; e < WE; e += 256) {
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
    for (int e = kHalo + tid; e < kHalo + W; e += 256) {
        const int k = lo - kHalo + e;
        const bool inner = (k > 0 && k < nx - 1);
        win.der(e, inner ? sy[e] * c.inv_b : 0.0, inner ? sz[e] * c.inv_b : 0.0);
    }
    __syncthreads();
}

}  // namespace

// The partial sums of the S blocks of a tile, added in split order, the
// implicit y equation (Picard) of its points, and the natural spline of the
// new layer on the tile.  For the spline the block also solves the y
// equation at the kHalo + 1 points either side of its tile (from the partial
// sums of the neighbouring tiles, with the same operations, hence the same
// values as their blocks) and runs the truncated PCR on that window, so the
// step needs no separate spline launch.  Window element e is the record
// t0 - kHalo - 1 + e (clamped to the grid); a thread takes e = tid + 256 u.
__global__ void __launch_bounds__(256) toeplitz_finish(const StepArgs s, int S)
{
    constexpr int W = kToepTile, WS = W + 2 * kHalo + 2, U = (WS + 255) / 256;
    __shared__ double2 wsm[2 * window_slots(1)];  // (y, z), then (M_y, M_z): WinStore64<1>
    __shared__ double R[4 * WS];
    const int tg = xcd_tile(blockIdx.x, gridDim.x);
    const InstDesc &d = block_desc(s, tg);
    const SweepArgs a = bind_instance(d, s.ws, s.s, s.stats != 0);
    const int tile = tg - d.tile_base, tid = threadIdx.x, t0 = tile * W;
    const Slot<false> prev = ring_slot<false>(a, a.n + 1), g = ring_slot<false>(a, a.n);
    // every load first: partial sums (tile i / W of the group, split order)
    // and y^{n+1} of the window's records
    double ys[U], zs[U], y1[U];
    const double *pp[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e = tid + u * 256;
        const int i = min(max(t0 - kHalo - 1 + e, 0), a.nx - 1), ti = i / W;
        pp[u] = s.part + (size_t)(d.tile_base + ti) * S * 2 * W + (i - ti * W);
        ys[u] = zs[u] = 0.0;
        y1[u] = e < WS ? prev.val(i).x : 0.0;
    }
    // four splits at a time, so their loads are in flight together; the
    // sums keep the split order
    for (int sp0 = 0; sp0 < S; sp0 += 4) {
        double vy[4][U], vz[4][U];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool in = sp0 + q < S && tid + u * 256 < WS;
                vy[q][u] = in ? pp[u][(sp0 + q) * 2 * W] : 0.0;
                vz[q][u] = in ? pp[u][(sp0 + q) * 2 * W + W] : 0.0;
            }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (sp0 + q < S) {
                    ys[u] += vy[q][u];
                    zs[u] += vz[q][u];
                }
    }
    const double c1 = toeplitz_constant(d.a.toep, a.K);
    const Driver<BSDE_DRIVER_LINEAR, double> f0(a.drv, a.n * a.dt);
    const bool last = a.n == a.n_stop;
    unsigned int it_max = 0, it_sum = 0, nonconv = 0;
    SplineRaw<U, double> raw;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e = tid + u * 256;
        if (e < WS) {
            int it;
            bool conv;
            const double y = picard_y(a, f0, y1[u], ys[u] + c1, zs[u], it, conv);
            raw.y[u] = y;
            raw.z[u] = zs[u];
            const int k = t0 - kHalo - 1 + e;  // the tile's own records are stored here
            if (k >= t0 && k < min(t0 + W, a.nx)) {
                g.set_val(k, y, zs[u]);
                if (last) {
                    a.fin_y[k] = y;
                    a.fin_z[k] = zs[u];
                }
                it_max = max(it_max, (unsigned int)it);
                it_sum += it;
                nonconv += conv ? 0u : 1u;
            }
        }
    }
    if (a.st_iter_max) {  // per-wave slots of the tile: wave w of the block takes t0 / 64 + w
        it_max = wave_max_u32(it_max);
        it_sum = wave_sum_u32(it_sum);
        nonconv = wave_sum_u32(nonconv);
        if ((tid & 63) == 0) {
            const int w = (t0 + tid) >> 6;
            a.st_iter_max[w] = max(a.st_iter_max[w], it_max);
            a.st_iter_sum[w] += it_sum;
            a.st_nonconv[w] += nonconv;
        }
    }
    if (last) return;  // no later step reads this layer's spline
    const WinStore64<1> win{wsm};
    if (t0 >= kHalo + 1 && t0 + W <= a.nx - kHalo - 1)
        spline_window_interior<256, U, 1>(W, win, R, WS, a.pcr, raw);
    else
        spline_window_ends<U>(a.nx, t0, W, win, R, WS, a.pcr, raw);
    const int kend = min(t0 + W, a.nx);
    for (int k = t0 + tid; k < kend; k += 256) {
        const double2 m = win.ders(k - t0 + kHalo);
        g.set_der(k, m.x, m.y);
    }
    // ghost records beyond the domain ends: the boundary value, M = 0
    if (tile == 0) {
        const double2 e0 = wsm[kHalo - t0];
        for (int k = tid; k < a.pad_l; k += 256) {
            g.set_val(k - a.pad_l, e0.x, e0.y);
            g.set_der(k - a.pad_l, 0.0, 0.0);
        }
    }
    if (tile == a.ntiles - 1) {
        const double2 e1 = wsm[a.nx - 1 - t0 + kHalo];
        for (int k = tid; k < a.pad_r; k += 256) {
            g.set_val(a.nx + k, e1.x, e1.y);
            g.set_der(a.nx + k, 0.0, 0.0);
        }
    }
}

hipError_t launch_sweep_toeplitz(const StepArgs &a, int tiles, int S, hipStream_t s)
{
    hipLaunchKernelGGL(sweep_toeplitz, dim3(tiles * S), dim3(256), toeplitz_lds_bytes(), s, a, S);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || S == 1) return e;
    hipLaunchKernelGGL(toeplitz_finish, dim3(tiles), dim3(256), 0, s, a, S);
    return hipGetLastError();
}

hipError_t set_toeplitz_lds_limit()
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&sweep_toeplitz),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)toeplitz_lds_bytes());
}

}  // namespace bsde

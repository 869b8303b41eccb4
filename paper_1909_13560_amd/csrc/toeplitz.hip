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
// adds them in a fixed order (deterministic) and finishes the points.
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

// The partial sums of the S blocks of a tile, added in split order, and the
// implicit y equation (Picard) of its points.
__global__ void __launch_bounds__(256) toeplitz_finish(const StepArgs s, int S)
{
    const int tg = xcd_tile(blockIdx.x, gridDim.x);
    const InstDesc &d = block_desc(s, tg);
    const SweepArgs a = bind_instance(d, s.ws, s.s, s.stats != 0);
    const int tile = tg - d.tile_base, tid = threadIdx.x;
    const double *p = s.part + (size_t)tg * S * 2 * kToepTile;
    double ys = 0.0, zs = 0.0;
    for (int sp = 0; sp < S; ++sp) {
        ys += p[sp * 2 * kToepTile + tid];
        zs += p[sp * 2 * kToepTile + kToepTile + tid];
    }
    Acc<1> acc;
    acc.Y[0] = ys + toeplitz_constant(d.a.toep, a.K);
    acc.Z[0] = zs;
    finish_points<1, BSDE_DRIVER_LINEAR, false>(a, tile * kToepTile + tid, acc,
                                                (tile * kToepTile + tid) >> 6);
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

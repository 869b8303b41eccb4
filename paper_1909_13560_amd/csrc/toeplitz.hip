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
// A wavefront computes 256 consecutive points as a 16 x 16 tile
// D[r][q] = sum_k A[r][k] B[k][q] of v_mfma_f64_16x16x4f64 products: point
// base + 16 q + p(r), A[r][k] = w[k - p(r)] (the band, shifted by the row's
// point offset) and B[k][q] = rec[base + 16 q + klo + k].  The row order p is
// chosen so that the four accumulator elements of a lane are consecutive
// points (the accumulator layout of the instruction keeps row r in lane
// group r % 4, element r / 4).  A block of four wavefronts stages the
// records its tiles read (1024 points plus the band) in LDS, the band in
// chunks of kChunk taps.
#include "device_common.h"
#include "kernels.h"

namespace bsde {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

// LDS element slot of window record e: one pad slot per 16 records, so the 16
// lanes of a row (records 16 apart) spread over the banks
__device__ inline int tslot(int e) { return e + (e >> 4); }

constexpr int kTilePts = 4 * 256;  // points per block (four 16 x 16 tiles)

}  // namespace

__host__ __device__ constexpr int toeplitz_window_slots()
{
    return (kTilePts + kToepChunk + 16) + (kTilePts + kToepChunk + 16) / 16 + 1;
}

size_t toeplitz_lds_bytes()
{
    return (size_t)4 * toeplitz_window_slots() * sizeof(double) +
           (size_t)4 * (kToepChunk + 32) * sizeof(double);
}

__global__ void __launch_bounds__(256) sweep_toeplitz(const StepArgs s)
{
    extern __shared__ double tsm[];
    constexpr int WS = toeplitz_window_slots();
    constexpr int WB = kToepChunk + 32;
    double *wy = tsm, *wmy = tsm + WS, *wz = tsm + 2 * WS, *wmz = tsm + 3 * WS;
    double *bev = tsm + 4 * WS, *bem = bev + WB, *bwv = bem + WB, *bwm = bwv + WB;

    const int idx = xcd_tile(blockIdx.x, gridDim.x);
    const InstDesc &d = block_desc(s, idx);
    const SweepArgs a = bind_instance(d, s.ws, s.s, s.stats != 0);
    const int tile = idx - d.tile_base;
    const int t0 = tile * kTilePts;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;  // A row / B column, and k row of the step
    // the per-layer entries are indexed by j at run time: read them from the
    // descriptor in memory (scalar loads), not from the private copy in a
    const ToepTable &T = d.a.toep;

    Acc<4> acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc.Y[q] = acc.Z[q] = 0.0;

    for (int j = 1; j <= a.K; ++j) {
        const Slot<false> g = ring_slot<false>(a, a.n + j);
        const int klo = T.klo[j], nb = T.nb[j];
        const double *band = T.w + T.off[j];  // ev, em, wv, wm: nb each
        v4d cey = {0, 0, 0, 0}, cwy = cey, cez = cey, cwz = cey;
        const int kend = nb + 15;  // k over which A[r][k] = w[k - r] can be non-zero
        for (int c0 = 0; c0 < kend; c0 += kToepChunk) {
            const int clen = min(kToepChunk, kend - c0);
            __syncthreads();  // the previous chunk's reads are done
            // records t0 + klo + c0 + e, e < kTilePts + clen + 16 (ghosts
            // outside the grid hold the boundary value and M = 0)
            for (int e = tid; e < kTilePts + clen + 16; e += 256) {
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
            const int ebase = 256 * wv + 16 * lr;  // B column of this lane: its tile column
            const int prow = 4 * (lr & 3) + (lr >> 2);  // point offset p(r) of A row r = lr
            for (int k4 = 0; k4 < clen; k4 += 4) {
                const int kk = k4 + lk;                // local k of this lane's row
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
        }
        // D[r][q] sits in lane q + 16 (r % 4), element r / 4, and row r is the
        // point offset p(r) = 4 (r % 4) + r / 4: this lane holds the points
        // base + 16 lr + 4 lk + i, i = 0..3, in order.  Linear driver: the
        // expectations of f are those of y and z combined; the host folded
        // the weights of eq (20) (Tables 1-2, the z form) into T.c*.
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            acc.Y[i] += T.cy_ey[j] * cey[i] + T.cy_ez[j] * cez[i] + T.cy_1[j];
            acc.Z[i] += T.cz_ez[j] * cez[i] + T.cz_wy[j] * cwy[i] + T.cz_wz[j] * cwz[i];
        }
    }
    finish_points<4, BSDE_DRIVER_LINEAR, false>(a, t0 + 256 * wv + 16 * lr + 4 * lk, acc,
                                                (tile * 256 + tid) >> 6);
}

hipError_t launch_sweep_toeplitz(const StepArgs &a, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(sweep_toeplitz, dim3(blocks), dim3(256), toeplitz_lds_bytes(), s, a);
    return hipGetLastError();
}

hipError_t set_toeplitz_lds_limit()
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&sweep_toeplitz),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)toeplitz_lds_bytes());
}

}  // namespace bsde

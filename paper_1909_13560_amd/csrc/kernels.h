// kernels.h -- host-side launchers of the FP64 kernels (kernels_f64.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>

#include "device_common.h"

namespace bsde {

bool fused_supported(int P, int G);
bool direct_p_supported(int P);
size_t node_table_lds(int nodes);

hipError_t launch_sweep_fused(int P, int G, const SweepArgs &a, int driver, int blocks,
                              size_t lds, hipStream_t s);
hipError_t set_fused_lds_limit(int P, int G, int driver, size_t lds);
hipError_t launch_sweep_direct(int P, const SweepArgs &a, int driver, int blocks, hipStream_t s);
hipError_t launch_spline(Rec64 *slot, int nx, int pad_l, int pad_r, const PcrCoef &c,
                         hipStream_t s);
hipError_t launch_scatter(Rec64 *ring, int npad, int pad_l, int nx, int N, int K,
                          const double *iy, const double *iz, hipStream_t s);
hipError_t launch_gather(const Rec64 *g, int nx, double *y0, double *z0,
                         unsigned long long *nonfinite, hipStream_t s);
hipError_t launch_clear(unsigned long long *p, size_t n, hipStream_t s);
hipError_t launch_reduce_stats(const unsigned int *imax, const unsigned long long *isum,
                               const unsigned long long *nonc, int nw, unsigned long long *totals,
                               hipStream_t s);

}  // namespace bsde

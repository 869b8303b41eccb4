// kernels.h -- host-side launchers of the sweep kernels (sweep.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>

#include "device_common.h"

namespace bsde {

// Instances handled by one scatter / gather launch (pointers travel as
// kernel arguments).
constexpr int kChunk = 32;

struct ScatterChunk {
    int count;
    int inst[kChunk];  // descriptor index
    const double *iy[kChunk];
    const double *iz[kChunk];
};

struct GatherChunk {
    int count;
    int inst[kChunk];
    double *y0[kChunk];
    double *z0[kChunk];
};

bool fused_supported(int P, int G);
bool direct_p_supported(int P);
size_t fused_window_lds(int P, bool f32);  // window + PCR arrays

hipError_t launch_sweep_fused(int P, int G, bool f32, int driver, const StepArgs &a, int blocks,
                              size_t lds, hipStream_t s);
hipError_t set_fused_lds_limit(int P, int G, bool f32, int driver, size_t lds);
hipError_t launch_sweep_direct(int P, bool f32, int driver, const StepArgs &a, int blocks,
                               size_t lds, hipStream_t s);
// state-dependent forward coefficients: one point per lane, nodes located per point
hipError_t launch_sweep_gather(bool f32, int driver, const StepArgs &a, int blocks, hipStream_t s);
// exact Gaussian expectations as banded Toeplitz products on FP64 matrix
// cores: kToepTile points per tile, linear driver, FP64.  S > 1 splits each
// tile's band over S blocks (partial sums in a.part: 2 kToepTile doubles per
// tile and split) and adds a finishing launch.
size_t toeplitz_lds_bytes();
int toeplitz_chunks(int nb);  // band chunks of a layer whose band has nb taps
hipError_t launch_sweep_toeplitz(const StepArgs &a, int tiles, int S, hipStream_t s);
hipError_t set_toeplitz_lds_limit();
// mode 0: initial layer s of every instance; mode 1: layer n0 - s (direct path)
hipError_t launch_spline(bool f32, const StepArgs &a, int mode, int blocks, hipStream_t s);
hipError_t launch_scatter(const ScatterChunk &c, char *ws, const InstDesc *desc, int blocks_x,
                          hipStream_t s);
hipError_t launch_gather(const GatherChunk &c, char *ws, const InstDesc *desc, int blocks_x,
                         unsigned long long *nonfinite, hipStream_t s);
hipError_t launch_clear(unsigned long long *p, size_t n, hipStream_t s);
// layers n_stop .. n_stop + K - 1 of the instance of `desc` from its ring in
// ws into ly, lz (K x nx each, row r = layer n_stop + r)
hipError_t launch_export_layers(bool f32, const InstDesc *desc, int K, int nx, char *ws,
                                double *ly, double *lz, hipStream_t s);
// totals[3 b + {0, 1, 2}] = max, sum, unconverged of descriptor b
hipError_t launch_reduce_stats(char *ws, const InstDesc *desc, int count,
                               unsigned long long *totals, hipStream_t s);

}  // namespace bsde

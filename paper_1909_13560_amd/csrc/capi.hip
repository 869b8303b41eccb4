// capi.hip -- plans, workspace layout, the backward time loop and the C ABI
// of include/bsde.h (arXiv:1909.13560, Section 3.1 steps 1-3).
//
// Workspace layout (caller-owned device memory):
//   per instance: ring of K+1 slots; layer n lives in slot n mod (K+1); a slot
//                 is two planes of pad_l ghost, n_x grid and pad_r ghost
//                 elements: (y, z), then (M_y, M_z) (16 bytes each in FP64,
//                 8 in FP32), so each launch writes whole planes; the FP32
//                 form adds a third plane, the rounding residuals (e_y, e_z)
//                 of the stored values (error feedback)
//   per instance: per-wavefront Picard counters (statistics)
//   totals      : 4 x u64 reduced statistics
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/bsde.h"
#include "kernels.h"
#include "plan_math.h"
#include "sweep2d.h"

namespace {

using bsde::kBlock;

enum SweepPath { PATH_FUSED = 0, PATH_DIRECT = 1, PATH_GATHER = 3, PATH_TOEPLITZ = 4 };

struct SweepConfig {
    int path = PATH_DIRECT;
    int P = 2;
    int G = 1;       // node groups per tile (fused path)
    size_t lds = 0;  // dynamic LDS bytes; 0 marks a fused shape that does not fit
};

constexpr int kMaxP = 4;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Instance {
    bsde_problem pb;
    int K, nx, pad_l, pad_r, npad;
    double dx, dt, h0;
    int m_min, m_max;
    double R;
    bool f32;
    bool gather;  // state-dependent forward coefficients: nodes located per point
    bool exact;   // exact Gaussian expectations (banded Toeplitz operators)
    std::vector<double> ctab;          // tabulated forward coefficients (host copy)
    const double *d_ctab = nullptr;    // and on the device
    bsde::GaussBand band[bsde::kMaxOrder + 1];  // per layer j (exact)
    int toep_off[bsde::kMaxOrder + 1] = {};       // band j in the device table
    const double *toep_w = nullptr;
    int steps;  // layers computed: N - K - n_stop + 1
    bsde::DriverParams drv;
    std::vector<int> m, win_lo, win_hi;
    std::vector<double> B, C, D, cfy, cfz, cz, cy, cyz, dw;
    bsde::NodeTable dtab;
    size_t ring_off, fin_off, stat_off;
    int nwaves;  // per-wave statistics slots (P = 1 has the most waves)
    int group;
};

// Instances sharing precision, driver and kernel shape: one launch per step
// serves all of them.  Members are sorted by their number of steps (most
// first), so the instances active at step s are a prefix.
struct Group {
    bool f32 = false;
    int driver = 0;
    SweepConfig cfg;
    std::vector<int> members;
    std::vector<int> tile_prefix, spline_prefix;  // members + 1 entries
    int *d_tile_inst = nullptr;    // grid tile -> instance (sized for P = 1)
    int *d_spline_inst = nullptr;  // spline tile -> instance
    int max_steps = 0;
    size_t part_off = 0;  // partial sums in the workspace: Toeplitz splits or direct chunks
    int dchunks = 0;      // direct sweep: node chunks per tile in that layout (0: no region)
    int active(int s, const std::vector<Instance> &inst) const
    {
        int lo = 0, hi = (int)members.size();  // members[0..lo) have steps > s
        while (lo < hi) {
            const int mid = (lo + hi) / 2;
            if (inst[members[mid]].steps > s)
                lo = mid + 1;
            else
                hi = mid;
        }
        return lo;
    }
};

// A two-dimensional instance (tensor grid).
struct Instance2 {
    bsde_problem pb;
    bool f32 = false;  // FP32 form: float ring planes with residual planes
    int K, n0, n1, pad0, pad0r, pad1, pad1r, npad0, npad1;
    int win;  // LDS window columns of the sweep kernel
    size_t plane;
    double dx0, dx1, dt, h0, R;
    std::vector<bsde::Node2Row> rows;
    std::vector<bsde::Node2> nodes;
    std::vector<int> m1;
    const bsde::Node2Row *d_rows = nullptr;
    const bsde::Node2 *d_nodes = nullptr;
    const int *d_m1 = nullptr;
    size_t ring_off, fin_off, stat_off;
    int nwaves;
};

}  // namespace

// A captured backward solve (hipGraph) for one set of buffers.
struct GraphEntry {
    const void *ws = nullptr;
    std::vector<bsde_io> io;
    bool stats = false;
    hipGraphExec_t exec = nullptr;
    unsigned long long last_use = 0;
};

constexpr int kMaxGraphs = 4;

struct bsde_plan_s {
    int device = 0;
    size_t max_lds = 65536;
    std::vector<Instance> inst;
    std::vector<Group> groups;
    std::vector<Instance2> inst2;       // two-dimensional plans (all instances d = 2)
    bsde::SplineFilter filter2;
    std::vector<bsde::InstDesc> desc;       // host copy of the descriptors
    bsde::InstDesc *d_desc = nullptr;
    void *d_tables = nullptr;
    size_t ws_bytes = 0;
    size_t stats_off = 0, stats_bytes = 0;  // statistics region of the workspace
    size_t totals_off = 0;                  // 3 u64 per instance + non-finite count
    bsde::PcrCoef pcr_base;                 // kappa, inv_b (s6 set per instance)
    bool use_graphs = true;
    std::mutex mu;                          // guards the graph cache
    hipStream_t capture_stream = nullptr;
    std::vector<GraphEntry> graphs;
    unsigned long long clock = 0;
    void drop_graphs()
    {
        for (GraphEntry &g : graphs) (void)hipGraphExecDestroy(g.exec);
        graphs.clear();
    }
};

namespace {

// Static workspace of bsde_solve_batched_static: a file-scope device array
// (each GPU the library runs on holds its own copy until the process ends).
// In host code `scratch` names a host-side stand-in, not a device address:
// the kernels get the address hipGetSymbolAddress returns for the device,
// looked up once per device at plan time (set-up) and kept in
// g_scratch_addr.
constexpr size_t kStaticWorkspaceBytes = BSDE_STATIC_WORKSPACE_BYTES;
__device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_addr[kMaxDevices];

// Device address of `scratch` on device dev (the current device).
bsde_status static_workspace(int dev, char **out)
{
    if (dev < 0 || dev >= kMaxDevices) return BSDE_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return BSDE_EDEVICE;
        g_scratch_addr[dev] = static_cast<char *>(p);
    }
    *out = g_scratch_addr[dev];
    return BSDE_OK;
}

#define HIP_OK(x)                                  \
    do {                                           \
        hipError_t e_ = (x);                       \
        if (e_ != hipSuccess) return BSDE_EDEVICE; \
    } while (0)

bool valid_problem(const bsde_problem &p)
{
    if (p.d != 1 && p.d != 2) return false;
    static_assert(bsde::kMaxK <= bsde::kMaxOrder, "descriptor window arrays hold K + 1 entries");
    if (p.k_y < 1 || p.k_y > bsde::kMaxK || p.k_z < 1 || p.k_z > bsde::kMaxK) return false;
    const int K = std::max(p.k_y, p.k_z);
    if (p.n_t < K || !(p.T > 0.0) || !std::isfinite(p.T)) return false;
    if (p.L < 1 || p.L > bsde::kMaxL) return false;
    if (p.n_x[0] < 4 || !(p.x_max[0] > p.x_min[0])) return false;
    if (!std::isfinite(p.x_min[0]) || !std::isfinite(p.x_max[0])) return false;
    if (p.tab_steps == 0) {
        if (p.coef_tab) return false;
        if (!std::isfinite(p.drift[0]) || !std::isfinite(p.vol[0][0])) return false;
        if (!std::isfinite(p.drift_x) || !std::isfinite(p.vol_x)) return false;
        // the diffusion coefficient b(x) = vol + vol_x x must be positive over the grid
        if (!(p.vol[0][0] + p.vol_x * p.x_min[0] > 0.0) ||
            !(p.vol[0][0] + p.vol_x * p.x_max[0] > 0.0))
            return false;
    } else {
        // tabulated coefficients: d = 1, one row or one per step, a finite,
        // b finite and positive, the affine slopes unused (0)
        if (p.d != 1 || !p.coef_tab || (p.tab_steps != 1 && p.tab_steps != p.n_t)) return false;
        if (p.drift_x != 0.0 || p.vol_x != 0.0) return false;
        const size_t nx = (size_t)p.n_x[0];
        for (int r = 0; r < p.tab_steps; ++r) {
            const double *ta = p.coef_tab + (size_t)2 * r * nx, *tb = ta + nx;
            for (size_t i = 0; i < nx; ++i)
                if (!std::isfinite(ta[i]) || !std::isfinite(tb[i]) || !(tb[i] > 0.0)) return false;
        }
    }
    if (p.driver < BSDE_DRIVER_LINEAR || p.driver > BSDE_DRIVER_EXP) return false;
    if (p.picard_max < 1) return false;
    if (p.prec != BSDE_FP64 && p.prec != BSDE_FP32_COMP) return false;
    if (p.n_stop < 0 || p.n_stop > p.n_t - K) return false;
    if (p.z_form != BSDE_ZFORM_EZ && p.z_form != BSDE_ZFORM_YDW) return false;
    if (p.quad != BSDE_QUAD_GH && p.quad != BSDE_QUAD_EXACT) return false;
    if (p.interp != BSDE_INTERP_SPLINE && p.interp != BSDE_INTERP_BICUBIC_FD) return false;
    if (p.interp == BSDE_INTERP_BICUBIC_FD && p.d != 2) return false;
    for (int i = 0; i < 8; ++i)
        if (!std::isfinite(p.p[i])) return false;
    if (p.driver == BSDE_DRIVER_BIDASK && p.p[3] == 0.0) return false;
    if (p.d == 2) {
        if (p.n_x[1] < 4 || !(p.x_max[1] > p.x_min[1])) return false;
        if (!std::isfinite(p.x_min[1]) || !std::isfinite(p.x_max[1])) return false;
        if (!std::isfinite(p.drift[1]) || !(p.vol[1][1] > 0.0) || !std::isfinite(p.vol[1][1]) ||
            !std::isfinite(p.vol[1][0]) || !std::isfinite(p.vol[0][1]))
            return false;
    }
    return true;
}

// R above BSDE_STABILITY_LIMIT by more than its own rounding (a grid built
// for R = 16 computes R = 16 to within a few ulps)
bool beyond_stability_limit(double R) { return R > BSDE_STABILITY_LIMIT * (1.0 + 1e-12); }

// What the one-dimensional path implements: every valid problem except the
// E[y dW]/dt z form in the FP32 form (it weighs the stored y by dW/dt ~
// 1/sqrt(dt), so the ring's rounding would enter z amplified by that) and
// exact expectations beyond the Toeplitz kernel's reach (linear driver,
// constant coefficients, FP64).
bool supported_1d(const bsde_problem &q)
{
    if (q.z_form == BSDE_ZFORM_YDW && q.prec == BSDE_FP32_COMP) return false;
    if (q.quad == BSDE_QUAD_EXACT &&
        (q.driver != BSDE_DRIVER_LINEAR || q.drift_x != 0.0 || q.vol_x != 0.0 ||
         q.tab_steps != 0 || q.prec != BSDE_FP64))
        return false;
    return true;
}

// What the two-dimensional path implements: vol lower triangular (any
// correlation, written with its Cholesky factor), the linear driver, FP64.
bool supported_2d(const bsde_problem &p)
{
    // the FP32 form stores the ring in single precision; with the E[y dW]/dt
    // z form its rounding would enter z amplified by dW/dt (as in 1-D)
    const bool prec_ok = p.prec == BSDE_FP64 ||
                         (p.prec == BSDE_FP32_COMP && p.z_form == BSDE_ZFORM_EZ);
    return p.vol[0][1] == 0.0 && p.driver == BSDE_DRIVER_LINEAR && prec_ok &&
           p.L <= 64 && p.drift_x == 0.0 && p.vol_x == 0.0 && p.tab_steps == 0 &&
           p.quad == BSDE_QUAD_GH &&
           (p.interp == BSDE_INTERP_SPLINE || (p.n_x[0] >= 5 && p.n_x[1] >= 5));
}

// Node tables of eq (20)-(21) on the uniform grid (Section 3.2): the node
// x_i + drift j dt + vol sqrt(2 j dt) a_l sits s = (drift j dt + vol sqrt(2 j dt) a_l)/dx
// cells from x_i, independent of i; s = m + phi with integer m.  The weights
// fold the Gauss-Hermite weight pi^{-1/2} w_l and the coefficients of
// Tables 1 and 2 into two accumulators per grid point:
//   Y = E[y^{n+K_y}] + K_y dt sum_{j=1}^{K_y} gamma_j E[f^{n+j}]
//   Z = (E[z^{n+1}] + sum_{j=1}^{K_z} gamma'_j (E[f^{n+j} dW] - E[z^{n+j}])) / gamma'_0 = z^n
bool build_instance(const bsde_problem &p, Instance &in)
{
    in.pb = p;
    in.K = std::max(p.k_y, p.k_z);
    in.nx = p.n_x[0];
    in.dt = p.T / p.n_t;
    in.dx = (p.x_max[0] - p.x_min[0]) / (in.nx - 1);
    in.f32 = p.prec == BSDE_FP32_COMP;
    in.gather = p.drift_x != 0.0 || p.vol_x != 0.0 || p.tab_steps > 0;
    in.exact = p.quad == BSDE_QUAD_EXACT;
    in.steps = p.n_t - in.K - p.n_stop + 1;
    const double vol = p.vol[0][0];
    // largest Gauss-Hermite spread per cell over the grid (b(x) is affine, or
    // tabulated)
    double bmax = std::max(vol + p.vol_x * p.x_min[0], vol + p.vol_x * p.x_max[0]);
    if (p.tab_steps > 0) {
        bmax = 0.0;
        for (int r = 0; r < p.tab_steps; ++r)
            for (int i = 0; i < in.nx; ++i)
                bmax = std::max(bmax, p.coef_tab[(size_t)(2 * r + 1) * in.nx + i]);
        // the plan keeps its own copy of the table
        in.ctab.assign(p.coef_tab, p.coef_tab + (size_t)2 * p.tab_steps * in.nx);
        in.pb.coef_tab = nullptr;
    }
    in.R = bmax * std::sqrt(2.0 * in.dt) / in.dx;
    // the constant-coefficient node offsets (the kernels' windows; the gather
    // kernel locates its nodes per point); with a table, drift and vol are
    // not used and the offsets take b's largest value
    const double drift_n = p.tab_steps > 0 ? 0.0 : p.drift[0];
    const double vol_n = p.tab_steps > 0 ? bmax : vol;
    double a[bsde::kMaxL], w[bsde::kMaxL], gy[8], gz[8];
    if (!bsde::gauss_hermite(p.L, a, w)) return false;
    if (!bsde::spline_gamma(1, p.k_y, gy) || !bsde::spline_gamma(2, p.k_z, gz)) return false;
    const double inv_sqrt_pi = 0.56418958354775628695;
    const int K = in.K, L = p.L;
    in.m.assign(K * L, 0);
    in.B.assign(K * L, 0.0);
    in.C = in.D = in.cfy = in.cfz = in.cz = in.cyz = in.dw = in.B;
    in.cy.assign(L, 0.0);
    in.win_lo.assign(K + 1, 0);
    in.win_hi.assign(K + 1, 0);
    in.m_min = 0;
    in.m_max = 0;
    const double dx26 = in.dx * in.dx / 6.0;
    for (int j = 1; j <= K; ++j) {
        const double sq = std::sqrt(2.0 * j * in.dt);
        int lo = INT32_MAX, hi = INT32_MIN;
        for (int l = 0; l < L; ++l) {
            const int k = (j - 1) * L + l;
            const double dW = sq * a[l];
            const double s = (drift_n * j * in.dt + vol_n * dW) / in.dx;
            const double fl = std::floor(s);
            if (!(std::fabs(fl) < 1e8)) return false;
            const int m = (int)fl;
            const double phi = s - fl;
            const double u = 1.0 - phi;
            const double wl = w[l] * inv_sqrt_pi;
            in.m[k] = m;
            in.dw[k] = dW;
            in.B[k] = phi;
            in.C[k] = dx26 * (u * u * u - u);
            in.D[k] = dx26 * (phi * phi * phi - phi);
            in.cfy[k] = (j <= p.k_y) ? p.k_y * in.dt * gy[j] * wl : 0.0;
            in.cfz[k] = (j <= p.k_z) ? gz[j] * wl * dW / gz[0] : 0.0;
            // the first term of the z equation: E[z^{n+1}] (eq (20)), or
            // E[y^{n+1} dW]/dt (eq (12) with l = 1) for the z form YDW
            const bool ydw = p.z_form == BSDE_ZFORM_YDW;
            in.cz[k] = ((j == 1 && !ydw ? 1.0 : 0.0) - (j <= p.k_z ? gz[j] : 0.0)) * wl / gz[0];
            in.cyz[k] = (j == 1 && ydw) ? wl * dW / (in.dt * gz[0]) : 0.0;
            if (j == p.k_y) in.cy[l] = wl;
            lo = std::min(lo, m);
            hi = std::max(hi, m);
        }
        if (j == 1) {  // the window of layer n+1 also covers the tile itself
            lo = std::min(lo, 0);
            hi = std::max(hi, 0);
        }
        in.win_lo[j] = lo;
        in.win_hi[j] = hi;
        in.m_min = std::min(in.m_min, lo);
        in.m_max = std::max(in.m_max, hi);
    }
    in.h0 = p.k_y * in.dt * gy[0];
    if (in.exact) {
        // exact Gaussian expectations: the band of every layer; the ghosts
        // cover the band and the Toeplitz kernel's window overhang
        for (int j = 1; j <= K; ++j) {
            bsde::GaussBand &b = in.band[j];
            if (!bsde::gaussian_spline_band(p.drift[0] * j * in.dt / in.dx,
                                            vol * std::sqrt(j * in.dt) / in.dx,
                                            std::sqrt(j * in.dt), in.dx, b))
                return false;
            in.m_min = std::min(in.m_min, b.klo);
            in.m_max = std::max(in.m_max, b.klo + (int)b.ev.size() - 1);
        }
    }
    in.pad_l = std::max(0, -in.m_min) + 1;
    // right ghosts cover the overhang of the last tile of any configuration
    in.pad_r = std::max(0, in.m_max) + kBlock * kMaxP + 2 + (in.exact ? 64 : 0);
    in.npad = in.pad_l + in.nx + in.pad_r;
    in.drv = bsde::DriverParams{p.p[0], p.p[1], p.p[2], p.p[3], p.p[4]};
    in.nwaves = (in.nx + kBlock - 1) / kBlock * (kBlock / 64);
    return true;
}

// Two-dimensional node tables (eq (20)-(21) with tensor Gauss-Hermite nodes):
// node (l0, l1) of layer n+j sits at x + drift j dt + vol sqrt(2 j dt) (a_l0, a_l1),
// i.e. s0 = (drift0 j dt + vol00 dW0)/dx0 (vol lower triangular) and
// s1 = (drift1 j dt + vol10 dW0 + vol11 dW1)/dx1 cells away, independent of
// the grid point.  Weights fold w_l0 w_l1 / pi with Tables 1 and 2 as in 1-D,
// z having one component per Brownian motion.
bsde_status build_instance2(const bsde_problem &p, Instance2 &in)
{
    in.pb = p;
    in.f32 = p.prec == BSDE_FP32_COMP;
    in.K = std::max(p.k_y, p.k_z);
    in.n0 = p.n_x[0];
    in.n1 = p.n_x[1];
    in.dt = p.T / p.n_t;
    in.dx0 = (p.x_max[0] - p.x_min[0]) / (in.n0 - 1);
    in.dx1 = (p.x_max[1] - p.x_min[1]) / (in.n1 - 1);
    in.R = std::max(p.vol[0][0] / in.dx0,
                    std::sqrt(p.vol[1][0] * p.vol[1][0] + p.vol[1][1] * p.vol[1][1]) / in.dx1) *
           std::sqrt(2.0 * in.dt);
    double a[bsde::kMaxL], w[bsde::kMaxL], gy[8], gz[8];
    if (!bsde::gauss_hermite(p.L, a, w)) return BSDE_EINVAL;
    if (!bsde::spline_gamma(1, p.k_y, gy) || !bsde::spline_gamma(2, p.k_z, gz)) return BSDE_EINVAL;
    const double inv_sqrt_pi = 0.56418958354775628695;
    const int K = in.K, L = p.L;
    in.rows.assign((size_t)K * L, bsde::Node2Row{});
    in.nodes.assign((size_t)K * L * L, bsde::Node2{});
    in.m1.assign((size_t)K * L * L, 0);
    int m0min = 0, m0max = 0, m1min = 0, m1max = 0;
    in.win = 0;
    const double d0 = in.dx0 * in.dx0 / 6.0, d1 = in.dx1 * in.dx1 / 6.0;
    // the interpolant of the layers (Section 3.3): the tensor natural spline
    // (second derivatives in the three derivative planes), or the paper's
    // bicubic from the values and finite-difference first and mixed
    // derivatives (in the same planes).  Either is v0 + B (v1 - v0) + C d0 +
    // D d1 per axis; for the bicubic B = h01(phi) (and 1 - B = h00(phi)),
    // C = dx h10(phi) = dx phi (1 - phi)^2, D = dx h11(phi) = -dx phi^2 (1 - phi).
    const bool bicubic = p.interp == BSDE_INTERP_BICUBIC_FD;
    for (int j = 1; j <= K; ++j) {
        const double sq = std::sqrt(2.0 * j * in.dt);
        for (int l0 = 0; l0 < L; ++l0) {
            const double dW0 = sq * a[l0];
            const double s0 = (p.drift[0] * j * in.dt + p.vol[0][0] * dW0) / in.dx0;
            const double f0 = std::floor(s0);
            if (!(std::fabs(f0) < 1e8)) return BSDE_EINVAL;
            const double ph0 = s0 - f0, u0 = 1.0 - ph0;
            bsde::Node2Row &row = in.rows[(size_t)(j - 1) * L + l0];
            row.m0 = (int)f0;
            if (bicubic) {  // Hermite basis: values, then dx-scaled slopes
                row.B0 = ph0 * ph0 * (3.0 - 2.0 * ph0);
                row.C0 = in.dx0 * ph0 * u0 * u0;
                row.D0 = -in.dx0 * ph0 * ph0 * u0;
            } else {
                row.B0 = ph0;
                row.C0 = d0 * (u0 * u0 * u0 - u0);
                row.D0 = d0 * (ph0 * ph0 * ph0 - ph0);
            }
            int lo = INT32_MAX, hi = INT32_MIN;
            for (int l1 = 0; l1 < L; ++l1) {
                const double dW1 = sq * a[l1];
                const double s1 =
                    (p.drift[1] * j * in.dt + p.vol[1][0] * dW0 + p.vol[1][1] * dW1) / in.dx1;
                const double f1 = std::floor(s1);
                if (!(std::fabs(f1) < 1e8)) return BSDE_EINVAL;
                const double ph1 = s1 - f1, u1 = 1.0 - ph1;
                const double wgt = w[l0] * inv_sqrt_pi * w[l1] * inv_sqrt_pi;
                const size_t k = ((size_t)(j - 1) * L + l0) * L + l1;
                bsde::Node2 &nd = in.nodes[k];
                if (bicubic) {
                    nd.B1 = ph1 * ph1 * (3.0 - 2.0 * ph1);
                    nd.C1 = in.dx1 * ph1 * u1 * u1;
                    nd.D1 = -in.dx1 * ph1 * ph1 * u1;
                } else {
                    nd.B1 = ph1;
                    nd.C1 = d1 * (u1 * u1 * u1 - u1);
                    nd.D1 = d1 * (ph1 * ph1 * ph1 - ph1);
                }
                nd.cfy = (j <= p.k_y) ? p.k_y * in.dt * gy[j] * wgt : 0.0;
                nd.cfz1 = (j <= p.k_z) ? gz[j] * wgt * dW0 / gz[0] : 0.0;
                nd.cfz2 = (j <= p.k_z) ? gz[j] * wgt * dW1 / gz[0] : 0.0;
                const bool ydw = p.z_form == BSDE_ZFORM_YDW;
                nd.cz = ((j == 1 && !ydw ? 1.0 : 0.0) - (j <= p.k_z ? gz[j] : 0.0)) * wgt / gz[0];
                nd.cy = (j == p.k_y) ? wgt : 0.0;
                nd.cyz1 = (j == 1 && ydw) ? wgt * dW0 / (in.dt * gz[0]) : 0.0;
                nd.cyz2 = (j == 1 && ydw) ? wgt * dW1 / (in.dt * gz[0]) : 0.0;
                in.m1[k] = (int)f1;
                lo = std::min(lo, (int)f1);
                hi = std::max(hi, (int)f1);
            }
            row.m1lo = lo;
            row.m1hi = hi;
            if (bsde::kTile2C + hi - lo + 2 > bsde::kWin2) return BSDE_EUNSUPPORTED;
            in.win = std::max(in.win, bsde::kTile2C + hi - lo + 2);
            m0min = std::min(m0min, row.m0);
            m0max = std::max(m0max, row.m0);
            m1min = std::min(m1min, lo);
            m1max = std::max(m1max, hi);
        }
    }
    in.h0 = p.k_y * in.dt * gy[0];
    // ghosts: node reach plus the overhang of the last tile (kTile2R rows,
    // kTile2C columns)
    in.pad0 = std::max(0, -m0min) + 1;
    in.pad0r = std::max(0, m0max) + bsde::kTile2R + 1;
    in.pad1 = std::max(0, -m1min) + 1;
    in.pad1r = std::max(0, m1max) + bsde::kTile2C + 3;
    in.npad0 = in.pad0 + in.n0 + in.pad0r;
    in.npad1 = in.pad1 + in.n1 + in.pad1r;
    in.plane = (size_t)in.npad0 * in.npad1;
    const int tiles = ((in.n0 + bsde::kTile2R - 1) / bsde::kTile2R) *
                      ((in.n1 + bsde::kTile2C - 1) / bsde::kTile2C);
    in.nwaves = tiles * bsde::kWaves2;
    return BSDE_OK;
}

bsde::Sweep2Args sweep2_args(const Instance2 &in, char *ws, bool stats)
{
    bsde::Sweep2Args a{};
    a.ring = ws + in.ring_off;
    a.plane = in.plane;
    a.n0 = in.n0;
    a.n1 = in.n1;
    a.npad1 = in.npad1;
    a.pad0 = in.pad0;
    a.pad1 = in.pad1;
    a.K = in.K;
    a.Ky = in.pb.k_y;
    a.L = in.pb.L;
    a.n_stop = in.pb.n_stop;
    a.rows = in.d_rows;
    a.nodes = in.d_nodes;
    a.m1 = in.d_m1;
    a.drv = bsde::DriverParams{in.pb.p[0], in.pb.p[1], in.pb.p[2], in.pb.p[3], in.pb.p[4]};
    a.dt = in.dt;
    a.h0 = in.h0;
    a.picard_max = in.pb.picard_max;
    a.picard_tol = in.pb.picard_tol;
    a.zform = in.pb.z_form;
    a.interp = in.pb.interp;
    a.half = (in.win + 1) / 2;
    a.fin = reinterpret_cast<double *>(ws + in.fin_off);
    if (stats) {
        unsigned long long *sum = reinterpret_cast<unsigned long long *>(ws + in.stat_off);
        a.st_iter_sum = sum;
        a.st_nonconv = sum + in.nwaves;
        a.st_iter_max = reinterpret_cast<unsigned int *>(sum + 2 * in.nwaves);
    }
    return a;
}

// The fused kernel with P points per lane and G node groups for every
// member of a group, or lds = 0 if some member's windows do not fit.
SweepConfig fused_config(const std::vector<Instance> &all, const std::vector<int> &members,
                         bool f32, int P, int G, size_t max_lds)
{
    SweepConfig c;
    c.path = PATH_FUSED;
    c.P = P;
    c.G = G;
    const int T = kBlock * P, NT = kBlock * G;
    size_t lds = 0;
    for (int b : members) {
        const Instance &in = all[b];
        // the fused kernel serves the E[z] form of the z equation only
        if (in.gather || in.exact || in.pb.z_form != BSDE_ZFORM_EZ)
            return SweepConfig{PATH_FUSED, P, G, 0};
        int wmax = 0, reach = 0;
        for (int j = 2; j <= in.K; ++j) {
            wmax = std::max(wmax, T + in.win_hi[j] - in.win_lo[j] + 1);
            reach = std::max(reach, in.win_hi[j] - in.win_lo[j] + 1);
        }
        const int reach1 = in.win_hi[1] - in.win_lo[1] + 1;
        const int w1 = T + reach1;
        const size_t window = bsde::fused_window_lds(P, f32);
        const size_t need = window + (size_t)in.K * in.pb.L * sizeof(int);
        const size_t reduce_bytes = (size_t)(G - 1) * kBlock * P * 2 * sizeof(double);
        const bool fits = reach <= bsde::kMaxReach2 && reach1 <= bsde::kMaxReach1 &&
                          wmax + bsde::kHalo <= bsde::window_elems(P) &&
                          w1 + 2 * bsde::kHalo <= bsde::window_elems(P) &&
                          w1 + 2 * bsde::kHalo + 2 <= bsde::pcr_values(P) &&
                          w1 + 2 * bsde::kHalo + 2 <= NT * bsde::pcr_slots(P, NT) &&
                          in.pb.L <= 64 && reduce_bytes <= window && need <= max_lds;
        if (!fits) return SweepConfig{PATH_FUSED, P, G, 0};
        lds = std::max(lds, need);
    }
    c.lds = lds;
    return c;
}

// Blocks per tile of the direct sweep with one point per lane: enough for
// about 1024 blocks on a small grid, at most 16 and at most the node chunks
// of a tile (its chunk sums go through the workspace).
int direct_splits(const std::vector<Instance> &all, const std::vector<int> &members)
{
    long tiles = 0;
    int chunks = 1;
    for (int b : members) {
        tiles += (all[b].nx + kBlock - 1) / kBlock;
        chunks = std::max(chunks, bsde::direct_chunks(all[b].K, all[b].pb.L));
    }
    const long want = (1024 + std::max(tiles, 1L) - 1) / std::max(tiles, 1L);
    return (int)std::max(1L, std::min<long>({want, 16L, (long)chunks}));
}

// S: blocks per tile (P = 1 only); 0 picks direct_splits.
SweepConfig direct_config(const std::vector<Instance> &all, const std::vector<int> &members,
                          bool f32, int P, int S = 0)
{
    SweepConfig c;
    c.path = PATH_DIRECT;
    c.P = P;
    (void)f32;
    const int smax = P == 1 ? direct_splits(all, members) : 1;
    c.G = S > 0 ? std::min(S, smax) : smax;
    c.lds = 0;  // the direct kernel uses no LDS
    return c;
}

// Default shape: the fused kernel with one point per lane (most waves for
// latency hiding), else the widest tile that fits; the direct kernel when no
// window fits in LDS.  BSDE_SWEEP = "fused:P:G" or "direct:P" overrides;
// bsde_autotune replaces the choice by the fastest measured shape.
bool group_gathers(const std::vector<Instance> &all, const std::vector<int> &members)
{
    for (int b : members)
        if (all[b].gather) return true;
    return false;
}

bool group_exact(const std::vector<Instance> &all, const std::vector<int> &members)
{
    for (int b : members)
        if (all[b].exact) return true;
    return false;
}

// The Toeplitz sweep takes tiles of kToepTile points (P = 1) and splits every
// tile's band chunks over S blocks (carried in the G field) so that a group
// with few tiles still launches about 1024 blocks: S = ceil(1024 / tiles),
// at most 16 and at most the largest member's chunk count.
int toeplitz_splits(const std::vector<Instance> &all, const std::vector<int> &members)
{
    long tiles = 0;
    int chunks = 1;
    for (int b : members) {
        const Instance &in = all[b];
        tiles += (in.nx + bsde::kToepTile - 1) / bsde::kToepTile;
        int c = 0;
        for (int j = 1; j <= in.K; ++j) c += bsde::toeplitz_chunks((int)in.band[j].ev.size());
        chunks = std::max(chunks, c);
    }
    const long want = (1024 + std::max(tiles, 1L) - 1) / std::max(tiles, 1L);
    return (int)std::max(1L, std::min<long>({want, 16L, (long)chunks}));
}

SweepConfig toeplitz_config(const std::vector<Instance> &all, const std::vector<int> &members)
{
    return SweepConfig{PATH_TOEPLITZ, 1, toeplitz_splits(all, members), bsde::toeplitz_lds_bytes()};
}

SweepConfig default_config(const std::vector<Instance> &all, const Group &g, size_t max_lds)
{
    if (group_gathers(all, g.members)) return SweepConfig{PATH_GATHER, 1, 1, 0};
    if (group_exact(all, g.members)) return toeplitz_config(all, g.members);
    const char *env = std::getenv("BSDE_SWEEP");
    if (env) {
        int P = 0, G = 1;
        if (std::sscanf(env, "fused:%d:%d", &P, &G) >= 1 && bsde::fused_supported(P, G)) {
            SweepConfig c = fused_config(all, g.members, g.f32, P, G, max_lds);
            if (c.lds) return c;
        }
        int S = 0;
        if (std::sscanf(env, "direct:%d:%d", &P, &S) >= 1 && bsde::direct_p_supported(P))
            return direct_config(all, g.members, g.f32, P, S);
    }
    const int ps[3] = {1, 2, 4};
    for (int P : ps) {
        SweepConfig c = fused_config(all, g.members, g.f32, P, 1, max_lds);
        if (c.lds) return c;
    }
    // the direct kernel: split over blocks on a small grid, else two points per lane
    const SweepConfig c1 = direct_config(all, g.members, g.f32, 1);
    return c1.G > 1 ? c1 : direct_config(all, g.members, g.f32, 2);
}

int sweep_tiles(const Instance &in, int P) { return (in.nx + kBlock * P - 1) / (kBlock * P); }
int spline_tiles(const Instance &in) { return (in.nx + bsde::kSplineTile - 1) / bsde::kSplineTile; }

// Bind a kernel shape to a group: tile numbering, descriptors, LDS limit.
bsde_status apply_config(bsde_plan_s &pl, Group &g, const SweepConfig &c)
{
    if (c.path == PATH_FUSED && c.lds > 65536)
        HIP_OK(bsde::set_fused_lds_limit(c.P, c.G, g.f32, g.driver, c.lds));
    if (c.path == PATH_TOEPLITZ && c.lds > 65536) HIP_OK(bsde::set_toeplitz_lds_limit());
    g.cfg = c;
    g.tile_prefix.assign(g.members.size() + 1, 0);
    g.spline_prefix.assign(g.members.size() + 1, 0);
    std::vector<int> tmap, smap;
    for (size_t k = 0; k < g.members.size(); ++k) {
        const int b = g.members[k];
        const Instance &in = pl.inst[b];
        bsde::InstDesc &d = pl.desc[b];
        d.tile_base = g.tile_prefix[k];
        d.spline_base = g.spline_prefix[k];
        d.spline_tiles = spline_tiles(in);
        d.a.ntiles = sweep_tiles(in, c.P);
        g.tile_prefix[k + 1] = g.tile_prefix[k] + d.a.ntiles;
        g.spline_prefix[k + 1] = g.spline_prefix[k] + d.spline_tiles;
        tmap.insert(tmap.end(), d.a.ntiles, b);
        smap.insert(smap.end(), d.spline_tiles, b);
    }
    HIP_OK(hipMemcpy(g.d_tile_inst, tmap.data(), tmap.size() * sizeof(int), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(g.d_spline_inst, smap.data(), smap.size() * sizeof(int),
                     hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(pl.d_desc, pl.desc.data(), pl.desc.size() * sizeof(bsde::InstDesc),
                     hipMemcpyHostToDevice));
    pl.drop_graphs();
    return BSDE_OK;
}

// Optional per-launch timing with hipEvent pairs (profiling entry point).
struct KernelTimer {
    std::vector<hipEvent_t> sweep, spline;  // start/stop pairs, in launch order
    hipError_t mark(std::vector<hipEvent_t> &v, hipStream_t s)
    {
        hipEvent_t e;
        hipError_t rc = hipEventCreate(&e);
        if (rc != hipSuccess) return rc;
        v.push_back(e);
        return hipEventRecord(e, s);
    }
    ~KernelTimer()
    {
        for (hipEvent_t e : sweep) (void)hipEventDestroy(e);
        for (hipEvent_t e : spline) (void)hipEventDestroy(e);
    }
};

bsde::StepArgs step_args(const bsde_plan_s &pl, const Group &g, char *ws, int s, bool stats,
                         bool spline_map)
{
    bsde::StepArgs a;
    a.ws = ws;
    if (g.members.size() == 1) {  // no tile map: every block is of this instance
        a.desc = pl.d_desc + g.members[0];
        a.tile_inst = nullptr;
    } else {
        a.desc = pl.d_desc;
        a.tile_inst = spline_map ? g.d_spline_inst : g.d_tile_inst;
    }
    a.s = s;
    a.stats = stats ? 1 : 0;
    a.part = (g.cfg.path == PATH_TOEPLITZ || g.cfg.path == PATH_DIRECT) && g.cfg.G > 1
                 ? reinterpret_cast<double *>(ws + g.part_off)
                 : nullptr;
    a.dsplit = g.cfg.path == PATH_DIRECT ? g.cfg.G : 1;
    a.dchunks = g.dchunks;
    return a;
}

// Step s of a group: layer n0 - s of every active member.
bsde_status enqueue_step(const bsde_plan_s &pl, const Group &g, char *ws, int s, bool stats,
                         hipStream_t st, KernelTimer *tm)
{
    const int act = g.active(s, pl.inst);
    if (act == 0) return BSDE_OK;
    const SweepConfig &c = g.cfg;
    const bsde::StepArgs a = step_args(pl, g, ws, s, stats, false);
    const int blocks = g.tile_prefix[act];
    if (tm) HIP_OK(tm->mark(tm->sweep, st));
    if (c.path == PATH_FUSED) {
        HIP_OK(bsde::launch_sweep_fused(c.P, c.G, g.f32, g.driver, a, blocks, c.lds, st));
        if (tm) HIP_OK(tm->mark(tm->sweep, st));
    } else {
        if (c.path == PATH_GATHER)
            HIP_OK(bsde::launch_sweep_gather(g.f32, g.driver, a, blocks, st));
        else if (c.path == PATH_TOEPLITZ)
            HIP_OK(bsde::launch_sweep_toeplitz(a, blocks, c.G, st));
        else
            HIP_OK(bsde::launch_sweep_direct(c.P, g.f32, g.driver, a, blocks, c.lds, st));
        if (tm) HIP_OK(tm->mark(tm->sweep, st));
        // natural spline of the new layer (the fused kernel does this in-kernel,
        // and so does the split Toeplitz sweep's finishing kernel)
        if (c.path == PATH_TOEPLITZ && c.G > 1) return BSDE_OK;
        if (tm) HIP_OK(tm->mark(tm->spline, st));
        HIP_OK(bsde::launch_spline(g.f32, step_args(pl, g, ws, s, false, true), 1,
                                   g.spline_prefix[act], st));
        if (tm) HIP_OK(tm->mark(tm->spline, st));
    }
    return BSDE_OK;
}

// Initial layers (scatter + splines) of every instance.
bsde_status enqueue_init(const bsde_plan_s &pl, char *ws, const bsde_io *io, hipStream_t s)
{
    const int count = (int)pl.inst.size();
    for (int b0 = 0; b0 < count; b0 += bsde::kChunk) {
        bsde::ScatterChunk c{};
        c.count = std::min(bsde::kChunk, count - b0);
        int nxmax = 1;
        for (int k = 0; k < c.count; ++k) {
            c.inst[k] = b0 + k;
            c.iy[k] = io[b0 + k].init_y;
            c.iz[k] = io[b0 + k].init_z;
            nxmax = std::max(nxmax, pl.inst[b0 + k].nx);
        }
        const int bx = std::min(1024, (nxmax + kBlock - 1) / kBlock);
        HIP_OK(bsde::launch_scatter(c, ws, pl.d_desc, bx, s));
    }
    for (const Group &g : pl.groups) {
        int kmax = 0;
        for (int b : g.members) kmax = std::max(kmax, pl.inst[b].K);
        for (int r = 0; r < kmax; ++r)
            HIP_OK(bsde::launch_spline(g.f32, step_args(pl, g, ws, r, false, true), 0,
                                       g.spline_prefix.back(), s));
    }
    return BSDE_OK;
}

bsde_status enqueue_gather(const bsde_plan_s &pl, char *ws, const bsde_io *io,
                           unsigned long long *nonfinite, hipStream_t s)
{
    const int count = (int)pl.inst.size();
    for (int b0 = 0; b0 < count; b0 += bsde::kChunk) {
        bsde::GatherChunk c{};
        c.count = std::min(bsde::kChunk, count - b0);
        int nxmax = 1;
        for (int k = 0; k < c.count; ++k) {
            c.inst[k] = b0 + k;
            c.y0[k] = io[b0 + k].y0;
            c.z0[k] = io[b0 + k].z0;
            nxmax = std::max(nxmax, pl.inst[b0 + k].nx);
        }
        const int bx = std::min(1024, (nxmax + kBlock - 1) / kBlock);
        HIP_OK(bsde::launch_gather(c, ws, pl.d_desc, bx, nonfinite, s));
    }
    return BSDE_OK;
}

// Two-dimensional plan: per instance, initial layers (values, tensor splines,
// ghosts) -> per step the sweep and the splines of the new layer -> outputs.
bsde_status enqueue_solve2(const bsde_plan_s &pl, char *ws, const bsde_io *io, bool stats,
                           unsigned long long *nonfinite, hipStream_t s, KernelTimer *tm)
{
    for (size_t b = 0; b < pl.inst2.size(); ++b) {
        const Instance2 &in = pl.inst2[b];
        bsde::Sweep2Args a = sweep2_args(in, ws, stats);
        bsde::SplineFilter f = pl.filter2;
        f.s6[0] = 6.0 / (in.dx0 * in.dx0) * pl.pcr_base.inv_b;
        f.s6[1] = 6.0 / (in.dx1 * in.dx1) * pl.pcr_base.inv_b;
        const int N = in.pb.n_t, K = in.K;
        a.n = N - K;
        // the derivative planes of a layer: tensor spline or finite differences
        auto interp_layer = [&](int slot) {
            return in.pb.interp == BSDE_INTERP_BICUBIC_FD
                       ? bsde::launch_fd2d(in.f32, a, slot, in.dx0, in.dx1, s)
                       : bsde::launch_spline2d(in.f32, a, slot, f, s);
        };
        HIP_OK(bsde::launch_scatter2d(in.f32, a, io[b].init_y, io[b].init_z, s));
        for (int r = 0; r < K; ++r) HIP_OK(interp_layer((N - K + 1 + r) % (K + 1)));
        for (int n = N - K; n >= in.pb.n_stop; --n) {
            a.n = n;
            if (tm) HIP_OK(tm->mark(tm->sweep, s));
            HIP_OK(bsde::launch_sweep2d(in.f32, a, s));
            if (tm) HIP_OK(tm->mark(tm->sweep, s));
            if (n > in.pb.n_stop) {
                if (tm) HIP_OK(tm->mark(tm->spline, s));
                HIP_OK(interp_layer(n % (K + 1)));
                if (tm) HIP_OK(tm->mark(tm->spline, s));
            }
        }
        HIP_OK(bsde::launch_gather2d(a, io[b].y0, io[b].z0, nonfinite, s));
    }
    return BSDE_OK;
}

// The whole solve: initial layers -> backward loop (all groups, step by
// step) -> outputs.
bsde_status enqueue_solve(const bsde_plan_s &pl, char *ws, const bsde_io *io, bool stats,
                          unsigned long long *nonfinite, hipStream_t s, KernelTimer *tm = nullptr)
{
    if (!pl.inst2.empty()) return enqueue_solve2(pl, ws, io, stats, nonfinite, s, tm);
    bsde_status rc = enqueue_init(pl, ws, io, s);
    if (rc != BSDE_OK) return rc;
    int smax = 0;
    for (const Group &g : pl.groups) smax = std::max(smax, g.max_steps);
    for (int st = 0; st < smax; ++st)
        for (const Group &g : pl.groups) {
            rc = enqueue_step(pl, g, ws, st, stats, s, tm);
            if (rc != BSDE_OK) return rc;
        }
    return enqueue_gather(pl, ws, io, nonfinite, s);
}

bsde_status finish_stats(bsde_plan_t plan, char *ws, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                         bsde_stats *st)
{
    const int count = (int)plan->desc.size();
    unsigned long long *tot = reinterpret_cast<unsigned long long *>(ws + plan->totals_off);
    HIP_OK(bsde::launch_reduce_stats(ws, plan->d_desc, count, tot, s));
    std::vector<unsigned long long> h(3 * (size_t)count + 1);
    HIP_OK(hipMemcpyAsync(h.data(), tot, h.size() * sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    unsigned long long mx = 0, sum = 0, nonc = 0;
    long long point_steps = 0;
    double R = 0.0;
    int unstable = 0;
    for (int b = 0; b < count; ++b) {
        mx = std::max(mx, h[3 * b]);
        sum += h[3 * b + 1];
        nonc += h[3 * b + 2];
        if (plan->inst2.empty()) {
            const Instance &in = plan->inst[b];
            point_steps += (long long)in.nx * in.steps;
            R = std::max(R, in.R);
            unstable += beyond_stability_limit(in.R) ? 1 : 0;
        } else {
            const Instance2 &in = plan->inst2[b];
            point_steps += (long long)in.n0 * in.n1 * (in.pb.n_t - in.K - in.pb.n_stop + 1);
            R = std::max(R, in.R);
            unstable += beyond_stability_limit(in.R) ? 1 : 0;
        }
    }
    float ms = 0.0f;
    HIP_OK(hipEventElapsedTime(&ms, e0, e1));
    st->picard_iter_max = (int)mx;
    st->picard_iter_mean = point_steps ? (double)sum / (double)point_steps : 0.0;
    st->picard_nonconverged = (long long)nonc;
    st->nonfinite = (long long)h[3 * (size_t)count];
    st->stability_ratio = R;
    st->unstable_instances = unstable;
    st->elapsed_ms = ms;
    if (st->nonfinite) return BSDE_ENONFINITE;
    if (st->picard_nonconverged) return BSDE_ENOCONV;
    return BSDE_OK;
}

bool same_io(const std::vector<bsde_io> &a, const bsde_io *b, int count)
{
    if ((int)a.size() != count) return false;
    for (int i = 0; i < count; ++i)
        if (a[i].init_y != b[i].init_y || a[i].init_z != b[i].init_z || a[i].y0 != b[i].y0 ||
            a[i].z0 != b[i].z0)
            return false;
    return true;
}

// The whole solve, replayed as one hipGraph launch: one capture per
// (workspace, buffers, statistics flag), kept in a small least-recently-used
// cache.  The graph holds kernel nodes only.
bsde_status launch_graph(bsde_plan_t plan, char *w, const bsde_io *io, int count, bool stats,
                         unsigned long long *nonfinite, hipStream_t s)
{
    std::lock_guard<std::mutex> lock(plan->mu);
    GraphEntry *hit = nullptr;
    for (GraphEntry &g : plan->graphs)
        if (g.ws == w && g.stats == stats && same_io(g.io, io, count)) hit = &g;
    if (!hit) {
        if (!plan->capture_stream)
            HIP_OK(hipStreamCreateWithFlags(&plan->capture_stream, hipStreamNonBlocking));
        hipStream_t cs = plan->capture_stream;
        HIP_OK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        const bsde_status rc = enqueue_solve(*plan, w, io, stats, nonfinite, cs);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(cs, &graph);
        if (rc != BSDE_OK || ec != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc != BSDE_OK ? rc : BSDE_EDEVICE;
        }
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return BSDE_EDEVICE;
        if ((int)plan->graphs.size() >= kMaxGraphs) {
            auto lru = std::min_element(plan->graphs.begin(), plan->graphs.end(),
                                        [](const GraphEntry &x, const GraphEntry &y) {
                                            return x.last_use < y.last_use;
                                        });
            (void)hipGraphExecDestroy(lru->exec);
            plan->graphs.erase(lru);
        }
        GraphEntry e;
        e.ws = w;
        e.io.assign(io, io + count);
        e.stats = stats;
        e.exec = exec;
        plan->graphs.push_back(e);
        hit = &plan->graphs.back();
    }
    hit->last_use = ++plan->clock;
    HIP_OK(hipGraphLaunch(hit->exec, s));
    return BSDE_OK;
}

bool valid_io(bsde_plan_t plan, void *ws, const bsde_io *io, int count)
{
    if (!plan || !ws || !io) return false;
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return false;
    for (int b = 0; b < count; ++b)
        if (!io[b].init_y || !io[b].init_z || !io[b].y0 || !io[b].z0) return false;
    return true;
}

// Two hipEvents released on every path out of the scope that made them.
struct EventPair {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool create() { return hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess; }
    ~EventPair()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

bsde_status solve_impl(bsde_plan_t plan, void *ws, const bsde_io *io, int count, void *stream,
                       bsde_stats *st)
{
    if (!valid_io(plan, ws, io, count)) return BSDE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    const bool stats = st != nullptr;
    EventPair ev;
    unsigned long long *nonfinite = nullptr;
    if (stats) {
        if (!ev.create()) return BSDE_EDEVICE;
        HIP_OK(hipEventRecord(ev.e0, s));
        // per-wave counters and the totals start at zero
        HIP_OK(bsde::launch_clear(reinterpret_cast<unsigned long long *>(w + plan->stats_off),
                                  plan->stats_bytes / 8, s));
        nonfinite = reinterpret_cast<unsigned long long *>(w + plan->totals_off) + 3 * count;
    }
    bsde_status rc = plan->use_graphs ? launch_graph(plan, w, io, count, stats, nonfinite, s)
                                      : enqueue_solve(*plan, w, io, stats, nonfinite, s);
    if (rc != BSDE_OK) return rc;
    if (!stats) return BSDE_OK;
    HIP_OK(hipEventRecord(ev.e1, s));
    HIP_OK(hipEventSynchronize(ev.e1));
    return finish_stats(plan, w, s, ev.e0, ev.e1, st);
}

}  // namespace

// --------------------------------------------------------------------------
// Plans of two-dimensional problems
// --------------------------------------------------------------------------
namespace {

void pcr_base_coefficients(bsde::PcrCoef &c)
{
    // PCR coefficients of the (1, 4, 1) system: round r eliminates the
    // neighbours at distance 2^r; a' = -a^2/b, b' = b - 2a^2/b
    double av = 1.0, bv = 4.0;
    for (int r = 0; r < bsde::kPcrRounds; ++r) {
        const double k = av / bv;
        c.kappa[r] = k;
        bv = bv - 2.0 * k * av;
        av = -k * av;
    }
    c.inv_b = 1.0 / bv;
    c.s6 = 0.0;
}

// The truncated PCR's filters (compile-time constants of the (1, 4, 1)
// system); the per-axis scale s6 is set per instance.
void pcr_filter(bsde::SplineFilter &f)
{
    constexpr bsde::SplineTaps t = bsde::spline_taps();
    for (int k = 0; k < bsde::kPcrTaps; ++k) f.c[k] = t.c[k];
    for (int k = 0; k < bsde::kPcrTaps + 2; ++k) f.d[k] = t.d[k];
    f.s6[0] = f.s6[1] = 0.0;
}

bsde_status plan_2d(const bsde_problem *pb, int batch, bsde_plan_t *out)
{
    for (int b = 0; b < batch; ++b)
        if (!supported_2d(pb[b])) return BSDE_EUNSUPPORTED;
    bsde_plan_s *pl = new (std::nothrow) bsde_plan_s;
    if (!pl) return BSDE_ENOMEM;
    pl->inst2.resize(batch);
    for (int b = 0; b < batch; ++b) {
        const bsde_status rc = build_instance2(pb[b], pl->inst2[b]);
        if (rc != BSDE_OK) {
            delete pl;
            return rc;
        }
    }
    pcr_base_coefficients(pl->pcr_base);
    pcr_filter(pl->filter2);
    char *sw = nullptr;
    if (hipGetDevice(&pl->device) != hipSuccess || static_workspace(pl->device, &sw) != BSDE_OK) {
        delete pl;
        return BSDE_EDEVICE;
    }
    {
        const char *g = std::getenv("BSDE_GRAPH");
        pl->use_graphs = !(g && g[0] == '0');
    }
    // device tables: node rows, nodes, axis-1 offsets; descriptors (statistics)
    size_t tbytes = 0;
    std::vector<size_t> toff(batch);
    for (int b = 0; b < batch; ++b) {
        const Instance2 &in = pl->inst2[b];
        toff[b] = tbytes;
        tbytes += align_up(in.rows.size() * sizeof(bsde::Node2Row), 256) +
                  align_up(in.nodes.size() * sizeof(bsde::Node2), 256) +
                  align_up(in.m1.size() * sizeof(int), 256);
    }
    const size_t desc_off = tbytes;
    tbytes += align_up((size_t)batch * sizeof(bsde::InstDesc), 256);
    if (hipMalloc(&pl->d_tables, tbytes) != hipSuccess) {
        delete pl;
        return BSDE_ENOMEM;
    }
    char *dev = static_cast<char *>(pl->d_tables);
    std::vector<char> host(desc_off);
    for (int b = 0; b < batch; ++b) {
        Instance2 &in = pl->inst2[b];
        size_t o = toff[b];
        auto put = [&](const void *src, size_t bytes) {
            std::memcpy(host.data() + o, src, bytes);
            void *d = dev + o;
            o += align_up(bytes, 256);
            return d;
        };
        in.d_rows = static_cast<const bsde::Node2Row *>(
            put(in.rows.data(), in.rows.size() * sizeof(bsde::Node2Row)));
        in.d_nodes =
            static_cast<const bsde::Node2 *>(put(in.nodes.data(), in.nodes.size() * sizeof(bsde::Node2)));
        in.d_m1 = static_cast<const int *>(put(in.m1.data(), in.m1.size() * sizeof(int)));
    }
    // workspace: rings (12 planes of doubles per layer, or 15 of floats in the
    // FP32 form), final layers, statistics
    size_t off = 0;
    for (Instance2 &in : pl->inst2) {
        in.ring_off = off;
        off += align_up((in.f32 ? (size_t)15 * sizeof(float) : (size_t)12 * sizeof(double)) *
                            (in.K + 1) * in.plane,
                        256);
    }
    for (Instance2 &in : pl->inst2) {
        in.fin_off = off;
        off += align_up((size_t)3 * in.n0 * in.n1 * sizeof(double), 256);
    }
    pl->stats_off = off;
    for (Instance2 &in : pl->inst2) {
        in.stat_off = off;
        off += align_up((size_t)in.nwaves * (2 * sizeof(unsigned long long) + sizeof(unsigned int)),
                        256);
    }
    pl->totals_off = off;
    off += align_up((3 * (size_t)batch + 1) * sizeof(unsigned long long), 256);
    pl->stats_bytes = off - pl->stats_off;
    pl->ws_bytes = off;
    pl->desc.resize(batch);
    for (int b = 0; b < batch; ++b) {
        bsde::InstDesc &d = pl->desc[b];
        std::memset(&d, 0, sizeof(d));
        d.stat_off = pl->inst2[b].stat_off;
        d.nwaves = pl->inst2[b].nwaves;
    }
    pl->d_desc = reinterpret_cast<bsde::InstDesc *>(dev + desc_off);
    if (hipMemcpy(pl->d_tables, host.data(), desc_off, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(pl->d_desc, pl->desc.data(), batch * sizeof(bsde::InstDesc),
                  hipMemcpyHostToDevice) != hipSuccess) {
        bsde_plan_destroy(pl);
        return BSDE_EDEVICE;
    }
    *out = pl;
    return BSDE_OK;
}

}  // namespace

// --------------------------------------------------------------------------
// C ABI
// --------------------------------------------------------------------------
extern "C" {

const char *bsde_status_string(bsde_status s)
{
    // a C caller may pass any int: read it as one (a value outside the
    // enumeration would be undefined as a C++ enum value)
    int v;
    std::memcpy(&v, &s, sizeof(v));
    switch (v) {
    case BSDE_OK: return "ok";
    case BSDE_EINVAL: return "invalid argument";
    case BSDE_ENOMEM: return "out of memory";
    case BSDE_EDEVICE: return "device (HIP) error";
    case BSDE_EUNSUPPORTED: return "unsupported problem";
    case BSDE_ENOCONV: return "Picard iteration did not converge at some point";
    case BSDE_ENONFINITE: return "non-finite value in the output";
    case BSDE_ESCRATCH:
        return "workspace larger than the static workspace (BSDE_STATIC_WORKSPACE_BYTES)";
    }
    return "unknown status";
}

bsde_status bsde_gauss_hermite(int L, double *a, double *w)
{
    if (!a || !w) return BSDE_EINVAL;
    return bsde::gauss_hermite(L, a, w) ? BSDE_OK : BSDE_EINVAL;
}

bsde_status bsde_gamma(int table, int K, double *g)
{
    if (!g) return BSDE_EINVAL;
    return bsde::spline_gamma(table, K, g) ? BSDE_OK : BSDE_EINVAL;
}

bsde_status bsde_initial_layers(const bsde_problem *pb, int substeps, void *ws, size_t ws_bytes,
                                double *init_y, double *init_z, void *stream)
{
    if (!pb || !ws || !init_y || !init_z || substeps < 1) return BSDE_EINVAL;
    if (!valid_problem(*pb)) return BSDE_EINVAL;
    const int K = std::max(pb->k_y, pb->k_z);
    const size_t np = pb->d == 1 ? (size_t)pb->n_x[0] : (size_t)pb->n_x[0] * pb->n_x[1];
    const double dt = pb->T / pb->n_t;
    // every segment plan has n_t = (N - r + 1) substeps steps; the count must
    // stay an int
    if ((long long)pb->n_t * substeps > INT32_MAX / 2) return BSDE_EINVAL;
    for (int r = 1; r < K; ++r) {
        // layer t_{N-r} from t_{N-r+1}: the 1-step scheme (K_y = K_z = 1) over
        // substeps steps of dt / substeps, absolute times kept (t = n dt')
        bsde_problem q = *pb;
        const int n_hi = pb->n_t - r + 1;
        q.k_y = q.k_z = 1;
        q.T = n_hi * dt;
        q.n_t = n_hi * substeps;
        q.n_stop = (n_hi - 1) * substeps;
        // coefficients tabulated per step: the row of t_{N-r}, held over the
        // segment's sub-steps
        if (pb->tab_steps > 1) {
            q.tab_steps = 1;
            q.coef_tab = pb->coef_tab + (size_t)2 * (pb->n_t - r) * pb->n_x[0];
        }
        bsde_plan_t plan = nullptr;
        bsde_status rc = bsde_plan(&q, 1, &plan);
        if (rc != BSDE_OK) return rc;
        plan->use_graphs = false;  // solved once: launch directly, no capture
        if (bsde_workspace_bytes(plan) > ws_bytes) {
            bsde_plan_destroy(plan);
            return BSDE_EINVAL;
        }
        const bsde_io io{init_y + (size_t)(K - r) * np, init_z + (size_t)(K - r) * np * pb->d,
                         init_y + (size_t)(K - 1 - r) * np,
                         init_z + (size_t)(K - 1 - r) * np * pb->d};
        // the plan (and its device tables) must outlive the enqueued work
        rc = bsde_solve_batched(plan, ws, &io, stream, nullptr);
        const hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
        bsde_plan_destroy(plan);
        if (rc != BSDE_OK) return rc;
        if (e != hipSuccess) return BSDE_EDEVICE;
    }
    return BSDE_OK;
}

bsde_status bsde_problem_info(const bsde_problem *pb, bsde_problem_info_t *info)
{
    if (!pb || !info) return BSDE_EINVAL;
    if (!valid_problem(*pb)) return BSDE_EINVAL;
    bsde_problem_info_t r{};
    r.K = std::max(pb->k_y, pb->k_z);
    if (pb->d == 1) {
        Instance in;
        if (!build_instance(*pb, in)) return BSDE_EINVAL;
        r.stability_ratio = in.R;
        r.node_reach = std::max(-in.m_min, in.m_max + 1);
        r.supported = supported_1d(*pb) ? 1 : 0;
    } else {
        Instance2 in;
        r.supported = supported_2d(*pb) ? 1 : 0;
        if (r.supported) {
            const bsde_status rc = build_instance2(*pb, in);
            if (rc == BSDE_EUNSUPPORTED) r.supported = 0;
            else if (rc != BSDE_OK) return rc;
        }
        const double dx0 = (pb->x_max[0] - pb->x_min[0]) / (pb->n_x[0] - 1);
        const double dx1 = (pb->x_max[1] - pb->x_min[1]) / (pb->n_x[1] - 1);
        const double dt = pb->T / pb->n_t;
        r.stability_ratio =
            std::max(std::hypot(pb->vol[0][0], pb->vol[0][1]) / dx0,
                     std::hypot(pb->vol[1][0], pb->vol[1][1]) / dx1) * std::sqrt(2.0 * dt);
        r.node_reach = r.supported ? in.pad0 - 1 : 0;
        if (r.supported) r.node_reach = std::max({r.node_reach, in.pad1 - 1, in.pad0r - bsde::kTile2R - 1});
    }
    r.stable = beyond_stability_limit(r.stability_ratio) ? 0 : 1;
    *info = r;
    return BSDE_OK;
}

bsde_status bsde_plan(const bsde_problem *pb, int batch, bsde_plan_t *out)
{
    if (!pb || !out || batch < 1) return BSDE_EINVAL;
    for (int b = 0; b < batch; ++b) {
        if (!valid_problem(pb[b])) return BSDE_EINVAL;
        if (pb[b].d != pb[0].d) return BSDE_EINVAL;
    }
    if (pb[0].d == 2) return plan_2d(pb, batch, out);
    bsde_plan_s *pl = new (std::nothrow) bsde_plan_s;
    if (!pl) return BSDE_ENOMEM;
    pl->inst.resize(batch);
    for (int b = 0; b < batch; ++b) {
        if (!supported_1d(pb[b])) {
            delete pl;
            return BSDE_EUNSUPPORTED;
        }
        if (!build_instance(pb[b], pl->inst[b])) {
            delete pl;
            return BSDE_EINVAL;
        }
        // the kernels address a ring plane by 32-bit byte offsets
        const Instance &in = pl->inst[b];
        if ((uint64_t)in.npad * (in.f32 ? sizeof(float2) : sizeof(double2)) >= (uint64_t(1) << 32)) {
            delete pl;
            return BSDE_EUNSUPPORTED;
        }
    }
    // PCR coefficients of the (1, 4, 1) system: round r eliminates the
    // neighbours at distance 2^r; a' = -a^2/b, b' = b - 2a^2/b
    {
        double av = 1.0, bv = 4.0;
        for (int r = 0; r < bsde::kPcrRounds; ++r) {
            const double k = av / bv;
            pl->pcr_base.kappa[r] = k;
            bv = bv - 2.0 * k * av;
            av = -k * av;
        }
        pl->pcr_base.inv_b = 1.0 / bv;
        pl->pcr_base.s6 = 0.0;
    }
    char *sw = nullptr;
    if (hipGetDevice(&pl->device) != hipSuccess || static_workspace(pl->device, &sw) != BSDE_OK) {
        delete pl;
        return BSDE_EDEVICE;
    }
    int lds_limit = 65536;
    if (hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock,
                              pl->device) != hipSuccess) {
        delete pl;
        return BSDE_EDEVICE;
    }
    pl->max_lds = (size_t)lds_limit;
    {
        const char *g = std::getenv("BSDE_GRAPH");
        pl->use_graphs = !(g && g[0] == '0');
    }
    // groups: same precision, driver and default kernel shape (an instance
    // whose windows do not fit a shape does not force it on the others);
    // members by number of steps, most first
    std::vector<SweepConfig> own(batch);
    for (int b = 0; b < batch; ++b) {
        Instance &in = pl->inst[b];
        Group one;
        one.f32 = in.f32;
        one.members = {b};
        own[b] = default_config(pl->inst, one, pl->max_lds);
        int gi = -1;
        for (size_t k = 0; k < pl->groups.size(); ++k) {
            const Group &g = pl->groups[k];
            const SweepConfig &c = own[g.members[0]];
            // the split count of the Toeplitz and direct sweeps follows the group
            if (g.f32 == in.f32 && g.driver == in.pb.driver && c.path == own[b].path &&
                (c.path == PATH_TOEPLITZ || (c.path == PATH_DIRECT && c.P == own[b].P) ||
                 (c.P == own[b].P && c.G == own[b].G)))
                gi = (int)k;
        }
        if (gi < 0) {
            pl->groups.emplace_back();
            pl->groups.back().f32 = in.f32;
            pl->groups.back().driver = in.pb.driver;
            gi = (int)pl->groups.size() - 1;
        }
        in.group = gi;
        pl->groups[gi].members.push_back(b);
    }
    for (Group &g : pl->groups) {
        std::stable_sort(g.members.begin(), g.members.end(), [&](int x, int y) {
            return pl->inst[x].steps > pl->inst[y].steps;
        });
        g.max_steps = pl->inst[g.members[0]].steps;
    }
    // device tables: per instance node records (both forms) and offsets; the
    // descriptors (with the window bounds); per group the tile maps
    size_t tbytes = 0;
    std::vector<size_t> toff(batch);
    for (int b = 0; b < batch; ++b) {
        const Instance &in = pl->inst[b];
        toff[b] = tbytes;
        const size_t kl = (size_t)in.K * in.pb.L;
        tbytes += align_up(kl * sizeof(int), 256) + align_up(kl * sizeof(bsde::NodeRec), 256) +
                  align_up(kl * sizeof(bsde::NodeRec32), 256) + align_up(kl * sizeof(double), 256);
        size_t nbw = 0;
        for (int j = 1; j <= in.K; ++j) nbw += 4 * in.band[j].ev.size();
        tbytes += align_up(nbw * sizeof(double), 256);
        tbytes += align_up(in.ctab.size() * sizeof(double), 256);
    }
    const size_t desc_off = tbytes;
    tbytes += align_up((size_t)batch * sizeof(bsde::InstDesc), 256);
    std::vector<size_t> map_off(pl->groups.size());
    for (size_t k = 0; k < pl->groups.size(); ++k) {
        size_t tiles = 0, stiles = 0;
        for (int b : pl->groups[k].members) {
            tiles += sweep_tiles(pl->inst[b], 1);
            stiles += spline_tiles(pl->inst[b]);
        }
        map_off[k] = tbytes;
        tbytes += align_up(tiles * sizeof(int), 256) + align_up(stiles * sizeof(int), 256);
    }
    if (hipMalloc(&pl->d_tables, std::max<size_t>(tbytes, 256)) != hipSuccess) {
        delete pl;
        return BSDE_ENOMEM;
    }
    char *dev = static_cast<char *>(pl->d_tables);
    std::vector<char> host(tbytes);
    for (int b = 0; b < batch; ++b) {
        Instance &in = pl->inst[b];
        const size_t kl = (size_t)in.K * in.pb.L;
        size_t o = toff[b];
        auto put = [&](const void *src, size_t bytes) {
            std::memcpy(host.data() + o, src, bytes);
            void *d = dev + o;
            o += align_up(bytes, 256);
            return d;
        };
        std::vector<bsde::NodeRec> recs(kl);
        std::vector<bsde::NodeRec32> recs32(kl);
        for (size_t k = 0; k < kl; ++k) {
            const int l = (int)(k % in.pb.L), j = (int)(k / in.pb.L) + 1;
            const double cy = (j == in.pb.k_y) ? in.cy[l] : 0.0;
            recs[k] = bsde::NodeRec{in.B[k],   in.C[k],  in.D[k], in.cfy[k],
                                    in.cfz[k], in.cz[k], cy,      in.cyz[k]};
            recs32[k] = bsde::NodeRec32{(float)in.B[k],   (float)in.C[k],   (float)in.D[k],
                                        (float)in.cfy[k], (float)in.cfz[k], (float)in.cz[k],
                                        (float)cy,        (float)in.cyz[k], in.cz[k],
                                        cy,               in.cyz[k],        0.0};
        }
        in.dtab.rec = static_cast<const bsde::NodeRec *>(put(recs.data(), kl * sizeof(bsde::NodeRec)));
        in.dtab.rec32 =
            static_cast<const bsde::NodeRec32 *>(put(recs32.data(), kl * sizeof(bsde::NodeRec32)));
        in.dtab.m = static_cast<const int *>(put(in.m.data(), kl * sizeof(int)));
        in.dtab.dw = static_cast<const double *>(put(in.dw.data(), kl * sizeof(double)));
        std::vector<double> bw;
        for (int j = 1; j <= in.K; ++j) {
            const bsde::GaussBand &bd = in.band[j];
            in.toep_off[j] = (int)bw.size();
            bw.insert(bw.end(), bd.ev.begin(), bd.ev.end());
            bw.insert(bw.end(), bd.em.begin(), bd.em.end());
            bw.insert(bw.end(), bd.wv.begin(), bd.wv.end());
            bw.insert(bw.end(), bd.wm.begin(), bd.wm.end());
        }
        in.toep_w = static_cast<const double *>(put(bw.data(), bw.size() * sizeof(double)));
        if (!in.ctab.empty())
            in.d_ctab = static_cast<const double *>(put(in.ctab.data(), in.ctab.size() * sizeof(double)));
    }
    if (hipMemcpy(pl->d_tables, host.data(), desc_off, hipMemcpyHostToDevice) != hipSuccess) {
        bsde_plan_destroy(pl);
        return BSDE_EDEVICE;
    }
    pl->d_desc = reinterpret_cast<bsde::InstDesc *>(dev + desc_off);
    for (size_t k = 0; k < pl->groups.size(); ++k) {
        Group &g = pl->groups[k];
        size_t tiles = 0;
        for (int b : g.members) tiles += sweep_tiles(pl->inst[b], 1);
        g.d_tile_inst = reinterpret_cast<int *>(dev + map_off[k]);
        g.d_spline_inst = reinterpret_cast<int *>(dev + map_off[k] + align_up(tiles * sizeof(int), 256));
    }
    // workspace: rings, then the final layers, then the statistics (per-wave
    // slots of every instance, then the totals)
    size_t off = 0;
    for (Instance &in : pl->inst) {
        in.ring_off = off;
        // planes of npad elements per slot: (y, z) and (M_y, M_z); the FP32
        // form adds the rounding residuals (e_y, e_z)
        off += align_up((size_t)(in.K + 1) * (in.f32 ? 3 * sizeof(float2) : 2 * sizeof(double2)) *
                            in.npad,
                        256);
    }
    for (Instance &in : pl->inst) {
        in.fin_off = off;
        off += align_up((size_t)2 * in.nx * sizeof(double), 256);
    }
    // partial sums of the split Toeplitz sweep: 2 kToepTile doubles per tile
    // and split
    for (Group &g : pl->groups) {
        if (!group_exact(pl->inst, g.members)) continue;
        const int S = toeplitz_splits(pl->inst, g.members);
        if (S == 1) continue;
        size_t tiles = 0;
        for (int b : g.members) tiles += sweep_tiles(pl->inst[b], 1);
        g.part_off = off;
        off += align_up(tiles * S * 2 * bsde::kToepTile * sizeof(double), 256);
    }
    // chunk sums of the split direct sweep: 2 kBlock doubles per tile and
    // node chunk (groups that may take it: neither exact nor gathering)
    for (Group &g : pl->groups) {
        if (group_exact(pl->inst, g.members) || group_gathers(pl->inst, g.members)) continue;
        if (direct_splits(pl->inst, g.members) == 1) continue;
        size_t tiles = 0;
        for (int b : g.members) {
            tiles += sweep_tiles(pl->inst[b], 1);
            g.dchunks = std::max(g.dchunks, bsde::direct_chunks(pl->inst[b].K, pl->inst[b].pb.L));
        }
        g.part_off = off;
        off += align_up(tiles * g.dchunks * 2 * kBlock * sizeof(double), 256);
    }
    pl->stats_off = off;
    for (Instance &in : pl->inst) {
        in.stat_off = off;
        off += align_up((size_t)in.nwaves * (2 * sizeof(unsigned long long) + sizeof(unsigned int)),
                        256);
    }
    pl->totals_off = off;
    off += align_up((3 * (size_t)batch + 1) * sizeof(unsigned long long), 256);
    pl->stats_bytes = off - pl->stats_off;
    pl->ws_bytes = off;
    // descriptors
    pl->desc.resize(batch);
    for (int b = 0; b < batch; ++b) {
        const Instance &in = pl->inst[b];
        bsde::InstDesc &d = pl->desc[b];
        std::memset(&d, 0, sizeof(d));
        bsde::SweepArgs &a = d.a;
        a.n_stop = in.pb.n_stop;
        a.tab = in.dtab;
        a.drv = in.drv;
        a.pcr = pl->pcr_base;
        a.pcr.s6 = 6.0 / (in.dx * in.dx);
        a.nx = in.nx;
        a.npad = in.npad;
        a.pad_l = in.pad_l;
        a.pad_r = in.pad_r;
        a.K = in.K;
        a.Ky = in.pb.k_y;
        a.L = in.pb.L;
        a.dt = in.dt;
        a.h0 = in.h0;
        a.picard_max = in.pb.picard_max;
        a.picard_tol = in.pb.picard_tol;
        a.zform = in.pb.z_form;
        a.x_min = in.pb.x_min[0];
        a.dx = in.dx;
        a.drift0 = in.pb.drift[0];
        a.drift_x = in.pb.drift_x;
        a.vol0 = in.pb.vol[0][0];
        a.vol_x = in.pb.vol_x;
        a.ctab = in.d_ctab;
        a.tab_steps = in.pb.tab_steps;
        if (in.exact) {
            // eq (20) for f = p0 y + p1 z + p3 with exact expectations:
            //   Y = E[y^{n+K_y}] + K_y dt sum_j gamma_j E[f^{n+j}]
            //   Z = (E[z^{n+1}] (or E[y^{n+1} dW]/dt) + sum_j gamma'_j (E[f dW] - E[z])) / gamma'_0
            double gy[8], gz[8];
            bsde::spline_gamma(1, in.pb.k_y, gy);
            bsde::spline_gamma(2, in.pb.k_z, gz);
            bsde::ToepTable &t = a.toep;
            t.w = in.toep_w;
            const double p0 = in.pb.p[0], p1 = in.pb.p[1], p3 = in.pb.p[3];
            const bool ydw = in.pb.z_form == BSDE_ZFORM_YDW;
            for (int j = 1; j <= in.K; ++j) {
                t.off[j] = in.toep_off[j];
                t.klo[j] = in.band[j].klo;
                t.nb[j] = (int)in.band[j].ev.size();
                const double fy = j <= in.pb.k_y ? in.pb.k_y * in.dt * gy[j] : 0.0;
                const double fz = j <= in.pb.k_z ? gz[j] : 0.0;
                t.cy_ey[j] = (j == in.pb.k_y ? 1.0 : 0.0) + fy * p0;
                t.cy_ez[j] = fy * p1;
                t.cy_1[j] = fy * p3;
                t.cz_ez[j] = ((j == 1 && !ydw ? 1.0 : 0.0) - fz) / gz[0];
                t.cz_wy[j] = (fz * p0 + (j == 1 && ydw ? 1.0 / in.dt : 0.0)) / gz[0];
                t.cz_wz[j] = fz * p1 / gz[0];
            }
        }
        d.ring_off = in.ring_off;
        d.fin_off = in.fin_off;
        d.stat_off = in.stat_off;
        d.nwaves = in.nwaves;
        d.n0 = in.pb.n_t - in.K;
        d.f32 = in.f32 ? 1 : 0;
        for (int j = 0; j <= in.K; ++j) {
            d.win_lo[j] = in.win_lo[j];
            d.win_hi[j] = in.win_hi[j];
        }
    }
    for (Group &g : pl->groups) {
        bsde_status rc = apply_config(*pl, g, default_config(pl->inst, g, pl->max_lds));
        if (rc != BSDE_OK) {
            bsde_plan_destroy(pl);
            return rc;
        }
    }
    *out = pl;
    return BSDE_OK;
}

void bsde_plan_destroy(bsde_plan_t plan)
{
    if (!plan) return;
    plan->drop_graphs();
    if (plan->capture_stream) (void)hipStreamDestroy(plan->capture_stream);
    if (plan->d_tables) (void)hipFree(plan->d_tables);
    delete plan;
}

size_t bsde_workspace_bytes(bsde_plan_t plan) { return plan ? plan->ws_bytes : 0; }

bsde_status bsde_solve(bsde_plan_t plan, void *ws, const double *init_y, const double *init_z,
                       double *y0, double *z0, void *stream, bsde_stats *st)
{
    if (!plan) return BSDE_EINVAL;
    if (plan->desc.size() != 1) return BSDE_EINVAL;
    bsde_io io{init_y, init_z, y0, z0};
    return solve_impl(plan, ws, &io, 1, stream, st);
}

bsde_status bsde_solve_batched(bsde_plan_t plan, void *ws, const bsde_io *io, void *stream,
                               bsde_stats *st)
{
    if (!plan) return BSDE_EINVAL;
    return solve_impl(plan, ws, io, (int)plan->desc.size(), stream, st);
}

bsde_status bsde_checkpoint_layers(bsde_plan_t plan, void *ws, int b, double *layers_y,
                                   double *layers_z, void *stream)
{
    if (!plan || !ws || !layers_y || !layers_z || b < 0) return BSDE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    if (!plan->inst2.empty()) {
        if (b >= (int)plan->inst2.size()) return BSDE_EINVAL;
        const Instance2 &in = plan->inst2[b];
        bsde::Sweep2Args a = sweep2_args(in, w, false);
        HIP_OK(bsde::launch_export2d(in.f32, a, layers_y, layers_z, s));
        return BSDE_OK;
    }
    if (b >= (int)plan->inst.size()) return BSDE_EINVAL;
    const Instance &in = plan->inst[b];
    HIP_OK(bsde::launch_export_layers(in.f32, plan->d_desc + b, in.K, in.nx, w, layers_y, layers_z,
                                      s));
    return BSDE_OK;
}

bsde_status bsde_solve_batched_static(bsde_plan_t plan, const bsde_io *io, void *stream)
{
    if (!plan || !io) return BSDE_EINVAL;
    const int count = (int)plan->desc.size();
    for (int b = 0; b < count; ++b)
        if (!io[b].init_y || !io[b].init_z || !io[b].y0 || !io[b].z0) return BSDE_EINVAL;
    if (plan->ws_bytes > kStaticWorkspaceBytes) return BSDE_ESCRATCH;
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev != plan->device) return BSDE_EINVAL;
    char *w = nullptr;
    const bsde_status rc = static_workspace(dev, &w);
    if (rc != BSDE_OK) return rc;
    // kernel launches only: no statistics (their counters would need
    // clearing and a host read-back), no graph capture
    return enqueue_solve(*plan, w, io, false, nullptr, static_cast<hipStream_t>(stream));
}

bsde_status bsde_profile_kernels(bsde_plan_t plan, void *ws, const bsde_io *io, void *stream,
                                 bsde_kernel_times *kt)
{
    const int count = plan ? (int)plan->desc.size() : 0;
    if (!kt || !valid_io(plan, ws, io, count)) return BSDE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    KernelTimer tm;
    bsde_status rc = enqueue_solve(*plan, w, io, false, nullptr, s, &tm);
    if (rc != BSDE_OK) return rc;
    HIP_OK(hipStreamSynchronize(s));
    double sw = 0.0, sp = 0.0;
    for (size_t i = 0; i + 1 < tm.sweep.size(); i += 2) {
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, tm.sweep[i], tm.sweep[i + 1]));
        sw += ms;
    }
    for (size_t i = 0; i + 1 < tm.spline.size(); i += 2) {
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, tm.spline[i], tm.spline[i + 1]));
        sp += ms;
    }
    kt->sweep_ms = sw;
    kt->sweep_launches = (int)(tm.sweep.size() / 2);
    kt->spline_ms = sp;
    kt->spline_launches = (int)(tm.spline.size() / 2);
    if (plan->groups.empty()) {  // two-dimensional plan
        const Instance2 &in = plan->inst2[0];
        kt->path = 2;
        kt->points_per_lane = 1;
        kt->node_groups = 1;
        kt->blocks = in.nwaves / bsde::kWaves2;
        kt->lds_bytes = 0;
        return BSDE_OK;
    }
    const Group &g = plan->groups[0];
    kt->path = g.cfg.path;
    kt->points_per_lane = g.cfg.P;
    kt->node_groups = g.cfg.G;
    kt->blocks = g.tile_prefix.back();
    kt->lds_bytes = (long long)g.cfg.lds;
    return BSDE_OK;
}

bsde_status bsde_autotune(bsde_plan_t plan, void *ws, const bsde_io *io, void *stream, int reps,
                          bsde_tune_report *rep)
{
    const int count = plan ? (int)plan->desc.size() : 0;
    if (!valid_io(plan, ws, io, count) || reps < 1) return BSDE_EINVAL;
    if (plan->groups.empty()) {  // two-dimensional plan: one kernel shape
        if (rep) *rep = bsde_tune_report{2, 1, 1, 0.0, 0};
        return BSDE_OK;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    std::lock_guard<std::mutex> lock(plan->mu);
    bsde_status rc = enqueue_init(*plan, w, io, s);
    if (rc != BSDE_OK) return rc;
    // the descriptors are rewritten (synchronously) for every candidate shape:
    // no kernel of the stream may still read them
    HIP_OK(hipStreamSynchronize(s));
    EventPair ev;
    if (!ev.create()) return BSDE_EDEVICE;
    hipEvent_t e0 = ev.e0, e1 = ev.e1;
    int tried = 0;
    for (Group &g : plan->groups) {
        std::vector<SweepConfig> cand;
        const int ps[3] = {1, 2, 4};
        for (int P : ps)
            for (int G = 1; G <= 2; ++G) {
                SweepConfig c = fused_config(plan->inst, g.members, g.f32, P, G, plan->max_lds);
                if (c.lds) cand.push_back(c);
            }
        if (group_gathers(plan->inst, g.members)) cand.assign(1, SweepConfig{PATH_GATHER, 1, 1, 0});
        if (group_exact(plan->inst, g.members)) cand.assign(1, toeplitz_config(plan->inst, g.members));
        if (cand.empty()) {
            cand.push_back(direct_config(plan->inst, g.members, g.f32, 1));
            cand.push_back(direct_config(plan->inst, g.members, g.f32, 2));
        }
        float best = 0.0f;
        SweepConfig best_c = g.cfg;
        // Timed steps: the first, and three more spread over the group's
        // steps, so that a batch's shrinking set of active instances weighs
        // in.  The warm-up runs steps 0 and 1, after which every plane of
        // every ring slot holds finite data (initial layers, their splines
        // and the warm-up's output), so any step does the work of a real one;
        // the solve reloads the initial layers afterwards.
        int sample[4] = {0, g.max_steps / 4, g.max_steps / 2, (3 * g.max_steps) / 4};
        const int nsample = g.max_steps >= 8 ? 4 : 1;
        // Two passes over the candidates, each keeping its faster pass: the
        // first candidate timed would otherwise run while the clocks ramp up.
        std::vector<float> t(cand.size(), 0.0f);
        for (int pass = 0; pass < 2 && rc == BSDE_OK; ++pass) {
            for (size_t ci = 0; ci < cand.size(); ++ci) {
                rc = apply_config(*plan, g, cand[ci]);
                if (rc != BSDE_OK) break;
                rc = enqueue_step(*plan, g, w, 0, false, s, nullptr);  // warm-up
                if (rc == BSDE_OK && nsample > 1) rc = enqueue_step(*plan, g, w, 1, false, s, nullptr);
                if (rc != BSDE_OK) break;
                auto timed_steps = [&](hipStream_t q) {
                    bsde_status r2 = BSDE_OK;
                    for (int r = 0; r < reps && r2 == BSDE_OK; ++r)
                        for (int k = 0; k < nsample && r2 == BSDE_OK; ++k)
                            r2 = enqueue_step(*plan, g, w, sample[k], false, q, nullptr);
                    return r2;
                };
                // the timed steps run the way a solve runs: replayed from a
                // graph (launches from a graph and direct launches rank the
                // shapes differently), or directly when the plan does not use
                // graphs
                hipGraphExec_t exec = nullptr;
                if (plan->use_graphs) {
                    if (!plan->capture_stream &&
                        hipStreamCreateWithFlags(&plan->capture_stream, hipStreamNonBlocking) != hipSuccess) {
                        rc = BSDE_EDEVICE;
                        break;
                    }
                    hipStream_t cs = plan->capture_stream;
                    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                        rc = BSDE_EDEVICE;
                        break;
                    }
                    rc = timed_steps(cs);
                    hipGraph_t graph = nullptr;
                    const hipError_t ec = hipStreamEndCapture(cs, &graph);
                    if (rc == BSDE_OK && ec == hipSuccess &&
                        hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
                        rc = BSDE_EDEVICE;
                    if (graph) (void)hipGraphDestroy(graph);
                    if (rc == BSDE_OK && ec != hipSuccess) rc = BSDE_EDEVICE;
                    if (rc == BSDE_OK && hipGraphLaunch(exec, s) != hipSuccess) rc = BSDE_EDEVICE;
                    if (rc != BSDE_OK) {
                        if (exec) (void)hipGraphExecDestroy(exec);
                        break;
                    }
                }
                float ms = 0.0f;
                if (hipEventRecord(e0, s) != hipSuccess) rc = BSDE_EDEVICE;
                if (rc == BSDE_OK) rc = exec ? (hipGraphLaunch(exec, s) == hipSuccess ? BSDE_OK : BSDE_EDEVICE)
                                             : timed_steps(s);
                if (rc == BSDE_OK &&
                    (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                     hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    rc = BSDE_EDEVICE;
                if (exec) (void)hipGraphExecDestroy(exec);
                if (rc != BSDE_OK) break;
                if (pass == 0) ++tried;
                if (t[ci] == 0.0f || ms < t[ci]) t[ci] = ms;
            }
        }
        for (size_t ci = 0; ci < cand.size() && rc == BSDE_OK; ++ci) {
            if (best == 0.0f || t[ci] < best) {
                best = t[ci];
                best_c = cand[ci];
            }
        }
        if (rc == BSDE_OK) rc = apply_config(*plan, g, best_c);
        if (rc != BSDE_OK) break;
        if (rep && &g == &plan->groups[0]) {
            rep->path = best_c.path;
            rep->points_per_lane = best_c.P;
            rep->node_groups = best_c.G;
            rep->best_ms_per_step = best / (reps * nsample);
        }
    }
    if (rep) rep->candidates = tried;
    return rc;
}

}  // extern "C"

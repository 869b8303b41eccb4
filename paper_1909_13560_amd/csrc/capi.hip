// capi.hip -- plans, workspace layout, the backward time loop and the C ABI
// of include/bsde.h (arXiv:1909.13560, Section 3.1 steps 1-3).
//
// Workspace layout (caller-owned device memory):
//   per instance: ring of K+1 slots; layer n lives in slot n mod (K+1); a slot
//                 is pad_l ghost records, n_x grid records, pad_r ghost records
//                 ({y, M_y, z, M_z}, 32 bytes each)
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

namespace {

using bsde::kBlock;
using bsde::Rec64;

enum SweepPath { PATH_FUSED = 0, PATH_DIRECT = 1 };

struct SweepConfig {
    int path = PATH_DIRECT;
    int P = 2;
    int G = 1;       // node groups per tile (fused path)
    int blocks = 0;
    size_t lds = 0;  // dynamic LDS bytes (fused path)
    int cap = 0, cap1 = 0;
};

constexpr int kMaxFusedP = 5;
constexpr int kMaxDirectP = 4;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Instance {
    bsde_problem pb;
    int K, nx, pad_l, pad_r, npad;
    double dx, dt, h0;
    int m_min, m_max;
    double R;
    bsde::DriverParams drv;
    std::vector<int> m, win_lo, win_hi;
    std::vector<double> A, B, C, D, cfy, cfz, cz, cy;
    bsde::NodeTable dtab;
    size_t ring_off, stat_off;
    int nwaves;  // per-wave statistics slots (largest launch of any configuration)
    SweepConfig cfg;
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
    void *d_tables = nullptr;
    size_t ws_bytes = 0;
    size_t totals_off = 0;
    bsde::PcrCoef pcr_base;  // kappa, inv_b (s6 set per instance)
    bool use_graphs = true;
    std::mutex mu;                    // guards the graph cache
    hipStream_t capture_stream = nullptr;
    std::vector<GraphEntry> graphs;
    unsigned long long clock = 0;
};

namespace {

#define HIP_OK(x)                                  \
    do {                                           \
        hipError_t e_ = (x);                       \
        if (e_ != hipSuccess) return BSDE_EDEVICE; \
    } while (0)

bool valid_problem(const bsde_problem &p)
{
    if (p.d != 1 && p.d != 2) return false;
    if (p.k_y < 1 || p.k_y > bsde::kMaxK || p.k_z < 1 || p.k_z > bsde::kMaxK) return false;
    const int K = std::max(p.k_y, p.k_z);
    if (p.n_t < K || !(p.T > 0.0) || !std::isfinite(p.T)) return false;
    if (p.L < 1 || p.L > bsde::kMaxL) return false;
    if (p.n_x[0] < 4 || !(p.x_max[0] > p.x_min[0])) return false;
    if (!std::isfinite(p.x_min[0]) || !std::isfinite(p.x_max[0])) return false;
    if (!std::isfinite(p.drift[0]) || !(p.vol[0][0] > 0.0) || !std::isfinite(p.vol[0][0]))
        return false;
    if (p.driver < BSDE_DRIVER_LINEAR || p.driver > BSDE_DRIVER_EXP) return false;
    if (p.picard_max < 1) return false;
    if (p.prec != BSDE_FP64 && p.prec != BSDE_FP32_COMP) return false;
    if (p.n_stop < 0 || p.n_stop > p.n_t - K) return false;
    for (int i = 0; i < 8; ++i)
        if (!std::isfinite(p.p[i])) return false;
    if (p.driver == BSDE_DRIVER_BIDASK && p.p[3] == 0.0) return false;
    return true;
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
    const double vol = p.vol[0][0];
    in.R = vol * std::sqrt(2.0 * in.dt) / in.dx;
    double a[bsde::kMaxL], w[bsde::kMaxL], gy[8], gz[8];
    if (!bsde::gauss_hermite(p.L, a, w)) return false;
    if (!bsde::spline_gamma(1, p.k_y, gy) || !bsde::spline_gamma(2, p.k_z, gz)) return false;
    const double inv_sqrt_pi = 0.56418958354775628695;
    const int K = in.K, L = p.L;
    in.m.assign(K * L, 0);
    in.A.assign(K * L, 0.0);
    in.B = in.C = in.D = in.cfy = in.cfz = in.cz = in.A;
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
            const double s = (p.drift[0] * j * in.dt + vol * dW) / in.dx;
            const double fl = std::floor(s);
            if (!(std::fabs(fl) < 1e8)) return false;
            const int m = (int)fl;
            const double phi = s - fl;
            const double u = 1.0 - phi;
            const double wl = w[l] * inv_sqrt_pi;
            in.m[k] = m;
            in.A[k] = u;
            in.B[k] = phi;
            in.C[k] = dx26 * (u * u * u - u);
            in.D[k] = dx26 * (phi * phi * phi - phi);
            in.cfy[k] = (j <= p.k_y) ? p.k_y * in.dt * gy[j] * wl : 0.0;
            in.cfz[k] = (j <= p.k_z) ? gz[j] * wl * dW / gz[0] : 0.0;
            in.cz[k] = ((j == 1 ? 1.0 : 0.0) - (j <= p.k_z ? gz[j] : 0.0)) * wl / gz[0];
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
    in.pad_l = std::max(0, -in.m_min) + 1;
    // right ghosts cover the overhang of the last tile of any configuration
    in.pad_r = std::max(0, in.m_max) + kBlock * std::max(kMaxFusedP, kMaxDirectP) + 2;
    in.npad = in.pad_l + in.nx + in.pad_r;
    in.drv = bsde::DriverParams{p.p[0], p.p[1], p.p[2], p.p[3], p.p[4]};
    in.nwaves = (in.nx + kBlock - 1) / kBlock * (kBlock / 64);  // P = 1 has the most waves
    return true;
}

// Dynamic LDS of the fused kernel with P points per lane and G node groups,
// or lds = 0 if the windows exceed the PCR work split or the device limit.
SweepConfig fused_config(const Instance &in, int P, int G, size_t max_lds)
{
    SweepConfig c;
    c.path = PATH_FUSED;
    c.P = P;
    c.G = G;
    const int T = kBlock * P, NT = kBlock * G;
    int wmax = 0, reach = 0;
    for (int j = 2; j <= in.K; ++j) {
        wmax = std::max(wmax, T + in.win_hi[j] - in.win_lo[j] + 1);
        reach = std::max(reach, in.win_hi[j] - in.win_lo[j] + 1);
    }
    const int w1 = T + in.win_hi[1] - in.win_lo[1] + 1;
    c.cap = bsde::window_slots(P);  // fixed per P: windows must fit, checked below
    c.cap1 = bsde::pcr_values(P);
    const size_t window_bytes = (size_t)c.cap * 2 * sizeof(double2) +
                                (size_t)c.cap1 * 4 * sizeof(double);
    c.lds = window_bytes + bsde::node_table_lds(in.K * in.pb.L);
    const bool fits = w1 + 2 * bsde::kHalo + 2 <= c.cap1 && w1 + 2 * bsde::kHalo <= bsde::window_elems(P) &&
                      wmax + bsde::kHalo <= bsde::window_elems(P) && in.pb.L <= 64;
    c.blocks = (in.nx + T - 1) / T;
    const size_t reduce_bytes = (size_t)(G - 1) * kBlock * P * 2 * sizeof(double);
    if (!fits || w1 + 2 * bsde::kHalo + 2 > NT * bsde::pcr_slots(P, NT) || c.lds > max_lds ||
        reduce_bytes > window_bytes || reach > bsde::kMaxReach2 ||
        in.win_hi[1] - in.win_lo[1] + 1 > bsde::kMaxReach1)
        c.lds = 0;
    return c;
}

SweepConfig direct_config(const Instance &in, int P)
{
    SweepConfig c;
    c.path = PATH_DIRECT;
    c.P = P;
    c.blocks = (in.nx + kBlock * P - 1) / (kBlock * P);
    c.lds = bsde::node_table_lds(in.K * in.pb.L);
    return c;
}

// Default choice: the fused kernel with one point per lane (most waves for
// latency hiding at the grid sizes of interest), the widest tile otherwise
// fitting; the direct kernel when no window fits in LDS.  BSDE_SWEEP =
// "fused:P:G" or "direct:P" overrides.
SweepConfig choose_config(const Instance &in, size_t max_lds, int num_cu)
{
    const char *env = std::getenv("BSDE_SWEEP");
    if (env) {
        int P = 0, G = 1;
        if (std::sscanf(env, "fused:%d:%d", &P, &G) >= 1 && bsde::fused_supported(P, G)) {
            SweepConfig c = fused_config(in, P, G, max_lds);
            if (c.lds) return c;
        }
        if (std::sscanf(env, "direct:%d", &P) == 1 && bsde::direct_p_supported(P))
            return direct_config(in, P);
    }
    (void)num_cu;
    const int ps[3] = {1, 2, 4};
    for (int P : ps) {
        SweepConfig c = fused_config(in, P, 1, max_lds);
        if (c.lds) return c;
    }
    return direct_config(in, 2);
}

bsde::PcrCoef pcr_for(const bsde_plan_s &pl, const Instance &in)
{
    bsde::PcrCoef c = pl.pcr_base;
    c.s6 = 6.0 / (in.dx * in.dx);
    return c;
}

bsde::SweepArgs sweep_args(const bsde_plan_s &pl, const Instance &in, char *ws, bool stats)
{
    bsde::SweepArgs a{};
    a.ring = reinterpret_cast<Rec64 *>(ws + in.ring_off);
    a.tab = in.dtab;
    a.drv = in.drv;
    a.pcr = pcr_for(pl, in);
    a.nx = in.nx;
    a.npad = in.npad;
    a.pad_l = in.pad_l;
    a.pad_r = in.pad_r;
    a.K = in.K;
    a.Ky = in.pb.k_y;
    a.L = in.pb.L;
    a.lds_cap = in.cfg.cap;
    a.lds_cap1 = in.cfg.cap1;
    a.dt = in.dt;
    a.h0 = in.h0;
    a.picard_max = in.pb.picard_max;
    a.picard_tol = in.pb.picard_tol;
    if (stats) {
        unsigned long long *sum = reinterpret_cast<unsigned long long *>(ws + in.stat_off);
        a.st_iter_sum = sum;
        a.st_nonconv = sum + in.nwaves;
        a.st_iter_max = reinterpret_cast<unsigned int *>(sum + 2 * in.nwaves);
    }
    return a;
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

// One time step n: layer n from layers n+1..n+K.
bsde_status enqueue_step(const Instance &in, bsde::SweepArgs &a, int n, hipStream_t s,
                         KernelTimer *tm)
{
    a.n = n;
    const SweepConfig &c = in.cfg;
    if (tm) HIP_OK(tm->mark(tm->sweep, s));
    if (c.path == PATH_FUSED) {
        HIP_OK(bsde::launch_sweep_fused(c.P, c.G, a, in.pb.driver, c.blocks, c.lds, s));
        if (tm) HIP_OK(tm->mark(tm->sweep, s));
    } else {
        HIP_OK(bsde::launch_sweep_direct(c.P, a, in.pb.driver, c.blocks, s));
        if (tm) HIP_OK(tm->mark(tm->sweep, s));
        // natural spline of the new layer (the fused kernel does this in-kernel)
        if (n > in.pb.n_stop) {
            if (tm) HIP_OK(tm->mark(tm->spline, s));
            Rec64 *slot = a.ring + (size_t)(n % (in.K + 1)) * in.npad;
            HIP_OK(bsde::launch_spline(slot, in.nx, in.pad_l, in.pad_r, a.pcr, s));
            if (tm) HIP_OK(tm->mark(tm->spline, s));
        }
    }
    return BSDE_OK;
}

// One instance: initial layers (with their splines) -> backward loop -> output.
bsde_status enqueue_instance(const bsde_plan_s &pl, const Instance &in, char *ws,
                             const double *iy, const double *iz, double *y0, double *z0,
                             hipStream_t s, bool stats, unsigned long long *nonfinite,
                             KernelTimer *tm = nullptr)
{
    const int K = in.K, N = in.pb.n_t;
    bsde::SweepArgs a = sweep_args(pl, in, ws, stats);
    HIP_OK(bsde::launch_scatter(a.ring, in.npad, in.pad_l, in.nx, N, K, iy, iz, s));
    for (int r = 0; r < K; ++r) {
        const int n = N - K + 1 + r;
        HIP_OK(bsde::launch_spline(a.ring + (size_t)(n % (K + 1)) * in.npad, in.nx, in.pad_l,
                                   in.pad_r, a.pcr, s));
    }
    for (int n = N - K; n >= in.pb.n_stop; --n) {
        bsde_status rc = enqueue_step(in, a, n, s, tm);
        if (rc != BSDE_OK) return rc;
    }
    const Rec64 *g = a.ring + (size_t)(in.pb.n_stop % (K + 1)) * in.npad + in.pad_l;
    HIP_OK(bsde::launch_gather(g, in.nx, y0, z0, nonfinite, s));
    return BSDE_OK;
}

bsde_status finish_stats(bsde_plan_t plan, char *ws, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                         bsde_stats *st)
{
    unsigned long long *tot = reinterpret_cast<unsigned long long *>(ws + plan->totals_off);
    unsigned long long agg[4] = {0, 0, 0, 0};
    unsigned long long h[4];
    long long point_steps = 0;
    for (const Instance &in : plan->inst) {
        unsigned long long *sum = reinterpret_cast<unsigned long long *>(ws + in.stat_off);
        unsigned int *mx = reinterpret_cast<unsigned int *>(sum + 2 * in.nwaves);
        HIP_OK(bsde::launch_reduce_stats(mx, sum, sum + in.nwaves, in.nwaves, tot, s));
        HIP_OK(hipMemcpyAsync(h, tot, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        agg[0] = std::max(agg[0], h[0]);
        agg[1] += h[1];
        agg[2] += h[2];
        point_steps += (long long)in.nx * (in.pb.n_t - in.K + 1 - in.pb.n_stop);
    }
    HIP_OK(hipMemcpyAsync(h, tot + 3, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    agg[3] = h[0];
    float ms = 0.0f;
    HIP_OK(hipEventElapsedTime(&ms, e0, e1));
    st->picard_iter_max = (int)agg[0];
    st->picard_iter_mean = point_steps ? (double)agg[1] / (double)point_steps : 0.0;
    st->picard_nonconverged = (long long)agg[2];
    st->nonfinite = (long long)agg[3];
    double R = 0.0;
    for (const Instance &in : plan->inst) R = std::max(R, in.R);
    st->stability_ratio = R;
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

// The whole backward loop of every instance, replayed as one hipGraph launch:
// one capture per (workspace, buffers, statistics flag), kept in a small
// least-recently-used cache.  The graph holds kernel nodes only.
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
        bsde_status rc = BSDE_OK;
        for (int b = 0; b < count && rc == BSDE_OK; ++b)
            rc = enqueue_instance(*plan, plan->inst[b], w, io[b].init_y, io[b].init_z, io[b].y0,
                                  io[b].z0, cs, stats, nonfinite);
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

bsde_status solve_impl(bsde_plan_t plan, void *ws, const bsde_io *io, int count, void *stream,
                       bsde_stats *st)
{
    if (!plan || !ws || !io) return BSDE_EINVAL;
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return BSDE_EINVAL;
    for (int b = 0; b < count; ++b)
        if (!io[b].init_y || !io[b].init_z || !io[b].y0 || !io[b].z0) return BSDE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    const bool stats = st != nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    unsigned long long *nonfinite = nullptr;
    if (stats) {
        HIP_OK(hipEventCreate(&e0));
        HIP_OK(hipEventCreate(&e1));
        HIP_OK(hipEventRecord(e0, s));
        // per-wave counters and the totals start at zero
        const size_t first = plan->inst[0].stat_off;
        const size_t n64 = (plan->totals_off - first) / 8 + 4;
        HIP_OK(bsde::launch_clear(reinterpret_cast<unsigned long long *>(w + first), n64, s));
        nonfinite = reinterpret_cast<unsigned long long *>(w + plan->totals_off) + 3;
    }
    if (plan->use_graphs) {
        bsde_status rc = launch_graph(plan, w, io, count, stats, nonfinite, s);
        if (rc != BSDE_OK) return rc;
    } else {
        for (int b = 0; b < count; ++b) {
            const Instance &in = plan->inst[b];
            bsde_status rc = enqueue_instance(*plan, in, w, io[b].init_y, io[b].init_z, io[b].y0,
                                              io[b].z0, s, stats, nonfinite);
            if (rc != BSDE_OK) return rc;
        }
    }
    if (!stats) return BSDE_OK;
    HIP_OK(hipEventRecord(e1, s));
    HIP_OK(hipEventSynchronize(e1));
    bsde_status rc = finish_stats(plan, w, s, e0, e1, st);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

}  // namespace

// --------------------------------------------------------------------------
// C ABI
// --------------------------------------------------------------------------
extern "C" {

const char *bsde_status_string(bsde_status s)
{
    switch (s) {
    case BSDE_OK: return "ok";
    case BSDE_EINVAL: return "invalid argument";
    case BSDE_ENOMEM: return "out of memory";
    case BSDE_EDEVICE: return "device (HIP) error";
    case BSDE_EUNSUPPORTED: return "unsupported problem";
    case BSDE_ENOCONV: return "Picard iteration did not converge at some point";
    case BSDE_ENONFINITE: return "non-finite value in the output";
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

bsde_status bsde_plan(const bsde_problem *pb, int batch, bsde_plan_t *out)
{
    if (!pb || !out || batch < 1) return BSDE_EINVAL;
    for (int b = 0; b < batch; ++b) {
        if (!valid_problem(pb[b])) return BSDE_EINVAL;
        if (pb[b].d != 1) return BSDE_EUNSUPPORTED;
        if (pb[b].prec != BSDE_FP64) return BSDE_EUNSUPPORTED;
    }
    bsde_plan_s *pl = new (std::nothrow) bsde_plan_s;
    if (!pl) return BSDE_ENOMEM;
    pl->inst.resize(batch);
    for (int b = 0; b < batch; ++b) {
        if (!build_instance(pb[b], pl->inst[b])) {
            delete pl;
            return BSDE_EINVAL;
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
    if (hipGetDevice(&pl->device) != hipSuccess) {
        delete pl;
        return BSDE_EDEVICE;
    }
    int lds_limit = 65536, num_cu = 256;
    if (hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock,
                              pl->device) != hipSuccess ||
        hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, pl->device) !=
            hipSuccess) {
        delete pl;
        return BSDE_EDEVICE;
    }
    pl->max_lds = (size_t)lds_limit;
    {
        const char *g = std::getenv("BSDE_GRAPH");
        pl->use_graphs = !(g && g[0] == '0');
    }
    for (Instance &in : pl->inst) {
        in.cfg = choose_config(in, pl->max_lds, num_cu);
        if (in.cfg.path == PATH_FUSED && in.cfg.lds > 65536 &&
            bsde::set_fused_lds_limit(in.cfg.P, in.cfg.G, in.pb.driver, in.cfg.lds) != hipSuccess)
            in.cfg = direct_config(in, 2);
    }
    // device tables
    size_t tbytes = 0;
    std::vector<size_t> toff(batch);
    for (int b = 0; b < batch; ++b) {
        const Instance &in = pl->inst[b];
        toff[b] = tbytes;
        const size_t kl = (size_t)in.K * in.pb.L;
        tbytes += align_up(kl * sizeof(int), 256) + align_up(kl * sizeof(bsde::NodeRec), 256) +
                  align_up(kl * sizeof(double), 256) + 2 * align_up((in.K + 1) * sizeof(int), 256);
    }
    if (hipMalloc(&pl->d_tables, std::max<size_t>(tbytes, 256)) != hipSuccess) {
        delete pl;
        return BSDE_ENOMEM;
    }
    std::vector<char> host(tbytes);
    for (int b = 0; b < batch; ++b) {
        Instance &in = pl->inst[b];
        const size_t kl = (size_t)in.K * in.pb.L;
        size_t o = toff[b];
        char *dev = static_cast<char *>(pl->d_tables);
        auto put = [&](const void *src, size_t bytes) {
            std::memcpy(host.data() + o, src, bytes);
            void *d = dev + o;
            o += align_up(bytes, 256);
            return d;
        };
        std::vector<bsde::NodeRec> recs(kl);
        std::vector<double> cyk(kl, 0.0);
        for (size_t k = 0; k < kl; ++k) {
            const int l = (int)(k % in.pb.L), j = (int)(k / in.pb.L) + 1;
            recs[k] = bsde::NodeRec{in.B[k], in.C[k], in.D[k], in.cfy[k], in.cfz[k], in.cz[k]};
            if (j == in.pb.k_y) cyk[k] = in.cy[l];
        }
        in.dtab.rec = static_cast<const bsde::NodeRec *>(put(recs.data(), kl * sizeof(bsde::NodeRec)));
        in.dtab.m = static_cast<const int *>(put(in.m.data(), kl * sizeof(int)));
        in.dtab.cy = static_cast<const double *>(put(cyk.data(), kl * sizeof(double)));
        in.dtab.win_lo = static_cast<const int *>(put(in.win_lo.data(), (in.K + 1) * sizeof(int)));
        in.dtab.win_hi = static_cast<const int *>(put(in.win_hi.data(), (in.K + 1) * sizeof(int)));
    }
    if (hipMemcpy(pl->d_tables, host.data(), tbytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(pl->d_tables);
        delete pl;
        return BSDE_EDEVICE;
    }
    // workspace: rings back to back, then per-wave stats, then totals
    size_t off = 0;
    for (Instance &in : pl->inst) {
        in.ring_off = off;
        off += align_up((size_t)(in.K + 1) * in.npad * sizeof(Rec64), 256);
    }
    for (Instance &in : pl->inst) {
        in.stat_off = off;
        off += align_up((size_t)in.nwaves * (2 * sizeof(unsigned long long) + sizeof(unsigned int)),
                        256);
    }
    pl->totals_off = off;
    off += 256;
    pl->ws_bytes = off;
    *out = pl;
    return BSDE_OK;
}

void bsde_plan_destroy(bsde_plan_t plan)
{
    if (!plan) return;
    for (GraphEntry &g : plan->graphs) (void)hipGraphExecDestroy(g.exec);
    if (plan->capture_stream) (void)hipStreamDestroy(plan->capture_stream);
    if (plan->d_tables) (void)hipFree(plan->d_tables);
    delete plan;
}

size_t bsde_workspace_bytes(bsde_plan_t plan) { return plan ? plan->ws_bytes : 0; }

bsde_status bsde_solve(bsde_plan_t plan, void *ws, const double *init_y, const double *init_z,
                       double *y0, double *z0, void *stream, bsde_stats *st)
{
    if (!plan) return BSDE_EINVAL;
    bsde_io io{init_y, init_z, y0, z0};
    return solve_impl(plan, ws, &io, 1, stream, st);
}

bsde_status bsde_solve_batched(bsde_plan_t plan, void *ws, const bsde_io *io, void *stream,
                               bsde_stats *st)
{
    if (!plan) return BSDE_EINVAL;
    return solve_impl(plan, ws, io, (int)plan->inst.size(), stream, st);
}

bsde_status bsde_profile_kernels(bsde_plan_t plan, void *ws, const double *init_y,
                                 const double *init_z, double *y0, double *z0, void *stream,
                                 bsde_kernel_times *kt)
{
    if (!plan || !ws || !init_y || !init_z || !y0 || !z0 || !kt) return BSDE_EINVAL;
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return BSDE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    KernelTimer tm;
    bsde_status rc =
        enqueue_instance(*plan, plan->inst[0], w, init_y, init_z, y0, z0, s, false, nullptr, &tm);
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
    const SweepConfig &c = plan->inst[0].cfg;
    kt->path = c.path;
    kt->points_per_lane = c.P;
    kt->node_groups = c.G;
    kt->blocks = c.blocks;
    kt->lds_bytes = (long long)c.lds;
    return BSDE_OK;
}

}  // extern "C"

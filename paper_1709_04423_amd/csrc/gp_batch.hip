// Batched form: many independent 2D SSCN problems of different sizes advanced
// together.
//
// Every problem keeps its own plan (tables, work grid, partial buffers); the
// batch adds per-problem sweep parameters in device memory and lists of
// wavefront-sized work items:
//   x items  (problem, first line, count): count x lines, one wavefront (scan solver),
//   y items  (problem, first line, count) for y lines of up to 512 points: count
//            lines, one wavefront (the same scan solver on the strided axis), or
//            (problem, 64-column group, segment) for longer ones: one wavefront
//            (windowed solver).
// A step is the x items of every problem followed by the y items of every
// problem.  Two ways to run nsteps steps:
//   - phased: two launches per step (all x items, then all y items);
//   - persistent (real time): ONE launch; each wavefront pops items from a
//     device queue ordered by (step, phase) and, before working on an item,
//     waits until its problem's items of the previous phase are done (per-
//     problem completion counters).  Every item depends only on items earlier
//     in the queue, all of which were taken by running wavefronts, so the
//     queue drains without deadlock whatever the grid size.  Waits are bounded:
//     past the limit the wavefront raises an error flag, every wavefront stops
//     taking items, the launch ends, and gp_batch_step returns GP_ETIMEOUT.
// The autotuner picks the run mode, lines per item, y segments and the
// persistent grid size by timing candidates on scratch copies, then refines the
// lines per item (and y segments) per line length: the problems' sides.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "gp_internal.h"
#include "gp_sweep_common.h"
#include "gp_window.h"
#include "gp_xscan.h"

namespace gp {

struct BatchItem {
    int prob;
    int seg;    // windowed y: segment index; scan y: the item's norm partial slot; x: unused
    int segs;   // windowed y: segments of this problem's lines; scan y and x: 0
    int count;  // x and scan y: lines in the item; windowed y: unused
    int64_t first;  // x and scan y: first line; windowed y: 64-column group
};

// Counters of the persistent launch: queue head, error flag, then per problem
// the number of finished x items and y items (monotonic over the launch).
constexpr int kCtrHead = 0, kCtrError = 1, kCtrFirstProblem = 4;
constexpr int kBatchWaves = 4;                 // wavefronts per workgroup of the batched kernels
constexpr unsigned kSpinLimit = 1u << 22;      // default bound of a dependency wait (polls, ~0.3 s)

// y lines solved as tiles by the scan solver: up to kBatchTileMaxQ points per
// lane (longer ones take the windowed items).
constexpr int kBatchTileMaxQ = 8;
inline bool batch_tiles(const AxisPlan &Y) { return Y.xq > 0 && Y.xq <= kBatchTileMaxQ; }

struct BatchConfig {
    int persistent = 0;  // 1: one launch for all steps (real time only)
    int lines = 4;       // lines per x item and per scan-solved y item
    int ysegs = 4;       // y segments per line (capped per problem)
    int grid = 1024;     // workgroups of the persistent launch
    unsigned spin_limit = kSpinLimit;  // polls before a dependency wait gives up
    // per line length (a problem's side): lines per item and y segments that
    // replace the two above for the lines of that length
    std::map<int64_t, int> side_lines, side_ysegs;
    int lines_for(int64_t len) const
    {
        const auto it = side_lines.find(len);
        return it == side_lines.end() ? lines : it->second;
    }
    int ysegs_for(int64_t len) const
    {
        const auto it = side_ysegs.find(len);
        return it == side_ysegs.end() ? ysegs : it->second;
    }
    // the settings that shape the item lists
    bool same_items(const BatchConfig &o) const
    {
        return lines == o.lines && ysegs == o.ysegs && side_lines == o.side_lines && side_ysegs == o.side_ysegs;
    }
};

}  // namespace gp

struct gp_batch {
    int count = 0;
    gp_mode mode = GP_REAL;
    gp_prec prec = GP_C64;
    int device = 0;
    std::vector<gp_plan *> plans;
    gp::BatchConfig cfg;
    // device data, rebuilt by prepare()
    gp::SweepParams *d_px = nullptr, *d_py = nullptr;
    gp::BatchItem *d_xi = nullptr, *d_yi = nullptr;
    int64_t nxi = 0, nyi = 0;
    int *d_ctr = nullptr;          // kCtrFirstProblem + 2 * count ints
    int *d_nx_per = nullptr, *d_ny_per = nullptr;
    int64_t *d_nparts = nullptr;   // y partials per problem (imaginary-time norm)
    size_t lds_wave = 0;           // ring bytes of one y wavefront (largest problem)
    int qmax = 1;                  // largest x points per lane over the problems
    int qmax_y = 0;                // largest y points per lane of the scan-solved y lines (0: none)
    int smax = 6;                  // most scan steps of any scan-solved line: 3 or 6 (sizes the solvers' registers)
    std::vector<const void *> bound; // psi pointers the device parameters were built for
    gp::BatchConfig bound_cfg;       // and the configuration they were built for
};

namespace gp {

static __device__ __forceinline__ int wave_first_lane_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ------------------------------------------------------------ item bodies

// Q range [QLO, QHI]: the points-per-lane of the x lines a kernel serves; only
// the solver variants in that range are compiled into it (their registers would
// be allocated even when not taken).  SMAX: the most scan steps of any of its
// lines (3 or 6).
// lds: the wavefront's LDS region (at least x_lds_bytes<R>(QHI) bytes).
template <typename R, int MODE, int FLAGS, int Q, int QLO, int QHI, int SMAX>
__device__ __forceinline__ bool x_item_q(const SweepParams &P, const BatchItem &it, typename CT<R>::V *xl)
{
    using V = typename CT<R>::V;
    if constexpr (QLO <= Q && Q <= QHI) {
        if (P.xq == Q) {
            double a = 0.0, b = 0.0, c = 0.0;
            x_scan_wave<R, MODE, FLAGS, Q, SMAX>(P, (const V *)P.psi, (V *)P.out, (const V *)P.tab, nullptr, it.first,
                                                 it.count, a, b, c, xl);
            return true;
        }
    }
    return false;
}

template <typename R, int MODE, int FLAGS, int QLO, int QHI, int SMAX>
__device__ __forceinline__ void run_x_item(const SweepParams &P0, const BatchItem &it, int64_t step, char *lds)
{
    using V = typename CT<R>::V;
    SweepParams P = P0;
    P.norm_total = P0.norm_total + ((step - 1) & 1);
    V *xl = (V *)lds;
    x_item_q<R, MODE, FLAGS, 1, QLO, QHI, SMAX>(P, it, xl) || x_item_q<R, MODE, FLAGS, 2, QLO, QHI, SMAX>(P, it, xl) ||
        x_item_q<R, MODE, FLAGS, 4, QLO, QHI, SMAX>(P, it, xl) || x_item_q<R, MODE, FLAGS, 8, QLO, QHI, SMAX>(P, it, xl) ||
        x_item_q<R, MODE, FLAGS, 16, QLO, QHI, SMAX>(P, it, xl);
}

// [QLO, QHI]: the points-per-lane of the scan-solved y lines a kernel serves
// (QHI = 0: windowed items only); SMAX as for x.
template <typename R, int MODE, int FLAGS, int Q, int QLO, int QHI, int SMAX>
__device__ __forceinline__ bool y_item_q(const SweepParams &P, const BatchItem &it, double &nacc,
                                         typename CT<R>::V *t)
{
    using V = typename CT<R>::V;
    if constexpr (QLO <= Q && Q <= QHI) {
        if (P.xq == Q) {
            col_tile_wave<R, MODE, FLAGS, Q, SMAX>(P, (const V *)P.psi, (V *)P.out, (const V *)P.tab, it.first,
                                                   it.count, nacc, t);
            return true;
        }
    }
    return false;
}

template <typename R, int MODE, int FLAGS, int QLO, int QHI, int SMAX>
__device__ __forceinline__ void run_y_item(const SweepParams &P0, const BatchItem &it, int64_t step, char *lds)
{
    using V = typename CT<R>::V;
    SweepParams P = P0;
    P.norm_out = P0.norm_out + (step & 1) * P0.n_norm;
    const V *src = (const V *)P.psi;
    V *dst = (V *)P.out;
    const V *tab = (const V *)P.tab;
    if constexpr (QHI > 0) {
        if (it.segs == 0) {  // scan solver on tiles of lines, one partial per item
            double nacc = 0.0;
            V *t = (V *)lds;
            y_item_q<R, MODE, FLAGS, 1, QLO, QHI, SMAX>(P, it, nacc, t) ||
                y_item_q<R, MODE, FLAGS, 2, QLO, QHI, SMAX>(P, it, nacc, t) ||
                y_item_q<R, MODE, FLAGS, 4, QLO, QHI, SMAX>(P, it, nacc, t) ||
                y_item_q<R, MODE, FLAGS, 8, QLO, QHI, SMAX>(P, it, nacc, t);
            if (FLAGS & F_NORM_OUT) {
                nacc = wave_sum(nacc);
                if ((threadIdx.x & (kLanes - 1)) == 0) P.norm_out[it.seg] = nacc;
            }
            return;
        }
    }
    if constexpr (QLO > 0) return;  // a scan-only kernel: no windowed items
    const int64_t ngroups = (P.nlines + kLanes - 1) / kLanes;
    const int64_t part = it.first + ngroups * it.seg;
    switch (P.D) {
    case 1: window_run<R, MODE, FLAGS, kStrided, 1, 4>(P, src, dst, tab, nullptr, lds, it.first, it.seg, it.segs, part); break;
    case 2: window_run<R, MODE, FLAGS, kStrided, 2, 4>(P, src, dst, tab, nullptr, lds, it.first, it.seg, it.segs, part); break;
    case 3: window_run<R, MODE, FLAGS, kStrided, 3, 4>(P, src, dst, tab, nullptr, lds, it.first, it.seg, it.segs, part); break;
    case 4: window_run<R, MODE, FLAGS, kStrided, 4, 4>(P, src, dst, tab, nullptr, lds, it.first, it.seg, it.segs, part); break;
    case 5: window_run<R, MODE, FLAGS, kStrided, 5, 4>(P, src, dst, tab, nullptr, lds, it.first, it.seg, it.segs, part); break;
    case 6: window_run<R, MODE, FLAGS, kStrided, 6, 4>(P, src, dst, tab, nullptr, lds, it.first, it.seg, it.segs, part); break;
    case 7: window_run<R, MODE, FLAGS, kStrided, 7, 4>(P, src, dst, tab, nullptr, lds, it.first, it.seg, it.segs, part); break;
    case 8: window_run<R, MODE, FLAGS, kStrided, 8, 4>(P, src, dst, tab, nullptr, lds, it.first, it.seg, it.segs, part); break;
    default: break;  // excluded when the batch is created (batch_supports)
    }
}

// ------------------------------------------------------------ phased kernels

// complex64 lines of up to 8 points per lane and at most 3 scan steps: at least
// three wavefronts per SIMD.  The line solves are latency-bound chains that two
// would leave the SIMD idle most of the time, and there the register cap costs
// no spills (elsewhere it would).
template <typename R, int MODE, int QLO, int QHI, int SMAX>
__global__ __launch_bounds__(kLanes *kBatchWaves, (sizeof(R) == 4 && QHI <= 8 && SMAX <= 3) ? 3 : 1) void k_batch_x(const SweepParams *__restrict__ px,
                                                                  const BatchItem *__restrict__ items, int64_t nitems,
                                                                  int64_t step, int renorm)
{
    __shared__ typename CT<R>::V xl[kBatchWaves][kLanes * (QHI + 1)];
    const int w = wave_first_lane_i(threadIdx.x / kLanes);
    const int64_t i = (int64_t)blockIdx.x * kBatchWaves + w;
    if (i >= nitems) return;  // whole wavefront
    const BatchItem it = items[i];
    if (MODE == GP_IMAG && renorm)
        run_x_item<R, MODE, F_FUSE_N | F_RENORM, QLO, QHI, SMAX>(px[it.prob], it, step, (char *)xl[w]);
    else
        run_x_item<R, MODE, F_FUSE_N, QLO, QHI, SMAX>(px[it.prob], it, step, (char *)xl[w]);
}

template <typename R, int MODE, int QLO, int QHI, int SMAX>
__global__ __launch_bounds__(kLanes *kBatchWaves) void k_batch_y(const SweepParams *__restrict__ py,
                                                                  const BatchItem *__restrict__ items, int64_t nitems,
                                                                  int64_t step, size_t lds_wave)
{
    extern __shared__ char lds_raw[];
    const int w = wave_first_lane_i(threadIdx.x / kLanes);
    const int64_t i = (int64_t)blockIdx.x * kBatchWaves + w;
    if (i >= nitems) return;
    const BatchItem it = items[i];
    run_y_item<R, MODE, MODE == GP_IMAG ? F_NORM_OUT : 0, QLO, QHI, SMAX>(py[it.prob], it, step,
                                                                        lds_raw + (size_t)w * lds_wave);
}

// Per problem: sum of its y partials of `step` (fixed order) into its norm total.
__global__ __launch_bounds__(256) void k_batch_norm_final(const SweepParams *__restrict__ py,
                                                          const int64_t *__restrict__ nparts, int64_t step)
{
    __shared__ double lds[256 / kLanes];
    const SweepParams &P = py[blockIdx.x];
    const double *part = P.norm_out + (step & 1) * P.n_norm;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < nparts[blockIdx.x]; i += blockDim.x) acc += part[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & (kLanes - 1)) == 0) lds[threadIdx.x / kLanes] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < 256 / kLanes; ++w) s += lds[w];
        // the x parameters read totals at P.norm_total + parity; y and x share the plan's buffer
        const_cast<double *>(P.norm_total)[step & 1] = s;
    }
}

// Per problem: psi <- psi / sqrt(dV * total of the last step).
template <typename R>
__global__ __launch_bounds__(256) void k_batch_scale(const SweepParams *__restrict__ py, int64_t last_step)
{
    using V = typename CT<R>::V;
    const SweepParams &P = py[blockIdx.x];
    const double s = 1.0 / sqrt(P.dV * P.norm_total[last_step & 1]);
    V *psi = (V *)P.out;
    const int64_t npts = P.n * P.nlines;
    for (int64_t i = threadIdx.x; i < npts; i += blockDim.x) {
        V v = psi[i];
        v.x = R((double)v.x * s);
        v.y = R((double)v.y * s);
        psi[i] = v;
    }
}

__global__ void k_fill_zero_i32(int *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ------------------------------------------------------------ persistent kernel

__device__ __forceinline__ bool wait_at_least(int *ctr, int target, int *error, unsigned limit)
{
    // lane 0 polls; the result is broadcast so the wavefront takes one branch
    int ok = 1;
    if ((threadIdx.x & (kLanes - 1)) == 0) {
        unsigned spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                ok = 0;
                break;
            }
            if (++spins > limit) {
                __hip_atomic_store(error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    ok = __shfl(ok, 0, kLanes);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // see the producers' grid writes
    return ok != 0;
}

template <typename R, int QMAX, int QY, int SMAX>
__global__ __launch_bounds__(kLanes *kBatchWaves) void k_batch_persistent(
    const SweepParams *__restrict__ px, const SweepParams *__restrict__ py, const BatchItem *__restrict__ xi,
    int64_t nxi, const BatchItem *__restrict__ yi, int64_t nyi, const int *__restrict__ nx_per,
    const int *__restrict__ ny_per, int64_t step0, int64_t nsteps, int *ctr, size_t lds_wave, unsigned limit)
{
    extern __shared__ char lds_raw[];
    const int w = wave_first_lane_i(threadIdx.x / kLanes);
    char *lds = lds_raw + (size_t)w * lds_wave;
    int *error = ctr + kCtrError;
    int *xdone = ctr + kCtrFirstProblem;
    const int64_t per_step = nxi + nyi;
    const int64_t total = per_step * nsteps;
    for (;;) {
        int64_t item = 0;
        if ((threadIdx.x & (kLanes - 1)) == 0)
            item = __hip_atomic_fetch_add(ctr + kCtrHead, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        item = __shfl(item, 0, kLanes);
        if (item >= total) break;
        if (__hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
        const int64_t sl = item / per_step;  // step within this launch
        const int64_t r = item - sl * per_step;
        if (r < nxi) {
            const BatchItem it = xi[r];
            int *ydone = xdone + 1;
            // the previous step's y items of this problem are done
            if (!wait_at_least(ydone + 2 * it.prob, (int)(sl * ny_per[it.prob]), error, limit)) break;
            run_x_item<R, GP_REAL, F_FUSE_N, 1, QMAX, SMAX>(px[it.prob], it, step0 + sl, lds);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if ((threadIdx.x & (kLanes - 1)) == 0)
                __hip_atomic_fetch_add(xdone + 2 * it.prob, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const BatchItem it = yi[r - nxi];
            // this step's x items of this problem are done
            if (!wait_at_least(xdone + 2 * it.prob, (int)((sl + 1) * nx_per[it.prob]), error, limit)) break;
            run_y_item<R, GP_REAL, 0, 0, QY, SMAX>(py[it.prob], it, step0 + sl, lds);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if ((threadIdx.x & (kLanes - 1)) == 0)
                __hip_atomic_fetch_add(xdone + 2 * it.prob + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ------------------------------------------------------------ host side

static void free_batch_device(gp_batch *b)
{
    (void)hipFree(b->d_px);
    (void)hipFree(b->d_py);
    (void)hipFree(b->d_xi);
    (void)hipFree(b->d_yi);
    (void)hipFree(b->d_ctr);
    (void)hipFree(b->d_nx_per);
    (void)hipFree(b->d_ny_per);
    (void)hipFree(b->d_nparts);
    b->d_px = b->d_py = nullptr;
    b->d_xi = b->d_yi = nullptr;
    b->d_ctr = b->d_nx_per = b->d_ny_per = nullptr;
    b->d_nparts = nullptr;
}

static gp_status upload(void **dst, const void *src, size_t bytes)
{
    hipError_t e = hipMalloc(dst, bytes > 0 ? bytes : 16);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(batch)");
    if (bytes > 0 && src) {  // src NULL: allocation only (filled on the device before use)
        e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(batch)");
    }
    return GP_OK;
}

// y segments of problem k (windowed y lines): at most the plan's count.
static int y_segments(const gp_plan *p, int want)
{
    const AxisPlan &A = p->ax[1];
    if (A.K < 0) return 1;
    return std::max(1, std::min(want, A.segs));
}

// (Re)build the device parameters and item lists for psis and the current config.
static gp_status prepare(gp_batch *b, void *const *psis)
{
    bool same = (int)b->bound.size() == b->count && b->bound_cfg.same_items(b->cfg);
    for (int k = 0; same && k < b->count; ++k) same = b->bound[k] == psis[k];
    if (same) return GP_OK;
    free_batch_device(b);
    std::vector<SweepParams> px(b->count), py(b->count);
    std::vector<std::vector<BatchItem>> xk(b->count), yk(b->count);  // per problem
    std::vector<int> nx_per(b->count), ny_per(b->count);
    std::vector<int64_t> nparts(b->count);
    size_t lds_wave = 0;
    auto lds_x = [&](int q) { return b->prec == GP_C128 ? x_lds_bytes<double>(q) : x_lds_bytes<float>(q); };
    auto lds_tile = [&](int q) {
        return b->prec == GP_C128 ? col_tile_lds_bytes<double>(q) : col_tile_lds_bytes<float>(q);
    };
    auto lds_ring = [&](int L) {
        return b->prec == GP_C128 ? window_lds_bytes<double, kStrided, 4>(L) : window_lds_bytes<float, kStrided, 4>(L);
    };
    for (int k = 0; k < b->count; ++k) {
        gp_plan *p = b->plans[k];
        // 2D: x psi -> work, y work -> psi
        px[k] = make_sweep_params(p, 0, psis[k], p->d_work, false, 0, nullptr);
        py[k] = make_sweep_params(p, 1, p->d_work, psis[k], false, 0, nullptr);
        px[k].norm_total = norm_total(p, 0);  // parity offsets are added in the kernels
        py[k].norm_total = norm_total(p, 0);
        py[k].norm_out = norm_partials(p, 0);
        const int64_t ny = p->n[1], nx = p->n[0];
        const int lx = b->cfg.lines_for(nx);
        for (int64_t l = 0; l < ny; l += lx) xk[k].push_back({k, 0, 1, (int)std::min<int64_t>(lx, ny - l), l});
        nx_per[k] = (int)xk[k].size();
        if (batch_tiles(p->ax[1])) {  // scan-solved y lines: items of whole tiles, one norm partial each
            const int64_t tl = b->prec == GP_C128 ? col_tile_lines<double>() : col_tile_lines<float>();
            int64_t per = std::max<int64_t>(b->cfg.lines_for(ny), (nx + p->n_norm - 1) / p->n_norm);
            per = (per + tl - 1) / tl * tl;
            for (int64_t l = 0; l < nx; l += per) {
                const int slot = (int)yk[k].size();
                yk[k].push_back({k, slot, 0, (int)std::min<int64_t>(per, nx - l), l});
            }
            nparts[k] = (int64_t)yk[k].size();
            lds_wave = std::max(lds_wave, lds_tile(p->ax[1].xq));
        } else {
            const int segs = y_segments(p, b->cfg.ysegs_for(ny));
            const int64_t groups = (nx + kLanes - 1) / kLanes;
            for (int s = 0; s < segs; ++s)
                for (int64_t g = 0; g < groups; ++g) yk[k].push_back({k, s, segs, 0, g});
            nparts[k] = groups * segs;
            lds_wave = std::max(lds_wave, lds_ring(p->ax[1].L));
        }
        ny_per[k] = (int)yk[k].size();
        // the persistent kernel's x items use the same region for their transposes
        lds_wave = std::max(lds_wave, lds_x(p->ax[0].xq));
    }
    std::vector<BatchItem> xi, yi;
    b->smax = 3;
    for (int k = 0; k < b->count; ++k) {
        xi.insert(xi.end(), xk[k].begin(), xk[k].end());
        yi.insert(yi.end(), yk[k].begin(), yk[k].end());
        const gp_plan *p = b->plans[k];
        if (p->ax[0].scan_steps > 3 || (batch_tiles(p->ax[1]) && p->ax[1].scan_steps > 3)) b->smax = 6;
    }
    gp_status st = upload((void **)&b->d_px, px.data(), px.size() * sizeof(SweepParams));
    if (st == GP_OK) st = upload((void **)&b->d_py, py.data(), py.size() * sizeof(SweepParams));
    if (st == GP_OK) st = upload((void **)&b->d_xi, xi.data(), xi.size() * sizeof(BatchItem));
    if (st == GP_OK) st = upload((void **)&b->d_yi, yi.data(), yi.size() * sizeof(BatchItem));
    if (st == GP_OK) st = upload((void **)&b->d_nx_per, nx_per.data(), nx_per.size() * sizeof(int));
    if (st == GP_OK) st = upload((void **)&b->d_ny_per, ny_per.data(), ny_per.size() * sizeof(int));
    if (st == GP_OK) st = upload((void **)&b->d_nparts, nparts.data(), nparts.size() * sizeof(int64_t));
    if (st == GP_OK) st = upload((void **)&b->d_ctr, nullptr, (kCtrFirstProblem + 2 * b->count) * sizeof(int));
    if (st != GP_OK) {
        free_batch_device(b);
        return st;
    }
    b->nxi = (int64_t)xi.size();
    b->nyi = (int64_t)yi.size();
    b->lds_wave = lds_wave;
    b->bound.assign(psis, psis + b->count);
    b->bound_cfg = b->cfg;
    return GP_OK;
}

template <typename R, int MODE, int QMAX, int QY, int SMAX>
static hipError_t run_phased(gp_batch *b, int64_t step0, int64_t nsteps, hipStream_t s)
{
    const unsigned gx = (unsigned)((b->nxi + kBatchWaves - 1) / kBatchWaves);
    const unsigned gy = (unsigned)((b->nyi + kBatchWaves - 1) / kBatchWaves);
    for (int64_t k = 0; k < nsteps; ++k) {
        const int64_t n = step0 + k;
        hipLaunchKernelGGL((k_batch_x<R, MODE, 1, QMAX, SMAX>), dim3(gx), dim3(kLanes * kBatchWaves), 0, s, b->d_px,
                           b->d_xi, b->nxi, n, (int)(k > 0));
        hipLaunchKernelGGL((k_batch_y<R, MODE, 0, QY, SMAX>), dim3(gy), dim3(kLanes * kBatchWaves),
                           kBatchWaves * b->lds_wave, s, b->d_py, b->d_yi, b->nyi, n, b->lds_wave);
        if (MODE == GP_IMAG)
            hipLaunchKernelGGL(k_batch_norm_final, dim3(b->count), dim3(256), 0, s, b->d_py, b->d_nparts, n);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (MODE == GP_IMAG)
        hipLaunchKernelGGL((k_batch_scale<R>), dim3(b->count), dim3(256), 0, s, b->d_py, step0 + nsteps - 1);
    return hipGetLastError();
}

template <typename R, int QMAX, int QY, int SMAX>
static hipError_t run_persistent(gp_batch *b, int64_t step0, int64_t nsteps, hipStream_t s)
{
    // the queue head and the per-problem counters are 32-bit: launches of at most 2^30 items
    const int64_t per_step = b->nxi + b->nyi;
    const int64_t chunk = std::max<int64_t>(1, ((int64_t)1 << 30) / per_step);
    const int64_t nctr = kCtrFirstProblem + 2 * b->count;
    for (int64_t k0 = 0; k0 < nsteps; k0 += chunk) {
        const int64_t m = std::min(chunk, nsteps - k0);
        hipLaunchKernelGGL(k_fill_zero_i32, dim3(1), dim3(256), 0, s, b->d_ctr, nctr);
        hipLaunchKernelGGL((k_batch_persistent<R, QMAX, QY, SMAX>), dim3((unsigned)b->cfg.grid), dim3(kLanes * kBatchWaves),
                           kBatchWaves * b->lds_wave, s, b->d_px, b->d_py, b->d_xi, b->nxi, b->d_yi, b->nyi,
                           b->d_nx_per, b->d_ny_per, step0 + k0, m, b->d_ctr, b->lds_wave, b->cfg.spin_limit);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename R, int QMAX, int QY, int SMAX>
static hipError_t run_batch_s(gp_batch *b, int64_t step0, int64_t nsteps, hipStream_t s)
{
    if (b->cfg.persistent && b->mode == GP_REAL) return run_persistent<R, QMAX, QY, SMAX>(b, step0, nsteps, s);
    return b->mode == GP_IMAG ? run_phased<R, GP_IMAG, QMAX, QY, SMAX>(b, step0, nsteps, s)
                              : run_phased<R, GP_REAL, QMAX, QY, SMAX>(b, step0, nsteps, s);
}

template <typename R, int QMAX, int QY>
static hipError_t run_batch_qy(gp_batch *b, int64_t step0, int64_t nsteps, hipStream_t s)
{
    return b->smax <= 3 ? run_batch_s<R, QMAX, QY, 3>(b, step0, nsteps, s)
                        : run_batch_s<R, QMAX, QY, 6>(b, step0, nsteps, s);
}

template <typename R, int QMAX>
static hipError_t run_batch_q(gp_batch *b, int64_t step0, int64_t nsteps, hipStream_t s)
{
    if (b->qmax_y == 0) return run_batch_qy<R, QMAX, 0>(b, step0, nsteps, s);
    if (b->qmax_y <= 2) return run_batch_qy<R, QMAX, 2>(b, step0, nsteps, s);
    if (b->qmax_y <= 4) return run_batch_qy<R, QMAX, 4>(b, step0, nsteps, s);
    return run_batch_qy<R, QMAX, 8>(b, step0, nsteps, s);
}

template <typename R>
static hipError_t run_batch_r(gp_batch *b, int64_t step0, int64_t nsteps, hipStream_t s)
{
    if (b->qmax <= 2) return run_batch_q<R, 2>(b, step0, nsteps, s);
    if (b->qmax <= 4) return run_batch_q<R, 4>(b, step0, nsteps, s);
    if (b->qmax <= 8) return run_batch_q<R, 8>(b, step0, nsteps, s);
    return run_batch_q<R, 16>(b, step0, nsteps, s);
}

static hipError_t run_batch(gp_batch *b, int64_t step0, int64_t nsteps, hipStream_t s)
{
    return b->prec == GP_C128 ? run_batch_r<double>(b, step0, nsteps, s) : run_batch_r<float>(b, step0, nsteps, s);
}

static gp_status check_error_flag(gp_batch *b, hipStream_t s)
{
    if (!(b->cfg.persistent && b->mode == GP_REAL)) return GP_OK;
    int flag = 0;
    hipError_t e = hipMemcpyAsync(&flag, b->d_ctr + kCtrError, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "batch error flag");
    if (flag) {
        set_error("persistent batch launch: a dependency wait exceeded its bound");
        return GP_ETIMEOUT;
    }
    return GP_OK;
}

// The batched kernels run the x sweep with the scan solver and the y sweep
// with the scan solver (y lines up to 512 points, exact) or the windowed solver
// of depth 1..8 blocks of 4 points, four wavefronts per workgroup each holding
// its ring (or x transpose buffer) in LDS.  A problem outside that (a longer y
// line that would need the exact two-pass solve or a deeper window, a ring set
// too large for the device's LDS) is rejected when the batch is created.  The
// y-sweep half of the check runs on the host before any HIP call.
static gp_status batch_y_supported(const AxisPlan &Y)
{
    if (Y.n <= (int64_t)kBatchTileMaxQ * kLanes) return GP_OK;  // scan solver
    if (Y.K < 0 || Y.B != 4 || Y.D < 1 || Y.D > 8)
        return set_error("batched y sweep needs a windowed solve of 1..8 blocks (dt/dx^2 too large)"),
               GP_EUNSUPPORTED;
    return GP_OK;
}

static gp_status batch_supports(const gp_plan *p, int max_lds)
{
    const AxisPlan &X = p->ax[0], &Y = p->ax[1];
    if (X.xq < 1 || X.xq > kXMaxQ) return set_error("batched x sweep needs 1 <= nx <= 1024"), GP_EUNSUPPORTED;
    const gp_status st = batch_y_supported(Y);
    if (st != GP_OK) return st;
    const size_t ring = batch_tiles(Y) ? (p->prec == GP_C128 ? col_tile_lds_bytes<double>(Y.xq)
                                                       : col_tile_lds_bytes<float>(Y.xq))
                        : p->prec == GP_C128 ? window_lds_bytes<double, kStrided, 4>(Y.L)
                                             : window_lds_bytes<float, kStrided, 4>(Y.L);
    const size_t xl = p->prec == GP_C128 ? x_lds_bytes<double>(X.xq) : x_lds_bytes<float>(X.xq);
    if (max_lds > 0 && (int64_t)kBatchWaves * (int64_t)std::max(ring, xl) > (int64_t)max_lds)
        return set_error("batched sweep's LDS (4 wavefronts' rings) exceeds the device limit"), GP_EUNSUPPORTED;
    return GP_OK;
}

static std::string cache_key(const gp_batch *b)
{
    std::vector<std::string> sizes;
    for (const gp_plan *p : b->plans) sizes.push_back(std::to_string(p->n[0]) + "x" + std::to_string(p->n[1]));
    std::sort(sizes.begin(), sizes.end());
    std::ostringstream os;
    os << (b->prec == GP_C128 ? "c128" : "c64") << (b->mode == GP_REAL ? "-real" : "-imag");
    for (const std::string &z : sizes) os << "-" << z;
    return os.str();
}

}  // namespace gp

using namespace gp;

extern "C" {

gp_status gp_batch_create(gp_batch **out, int count, const int64_t *n, const double *dx, const double *dt,
                          gp_mode mode, const gp_trap *traps, const double *g, gp_prec prec)
{
    if (!out || count < 1 || !n || !dx || !dt || !traps || !g) return set_error("bad argument"), GP_EINVAL;
    *out = nullptr;
    if (mode != GP_IMAG && mode != GP_REAL) return set_error("bad mode"), GP_EINVAL;
    if (prec != GP_C128 && prec != GP_C64) return set_error("bad precision"), GP_EINVAL;
    for (int k = 0; k < count; ++k) {
        if (n[2 * k] < 1 || n[2 * k + 1] < 1 || n[2 * k] > 64 * kXMaxQ)
            return set_error("batch problems need 1 <= n <= 1024 per axis"), GP_EINVAL;
        if (!(dx[k] > 0.0) || !(dt[k] > 0.0) || !std::isfinite(dx[k]) || !std::isfinite(dt[k]))
            return set_error("dx and dt must be finite and > 0"), GP_EINVAL;
        if (traps[k].sched_len != 0)
            return set_error("batched problems take static traps (no schedule)"), GP_EUNSUPPORTED;
        const gp_status st =
            batch_y_supported(preview_axis(n[2 * k + 1], n[2 * k], dx[k], dt[k], mode, prec, 4, false));
        if (st != GP_OK) return st;
    }
    gp_batch *b = new (std::nothrow) gp_batch();
    if (!b) return set_error("host allocation failed"), GP_ENOMEM;
    b->count = count;
    b->mode = mode;
    b->prec = prec;
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) {
        gp_batch_destroy(b);
        return hip_fail(e, "hipGetDevice");
    }
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device) != hipSuccess)
        max_lds = 0;
    for (int k = 0; k < count; ++k) {
        gp_trap trap{};
        trap.omega[0] = traps[k].omega[0];
        trap.omega[1] = traps[k].omega[1];
        const double dxs[2] = {dx[k], dx[k]};
        gp_plan *p = nullptr;
        gp_status st = gp_plan_create(&p, 2, n + 2 * k, dxs, dt[k], mode, &trap, g[k], prec);
        if (st != GP_OK) {
            gp_batch_destroy(b);
            return st;
        }
        b->plans.push_back(p);
        b->qmax = std::max(b->qmax, p->ax[0].xq);
        if (batch_tiles(p->ax[1])) b->qmax_y = std::max(b->qmax_y, p->ax[1].xq);
        st = batch_supports(p, max_lds);
        if (st != GP_OK) {
            gp_batch_destroy(b);
            return st;
        }
    }
    *out = b;
    return GP_OK;
}

gp_status gp_batch_destroy(gp_batch *b)
{
    if (!b) return GP_OK;
    free_batch_device(b);
    for (gp_plan *p : b->plans) gp_plan_destroy(p);
    delete b;
    return GP_OK;
}

gp_status gp_batch_step(gp_batch *b, void *const *psis, int64_t nsteps, void *stream)
{
    if (!b || !psis || nsteps < 0) return set_error("bad argument"), GP_EINVAL;
    for (int k = 0; k < b->count; ++k)
        if (!psis[k]) return set_error("NULL problem grid"), GP_EINVAL;
    if (nsteps == 0) return GP_OK;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSetDevice(b->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    gp_status st = prepare(b, psis);
    if (st != GP_OK) return st;
    const int64_t step0 = b->plans[0]->step;
    e = run_batch(b, step0, nsteps, s);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    st = check_error_flag(b, s);
    if (st != GP_OK) return st;  // the grids are not advanced consistently: step indices stay put
    for (gp_plan *p : b->plans) p->step += nsteps;
    return GP_OK;
}

gp_status gp_batch_observables(gp_batch *b, int k, const void *psi, gp_obs *out, void *stream)
{
    if (!b || k < 0 || k >= b->count) return set_error("bad batch or index"), GP_EINVAL;
    return gp_observables(b->plans[k], psi, out, stream);
}

gp_status gp_batch_autotune(gp_batch *b, const char *cache_path, void *stream)
{
    if (!b) return set_error("bad batch"), GP_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSetDevice(b->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const std::string key = cache_key(b);
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream is(line);
            std::string k2;
            BatchConfig c;
            c.spin_limit = b->cfg.spin_limit;
            if (!(is >> k2 >> c.persistent >> c.lines >> c.ysegs >> c.grid) || k2 != key) continue;
            // optional per-side settings: "sides" then "len:lines:ysegs" triples
            std::string tok;
            bool ok = true;
            if (is >> tok) {
                ok = tok == "sides";
                while (ok && is >> tok) {
                    long long len = 0;
                    int ln = 0, ys = 0;
                    ok = std::sscanf(tok.c_str(), "%lld:%d:%d", &len, &ln, &ys) == 3 && len > 0 && ln >= 1 &&
                         ln <= 64 && ys >= 1 && ys <= 64;
                    if (ok) {
                        c.side_lines[len] = ln;
                        c.side_ysegs[len] = ys;
                    }
                }
            }
            if (!ok) continue;
            b->cfg = c;
            b->bound.clear();
            return GP_OK;
        }
    }
    // scratch copies of every problem (Gaussian-like content does not matter for timing)
    std::vector<void *> scratch(b->count, nullptr);
    for (int k = 0; k < b->count; ++k) {
        const gp_plan *p = b->plans[k];
        const size_t bytes = (size_t)p->npts * elem_bytes(b->prec);
        e = hipMalloc(&scratch[k], bytes);
        if (e == hipSuccess) e = hipMemsetAsync(scratch[k], 0, bytes, s);
        if (e != hipSuccess) {
            for (void *q : scratch) (void)hipFree(q);
            return hip_fail(e, "autotune scratch");
        }
    }
    const BatchConfig saved = b->cfg;
    std::vector<int64_t> saved_steps;
    for (gp_plan *p : b->plans) saved_steps.push_back(p->step);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        for (void *q : scratch) (void)hipFree(q);
        return hip_fail(e, "autotune events");
    }
    gp_status st = GP_OK;
    const int64_t steps = 10;
    // ms for `steps` steps under config c (+inf when it cannot run)
    auto time_cfg = [&](const BatchConfig &c) -> float {
        b->cfg = c;
        st = prepare(b, scratch.data());
        if (st != GP_OK) return 1e30f;
        if (run_batch(b, 0, 2, s) != hipSuccess) return 1e30f;  // warm-up
        if (hipEventRecord(e0, s) != hipSuccess) return 1e30f;
        const hipError_t er = run_batch(b, 0, steps, s);
        if (hipEventRecord(e1, s) != hipSuccess || er != hipSuccess) return 1e30f;
        if (hipEventSynchronize(e1) != hipSuccess) return 1e30f;
        if (check_error_flag(b, s) != GP_OK) return 1e30f;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 1e30f;
        return ms;
    };
    // 1. one setting for every problem
    std::vector<BatchConfig> cands;
    for (int lines : {1, 2, 4})
        for (int ysegs : {1, 2, 4, 8, 16, 32}) {
            BatchConfig c;
            c.spin_limit = b->cfg.spin_limit;
            c.persistent = 0;
            c.lines = lines;
            c.ysegs = ysegs;
            cands.push_back(c);
            if (b->mode == GP_REAL)
                for (int grid : {256, 512, 1024, 2048}) {
                    c.persistent = 1;
                    c.grid = grid;
                    cands.push_back(c);
                }
        }
    float best = 1e30f;
    BatchConfig best_cfg = saved;
    for (const BatchConfig &c : cands) {
        const float ms = time_cfg(c);
        if (st != GP_OK) break;
        if (ms < best) {
            best = ms;
            best_cfg = c;
        }
    }
    // 2. per line length, largest total first: lines per item (x lines and
    // scan-solved y lines of that length) and y segments (windowed y lines),
    // kept when at least 1% faster
    if (st == GP_OK && best < 1e29f) {
        std::map<int64_t, int64_t> pts_x, pts_yw;  // points on lines of each length
        for (const gp_plan *p : b->plans) {
            pts_x[p->n[0]] += p->npts;
            if (batch_tiles(p->ax[1]))
                pts_x[p->n[1]] += p->npts;
            else
                pts_yw[p->n[1]] += p->npts;
        }
        auto by_size = [](const std::map<int64_t, int64_t> &m) {
            std::vector<std::pair<int64_t, int64_t>> v(m.begin(), m.end());
            std::sort(v.begin(), v.end(), [](const auto &a, const auto &c) { return a.second > c.second; });
            return v;
        };
        for (const auto &[len, pts] : by_size(pts_x))
            for (int lines : {1, 2, 4, 8}) {
                if (st != GP_OK || lines == best_cfg.lines_for(len)) continue;
                BatchConfig c = best_cfg;
                c.side_lines[len] = lines;
                const float ms = time_cfg(c);
                if (st != GP_OK) break;
                if (ms < 0.99f * best) {
                    best = ms;
                    best_cfg = c;
                }
            }
        for (const auto &[len, pts] : by_size(pts_yw))
            for (int ysegs : {1, 2, 4, 8, 16, 32}) {
                if (st != GP_OK || ysegs == best_cfg.ysegs_for(len)) continue;
                BatchConfig c = best_cfg;
                c.side_ysegs[len] = ysegs;
                const float ms = time_cfg(c);
                if (st != GP_OK) break;
                if (ms < 0.99f * best) {
                    best = ms;
                    best_cfg = c;
                }
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (void *q : scratch) (void)hipFree(q);
    for (int k = 0; k < b->count; ++k) b->plans[k]->step = saved_steps[k];
    b->cfg = st == GP_OK ? best_cfg : saved;
    b->bound.clear();  // rebuild for the caller's grids on the next step
    if (st != GP_OK) return st;
    if (cache_path) {
        std::ofstream o(cache_path, std::ios::app);
        o << key << " " << b->cfg.persistent << " " << b->cfg.lines << " " << b->cfg.ysegs << " " << b->cfg.grid;
        std::map<int64_t, int> sides;
        for (const auto &kv : b->cfg.side_lines) sides[kv.first] = 1;
        for (const auto &kv : b->cfg.side_ysegs) sides[kv.first] = 1;
        if (!sides.empty()) {
            o << " sides";
            for (const auto &kv : sides)
                o << " " << kv.first << ":" << b->cfg.lines_for(kv.first) << ":" << b->cfg.ysegs_for(kv.first);
        }
        o << "\n";
    }
    return GP_OK;
}

gp_status gp_autotune(gp_batch *b, const char *cache_path) { return gp_batch_autotune(b, cache_path, nullptr); }

gp_status gp_batch_set_wait_limit(gp_batch *b, uint32_t polls)
{
    if (!b || polls < 1) return set_error("bad argument"), GP_EINVAL;
    b->cfg.spin_limit = polls;
    return GP_OK;
}

gp_status gp_batch_get_config(const gp_batch *b, int *persistent, int *lines, int *ysegs, int *grid)
{
    if (!b || !persistent || !lines || !ysegs || !grid) return set_error("bad argument"), GP_EINVAL;
    *persistent = b->cfg.persistent;
    *lines = b->cfg.lines;
    *ysegs = b->cfg.ysegs;
    *grid = b->cfg.grid;
    return GP_OK;
}

gp_status gp_batch_set_config(gp_batch *b, int persistent, int lines, int ysegs, int grid)
{
    if (!b || persistent < 0 || persistent > 1 || lines < 1 || lines > 64 || ysegs < 1 || ysegs > 64 || grid < 1 ||
        grid > 65536)
        return set_error("bad argument"), GP_EINVAL;
    if (persistent && b->mode != GP_REAL) return set_error("persistent batches run real time only"), GP_EUNSUPPORTED;
    b->cfg.persistent = persistent;
    b->cfg.lines = lines;
    b->cfg.ysegs = ysegs;
    b->cfg.grid = grid;
    b->cfg.side_lines.clear();
    b->cfg.side_ysegs.clear();
    b->bound.clear();
    return GP_OK;
}

gp_status gp_batch_set_side_config(gp_batch *b, int64_t side, int lines, int ysegs)
{
    if (!b || side < 1 || lines < 1 || lines > 64 || ysegs < 1 || ysegs > 64)
        return set_error("bad argument"), GP_EINVAL;
    b->cfg.side_lines[side] = lines;
    b->cfg.side_ysegs[side] = ysegs;
    b->bound.clear();
    return GP_OK;
}

gp_status gp_batch_get_side_config(const gp_batch *b, int64_t side, int *lines, int *ysegs)
{
    if (!b || side < 1 || !lines || !ysegs) return set_error("bad argument"), GP_EINVAL;
    *lines = b->cfg.lines_for(side);
    *ysegs = b->cfg.ysegs_for(side);
    return GP_OK;
}

}  // extern "C"

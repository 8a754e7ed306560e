// The x and y sweeps of a 3D step fused over xy-planes.
//
// The CN substeps along x and y act on one xy-plane at a time, and the y
// sweep's windowed solver consumes rows in order, so the x sweep's output never
// needs to reach HBM: one workgroup walks the rows of one plane (or one segment
// of its rows) in blocks of four.  Each of its four wavefronts x-solves one row
// of the block (potential substep on load, the same affine-scan solve as the x
// kernel) into an LDS tile; then every thread takes one column of the tile and
// advances that column's windowed y solve (the strided-sweep solver with its LDS
// ring), writing finished rows of the y output.  The grid is read once and
// written once for both substeps.
//
// Segments of a plane's rows start their y elimination DW blocks early from
// zero state, like the strided sweeps' segments; the x rows of those warm-up
// blocks are solved again by the segment that needs them.
#include <algorithm>

#include "gp_internal.h"
#include "gp_sweep_common.h"
#include "gp_window.h"
#include "gp_xscan.h"

namespace gp {

namespace {

constexpr int kXYWaves = 4;  // wavefronts per workgroup = rows per block of the y window
constexpr int kXYAhead = 1;  // blocks whose rows are loaded ahead
constexpr int kXYMaxScan = 3;  // x scan steps the fused kernel supports

// Tile slot of point q of a row: the low three bits (one 128-byte group of
// 16-byte values) are permuted by the next three, so the coalesced row
// (lane + 64 i), the solver's consecutive points (lane Q + i) and the column
// reads each hit eight distinct 16-byte bank groups per eight lanes.
__device__ __forceinline__ int xy_slot(int q) { return q ^ ((q >> 3) & 7); }

// Row y = jb B + w of plane k (zeros past the plane or past block j1).
template <typename R, int Q>
__device__ __forceinline__ void xy_load_row(const typename CT<R>::V *src, int jb, int j1, int w, int64_t k,
                                            int64_t nx, int64_t ny, int lane, typename CT<R>::V (&dst_row)[Q])
{
    using V = typename CT<R>::V;
    const int64_t y = (int64_t)jb * kXYWaves + w;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        dst_row[i] = (jb < j1 && y < ny && lane + kLanes * i < nx) ? src[(y + ny * k) * nx + lane + kLanes * i]
                                                                   : to_v<V>(cp<R>{R(0), R(0)});
}

template <typename R, int MODE, int XFLAGS, int Q, int DW>
__global__ __launch_bounds__(kLanes *kXYWaves) void k_sweep_xy(SweepParams PX, SweepParams PY,
                                                                const typename CT<R>::V *src,
                                                                typename CT<R>::V *dst,
                                                                const typename CT<R>::V *__restrict__ tabx,
                                                                const typename CT<R>::V *__restrict__ taby)
{
    using V = typename CT<R>::V;
    constexpr int B = kXYWaves;
    __shared__ V tile[B][kLanes * Q];
    extern __shared__ char ring_raw[];
    const int lane = threadIdx.x & (kLanes - 1);
    // wave-uniform by construction; stated so, the y solver's table rows (whose
    // addresses depend only on the block) are read as scalar loads, outside the
    // vector memory counter that the prefetched rows occupy
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    const int64_t nx = PX.n, ny = PY.n;
    const int64_t k = blockIdx.y;  // plane
    const int cw = (int)(nx / kLanes);  // wavefronts with columns in the y part
    const size_t ringb = (size_t)(PY.lmask + 1) * kLanes * sizeof(V);
    const cp<R> zero = {R(0), R(0)};

    // y solver of this wavefront's 64 columns: y lines l = x + nx k
    WindowSweep<R, MODE, 0, kStrided, DW, 4> Y(PY, nullptr, dst, taby, nullptr, ring_raw + w * ringb,
                                                k * cw + w, (int)blockIdx.x, (int)gridDim.x, 0);
    const int j0 = Y.o_lo - DW > 0 ? Y.o_lo - DW : 0;
    const int j1 = Y.o_hi + DW;  // exclusive; uniform over the workgroup

    const int S = PX.scan_steps;  // at most kXYMaxScan (checked on the host)
    XConsts<R, Q, kXYMaxScan> KX;
    x_consts_load<R, Q, kXYMaxScan>(PX, tabx, (const V *)PX.xmul, lane, KX);
    const double renorm = (XFLAGS & F_RENORM) ? 1.0 / sqrt(PX.dV * PX.norm_total[0]) : 1.0;
    // this wavefront's rows of the next kXYAhead blocks stay in flight while a
    // block is solved (one slot per block; the loop is unrolled over the slots so
    // every slot index is a compile-time constant)
    V ahead[kXYAhead][Q];
#pragma unroll
    for (int t = 0; t < kXYAhead; ++t) xy_load_row<R, Q>(src, j0 + t, j1, w, k, nx, ny, lane, ahead[t]);
    V *row = tile[w];
#pragma unroll 1
    for (int jb = j0; jb < j1; jb += kXYAhead) {
#pragma unroll
        for (int t = 0; t < kXYAhead; ++t) {
            const int j = jb + t;
            if (j >= j1) break;  // uniform over the workgroup
            const int64_t y = (int64_t)j * B + w;
            cp<R> u[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) u[i] = from_v<R>(ahead[t][i]);
            if (y < ny) {  // uniform over the wavefront
                LineCtx<R> L = line_ctx_of<R>(PX, y + ny * k);
                if (XFLAGS & F_RENORM) L.scale = renorm;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const int64_t q = lane + kLanes * i;
                    if ((XFLAGS & F_FUSE_N) && q < nx) u[i] = potential_substep<R, MODE, XFLAGS>(u[i], q, PX, L);
                }
                if (Q > 1) {  // coalesced -> Q consecutive points per lane
#pragma unroll
                    for (int i = 0; i < Q; ++i) row[xy_slot(lane + kLanes * i)] = to_v<V>(u[i]);
                    wave_lds_sync();
#pragma unroll
                    for (int i = 0; i < Q; ++i) u[i] = from_v<R>(row[xy_slot(lane * Q + i)]);
                }
                x_line_solve<R, MODE, Q, kXYMaxScan>(PX, KX, S, lane, u);
#pragma unroll
                for (int i = 0; i < Q; ++i) row[xy_slot(lane * Q + i)] = to_v<V>(u[i]);
            } else {  // rows past the plane are the y solver's zero rows
#pragma unroll
                for (int i = 0; i < Q; ++i) row[xy_slot(lane * Q + i)] = to_v<V>(zero);
            }
            // the next rows are requested only now: the vector memory counter is
            // in order, so waiting for the x solve's table loads would otherwise
            // wait for them too
            xy_load_row<R, Q>(src, j + kXYAhead, j1, w, k, nx, ny, lane, ahead[t]);
            __syncthreads();
            if (w < cw) {
                V buf[B];
#pragma unroll
                for (int r = 0; r < B; ++r) buf[r] = tile[r][xy_slot(w * kLanes + lane)];
                Y.template process<false>(buf, j);  // tile rows are zero off the grid
            }
            __syncthreads();
        }
    }
}

template <typename R, int MODE, int XFLAGS, int Q, int DW>
static void launch_xy_dw(const gp_plan *p, const SweepParams &PX, const SweepParams &PY, hipStream_t s)
{
    using V = typename CT<R>::V;
    const size_t ring = (size_t)kXYWaves * (PY.lmask + 1) * kLanes * sizeof(V);
    hipLaunchKernelGGL((k_sweep_xy<R, MODE, XFLAGS, Q, DW>), dim3((unsigned)p->xy_segs, (unsigned)p->n[2]),
                       dim3(kLanes * kXYWaves), ring, s, PX, PY, (const V *)PX.psi, (V *)PY.out,
                       (const V *)PX.tab, (const V *)PY.tab);
}

template <typename R, int MODE, int XFLAGS, int Q>
static hipError_t launch_xy_q(const gp_plan *p, const SweepParams &PX, const SweepParams &PY, hipStream_t s)
{
    switch (p->ax[1].D) {
    case 2: launch_xy_dw<R, MODE, XFLAGS, Q, 2>(p, PX, PY, s); break;
    case 3: launch_xy_dw<R, MODE, XFLAGS, Q, 3>(p, PX, PY, s); break;
    case 4: launch_xy_dw<R, MODE, XFLAGS, Q, 4>(p, PX, PY, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R, int MODE, int XFLAGS>
static hipError_t launch_xy_flags(const gp_plan *p, const SweepParams &PX, const SweepParams &PY, hipStream_t s)
{
    switch (p->ax[0].xq) {
    case 2: return launch_xy_q<R, MODE, XFLAGS, 2>(p, PX, PY, s);
    case 4: return launch_xy_q<R, MODE, XFLAGS, 4>(p, PX, PY, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename R>
static hipError_t launch_xy_r(const gp_plan *p, const SweepParams &PX, const SweepParams &PY, int flags,
                              hipStream_t s)
{
    if (p->mode == GP_IMAG)
        return (flags & F_RENORM) ? launch_xy_flags<R, GP_IMAG, F_FUSE_N | F_RENORM>(p, PX, PY, s)
                                  : launch_xy_flags<R, GP_IMAG, F_FUSE_N>(p, PX, PY, s);
    return launch_xy_flags<R, GP_REAL, F_FUSE_N>(p, PX, PY, s);
}

}  // namespace

size_t xy_lds_bytes(const gp_plan *p)
{
    const size_t eb = elem_bytes(p->prec);
    return (size_t)kXYWaves * kLanes * (size_t)p->ax[0].xq * eb +
           (size_t)kXYWaves * (size_t)p->ax[1].L * kLanes * eb;
}

int xy_choose_segments(const gp_plan *p, int64_t max_lds)
{
    if (p->ndim != 3) return 0;
    const AxisPlan &X = p->ax[0], &Y = p->ax[1];
    if (X.xq != 2 && X.xq != 4) return 0;
    if (X.scan_steps > kXYMaxScan) return 0;
    if (p->n[0] % kLanes != 0 || p->n[0] > (int64_t)kLanes * X.xq) return 0;
    if (Y.K < 0 || Y.B != 4 || Y.D < 2 || Y.D > 4) return 0;
    if ((int64_t)xy_lds_bytes(p) > max_lds) return 0;
    // about two workgroups per CU of a 256-CU device, each segment at least
    // four windows long
    const int64_t nb = (p->n[1] + 3) / 4;
    int segs = (int)((512 + p->n[2] - 1) / p->n[2]);
    const int most = (int)std::max<int64_t>(1, nb / (4 * (Y.D + 1)));
    if (segs > most) segs = most;
    return segs < 1 ? 1 : segs;
}

hipError_t launch_xy(gp_plan *p, const void *src, void *dst, int flags, int64_t step_index, hipStream_t s)
{
    SweepParams PX = make_sweep_params(p, 0, src, nullptr, false, step_index, nullptr);
    SweepParams PY = make_sweep_params(p, 1, nullptr, dst, false, step_index, nullptr);
    timing_begin(p, K_SWEEP_XY, s);
    const hipError_t e = p->prec == GP_C128 ? launch_xy_r<double>(p, PX, PY, flags, s)
                                            : launch_xy_r<float>(p, PX, PY, flags, s);
    timing_end(p, s);
    return e;
}

}  // namespace gp

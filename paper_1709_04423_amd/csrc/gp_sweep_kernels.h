// Line-sweep kernels of the SSCN step: one Crank-Nicolson kinetic substep
// along one axis over every grid line, with the pointwise potential/nonlinear
// substep fused into the first axis's loads, the imaginary-time norm partials
// fused into the last axis's stores, and the adjoint of the potential substep
// fused into the adjoint x sweep's stores.
//
// Mapping: one grid line per lane, 64 lines per wavefront (= workgroup).  For
// the strided axes the 64 lines of a wavefront are adjacent in x, so every
// load/store instruction moves one contiguous row segment.
//
// Solver: the Thomas algorithm on the constant-coefficient tridiagonal CN
// system (scaled to unit off-diagonals, see below), streamed in blocks of
// kBlock points.  Forward elimination is exact and runs as the values stream
// in; the eliminated values go to a per-lane ring in LDS.  Back substitution
// u_t = y_t - c'_t u_{t+1} runs per output block of kBlock points, starting K
// points past the block with u = 0: the neglected term is multiplied by
// prod |c'| <= rho^(K+1) before it reaches an output.  K = D kBlock - 1 for a
// compile-time D (1..4), the smallest with rho^(K+1) below 2^-60 (FP64) or
// 2^-44 (FP32), so the back substitution is fully unrolled.  Rows past the end of
// a line hold c' = 0, so the tail of every line is exact.  Each point is read
// once and written once.  When the window does not fit in LDS, k_sweep_exact
// runs the plain two-pass Thomas algorithm (eliminated values stored in
// place, then read back).
#pragma once

#include "gp_internal.h"
#include "gp_sweep_common.h"
#include "gp_window.h"

namespace gp {

// Access patterns of the windowed solver.
//  kStrided: lane = line, point q of the line at base + q*stride; used for the
//    y and z axes, whose 64 lines per wavefront are adjacent in memory, so each
//    load/store instruction moves one contiguous row.
//  kTransposed: the 64 lines of a wavefront are 64 consecutive x lines (length
//    n, stride 1).  Each block of kBlock points of the 64 lines is loaded with
//    coalesced instructions (instruction i, lane -> line 4i + lane/16, point
//    lane%16) and transposed through an LDS tile to the one-line-per-lane layout
//    of the solver; outputs go back the same way.
template <typename R, int MODE, int FLAGS, int ACC, int DW, int BB>
__global__ __launch_bounds__(kLanes) void k_sweep_window(SweepParams P, const typename CT<R>::V *src,
                                                         typename CT<R>::V *dst,
                                                         const typename CT<R>::V *__restrict__ tab,
                                                         const typename CT<R>::V *__restrict__ state)
{
    extern __shared__ char lds_raw[];
    window_run<R, MODE, FLAGS, ACC, DW, BB>(P, src, dst, tab, state, lds_raw, blockIdx.x, blockIdx.y, gridDim.y,
                                           blockIdx.x + (int64_t)gridDim.x * blockIdx.y);
}

// Plain two-pass Thomas algorithm: forward elimination stores d in place,
// back substitution reads it back.  Exact for any window; twice the traffic.
template <typename R, int MODE, int FLAGS>
__global__ __launch_bounds__(kLanes) void k_sweep_exact(SweepParams P, const typename CT<R>::V *src,
                                                        typename CT<R>::V *dst,
                                                        const typename CT<R>::V *__restrict__ tab,
                                                        const typename CT<R>::V *__restrict__ state)
{
    using V = typename CT<R>::V;
    const int lane = threadIdx.x;
    const LineCtx<R> L = line_setup<R, FLAGS>(P, blockIdx.x, lane);
    const int64_t n = P.n, stride = P.stride, base = L.base;
    double nacc = 0.0, acc_w = 0.0, acc_g = 0.0;

    if (L.active) {
        cp<R> um1 = {R(0), R(0)}, dprev = {R(0), R(0)};
        cp<R> u0 = from_v<R>(src[base]);
        if (FLAGS & F_FUSE_N) u0 = potential_substep<R, MODE, FLAGS>(u0, 0, P, L);
        for (int64_t q = 1; q <= n; ++q) {
            cp<R> up1 = {R(0), R(0)};
            if (q < n) {
                up1 = from_v<R>(src[base + q * stride]);
                if (FLAGS & F_FUSE_N) up1 = potential_substep<R, MODE, FLAGS>(up1, q, P, L);
            }
            const cp<R> d = cn_elim<MODE, R>(cn_rhs<MODE, R>(um1, u0, up1, tab[3 * q + 1], tab[3 * q + 2]), dprev,
                                             tab[3 * q]);
            dst[base + (q - 1) * stride] = to_v<V>(d);
            dprev = d;
            um1 = u0;
            u0 = up1;
        }
        cp<R> v = {R(0), R(0)};
        for (int64_t t = n - 1; t >= 0; --t) {
            const int64_t addr = base + t * stride;
            v = cn_back<MODE, R>(from_v<R>(dst[addr]), tab[3 * (t + 1)], v);
            cp<R> w = v;
            if (FLAGS & F_NORM_OUT) nacc += (double)w.re * (double)w.re + (double)w.im * (double)w.im;
            if (FLAGS & F_ADJ_N) w = potential_adjoint<R, MODE, FLAGS>(w, t, state, addr, P, L, acc_w, acc_g);
            dst[addr] = to_v<V>(w);
        }
    }
    write_partials<R, FLAGS>(P, lane, nacc, acc_w, acc_g, blockIdx.x);
}

// -------------------------------------------------------------- dispatch

template <typename R, int MODE, int FLAGS, int ACC, int DW, int BB>
static void launch_window(const AxisPlan &A, const SweepParams &P, const void *tab, hipStream_t s)
{
    using V = typename CT<R>::V;
    const dim3 grid((unsigned)((A.nlines + kLanes - 1) / kLanes), (unsigned)A.segs);
    const size_t lds = window_lds_bytes<R, ACC, BB>(A.L);
    hipLaunchKernelGGL((k_sweep_window<R, MODE, FLAGS, ACC, DW, BB>), grid, dim3(kLanes), lds, s, P,
                       (const V *)P.psi, (V *)P.out, (const V *)tab, (const V *)P.state);
}

template <typename R, int MODE, int FLAGS, int ACC>
static hipError_t launch_window_d(const AxisPlan &A, const SweepParams &P, const void *tab, hipStream_t s)
{
    if (ACC == kTransposed) {  // blocks of 16 points
        if (A.B != 16) return hipErrorInvalidValue;
        switch (A.D) {
        case 1: launch_window<R, MODE, FLAGS, ACC, 1, 16>(A, P, tab, s); break;
        case 2: launch_window<R, MODE, FLAGS, ACC, 2, 16>(A, P, tab, s); break;
        case 3: launch_window<R, MODE, FLAGS, ACC, 3, 16>(A, P, tab, s); break;
        case 4: launch_window<R, MODE, FLAGS, ACC, 4, 16>(A, P, tab, s); break;
        default: return hipErrorInvalidValue;
        }
    } else {  // blocks of 4 points (strided axes, both precisions)
        if (A.B != 4) return hipErrorInvalidValue;
        switch (A.D) {
        case 1: launch_window<R, MODE, FLAGS, ACC, 1, 4>(A, P, tab, s); break;
        case 2: launch_window<R, MODE, FLAGS, ACC, 2, 4>(A, P, tab, s); break;
        case 3: launch_window<R, MODE, FLAGS, ACC, 3, 4>(A, P, tab, s); break;
        case 4: launch_window<R, MODE, FLAGS, ACC, 4, 4>(A, P, tab, s); break;
        case 5: launch_window<R, MODE, FLAGS, ACC, 5, 4>(A, P, tab, s); break;
        case 6: launch_window<R, MODE, FLAGS, ACC, 6, 4>(A, P, tab, s); break;
        case 7: launch_window<R, MODE, FLAGS, ACC, 7, 4>(A, P, tab, s); break;
        case 8: launch_window<R, MODE, FLAGS, ACC, 8, 4>(A, P, tab, s); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

template <typename R, int MODE, int FLAGS>
static hipError_t launch_one(const AxisPlan &A, const SweepParams &P, bool exact, bool transposed, const void *tab,
                             hipStream_t s)
{
    using V = typename CT<R>::V;
    if (exact) {
        const unsigned grid = (unsigned)((A.nlines + kLanes - 1) / kLanes);
        hipLaunchKernelGGL((k_sweep_exact<R, MODE, FLAGS>), dim3(grid), dim3(kLanes), 0, s, P,
                           (const V *)P.psi, (V *)P.out, (const V *)tab, (const V *)P.state);
        return hipGetLastError();
    }
    if (transposed) return launch_window_d<R, MODE, FLAGS, kTransposed>(A, P, tab, s);
    return launch_window_d<R, MODE, FLAGS, kStrided>(A, P, tab, s);
}

template <typename R, int MODE>
static hipError_t dispatch_flags(const AxisPlan &A, const SweepParams &P, int flags, bool exact, bool tr,
                                 const void *tab, hipStream_t s)
{
    if (MODE == GP_IMAG) {
        switch (flags) {
        case 0: return launch_one<R, MODE, 0>(A, P, exact, tr, tab, s);
        case F_FUSE_N: return launch_one<R, MODE, F_FUSE_N>(A, P, exact, tr, tab, s);
        case F_FUSE_N | F_RENORM: return launch_one<R, MODE, F_FUSE_N | F_RENORM>(A, P, exact, tr, tab, s);
        case F_NORM_OUT: return launch_one<R, MODE, F_NORM_OUT>(A, P, exact, tr, tab, s);
        case F_FUSE_N | F_NORM_OUT: return launch_one<R, MODE, F_FUSE_N | F_NORM_OUT>(A, P, exact, tr, tab, s);
        case F_FUSE_N | F_RENORM | F_NORM_OUT:
            return launch_one<R, MODE, F_FUSE_N | F_RENORM | F_NORM_OUT>(A, P, exact, tr, tab, s);
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (flags) {
        case 0: return launch_one<R, MODE, 0>(A, P, exact, tr, tab, s);
        case F_FUSE_N: return launch_one<R, MODE, F_FUSE_N>(A, P, exact, tr, tab, s);
        case F_ADJ_N: return launch_one<R, MODE, F_ADJ_N>(A, P, exact, tr, tab, s);
        default: return hipErrorInvalidValue;
        }
    }
}

}  // namespace gp

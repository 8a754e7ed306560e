// x sweep kernel (contiguous axis, one wavefront per line; see gp_xscan.h) and its dispatch.
#include "gp_internal.h"
#include "gp_sweep_common.h"
#include "gp_xscan.h"

namespace gp {

template <typename R, int MODE, int FLAGS, int Q, int SMAX>
__global__ __launch_bounds__(kLanes *kXWaves) void k_sweep_x_scan(SweepParams P, const typename CT<R>::V *src,
                                                                   typename CT<R>::V *dst,
                                                                   const typename CT<R>::V *__restrict__ tab,
                                                                   const typename CT<R>::V *__restrict__ state)
{
    using V = typename CT<R>::V;
    const int lane = threadIdx.x & (kLanes - 1);
    const int wave = threadIdx.x / kLanes;
    __shared__ V xl[kXWaves][kLanes * (Q + 1)];
    double nacc = 0.0, acc_w = 0.0, acc_g = 0.0;
    if constexpr (Q >= kXLdsQ) {  // table rows in LDS, one copy for the workgroup
        __shared__ V kc[3 * Q * kLanes];
        x_rows_to_lds<R, Q>(P, tab, kc);
        __syncthreads();
        x_scan_wave<R, MODE, FLAGS, Q, SMAX, true>(P, src, dst, tab, state,
                                                   ((int64_t)blockIdx.x * kXWaves + wave) * P.xlpw, P.xlpw, nacc,
                                                   acc_w, acc_g, xl[wave], kc);
    } else {
        x_scan_wave<R, MODE, FLAGS, Q, SMAX>(P, src, dst, tab, state, ((int64_t)blockIdx.x * kXWaves + wave) * P.xlpw,
                                             P.xlpw, nacc, acc_w, acc_g, xl[wave]);
    }
    if (FLAGS & (F_NORM_OUT | F_ADJ_N)) {
        __shared__ double red[kXWaves][3];
        nacc = wave_sum(nacc);
        acc_w = wave_sum(acc_w);
        acc_g = wave_sum(acc_g);
        if (lane == 0) {
            red[wave][0] = nacc;
            red[wave][1] = acc_w;
            red[wave][2] = acc_g;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = 0.0, b = 0.0, c = 0.0;
            for (int w = 0; w < kXWaves; ++w) {
                a += red[w][0];
                b += red[w][1];
                c += red[w][2];
            }
            if (FLAGS & F_NORM_OUT) P.norm_out[blockIdx.x] = a;
            if (FLAGS & F_ADJ_N) {
                P.adj_out[2 * blockIdx.x] = b;
                P.adj_out[2 * blockIdx.x + 1] = c;
            }
        }
        if ((FLAGS & F_ADJ_N) && P.adj_done) {
            // the last workgroup to finish reduces every workgroup's partials,
            // in the fixed order of the separate reduce kernel
            __shared__ int last;
            if (threadIdx.x == 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                const int done = __hip_atomic_fetch_add(P.adj_done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                last = done == (int)gridDim.x - 1;
            }
            __syncthreads();
            if (last && wave == 0) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                double sw = 0.0, sg = 0.0;
                for (int i = lane; i < (int)gridDim.x; i += kLanes) {
                    sw += __hip_atomic_load(P.adj_out + 2 * i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    sg += __hip_atomic_load(P.adj_out + 2 * i + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                sw = wave_sum(sw);
                sg = wave_sum(sg);
                if (lane == 0) {
                    if (P.adj_dsched) *P.adj_dsched = P.adj_coeff * sw;
                    if (P.adj_dg) *P.adj_dg += P.dt * sg;
                    __hip_atomic_store(P.adj_done, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    }
}

// Scan steps: most plans need at most 3 (a carry reaches Q 8 points); the
// variant for up to 6 reserves registers for the longer scans.
template <typename R, int MODE, int FLAGS, int Q>
static void launch_q(const SweepParams &P, const void *tab, hipStream_t s)
{
    using V = typename CT<R>::V;
    const int64_t per_group = (int64_t)kXWaves * P.xlpw;
    const unsigned grid = (unsigned)((P.nlines + per_group - 1) / per_group);
    if (P.scan_steps <= 3)
        hipLaunchKernelGGL((k_sweep_x_scan<R, MODE, FLAGS, Q, 3>), dim3(grid), dim3(kLanes * kXWaves), 0, s, P,
                           (const V *)P.psi, (V *)P.out, (const V *)tab, (const V *)P.state);
    else
        hipLaunchKernelGGL((k_sweep_x_scan<R, MODE, FLAGS, Q, 6>), dim3(grid), dim3(kLanes * kXWaves), 0, s, P,
                           (const V *)P.psi, (V *)P.out, (const V *)tab, (const V *)P.state);
}

template <typename R, int MODE, int FLAGS>
static hipError_t launch_x_flags(const SweepParams &P, int Q, const void *tab, hipStream_t s)
{
    switch (Q) {
    case 1: launch_q<R, MODE, FLAGS, 1>(P, tab, s); break;
    case 2: launch_q<R, MODE, FLAGS, 2>(P, tab, s); break;
    case 4: launch_q<R, MODE, FLAGS, 4>(P, tab, s); break;
    case 8: launch_q<R, MODE, FLAGS, 8>(P, tab, s); break;
    case 16: launch_q<R, MODE, FLAGS, 16>(P, tab, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R, int MODE>
static hipError_t launch_x_mode(const SweepParams &P, int flags, int Q, const void *tab, hipStream_t s)
{
    if (MODE == GP_IMAG) {
        switch (flags) {
        case 0: return launch_x_flags<R, MODE, 0>(P, Q, tab, s);
        case F_FUSE_N: return launch_x_flags<R, MODE, F_FUSE_N>(P, Q, tab, s);
        case F_FUSE_N | F_RENORM: return launch_x_flags<R, MODE, F_FUSE_N | F_RENORM>(P, Q, tab, s);
        case F_NORM_OUT: return launch_x_flags<R, MODE, F_NORM_OUT>(P, Q, tab, s);
        case F_FUSE_N | F_NORM_OUT: return launch_x_flags<R, MODE, F_FUSE_N | F_NORM_OUT>(P, Q, tab, s);
        case F_FUSE_N | F_RENORM | F_NORM_OUT:
            return launch_x_flags<R, MODE, F_FUSE_N | F_RENORM | F_NORM_OUT>(P, Q, tab, s);
        default: return hipErrorInvalidValue;
        }
    }
    switch (flags) {
    case 0: return launch_x_flags<R, MODE, 0>(P, Q, tab, s);
    case F_FUSE_N: return launch_x_flags<R, MODE, F_FUSE_N>(P, Q, tab, s);
    case F_FUSE_N | F_COPY_IN: return launch_x_flags<R, MODE, F_FUSE_N | F_COPY_IN>(P, Q, tab, s);
    case F_ADJ_N: return launch_x_flags<R, MODE, F_ADJ_N>(P, Q, tab, s);
    default: return hipErrorInvalidValue;
    }
}

// Strided axis with the scan solver: workgroup b's wavefront w takes lines
// b 4 lpw + w + 4 li (li < lpw), so its four wavefronts work on neighbouring
// lines at every moment; one FP64 norm partial per workgroup (F_NORM_OUT).
template <typename R, int MODE, int FLAGS, int Q, int SMAX>
__global__ __launch_bounds__(kLanes *kXWaves) void k_sweep_col_scan(SweepParams P, const typename CT<R>::V *src,
                                                                     typename CT<R>::V *dst,
                                                                     const typename CT<R>::V *__restrict__ tab)
{
    using V = typename CT<R>::V;
    const int lane = threadIdx.x & (kLanes - 1);
    const int wave = threadIdx.x / kLanes;
    double nacc = 0.0;
    const int64_t first = (int64_t)blockIdx.x * kXWaves * P.xlpw + wave;
    if constexpr (Q >= kXLdsQ) {
        __shared__ V kc[3 * Q * kLanes];
        x_rows_to_lds<R, Q>(P, tab, kc);
        __syncthreads();
        col_scan_wave<R, MODE, FLAGS, Q, SMAX, true>(P, src, dst, tab, first, P.xlpw, kXWaves, nacc, kc);
    } else {
        col_scan_wave<R, MODE, FLAGS, Q, SMAX>(P, src, dst, tab, first, P.xlpw, kXWaves, nacc);
    }
    if (FLAGS & F_NORM_OUT) {
        __shared__ double red[kXWaves];
        nacc = wave_sum(nacc);
        if (lane == 0) red[wave] = nacc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = 0.0;
            for (int w = 0; w < kXWaves; ++w) a += red[w];
            P.norm_out[blockIdx.x] = a;
        }
    }
}

template <typename R, int MODE, int FLAGS, int Q>
static void launch_col_q(const SweepParams &P, const void *tab, hipStream_t s)
{
    using V = typename CT<R>::V;
    const int64_t per_group = (int64_t)kXWaves * P.xlpw;
    const unsigned grid = (unsigned)((P.nlines + per_group - 1) / per_group);
    if (P.scan_steps <= 3)
        hipLaunchKernelGGL((k_sweep_col_scan<R, MODE, FLAGS, Q, 3>), dim3(grid), dim3(kLanes * kXWaves), 0, s, P,
                           (const V *)P.psi, (V *)P.out, (const V *)tab);
    else
        hipLaunchKernelGGL((k_sweep_col_scan<R, MODE, FLAGS, Q, 6>), dim3(grid), dim3(kLanes * kXWaves), 0, s, P,
                           (const V *)P.psi, (V *)P.out, (const V *)tab);
}

template <typename R, int MODE, int FLAGS>
static hipError_t launch_col_flags(const SweepParams &P, int Q, const void *tab, hipStream_t s)
{
    switch (Q) {
    case 1: launch_col_q<R, MODE, FLAGS, 1>(P, tab, s); break;
    case 2: launch_col_q<R, MODE, FLAGS, 2>(P, tab, s); break;
    case 4: launch_col_q<R, MODE, FLAGS, 4>(P, tab, s); break;
    case 8: launch_col_q<R, MODE, FLAGS, 8>(P, tab, s); break;
    case 16: launch_col_q<R, MODE, FLAGS, 16>(P, tab, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R, int MODE>
static hipError_t launch_col_mode(const SweepParams &P, int flags, int Q, const void *tab, hipStream_t s)
{
    switch (flags) {
    case 0: return launch_col_flags<R, MODE, 0>(P, Q, tab, s);
    case F_NORM_OUT: return launch_col_flags<R, MODE, F_NORM_OUT>(P, Q, tab, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_col_scan(const gp_plan *p, int axis, const SweepParams &P, int flags, const void *tab,
                           hipStream_t s)
{
    const int Q = p->ax[axis].xq;
    if (p->prec == GP_C128)
        return p->mode == GP_IMAG ? launch_col_mode<double, GP_IMAG>(P, flags, Q, tab, s)
                                  : launch_col_mode<double, GP_REAL>(P, flags, Q, tab, s);
    return p->mode == GP_IMAG ? launch_col_mode<float, GP_IMAG>(P, flags, Q, tab, s)
                              : launch_col_mode<float, GP_REAL>(P, flags, Q, tab, s);
}

// A 1D run in one launch.  A 1D grid is one line, solved by one wavefront, so
// consecutive steps need no ordering across workgroups: the wavefront runs them
// in turn, each exactly as the x sweep kernel would (the same routine and
// flags: potential substep on load, deferred renormalisation in imaginary
// time), and keeps the imaginary-time norm total in LDS, where the separate
// launches pass it through the norm kernel.  The total is the same sum as the
// separate kernels form (their extra terms are zeros), so the results are too.
// Each lane reloads only the points it stored itself.  *total_out receives the
// last step's norm total (the scale applied after the call).
template <typename R, int MODE, int Q, int SMAX>
__global__ __launch_bounds__(kLanes) void k_steps_1d(SweepParams P, typename CT<R>::V *psi,
                                                     const typename CT<R>::V *__restrict__ tab, int64_t nsteps,
                                                     double *total_out)
{
    using V = typename CT<R>::V;
    constexpr bool kImag = MODE == GP_IMAG;
    constexpr int kFlags = F_FUSE_N | (kImag ? F_NORM_OUT : 0);
    const int lane = threadIdx.x & (kLanes - 1);
    __shared__ V xl[kLanes * (Q + 1)];
    __shared__ double tot;
    SweepParams Pr = P;  // renormalising steps read the previous step's total from LDS
    Pr.norm_total = &tot;
    for (int64_t k = 0; k < nsteps; ++k) {
        double nacc = 0.0, acc_w = 0.0, acc_g = 0.0;
        if (kImag && k > 0)
            x_scan_wave<R, MODE, kFlags | F_RENORM, Q, SMAX>(Pr, psi, psi, tab, nullptr, 0, 1, nacc, acc_w, acc_g, xl);
        else
            x_scan_wave<R, MODE, kFlags, Q, SMAX>(P, psi, psi, tab, nullptr, 0, 1, nacc, acc_w, acc_g, xl);
        if constexpr (kImag) {
            nacc = wave_sum(nacc);
            __syncthreads();  // every lane has read the previous total
            if (lane == 0) tot = nacc;
            __syncthreads();
        }
    }
    if (kImag && lane == 0 && nsteps > 0) *total_out = tot;
}

template <typename R, int MODE, int Q>
static hipError_t launch_steps_1d_q(const SweepParams &P, void *psi, int64_t nsteps, double *total_out,
                                    hipStream_t s)
{
    using V = typename CT<R>::V;
    if (P.scan_steps <= 3)
        hipLaunchKernelGGL((k_steps_1d<R, MODE, Q, 3>), dim3(1), dim3(kLanes), 0, s, P, (V *)psi, (const V *)P.tab,
                           nsteps, total_out);
    else
        hipLaunchKernelGGL((k_steps_1d<R, MODE, Q, 6>), dim3(1), dim3(kLanes), 0, s, P, (V *)psi, (const V *)P.tab,
                           nsteps, total_out);
    return hipGetLastError();
}

template <typename R, int MODE>
static hipError_t launch_steps_1d_mode(const SweepParams &P, int Q, void *psi, int64_t nsteps, double *total_out,
                                       hipStream_t s)
{
    switch (Q) {
    case 1: return launch_steps_1d_q<R, MODE, 1>(P, psi, nsteps, total_out, s);
    case 2: return launch_steps_1d_q<R, MODE, 2>(P, psi, nsteps, total_out, s);
    case 4: return launch_steps_1d_q<R, MODE, 4>(P, psi, nsteps, total_out, s);
    case 8: return launch_steps_1d_q<R, MODE, 8>(P, psi, nsteps, total_out, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_steps_1d(const gp_plan *p, void *psi, int64_t nsteps, double *total_out, hipStream_t s)
{
    const SweepParams P = make_sweep_params(p, 0, psi, psi, false, p->step, nullptr);
    const int Q = p->ax[0].xq;
    if (p->prec == GP_C128)
        return p->mode == GP_IMAG ? launch_steps_1d_mode<double, GP_IMAG>(P, Q, psi, nsteps, total_out, s)
                                  : launch_steps_1d_mode<double, GP_REAL>(P, Q, psi, nsteps, total_out, s);
    return p->mode == GP_IMAG ? launch_steps_1d_mode<float, GP_IMAG>(P, Q, psi, nsteps, total_out, s)
                              : launch_steps_1d_mode<float, GP_REAL>(P, Q, psi, nsteps, total_out, s);
}

hipError_t launch_x_scan(const gp_plan *p, const SweepParams &P, int flags, const void *tab, hipStream_t s)
{
    const int Q = p->ax[0].xq;
    if (p->prec == GP_C128)
        return p->mode == GP_IMAG ? launch_x_mode<double, GP_IMAG>(P, flags, Q, tab, s)
                                  : launch_x_mode<double, GP_REAL>(P, flags, Q, tab, s);
    return p->mode == GP_IMAG ? launch_x_mode<float, GP_IMAG>(P, flags, Q, tab, s)
                              : launch_x_mode<float, GP_REAL>(P, flags, Q, tab, s);
}

}  // namespace gp

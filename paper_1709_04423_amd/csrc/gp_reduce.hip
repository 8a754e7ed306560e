// Reductions and pointwise passes: final imaginary-time renormalisation,
// observables (FP64 accumulation, deterministic fixed-order block sums),
// the per-step reduction of the adjoint's gradient partials, and a plain copy
// kernel used to calibrate bandwidth and memory counters.
#include "gp_internal.h"

namespace gp {

namespace {

template <typename R> struct VT;
template <> struct VT<double> {
    using V = double2;
};
template <> struct VT<float> {
    using V = float2;
};

__device__ __forceinline__ double wsum(double v)
{
    for (int off = kLanes / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kLanes);
    return v;
}


template <typename R>
__global__ __launch_bounds__(256) void k_scale(typename VT<R>::V *__restrict__ psi, int64_t npts,
                                               const double *__restrict__ total, double dV)
{
    const double s = 1.0 / sqrt(dV * total[0]);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts;
         i += (int64_t)gridDim.x * blockDim.x) {
        typename VT<R>::V v = psi[i];
        v.x = R((double)v.x * s);
        v.y = R((double)v.y * s);
        psi[i] = v;
    }
}

// Sum of the per-workgroup norm partials of one step in a fixed order.
__global__ __launch_bounds__(256) void k_norm_final(const double *__restrict__ part, int64_t np,
                                                    double *__restrict__ total)
{
    __shared__ double lds[256 / kLanes];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < np; i += blockDim.x) acc += part[i];
    acc = wsum(acc);
    const int lane = threadIdx.x & (kLanes - 1), wave = threadIdx.x / kLanes;
    if (lane == 0) lds[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < 256 / kLanes; ++w) s += lds[w];
        total[0] = s;
    }
}

struct ObsParams {
    int64_t nx, ny, nz;
    int ndim;
    double x0[3], dx[3], hw2[3];
};

__device__ __forceinline__ double abs2d(double re, double im) { return re * re + im * im; }

// Fixed-order reduction of kObsFields values over a 256-thread block.
__device__ void block_reduce_fields(double *acc, double *out)
{
    __shared__ double lds[256 / kLanes][kObsFields];
    const int lane = threadIdx.x & (kLanes - 1), wave = threadIdx.x / kLanes;
    for (int f = 0; f < kObsFields; ++f) {
        double v = wsum(acc[f]);
        if (lane == 0) lds[wave][f] = v;
    }
    __syncthreads();
    if (threadIdx.x < kObsFields) {
        double s = 0.0;
        for (int w = 0; w < 256 / kLanes; ++w) s += lds[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// One thread per (i, j) column, marching along z.  Fields:
// 0 sum|u|^2, 1 sum V|u|^2, 2 sum|u|^4, 3-5 sum x_a^2|u|^2, 6-8 kinetic sums per axis.
template <typename R>
__global__ __launch_bounds__(256) void k_observables(const typename VT<R>::V *__restrict__ psi,
                                                     ObsParams O, double *__restrict__ part)
{
    double acc[kObsFields];
    for (int f = 0; f < kObsFields; ++f) acc[f] = 0.0;
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col < O.nx * O.ny) {
        const int64_t i = col % O.nx, j = col / O.nx;
        const double x = ((double)i + O.x0[0]) * O.dx[0];
        const double y = ((double)j + O.x0[1]) * O.dx[1];
        const int64_t plane = O.nx * O.ny;
        double pr = 0.0, pi = 0.0;  // previous value along z (ghost 0 before k = 0)
        for (int64_t k = 0; k < O.nz; ++k) {
            const double z = ((double)k + O.x0[2]) * O.dx[2];
            const int64_t at = col + k * plane;
            const typename VT<R>::V u = psi[at];
            const double ur = u.x, ui = u.y;
            const double d = abs2d(ur, ui);
            acc[0] += d;
            acc[1] += (O.hw2[0] * x * x + O.hw2[1] * y * y + O.hw2[2] * z * z) * d;
            acc[2] += d * d;
            acc[3] += x * x * d;
            acc[4] += y * y * d;
            acc[5] += z * z * d;
            // x: |u_{i+1} - u_i|^2 with u_nx = 0, plus |u_0|^2 for the i = -1 term
            {
                double nr = 0.0, ni = 0.0;
                if (i + 1 < O.nx) {
                    const typename VT<R>::V w = psi[at + 1];
                    nr = w.x;
                    ni = w.y;
                }
                acc[6] += abs2d(nr - ur, ni - ui) + (i == 0 ? d : 0.0);
            }
            if (O.ndim >= 2) {
                double nr = 0.0, ni = 0.0;
                if (j + 1 < O.ny) {
                    const typename VT<R>::V w = psi[at + O.nx];
                    nr = w.x;
                    ni = w.y;
                }
                acc[7] += abs2d(nr - ur, ni - ui) + (j == 0 ? d : 0.0);
            }
            if (O.ndim >= 3) acc[8] += abs2d(ur - pr, ui - pi);
            pr = ur;
            pi = ui;
        }
        if (O.ndim >= 3) acc[8] += abs2d(pr, pi);
    }
    __shared__ double out[kObsFields];
    block_reduce_fields(acc, out);
    __syncthreads();
    if (threadIdx.x < kObsFields) part[(int64_t)blockIdx.x * kObsFields + threadIdx.x] = out[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_obs_final(const double *__restrict__ part, int64_t nblocks,
                                                   double *__restrict__ out)
{
    double acc[kObsFields];
    for (int f = 0; f < kObsFields; ++f) {
        double s = 0.0;
        for (int64_t b = threadIdx.x; b < nblocks; b += blockDim.x) s += part[b * kObsFields + f];
        acc[f] = s;
    }
    __shared__ double res[kObsFields];
    block_reduce_fields(acc, res);
    __syncthreads();
    if (threadIdx.x < kObsFields) out[threadIdx.x] = res[threadIdx.x];
}

// dsched[k] = dt * omega_s(n) * sum w x_s^2 ;  dg += dt * sum w |u|^2
__global__ __launch_bounds__(64) void k_adj_reduce(const double *__restrict__ part, int np, double coeff,
                                                   double dt, double *dsched_k, double *dg)
{
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < np; i += kLanes) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    a = wsum(a);
    b = wsum(b);
    if (threadIdx.x == 0) {
        if (dsched_k) *dsched_k = coeff * a;
        if (dg) *dg += dt * b;
    }
}

__global__ __launch_bounds__(256) void k_copy(double2 *__restrict__ dst, const double2 *__restrict__ src,
                                              int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace

int64_t obs_groups(const gp_plan *p)
{
    const int64_t cols = p->n[0] * (p->ndim >= 2 ? p->n[1] : 1);
    return (cols + kObsThreads - 1) / kObsThreads;
}

hipError_t launch_scale(gp_plan *p, void *psi, hipStream_t s)
{
    const double *total = norm_total(p, p->step - 1);  // written after the last step's final sweep
    int64_t grid = (p->npts + 255) / 256;
    if (grid > 4096) grid = 4096;
    timing_begin(p, K_SCALE, s);
    if (p->prec == GP_C128)
        hipLaunchKernelGGL(k_scale<double>, dim3((unsigned)grid), dim3(256), 0, s, (double2 *)psi, p->npts, total,
                           p->dV);
    else
        hipLaunchKernelGGL(k_scale<float>, dim3((unsigned)grid), dim3(256), 0, s, (float2 *)psi, p->npts, total,
                           p->dV);
    timing_end(p, s);
    return hipGetLastError();
}

hipError_t launch_norm_final(gp_plan *p, int64_t step_index, hipStream_t s)
{
    timing_begin(p, K_NORM_FINAL, s);
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(256), 0, s, norm_partials(p, step_index),
                       sweep_groups(p, p->ndim - 1), norm_total(p, step_index));
    timing_end(p, s);
    return hipGetLastError();
}

hipError_t launch_observables(gp_plan *p, const void *psi, hipStream_t s)
{
    ObsParams O{};
    O.nx = p->n[0];
    O.ny = p->ndim >= 2 ? p->n[1] : 1;
    O.nz = p->ndim >= 3 ? p->n[2] : 1;
    O.ndim = p->ndim;
    for (int a = 0; a < 3; ++a) {
        O.x0[a] = a < p->ndim ? coord0(p->n[a]) : 0.0;
        O.dx[a] = a < p->ndim ? p->dx[a] : 0.0;
        O.hw2[a] = a < p->ndim ? 0.5 * p->omega[a] * p->omega[a] : 0.0;
    }
    const int64_t nb = obs_groups(p);
    timing_begin(p, K_OBS, s);
    if (p->prec == GP_C128)
        hipLaunchKernelGGL(k_observables<double>, dim3((unsigned)nb), dim3(kObsThreads), 0, s,
                           (const double2 *)psi, O, p->d_obs);
    else
        hipLaunchKernelGGL(k_observables<float>, dim3((unsigned)nb), dim3(kObsThreads), 0, s,
                           (const float2 *)psi, O, p->d_obs);
    timing_end(p, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    timing_begin(p, K_OBS_FINAL, s);
    hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(256), 0, s, p->d_obs, nb, p->d_obs + nb * kObsFields);
    timing_end(p, s);
    return hipGetLastError();
}

hipError_t launch_adj_reduce(gp_plan *p, int64_t nparts, double coeff, double *dsched_k, double *dg,
                             hipStream_t s)
{
    timing_begin(p, K_ADJ_REDUCE, s);
    hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(64), 0, s, p->d_adj, (int)nparts, coeff, p->dt,
                       dsched_k, dg);
    timing_end(p, s);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, int64_t bytes, hipStream_t s)
{
    const int64_t n = bytes / 16;
    int64_t grid = (n + 255) / 256;
    if (grid > 65536) grid = 65536;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)grid), dim3(256), 0, s, (double2 *)dst, (const double2 *)src, n);
    return hipGetLastError();
}

}  // namespace gp

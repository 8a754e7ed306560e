// Reductions and pointwise passes: final imaginary-time renormalisation,
// observables (FP64 accumulation, deterministic fixed-order block sums),
// the per-step reduction of the adjoint's gradient partials, and a plain copy
// kernel used to calibrate bandwidth and memory counters.
#include <cmath>
#include <mutex>
#include <string>

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

// Sum of the per-workgroup norm partials of one step in a fixed order.  Each
// thread adds its partials i = t, t + 256, ... in that order; they are loaded
// eight at a time before the adds (a missing one as +0, which leaves the
// non-negative sum unchanged), so the loads overlap instead of each one waiting
// for the last: the same sums, bit for bit.
__global__ __launch_bounds__(256) void k_norm_final(const double *__restrict__ part, int64_t np,
                                                    double *__restrict__ total)
{
    __shared__ double lds[256 / kLanes];
    constexpr int kBatch = 8;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < np; i += kBatch * (int64_t)blockDim.x) {
        double v[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int64_t j = i + k * (int64_t)blockDim.x;
            v[k] = j < np ? part[j] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) acc += v[k];
    }
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
    int64_t cx, cy, cz;  // tiles along x (64 columns), y (kObsTileRows rows), z (zc planes)
    int64_t zc;
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

constexpr int kObsRows = 4;                       // rows per wavefront
constexpr int kObsTileRows = kObsRows * (kObsThreads / kLanes);  // rows per workgroup

// Observables of one tile: 64 columns (one per lane) by kObsTileRows rows (the
// workgroup's wavefronts stacked along y), marching through zc planes.  The
// kinetic sums use backward differences: point p adds |u_p - u_{p-1}|^2 along
// each axis (u_{-1} = 0) and the last point of a line also adds |u_{N-1}|^2 --
// the same terms as the forward differences over i = -1..N-1.  The previous
// value along z stays in registers and the one along x comes from the next
// lower lane, so each point is read once; only the tile's edges (the column
// left of it, the row below it, the plane before it) are read again.
// Fields: 0 sum|u|^2, 1 sum V|u|^2, 2 sum|u|^4, 3-5 sum x_a^2|u|^2, 6-8 kinetic sums per axis.
template <typename R>
__global__ __launch_bounds__(kObsThreads) void k_observables(const typename VT<R>::V *__restrict__ psi,
                                                             ObsParams O, double *__restrict__ part)
{
    using V = typename VT<R>::V;
    const int lane = threadIdx.x & (kLanes - 1), w = threadIdx.x / kLanes;
    int64_t b = blockIdx.x;
    const int64_t bx = b % O.cx;
    b /= O.cx;
    const int64_t by = b % O.cy, bz = b / O.cy;
    const int64_t i = bx * kLanes + lane;
    const int64_t j0 = by * kObsTileRows + (int64_t)w * kObsRows;
    const int64_t k0 = bz * O.zc, k1 = min(k0 + O.zc, O.nz);
    const int64_t plane = O.nx * O.ny;
    const bool xin = i < O.nx;
    const double x = ((double)i + O.x0[0]) * O.dx[0];
    double acc[kObsFields];
    for (int f = 0; f < kObsFields; ++f) acc[f] = 0.0;
    auto ld = [&](int64_t ii, int64_t jj, int64_t kk, bool ok) -> V {
        V v;
        v.x = R(0);
        v.y = R(0);
        if (ok) v = psi[ii + O.nx * jj + plane * kk];
        return v;
    };
    V zprev[kObsRows];
#pragma unroll
    for (int r = 0; r < kObsRows; ++r) zprev[r] = ld(i, j0 + r, k0 - 1, xin && k0 > 0 && j0 + r < O.ny);
    for (int64_t k = k0; k < k1; ++k) {
        const double z = ((double)k + O.x0[2]) * O.dx[2];
        V u[kObsRows], left[kObsRows];
#pragma unroll
        for (int r = 0; r < kObsRows; ++r) u[r] = ld(i, j0 + r, k, xin && j0 + r < O.ny);
        V below = ld(i, j0 - 1, k, xin && j0 >= 1 && j0 - 1 < O.ny);
#pragma unroll
        for (int r = 0; r < kObsRows; ++r) {
            left[r].x = __shfl_up(u[r].x, 1, kLanes);
            left[r].y = __shfl_up(u[r].y, 1, kLanes);
            if (lane == 0) left[r] = ld(i - 1, j0 + r, k, xin && i >= 1 && j0 + r < O.ny);
        }
#pragma unroll
        for (int r = 0; r < kObsRows; ++r) {
            const int64_t j = j0 + r;
            if (xin && j < O.ny) {
                const double y = ((double)j + O.x0[1]) * O.dx[1];
                const double ur = u[r].x, ui = u[r].y;
                const double d = abs2d(ur, ui);
                acc[0] += d;
                acc[1] += (O.hw2[0] * x * x + O.hw2[1] * y * y + O.hw2[2] * z * z) * d;
                acc[2] += d * d;
                acc[3] += x * x * d;
                acc[4] += y * y * d;
                acc[5] += z * z * d;
                acc[6] += abs2d(ur - (double)left[r].x, ui - (double)left[r].y) + (i == O.nx - 1 ? d : 0.0);
                if (O.ndim >= 2) {
                    const V pv = r == 0 ? below : u[r - 1];
                    acc[7] += abs2d(ur - (double)pv.x, ui - (double)pv.y) + (j == O.ny - 1 ? d : 0.0);
                }
                if (O.ndim >= 3)
                    acc[8] += abs2d(ur - (double)zprev[r].x, ui - (double)zprev[r].y) + (k == O.nz - 1 ? d : 0.0);
            }
            zprev[r] = u[r];
        }
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

// Tiling of the observables kernel: 64-column by kObsTileRows-row tiles, and the
// z extent split into chunks of at least 8 planes until about 1024 workgroups run.
static void obs_tiling(int ndim, const int64_t *n, int64_t &cx, int64_t &cy, int64_t &cz, int64_t &zc)
{
    const int64_t nx = n[0], ny = ndim >= 2 ? n[1] : 1, nz = ndim >= 3 ? n[2] : 1;
    cx = (nx + kLanes - 1) / kLanes;
    cy = (ny + kObsTileRows - 1) / kObsTileRows;
    const int64_t base = cx * cy;
    int64_t want = (1024 + base - 1) / base;
    const int64_t most = (nz + 7) / 8;
    if (want > most) want = most;
    if (want < 1) want = 1;
    zc = (nz + want - 1) / want;
    cz = (nz + zc - 1) / zc;
}

int64_t obs_groups_of(int ndim, const int64_t *n)
{
    int64_t cx, cy, cz, zc;
    obs_tiling(ndim, n, cx, cy, cz, zc);
    return cx * cy * cz;
}

int64_t obs_groups(const gp_plan *p) { return obs_groups_of(p->ndim, p->n); }

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
    const int64_t np = p->geom == GP_AXIAL ? radial_norm_groups(p) : sweep_groups(p, p->ndim - 1);
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(256), 0, s, norm_partials(p, step_index), np,
                       norm_total(p, step_index));
    timing_end(p, s);
    return hipGetLastError();
}

// The observables kernels of a grid into `part` (nb = obs_groups_of partial rows
// of kObsFields, then the final sums in row nb).  Shared by the plan's entry
// point and the plan-free one.
static hipError_t launch_obs_kernels(int ndim, const int64_t *n, const double *dx, const double *omega, gp_prec prec,
                                     const void *psi, double *part, gp_plan *timed, hipStream_t s)
{
    ObsParams O{};
    O.nx = n[0];
    O.ny = ndim >= 2 ? n[1] : 1;
    O.nz = ndim >= 3 ? n[2] : 1;
    O.ndim = ndim;
    obs_tiling(ndim, n, O.cx, O.cy, O.cz, O.zc);
    for (int a = 0; a < 3; ++a) {
        O.x0[a] = a < ndim ? coord0(n[a]) : 0.0;
        O.dx[a] = a < ndim ? dx[a] : 0.0;
        O.hw2[a] = a < ndim ? 0.5 * omega[a] * omega[a] : 0.0;
    }
    const int64_t nb = obs_groups_of(ndim, n);
    if (timed) timing_begin(timed, K_OBS, s);
    if (prec == GP_C128)
        hipLaunchKernelGGL(k_observables<double>, dim3((unsigned)nb), dim3(kObsThreads), 0, s,
                           (const double2 *)psi, O, part);
    else
        hipLaunchKernelGGL(k_observables<float>, dim3((unsigned)nb), dim3(kObsThreads), 0, s,
                           (const float2 *)psi, O, part);
    if (timed) timing_end(timed, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (timed) timing_begin(timed, K_OBS_FINAL, s);
    hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(256), 0, s, part, nb, part + nb * kObsFields);
    if (timed) timing_end(timed, s);
    return hipGetLastError();
}

hipError_t launch_obs_final(gp_plan *p, double *part, int64_t nb, hipStream_t s)
{
    timing_begin(p, K_OBS_FINAL, s);
    hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(256), 0, s, part, nb, part + nb * kObsFields);
    timing_end(p, s);
    return hipGetLastError();
}

hipError_t launch_observables(gp_plan *p, const void *psi, hipStream_t s)
{
    // the trap of the last step taken (a schedule may change it), or of step 0 before any step
    double w[3];
    omega_at_step(p, p->step > 0 ? p->step - 1 : 0, w);
    return launch_obs_kernels(p->ndim, p->n, p->dx, w, p->prec, psi, p->d_obs, p, s);
}

void obs_from_sums(const double *f, int ndim, const double *dx, double g, gp_obs *out)
{
    double dv = 1.0;
    for (int a = 0; a < ndim; ++a) dv *= dx[a];
    out->norm = dv * f[0];
    out->epot = dv * f[1];
    out->eint = 0.5 * g * dv * f[2];
    out->ekin = 0.0;
    for (int a = 0; a < ndim; ++a) out->ekin += 0.5 * dv * f[6 + a] / (dx[a] * dx[a]);
    out->energy = out->ekin + out->epot + out->eint;
    out->mu = out->ekin + out->epot + 2.0 * out->eint;
    for (int a = 0; a < 3; ++a) out->rms[a] = a < ndim ? std::sqrt(dv * f[3 + a] / out->norm) : 0.0;
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

// ------------------------------------------------------------ observables without allocation

namespace gp {

namespace {

// Partial sums of gp_observables_noalloc: GP_OBS_NOALLOC_MAX_GROUPS rows of
// kObsFields FP64 values and the row of final sums, in a static device array
// (one copy on every device the library runs on, held until the process ends).
constexpr int64_t kObsScratchGroups = GP_OBS_NOALLOC_MAX_GROUPS;
__device__ __align__(256) double scratch[(kObsScratchGroups + 1) * kObsFields];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch` per device (host copy of the symbol is not it)

// The array's device address on the current device, looked up once per device.
gp_status scratch_address(int dev, double **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        double *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(observables scratch)");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return GP_OK;
}

}  // namespace

}  // namespace gp

extern "C" gp_status gp_observables_noalloc(int ndim, const int64_t *n, const double *dx, const double *omega,
                                            double g, gp_prec prec, const void *psi, gp_obs *out, void *stream)
{
    using namespace gp;
    if (ndim < 1 || ndim > 3 || !n || !dx || !psi || !out) return set_error("bad argument"), GP_EINVAL;
    if (prec != GP_C128 && prec != GP_C64) return set_error("bad precision"), GP_EINVAL;
    if (!std::isfinite(g)) return set_error("g must be finite"), GP_EINVAL;
    double w[3] = {0.0, 0.0, 0.0};
    int64_t npts = 1;
    for (int a = 0; a < ndim; ++a) {
        if (n[a] < 1 || n[a] > ((int64_t)1 << 31) || npts > ((int64_t)1 << 40) / n[a])
            return set_error("grid size must be 1..2^31 per axis and 2^40 in all"), GP_EINVAL;
        if (!(dx[a] > 0.0) || !std::isfinite(dx[a])) return set_error("dx must be finite and > 0"), GP_EINVAL;
        if (omega) {
            if (!std::isfinite(omega[a])) return set_error("omega must be finite"), GP_EINVAL;
            w[a] = omega[a];
        }
        npts *= n[a];
    }
    const int64_t nb = obs_groups_of(ndim, n);
    if (nb > kObsScratchGroups)
        return set_error("grid too large for the static observables scratch (ceil(nx/64) ceil(ny/16) > " +
                         std::to_string(kObsScratchGroups) + ")"),
               GP_EUNSUPPORTED;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return set_error("device index beyond the scratch table"), GP_EUNSUPPORTED;
    double *part = nullptr;
    gp_status st = scratch_address(dev, &part);
    if (st != GP_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    e = launch_obs_kernels(ndim, n, dx, w, prec, psi, part, nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "observables launch");
    double f[kObsFields];
    e = hipMemcpyAsync(f, part + nb * kObsFields, sizeof(f), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(observables)");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    obs_from_sums(f, ndim, dx, g, out);
    if (!std::isfinite(out->norm) || !std::isfinite(out->energy)) {
        set_error("non-finite norm or energy");
        return GP_ENONFINITE;
    }
    return GP_OK;
}


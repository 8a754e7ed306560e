// Density outputs of the paper's programs ("Summary of revisions": the
// condensate density, reduced -- integrated -- 1d and 2d densities, and in real
// time the rms sizes as the dynamics evolves after a perturbation), computed on
// the device next to the step's output.
//
//  - gp_density: |psi|^2 at every point (FP64).
//  - gp_density_reduced: |psi|^2 integrated over the axes not kept, one axis at a
//    time, slowest first.  Integrating x (contiguous) is one wavefront per row
//    (lane-strided partial sums, then a fixed butterfly); integrating a strided
//    axis is one thread per output value summing along the axis in index order,
//    with loads coalesced across the threads.  Every sum has a fixed order, so
//    results are reproducible bit for bit.  An intermediate (after the first of
//    two integrations) goes to the plan's work grid.
//  - gp_step_series: gp_step in blocks of `every` steps with the observables of
//    the state before the first block and after each block written, as FP64
//    records, to a device buffer: no host synchronisation.
#include <cmath>

#include "gp_internal.h"
#include "gp_sweep_common.h"

namespace gp {

namespace {

template <typename T> struct Abs2;
template <> struct Abs2<double2> {
    __device__ static double of(double2 v) { return v.x * v.x + v.y * v.y; }
};
template <> struct Abs2<float2> {
    __device__ static double of(float2 v) { return (double)v.x * (double)v.x + (double)v.y * (double)v.y; }
};
template <> struct Abs2<double> {
    __device__ static double of(double v) { return v; }  // already a density
};

template <typename T>
__global__ __launch_bounds__(256) void k_density(const T *__restrict__ psi, int64_t npts, double *__restrict__ out)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += (int64_t)gridDim.x * blockDim.x)
        out[p] = Abs2<T>::of(psi[p]);
}

// out[r] = scale * sum_i wt_i |in[r len + i]|^2, one wavefront per row; wt_i is
// the radial cell weight (i + 1/2) dr when radial_dr > 0, else 1.
template <typename T>
__global__ __launch_bounds__(256) void k_integrate_rows(const T *__restrict__ in, int64_t nrows, int64_t len,
                                                        double scale, double radial_dr, double *__restrict__ out)
{
    const int lane = threadIdx.x & (kLanes - 1);
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / kLanes) + threadIdx.x / kLanes;
    if (row >= nrows) return;  // whole wavefront
    double acc = 0.0;
    for (int64_t i = lane; i < len; i += kLanes) {
        const double d = Abs2<T>::of(in[row * len + i]);
        acc += radial_dr > 0.0 ? ((double)i + 0.5) * radial_dr * d : d;
    }
    acc = wave_sum(acc);
    if (lane == 0) out[row] = scale * acc;
}

// out[o inner + i] = scale * sum_k |in[(o len + k) inner + i]|^2, one thread per output.
template <typename T>
__global__ __launch_bounds__(256) void k_integrate_strided(const T *__restrict__ in, int64_t inner, int64_t len,
                                                           int64_t outer, double scale, double *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= inner * outer) return;
    const int64_t i = t % inner, o = t / inner;
    double acc = 0.0;
    for (int64_t k = 0; k < len; ++k) acc += Abs2<T>::of(in[(o * len + k) * inner + i]);
    out[t] = scale * acc;
}

// One axis integrated out of a (n0, n1, n2) array (x fastest).
template <typename T>
void integrate_axis(const T *in, const int64_t *dims, int axis, double scale, double radial_dr, double *out,
                    hipStream_t s)
{
    int64_t inner = 1, outer = 1;
    for (int b = 0; b < axis; ++b) inner *= dims[b];
    for (int b = axis + 1; b < 3; ++b) outer *= dims[b];
    const int64_t len = dims[axis];
    if (inner == 1) {
        const int64_t rows_per_block = 256 / kLanes;
        hipLaunchKernelGGL((k_integrate_rows<T>), dim3((unsigned)((outer + rows_per_block - 1) / rows_per_block)),
                           dim3(256), 0, s, in, outer, len, scale, radial_dr, out);
    } else {
        hipLaunchKernelGGL((k_integrate_strided<T>), dim3((unsigned)((inner * outer + 255) / 256)), dim3(256), 0, s,
                           in, inner, len, outer, scale, out);
    }
}

// Observables from the final sums, on the device, in the order of the host's
// formulas: record = step index, norm, mu, energy, ekin, epot, eint, rms[0..2].
struct ObsConv {
    int geom, ndim;
    double dx[3], g, measure;  // measure: prod dx (Cartesian) or the symmetric trap's m
};

__global__ void k_obs_record(const double *__restrict__ f, ObsConv c, int64_t step, double *__restrict__ rec)
{
    if (threadIdx.x != 0) return;
    double norm, epot, eint, ekin = 0.0, r[3] = {0.0, 0.0, 0.0};
    if (c.geom == GP_CARTESIAN) {
        double dv = 1.0;
        for (int a = 0; a < c.ndim; ++a) dv *= c.dx[a];
        norm = dv * f[0];
        epot = dv * f[1];
        eint = 0.5 * c.g * dv * f[2];
        for (int a = 0; a < c.ndim; ++a) ekin += 0.5 * dv * f[6 + a] / (c.dx[a] * c.dx[a]);
        for (int a = 0; a < c.ndim; ++a) r[a] = sqrt(dv * f[3 + a] / norm);
    } else {
        const double m = c.measure;
        norm = m * f[0];
        epot = m * f[1];
        eint = 0.5 * c.g * m * f[2];
        ekin = 0.5 * m * f[6] / (c.dx[0] * c.dx[0]);
        if (c.geom == GP_AXIAL) ekin += 0.5 * m * f[7] / (c.dx[1] * c.dx[1]);
        r[0] = sqrt(f[3] / f[0]);
        if (c.geom == GP_AXIAL) r[1] = sqrt(f[4] / f[0]);
    }
    rec[0] = (double)step;
    rec[1] = norm;
    rec[2] = ekin + epot + 2.0 * eint;
    rec[3] = ekin + epot + eint;
    rec[4] = ekin;
    rec[5] = epot;
    rec[6] = eint;
    rec[7] = r[0];
    rec[8] = r[1];
    rec[9] = r[2];
}

gp_status density_prologue(gp_plan *p, hipStream_t *s, void *stream)
{
    *s = (hipStream_t)stream;
    const hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    return GP_OK;
}

// Observables of psi into one series record (device).
hipError_t record_obs(gp_plan *p, const void *psi, double *rec, hipStream_t s)
{
    int64_t nb = p->n_obs_blocks;
    hipError_t e;
    if (p->geom != GP_CARTESIAN) {
        nb = radial_norm_groups(p);
        e = launch_radial_obs(p, psi, p->d_obs, nb, s);
        if (e == hipSuccess) e = launch_obs_final(p, p->d_obs, nb, s);
    } else {
        e = launch_observables(p, psi, s);
    }
    if (e != hipSuccess) return e;
    ObsConv c{};
    c.geom = p->geom;
    c.ndim = p->ndim;
    for (int a = 0; a < 3; ++a) c.dx[a] = a < p->ndim ? p->dx[a] : 0.0;
    c.g = p->g;
    c.measure = p->dV;
    hipLaunchKernelGGL(k_obs_record, dim3(1), dim3(64), 0, s, p->d_obs + nb * kObsFields, c, p->step, rec);
    return hipGetLastError();
}

}  // namespace

}  // namespace gp

using namespace gp;

extern "C" {

gp_status gp_density(gp_plan *p, const void *psi, double *out, void *stream)
{
    if (!p || !psi || !out) return set_error("NULL argument"), GP_EINVAL;
    hipStream_t s;
    gp_status st = density_prologue(p, &s, stream);
    if (st != GP_OK) return st;
    int64_t grid = (p->npts + 255) / 256;
    if (grid > 4096) grid = 4096;
    if (p->prec == GP_C128)
        hipLaunchKernelGGL(k_density<double2>, dim3((unsigned)grid), dim3(256), 0, s, (const double2 *)psi, p->npts,
                           out);
    else
        hipLaunchKernelGGL(k_density<float2>, dim3((unsigned)grid), dim3(256), 0, s, (const float2 *)psi, p->npts,
                           out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GP_OK : hip_fail(e, "density launch");
}

gp_status gp_density_reduced(gp_plan *p, const void *psi, int keep_mask, double *out, void *stream)
{
    if (!p || !psi || !out) return set_error("NULL argument"), GP_EINVAL;
    if (p->geom == GP_CIRCULAR || p->geom == GP_SPHERICAL)
        return set_error("a radial plan's density is already one-dimensional"), GP_EINVAL;
    const int all = (1 << p->ndim) - 1;
    if (keep_mask <= 0 || keep_mask >= all || (keep_mask & ~all))
        return set_error("keep_mask must keep at least one axis and integrate at least one"), GP_EINVAL;
    hipStream_t s;
    gp_status st = density_prologue(p, &s, stream);
    if (st != GP_OK) return st;
    const double pi = 3.14159265358979323846;
    int64_t dims[3] = {p->n[0], p->ndim >= 2 ? p->n[1] : 1, p->ndim >= 3 ? p->n[2] : 1};
    int todo[3], nt = 0;
    for (int a = p->ndim - 1; a >= 0; --a)  // slowest first
        if (!(keep_mask & (1 << a))) todo[nt++] = a;
    const void *in = psi;
    bool in_is_density = false;
    for (int t = 0; t < nt; ++t) {
        const int a = todo[t];
        double *dst = t + 1 < nt ? (double *)p->d_work : out;
        // integrating the radial axis of an axial plan carries its weights 2 pi r_i drho
        const bool rad = p->geom == GP_AXIAL && a == 0;
        const double scale = rad ? 2.0 * pi * p->dx[0] : p->dx[a];
        const double rdr = rad ? p->dx[0] : 0.0;
        if (in_is_density)
            integrate_axis<double>((const double *)in, dims, a, scale, rdr, dst, s);
        else if (p->prec == GP_C128)
            integrate_axis<double2>((const double2 *)in, dims, a, scale, rdr, dst, s);
        else
            integrate_axis<float2>((const float2 *)in, dims, a, scale, rdr, dst, s);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "reduced density launch");
        dims[a] = 1;
        in = dst;
        in_is_density = true;
    }
    return GP_OK;
}

gp_status gp_step_series(gp_plan *p, void *psi, int64_t nsteps, int64_t every, double *out, void *stream)
{
    if (!p || !psi || !out || nsteps < 0 || every < 1 || nsteps % every != 0)
        return set_error("bad argument (nsteps must be a non-negative multiple of every >= 1)"), GP_EINVAL;
    hipStream_t s;
    gp_status st = density_prologue(p, &s, stream);
    if (st != GP_OK) return st;
    hipError_t e = record_obs(p, psi, out, s);
    if (e != hipSuccess) return hip_fail(e, "series record launch");
    for (int64_t r = 1; r <= nsteps / every; ++r) {
        st = gp_step(p, psi, every, stream);
        if (st != GP_OK) return st;
        e = record_obs(p, psi, out + r * GP_SERIES_FIELDS, s);
        if (e != hipSuccess) return hip_fail(e, "series record launch");
    }
    return GP_OK;
}

}  // extern "C"

// Symmetric traps: the circularly symmetric 2D, spherically symmetric 3D and
// axially symmetric 3D problems of the paper's "Nature of problem", on the
// cell-centred radial grid r_i = (i + 1/2) dr.
//
// The radial Crank-Nicolson substep solves (W + k S) psi' = (W - k S) psi with
// W the cell weights and S the symmetric finite-volume stiffness (k = i dt/2 in
// real time, dt/2 in imaginary time; the coefficients vary along the line).
// One wavefront solves one radial line with Q = n/64 consecutive points per
// lane, as the Cartesian x solver does, but with every row's own coefficients:
//     forward   y_p = alpha_p y_{p-1} + m_p rhs_p,   alpha_p = -m_p l_p,
//     backward  u'_p = -c'_p u'_{p+1} + y_p,
//     rhs_p = beta_p u_p - (l_p u_{p-1} + l_{p+1} u_{p+1}),
// where l_p are the sub-diagonal entries, m_p the inverted Thomas pivots, c'_p
// the eliminated super-diagonal and beta_p the explicit diagonal, all from the
// host (long double, rounded once).  Each lane composes its points' affine maps,
// a six-step Hillis-Steele scan over the lanes combines them (exact: every
// carry reaches the whole line) with host-precomputed multipliers, and each
// lane applies its carry.  The potential + nonlinear substep (and the
// imaginary-time renormalisation) is applied on load; in imaginary time the
// epilogue writes the weighted norm partial sum w_p |u'_p|^2.
#include <cmath>

#include "gp_internal.h"
#include "gp_sweep_common.h"
#include "gp_xscan.h"

namespace gp {

namespace {

constexpr int kRWaves = 4;  // lines (wavefronts) per workgroup

// Cell weight w_i (cell volume over dr) of a d-dimensional radial grid.
__device__ __forceinline__ double radial_weight(int64_t i, double dr, int d)
{
    const double r = ((double)i + 0.5) * dr;
    return d == 3 ? r * r + dr * dr / 12.0 : r;
}

// One wavefront solves radial line `line` (src -> dst), adding the weighted
// norm of its output to nacc when FLAGS has F_NORM_OUT.
template <typename R, int MODE, int FLAGS, int Q>
__device__ __forceinline__ void radial_line_wave(const SweepParams &P, const typename CT<R>::V *src,
                                                 typename CT<R>::V *dst, const typename CT<R>::V *__restrict__ rows,
                                                 const typename CT<R>::V *__restrict__ rmul, int64_t line, int lane,
                                                 double &nacc)
{
    using V = typename CT<R>::V;
    const int64_t n = P.n;
    const cp<R> zero = {R(0), R(0)};
    {
        const int64_t base = line * n;
        LineCtx<R> L = line_ctx_of<R>(P, line);
        if (FLAGS & F_RENORM) L.scale = 1.0 / sqrt(P.dV * P.norm_total[0]);
        cp<R> u[Q], f[Q];
        cp<R> al[Q], mm[Q], cn[Q], bt[Q], sb[Q], sp[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int64_t q = (int64_t)lane * Q + i;
            const bool in = q < n;
            u[i] = in ? from_v<R>(src[base + q]) : zero;
            if ((FLAGS & F_FUSE_N) && in) u[i] = potential_substep<R, MODE, FLAGS>(u[i], q, P, L);
            const V *row = rows + 6 * (in ? q : 0);
            al[i] = in ? from_v<R>(row[0]) : zero;
            mm[i] = in ? from_v<R>(row[1]) : zero;
            cn[i] = in ? from_v<R>(row[2]) : zero;  // -c'_p (the backward multiplier)
            bt[i] = in ? from_v<R>(row[3]) : zero;
            sb[i] = in ? from_v<R>(row[4]) : zero;
            sp[i] = in ? from_v<R>(row[5]) : zero;
        }
        cp<R> left = shfl_up_c(u[Q - 1], 1);
        cp<R> right = shfl_down_c(u[0], 1);
        if (lane == 0) left = zero;
        if (lane == kLanes - 1) right = zero;
        // forward: f_p = m_p rhs_p, composed over the lane's points
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const cp<R> um1 = i == 0 ? left : u[i - 1];
            const cp<R> up1 = i == Q - 1 ? right : u[i + 1];
            cp<R> rhs = kmul<MODE>(bt[i], u[i]);
            const cp<R> lo = kmul<MODE>(sb[i], um1), hi = kmul<MODE>(sp[i], up1);
            rhs.re -= lo.re + hi.re;
            rhs.im -= lo.im + hi.im;
            f[i] = kmul<MODE>(mm[i], rhs);
        }
        cp<R> F = f[0];
#pragma unroll
        for (int i = 1; i < Q; ++i) F = kfma<MODE>(al[i], F, f[i]);
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            const cp<R> Fp = shfl_up_c(F, 1 << s);
            if (lane >= (1 << s)) F = kfma<MODE>(from_v<R>(rmul[s * kLanes + lane]), Fp, F);
        }
        cp<R> y = shfl_up_c(F, 1);
        if (lane == 0) y = zero;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            y = kfma<MODE>(al[i], y, f[i]);
            f[i] = y;
        }
        // backward: u'_p = -c'_p u'_{p+1} + y_p
        cp<R> G = f[Q - 1];
#pragma unroll
        for (int i = Q - 2; i >= 0; --i) G = kfma<MODE>(cn[i], G, f[i]);
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            const cp<R> Gp = shfl_down_c(G, 1 << s);
            if (lane + (1 << s) < kLanes) G = kfma<MODE>(from_v<R>(rmul[(6 + s) * kLanes + lane]), Gp, G);
        }
        cp<R> v = shfl_down_c(G, 1);
        if (lane == kLanes - 1) v = zero;
#pragma unroll
        for (int i = Q - 1; i >= 0; --i) {
            v = kfma<MODE>(cn[i], v, f[i]);
            const int64_t q = (int64_t)lane * Q + i;
            if (q < n) {
                if (FLAGS & F_NORM_OUT)
                    nacc += radial_weight(q, P.dx[0], P.radial_d) * ((double)v.re * (double)v.re +
                                                                     (double)v.im * (double)v.im);
                dst[base + q] = to_v<V>(v);
            }
        }
    }
}

template <typename R, int MODE, int FLAGS, int Q>
__global__ __launch_bounds__(kLanes *kRWaves) void k_radial_line(SweepParams P, const typename CT<R>::V *src,
                                                                 typename CT<R>::V *dst,
                                                                 const typename CT<R>::V *__restrict__ rows,
                                                                 const typename CT<R>::V *__restrict__ rmul)
{
    const int lane = threadIdx.x & (kLanes - 1);
    const int wave = threadIdx.x / kLanes;
    const int64_t line = (int64_t)blockIdx.x * kRWaves + wave;
    double nacc = 0.0;
    if (line < P.nlines)  // uniform across the wavefront
        radial_line_wave<R, MODE, FLAGS, Q>(P, src, dst, rows, rmul, line, lane, nacc);
    if (FLAGS & F_NORM_OUT) {
        __shared__ double red[kRWaves];
        nacc = wave_sum(nacc);
        if (lane == 0) red[wave] = nacc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = 0.0;
            for (int k = 0; k < kRWaves; ++k) a += red[k];
            P.norm_out[blockIdx.x] = a;
        }
    }
}

// A circular or spherical run (one radial line) in one launch, as the
// Cartesian 1D run: one wavefront takes the steps in turn through the line
// kernel's routine and flags, with the imaginary-time norm total kept in LDS
// (the separate launches sum the same value with zeros).  *total_out receives
// the last step's total.
template <int MODE, int Q>
__global__ __launch_bounds__(kLanes) void k_radial_steps(SweepParams P, typename CT<double>::V *psi,
                                                         const typename CT<double>::V *__restrict__ rows,
                                                         const typename CT<double>::V *__restrict__ rmul,
                                                         int64_t nsteps, double *total_out)
{
    constexpr bool kImag = MODE == GP_IMAG;
    constexpr int kFlags = F_FUSE_N | (kImag ? F_NORM_OUT : 0);
    const int lane = threadIdx.x & (kLanes - 1);
    __shared__ double tot;
    SweepParams Pr = P;  // renormalising steps read the previous step's total from LDS
    Pr.norm_total = &tot;
    for (int64_t k = 0; k < nsteps; ++k) {
        double nacc = 0.0;
        if (kImag && k > 0)
            radial_line_wave<double, MODE, kFlags | F_RENORM, Q>(Pr, psi, psi, rows, rmul, 0, lane, nacc);
        else
            radial_line_wave<double, MODE, kFlags, Q>(P, psi, psi, rows, rmul, 0, lane, nacc);
        if constexpr (kImag) {
            nacc = wave_sum(nacc);
            __syncthreads();  // every lane has read the previous total
            if (lane == 0) tot = nacc;
            __syncthreads();
        }
    }
    if (kImag && lane == 0 && nsteps > 0) *total_out = tot;
}

template <int MODE>
hipError_t launch_radial_steps_mode(const SweepParams &P, const AxisPlan &A, void *psi, int64_t nsteps,
                                    double *total_out, hipStream_t s)
{
    using V = CT<double>::V;
    const V *rows = (const V *)A.d_rtab, *rmul = (const V *)A.d_rmul;
    switch (A.rq) {
    case 1: hipLaunchKernelGGL((k_radial_steps<MODE, 1>), dim3(1), dim3(kLanes), 0, s, P, (V *)psi, rows, rmul, nsteps, total_out); break;
    case 2: hipLaunchKernelGGL((k_radial_steps<MODE, 2>), dim3(1), dim3(kLanes), 0, s, P, (V *)psi, rows, rmul, nsteps, total_out); break;
    case 4: hipLaunchKernelGGL((k_radial_steps<MODE, 4>), dim3(1), dim3(kLanes), 0, s, P, (V *)psi, rows, rmul, nsteps, total_out); break;
    case 8: hipLaunchKernelGGL((k_radial_steps<MODE, 8>), dim3(1), dim3(kLanes), 0, s, P, (V *)psi, rows, rmul, nsteps, total_out); break;
    case 16: hipLaunchKernelGGL((k_radial_steps<MODE, 16>), dim3(1), dim3(kLanes), 0, s, P, (V *)psi, rows, rmul, nsteps, total_out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Weighted norm partials sum w_i |psi_ij|^2 of an axial grid (rho fastest), one
// per workgroup, each thread summing a fixed strided set of points.
template <typename R>
__global__ __launch_bounds__(256) void k_radial_norm(const typename CT<R>::V *__restrict__ psi, int64_t nr,
                                                     int64_t npts, double dr, int d, double *__restrict__ part)
{
    double acc = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += (int64_t)gridDim.x * blockDim.x) {
        const typename CT<R>::V u = psi[p];
        acc += radial_weight(p % nr, dr, d) * ((double)u.x * (double)u.x + (double)u.y * (double)u.y);
    }
    __shared__ double red[256 / kLanes];
    acc = wave_sum(acc);
    if ((threadIdx.x & (kLanes - 1)) == 0) red[threadIdx.x / kLanes] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < 256 / kLanes; ++k) s += red[k];
        part[blockIdx.x] = s;
    }
}

// Observable sums of a symmetric-trap grid, one point per thread (grid-stride),
// into per-workgroup rows of kObsFields: 0 sum w|u|^2, 1 sum w V|u|^2, 2 sum w|u|^4,
// 3 sum w r^2|u|^2, 4 sum w z^2|u|^2, 6 radial faces a_{i+1/2}|u_{i+1} - u_i|^2
// (the outer face to the zero ghost included), 7 z: w |u_j - u_{j-1}|^2 with zero ghosts.
struct RadialObs {
    int64_t nr, nz, npts;
    double dr, dz, z0, hw_r, hw_z;
    int d;
};

template <typename R>
__global__ __launch_bounds__(256) void k_radial_obs(const typename CT<R>::V *__restrict__ psi, RadialObs O,
                                                    double *__restrict__ part)
{
    double acc[kObsFields];
    for (int f = 0; f < kObsFields; ++f) acc[f] = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < O.npts; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = p % O.nr, j = p / O.nr;
        const typename CT<R>::V u = psi[p];
        const double ur = u.x, ui = u.y, dd = ur * ur + ui * ui;
        const double w = radial_weight(i, O.dr, O.d), r = ((double)i + 0.5) * O.dr;
        const double z = ((double)j + O.z0) * O.dz;
        acc[0] += w * dd;
        acc[1] += w * (O.hw_r * r * r + O.hw_z * z * z) * dd;
        acc[2] += w * dd * dd;
        acc[3] += w * r * r * dd;
        acc[4] += w * z * z * dd;
        double nr_ = 0.0, ni_ = 0.0;
        if (i + 1 < O.nr) {
            const typename CT<R>::V v = psi[p + 1];
            nr_ = v.x;
            ni_ = v.y;
        }
        const double face = O.d == 3 ? ((double)(i + 1) * O.dr) * ((double)(i + 1) * O.dr) : (double)(i + 1) * O.dr;
        acc[6] += face * ((nr_ - ur) * (nr_ - ur) + (ni_ - ui) * (ni_ - ui));
        if (O.nz > 1) {
            double pr = 0.0, pi = 0.0;
            if (j > 0) {
                const typename CT<R>::V v = psi[p - O.nr];
                pr = v.x;
                pi = v.y;
            }
            acc[7] += w * ((ur - pr) * (ur - pr) + (ui - pi) * (ui - pi) + (j == O.nz - 1 ? dd : 0.0));
        }
    }
    __shared__ double red[256 / kLanes][kObsFields];
    const int lane = threadIdx.x & (kLanes - 1), wave = threadIdx.x / kLanes;
    for (int f = 0; f < kObsFields; ++f) {
        const double v = wave_sum(acc[f]);
        if (lane == 0) red[wave][f] = v;
    }
    __syncthreads();
    if (threadIdx.x < kObsFields) {
        double s = 0.0;
        for (int k = 0; k < 256 / kLanes; ++k) s += red[k][threadIdx.x];
        part[(int64_t)blockIdx.x * kObsFields + threadIdx.x] = s;
    }
}

template <int MODE, int FLAGS, int Q>
void launch_line_q(const SweepParams &P, const AxisPlan &A, hipStream_t s)
{
    using V = CT<double>::V;
    const unsigned grid = (unsigned)((P.nlines + kRWaves - 1) / kRWaves);
    hipLaunchKernelGGL((k_radial_line<double, MODE, FLAGS, Q>), dim3(grid), dim3(kLanes * kRWaves), 0, s, P,
                       (const V *)P.psi, (V *)P.out, (const V *)A.d_rtab, (const V *)A.d_rmul);
}

template <int MODE, int FLAGS>
hipError_t launch_line_flags(const SweepParams &P, const AxisPlan &A, hipStream_t s)
{
    switch (A.rq) {
    case 1: launch_line_q<MODE, FLAGS, 1>(P, A, s); break;
    case 2: launch_line_q<MODE, FLAGS, 2>(P, A, s); break;
    case 4: launch_line_q<MODE, FLAGS, 4>(P, A, s); break;
    case 8: launch_line_q<MODE, FLAGS, 8>(P, A, s); break;
    case 16: launch_line_q<MODE, FLAGS, 16>(P, A, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

int64_t radial_line_groups(const gp_plan *p) { return (p->ax[0].nlines + kRWaves - 1) / kRWaves; }
int64_t radial_norm_groups(const gp_plan *p) { return std::min<int64_t>(256, (p->npts + 255) / 256); }

hipError_t launch_radial_line(gp_plan *p, const void *src, void *dst, int flags, int64_t step_index, hipStream_t s)
{
    SweepParams P = make_sweep_params(p, 0, src, dst, false, step_index, nullptr);
    timing_begin(p, K_SWEEP_X, s);
    hipError_t e;
    if (p->mode == GP_IMAG) {
        switch (flags) {
        case F_FUSE_N: e = launch_line_flags<GP_IMAG, F_FUSE_N>(P, p->ax[0], s); break;
        case F_FUSE_N | F_RENORM: e = launch_line_flags<GP_IMAG, F_FUSE_N | F_RENORM>(P, p->ax[0], s); break;
        case F_FUSE_N | F_NORM_OUT: e = launch_line_flags<GP_IMAG, F_FUSE_N | F_NORM_OUT>(P, p->ax[0], s); break;
        case F_FUSE_N | F_RENORM | F_NORM_OUT:
            e = launch_line_flags<GP_IMAG, F_FUSE_N | F_RENORM | F_NORM_OUT>(P, p->ax[0], s);
            break;
        default: e = hipErrorInvalidValue;
        }
    } else {
        e = flags == F_FUSE_N ? launch_line_flags<GP_REAL, F_FUSE_N>(P, p->ax[0], s) : hipErrorInvalidValue;
    }
    timing_end(p, s);
    return e;
}

hipError_t launch_radial_steps(gp_plan *p, void *psi, int64_t nsteps, double *total_out, hipStream_t s)
{
    const SweepParams P = make_sweep_params(p, 0, psi, psi, false, p->step, nullptr);
    timing_begin(p, K_SWEEP_X, s);
    const hipError_t e = p->mode == GP_IMAG
                             ? launch_radial_steps_mode<GP_IMAG>(P, p->ax[0], psi, nsteps, total_out, s)
                             : launch_radial_steps_mode<GP_REAL>(P, p->ax[0], psi, nsteps, total_out, s);
    timing_end(p, s);
    return e;
}

hipError_t launch_radial_norm(gp_plan *p, const void *psi, int64_t step_index, hipStream_t s)
{
    const int64_t nb = radial_norm_groups(p);
    timing_begin(p, K_RADIAL_NORM, s);
    hipLaunchKernelGGL(k_radial_norm<double>, dim3((unsigned)nb), dim3(256), 0, s, (const double2 *)psi, p->n[0],
                       p->npts, p->dx[0], radial_dim(p->geom), norm_partials(p, step_index));
    timing_end(p, s);
    return hipGetLastError();
}

hipError_t launch_radial_obs(gp_plan *p, const void *psi, double *part, int64_t nb, hipStream_t s)
{
    double w[3];
    omega_at_step(p, p->step > 0 ? p->step - 1 : 0, w);
    RadialObs O{};
    O.nr = p->n[0];
    O.nz = p->geom == GP_AXIAL ? p->n[1] : 1;
    O.npts = p->npts;
    O.dr = p->dx[0];
    O.dz = p->geom == GP_AXIAL ? p->dx[1] : 0.0;
    O.z0 = p->geom == GP_AXIAL ? coord0(p->n[1]) : 0.0;
    O.hw_r = 0.5 * w[0] * w[0];
    O.hw_z = p->geom == GP_AXIAL ? 0.5 * w[1] * w[1] : 0.0;
    O.d = radial_dim(p->geom);
    timing_begin(p, K_OBS, s);
    hipLaunchKernelGGL(k_radial_obs<double>, dim3((unsigned)nb), dim3(256), 0, s, (const double2 *)psi, O, part);
    timing_end(p, s);
    return hipGetLastError();
}

}  // namespace gp

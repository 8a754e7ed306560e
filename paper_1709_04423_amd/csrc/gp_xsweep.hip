// x sweep (contiguous axis) with one wavefront per grid line.
//
// Each lane holds Q = n/64 (rounded up to a power of two) consecutive points
// of the line, so every load and store of a wavefront is one contiguous
// segment, and many lines per CU are in flight at once (no LDS, modest
// registers).  The two Thomas recurrences of the scaled CN system are first-
// order affine recurrences along the line,
//     forward   y_p = -c'_p y_{p-1} + c'_p rhs_p,
//     backward  u'_p = -c'_p u'_{p+1} + y_p,
// so each lane composes the affine maps of its Q points into one map, the
// lanes combine their maps with a Hillis-Steele scan over shuffles, and each
// lane then applies its incoming carry to its own points.  A scan of S steps
// lets a carry travel Q 2^S points; the influence of points further away is
// multiplied by prod |c'| <= rho^(Q 2^S), and the host picks S as the smallest
// with Q 2^S > K (the same bound as the windowed solver) -- S = 6 is the full
// scan and exact.  The potential substep is applied to the loaded values, and
// the norm / adjoint epilogues to the stored ones, as in the other sweeps.
#include "gp_internal.h"
#include "gp_sweep_common.h"

namespace gp {

constexpr int kXWaves = kXWavesPerGroup;  // lines (wavefronts) per workgroup

template <typename R>
__device__ __forceinline__ cp<R> cmul(cp<R> a, cp<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cp<R> cfma(cp<R> a, cp<R> b, cp<R> c)  // a*b + c
{
    return {a.re * b.re - a.im * b.im + c.re, a.re * b.im + a.im * b.re + c.im};
}
template <typename R> __device__ __forceinline__ cp<R> shfl_up_c(cp<R> v, int d)
{
    return {__shfl_up(v.re, d, kLanes), __shfl_up(v.im, d, kLanes)};
}
template <typename R> __device__ __forceinline__ cp<R> shfl_down_c(cp<R> v, int d)
{
    return {__shfl_down(v.re, d, kLanes), __shfl_down(v.im, d, kLanes)};
}

// Table row of point q: (c', beta, beta_lo); constant past q_const, zero past n.
template <typename R, typename V>
__device__ __forceinline__ void row_of(const SweepParams &P, const V *__restrict__ tab, int64_t q, V &c, V &b,
                                       V &blo)
{
    if (q >= P.n) {
        c.x = c.y = b.x = b.y = blo.x = blo.y = R(0);
    } else if (q >= P.q_const) {
        c.x = R(P.c_inf[0]);
        c.y = R(P.c_inf[1]);
        b.x = R(P.b_inf[0]);
        b.y = R(P.b_inf[1]);
        blo.x = R(P.b_inf[2]);
        blo.y = R(0);
    } else {
        c = tab[3 * (q + 1)];
        b = tab[3 * (q + 1) + 1];
        blo = tab[3 * (q + 1) + 2];
    }
}

template <typename R, int MODE, int FLAGS, int Q>
__global__ __launch_bounds__(kLanes *kXWaves) void k_sweep_x_scan(SweepParams P, const typename CT<R>::V *src,
                                                                   typename CT<R>::V *dst,
                                                                   const typename CT<R>::V *__restrict__ tab,
                                                                   const typename CT<R>::V *__restrict__ state)
{
    using V = typename CT<R>::V;
    const int lane = threadIdx.x & (kLanes - 1);
    const int wave = threadIdx.x / kLanes;
    const int64_t line = (int64_t)blockIdx.x * kXWaves + wave;
    const bool active = line < P.nlines;
    const int64_t n = P.n;
    const int64_t base = (active ? line : 0) * n;
    const int64_t q0 = (int64_t)lane * Q;

    LineCtx<R> L = line_ctx_of<R>(P, active ? line : 0);
    if (FLAGS & F_RENORM) L.scale = 1.0 / sqrt(P.dV * wave_sum_partials(P.norm_in, P.nnorm_in, lane));

    // load Q consecutive points (one contiguous segment per wavefront)
    cp<R> u[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int64_t q = q0 + i;
        u[i] = (active && q < n) ? from_v<R>(src[base + q]) : cp<R>{R(0), R(0)};
        if ((FLAGS & F_FUSE_N) && q < n) u[i] = potential_substep<R, MODE, FLAGS>(u[i], q, P, L);
    }
    // neighbours across lane boundaries (zero ghosts at the line ends)
    cp<R> left = shfl_up_c(u[Q - 1], 1);
    cp<R> right = shfl_down_c(u[0], 1);
    if (lane == 0) left = {R(0), R(0)};
    if (lane == kLanes - 1) right = {R(0), R(0)};

    // forward maps y_p = a_p y_{p-1} + f_p with a_p = -c'_p, f_p = c'_p rhs_p
    cp<R> cc[Q], f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        V c, b, blo;
        row_of<R>(P, tab, q0 + i, c, b, blo);
        const cp<R> um1 = i == 0 ? left : u[i - 1];
        const cp<R> up1 = i == Q - 1 ? right : u[i + 1];
        const cp<R> rhs = cn_rhs<MODE, R>(um1, u[i], up1, b, blo);
        cc[i] = from_v<R>(c);
        f[i] = cmul(cc[i], rhs);
    }
    // compose this lane's maps: y_last = A y_in + F
    cp<R> A = {-cc[0].re, -cc[0].im}, F = f[0];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const cp<R> a = {-cc[i].re, -cc[i].im};
        F = cfma(a, F, f[i]);
        A = cmul(a, A);
    }
    for (int s = 0; s < P.scan_steps; ++s) {
        const int d = 1 << s;
        const cp<R> Ap = shfl_up_c(A, d), Fp = shfl_up_c(F, d);
        if (lane >= d) {
            F = cfma(A, Fp, F);
            A = cmul(A, Ap);
        }
    }
    cp<R> y = shfl_up_c(F, 1);
    if (lane == 0) y = {R(0), R(0)};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        y = cfma({-cc[i].re, -cc[i].im}, y, f[i]);
        f[i] = y;  // f now holds the eliminated values y_p
    }
    // backward maps u'_p = b_p u'_{p+1} + y_p with b_p = -c'_p, composed from the top
    cp<R> Bm = {-cc[Q - 1].re, -cc[Q - 1].im}, G = f[Q - 1];
#pragma unroll
    for (int i = Q - 2; i >= 0; --i) {
        const cp<R> b = {-cc[i].re, -cc[i].im};
        G = cfma(b, G, f[i]);
        Bm = cmul(b, Bm);
    }
    for (int s = 0; s < P.scan_steps; ++s) {
        const int d = 1 << s;
        const cp<R> Bp = shfl_down_c(Bm, d), Gp = shfl_down_c(G, d);
        if (lane + d < kLanes) {
            G = cfma(Bm, Gp, G);
            Bm = cmul(Bm, Bp);
        }
    }
    cp<R> v = shfl_down_c(G, 1);
    if (lane == kLanes - 1) v = {R(0), R(0)};
#pragma unroll
    for (int i = Q - 1; i >= 0; --i) {
        v = cfma({-cc[i].re, -cc[i].im}, v, f[i]);
        u[i] = v;
    }

    // epilogue and store
    double nacc = 0.0, acc_w = 0.0, acc_g = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int64_t q = q0 + i;
        if (active && q < n) {
            cp<R> w = u[i];
            if (FLAGS & F_NORM_OUT) nacc += (double)w.re * (double)w.re + (double)w.im * (double)w.im;
            if (FLAGS & F_ADJ_N) w = potential_adjoint<R, MODE, FLAGS>(w, q, state, base + q, P, L, acc_w, acc_g);
            dst[base + q] = to_v<V>(w);
        }
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
    }
}

template <typename R, int MODE, int FLAGS, int Q>
static void launch_q(const SweepParams &P, const void *tab, hipStream_t s)
{
    using V = typename CT<R>::V;
    const unsigned grid = (unsigned)((P.nlines + kXWaves - 1) / kXWaves);
    hipLaunchKernelGGL((k_sweep_x_scan<R, MODE, FLAGS, Q>), dim3(grid), dim3(kLanes * kXWaves), 0, s, P,
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
    case F_ADJ_N: return launch_x_flags<R, MODE, F_ADJ_N>(P, Q, tab, s);
    default: return hipErrorInvalidValue;
    }
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

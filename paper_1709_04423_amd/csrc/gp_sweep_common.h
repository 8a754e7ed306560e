// Device helpers shared by the sweep kernels: complex values, the scaled CN
// recurrences, the potential substep and its adjoint, wavefront reductions.
#pragma once

#include "gp_internal.h"

namespace gp {

template <typename R> struct CT;
template <> struct CT<double> {
    using V = double2;
};
template <> struct CT<float> {
    using V = float2;
};

template <typename R> struct cp {
    R re, im;
};

template <typename R, typename V> __device__ __forceinline__ cp<R> from_v(V v) { return {v.x, v.y}; }
template <typename V, typename R> __device__ __forceinline__ V to_v(cp<R> c)
{
    V v;
    v.x = c.re;
    v.y = c.im;
    return v;
}

// The solver works on the CN system divided by the off-diagonal e, which has
// unit off-diagonals:  tridiag(1, delta_p, 1) u' = beta_p u - (u_{p-1} + u_{p+1}).
// The Thomas factorisation of the left side, LU with L = diag(1/c'_p) + S^-,
// U = I + diag(c'_p) S^+, needs one table value per row:
//     y_p = (rhs_p - y_{p-1}) c'_p          (forward elimination)
//     u'_p = y_p - c'_p u'_{p+1}             (back substitution)
// and the c' as stored define delta_p = 1/c'_p + c'_{p-1} exactly.  The host
// derives beta_p from those same stored values: in real time beta_p =
// -conj(delta_p), whose imaginary part is carried as a float pair (hi + lo).
// That keeps the Hermitian part of the map's two sides equal to working
// precision squared, so the real-time substep stays unitary in the interior of
// every line even when the table is rounded to FP32.  Table row r (point
// p = r - 1) holds three values: c'_p, (Re beta_p, Im beta_p hi), (Im beta_p lo, 0).
template <int MODE, typename R, typename V>
__device__ __forceinline__ cp<R> cn_rhs(cp<R> um1, cp<R> u, cp<R> up1, V beta, V beta_lo)
{
    const R sr = um1.re + up1.re, si = um1.im + up1.im;
    if (MODE == GP_IMAG) return {beta.x * u.re - sr, beta.x * u.im - si};
    // The small part (a discrete Laplacian plus the lo correction) is formed
    // first and the large i Im(beta) u term added last: added after it, the lo
    // correction would fall below that sum's rounding and be lost every time,
    // which biases the norm by the rounding of Im(beta) per sweep.
    R re = beta.x * u.re - sr;
    R im = beta.x * u.im - si;
    re -= beta_lo.x * u.im;
    im += beta_lo.x * u.re;
    re -= beta.y * u.im;
    im += beta.y * u.re;
    return {re, im};
}

// y = (rhs - y_prev) c'
template <int MODE, typename R, typename V>
__device__ __forceinline__ cp<R> cn_elim(cp<R> rhs, cp<R> yprev, V c)
{
    const R wr = rhs.re - yprev.re, wi = rhs.im - yprev.im;
    if (MODE == GP_IMAG) return {wr * c.x, wi * c.x};
    return {wr * c.x - wi * c.y, wr * c.y + wi * c.x};
}

// v = y - c' v
template <int MODE, typename R, typename V>
__device__ __forceinline__ cp<R> cn_back(cp<R> y, V c, cp<R> v)
{
    if (MODE == GP_IMAG) return {y.re - c.x * v.re, y.im - c.x * v.im};
    return {y.re - (c.x * v.re - c.y * v.im), y.im - (c.x * v.im + c.y * v.re)};
}

// Sum of np FP64 partials in a fixed order; every lane of the wavefront gets
// the same bits (lane-strided sums, then an xor butterfly of commutative adds).
__device__ __forceinline__ double wave_sum_partials(const double *part, int np, int lane)
{
    double acc = 0.0;
    for (int i = lane; i < np; i += kLanes) acc += part[i];
    for (int off = kLanes / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kLanes);
    return acc;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = kLanes / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kLanes);
    return v;
}

// Phase factors of the potential substep.  Real time multiplies by
// e^{-i theta} = 1 - h - i s with s = sin(theta) and h = 1 - cos(theta) =
// 2 sin^2(theta/2), applied as u + (s-term - h u): h is computed to full
// relative precision instead of rounding cos(theta) next to 1, so |1 - h - i s|
// differs from 1 by about eps h, not eps.  Near the Thomas-Fermi plateau theta
// is almost the same at every point, and a rounded cos(theta) would then scale
// the norm by the same factor every step (an FP32 drift of order 1e-5 per
// 1000 steps).  The angle is small in practice (|theta| = dt (V + g|psi|^2)
// ~ 0.06 on the 256^3 workload), so for |theta| <= 1/8 the Taylor series are
// evaluated in Horner form with coefficients (-1)^k/(2k+1)! for sin,
// (-1)^(k+1)/(2k)! for h and 1/k! for exp -- through theta^11, theta^10 and
// theta^11 in FP64 (first omitted term below 4e-18 relative) and theta^7,
// theta^6, theta^6 in FP32 (below 2e-10) -- and larger angles use the library
// sin and cos of theta/2.
template <typename R> struct Taylor {
    static constexpr R s3 = R(-1.0 / 6.0), s5 = R(1.0 / 120.0), s7 = R(-1.0 / 5040.0),
                       s9 = R(1.0 / 362880.0), s11 = R(-1.0 / 39916800.0);
    static constexpr R h2 = R(1.0 / 2.0), h4 = R(-1.0 / 24.0), h6 = R(1.0 / 720.0),
                       h8 = R(-1.0 / 40320.0), h10 = R(1.0 / 3628800.0);
    static constexpr R e2 = R(1.0 / 2.0), e3 = R(1.0 / 6.0), e4 = R(1.0 / 24.0), e5 = R(1.0 / 120.0),
                       e6 = R(1.0 / 720.0), e7 = R(1.0 / 5040.0), e8 = R(1.0 / 40320.0),
                       e9 = R(1.0 / 362880.0), e10 = R(1.0 / 3628800.0), e11 = R(1.0 / 39916800.0);
};

// s = sin(t), h = 1 - cos(t)
__device__ __forceinline__ void phase_r(double t, double *s, double *h)
{
    using T = Taylor<double>;
    if (fabs(t) <= 0.125) {
        const double t2 = t * t;
        *s = t + t * t2 * (T::s3 + t2 * (T::s5 + t2 * (T::s7 + t2 * (T::s9 + t2 * T::s11))));
        *h = t2 * (T::h2 + t2 * (T::h4 + t2 * (T::h6 + t2 * (T::h8 + t2 * T::h10))));
    } else {
        double sh, ch;
        sincos(0.5 * t, &sh, &ch);
        *s = 2.0 * sh * ch;
        *h = 2.0 * sh * sh;
    }
}
__device__ __forceinline__ void phase_r(float t, float *s, float *h)
{
    using T = Taylor<float>;
    if (fabsf(t) <= 0.125f) {
        const float t2 = t * t;
        *s = t + t * t2 * (T::s3 + t2 * (T::s5 + t2 * T::s7));
        *h = t2 * (T::h2 + t2 * (T::h4 + t2 * T::h6));
    } else {
        float sh, ch;
        sincosf(0.5f * t, &sh, &ch);
        *s = 2.0f * sh * ch;
        *h = 2.0f * sh * sh;
    }
}

// u e^{-i sg t} for sg = +1 / -1 given s = sin t, h = 1 - cos t
template <typename R>
__device__ __forceinline__ cp<R> rotate(cp<R> u, R s, R h, R sg)
{
    const R ss = sg * s;
    return {u.re + (ss * u.im - h * u.re), u.im - (ss * u.re + h * u.im)};
}

__device__ __forceinline__ double exp_r(double t)
{
    using T = Taylor<double>;
    if (fabs(t) <= 0.125)
        return 1.0 + t * (1.0 + t * (T::e2 + t * (T::e3 + t * (T::e4 + t * (T::e5 + t * (T::e6 + t * (T::e7 +
               t * (T::e8 + t * (T::e9 + t * (T::e10 + t * T::e11))))))))));
    return exp(t);
}
__device__ __forceinline__ float exp_r(float t)
{
    using T = Taylor<float>;
    if (fabsf(t) <= 0.125f)
        return 1.0f + t * (1.0f + t * (T::e2 + t * (T::e3 + t * (T::e4 + t * (T::e5 + t * T::e6)))));
    return expf(t);
}

// Per-line state shared by the sweep kernels.
template <typename R> struct LineCtx {
    int64_t base;
    bool active;
    double scale;   // imaginary-time renormalisation of loaded values
    R vperp;        // potential of the line's fixed coordinates (axis 0 lines)
    R hw0;          // 1/2 omega_x^2 of this step
    R ysq, zsq;     // squared fixed coordinates (schedule gradient)
};

template <typename R, int FLAGS>
__device__ __forceinline__ LineCtx<R> line_setup(const SweepParams &P, int64_t group, int lane)
{
    LineCtx<R> L;
    const int64_t line = group * kLanes + lane;
    L.active = line < P.nlines;
    const int64_t l = L.active ? line : 0;
    L.base = (l % P.m1) * P.s1 + (l / P.m1) * P.s2;
    L.scale = 1.0;
    if (FLAGS & F_RENORM) L.scale = 1.0 / sqrt(P.dV * P.norm_total[0]);
    L.vperp = R(0);
    L.hw0 = R(P.hw2[0]);
    L.ysq = R(0);
    L.zsq = R(0);
    if (FLAGS & (F_FUSE_N | F_ADJ_N)) {
        const double y = ((double)(l % P.ny) + P.x0[1]) * P.dx[1];
        const double z = ((double)(l / P.ny) + P.x0[2]) * P.dx[2];
        L.vperp = R(P.hw2[1] * y * y + P.hw2[2] * z * z);
        L.ysq = R(y * y);
        L.zsq = R(z * z);
    }
    return L;
}

// Per-line potential data of an axis-0 line given its index (transposed layout).
template <typename R>
__device__ __forceinline__ LineCtx<R> line_ctx_of(const SweepParams &P, int64_t line)
{
    LineCtx<R> L;
    L.base = line * P.n;
    L.active = true;
    L.scale = 1.0;
    const uint32_t l = (uint32_t)line, ny = (uint32_t)P.ny;
    const double y = ((double)(l % ny) + P.x0[1]) * P.dx[1];
    const double z = ((double)(l / ny) + P.x0[2]) * P.dx[2];
    L.vperp = R(P.hw2[1] * y * y + P.hw2[2] * z * z);
    L.hw0 = R(P.hw2[0]);
    L.ysq = R(y * y);
    L.zsq = R(z * z);
    return L;
}

// Potential + nonlinear substep on one value at point q of an axis-0 line.
template <typename R, int MODE, int FLAGS>
__device__ __forceinline__ cp<R> potential_substep(cp<R> u, int64_t q, const SweepParams &P,
                                                   const LineCtx<R> &L)
{
    if (FLAGS & F_RENORM) {
        u.re = R((double)u.re * L.scale);
        u.im = R((double)u.im * L.scale);
    }
    const R x = R(((double)q + P.x0[0]) * P.dx[0]);
    const R theta = R(P.dt) * (L.vperp + L.hw0 * x * x + R(P.g) * (u.re * u.re + u.im * u.im));
    if (MODE == GP_REAL) {
        R s, h;
        phase_r(theta, &s, &h);
        return rotate(u, s, h, R(1));
    }
    const R f = exp_r(-theta);
    return {u.re * f, u.im * f};
}

// The potential substep on Q values of one line, at points q0 + qs i, with the
// same arithmetic as potential_substep.  The series branch is taken for all Q
// values together, with no per-value branch, so their dependency chains
// interleave; values whose angle exceeds the series range (rare; the wavefront
// checks once) are redone with the library functions.
template <typename R, int MODE, int FLAGS, int Q>
__device__ __forceinline__ void potential_substep_n(cp<R> *u, int q0, int qs, const SweepParams &P,
                                                    const LineCtx<R> &L)
{
    R th[Q];
    bool big = false;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (FLAGS & F_RENORM) {
            u[i].re = R((double)u[i].re * L.scale);
            u[i].im = R((double)u[i].im * L.scale);
        }
        const R x = R(((double)(q0 + qs * i) + P.x0[0]) * P.dx[0]);
        th[i] = R(P.dt) * (L.vperp + L.hw0 * x * x + R(P.g) * (u[i].re * u[i].re + u[i].im * u[i].im));
        big |= !(fabs(th[i]) <= R(0.125));
    }
    using T = Taylor<R>;
    if (MODE == GP_REAL) {
        R sn[Q], h[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const R t = th[i], t2 = t * t;
            if (sizeof(R) == 8) {
                sn[i] = t + t * t2 * (T::s3 + t2 * (T::s5 + t2 * (T::s7 + t2 * (T::s9 + t2 * T::s11))));
                h[i] = t2 * (T::h2 + t2 * (T::h4 + t2 * (T::h6 + t2 * (T::h8 + t2 * T::h10))));
            } else {
                sn[i] = t + t * t2 * (T::s3 + t2 * (T::s5 + t2 * T::s7));
                h[i] = t2 * (T::h2 + t2 * (T::h4 + t2 * T::h6));
            }
        }
        if (__builtin_expect(__builtin_amdgcn_ballot_w64(big) != 0, 0)) {
#pragma unroll
            for (int i = 0; i < Q; ++i)
                if (!(fabs(th[i]) <= R(0.125))) phase_r(th[i], &sn[i], &h[i]);
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) u[i] = rotate(u[i], sn[i], h[i], R(1));
        return;
    }
    R f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const R t = -th[i];
        if (sizeof(R) == 8)
            f[i] = 1.0 + t * (1.0 + t * (T::e2 + t * (T::e3 + t * (T::e4 + t * (T::e5 + t * (T::e6 + t * (T::e7 +
                   t * (T::e8 + t * (T::e9 + t * (T::e10 + t * T::e11))))))))));
        else
            f[i] = R(1) + t * (R(1) + t * (T::e2 + t * (T::e3 + t * (T::e4 + t * (T::e5 + t * T::e6)))));
    }
    if (__builtin_expect(__builtin_amdgcn_ballot_w64(big) != 0, 0)) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
            if (!(fabs(th[i]) <= R(0.125))) f[i] = exp_r(-th[i]);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) u[i] = {u[i].re * f[i], u[i].im * f[i]};
}

// In groups of at most four values: enough independent chains to fill the
// pipeline without holding every value's angle, sine and cosine at once.
template <typename R, int MODE, int FLAGS, int Q>
__device__ __forceinline__ void potential_substep_q(cp<R> (&u)[Q], int q0, int qs, const SweepParams &P,
                                                    const LineCtx<R> &L)
{
    constexpr int G = Q < 4 ? Q : 4;
#pragma unroll
    for (int i = 0; i < Q; i += G) potential_substep_n<R, MODE, FLAGS, G>(u + i, q0 + qs * i, qs, P, L);
}

// Adjoint of the potential substep at point t: lam (gradient of its output)
// -> gradient of its input; accumulates the schedule and g gradient sums.
template <typename R, int MODE, int FLAGS, typename V>
__device__ __forceinline__ cp<R> potential_adjoint(cp<R> lam, int64_t t, const V *state,
                                                   int64_t addr, const SweepParams &P,
                                                   const LineCtx<R> &L, double &acc_w,
                                                   double &acc_g)
{
    const cp<R> psi = from_v<R>(state[addr]);
    const R x = R(((double)t + P.x0[0]) * P.dx[0]);
    const R d = psi.re * psi.re + psi.im * psi.im;
    const R theta = R(P.dt) * (L.vperp + L.hw0 * x * x + R(P.g) * d);
    R s, h;
    phase_r(theta, &s, &h);
    const cp<R> u = rotate(psi, s, h, R(1));  // u = psi e^{-i theta}
    const R w = lam.re * u.im - lam.im * u.re;  // Im(conj(lam) u)
    const R k2 = R(2) * R(P.dt) * R(P.g) * w;
    const R xs2 = P.sched_axis == 0 ? x * x : (P.sched_axis == 1 ? L.ysq : L.zsq);
    acc_w += (double)w * (double)xs2;
    acc_g += (double)w * (double)d;
    const cp<R> l = rotate(lam, s, h, R(-1));  // lam e^{+i theta}
    return {l.re + k2 * psi.re, l.im + k2 * psi.im};
}

// potential_adjoint on Q values at points q0 + qs i (those below n), with the
// forward state already loaded (st), the series branch shared by all values as
// in potential_substep_n and the sums accumulated in order of i.
template <typename R, int MODE, int FLAGS, int Q, typename V>
__device__ __forceinline__ void potential_adjoint_q(cp<R> (&lam)[Q], const V (&st)[Q], int q0, int qs, int64_t n,
                                                    const SweepParams &P, const LineCtx<R> &L, double &acc_w,
                                                    double &acc_g)
{
    using T = Taylor<R>;
    cp<R> psi[Q];
    R x[Q], d[Q], sn[Q], h[Q];
    bool big = false;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        psi[i] = from_v<R>(st[i]);
        x[i] = R(((double)(q0 + qs * i) + P.x0[0]) * P.dx[0]);
        d[i] = psi[i].re * psi[i].re + psi[i].im * psi[i].im;
        const R t = R(P.dt) * (L.vperp + L.hw0 * x[i] * x[i] + R(P.g) * d[i]), t2 = t * t;
        big |= !(fabs(t) <= R(0.125));
        if (sizeof(R) == 8) {
            sn[i] = t + t * t2 * (T::s3 + t2 * (T::s5 + t2 * (T::s7 + t2 * (T::s9 + t2 * T::s11))));
            h[i] = t2 * (T::h2 + t2 * (T::h4 + t2 * (T::h6 + t2 * (T::h8 + t2 * T::h10))));
        } else {
            sn[i] = t + t * t2 * (T::s3 + t2 * (T::s5 + t2 * T::s7));
            h[i] = t2 * (T::h2 + t2 * (T::h4 + t2 * T::h6));
        }
    }
    if (__builtin_expect(__builtin_amdgcn_ballot_w64(big) != 0, 0)) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const R t = R(P.dt) * (L.vperp + L.hw0 * x[i] * x[i] + R(P.g) * d[i]);
            if (!(fabs(t) <= R(0.125))) phase_r(t, &sn[i], &h[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const cp<R> u = rotate(psi[i], sn[i], h[i], R(1));  // u = psi e^{-i theta}
        const R w = lam[i].re * u.im - lam[i].im * u.re;   // Im(conj(lam) u)
        const R k2 = R(2) * R(P.dt) * R(P.g) * w;
        const R xs2 = P.sched_axis == 0 ? x[i] * x[i] : (P.sched_axis == 1 ? L.ysq : L.zsq);
        if (q0 + qs * i < n) {
            acc_w += (double)w * (double)xs2;
            acc_g += (double)w * (double)d[i];
        }
        const cp<R> l = rotate(lam[i], sn[i], h[i], R(-1));  // lam e^{+i theta}
        lam[i] = {l.re + k2 * psi[i].re, l.im + k2 * psi[i].im};
    }
}

// Wavefront sums of the epilogue accumulators, written to partial slot g.
template <typename R, int FLAGS>
__device__ __forceinline__ void write_partials(const SweepParams &P, int lane, double nacc,
                                               double acc_w, double acc_g, int64_t g)
{
    if (FLAGS & F_NORM_OUT) {
        nacc = wave_sum(nacc);
        if (lane == 0) P.norm_out[g] = nacc;
    }
    if (FLAGS & F_ADJ_N) {
        acc_w = wave_sum(acc_w);
        acc_g = wave_sum(acc_g);
        if (lane == 0) {
            P.adj_out[2 * g] = acc_w;
            P.adj_out[2 * g + 1] = acc_g;
        }
    }
}

}  // namespace gp

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
// prod |c'| <= rho^(K+1) before it reaches an output, and the host picks K so
// that rho^(K+1) is below 2^-60 (FP64) or 2^-48 (FP32).  Rows past the end of
// a line hold c' = 0, so the tail of every line is exact.  Each point is read
// once and written once.  When the window does not fit in LDS, k_sweep_exact
// runs the plain two-pass Thomas algorithm (eliminated values stored in
// place, then read back).
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

__device__ __forceinline__ void sincos_r(double t, double *s, double *c) { sincos(t, s, c); }
__device__ __forceinline__ void sincos_r(float t, float *s, float *c) { sincosf(t, s, c); }
__device__ __forceinline__ double exp_r(double t) { return exp(t); }
__device__ __forceinline__ float exp_r(float t) { return expf(t); }

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
__device__ __forceinline__ LineCtx<R> line_setup(const SweepParams &P, int lane)
{
    LineCtx<R> L;
    const int64_t line = (int64_t)blockIdx.x * kLanes + lane;
    L.active = line < P.nlines;
    const int64_t l = L.active ? line : 0;
    L.base = (l % P.m1) * P.s1 + (l / P.m1) * P.s2;
    L.scale = 1.0;
    if (FLAGS & F_RENORM) L.scale = 1.0 / sqrt(P.dV * wave_sum_partials(P.norm_in, P.nnorm_in, lane));
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
        R s, c;
        sincos_r(theta, &s, &c);
        return {u.re * c + u.im * s, u.im * c - u.re * s};
    }
    const R f = exp_r(-theta);
    return {u.re * f, u.im * f};
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
    R s, c;
    sincos_r(theta, &s, &c);
    const R ur = psi.re * c + psi.im * s;  // u = psi e^{-i theta}
    const R ui = psi.im * c - psi.re * s;
    const R w = lam.re * ui - lam.im * ur;  // Im(conj(lam) u)
    const R k2 = R(2) * R(P.dt) * R(P.g) * w;
    const R xs2 = P.sched_axis == 0 ? x * x : (P.sched_axis == 1 ? L.ysq : L.zsq);
    acc_w += (double)w * (double)xs2;
    acc_g += (double)w * (double)d;
    return {lam.re * c - lam.im * s + k2 * psi.re, lam.re * s + lam.im * c + k2 * psi.im};
}

template <typename R, int FLAGS>
__device__ __forceinline__ void write_partials(const SweepParams &P, int lane, double nacc,
                                               double acc_w, double acc_g)
{
    if (FLAGS & F_NORM_OUT) {
        nacc = wave_sum(nacc);
        if (lane == 0) P.norm_out[blockIdx.x] = nacc;
    }
    if (FLAGS & F_ADJ_N) {
        acc_w = wave_sum(acc_w);
        acc_g = wave_sum(acc_g);
        if (lane == 0) {
            P.adj_out[2 * blockIdx.x] = acc_w;
            P.adj_out[2 * blockIdx.x + 1] = acc_g;
        }
    }
}

// Access patterns of the windowed solver.
//  kStrided: lane = line, point q of the line at base + q*stride; used for the
//    y and z axes, whose 64 lines per wavefront are adjacent in memory, so each
//    load/store instruction moves one contiguous row.
//  kTransposed: the 64 lines of a wavefront are 64 consecutive x lines (length
//    n, stride 1).  Each block of kBlock points of the 64 lines is loaded with
//    coalesced instructions (instruction i, lane -> line 4i + lane/16, point
//    lane%16) and transposed through an LDS tile to the one-line-per-lane layout
//    of the solver; outputs go back the same way.
enum Access { kStrided = 0, kTransposed = 1 };
constexpr int kTilePitch = kBlock + 1;  // tile row pitch in values: conflict-free b128 access

template <typename R, int MODE, int FLAGS, int ACC> struct WindowSweep {
    using V = typename CT<R>::V;
    static constexpr int B = kBlock;
    const SweepParams &P;
    V *__restrict__ psi;
    const V *__restrict__ tab;
    const V *__restrict__ state;
    V *ring;
    V *tile;
    LineCtx<R> L;
    int lane;
    int64_t n, stride, base, l0;
    int lmask;
    cp<R> um1, u0, dprev;
    double nacc, acc_w, acc_g;

    __device__ __forceinline__ WindowSweep(const SweepParams &P_, V *psi_, const V *tab_, const V *state_, char *lds)
        : P(P_), psi(psi_), tab(tab_), state(state_)
    {
        lane = threadIdx.x;
        L = line_setup<R, FLAGS>(P, lane);
        n = P.n;
        stride = P.stride;
        base = L.base;
        l0 = (int64_t)blockIdx.x * kLanes;
        lmask = P.lmask;
        ring = reinterpret_cast<V *>(lds);
        tile = ring + (size_t)(lmask + 1) * kLanes;
        um1 = u0 = dprev = cp<R>{R(0), R(0)};
        nacc = acc_w = acc_g = 0.0;
    }

    __device__ __forceinline__ static V zero() { return to_v<V>(cp<R>{R(0), R(0)}); }

    // Issue the loads of block j.
    __device__ __forceinline__ void load(V (&buf)[B], int j) const
    {
        const int64_t q0 = (int64_t)j * B;
        if (ACC == kStrided) {
#pragma unroll
            for (int k = 0; k < B; ++k) buf[k] = (L.active && q0 + k < n) ? psi[base + (q0 + k) * stride] : zero();
        } else {
            const int pt = lane & (B - 1);
            const int64_t q = q0 + pt;
#pragma unroll
            for (int i = 0; i < B; ++i) {
                const int64_t line = l0 + i * (kLanes / B) + lane / B;
                buf[i] = (line < P.nlines && q < n) ? psi[line * n + q] : zero();
            }
        }
    }

    // Solve block j (values in buf) and write output block j - D.
    __device__ __forceinline__ void process(V (&buf)[B], int j)
    {
        V own[B];
        if (ACC == kTransposed) {
#pragma unroll
            for (int i = 0; i < B; ++i)
                tile[(i * (kLanes / B) + lane / B) * kTilePitch + (lane & (B - 1))] = buf[i];
            __syncthreads();
#pragma unroll
            for (int k = 0; k < B; ++k) own[k] = tile[lane * kTilePitch + k];
            __syncthreads();
        } else {
#pragma unroll
            for (int k = 0; k < B; ++k) own[k] = buf[k];
        }
        // forward elimination of points p = jB-1 .. jB+B-2 (u_{p+1} = own[k])
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int64_t q = (int64_t)j * B + k;
            cp<R> up1 = from_v<R>(own[k]);
            if ((FLAGS & F_FUSE_N) && q < n) up1 = potential_substep<R, MODE, FLAGS>(up1, q, P, L);
            const cp<R> rhs = cn_rhs<MODE, R>(um1, u0, up1, tab[3 * q + 1], tab[3 * q + 2]);  // row p+1 = q
            const cp<R> d = cn_elim<MODE, R>(rhs, dprev, tab[3 * q]);
            ring[(int)(q & lmask) * kLanes + lane] = to_v<V>(d);
            dprev = d;
            um1 = u0;
            u0 = up1;
        }
        // back substitution of output block o = j - D
        const int o = j - P.D;
        if (o < 0) return;
        const int64_t ob = (int64_t)o * B;
        cp<R> v = {R(0), R(0)};
        for (int64_t t = ob + B - 1 + P.K; t >= ob + B; --t)
            v = cn_back<MODE, R>(from_v<R>(ring[(int)((t + 1) & lmask) * kLanes + lane]), tab[3 * (t + 1)], v);
        cp<R> out[B];
#pragma unroll
        for (int k = B - 1; k >= 0; --k) {
            const int64_t t = ob + k;
            v = cn_back<MODE, R>(from_v<R>(ring[(int)((t + 1) & lmask) * kLanes + lane]), tab[3 * (t + 1)], v);
            out[k] = v;
        }
        if (ACC == kStrided) {
#pragma unroll
            for (int k = 0; k < B; ++k) {
                const int64_t t = ob + k;
                if (t < n) {
                    cp<R> w = out[k];
                    const int64_t addr = base + t * stride;
                    if (FLAGS & F_NORM_OUT) nacc += (double)w.re * (double)w.re + (double)w.im * (double)w.im;
                    if (FLAGS & F_ADJ_N)
                        if (L.active) w = potential_adjoint<R, MODE, FLAGS>(w, t, state, addr, P, L, acc_w, acc_g);
                    if (L.active) psi[addr] = to_v<V>(w);
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < B; ++k) tile[lane * kTilePitch + k] = to_v<V>(out[k]);
            __syncthreads();
            const int pt = lane & (B - 1);
            const int64_t t = ob + pt;
#pragma unroll
            for (int i = 0; i < B; ++i) {
                const int lo = i * (kLanes / B) + lane / B;
                const int64_t line = l0 + lo;
                cp<R> w = from_v<R>(tile[lo * kTilePitch + pt]);
                if (line < P.nlines && t < n) {
                    const int64_t addr = line * n + t;
                    if (FLAGS & F_NORM_OUT) nacc += (double)w.re * (double)w.re + (double)w.im * (double)w.im;
                    if (FLAGS & F_ADJ_N) {
                        const LineCtx<R> Lw = line_ctx_of<R>(P, line);
                        w = potential_adjoint<R, MODE, FLAGS>(w, t, state, addr, P, Lw, acc_w, acc_g);
                    }
                    psi[addr] = to_v<V>(w);
                }
            }
            __syncthreads();
        }
    }

    __device__ __forceinline__ void finish()
    {
        if (ACC == kStrided && !L.active) {
            nacc = 0.0;
            acc_w = 0.0;
            acc_g = 0.0;
        }
        write_partials<R, FLAGS>(P, lane, nacc, acc_w, acc_g);
    }
};

// Streaming solver with a windowed back substitution (see the file header).
// The block loop is unrolled by two over ping-pong buffers, so the loads of
// block j+1 stay in flight while block j is solved.
template <typename R, int MODE, int FLAGS, int ACC>
__global__ __launch_bounds__(kLanes) void k_sweep_window(SweepParams P,
                                                         typename CT<R>::V *__restrict__ psi,
                                                         const typename CT<R>::V *__restrict__ tab,
                                                         const typename CT<R>::V *__restrict__ state)
{
    using V = typename CT<R>::V;
    extern __shared__ char lds_raw[];
    WindowSweep<R, MODE, FLAGS, ACC> S(P, psi, tab, state, lds_raw);
    const int nit = P.nblocks + P.D;
    V a[kBlock], b[kBlock];
    S.load(a, 0);
    for (int j = 0; j < nit; j += 2) {
        if (j + 1 < nit) S.load(b, j + 1);
        S.process(a, j);
        if (j + 1 >= nit) break;
        if (j + 2 < nit) S.load(a, j + 2);
        S.process(b, j + 1);
    }
    S.finish();
}

// Plain two-pass Thomas algorithm: forward elimination stores d in place,
// back substitution reads it back.  Exact for any window; twice the traffic.
template <typename R, int MODE, int FLAGS>
__global__ __launch_bounds__(kLanes) void k_sweep_exact(SweepParams P,
                                                        typename CT<R>::V *__restrict__ psi,
                                                        const typename CT<R>::V *__restrict__ tab,
                                                        const typename CT<R>::V *__restrict__ state)
{
    using V = typename CT<R>::V;
    const int lane = threadIdx.x;
    const LineCtx<R> L = line_setup<R, FLAGS>(P, lane);
    const int64_t n = P.n, stride = P.stride, base = L.base;
    double nacc = 0.0, acc_w = 0.0, acc_g = 0.0;

    if (L.active) {
        cp<R> um1 = {R(0), R(0)}, dprev = {R(0), R(0)};
        cp<R> u0 = from_v<R>(psi[base]);
        if (FLAGS & F_FUSE_N) u0 = potential_substep<R, MODE, FLAGS>(u0, 0, P, L);
        for (int64_t q = 1; q <= n; ++q) {
            cp<R> up1 = {R(0), R(0)};
            if (q < n) {
                up1 = from_v<R>(psi[base + q * stride]);
                if (FLAGS & F_FUSE_N) up1 = potential_substep<R, MODE, FLAGS>(up1, q, P, L);
            }
            const cp<R> d = cn_elim<MODE, R>(cn_rhs<MODE, R>(um1, u0, up1, tab[3 * q + 1], tab[3 * q + 2]), dprev,
                                             tab[3 * q]);
            psi[base + (q - 1) * stride] = to_v<V>(d);
            dprev = d;
            um1 = u0;
            u0 = up1;
        }
        cp<R> v = {R(0), R(0)};
        for (int64_t t = n - 1; t >= 0; --t) {
            const int64_t addr = base + t * stride;
            v = cn_back<MODE, R>(from_v<R>(psi[addr]), tab[3 * (t + 1)], v);
            cp<R> w = v;
            if (FLAGS & F_NORM_OUT) nacc += (double)w.re * (double)w.re + (double)w.im * (double)w.im;
            if (FLAGS & F_ADJ_N) w = potential_adjoint<R, MODE, FLAGS>(w, t, state, addr, P, L, acc_w, acc_g);
            psi[addr] = to_v<V>(w);
        }
    }
    write_partials<R, FLAGS>(P, lane, nacc, acc_w, acc_g);
}

// -------------------------------------------------------------- dispatch

template <typename R, int MODE, int FLAGS>
static hipError_t launch_one(const AxisPlan &A, const SweepParams &P, bool exact, bool transposed, const void *tab,
                             hipStream_t s)
{
    using V = typename CT<R>::V;
    const unsigned grid = (unsigned)((A.nlines + kLanes - 1) / kLanes);
    if (exact) {
        hipLaunchKernelGGL((k_sweep_exact<R, MODE, FLAGS>), dim3(grid), dim3(kLanes), 0, s, P,
                           (V *)P.psi, (const V *)tab, (const V *)P.state);
    } else if (transposed) {
        const size_t lds = ((size_t)A.L * kLanes + (size_t)kLanes * kTilePitch) * sizeof(V);
        hipLaunchKernelGGL((k_sweep_window<R, MODE, FLAGS, kTransposed>), dim3(grid), dim3(kLanes), lds, s, P,
                           (V *)P.psi, (const V *)tab, (const V *)P.state);
    } else {
        const size_t lds = (size_t)A.L * kLanes * sizeof(V);
        hipLaunchKernelGGL((k_sweep_window<R, MODE, FLAGS, kStrided>), dim3(grid), dim3(kLanes), lds, s, P,
                           (V *)P.psi, (const V *)tab, (const V *)P.state);
    }
    return hipGetLastError();
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

int64_t sweep_groups(const gp_plan *p, int axis)
{
    return (p->ax[axis].nlines + kLanes - 1) / kLanes;
}

void omega_at_step(const gp_plan *p, int64_t step, double w[3])
{
    for (int a = 0; a < 3; ++a) w[a] = a < p->ndim ? p->omega[a] : 0.0;
    if (!p->sched.empty() && step >= 0 && step < (int64_t)p->sched.size()) w[p->sched_axis] = p->sched[step];
}

hipError_t launch_sweep(gp_plan *p, int axis, void *psi, int flags, bool adjoint, int64_t step_index,
                        const void *state, hipStream_t s)
{
    const AxisPlan &A = p->ax[axis];
    SweepParams P{};
    P.psi = psi;
    P.state = state;
    P.n = A.n;
    P.stride = A.stride;
    P.nlines = A.nlines;
    P.m1 = A.m1;
    P.s1 = A.s1;
    P.s2 = A.s2;
    P.K = A.K < 0 ? 0 : A.K;
    P.lmask = A.L > 0 ? A.L - 1 : 0;
    P.D = A.D;
    P.nblocks = (int)((A.n + kBlock - 1) / kBlock);
    P.dt = p->dt;
    P.g = p->g;
    double w[3];
    omega_at_step(p, step_index, w);
    for (int a = 0; a < 3; ++a) {
        P.hw2[a] = a < p->ndim ? 0.5 * w[a] * w[a] : 0.0;
        P.x0[a] = a < p->ndim ? coord0(p->n[a]) : 0.0;
        P.dx[a] = a < p->ndim ? p->dx[a] : 0.0;
    }
    P.ny = p->ndim >= 2 ? p->n[1] : 1;
    P.sched_axis = p->sched_axis;
    const int parity = (int)(step_index & 1);
    P.norm_in = p->d_norm + (1 - parity) * p->n_norm;
    P.nnorm_in = (int)sweep_groups(p, p->ndim - 1);
    P.dV = p->dV;
    P.norm_out = p->d_norm + parity * p->n_norm;
    P.adj_out = p->d_adj;
    const bool exact = A.K < 0;
    // x lines are contiguous: coalesce through the LDS tile when ring + tile fit
    const size_t tr_lds = ((size_t)A.L * kLanes + (size_t)kLanes * kTilePitch) * elem_bytes(p->prec);
    const bool tr = axis == 0 && tr_lds <= (size_t)kMaxLdsBytes;
    const void *tab = adjoint ? A.d_tab_adj : A.d_tab;
    int kind = exact ? K_SWEEP_EXACT : (axis == 0 ? K_SWEEP_X : (axis == 1 ? K_SWEEP_Y : K_SWEEP_Z));
    if (flags & F_ADJ_N) kind = K_ADJ_X;
    else if (adjoint) kind = K_ADJ_YZ;
    timing_begin(p, kind, s);
    hipError_t e;
    if (p->prec == GP_C128)
        e = p->mode == GP_IMAG ? dispatch_flags<double, GP_IMAG>(A, P, flags, exact, tr, tab, s)
                               : dispatch_flags<double, GP_REAL>(A, P, flags, exact, tr, tab, s);
    else
        e = p->mode == GP_IMAG ? dispatch_flags<float, GP_IMAG>(A, P, flags, exact, tr, tab, s)
                               : dispatch_flags<float, GP_REAL>(A, P, flags, exact, tr, tab, s);
    timing_end(p, s);
    return e;
}

}  // namespace gp

// x sweep (contiguous axis): one wavefront per grid line, shared by the x kernel
// and the batched kernels.
//
// Each lane solves Q = n/64 (rounded up to a power of two) consecutive points
// of the line.  Global loads and stores are coalesced instead (lane L moves
// points L + 64 i, so each instruction covers one contiguous 1 KB / 512 B row
// of the line), and a per-wavefront LDS buffer transposes between the two
// layouts; lane-strided global access would touch four times as many cache
// lines per instruction and caps streaming well below the coalesced rate.  The
// buffer holds 64 (Q + 1) values with one pad slot after every Q, which keeps
// both access patterns free of bank conflicts.
//
// The two Thomas recurrences of the scaled CN system are first-order affine
// recurrences along the line,
//     forward   y_p = -c'_p y_{p-1} + c'_p rhs_p,
//     backward  u'_p = -c'_p u'_{p+1} + y_p,
// so each lane composes the affine maps of its Q points into one map, the
// lanes combine their maps with a Hillis-Steele scan over shuffles, and each
// lane then applies its incoming carry to its own points.  A scan of S steps
// lets a carry travel Q 2^S points; the influence of points further away is
// multiplied by prod |c'| <= rho^(Q 2^S), and the host picks S as the smallest
// with Q 2^S > K (the same bound as the windowed solver) -- S = 6 is the full
// scan and exact.  The potential substep is applied to the loaded values, and
// the norm / adjoint epilogues to the stored ones (both in the coalesced
// layout), as in the other sweeps.
#pragma once

#include <type_traits>

#include "gp_sweep_common.h"

namespace gp {

constexpr int kXWaves = kXWavesPerGroup;  // lines (wavefronts) per workgroup

// Bytes of one wavefront's transpose buffer for Q points per lane.
template <typename R> __host__ __device__ constexpr size_t x_lds_bytes(int Q)
{
    return (size_t)kLanes * (Q + 1) * sizeof(typename CT<R>::V);
}

// Orders one wavefront's LDS accesses (its lanes exchange values through LDS).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename R> __device__ __forceinline__ cp<R> cmul(cp<R> a, cp<R> b)
{
    return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
template <typename R> __device__ __forceinline__ cp<R> cfma(cp<R> a, cp<R> b, cp<R> c)  // a*b + c
{
    return {fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}
// Products with a CN coefficient or scan multiplier k.  In imaginary time
// every coefficient is real (c', beta and their products), so only k.re is
// used there: half the registers and arithmetic of a complex product.
template <int MODE, typename R> __device__ __forceinline__ cp<R> kmul(cp<R> k, cp<R> v)
{
    if (MODE == GP_IMAG) return {k.re * v.re, k.re * v.im};
    return cmul(k, v);
}
template <int MODE, typename R> __device__ __forceinline__ cp<R> kfma(cp<R> k, cp<R> v, cp<R> w)  // k*v + w
{
    if (MODE == GP_IMAG) return {fma(k.re, v.re, w.re), fma(k.re, v.im, w.im)};
    return cfma(k, v, w);
}
// Whole-wavefront shifts by one lane as DPP moves (wave_shr:1 / wave_shl:1): a
// VALU operation instead of an LDS permute round trip, on the scan's critical
// chain.  The lane shifted in from outside the wavefront receives 0 (callers
// discard or zero those lanes anyway).
__device__ __forceinline__ int dpp_shr1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, false); }
__device__ __forceinline__ int dpp_shl1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, false); }

template <bool UP> __device__ __forceinline__ double dpp_shift1(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = (int)(b & 0xffffffffLL), hi = (int)(b >> 32);
    const int slo = UP ? dpp_shr1(lo) : dpp_shl1(lo), shi = UP ? dpp_shr1(hi) : dpp_shl1(hi);
    return __longlong_as_double(((long long)shi << 32) | (long long)(unsigned)slo);
}
template <bool UP> __device__ __forceinline__ float dpp_shift1(float v)
{
    const int b = __float_as_int(v);
    return __int_as_float(UP ? dpp_shr1(b) : dpp_shl1(b));
}

// Lane L receives lane L - d (UP) or L + d: shifts of 1, 2 and 4 lanes are that
// many DPP moves, longer ones a permute.  d is a compile-time constant wherever
// these are used in unrolled loops, so the branch folds away.
template <bool UP, typename R> __device__ __forceinline__ R lane_shift(R v, int d)
{
    if (d == 1 || d == 2 || d == 4) {
        for (int k = 0; k < d; ++k) v = dpp_shift1<UP>(v);
        return v;
    }
    return UP ? __shfl_up(v, d, kLanes) : __shfl_down(v, d, kLanes);
}
template <typename R> __device__ __forceinline__ cp<R> shfl_up_c(cp<R> v, int d)
{
    return {lane_shift<true>(v.re, d), lane_shift<true>(v.im, d)};
}
template <typename R> __device__ __forceinline__ cp<R> shfl_down_c(cp<R> v, int d)
{
    return {lane_shift<false>(v.re, d), lane_shift<false>(v.im, d)};
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

// Line `line` (clamped to the last line), coalesced: lane L gets points
// L + 64 i (clamped to the last point).  Loads are unconditional from in-bounds
// addresses and the caller zeroes points past n when it uses them: a load under
// a branch, or a select right after it, would make the wavefront wait for it
// at once, the prefetched line included.
template <typename R, int Q>
__device__ __forceinline__ void x_load_line(const typename CT<R>::V *src, int64_t line, int64_t nlines, int64_t n,
                                            int lane, typename CT<R>::V (&dst)[Q])
{
    const int64_t lc = line < nlines ? line : nlines - 1;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int64_t q = lane + kLanes * i;
        dst[i] = src[lc * n + (q < n ? q : n - 1)];
    }
}

// Per-lane constants of the x solve: the table rows of the lane's Q points and
// the multipliers of its composed maps before each of the first SMAX scan
// steps (host table xmul: rows s = 0..5 forward, 6..11 backward, one value per
// lane).  Loaded once, ahead of the line loop: loaded at their point of use,
// each multiplier would be one more memory round trip per line, in sequence.
template <typename R, int Q, int SMAX> struct XConsts {
    using V = typename CT<R>::V;
    V c_[Q], b_[Q], blo_[Q];
    V mf[SMAX], mb[SMAX];
    __device__ __forceinline__ V c(int i) const { return c_[i]; }
    __device__ __forceinline__ V b(int i) const { return b_[i]; }
    __device__ __forceinline__ V blo(int i) const { return blo_[i]; }
};

// The same constants with the table rows in LDS, one copy per workgroup (all
// its wavefronts solve lines of one axis): for 16 points per lane the rows
// would take 48 registers (complex64) or 192 (complex128) per lane.  Row k of
// point i of lane L at kc[(k Q + i) 64 + L]: consecutive lanes, no conflicts.
template <typename R, int Q, int SMAX> struct XConstsLds {
    using V = typename CT<R>::V;
    const V *kc;
    int lane;
    V mf[SMAX], mb[SMAX];
    __device__ __forceinline__ V c(int i) const { return kc[(0 * Q + i) * kLanes + lane]; }
    __device__ __forceinline__ V b(int i) const { return kc[(1 * Q + i) * kLanes + lane]; }
    __device__ __forceinline__ V blo(int i) const { return kc[(2 * Q + i) * kLanes + lane]; }
};

// Fills a workgroup's LDS rows (3 Q 64 values) for XConstsLds; the caller
// synchronises the workgroup afterwards.
template <typename R, int Q>
__device__ __forceinline__ void x_rows_to_lds(const SweepParams &P, const typename CT<R>::V *__restrict__ tab,
                                              typename CT<R>::V *kc)
{
    using V = typename CT<R>::V;
    for (int t = threadIdx.x; t < Q * kLanes; t += blockDim.x) {
        const int i = t / kLanes, L = t % kLanes;
        V c, b, blo;
        row_of<R>(P, tab, (int64_t)L * Q + i, c, b, blo);
        kc[(0 * Q + i) * kLanes + L] = c;
        kc[(1 * Q + i) * kLanes + L] = b;
        kc[(2 * Q + i) * kLanes + L] = blo;
    }
}

template <typename R, int Q, int SMAX>
__device__ __forceinline__ void x_mul_load(const SweepParams &P, const typename CT<R>::V *__restrict__ xmul, int lane,
                                           typename CT<R>::V (&mf)[SMAX], typename CT<R>::V (&mb)[SMAX])
{
    const int last = P.scan_steps > 0 ? P.scan_steps - 1 : 0;
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {  // unconditional loads (steps past S are not used)
        const int r = s < last ? s : last;
        mf[s] = xmul[r * kLanes + lane];
        mb[s] = xmul[(6 + r) * kLanes + lane];
    }
}

template <typename R, int Q, int SMAX>
__device__ __forceinline__ void x_consts_load(const SweepParams &P, const typename CT<R>::V *__restrict__ tab,
                                              const typename CT<R>::V *__restrict__ xmul, int lane,
                                              XConsts<R, Q, SMAX> &K)
{
    const int64_t q0 = (int64_t)lane * Q;
#pragma unroll
    for (int i = 0; i < Q; ++i) row_of<R>(P, tab, q0 + i, K.c_[i], K.b_[i], K.blo_[i]);
    x_mul_load<R, Q, SMAX>(P, xmul, lane, K.mf, K.mb);
}

// Solves one line held as Q consecutive points per lane (u, in the potential
// substep's output) and leaves the CN sweep's result in u, same layout.  Data
// moves only through registers and cross-lane shuffles; the table rows come
// from K (XConsts: registers, XConstsLds: the workgroup's LDS copy); S <= SMAX
// scan steps.
template <typename R, int MODE, int Q, int SMAX, typename KC>
__device__ __forceinline__ void x_line_solve(const SweepParams &P, const KC &K, int S, int lane, cp<R> (&u)[Q])
{
    const cp<R> zero = {R(0), R(0)};
    cp<R> left = shfl_up_c(u[Q - 1], 1);
    cp<R> right = shfl_down_c(u[0], 1);
    if (lane == 0) left = zero;
    if (lane == kLanes - 1) right = zero;

    // forward: f_p = c'_p rhs_p = -a_p rhs_p, y_p = a_p y_{p-1} + f_p
    cp<R> f[Q];
    auto ac = [&](int i) -> cp<R> {
        const auto c = K.c(i);
        return {-c.x, MODE == GP_IMAG ? R(0) : -c.y};
    };
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const cp<R> um1 = i == 0 ? left : u[i - 1];
        const cp<R> up1 = i == Q - 1 ? right : u[i + 1];
        const cp<R> rhs = cn_rhs<MODE, R>(um1, u[i], up1, K.b(i), K.blo(i));
        f[i] = kmul<MODE>(from_v<R>(K.c(i)), rhs);
    }
    cp<R> F = f[0];
#pragma unroll
    for (int i = 1; i < Q; ++i) F = kfma<MODE>(ac(i), F, f[i]);
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
        if (s < S) {  // uniform
            const cp<R> Fp = shfl_up_c(F, 1 << s);
            if (lane >= (1 << s)) F = kfma<MODE>(from_v<R>(K.mf[s]), Fp, F);
        }
    }
    cp<R> y = shfl_up_c(F, 1);
    if (lane == 0) y = zero;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        y = kfma<MODE>(ac(i), y, f[i]);
        f[i] = y;
    }
    // backward: u'_p = a_p u'_{p+1} + y_p
    cp<R> G = f[Q - 1];
#pragma unroll
    for (int i = Q - 2; i >= 0; --i) G = kfma<MODE>(ac(i), G, f[i]);
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
        if (s < S) {  // uniform
            const cp<R> Gp = shfl_down_c(G, 1 << s);
            if (lane + (1 << s) < kLanes) G = kfma<MODE>(from_v<R>(K.mb[s]), Gp, G);
        }
    }
    cp<R> v = shfl_down_c(G, 1);
    if (lane == kLanes - 1) v = zero;
#pragma unroll
    for (int i = Q - 1; i >= 0; --i) {
        v = kfma<MODE>(ac(i), v, f[i]);
        u[i] = v;
    }
}

// Each wavefront solves a run of lines in turn.  Everything that depends only
// on the position along the line is computed once: the table rows of the
// lane's points are loaded before the line loop, and the multiplier halves of
// the lane's composed maps at every scan step come precomputed from the host
// (their products involve only the table), so per line only the data halves
// (the F and G of the affine maps) are composed and scanned.

// One wavefront solves lines first .. first+count-1 (those below P.nlines),
// adding its epilogue sums to nacc / acc_w / acc_g.
// xl: this wavefront's LDS buffer of x_lds_bytes<R>(Q) bytes.
// KLDS: the table rows come from the workgroup's LDS copy kc (XConstsLds).
template <typename R, int MODE, int FLAGS, int Q, int SMAX = 6, bool KLDS = false>
__device__ __forceinline__ void x_scan_wave(const SweepParams &P, const typename CT<R>::V *src,
                                            typename CT<R>::V *dst, const typename CT<R>::V *__restrict__ tab,
                                            const typename CT<R>::V *__restrict__ state, int64_t first, int count,
                                            double &nacc, double &acc_w, double &acc_g, typename CT<R>::V *xl,
                                            const typename CT<R>::V *kc = nullptr)
{
    using V = typename CT<R>::V;
    const int lane = threadIdx.x & (kLanes - 1);
    const int64_t n = P.n;
    auto pad = [](int q) { return q + q / Q; };  // slot of point q in xl
    const int S = P.scan_steps;
    const cp<R> zero = {R(0), R(0)};
    std::conditional_t<KLDS, XConstsLds<R, Q, SMAX>, XConsts<R, Q, SMAX>> K;  // scan steps S <= SMAX
    if constexpr (KLDS) {
        K.kc = kc;
        K.lane = lane;
        x_mul_load<R, Q, SMAX>(P, (const V *)P.xmul, lane, K.mf, K.mb);
    } else {
        x_consts_load<R, Q, SMAX>(P, tab, (const V *)P.xmul, lane, K);
    }
    const double renorm = (FLAGS & F_RENORM) ? 1.0 / sqrt(P.dV * P.norm_total[0]) : 1.0;
    V nxt[Q];  // the next line's values, loaded while the current one is solved
    x_load_line<R, Q>(src, first, P.nlines, n, lane, nxt);
#pragma unroll 1
    for (int li = 0; li < count; ++li) {
        const int64_t line = first + li;
        if (line >= P.nlines) break;  // uniform across the wavefront
        const int64_t base = line * n;
        LineCtx<R> L = line_ctx_of<R>(P, line);
        if (FLAGS & F_RENORM) L.scale = renorm;

        cp<R> u[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) u[i] = lane + kLanes * i < n ? from_v<R>(nxt[i]) : zero;
        if (FLAGS & F_COPY_IN) {  // the input state, as loaded
#pragma unroll
            for (int i = 0; i < Q; ++i)
                if (lane + kLanes * i < n) ((V *)P.copy_out)[base + lane + kLanes * i] = nxt[i];
        }
        // the adjoint's forward state, requested before the solve so that its
        // latency overlaps it (clamped in-bounds addresses; used below n only)
        V stv[(FLAGS & F_ADJ_N) ? Q : 1];
        if constexpr ((FLAGS & F_ADJ_N) != 0) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int64_t q = lane + kLanes * i;
                stv[i] = state[base + (q < n ? q : n - 1)];
            }
        }
        if (li + 1 < count) {
            const int64_t nl = line + 1;
            x_load_line<R, Q>(src, nl, P.nlines, n, lane, nxt);
        }
        // points past the line's end are zeros and stay zeros
        if (FLAGS & F_FUSE_N) potential_substep_q<R, MODE, FLAGS, Q>(u, lane, kLanes, P, L);
        if (Q > 1) {  // coalesced -> Q consecutive points per lane
#pragma unroll
            for (int i = 0; i < Q; ++i) xl[pad(lane + kLanes * i)] = to_v<V>(u[i]);
            wave_lds_sync();
#pragma unroll
            for (int i = 0; i < Q; ++i) u[i] = from_v<R>(xl[pad(lane * Q + i)]);
        }
        x_line_solve<R, MODE, Q, SMAX>(P, K, S, lane, u);
        if (Q > 1) {  // back to the coalesced layout
#pragma unroll
            for (int i = 0; i < Q; ++i) xl[pad(lane * Q + i)] = to_v<V>(u[i]);
            wave_lds_sync();
#pragma unroll
            for (int i = 0; i < Q; ++i) u[i] = from_v<R>(xl[pad(lane + kLanes * i)]);
            wave_lds_sync();
        }
        if constexpr ((FLAGS & F_ADJ_N) != 0)
            potential_adjoint_q<R, MODE, FLAGS, Q>(u, stv, lane, kLanes, n, P, L, acc_w, acc_g);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int64_t q = lane + kLanes * i;
            if (q < n) {
                const cp<R> w = u[i];
                if (FLAGS & F_NORM_OUT) nacc += (double)w.re * (double)w.re + (double)w.im * (double)w.im;
                dst[base + q] = to_v<V>(w);
            }
        }
    }
}

// The same scan solver on a strided axis (a 2D grid's y lines): one wavefront
// per line, lane L loading points L Q .. L Q + Q - 1 straight into the
// solver's layout (no transpose), at stride P.stride from the line's base.
// Each load touches one point of 64 rows; the wavefronts of a workgroup take
// neighbouring lines at the same time (line first + w + lstep li for
// wavefront w), so they share the cache lines of those rows.  No potential
// substep (the x sweep carries it); F_NORM_OUT sums |u'|^2 into nacc.
template <typename R, int Q>
__device__ __forceinline__ void col_load_line(const typename CT<R>::V *src, const SweepParams &P, int64_t line,
                                              int lane, typename CT<R>::V (&dst)[Q])
{
    const int64_t lc = line < P.nlines ? line : P.nlines - 1;
    const int64_t base = (lc % P.m1) * P.s1 + (lc / P.m1) * P.s2;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int64_t q = (int64_t)lane * Q + i;
        dst[i] = src[base + (q < P.n ? q : P.n - 1) * P.stride];
    }
}

template <typename R, int MODE, int FLAGS, int Q, int SMAX = 6, bool KLDS = false>
__device__ __forceinline__ void col_scan_wave(const SweepParams &P, const typename CT<R>::V *src,
                                              typename CT<R>::V *dst, const typename CT<R>::V *__restrict__ tab,
                                              int64_t first, int count, int64_t lstep, double &nacc,
                                              const typename CT<R>::V *kc = nullptr)
{
    using V = typename CT<R>::V;
    const int lane = threadIdx.x & (kLanes - 1);
    const int64_t n = P.n;
    const cp<R> zero = {R(0), R(0)};
    std::conditional_t<KLDS, XConstsLds<R, Q, SMAX>, XConsts<R, Q, SMAX>> K;
    if constexpr (KLDS) {
        K.kc = kc;
        K.lane = lane;
        x_mul_load<R, Q, SMAX>(P, (const V *)P.xmul, lane, K.mf, K.mb);
    } else {
        x_consts_load<R, Q, SMAX>(P, tab, (const V *)P.xmul, lane, K);
    }
    V nxt[Q];
    col_load_line<R, Q>(src, P, first, lane, nxt);
#pragma unroll 1
    for (int li = 0; li < count; ++li) {
        const int64_t line = first + li * lstep;
        if (line >= P.nlines) break;  // uniform across the wavefront
        const int64_t base = (line % P.m1) * P.s1 + (line / P.m1) * P.s2;
        cp<R> u[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) u[i] = (int64_t)lane * Q + i < n ? from_v<R>(nxt[i]) : zero;
        if (li + 1 < count) col_load_line<R, Q>(src, P, line + lstep, lane, nxt);
        x_line_solve<R, MODE, Q, SMAX>(P, K, P.scan_steps, lane, u);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int64_t q = (int64_t)lane * Q + i;
            if (q < n) {
                if (FLAGS & F_NORM_OUT)
                    nacc += (double)u[i].re * (double)u[i].re + (double)u[i].im * (double)u[i].im;
                dst[base + q * P.stride] = to_v<V>(u[i]);
            }
        }
    }
}

// Strided lines in tiles: one wavefront loads a tile of T neighbouring lines
// (T values = 32 bytes of each row, so four such tiles fill a 128-byte cache
// line) with every load instruction covering 64/T rows, keeps it in LDS in the
// solver's padded layout, solves the tile's lines one after another from LDS
// and stores the tile back the same way.  Against one line per load pass this
// reads each row segment once per tile instead of once per line.  Lines first ..
// first + count - 1 (those below P.nlines), T at a time; lds: this wavefront's
// col_tile_lds_bytes<R>(Q) bytes.  F_NORM_OUT sums |u'|^2 into nacc.
template <typename R> __host__ __device__ constexpr int col_tile_lines() { return 32 / (int)sizeof(typename CT<R>::V); }
// One line's LDS slots: the padded layout plus one value, so that the T lines'
// slots of a row fall in different banks.
__host__ __device__ constexpr int col_tile_stride(int Q) { return kLanes * (Q + 1) + 1; }
template <typename R> __host__ __device__ constexpr size_t col_tile_lds_bytes(int Q)
{
    return (size_t)col_tile_lines<R>() * col_tile_stride(Q) * sizeof(typename CT<R>::V);
}

template <typename R, int MODE, int FLAGS, int Q, int SMAX = 6>
__device__ __forceinline__ void col_tile_wave(const SweepParams &P, const typename CT<R>::V *src,
                                              typename CT<R>::V *dst, const typename CT<R>::V *__restrict__ tab,
                                              int64_t first, int count, double &nacc, typename CT<R>::V *lds)
{
    using V = typename CT<R>::V;
    constexpr int T = col_tile_lines<R>();
    constexpr int RPI = kLanes / T;         // rows per load instruction
    constexpr int NLD = kLanes * Q / RPI;   // load instructions per tile (rows 0 .. 64 Q - 1)
    constexpr int LSTR = col_tile_stride(Q);  // LDS values per line
    const int lane = threadIdx.x & (kLanes - 1);
    const int lc = lane % T, lr = lane / T;
    const int64_t n = P.n;
    const cp<R> zero = {R(0), R(0)};
    XConsts<R, Q, SMAX> K;
    x_consts_load<R, Q, SMAX>(P, tab, (const V *)P.xmul, lane, K);
#pragma unroll 1
    for (int c0 = 0; c0 < count; c0 += T) {
        const int64_t line = first + c0 + lc;
        const bool mine = c0 + lc < count && line < P.nlines;  // this lane's line of the tile exists
        const int64_t lcl = line < P.nlines ? line : P.nlines - 1;
        const int64_t base = (lcl % P.m1) * P.s1 + (lcl / P.m1) * P.s2;
        V *col = lds + lc * LSTR;
        // loads in groups of 128 bytes per lane (16 complex64 or 8 complex128
        // values), all in flight together: a full unroll would hold the whole
        // tile in registers next to the solver's constants
        constexpr int GRP = NLD < 128 / (int)sizeof(V) ? NLD : 128 / (int)sizeof(V);
#pragma unroll 1
        for (int k0 = 0; k0 < NLD; k0 += GRP) {
            V v[GRP];
#pragma unroll
            for (int k = 0; k < GRP; ++k) {  // rows past the line's end are zeros
                const int r = lr + RPI * (k0 + k);
                v[k] = src[base + (r < n ? r : n - 1) * P.stride];
            }
#pragma unroll
            for (int k = 0; k < GRP; ++k) {
                const int r = lr + RPI * (k0 + k);
                col[r + r / Q] = r < n ? v[k] : to_v<V>(zero);
            }
        }
        wave_lds_sync();
        int nt = count - c0 < T ? count - c0 : T;  // lines of this tile
        if (P.nlines - (first + c0) < nt) nt = (int)(P.nlines - (first + c0));
#pragma unroll 1
        for (int c = 0; c < nt; ++c) {
            V *cl = lds + c * LSTR;
            cp<R> u[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) u[i] = from_v<R>(cl[lane * (Q + 1) + i]);
            x_line_solve<R, MODE, Q, SMAX>(P, K, P.scan_steps, lane, u);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                cl[lane * (Q + 1) + i] = to_v<V>(u[i]);
                if ((FLAGS & F_NORM_OUT) && (int64_t)lane * Q + i < n)
                    nacc += (double)u[i].re * (double)u[i].re + (double)u[i].im * (double)u[i].im;
            }
        }
        wave_lds_sync();
        if (mine) {
#pragma unroll 8
            for (int k = 0; k < NLD; ++k) {
                const int r = lr + RPI * k;
                if (r < n) dst[base + r * P.stride] = col[r + r / Q];
            }
        }
        wave_lds_sync();  // the next tile's loads overwrite these slots
    }
}

}  // namespace gp

// Windowed streaming line solver of the strided sweeps (one wavefront, one
// line per lane), shared by the per-axis kernels and the batched kernels.
#pragma once

#include "gp_sweep_common.h"

namespace gp {

enum Access { kStrided = 0, kTransposed = 1 };

// One wavefront streaming its 64 lines (one per lane) in blocks of BB points.
// A line may be split into `segs` segments: segment s writes the
// output blocks [s nb/segs, (s+1) nb/segs) and starts its forward elimination
// DW blocks earlier from y = 0 -- after at least K + 1 recurrence steps that
// start has decayed below the window bound, as in the back substitution.
template <typename R, int MODE, int FLAGS, int ACC, int DW, int BB> struct WindowSweep {
    using V = typename CT<R>::V;
    static constexpr int B = BB;
    static constexpr int kPitch = BB + 1;  // tile row pitch in values: conflict-free b128 access
    const SweepParams &P;
    const V *src;  // input grid (may equal dst: each point is read before it is written)
    V *dst;        // output grid
    const V *__restrict__ tab;
    const V *__restrict__ state;
    V *ring;
    V *tile;
    LineCtx<R> L;
    int lane;
    int64_t n, stride, base, l0;
    int lmask;
    int o_lo, o_hi;  // output blocks of this segment
    int64_t part;    // partial slot of this wavefront's epilogue sums
    cp<R> um1, u0, dprev;
    double nacc, acc_w, acc_g;

    // group: which 64 lines; s of segs: which part of them; lds: this wavefront's ring (+ tile)
    __device__ __forceinline__ WindowSweep(const SweepParams &P_, const V *src_, V *dst_, const V *tab_,
                                           const V *state_, char *lds, int64_t group, int s, int segs,
                                           int64_t part_)
        : P(P_), src(src_), dst(dst_), tab(tab_), state(state_), part(part_)
    {
        lane = threadIdx.x & (kLanes - 1);
        L = line_setup<R, FLAGS>(P, group, lane);
        n = P.n;
        stride = P.stride;
        base = L.base;
        l0 = group * kLanes;
        lmask = P.lmask;
        ring = reinterpret_cast<V *>(lds);
        tile = ring + (size_t)(lmask + 1) * kLanes;
        const int nb = P.nblocks;
        o_lo = (int)((int64_t)s * nb / segs);
        o_hi = (int)((int64_t)(s + 1) * nb / segs);
        um1 = u0 = dprev = cp<R>{R(0), R(0)};
        nacc = acc_w = acc_g = 0.0;
    }

    __device__ __forceinline__ static V zero() { return to_v<V>(cp<R>{R(0), R(0)}); }

    __device__ __forceinline__ V load_point(int64_t q) const
    {
        return (L.active && q >= 0 && q < n) ? src[base + q * stride] : zero();
    }

    // Values u_{q-2}, u_{q-1} before the first eliminated point of block j0.
    __device__ __forceinline__ void start(int j0)
    {
        if (j0 == 0) return;  // ghosts
        const int64_t q = (int64_t)j0 * B;
        um1 = from_v<R>(load_point(q - 2));
        u0 = from_v<R>(load_point(q - 1));
        if (FLAGS & F_FUSE_N) {
            um1 = potential_substep<R, MODE, FLAGS>(um1, q - 2, P, L);
            u0 = potential_substep<R, MODE, FLAGS>(u0, q - 1, P, L);
        }
    }

    // Issue the loads of block j.  Every lane loads unconditionally from an
    // in-bounds address (point index clamped to the line, inactive lanes on
    // line 0); what lies outside the grid is zeroed only when the block is
    // used (process).  Loads under branches, or a select right after them,
    // would make the wavefront wait for them at once, the prefetched block
    // included.
    __device__ __forceinline__ void load(V (&buf)[B], int j) const
    {
        const int64_t q0 = (int64_t)j * B;
        if (ACC == kStrided) {
#pragma unroll
            for (int k = 0; k < B; ++k) {
                const int64_t q = q0 + k;
                buf[k] = src[base + (q < n ? q : n - 1) * stride];
            }
        } else {
            const int pt = lane & (B - 1);
            const int64_t q = q0 + pt;
#pragma unroll
            for (int i = 0; i < B; ++i) {
                const int64_t line = l0 + i * (kLanes / B) + lane / B;
                buf[i] = src[(line < P.nlines ? line : P.nlines - 1) * n + (q < n ? q : n - 1)];
            }
        }
    }

    // Whether the value load() put in slot k of block j lies on the grid.
    __device__ __forceinline__ bool loaded_ok(int j, int k) const
    {
        if (ACC == kStrided) return L.active && (int64_t)j * B + k < n;
        const int64_t line = l0 + k * (kLanes / B) + lane / B;
        return line < P.nlines && (int64_t)j * B + (lane & (B - 1)) < n;
    }

    // Solve block j (values in buf, as load() left them; MASKED = false when the
    // caller supplies values already zero off the grid) and write output block
    // j - DW if this segment owns it.
    template <bool MASKED = true> __device__ __forceinline__ void process(V (&buf)[B], int j)
    {
        V own[B];
        if (ACC == kTransposed) {
#pragma unroll
            for (int i = 0; i < B; ++i)
                tile[(i * (kLanes / B) + lane / B) * kPitch + (lane & (B - 1))] = loaded_ok(j, i) ? buf[i] : zero();
            __syncthreads();
#pragma unroll
            for (int k = 0; k < B; ++k) own[k] = tile[lane * kPitch + k];
            __syncthreads();
        } else {
#pragma unroll
            for (int k = 0; k < B; ++k) own[k] = (!MASKED || loaded_ok(j, k)) ? buf[k] : zero();
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
        // back substitution of output block o = j - DW, window K = DW*B - 1: it
        // starts at the newest eliminated point, jB + B - 2 = ob + (DW+1)B - 2
        const int o = j - DW;
        if (o < o_lo || o >= o_hi) return;
        const int64_t ob = (int64_t)o * B;
        cp<R> v = {R(0), R(0)};
#pragma unroll
        for (int i = (DW + 1) * B - 2; i >= B; --i) {
            const int64_t t = ob + i;
            v = cn_back<MODE, R>(from_v<R>(ring[(int)((t + 1) & lmask) * kLanes + lane]), tab[3 * (t + 1)], v);
        }
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
                    if (L.active) dst[addr] = to_v<V>(w);
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < B; ++k) tile[lane * kPitch + k] = to_v<V>(out[k]);
            __syncthreads();
            const int pt = lane & (B - 1);
            const int64_t t = ob + pt;
#pragma unroll
            for (int i = 0; i < B; ++i) {
                const int lo = i * (kLanes / B) + lane / B;
                const int64_t line = l0 + lo;
                cp<R> w = from_v<R>(tile[lo * kPitch + pt]);
                if (line < P.nlines && t < n) {
                    const int64_t addr = line * n + t;
                    if (FLAGS & F_NORM_OUT) nacc += (double)w.re * (double)w.re + (double)w.im * (double)w.im;
                    if (FLAGS & F_ADJ_N) {
                        const LineCtx<R> Lw = line_ctx_of<R>(P, line);
                        w = potential_adjoint<R, MODE, FLAGS>(w, t, state, addr, P, Lw, acc_w, acc_g);
                    }
                    dst[addr] = to_v<V>(w);
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
        write_partials<R, FLAGS>(P, lane, nacc, acc_w, acc_g, part);
    }
};

// Streaming solver with a windowed back substitution, run by one wavefront.
// The block loop is unrolled by two over ping-pong buffers, so the loads of
// block j+1 stay in flight while block j is solved.
template <typename R, int MODE, int FLAGS, int ACC, int DW, int BB>
__device__ __forceinline__ void window_run(const SweepParams &P, const typename CT<R>::V *src,
                                           typename CT<R>::V *dst, const typename CT<R>::V *tab,
                                           const typename CT<R>::V *state, char *lds, int64_t group, int seg,
                                           int segs, int64_t part)
{
    using V = typename CT<R>::V;
    WindowSweep<R, MODE, FLAGS, ACC, DW, BB> S(P, src, dst, tab, state, lds, group, seg, segs, part);
    const int j0 = S.o_lo - DW > 0 ? S.o_lo - DW : 0;
    const int j1 = S.o_hi + DW;  // exclusive: the last output block o_hi-1 is written at j = o_hi-1+DW
    S.start(j0);
    V a[BB], b[BB];
    S.load(a, j0);
    // the next block's loads are issued unconditionally (past the segment's end
    // they repeat its last block, a cache hit): loads under a branch would make
    // the wavefront wait for all of them before solving the current block
    for (int j = j0; j < j1; j += 2) {
        S.load(b, j + 1 < j1 ? j + 1 : j1 - 1);
        S.process(a, j);
        if (j + 1 >= j1) break;
        S.load(a, j + 2 < j1 ? j + 2 : j1 - 1);
        S.process(b, j + 1);
    }
    S.finish();
}

// LDS bytes of one wavefront's ring (+ transposed tile).
template <typename R, int ACC, int BB> __host__ __device__ constexpr size_t window_lds_bytes(int L)
{
    return ((size_t)L * kLanes + (ACC == kTransposed ? (size_t)kLanes * (BB + 1) : 0)) * sizeof(typename CT<R>::V);
}

}  // namespace gp

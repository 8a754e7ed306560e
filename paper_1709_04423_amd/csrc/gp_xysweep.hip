// The x and y sweeps of a 3D step fused over xy-planes.
//
// The CN substeps along x and y act on one xy-plane at a time, and the y
// sweep's windowed solver consumes rows in order, so the x sweep's output never
// needs to reach HBM: one workgroup walks the rows of one plane (or one segment
// of its rows) in blocks of four.  Each of its four wavefronts x-solves one row
// of the block (potential substep on load, the same affine-scan solve as the x
// kernel) into an LDS tile; then every thread takes one column of the tile and
// advances that column's windowed y solve (the strided-sweep solver with its LDS
// ring), writing finished rows of the y output.  The grid is read once and
// written once for both substeps.
//
// Segments of a plane's rows start their y elimination DW blocks early from
// zero state, like the strided sweeps' segments; the x rows of those warm-up
// blocks are solved again by the segment that needs them.
#include <algorithm>
#include <utility>

#include "gp_internal.h"
#include "gp_sweep_common.h"
#include "gp_window.h"
#include "gp_xscan.h"

namespace gp {

namespace {

constexpr int kXYWaves = 4;  // wavefronts per workgroup = rows per block of the y window
constexpr int kXYAhead = 1;  // blocks whose rows are loaded ahead
constexpr int kXYMaxScan = 3;  // x scan steps the fused kernel supports

// Tile slot of point q of a row, for values of E bytes.  E = 16: the low three
// bits (one 128-byte group) are permuted by the next three, so the coalesced row
// (lane + 64 i), the solver's consecutive points (lane Q + i) and the column
// reads each hit eight distinct 16-byte bank groups per eight lanes.  E = 8:
// the low two bits are permuted by bits 4-5, so each sixteen lanes of those
// patterns hit sixteen distinct 8-byte bank pairs (the 16-byte permutation
// leaves the consecutive-points pattern two-way conflicted there).
template <int E> __device__ __forceinline__ int xy_slot(int q)
{
    if constexpr (E == 8) return q ^ ((q >> 4) & 3);
    return q ^ ((q >> 3) & 7);
}

// Row y = jb B + w of plane k (zeros past the plane or past block j1).
template <typename R, int Q>
__device__ __forceinline__ void xy_load_row(const typename CT<R>::V *src, int jb, int j1, int w, int64_t k,
                                            int64_t nx, int64_t ny, int lane, typename CT<R>::V (&dst_row)[Q])
{
    using V = typename CT<R>::V;
    const int64_t y = (int64_t)jb * kXYWaves + w;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        dst_row[i] = (jb < j1 && y < ny && lane + kLanes * i < nx) ? src[(y + ny * k) * nx + lane + kLanes * i]
                                                                   : to_v<V>(cp<R>{R(0), R(0)});
}

template <typename R, int MODE, int XFLAGS, int Q, int DW>
__global__ __launch_bounds__(kLanes *kXYWaves) void k_sweep_xy(SweepParams PX, SweepParams PY,
                                                                const typename CT<R>::V *src,
                                                                typename CT<R>::V *dst,
                                                                const typename CT<R>::V *__restrict__ tabx,
                                                                const typename CT<R>::V *__restrict__ taby)
{
    using V = typename CT<R>::V;
    constexpr int B = kXYWaves;
    __shared__ V tile[B][kLanes * Q];
    extern __shared__ char ring_raw[];
    const int lane = threadIdx.x & (kLanes - 1);
    // wave-uniform by construction; stated so, the y solver's table rows (whose
    // addresses depend only on the block) are read as scalar loads, outside the
    // vector memory counter that the prefetched rows occupy
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    const int64_t nx = PX.n, ny = PY.n;
    const int64_t k = blockIdx.y;  // plane
    const int cw = (int)(nx / kLanes);  // wavefronts with columns in the y part
    const size_t ringb = (size_t)(PY.lmask + 1) * kLanes * sizeof(V);
    const cp<R> zero = {R(0), R(0)};

    // y solver of this wavefront's 64 columns: y lines l = x + nx k
    WindowSweep<R, MODE, 0, kStrided, DW, 4> Y(PY, nullptr, dst, taby, nullptr, ring_raw + w * ringb,
                                                k * cw + w, (int)blockIdx.x, (int)gridDim.x, 0);
    const int j0 = Y.o_lo - DW > 0 ? Y.o_lo - DW : 0;
    const int j1 = Y.o_hi + DW;  // exclusive; uniform over the workgroup

    const int S = PX.scan_steps;  // at most kXYMaxScan (checked on the host)
    XConsts<R, Q, kXYMaxScan> KX;
    x_consts_load<R, Q, kXYMaxScan>(PX, tabx, (const V *)PX.xmul, lane, KX);
    const double renorm = (XFLAGS & F_RENORM) ? 1.0 / sqrt(PX.dV * PX.norm_total[0]) : 1.0;
    // this wavefront's rows of the next kXYAhead blocks stay in flight while a
    // block is solved (one slot per block; the loop is unrolled over the slots so
    // every slot index is a compile-time constant)
    V ahead[kXYAhead][Q];
#pragma unroll
    for (int t = 0; t < kXYAhead; ++t) xy_load_row<R, Q>(src, j0 + t, j1, w, k, nx, ny, lane, ahead[t]);
    V *row = tile[w];
#pragma unroll 1
    for (int jb = j0; jb < j1; jb += kXYAhead) {
#pragma unroll
        for (int t = 0; t < kXYAhead; ++t) {
            const int j = jb + t;
            if (j >= j1) break;  // uniform over the workgroup
            const int64_t y = (int64_t)j * B + w;
            cp<R> u[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) u[i] = from_v<R>(ahead[t][i]);
            if (y < ny) {  // uniform over the wavefront
                LineCtx<R> L = line_ctx_of<R>(PX, y + ny * k);
                if (XFLAGS & F_RENORM) L.scale = renorm;
                // points past the row's end are zeros and stay zeros
                if (XFLAGS & F_FUSE_N) potential_substep_q<R, MODE, XFLAGS, Q>(u, lane, kLanes, PX, L);
                if (Q > 1) {  // coalesced -> Q consecutive points per lane
#pragma unroll
                    for (int i = 0; i < Q; ++i) row[xy_slot<(int)sizeof(V)>(lane + kLanes * i)] = to_v<V>(u[i]);
                    wave_lds_sync();
#pragma unroll
                    for (int i = 0; i < Q; ++i) u[i] = from_v<R>(row[xy_slot<(int)sizeof(V)>(lane * Q + i)]);
                }
                x_line_solve<R, MODE, Q, kXYMaxScan>(PX, KX, S, lane, u);
#pragma unroll
                for (int i = 0; i < Q; ++i) row[xy_slot<(int)sizeof(V)>(lane * Q + i)] = to_v<V>(u[i]);
            } else {  // rows past the plane are the y solver's zero rows
#pragma unroll
                for (int i = 0; i < Q; ++i) row[xy_slot<(int)sizeof(V)>(lane * Q + i)] = to_v<V>(zero);
            }
            // the next rows are requested only now: the vector memory counter is
            // in order, so waiting for the x solve's table loads would otherwise
            // wait for them too
            xy_load_row<R, Q>(src, j + kXYAhead, j1, w, k, nx, ny, lane, ahead[t]);
            __syncthreads();
            if (w < cw) {
                V buf[B];
#pragma unroll
                for (int r = 0; r < B; ++r) buf[r] = tile[r][xy_slot<(int)sizeof(V)>(w * kLanes + lane)];
                Y.template process<false>(buf, j);  // tile rows are zero off the grid
            }
            __syncthreads();
        }
    }
}

// f(integral_constant<int, 0>) .. f(integral_constant<int, N-1>), in order: a loop
// whose index is a compile-time constant in every copy.
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F> __device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// y solver of one column (one lane) with its elimination window in registers:
// the window holds the eliminated values of the last DW + 1 blocks of four rows,
// and the block loop is unrolled by DW + 1 so block j's values live in slot
// u = (j - j0) mod (DW + 1), a compile-time index in every unrolled copy.
// The elimination is WindowSweep::process's (same order, same table rows), only
// the ring moved from LDS to registers.  Away from the line's start and end
// every table row a block touches is the constant row (the Thomas factors have
// converged to rounding: rows of points q_const .. n-1 are equal bit for bit),
// and CR = true takes it from registers instead of the table: no loads and no
// waits for them in the steady state.  With a constant c' the windowed back
// substitution also splits by blocks: x_{mB} = S_m + (-c')^B x_{(m+1)B}, where
// S_m (the block's back substitution from a zero after it) is formed once when
// block m is eliminated.  The output block then costs DW - 1 of those steps and
// B - 1 single-point steps instead of (DW + 1) B - 1 of the latter -- the same
// truncated window, summed in another order.  SUMS selects it; the kernel uses
// it in complex128 only -- in complex64 the reordered sums bias the long-run
// observables (after 2000 imaginary and 2000 real steps at 256^3 the chemical
// potential moves 4e-6 from the FP64 result instead of 3e-7) -- and in real
// time only for rows of up to 128 points: with 4 points per lane the DW + 1
// sums would push the kernel past 256 registers (one wavefront per SIMD).
template <typename R, int MODE, int DW, bool SUMS> struct YRegSolver {
    using V = typename CT<R>::V;
    static constexpr int B = kXYWaves;
    static constexpr bool kSums = SUMS;
    cp<R> d[DW + 1][B];
    cp<R> bs[kSums ? DW + 1 : 1];  // S_m of the block in each slot
    cp<R> um1, u0, dprev;
    int o_lo, o_hi;
    int64_t base, stride, n;
    V rc, rb, rblo;  // the constant row (c', beta, beta_lo)
    cp<R> cB;        // (-c')^B

    // field k of table row t (row t belongs to point t - 1)
    template <bool CR> __device__ __forceinline__ V row(const V *__restrict__ tab, int64_t t, int k) const
    {
        if constexpr (CR) return k == 0 ? rc : (k == 1 ? rb : rblo);
        return tab[3 * t + k];
    }

    // whether block j's rows are all the constant row: elimination rows jB ..
    // jB+B-1 and back-substitution rows (j-DW)B+1 .. jB+B-1 within q_const+1 .. n
    __device__ __forceinline__ static bool const_rows(int j, int64_t q_const, int64_t n)
    {
        return (int64_t)(j - DW) * B >= q_const && (int64_t)j * B + B - 1 <= n;
    }

    // block j (rows jB .. jB+3 in v), stored in slot U; writes output block j - DW
    template <int U, bool CR>
    __device__ __forceinline__ void process(const cp<R> (&v)[B], int j, const V *__restrict__ tab, V *dst)
    {
        static_for<B>([&](auto K) {  // eliminated point p = jB + K - 1, table row q = p + 1
            constexpr int k = decltype(K)::value;
            const int64_t q = (int64_t)j * B + k;
            const cp<R> rhs = cn_rhs<MODE, R>(um1, u0, v[k], row<CR>(tab, q, 1), row<CR>(tab, q, 2));
            const cp<R> e = cn_elim<MODE, R>(rhs, dprev, row<CR>(tab, q, 0));
            d[U][k] = e;
            dprev = e;
            um1 = u0;
            u0 = v[k];
        });
        if constexpr (kSums) {  // S_j with the constant c' (used only where every row is)
            cp<R> sj = d[U][B - 1];
            static_for<B - 1>([&](auto I) { sj = cn_back<MODE, R>(d[U][B - 2 - decltype(I)::value], rc, sj); });
            bs[U] = sj;
        }
        const int o = j - DW;
        if (o < o_lo || o >= o_hi) return;  // uniform
        const int64_t ob = (int64_t)o * B;
        cp<R> out[B];
        if constexpr (CR && kSums) {
            // x_{(o+1)B} = S_{o+1} + (-c')^B (S_{o+2} + ... (-c')^B S_j); block j - i is
            // in slot (U + DW + 1 - i) mod (DW + 1)
            cp<R> x = bs[U];
            static_for<DW - 1>([&](auto I) {
                constexpr int i = decltype(I)::value + 1;
                x = kfma<MODE>(cB, x, bs[(U + DW + 1 - i) % (DW + 1)]);
            });
            out[B - 1] = x;
            constexpr int so = (U + 1) % (DW + 1);  // block o
            static_for<B - 1>([&](auto I) {
                constexpr int k = B - 2 - decltype(I)::value;
                x = cn_back<MODE, R>(d[so][k + 1], rc, x);
                out[k] = x;
            });
        } else {
            cp<R> x = {R(0), R(0)};
            // q = t + 1 from ob + (DW+1)B - 1 down to ob + 1; block (q - ob) / B of the
            // window is slot (U + 1 + (q - ob) / B) mod (DW + 1).  Expanded as a fold
            // so every slot index is a constant (a rolled loop would put d in scratch).
            constexpr int L = (DW + 1) * B - 1;
            static_for<L>([&](auto I) {
                constexpr int i = L - decltype(I)::value;
                x = cn_back<MODE, R>(d[(U + 1 + i / B) % (DW + 1)][i % B], row<CR>(tab, ob + i, 0), x);
                if constexpr (i <= B) out[i - 1] = x;
            });
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int64_t t = ob + k;
            if (t < n) dst[base + t * stride] = to_v<V>(out[k]);
        }
    }
};

template <typename R, int MODE, int XFLAGS, int Q, int DW>
__global__ __launch_bounds__(kLanes *kXYWaves) void k_sweep_xy_reg(SweepParams PX, SweepParams PY,
                                                                    const typename CT<R>::V *src,
                                                                    typename CT<R>::V *dst,
                                                                    const typename CT<R>::V *__restrict__ tabx,
                                                                    const typename CT<R>::V *__restrict__ taby)
{
    using V = typename CT<R>::V;
    constexpr int B = kXYWaves;
    __shared__ V tile[2][B][kLanes * Q];
    const int lane = threadIdx.x & (kLanes - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    const int64_t nx = PX.n, ny = PY.n;
    const int64_t k = blockIdx.y;
    const int cw = (int)(nx / kLanes);
    const cp<R> zero = {R(0), R(0)};

    constexpr bool kYSums = sizeof(R) == 8 && (MODE == GP_IMAG || Q <= 2);
    YRegSolver<R, MODE, DW, kYSums> Y;
    {
        const int nb = PY.nblocks, segs = (int)gridDim.x, sg = (int)blockIdx.x;
        Y.o_lo = (int)((int64_t)sg * nb / segs);
        Y.o_hi = (int)((int64_t)(sg + 1) * nb / segs);
        Y.um1 = Y.u0 = Y.dprev = zero;
        Y.base = (int64_t)(w * kLanes + lane) + nx * ny * k;
        Y.stride = nx;
        Y.n = ny;
        Y.rc = V{R(PY.c_inf[0]), R(PY.c_inf[1])};
        Y.rb = V{R(PY.b_inf[0]), R(PY.b_inf[1])};
        Y.rblo = V{R(PY.b_inf[2]), R(0)};
        const cp<R> mc = {-Y.rc.x, -Y.rc.y};
        Y.cB = mc;
        for (int b = 1; b < B; ++b) Y.cB = cmul(Y.cB, mc);
    }
    const int j0 = Y.o_lo - DW > 0 ? Y.o_lo - DW : 0;
    const int j1 = Y.o_hi + DW;  // exclusive, uniform over the workgroup

    const int S = PX.scan_steps;
    XConsts<R, Q, kXYMaxScan> KX;
    x_consts_load<R, Q, kXYMaxScan>(PX, tabx, (const V *)PX.xmul, lane, KX);
    const double renorm = (XFLAGS & F_RENORM) ? 1.0 / sqrt(PX.dV * PX.norm_total[0]) : 1.0;

    // x-solve this wavefront's row of block j into tile[j & 1] (rows past the
    // plane, or blocks past j1, are zero rows), from values `in` loaded earlier
    auto x_row = [&](int j, V (&in)[Q]) {
        V *row = tile[j & 1][w];
        const int64_t y = (int64_t)j * B + w;
        if (j < j1 && y < ny) {  // uniform over the wavefront
            cp<R> u[Q];
            LineCtx<R> L = line_ctx_of<R>(PX, y + ny * k);
            if (XFLAGS & F_RENORM) L.scale = renorm;
#pragma unroll
            for (int i = 0; i < Q; ++i) u[i] = from_v<R>(in[i]);
            // points past the row's end are zeros and stay zeros
            if (XFLAGS & F_FUSE_N) potential_substep_q<R, MODE, XFLAGS, Q>(u, lane, kLanes, PX, L);
            if (Q > 1) {
#pragma unroll
                for (int i = 0; i < Q; ++i) row[xy_slot<(int)sizeof(V)>(lane + kLanes * i)] = to_v<V>(u[i]);
                wave_lds_sync();
#pragma unroll
                for (int i = 0; i < Q; ++i) u[i] = from_v<R>(row[xy_slot<(int)sizeof(V)>(lane * Q + i)]);
                wave_lds_sync();
            }
            x_line_solve<R, MODE, Q, kXYMaxScan>(PX, KX, S, lane, u);
#pragma unroll
            for (int i = 0; i < Q; ++i) row[xy_slot<(int)sizeof(V)>(lane * Q + i)] = to_v<V>(u[i]);
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i) row[xy_slot<(int)sizeof(V)>(lane * Q + i)] = to_v<V>(zero);
        }
    };

    V ahead[Q];
    xy_load_row<R, Q>(src, j0, j1, w, k, nx, ny, lane, ahead);
    x_row(j0, ahead);
    xy_load_row<R, Q>(src, j0 + 1, j1, w, k, nx, ny, lane, ahead);
    __syncthreads();
    int u = 0;  // window slot of block j: (j - j0) mod (DW + 1)
#pragma unroll 1
    for (int j = j0; j < j1; ++j) {
        // the next block's x solve (its rows were loaded a block ago), then the
        // request for the rows after it
        x_row(j + 1, ahead);
        xy_load_row<R, Q>(src, j + 2, j1, w, k, nx, ny, lane, ahead);
        if (w < cw) {
            cp<R> v[B];
#pragma unroll
            for (int r = 0; r < B; ++r) v[r] = from_v<R>(tile[j & 1][r][xy_slot<(int)sizeof(V)>(w * kLanes + lane)]);
            // one copy of the y step per window slot, so the slot index is a constant
            const bool cr = YRegSolver<R, MODE, DW, kYSums>::const_rows(j, PY.q_const, ny);
            static_for<DW + 1>([&](auto U) {
                if (u == decltype(U)::value) {
                    if (cr)
                        Y.template process<decltype(U)::value, true>(v, j, taby, dst);
                    else
                        Y.template process<decltype(U)::value, false>(v, j, taby, dst);
                }
            });
        }
        u = u == DW ? 0 : u + 1;
        __syncthreads();
    }
}

// Launch the fused kernel of the plan's shape, or (occ != nullptr) only report
// how many of its workgroups one CU holds at once.
template <typename R, int MODE, int XFLAGS, int Q, int DW>
static hipError_t launch_xy_dw(const gp_plan *p, const SweepParams &PX, const SweepParams &PY, hipStream_t s,
                               int variant, int *occ)
{
    using V = typename CT<R>::V;
    const dim3 grid((unsigned)p->xy_segs, (unsigned)p->n[2]), block(kLanes * kXYWaves);
    if (variant == 2) {  // elimination window in registers, double-buffered tile
        const auto kern = k_sweep_xy_reg<R, MODE, XFLAGS, Q, DW>;
        if (occ) return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, kern, (int)block.x, 0);
        hipLaunchKernelGGL(kern, grid, block, 0, s, PX, PY, (const V *)PX.psi, (V *)PY.out, (const V *)PX.tab,
                           (const V *)PY.tab);
        return hipGetLastError();
    }
    const auto kern = k_sweep_xy<R, MODE, XFLAGS, Q, DW>;
    const size_t ring = (size_t)kXYWaves * (size_t)p->ax[1].L * kLanes * sizeof(V);
    if (occ) return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, kern, (int)block.x, ring);
    hipLaunchKernelGGL(kern, grid, block, ring, s, PX, PY, (const V *)PX.psi, (V *)PY.out, (const V *)PX.tab,
                       (const V *)PY.tab);
    return hipGetLastError();
}

template <typename R, int MODE, int XFLAGS, int Q>
static hipError_t launch_xy_q(const gp_plan *p, const SweepParams &PX, const SweepParams &PY, hipStream_t s,
                              int variant, int *occ)
{
    switch (p->ax[1].D) {
    case 2: return launch_xy_dw<R, MODE, XFLAGS, Q, 2>(p, PX, PY, s, variant, occ);
    case 3: return launch_xy_dw<R, MODE, XFLAGS, Q, 3>(p, PX, PY, s, variant, occ);
    case 4: return launch_xy_dw<R, MODE, XFLAGS, Q, 4>(p, PX, PY, s, variant, occ);
    default: return hipErrorInvalidValue;
    }
}

template <typename R, int MODE, int XFLAGS>
static hipError_t launch_xy_flags(const gp_plan *p, const SweepParams &PX, const SweepParams &PY, hipStream_t s,
                                  int variant, int *occ)
{
    switch (p->ax[0].xq) {
    case 2: return launch_xy_q<R, MODE, XFLAGS, 2>(p, PX, PY, s, variant, occ);
    case 4: return launch_xy_q<R, MODE, XFLAGS, 4>(p, PX, PY, s, variant, occ);
    default: return hipErrorInvalidValue;
    }
}

template <typename R>
static hipError_t launch_xy_r(const gp_plan *p, const SweepParams &PX, const SweepParams &PY, int flags,
                              hipStream_t s, int variant, int *occ)
{
    if (p->mode == GP_IMAG)
        return (flags & F_RENORM) ? launch_xy_flags<R, GP_IMAG, F_FUSE_N | F_RENORM>(p, PX, PY, s, variant, occ)
                                  : launch_xy_flags<R, GP_IMAG, F_FUSE_N>(p, PX, PY, s, variant, occ);
    return launch_xy_flags<R, GP_REAL, F_FUSE_N>(p, PX, PY, s, variant, occ);
}

hipError_t xy_dispatch(const gp_plan *p, const SweepParams &PX, const SweepParams &PY, int flags, hipStream_t s,
                       int variant, int *occ)
{
    return p->prec == GP_C128 ? launch_xy_r<double>(p, PX, PY, flags, s, variant, occ)
                              : launch_xy_r<float>(p, PX, PY, flags, s, variant, occ);
}

}  // namespace

size_t xy_lds_bytes(const gp_plan *p, int variant)
{
    const size_t eb = elem_bytes(p->prec);
    const size_t tile = (size_t)kXYWaves * kLanes * (size_t)p->ax[0].xq * eb;
    if (variant == 2) return 2 * tile;
    return tile + (size_t)kXYWaves * (size_t)p->ax[1].L * kLanes * eb;
}

int xy_choose_segments(const gp_plan *p, int variant, int64_t max_lds)
{
    if (p->ndim != 3) return 0;
    const AxisPlan &X = p->ax[0], &Y = p->ax[1];
    if (X.xq != 2 && X.xq != 4) return 0;
    if (X.scan_steps > kXYMaxScan) return 0;
    if (p->n[0] % kLanes != 0 || p->n[0] > (int64_t)kLanes * X.xq) return 0;
    if (Y.K < 0 || Y.B != 4 || Y.D < 2 || Y.D > 4) return 0;
    if ((int64_t)xy_lds_bytes(p, variant) > max_lds) return 0;
    // as many workgroups as the device holds at once (its CUs times what one CU
    // holds of this kernel), in segments of at least two windows: an idle CU
    // costs more than the warm-up rows a segment repeats, and workgroups beyond
    // what the device holds would only queue
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || cus < 1)
        cus = 256;
    const SweepParams none{};
    if (xy_dispatch(p, none, none, F_FUSE_N, nullptr, variant, &per_cu) != hipSuccess || per_cu < 1) per_cu = 2;
    const int64_t nb = (p->n[1] + 3) / 4;
    int64_t segs = (int64_t)cus * per_cu / p->n[2];
    const int64_t most = std::max<int64_t>(1, nb / (2 * (Y.D + 1)));
    segs = std::min(segs, most);
    return (int)std::max<int64_t>(1, segs);
}

hipError_t launch_xy(gp_plan *p, const void *src, void *dst, int flags, int64_t step_index, hipStream_t s)
{
    SweepParams PX = make_sweep_params(p, 0, src, nullptr, false, step_index, nullptr);
    SweepParams PY = make_sweep_params(p, 1, nullptr, dst, false, step_index, nullptr);
    timing_begin(p, K_SWEEP_XY, s);
    const hipError_t e = xy_dispatch(p, PX, PY, flags, s, p->xy_variant, nullptr);
    timing_end(p, s);
    return e;
}

}  // namespace gp

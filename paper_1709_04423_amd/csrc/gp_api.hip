// Host runtime of libgp: argument checking, plan construction (FP64 Thomas
// tables on the host, device buffers), the per-step launch sequence, the
// adjoint driver, observables and the measurement aids.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gp_internal.h"

namespace gp {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

gp_status hip_fail(hipError_t e, const char *what)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return GP_EHIP;
}

static gp_status alloc(void **ptr, size_t bytes, int64_t &counter)
{
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
        *ptr = nullptr;
        set_error(std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? GP_ENOMEM : GP_EHIP;
    }
    counter += (int64_t)bytes;
    return GP_OK;
}

size_t elem_bytes(gp_prec prec) { return prec == GP_C128 ? 16 : 8; }

double coord0(int64_t n) { return -0.5 * (double)n; }

void timing_begin(gp_plan *p, int kind, hipStream_t s)
{
    Timing &T = p->timing;
    if (T.capacity == 0 || T.used >= T.capacity) return;
    T.kind[T.used] = kind;
    (void)hipEventRecord(T.ev[2 * T.used], s);  // instrumentation only
}

void timing_end(gp_plan *p, hipStream_t s)
{
    Timing &T = p->timing;
    if (T.capacity == 0 || T.used >= T.capacity) return;
    (void)hipEventRecord(T.ev[2 * T.used + 1], s);
    ++T.used;
}

// c'_p of the scaled CN system tridiag(1, b/e, 1) for p = 0..n-1 (equal to
// e m_p of the Thomas algorithm on tridiag(e, b, e)), in extended precision:
//   c'_0 = 1/(b/e),  c'_p = 1/(b/e - c'_{p-1});
//   real time b/e = -2 + i/r, imaginary time b/e = -2 - 1/r,  r = dt/(4 dx^2).
// rho = max |c'_p| over p < n-1: the contraction factor of the back substitution.
static void thomas_c(int64_t n, double r, gp_mode mode, std::vector<std::complex<long double>> &c,
                     double &rho)
{
    using cl = std::complex<long double>;
    const long double kappa = 1.0L / (long double)r;
    const cl be = mode == GP_REAL ? cl(-2.0L, kappa) : cl(-2.0L - kappa, 0.0L);
    c.assign(n, cl(0.0L, 0.0L));
    cl prev(0.0L, 0.0L);
    rho = 0.0;
    for (int64_t p = 0; p < n; ++p) {
        c[p] = 1.0L / (be - prev);
        prev = c[p];
        if (p + 1 < n) rho = std::fmax(rho, (double)std::abs(c[p]));
    }
}

// Device rows (p = -1 .. rows-2) of precision T: c'_p rounded to T, and the
// explicit-side diagonal beta_p derived from the rounded c' values:
//   delta_p = 1/c'_p + c'_{p-1} (the diagonal the stored factors multiply out to),
//   real time beta_p = -conj(delta_p), imaginary time beta_p = -2/r - delta_p,
// with Im beta_p split into T hi + T lo.  conj conjugates every entry (the
// adjoint map).  Rows outside the line are zero.
template <typename T>
static void table_rows(const std::vector<std::complex<long double>> &c, int64_t rows, double r, gp_mode mode,
                       bool conj, std::vector<T> &out)
{
    using cl = std::complex<long double>;
    const int64_t n = (int64_t)c.size();
    out.assign(6 * rows, T(0));
    cl prev(0.0L, 0.0L);
    const long double sg = conj ? -1.0L : 1.0L;
    for (int64_t p = 0; p < n; ++p) {
        const T cr = (T)c[p].real(), ci = (T)c[p].imag();
        const cl cs((long double)cr, (long double)ci);
        const cl delta = 1.0L / cs + prev;
        prev = cs;
        cl beta = mode == GP_REAL ? -std::conj(delta) : cl(-2.0L / (long double)r, 0.0L) - delta;
        const T br = (T)beta.real();
        const T bi_hi = (T)beta.imag();
        const T bi_lo = (T)(beta.imag() - (long double)bi_hi);
        T *row = &out[6 * (p + 1)];
        row[0] = cr;
        row[1] = (T)(sg * ci);
        row[2] = br;
        row[3] = (T)(sg * bi_hi);
        row[4] = (T)(sg * bi_lo);
        row[5] = T(0);
    }
}

// Window: blocks of B points (4 on the strided axes, 16 for transposed x
// lines), D = ceil((Kmin + 1) / B) for the smallest Kmin with rho^(Kmin+1) <=
// tol, used as K = D B - 1 (the back substitution then starts at the newest
// eliminated point); ring of next_pow2((D+1) B) slots.  K = -1 selects the
// exact two-pass solver when K + 1 > kMaxWindowPoints or the ring (plus the
// transposed tile) does not fit in LDS.  Lines are split into segments until
// about two (complex128) or four (complex64) wavefronts per SIMD are in
// flight, keeping every segment at least four windows long; grids too small for
// one wavefront per SIMD are split further, down to one window per segment.
constexpr int64_t kMinSweepWaves = 1024;  // one wavefront per SIMD of a 256-CU device

static void choose_window(AxisPlan &A, gp_prec prec, int B, bool tile)
{
    const double tol = prec == GP_C128 ? std::ldexp(1.0, -60) : std::ldexp(1.0, -44);
    int Kmin = 0;
    double bound = A.rho;
    while (bound > tol && Kmin < 100000) {
        bound *= A.rho;
        ++Kmin;
    }
    A.kmin = Kmin;
    A.B = B;
    const int D = (Kmin + 1 + B - 1) / B;
    int L = 1;
    while (L < (D + 1) * B) L <<= 1;
    const int64_t eb = (int64_t)elem_bytes(prec);
    const int64_t lds = (int64_t)L * kLanes * eb + (tile ? (int64_t)kLanes * (B + 1) * eb : 0);
    const int64_t nblocks = (A.n + B - 1) / B;
    A.segs = 1;
    if (D * B <= kMaxWindowPoints && lds <= kMaxLdsBytes) {
        A.K = D * B - 1;
        A.D = D;
        A.L = L;
        A.bound = std::pow(A.rho, A.K + 1);
        A.npad = (nblocks + D) * B;
        const int64_t waves = (A.nlines + kLanes - 1) / kLanes;
        // about 2 wavefronts per SIMD for complex128 rows, 4 for complex64 (same bytes in flight)
        const int64_t target = prec == GP_C128 ? 2048 : 4096;
        if (!tile) {
            while (A.segs < 8 && waves * A.segs < target && nblocks / (A.segs + 1) >= 4 * (D + 1)) ++A.segs;
            // small grids leave the device mostly idle and each wavefront's
            // sequential chain sets the time: keep splitting, down to segments
            // of one window, until about one wavefront per SIMD is busy
            while (A.segs < 64 && waves * A.segs < kMinSweepWaves && nblocks / (A.segs + 1) >= D + 1) ++A.segs;
        }
    } else {
        A.K = -1;
        A.D = 0;
        A.L = 0;
        A.bound = 0.0;
        A.npad = A.n + 1;
    }
    if (A.npad < A.n + 1) A.npad = A.n + 1;
}

AxisPlan preview_axis(int64_t n, int64_t nlines, double dx, double dt, gp_mode mode, gp_prec prec, int B, bool tile)
{
    AxisPlan A;
    A.n = n;
    A.nlines = nlines;
    A.r = dt / (4.0 * dx * dx);
    std::vector<std::complex<long double>> c;
    thomas_c(A.n, A.r, mode, c, A.rho);
    choose_window(A, prec, B, tile);
    return A;
}

// x sweep with one wavefront per line: Q = points per lane (power of two,
// n <= 64 Q <= 64 kXMaxQ) and scan steps S = smallest with Q 2^S > Kmin (full
// scan, S = 6, when that is not below 64 lanes).
static void x_scan_setup(AxisPlan &A)
{
    A.xq = 0;
    int Q = 1;
    while ((int64_t)Q * kLanes < A.n) Q <<= 1;
    if (Q > kXMaxQ) return;
    A.xq = Q;
    // lines per wavefront: 4 on large grids (the next line's load overlaps the
    // current solve), fewer while that would leave under 1024 workgroups
    A.xlpw = 4;
    while (A.xlpw > 1 && A.nlines < (int64_t)1024 * kXWavesPerGroup * A.xlpw) A.xlpw >>= 1;
    int S = 0;
    while (S < 6 && (int64_t)Q * (1 << S) <= A.kmin) ++S;
    A.scan_steps = S;
}

// The first point from which the stored table rows no longer change (the
// Thomas factors have converged to the table's rounding), and that row.
template <typename T>
static void const_row_setup(AxisPlan &A, const std::vector<std::complex<long double>> &c, gp_mode mode)
{
    std::vector<T> rows;
    table_rows<T>(c, A.n + 1, A.r, mode, false, rows);
    int64_t qc = A.n;
    auto same = [&](int64_t a, int64_t b) {
        for (int k = 0; k < 6; ++k)
            if (rows[6 * (a + 1) + k] != rows[6 * (b + 1) + k]) return false;
        return true;
    };
    while (qc > 0 && same(qc - 1, A.n - 1)) --qc;
    A.q_const = qc;
    const T *r = &rows[6 * A.n];  // row of point n-1
    A.c_inf[0] = (double)r[0];
    A.c_inf[1] = (double)r[1];
    A.b_inf[0] = (double)r[2];
    A.b_inf[1] = (double)r[3];
    A.b_inf[2] = (double)r[4];
}

// Multipliers of the x scan kernel's composed affine maps, per lane and scan
// step, exactly as the kernel would compute them: lane L holds points
// L Q .. L Q + Q - 1 with a_p = -c'_p (zero past the line); its forward map
// multiplier is prod a_p over its points, and scan step s (d = 2^s) multiplies
// lane L's by lane L-d's (forward) or L+d's (backward) when that lane exists.
// Rows 0..5: forward multiplier before step s; rows 6..11: backward.
template <typename T>
static std::vector<T> x_scan_multipliers(const std::vector<std::complex<long double>> &c, int Q, bool conj)
{
    using cl = std::complex<long double>;
    const int64_t n = (int64_t)c.size();
    std::vector<cl> f(kLanes, cl(1.0L, 0.0L)), b(kLanes, cl(1.0L, 0.0L));
    for (int L = 0; L < kLanes; ++L)
        for (int i = 0; i < Q; ++i) {
            const int64_t p = (int64_t)L * Q + i;
            const T cr = p < n ? (T)c[p].real() : T(0), ci = p < n ? (T)c[p].imag() : T(0);
            const cl a(-(long double)cr, -(long double)ci * (conj ? -1.0L : 1.0L));
            f[L] *= a;
            b[L] *= a;
        }
    std::vector<T> out(2 * 12 * kLanes, T(0));
    for (int s = 0; s < 6; ++s) {
        for (int L = 0; L < kLanes; ++L) {
            out[2 * (s * kLanes + L)] = (T)f[L].real();
            out[2 * (s * kLanes + L) + 1] = (T)f[L].imag();
            out[2 * ((6 + s) * kLanes + L)] = (T)b[L].real();
            out[2 * ((6 + s) * kLanes + L) + 1] = (T)b[L].imag();
        }
        const int d = 1 << s;
        std::vector<cl> f2 = f, b2 = b;
        for (int L = 0; L < kLanes; ++L) {
            if (L >= d) f2[L] = f[L] * f[L - d];
            if (L + d < kLanes) b2[L] = b[L] * b[L + d];
        }
        f = f2;
        b = b2;
    }
    return out;
}

template <typename T>
static gp_status upload_x_multipliers(gp_plan *p, AxisPlan &A, const std::vector<std::complex<long double>> &c,
                                      bool conj, void **dst)
{
    std::vector<T> h = x_scan_multipliers<T>(c, A.xq, conj);
    gp_status st = alloc(dst, h.size() * sizeof(T), p->device_bytes);
    if (st != GP_OK) return st;
    hipError_t e = hipMemcpy(*dst, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(x multipliers)");
    return GP_OK;
}

// Upload one axis's table (forward or conjugate) to the device.
static gp_status upload_table(gp_plan *p, AxisPlan &A, const std::vector<std::complex<long double>> &c, bool conj,
                              void **dst)
{
    const int64_t rows = A.npad + 1;
    hipError_t e;
    gp_status st;
    if (p->prec == GP_C128) {
        std::vector<double> h;
        table_rows<double>(c, rows, A.r, p->mode, conj, h);
        st = alloc(dst, h.size() * sizeof(double), p->device_bytes);
        if (st != GP_OK) return st;
        e = hipMemcpy(*dst, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice);
    } else {
        std::vector<float> h;
        table_rows<float>(c, rows, A.r, p->mode, conj, h);
        st = alloc(dst, h.size() * sizeof(float), p->device_bytes);
        if (st != GP_OK) return st;
        e = hipMemcpy(*dst, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(table)");
    return GP_OK;
}

// Radial axis of a symmetric-trap plan: the rows of the finite-volume CN system
// (W + k S) psi' = (W - k S) psi on r_i = (i + 1/2) dr, k = i dt/2 (real time) or
// dt/2 (imaginary time), with face areas a_{i+1/2} = ((i+1) dr)^(d-1), weights
// w_i = r_i (d = 2) or r_i^2 + dr^2/12 (d = 3) and S = -1/2 W L:
//   l_i = k s_{i,i-1}, diagonal w_i + k s_ii, u_i = k s_{i,i+1} (the wall coupling
//   of the last row dropped: the ghost is zero);
//   Thomas: m_i = 1/(diag_i - l_i c'_{i-1}), c'_i = u_i m_i;
//   row p = (alpha_p = -m_p l_p, m_p, -c'_p, beta_p = w_p - k s_pp, l_p, u_p),
// in long double, rounded once to double.  Rows past n are zero.  Also the scan
// multipliers of the one-wavefront solver (Q points per lane): rows s = 0..5
// forward, 6..11 backward, the lane's composite multiplier before scan step s.
static void radial_tables(int64_t n, double dr, double dt, gp_mode mode, int d, int Q, std::vector<double> &rows,
                          std::vector<double> &mul, double &rho)
{
    using cl = std::complex<long double>;
    const int64_t nrows = (int64_t)Q * kLanes;
    const long double tau = 0.5L * (long double)dt, h2 = (long double)dr * (long double)dr;
    const cl k = mode == GP_REAL ? cl(0.0L, tau) : cl(tau, 0.0L);
    std::vector<cl> fa(nrows, cl(0.0L, 0.0L)), ba(nrows, cl(0.0L, 0.0L));
    rows.assign(12 * nrows, 0.0);
    cl cprev(0.0L, 0.0L);
    rho = 0.0;
    auto face = [&](int64_t i) {
        const long double r = (long double)i * (long double)dr;
        return d == 3 ? r * r : r;
    };
    for (int64_t i = 0; i < n; ++i) {
        const long double r = ((long double)i + 0.5L) * (long double)dr;
        const long double w = d == 3 ? r * r + h2 / 12.0L : r;
        const long double lo = face(i), hi = face(i + 1);
        const long double sdd = (lo + hi) / (2.0L * h2), slo = -lo / (2.0L * h2), shi = -hi / (2.0L * h2);
        const cl sub = k * slo, dia = cl(w, 0.0L) + k * sdd, sup = i + 1 < n ? k * shi : cl(0.0L, 0.0L);
        const cl m = 1.0L / (dia - sub * cprev);
        const cl c = sup * m;
        const cl vals[6] = {-sub * m, m, -c, cl(w, 0.0L) - k * sdd, sub, sup};
        for (int j = 0; j < 6; ++j) {
            rows[12 * i + 2 * j] = (double)vals[j].real();
            rows[12 * i + 2 * j + 1] = (double)vals[j].imag();
        }
        fa[i] = cl((long double)(double)vals[0].real(), (long double)(double)vals[0].imag());
        ba[i] = cl((long double)(double)vals[2].real(), (long double)(double)vals[2].imag());
        if (i + 1 < n) rho = std::fmax(rho, (double)std::abs(c));
        cprev = c;
    }
    std::vector<cl> f(kLanes, cl(1.0L, 0.0L)), b(kLanes, cl(1.0L, 0.0L));
    for (int L = 0; L < kLanes; ++L)
        for (int i = 0; i < Q; ++i) {
            f[L] *= fa[(int64_t)L * Q + i];
            b[L] *= ba[(int64_t)L * Q + i];
        }
    mul.assign(2 * 12 * kLanes, 0.0);
    for (int st = 0; st < 6; ++st) {
        for (int L = 0; L < kLanes; ++L) {
            mul[2 * (st * kLanes + L)] = (double)f[L].real();
            mul[2 * (st * kLanes + L) + 1] = (double)f[L].imag();
            mul[2 * ((6 + st) * kLanes + L)] = (double)b[L].real();
            mul[2 * ((6 + st) * kLanes + L) + 1] = (double)b[L].imag();
        }
        const int dd = 1 << st;
        std::vector<cl> f2 = f, b2 = b;
        for (int L = 0; L < kLanes; ++L) {
            if (L >= dd) f2[L] = f[L] * f[L - dd];
            if (L + dd < kLanes) b2[L] = b[L] * b[L + dd];
        }
        f = f2;
        b = b2;
    }
}

static gp_status upload_doubles(gp_plan *p, const std::vector<double> &h, void **dst)
{
    gp_status st = alloc(dst, h.size() * sizeof(double), p->device_bytes);
    if (st != GP_OK) return st;
    hipError_t e = hipMemcpy(*dst, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(radial table)");
    return GP_OK;
}

static void free_plan(gp_plan *p)
{
    if (!p) return;
    for (int a = 0; a < 3; ++a) {
        if (p->ax[a].d_rtab) (void)hipFree(p->ax[a].d_rtab);
        if (p->ax[a].d_rmul) (void)hipFree(p->ax[a].d_rmul);
        if (p->ax[a].d_tab) (void)hipFree(p->ax[a].d_tab);
        if (p->ax[a].d_tab_adj) (void)hipFree(p->ax[a].d_tab_adj);
        if (p->ax[a].d_xmul) (void)hipFree(p->ax[a].d_xmul);
        if (p->ax[a].d_xmul_adj) (void)hipFree(p->ax[a].d_xmul_adj);
    }
    if (p->d_work) (void)hipFree(p->d_work);
    if (p->d_norm) (void)hipFree(p->d_norm);
    if (p->d_adj) (void)hipFree(p->d_adj);
    if (p->d_adj_done) (void)hipFree(p->d_adj_done);
    if (p->d_obs) (void)hipFree(p->d_obs);
    for (hipEvent_t e : p->timing.ev) (void)hipEventDestroy(e);
    delete p;
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Buffers of the sweep along `axis`: the strided sweeps run out of place (a
// segmented line would otherwise read points its neighbour segment has already
// written), and the last sweep of a step writes the caller's grid.
//   forward  3D: x psi->psi, y psi->work, z work->psi;  2D: x psi->work, y work->psi
//   adjoint  3D: z lam->work, y work->lam, x lam->lam;  2D: y lam->work, x work->lam
static void sweep_buffers(gp_plan *p, void *grid, int axis, bool adjoint, void **src, void **dst)
{
    void *w = p->d_work;
    *src = *dst = grid;
    if (p->ndim == 3) {
        if (!adjoint) {
            if (axis == 1) *dst = w;
            if (axis == 2) *src = w;
        } else {
            if (axis == 2) *dst = w;
            if (axis == 1) *src = w;
        }
    } else if (p->ndim == 2) {
        if (!adjoint) {
            if (axis == 0) *dst = w;
            if (axis == 1) *src = w;
        } else {
            if (axis == 1) *dst = w;
            if (axis == 0) *src = w;
        }
    }
}

}  // namespace gp

using namespace gp;

extern "C" {

const char *gp_strerror(gp_status s)
{
    switch (s) {
    case GP_OK: return "ok";
    case GP_EINVAL: return "invalid argument";
    case GP_ENOMEM: return "out of memory";
    case GP_EHIP: return "HIP runtime error";
    case GP_ENONFINITE: return "non-finite result";
    case GP_EUNSUPPORTED: return "unsupported";
    case GP_ETIMEOUT: return "device wait timed out";
    }
    return "unknown status";
}

const char *gp_last_error(void) { return g_last_error.c_str(); }

const char *gp_kernel_name(int kind)
{
    static const char *names[GP_NUM_KERNEL_KINDS] = {
        "sweep_x", "sweep_y", "sweep_z", "sweep_exact", "scale", "observables",
        "observables_final", "adjoint_x", "adjoint_yz", "adjoint_reduce", "batch", "copy", "norm_final",
        "sweep_xy", "radial_norm"};
    if (kind < 0 || kind >= GP_NUM_KERNEL_KINDS) return "unknown";
    return names[kind];
}

}  // extern "C"

// Plan of either kind: Cartesian (geom GP_CARTESIAN, ndim 1..3) or a symmetric
// trap (radial axis 0; ndim 1, or 2 for axial).
static gp_status create_plan(gp_plan **out, int geom, int ndim, const int64_t *n, const double *dx, double dt,
                             gp_mode mode, const gp_trap *trap, double g, gp_prec prec)
{
    if (!out) return set_error("out is NULL"), GP_EINVAL;
    *out = nullptr;
    if (ndim < 1 || ndim > 3) return set_error("ndim must be 1, 2 or 3"), GP_EINVAL;
    if (!n || !dx) return set_error("n or dx is NULL"), GP_EINVAL;
    for (int a = 0; a < ndim; ++a) {
        if (n[a] < 1) return set_error("grid size must be >= 1"), GP_EINVAL;
        if (!finite_pos(dx[a])) return set_error("dx must be finite and > 0"), GP_EINVAL;
    }
    if (!finite_pos(dt)) return set_error("dt must be finite and > 0"), GP_EINVAL;
    if (mode != GP_IMAG && mode != GP_REAL) return set_error("bad mode"), GP_EINVAL;
    if (prec != GP_C128 && prec != GP_C64) return set_error("bad precision"), GP_EINVAL;
    if (!std::isfinite(g)) return set_error("g must be finite"), GP_EINVAL;
    int64_t npts = 1;
    for (int a = 0; a < ndim; ++a) {
        if (n[a] > ((int64_t)1 << 31) || npts > ((int64_t)1 << 40) / n[a])
            return set_error("grid too large"), GP_EINVAL;
        npts *= n[a];
    }
    if (trap) {
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(trap->omega[a])) return set_error("omega must be finite"), GP_EINVAL;
        if (trap->sched_len < 0 || (trap->sched_len > 0 && !trap->omega_sched))
            return set_error("bad trap schedule"), GP_EINVAL;
        if (trap->sched_len > 0 && (trap->sched_axis < 0 || trap->sched_axis >= ndim))
            return set_error("schedule axis out of range"), GP_EINVAL;
        for (int64_t k = 0; k < trap->sched_len; ++k)
            if (!std::isfinite(trap->omega_sched[k])) return set_error("schedule value not finite"), GP_EINVAL;
    }

    const bool radial = geom != GP_CARTESIAN;
    if (radial && prec != GP_C128)
        return set_error("symmetric-trap plans run in complex128 only"), GP_EUNSUPPORTED;
    if (radial && n[0] > (int64_t)kLanes * kXMaxQ)
        return set_error("symmetric-trap plans take at most 1024 radial points"), GP_EUNSUPPORTED;

    gp_plan *p = new (std::nothrow) gp_plan();
    if (!p) return set_error("host allocation failed"), GP_ENOMEM;
    p->geom = geom;
    p->ndim = ndim;
    p->dt = dt;
    p->mode = mode;
    p->prec = prec;
    p->g = g;
    p->npts = npts;
    p->dV = 1.0;
    for (int a = 0; a < ndim; ++a) {
        p->n[a] = n[a];
        p->dx[a] = dx[a];
        p->dV *= dx[a];
    }
    if (radial) {  // norm = m sum w |psi|^2
        const double pi = 3.14159265358979323846;
        p->dV = geom == GP_CIRCULAR ? 2.0 * pi * dx[0] : geom == GP_SPHERICAL ? 4.0 * pi * dx[0]
                                                                              : 2.0 * pi * dx[0] * dx[1];
    }
    if (trap) {
        for (int a = 0; a < ndim; ++a) p->omega[a] = trap->omega[a];
        if (trap->sched_len > 0) p->sched.assign(trap->omega_sched, trap->omega_sched + trap->sched_len);
        p->sched_axis = trap->sched_len > 0 ? trap->sched_axis : 0;
    }
    std::vector<double> rrows, rmul;

    // host-side plan of each axis: line addressing, tables, window
    const int64_t nx = p->n[0], ny = p->n[1];
    std::vector<std::complex<long double>> cs[3];
    for (int a = 0; a < ndim; ++a) {
        AxisPlan &A = p->ax[a];
        A.n = n[a];
        A.nlines = npts / n[a];
        if (a == 0) {  // line l = j + ny k -> first element l * nx, stride 1
            A.stride = 1;
            A.m1 = 1;
            A.s1 = 0;
            A.s2 = nx;
        } else if (a == 1) {  // line l = i + nx k -> i + nx ny k, stride nx
            A.stride = nx;
            A.m1 = nx;
            A.s1 = 1;
            A.s2 = nx * ny;
        } else {  // line l = i + nx j -> l, stride nx ny
            A.stride = nx * ny;
            A.m1 = A.nlines;
            A.s1 = 1;
            A.s2 = 0;
        }
        A.r = dt / (4.0 * dx[a] * dx[a]);
        if (radial && a == 0) {  // variable-coefficient radial line: one wavefront per line, full scan
            int Q = 1;
            while ((int64_t)Q * kLanes < A.n) Q <<= 1;
            A.rq = Q;
            A.K = -1;
            A.npad = (int64_t)Q * kLanes;
            radial_tables(A.n, dx[0], dt, mode, radial_dim(geom), Q, rrows, rmul, A.rho);
            continue;
        }
        thomas_c(A.n, A.r, mode, cs[a], A.rho);
        // strided axes stream blocks of 4 rows per wavefront
        choose_window(A, prec, a == 0 ? kBlock : 4, a == 0);
        if (prec == GP_C128)
            const_row_setup<double>(A, cs[a], mode);
        else
            const_row_setup<float>(A, cs[a], mode);
        // a 2D grid's y lines are too few for the windowed solver to fill the
        // device: one wavefront per line with the scan solver instead
        if (a == 0 || (a == 1 && ndim == 2 && A.n <= (int64_t)kColMaxQ * kLanes)) {
            x_scan_setup(A);
            if (A.xq > 0 && A.npad < (int64_t)A.xq * kLanes) A.npad = (int64_t)A.xq * kLanes;
        }
    }

    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        free_plan(p);
        return hip_fail(e, "hipGetDevice");
    }
    gp_status st = GP_OK;
    if (radial) {
        st = upload_doubles(p, rrows, &p->ax[0].d_rtab);
        if (st == GP_OK) st = upload_doubles(p, rmul, &p->ax[0].d_rmul);
    }
    for (int a = radial ? 1 : 0; a < ndim && st == GP_OK; ++a) {
        st = upload_table(p, p->ax[a], cs[a], false, &p->ax[a].d_tab);
        if (st == GP_OK && mode == GP_REAL) st = upload_table(p, p->ax[a], cs[a], true, &p->ax[a].d_tab_adj);
        if (st == GP_OK && p->ax[a].xq > 0) {
            for (int cj = 0; cj < (mode == GP_REAL ? 2 : 1) && st == GP_OK; ++cj) {
                void **dst = cj ? &p->ax[a].d_xmul_adj : &p->ax[a].d_xmul;
                st = prec == GP_C128 ? upload_x_multipliers<double>(p, p->ax[a], cs[a], cj != 0, dst)
                                     : upload_x_multipliers<float>(p, p->ax[a], cs[a], cj != 0, dst);
            }
        }
    }
    int64_t maxg = 1;
    for (int a = 0; a < ndim; ++a) maxg = std::max(maxg, sweep_groups(p, a));
    if (radial) maxg = std::max(maxg, radial_norm_groups(p));
    p->n_norm = maxg;
    p->n_adj = maxg;
    p->n_obs_blocks = radial ? std::max<int64_t>(obs_groups(p), radial_norm_groups(p)) : obs_groups(p);
    if (st == GP_OK && ndim >= 2) st = alloc(&p->d_work, (size_t)npts * elem_bytes(prec), p->device_bytes);
    if (st == GP_OK) st = alloc((void **)&p->d_norm, (2 * maxg + 2) * sizeof(double), p->device_bytes);
    if (st == GP_OK) st = alloc((void **)&p->d_adj, 2 * maxg * sizeof(double), p->device_bytes);
    if (st == GP_OK && mode == GP_REAL) {
        st = alloc((void **)&p->d_adj_done, sizeof(int), p->device_bytes);
        if (st == GP_OK && hipMemset(p->d_adj_done, 0, sizeof(int)) != hipSuccess) {
            set_error("hipMemset(adjoint counter)");
            st = GP_EHIP;
        }
    }
    if (st == GP_OK)
        st = alloc((void **)&p->d_obs, (p->n_obs_blocks + 1) * kObsFields * sizeof(double), p->device_bytes);
    if (st != GP_OK) {
        free_plan(p);
        return st;
    }
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device) != hipSuccess)
        max_lds = 0;
    p->max_lds = max_lds;
    p->xy_segs = radial ? 0 : xy_choose_segments(p, p->xy_variant, max_lds);
    *out = p;
    return GP_OK;
}

extern "C" {

gp_status gp_plan_create(gp_plan **out, int ndim, const int64_t *n, const double *dx, double dt, gp_mode mode,
                         const gp_trap *trap, double g, gp_prec prec)
{
    return create_plan(out, GP_CARTESIAN, ndim, n, dx, dt, mode, trap, g, prec);
}

gp_status gp_plan_create_sym(gp_plan **out, gp_geometry geom, const int64_t *n, const double *dx, double dt,
                             gp_mode mode, const gp_trap *trap, double g, gp_prec prec)
{
    if (geom != GP_CIRCULAR && geom != GP_SPHERICAL && geom != GP_AXIAL) {
        if (out) *out = nullptr;
        return set_error("geometry must be GP_CIRCULAR, GP_SPHERICAL or GP_AXIAL"), GP_EINVAL;
    }
    return create_plan(out, geom, geom == GP_AXIAL ? 2 : 1, n, dx, dt, mode, trap, g, prec);
}

gp_status gp_plan_destroy(gp_plan *plan)
{
    free_plan(plan);
    return GP_OK;
}

gp_status gp_plan_set_step(gp_plan *plan, int64_t step)
{
    if (!plan || step < 0) return set_error("bad plan or step"), GP_EINVAL;
    plan->step = step;
    return GP_OK;
}

gp_status gp_plan_get_info(const gp_plan *plan, gp_plan_info *info)
{
    if (!plan || !info) return set_error("NULL argument"), GP_EINVAL;
    std::memset(info, 0, sizeof(*info));
    info->ndim = plan->ndim;
    for (int a = 0; a < 3; ++a) {
        info->n[a] = a < plan->ndim ? plan->n[a] : 1;
        info->window[a] = a < plan->ndim ? plan->ax[a].K : 0;
        if (a < plan->ndim && plan->ax[a].xq > 0)  // scan solver: a carry reaches Q 2^S points (S = 6: whole line)
            info->window[a] = plan->ax[a].scan_steps >= 6 ? -1 : plan->ax[a].xq * (1 << plan->ax[a].scan_steps) - 1;
        info->rho[a] = a < plan->ndim ? plan->ax[a].rho : 0.0;
        info->window_bound[a] = a < plan->ndim ? plan->ax[a].bound : 0.0;
    }
    info->step = plan->step;
    info->device_bytes = plan->device_bytes;
    info->xy_fused = plan->xy_enabled ? plan->xy_segs : 0;
    return GP_OK;
}

gp_status gp_plan_set_xy_fusion(gp_plan *plan, int enable)
{
    if (!plan || enable < 0 || enable > 2) return set_error("bad plan or flag"), GP_EINVAL;
    plan->xy_enabled = enable != 0;
    if (enable && enable != plan->xy_variant && plan->geom == GP_CARTESIAN) {
        const hipError_t e = hipSetDevice(plan->device);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
        plan->xy_variant = enable;
        plan->xy_segs = xy_choose_segments(plan, enable, plan->max_lds);
    }
    return GP_OK;
}

gp_status gp_osc_length(double mass_amu, double freq_hz, double *l_micron)
{
    if (!l_micron || !(mass_amu > 0.0) || !(freq_hz > 0.0) || !std::isfinite(mass_amu) || !std::isfinite(freq_hz))
        return set_error("mass and frequency must be finite and > 0"), GP_EINVAL;
    const double hbar = 1.054571817e-34, amu = 1.66053906660e-27, pi = 3.14159265358979323846;
    *l_micron = std::sqrt(hbar / (mass_amu * amu * 2.0 * pi * freq_hz)) * 1e6;
    return GP_OK;
}

gp_status gp_nonlinearity(int ndim, double natoms, double a_bohr, double l_micron, double confine, double *g)
{
    if (!g || ndim < 1 || ndim > 3 || !std::isfinite(natoms) || natoms < 0.0 || !std::isfinite(a_bohr) ||
        !(l_micron > 0.0) || !std::isfinite(l_micron) || (ndim < 3 && (!(confine > 0.0) || !std::isfinite(confine))))
        return set_error("bad physical input"), GP_EINVAL;
    const double bohr = 5.29177210903e-11, pi = 3.14159265358979323846;
    const double na_l = natoms * a_bohr * bohr / (l_micron * 1e-6);  // N a / l
    if (ndim == 3)
        *g = 4.0 * pi * na_l;
    else if (ndim == 2)  // integral of the z ground state's |zeta|^4 = sqrt(lambda / (2 pi))
        *g = 4.0 * pi * na_l * std::sqrt(confine / (2.0 * pi));
    else  // integral of the transverse (2D) ground state's |zeta|^4 = nu / (2 pi)
        *g = 4.0 * pi * na_l * confine / (2.0 * pi);
    return GP_OK;
}

gp_status gp_thomas_table(int64_t n, double dx, double dt, gp_mode mode, gp_prec prec, int adjoint, double *c,
                          double *beta, int *window, double *rho)
{
    if (n < 1 || n > ((int64_t)1 << 31) || !finite_pos(dx) || !finite_pos(dt) || !c || !beta || !window || !rho)
        return set_error("bad argument"), GP_EINVAL;
    if (mode != GP_IMAG && mode != GP_REAL) return set_error("bad mode"), GP_EINVAL;
    if (prec != GP_C128 && prec != GP_C64) return set_error("bad precision"), GP_EINVAL;
    AxisPlan A;
    A.n = n;
    A.r = dt / (4.0 * dx * dx);
    std::vector<std::complex<long double>> cs;
    A.nlines = 1;
    thomas_c(n, A.r, mode, cs, A.rho);
    choose_window(A, prec, 4, false);
    const int64_t rows = n + 1;
    auto emit = [&](auto &h) {
        for (int64_t q = 0; q < n; ++q) {
            const auto *row = &h[6 * (q + 1)];
            c[2 * q] = (double)row[0];
            c[2 * q + 1] = (double)row[1];
            beta[2 * q] = (double)row[2];
            beta[2 * q + 1] = (double)row[3] + (double)row[4];
        }
    };
    if (prec == GP_C128) {
        std::vector<double> h;
        table_rows<double>(cs, rows, A.r, mode, adjoint != 0, h);
        emit(h);
    } else {
        std::vector<float> h;
        table_rows<float>(cs, rows, A.r, mode, adjoint != 0, h);
        emit(h);
    }
    *window = A.K;
    *rho = A.rho;
    return GP_OK;
}

// nsteps Cartesian steps from step index p->step (the index is not advanced).
// states != null (real time): the state before step k is written to
// states + k * grid bytes, by the x scan kernel as it loads (otherwise a copy).
static gp_status cartesian_steps(gp_plan *p, void *psi, int64_t nsteps, void *states, hipStream_t s)
{
    const bool imag = p->mode == GP_IMAG;
    const bool fused = p->ndim == 3 && p->xy_segs > 0 && p->xy_enabled;
    const size_t bytes = (size_t)p->npts * elem_bytes(p->prec);
    hipError_t e;
    if (p->ndim == 1 && !states && p->sched.empty() && p->ax[0].xq > 0 && p->ax[0].xq <= k1DMaxQ) {
        // one line: the whole run in one launch
        timing_begin(p, K_SWEEP_X, s);
        e = launch_steps_1d(p, psi, nsteps, norm_total(p, p->step + nsteps - 1), s);
        timing_end(p, s);
        return e == hipSuccess ? GP_OK : hip_fail(e, "1D steps launch");
    }
    for (int64_t k = 0; k < nsteps; ++k) {
        const int64_t n = p->step + k;
        void *copy_to = states ? (char *)states + (size_t)k * bytes : nullptr;
        const bool copy_in_x = copy_to && !fused && p->ax[0].xq > 0;
        if (copy_to && !copy_in_x) {
            e = launch_copy(copy_to, psi, (int64_t)bytes, s);
            if (e != hipSuccess) return hip_fail(e, "state copy launch");
        }
        if (fused) {  // x and y in one pass psi -> work, then z work -> psi
            e = launch_xy(p, psi, p->d_work, F_FUSE_N | ((imag && k > 0) ? F_RENORM : 0), n, s);
            if (e != hipSuccess) return hip_fail(e, "fused x+y sweep launch");
        }
        for (int a = fused ? 2 : 0; a < p->ndim; ++a) {
            int flags = 0;
            if (a == 0) flags |= F_FUSE_N | ((imag && k > 0) ? F_RENORM : 0);
            if (imag && a == p->ndim - 1) flags |= F_NORM_OUT;
            SweepExtras x;
            if (a == 0 && copy_in_x) {
                flags |= F_COPY_IN;
                x.copy_out = copy_to;
            }
            void *src, *dst;
            sweep_buffers(p, psi, a, false, &src, &dst);
            e = launch_sweep(p, a, src, dst, flags, false, n, nullptr, s, &x);
            if (e != hipSuccess) return hip_fail(e, "sweep launch");
        }
        if (imag) {
            e = launch_norm_final(p, n, s);
            if (e != hipSuccess) return hip_fail(e, "norm launch");
        }
    }
    return GP_OK;
}

gp_status gp_step(gp_plan *p, void *psi, int64_t nsteps, void *stream)
{
    if (!p || !psi || nsteps < 0) return set_error("bad plan, psi or nsteps"), GP_EINVAL;
    if (nsteps == 0) return GP_OK;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const bool imag = p->mode == GP_IMAG;
    if (p->geom != GP_CARTESIAN && p->ndim == 1 && p->sched.empty()) {  // one radial line: one launch
        e = launch_radial_steps(p, psi, nsteps, norm_total(p, p->step + nsteps - 1), s);
        if (e != hipSuccess) return hip_fail(e, "symmetric-trap steps launch");
        p->step += nsteps;
        if (imag) {
            e = launch_scale(p, psi, s);
            if (e != hipSuccess) return hip_fail(e, "scale launch");
        }
        return GP_OK;
    }
    if (p->geom != GP_CARTESIAN) {  // symmetric trap: radial line solver, then z (axial)
        for (int64_t k = 0; k < nsteps; ++k) {
            const int64_t n = p->step + k;
            const int fl = F_FUSE_N | ((imag && k > 0) ? F_RENORM : 0);
            if (p->ndim == 1) {
                e = launch_radial_line(p, psi, psi, fl | (imag ? F_NORM_OUT : 0), n, s);
            } else {
                e = launch_radial_line(p, psi, p->d_work, fl, n, s);
                if (e == hipSuccess) e = launch_sweep(p, 1, p->d_work, psi, 0, false, n, nullptr, s);
                if (e == hipSuccess && imag) e = launch_radial_norm(p, psi, n, s);
            }
            if (e == hipSuccess && imag) e = launch_norm_final(p, n, s);
            if (e != hipSuccess) return hip_fail(e, "symmetric-trap step launch");
        }
        p->step += nsteps;
        if (imag) {
            e = launch_scale(p, psi, s);
            if (e != hipSuccess) return hip_fail(e, "scale launch");
        }
        return GP_OK;
    }
    const gp_status st = cartesian_steps(p, psi, nsteps, nullptr, s);
    if (st != GP_OK) return st;
    p->step += nsteps;
    if (imag) {
        e = launch_scale(p, psi, s);
        if (e != hipSuccess) return hip_fail(e, "scale launch");
    }
    return GP_OK;
}

gp_status gp_observables(gp_plan *p, const void *psi, gp_obs *out, void *stream)
{
    if (!p || !psi || !out) return set_error("NULL argument"), GP_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    int64_t nb = p->n_obs_blocks;
    if (p->geom != GP_CARTESIAN) {
        nb = radial_norm_groups(p);
        e = launch_radial_obs(p, psi, p->d_obs, nb, s);
        if (e == hipSuccess) e = launch_obs_final(p, p->d_obs, nb, s);
    } else {
        e = launch_observables(p, psi, s);
    }
    if (e != hipSuccess) return hip_fail(e, "observables launch");
    double f[kObsFields];
    e = hipMemcpyAsync(f, p->d_obs + nb * kObsFields, sizeof(f), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(observables)");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (p->geom != GP_CARTESIAN) {  // weighted sums; m = the measure factor held in dV
        const double m = p->dV;
        out->norm = m * f[0];
        out->epot = m * f[1];
        out->eint = 0.5 * p->g * m * f[2];
        out->ekin = 0.5 * m * f[6] / (p->dx[0] * p->dx[0]);
        if (p->geom == GP_AXIAL) out->ekin += 0.5 * m * f[7] / (p->dx[1] * p->dx[1]);
        out->energy = out->ekin + out->epot + out->eint;
        out->mu = out->ekin + out->epot + 2.0 * out->eint;
        out->rms[0] = std::sqrt(f[3] / f[0]);
        out->rms[1] = p->geom == GP_AXIAL ? std::sqrt(f[4] / f[0]) : 0.0;
        out->rms[2] = 0.0;
    } else {
        obs_from_sums(f, p->ndim, p->dx, p->g, out);
    }
    if (!std::isfinite(out->norm) || !std::isfinite(out->energy)) {
        set_error("non-finite norm or energy");
        return GP_ENONFINITE;
    }
    return GP_OK;
}

gp_status gp_step_record(gp_plan *p, void *psi, int64_t nsteps, void *states, void *stream)
{
    if (!p || !psi || !states || nsteps < 0) return set_error("bad argument"), GP_EINVAL;
    if (p->mode != GP_REAL) return set_error("recording needs a real-time plan"), GP_EUNSUPPORTED;
    if (p->geom != GP_CARTESIAN) return set_error("the adjoint form runs on Cartesian plans"), GP_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const gp_status st = cartesian_steps(p, psi, nsteps, states, s);
    if (st != GP_OK) return st;
    p->step += nsteps;
    return GP_OK;
}

gp_status gp_step_adjoint(gp_plan *p, const void *states, void *lambda, int64_t n_first, int64_t nsteps,
                          double *dsched, double *dg, void *stream)
{
    if (!p || !states || !lambda || nsteps < 0 || n_first < 0) return set_error("bad argument"), GP_EINVAL;
    if (p->mode != GP_REAL) return set_error("adjoint needs a real-time plan"), GP_EUNSUPPORTED;
    if (p->geom != GP_CARTESIAN) return set_error("the adjoint form runs on Cartesian plans"), GP_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const size_t bytes = (size_t)p->npts * elem_bytes(p->prec);
    const int64_t nparts = sweep_groups(p, 0);
    for (int64_t k = nsteps - 1; k >= 0; --k) {
        const int64_t n = n_first + k;
        const void *st = (const char *)states + (size_t)k * bytes;
        double w[3];
        omega_at_step(p, n, w);
        const double coeff = p->dt * w[p->sched_axis];
        // the x scan kernel reduces the gradient sums itself (its last workgroup)
        const bool fold = p->ax[0].xq > 0 && p->d_adj_done;
        SweepExtras x;
        if (fold) {
            x.adj_done = p->d_adj_done;
            x.adj_dsched = dsched ? dsched + k : nullptr;
            x.adj_dg = dg;
            x.adj_coeff = coeff;
        }
        for (int a = p->ndim - 1; a >= 0; --a) {
            void *src, *dst;
            sweep_buffers(p, lambda, a, true, &src, &dst);
            e = launch_sweep(p, a, src, dst, a == 0 ? F_ADJ_N : 0, true, n, st, s, a == 0 ? &x : nullptr);
            if (e != hipSuccess) return hip_fail(e, "adjoint sweep launch");
        }
        if (!fold) {
            e = launch_adj_reduce(p, nparts, coeff, dsched ? dsched + k : nullptr, dg, s);
            if (e != hipSuccess) return hip_fail(e, "adjoint reduce launch");
        }
    }
    return GP_OK;
}

gp_status gp_plan_timing_enable(gp_plan *p, int64_t capacity)
{
    if (!p || capacity < 0) return set_error("bad argument"), GP_EINVAL;
    Timing &T = p->timing;
    for (hipEvent_t ev : T.ev) (void)hipEventDestroy(ev);
    T.ev.clear();
    T.kind.clear();
    T.used = 0;
    T.capacity = 0;
    if (capacity == 0) return GP_OK;
    T.ev.resize(2 * capacity);
    T.kind.resize(capacity);
    for (int64_t i = 0; i < 2 * capacity; ++i) {
        hipError_t e = hipEventCreate(&T.ev[i]);
        if (e != hipSuccess) {
            T.ev.resize(i);
            return hip_fail(e, "hipEventCreate");
        }
    }
    T.capacity = capacity;
    return GP_OK;
}

gp_status gp_plan_timing_read(gp_plan *p, int64_t *counts, double *total_ms)
{
    if (!p || !counts || !total_ms) return set_error("bad argument"), GP_EINVAL;
    for (int k = 0; k < GP_NUM_KERNEL_KINDS; ++k) {
        counts[k] = 0;
        total_ms[k] = 0.0;
    }
    Timing &T = p->timing;
    if (T.used > 0) {
        hipError_t e = hipEventSynchronize(T.ev[2 * T.used - 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    }
    for (int64_t i = 0; i < T.used; ++i) {
        float ms = 0.0f;
        hipError_t e = hipEventElapsedTime(&ms, T.ev[2 * i], T.ev[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        counts[T.kind[i]] += 1;
        total_ms[T.kind[i]] += ms;
    }
    T.used = 0;
    return GP_OK;
}

gp_status gp_copy_probe(void *dst, const void *src, int64_t bytes, void *stream)
{
    if (!dst || !src || bytes <= 0 || bytes % 16) return set_error("bad copy arguments"), GP_EINVAL;
    hipError_t e = launch_copy(dst, src, bytes, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "copy launch");
    return GP_OK;
}

}  // extern "C"

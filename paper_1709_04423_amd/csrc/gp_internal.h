// Internal declarations of libgp (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "gp.h"

namespace gp {

// Kinds of kernel launches, for per-kernel timing.
enum KernelKind {
    K_SWEEP_X = 0,
    K_SWEEP_Y = 1,
    K_SWEEP_Z = 2,
    K_SWEEP_EXACT = 3,
    K_SCALE = 4,
    K_OBS = 5,
    K_OBS_FINAL = 6,
    K_ADJ_X = 7,
    K_ADJ_YZ = 8,
    K_ADJ_REDUCE = 9,
    K_BATCH = 10,
    K_COPY = 11,
    K_NORM_FINAL = 12,
    K_SWEEP_XY = 13,
    K_RADIAL_NORM = 14,
};

// Flags of the line-sweep kernel.
enum SweepFlags {
    F_FUSE_N = 1,   // potential + nonlinear substep applied to every value at load (axis 0)
    F_RENORM = 2,   // scale loaded values by 1/sqrt(dV * sum of norm partials) first
    F_NORM_OUT = 4, // write an FP64 per-workgroup partial of sum |u'|^2
    F_ADJ_N = 8,    // adjoint of the potential substep applied at store (axis 0)
    F_COPY_IN = 16, // also write every loaded input value to copy_out (axis 0 scan kernel)
};

constexpr int kLanes = 64;      // one wavefront = one workgroup of the sweeps
constexpr int kBlock = 16;      // points per block of the transposed x solver (strided axes use 4)
constexpr int kMaxLdsBytes = 64 * 1024;
constexpr int kMaxWindowPoints = 32; // largest compiled window (K + 1 = D B points)

// Everything a sweep launch needs; passed by value as the kernel argument.
struct SweepParams {
    void *psi;            // input grid
    void *out;            // output grid (may equal psi)
    const void *state;    // F_ADJ_N: input state of the step being reversed
    int64_t n;            // line length
    int64_t stride;       // element stride along the line
    int64_t nlines;       // number of lines
    int64_t m1, s1, s2;   // first element of line l: (l % m1) * s1 + (l / m1) * s2
    const void *tab;      // Thomas table rows p = -1 .. npad-1: c'_p, beta_p, beta_p lo (precision of psi)
    int K;                // back-substitution window
    int lmask;            // ring slots - 1 (power of two)
    int D;                // window depth in blocks (K = D kBlock - 1)
    int nblocks;          // ceil(n / kBlock)
    // x sweep with one wavefront per line: scan steps and the constant interior row
    int scan_steps;
    int64_t q_const;      // rows of points q >= q_const all equal (c_inf, b_inf)
    double c_inf[2];      // c'_q (re, im)
    double b_inf[3];      // beta_q (re, im hi, im lo)
    const void *xmul;     // x scan multipliers: 12 rows x 64 lanes (forward steps 0..5, backward 0..5)
    int xq;               // x scan points per lane (0: not the scan kernel)
    int xlpw;             // x scan lines per wavefront
    // potential substep on axis 0
    double dt, g;
    double hw2[3];        // 1/2 omega_a^2 of this step
    double x0[3], dx[3];  // coordinate of index i on axis a: (i + x0[a]) * dx[a]
    int64_t ny;           // axis-0 line index l -> (j, k) = (l % ny, l / ny)
    int sched_axis;       // F_ADJ_N: axis whose x^2 weights the schedule gradient
    // imaginary-time renormalisation
    const double *norm_total;  // F_RENORM: dV-less sum |psi|^2 of the previous step (one value)
    double dV;
    double *norm_out;     // F_NORM_OUT partials, one per workgroup
    int64_t n_norm;       // partial slots per step parity (batched kernels offset by parity)
    double *adj_out;      // F_ADJ_N partials, two per workgroup
    // F_ADJ_N in the x scan kernel: the last workgroup to finish sums the
    // partials (adj_done counts finished workgroups and is reset by that one)
    // into *adj_dsched = adj_coeff sum_w and *adj_dg += dt sum_g
    int *adj_done;
    double *adj_dsched, *adj_dg;
    double adj_coeff;
    void *copy_out;       // F_COPY_IN: where the input values are copied
    int radial_d;         // symmetric traps: dimension of the radial axis 0 (2 or 3; 0 Cartesian)
};

struct AxisPlan {
    int64_t n = 1, stride = 1, nlines = 1, m1 = 1, s1 = 0, s2 = 0;
    double r = 0.0;
    double rho = 0.0;
    int K = 0;            // window; -1 = exact two-pass solver
    int D = 0, L = 0;
    int B = 4;            // points per block of the windowed solver
    int segs = 1;         // segments per line (windowed solver)
    int64_t npad = 0;     // table rows after the p = -1 row
    double bound = 0.0;
    int kmin = 0;         // smallest window meeting the precision's bound
    int xq = 0;           // x sweep: points per lane of the one-wavefront-per-line kernel (0: not used)
    int xlpw = 1;         // x sweep: lines each wavefront solves in turn (1, 2 or 4)
    int scan_steps = 6;   // x sweep: Hillis-Steele steps (6 = full, exact)
    int64_t q_const = 0;  // first point from which every table row is identical
    double c_inf[2] = {0.0, 0.0}, b_inf[3] = {0.0, 0.0, 0.0};
    std::vector<double> c;             // FP64 c'_p (interleaved complex), before rounding
    void *d_tab = nullptr;             // device table (forward)
    void *d_tab_adj = nullptr;         // device table (conjugate)
    void *d_xmul = nullptr;            // x scan multipliers (forward map)
    void *d_xmul_adj = nullptr;        // x scan multipliers (conjugate map)
    // radial axis of a symmetric-trap plan (axis 0): per-row coefficients and scan multipliers
    void *d_rtab = nullptr;            // rows p = 0..64 rq - 1: alpha, m, -c', beta, l_p, l_{p+1} (complex)
    void *d_rmul = nullptr;            // 12 x 64 complex: forward / backward lane multipliers per scan step
    int rq = 0;                        // points per lane of the radial line solver
};

struct Timing {
    std::vector<hipEvent_t> ev;
    std::vector<int> kind;
    int64_t used = 0;
    int64_t capacity = 0;
};

}  // namespace gp

struct gp_plan {
    int geom = GP_CARTESIAN;        // gp_geometry: symmetric traps solve a radial axis 0
    int ndim = 1;
    int64_t n[3] = {1, 1, 1};
    double dx[3] = {1.0, 1.0, 1.0};
    double dt = 0.0;
    gp_mode mode = GP_IMAG;
    gp_prec prec = GP_C128;
    double g = 0.0;
    double omega[3] = {0.0, 0.0, 0.0};
    std::vector<double> sched;
    int sched_axis = 0;
    int64_t step = 0;
    int64_t npts = 1;
    double dV = 1.0;
    int device = 0;
    gp::AxisPlan ax[3];
    void *d_work = nullptr;         // second grid: the strided sweeps run out of place
    double *d_norm = nullptr;       // norm partials of the last sweep
    int64_t n_norm = 0;
    double *d_adj = nullptr;        // adjoint partials (2 per workgroup)
    int *d_adj_done = nullptr;      // finished-workgroup counter of the x adjoint sweep (zero between launches)
    int64_t n_adj = 0;
    double *d_obs = nullptr;        // observable partials + final sums
    int64_t n_obs_blocks = 0;
    int64_t device_bytes = 0;
    int xy_segs = 0;                // 3D: row segments per plane of the fused x+y kernel (0: not fusable)
    bool xy_enabled = true;         // use the fused kernel when xy_segs > 0
    int xy_variant = 2;             // fused kernel: 1 LDS elimination window, 2 window in registers
    int max_lds = 0;                // LDS bytes a workgroup may use on the plan's device
    gp::Timing timing;
};

namespace gp {

void set_error(const std::string &msg);
gp_status hip_fail(hipError_t e, const char *what);

// Launch helpers (stream-ordered, asynchronous).
void timing_begin(gp_plan *p, int kind, hipStream_t s);
void timing_end(gp_plan *p, hipStream_t s);

size_t elem_bytes(gp_prec prec);
double coord0(int64_t n);  // x0 such that x_i = (i + x0) dx

// Extras of a sweep launch beyond its grids (null: not used): the x scan
// kernel's folded adjoint reduce (F_ADJ_N) and its input copy (F_COPY_IN).
struct SweepExtras {
    int *adj_done = nullptr;
    double *adj_dsched = nullptr, *adj_dg = nullptr;
    double adj_coeff = 0.0;
    void *copy_out = nullptr;
};

// Sweep along one axis; flags per SweepFlags; adjoint selects the conjugate map.
hipError_t launch_sweep(gp_plan *p, int axis, const void *src, void *dst, int flags, bool adjoint,
                        int64_t step_index, const void *state, hipStream_t s, const SweepExtras *extras = nullptr);
SweepParams make_sweep_params(const gp_plan *p, int axis, const void *src, void *dst, bool adjoint,
                              int64_t step_index, const void *state);
// Windowed / two-pass sweep of one axis in one precision (gp_sweep_c128.hip, gp_sweep_c64.hip).
hipError_t dispatch_sweep_c128(const AxisPlan &A, const SweepParams &P, gp_mode mode, int flags, bool exact,
                               bool tr, const void *tab, hipStream_t s);
hipError_t dispatch_sweep_c64(const AxisPlan &A, const SweepParams &P, gp_mode mode, int flags, bool exact,
                              bool tr, const void *tab, hipStream_t s);
hipError_t launch_scale(gp_plan *p, void *psi, hipStream_t s);
hipError_t launch_norm_final(gp_plan *p, int64_t step_index, hipStream_t s);
// norm totals: one value per step parity, after the 2 x n_norm partials
inline double *norm_partials(gp_plan *p, int64_t step) { return p->d_norm + (step & 1) * p->n_norm; }
inline double *norm_total(gp_plan *p, int64_t step) { return p->d_norm + 2 * p->n_norm + (step & 1); }
hipError_t launch_x_scan(const gp_plan *p, const SweepParams &P, int flags, const void *tab, hipStream_t s);
// nsteps 1D steps from step p->step in one launch (one wavefront; x points per
// lane 1..8, static trap); *total_out gets the last step's norm total.
constexpr int k1DMaxQ = 8;
hipError_t launch_steps_1d(const gp_plan *p, void *psi, int64_t nsteps, double *total_out, hipStream_t s);
// Strided axis solved with the scan solver (AxisPlan::xq > 0 on an axis other
// than 0): flags 0 or F_NORM_OUT.
hipError_t launch_col_scan(const gp_plan *p, int axis, const SweepParams &P, int flags, const void *tab,
                           hipStream_t s);
constexpr int kColMaxQ = 16;  // longest strided line of the scan solver: 64 kColMaxQ points
constexpr int kXLdsQ = 16;    // from this many points per lane the scan kernels keep the table rows in LDS
// Fused x and y sweeps of a 3D step (src -> dst, x flags as for the x sweep).
hipError_t launch_xy(gp_plan *p, const void *src, void *dst, int flags, int64_t step_index, hipStream_t s);
size_t xy_lds_bytes(const gp_plan *p, int variant);
// Row segments per plane of the fused kernel variant on this plan's device (0:
// the shape is not fusable).
int xy_choose_segments(const gp_plan *p, int variant, int64_t max_lds);
constexpr int kXWavesPerGroup = 4;  // wavefronts per workgroup of the x scan kernel
constexpr int kXMaxQ = 16;          // largest points per lane of the x scan kernel
hipError_t launch_observables(gp_plan *p, const void *psi, hipStream_t s);
hipError_t launch_obs_final(gp_plan *p, double *part, int64_t nb, hipStream_t s);  // row nb = sums of rows 0..nb-1
// Observables from the kObsFields final sums (norm, E parts, mu, rms) of a grid.
void obs_from_sums(const double *f, int ndim, const double *dx, double g, gp_obs *out);
hipError_t launch_adj_reduce(gp_plan *p, int64_t nparts, double hw_coeff, double *dsched_k,
                             double *dg, hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, int64_t bytes, hipStream_t s);

// Number of workgroups a sweep along `axis` launches.
int64_t sweep_groups(const gp_plan *p, int axis);
int64_t obs_groups(const gp_plan *p);
int64_t obs_groups_of(int ndim, const int64_t *n);  // workgroups of the observables kernel for a grid
constexpr int kObsFields = 10;
constexpr int kObsThreads = 256;

void omega_at_step(const gp_plan *p, int64_t step, double w[3]);

// Symmetric traps (gp_radial.hip).
inline int radial_dim(int geom) { return geom == GP_SPHERICAL ? 3 : 2; }
double axis_x0(const gp_plan *p, int axis);  // coordinate of index i on an axis: (i + x0) dx
int64_t radial_line_groups(const gp_plan *p);
int64_t radial_norm_groups(const gp_plan *p);
hipError_t launch_radial_line(gp_plan *p, const void *src, void *dst, int flags, int64_t step_index, hipStream_t s);
hipError_t launch_radial_norm(gp_plan *p, const void *psi, int64_t step_index, hipStream_t s);
// nsteps steps of a circular or spherical plan (one radial line) from p->step in
// one launch; *total_out gets the last step's norm total.
hipError_t launch_radial_steps(gp_plan *p, void *psi, int64_t nsteps, double *total_out, hipStream_t s);
hipError_t launch_radial_obs(gp_plan *p, const void *psi, double *part, int64_t nb, hipStream_t s);

// Window choice of one axis exactly as gp_plan_create makes it (host only, no
// device tables): for checks that must run before any HIP call.
AxisPlan preview_axis(int64_t n, int64_t nlines, double dx, double dt, gp_mode mode, gp_prec prec, int B,
                      bool tile);

}  // namespace gp

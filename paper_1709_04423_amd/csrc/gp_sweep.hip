// Plan-level side of the line sweeps: sweep parameters, workgroup counts and
// the launch of one axis's sweep (the kernels are in gp_sweep_kernels.h, one
// translation unit per precision).
#include "gp_internal.h"

namespace gp {

double axis_x0(const gp_plan *p, int axis)
{
    // radial axes are cell-centred from r = 0: r_i = (i + 1/2) dr
    if (axis == 0 && p->geom != GP_CARTESIAN) return 0.5;
    return coord0(p->n[axis]);
}

int64_t sweep_groups(const gp_plan *p, int axis)
{
    if (axis == 0 && p->geom != GP_CARTESIAN) return radial_line_groups(p);
    const AxisPlan &A = p->ax[axis];
    if (A.xq > 0) return (A.nlines + kXWavesPerGroup * A.xlpw - 1) / (kXWavesPerGroup * A.xlpw);
    const int64_t g = (A.nlines + kLanes - 1) / kLanes;
    return A.K < 0 ? g : g * A.segs;
}

void omega_at_step(const gp_plan *p, int64_t step, double w[3])
{
    for (int a = 0; a < 3; ++a) w[a] = a < p->ndim ? p->omega[a] : 0.0;
    if (!p->sched.empty() && step >= 0 && step < (int64_t)p->sched.size()) w[p->sched_axis] = p->sched[step];
}

SweepParams make_sweep_params(const gp_plan *p, int axis, const void *src, void *dst, bool adjoint,
                              int64_t step_index, const void *state)
{
    const AxisPlan &A = p->ax[axis];
    SweepParams P{};
    P.psi = const_cast<void *>(src);
    P.out = dst;
    P.state = state;
    P.n = A.n;
    P.stride = A.stride;
    P.nlines = A.nlines;
    P.m1 = A.m1;
    P.s1 = A.s1;
    P.s2 = A.s2;
    P.tab = adjoint ? A.d_tab_adj : A.d_tab;
    P.K = A.K < 0 ? 0 : A.K;
    P.lmask = A.L > 0 ? A.L - 1 : 0;
    P.D = A.D;
    P.nblocks = A.B > 0 ? (int)((A.n + A.B - 1) / A.B) : 0;
    P.dt = p->dt;
    P.g = p->g;
    double w[3];
    omega_at_step(p, step_index, w);
    for (int a = 0; a < 3; ++a) {
        P.hw2[a] = a < p->ndim ? 0.5 * w[a] * w[a] : 0.0;
        P.x0[a] = a < p->ndim ? axis_x0(p, a) : 0.0;
        P.dx[a] = a < p->ndim ? p->dx[a] : 0.0;
    }
    P.ny = p->ndim >= 2 ? p->n[1] : 1;
    P.sched_axis = p->sched_axis;
    P.norm_total = norm_total(const_cast<gp_plan *>(p), step_index - 1);
    P.dV = p->dV;
    P.norm_out = norm_partials(const_cast<gp_plan *>(p), step_index);
    P.n_norm = p->n_norm;
    P.adj_out = p->d_adj;
    P.scan_steps = A.scan_steps;
    P.q_const = A.q_const;
    const double sg = adjoint ? -1.0 : 1.0;  // the conjugate map's constants
    P.c_inf[0] = A.c_inf[0];
    P.c_inf[1] = sg * A.c_inf[1];
    P.b_inf[0] = A.b_inf[0];
    P.b_inf[1] = sg * A.b_inf[1];
    P.b_inf[2] = sg * A.b_inf[2];
    P.xmul = adjoint ? A.d_xmul_adj : A.d_xmul;
    P.xq = A.xq;
    P.xlpw = A.xlpw;
    P.radial_d = p->geom == GP_CARTESIAN ? 0 : radial_dim(p->geom);
    return P;
}

hipError_t launch_sweep(gp_plan *p, int axis, const void *src, void *dst, int flags, bool adjoint,
                        int64_t step_index, const void *state, hipStream_t s, const SweepExtras *extras)
{
    const AxisPlan &A = p->ax[axis];
    SweepParams P = make_sweep_params(p, axis, src, dst, adjoint, step_index, state);
    if (extras) {
        P.adj_done = extras->adj_done;
        P.adj_dsched = extras->adj_dsched;
        P.adj_dg = extras->adj_dg;
        P.adj_coeff = extras->adj_coeff;
        P.copy_out = extras->copy_out;
    }
    const bool exact = A.K < 0;
    const bool tr = axis == 0;  // x lines too long for the scan kernel: coalesced through an LDS tile
    const void *tab = P.tab;
    int kind = exact ? K_SWEEP_EXACT : (axis == 0 ? K_SWEEP_X : (axis == 1 ? K_SWEEP_Y : K_SWEEP_Z));
    if (flags & F_ADJ_N) kind = K_ADJ_X;
    else if (adjoint) kind = K_ADJ_YZ;
    if (axis == 0 && A.xq > 0) {  // one wavefront per x line
        timing_begin(p, (flags & F_ADJ_N) ? K_ADJ_X : K_SWEEP_X, s);
        hipError_t e = launch_x_scan(p, P, flags, tab, s);
        timing_end(p, s);
        return e;
    }
    if (A.xq > 0) {  // strided axis, one wavefront per line
        timing_begin(p, kind, s);
        hipError_t e = launch_col_scan(p, axis, P, flags, tab, s);
        timing_end(p, s);
        return e;
    }
    timing_begin(p, kind, s);
    hipError_t e;
    if (p->prec == GP_C128)
        e = dispatch_sweep_c128(A, P, p->mode, flags, exact, tr, tab, s);
    else
        e = dispatch_sweep_c64(A, P, p->mode, flags, exact, tr, tab, s);
    timing_end(p, s);
    return e;
}

}  // namespace gp

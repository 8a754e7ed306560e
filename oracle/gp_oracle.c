/*
 * gp_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow FP64 CPU reference of the split-step Crank-Nicolson (SSCN)
 * time step for the dimensionless Gross-Pitaevskii equation
 *
 *     i dpsi/dt = [ -1/2 laplacian + V + g |psi|^2 ] psi,   V = 1/2 sum_a w_a^2 x_a^2,
 *
 * in 1, 2 or 3 dimensions, in imaginary time (stationary states) and real time
 * (dynamics).  The paper (program summary, "Solution method" and "Nature of
 * problem") names the method -- split-step Crank-Nicolson discretisation in
 * space and time, propagated in imaginary or real time -- and defers the
 * formulas to its earlier publications; the readings used where it is silent
 * are listed below and in the design notes.
 *
 * Only tests/, the package smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header, table or helper with the GPU
 * path; nothing here is tuned.  OpenMP splits independent grid lines over host
 * cores (as the paper's OpenMP programs do) only to time a CPU baseline; every
 * floating-point reduction is a serial, compensated sum in a fixed order, so
 * results do not depend on the thread count and sums stay within a few ulps of
 * their exact value on any grid size.
 *
 * Readings of the paper (it states none of these):
 *  - grid: x_{a,i} = -N_a dx_a / 2 + i dx_a, i = 0..N_a-1; dV = prod dx_a;
 *  - Laplacian: 3-point second difference per axis, zero values at the ghost
 *    points i = -1 and i = N_a (zero Dirichlet walls);
 *  - one step (Lie splitting): pointwise potential + nonlinear propagator with
 *    |psi|^2 taken before the substep, then one Crank-Nicolson kinetic substep
 *    per axis in the order x, y, z; imaginary time then renormalises to 1;
 *  - CN substep along axis a with r = dt / (4 dx_a^2):
 *        real time : b = 1 + 2 i r, e = -i r;     imaginary time: b = 1 + 2 r, e = -r
 *        solve  b u'_i + e (u'_{i-1} + u'_{i+1}) = (2 - b) u_i - e (u_{i-1} + u_{i+1})
 *    with the plain Thomas algorithm (no pivoting; |b| > 2|e| always holds);
 *  - observables: rectangle sums; kinetic energy from forward differences over
 *    i = -1..N_a-1 with zero ghosts (equal to <psi, T psi> for the same T);
 *    mu = Ekin + Epot + 2 Eint, E = Ekin + Epot + Eint, uncentred rms sizes;
 *  - trap schedule: step n may replace w on one axis by sched[n] (0 <= n < len).
 *
 * Array layout: complex128 values stored as interleaved (re, im) doubles, x the
 * fastest index: p = i + N0 (j + N1 k).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORACLE_IMAG 0
#define ORACLE_REAL 1

/* ------------------------------------------------------------------ grid */

static double coord(int64_t i, int64_t n, double dx)
{
    return (double)i * dx - 0.5 * (double)n * dx;
}

static int64_t total_points(int ndim, const int64_t *n)
{
    int64_t t = 1;
    for (int a = 0; a < ndim; ++a) t *= n[a];
    return t;
}

static int64_t axis_stride(int ndim, const int64_t *n, int axis)
{
    int64_t s = 1;
    for (int a = 0; a < axis && a < ndim; ++a) s *= n[a];
    return s;
}

/* Trap frequency of axis a during step `step` (schedule overrides one axis). */
static double omega_at(const double *omega, const double *sched, int64_t sched_len,
                       int sched_axis, int64_t step, int a)
{
    if (sched && a == sched_axis && step >= 0 && step < sched_len) return sched[step];
    return omega[a];
}

static void point_coords(int ndim, const int64_t *n, const double *dx, int64_t p, double *x)
{
    int64_t rem = p;
    for (int a = 0; a < ndim; ++a) {
        int64_t i = rem % n[a];
        rem /= n[a];
        x[a] = coord(i, n[a], dx[a]);
    }
}

/* Compensated (Neumaier) running sum.  Every reduction of the oracle is the
 * plain sum of its definition taken in index order; a bare FP64 running sum
 * over 10^6..10^7 smoothly varying terms drifts by ~1e-12 relative, which is
 * the size of the GPU parity bar, while the compensated sum keeps the error
 * near 2 eps sum|x_i| whatever the grid size. */
typedef struct {
    double s, c;
} ksum;

static void ksum_add(ksum *k, double x)
{
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x))
        k->c += (k->s - t) + x;
    else
        k->c += (x - t) + k->s;
    k->s = t;
}

static double ksum_value(const ksum *k) { return k->s + k->c; }

static double potential(int ndim, const double *x, const double *w)
{
    double v = 0.0;
    for (int a = 0; a < ndim; ++a) v += 0.5 * w[a] * w[a] * x[a] * x[a];
    return v;
}

static double abs2(cplx z) { return creal(z) * creal(z) + cimag(z) * cimag(z); }

/* --------------------------------------------------- Crank-Nicolson parts */

/* Coefficients of the implicit side of the CN substep along one axis.
 * `adjoint` conjugates them: the Hermitian adjoint of the real-time CN map is
 * the same map with dt -> -dt. */
static void cn_coefficients(double dt, double dxa, int mode, int adjoint, cplx *b, cplx *e)
{
    double r = dt / (4.0 * dxa * dxa);
    if (mode == ORACLE_REAL) {
        *b = 1.0 + 2.0 * I * r;
        *e = -I * r;
    } else {
        *b = 1.0 + 2.0 * r;
        *e = -r;
    }
    if (adjoint) {
        *b = conj(*b);
        *e = conj(*e);
    }
}

/* Plain Thomas algorithm for tridiag(e, b, e) x = rhs of size n.
 * work holds n values.  Returns 0, or -1 if the matrix is not strictly
 * diagonally dominant (then the elimination is not known to be stable).
 *
 * The elimination factors and every product with them are carried in long
 * double (64-bit significand) and each result is rounded once to double.  The
 * factors are the same on every grid line (constant coefficients), so rounding
 * them to double would perturb the solved matrix identically on all lines: the
 * real-time Crank-Nicolson map, unitary in exact arithmetic, then changes the
 * norm by a fixed ~1e-16 per sweep (7e-13 over 1000 steps of a 128^3 grid).
 * Rounded in long double that perturbation is 2^11 times smaller, and the
 * remaining roundings of the data are unbiased. */
typedef long double complex lcplx;

static int thomas(int64_t n, cplx b, cplx e, const cplx *rhs, cplx *x, lcplx *work)
{
    if (n <= 0) return 0;
    if (!(cabs(b) > 2.0 * cabs(e))) return -1;
    const lcplx bl = b, el = e;
    work[0] = el / bl;
    x[0] = (cplx)((lcplx)rhs[0] / bl);
    for (int64_t i = 1; i < n; ++i) {
        const lcplx denom = bl - el * work[i - 1];
        work[i] = el / denom;
        x[i] = (cplx)(((lcplx)rhs[i] - el * (lcplx)x[i - 1]) / denom);
    }
    for (int64_t i = n - 2; i >= 0; --i) x[i] = (cplx)((lcplx)x[i] - work[i] * (lcplx)x[i + 1]);
    return 0;
}

/* One CN kinetic substep along `axis`, in place, over every line of the grid. */
static int cn_axis(int ndim, const int64_t *n, const double *dx, double dt, int mode,
                   int axis, int adjoint, cplx *psi)
{
    cplx b, e;
    cn_coefficients(dt, dx[axis], mode, adjoint, &b, &e);
    if (!(cabs(b) > 2.0 * cabs(e))) return -1;
    const int64_t len = n[axis];
    const int64_t stride = axis_stride(ndim, n, axis);
    const int64_t nlines = total_points(ndim, n) / len;
    int status = 0;

#pragma omp parallel
    {
        cplx *u = (cplx *)malloc(sizeof(cplx) * (size_t)len);
        cplx *rhs = (cplx *)malloc(sizeof(cplx) * (size_t)len);
        cplx *out = (cplx *)malloc(sizeof(cplx) * (size_t)len);
        lcplx *work = (lcplx *)malloc(sizeof(lcplx) * (size_t)len);
#pragma omp for schedule(static)
        for (int64_t line = 0; line < nlines; ++line) {
            /* first point of the line: split the line index into the part
             * below the axis (inner) and above it (outer). */
            int64_t inner = line % stride;
            int64_t outer = line / stride;
            int64_t base = inner + outer * stride * len;
            for (int64_t i = 0; i < len; ++i) u[i] = psi[base + i * stride];
            for (int64_t i = 0; i < len; ++i) {
                cplx left = (i > 0) ? u[i - 1] : 0.0;
                cplx right = (i + 1 < len) ? u[i + 1] : 0.0;
                rhs[i] = (2.0 - b) * u[i] - e * (left + right);
            }
            if (thomas(len, b, e, rhs, out, work) != 0) {
#pragma omp atomic write
                status = -1;
            }
            for (int64_t i = 0; i < len; ++i) psi[base + i * stride] = out[i];
        }
        free(u);
        free(rhs);
        free(out);
        free(work);
    }
    return status;
}

/* Pointwise potential + nonlinear propagator for step `step`. */
static void nonlinear(int ndim, const int64_t *n, const double *dx, double dt, int mode,
                      const double *omega, const double *sched, int64_t sched_len,
                      int sched_axis, int64_t step, double g, cplx *psi)
{
    double w[3];
    for (int a = 0; a < ndim; ++a) w[a] = omega_at(omega, sched, sched_len, sched_axis, step, a);
    const int64_t total = total_points(ndim, n);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < total; ++p) {
        double x[3];
        point_coords(ndim, n, dx, p, x);
        double theta = dt * (potential(ndim, x, w) + g * abs2(psi[p]));
        if (mode == ORACLE_REAL)
            psi[p] *= cexp(-I * theta);
        else
            psi[p] *= exp(-theta);
    }
}

static double norm_of(int ndim, const int64_t *n, const double *dx, const cplx *psi)
{
    double dv = 1.0;
    for (int a = 0; a < ndim; ++a) dv *= dx[a];
    ksum s = {0.0, 0.0};
    const int64_t total = total_points(ndim, n);
    for (int64_t p = 0; p < total; ++p) ksum_add(&s, abs2(psi[p]));
    return ksum_value(&s) * dv;
}

static int check_args(int ndim, const int64_t *n, const double *dx, double dt, int mode)
{
    if (ndim < 1 || ndim > 3 || !n || !dx) return -2;
    for (int a = 0; a < ndim; ++a)
        if (n[a] < 1 || !(dx[a] > 0.0)) return -2;
    if (!(dt > 0.0) || (mode != ORACLE_IMAG && mode != ORACLE_REAL)) return -2;
    return 0;
}

/* ------------------------------------------------------------ public API */

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Number of OpenMP threads for the line loops (results do not depend on it). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Thomas solve of tridiag(e, b, e) x = rhs; arrays interleaved (re, im). */
int oracle_thomas(int64_t n, double br, double bi, double er, double ei, const double *rhs,
                  double *x)
{
    if (n < 0) return -2;
    lcplx *work = (lcplx *)malloc(sizeof(lcplx) * (size_t)(n > 0 ? n : 1));
    int s = thomas(n, br + I * bi, er + I * ei, (const cplx *)rhs, (cplx *)x, work);
    free(work);
    return s;
}

/* One CN kinetic substep along one axis (adjoint != 0: the conjugate map). */
int oracle_cn_axis(int ndim, const int64_t *n, const double *dx, double dt, int mode, int axis,
                   int adjoint, double *psi)
{
    int s = check_args(ndim, n, dx, dt, mode);
    if (s) return s;
    if (axis < 0 || axis >= ndim) return -2;
    return cn_axis(ndim, n, dx, dt, mode, axis, adjoint, (cplx *)psi);
}

/* Pointwise potential + nonlinear substep alone (step index selects the schedule). */
int oracle_nonlinear(int ndim, const int64_t *n, const double *dx, double dt, int mode,
                     const double *omega, const double *sched, int64_t sched_len,
                     int sched_axis, int64_t step, double g, double *psi)
{
    int s = check_args(ndim, n, dx, dt, mode);
    if (s) return s;
    nonlinear(ndim, n, dx, dt, mode, omega, sched, sched_len, sched_axis, step, g, (cplx *)psi);
    return 0;
}

/* `nsteps` full SSCN steps, the first with schedule index n0. */
int oracle_step(int ndim, const int64_t *n, const double *dx, double dt, int mode,
                const double *omega, const double *sched, int64_t sched_len, int sched_axis,
                double g, int64_t n0, int64_t nsteps, double *psi_ri)
{
    int s = check_args(ndim, n, dx, dt, mode);
    if (s) return s;
    cplx *psi = (cplx *)psi_ri;
    const int64_t total = total_points(ndim, n);
    for (int64_t k = 0; k < nsteps; ++k) {
        nonlinear(ndim, n, dx, dt, mode, omega, sched, sched_len, sched_axis, n0 + k, g, psi);
        for (int a = 0; a < ndim; ++a)
            if (cn_axis(ndim, n, dx, dt, mode, a, 0, psi) != 0) return -1;
        if (mode == ORACLE_IMAG) {
            double nrm = norm_of(ndim, n, dx, psi);
            if (!(nrm > 0.0) || !isfinite(nrm)) return -3;
            double scale = 1.0 / sqrt(nrm);
            for (int64_t p = 0; p < total; ++p) psi[p] *= scale;
        }
    }
    return 0;
}

/* Observables of psi with static trap omega:
 * out = {norm, mu, energy, ekin, epot, eint, rms_x, rms_y, rms_z}. */
int oracle_observables(int ndim, const int64_t *n, const double *dx, const double *omega,
                       double g, const double *psi_ri, double *out)
{
    if (ndim < 1 || ndim > 3) return -2;
    const cplx *psi = (const cplx *)psi_ri;
    const int64_t total = total_points(ndim, n);
    double dv = 1.0;
    for (int a = 0; a < ndim; ++a) dv *= dx[a];

    ksum sum_n = {0.0, 0.0}, sum_v = {0.0, 0.0}, sum_4 = {0.0, 0.0};
    ksum sum_x2[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    for (int64_t p = 0; p < total; ++p) {
        double x[3];
        point_coords(ndim, n, dx, p, x);
        double d = abs2(psi[p]);
        ksum_add(&sum_n, d);
        ksum_add(&sum_v, potential(ndim, x, omega) * d);
        ksum_add(&sum_4, d * d);
        for (int a = 0; a < ndim; ++a) ksum_add(&sum_x2[a], x[a] * x[a] * d);
    }

    /* kinetic: forward differences along each axis, ghosts zero on both ends */
    double ekin = 0.0;
    for (int a = 0; a < ndim; ++a) {
        const int64_t len = n[a];
        const int64_t stride = axis_stride(ndim, n, a);
        const int64_t nlines = total / len;
        ksum s = {0.0, 0.0};
        for (int64_t line = 0; line < nlines; ++line) {
            int64_t base = (line % stride) + (line / stride) * stride * len;
            for (int64_t i = -1; i < len; ++i) {
                cplx lo = (i >= 0) ? psi[base + i * stride] : 0.0;
                cplx hi = (i + 1 < len) ? psi[base + (i + 1) * stride] : 0.0;
                ksum_add(&s, abs2(hi - lo));
            }
        }
        ekin += 0.5 * dv * ksum_value(&s) / (dx[a] * dx[a]);
    }

    double norm = dv * ksum_value(&sum_n);
    double epot = dv * ksum_value(&sum_v);
    double eint = 0.5 * g * dv * ksum_value(&sum_4);
    out[0] = norm;
    out[1] = ekin + epot + 2.0 * eint;
    out[2] = ekin + epot + eint;
    out[3] = ekin;
    out[4] = epot;
    out[5] = eint;
    for (int a = 0; a < 3; ++a) out[6 + a] = (a < ndim) ? sqrt(dv * ksum_value(&sum_x2[a]) / norm) : 0.0;
    return 0;
}

/* Adjoint of one real-time step n (schedule index `step`), in the gradient
 * convention G = dL/dRe + i dL/dIm.
 *
 * Forward step: u = psi e^{-i theta}, theta = dt (V_n + g |psi|^2); then the CN
 * maps X, Y, Z.  Given lambda = G of the step output and psi = the step input,
 * on return lambda = G of the step input and
 *   *dtheta_w = dt * sum_p w_p x_{s,p}^2   (times w_s(n) gives dL/dw_s(n)),
 *   *dg       = dt * sum_p w_p |u_p|^2,
 * with w = Im(conj(lambda_u) u) and lambda_u the gradient of u. */
int oracle_adjoint_step(int ndim, const int64_t *n, const double *dx, double dt,
                        const double *omega, const double *sched, int64_t sched_len,
                        int sched_axis, double g, int64_t step, const double *psi_ri,
                        double *lambda_ri, double *dtheta_w, double *dg)
{
    int s = check_args(ndim, n, dx, dt, ORACLE_REAL);
    if (s) return s;
    cplx *lam = (cplx *)lambda_ri;
    const cplx *psi = (const cplx *)psi_ri;

    /* the CN maps in reverse order, each replaced by its adjoint */
    for (int a = ndim - 1; a >= 0; --a)
        if (cn_axis(ndim, n, dx, dt, ORACLE_REAL, a, 1, lam) != 0) return -1;

    double w_axis[3];
    for (int a = 0; a < ndim; ++a)
        w_axis[a] = omega_at(omega, sched, sched_len, sched_axis, step, a);
    const int64_t total = total_points(ndim, n);
    ksum sum_wx = {0.0, 0.0}, sum_wd = {0.0, 0.0};
    for (int64_t p = 0; p < total; ++p) {
        double x[3];
        point_coords(ndim, n, dx, p, x);
        double d = abs2(psi[p]);
        double theta = dt * (potential(ndim, x, w_axis) + g * d);
        cplx u = psi[p] * cexp(-I * theta);
        double w = cimag(conj(lam[p]) * u);
        lam[p] = cexp(I * theta) * lam[p] + 2.0 * dt * g * w * psi[p];
        int sa = (sched_axis >= 0 && sched_axis < ndim) ? sched_axis : 0;
        ksum_add(&sum_wx, w * x[sa] * x[sa]);
        ksum_add(&sum_wd, w * d);
    }
    *dtheta_w = dt * ksum_value(&sum_wx);
    *dg = dt * ksum_value(&sum_wd);
    return 0;
}

/* ====================================================== symmetric traps ==
 * The paper's programs also solve the equation for three trap symmetries that
 * reduce the dimension ("Nature of problem"): circularly symmetric 2D traps
 * (psi(r)), spherically symmetric 3D traps (psi(r)) and axially symmetric 3D
 * traps (psi(rho, z)).  The discretisation is left to the earlier papers, so
 * the reading used here (and by the GPU path) is:
 *  - cell-centred radial grid r_i = (i + 1/2) dr, i = 0..N-1, zero ghost at
 *    i = N (the outer wall); no boundary condition is needed at r = 0 because
 *    the face there has zero area;
 *  - finite-volume radial Laplacian in d dimensions (d = 2 circular and axial,
 *    3 spherical): with face areas a_{i+1/2} = ((i+1) dr)^(d-1) and cell
 *    weights w_i = [ r_{i+1/2}^d - r_{i-1/2}^d ] / (d dr) (the exact cell volume
 *    over dr: r_i in 2D, r_i^2 + dr^2/12 in 3D),
 *        (L psi)_i = [ a_{i+1/2} (psi_{i+1} - psi_i) - a_{i-1/2} (psi_i - psi_{i-1}) ] / (w_i dr^2),
 *    which is self-adjoint in <u, v> = sum_i w_i conj(u_i) v_i: with
 *    S = -1/2 W L (symmetric tridiagonal) the CN substep solves
 *        (W + i tau S) psi' = (W - i tau S) psi,   tau = dt/2 (real time),
 *        (W + tau S) psi' = (W - tau S) psi                  (imaginary time),
 *    so real-time substeps conserve sum w |psi|^2 exactly;
 *  - axial: the rho substep as above (d = 2), then a Cartesian CN substep
 *    along z with the z grid of the Cartesian programs; the two commute;
 *  - norm = m sum_i w_i |psi_i|^2 with m = 2 pi dr (circular), 4 pi dr
 *    (spherical), 2 pi drho dz (axial); V = 1/2 (w_r^2 r^2 + w_z^2 z^2).
 * Observables: E_kin = m/2 [ sum_faces a |psi_{i+1} - psi_i|^2 / dr^2 (the outer
 * face to the zero ghost included) + sum w |psi_{j+1} - psi_j|^2 / dz^2 (axial,
 * z faces as in the Cartesian programs) ], which is <psi, T psi>; E_pot, E_int,
 * norm as weighted sums; rms[0] = sqrt(<r^2>) (rho^2 for axial), rms[1] =
 * sqrt(<z^2>) (axial). */

#define ORACLE_CIRCULAR 1
#define ORACLE_SPHERICAL 2
#define ORACLE_AXIAL 3

static int radial_dim(int geom) { return geom == ORACLE_SPHERICAL ? 3 : 2; }

static double radial_face(int64_t i, double dr, int d)  /* a_{i-1/2} = (i dr)^(d-1) */
{
    double r = (double)i * dr;
    return d == 3 ? r * r : r;
}

static double radial_weight(int64_t i, double dr, int d)
{
    double r = ((double)i + 0.5) * dr;
    return d == 3 ? r * r + dr * dr / 12.0 : r;
}

static double radial_measure(int geom, const double *dx)
{
    const double pi = 3.14159265358979323846;
    if (geom == ORACLE_CIRCULAR) return 2.0 * pi * dx[0];
    if (geom == ORACLE_SPHERICAL) return 4.0 * pi * dx[0];
    return 2.0 * pi * dx[0] * dx[1];
}

/* General tridiagonal solve: sub[i] x_{i-1} + diag[i] x_i + sup[i] x_{i+1} = rhs[i]
 * (Thomas; factors and products in long double, results rounded to double). */
static int thomas_general(int64_t n, const cplx *sub, const cplx *diag, const cplx *sup, const cplx *rhs, cplx *x,
                          lcplx *work)
{
    if (n <= 0) return 0;
    lcplx den = diag[0];
    work[0] = (lcplx)sup[0] / den;
    x[0] = (cplx)((lcplx)rhs[0] / den);
    for (int64_t i = 1; i < n; ++i) {
        den = (lcplx)diag[i] - (lcplx)sub[i] * work[i - 1];
        if (cabsl(den) == 0.0L) return -1;
        work[i] = (lcplx)sup[i] / den;
        x[i] = (cplx)(((lcplx)rhs[i] - (lcplx)sub[i] * (lcplx)x[i - 1]) / den);
    }
    for (int64_t i = n - 2; i >= 0; --i) x[i] = (cplx)((lcplx)x[i] - work[i] * (lcplx)x[i + 1]);
    return 0;
}

/* One radial CN substep on every radial line (axis 0, contiguous). */
static int radial_cn(int geom, const int64_t *n, const double *dx, double dt, int mode, cplx *psi)
{
    const int d = radial_dim(geom);
    const int64_t nr = n[0], nlines = geom == ORACLE_AXIAL ? n[1] : 1;
    const double dr = dx[0], tau = 0.5 * dt;
    const cplx k = mode == ORACLE_REAL ? I * tau : tau;  /* implicit side W + k S, explicit W - k S */
    cplx *sub = malloc(sizeof(cplx) * nr), *dia = malloc(sizeof(cplx) * nr), *sup = malloc(sizeof(cplx) * nr);
    cplx *rhs = malloc(sizeof(cplx) * nr), *out = malloc(sizeof(cplx) * nr);
    lcplx *work = malloc(sizeof(lcplx) * nr);
    int status = 0;
    for (int64_t line = 0; line < nlines && status == 0; ++line) {
        cplx *u = psi + line * nr;
        for (int64_t i = 0; i < nr; ++i) {
            const double lo = radial_face(i, dr, d), hi = radial_face(i + 1, dr, d), w = radial_weight(i, dr, d);
            const double s_d = (lo + hi) / (2.0 * dr * dr), s_lo = -lo / (2.0 * dr * dr), s_hi = -hi / (2.0 * dr * dr);
            sub[i] = k * s_lo;
            dia[i] = w + k * s_d;
            sup[i] = k * s_hi;
            cplx ex = (w - k * s_d) * u[i];
            if (i > 0) ex -= k * s_lo * u[i - 1];
            if (i + 1 < nr) ex -= k * s_hi * u[i + 1];
            rhs[i] = ex;
        }
        status = thomas_general(nr, sub, dia, sup, rhs, out, work);
        for (int64_t i = 0; i < nr; ++i) u[i] = out[i];
    }
    free(sub); free(dia); free(sup); free(rhs); free(out); free(work);
    return status;
}

static double radial_norm(int geom, const int64_t *n, const double *dx, const cplx *psi)
{
    const int d = radial_dim(geom);
    const int64_t nr = n[0], nz = geom == ORACLE_AXIAL ? n[1] : 1;
    ksum s = {0.0, 0.0};
    for (int64_t j = 0; j < nz; ++j)
        for (int64_t i = 0; i < nr; ++i) ksum_add(&s, radial_weight(i, dx[0], d) * abs2(psi[j * nr + i]));
    return radial_measure(geom, dx) * ksum_value(&s);
}

static double radial_potential(int geom, const int64_t *n, const double *dx, const double *omega, int64_t i, int64_t j)
{
    const double r = ((double)i + 0.5) * dx[0];
    double v = 0.5 * omega[0] * omega[0] * r * r;
    if (geom == ORACLE_AXIAL) {
        const double z = coord(j, n[1], dx[1]);
        v += 0.5 * omega[1] * omega[1] * z * z;
    }
    return v;
}

static int check_radial(int geom, const int64_t *n, const double *dx, double dt, int mode)
{
    if (geom != ORACLE_CIRCULAR && geom != ORACLE_SPHERICAL && geom != ORACLE_AXIAL) return -2;
    const int nd = geom == ORACLE_AXIAL ? 2 : 1;
    return check_args(nd, n, dx, dt, mode);
}

/* `nsteps` SSCN steps of a symmetric-trap problem: potential + nonlinear
 * substep, CN along r (rho), then along z (axial), imaginary-time renormalisation.
 * psi: (n[1], n[0]) for axial (rho fastest), (n[0]) otherwise. */
int oracle_radial_step(int geom, const int64_t *n, const double *dx, double dt, int mode, const double *omega,
                       double g, int64_t nsteps, double *psi_ri)
{
    int s = check_radial(geom, n, dx, dt, mode);
    if (s) return s;
    cplx *psi = (cplx *)psi_ri;
    const int64_t nr = n[0], nz = geom == ORACLE_AXIAL ? n[1] : 1;
    const int64_t zn[2] = {nr, nz};
    for (int64_t k = 0; k < nsteps; ++k) {
        for (int64_t j = 0; j < nz; ++j)
            for (int64_t i = 0; i < nr; ++i) {
                cplx *p = &psi[j * nr + i];
                const double theta = dt * (radial_potential(geom, n, dx, omega, i, j) + g * abs2(*p));
                if (mode == ORACLE_REAL)
                    *p *= cexp(-I * theta);
                else
                    *p *= exp(-theta);
            }
        if (radial_cn(geom, n, dx, dt, mode, psi) != 0) return -1;
        if (geom == ORACLE_AXIAL && cn_axis(2, zn, dx, dt, mode, 1, 0, psi) != 0) return -1;
        if (mode == ORACLE_IMAG) {
            const double nrm = radial_norm(geom, n, dx, psi);
            if (!(nrm > 0.0) || !isfinite(nrm)) return -3;
            const double scale = 1.0 / sqrt(nrm);
            for (int64_t p = 0; p < nr * nz; ++p) psi[p] *= scale;
        }
    }
    return 0;
}

/* out = {norm, mu, energy, ekin, epot, eint, rms_r (rho), rms_z, 0}. */
int oracle_radial_observables(int geom, const int64_t *n, const double *dx, const double *omega, double g,
                              const double *psi_ri, double *out)
{
    if (geom != ORACLE_CIRCULAR && geom != ORACLE_SPHERICAL && geom != ORACLE_AXIAL) return -2;
    const cplx *psi = (const cplx *)psi_ri;
    const int d = radial_dim(geom);
    const int64_t nr = n[0], nz = geom == ORACLE_AXIAL ? n[1] : 1;
    const double dr = dx[0], m = radial_measure(geom, dx);
    ksum sn = {0, 0}, sv = {0, 0}, s4 = {0, 0}, sr2 = {0, 0}, sz2 = {0, 0}, kr = {0, 0}, kz = {0, 0};
    for (int64_t j = 0; j < nz; ++j) {
        for (int64_t i = 0; i < nr; ++i) {
            const cplx u = psi[j * nr + i];
            const double w = radial_weight(i, dr, d), dd = abs2(u), r = ((double)i + 0.5) * dr;
            ksum_add(&sn, w * dd);
            ksum_add(&sv, w * radial_potential(geom, n, dx, omega, i, j) * dd);
            ksum_add(&s4, w * dd * dd);
            ksum_add(&sr2, w * r * r * dd);
            if (geom == ORACLE_AXIAL) {
                const double z = coord(j, nz, dx[1]);
                ksum_add(&sz2, w * z * z * dd);
            }
            /* radial faces i+1/2: to the next cell, or to the zero ghost past the last */
            const cplx nxt = (i + 1 < nr) ? psi[j * nr + i + 1] : 0.0;
            ksum_add(&kr, radial_face(i + 1, dr, d) * abs2(nxt - u));
        }
    }
    if (geom == ORACLE_AXIAL)
        for (int64_t i = 0; i < nr; ++i) {
            const double w = radial_weight(i, dr, d);
            for (int64_t j = -1; j < nz; ++j) {
                const cplx lo = j >= 0 ? psi[j * nr + i] : 0.0, hi = j + 1 < nz ? psi[(j + 1) * nr + i] : 0.0;
                ksum_add(&kz, w * abs2(hi - lo));
            }
        }
    const double norm = m * ksum_value(&sn);
    double ekin = 0.5 * m * ksum_value(&kr) / (dr * dr);
    if (geom == ORACLE_AXIAL) ekin += 0.5 * m * ksum_value(&kz) / (dx[1] * dx[1]);
    const double epot = m * ksum_value(&sv), eint = 0.5 * g * m * ksum_value(&s4);
    out[0] = norm;
    out[1] = ekin + epot + 2.0 * eint;
    out[2] = ekin + epot + eint;
    out[3] = ekin;
    out[4] = epot;
    out[5] = eint;
    out[6] = sqrt(m * ksum_value(&sr2) / norm);
    out[7] = geom == ORACLE_AXIAL ? sqrt(m * ksum_value(&sz2) / norm) : 0.0;
    out[8] = 0.0;
    return 0;
}


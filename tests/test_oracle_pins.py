"""Pins of the FP64 CPU oracle against facts the mathematics fixes.

The paper prints no worked example for the SSCN step (it defers formulas and
outputs to its earlier publications), so every pin here is a closed form, an
invariant, a library routine solving the same problem another way, or a
convergence order.  Each is chosen so that a plausible slip in the oracle (a
dropped term, a wrong sign, an index shift, a transposed axis) fails at least
one of them.
"""
import numpy as np
import pytest
import scipy.fft
import scipy.sparse as sp
from scipy.linalg import eigh_tridiagonal

import oracle
from paper_1709_04423_amd import inputs


def coords(n, dx):
    return (np.arange(n) - n / 2.0) * dx


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


def cn_bte(dt, dx, mode):
    r = dt / (4 * dx * dx)
    return (1 + 2j * r, -1j * r) if mode == oracle.REAL else (1 + 2 * r, -r)


def laplace_1d(n, dx):
    """-1/2 d^2/dx^2 with zero ghosts, as a sparse matrix."""
    main = np.full(n, 1.0 / dx**2)
    off = np.full(n - 1, -0.5 / dx**2)
    return sp.diags([off, main, off], [-1, 0, 1], format="csr")


def kinetic_op(shape, dx):
    """T = sum_a -1/2 D_a^2 on a (Nz, Ny, Nx)-ordered grid (x fastest), via Kronecker sums."""
    n = shape[::-1]
    dims = len(n)
    T = None
    for a in range(dims):
        mats = [sp.identity(n[b], format="csr") for b in range(dims)]
        mats[a] = laplace_1d(n[a], dx[a])
        # kron order: slowest axis first
        m = mats[dims - 1]
        for b in range(dims - 2, -1, -1):
            m = sp.kron(m, mats[b], format="csr")
        T = m if T is None else T + m
    return T


# ---------------------------------------------------------------- Thomas

@pytest.mark.parametrize("mode", [oracle.IMAG, oracle.REAL])
@pytest.mark.parametrize("conj", [False, True])
def test_thomas_matches_dense_lu(mode, conj):
    rng = np.random.default_rng(1)
    for n in range(1, 17):
        for dt, dx in ((1e-3, 0.05), (0.1, 0.1), (2.0, 0.3)):
            b, e = cn_bte(dt, dx, mode)
            if conj:
                b, e = np.conj(b), np.conj(e)
            A = np.diag(np.full(n, b, dtype=complex))
            if n > 1:
                A += np.diag(np.full(n - 1, e, dtype=complex), 1) + np.diag(np.full(n - 1, e, dtype=complex), -1)
            rhs = rng.standard_normal(n) + 1j * rng.standard_normal(n)
            x = oracle.thomas(complex(b), complex(e), rhs)
            ref = np.linalg.solve(A, rhs)
            assert rel(x, ref) <= 1e-14, (n, dt, dx)


# ------------------------------------------------------ CN substep vs DST

def dst_cn(u, dt, dx, mode, axis):
    """CN substep by diagonalising the Dirichlet 3-point Laplacian with DST-I."""
    n = u.shape[axis]
    k = np.arange(1, n + 1)
    lam = (1 - np.cos(np.pi * k / (n + 1))) / dx**2  # eigenvalues of -1/2 D^2
    tau = dt / 2
    mult = (1 - 1j * tau * lam) / (1 + 1j * tau * lam) if mode == oracle.REAL else (1 - tau * lam) / (1 + tau * lam)
    shape = [1] * u.ndim
    shape[axis] = n
    c = scipy.fft.dst(u, type=1, norm="ortho", axis=axis)
    c = c * mult.reshape(shape)
    return scipy.fft.idst(c, type=1, norm="ortho", axis=axis)


@pytest.mark.parametrize("mode", [oracle.IMAG, oracle.REAL])
def test_cn_substep_matches_dst_1d(mode):
    u = inputs.random_field((256,), 3)
    for dt, dx in ((5e-4, 0.05), (1e-2, 0.05), (0.3, 0.1)):
        got = oracle.cn_axis(u, dx, dt, mode, 0)
        assert rel(got, dst_cn(u, dt, dx, mode, 0)) <= 1e-13


@pytest.mark.parametrize("mode", [oracle.IMAG, oracle.REAL])
def test_cn_substeps_3d_match_dst(mode):
    # anisotropic sizes and spacings so a transposed axis is caught
    shape = (7, 11, 13)  # (Nz, Ny, Nx)
    dx = (0.11, 0.13, 0.17)  # x, y, z
    u = inputs.random_field(shape, 4)
    dt = 0.02
    got = u
    ref = u
    for a in range(3):
        got = oracle.cn_axis(got, dx, dt, mode, a)
        ref = dst_cn(ref, dt, dx[a], mode, 2 - a)
        assert rel(got, ref) <= 1e-13, a


def test_cn_real_is_unitary_and_adjoint_is_inverse():
    u = inputs.random_field((9, 10, 12), 5)
    dx = (0.1, 0.2, 0.15)
    for a in range(3):
        v = oracle.cn_axis(u, dx, 0.05, oracle.REAL, a)
        assert abs(np.linalg.norm(v) / np.linalg.norm(u) - 1) <= 1e-14
        w = oracle.cn_axis(v, dx, 0.05, oracle.REAL, a, adjoint=True)
        assert rel(w, u) <= 1e-14


@pytest.mark.parametrize("mode", [oracle.IMAG, oracle.REAL])
def test_cn_adjoint_dot_product(mode):
    rng = np.random.default_rng(6)
    shape, dx = (6, 8, 10), (0.1, 0.12, 0.09)
    a = inputs.random_field(shape, 7)
    lam = inputs.random_field(shape, 8)
    for ax in range(3):
        lhs = np.vdot(lam, oracle.cn_axis(a, dx, 0.03, mode, ax)).real
        rhs = np.vdot(oracle.cn_axis(lam, dx, 0.03, mode, ax, adjoint=True), a).real
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


# ------------------------------------------------------- N substep

def test_nonlinear_modulus_and_semigroup():
    shape, dx, om, g = (8, 10, 12), (0.2, 0.25, 0.3), (1.0, 2.0, 3.0), 37.0
    u = inputs.random_field(shape, 9) * 0.3
    v = oracle.nonlinear(u, dx, 0.01, oracle.REAL, om, g)
    np.testing.assert_allclose(np.abs(v), np.abs(u), rtol=1e-15, atol=0)
    # real time: |psi| is conserved, so two substeps of dt compose to one of 2 dt
    v2 = oracle.nonlinear(oracle.nonlinear(u, dx, 0.01, oracle.REAL, om, g), dx, 0.01, oracle.REAL, om, g)
    assert rel(v2, oracle.nonlinear(u, dx, 0.02, oracle.REAL, om, g)) <= 1e-13
    # imaginary time, g = 0: pure decay, composes the same way
    w2 = oracle.nonlinear(oracle.nonlinear(u, dx, 0.01, oracle.IMAG, om, 0.0), dx, 0.01, oracle.IMAG, om, 0.0)
    assert rel(w2, oracle.nonlinear(u, dx, 0.02, oracle.IMAG, om, 0.0)) <= 1e-14
    # the potential vanishes only at the grid origin (index N/2 on every axis)
    z = oracle.nonlinear(np.ones(shape, complex), dx, 0.5, oracle.IMAG, om, 0.0)
    idx = np.unravel_index(np.argmax(np.abs(z)), shape)
    assert idx == (shape[0] // 2, shape[1] // 2, shape[2] // 2) and abs(z[idx] - 1) < 1e-15


def test_schedule_overrides_one_axis():
    shape, dx = (6, 8), (0.2, 0.25)
    u = inputs.random_field(shape, 10)
    sched = np.array([0.7, 1.3, 2.1])
    a = oracle.nonlinear(u, dx, 0.05, oracle.REAL, (1.0, 1.0), 3.0, sched, 0, 1)
    b = oracle.nonlinear(u, dx, 0.05, oracle.REAL, (1.3, 1.0), 3.0)
    assert rel(a, b) == 0
    c = oracle.nonlinear(u, dx, 0.05, oracle.REAL, (1.0, 1.0), 3.0, sched, 1, 5)  # past the end
    d = oracle.nonlinear(u, dx, 0.05, oracle.REAL, (1.0, 1.0), 3.0)
    assert rel(c, d) == 0


# ------------------------------------------------------- observables

def test_observables_of_gaussian_closed_forms():
    # rectangle sums of a well-resolved Gaussian are exact up to the rounding of
    # a serial sum over ~2e6 points (Poisson summation: aliasing ~ exp(-600))
    n, dx, om, g = (160, 120, 100), (0.1, 0.08, 0.07), (1.0, 2.0, 3.0), 10.0
    psi = inputs.gaussian(n, dx, om)
    o = oracle.observables(psi, dx, om, g)
    assert abs(o["norm"] - 1) < 2e-12
    for a in range(3):
        assert abs(o[("rms_x", "rms_y", "rms_z")[a]] - np.sqrt(0.5 / om[a])) < 2e-12
    assert abs(o["epot"] - sum(om) / 4) < 2e-12
    eint = 0.5 * g * np.prod([np.sqrt(w / (2 * np.pi)) for w in om])
    assert abs(o["eint"] - eint) < 1e-12 * eint
    # kinetic term: <psi, T psi> for the same 3-point T, built independently
    T = kinetic_op(psi.shape, dx)
    ek = np.prod(dx) * np.vdot(psi.ravel(), T @ psi.ravel()).real
    assert abs(o["ekin"] - ek) < 1e-12 * ek
    # and the continuum value sum(w)/4 up to the O(dx^2) lattice error
    assert abs(o["ekin"] - sum(om) / 4) < 0.01
    assert abs(o["mu"] - (o["ekin"] + o["epot"] + 2 * o["eint"])) < 1e-13
    assert abs(o["energy"] - (o["ekin"] + o["epot"] + o["eint"])) < 1e-13


def test_observable_sums_are_correctly_rounded_sums():
    # the observables are plain rectangle sums; on a 10^6-point grid the oracle
    # must return them to within a few ulps of math.fsum (correctly rounded) of
    # the same per-point terms, so its own summation error stays far below the
    # 1e-12 GPU parity bar (a bare running sum drifts by ~1e-13..1e-12 here)
    from math import fsum
    # Thomas-Fermi profile sqrt(max(mu - V, 0) / g) plus seeded noise: a plateau
    # of nearly equal terms, where rounding errors of a running sum add up
    n, dx, omega, g = (128, 96, 80), (0.1, 0.12, 0.15), (1.0, 1.3, 0.8), 250.0
    xs = [np.arange(n[a]) * dx[a] - 0.5 * n[a] * dx[a] for a in range(3)]
    V = (0.5 * omega[0] * omega[0] * xs[0] * xs[0])[None, None, :] \
        + (0.5 * omega[1] * omega[1] * xs[1] * xs[1])[None, :, None]
    V = V + (0.5 * omega[2] * omega[2] * xs[2] * xs[2])[:, None, None]
    tf = np.sqrt(np.maximum(4.0 - V, 0.0) / g)
    psi = tf / np.sqrt(dx[0] * dx[1] * dx[2] * np.sum(tf * tf)) + 1e-6 * inputs.random_field(tf.shape, 77)
    o = oracle.observables(psi, dx, omega, g)
    d = psi.real * psi.real + psi.imag * psi.imag
    dv = dx[0] * dx[1] * dx[2]
    norm = dv * fsum(d.ravel())
    epot = dv * fsum((V * d).ravel())
    eint = 0.5 * g * dv * fsum((d * d).ravel())
    ekin = 0.0
    for a in range(3):
        ax = 2 - a
        pad = [(0, 0)] * 3
        pad[ax] = (1, 1)
        diff = np.diff(np.pad(psi, pad), axis=ax)
        ekin += 0.5 * dv * fsum((diff.real * diff.real + diff.imag * diff.imag).ravel()) / (dx[a] * dx[a])
    ref = {"norm": norm, "epot": epot, "eint": eint, "ekin": ekin, "energy": ekin + epot + eint,
           "mu": ekin + epot + 2 * eint}
    for k, v in ref.items():
        assert abs(o[k] - v) <= 4e-15 * abs(v), (k, o[k], v)


def test_kinetic_energy_random_field_2d():
    shape, dx = (13, 17), (0.3, 0.2)
    psi = inputs.random_field(shape, 11)
    o = oracle.observables(psi, dx, (0.0, 0.0), 0.0)
    T = kinetic_op(shape, dx)
    ek = np.prod(dx) * np.vdot(psi.ravel(), T @ psi.ravel()).real
    assert abs(o["ekin"] - ek) < 1e-12 * ek
    assert o["epot"] == 0.0


# ------------------------------------------------- imaginary-time physics

def lambda_min(n, dx, w):
    x = coords(n, dx)
    d = 1 / dx**2 + 0.5 * w * w * x * x
    e = np.full(n - 1, -0.5 / dx**2)
    return float(eigh_tridiagonal(d, e, eigvals_only=True, select="i", select_range=(0, 0))[0])


def test_1d_g0_ground_state_matches_eigh_tridiagonal():
    w = inputs.ONE_D
    lam = lambda_min(512, w.dx, 1.0)
    assert abs(lam - 0.4999218627873122) < 1e-13
    psi = oracle.step(inputs.gaussian(w.n, w.dx, w.omega), w.dx, w.dt, oracle.IMAG, w.omega, 0.0, w.steps)
    o = oracle.observables(psi, w.dx, w.omega, 0.0)
    assert abs(o["norm"] - 1) < 1e-14
    assert abs(o["mu"] - lam) < 1e-6
    assert o["mu"] == o["energy"]
    assert abs(o["rms_x"] - np.sqrt(0.5)) < 1e-3


def test_3d_g0_ground_state_is_separable():
    n, dx, om = (24, 20, 16), (0.4, 0.3, 0.25), (1.0, 2.0, 3.0)
    lam = sum(lambda_min(n[a], dx[a], om[a]) for a in range(3))
    psi = oracle.step(inputs.gaussian(n, dx, om), dx, 2e-3, oracle.IMAG, om, 0.0, 1500)
    o = oracle.observables(psi, dx, om, 0.0)
    assert abs(o["mu"] - lam) < 1e-5
    assert abs(o["mu"] - 3.0) < 0.1  # continuum sum(w)/2 up to lattice error


def ground_state_1d(g, n=512, dx=0.05, dt=5e-4, steps=10_000):
    psi = inputs.gaussian((n,), dx, (1.0,))
    return oracle.step(psi, dx, dt, oracle.IMAG, (1.0,), g, steps)


def test_1d_ground_state_virial_and_self_consistency():
    g, dx = 62.74, 0.05
    psi = ground_state_1d(g)
    o = oracle.observables(psi, dx, (1.0,), g)
    # virial theorem for a harmonic trap in d = 1: 2 Ekin - 2 Epot + Eint = 0
    vir = 2 * o["ekin"] - 2 * o["epot"] + o["eint"]
    assert abs(vir) < 2e-3 * o["energy"]
    # psi is an eigenvector of H[psi] = T + V + g |psi|^2 with eigenvalue mu
    x = coords(512, dx)
    H = laplace_1d(512, dx) + sp.diags(0.5 * x * x + g * np.abs(psi) ** 2)
    res = H @ psi - o["mu"] * psi
    assert np.linalg.norm(res) / np.linalg.norm(psi) < 2e-2
    # Rayleigh quotient of the self-consistent H is mu
    rq = np.vdot(psi, H @ psi).real / np.vdot(psi, psi).real
    assert abs(rq - o["mu"]) < 1e-10 * o["mu"]


def test_thomas_fermi_trend_1d():
    # mu/mu_TF - 1 > 0 and shrinks as g grows; wide box so the cloud never touches the walls
    ratios = []
    for g in (62.74, 1000.0, 10000.0):
        psi = inputs.gaussian((2048,), 0.05, (1.0,))
        psi = oracle.step(psi, 0.05, 1e-3, oracle.IMAG, (1.0,), g, 8000)
        mu = oracle.observables(psi, 0.05, (1.0,), g)["mu"]
        mu_tf = 0.5 * (1.5 * g) ** (2.0 / 3.0)
        ratios.append(mu / mu_tf - 1)
    assert all(r > 0 for r in ratios)
    assert ratios[0] > ratios[1] > ratios[2]
    assert ratios[2] < 0.01


def test_dt_convergence_of_ground_state():
    g = 62.74
    mus = [oracle.observables(ground_state_1d(g, dt=dt, steps=int(5.0 / dt)), 0.05, (1.0,), g)["mu"]
           for dt in (2e-3, 1e-3, 5e-4)]
    d1, d2 = abs(mus[0] - mus[1]), abs(mus[1] - mus[2])
    assert d2 < 0.6 * d1  # at least first order in dt


# ------------------------------------------------------ real-time physics

def test_real_time_norm_and_energy_conservation():
    n, dx, om, g = (40, 48), (0.2, 0.2), (1.0, 1.3), 50.0
    psi0 = oracle.step(inputs.gaussian(n, dx, om), dx, 2e-3, oracle.IMAG, om, g, 400)
    om_q = (0.8, 1.3)  # perturbed trap
    e_dev = []
    for dt in (2e-3, 1e-3):
        psi = psi0
        e0 = oracle.observables(psi, dx, om_q, g)["energy"]
        n0 = oracle.observables(psi, dx, om_q, g)["norm"]
        dev = 0.0
        for _ in range(10):
            psi = oracle.step(psi, dx, dt, oracle.REAL, om_q, g, int(0.1 / dt))
            o = oracle.observables(psi, dx, om_q, g)
            # unitary substeps: only rounding of the phase factor (~5e-16 per step) moves it
            assert abs(o["norm"] - n0) < 1e-12
            dev = max(dev, abs(o["energy"] - e0))
        e_dev.append(dev)
    assert e_dev[0] < 1e-2
    assert 1.5 < e_dev[0] / e_dev[1] < 2.6  # first order in dt (Lie splitting)


def test_reversibility_of_one_real_step():
    shape, dx, om, g, dt = (10, 12, 14), (0.15, 0.2, 0.25), (1.0, 2.0, 3.0), 20.0, 0.01
    psi = inputs.random_field(shape, 12) * 0.3
    out = oracle.step(psi, dx, dt, oracle.REAL, om, g)
    back = out
    for a in (2, 1, 0):
        back = oracle.cn_axis(back, dx, dt, oracle.REAL, a, adjoint=True)
    # undo the N substep: |u| = |psi|, so theta is known from u itself
    x = [coords(shape[::-1][a], dx[a]) for a in range(3)]
    V = 0.5 * ((om[0] * x[0][None, None, :]) ** 2 + (om[1] * x[1][None, :, None]) ** 2
               + (om[2] * x[2][:, None, None]) ** 2)
    back = back * np.exp(1j * dt * (V + g * np.abs(back) ** 2))
    assert rel(back, psi) <= 1e-13


def test_g0_quench_closed_form():
    # <x^2>(t) after w0 = 1 -> w1 = 0.5: cos^2(w1 t)/(2 w0) + (w0/2) sin^2(w1 t)/w1^2
    ref = np.cos(0.5) ** 2 / 2 + 0.5 * np.sin(0.5) ** 2 / 0.25
    assert abs(ref - 0.84477) < 1e-5
    floors = []
    for n, dx in ((512, 0.05), (1024, 0.025)):
        gs = oracle.step(inputs.gaussian((n,), dx, (1.0,)), dx, 5e-4, oracle.IMAG, (1.0,), 0.0, 20000)
        errs = []
        for dt in (2e-3, 1e-3, 5e-4):
            psi = oracle.step(gs, dx, dt, oracle.REAL, (0.5,), 0.0, int(round(1.0 / dt)))
            errs.append(oracle.observables(psi, dx, (0.5,), 0.0)["rms_x"] ** 2 - ref)
        # first order in dt (Lie splitting): successive differences halve
        ratio = (errs[0] - errs[1]) / (errs[1] - errs[2])
        assert 1.8 < ratio < 2.2
        floors.append(2 * errs[2] - errs[1])  # dt -> 0 extrapolation: O(dx^2) lattice error
    assert abs(floors[0]) < 6e-4
    assert 3.0 < floors[0] / floors[1] < 5.0  # second order in dx


def test_kohn_mode_of_displaced_ground_state():
    # centre of mass oscillates at the trap frequency for any g (Kohn theorem)
    n, dx, g, x0 = 1024, 0.04, 40.0, 1.0
    gs = ground_state_1d(g, n=n, dx=dx, dt=1e-3, steps=6000)
    x = coords(n, dx)
    # displace by x0 via interpolation on the grid (shift by an integer number of cells)
    shift = int(round(x0 / dx))
    psi = np.roll(gs, shift)
    dt = 1e-3
    com = []
    for t_target in (np.pi / 2, np.pi):
        steps = int(round(t_target / dt))
        p = oracle.step(psi, dx, dt, oracle.REAL, (1.0,), g, steps)
        com.append(dx * np.sum(x * np.abs(p) ** 2) / (dx * np.sum(np.abs(p) ** 2)))
    xs = shift * dx
    assert abs(com[0]) < 5e-3 * xs
    assert abs(com[1] + xs) < 5e-3 * xs


# ------------------------------------------------------------ adjoint

def _richardson(f, h):
    d1 = (f(h) - f(-h)) / (2 * h)
    d2 = (f(h / 2) - f(-h / 2)) / h
    return (4 * d2 - d1) / 3


# The reverse sweep is pinned against central differences of the oracle's own
# forward map on every branch it has: the schedule on x, y and z (the weight
# x_s^2 of the schedule gradient comes from a different coordinate on each),
# 2D and 3D grids (one, two or three adjoint CN sweeps), g, and the initial state.
ADJOINT_CASES = [
    # (grid x first, dx, trap, g, dt, T, schedule axis)
    ((16, 12), (0.3, 0.35), (1.0, 1.0), 30.0, 5e-3, 20, 0),
    ((12, 16), (0.35, 0.3), (1.0, 1.2), 25.0, 5e-3, 16, 1),
    ((8, 10, 12), (0.45, 0.4, 0.35), (1.0, 1.3, 0.9), 15.0, 5e-3, 10, 2),
    ((10, 8, 9), (0.4, 0.45, 0.42), (1.1, 0.9, 1.0), 12.0, 5e-3, 8, 1),
]


@pytest.mark.parametrize("case", ADJOINT_CASES, ids=lambda c: f"{len(c[0])}d-axis{c[6]}")
def test_adjoint_matches_finite_differences(case):
    n, dx, om, g, dt, T, ax = case
    psi0 = inputs.gaussian(n, dx, om).astype(complex) + 0.02 * inputs.random_field(tuple(n[::-1]), 16)
    tgt_om = list(om)
    tgt_om[ax] = 1.4 * om[ax]
    tgt = inputs.gaussian(n, dx, tgt_om)
    sched = om[ax] * inputs.gamma_schedule(T)

    def loss(sc, gg, p0=psi0):
        psi = oracle.step(p0, dx, dt, oracle.REAL, om, gg, T, sc, ax, 0)
        return oracle.overlap_loss(psi, tgt, dx)[0]

    L, dsched, dg, lam0 = oracle.gradient(psi0, tgt, dx, dt, om, g, sched, ax)
    assert abs(L - loss(sched, g)) < 1e-15

    rng = np.random.default_rng(13 + ax)
    v = rng.standard_normal(T)
    v /= np.linalg.norm(v)
    fd = _richardson(lambda h: loss(sched + h * v, g), 1e-3)
    assert abs(fd - dsched @ v) <= 1e-8 * max(abs(fd), 1e-12) + 1e-12
    # single entries: rounding of the loss (~1e-16) divided by h = 1e-3 puts a
    # noise floor of a few 1e-13 under each Richardson difference
    for k in (0, T // 2, T - 1):
        e = np.zeros(T)
        e[k] = 1
        fd = _richardson(lambda h: loss(sched + h * e, g), 1e-3)
        assert abs(fd - dsched[k]) <= 1e-8 * abs(dsched).max() + 2e-12, k
    fd = _richardson(lambda h: loss(sched, g + h), 1e-2)
    assert abs(fd - dg) <= 1e-8 * abs(dg)
    # gradient w.r.t. the initial state, along a random complex direction
    d = inputs.random_field(psi0.shape, 14)
    d /= np.linalg.norm(d)
    fd = _richardson(lambda h: loss(sched, g, psi0 + h * d), 1e-3)
    assert abs(fd - np.vdot(lam0, d).real) <= 1e-8 * abs(fd)


def test_adjoint_schedule_weight_uses_the_schedule_axis():
    # the same step reversed with the schedule on each axis of an anisotropic 3D
    # grid: the schedule gradients differ by the weight x_s^2 alone, so with the
    # gradient lambda and the state fixed they must reproduce sum w x_s^2 for the
    # matching coordinate (a swapped axis index gives a different, nonzero value)
    n, dx, om, g, dt = (6, 8, 10), (0.5, 0.4, 0.3), (1.0, 1.0, 1.0), 20.0, 1e-2
    psi = inputs.gaussian(n, dx, om) + 0.1 * inputs.random_field((10, 8, 6), 17)
    lam = inputs.random_field((10, 8, 6), 18)
    x = [coords(n[a], dx[a]) for a in range(3)]
    X2 = [x[0][None, None, :] ** 2 * np.ones((10, 8, 6)), x[1][None, :, None] ** 2 * np.ones((10, 8, 6)),
          x[2][:, None, None] ** 2 * np.ones((10, 8, 6))]
    got = [oracle.adjoint_step(psi, lam, dx, dt, om, g, np.array([1.0]), a, 0)[1] for a in range(3)]
    # w from the definition: lambda_u = CN adjoints of lambda, u = psi e^{-i theta}
    lu = lam
    for a in (2, 1, 0):
        lu = oracle.cn_axis(lu, dx, dt, oracle.REAL, a, adjoint=True)
    V = 0.5 * (X2[0] + X2[1] + X2[2])
    u = psi * np.exp(-1j * dt * (V + g * np.abs(psi) ** 2))
    w = (np.conj(lu) * u).imag
    for a in range(3):
        assert abs(got[a] - dt * np.sum(w * X2[a])) <= 1e-12 * abs(got[a]), a
    assert len({round(v, 12) for v in got}) == 3


def test_threads_do_not_change_results():
    # fixed-order reductions: identical bits whatever the OpenMP thread count
    import subprocess, sys, json, os
    code = ("import numpy as np, oracle; from paper_1709_04423_amd import inputs;"
            "p=inputs.random_field((12,14,16),15);"
            "q=oracle.step(p,(0.1,0.1,0.1),1e-3,oracle.IMAG,(1,2,3),5.0,3);"
            "print(oracle.observables(q,(0.1,0.1,0.1),(1,2,3),5.0)['mu'].hex(), float(np.abs(q).sum()).hex())")
    outs = []
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for t in ("1", "4"):
        env = dict(os.environ, OMP_NUM_THREADS=t, PYTHONPATH=root)
        outs.append(subprocess.check_output([sys.executable, "-c", code], env=env, cwd=root).decode())
    assert outs[0] == outs[1]


# ------------------------------------------------------- density outputs

def test_reduced_densities_of_a_product_state_are_its_marginals():
    # a product of 1D Gaussians: integrating out axes leaves the product of the
    # remaining 1D factors times the Riemann sums of the integrated ones
    n, dx, om = (40, 30, 20), (0.2, 0.25, 0.3), (1.0, 2.0, 3.0)
    psi = inputs.gaussian(n, dx, om)
    f = [np.abs(inputs.gaussian((n[a],), dx[a], (om[a],))) ** 2 for a in range(3)]
    m = [dx[a] * np.sum(f[a]) for a in range(3)]  # Riemann sum of each factor
    for keep in range(3):
        got = oracle.reduced_density(psi, dx, [keep])
        others = [a for a in range(3) if a != keep]
        assert np.allclose(got, f[keep] * m[others[0]] * m[others[1]], rtol=1e-14, atol=0)
    got = oracle.reduced_density(psi, dx, [0, 2])  # integrate y out: (Nz, Nx)
    assert np.allclose(got, np.outer(f[2], f[0]) * m[1], rtol=1e-14, atol=0)
    assert abs(dx[0] * np.sum(oracle.reduced_density(psi, dx, [0])) - oracle.observables(psi, dx, om, 0)["norm"]) < 1e-14


def test_reduced_density_integrates_to_the_norm_on_a_random_field():
    psi = inputs.random_field((9, 11, 13), 21)
    dx = (0.1, 0.2, 0.3)
    norm = oracle.observables(psi, dx, (0, 0, 0), 0.0)["norm"]
    for keep in ([0], [1], [2], [0, 1], [1, 2], [0, 2]):
        d = oracle.reduced_density(psi, dx, keep)
        cell = np.prod([dx[a] for a in keep])
        assert abs(cell * np.sum(d) - norm) <= 1e-13 * norm, keep


def test_series_records_the_observables_of_each_step_block():
    n, dx, om, g, dt = (24, 20), (0.2, 0.25), (1.0, 1.3), 20.0, 1e-3
    psi = inputs.gaussian(n, dx, om) + 0.01 * inputs.random_field((20, 24), 22)
    rec = oracle.series(psi, dx, dt, oracle.REAL, om, g, 30, 10)
    assert len(rec) == 4
    assert rec[0] == oracle.observables(psi, dx, om, g)
    assert rec[3] == oracle.observables(oracle.step(psi, dx, dt, oracle.REAL, om, g, 30), dx, om, g)

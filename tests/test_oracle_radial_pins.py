"""Pins of the oracle's symmetric-trap programs (circular 2D, spherical 3D,
axial 3D; "Nature of problem") against what the mathematics fixes:

  - g = 0 ground states converge to the continuum oscillator energies (1, 3/2,
    1 + lambda/2) at second order in the radial spacing, and equal the lowest
    eigenvalue of the same discrete operator from scipy's tridiagonal solver;
  - axial at g = 0 is separable: its mu is the circular mu plus the 1D Cartesian
    z-oscillator mu on the same grids, to rounding;
  - g > 0: the circular ground state agrees with the 2D Cartesian oracle as both
    grids are refined; the virial theorem 2 Ekin - 2 Epot + d Eint = 0 and the
    Thomas-Fermi trend hold;
  - real time: the weighted norm is conserved, and after a trap quench the
    circular mean square radius oscillates at exactly twice the new trap
    frequency for any g (the 2D scale symmetry);
  - one CN substep equals a dense solve of the weighted Crank-Nicolson system.
"""
import numpy as np
import pytest
from scipy.linalg import eigh_tridiagonal

import oracle
from paper_1709_04423_amd import inputs

C, S, A = oracle.CIRCULAR, oracle.SPHERICAL, oracle.AXIAL


def r_grid(n, dr):
    return (np.arange(n) + 0.5) * dr


def gauss_r(n, dr):
    r = r_grid(n, dr)
    return np.exp(-0.5 * r * r).astype(complex)


def ground(geom, n, dr, g, omega=(1.0,), dt=1e-3, steps=6000, dz=None, nz=None):
    if geom == A:
        r = r_grid(n, dr)
        z = (np.arange(nz) - nz / 2) * dz
        psi = np.exp(-0.5 * omega[0] * r[None, :] ** 2 - 0.5 * omega[1] * z[:, None] ** 2).astype(complex)
        dx = (dr, dz)
    else:
        psi = gauss_r(n, dr)
        dx = dr
    psi = oracle.radial_step(psi, geom, dx, dt, oracle.IMAG, omega, g, steps)
    return psi, oracle.radial_observables(psi, geom, dx, omega, g)


def fv_operator(n, dr, d, omega):
    """Symmetric form of T + V for the finite-volume radial grid (W^-1/2 (S + W V) W^-1/2)."""
    i = np.arange(n)
    lo = (i * dr) ** (d - 1)
    hi = ((i + 1) * dr) ** (d - 1)
    r = (i + 0.5) * dr
    w = r if d == 2 else r * r + dr * dr / 12
    diag = (lo + hi) / (2 * dr * dr) / w + 0.5 * omega * omega * r * r
    off = -hi[:-1] / (2 * dr * dr) / np.sqrt(w[:-1] * w[1:])
    return diag, off


@pytest.mark.parametrize("geom,exact,d", [(C, 1.0, 2), (S, 1.5, 3)])
def test_g0_ground_state_second_order_and_eigensolver(geom, exact, d):
    errs = []
    for n, dr in ((120, 0.1), (240, 0.05)):
        _, o = ground(geom, n, dr, 0.0, dt=1e-3, steps=6000)
        diag, off = fv_operator(n, dr, d, 1.0)
        lam = eigh_tridiagonal(diag, off, eigvals_only=True, select="i", select_range=(0, 0))[0]
        assert abs(o["mu"] - lam) < 2e-6, (n, o["mu"], lam)  # Lie-splitting fixed point: O(dt^2)
        assert abs(o["mu"] - o["energy"]) < 1e-14
        errs.append(o["mu"] - exact)
    assert abs(errs[1]) < 1e-3
    assert 3.5 < errs[0] / errs[1] < 4.5  # second order in dr


def test_axial_g0_is_separable():
    nr, dr, nz, dz, lam = 80, 0.1, 96, 0.08, 2.0
    _, oa = ground(A, nr, dr, 0.0, omega=(1.0, lam), dt=2e-3, steps=5000, dz=dz, nz=nz)
    _, oc = ground(C, nr, dr, 0.0, dt=2e-3, steps=5000)
    z1 = oracle.step(inputs.gaussian((nz,), dz, (lam,)), dz, 2e-3, oracle.IMAG, (lam,), 0.0, 5000)
    o1 = oracle.observables(z1, dz, (lam,), 0.0)
    assert abs(oa["mu"] - (oc["mu"] + o1["mu"])) < 1e-11
    assert abs(oa["rms_r"] - oc["rms_r"]) < 1e-11 and abs(oa["rms_z"] - o1["rms_x"]) < 1e-11
    assert abs(oa["mu"] - (1.0 + lam / 2)) < 5e-3


def test_circular_agrees_with_cartesian_2d_as_grids_refine():
    g = 30.0
    _, o_cir = ground(C, 320, 0.025, g, dt=1e-3, steps=6000)
    gaps = []
    for n, dx in ((80, 0.2), (160, 0.1)):
        psi = oracle.step(inputs.gaussian((n, n), dx, (1.0, 1.0)), dx, 1e-3, oracle.IMAG, (1.0, 1.0), g, 6000)
        o = oracle.observables(psi, dx, (1.0, 1.0), g)
        gaps.append(abs(o["mu"] - o_cir["mu"]))
    assert gaps[1] < 0.5 * gaps[0] and gaps[1] < 5e-3


@pytest.mark.parametrize("geom,d", [(C, 2), (S, 3)])
def test_virial_and_thomas_fermi_trend(geom, d):
    ratios = []
    for g in (50.0, 500.0, 5000.0):
        _, o = ground(geom, 400, 0.05, g, dt=2e-3, steps=5000)
        vir = 2 * o["ekin"] - 2 * o["epot"] + d * o["eint"]
        assert abs(vir) < 5e-3 * o["energy"], (g, vir)
        mu_tf = np.sqrt(g / np.pi) if d == 2 else 0.5 * (15 * g / (4 * np.pi)) ** 0.4
        ratios.append(o["mu"] / mu_tf - 1)
    assert all(r > 0 for r in ratios) and ratios[0] > ratios[1] > ratios[2]


@pytest.mark.parametrize("geom", [C, S, A])
def test_real_time_conserves_weighted_norm(geom):
    if geom == A:
        psi, _ = ground(A, 60, 0.12, 40.0, omega=(1.0, 2.0), dt=5e-3, steps=300, dz=0.1, nz=64)
        dx, om = (0.12, 0.1), (0.8, 2.0)
    else:
        psi, _ = ground(geom, 200, 0.05, 40.0, dt=5e-3, steps=300)
        dx, om = 0.05, (0.8,)
    n0 = oracle.radial_observables(psi, geom, dx, om, 40.0)["norm"]
    e0 = oracle.radial_observables(psi, geom, dx, om, 40.0)["energy"]
    p = oracle.radial_step(psi, geom, dx, 1e-3, oracle.REAL, om, 40.0, 500)
    o = oracle.radial_observables(p, geom, dx, om, 40.0)
    assert abs(o["norm"] - n0) < 1e-13
    assert abs(o["energy"] - e0) < 1e-2 * abs(e0)


def test_circular_breathing_mode_at_twice_the_trap_frequency():
    # after w: 1 -> 1.25 the mean square radius oscillates at 2 w = 2.5 for any g
    w1, g, dt = 1.25, 20.0, 5e-4
    psi, _ = ground(C, 320, 0.025, g, dt=1e-3, steps=6000)
    period = 2 * np.pi / (2 * w1)
    r2 = []
    for t in (0.0, period / 2, period):
        p = psi if t == 0 else oracle.radial_step(psi, C, 0.025, dt, oracle.REAL, (w1,), g, int(round(t / dt)))
        r2.append(oracle.radial_observables(p, C, 0.025, (w1,), g)["rms_r"] ** 2)
    amp = abs(r2[1] - r2[0])
    assert amp > 0.1 * r2[0]                 # a real oscillation
    assert abs(r2[2] - r2[0]) < 5e-3 * amp   # back to the start after one period


@pytest.mark.parametrize("mode", [oracle.IMAG, oracle.REAL])
@pytest.mark.parametrize("geom,d", [(C, 2), (S, 3)])
def test_one_substep_equals_dense_weighted_cn_solve(geom, d, mode):
    n, dr, dt = 23, 0.15, 0.07
    rng = np.random.default_rng(5)
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    i = np.arange(n)
    lo, hi = (i * dr) ** (d - 1), ((i + 1) * dr) ** (d - 1)
    r = (i + 0.5) * dr
    w = r if d == 2 else r * r + dr * dr / 12
    Smat = np.diag((lo + hi) / (2 * dr * dr)) - np.diag(hi[:-1] / (2 * dr * dr), 1) - np.diag(hi[:-1] / (2 * dr * dr), -1)
    k = 1j * dt / 2 if mode == oracle.REAL else dt / 2
    ref = np.linalg.solve(np.diag(w) + k * Smat, (np.diag(w) - k * Smat) @ u)
    # one step of the oracle with g = 0 and no trap is exactly one CN substep
    got = oracle.radial_step(u, geom, dr, dt, mode, (0.0,), 0.0, 1)
    if mode == oracle.IMAG:  # the imaginary-time step renormalises afterwards
        ref = ref / np.sqrt(oracle.radial_observables(ref, geom, dr, (0.0,), 0.0)["norm"])
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)

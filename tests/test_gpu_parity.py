"""GPU parity: the HIP path (called through the C ABI) against the FP64 oracle,
element by element on the same seeded inputs.

FP64 (complex128) bar: every element within 1e-12 of the oracle, relative to
the largest |psi| (the FP64 parity bar: 1e-12 relative), and observables within
1e-12 relative.  FP32-bulk (complex64) bar: 1e-5 relative on norm, mu and energy
and on the elements (relative to max |psi|).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1709_04423_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_04423_amd import binding
    binding.lib()
    return binding


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def max_rel(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def run_case(gp, n, dx, dt, mode, omega, g, steps, prec=0, psi0=None, seed=0):
    shape = tuple(n[::-1])
    if psi0 is None:
        psi0 = inputs.gaussian(n, dx, omega) + 0.05 * inputs.random_field(shape, seed)
    dtype = np.complex128 if prec == 0 else np.complex64
    plan = gp.Plan(n, dx, dt, mode, omega, g, prec)
    say(f"case n={n} dx={dx} dt={dt} mode={mode} g={g} steps={steps} prec={prec} info={plan.info()}")
    psi = to_dev(psi0.astype(dtype))
    plan.step(psi, steps)
    torch.cuda.synchronize()
    got = psi.cpu().numpy().astype(np.complex128)
    ref = oracle.step(psi0.astype(dtype).astype(np.complex128), dx, dt, mode, omega, g, steps)
    return plan, psi, got, ref


CASES_FP64 = [
    # (n (x first), dx, dt, omega, g, steps)
    ((512,), (0.05,), 5e-4, (1.0,), 62.74, 1),
    ((512,), (0.05,), 5e-4, (1.0,), 62.74, 40),
    ((37,), (0.2,), 1e-2, (1.0,), 5.0, 3),
    ((1,), (0.2,), 1e-2, (1.0,), 5.0, 2),
    # 1D lines of 2 and 4 points per lane (a whole 1D run is one launch)
    ((100,), (0.1,), 1e-3, (1.0,), 20.0, 5),
    ((200,), (0.08,), 1e-3, (1.0,), 40.0, 4),
    ((70, 45), (0.1, 0.12), 1e-3, (1.0, 1.5), 30.0, 3),
    ((33, 130), (0.1, 0.05), 2e-3, (1.0, 0.7), 100.0, 2),
    ((64, 64), (0.1, 0.1), 1e-3, (1.0, 1.0), 200.0, 5),
    ((37, 29, 23), (0.2, 0.25, 0.3), 1e-3, (1.0, 2.0, 3.0), 50.0, 2),
    ((64, 48, 40), (0.2, 0.2, 0.25), 5e-4, (1.0, 1.0, 4.0), 100.0, 3),
    ((17, 1, 5), (0.3, 0.3, 0.3), 1e-2, (1.0, 1.0, 1.0), 3.0, 2),
    # long ragged strided lines: split into several segments per line
    ((40, 301, 20), (0.2, 0.04, 0.3), 2e-4, (1.0, 1.0, 2.0), 20.0, 2),
    ((50, 701), (0.2, 0.03), 2e-4, (1.0, 1.0), 20.0, 3),
    ((24, 20, 517), (0.3, 0.3, 0.025), 1e-4, (1.0, 1.0, 1.0), 20.0, 2),
    # lines of 513-1024 points: the scan solvers with their table rows in LDS (x, and 2D y)
    ((1000,), (0.02,), 1e-4, (1.0,), 10.0, 3),
    ((700, 30), (0.03, 0.3), 2e-4, (1.0, 1.0), 20.0, 2),
    ((60, 1000), (0.3, 0.02), 1e-4, (1.0, 1.0), 20.0, 2),
    # x lines longer than the scan kernel takes (64 x 16 points): windowed x solver
    ((2000,), (0.02,), 1e-4, (1.0,), 10.0, 3),
    ((1500, 12), (0.02, 0.3), 1e-4, (1.0, 1.0), 10.0, 2),
]


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("case", CASES_FP64, ids=lambda c: "x".join(map(str, c[0])) + f"_s{c[5]}")
def test_step_fp64_matches_oracle(gp, case, mode):
    n, dx, dt, omega, g, steps = case
    _, _, got, ref = run_case(gp, n, dx, dt, mode, omega, g, steps)
    err = max_rel(got, ref)
    say(f"  max rel err {err:.3e}")
    assert err <= FP64_TOL


@pytest.mark.parametrize("mode", [0, 1])
def test_exact_two_pass_path_matches_oracle(gp, mode):
    # dt/dx^2 large: the Thomas recurrence contracts slowly, the window does not
    # fit in LDS and the exact two-pass solver runs instead
    n, dx, dt, omega, g = (40, 36, 20), (0.05, 0.05, 0.05), 0.2, (1.0, 1.0, 1.0), 10.0
    plan, _, got, ref = run_case(gp, n, dx, dt, mode, omega, g, 2)
    assert min(plan.info()["window"][:3]) == -1
    assert max_rel(got, ref) <= FP64_TOL


def test_window_and_exact_paths_agree_on_medium_window(gp):
    # r = 0.3: window K ~ 30, still in LDS; compare against the oracle
    n, dx, dt, omega, g = (96, 80, 50), (0.05, 0.05, 0.05), 0.003, (1.0, 1.0, 1.0), 10.0
    plan, _, got, ref = run_case(gp, n, dx, dt, 1, omega, g, 2)
    w = plan.info()["window"]
    say(f"  windows {w}")
    assert all(k >= 16 for k in w[1:])  # strided axes: windowed solver with a deep window
    assert w[0] >= 16 or w[0] == -1     # x: scan kernel reaching as far (or the whole line)
    assert max_rel(got, ref) <= FP64_TOL


@pytest.mark.parametrize("mode", [0, 1])
def test_observables_match_oracle(gp, mode):
    for n, dx, omega, g in [((512,), (0.05,), (1.0,), 62.74), ((70, 45), (0.1, 0.12), (1.0, 1.5), 30.0),
                            ((37, 29, 23), (0.2, 0.25, 0.3), (1.0, 2.0, 3.0), 50.0)]:
        psi0 = inputs.gaussian(n, dx, omega) + 0.05 * inputs.random_field(tuple(n[::-1]), 3)
        plan = gp.Plan(n, dx, 1e-3, mode, omega, g, 0)
        say(f"observables n={n}")
        o = plan.observables(to_dev(psi0))
        r = oracle.observables(psi0, dx, omega, g)
        for k in ("norm", "mu", "energy", "ekin", "epot", "eint", "rms_x", "rms_y", "rms_z"):
            if r[k] == 0.0:
                assert o[k] == 0.0
            else:
                assert abs(o[k] - r[k]) <= FP64_TOL * abs(r[k]), (k, o[k], r[k])


def test_imag_time_returns_unit_norm_and_matches_oracle_observables(gp):
    w = inputs.ONE_D
    psi0 = inputs.gaussian(w.n, w.dx, w.omega)
    plan = gp.Plan(w.n, w.dx, w.dt, 0, w.omega, w.g)
    psi = to_dev(psi0)
    say("1d imag 2000 steps")
    plan.step(psi, 2000)
    o = plan.observables(psi)
    ref = oracle.step(psi0, w.dx, w.dt, 0, w.omega, w.g, 2000)
    r = oracle.observables(ref, w.dx, w.omega, w.g)
    for k in ("norm", "mu", "energy", "rms_x"):
        assert abs(o[k] - r[k]) <= FP64_TOL * abs(r[k]), (k, o[k], r[k])
    assert max_rel(psi.cpu().numpy(), ref) <= FP64_TOL


def test_steps_split_across_calls_equal_one_call(gp):
    n, dx, dt, omega, g = (40, 30, 20), (0.2, 0.2, 0.2), 1e-3, (1.0, 1.2, 1.4), 20.0
    psi0 = inputs.gaussian(n, dx, omega) + 0.05 * inputs.random_field(tuple(n[::-1]), 5)
    for mode in (0, 1):
        a = gp.Plan(n, dx, dt, mode, omega, g)
        b = gp.Plan(n, dx, dt, mode, omega, g)
        pa, pb = to_dev(psi0), to_dev(psi0)
        a.step(pa, 6)
        for _ in range(3):
            b.step(pb, 2)
        ga, gb = pa.cpu().numpy(), pb.cpu().numpy()
        if mode == 1:
            assert np.array_equal(ga, gb)  # same kernels, same order: identical bits
        else:
            # imaginary time renormalises at the end of each call: rounding differs
            assert max_rel(ga, gb) <= FP64_TOL
        assert a.info()["step"] == 6 and b.info()["step"] == 6


def test_1d_steps_split_across_calls_equal_one_call(gp):
    # a 1D call runs all its steps in one launch: splitting the call changes
    # nothing in real time, and only the end-of-call renormalisation's rounding
    # in imaginary time
    n, dx, dt, omega, g = (300,), (0.06,), 1e-3, (1.0,), 30.0
    psi0 = inputs.gaussian(n, dx, omega) + 0.05 * inputs.random_field(n, 9)
    for mode in (0, 1):
        a = gp.Plan(n, dx, dt, mode, omega, g)
        b = gp.Plan(n, dx, dt, mode, omega, g)
        pa, pb = to_dev(psi0), to_dev(psi0)
        a.step(pa, 12)
        for _ in range(4):
            b.step(pb, 3)
        ga, gb = pa.cpu().numpy(), pb.cpu().numpy()
        if mode == 1:
            assert np.array_equal(ga, gb)
        else:
            assert max_rel(ga, gb) <= FP64_TOL
        assert a.info()["step"] == 12 and b.info()["step"] == 12


def test_zero_steps_is_a_no_op(gp):
    psi0 = inputs.random_field((8, 9, 10), 6)
    plan = gp.Plan((10, 9, 8), (0.1, 0.1, 0.1), 1e-3, 0, (1, 1, 1), 1.0)
    psi = to_dev(psi0)
    plan.step(psi, 0)
    assert np.array_equal(psi.cpu().numpy(), psi0)


def test_schedule_matches_oracle(gp):
    n, dx, dt, g = (48, 40), (0.15, 0.15), 1e-3, 40.0
    sched = inputs.gamma_schedule(8)
    psi0 = inputs.gaussian(n, dx, (1.0, 1.0)) + 0.02 * inputs.random_field((40, 48), 7)
    plan = gp.Plan(n, dx, dt, 1, (1.0, 1.0), g, 0, sched=sched, sched_axis=0)
    psi = to_dev(psi0)
    plan.step(psi, 5)
    plan.step(psi, 6)  # runs past the end of the schedule: static omega afterwards
    ref = oracle.step(psi0, dx, dt, 1, (1.0, 1.0), g, 11, sched, 0, 0)
    assert max_rel(psi.cpu().numpy(), ref) <= FP64_TOL


@pytest.mark.parametrize("mode", [0, 1])
def test_fp32_bulk_matches_oracle(gp, mode):
    n, dx, dt, omega, g = (64, 48, 40), (0.2, 0.2, 0.25), 5e-4, (1.0, 1.0, 4.0), 100.0
    psi0 = inputs.noisy_gaussian(n, dx, omega, 11)
    plan, psi, got, ref = run_case(gp, n, dx, dt, mode, omega, g, 20, prec=1, psi0=psi0)
    err = max_rel(got, ref)
    say(f"  fp32 max rel err {err:.3e}")
    assert err <= FP32_TOL
    o = plan.observables(psi)
    r = oracle.observables(ref, dx, omega, g)
    for k in ("norm", "mu", "energy"):
        assert abs(o[k] - r[k]) <= FP32_TOL * abs(r[k]), (k, o[k], r[k])


def test_headline_grid_few_steps_matches_oracle(gp):
    # full 256^3 grid, the launch configuration the benchmark times, 2 steps per mode
    w = inputs.HEADLINE_3D
    psi0 = inputs.headline_initial()
    for mode in (0, 1):
        plan = gp.Plan(w.n, w.dx, w.dt, mode, w.omega, w.g)
        say(f"256^3 mode {mode}")
        psi = to_dev(psi0)
        plan.step(psi, 2)
        got = psi.cpu().numpy()
        ref = oracle.step(psi0, w.dx, w.dt, mode, w.omega, w.g, 2)
        err = max_rel(got, ref)
        say(f"  256^3 max rel err {err:.3e}")
        assert err <= FP64_TOL
        del psi
        torch.cuda.empty_cache()

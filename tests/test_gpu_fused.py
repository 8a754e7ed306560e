"""Fused x+y sweep of 3D steps (both variants: the y window in LDS, 1, and in
registers, 2): against the FP64 oracle, against the same plan with the sweeps
run as separate kernels, over x extents 128/192/256, ragged y extents and
several row segments per plane, in both modes and precisions."""
import sys

import numpy as np
import pytest

import oracle
from paper_1709_04423_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


CASES = [
    # (n (x first), dx, dt, omega, g, steps, expected row segments > 1)
    ((128, 22, 20), (0.2, 0.2, 0.25), 1e-3, (1.0, 1.5, 2.0), 50.0, 3, False),
    ((192, 201, 8), (0.1, 0.1, 0.3), 1e-3, (1.0, 1.2, 2.0), 80.0, 3, True),
    ((256, 42, 6), (0.05, 0.1, 0.3), 5e-4, (1.0, 2.0, 3.0), 200.0, 2, False),
    ((256, 130, 3), (0.05, 0.08, 0.4), 5e-4, (1.0, 1.0, 1.0), 20.0, 2, True),
]


def initial(n, dx, omega, seed):
    return inputs.gaussian(n, dx, omega) + 0.05 * inputs.random_field(tuple(n[::-1]), seed)


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[0])))
def test_fused_step_matches_oracle_and_separate_sweeps(gp, case, mode, variant):
    n, dx, dt, omega, g, steps, multi = case
    psi0 = initial(n, dx, omega, 7)
    plan = gp.Plan(n, dx, dt, mode, omega, g)
    plan.set_xy_fusion(variant)
    info = plan.info()
    say(f"fused n={n} mode={mode} variant={variant} info={info}")
    assert info["xy_fused"] >= 1
    assert (info["xy_fused"] > 1) == multi
    psi = to_dev(psi0)
    plan.step(psi, steps)
    got = psi.cpu().numpy()
    ref = oracle.step(psi0, dx, dt, mode, omega, g, steps)
    assert max_rel(got, ref) <= 1e-12
    # the same plan with separate x and y kernels
    sep = gp.Plan(n, dx, dt, mode, omega, g)
    sep.set_xy_fusion(False)
    assert sep.info()["xy_fused"] == 0
    psi2 = to_dev(psi0)
    sep.step(psi2, steps)
    assert max_rel(got, psi2.cpu().numpy()) <= 1e-13
    o, r = plan.observables(psi), oracle.observables(ref, dx, omega, g)
    for k in ("norm", "mu", "energy"):
        assert abs(o[k] - r[k]) <= 1e-12 * abs(r[k]), k


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("mode", [0, 1])
def test_fused_step_fp32(gp, mode, variant):
    n, dx, dt, omega, g, steps, _ = CASES[1]
    psi0 = initial(n, dx, omega, 8)
    plan = gp.Plan(n, dx, dt, mode, omega, g, gp.GP_C64)
    plan.set_xy_fusion(variant)
    say(f"fused fp32 n={n} mode={mode} variant={variant} info={plan.info()}")
    assert plan.info()["xy_fused"] >= 1
    psi = to_dev(psi0.astype(np.complex64))
    plan.step(psi, steps)
    ref = oracle.step(psi0.astype(np.complex64).astype(np.complex128), dx, dt, mode, omega, g, steps)
    assert max_rel(psi.cpu().numpy().astype(np.complex128), ref) <= 1e-5
    o, r = plan.observables(psi), oracle.observables(ref, dx, omega, g)
    for k in ("norm", "mu", "energy"):
        assert abs(o[k] - r[k]) <= 1e-5 * abs(r[k]), k


def test_unfusable_shapes_use_separate_sweeps(gp):
    for n in ((100, 40, 10), (64, 64, 8), (512, 16, 4), (40, 30)):
        dx = tuple([0.2] * len(n))
        plan = gp.Plan(n, dx, 1e-3, gp.GP_REAL, tuple([1.0] * len(n)), 10.0)
        assert plan.info()["xy_fused"] == 0, n


def test_fused_headline_grid_matches_separate_sweeps(gp):
    # 256^3 workload, 3 imaginary then 3 real steps, fused against separate kernels
    w = inputs.HEADLINE_3D
    psi0 = to_dev(inputs.headline_initial())
    out = []
    for fuse in (2, 1, 0):
        psi = psi0.clone()
        for mode in (gp.GP_IMAG, gp.GP_REAL):
            plan = gp.Plan(w.n, w.dx, w.dt, mode, w.omega, w.g)
            plan.set_xy_fusion(fuse)
            assert (plan.info()["xy_fused"] > 0) == (fuse > 0)
            plan.step(psi, 3)
        out.append(psi)
    for k, fuse in enumerate((2, 1)):
        d = float((out[k] - out[2]).abs().max() / out[2].abs().max())
        say(f"256^3 fused variant {fuse} vs separate: {d:.2e}")
        assert d <= 1e-13

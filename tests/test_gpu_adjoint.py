"""GPU adjoint (gp_step_adjoint through the C ABI) against the FP64 oracle's
adjoint, and long-run conservation checks of the forward path."""
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


def gpu_gradient(gp, psi0, tgt, n, dx, dt, omega, g, sched, prec=0, sched_axis=0):
    """Full-storage reverse sweep on the GPU: forward states, loss gradient, adjoint steps."""
    T = len(sched)
    dtype = torch.complex128 if prec == 0 else torch.complex64
    plan = gp.Plan(n, dx, dt, gp.GP_REAL, omega, g, prec, sched=sched, sched_axis=sched_axis)
    states = torch.empty((T,) + tuple(n[::-1]), dtype=dtype, device="cuda")
    psi = to_dev(psi0).to(dtype)
    for k in range(T):
        states[k].copy_(psi)
        plan.step(psi, 1)
    psiT = psi.to(torch.complex128)
    tg = to_dev(tgt)
    dv = float(np.prod(dx))
    c = dv * torch.sum(tg.conj() * psiT)
    lam = (-2.0 * c * dv * tg).to(dtype).contiguous()
    dsched = torch.zeros(T, dtype=torch.float64, device="cuda")
    dg = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan.adjoint(states, lam, 0, T, dsched, dg)
    torch.cuda.synchronize()
    return (1 - abs(c.item()) ** 2, dsched.cpu().numpy(), float(dg.item()), lam.cpu().numpy().astype(np.complex128))


@pytest.mark.parametrize("n,sched_axis", [((48, 40), 0), ((37, 29), 1), ((20, 18, 16), 2)])
def test_adjoint_matches_oracle_fp64(gp, n, sched_axis):
    dx = tuple([0.25] * len(n))
    omega = tuple([1.0] * len(n))
    dt, g, T = 2e-3, 40.0, 24
    psi0 = inputs.gaussian(n, dx, omega) + 0.02 * inputs.random_field(tuple(n[::-1]), 21)
    tgt = inputs.gaussian(n, dx, tuple([1.3] + [1.0] * (len(n) - 1)))
    sched = inputs.gamma_schedule(T)
    say(f"adjoint n={n} axis={sched_axis}")
    L, ds, dg, lam0 = gpu_gradient(gp, psi0, tgt, n, dx, dt, omega, g, sched, 0, sched_axis)
    Lr, dsr, dgr, lamr = oracle.gradient(psi0, tgt, dx, dt, omega, g, sched, sched_axis)
    assert abs(L - Lr) <= 1e-12 * abs(Lr)
    assert np.max(np.abs(ds - dsr)) <= 1e-10 * np.max(np.abs(dsr))
    assert abs(dg - dgr) <= 1e-10 * abs(dgr)
    assert np.max(np.abs(lam0 - lamr)) <= 1e-12 * np.max(np.abs(lamr))


def test_adjoint_fp32_error_is_small(gp):
    n, dx, omega, dt, g, T = (64, 48), (0.2, 0.2), (1.0, 1.0), 1e-3, 100.0, 40
    psi0 = inputs.gaussian(n, dx, omega)
    tgt = inputs.gaussian(n, dx, (1.5, 1.0))
    sched = inputs.gamma_schedule(T)
    _, ds, dg, _ = gpu_gradient(gp, psi0, tgt, n, dx, dt, omega, g, sched, 1)
    _, dsr, dgr, _ = oracle.gradient(psi0, tgt, dx, dt, omega, g, sched)
    err_s = np.max(np.abs(ds - dsr)) / np.max(np.abs(dsr))
    err_g = abs(dg - dgr) / abs(dgr)
    say(f"fp32 adjoint errors: dsched {err_s:.2e}, dg {err_g:.2e}")
    assert err_s < 1e-3 and err_g < 1e-3


def test_fp32_real_time_norm_drift(gp):
    # the rounded tables keep the substeps unitary: norm drift over 1000 steps
    # comes only from rounding noise
    n, dx, omega, dt, g = (64, 64, 64), (0.15, 0.15, 0.15), (1.0, 1.0, 1.5), 1e-3, 100.0
    psi0 = inputs.noisy_gaussian(n, dx, omega, 31)
    plan = gp.Plan(n, dx, dt, gp.GP_REAL, omega, g, gp.GP_C64)
    psi = to_dev(psi0.astype(np.complex64))
    o0 = plan.observables(psi)
    plan.step(psi, 1000)
    o1 = plan.observables(psi)
    say(f"fp32 norm drift {o1['norm'] - o0['norm']:.3e}")
    assert abs(o1["norm"] - o0["norm"]) < 2e-6


def test_fp64_long_real_run_matches_oracle(gp):
    n, dx, omega, dt, g = (96, 80, 64), (0.12, 0.12, 0.12), (1.0, 1.2, 1.5), 1e-3, 100.0
    psi0 = inputs.noisy_gaussian(n, dx, omega, 32)
    plan = gp.Plan(n, dx, dt, gp.GP_REAL, omega, g)
    psi = to_dev(psi0)
    say("fp64 300 real steps 96x80x64")
    plan.step(psi, 300)
    ref = oracle.step(psi0, dx, dt, oracle.REAL, omega, g, 300)
    got = psi.cpu().numpy()
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    say(f"  max rel err {err:.2e}")
    assert err <= 1e-12
    o = plan.observables(psi)
    r = oracle.observables(ref, dx, omega, g)
    for k in ("norm", "mu", "energy"):
        assert abs(o[k] - r[k]) <= 1e-12 * abs(r[k])


def test_autograd_fp32_gradient_error(gp):
    from paper_1709_04423_amd import adjoint
    n, dx, dt, g, T = (96, 80), (0.15, 0.15), 1e-3, 200.0, 200
    sched = inputs.gamma_schedule(T)
    psi0 = inputs.gaussian(n, dx, (1.0, 1.0))
    tgt = inputs.gaussian(n, dx, (1.5, 1.0))
    psi = to_dev(psi0.astype(np.complex64))
    s = torch.tensor(sched, dtype=torch.float64, device="cuda", requires_grad=True)
    loss = adjoint.overlap_loss(adjoint.evolve(psi, s, g, n, dx, dt, (1.0, 1.0)), to_dev(tgt.astype(np.complex64)), dx)
    loss.backward()
    _, dsr, _, _ = oracle.gradient(psi0, tgt, dx, dt, (1.0, 1.0), g, sched)
    err = np.max(np.abs(s.grad.cpu().numpy() - dsr)) / np.max(np.abs(dsr))
    say(f"fp32 schedule-gradient error {err:.2e}")
    assert err < 1e-3


@pytest.mark.parametrize("n", [(48, 40, 36), (64, 50), (128, 30, 12)])
def test_step_record_stores_each_step_input(gp, n):
    # the x sweep writes the recorded state as it loads (1D/2D/unfused 3D); the
    # fused 3D sweep is preceded by a copy
    dx = (0.2, 0.2, 0.25)[:len(n)]
    dt, omega, g, m = 1e-3, (1.0, 1.5, 2.0)[:len(n)], 60.0, 5
    psi0 = to_dev(inputs.noisy_gaussian(n, dx, omega, 44))
    plan = gp.Plan(n, dx, dt, gp.GP_REAL, omega, g)
    psi = psi0.clone()
    states = torch.empty((m,) + tuple(n[::-1]), dtype=psi.dtype, device="cuda")
    plan.step_record(psi, m, states)
    ref = gp.Plan(n, dx, dt, gp.GP_REAL, omega, g)
    chk = psi0.clone()
    for k in range(m):
        assert torch.equal(states[k], chk), k
        ref.step(chk, 1)
    assert torch.equal(psi, chk)
    assert plan.info()["step"] == m
    imag = gp.Plan(n, dx, dt, gp.GP_IMAG, omega, g)
    with pytest.raises(gp.GpError) as e:
        imag.step_record(psi0.clone(), 2, states)
    assert e.value.status == gp.GP_EUNSUPPORTED

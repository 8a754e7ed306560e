"""Full-length runs of the named workloads on the GPU (through the C ABI)
against values the FP64 oracle stored in tests/golden/ (written by
tests/golden/make_golden.py, which calls only oracle/).

  - 256^3, dx 0.05, trap (1, 2, 3), g 1000, dt 2e-4: 2000 imaginary-time steps
    from the seeded noisy Gaussian, then 2000 real-time steps -- complex128 within
    1e-12 and complex64 bulk within 1e-5 of the oracle in norm, mu and energy;
  - 128^3 quench: the oracle's ground state of the trap (1, 1, 4), then w_x -> 0.5
    and 1000 real-time steps, complex128 within 1e-12;
  - 256^2 adjoint: gradient over 2000 real-time steps between the oracle's
    ground states at gamma = 1 and 1.5, within 1e-9 of the oracle's gradient
    and 1e-6 of central differences.
Inputs that are oracle results (the ground states) are recomputed here with the
same oracle calls and checked bit for bit against the stored hashes.
"""
import importlib.util
import json
import os
import sys

import numpy as np
import pytest

from paper_1709_04423_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
FP64_TOL, FP32_TOL = 1e-12, 1e-5
# complex64 after each 2000-step phase: the level the bulk arithmetic reaches
# (about 3e-7), well inside the 1e-5 target -- a reordering of the solver's sums
# that biases the rounding shows up here first
FP32_PHASE_END_TOL = 1e-6


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def load_golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated (python tests/golden/make_golden.py)")
    return json.load(open(path))


def make_golden():
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(GOLDEN, "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_04423_amd import binding
    binding.lib()
    return binding


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def check(got, ref, fields, tol, what):
    errs = {k: abs(got[k] - ref[k]) / abs(ref[k]) for k in fields if ref[k] != 0.0}
    say(f"  {what}: " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()))
    for k, e in errs.items():
        assert e <= tol, (what, k, got[k], ref[k])


@pytest.mark.parametrize("prec", [0, 1], ids=["c128", "c64"])
def test_headline_2000_imag_then_2000_real_against_oracle(gp, prec):
    ref = load_golden("headline_256cubed.json")
    w = inputs.HEADLINE_3D
    psi0 = inputs.headline_initial()
    assert make_golden().sha(psi0) == ref["psi0_sha256"]
    dtype = np.complex128 if prec == 0 else np.complex64
    tol = FP64_TOL if prec == 0 else FP32_TOL
    fields = ("norm", "mu", "energy", "ekin", "epot", "eint", "rms_x", "rms_y", "rms_z") if prec == 0 \
        else ("norm", "mu", "energy", "rms_x", "rms_y", "rms_z")
    psi = to_dev(psi0.astype(dtype))
    for mode, key in ((gp.GP_IMAG, "imag"), (gp.GP_REAL, "real")):
        plan = gp.Plan(w.n, w.dx, w.dt, mode, w.omega, w.g, prec)
        done = 0
        for mark in sorted(int(m) for m in ref[key]):
            plan.step(psi, mark - done)
            done = mark
            if mark >= 20:
                check(plan.observables(psi), ref[key][str(mark)], fields, tol, f"{key} {mark}")
        if prec == 1:
            check(plan.observables(psi), ref[key][str(done)], ("norm", "mu", "energy"), FP32_PHASE_END_TOL,
                  f"{key} {done} (phase end)")
    del psi
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def quench_ground_state():
    mg = make_golden()
    ref = load_golden("quench_128cubed.json")
    say("oracle ground state of the 128^3 trap (1, 1, 4)")
    psi, steps, mu, _ = mg.quench_ground_state()
    assert steps == ref["ground_state"]["steps"] and mg.sha(psi) == ref["ground_state"]["sha256"]
    return psi, ref


def test_quench_1000_real_steps_from_oracle_ground_state(gp, quench_ground_state):
    psi0, ref = quench_ground_state
    w = inputs.QUENCH_3D
    plan = gp.Plan(w.n, w.dx, w.dt, gp.GP_REAL, w.omega, w.g)
    psi = to_dev(psi0)
    fields = ("norm", "mu", "energy", "ekin", "epot", "eint", "rms_x", "rms_y", "rms_z")
    check(plan.observables(psi), ref["after_quench_t0"], fields, FP64_TOL, "t = 0")
    done = 0
    for mark in sorted(int(m) for m in ref["real"]):
        plan.step(psi, mark - done)
        done = mark
        check(plan.observables(psi), ref["real"][str(mark)], fields, FP64_TOL, f"real {mark}")
    # conservation over the run: norm to rounding, energy within the splitting error
    assert abs(ref["real"]["1000"]["norm"] - ref["after_quench_t0"]["norm"]) < 1e-12


def test_quench_ground_state_on_gpu_matches_oracle(gp, quench_ground_state):
    # the same imaginary-time recipe (dt 1e-2 from the Gaussian, 100-step blocks,
    # stop when mu changes by < 1e-12) on the GPU reaches the oracle's state
    psi_ref, ref = quench_ground_state
    w = inputs.QUENCH_3D
    before = w.extra["omega_before"]
    plan = gp.Plan(w.n, w.dx, 1e-2, gp.GP_IMAG, before, w.g)
    psi = to_dev(inputs.gaussian(w.n, w.dx, before))
    for _ in range(ref["ground_state"]["steps"] // 100):
        plan.step(psi, 100)
    check(plan.observables(psi), ref["ground_state"]["obs"], ("norm", "mu", "energy", "rms_x", "rms_z"), FP64_TOL,
          "ground state")
    err = float(np.max(np.abs(psi.cpu().numpy() - psi_ref)) / np.max(np.abs(psi_ref)))
    say(f"  ground state max rel err {err:.2e}")
    assert err <= FP64_TOL


@pytest.fixture(scope="module")
def adjoint_inputs():
    mg = make_golden()
    ref = load_golden("adjoint_256sq.json")
    say("oracle ground states at gamma = 1 and 1.5 (256^2)")
    gs = mg.adjoint_ground_states()
    for key in ("start", "target"):
        assert mg.sha(gs[key][0]) == ref["ground_states"][key]["sha256"], key
    return gs["start"][0], gs["target"][0], ref


@pytest.mark.parametrize("prec", [0, 1], ids=["c128", "c64"])
def test_adjoint_gradient_between_ground_states(gp, adjoint_inputs, prec):
    from paper_1709_04423_amd import adjoint
    psi0, tgt, ref = adjoint_inputs
    w = inputs.ADJOINT_2D
    sched = inputs.gamma_schedule(w.steps)
    dt_ = torch.complex128 if prec == 0 else torch.complex64
    psi = to_dev(psi0).to(dt_).requires_grad_(True)
    s = torch.tensor(sched, dtype=torch.float64, device="cuda", requires_grad=True)
    g = torch.tensor(w.g, dtype=torch.float64, device="cuda", requires_grad=True)
    tg = to_dev(tgt).to(dt_)
    loss = adjoint.overlap_loss(adjoint.evolve(psi, s, g, w.n, w.dx, w.dt, (1.0, 1.0)), tg, w.dx)
    loss.backward()
    gr = ref["gradient"]
    ds = s.grad.cpu().numpy()
    dsr = np.array(gr["dsched"])
    e_loss = abs(loss.item() - gr["loss"]) / abs(gr["loss"])
    e_ds = float(np.max(np.abs(ds - dsr)) / np.max(np.abs(dsr)))
    e_dg = abs(g.grad.item() - gr["dg"]) / abs(gr["dg"])
    say(f"  {'c128' if prec == 0 else 'c64'}: loss {e_loss:.1e}, dsched {e_ds:.1e}, dg {e_dg:.1e}")
    if prec == 0:
        assert e_loss <= 1e-12 and e_ds <= 1e-9 and e_dg <= 1e-9
    else:
        # the loss 1 - |c|^2 (~0.07 here) is a difference next to 1: FP32 rounding of
        # |c|^2 is bounded absolutely, so its relative error is ~14x larger
        assert abs(loss.item() - gr["loss"]) <= 1e-5 and e_ds <= 1e-3 and e_dg <= 1e-3
        return

    # central differences with Richardson extrapolation through the GPU forward path
    def loss_at(sc, gg):
        with torch.no_grad():
            out = adjoint.evolve(to_dev(psi0), torch.tensor(sc, device="cuda"), gg, w.n, w.dx, w.dt, (1.0, 1.0))
            return float(adjoint.overlap_loss(out, tg, w.dx).item())

    def richardson(f, h):
        d1 = (f(h) - f(-h)) / (2 * h)
        d2 = (f(h / 2) - f(-h / 2)) / h
        return (4 * d2 - d1) / 3

    v = np.random.default_rng(41).standard_normal(len(sched))
    v /= np.linalg.norm(v)
    fd_s = richardson(lambda h: loss_at(sched + h * v, w.g), 1e-3)
    fd_g = richardson(lambda h: loss_at(sched, w.g + h), 1e-2)
    rel_s = abs(fd_s - ds @ v) / abs(fd_s)
    rel_g = abs(fd_g - g.grad.item()) / abs(fd_g)
    say(f"  FD check: schedule {rel_s:.2e}, g {rel_g:.2e}")
    assert rel_s <= 1e-6 and rel_g <= 1e-6

"""The SSCN workloads at their full sizes on the GPU, against the FP64 oracle
(element by element where the oracle finishes in seconds, else on the
observables and on conservation properties that hold at any size)."""
import sys

import numpy as np
import pytest
from scipy.linalg import eigh_tridiagonal

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


def max_rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("g", [0.0, 62.74])
def test_1d_imaginary_time_full_run(gp, g):
    # N = 512 on [-12.8, 12.8), V = x^2/2, dt = 5e-4, 10,000 steps from pi^-1/4 exp(-x^2/2)
    w = inputs.ONE_D
    psi0 = inputs.gaussian(w.n, w.dx, w.omega)
    plan = gp.Plan(w.n, w.dx, w.dt, gp.GP_IMAG, w.omega, g)
    psi = to_dev(psi0)
    say(f"1d g={g} 10^4 steps")
    plan.step(psi, w.steps)
    o = plan.observables(psi)
    ref = oracle.step(psi0, w.dx, w.dt, oracle.IMAG, w.omega, g, w.steps)
    r = oracle.observables(ref, w.dx, w.omega, g)
    assert max_rel(psi.cpu().numpy(), ref) <= 1e-12
    for k in ("norm", "mu", "energy", "rms_x"):
        assert abs(o[k] - r[k]) <= 1e-12 * abs(r[k]), k
    if g == 0.0:
        x = (np.arange(512) - 256) * w.dx
        lam = eigh_tridiagonal(1 / w.dx**2 + 0.5 * x * x, np.full(511, -0.5 / w.dx**2), eigvals_only=True,
                               select="i", select_range=(0, 0))[0]
        assert abs(o["mu"] - lam) < 1e-6
    say(f"  mu {o['mu']:.14f} (oracle {r['mu']:.14f}) E {o['energy']:.14f} rms {o['rms_x']:.14f}")


def test_3d_128_real_time_full_size_parity(gp):
    # the 128^3 quench grid (dx = 0.1, trap (0.5, 1, 4), g = 100, dt = 1e-3), 100 steps
    w = inputs.QUENCH_3D
    psi0 = inputs.noisy_gaussian(w.n, w.dx, w.extra["omega_before"], inputs.seed_for(1), 1e-3)
    plan = gp.Plan(w.n, w.dx, w.dt, gp.GP_REAL, w.omega, w.g)
    psi = to_dev(psi0)
    say("128^3 100 real steps")
    plan.step(psi, 100)
    ref = oracle.step(psi0, w.dx, w.dt, oracle.REAL, w.omega, w.g, 100)
    assert max_rel(psi.cpu().numpy(), ref) <= 1e-12
    o = plan.observables(psi)
    r = oracle.observables(ref, w.dx, w.omega, w.g)
    for k in ("norm", "mu", "energy"):
        assert abs(o[k] - r[k]) <= 1e-12 * abs(r[k]), k


def test_3d_128_quench_workflow_conserves_norm_and_energy(gp):
    # ground state of the unquenched trap by imaginary time, then w_x 1 -> 0.5
    # and 1000 real-time steps: norm conserved to rounding, energy bounded (Lie splitting, O(dt))
    w = inputs.QUENCH_3D
    before = w.extra["omega_before"]
    psi = to_dev(inputs.gaussian(w.n, w.dx, before))
    prep = gp.Plan(w.n, w.dx, w.dt, gp.GP_IMAG, before, w.g)
    say("128^3 ground state")
    prep.step(psi, 1500)
    real = gp.Plan(w.n, w.dx, w.dt, gp.GP_REAL, w.omega, w.g)
    o0 = real.observables(psi)
    rms0 = o0["rms_x"]
    energies = []
    for _ in range(10):
        real.step(psi, 100)
        o = real.observables(psi)
        energies.append(o["energy"])
        assert abs(o["norm"] - o0["norm"]) < 5e-12  # the oracle drifts 8e-13 over these 1000 steps
    say(f"  E0 {o0['energy']:.10f} E range {min(energies):.10f}..{max(energies):.10f} rms_x {rms0:.4f} -> {o['rms_x']:.4f}")
    # the oracle's energy stays within 4e-5 of E(0) on this run (Lie splitting error, bounded)
    assert max(abs(e - o0["energy"]) for e in energies) < 1e-4 * abs(o0["energy"])
    assert o["rms_x"] > rms0  # the cloud expands along the weakened axis


def test_headline_grid_20_steps_both_precisions(gp):
    # 256^3, dx = 0.05, trap (1, 2, 3), g = 1000, dt = 2e-4: 20 imaginary then 20 real steps
    w = inputs.HEADLINE_3D
    psi0 = inputs.headline_initial()
    say("oracle 256^3 20 imag + 20 real")
    ref_i = oracle.step(psi0, w.dx, w.dt, oracle.IMAG, w.omega, w.g, 20)
    ref_r = oracle.step(ref_i, w.dx, w.dt, oracle.REAL, w.omega, w.g, 20)
    r = oracle.observables(ref_r, w.dx, w.omega, w.g)
    for prec, tol, dtype in ((gp.GP_C128, 1e-12, np.complex128), (gp.GP_C64, 1e-5, np.complex64)):
        psi = to_dev(psi0.astype(dtype))
        gp.Plan(w.n, w.dx, w.dt, gp.GP_IMAG, w.omega, w.g, prec).step(psi, 20)
        if prec == gp.GP_C128:
            assert max_rel(psi.cpu().numpy(), ref_i) <= tol
        plan = gp.Plan(w.n, w.dx, w.dt, gp.GP_REAL, w.omega, w.g, prec)
        plan.step(psi, 20)
        o = plan.observables(psi)
        errs = {k: abs(o[k] - r[k]) / abs(r[k]) for k in ("norm", "mu", "energy")}
        say(f"  prec {prec}: psi err {max_rel(psi.cpu().numpy().astype(np.complex128), ref_r):.2e} obs errs {errs}")
        assert max_rel(psi.cpu().numpy().astype(np.complex128), ref_r) <= tol
        for k, e in errs.items():
            assert e <= tol, k
        del psi
        torch.cuda.empty_cache()


def test_batch_64_problems_1000_steps_fp32_against_oracle(gp, tmp_path):
    # 64 uneven 2D problems (sides from {128..512}, g ~ U[10, 500], nu ~ U[0.5, 2]),
    # complex64 bulk, autotuned launch, 1000 real-time steps; sampled problems
    # checked against the FP64 oracle per observable, every problem for norm
    probs = inputs.batch_problems()
    sizes = [p.n for p in probs]
    b = gp.Batch(sizes, 0.05, 1e-3, gp.GP_REAL, [p.omega for p in probs], [p.g for p in probs], gp.GP_C64)
    say("batch 64 autotune")
    cfg = b.autotune(str(tmp_path / "tune.txt"))
    say(f"  config {cfg}")
    init = [inputs.gaussian(p.n, p.dx, p.omega) for p in probs]
    psis = [to_dev(a.astype(np.complex64)) for a in init]
    # the walls cut the Gaussians' tails, so each problem keeps its own starting norm
    n0 = [b.observables(k, psis[k])["norm"] for k in range(len(probs))]
    say("batch 64 x 1000 steps")
    b.step(psis, 1000)
    torch.cuda.synchronize()
    drift = [abs(b.observables(k, psis[k])["norm"] - n0[k]) / n0[k] for k in range(len(probs))]
    say(f"  largest FP32 norm drift {max(drift):.2e} (problem {int(np.argmax(drift))})")
    assert max(drift) < 1e-5
    by_size = sorted(range(len(probs)), key=lambda k: probs[k].points)
    for k in (by_size[0], by_size[len(by_size) // 2], by_size[-1]):
        p = probs[k]
        o = b.observables(k, psis[k])
        ref = oracle.step(init[k], p.dx, p.dt, oracle.REAL, p.omega, p.g, 1000)
        r = oracle.observables(ref, p.dx, p.omega, p.g)
        errs = {f: abs(o[f] - r[f]) / abs(r[f]) for f in ("norm", "mu", "energy")}
        say(f"  problem {k} {p.n} g={p.g:.1f}: {errs}")
        for f, e in errs.items():
            assert e <= 1e-5, (k, f)

"""The stationary -> dynamic workflow on the GPU: a ground state from physical
inputs by imaginary time, stored and read back into a real-time run (the
hand-over with the same mesh and nonlinearity), a trap quench, and the rms
series of the dynamics -- against the oracle running the same recipe."""
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
def wf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_04423_amd import binding, workflow
    binding.lib()
    return workflow


def test_ground_state_store_quench_and_rms_series(wf, tmp_path):
    p = wf.Problem.from_physics((96, 80), (0.15, 0.15), (1.0, 1.4), natoms=5000, a_bohr=50.0, l_micron=1.0,
                                confine=10.0)
    say(f"g_2D = {p.g:.6f}")
    psi0 = inputs.gaussian(p.n, p.dx, p.omega)
    psi, steps, obs = wf.ground_state(p, 2e-3, psi=torch.from_numpy(psi0).to("cuda"), tol=1e-12)
    ref = oracle.step(psi0, p.dx, 2e-3, oracle.IMAG, p.omega, p.g, steps)
    r = oracle.observables(ref, p.dx, p.omega, p.g)
    say(f"ground state after {steps} steps: mu {obs['mu']:.14f} (oracle {r['mu']:.14f})")
    assert abs(obs["mu"] - r["mu"]) <= 1e-12 * r["mu"]
    path = str(tmp_path / "gs")
    wf.save_state(path, psi, p)
    q = wf.perturb(p, "trap", 0.8, axis=0)
    psi_rt = wf.load_state(path, q)
    rec = wf.dynamics(q, psi_rt, 1e-3, 2000, 100)
    assert rec.shape == (21, 10)
    rms_x = rec[:, 7]
    say(f"rms_x range {rms_x.min():.6f} .. {rms_x.max():.6f}")
    assert rms_x.max() - rms_x.min() > 0.01 * rms_x[0]      # the quench starts a breathing oscillation
    assert np.max(np.abs(rec[:, 1] - rec[0, 1])) < 1e-13     # norm conserved along the run
    fin = oracle.observables(oracle.step(ref, p.dx, 1e-3, oracle.REAL, q.omega, q.g, 2000), p.dx, q.omega, q.g)
    assert abs(rec[-1, 3] - fin["energy"]) <= 1e-12 * abs(fin["energy"])
    assert abs(rec[-1, 7] - fin["rms_x"]) <= 1e-12 * fin["rms_x"]
    with pytest.raises(ValueError):
        wf.load_state(path, wf.perturb(p, "nonlinearity", 0.5))

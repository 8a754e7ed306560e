"""Physical-input front end (host only): the dimensionless nonlinearity from
the number of atoms, scattering length and oscillator length, with the 2D and
1D reductions pinned by integrating the tight direction's ground state
numerically, and the stored-state hand-over checks of the workflow."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from paper_1709_04423_amd import binding, workflow


def test_three_dimensional_nonlinearity_and_oscillator_length():
    # g = 4 pi N a / l in units of l; 87Rb (86.909 u) at 100 Hz has l = 1.0785 um
    g = binding.nonlinearity(3, 2000, 100.0, 1.0)
    assert abs(g - 4 * math.pi * 2000 * 100 * 5.29177210903e-11 / 1e-6) < 1e-12 * g
    assert abs(binding.osc_length(86.909, 100.0) - 1.0785) < 5e-4


@pytest.mark.parametrize("lam", [4.0, 10.0, 50.0])
def test_two_and_one_dimensional_reductions_integrate_the_tight_ground_state(lam):
    g3 = binding.nonlinearity(3, 1500, 80.0, 1.3)
    # 2D: the z ground state (lam/pi)^(1/4) exp(-lam z^2 / 2), integral of its fourth power
    z4, _ = quad(lambda z: (lam / math.pi) * math.exp(-2 * lam * z * z), -np.inf, np.inf)
    assert abs(binding.nonlinearity(2, 1500, 80.0, 1.3, lam) - g3 * z4) < 1e-12 * g3 * z4
    # 1D: the transverse 2D ground state (nu/pi)^(1/2) exp(-nu r^2 / 2)
    r4, _ = quad(lambda r: (lam / math.pi) ** 2 * math.exp(-2 * lam * r * r) * 2 * math.pi * r, 0, np.inf)
    assert abs(binding.nonlinearity(1, 1500, 80.0, 1.3, lam) - g3 * r4) < 1e-12 * g3 * r4


def test_bad_physical_inputs():
    for args in ((4, 1, 1, 1, 1), (3, -1, 1, 1, 1), (3, 1, 1, 0.0, 1), (2, 1, 1, 1, 0.0), (1, 1, 1, 1, -1.0),
                 (3, float("nan"), 1, 1, 1)):
        with pytest.raises(binding.GpError) as e:
            binding.nonlinearity(*args)
        assert e.value.status == binding.GP_EINVAL
    with pytest.raises(binding.GpError):
        binding.osc_length(0.0, 100.0)


def test_stored_state_needs_the_same_mesh_and_nonlinearity(tmp_path):
    torch = pytest.importorskip("torch")
    p = workflow.Problem((16, 12), (0.2, 0.25), (1.0, 1.5), 30.0)
    psi = torch.arange(12 * 16, dtype=torch.float64).reshape(12, 16).to(torch.complex128)
    path = str(tmp_path / "state")
    workflow.save_state(path, psi, p)
    back = workflow.load_state(path, workflow.perturb(p, "trap", 0.5, axis=0), device="cpu")
    assert torch.equal(back, psi)  # a different trap is a perturbation: allowed
    for bad in (workflow.Problem((16, 12), (0.2, 0.2), (1.0, 1.5), 30.0),
                workflow.perturb(p, "nonlinearity", 2.0),
                workflow.Problem((16, 13), (0.2, 0.25), (1.0, 1.5), 30.0)):
        with pytest.raises(ValueError):
            workflow.load_state(path, bad, device="cpu")
    with pytest.raises(ValueError):
        workflow.perturb(p, "kick", 1.0)

"""gp_observables_noalloc (the entry point for callers that cannot allocate)
against gp_observables of a plan of the same grid, through the C ABI: the same
kernels and order, so bitwise equal; two calls in a row, the second on a smaller
grid, so partials left in the shared static array from the first cannot leak
into the second."""
import ctypes
import sys

import numpy as np
import pytest

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
    L = binding.lib()
    L.gp_observables_noalloc.argtypes = [ctypes.c_int, binding.c_i64p, binding.c_dp, binding.c_dp, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(binding.GpObs),
                                         ctypes.c_void_p]
    L.gp_observables_noalloc.restype = ctypes.c_int
    return binding


def noalloc(gp, psi, n, dx, omega, g, prec):
    L = gp.lib()
    nd = len(n)
    o = gp.GpObs()
    st = L.gp_observables_noalloc(nd, (ctypes.c_int64 * nd)(*n), (ctypes.c_double * nd)(*dx),
                                  (ctypes.c_double * nd)(*omega), g, prec, ctypes.c_void_p(psi.data_ptr()),
                                  ctypes.byref(o), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    gp.check(st, "gp_observables_noalloc")
    return o.as_dict()


CASES = [  # (n x first, dx, omega, g, prec): a large grid first, then smaller ones
    ((256, 256, 256), (0.05, 0.05, 0.05), (1.0, 2.0, 3.0), 1000.0, 0),
    ((37, 29, 23), (0.2, 0.25, 0.3), (1.0, 2.0, 3.0), 50.0, 0),
    ((96, 80, 64), (0.12, 0.12, 0.12), (1.0, 1.2, 1.5), 100.0, 1),
    ((70, 45), (0.1, 0.12), (1.0, 1.5), 30.0, 0),
    ((512,), (0.05,), (1.0,), 62.74, 0),
]


def test_noalloc_matches_plan_observables_two_calls_in_a_row(gp):
    for n, dx, omega, g, prec in CASES:
        dtype = np.complex128 if prec == 0 else np.complex64
        psi0 = inputs.gaussian(n, dx, omega) + 0.05 * inputs.random_field(tuple(n[::-1]), 9)
        psi = torch.from_numpy(psi0.astype(dtype)).to("cuda")
        plan = gp.Plan(n, dx, 1e-3, gp.GP_IMAG, omega, g, prec)
        ref = plan.observables(psi)
        for call in range(2):  # the second call reuses the array the first left filled
            got = noalloc(gp, psi, n, dx, omega, g, prec)
            say(f"n={n} prec={prec} call {call}: mu {got['mu']:.15f}")
            assert got == ref, (n, call)
        del psi, plan
        torch.cuda.empty_cache()


def test_noalloc_rejects_bad_and_oversized_grids(gp):
    L = gp.lib()
    psi = torch.zeros(8, dtype=torch.complex128, device="cuda")
    o = gp.GpObs()
    one = (ctypes.c_int64 * 1)(8)
    dx = (ctypes.c_double * 1)(0.1)
    assert L.gp_observables_noalloc(0, one, dx, None, 0.0, 0, ctypes.c_void_p(psi.data_ptr()), ctypes.byref(o),
                                    None) == gp.GP_EINVAL
    assert L.gp_observables_noalloc(1, one, dx, None, 0.0, 0, None, ctypes.byref(o), None) == gp.GP_EINVAL
    big = (ctypes.c_int64 * 1)(8192 * 64 + 1)  # one group more than the static array holds
    assert L.gp_observables_noalloc(1, big, dx, None, 0.0, 0, ctypes.c_void_p(psi.data_ptr()), ctypes.byref(o),
                                    None) == gp.GP_EUNSUPPORTED

"""Host-side checks of the C ABI: the library loads, exports every symbol that
include/gp.h declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

from paper_1709_04423_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "gp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gp_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = binding.lib()
    names = declared_functions()
    assert len(names) >= 19
    for name in names:
        assert hasattr(L, name), name


def test_header_is_plain_c():
    # the boundary takes plain pointers and sizes: no torch or HIP types in it
    text = open(os.path.join(ROOT, "include", "gp.h")).read()
    code = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    for word in ("torch", "at::", "hipStream_t", "#include <hip", "std::"):
        assert word not in code


def test_status_strings():
    L = binding.lib()
    assert L.gp_strerror(binding.GP_EINVAL) == b"invalid argument"
    assert L.gp_strerror(binding.GP_OK) == b"ok"
    assert binding.kernel_names()[0] == "sweep_x"


def _create(ndim, n, dx, dt, mode=0, prec=0, g=0.0, trap=None):
    L = binding.lib()
    h = ctypes.c_void_p()
    n_arr = (ctypes.c_int64 * max(ndim, 1))(*n) if n is not None else None
    dx_arr = (ctypes.c_double * max(ndim, 1))(*dx) if dx is not None else None
    st = L.gp_plan_create(ctypes.byref(h), ndim, n_arr, dx_arr, dt, mode,
                          ctypes.byref(trap) if trap is not None else None, g, prec)
    return st, h


@pytest.mark.parametrize("args", [
    (0, [4], [0.1], 0.01),            # ndim
    (4, [4, 4, 4, 4], [0.1] * 4, 0.01),
    (1, [0], [0.1], 0.01),            # empty axis
    (1, [-3], [0.1], 0.01),
    (1, [8], [0.0], 0.01),            # dx
    (1, [8], [-0.1], 0.01),
    (1, [8], [float("nan")], 0.01),
    (1, [8], [0.1], 0.0),             # dt
    (1, [8], [0.1], -1e-3),
    (1, [8], [0.1], float("inf")),
    (2, [1 << 32, 8], [0.1, 0.1], 0.01),  # too large
])
def test_plan_create_rejects_bad_geometry(args):
    st, h = _create(*args)
    assert st == binding.GP_EINVAL
    assert not h.value


def test_plan_create_rejects_bad_enums_and_trap():
    assert _create(1, [8], [0.1], 0.01, mode=2)[0] == binding.GP_EINVAL
    assert _create(1, [8], [0.1], 0.01, prec=7)[0] == binding.GP_EINVAL
    assert _create(1, [8], [0.1], 0.01, g=float("nan"))[0] == binding.GP_EINVAL
    t = binding.GpTrap()
    t.sched_len = 3  # schedule length without an array
    assert _create(1, [8], [0.1], 0.01, trap=t)[0] == binding.GP_EINVAL
    arr = (ctypes.c_double * 3)(1.0, 1.1, 1.2)
    t.omega_sched = ctypes.cast(arr, binding.c_dp)
    t.sched_axis = 1  # axis beyond ndim = 1
    assert _create(1, [8], [0.1], 0.01, trap=t)[0] == binding.GP_EINVAL
    t.sched_axis = 0
    t.omega[1] = float("inf")
    assert _create(1, [8], [0.1], 0.01, trap=t)[0] == binding.GP_EINVAL
    assert binding.lib().gp_plan_create(None, 1, None, None, 0.1, 0, None, 0.0, 0) == binding.GP_EINVAL


def test_null_handles_are_rejected():
    L = binding.lib()
    obs = binding.GpObs()
    assert L.gp_step(None, None, 1, None) == binding.GP_EINVAL
    assert L.gp_observables(None, None, ctypes.byref(obs), None) == binding.GP_EINVAL
    assert L.gp_plan_set_step(None, 0) == binding.GP_EINVAL
    assert L.gp_plan_get_info(None, None) == binding.GP_EINVAL
    assert L.gp_step_adjoint(None, None, None, 0, 1, None, None, None) == binding.GP_EINVAL
    assert L.gp_step_record(None, None, 1, None, None) == binding.GP_EINVAL
    assert L.gp_plan_set_xy_fusion(None, 1) == binding.GP_EINVAL
    assert L.gp_batch_set_config(None, 0, 1, 1, 1) == binding.GP_EINVAL
    iv = ctypes.c_int()
    assert L.gp_batch_set_side_config(None, 128, 1, 1) == binding.GP_EINVAL
    assert L.gp_batch_get_side_config(None, 128, ctypes.byref(iv), ctypes.byref(iv)) == binding.GP_EINVAL
    assert L.gp_plan_timing_enable(None, 4) == binding.GP_EINVAL
    assert L.gp_copy_probe(None, None, 16, None) == binding.GP_EINVAL
    assert L.gp_plan_destroy(None) == binding.GP_OK
    assert L.gp_batch_destroy(None) == binding.GP_OK
    h = ctypes.c_void_p()
    assert L.gp_batch_create(ctypes.byref(h), 0, None, None, None, 1, None, None, 1) == binding.GP_EINVAL
    assert L.gp_batch_step(None, None, 1, None) == binding.GP_EINVAL
    # the no-allocation observables check their arguments before any HIP call
    one = (ctypes.c_int64 * 1)(8)
    dx = (ctypes.c_double * 1)(0.1)
    assert L.gp_observables_noalloc(0, one, dx, None, 0.0, 0, None, ctypes.byref(obs), None) == binding.GP_EINVAL
    assert L.gp_observables_noalloc(1, one, dx, None, 0.0, 0, None, ctypes.byref(obs), None) == binding.GP_EINVAL
    bad = (ctypes.c_double * 1)(-0.1)
    assert L.gp_observables_noalloc(1, one, bad, None, 0.0, 0, ctypes.c_void_p(16), ctypes.byref(obs),
                                    None) == binding.GP_EINVAL
    big = (ctypes.c_int64 * 1)(8192 * 64 + 1)
    assert L.gp_observables_noalloc(1, big, dx, None, 0.0, 0, ctypes.c_void_p(16), ctypes.byref(obs),
                                    None) == binding.GP_EUNSUPPORTED


def _batch_create(sizes, dx, dt, mode, prec, traps=None):
    L = binding.lib()
    k = len(sizes)
    n = (ctypes.c_int64 * (2 * k))(*[v for s in sizes for v in s])
    dxa = (ctypes.c_double * k)(*[dx] * k)
    dta = (ctypes.c_double * k)(*[dt] * k)
    if traps is None:
        traps = (binding.GpTrap * k)()
        for t in traps:
            t.omega[0] = t.omega[1] = 1.0
    ga = (ctypes.c_double * k)(*[10.0] * k)
    h = ctypes.c_void_p()
    return L.gp_batch_create(ctypes.byref(h), k, n, dxa, dta, mode, traps, ga, prec), h


def test_batch_create_rejects_problems_the_batched_kernels_do_not_run():
    # dx = 0.05, dt = 5e-3 in complex128 real time: the y recurrence contracts so
    # slowly that its window would exceed 8 blocks (or the exact solver would be
    # needed) on a y line too long for the scan solver (over 512 points); the
    # batch must refuse it up front instead of skipping the y sweep
    st, h = _batch_create([(64, 64), (128, 600)], 0.05, 5e-3, binding.GP_REAL, binding.GP_C128)
    assert st == binding.GP_EUNSUPPORTED and not h.value
    assert b"windowed" in binding.lib().gp_last_error()
    # a per-problem trap schedule is not supported by the batched launch
    traps = (binding.GpTrap * 1)()
    arr = (ctypes.c_double * 2)(1.0, 1.1)
    traps[0].omega_sched = ctypes.cast(arr, binding.c_dp)
    traps[0].sched_len = 2
    st, h = _batch_create([(64, 64)], 0.1, 1e-3, binding.GP_REAL, binding.GP_C64, traps)
    assert st == binding.GP_EUNSUPPORTED
    # bad spacing / time step
    assert _batch_create([(64, 64)], 0.0, 1e-3, binding.GP_REAL, binding.GP_C64)[0] == binding.GP_EINVAL
    assert _batch_create([(64, 64)], 0.1, float("nan"), binding.GP_REAL, binding.GP_C64)[0] == binding.GP_EINVAL
    assert binding.lib().gp_autotune(None, None) == binding.GP_EINVAL


def test_symmetric_trap_plan_arguments_checked_before_hip():
    L = binding.lib()
    h = ctypes.c_void_p()
    n = (ctypes.c_int64 * 2)(64, 32)
    dx = (ctypes.c_double * 2)(0.1, 0.1)
    # GP_CARTESIAN and out-of-range values are not symmetric geometries
    for geom in (0, 4, -1):
        assert L.gp_plan_create_sym(ctypes.byref(h), geom, n, dx, 1e-3, 0, None, 0.0, 0) == binding.GP_EINVAL
    assert L.gp_plan_create_sym(ctypes.byref(h), binding.GP_AXIAL, n, dx, -1.0, 0, None, 0.0, 0) == binding.GP_EINVAL
    # complex64 and radial lines beyond 1024 points are refused before any device work
    assert L.gp_plan_create_sym(ctypes.byref(h), binding.GP_CIRCULAR, n, dx, 1e-3, 0, None, 0.0,
                                1) == binding.GP_EUNSUPPORTED
    big = (ctypes.c_int64 * 1)(1025)
    assert L.gp_plan_create_sym(ctypes.byref(h), binding.GP_SPHERICAL, big, dx, 1e-3, 0, None, 0.0,
                                0) == binding.GP_EUNSUPPORTED
    assert not h.value


def test_binding_refuses_missing_library(monkeypatch, tmp_path):
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        binding.lib()

"""ctypes binding of libgp (``include/gp.h``): argument marshalling only.

Every step of the solver runs in the HIP kernels of ``libgp.so``; this module
passes torch tensors' device pointers and the current HIP stream across the C
ABI and turns status codes into exceptions.  It raises if the library is not
built -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgp.so")

GP_OK, GP_EINVAL, GP_ENOMEM, GP_EHIP, GP_ENONFINITE, GP_EUNSUPPORTED, GP_ETIMEOUT = 0, -1, -2, -3, -4, -5, -6
GP_IMAG, GP_REAL = 0, 1
GP_C128, GP_C64 = 0, 1
GP_CARTESIAN, GP_CIRCULAR, GP_SPHERICAL, GP_AXIAL = 0, 1, 2, 3
GP_NUM_KERNEL_KINDS = 15

c_i64p = ctypes.POINTER(ctypes.c_int64)
c_dp = ctypes.POINTER(ctypes.c_double)


class GpTrap(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double * 3), ("omega_sched", c_dp), ("sched_len", ctypes.c_int64),
                ("sched_axis", ctypes.c_int)]


class GpObs(ctypes.Structure):
    _fields_ = [("norm", ctypes.c_double), ("mu", ctypes.c_double), ("energy", ctypes.c_double),
                ("ekin", ctypes.c_double), ("epot", ctypes.c_double), ("eint", ctypes.c_double),
                ("rms", ctypes.c_double * 3)]

    def as_dict(self) -> dict:
        return {"norm": self.norm, "mu": self.mu, "energy": self.energy, "ekin": self.ekin,
                "epot": self.epot, "eint": self.eint, "rms_x": self.rms[0], "rms_y": self.rms[1],
                "rms_z": self.rms[2]}


class GpPlanInfo(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int64 * 3), ("window", ctypes.c_int * 3),
                ("rho", ctypes.c_double * 3), ("window_bound", ctypes.c_double * 3),
                ("step", ctypes.c_int64), ("device_bytes", ctypes.c_int64), ("xy_fused", ctypes.c_int)]


class GpError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str):
        super().__init__(f"{what}: status {status} ({detail})")
        self.status = status


_lib = None


def lib():
    """Load libgp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                              "python paper_1709_04423_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        pp = ctypes.POINTER(ctypes.c_void_p)
        sig = {
            "gp_plan_create": [pp, i32, c_i64p, c_dp, d, i32, ctypes.POINTER(GpTrap), d, i32],
            "gp_plan_create_sym": [pp, i32, c_i64p, c_dp, d, i32, ctypes.POINTER(GpTrap), d, i32],
            "gp_plan_destroy": [vp],
            "gp_step": [vp, vp, i64, vp],
            "gp_observables": [vp, vp, ctypes.POINTER(GpObs), vp],
            "gp_plan_set_step": [vp, i64],
            "gp_plan_get_info": [vp, ctypes.POINTER(GpPlanInfo)],
            "gp_plan_set_xy_fusion": [vp, i32],
            "gp_thomas_table": [i64, d, d, i32, i32, i32, c_dp, c_dp, ctypes.POINTER(ctypes.c_int), c_dp],
            "gp_step_adjoint": [vp, vp, vp, i64, i64, vp, vp, vp],
            "gp_step_record": [vp, vp, i64, vp, vp],
            "gp_batch_create": [pp, i32, c_i64p, c_dp, c_dp, i32, ctypes.POINTER(GpTrap), c_dp, i32],
            "gp_autotune": [vp, ctypes.c_char_p],
            "gp_batch_destroy": [vp],
            "gp_batch_step": [vp, pp, i64, vp],
            "gp_batch_autotune": [vp, ctypes.c_char_p, vp],
            "gp_batch_observables": [vp, i32, vp, ctypes.POINTER(GpObs), vp],
            "gp_batch_get_config": [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                    ctypes.POINTER(i32)],
            "gp_batch_set_config": [vp, i32, i32, i32, i32],
            "gp_batch_set_side_config": [vp, i64, i32, i32],
            "gp_batch_get_side_config": [vp, i64, ctypes.POINTER(i32), ctypes.POINTER(i32)],
            "gp_batch_set_wait_limit": [vp, ctypes.c_uint32],
            "gp_plan_timing_enable": [vp, i64],
            "gp_plan_timing_read": [vp, c_i64p, c_dp],
            "gp_copy_probe": [vp, vp, i64, vp],
            "gp_observables_noalloc": [i32, c_i64p, c_dp, c_dp, d, i32, vp, ctypes.POINTER(GpObs), vp],
            "gp_density": [vp, vp, vp, vp],
            "gp_nonlinearity": [i32, d, d, d, d, c_dp],
            "gp_osc_length": [d, d, c_dp],
            "gp_density_reduced": [vp, vp, i32, vp, vp],
            "gp_step_series": [vp, vp, i64, i64, vp, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.gp_strerror.argtypes = [ctypes.c_int]
        L.gp_strerror.restype = ctypes.c_char_p
        L.gp_last_error.argtypes = []
        L.gp_last_error.restype = ctypes.c_char_p
        L.gp_kernel_name.argtypes = [ctypes.c_int]
        L.gp_kernel_name.restype = ctypes.c_char_p
        _lib = L
    return _lib


def check(status: int, what: str) -> None:
    if status != GP_OK:
        L = lib()
        raise GpError(status, what, f"{L.gp_strerror(status).decode()}: {L.gp_last_error().decode()}")


def kernel_names():
    return [lib().gp_kernel_name(k).decode() for k in range(GP_NUM_KERNEL_KINDS)]


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _prec_of(dtype) -> int:
    import torch
    if dtype == torch.complex128:
        return GP_C128
    if dtype == torch.complex64:
        return GP_C64
    raise TypeError(f"psi must be complex128 or complex64, got {dtype}")


def _check_psi(psi, shape, prec):
    import torch
    if not isinstance(psi, torch.Tensor) or not psi.is_cuda:
        raise TypeError("psi must be a CUDA (HIP) tensor")
    if tuple(psi.shape) != tuple(shape):
        raise ValueError(f"psi has shape {tuple(psi.shape)}, plan expects {tuple(shape)}")
    if not psi.is_contiguous():
        raise ValueError("psi must be contiguous")
    if _prec_of(psi.dtype) != prec:
        raise TypeError("psi dtype does not match the plan precision")


def _check_f64(t, shape):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() \
            or tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected a contiguous float64 device tensor of shape {shape}")


class Plan:
    """Owns a gp_plan.  Grid sizes and spacings are given x first; tensors are
    (Nz, Ny, Nx)-shaped, x fastest.  geometry: GP_CARTESIAN (gp_plan_create) or a
    symmetric trap (gp_plan_create_sym): GP_CIRCULAR / GP_SPHERICAL with n = (N_r,),
    GP_AXIAL with n = (N_rho, N_z) and a (N_z, N_rho) tensor."""

    def __init__(self, n: Sequence[int], dx, dt: float, mode: int, omega=(0.0, 0.0, 0.0), g: float = 0.0,
                 prec: int = GP_C128, sched=None, sched_axis: int = 0, geometry: int = GP_CARTESIAN):
        L = lib()
        self.n = tuple(int(v) for v in n)
        self.ndim = len(self.n)
        dxs = [float(v) for v in (dx if hasattr(dx, "__len__") else [dx] * self.ndim)]
        if len(dxs) != self.ndim:
            raise ValueError("dx must have one entry per axis")
        self.dx = tuple(dxs)
        self.dt, self.mode, self.g, self.prec = float(dt), int(mode), float(g), int(prec)
        om = list(omega if hasattr(omega, "__len__") else [omega] * self.ndim)
        self.omega = tuple(float(v) for v in om) + (0.0,) * (3 - len(om))
        trap = GpTrap()
        for a in range(3):
            trap.omega[a] = self.omega[a]
        self._sched = None
        if sched is not None:
            import numpy as np
            self._sched = np.ascontiguousarray(sched, dtype=np.float64)
            trap.omega_sched = self._sched.ctypes.data_as(c_dp)
            trap.sched_len = len(self._sched)
            trap.sched_axis = int(sched_axis)
        n_arr = (ctypes.c_int64 * self.ndim)(*self.n)
        dx_arr = (ctypes.c_double * self.ndim)(*self.dx)
        h = ctypes.c_void_p()
        self.geometry = int(geometry)
        if self.geometry == GP_CARTESIAN:
            check(L.gp_plan_create(ctypes.byref(h), self.ndim, n_arr, dx_arr, self.dt, self.mode,
                                   ctypes.byref(trap), self.g, self.prec), "gp_plan_create")
        else:
            check(L.gp_plan_create_sym(ctypes.byref(h), self.geometry, n_arr, dx_arr, self.dt, self.mode,
                                       ctypes.byref(trap), self.g, self.prec), "gp_plan_create_sym")
        self._h = h

    @property
    def shape(self):
        return tuple(self.n[::-1])

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().gp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, psi, nsteps: int = 1, stream=None):
        _check_psi(psi, self.shape, self.prec)
        check(lib().gp_step(self._h, ctypes.c_void_p(psi.data_ptr()), int(nsteps), _stream_handle(stream)),
              "gp_step")
        return psi

    def observables(self, psi, stream=None) -> dict:
        _check_psi(psi, self.shape, self.prec)
        o = GpObs()
        check(lib().gp_observables(self._h, ctypes.c_void_p(psi.data_ptr()), ctypes.byref(o),
                                   _stream_handle(stream)), "gp_observables")
        return o.as_dict()

    def step_record(self, psi, nsteps: int, states, stream=None):
        """nsteps real-time steps of psi in place, states[k] = input of the k-th one."""
        _check_psi(psi, self.shape, self.prec)
        if not states.is_cuda or states.dtype != psi.dtype or not states.is_contiguous() or states.dim() != psi.dim() + 1 \
                or tuple(states.shape[1:]) != tuple(psi.shape) or states.shape[0] < nsteps:
            raise ValueError("states must be a contiguous (>= nsteps, *psi.shape) tensor of psi's dtype")
        check(lib().gp_step_record(self._h, ctypes.c_void_p(psi.data_ptr()), int(nsteps),
                                   ctypes.c_void_p(states.data_ptr()), _stream_handle(stream)), "gp_step_record")
        return psi

    def density(self, psi, out=None, stream=None):
        """|psi|^2 on the grid (float64 device tensor of psi's shape)."""
        import torch
        _check_psi(psi, self.shape, self.prec)
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=psi.device)
        _check_f64(out, tuple(self.shape))
        check(lib().gp_density(self._h, ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                               _stream_handle(stream)), "gp_density")
        return out

    def density_reduced(self, psi, keep, stream=None):
        """|psi|^2 integrated over the axes not in `keep` (axis numbers, x = 0): a float64
        tensor over the kept axes (slowest first, as the grid)."""
        import torch
        _check_psi(psi, self.shape, self.prec)
        mask = 0
        for a in keep:
            mask |= 1 << int(a)
        kept = tuple(self.n[a] for a in sorted(keep))[::-1]
        out = torch.empty(kept, dtype=torch.float64, device=psi.device)
        check(lib().gp_density_reduced(self._h, ctypes.c_void_p(psi.data_ptr()), mask,
                                       ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)), "gp_density_reduced")
        return out

    def step_series(self, psi, nsteps: int, every: int, stream=None):
        """Steps as step() with the observables every `every` steps: a float64 device tensor of
        shape (nsteps/every + 1, 10): step, norm, mu, energy, ekin, epot, eint, rms[3]."""
        import torch
        _check_psi(psi, self.shape, self.prec)
        if every < 1 or nsteps < 0 or nsteps % every:
            raise ValueError("nsteps must be a non-negative multiple of every >= 1")
        out = torch.empty((nsteps // every + 1, 10), dtype=torch.float64, device=psi.device)
        check(lib().gp_step_series(self._h, ctypes.c_void_p(psi.data_ptr()), int(nsteps), int(every),
                                   ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)), "gp_step_series")
        return out

    def set_step(self, step: int):
        check(lib().gp_plan_set_step(self._h, int(step)), "gp_plan_set_step")

    def info(self) -> dict:
        i = GpPlanInfo()
        check(lib().gp_plan_get_info(self._h, ctypes.byref(i)), "gp_plan_get_info")
        return {"ndim": i.ndim, "n": tuple(i.n), "window": tuple(i.window), "rho": tuple(i.rho),
                "window_bound": tuple(i.window_bound), "step": i.step, "device_bytes": i.device_bytes,
                "xy_fused": i.xy_fused}

    def set_xy_fusion(self, enable):
        """3D: skip (0/False) the fused x+y sweep, or use it where the shape allows:
        2 (the default) with the y window in registers, 1 (True) with it in LDS."""
        check(lib().gp_plan_set_xy_fusion(self._h, int(enable)), "gp_plan_set_xy_fusion")

    def adjoint(self, states, lam, n_first: int, nsteps: int, dsched=None, dg=None, stream=None):
        """Reverse nsteps real-time steps (see gp_step_adjoint)."""
        import torch
        if states.shape[0] < nsteps or tuple(states.shape[1:]) != self.shape or not states.is_contiguous():
            raise ValueError("states must be a contiguous (nsteps, *grid) tensor")
        _check_psi(lam, self.shape, self.prec)
        if _prec_of(states.dtype) != self.prec:
            raise TypeError("states dtype does not match the plan precision")
        for t in (dsched, dg):
            if t is not None and (t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous()):
                raise TypeError("dsched and dg must be contiguous float64 device tensors")
        if dsched is not None and dsched.numel() < nsteps:
            raise ValueError("dsched too short")
        check(lib().gp_step_adjoint(self._h, ctypes.c_void_p(states.data_ptr()), ctypes.c_void_p(lam.data_ptr()),
                                    int(n_first), int(nsteps),
                                    ctypes.c_void_p(dsched.data_ptr()) if dsched is not None else None,
                                    ctypes.c_void_p(dg.data_ptr()) if dg is not None else None,
                                    _stream_handle(stream)), "gp_step_adjoint")
        return lam

    def timing_enable(self, capacity: int):
        check(lib().gp_plan_timing_enable(self._h, int(capacity)), "gp_plan_timing_enable")

    def timing_read(self) -> dict:
        counts = (ctypes.c_int64 * GP_NUM_KERNEL_KINDS)()
        ms = (ctypes.c_double * GP_NUM_KERNEL_KINDS)()
        check(lib().gp_plan_timing_read(self._h, counts, ms), "gp_plan_timing_read")
        names = kernel_names()
        return {names[k]: (counts[k], ms[k]) for k in range(GP_NUM_KERNEL_KINDS) if counts[k]}


class Batch:
    """Owns a gp_batch of independent 2D problems (sizes x first)."""

    def __init__(self, sizes, dx, dt, mode, omega, g, prec=GP_C64):
        import numpy as np
        L = lib()
        self.count = len(sizes)
        self.sizes = [tuple(int(v) for v in s) for s in sizes]
        self.prec = int(prec)
        n = np.ascontiguousarray(np.array(self.sizes, dtype=np.int64).reshape(-1))
        dxa = np.ascontiguousarray(np.broadcast_to(np.asarray(dx, dtype=np.float64), (self.count,)))
        dta = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (self.count,)))
        om = np.asarray(omega, dtype=np.float64).reshape(self.count, 2)
        traps = (GpTrap * self.count)()
        for k in range(self.count):
            traps[k].omega[0], traps[k].omega[1] = float(om[k, 0]), float(om[k, 1])
        ga = np.ascontiguousarray(np.broadcast_to(np.asarray(g, dtype=np.float64), (self.count,)))
        h = ctypes.c_void_p()
        check(L.gp_batch_create(ctypes.byref(h), self.count, n.ctypes.data_as(c_i64p), dxa.ctypes.data_as(c_dp),
                                dta.ctypes.data_as(c_dp), int(mode), traps, ga.ctypes.data_as(c_dp),
                                self.prec), "gp_batch_create")
        self._h = h

    def shape(self, k):
        return self.sizes[k][::-1]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().gp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, psis, nsteps=1, stream=None):
        if len(psis) != self.count:
            raise ValueError("one grid per problem")
        for k, p in enumerate(psis):
            _check_psi(p, self.shape(k), self.prec)
        arr = (ctypes.c_void_p * self.count)(*[p.data_ptr() for p in psis])
        check(lib().gp_batch_step(self._h, arr, int(nsteps), _stream_handle(stream)), "gp_batch_step")
        return psis

    def autotune(self, cache_path=None, stream=None):
        check(lib().gp_batch_autotune(self._h, cache_path.encode() if cache_path else None, _stream_handle(stream)),
              "gp_batch_autotune")
        return self.config()

    def config(self):
        v = [ctypes.c_int() for _ in range(4)]
        check(lib().gp_batch_get_config(self._h, *[ctypes.byref(x) for x in v]), "gp_batch_get_config")
        return {"persistent": v[0].value, "lines": v[1].value, "ysegs": v[2].value, "grid": v[3].value}

    def set_config(self, persistent=0, lines=4, ysegs=4, grid=1024):
        check(lib().gp_batch_set_config(self._h, int(persistent), int(lines), int(ysegs), int(grid)),
              "gp_batch_set_config")

    def set_side_config(self, side, lines, ysegs):
        check(lib().gp_batch_set_side_config(self._h, int(side), int(lines), int(ysegs)), "gp_batch_set_side_config")

    def side_config(self, side):
        v = [ctypes.c_int() for _ in range(2)]
        check(lib().gp_batch_get_side_config(self._h, int(side), *[ctypes.byref(x) for x in v]),
              "gp_batch_get_side_config")
        return {"lines": v[0].value, "ysegs": v[1].value}

    def set_wait_limit(self, polls):
        check(lib().gp_batch_set_wait_limit(self._h, int(polls)), "gp_batch_set_wait_limit")

    def observables(self, k, psi, stream=None):
        _check_psi(psi, self.shape(k), self.prec)
        o = GpObs()
        check(lib().gp_batch_observables(self._h, int(k), ctypes.c_void_p(psi.data_ptr()), ctypes.byref(o),
                                         _stream_handle(stream)), "gp_batch_observables")
        return o.as_dict()


def thomas_table(n: int, dx: float, dt: float, mode: int, prec: int = GP_C128, adjoint: bool = False):
    """One axis's Thomas table as a plan stores it (host only): (c', beta, window K, rho)."""
    import numpy as np
    c = np.zeros(2 * n)
    beta = np.zeros(2 * n)
    K = ctypes.c_int()
    rho = ctypes.c_double()
    check(lib().gp_thomas_table(int(n), float(dx), float(dt), int(mode), int(prec), int(adjoint),
                                c.ctypes.data_as(c_dp), beta.ctypes.data_as(c_dp), ctypes.byref(K),
                                ctypes.byref(rho)), "gp_thomas_table")
    return c.view(np.complex128), beta.view(np.complex128), K.value, rho.value


def nonlinearity(ndim: int, natoms: float, a_bohr: float, l_micron: float, confine: float = 1.0) -> float:
    """gp_nonlinearity: dimensionless g from N, a (Bohr radii), l (micrometres) and the
    confinement ratio lambda (2D) or nu (1D)."""
    g = ctypes.c_double()
    check(lib().gp_nonlinearity(int(ndim), float(natoms), float(a_bohr), float(l_micron), float(confine),
                                ctypes.byref(g)), "gp_nonlinearity")
    return g.value


def osc_length(mass_amu: float, freq_hz: float) -> float:
    """gp_osc_length: sqrt(hbar / (m 2 pi f)) in micrometres."""
    v = ctypes.c_double()
    check(lib().gp_osc_length(float(mass_amu), float(freq_hz), ctypes.byref(v)), "gp_osc_length")
    return v.value


def observables_noalloc(psi, dx, omega=None, g: float = 0.0, stream=None) -> dict:
    """gp_observables_noalloc: observables of psi (x-first spacings dx, trap omega)
    without a plan; the library allocates nothing (static partial-sum array)."""
    n = tuple(int(v) for v in psi.shape[::-1])
    nd = len(n)
    prec = _prec_of(psi.dtype)
    _check_psi(psi, psi.shape, prec)
    dxs = [float(v) for v in (dx if hasattr(dx, "__len__") else [dx] * nd)]
    om = None if omega is None else (ctypes.c_double * nd)(*[float(v) for v in omega])
    o = GpObs()
    check(lib().gp_observables_noalloc(nd, (ctypes.c_int64 * nd)(*n), (ctypes.c_double * nd)(*dxs), om, float(g),
                                       prec, ctypes.c_void_p(psi.data_ptr()), ctypes.byref(o), _stream_handle(stream)),
          "gp_observables_noalloc")
    return o.as_dict()


def copy_probe(dst, src, stream=None):
    nbytes = src.numel() * src.element_size()
    check(lib().gp_copy_probe(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                              _stream_handle(stream)), "gp_copy_probe")

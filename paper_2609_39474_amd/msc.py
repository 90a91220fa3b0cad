"""ctypes binding of the HIP library ``libmsc_hip.so`` (C ABI in include/msc.h).

Argument marshalling only: every step of the method runs in the library's
kernels.  The functions keep the C names; ``Solver`` is a thin convenience
wrapper over one context.  Arrays cross the boundary as FP64 numpy arrays in
the canonical layout (populations ``f[k, x, y(, z)]``, hydrodynamic fields
``m[b, x, y(, z)]``).  PyTorch supplies the stream (and, on request, device
memory through its caching allocator).

Loading fails loudly when the library has not been built: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmsc_hip.so")

MSC_OK = 0
MSC_ERR_INVALID_ARG = 1
MSC_ERR_OUT_OF_MEMORY = 2
MSC_ERR_DEVICE = 3
MSC_ERR_STATE = 4
MSC_ERR_NONCONVERGED = 5
MSC_ERR_NONFINITE = 6
MSC_ERR_UNSUPPORTED = 7

MSC_D2Q9 = 2
MSC_D3Q19 = 3
MSC_CORRECTOR_PICARD = 0
MSC_CORRECTOR_SHADOW = 1
MSC_CORRECTOR_FULL_SYMBOL = 2
MSC_CORRECTOR_WALL_KINETIC = 3
MSC_BOUNDARY_PERIODIC = 0
MSC_BOUNDARY_CAVITY = 1
MSC_WALL_FROZEN = 0
MSC_WALL_ADAPTIVE = 1
MSC_STORAGE_FP64 = 0
MSC_STORAGE_FP32 = 1
MSC_STORAGE_FP16_DEV = 2

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class msc_params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("tau_plus", ctypes.c_double),
        ("tau_minus", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("k_max", ctypes.c_int32),
        ("n_min", ctypes.c_int32),
        ("corrector", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("inputs_on_device", ctypes.c_int32),
        ("extrap_states", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("alloc_fn", ALLOC_FN),
        ("free_fn", FREE_FN),
        ("alloc_user", ctypes.c_void_p),
        ("boundary", ctypes.c_int32),
        ("wall_operator", ctypes.c_int32),
        ("u_lid", ctypes.c_double),
        ("wall_forced", ctypes.c_int32),
        ("wall_restart", ctypes.c_int32),
        ("krylov_tol", ctypes.c_double),
    ]


class msc_step_stats(ctypes.Structure):
    _fields_ = [
        ("q", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("R_first", ctypes.c_double),
        ("R_final", ctypes.c_double),
        ("rho_obs", ctypes.c_double),
        ("converged", ctypes.c_int32),
        ("refreshes", ctypes.c_int32),
    ]


# every entry point declared in include/msc.h, with ctypes signatures
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p
SIGNATURES = {
    "msc_params_default": (ctypes.c_int, [ctypes.POINTER(msc_params), ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_double, ctypes.c_double]),
    "msc_init": (ctypes.c_int, [ctypes.POINTER(msc_params), _vp, _vp, ctypes.POINTER(_vp)]),
    "msc_bdf2_step": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(msc_step_stats)]),
    "msc_explicit_step": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "msc_moments": (ctypes.c_int, [_vp, _vp, _vp]),
    "msc_free": (None, [_vp]),
    "msc_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "msc_last_error": (ctypes.c_char_p, [_vp]),
    "msc_export_tables": (ctypes.c_int, [_vp, _ip, _ip, ctypes.POINTER(ctypes.c_uint8)]),
    "msc_get_populations": (ctypes.c_int, [_vp, _dp]),
    "msc_set_populations": (ctypes.c_int, [_vp, _dp]),
    "msc_sweep": (ctypes.c_int, [_vp, _dp, _dp, ctypes.c_double, _dp, _dp, _dp]),
    "msc_correct": (ctypes.c_int, [_vp, _dp, _dp, ctypes.c_double, _dp, _dp, _dp]),
    "msc_set_schedule": (ctypes.c_int, [_vp, _ip, ctypes.c_int32]),
    "msc_state_size": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64)]),
    "msc_get_state": (ctypes.c_int, [_vp, _dp, ctypes.POINTER(ctypes.c_int64)]),
    "msc_set_state": (ctypes.c_int, [_vp, _dp, ctypes.c_int64]),
    "msc_set_kernel_timing": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "msc_kernel_time": (ctypes.c_int, [_vp, ctypes.c_int32, _dp, ctypes.POINTER(ctypes.c_int64), _dp]),
    "msc_krylov_stats": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int64), _dp]),
    "msc_set_tuning": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32]),
    "msc_set_recording": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "msc_recorded_steps": (ctypes.c_int, [_vp, _ip]),
    "msc_bdf2_adjoint": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, ctypes.c_int32]),
    "msc_init_adjoint": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32]),
    "msc_sweep_noalloc": (ctypes.c_int, [ctypes.c_int32, _ip, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                         _vp, _vp, ctypes.c_double, _vp, _vp, _vp, _vp]),
}

_lib = None


def lib():
    """Load libmsc_hip.so (built by ``build()`` of the repository entry point)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
        # PyTorch ships its own HIP runtime.  Importing it first makes the
        # library bind to that same runtime (one runtime per process), so that
        # torch streams and allocations are valid here and torch can still
        # initialise the GPU after the library has used it.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class MscError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{lib().msc_status_string(status).decode()} ({status}): {msg}")


def _dptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def msc_params_default(lattice, n, dt, eps):
    p = msc_params()
    rc = lib().msc_params_default(ctypes.byref(p), lattice, n, dt, eps)
    if rc != MSC_OK:
        raise MscError(rc)
    return p


class TorchAllocator:
    """Device memory from torch's caching allocator (alloc_fn/free_fn hooks)."""

    def __init__(self):
        import torch

        self._torch = torch
        self._alloc = ALLOC_FN(self._a)
        self._free = FREE_FN(self._f)

    def _a(self, nbytes, user):
        try:
            return int(self._torch.cuda.caching_allocator_alloc(int(nbytes)))
        except Exception:
            return None

    def _f(self, ptr, user):
        if ptr:
            self._torch.cuda.caching_allocator_delete(int(ptr))

    def install(self, p: msc_params):
        p.alloc_fn = self._alloc
        p.free_fn = self._free


class Solver:
    """One library context.  Raises MscError on any non-OK status except the
    step failures that ``bdf2_step(..., raise_on_fail=False)`` returns."""

    def __init__(self, params: msc_params, phat0, u0, stream=None, torch_alloc=False):
        """phat0, u0: host arrays, or device FP64 tensors (anything with
        ``data_ptr``), which sets params.inputs_on_device: msc_moments then
        writes device pointers too (``moments_device``)."""
        self.params = params
        self.d = 2 if params.lattice == MSC_D2Q9 else 3
        self.Q = 9 if self.d == 2 else 19
        self.shape = tuple(params.n[: self.d])
        self.NS = int(np.prod(self.shape))
        self._keep = []
        if stream is not None:
            params.stream = ctypes.c_void_p(int(stream))
        if torch_alloc:
            ta = TorchAllocator()
            ta.install(params)
            self._keep.append(ta)
        self.on_device = hasattr(phat0, "data_ptr")
        if self.on_device:
            assert tuple(phat0.shape) == self.shape and tuple(u0.shape) == (self.d,) + self.shape
            assert phat0.is_contiguous() and u0.is_contiguous()
            params.inputs_on_device = 1
            p_ptr, u_ptr = phat0.data_ptr(), u0.data_ptr()
        else:
            params.inputs_on_device = 0
            phat0 = _f64(phat0)
            u0 = _f64(u0)
            assert phat0.shape == self.shape and u0.shape == (self.d,) + self.shape
            p_ptr, u_ptr = phat0.ctypes.data, u0.ctypes.data
        h = ctypes.c_void_p()
        rc = lib().msc_init(ctypes.byref(params), ctypes.c_void_p(p_ptr), ctypes.c_void_p(u_ptr), ctypes.byref(h))
        if rc != MSC_OK:
            raise MscError(rc, "msc_init")
        self.h = h

    # -- lifecycle
    def close(self):
        if getattr(self, "h", None):
            lib().msc_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != MSC_OK:
            raise MscError(rc, f"{what}: {lib().msc_last_error(self.h).decode()}")

    # -- march
    def bdf2_step(self, nsteps, raise_on_fail=True):
        st = (msc_step_stats * max(1, nsteps))()
        rc = lib().msc_bdf2_step(self.h, nsteps, st)
        stats = [dict(q=s.q, iters=s.iters, R_first=s.R_first, R_final=s.R_final, rho_obs=s.rho_obs,
                      converged=s.converged, refreshes=s.refreshes) for s in st[:nsteps]]
        if rc != MSC_OK and raise_on_fail:
            self._check(rc, "msc_bdf2_step")
        return rc, stats

    def explicit_step(self, nsteps):
        self._check(lib().msc_explicit_step(self.h, int(nsteps)), "msc_explicit_step")

    def moments_device(self, phat_ptr, u_ptr):
        assert self.on_device
        self._check(lib().msc_moments(self.h, ctypes.c_void_p(int(phat_ptr)), ctypes.c_void_p(int(u_ptr))),
                    "msc_moments")

    def moments(self):
        if self.on_device:
            raise ValueError("context created from device inputs: use moments_device")
        m = np.zeros((self.d + 1,) + self.shape)
        self._check(lib().msc_moments(self.h, m.ctypes.data, m[1:].ctypes.data), "msc_moments")
        return m

    def populations(self):
        f = np.zeros((self.Q,) + self.shape)
        self._check(lib().msc_get_populations(self.h, _dptr(f)), "msc_get_populations")
        return f

    def set_populations(self, f):
        f = _f64(f)
        self._check(lib().msc_set_populations(self.h, _dptr(f)), "msc_set_populations")

    # -- diagnostics
    def sweep(self, f, h, a):
        f = _f64(f)
        h = _f64(h)
        fT = np.zeros_like(f)
        Pr = np.zeros((self.d + 1,) + self.shape)
        R = ctypes.c_double()
        self._check(lib().msc_sweep(self.h, _dptr(f), _dptr(h), a, _dptr(fT), _dptr(Pr), ctypes.byref(R)),
                    "msc_sweep")
        return fT, Pr, R.value

    def correct(self, f, h, a):
        f = _f64(f)
        h = _f64(h)
        fn = np.zeros_like(f)
        dm = np.zeros((self.d + 1,) + self.shape)
        R = ctypes.c_double()
        self._check(lib().msc_correct(self.h, _dptr(f), _dptr(h), a, _dptr(fn), _dptr(dm), ctypes.byref(R)),
                    "msc_correct")
        return fn, dm, R.value

    def tables(self):
        nbr = np.zeros(self.Q * self.NS, dtype=np.int32)
        sidx = np.zeros(int(sum(self.shape)), dtype=np.int32)
        mask = np.zeros(self.NS, dtype=np.uint8)
        self._check(lib().msc_export_tables(self.h, nbr.ctypes.data_as(_ip), sidx.ctypes.data_as(_ip),
                                            mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))),
                    "msc_export_tables")
        return nbr.reshape(self.Q, self.NS), sidx, mask

    def set_schedule(self, K):
        if K is None:
            self._check(lib().msc_set_schedule(self.h, None, 0), "msc_set_schedule")
            return
        K = np.ascontiguousarray(K, dtype=np.int32)
        self._check(lib().msc_set_schedule(self.h, K.ctypes.data_as(_ip), len(K)), "msc_set_schedule")

    def state_size(self):
        n = ctypes.c_int64()
        self._check(lib().msc_state_size(self.h, ctypes.byref(n)), "msc_state_size")
        return n.value

    def get_state(self):
        s = np.zeros(self.state_size())
        bc = ctypes.c_int64()
        self._check(lib().msc_get_state(self.h, _dptr(s), ctypes.byref(bc)), "msc_get_state")
        return s, bc.value

    def set_state(self, s, bdf_count):
        s = _f64(s)
        self._check(lib().msc_set_state(self.h, _dptr(s), int(bdf_count)), "msc_set_state")

    def set_kernel_timing(self, on):
        self._check(lib().msc_set_kernel_timing(self.h, 1 if on else 0), "msc_set_kernel_timing")

    def kernel_time(self, kind):
        sec = ctypes.c_double()
        n = ctypes.c_int64()
        b = ctypes.c_double()
        self._check(lib().msc_kernel_time(self.h, kind, ctypes.byref(sec), ctypes.byref(n), ctypes.byref(b)),
                    "msc_kernel_time")
        return sec.value, n.value, b.value

    def krylov_stats(self):
        """(solves, GMRES iterations, refreshes, worst final relative residual)
        of the wall corrector since creation."""
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        w = ctypes.c_double()
        self._check(lib().msc_krylov_stats(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                           ctypes.byref(w)), "msc_krylov_stats")
        return a.value, b.value, c.value, w.value

    def set_tuning(self, key, value):
        self._check(lib().msc_set_tuning(self.h, key, value), "msc_set_tuning")

    # -- adjoint
    def set_recording(self, on):
        self._check(lib().msc_set_recording(self.h, 1 if on else 0), "msc_set_recording")

    def recorded_steps(self):
        n = ctypes.c_int32()
        self._check(lib().msc_recorded_steps(self.h, ctypes.byref(n)), "msc_recorded_steps")
        return n.value

    def bdf2_adjoint(self, nsteps, lam):
        """Host FP64 state-layout adjoint in, adjoint before the nsteps steps out."""
        lam = np.array(lam, dtype=np.float64, copy=True)
        self._check(lib().msc_bdf2_adjoint(self.h, int(nsteps), lam.ctypes.data, 0), "msc_bdf2_adjoint")
        return lam

    def bdf2_adjoint_device(self, nsteps, lam_ptr):
        """In-place on a device FP64 buffer (pointer as int)."""
        self._check(lib().msc_bdf2_adjoint(self.h, int(nsteps), ctypes.c_void_p(int(lam_ptr)), 1),
                    "msc_bdf2_adjoint")

    def init_adjoint(self, phat0, u0, lam):
        phat0, u0, lam = _f64(phat0), _f64(u0), _f64(lam)
        lp = np.zeros(self.shape)
        lu = np.zeros((self.d,) + self.shape)
        self._check(lib().msc_init_adjoint(self.h, phat0.ctypes.data, u0.ctypes.data, lam.ctypes.data,
                                           lp.ctypes.data, lu.ctypes.data, 0), "msc_init_adjoint")
        return lp, lu

    def init_adjoint_device(self, phat0_ptr, u0_ptr, lam_ptr, lp_ptr, lu_ptr):
        ptrs = [ctypes.c_void_p(int(p)) for p in (phat0_ptr, u0_ptr, lam_ptr, lp_ptr, lu_ptr)]
        self._check(lib().msc_init_adjoint(self.h, *ptrs, 1), "msc_init_adjoint")


def sweep_noalloc(d, n, storage, f_ptr, h_ptr, a, fT_ptr, Pr_ptr, R_ptr=None, stream=None, tau_plus=1.0,
                  tau_minus=1.0):
    """msc_sweep_noalloc on device pointers (ints): one sweep with no context
    and no device allocation.  storage "fp64" or "fp32"; R_ptr may be None.
    Enqueues on ``stream`` and returns without synchronising."""
    ext = (ctypes.c_int32 * 3)(*(list(n) + [1] * (3 - len(n))))
    st = {"fp64": MSC_STORAGE_FP64, "fp32": MSC_STORAGE_FP32, "fp16dev": MSC_STORAGE_FP16_DEV}[storage]
    rc = lib().msc_sweep_noalloc(MSC_D2Q9 if d == 2 else MSC_D3Q19, ext, tau_plus, tau_minus, st, f_ptr, h_ptr, a,
                                 fT_ptr, Pr_ptr, R_ptr, stream)
    if rc != MSC_OK:
        raise MscError(rc, "msc_sweep_noalloc")


def make_params(d, N, *, dt, eps, storage="fp64", corrector="shadow", tau_plus=1.0, tau_minus=1.0,
                k_max=300, n_min=None, extrap_states=0, boundary="periodic", u_lid=0.0, wall_operator="frozen",
                wall_forced=0, wall_restart=0, krylov_tol=0.0):
    p = msc_params_default(MSC_D2Q9 if d == 2 else MSC_D3Q19, N, dt, eps)
    p.storage = {"fp64": MSC_STORAGE_FP64, "fp32": MSC_STORAGE_FP32, "fp16dev": MSC_STORAGE_FP16_DEV}[storage]
    p.corrector = {"shadow": MSC_CORRECTOR_SHADOW, "picard": MSC_CORRECTOR_PICARD,
                   "full_symbol": MSC_CORRECTOR_FULL_SYMBOL, "wall_kinetic": MSC_CORRECTOR_WALL_KINETIC}[corrector]
    p.boundary = {"periodic": MSC_BOUNDARY_PERIODIC, "cavity": MSC_BOUNDARY_CAVITY}[boundary]
    p.u_lid = u_lid
    p.wall_operator = {"frozen": MSC_WALL_FROZEN, "adaptive": MSC_WALL_ADAPTIVE}[wall_operator]
    p.wall_forced = wall_forced
    p.wall_restart = wall_restart
    p.krylov_tol = krylov_tol
    p.tau_plus = tau_plus
    p.tau_minus = tau_minus
    p.k_max = k_max
    p.extrap_states = extrap_states
    if n_min is not None:
        p.n_min = n_min
    return p

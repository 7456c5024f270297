"""Python binding of liblbm (ctypes): argument marshalling only.

Every function here has the name and meaning of the C entry point declared
in ``include/lbm.h``; all work runs in the HIP library.  Host arrays are
numpy FP64; device arrays are torch CUDA (HIP) tensors, passed by pointer.
Importing this module raises if ``liblbm.so`` has not been built -- there is
no fallback path.
"""
import ctypes
import os

import numpy as np

# One HIP runtime per process: PyTorch ships its own libamdhip64 with the
# same soname as the system one liblbm links against.  Loading torch first
# makes liblbm bind to the runtime torch already holds; the other order
# would bring up a second runtime, and torch's would then see no GPU.
try:
    import torch  # noqa: F401
except ImportError:  # torch is optional for host-array use of the library
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ESTATE, LBM_ENONFINITE = 0, -1, -2, -3, -4, -5
LBM_EBUSY = -6
LBM_ESCRATCH = -7
LBM_D2Q37, LBM_D3Q107 = 37, 107
LBM_BC_PERIODIC, LBM_BC_ZERO_GRADIENT = 0, 1
LBM_FP64, LBM_FP32_DEV, LBM_FP16_SCALED = 0, 1, 2
LBM_VARIANT_AUTO, LBM_VARIANT_LANE, LBM_VARIANT_SPLIT, LBM_VARIANT_TWO_PASS = 0, 1, 2, 3
LBM_VARIANT_SPLIT_LDS = 4
LBM_COLLISION_PAPER, LBM_COLLISION_ENERGY_CONSERVING = 0, 1


def LBM_BC(bx, by, bz=0):
    return (bx & 3) | ((by & 3) << 2) | ((bz & 3) << 4)


class LBMError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {lbm_strerror(code)} ({code})")


class NonFiniteError(LBMError):
    def __init__(self, code, where, totals):
        super().__init__(code, where)
        self.totals = totals


class _Info(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("q", ctypes.c_int), ("precision", ctypes.c_int),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("bc", ctypes.c_uint32),
                ("gamma", ctypes.c_double), ("delta", ctypes.c_double),
                ("tau_f", ctypes.c_double), ("tau_g", ctypes.c_double), ("r", ctypes.c_double),
                ("steps", ctypes.c_int64), ("device_bytes", ctypes.c_size_t),
                ("scheme", ctypes.c_int), ("dt", ctypes.c_double), ("collision", ctypes.c_int)]


class lbm_request(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("gamma", ctypes.c_double), ("tau_f", ctypes.c_double),
                ("tau_g", ctypes.c_double), ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("nz", ctypes.c_int64), ("bc", ctypes.c_uint32), ("steps", ctypes.c_int64)]


class _PoolInfo(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("used_bytes", ctypes.c_size_t),
                ("largest_free_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int),
                ("resident", ctypes.c_int), ("graphs", ctypes.c_int)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1608_06345_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, d, i64, i32 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int64, ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "lbm_create": [i32, i32, d, d, d, i64, i64, i64, ctypes.c_uint32, ctypes.POINTER(vp)],
        "lbm_create_ex": [i32, i32, d, d, d, i64, i64, i64, ctypes.c_uint32, i32,
                          ctypes.POINTER(vp)],
        "lbm_create_fd": [i32, i32, d, d, d, d, i64, i64, i64, ctypes.c_uint32, i32,
                          ctypes.POINTER(vp)],
        "lbm_destroy": [vp],
        "lbm_set_stream": [vp, vp],
        "lbm_set_variant": [vp, i32],
        "lbm_set_collision": [vp, i32],
        "lbm_synchronize": [vp],
        "lbm_init_fields": [vp, dp, dp, dp],
        "lbm_init_fields_dev": [vp, vp, vp, vp],
        "lbm_step": [vp, i64],
        "lbm_moments": [vp, dp, dp, dp],
        "lbm_moments_dev": [vp, vp, vp, vp],
        "lbm_moments_noalloc": [vp, dp, dp, dp],
        "lbm_temperature": [vp, dp],
        "lbm_temperature_dev": [vp, vp],
        "lbm_totals": [vp, dp, dp, dp],
        "lbm_get_info": [vp, ctypes.POINTER(_Info)],
        "lbm_lattice": [i32, ctypes.POINTER(ctypes.c_int8), dp, dp],
        "lbm_pool_create": [ctypes.c_size_t, i32, i32, ctypes.POINTER(vp)],
        "lbm_pool_destroy": [vp],
        "lbm_pool_set_stream": [vp, vp],
        "lbm_pool_admit": [vp, ctypes.POINTER(lbm_request), dp, dp, dp, ctypes.POINTER(i32)],
        "lbm_pool_admit_dev": [vp, ctypes.POINTER(lbm_request), vp, vp, vp, ctypes.POINTER(i32)],
        "lbm_pool_run": [vp, i32],
        "lbm_pool_run_eager": [vp, i32],
        "lbm_pool_poll": [vp, ctypes.POINTER(i32), i32, ctypes.POINTER(i32)],
        "lbm_pool_slot_steps": [vp, i32, ctypes.POINTER(i64)],
        "lbm_pool_moments": [vp, i32, dp, dp, dp],
        "lbm_pool_moments_dev": [vp, i32, vp, vp, vp],
        "lbm_pool_totals": [vp, i32, dp, dp, dp],
        "lbm_pool_temperature": [vp, i32, dp],
        "lbm_pool_release": [vp, i32],
        "lbm_pool_get_info": [vp, ctypes.POINTER(_PoolInfo)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.lbm_footprint_bytes.argtypes = [i32, i32, i32, i64, i64, i64]
    lib.lbm_footprint_bytes.restype = ctypes.c_size_t
    lib.lbm_pool_request_bytes.argtypes = [ctypes.POINTER(lbm_request), i32]
    lib.lbm_pool_request_bytes.restype = ctypes.c_size_t
    lib.lbm_strerror.argtypes = [i32]
    lib.lbm_strerror.restype = ctypes.c_char_p
    return lib


_lib = _load()


def _check(rc, where):
    if rc != LBM_OK:
        raise LBMError(rc, where)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _host(a, n):
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    if a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _dev_ptr(t, n):
    if not (hasattr(t, "is_cuda") and t.is_cuda):
        raise TypeError("expected a device (torch CUDA/HIP) tensor")
    if t.dtype.__repr__() != "torch.float64" or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"expected a contiguous float64 device tensor of {n} values")
    return ctypes.c_void_p(t.data_ptr())


def lbm_strerror(code):
    return _lib.lbm_strerror(int(code)).decode()


def lbm_create_ex(dim, velocity_set, gamma, tau_f, tau_g, nx, ny, nz, bc, precision):
    h = ctypes.c_void_p()
    _check(_lib.lbm_create_ex(dim, velocity_set, gamma, tau_f, tau_g, nx, ny, nz, bc,
                              precision, ctypes.byref(h)), "lbm_create_ex")
    return h


def lbm_create_fd(dim, velocity_set, gamma, tau_f, tau_g, dt, nx, ny, nz, bc, precision):
    h = ctypes.c_void_p()
    _check(_lib.lbm_create_fd(dim, velocity_set, gamma, tau_f, tau_g, dt, nx, ny, nz, bc,
                              precision, ctypes.byref(h)), "lbm_create_fd")
    return h


def lbm_create_fd_rc(dim, velocity_set, gamma, tau_f, tau_g, dt, nx, ny, nz, bc,
                     precision=LBM_FP64):
    """Raw status code of lbm_create_fd (for error-path tests); destroys a
    handle that was created."""
    h = ctypes.c_void_p()
    rc = _lib.lbm_create_fd(dim, velocity_set, gamma, tau_f, tau_g, dt, nx, ny, nz, bc,
                            precision, ctypes.byref(h))
    if rc == LBM_OK:
        _lib.lbm_destroy(h)
    return rc


def lbm_create(dim, velocity_set, gamma, tau_f, tau_g, nx, ny, nz, bc):
    h = ctypes.c_void_p()
    _check(_lib.lbm_create(dim, velocity_set, gamma, tau_f, tau_g, nx, ny, nz, bc,
                           ctypes.byref(h)), "lbm_create")
    return h


def lbm_create_rc(dim, velocity_set, gamma, tau_f, tau_g, nx, ny, nz, bc,
                  precision=LBM_FP64):
    """Raw status code of lbm_create_ex (for error-path tests); destroys a
    handle that was created."""
    h = ctypes.c_void_p()
    rc = _lib.lbm_create_ex(dim, velocity_set, gamma, tau_f, tau_g, nx, ny, nz, bc,
                            precision, ctypes.byref(h))
    if rc == LBM_OK:
        _lib.lbm_destroy(h)
    return rc


def lbm_destroy(h):
    _check(_lib.lbm_destroy(h), "lbm_destroy")


def lbm_set_stream(h, stream):
    """``stream``: a torch stream, a raw hipStream_t integer, or None / 0 for
    the null stream."""
    ptr = getattr(stream, "cuda_stream", stream)
    _check(_lib.lbm_set_stream(h, ctypes.c_void_p(ptr or 0)), "lbm_set_stream")


def lbm_set_variant(h, variant):
    _check(_lib.lbm_set_variant(h, int(variant)), "lbm_set_variant")


def lbm_set_collision(h, mode):
    _check(_lib.lbm_set_collision(h, int(mode)), "lbm_set_collision")


def lbm_synchronize(h):
    _check(_lib.lbm_synchronize(h), "lbm_synchronize")


def lbm_get_info(h):
    info = _Info()
    _check(_lib.lbm_get_info(h, ctypes.byref(info)), "lbm_get_info")
    return {name: getattr(info, name) for name, _ in _Info._fields_}


def lbm_init_fields(h, rho, u, T):
    inf = lbm_get_info(h)
    n = inf["nx"] * inf["ny"] * inf["nz"]
    rho, u, T = _host(rho, n), _host(u, inf["dim"] * n), _host(T, n)
    _check(_lib.lbm_init_fields(h, _dp(rho), _dp(u), _dp(T)), "lbm_init_fields")


def lbm_init_fields_dev(h, rho, u, T):
    inf = lbm_get_info(h)
    n = inf["nx"] * inf["ny"] * inf["nz"]
    _check(_lib.lbm_init_fields_dev(h, _dev_ptr(rho, n), _dev_ptr(u, inf["dim"] * n),
                                    _dev_ptr(T, n)), "lbm_init_fields_dev")


def lbm_step(h, n):
    _check(_lib.lbm_step(h, int(n)), "lbm_step")


def lbm_moments(h):
    """(rho [cells], u [dim][cells], E [cells]) of S_n as FP64 numpy arrays."""
    inf = lbm_get_info(h)
    n = inf["nx"] * inf["ny"] * inf["nz"]
    rho, u, E = np.empty(n), np.empty((inf["dim"], n)), np.empty(n)
    _check(_lib.lbm_moments(h, _dp(rho), _dp(u), _dp(E)), "lbm_moments")
    return rho, u, E


def lbm_moments_noalloc(h):
    """As lbm_moments, staged through the library's fixed device scratch
    (no device allocation)."""
    inf = lbm_get_info(h)
    n = inf["nx"] * inf["ny"] * inf["nz"]
    rho, u, E = np.empty(n), np.empty((inf["dim"], n)), np.empty(n)
    _check(_lib.lbm_moments_noalloc(h, _dp(rho), _dp(u), _dp(E)), "lbm_moments_noalloc")
    return rho, u, E


def lbm_moments_noalloc_rc(h):
    """Raw status code of lbm_moments_noalloc (for error-path tests)."""
    inf = lbm_get_info(h)
    n = inf["nx"] * inf["ny"] * inf["nz"]
    rho, u, E = np.empty(n), np.empty((inf["dim"], n)), np.empty(n)
    return _lib.lbm_moments_noalloc(h, _dp(rho), _dp(u), _dp(E))


def lbm_moments_dev(h, rho, u, E):
    inf = lbm_get_info(h)
    n = inf["nx"] * inf["ny"] * inf["nz"]
    _check(_lib.lbm_moments_dev(h, _dev_ptr(rho, n), _dev_ptr(u, inf["dim"] * n),
                                _dev_ptr(E, n)), "lbm_moments_dev")


def lbm_temperature(h):
    """T [cells] of S_n as an FP64 numpy array (formed by the library)."""
    inf = lbm_get_info(h)
    T = np.empty(inf["nx"] * inf["ny"] * inf["nz"])
    _check(_lib.lbm_temperature(h, _dp(T)), "lbm_temperature")
    return T


def lbm_temperature_dev(h, T):
    inf = lbm_get_info(h)
    _check(_lib.lbm_temperature_dev(h, _dev_ptr(T, inf["nx"] * inf["ny"] * inf["nz"])),
           "lbm_temperature_dev")


def lbm_totals(h):
    """(mass, momentum [dim], energy); NonFiniteError if any is NaN/Inf."""
    inf = lbm_get_info(h)
    mass, energy = np.zeros(1), np.zeros(1)
    mom = np.zeros(3)
    rc = _lib.lbm_totals(h, _dp(mass), _dp(mom), _dp(energy))
    out = (float(mass[0]), mom[:inf["dim"]].copy(), float(energy[0]))
    if rc == LBM_ENONFINITE:
        raise NonFiniteError(rc, "lbm_totals", out)
    _check(rc, "lbm_totals")
    return out


def lbm_footprint_bytes(dim, velocity_set, precision, nx, ny, nz):
    return int(_lib.lbm_footprint_bytes(dim, velocity_set, precision, nx, ny, nz))


def lbm_lattice(velocity_set):
    """(e [q][3] int8, w [q] FP64, r) of the library's lattice."""
    q = _lib.lbm_lattice(velocity_set, None, None, None)
    if q < 0:
        raise LBMError(q, "lbm_lattice")
    e = np.zeros((q, 3), dtype=np.int8)
    w = np.zeros(q)
    r = np.zeros(1)
    _lib.lbm_lattice(velocity_set, e.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), _dp(w),
                     _dp(r))
    return e, w, float(r[0])


class Solver:
    """One solve behind a handle; closes it on ``close()`` / exit.  With
    ``dt`` it advances by the finite-difference form (``lbm_create_fd``),
    else by lattice streaming."""

    def __init__(self, dim, gamma, tau_f, tau_g, nx, ny, nz=1, bc=0, precision=LBM_FP64,
                 dt=None, collision=LBM_COLLISION_PAPER):
        vs = LBM_D2Q37 if dim == 2 else LBM_D3Q107
        if dt is None:
            self.h = lbm_create_ex(dim, vs, gamma, tau_f, tau_g, nx, ny, nz, bc, precision)
        else:
            self.h = lbm_create_fd(dim, vs, gamma, tau_f, tau_g, dt, nx, ny, nz, bc, precision)
        if collision != LBM_COLLISION_PAPER:
            lbm_set_collision(self.h, collision)
        self.dim = dim
        self.ncells = nx * ny * nz

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def close(self):
        if self.h is not None:
            lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def info(self):
        return lbm_get_info(self.h)

    def init_fields(self, rho, u, T):
        lbm_init_fields(self.h, rho, u, T)

    def step(self, n=1):
        lbm_step(self.h, n)

    def moments(self):
        return lbm_moments(self.h)

    def temperature(self):
        return lbm_temperature(self.h)

    def totals(self):
        return lbm_totals(self.h)

    def synchronize(self):
        lbm_synchronize(self.h)

    def set_stream(self, stream):
        lbm_set_stream(self.h, stream)

    def set_variant(self, variant):
        lbm_set_variant(self.h, variant)


# --------------------------------------------------------------------------
# Batched multi-solve pool


def make_request(dim, gamma, tau_f, tau_g, nx, ny, nz=1, bc=0, steps=0):
    return lbm_request(dim, gamma, tau_f, tau_g, nx, ny, nz if dim == 3 else 1, bc, steps)


def lbm_pool_request_bytes(req, precision):
    return int(_lib.lbm_pool_request_bytes(ctypes.byref(req), precision))


def lbm_pool_create(budget_bytes, max_slots, precision):
    p = ctypes.c_void_p()
    _check(_lib.lbm_pool_create(int(budget_bytes), int(max_slots), int(precision),
                                ctypes.byref(p)), "lbm_pool_create")
    return p


def lbm_pool_create_rc(budget_bytes, max_slots, precision):
    p = ctypes.c_void_p()
    rc = _lib.lbm_pool_create(int(budget_bytes), int(max_slots), int(precision),
                              ctypes.byref(p))
    if rc == LBM_OK:
        _lib.lbm_pool_destroy(p)
    return rc


def lbm_pool_destroy(p):
    _check(_lib.lbm_pool_destroy(p), "lbm_pool_destroy")


class Pool:
    """A batched multi-solve pool (see lbm.h).  ``admit`` returns the slot,
    or None when the pool has no room right now (EBUSY)."""

    def __init__(self, budget_bytes, max_slots, precision=LBM_FP32_DEV):
        self.p = lbm_pool_create(budget_bytes, max_slots, precision)
        self.precision = precision
        self.requests = {}

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def close(self):
        if self.p is not None:
            lbm_pool_destroy(self.p)
            self.p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        ptr = getattr(stream, "cuda_stream", stream)
        _check(_lib.lbm_pool_set_stream(self.p, ctypes.c_void_p(ptr or 0)), "lbm_pool_set_stream")

    def admit(self, req, rho, u, T):
        n = req.nx * req.ny * req.nz
        rho, u, T = _host(rho, n), _host(u, req.dim * n), _host(T, n)
        slot = ctypes.c_int(-1)
        rc = _lib.lbm_pool_admit(self.p, ctypes.byref(req), _dp(rho), _dp(u), _dp(T),
                                 ctypes.byref(slot))
        if rc == LBM_EBUSY:
            return None
        _check(rc, "lbm_pool_admit")
        self.requests[slot.value] = req
        return slot.value

    def admit_dev(self, req, rho, u, T):
        n = req.nx * req.ny * req.nz
        slot = ctypes.c_int(-1)
        rc = _lib.lbm_pool_admit_dev(self.p, ctypes.byref(req), _dev_ptr(rho, n),
                                     _dev_ptr(u, req.dim * n), _dev_ptr(T, n),
                                     ctypes.byref(slot))
        if rc == LBM_EBUSY:
            return None
        _check(rc, "lbm_pool_admit_dev")
        self.requests[slot.value] = req
        return slot.value

    def run(self, ticks):
        _check(_lib.lbm_pool_run(self.p, int(ticks)), "lbm_pool_run")

    def run_eager(self, ticks):
        _check(_lib.lbm_pool_run_eager(self.p, int(ticks)), "lbm_pool_run_eager")

    def poll(self, max_finished=1024):
        buf = (ctypes.c_int * max_finished)()
        n = ctypes.c_int(0)
        _check(_lib.lbm_pool_poll(self.p, buf, max_finished, ctypes.byref(n)), "lbm_pool_poll")
        return [buf[i] for i in range(n.value)]

    def steps_done(self, slot):
        v = ctypes.c_int64(0)
        _check(_lib.lbm_pool_slot_steps(self.p, slot, ctypes.byref(v)), "lbm_pool_slot_steps")
        return v.value

    def moments(self, slot):
        req = self.requests[slot]
        n = req.nx * req.ny * req.nz
        rho, u, E = np.empty(n), np.empty((req.dim, n)), np.empty(n)
        _check(_lib.lbm_pool_moments(self.p, slot, _dp(rho), _dp(u), _dp(E)), "lbm_pool_moments")
        return rho, u, E

    def totals(self, slot):
        req = self.requests[slot]
        mass, energy, mom = np.zeros(1), np.zeros(1), np.zeros(3)
        rc = _lib.lbm_pool_totals(self.p, slot, _dp(mass), _dp(mom), _dp(energy))
        out = (float(mass[0]), mom[:req.dim].copy(), float(energy[0]))
        if rc == LBM_ENONFINITE:
            raise NonFiniteError(rc, "lbm_pool_totals", out)
        _check(rc, "lbm_pool_totals")
        return out

    def temperature(self, slot):
        req = self.requests[slot]
        T = np.empty(req.nx * req.ny * req.nz)
        _check(_lib.lbm_pool_temperature(self.p, slot, _dp(T)), "lbm_pool_temperature")
        return T

    def release(self, slot):
        _check(_lib.lbm_pool_release(self.p, slot), "lbm_pool_release")
        self.requests.pop(slot, None)

    def info(self):
        inf = _PoolInfo()
        _check(_lib.lbm_pool_get_info(self.p, ctypes.byref(inf)), "lbm_pool_get_info")
        return {name: getattr(inf, name) for name, _ in _PoolInfo._fields_}

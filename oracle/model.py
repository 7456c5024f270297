"""ctypes wrapper of the C oracle (``lbm_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).

``build()`` compiles ``liboracle.so`` next to this file with gcc (-O2,
OpenMP).  ``OracleLBM`` holds one solve: the two reduced distributions g
(mass) and h (energy) in FP64, cell-major ``[cells][Q]``.
"""
import ctypes
import os
import subprocess

import numpy as np

from .lattice import delta_from_gamma, lattice

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force=True):
    """Compile the C oracle (plain gcc; no GPU code)."""
    if not force and os.path.exists(_LIB) and \
            os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                           "-std=c99", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


class _Model(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int), ("Q", ctypes.c_int),
                ("e", ctypes.POINTER(ctypes.c_long)),
                ("w", ctypes.POINTER(ctypes.c_double)),
                ("r", ctypes.c_double), ("delta", ctypes.c_double),
                ("tau_f", ctypes.c_double), ("tau_g", ctypes.c_double),
                ("n", ctypes.c_long * 3), ("open_end", ctypes.c_int * 3),
                ("energy_fix", ctypes.c_int)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d = P(ctypes.c_double)
        m = P(_Model)
        lib.orc_feq.argtypes = [m, ctypes.c_double, d, ctypes.c_double, d]
        lib.orc_macro.argtypes = [m, d, d, d, d, d, d]
        lib.orc_collide_cell.argtypes = [m, d, d]
        lib.orc_init.argtypes = [m, d, d, d, d, d]
        lib.orc_step.argtypes = [m, d, d, ctypes.c_long]
        lib.orc_step.restype = ctypes.c_int
        lib.orc_fd_step.argtypes = [m, d, d, ctypes.c_long, ctypes.c_double]
        lib.orc_fd_step.restype = ctypes.c_int
        lib.orc_moments.argtypes = [m, d, d, d, d, d]
        lib.orc_totals.argtypes = [m, d, d, d, d, d]
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_threads():
    return _load().orc_num_threads()


def set_num_threads(n):
    _load().orc_set_num_threads(int(n))


class OracleLBM:
    """One solve of the two-distribution scheme on an nx x ny (x nz) grid.

    ``open_end``: per axis, True for the zero-gradient (open) end condition,
    False for periodic.  ``rho``/``T`` are ``[cells]`` and ``u`` is
    ``[dim][cells]`` with cell = x + nx (y + ny z).

    ``dt``: None for the lattice scheme (collide, then stream e_i cells per
    step; tau in lattice units), or the time step of the finite-difference
    form of Sec. III (grid step 1, speeds xi_i = r e_i; tau_f and tau_g then
    in the units of dt).

    ``energy_fix``: the energy-conserving collision for tau_f != tau_g (a
    mode beyond the paper; see energy_fix_kappa in the C source).
    """

    def __init__(self, dim, gamma, tau_f, tau_g, nx, ny, nz=1,
                 open_end=(False, False, False), delta=None, dt=None, energy_fix=False):
        self.lat = lattice(dim)
        self.dim = dim
        self.delta = delta_from_gamma(gamma, dim) if delta is None else delta
        self.gamma = gamma
        self.shape = (nx, ny, nz if dim == 3 else 1)
        if dim == 2 and nz != 1:
            raise ValueError("nz must be 1 in 2D")
        self._e = np.ascontiguousarray(self.lat.e, dtype=np.int64)
        self._w = np.ascontiguousarray(self.lat.w, dtype=np.float64)
        m = _Model()
        m.D, m.Q = dim, self.lat.Q
        m.e = self._e.ctypes.data_as(ctypes.POINTER(ctypes.c_long))
        m.w = _dp(self._w)
        m.r = self.lat.r
        m.delta = self.delta
        m.tau_f, m.tau_g = tau_f, tau_g
        for k in range(3):
            m.n[k] = self.shape[k]
            m.open_end[k] = 1 if open_end[k] else 0
        m.energy_fix = 1 if energy_fix else 0
        self._m = m
        self.ncells = nx * ny * self.shape[2]
        self.g = np.zeros((self.ncells, self.lat.Q))
        self.h = np.zeros((self.ncells, self.lat.Q))
        self.steps = 0
        self.dt = dt

    @property
    def Q(self):
        return self.lat.Q

    # per-cell primitives (used by the pins) -------------------------------
    def feq(self, rho, u, theta):
        F = np.zeros(self.Q)
        uu = np.zeros(3)
        uu[:self.dim] = u
        _load().orc_feq(ctypes.byref(self._m), float(rho), _dp(uu),
                        float(theta), _dp(F))
        return F

    def macro(self, g, h):
        g = np.ascontiguousarray(g, dtype=np.float64)
        h = np.ascontiguousarray(h, dtype=np.float64)
        u = np.zeros(3)
        rho, E, T = (ctypes.c_double(), ctypes.c_double(), ctypes.c_double())
        _load().orc_macro(ctypes.byref(self._m), _dp(g), _dp(h),
                          ctypes.cast(ctypes.byref(rho), ctypes.POINTER(ctypes.c_double)),
                          _dp(u),
                          ctypes.cast(ctypes.byref(E), ctypes.POINTER(ctypes.c_double)),
                          ctypes.cast(ctypes.byref(T), ctypes.POINTER(ctypes.c_double)))
        return rho.value, u[:self.dim].copy(), E.value, T.value

    def collide_cell(self, g, h):
        g = np.array(g, dtype=np.float64)
        h = np.array(h, dtype=np.float64)
        _load().orc_collide_cell(ctypes.byref(self._m), _dp(g), _dp(h))
        return g, h

    # whole-grid operations -------------------------------------------------
    def init_fields(self, rho, u, T):
        n = self.ncells
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(n)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.dim, n)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(n)
        _load().orc_init(ctypes.byref(self._m), _dp(rho), _dp(u), _dp(T),
                         _dp(self.g), _dp(self.h))
        self.steps = 0

    def set_state(self, g, h):
        self.g = np.ascontiguousarray(g, dtype=np.float64).reshape(self.ncells, self.Q).copy()
        self.h = np.ascontiguousarray(h, dtype=np.float64).reshape(self.ncells, self.Q).copy()

    def step(self, n=1):
        if self.dt is None:
            rc = _load().orc_step(ctypes.byref(self._m), _dp(self.g), _dp(self.h),
                                  int(n))
        else:
            rc = _load().orc_fd_step(ctypes.byref(self._m), _dp(self.g), _dp(self.h),
                                     int(n), float(self.dt))
        if rc != 0:
            raise MemoryError("oracle step could not allocate")
        self.steps += n

    def moments(self):
        """(rho [cells], u [dim][cells], E [cells]) of the current state."""
        n = self.ncells
        rho, u, E = np.zeros(n), np.zeros((self.dim, n)), np.zeros(n)
        _load().orc_moments(ctypes.byref(self._m), _dp(self.g), _dp(self.h),
                            _dp(rho), _dp(u), _dp(E))
        return rho, u, E

    def temperature(self, u, E):
        """T from the specific total energy: E = u^2/2 + (D+delta) T/2."""
        return (2.0 * E - np.sum(u * u, axis=0)) / (self.dim + self.delta)

    def totals(self):
        mass = ctypes.c_double()
        energy = ctypes.c_double()
        mom = np.zeros(3)
        _load().orc_totals(ctypes.byref(self._m), _dp(self.g), _dp(self.h),
                           ctypes.cast(ctypes.byref(mass), ctypes.POINTER(ctypes.c_double)),
                           _dp(mom),
                           ctypes.cast(ctypes.byref(energy), ctypes.POINTER(ctypes.c_double)))
        return mass.value, mom[:self.dim].copy(), energy.value

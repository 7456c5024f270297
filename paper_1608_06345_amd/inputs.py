"""Seeded synthetic initial fields (rho, u, T) for the workloads.

This module holds no arithmetic of the lattice Boltzmann method: it only
produces macroscopic initial data, which both the HIP path and the oracle
consume.  Fields are FP64, cell-major with x fastest: ``rho[cells]``,
``u[dim][cells]``, ``T[cells]``, cell = x + nx (y + ny z).

Recipes
-------
smooth   rho = 1 + a_rho s_rho, u_c = a_u s_uc, T = 1 + a_T s_T, where each s
         is an independent sum of 8 Fourier modes
         s(x) = sum_m a_m cos(2 pi k_m . (x / N) + phi_m),
         a_m ~ U[-1, 1], k_m integer with 1 <= max_d |k_m,d| <= 8,
         phi_m ~ U[0, 2 pi).  Defaults a_rho = a_T = 0.01, a_u = 0.02.
sod      a two-state shock tube along x (left state for cells x < nx // 2),
         uniform across y and z; T = p / rho (dimensionless equation of
         state p = rho T).
"""
import math

import numpy as np


def _modes(rng, dim, nmodes, kmax):
    amp = rng.uniform(-1.0, 1.0, nmodes)
    phase = rng.uniform(0.0, 2.0 * math.pi, nmodes)
    ks = []
    while len(ks) < nmodes:
        k = rng.integers(-kmax, kmax + 1, dim)
        if np.max(np.abs(k)) >= 1:
            ks.append(k)
    return amp, np.array(ks), phase


def _mode_sum(shape, amp, ks, phase):
    """sum_m amp_m cos(2 pi k_m . x / N + phase_m) on a grid (x fastest)."""
    dim = ks.shape[1]
    nx, ny, nz = shape
    # separable evaluation: cos(a + b + c) through complex exponentials
    xs = [np.arange(n, dtype=np.float64) / n for n in (nx, ny, nz)[:dim]]
    out = np.zeros((nz, ny, nx) if dim == 3 else (ny, nx))
    for m in range(len(amp)):
        ex = np.exp(2j * math.pi * ks[m, 0] * xs[0])
        ey = np.exp(2j * math.pi * ks[m, 1] * xs[1])
        if dim == 3:
            ez = np.exp(2j * math.pi * ks[m, 2] * xs[2])
            z = ez[:, None, None] * ey[None, :, None] * ex[None, None, :]
        else:
            z = ey[:, None] * ex[None, :]
        out += amp[m] * np.real(z * np.exp(1j * phase[m]))
    return out.reshape(-1)


def smooth_fields(dim, nx, ny, nz=1, seed=0, a_rho=0.01, a_u=0.02, a_T=0.01,
                  nmodes=8, kmax=8):
    """Smooth low-mode perturbation of the rest state rho = T = 1, u = 0."""
    if dim == 2:
        nz = 1
    shape = (nx, ny, nz)
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(2 + dim)
    rngs = [np.random.default_rng(c) for c in children]
    s_rho = _mode_sum(shape, *_modes(rngs[0], dim, nmodes, kmax))
    s_T = _mode_sum(shape, *_modes(rngs[1], dim, nmodes, kmax))
    u = np.stack([_mode_sum(shape, *_modes(rngs[2 + c], dim, nmodes, kmax))
                  for c in range(dim)])
    return 1.0 + a_rho * s_rho, a_u * u, 1.0 + a_T * s_T


def sod_fields(dim, nx, ny, nz=1, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1),
               x_d=None):
    """Shock tube along x: ``left``/``right`` are (rho, u_x, p)."""
    if dim == 2:
        nz = 1
    if x_d is None:
        x_d = nx // 2
    n = nx * ny * nz
    x = np.arange(n) % nx
    is_left = x < x_d
    rho = np.where(is_left, left[0], right[0]).astype(np.float64)
    ux = np.where(is_left, left[1], right[1]).astype(np.float64)
    p = np.where(is_left, left[2], right[2]).astype(np.float64)
    u = np.zeros((dim, n))
    u[0] = ux
    return rho, u, p / rho


def uniform_fields(dim, nx, ny, nz=1, rho=1.0, u=(0.0, 0.0, 0.0), T=1.0):
    if dim == 2:
        nz = 1
    n = nx * ny * nz
    uu = np.zeros((dim, n))
    for c in range(dim):
        uu[c] = u[c]
    return np.full(n, float(rho)), uu, np.full(n, float(T))


def shear_wave_fields(dim, nx, ny, nz=1, seed=0, amp=0.05, background=0.25):
    """Long transverse (shear) and longitudinal waves along x with seeded
    phases, on top of the ``smooth`` recipe scaled by ``background``.  The
    waves span the whole x extent, so viscosity damps them slowly and the
    flow is still of useful size after thousands of steps; the background
    modes give every lattice direction work to do early on."""
    if dim == 2:
        nz = 1
    rho, u, T = smooth_fields(dim, nx, ny, nz, seed=seed, a_rho=0.01 * background,
                              a_u=0.02 * background, a_T=0.01 * background)
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(4)[3])
    ph = rng.uniform(0.0, 2.0 * math.pi, 4)
    x = (np.arange(nx * ny * nz) % nx) / nx
    u[1] += amp * np.sin(2 * math.pi * x + ph[0])
    if dim == 3:
        u[2] += 0.6 * amp * np.cos(2 * math.pi * x + ph[1])
    rho += 0.2 * amp * np.cos(2 * math.pi * x + ph[2])
    T += 0.2 * amp * np.cos(2 * math.pi * x + ph[3])
    return rho, u, T


def smooth_fields_device(dim, nx, ny, nz=1, seed=0, a_rho=0.01, a_u=0.02, a_T=0.01,
                         nmodes=8, kmax=8, device="cuda"):
    """The ``smooth`` recipe (same seeded draws as smooth_fields), evaluated
    with torch on ``device``: (rho, u, T) as contiguous float64 tensors."""
    import torch

    if dim == 2:
        nz = 1
    shape = (nx, ny, nz)
    ss = np.random.SeedSequence(seed)
    rngs = [np.random.default_rng(c) for c in ss.spawn(2 + dim)]
    axes = [torch.arange(n, dtype=torch.float64, device=device) / n for n in shape[:dim]]

    def mode_sum(amp, ks, phase):
        out = torch.zeros(tuple(reversed(shape[:dim])), dtype=torch.float64, device=device)
        for m in range(len(amp)):
            arg = None
            for d in range(dim):
                a = 2 * math.pi * float(ks[m, d]) * axes[d]
                view = [1] * dim
                view[dim - 1 - d] = -1
                a = a.reshape(view)
                arg = a if arg is None else arg + a
            out += float(amp[m]) * torch.cos(arg + float(phase[m]))
        return out.reshape(-1)

    s_rho = mode_sum(*_modes(rngs[0], dim, nmodes, kmax))
    s_T = mode_sum(*_modes(rngs[1], dim, nmodes, kmax))
    u = torch.stack([mode_sum(*_modes(rngs[2 + c], dim, nmodes, kmax)) for c in range(dim)])
    return ((1.0 + a_rho * s_rho).contiguous(), (a_u * u).contiguous(),
            (1.0 + a_T * s_T).contiguous())

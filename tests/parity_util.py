"""Shared helpers of the GPU parity tests: run the same seeded case through
the HIP library and through the oracle, and compare the macroscopic fields.

Error metrics (the bar is stated on rho, u and T):
  rho, T  max over cells of |gpu - oracle| / |oracle|  (pointwise relative)
  u       max |gpu - oracle| / max |oracle|  (u crosses zero, so a pointwise
          relative error is undefined there; this is the literal "relative
          error in u" over the field)
"""
import numpy as np

from paper_1608_06345_amd import lbm

TOL_FP64 = 1e-12
TOL_FP32 = 1e-5


def gpu_run(dim, gamma, tf, tg, shape, fields, steps, bc=0, precision=lbm.LBM_FP64,
            variant=lbm.LBM_VARIANT_AUTO, dt=None):
    """``dt`` selects the finite-difference form (lbm_create_fd)."""
    nx, ny, nz = shape
    with lbm.Solver(dim, gamma, tf, tg, nx, ny, nz, bc=bc, precision=precision, dt=dt) as s:
        s.set_variant(variant)
        s.init_fields(*fields)
        s.step(steps)
        rho, u, E = s.moments()
        T = s.temperature()
        tot = s.totals()
    return rho, u, T, tot


def oracle_run(dim, gamma, tf, tg, shape, fields, steps, open_end=(False, False, False),
               dt=None):
    from oracle.model import OracleLBM
    o = OracleLBM(dim, gamma, tf, tg, *shape, open_end=open_end, dt=dt)
    o.init_fields(*fields)
    o.step(steps)
    rho, u, E = o.moments()
    return rho, u, o.temperature(u, E), o.totals()


def open_of(bc):
    return tuple(((bc >> (2 * k)) & 3) == lbm.LBM_BC_ZERO_GRADIENT for k in range(3))


def errors(a, b):
    """(rho, u, T) errors of run a against run b (each: rho, u, T, ...)."""
    rho_a, u_a, T_a = a[:3]
    rho_b, u_b, T_b = b[:3]
    e_rho = float(np.max(np.abs(rho_a - rho_b) / np.abs(rho_b)))
    e_T = float(np.max(np.abs(T_a - T_b) / np.abs(T_b)))
    scale = float(np.max(np.abs(u_b)))
    e_u = float(np.max(np.abs(u_a - u_b))) / (scale if scale > 0 else 1.0)
    return e_rho, e_u, e_T


def assert_close(a, b, tol, what=""):
    e = errors(a, b)
    assert max(e) <= tol, f"{what}: rho/u/T errors {e} exceed {tol}"
    return e


def periodic_window(fields, shape, dim, center, half):
    """Initial fields on the (2 half + 1)^dim window around ``center`` of a
    periodic grid (wrapped), as flat arrays of the window grid."""
    rho, u, T = fields
    nx, ny, nz = shape
    idx = [np.arange(c - half, c + half + 1) % n for c, n in zip(center, (nx, ny, nz)[:dim])]
    if dim == 2:
        cell = idx[0][None, :] + nx * idx[1][:, None]
    else:
        cell = idx[0][None, None, :] + nx * (idx[1][None, :, None] + ny * idx[2][:, None, None])
    cell = cell.reshape(-1)
    return rho[cell], u[:, cell], T[cell]


def oracle_sample(dim, gamma, tf, tg, fields, shape, centers, steps, dt=None):
    """Oracle moments at sampled cells of a periodic grid after ``steps``
    steps, each from its own window: a cell's state after n steps depends
    only on the initial data within 3n cells (populations move at most 3
    cells per step; the finite-difference stencil reaches 2 cells), so a
    window of that half-width reproduces it exactly -- whatever happens at
    the window's own edges reaches at most that far inward in n steps."""
    half = (3 if dt is None else 2) * steps
    w = 2 * half + 1
    out = []
    for c in centers:
        f = periodic_window(fields, shape, dim, c, half)
        wshape = (w, w, w if dim == 3 else 1)
        rho, u, T, _ = oracle_run(dim, gamma, tf, tg, wshape, f, steps, dt=dt)
        mid = half + w * half + (w * w * half if dim == 3 else 0)
        out.append((rho[mid], u[:, mid], T[mid]))
    return out

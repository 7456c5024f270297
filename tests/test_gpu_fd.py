"""The finite-difference form (Sec. III, lbm_create_fd) on the GPU against
the FP64 oracle's finite-difference step, on identical seeded inputs.

Time steps are inside the scheme's stability region.  Forward Euler with
the upwind-biased difference alone amplifies every Fourier mode a little;
the BGK relaxation damps the departures from equilibrium and makes the
scheme stable for Courant numbers c = |xi_a| dt (per axis) up to about
0.6-0.7 on one axis, which for D2Q37's fastest population (3r, 3r) means
3 r dt <= 0.30-0.36 at dt / tau = 0.2-1.  The cases use 3 r dt = 0.25 (2D)
and 0.3 (3D) with dt / tau about 0.6-0.7.

Bars as for the lattice scheme: FP64 1e-12, FP32 deviation storage 1e-5 on
smooth fields after 1000 steps (u relative to its field maximum).  Half
storage is refused for this form (lbm_create_fd returns EINVAL)."""
import numpy as np
import pytest

from paper_1608_06345_amd import lbm
from paper_1608_06345_amd.inputs import shear_wave_fields, smooth_fields, sod_fields
from parity_util import (TOL_FP32, TOL_FP64, assert_close, gpu_run, open_of, oracle_run,
                         oracle_sample)
from shock_cases import FP32_BAR, FP64_BAR

pytestmark = pytest.mark.gpu

R = lbm.lbm_lattice(37)[2]
P64, P32 = lbm.LBM_FP64, lbm.LBM_FP32_DEV
AUTO, LANE, SPLIT = lbm.LBM_VARIANT_AUTO, lbm.LBM_VARIANT_LANE, lbm.LBM_VARIANT_SPLIT
TWO = lbm.LBM_VARIANT_TWO_PASS

CASE2D = dict(shape=(125, 111, 1), gamma=1.4, tf=0.1, tg=0.12, dt=0.25 / (3 * R))
CASE3D = dict(shape=(48, 13, 11), gamma=1.4, tf=0.12, tg=0.12, dt=0.3 / (3 * R))


def _args(c):
    return c["gamma"], c["tf"], c["tg"], c["shape"]


@pytest.fixture(scope="module")
def fd2d():
    c = CASE2D
    f = smooth_fields(2, *c["shape"], seed=2, kmax=1)
    return f, oracle_run(2, *_args(c), f, 1000, dt=c["dt"])


@pytest.fixture(scope="module")
def fd3d():
    c = CASE3D
    f = shear_wave_fields(3, *c["shape"], seed=3)
    return f, oracle_run(3, *_args(c), f, 1000, dt=c["dt"])


# TWO is the two-pass step (moments pass, then chunks of populations);
# LANE and SPLIT the fused kernel in either layout
@pytest.mark.parametrize("precision,variant,tol", [
    (P64, TWO, TOL_FP64), (P32, TWO, TOL_FP32), (P64, LANE, TOL_FP64), (P64, SPLIT, TOL_FP64),
    (P32, LANE, TOL_FP32), (P32, SPLIT, TOL_FP32)])
def test_fd_2d_smooth_1000_steps(fd2d, precision, variant, tol):
    c = CASE2D
    f, o = fd2d
    g = gpu_run(2, *_args(c), f, 1000, precision=precision, variant=variant, dt=c["dt"])
    e = assert_close(g, o, tol, "FD D2Q37")
    print(f"\nPARITY FD D2Q37 1000 steps precision={precision} variant={variant} rho/u/T={e} "
          f"max|u|={np.max(np.abs(o[1])):.3g}")


@pytest.mark.parametrize("precision,variant,tol", [
    (P64, TWO, TOL_FP64), (P32, TWO, TOL_FP32), (P64, SPLIT, TOL_FP64), (P32, SPLIT, TOL_FP32)])
def test_fd_3d_smooth_1000_steps(fd3d, precision, variant, tol):
    c = CASE3D
    f, o = fd3d
    g = gpu_run(3, *_args(c), f, 1000, precision=precision, variant=variant, dt=c["dt"])
    e = assert_close(g, o, tol, "FD D3Q107")
    print(f"\nPARITY FD D3Q107 1000 steps precision={precision} variant={variant} rho/u/T={e} "
          f"max|u|={np.max(np.abs(o[1])):.3g}")


@pytest.mark.parametrize("dim,shape,bc", [
    (2, (1, 1, 1), 0), (2, (2, 3, 1), 0), (2, (5, 1, 1), 0), (2, (4, 4, 1), lbm.LBM_BC(1, 1)),
    (2, (70, 20, 1), lbm.LBM_BC(1, 0)), (3, (1, 1, 1), 0), (3, (3, 2, 1), 0),
    (3, (7, 6, 5), lbm.LBM_BC(1, 1, 1)), (3, (9, 2, 4), lbm.LBM_BC(1, 0, 1)),
    (3, (40, 17, 19), lbm.LBM_BC(0, 1, 0))])
@pytest.mark.parametrize("precision,tol", [(P64, TOL_FP64), (P32, TOL_FP32)])
def test_fd_tiny_open_and_banded_grids(dim, shape, bc, precision, tol):
    # (70, 20) and (40, 17, 19): several waves per row, ragged last segment;
    # both the two-pass step and the fused kernel
    dt = 0.25 / (3 * R)
    f = smooth_fields(dim, *shape, seed=13, a_rho=0.05, a_u=0.05, a_T=0.05)
    o = oracle_run(dim, 1.4, 0.1, 0.12, shape, f, 30, open_end=open_of(bc), dt=dt)
    for variant in (TWO, LANE if dim == 2 else SPLIT):
        g = gpu_run(dim, 1.4, 0.1, 0.12, shape, f, 30, bc=bc, precision=precision, dt=dt,
                    variant=variant)
        assert_close(g, o, tol, f"FD {shape} bc={bc} variant={variant}")


@pytest.mark.parametrize("precision", [P64, P32])
def test_fd_sod_shock_tube(precision):
    """Sod 200x4 with open ends, dt = 0.25 / (3r), tau = 0.1 / r: parity
    with the oracle and L1 against the exact Riemann solution at t = 48 / r."""
    from oracle.riemann import l1_errors, shock_tube_profile
    shape = (200, 4, 1)
    bc = lbm.LBM_BC(lbm.LBM_BC_ZERO_GRADIENT, lbm.LBM_BC_PERIODIC)
    dt, tau = 0.25 / (3 * R), 0.1 / R
    steps = int(round((48.0 / R) / dt))
    f = sod_fields(2, *shape)
    o = oracle_run(2, 1.4, tau, tau, shape, f, steps, open_end=(True, False, False), dt=dt)
    g = gpu_run(2, 1.4, tau, tau, shape, f, steps, bc=bc, precision=precision, dt=dt)
    e = (np.max(np.abs(g[0] - o[0]) / o[0]), np.max(np.abs(g[1] - o[1])),
         np.max(np.abs(g[2] - o[2]) / o[2]))
    print(f"\nPARITY FD Sod 200x4 {steps} steps precision={precision} rho/u(abs)/T={e}")
    # the shock-tube bars of shock_cases.py (float-model evidence)
    assert max(e) < (FP64_BAR if precision == P64 else FP32_BAR)["fd_sod200"]
    ex = shock_tube_profile((1, 0, 1), (0.125, 0, 0.1), 1.4, 200, steps * dt * R, R)
    l1 = l1_errors(g[0][:200], g[1][0][:200], (g[0] * g[2])[:200], *ex)
    print(f"FD Sod L1 against the exact solution rho/u/p = {l1}")
    assert l1[0] < 0.015 and l1[1] < 0.03 and l1[2] < 0.015, l1


@pytest.mark.parametrize("dim,tf,tg", [(2, 0.1, 0.1), (3, 0.12, 0.12), (2, 0.1, 0.15)])
def test_fd_conservation_and_totals(dim, tf, tg):
    shape = (45, 38, 1) if dim == 2 else (21, 18, 17)
    dt = 0.25 / (3 * R)
    f = smooth_fields(dim, *shape, seed=8, a_rho=0.05, a_u=0.05, a_T=0.05)
    o = oracle_run(dim, 1.4, tf, tg, shape, f, 100, dt=dt)
    g = gpu_run(dim, 1.4, tf, tg, shape, f, 100, dt=dt)
    g0 = gpu_run(dim, 1.4, tf, tg, shape, f, 0, dt=dt)
    (mo, po, eo), (mg, pg, eg), (m0, p0, e0) = o[3], g[3], g0[3]
    assert mg == pytest.approx(mo, rel=1e-13)
    assert np.allclose(pg, po, rtol=0, atol=1e-11)
    assert eg == pytest.approx(eo, rel=1e-13)
    # periodic: mass and momentum are conserved (and energy when tf == tg)
    assert mg == pytest.approx(m0, rel=1e-13)
    assert np.allclose(pg, p0, rtol=0, atol=1e-10)
    if tf == tg:
        assert eg == pytest.approx(e0, rel=1e-13)


def test_fd_step_zero_and_determinism():
    shape = (40, 9, 1)
    dt = 0.25 / (3 * R)
    f = smooth_fields(2, *shape, seed=21)
    g0 = gpu_run(2, 1.4, 0.1, 0.1, shape, f, 0, dt=dt)
    assert np.max(np.abs(g0[0] - f[0])) < 1e-14 and np.max(np.abs(g0[2] - f[2])) < 1e-13
    a = gpu_run(2, 1.4, 0.1, 0.1, shape, f, 30, precision=P32, dt=dt)
    b = gpu_run(2, 1.4, 0.1, 0.1, shape, f, 30, precision=P32, dt=dt)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
    with lbm.Solver(2, 1.4, 0.1, 0.1, *shape, dt=dt) as s:
        assert s.info["scheme"] == 1 and s.info["dt"] == dt
    with lbm.Solver(2, 1.4, 0.7, 0.7, *shape) as s:  # two passes: finite differences only
        with pytest.raises(lbm.LBMError) as ei:
            s.set_variant(TWO)
        assert ei.value.code == lbm.LBM_EINVAL


@pytest.mark.parametrize("dim", [3, 2])
def test_fd_full_size_sampled_cells(dim):
    """The benchmark's full grids (D3Q107 256^3, D2Q37 4096^2) in the launch
    configuration bench.py times, FP32: sampled cells against oracle windows
    (half-width 2n: the stencil reaches two cells per step)."""
    if dim == 3:
        shape, tf, centers = (256, 256, 256), 0.12, [(0, 0, 0), (255, 255, 255), (128, 3, 250),
                                                   (7, 131, 64), (254, 0, 127)]
        dt = 0.3 / (3 * R)
    else:
        shape, tf, centers = (4096, 4096, 1), 0.1, [(0, 0), (4095, 4095), (2048, 5), (3, 2047),
                                                  (1234, 3210)]
        dt = 0.25 / (3 * R)
    steps = 4
    f = smooth_fields(dim, *shape, seed=3 if dim == 3 else 2)
    ref = oracle_sample(dim, 1.4, tf, tf, f, shape, centers, steps, dt=dt)
    nx, ny, nz = shape
    with lbm.Solver(dim, 1.4, tf, tf, nx, ny, nz, precision=P32, dt=dt) as s:
        s.init_fields(*f)
        s.step(steps)
        rho, u, E = s.moments()
        T = s.temperature()
    umax = max(np.max(np.abs(r[1])) for r in ref)
    worst = [0.0, 0.0, 0.0]
    for cen, (r_o, u_o, T_o) in zip(centers, ref):
        cell = cen[0] + nx * (cen[1] + (ny * cen[2] if dim == 3 else 0))
        worst[0] = max(worst[0], abs(rho[cell] - r_o) / r_o)
        worst[1] = max(worst[1], np.max(np.abs(u[:, cell] - u_o)) / umax)
        worst[2] = max(worst[2], abs(T[cell] - T_o) / T_o)
    print(f"\nPARITY FD full-size D{dim} FP32 sampled rho/u/T={worst}")
    assert max(worst) <= TOL_FP32, worst


def _tile_x(fields, shape, times):
    """Fields of a grid repeated ``times`` over x (flat arrays, x fastest)."""
    nx, ny, nz = shape
    rho, u, T = fields
    rep = lambda a: np.concatenate([a.reshape(nz, ny, nx)] * times, axis=-1).reshape(-1)
    return rep(rho), np.stack([rep(c) for c in u]), rep(T)


@pytest.mark.parametrize("dim,shape,bc", [
    (3, (128, 6, 5), lbm.LBM_BC(0, 1, 0)), (3, (128, 4, 7), lbm.LBM_BC(0, 0, 1)),
    (2, (128, 9, 1), lbm.LBM_BC(0, 1)), (2, (256, 5, 1), 0)])
@pytest.mark.parametrize("precision,tol", [(P64, TOL_FP64), (P32, TOL_FP32)])
def test_fd_lds_kernel_against_per_cell_kernel(dim, shape, bc, precision, tol):
    """Rows of whole 256-cell tiles take the LDS-staged update kernel, other
    widths the one-lane-per-cell kernel; both run FdCell's per-cell steps.
    Two periodic copies of a grid along x, run on the doubled grid (LDS
    kernel), must give each copy the original grid's state (per-cell kernel
    when its width is 128; 256 -> 512 compares the LDS kernel with itself
    across tile boundaries, bitwise).  Between the two kernels the compiler
    fuses multiply-adds differently (it contracts per basic block), so they
    agree to rounding: the parity bars, far below a wrong stencil value."""
    dt = 0.25 / (3 * R)
    f = smooth_fields(dim, *shape, seed=17, a_rho=0.05, a_u=0.05, a_T=0.05)
    wide = (2 * shape[0], shape[1], shape[2])
    a = gpu_run(dim, 1.4, 0.1, 0.12, shape, f, 25, bc=bc, precision=precision, dt=dt,
                variant=TWO)
    b = gpu_run(dim, 1.4, 0.1, 0.12, wide, _tile_x(f, shape, 2), 25, bc=bc,
                precision=precision, dt=dt, variant=TWO)
    nx, ny, nz = shape
    halves = []
    for k in range(2):
        halves.append([y.reshape(-1, nz, ny, 2 * nx)[..., k * nx:(k + 1) * nx].reshape(y.shape[:-1] + (-1,))
                       for y in b[:3]])
    for h in halves:
        e = assert_close(h, a, tol, f"LDS vs per-cell kernel {shape} bc={bc}")
    print(f"\nFD LDS vs per-cell {shape} bc={bc} precision={precision}: rho/u/T {e}")
    if shape[0] % 256 == 0:  # the same kernel on both grids
        for x, y in zip(a[:3], halves[0]):
            assert np.array_equal(x, y)
    for x, y in zip(halves[0], halves[1]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("dim,shape,bc", [
    (3, (256, 5, 3), lbm.LBM_BC(1, 0, 1)), (3, (256, 3, 4), lbm.LBM_BC(0, 1, 0)),
    (2, (512, 7, 1), lbm.LBM_BC(1, 0)), (2, (256, 2, 1), 0)])
@pytest.mark.parametrize("precision,tol", [(P64, TOL_FP64), (P32, TOL_FP32)])
def test_fd_lds_kernel_against_oracle(dim, shape, bc, precision, tol):
    """The LDS-staged update (rows of whole tiles) with open and periodic
    ends, and rows of two tiles whose halos come from the neighbour tile."""
    dt = 0.25 / (3 * R)
    f = smooth_fields(dim, *shape, seed=19, a_rho=0.05, a_u=0.05, a_T=0.05)
    o = oracle_run(dim, 1.4, 0.1, 0.12, shape, f, 20, open_end=open_of(bc), dt=dt)
    g = gpu_run(dim, 1.4, 0.1, 0.12, shape, f, 20, bc=bc, precision=precision, dt=dt,
                variant=TWO)
    e = assert_close(g, o, tol, f"FD LDS {shape} bc={bc}")
    print(f"\nPARITY FD LDS {shape} bc={bc} precision={precision} rho/u/T={e}")


_LDS_1000 = {}


@pytest.mark.parametrize("dim,shape", [(2, (256, 12, 1)), (3, (256, 6, 4))])
@pytest.mark.parametrize("precision,tol", [(P64, TOL_FP64), (P32, TOL_FP32)])
def test_fd_lds_kernel_1000_steps(dim, shape, precision, tol):
    """The LDS-staged update over 1000 steps, against the oracle."""
    c = CASE2D if dim == 2 else CASE3D
    if dim == 2:
        f = smooth_fields(2, *shape, seed=2, kmax=1)
    else:
        f = shear_wave_fields(3, *shape, seed=3)
    if dim not in _LDS_1000:  # one oracle run per grid
        _LDS_1000[dim] = oracle_run(dim, c["gamma"], c["tf"], c["tg"], shape, f, 1000,
                                    dt=c["dt"])
    o = _LDS_1000[dim]
    g = gpu_run(dim, c["gamma"], c["tf"], c["tg"], shape, f, 1000, precision=precision,
                variant=TWO, dt=c["dt"])
    e = assert_close(g, o, tol, f"FD LDS {shape} 1000 steps")
    print(f"\nPARITY FD LDS {shape} 1000 steps precision={precision} rho/u/T={e}")

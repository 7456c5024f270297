"""The D3Q107 lattice step with the pulled rows staged in LDS
(LBM_VARIANT_SPLIT_LDS) against the split kernel it restages and against
the FP64 oracle, on identical seeded inputs: periodic and open ends, rows of
one and two 128-cell tiles (the x halo from the neighbour tile or across the
domain end), FP64, FP32 deviation and half storage, and the full benchmark
grid on sampled cells."""
import numpy as np
import pytest

from paper_1608_06345_amd import lbm
from paper_1608_06345_amd.inputs import smooth_fields, sod_fields
from parity_util import (TOL_FP32, TOL_FP64, assert_close, gpu_run, open_of, oracle_run,
                         oracle_sample)

pytestmark = pytest.mark.gpu

P64, P32, P16 = lbm.LBM_FP64, lbm.LBM_FP32_DEV, lbm.LBM_FP16_SCALED
SPLIT, LDS = lbm.LBM_VARIANT_SPLIT, lbm.LBM_VARIANT_SPLIT_LDS


@pytest.mark.parametrize("shape,bc", [((128, 9, 5), 0), ((256, 4, 6), lbm.LBM_BC(1, 1, 0)),
                                      ((128, 3, 2), lbm.LBM_BC(0, 0, 1))])
@pytest.mark.parametrize("precision", [P64, P32, P16])
def test_lds_matches_split_kernel(shape, bc, precision):
    f = smooth_fields(3, *shape, seed=23, a_rho=0.05, a_u=0.05, a_T=0.05)
    a = gpu_run(3, 1.4, 0.65, 0.75, shape, f, 40, bc=bc, precision=precision, variant=SPLIT)
    b = gpu_run(3, 1.4, 0.65, 0.75, shape, f, 40, bc=bc, precision=precision, variant=LDS)
    same = all(np.array_equal(x, y) for x, y in zip(a[:3], b[:3]))
    tol = {P64: TOL_FP64, P32: TOL_FP32, P16: 1e-3}[precision]
    e = assert_close(b, a, tol, f"LDS vs split {shape} bc={bc}")
    print(f"\nSPLIT_LDS vs SPLIT {shape} bc={bc} precision={precision}: rho/u/T {e}, "
          f"bitwise {same}")


@pytest.mark.parametrize("shape,bc", [((256, 5, 3), lbm.LBM_BC(1, 0, 1)),
                                      ((128, 4, 4), 0)])
@pytest.mark.parametrize("precision,tol", [(P64, TOL_FP64), (P32, TOL_FP32)])
def test_lds_against_oracle(shape, bc, precision, tol):
    f = smooth_fields(3, *shape, seed=29, a_rho=0.05, a_u=0.05, a_T=0.05)
    o = oracle_run(3, 1.4, 0.65, 0.75, shape, f, 30, open_end=open_of(bc))
    g = gpu_run(3, 1.4, 0.65, 0.75, shape, f, 30, bc=bc, precision=precision, variant=LDS)
    e = assert_close(g, o, tol, f"SPLIT_LDS {shape} bc={bc}")
    print(f"\nPARITY SPLIT_LDS {shape} bc={bc} precision={precision} rho/u/T={e}")


def test_lds_shock_tube_open_ends():
    """Sod along x in a 256 x 4 x 4 box, open in x: the halo at the domain
    ends is the clamped end cell."""
    shape = (256, 4, 4)
    bc = lbm.LBM_BC(lbm.LBM_BC_ZERO_GRADIENT, lbm.LBM_BC_PERIODIC, lbm.LBM_BC_PERIODIC)
    f = sod_fields(3, *shape)
    o = oracle_run(3, 1.4, 0.6, 0.6, shape, f, 60, open_end=(True, False, False))
    g = gpu_run(3, 1.4, 0.6, 0.6, shape, f, 60, bc=bc, precision=P64, variant=LDS)
    e = (np.max(np.abs(g[0] - o[0]) / o[0]), np.max(np.abs(g[1] - o[1])),
         np.max(np.abs(g[2] - o[2]) / o[2]))
    print(f"\nPARITY SPLIT_LDS Sod 256x4x4 60 steps rho/u(abs)/T={e}")
    assert max(e) < TOL_FP64


@pytest.mark.parametrize("precision,tol", [(P32, TOL_FP32), (P16, 1e-3)])
def test_lds_full_size_sampled_cells(precision, tol):
    """D3Q107 256^3 (the benchmark grid and fields), 4 steps, sampled cells
    against oracle windows."""
    shape, steps = (256, 256, 256), 4
    centers = [(0, 0, 0), (255, 255, 255), (128, 3, 250), (127, 131, 64), (129, 100, 1)]
    f = smooth_fields(3, *shape, seed=3)
    ref = oracle_sample(3, 1.4, 0.65, 0.65, f, shape, centers, steps)
    nx, ny, nz = shape
    with lbm.Solver(3, 1.4, 0.65, 0.65, nx, ny, nz, precision=precision) as s:
        s.set_variant(LDS)
        s.init_fields(*f)
        s.step(steps)
        rho, u, E = s.moments()
        T = s.temperature()
    umax = max(np.max(np.abs(r[1])) for r in ref)
    worst = [0.0, 0.0, 0.0]
    for cen, (r_o, u_o, T_o) in zip(centers, ref):
        cell = cen[0] + nx * (cen[1] + ny * cen[2])
        worst[0] = max(worst[0], abs(rho[cell] - r_o) / r_o)
        worst[1] = max(worst[1], np.max(np.abs(u[:, cell] - u_o)) / umax)
        worst[2] = max(worst[2], abs(T[cell] - T_o) / T_o)
    print(f"\nPARITY SPLIT_LDS full-size precision={precision} sampled rho/u/T={worst}")
    assert max(worst) <= tol, worst


def test_lds_variant_refused_where_it_does_not_apply():
    for args, kw in [((2, 1.4, 0.7, 0.7, 128, 8, 1), {}), ((3, 1.4, 0.7, 0.7, 100, 4, 4), {}),
                     ((3, 1.4, 0.12, 0.12, 128, 4, 4), dict(dt=0.05))]:
        with lbm.Solver(*args, **kw) as s:
            with pytest.raises(lbm.LBMError) as ei:
                s.set_variant(LDS)
            assert ei.value.code == lbm.LBM_EINVAL

"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (AUTO kernel layout, whole-row XCD mapping): D3Q107 256^3 and D2Q37
4096^2, FP64, FP32 deviation storage and half-precision scaled storage, on
the benchmark's own seeded fields.

The oracle cannot step these grids, so it computes sampled cells one by one:
after n steps a cell depends only on the initial data within 3n cells, and
the oracle runs that periodic window (corners and edges included, where the
window wraps around the grid).  Over longer runs, properties that hold at any
size are checked: mass and momentum totals (and energy where tau_f = tau_g)
are conserved, and a repeated run is bitwise identical."""
import numpy as np
import pytest

from paper_1608_06345_amd import lbm
from paper_1608_06345_amd.inputs import smooth_fields
from parity_util import TOL_FP32, TOL_FP64, oracle_sample

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

CASES = {
    3: dict(shape=(256, 256, 256), gamma=1.4, tf=0.65, tg=0.65, seed=3),
    2: dict(shape=(4096, 4096, 1), gamma=1.4, tf=0.7, tg=0.8, seed=2),
}
# steps before the sampled comparison: 20 in 3D (each sampled cell's
# oracle window is 121^3 cells), 100 in 2D (601^2)
STEPS = {3: 20, 2: 100}


@pytest.fixture(scope="module", params=[3, 2])
def case(request):
    dim = request.param
    c = CASES[dim]
    f = smooth_fields(dim, *c["shape"], seed=c["seed"])
    nx, ny, nz = c["shape"]
    if dim == 3:
        centers = [(0, 0, 0), (255, 255, 255), (128, 3, 250), (7, 131, 64)]
    else:
        centers = [(0, 0), (4095, 4095), (2048, 5), (3, 2047), (1234, 3210), (4094, 1)]
    ref = oracle_sample(dim, c["gamma"], c["tf"], c["tg"], f, c["shape"], centers, STEPS[dim])
    return dim, c, f, centers, ref


# half storage rounds each scaled deviation to 11 bits: after tens of steps
# the moments carry ~1e-5 of it (the 1000-step bars are in test_gpu_fp16)
TOL_FP16_SHORT = 1e-3


@pytest.mark.parametrize("precision,tol", [(lbm.LBM_FP64, TOL_FP64),
                                           (lbm.LBM_FP32_DEV, TOL_FP32),
                                           (lbm.LBM_FP16_SCALED, TOL_FP16_SHORT)])
def test_full_size_sampled_cells(case, precision, tol):
    dim, c, f, centers, ref = case
    nx, ny, nz = c["shape"]
    with lbm.Solver(dim, c["gamma"], c["tf"], c["tg"], nx, ny, nz, precision=precision) as s:
        s.init_fields(*f)
        s.step(STEPS[dim])
        rho, u, E = s.moments()
        T = s.temperature()
        m0, p0, e0 = s.totals()
        s.step(96)
        m1, p1, e1 = s.totals()
    umax = max(np.max(np.abs(r[1])) for r in ref)
    worst = [0.0, 0.0, 0.0]
    for cen, (r_o, u_o, T_o) in zip(centers, ref):
        cell = cen[0] + nx * (cen[1] + (ny * cen[2] if dim == 3 else 0))
        worst[0] = max(worst[0], abs(rho[cell] - r_o) / r_o)
        worst[1] = max(worst[1], np.max(np.abs(u[:, cell] - u_o)) / umax)
        worst[2] = max(worst[2], abs(T[cell] - T_o) / T_o)
    print(f"\nPARITY full-size D{dim} {STEPS[dim]} steps precision={precision} "
          f"sampled rho/u/T={worst}")
    assert max(worst) <= tol, worst
    # conservation over 96 further steps (energy only where tau_f = tau_g)
    # (half storage rounds every stored value independently each step: the
    # totals random-walk, ~1e-9 of the mass over these steps)
    crel = {lbm.LBM_FP64: 1e-13, lbm.LBM_FP32_DEV: 1e-9, lbm.LBM_FP16_SCALED: 1e-7}[precision]
    assert abs(m1 - m0) <= crel * m0
    assert np.max(np.abs(p1 - p0)) <= crel * m0
    if c["tf"] == c["tg"]:
        assert abs(e1 - e0) <= crel * e0
    print(f"conservation D{dim} precision={precision}: dmass={m1 - m0:.3e} "
          f"dmom={np.max(np.abs(p1 - p0)):.3e} denergy={e1 - e0:.3e}")

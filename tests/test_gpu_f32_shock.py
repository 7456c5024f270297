"""Shock tubes in FP32 deviation storage and FP64 on the GPU, against the
oracle and against the float model of the same step (f32_model.py), with
the bars of shock_cases.py: each 3-4 times the largest difference that
correct evaluations of the step in the same floating-point type show
against the oracle on that case (the CPU test test_f32_model.py measures
them).  The GPU is one more such evaluation, with fused multiply-adds and
its own summation order; its difference to the oracle, and to one model
evaluation, must stay within the bar.
"""
import numpy as np
import pytest

from paper_1608_06345_amd import lbm
from paper_1608_06345_amd.inputs import sod_fields
from parity_util import oracle_run
from shock_cases import CASES, FP32_BAR, FP64_BAR

pytestmark = pytest.mark.gpu


def _metric(a, b, kind, nx):
    """a, b: (rho, u, T) on the first nx cells."""
    if kind == "pointwise":
        return max(float(np.max(np.abs(a[0] - b[0]) / b[0])),
                   float(np.max(np.abs(a[1] - b[1]))),
                   float(np.max(np.abs(a[2] - b[2]) / b[2])))
    return max(float(np.sum(np.abs(x - y)) / np.sum(np.abs(y)))
               for x, y in ((a[0], b[0]), (a[1], b[1]), (a[2], b[2])))


@pytest.fixture(scope="module")
def references():
    """Oracle and float32 model (pairwise order) per case, quasi-1D."""
    from f32_model import DevModel
    out = {}
    for name, (dim, gamma, tau, nx, left, right, steps, dt, kind) in CASES.items():
        f = sod_fields(dim, nx, 1, 1, left=left, right=right)
        o = oracle_run(dim, gamma, tau, tau, (nx, 1, 1), f, steps, open_end=(True, False, False),
                       dt=dt)
        m = DevModel(dim, gamma, tau, tau, nx, 1, 1, open_end=(True, False, False),
                     dtype=np.float32, dt=dt)
        m.init_fields(*f)
        m.step(steps)
        rm, um, Tm = m.moments()
        out[name] = ((o[0], o[1][0], o[2]), (rm, um[0], Tm))
    return out


def _gpu(name, precision, variant=lbm.LBM_VARIANT_AUTO):
    dim, gamma, tau, nx, left, right, steps, dt, kind = CASES[name]
    shape = (nx, 4, 1) if dim == 2 else (nx, 4, 4)
    bc = lbm.LBM_BC(lbm.LBM_BC_ZERO_GRADIENT, lbm.LBM_BC_PERIODIC, lbm.LBM_BC_PERIODIC)
    f = sod_fields(dim, *shape, left=left, right=right)
    with lbm.Solver(dim, gamma, tau, tau, *shape, bc=bc, precision=precision, dt=dt) as s:
        s.set_variant(variant)
        s.init_fields(*f)
        s.step(steps)
        rho, u, _ = s.moments()
        T = s.temperature()
    rows = rho.reshape(-1, nx)
    assert np.all(rows == rows[0])  # quasi-1D: every transverse row identical
    return rho[:nx], u[0][:nx], T[:nx]


VARIANTS = [(n, lbm.LBM_VARIANT_AUTO) for n in CASES] + [("fd_sod200", lbm.LBM_VARIANT_LANE)]


@pytest.mark.parametrize("name,variant", VARIANTS)
def test_fp32_shock_within_float32_family(references, name, variant):
    kind = CASES[name][8]
    nx = CASES[name][3]
    ref, model = references[name]
    g = _gpu(name, lbm.LBM_FP32_DEV, variant)
    e_oracle = _metric(g, ref, kind, nx)
    e_model = _metric(g, model, kind, nx)
    e_model_oracle = _metric(model, ref, kind, nx)
    print(f"\nFP32 {name} variant={variant} ({kind}): GPU-oracle {e_oracle:.2e}, "
          f"GPU-model {e_model:.2e}, model-oracle {e_model_oracle:.2e}, bar {FP32_BAR[name]:.1e}")
    assert e_oracle <= FP32_BAR[name]
    assert e_model <= FP32_BAR[name]


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_shock_within_float64_family(references, name):
    kind = CASES[name][8]
    nx = CASES[name][3]
    ref, _ = references[name]
    g = _gpu(name, lbm.LBM_FP64)
    e = _metric(g, ref, kind, nx)
    print(f"\nFP64 {name} ({kind}): GPU-oracle {e:.2e}, bar {FP64_BAR[name]:.1e}")
    assert e <= FP64_BAR[name]

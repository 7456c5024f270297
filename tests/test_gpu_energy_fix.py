"""The energy-conserving collision mode (lbm_set_collision; beyond the
paper) on the GPU against the oracle's mode of the same name.

  * parity with the FP64 oracle for tau_f != tau_g: lattice scheme in 2D and
    3D (FP64 1e-12, FP32 deviation storage 1e-5) and the finite-difference
    form;
  * total energy is conserved to round-off with tau_f != tau_g, where the
    paper's collision drifts;
  * at tau_f = tau_g the mode is the paper's collision bit for bit;
  * the mode must be chosen before a state exists."""
import numpy as np
import pytest

from paper_1608_06345_amd import lbm
from paper_1608_06345_amd.inputs import shear_wave_fields, smooth_fields
from parity_util import TOL_FP32, TOL_FP64, assert_close

pytestmark = pytest.mark.gpu

EC = lbm.LBM_COLLISION_ENERGY_CONSERVING
R = lbm.lbm_lattice(37)[2]


def _gpu(dim, gamma, tf, tg, shape, f, steps, precision, collision, dt=None):
    with lbm.Solver(dim, gamma, tf, tg, *shape, precision=precision, dt=dt,
                    collision=collision) as s:
        assert s.info["collision"] == collision
        s.init_fields(*f)
        t0 = s.totals()
        s.step(steps)
        rho, u, E = s.moments()
        return rho, u, s.temperature(), t0, s.totals()


def _oracle(dim, gamma, tf, tg, shape, f, steps, dt=None):
    from oracle.model import OracleLBM
    o = OracleLBM(dim, gamma, tf, tg, *shape, dt=dt, energy_fix=True)
    o.init_fields(*f)
    o.step(steps)
    rho, u, E = o.moments()
    return rho, u, o.temperature(u, E)


@pytest.mark.parametrize("dim,gamma,tf,tg", [(2, 1.4, 0.7, 0.9), (3, 1.4, 0.9, 0.6),
                                             (2, 2.0, 0.6, 1.1)])
@pytest.mark.parametrize("precision,tol", [(lbm.LBM_FP64, TOL_FP64), (lbm.LBM_FP32_DEV, TOL_FP32)])
def test_energy_fix_parity_lattice(dim, gamma, tf, tg, precision, tol):
    # 150 steps, as for the paper collision's two-tau cases: on these small
    # grids the flow decays, and u is measured against its field maximum
    shape = (37, 29, 1) if dim == 2 else (24, 7, 5)
    f = shear_wave_fields(dim, *shape, seed=11)
    o = _oracle(dim, gamma, tf, tg, shape, f, 150)
    g = _gpu(dim, gamma, tf, tg, shape, f, 150, precision, EC)
    e = assert_close(g[:3], o, tol, f"energy fix D{dim}")
    print(f"\nPARITY energy-conserving D{dim} gamma={gamma} tau={tf}/{tg} precision={precision} "
          f"rho/u/T={e} max|u|={np.max(np.abs(o[1])):.3g}")


def test_energy_fix_parity_finite_difference():
    shape = (45, 38, 1)
    dt = 0.25 / (3 * R)
    f = smooth_fields(2, *shape, seed=8, a_rho=0.05, a_u=0.05, a_T=0.05)
    o = _oracle(2, 1.4, 0.1, 0.15, shape, f, 300, dt=dt)
    g = _gpu(2, 1.4, 0.1, 0.15, shape, f, 300, lbm.LBM_FP64, EC, dt=dt)
    e = assert_close(g[:3], o, TOL_FP64, "energy fix FD")
    print(f"\nPARITY energy-conserving FD D2 rho/u/T={e}")


@pytest.mark.parametrize("dim,shape,steps", [(2, (256, 6, 1), 300), (2, (45, 38, 1), 300),
                                              (3, (256, 4, 3), 100)])
@pytest.mark.parametrize("precision,tol", [(lbm.LBM_FP64, TOL_FP64), (lbm.LBM_FP32_DEV, TOL_FP32)])
def test_energy_fix_parity_finite_difference_two_pass(dim, shape, steps, precision, tol):
    """The two-pass finite-difference step with the energy-conserving
    collision (kappa rho in the record): the LDS-staged update kernel (rows of
    whole 256-cell tiles) and the one-lane kernel (45 wide)."""
    dt = (0.25 if dim == 2 else 0.3) / (3 * R)
    tf, tg = (0.1, 0.15) if dim == 2 else (0.12, 0.16)
    f = smooth_fields(dim, *shape, seed=8, a_rho=0.05, a_u=0.05, a_T=0.05)
    o = _oracle(dim, 1.4, tf, tg, shape, f, steps, dt=dt)
    with lbm.Solver(dim, 1.4, tf, tg, *shape, precision=precision, dt=dt, collision=EC) as s:
        s.set_variant(lbm.LBM_VARIANT_TWO_PASS)
        s.init_fields(*f)
        s.step(steps)
        rho, u, E = s.moments()
        g = (rho, u, s.temperature())
    e = assert_close(g, o, tol, f"energy fix FD two-pass {shape}")
    print(f"\nPARITY energy-conserving FD two-pass D{dim} {shape} precision={precision} rho/u/T={e}")


@pytest.mark.parametrize("dim,dt", [(2, None), (3, None), (2, 0.25 / (3 * R))])
def test_energy_fix_conserves_total_energy(dim, dt):
    shape = (45, 38, 1) if dim == 2 else (21, 18, 17)
    tf, tg = (0.7, 0.95) if dt is None else (0.1, 0.15)
    f = smooth_fields(dim, *shape, seed=8, a_rho=0.05, a_u=0.05, a_T=0.05)
    # FP32: each population's float update rounds independently, so the
    # totals random-walk at ~1e-9 per 100 steps on these strongly perturbed
    # fields (amplitude 0.05 per mode); the paper's collision drifts ~1e-4
    for precision, rel in ((lbm.LBM_FP64, 1e-13), (lbm.LBM_FP32_DEV, 1e-7)):
        *_, (m0, p0, e0), (m1, p1, e1) = _gpu(dim, 1.4, tf, tg, shape, f, 200, precision, EC,
                                              dt=dt)
        *_, (_, _, q0), (_, _, q1) = _gpu(dim, 1.4, tf, tg, shape, f, 200, precision,
                                          lbm.LBM_COLLISION_PAPER, dt=dt)
        print(f"\nD{dim} dt={dt} precision={precision}: energy drift fixed {(e1 - e0) / e0:.2e}, "
              f"paper {(q1 - q0) / q0:.2e}")
        assert abs(e1 - e0) <= rel * e0
        assert abs(m1 - m0) <= rel * m0
        assert abs(q1 - q0) > 100 * rel * q0


def test_energy_fix_equals_paper_at_equal_tau():
    shape = (33, 20, 1)
    f = smooth_fields(2, *shape, seed=3)
    for precision in (lbm.LBM_FP64, lbm.LBM_FP32_DEV):
        a = _gpu(2, 1.4, 0.8, 0.8, shape, f, 50, precision, EC)
        b = _gpu(2, 1.4, 0.8, 0.8, shape, f, 50, precision, lbm.LBM_COLLISION_PAPER)
        for x, y in zip(a[:3], b[:3]):
            assert np.array_equal(x, y)


def test_collision_mode_errors():
    with lbm.Solver(2, 1.4, 0.7, 0.8, 8, 8) as s:
        with pytest.raises(lbm.LBMError) as ei:
            lbm.lbm_set_collision(s.h, 5)
        assert ei.value.code == lbm.LBM_EINVAL
        lbm.lbm_set_collision(s.h, EC)
        s.init_fields(*smooth_fields(2, 8, 8, seed=1))
        with pytest.raises(lbm.LBMError) as ei:
            lbm.lbm_set_collision(s.h, lbm.LBM_COLLISION_PAPER)
        assert ei.value.code == lbm.LBM_ESTATE

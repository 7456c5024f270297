"""Pins of total energy under two relaxation times, and of the oracle's
energy-conserving collision mode (beyond the paper; a separate mode).

With rates a_f, a_g (1/tau per lattice step, dt/tau per finite-difference
step) the paper's BGK step moves sum xi^2 g / 2 toward rho (u^2 + D T) / 2
at rate a_f and sum h toward the complement at rate a_g, so a cell's total
energy changes by exactly (a_f - a_g) (E_tr^eq - E_tr).  That closed form
is computed here from the populations with numpy, independently of the
oracle's code.  The fixed mode must instead conserve energy cell by cell,
keep mass and momentum, and reduce to the paper's collision bit for bit
when tau_f = tau_g."""
import numpy as np
import pytest

from oracle.model import OracleLBM
from paper_1608_06345_amd.inputs import smooth_fields


def _perturbed_cell(o, seed):
    """A non-equilibrium cell: the equilibrium of some state, perturbed."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-0.1, 0.1, o.dim)
    F = o.feq(1.1, u, 0.95)
    g = F * (1 + 0.05 * rng.uniform(-1, 1, o.Q))
    h = 0.5 * o.delta * 0.9 * F * (1 + 0.05 * rng.uniform(-1, 1, o.Q))
    return g, h


def _energies(o, g, h):
    xi = o.lat.r * o.lat.e.astype(np.float64)
    q = np.sum(xi * xi, axis=1)
    rho = g.sum()
    u = (g @ xi) / rho
    e_tr = 0.5 * np.dot(q, g)
    e_tot = e_tr + h.sum()
    T = (2 * e_tot / rho - u @ u) / (o.dim + o.delta)
    e_tr_eq = 0.5 * rho * (u @ u + o.dim * T)
    return rho, rho * u, e_tot, e_tr, e_tr_eq


@pytest.mark.parametrize("dim,tf,tg", [(2, 0.7, 0.8), (3, 0.9, 0.6), (2, 1.3, 0.55)])
def test_paper_collision_energy_change_is_the_closed_form(dim, tf, tg):
    o = OracleLBM(dim, 1.4, tf, tg, 1, 1, 1)
    for seed in range(5):
        g, h = _perturbed_cell(o, seed)
        rho, j, e0, e_tr, e_tr_eq = _energies(o, g, h)
        g2, h2 = o.collide_cell(g, h)
        _, j2, e1, _, _ = _energies(o, g2, h2)
        want = (1 / tf - 1 / tg) * (e_tr_eq - e_tr)
        assert abs(want) > 1e-6  # a real change, not round-off
        assert (e1 - e0) == pytest.approx(want, rel=1e-9, abs=1e-15)
        assert g2.sum() == pytest.approx(rho, rel=1e-14)
        assert np.allclose(j2, j, rtol=0, atol=1e-15)


@pytest.mark.parametrize("dim,tf,tg", [(2, 0.7, 0.8), (3, 0.9, 0.6), (2, 1.3, 0.55)])
def test_energy_fix_conserves_energy_per_cell(dim, tf, tg):
    o = OracleLBM(dim, 1.4, tf, tg, 1, 1, 1, energy_fix=True)
    for seed in range(5):
        g, h = _perturbed_cell(o, seed)
        rho, j, e0, _, _ = _energies(o, g, h)
        g2, h2 = o.collide_cell(g, h)
        rho2, j2, e1, _, _ = _energies(o, g2, h2)
        assert e1 == pytest.approx(e0, rel=1e-14)
        assert rho2 == pytest.approx(rho, rel=1e-14)
        assert np.allclose(j2, j, rtol=0, atol=1e-15)
        # g relaxes exactly as in the paper's collision; only h's target moves
        p = OracleLBM(dim, 1.4, tf, tg, 1, 1, 1)
        g3, h3 = p.collide_cell(g, h)
        assert np.array_equal(g2, g3)
        assert not np.allclose(h2, h3, rtol=0, atol=1e-14)


@pytest.mark.parametrize("dt", [None, 0.07])
def test_energy_fix_equals_paper_at_equal_tau(dt):
    shape = (17, 11, 1)
    f = smooth_fields(2, *shape, seed=5, a_rho=0.05, a_u=0.05, a_T=0.05)
    tau = 0.7 if dt is None else 0.1
    a = OracleLBM(2, 1.4, tau, tau, *shape, dt=dt)
    b = OracleLBM(2, 1.4, tau, tau, *shape, dt=dt, energy_fix=True)
    a.init_fields(*f)
    b.init_fields(*f)
    a.step(30)
    b.step(30)
    assert np.array_equal(a.g, b.g) and np.array_equal(a.h, b.h)


@pytest.mark.parametrize("dim,dt", [(2, None), (3, None), (2, 0.07)])
def test_energy_fix_conserves_total_energy_over_a_run(dim, dt):
    shape = (23, 19, 1) if dim == 2 else (11, 9, 8)
    f = smooth_fields(dim, *shape, seed=6, a_rho=0.05, a_u=0.05, a_T=0.05)
    tf, tg = (0.7, 0.95) if dt is None else (0.1, 0.15)
    fixed = OracleLBM(dim, 1.4, tf, tg, *shape, dt=dt, energy_fix=True)
    paper = OracleLBM(dim, 1.4, tf, tg, *shape, dt=dt)
    for o in (fixed, paper):
        o.init_fields(*f)
    m0, p0, e0 = fixed.totals()
    fixed.step(150)
    paper.step(150)
    m1, p1, e1 = fixed.totals()
    _, _, e_paper = paper.totals()
    assert e1 == pytest.approx(e0, rel=1e-13)
    assert m1 == pytest.approx(m0, rel=1e-13)
    assert np.allclose(p1, p0, rtol=0, atol=1e-11)
    assert abs(e_paper - e0) > 1e-7 * e0  # the paper's collision drifts here

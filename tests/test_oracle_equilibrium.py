"""Pins of the oracle's equilibrium and collision (Secs. II-IV).

The fourth-order equilibrium must reproduce every velocity moment of the
reduced Maxwellian rho (2 pi theta)^(-D/2) exp(-|xi-u|^2 / 2 theta) up to
degree 4 (that is what "fourth-order accuracy" of Sec. IV means with a
degree-9 quadrature).  The reference moments here come from a product
Gauss-Hermite rule of numpy applied to the shifted, scaled Gaussian itself,
so they share nothing with the Hermite formula under test.  A dropped term,
a wrong sign or an exchanged xi/u in any of the k = 0..4 contractions breaks
at least one of these moments.

Collision pins: exact conservation of mass and momentum, of total energy
when tau_f = tau_g, and the closed-form energy change when they differ
(from the energy split of Sec. II); a uniform equilibrium is a fixed point.
"""
import itertools
import math

import numpy as np
import pytest

from oracle.model import OracleLBM


def _maxwellian_moment(rho, u, theta, alpha):
    x, w = np.polynomial.hermite_e.hermegauss(12)
    w = w / math.sqrt(2 * math.pi)
    out = rho
    for k, a in enumerate(alpha):
        out *= np.sum(w * (u[k] + math.sqrt(theta) * x) ** a)
    return out


def _states(dim, n, seed):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        rho = rng.uniform(0.5, 2.0)
        u = rng.uniform(-0.3, 0.3, dim)
        theta = rng.uniform(0.8, 1.25)
        yield rho, u, theta


@pytest.mark.parametrize("dim", [2, 3])
def test_equilibrium_moments_to_degree_four(dim):
    o = OracleLBM(dim, 1.4, 0.8, 0.8, 1, 1, 1)
    xi = o.lat.xi
    for rho, u, theta in _states(dim, 6, 11 + dim):
        F = o.feq(rho, u, theta)
        for alpha in itertools.product(range(5), repeat=dim):
            if sum(alpha) > 4:
                continue
            disc = np.sum(F * np.prod(xi ** np.array(alpha), axis=1))
            ref = _maxwellian_moment(rho, u, theta, alpha)
            assert abs(disc - ref) <= 1e-13 * max(1.0, abs(ref)), (alpha, disc, ref)


@pytest.mark.parametrize("dim", [2, 3])
def test_equilibrium_is_fourth_order_only(dim):
    # moments of degree 5 carry the truncation error O(u^5): they must not
    # match for a moving state (otherwise the test above would be vacuous
    # about the expansion order)
    o = OracleLBM(dim, 1.4, 0.8, 0.8, 1, 1, 1)
    rho, u, theta = 1.0, np.full(dim, 0.3), 1.1
    F = o.feq(rho, u, theta)
    alpha = (5,) + (0,) * (dim - 1)
    disc = np.sum(F * o.lat.xi[:, 0] ** 5)
    ref = _maxwellian_moment(rho, u, theta, alpha)
    assert abs(disc - ref) > 1e-4


def _printed_feq(o, rho, u, theta):
    """The k = 2..4 contractions exactly as typeset in Sec. IV."""
    D = o.dim
    U = float(np.dot(u, u))
    F = np.zeros(o.Q)
    for i in range(o.Q):
        xi = o.lat.xi[i]
        c = float(np.dot(xi, u))
        q = float(np.dot(xi, xi))
        t = theta - 1
        h2 = c * c + t * (theta ** 2 - D) - U
        h3 = c * (c * c - 3 * U + 3 * t * (U - D - 2))
        h4 = (c ** 4 - 6 * c * c * U + 3 * U * U
              + 6 * t * (c * c * (U - D - 4) + (D + 2 - U) * q)
              + 3 * t * t * (U * U - 2 * (D + 2) * U + D * (D + 2)))
        F[i] = o.lat.w[i] * rho * (1 + c + h2 / 2 + h3 / 6 + h4 / 24)
    return F


def test_printed_equilibrium_breaks_the_moments():
    # documents the reading of the garbled k=2..4 lines: taken literally they
    # do not reproduce even the energy moment
    o = OracleLBM(2, 1.4, 0.8, 0.8, 1, 1, 1)
    rho, u, theta = 1.0, np.array([0.1, -0.05]), 1.1
    F = _printed_feq(o, rho, u, theta)
    e2 = np.sum(F * np.sum(o.lat.xi ** 2, axis=1))
    ref = rho * (np.dot(u, u) + 2 * theta)
    assert abs(e2 - ref) > 1e-3


def _perturbed(o, rho, u, theta, rng, eps=0.02):
    F = o.feq(rho, u, theta)
    g = F * (1 + eps * rng.standard_normal(o.Q))
    h = 0.5 * o.delta * theta * F * (1 + eps * rng.standard_normal(o.Q))
    return g, h


@pytest.mark.parametrize("dim", [2, 3])
def test_collision_conserves_mass_momentum_energy(dim):
    rng = np.random.default_rng(5)
    o = OracleLBM(dim, 1.4, 0.65, 0.65, 1, 1, 1)
    xi = o.lat.xi
    q = 0.5 * np.sum(xi ** 2, axis=1)
    for rho, u, theta in _states(dim, 5, 3):
        g, h = _perturbed(o, rho, u, theta, rng)
        g2, h2 = o.collide_cell(g, h)
        assert np.sum(g2) == pytest.approx(np.sum(g), rel=1e-14)
        assert np.allclose(xi.T @ g2, xi.T @ g, rtol=0, atol=1e-14)
        e1 = np.sum(q * g) + np.sum(h)
        e2 = np.sum(q * g2) + np.sum(h2)
        assert e2 == pytest.approx(e1, rel=1e-14)
        assert not np.allclose(g2, g)


@pytest.mark.parametrize("dim", [2, 3])
def test_two_tau_energy_change_closed_form(dim):
    # With tau_f != tau_g only the sum is not conserved: from the energy
    # split (translational part sum xi^2 g / 2, internal part sum h) and the
    # equilibrium moments, one collision changes rho E by
    # (1/tau_f - 1/tau_g) (E_tr_eq - E_tr),  E_tr_eq = rho (u^2 + D T) / 2.
    rng = np.random.default_rng(9)
    tf, tg = 0.7, 0.8
    o = OracleLBM(dim, 1.4, tf, tg, 1, 1, 1)
    q = 0.5 * np.sum(o.lat.xi ** 2, axis=1)
    for rho, u, theta in _states(dim, 5, 4):
        g, h = _perturbed(o, rho, u, theta, rng)
        r_, uu, E, T = o.macro(g, h)
        e_tr = np.sum(q * g)
        e_tr_eq = 0.5 * r_ * (np.dot(uu, uu) + dim * T)
        g2, h2 = o.collide_cell(g, h)
        d_e = (np.sum(q * g2) + np.sum(h2)) - (np.sum(q * g) + np.sum(h))
        pred = (1 / tf - 1 / tg) * (e_tr_eq - e_tr)
        assert abs(d_e - pred) < 1e-13 * max(1.0, abs(r_ * E))
        assert abs(pred) > 1e-8


@pytest.mark.parametrize("dim,gamma", [(2, 1.4), (3, 1.4), (3, 5.0 / 3.0)])
def test_equilibrium_fixed_point_and_energy(dim, gamma):
    o = OracleLBM(dim, gamma, 0.6, 0.9, 1, 1, 1)
    for rho, u, theta in _states(dim, 4, 21):
        F = o.feq(rho, u, theta)
        H = 0.5 * o.delta * theta * F
        r_, uu, E, T = o.macro(F, H)
        assert r_ == pytest.approx(rho, rel=1e-14)
        assert np.allclose(uu, u, rtol=0, atol=1e-14)
        assert T == pytest.approx(theta, rel=1e-13)
        # dimensionless specific energy (Sec. II): E = u^2/2 + (D+delta) T/2
        assert E == pytest.approx(0.5 * np.dot(u, u) + 0.5 * (dim + o.delta) * theta,
                                  rel=1e-13)
        g2, h2 = o.collide_cell(F, H)
        assert np.max(np.abs(g2 - F)) < 1e-15
        assert np.max(np.abs(h2 - H)) < 1e-15

"""Pins of the oracle's exact Riemann solver (the analytical shock-tube
solution the paper compares with, Sec. V).

Independent of the solver's iteration: the Rankine-Hugoniot conditions
across the shock, constant entropy and Riemann invariant through the
rarefaction fan, continuity of pressure and velocity at the contact, the
textbook star values of Sod's problem (golden file), and mirror symmetry.
"""
import math
import os

import numpy as np
import pytest

from oracle.riemann import RiemannSolution

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CASES = [((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4),
         ((4.0, 0.0, 4.0), (1.0, 0.0, 1.0), 1.4),
         ((2.0, 0.1, 5.0), (1.0, -0.2, 0.4), 1.25),
         ((1.0, 0.0, 10.0), (1.0, 0.0, 1.0), 5.0 / 3.0)]


def _energy(rho, u, p, g):
    return p / (g - 1) + 0.5 * rho * u * u


def test_sod_star_values():
    line = [l for l in open(os.path.join(GOLDEN, "sod_exact_star.txt"))
            if not l.startswith("#")][0].split()
    p, u, rl, rr = map(float, line)
    s = RiemannSolution((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4)
    assert s.p_star == pytest.approx(p, abs=6e-6)
    assert s.u_star == pytest.approx(u, abs=6e-6)
    assert s.rho_star_l == pytest.approx(rl, abs=6e-6)
    assert s.rho_star_r == pytest.approx(rr, abs=6e-6)


@pytest.mark.parametrize("left,right,gamma", CASES)
def test_shock_jump_conditions(left, right, gamma):
    s = RiemannSolution(left, right, gamma)
    ws = s.wave_speeds()
    assert "right_shock" in ws
    S = ws["right_shock"]
    r1, u1, p1 = s.sample(np.array([S + 1e-9]))
    r2, u2, p2 = s.sample(np.array([S - 1e-9]))
    r1, u1, p1, r2, u2, p2 = map(float, (r1[0], u1[0], p1[0], r2[0], u2[0], p2[0]))
    m1, m2 = r1 * (u1 - S), r2 * (u2 - S)
    assert m1 == pytest.approx(m2, rel=1e-10)
    assert r1 * (u1 - S) ** 2 + p1 == pytest.approx(r2 * (u2 - S) ** 2 + p2, rel=1e-10)
    f1 = (_energy(r1, u1, p1, gamma) + p1) * u1 - S * _energy(r1, u1, p1, gamma)
    f2 = (_energy(r2, u2, p2, gamma) + p2) * u2 - S * _energy(r2, u2, p2, gamma)
    assert f1 == pytest.approx(f2, rel=1e-10, abs=1e-12)


@pytest.mark.parametrize("left,right,gamma", CASES)
def test_rarefaction_invariants(left, right, gamma):
    s = RiemannSolution(left, right, gamma)
    ws = s.wave_speeds()
    assert "left_head" in ws
    S = np.linspace(ws["left_head"] - 0.1, ws["left_tail"] + 0.05, 40)
    rho, u, p = s.sample(S)
    entropy = p / rho ** gamma
    assert np.max(np.abs(entropy / entropy[0] - 1)) < 1e-12
    a = np.sqrt(gamma * p / rho)
    inv = u + 2 * a / (gamma - 1)
    assert np.max(np.abs(inv - inv[0])) < 1e-12
    inside = (S > ws["left_head"]) & (S < ws["left_tail"])
    assert np.allclose((u - a)[inside], S[inside], atol=1e-12)  # fan: S = u - a


@pytest.mark.parametrize("left,right,gamma", CASES)
def test_contact(left, right, gamma):
    s = RiemannSolution(left, right, gamma)
    c = s.wave_speeds()["contact"]
    rho, u, p = s.sample(np.array([c - 1e-9, c + 1e-9]))
    assert p[0] == pytest.approx(p[1], rel=1e-12)
    assert u[0] == pytest.approx(u[1], rel=1e-12)


def test_mirror_symmetry():
    a = RiemannSolution((1.0, 0.3, 1.0), (1.0, -0.3, 1.0), 1.4)
    assert abs(a.u_star) < 1e-14
    b = RiemannSolution((0.7, 0.0, 2.0), (1.3, 0.0, 0.5), 1.3)
    c = RiemannSolution((1.3, 0.0, 0.5), (0.7, 0.0, 2.0), 1.3)
    assert b.p_star == pytest.approx(c.p_star, rel=1e-13)
    assert b.u_star == pytest.approx(-c.u_star, rel=1e-13)

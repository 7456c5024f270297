"""Pins of the oracle's lattice generator (Sec. IV, Tables I and II).

What pins it, independent of the generator's own equations:
  * the paper's printed weights and scale (golden files) to their 9 digits;
  * the Gaussian moments of every monomial up to degree 9, taken from
    numpy's Gauss-Hermite rule (a library routine, not the generator's
    double-factorial formula), and the failure at degree 10 that marks the
    quadrature's exact degree;
  * the worked time conversion of Sec. V;
  * gamma <-> delta from the definition in Sec. II and the examples of Sec. V.
"""
import itertools
import math
import os

import numpy as np
import pytest

from oracle.lattice import delta_from_gamma, group_members, lattice

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_table(name, dim):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        rows.append((tuple(int(v) for v in f[:dim]), int(f[dim]), float(f[dim + 1])))
    return rows


def _gauss_moment_1d(a):
    # E[z^a], z ~ N(0,1), from numpy's probabilists' Gauss-Hermite rule
    x, w = np.polynomial.hermite_e.hermegauss(30)
    return float(np.sum(w * x ** a) / math.sqrt(2 * math.pi))


@pytest.mark.parametrize("dim,name,Q", [(2, "table1_d2q37.txt", 37),
                                        (3, "table2_d3q107.txt", 107)])
def test_printed_tables(dim, name, Q):
    lat = lattice(dim)
    assert lat.Q == Q
    rows = _read_table(name, dim)
    assert sum(k for _, k, _ in rows) == Q
    for rep, k, w_printed in rows:
        members = group_members(rep)
        assert len(members) == k
        idx = [i for i in range(lat.Q) if tuple(lat.e[i]) in members]
        assert len(idx) == k
        w = lat.w[idx]
        assert np.all(w == w[0])
        # 9 printed digits: agreement to a few units in the last digit
        assert abs(w[0] - w_printed) <= 2e-7 * w_printed + 1e-12, (rep, w[0], w_printed)


def test_printed_scale_and_time_conversion():
    r = lattice(2).r
    assert r == lattice(3).r
    assert abs(r - 1.19697977) < 5e-9  # Table I / II captions
    line = [l for l in open(os.path.join(GOLDEN, "time_conversion.txt"))
            if not l.startswith("#")][0].split()
    step, X, r_sec5, t_printed = int(line[0]), int(line[1]), float(line[2]), float(line[3])
    assert abs(r - r_sec5) < 1e-8
    assert round(step / (X * r), 4) == t_printed


@pytest.mark.parametrize("dim", [2, 3])
def test_quadrature_degree_nine(dim):
    lat = lattice(dim)
    worst = 0.0
    for alpha in itertools.product(range(10), repeat=dim):
        if sum(alpha) > 9:
            continue
        disc = np.sum(lat.w * np.prod(lat.xi ** np.array(alpha), axis=1))
        exact = np.prod([_gauss_moment_1d(a) for a in alpha])
        worst = max(worst, abs(disc - exact) / max(1.0, abs(exact)))
    assert worst < 5e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_quadrature_fails_at_degree_ten(dim):
    lat = lattice(dim)
    errs = []
    for alpha in itertools.product(range(11), repeat=dim):
        if sum(alpha) != 10:
            continue
        disc = np.sum(lat.w * np.prod(lat.xi ** np.array(alpha), axis=1))
        exact = np.prod([_gauss_moment_1d(a) for a in alpha])
        errs.append(abs(disc - exact) / abs(exact) if exact else abs(disc))
    assert max(errs) > 1e-3


@pytest.mark.parametrize("dim", [2, 3])
def test_lattice_symmetry(dim):
    lat = lattice(dim)
    # closed under negation and axis permutation, all in {-3..3}^D
    s = {tuple(v) for v in lat.e}
    assert len(s) == lat.Q
    for v in s:
        assert tuple(-a for a in v) in s
        for p in itertools.permutations(v):
            assert p in s
    assert np.max(np.abs(lat.e)) == 3


def test_delta_from_gamma():
    assert delta_from_gamma(1.4, 2) == pytest.approx(3.0, abs=1e-12)  # Sec. V, 2D
    assert delta_from_gamma(1.4, 3) == pytest.approx(2.0, abs=1e-12)  # Sec. V, 3D
    assert delta_from_gamma(5.0 / 3.0, 3) == 0.0
    assert delta_from_gamma(2.0, 2) == 0.0
    for D in (2, 3):
        d = delta_from_gamma(1.25, D)
        assert (d + D + 2) / (d + D) == pytest.approx(1.25, rel=1e-14)
    with pytest.raises(ValueError):
        delta_from_gamma(1.7, 3)
    with pytest.raises(ValueError):
        delta_from_gamma(1.0, 2)

"""Oracle lattice generator: D2Q37 and D3Q107 (Sec. IV, Tables I and II).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper builds both velocity sets by Gauss-Hermite quadrature on scaled
integer lattices: every discrete velocity is ``xi_i = r * e_i`` with integer
``e_i``, and the weights make the discrete sums reproduce the moments of the
standard normal weight function.  The tables print the symmetry groups,
member counts and 9-digit weights; the scale ``r`` is printed as 1.19697977.

This module derives the constants itself instead of trusting the printed
digits: the unknowns are the group weights ``w_g`` and ``s = r**2``; the
equations are the Gaussian moment conditions

    sum_i w_i xi_i^alpha = prod_k (alpha_k - 1)!!      (all alpha_k even)

for every even multi-index with total degree <= 8, one per multi-index up to
axis permutation (odd moments vanish by the lattice symmetry).  In 2D that is
9 equations for 8 weights and s, in 3D 11 equations for 10 weights and s.
Newton's method in 40-digit arithmetic, started from the printed table,
converges to the unique nearby solution.

Reading of the tables (they are partly garbled in the source):
  * Table I lists k = 4 for Perm(2r, r) and Perm(3r, r); all sign and axis
    permutations of those give 8 members each, and only with 8 do the groups
    add up to 37 velocities.
  * The text names the 3D set "D3Q105"; Table II's groups add up to 107.
"""
import itertools
from functools import lru_cache

import mpmath as mp
import numpy as np

# Group representatives in units of r, and the printed weights (Table I,
# Table II), used only as the Newton starting point and as the pin.
D2Q37_GROUPS = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (3, 0), (3, 1), (3, 3)]
D2Q37_PRINTED_W = [2.03916918e-1, 1.27544846e-1, 4.37537182e-2, 8.13659044e-3,
                   9.40079914e-3, 6.95051049e-4, 3.04298494e-5, 2.81093762e-5]
D3Q107_GROUPS = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 1, 1), (2, 0, 0),
                 (2, 1, 1), (2, 2, 0), (2, 2, 2), (3, 0, 0), (3, 1, 1)]
D3Q107_PRINTED_W = [1.603003550e-1, 2.390868500e-2, 4.169870315e-2,
                    5.166346780e-3, 1.227117147e-2, 2.676524495e-3,
                    9.685223338e-4, 2.170763000e-5, 2.453010230e-4,
                    1.417071270e-4]
PRINTED_R = 1.19697977


def group_members(rep):
    """All distinct vectors obtained from ``rep`` by axis permutation and
    sign changes ("Perm" in Tables I and II)."""
    out = set()
    for p in itertools.permutations(rep):
        for s in itertools.product((1, -1), repeat=len(rep)):
            out.add(tuple(a * b for a, b in zip(p, s)))
    return sorted(out, reverse=True)


def _double_factorial(n):
    return 1 if n <= 0 else n * _double_factorial(n - 2)


def _gaussian_moment(alpha):
    """E[z^alpha] for a standard normal vector z (odd -> 0)."""
    out = 1
    for a in alpha:
        if a % 2:
            return 0
        out *= _double_factorial(a - 1)
    return out


def _conditions(dim, degree):
    """Even multi-indices of total degree <= ``degree``, one per orbit
    under axis permutation (sorted, largest first)."""
    out = []
    for a in itertools.product(range(0, degree + 1, 2), repeat=dim):
        if sum(a) <= degree and list(a) == sorted(a, reverse=True):
            out.append(a)
    return out


@lru_cache(maxsize=None)
def _solve(dim, dps=40):
    groups = D2Q37_GROUPS if dim == 2 else D3Q107_GROUPS
    printed = D2Q37_PRINTED_W if dim == 2 else D3Q107_PRINTED_W
    members = [group_members(g) for g in groups]
    conds = _conditions(dim, 8)
    assert len(conds) == len(groups) + 1
    with mp.workdps(dps):
        # sum over a group's members of e^alpha (integers, exact)
        msum = [[sum(int(np.prod([e[k] ** a[k] for k in range(dim)]))
                     for e in mem) for mem in members] for a in conds]

        def residual(*x):
            w, s = x[:-1], x[-1]
            return [sum(w[g] * msum[c][g] for g in range(len(groups)))
                    * s ** (sum(conds[c]) // 2) - _gaussian_moment(conds[c])
                    for c in range(len(conds))]

        x0 = [mp.mpf(v) for v in printed] + [mp.mpf(PRINTED_R) ** 2]
        sol = mp.findroot(residual, x0, tol=mp.mpf(10) ** (-(dps - 5)))
        w = [sol[g] for g in range(len(groups))]
        s = sol[len(groups)]
        return ([mp.nstr(v, dps - 5) for v in w], mp.nstr(mp.sqrt(s), dps - 5),
                members)


class Lattice:
    """A velocity set: integer vectors ``e`` (Q x D), FP64 weights ``w`` (Q),
    scale ``r`` (xi = r e), group index of every velocity and the weights in
    40-digit strings (``w_exact``, ``r_exact``)."""

    def __init__(self, dim):
        if dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        w_str, r_str, members = _solve(dim)
        self.dim = dim
        self.r_exact = r_str
        self.w_group_exact = w_str
        self.r = float(mp.mpf(r_str))
        e, w, grp = [], [], []
        for g, mem in enumerate(members):
            for v in mem:
                e.append(v)
                w.append(float(mp.mpf(w_str[g])))
                grp.append(g)
        self.e = np.array(e, dtype=np.int64)
        self.w = np.array(w, dtype=np.float64)
        self.group = np.array(grp, dtype=np.int64)
        self.Q = len(e)
        self.xi = self.r * self.e.astype(np.float64)

    @property
    def name(self):
        return f"D{self.dim}Q{self.Q}"


@lru_cache(maxsize=None)
def lattice(dim):
    """D2Q37 for ``dim == 2``, D3Q107 for ``dim == 3``."""
    return Lattice(dim)


def delta_from_gamma(gamma, dim):
    """Internal degrees of freedom from the specific-heat ratio: the paper
    defines gamma = (delta + D + 2) / (delta + D) (Sec. II), so
    delta = 2 / (gamma - 1) - D.  A result within 1e-9 of zero is taken as
    zero (gamma = 5/3 in 3D); a negative one is rejected as unphysical."""
    if not gamma > 1.0:
        raise ValueError("gamma must exceed 1")
    d = 2.0 / (gamma - 1.0) - dim
    if abs(d) < 1e-9:
        d = 0.0
    if d < 0:
        raise ValueError(f"gamma={gamma} needs delta={d} < 0 in {dim}D")
    return d

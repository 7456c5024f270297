"""A numpy model of the FP32 deviation-storage step, for the tests only.

It evaluates the lattice scheme (Sec. II moments, Sec. IV equilibrium, BGK
relaxation, lattice streaming with the Sec. V time step) the way the FP32
storage path does, in a chosen floating-point type:

  * populations are held as deviations from the rest equilibrium,
    g~_i = g_i - w_i and h~_i = h_i - (delta/2) w_i (rho0 = T0 = 1);
  * the moments, the temperature offset t = T - 1 and the equilibrium
    targets are formed directly on the deviations, F_i - w_i =
    w_i (rho (P_i - 1) + (rho - 1)), so the rest-state part is never rounded;
  * the float residuals of the targets' mass, momentum and energy sums are
    folded back into the rest and axis populations (exact in exact
    arithmetic: the quadrature identities of Sec. IV make them zero).

With dtype=np.float64 it is the oracle's arithmetic reordered, so it must
match the oracle to round-off; with dtype=np.float32 it shows what float
arithmetic alone costs on a given case.  It shares nothing with the HIP
library: it is written from the method, with the lattice of the oracle's own
generator.  Every elementary operation rounds once (numpy has no fused
multiply-add), where the GPU fuses multiply-adds: the two float32
evaluations differ at the rounding level in every step.
"""
import numpy as np

from oracle.lattice import delta_from_gamma, lattice


class DevModel:
    """One solve on an nx x ny (x nz) grid; ``open_end`` per axis (zero
    gradient: the pull source is clamped), else periodic.

    ``order`` picks one of several evaluation orders of the same arithmetic,
    to show how far apart two correct evaluations in one floating-point type
    land:
      "pairwise"    numpy's own sums over the populations (pairwise),
      "sequential"  sums over the populations one after the other,
      "perturbed"   pairwise, and after every collision each stored value
                    is moved by -1, 0 or +1 unit in the last place (seeded):
                    a stand-in for any other rounding sequence;
      "widesum"     sequential, with the sums of the targets accumulated in
                    float64 and rounded once;
      "nofold"      sequential, without the exact-moment fold (the targets
                    as the equilibrium gives them).
    ``dt``: None for lattice streaming, else the time step of the
    finite-difference form of Sec. III (grid step 1, speeds r e_i, rates
    dt/tau): forward Euler with the third-order upwind-biased convection per
    axis, every term at time t.
    """

    def __init__(self, dim, gamma, tau_f, tau_g, nx, ny=1, nz=1,
                 open_end=(False, False, False), dtype=np.float32, order="pairwise",
                 dt=None, seed=0):
        lat = lattice(dim)
        self.dim, self.ft = dim, dtype
        self.shape = (nx, ny, nz if dim == 3 else 1)
        self.e = np.asarray(lat.e, dtype=np.int64)           # [Q][D]
        self.w64 = np.asarray(lat.w, dtype=np.float64)
        self.r64 = float(lat.r)
        self.delta = delta_from_gamma(gamma, dim)
        self.Q = self.e.shape[0]
        self.open_end = open_end
        T = dtype
        self.w = self.w64.astype(T)
        self.r = T(self.r64)
        self.r2 = T(self.r64 * self.r64)
        self.hd = T(0.5 * self.delta)
        self.inv_dof = T(1.0 / (dim + self.delta))
        self.half_dof = T(0.5 * dim) + T(0.5 * self.delta)
        self.fd = dt is not None
        self.om_f = T(dt / tau_f) if self.fd else T(1.0 / tau_f)
        self.om_g = T(dt / tau_g) if self.fd else T(1.0 / tau_g)
        self.cs = T(dt * self.r64 / 6.0) if self.fd else T(0)
        self.order = order
        self.rng = np.random.default_rng(seed)
        self.ef = self.e.astype(T)                          # [Q][D]
        self.qn = np.sum(self.e * self.e, axis=1)          # |e|^2 per population
        self.qf = self.qn.astype(T)
        self.l1 = np.sum(np.abs(self.e), axis=1)           # |e|_1 per population
        self.rest = int(np.flatnonzero(self.qn == 0)[0])
        # axis populations: +e_k and -e_k of each axis k
        self.axis = [(int(np.flatnonzero((self.qn == 1) & (self.e[:, k] == 1))[0]),
                      int(np.flatnonzero((self.qn == 1) & (self.e[:, k] == -1))[0]))
                     for k in range(dim)]

    # -- equilibrium in deviation form ---------------------------------------
    def _targets(self, u, t, T):
        """P_i - 1 [cells][Q] in type T, the 4th-order equilibrium polynomial
        (corrected Sec. IV form) less its rest value, from u [cells][D] and
        t = T - 1 [cells]: F_i - w_i = w_i (rho (P_i - 1) + (rho - 1))."""
        D = self.dim
        U = np.sum(u * u, axis=1)                         # [cells]
        c = (u @ (self.ef.T * self.r)).astype(T)          # xi_i . u, [cells][Q]
        q = self.r2 * self.qf                             # shell |xi|^2, [Q]
        Dd = T(D)
        t_, U_ = t[:, None], U[:, None]
        a0m1 = (T(0.5) * (t_ * (q - Dd) - U_)
                + T(1.0 / 24.0) * (T(3) * U_ * U_ + T(6) * t_ * (Dd + T(2) - q) * U_
                                   + T(3) * t_ * t_ * (q * q - T(2) * (Dd + T(2)) * q
                                                       + Dd * (Dd + T(2)))))
        a1 = T(1) - T(0.5) * U_ + T(0.5) * t_ * (q - Dd - T(2))
        a2 = T(0.5) - T(0.25) * U_ + T(0.25) * t_ * (q - Dd - T(4))
        c2 = c * c
        even = a0m1 + c2 * (a2 + c2 * T(1.0 / 24.0))
        odd = c * (a1 + c2 * T(1.0 / 6.0))
        return even + odd                                 # P_i - 1

    def init_fields(self, rho, u, T_field):
        """S_0: the equilibrium of the fields, formed in float64 and rounded
        once to the storage type."""
        n = rho.size
        D = self.dim
        rho = np.asarray(rho, dtype=np.float64).reshape(n)
        u = np.asarray(u, dtype=np.float64).reshape(D, n).T
        Tf = np.asarray(T_field, dtype=np.float64).reshape(n)
        save = (self.ft, self.ef, self.r, self.r2, self.qf)
        self.ef, self.r, self.r2 = self.e.astype(np.float64), self.r64, self.r64 ** 2
        self.qf = self.qn.astype(np.float64)
        pm1 = self._targets(u, Tf - 1.0, np.float64)
        self.ft, self.ef, self.r, self.r2, self.qf = save
        Fdev = self.w64 * (rho[:, None] * pm1 + (rho - 1.0)[:, None])
        hd = 0.5 * self.delta
        self.g = Fdev.astype(self.ft)
        self.h = (hd * Tf[:, None] * Fdev + hd * self.w64 * (Tf - 1.0)[:, None]).astype(self.ft)

    def _sum(self, a, weights=None):
        """Sum over the populations (axis 1), optionally weighted."""
        if weights is not None:
            a = a * weights
        if self.order in ("sequential", "widesum", "nofold"):
            acc = np.zeros(a.shape[0], dtype=a.dtype)
            for i in range(a.shape[1]):
                acc = acc + a[:, i]
            return acc
        return np.sum(a, axis=1)

    def _vsum(self, a):
        """[cells][D] momentum-like sums sum_i e_i a_i."""
        return np.stack([self._sum(a, self.ef[:, k]) for k in range(self.dim)], axis=1)

    # -- one collision ---------------------------------------------------------
    def collide(self):
        T = self.ft
        D = self.dim
        g, h = self.g, self.h
        if self.fd:  # the time-n values the convection differences
            self._g0, self._h0 = g.copy(), h.copy()
        s0 = self._sum(g)
        sj = self._vsum(g)                                # [cells][D], lattice units
        se = self._sum(g, self.qf)
        sh = self._sum(h)
        drho = s0
        rho = T(1) + drho
        inv_rho = T(1) / rho
        u = (self.r * sj) * inv_rho[:, None]
        U = np.sum(u * u, axis=1)
        X = T(0.5) * self.r2 * se + sh
        t = (T(2) * (X - drho * self.half_dof) * inv_rho - U) * self.inv_dof
        pm1 = self._targets(u, t, T)
        hd = self.hd
        hdT = hd * (T(1) + t)
        want_e = (rho * U + T(D) * (drho + rho * t)) / self.r2
        for dist, arho, beta, om, want_m, je in (
                (g, rho, drho, self.om_f, drho, True),
                (h, hdT * rho, hdT * drho + hd * t, self.om_g, hd * (drho + rho * t), False)):
            tgt = self.w * (arho[:, None] * pm1 + beta[:, None])
            # fold the float residuals of the target moments back in
            if self.order == "widesum":
                wide = tgt.astype(np.float64)
                dm = want_m - np.sum(wide, axis=1).astype(T)
            else:
                dm = want_m - self._sum(tgt)
            if self.order == "nofold":
                dm = dm * T(0)
            if je and self.order == "nofold":
                de = dm
                dj = np.zeros_like(sj)
            elif je and self.order == "widesum":
                de = want_e - (wide @ self.qn.astype(np.float64)).astype(T)
                dj = sj - (wide @ self.e.astype(np.float64)).astype(T)
            elif je:
                de = want_e - self._sum(tgt, self.qf)
                dj = sj - self._vsum(tgt)
                tgt[:, self.rest] += dm - de
                for k, (ip, im) in enumerate(self.axis):
                    tgt[:, ip] += de * T(1.0 / (2 * D)) + T(0.5) * dj[:, k]
                    tgt[:, im] += de * T(1.0 / (2 * D)) - T(0.5) * dj[:, k]
            else:
                tgt[:, self.rest] += dm
            if self.fd:  # the convection's centre term 3 |e|_1 (dt r / 6) p
                kc = T(3) * self.l1.astype(T) * self.cs
                dist[...] = (dist - kc * dist) + om * (tgt - dist)
            else:
                dist += om * (tgt - dist)
        if self.order == "perturbed":
            for dist in (g, h):
                ulp = np.spacing(np.abs(dist)).astype(T)
                dist += self.rng.integers(-1, 2, size=dist.shape).astype(T) * ulp

    # -- streaming (exact: a permutation) ---------------------------------------
    def stream(self):
        """Population i moves e_i cells: each cell pulls from x - e_i."""
        for dist in (self.g, self.h):
            out = np.empty_like(dist)
            for i in range(self.Q):
                e = [int(v) for v in self.e[i]] + [0] * (3 - self.dim)
                out[:, i] = dist[self._source([-v for v in e]), i]
            dist[...] = out

    def _source(self, shift):
        """Cell index each cell reads `shift` (per axis) away: periodic wrap
        or clamp at an open end."""
        shift = tuple(shift)
        cache = self.__dict__.setdefault("_src_cache", {})
        if shift in cache:
            return cache[shift]
        nx, ny, nz = self.shape
        cells = np.arange(nx * ny * nz)
        coord = (cells % nx, (cells // nx) % ny, cells // (nx * ny))
        src = []
        for c, d, n, op in zip(coord, shift, (nx, ny, nz), self.open_end):
            s = c + d
            src.append(np.clip(s, 0, n - 1) if op else s % n)
        cache[shift] = src[0] + nx * (src[1] + ny * src[2])
        return cache[shift]

    def convect(self):
        """Finite differences: subtract the neighbour terms
        (dt r / 6) sum_a |e_a| [p(x - 2s) - 6 p(x - s) + 2 p(x + s)],
        s = sign(e_a), of the time-n values."""
        T = self.ft
        for dist, old in ((self.g, self._g0), (self.h, self._h0)):
            for i in range(self.Q):
                nb = np.zeros(dist.shape[0], dtype=T)
                for a in range(self.dim):
                    e = int(self.e[i, a])
                    if e == 0:
                        continue
                    sg = 1 if e > 0 else -1

                    def at(d):
                        shift = [0, 0, 0]
                        shift[a] = d
                        return old[self._source(shift), i]
                    nb = nb + T(abs(e)) * ((at(-2 * sg) - T(6) * at(-sg)) + T(2) * at(sg))
                dist[:, i] = dist[:, i] - self.cs * nb

    def step(self, n=1):
        for _ in range(n):
            self.collide()
            if self.fd:
                self.convect()
            else:
                self.stream()

    def moments(self):
        """(rho, u [D][cells], T) of the current state, summed in float64."""
        g = self.g.astype(np.float64)
        h = self.h.astype(np.float64)
        rho = 1.0 + np.sum(g, axis=1)
        mom = self.r64 * (g @ self.e.astype(np.float64))
        rhoE = (0.5 * self.r64 ** 2 * (g @ self.qn.astype(np.float64)) + np.sum(h, axis=1)
                + 0.5 * (self.dim + self.delta))
        u = (mom / rho[:, None]).T
        E = rhoE / rho
        T = (2.0 * E - np.sum(u * u, axis=0)) / (self.dim + self.delta)
        return rho, u, T

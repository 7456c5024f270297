// Device code shared by the single-solve kernels (kernels.hip, fd.hip) and
// the batched multi-solve kernels (pool.hip): memory helpers, the pull
// offsets, the moments, the 4th-order equilibrium, the BGK relaxation (with
// the finite-difference and energy-conserving variants), the storage
// precisions, and the whole per-cell collision in the two register layouts.
#pragma once

#include <type_traits>

#include "lbm_internal.h"

namespace lbm {
namespace core {

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <typename T>
__device__ __forceinline__ T load_at(const char* base, uint32_t byte_off) {
    return *reinterpret_cast<const T*>(base + byte_off);
}

// Populations are written once per step and read back only in the next
// launch, far beyond what L2 holds: stream them out non-temporally so they do
// not evict the lines that neighbouring waves are still pulling from.
template <typename T>
__device__ __forceinline__ void store_at(char* base, uint32_t byte_off, T v) {
    __builtin_nontemporal_store(v, reinterpret_cast<T*>(base + byte_off));
}

// Ordinary (cached) store, for the split layout in half storage: its lanes
// write single halves into the g/h words (g lanes the low, h lanes the high
// halves of one line).  Through the cache or streamed measured the same
// (6.2 ms per D3Q107 256^3 step); the one-lane kernel, which AUTO takes in
// half storage, stores whole words.
template <typename T>
__device__ __forceinline__ void store_cached(char* base, uint32_t byte_off, T v) {
    *reinterpret_cast<T*>(base + byte_off) = v;
}

// Source coordinate of a pull along one axis: x - e, wrapped (periodic) or
// clamped (zero gradient).
__device__ __forceinline__ int pull_coord(int x, int e, int n, bool open_end) {
    int s = x - e;
    if (open_end) return s < 0 ? 0 : (s > n - 1 ? n - 1 : s);
    if (n >= 3) return s < 0 ? s + n : (s >= n ? s - n : s);
    s %= n;
    return s < 0 ? s + n : s;
}

// Per-axis source offsets (in cells) for shifts e = -3..3, index e + 3.
template <int D>
struct PullTable {
    int x[7], y[7], z[7];
    __device__ __forceinline__ void fill(int cx, int cy, int cz, int nx, int ny,
                                         int nz, int nxy, uint32_t open_end,
                                         bool stream) {
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            const int e = stream ? k - 3 : 0;
            x[k] = pull_coord(cx, e, nx, open_end & 1u);
            y[k] = pull_coord(cy, e, ny, open_end & 2u) * nx;
            if constexpr (D == 3) z[k] = pull_coord(cz, e, nz, open_end & 4u) * nxy;
        }
    }
    // source cell of the population with lattice vector (EX, EY, EZ)
    template <int EX, int EY, int EZ>
    __device__ __forceinline__ int src() const {
        if constexpr (D == 3) return x[EX + 3] + y[EY + 3] + z[EZ + 3];
        else return x[EX + 3] + y[EY + 3];
    }
};


// Cell -> (x, y, z).
__device__ __forceinline__ void coords(int cell, int nx, int nxy, int& x, int& y,
                                       int& z) {
    z = cell / nxy;
    const int rem = cell - z * nxy;
    y = rem / nx;
    x = rem - y * nx;
}

// The 4th-order equilibrium of one cell, as a polynomial in c = xi . u per
// shell |xi|^2 = q (one shell per group):
//   P(c) = A0 + A1 c + A2 c^2 + c^3/6 + c^4/24,
//   A0 - 1 = (-U + t(q-D))/2 + (3U^2 + 6t(D+2-q)U + 3t^2(q^2-2(D+2)q+D(D+2)))/24
//   A1 = 1 - U/2 + t(q-D-2)/2,  A2 = 1/2 - U/4 + t(q-D-4)/4,
// U = |u|^2, t = T - 1, and F_i = w_i rho P(c_i).  The coefficients are
// formed per group at the point of use, which keeps register live ranges
// short.  In deviation storage (DEV) A0 is returned as A0 - 1, so that the
// rest-state part w_i is never formed in float:
//   F_i - w_i = w_i (rho (P_i - 1) + (rho - 1)).
template <int D, typename T, bool DEV>
struct Equilibrium {
    T U, t, r2, ru[3];

    __device__ __forceinline__ void setup(const T* u, T t_, T r) {
        U = D == 3 ? u[0] * u[0] + u[1] * u[1] + u[2] * u[2] : u[0] * u[0] + u[1] * u[1];
        t = t_;
        r2 = r * r;
#pragma unroll
        for (int k = 0; k < 3; ++k) ru[k] = k < D ? r * u[k] : T(0);
    }

    template <int QN>
    __device__ __forceinline__ void coef(T& A0, T& A1, T& A2) const {
        const T q = r2 * T(QN);
        constexpr T Dd = T(D);
        const T a0m1 = T(0.5) * (t * (q - Dd) - U) +
                       T(1.0 / 24.0) * (T(3) * U * U + T(6) * t * (Dd + T(2) - q) * U +
                                        T(3) * t * t * (q * q - T(2) * (Dd + T(2)) * q +
                                                        Dd * (Dd + T(2))));
        A0 = DEV ? a0m1 : T(1) + a0m1;
        A1 = T(1) - T(0.5) * U + T(0.5) * t * (q - Dd - T(2));
        A2 = T(0.5) - T(0.25) * U + T(0.25) * t * (q - Dd - T(4));
    }

    // c = xi_i . u for the lattice vector V
    template <int EX, int EY, int EZ>
    __device__ __forceinline__ T dot() const {
        T c = T(0);
        if constexpr (EX != 0) c += T(EX) * ru[0];
        if constexpr (EY != 0) c += T(EY) * ru[1];
        if constexpr (D == 3 && EZ != 0) c += T(EZ) * ru[2];
        return c;
    }
};

// Fused multiply-add, written out.  The target and relaxation code below
// turns implicit contraction off and states each fused operation itself.
template <typename T>
__device__ __forceinline__ T fmadd(T a, T b, T c) {
    if constexpr (std::is_same_v<T, float>)
        return __builtin_fmaf(a, b, c);
    else
        return __builtin_fma(a, b, c);
}

// BGK targets of a +- pair of populations with c = xi . u (c for the first
// of the pair, -c for the second):
//   t = w (arho P(+-c) + beta),  P(c) = A0 + A1 c + A2 c^2 + c^3/6 + c^4/24,
// each rounded once.  The exact-moment correction of deviation storage sums
// these very values, and the relaxation uses them.  Contraction is off here:
// a multiply w * (...) fused into a later sum would let that sum see the
// unrounded target, and the correction would then not cancel the rounding
// of the targets it is applied to (measured: 10x the float32 error on a
// shock tube).  pair_parts forms the even and odd parts of P(c), P(+-c) =
// even +- odd, which do not depend on the distribution; pair_finish the two
// targets of one distribution from them.
template <typename T>
__device__ __forceinline__ void pair_parts(T A0, T A1, T A2, T c, T& even, T& odd) {
#pragma clang fp contract(off)
    const T c2 = c * c;
    even = fmadd(c2, fmadd(c2, T(1.0 / 24.0), A2), A0);
    odd = c * fmadd(c2, T(1.0 / 6.0), A1);
}

template <typename T>
__device__ __forceinline__ void pair_finish(T even, T odd, T w, T arho, T beta, T& tp, T& tm) {
#pragma clang fp contract(off)
    tp = w * fmadd(arho, even + odd, beta);
    tm = w * fmadd(arho, even - odd, beta);
}

template <typename T>
__device__ __forceinline__ void pair_targets(T A0, T A1, T A2, T c, T w, T arho, T beta, T& tp,
                                             T& tm) {
    T even, odd;
    pair_parts(A0, A1, A2, c, even, odd);
    pair_finish(even, odd, w, arho, beta, tp, tm);
}

// Target of the rest population (c = 0), rounded once as above.
template <typename T>
__device__ __forceinline__ T rest_target(T A0, T w, T arho, T beta) {
#pragma clang fp contract(off)
    return w * fmadd(arho, A0, beta);
}

// One relaxation p + omega (t - p); with the finite-difference centre term
// kc p (kc = 0: none) taken from the pre-collision value first.
template <typename T>
__device__ __forceinline__ T relax_value(T p, T t, T omega, T kc) {
#pragma clang fp contract(off)
    return fmadd(omega, t - p, fmadd(-kc, p, p));
}
template <typename T>
__device__ __forceinline__ T relax_value(T p, T t, T omega) {
#pragma clang fp contract(off)
    return fmadd(omega, t - p, p);
}

// First velocity index of group g (velocities are ordered group by group).
template <int D>
constexpr int group_start(int g) {
    int s = 0;
    for (int k = 0; k < g; ++k) s += kVelSet<D>.count[k];
    return s;
}

// Group weight in the arithmetic type (the parameters carry both).
template <typename T>
__device__ __forceinline__ T weight(const Physics& ph, int g);
template <>
__device__ __forceinline__ double weight<double>(const Physics& ph, int g) { return ph.w[g]; }
template <>
__device__ __forceinline__ float weight<float>(const Physics& ph, int g) { return ph.wf[g]; }

// Storage precisions.  T is the arithmetic type of the collision, S the type
// a population is stored in.  F16 stores the deviation of a population from
// its rest equilibrium divided by its weight, (g_i - w_i) / w_i and
// (h_i - (delta/2) w_i) / w_i: dividing by w_i (which spans 3e-5 .. 0.2)
// makes every population's stored value of the same size, so one half-
// precision format serves all of them.  Loads multiply w_i back and the
// collision runs in float exactly as for F32Dev.
struct F64 {
    using T = double;
    using S = double;
    static constexpr bool kDev = false, kScaled = false;
};
struct F32Dev {
    using T = float;
    using S = float;
    static constexpr bool kDev = true, kScaled = false;
};
struct F16Dev {
    using T = float;
    using S = _Float16;
    static constexpr bool kDev = true, kScaled = true;
};

// Moment sums over one set of Q populations p (scaled lattice units):
// s0 = sum p, sj = sum e p, se = sum |e|^2 p.
template <int D, typename T, class Get>
__device__ __forceinline__ void moment_sums_of(Get&& get, T& s0, T* sj, T& se) {
    constexpr VelSet<D> V = kVelSet<D>;
    constexpr int Q = VelSet<D>::Q;
    T a0 = 0, ax = 0, ay = 0, az = 0, ae = 0;
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr Vel v = V.v[i];
        const T x = get(I);
        a0 += x;
        if constexpr (v.x != 0) ax += T(v.x) * x;
        if constexpr (v.y != 0) ay += T(v.y) * x;
        if constexpr (D == 3 && v.z != 0) az += T(v.z) * x;
        if constexpr (V.qn[v.group] != 0) ae += T(V.qn[v.group]) * x;
    });
    s0 = a0;
    sj[0] = ax;
    sj[1] = ay;
    if constexpr (D == 3) sj[2] = az;
    se = ae;
}

template <int D, typename T>
__device__ __forceinline__ void moment_sums(const T* p, T& s0, T* sj, T& se) {
    moment_sums_of<D, T>([&](auto I) { return p[decltype(I)::value]; }, s0, sj, se);
}

// |e|_1 of a lattice vector.
__host__ __device__ constexpr int l1_of(Vel v) {
    return (v.x < 0 ? -v.x : v.x) + (v.y < 0 ? -v.y : v.y) + (v.z < 0 ? -v.z : v.z);
}

// Energy-conserving collision coefficient 1 - tau_g / tau_f (0 when off), in T.
template <typename T>
__device__ __forceinline__ T ec_coef(const Physics& ph);
template <>
__device__ __forceinline__ double ec_coef<double>(const Physics& ph) { return ph.ec; }
template <>
__device__ __forceinline__ float ec_coef<float>(const Physics& ph) { return ph.ecf; }

// Convection scale dt r / 6 of the finite-difference form, in T.
template <typename T>
__device__ __forceinline__ T fd_scale(const Physics& ph);
template <>
__device__ __forceinline__ double fd_scale<double>(const Physics& ph) { return ph.fd_cs; }
template <>
__device__ __forceinline__ float fd_scale<float>(const Physics& ph) { return ph.fd_csf; }

// Relax one set of populations toward their BGK targets with rate omega:
//   t_i = w_i (alpha rho P~(c_i) + beta),
// i.e. t_i = F_i for g (alpha = 1) and t_i = (delta/2) T F_i for h
// (alpha = (delta/2) T); in deviation storage beta carries the rest-state
// shift: beta = rho - 1 for g and (delta/2)(T (rho - 1) + T - 1) for h, and
// then t_i is the target minus its rest value.
//
// Deviation storage (DEV) also makes the targets' discrete moments exact.
// The weights, rounded to float, miss the quadrature identities by ~3e-8
// relative, which would bias mass, momentum and energy by the same order in
// every collision, always with the same sign.  In exact arithmetic
// sum t_i = want_m, sum e_i t_i = want_j and sum |e_i|^2 t_i = want_e hold
// already; here the float residuals of those sums are folded back into the
// rest population and the 2D axis populations (group |e| = 1):
//   mass     into the rest population,
//   momentum +d/2 and -d/2 into the +e_k / -e_k pair (no mass, no energy),
//   energy   +d/(2D) into each axis population, -d into the rest (no mass,
//            no momentum).
// je_on = 0 restricts the correction to the mass (used for h, whose only
// conserved moment is its sum).
//
// FD (the finite-difference form, Sec. III): omega is dt / tau, and each
// population also loses the centre term of its upwind-biased convection,
// 3 |e_i|_1 (dt r / 6) p_i, taken from the pre-collision value; the
// neighbour terms are added by convect_store_* below.
//
// relax_k does this for K distributions of one cell at once (K = 2: g and h
// of a lane that holds both): each pair's polynomial is formed once and
// serves every distribution.  Per distribution the arithmetic, and the order
// of every sum, is that of K = 1.  p.get<k, i>() / p.set<k, i>(v):
// population i of distribution k; r[k]: its parameters; relax: one
// distribution held in an array.
template <typename T>
struct RelaxPar {
    T arho, beta, omega, want_m, want_e, je_on;
};

template <int D, typename T, bool DEV, bool FD, int K, class Acc>
__device__ __forceinline__ void relax_k(const Acc& p, const Equilibrium<D, T, DEV>& eq,
                                        const Physics& a, const RelaxPar<T>* r,
                                        const T* want_j) {
#pragma clang fp contract(off)
    constexpr VelSet<D> V = kVelSet<D>;
    constexpr int G = VelSet<D>::G;
    // p + omega (t - p), less the convection centre term in FD
    auto update = [&](auto Kc, auto Ic, T t, auto L1) {
        constexpr int k = decltype(Kc)::value;
        constexpr int i = decltype(Ic)::value;
        constexpr int l1 = decltype(L1)::value;
        const T pi = p.template get<k, i>();
        if constexpr (FD && l1 != 0) {
            const T kc = T(3 * l1) * fd_scale<T>(a);
            p.template set<k, i>(relax_value(pi, t, r[k].omega, kc));
        } else {
            p.template set<k, i>(relax_value(pi, t, r[k].omega));
        }
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    static_assert(V.v[1].group == 1 && V.v[2 * D].group == 1 && V.v[2 * D + 1].group == 2,
                  "the axis populations must follow the rest population");
    T sm[K], sjx[K], sjy[K], sjz[K], se[K];
    T t1[K][2 * D];  // targets of the axis populations, corrected below
#pragma unroll
    for (int k = 0; k < K; ++k) sm[k] = sjx[k] = sjy[k] = sjz[k] = se[k] = T(0);
    static_for<1, G>([&](auto Gi) {
        constexpr int g = decltype(Gi)::value;
        T A0, A1, A2;
        eq.template coef<V.qn[g]>(A0, A1, A2);
        const T w = weight<T>(a, g);
        constexpr int first = group_start<D>(g);
        static_for<0, V.count[g] / 2>([&](auto Pi) {
            constexpr int i = first + 2 * decltype(Pi)::value;
            constexpr Vel v = V.v[i];
            const T c = eq.template dot<v.x, v.y, v.z>();
            T even, odd;
            pair_parts(A0, A1, A2, c, even, odd);
            static_for<0, K>([&](auto Kc) {
                constexpr int k = decltype(Kc)::value;
                T tp, tm;
                pair_finish(even, odd, w, r[k].arho, r[k].beta, tp, tm);
                if constexpr (DEV) {
                    const T sum = tp + tm;
                    const T dif = tp - tm;
                    sm[k] += sum;
                    if constexpr (v.x != 0) sjx[k] = fmadd(T(v.x), dif, sjx[k]);
                    if constexpr (v.y != 0) sjy[k] = fmadd(T(v.y), dif, sjy[k]);
                    if constexpr (D == 3 && v.z != 0) sjz[k] = fmadd(T(v.z), dif, sjz[k]);
                    se[k] = fmadd(T(V.qn[g]), sum, se[k]);
                }
                if constexpr (DEV && g == 1) {
                    t1[k][i - 1] = tp;
                    t1[k][i] = tm;
                } else {
                    update(Kc, std::integral_constant<int, i>{}, tp,
                           std::integral_constant<int, l1_of(v)>{});
                    update(Kc, std::integral_constant<int, i + 1>{}, tm,
                           std::integral_constant<int, l1_of(v)>{});
                }
            });
        });
    });
    T A0, A1, A2;
    eq.template coef<0>(A0, A1, A2);
    static_for<0, K>([&](auto Kc) {
        constexpr int k = decltype(Kc)::value;
        T t0 = rest_target(A0, weight<T>(a, 0), r[k].arho, r[k].beta);
        if constexpr (DEV) {
            sm[k] += t0;
            const T je_on = r[k].je_on;
            const T dm = r[k].want_m - sm[k];
            const T de = je_on * (r[k].want_e - se[k]);
            const T dj[3] = {je_on * (want_j[0] - sjx[k]), je_on * (want_j[1] - sjy[k]),
                             D == 3 ? je_on * (want_j[2] - sjz[k]) : T(0)};
            t0 += dm - de;
            const T de_axis = de * T(1.0 / (2 * D));
            static_for<0, D>([&](auto I) {
                constexpr int q = decltype(I)::value;
                constexpr Vel v = V.v[1 + 2 * q];  // +e_axis (first of its pair)
                constexpr int axis = v.x != 0 ? 0 : (v.y != 0 ? 1 : 2);
                const T half = T(0.5) * dj[axis];
                const T tp = t1[k][2 * q] + de_axis + half;
                const T tm = t1[k][2 * q + 1] + de_axis - half;
                update(Kc, std::integral_constant<int, 1 + 2 * q>{}, tp, I1{});
                update(Kc, std::integral_constant<int, 2 + 2 * q>{}, tm, I1{});
            });
        }
        update(Kc, I0{}, t0, I0{});
    });
}

// One distribution held in an array.
template <typename T>
struct ArrayAcc1 {
    T* p;
    template <int K, int I>
    __device__ __forceinline__ T get() const { return p[I]; }
    template <int K, int I>
    __device__ __forceinline__ void set(T v) const { p[I] = v; }
};

// Distribution K0 of a two-distribution accessor, as a one-distribution one.
template <int K0, class Acc>
struct Slice {
    const Acc& p;
    template <int K, int I>
    __device__ __forceinline__ auto get() const { return p.template get<K0, I>(); }
    template <int K, int I, typename V>
    __device__ __forceinline__ void set(V v) const { p.template set<K0, I>(v); }
};

// The BGK relaxation of one distribution (the parameters as in RelaxPar).
template <int D, typename T, bool DEV, bool FD = false>
__device__ __forceinline__ void relax(T* p, const Equilibrium<D, T, DEV>& eq,
                                      const Physics& a, T arho, T beta, T omega, T want_m,
                                      const T* want_j, T want_e, T je_on) {
    const RelaxPar<T> r{arho, beta, omega, want_m, want_e, je_on};
    relax_k<D, T, DEV, FD, 1>(ArrayAcc1<T>{p}, eq, a, &r, want_j);
}

// Macroscopic state of a cell from the moment sums.
template <int D, typename T, bool DEV>
__device__ __forceinline__ void macro(T s0, const T* sj, T se, T sh, T r,
                                      double inv_dof, double half_delta, T& rho,
                                      T& drho, T* u, T& t) {
    const T r2 = r * r;
    if constexpr (DEV) {
        drho = s0;
        rho = T(1) + drho;
    } else {
        rho = s0;
        drho = s0 - T(1);
    }
    const T inv_rho = T(1) / rho;
#pragma unroll
    for (int k = 0; k < D; ++k) u[k] = r * sj[k] * inv_rho;
    const T U = D == 3 ? u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
                       : u[0] * u[0] + u[1] * u[1];
    const T X = T(0.5) * r2 * se + sh;  // sum xi^2 g/2 + sum h (deviations in DEV)
    if constexpr (DEV) {
        // t = T - 1 = (2 (X - drho (D+delta)/2) / rho - U) / (D+delta): no
        // cancellation against the rest energy in float
        const T half_dof = T(0.5 * double(D)) + T(half_delta);
        t = (T(2) * (X - drho * half_dof) * inv_rho - U) * T(inv_dof);
    } else {
        t = (T(2) * X * inv_rho - U) * T(inv_dof) - T(1);
    }
}


// ---------------------------------------------------------------------------
// Pull offsets of one wave's row segment.  y, z and every pull offset along
// them are wave-uniform (scalar registers); per lane only the seven x offsets
// (shifts -3..3, wrapped or clamped) are held.  A population load is then one
// scalar base plus one of those seven lane offsets.
template <typename T>
struct RowOffsets {
    uint32_t xo[7];  // per lane
    uint32_t yo[7];  // wave-uniform
    uint32_t zo[7];  // wave-uniform
    uint32_t own;    // per lane: byte offset of the lane's own cell in its row
    uint32_t row;    // wave-uniform: byte offset of the row start
};

// Fill the offsets for the lane's cell x of row (y, z); `stream` = false
// points every pull at the cell itself (collision without streaming).
template <int D, typename T>
__device__ __forceinline__ void fill_row_offsets(RowOffsets<T>& o, int x, int y, int z, int nx,
                                                 int ny, int nz, int nxy, uint32_t open_end,
                                                 bool stream, uint32_t role_off) {
    constexpr uint32_t cb = cell_bytes(sizeof(T));
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        const int e = stream ? k - 3 : 0;
        o.xo[k] = (uint32_t)pull_coord(x, e, nx, open_end & 1u) * cb + role_off;
        o.yo[k] = (uint32_t)(pull_coord(y, e, ny, open_end & 2u) * nx) * cb;
        if constexpr (D == 3)
            o.zo[k] = (uint32_t)(pull_coord(z, e, nz, open_end & 4u) * nxy) * cb;
        else
            o.zo[k] = 0;
    }
    o.own = (uint32_t)x * cb + role_off;
    o.row = (uint32_t)(y * nx + z * nxy) * cb;
}

// Energy-conserving collision (a mode beyond the paper).  With rates a_f,
// a_g the BGK step changes a cell's total energy by (a_f - a_g)
// (E_tr^eq - E_tr), E_tr = sum xi^2 g / 2 and E_tr^eq = rho (u^2 + D T) / 2,
// because sum h relaxes at the other rate toward the complement.  h relaxed
// toward ((delta/2) T + kappa) F with
//   kappa rho = (1 - a_f / a_g) (E_tr^eq - E_tr)
// conserves energy exactly.  Returns kappa rho; a signed zero when the mode
// is off (coefficient 0), which leaves every target bit-identical.  In
// deviation storage E_tr^eq - E_tr = (r^2 / 2)(want_e - se), both sums over
// deviations.
template <int D, typename T, bool DEV>
__device__ __forceinline__ T energy_fix_kr(const Physics& ph, T rho,
                                           const Equilibrium<D, T, DEV>& eq, T want_e, T se) {
    T diff;
    if constexpr (DEV) {
        diff = T(0.5) * eq.r2 * (want_e - se);
    } else {
        diff = T(0.5) * (rho * (eq.U + T(D) * (T(1) + eq.t)) - eq.r2 * se);
    }
    return ec_coef<T>(ph) * diff;
}

// Collision of one cell, one lane holding all 2Q populations, reached
// through p.get<k, i>() / p.set<k, i>() with k = 0 for g and k = 1 for h.
// JOINT relaxes g and h in one pass over the pairs (relax_k with K = 2);
// otherwise g, then h.
template <int D, class P, bool FD, bool JOINT, class Acc>
__device__ __forceinline__ void collide_lane_acc(const Acc& p, const Physics& ph) {
    using T = typename P::T;
    constexpr bool DEV = P::kDev;
    T s0, sj[3] = {0, 0, 0}, se, sh, dummy_j[3], dummy_e;
    moment_sums_of<D, T>([&](auto I) { return p.template get<0, decltype(I)::value>(); }, s0, sj,
                         se);
    moment_sums_of<D, T>([&](auto I) { return p.template get<1, decltype(I)::value>(); }, sh,
                         dummy_j, dummy_e);
    T rho, drho, u[3] = {0, 0, 0}, t;
    macro<D, T, DEV>(s0, sj, se, sh, T(ph.r), ph.inv_dof, ph.half_delta, rho, drho, u, t);
    Equilibrium<D, T, DEV> eq;
    eq.setup(u, t, T(ph.r));
    const T hd = T(ph.half_delta);
    const T hdT = hd * (T(1) + t);
    // BGK targets: F for g; (delta/2) T F for h (shifted by the rest state in
    // deviation storage), plus kappa F in the energy-conserving mode; exact
    // target moments for the correction
    const T want_e = (rho * eq.U + T(D) * (drho + rho * t)) / eq.r2;
    const T kr = energy_fix_kr<D, T, DEV>(ph, rho, eq, want_e, se);
    const T beta_g = DEV ? drho : T(0);
    const T beta_h = DEV ? hdT * drho + hd * t + kr : T(0);
    const RelaxPar<T> r[2] = {{rho, beta_g, T(ph.omega_f), drho, want_e, T(1)},
                              {hdT * rho + kr, beta_h, T(ph.omega_g), hd * (drho + rho * t) + kr,
                               T(0), T(0)}};
    if constexpr (JOINT) {
        relax_k<D, T, DEV, FD, 2>(p, eq, ph, r, sj);
    } else {
        relax_k<D, T, DEV, FD, 1>(Slice<0, Acc>{p}, eq, ph, &r[0], sj);
        relax_k<D, T, DEV, FD, 1>(Slice<1, Acc>{p}, eq, ph, &r[1], sj);
    }
}

// g[] and h[] arrays.
template <typename T>
struct LaneAcc {
    T* g;
    T* h;
    template <int K, int I>
    __device__ __forceinline__ T get() const { return K ? h[I] : g[I]; }
    template <int K, int I>
    __device__ __forceinline__ void set(T v) const { (K ? h : g)[I] = v; }
};

template <int D, class P, bool FD = false>
__device__ __forceinline__ void collide_lane(typename P::T* g, typename P::T* h,
                                             const Physics& ph) {
    using T = typename P::T;
    collide_lane_acc<D, P, FD, false>(LaneAcc<T>{g, h}, ph);
}

// Collision of one cell in the split layout: lane l < 32 holds the g
// populations of its cell, lane l + 32 the h populations of the same cell
// (role 1).  The moment sums are exchanged between the halves (lane ^ 32);
// both halves evaluate the same equilibrium, each relaxes its own
// distribution.  Every lane of the wave must take part (the exchange).
template <int D, class P, bool FD = false>
__device__ __forceinline__ void collide_split(typename P::T* p, int role, const Physics& ph) {
    using T = typename P::T;
    constexpr bool DEV = P::kDev;
    T s0, sj[3] = {0, 0, 0}, se;
    moment_sums<D, T>(p, s0, sj, se);
    const T o0 = __shfl_xor(s0, 32);
    T oj[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < D; ++k) oj[k] = __shfl_xor(sj[k], 32);
    const T oe = __shfl_xor(se, 32);
    const T g0 = role ? o0 : s0;
    T gj[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < D; ++k) gj[k] = role ? oj[k] : sj[k];
    const T ge = role ? oe : se;
    const T sh = role ? s0 : o0;

    T rho, drho, u[3] = {0, 0, 0}, t;
    macro<D, T, DEV>(g0, gj, ge, sh, T(ph.r), ph.inv_dof, ph.half_delta, rho, drho, u, t);
    Equilibrium<D, T, DEV> eq;
    eq.setup(u, t, T(ph.r));
    const T hd = T(ph.half_delta);
    const T hdT = hd * (T(1) + t);
    const T want_e = (rho * eq.U + T(D) * (drho + rho * t)) / eq.r2;
    const T kr = energy_fix_kr<D, T, DEV>(ph, rho, eq, want_e, ge);
    const T arho = role ? hdT * rho + kr : rho;
    const T beta = DEV ? (role ? hdT * drho + hd * t + kr : drho) : T(0);
    const T want_m = role ? hd * (drho + rho * t) + kr : drho;
    relax<D, T, DEV, FD>(p, eq, ph, arho, beta, role ? T(ph.omega_g) : T(ph.omega_f), want_m, gj,
                         want_e, role ? T(0) : T(1));
}

// Pull the lane's cell (lane layout): g and h of every population.
// Half storage: each conversion and its weight scaling are one mixed-
// precision FMA with a zero addend, written out as such:
//   load   x = half(raw) * w_g          (v_fma_mix_f32, f16 source: exact
//                                         widening, one rounding in float)
//   store  raw = half(x * (1/w_g))       (v_fma_mixlo_f16: one rounding to
//                                         half, round to nearest even)
// The load converts in place (tied operand), so the load's destination
// register becomes the float.  Left to itself the compiler folds the
// conversions into the neighbouring FMAs instead, which keeps the half
// values live beside their float copies and costs 60-80 registers (an
// occupancy step).
//
// Stored value -> arithmetic value of a population of group g.
template <class P>
__device__ __forceinline__ typename P::T from_store(typename P::S raw, const Physics& ph, int g) {
    using T = typename P::T;
    if constexpr (P::kScaled) {
        static_assert(std::is_same_v<typename P::S, _Float16> && std::is_same_v<T, float>);
        float x = __builtin_bit_cast(float, (uint32_t)__builtin_bit_cast(uint16_t, raw));
        asm("v_fma_mix_f32 %0, %0, %1, 0 op_sel_hi:[1,0,0]" : "+v"(x) : "s"(weight<T>(ph, g)));
        return x;
    } else {
        return T(raw);
    }
}

// Arithmetic value -> stored value.
template <class P>
__device__ __forceinline__ typename P::S to_store(typename P::T v, const Physics& ph, int g) {
    if constexpr (P::kScaled) {
        static_assert(std::is_same_v<typename P::S, _Float16> && std::is_same_v<typename P::T, float>);
        _Float16 r;
        asm("v_fma_mixlo_f16 %0, %1, %2, 0 op_sel_hi:[0,0,0]" : "=v"(r) : "v"(v), "s"(ph.inv_wf[g]));
        return r;
    } else {
        return typename P::S(v);
    }
}

// PULL = false reads every population at the cell itself (the centre values
// of the finite-difference form).
template <int D, class P, bool PULL = true>
__device__ __forceinline__ void load_lane(const char* src, uint32_t plane,
                                          const RowOffsets<typename P::S>& o, typename P::T* g,
                                          typename P::T* h, const Physics& ph) {
    using S = typename P::S;
    constexpr VelSet<D> V = kVelSet<D>;
    static_for<0, VelSet<D>::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr Vel v = V.v[i];
        constexpr int kx = PULL ? v.x + 3 : 3, ky = PULL ? v.y + 3 : 3, kz = PULL ? v.z + 3 : 3;
        const char* base = src + (size_t)(2 * i) * plane + o.yo[ky] + o.zo[kz];
        g[i] = from_store<P>(load_at<S>(base, o.xo[kx]), ph, v.group);
        h[i] = from_store<P>(load_at<S>(base + h_offset(sizeof(S), plane), o.xo[kx]), ph, v.group);
    });
}

template <int D, class P>
__device__ __forceinline__ void store_lane(char* dst, uint32_t plane,
                                           const RowOffsets<typename P::S>& o,
                                           const typename P::T* g, const typename P::T* h,
                                           const Physics& ph) {
    constexpr VelSet<D> V = kVelSet<D>;
    char* row = dst + o.row;
    const uint32_t ho = h_offset(sizeof(typename P::S), plane);
    static_for<0, VelSet<D>::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int grp = V.v[i].group;
        char* base = row + (size_t)(2 * i) * plane;
        store_at(base, o.own, to_store<P>(g[i], ph, grp));
        store_at(base + ho, o.own, to_store<P>(h[i], ph, grp));
    });
}

// Pull the lane's half of its cell (split layout; the role offset is in o).
template <int D, class P, bool PULL = true>
__device__ __forceinline__ void load_split(const char* src, uint32_t plane,
                                           const RowOffsets<typename P::S>& o, typename P::T* p,
                                           const Physics& ph) {
    using S = typename P::S;
    constexpr VelSet<D> V = kVelSet<D>;
    static_for<0, VelSet<D>::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr Vel v = V.v[i];
        constexpr int kx = PULL ? v.x + 3 : 3, ky = PULL ? v.y + 3 : 3, kz = PULL ? v.z + 3 : 3;
        const char* base = src + (size_t)(2 * i) * plane + o.yo[ky] + o.zo[kz];
        p[i] = from_store<P>(load_at<S>(base, o.xo[kx]), ph, v.group);
    });
}

template <int D, class P>
__device__ __forceinline__ void store_split(char* dst, uint32_t plane,
                                            const RowOffsets<typename P::S>& o,
                                            const typename P::T* p, const Physics& ph) {
    constexpr VelSet<D> V = kVelSet<D>;
    char* row = dst + o.row;
    static_for<0, VelSet<D>::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const auto x = to_store<P>(p[i], ph, V.v[i].group);
        if constexpr (sizeof(typename P::S) == 2)
            store_cached(row + (size_t)(2 * i) * plane, o.own, x);
        else
            store_at(row + (size_t)(2 * i) * plane, o.own, x);
    });
}


// Half storage, one lane per cell.  The lane holds its cell's 107 (D3Q107) or
// 37 (D2Q37) g/h words -- g in the low half, h in the high half -- loaded and
// stored as whole 32-bit words, a wave's access covering 64 cells (256
// bytes).  A value is converted where it is used, by the conversions of
// from_store and to_store (one mixed-precision FMA with the weight), so each
// population goes through exactly the arithmetic of the other layouts; only
// the float is formed twice (moment sums, then relaxation) instead of being
// kept, which keeps 214 values in 107 registers.  The relaxed value goes
// straight back into its half of the word (v_fma_mixlo/mixhi_f16 leave the
// other half as it is).  volatile: a conversion must not be merged with the
// other one of the same word, which would keep the float live.
template <bool HI>
__device__ __forceinline__ float half_of(uint32_t w, float scale) {
    float x;
    if constexpr (HI)
        asm volatile("v_fma_mix_f32 %0, %1, %2, 0 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
                     : "=v"(x) : "v"(w), "s"(scale));
    else
        asm volatile("v_fma_mix_f32 %0, %1, %2, 0 op_sel_hi:[1,0,0]"
                     : "=v"(x) : "v"(w), "s"(scale));
    return x;
}

template <bool HI>
__device__ __forceinline__ void set_half(uint32_t& w, float v, float inv_scale) {
    if constexpr (HI)
        asm volatile("v_fma_mixhi_f16 %0, %1, %2, 0 op_sel_hi:[0,0,0]"
                     : "+v"(w) : "v"(v), "s"(inv_scale));
    else
        asm volatile("v_fma_mixlo_f16 %0, %1, %2, 0 op_sel_hi:[0,0,0]"
                     : "+v"(w) : "v"(v), "s"(inv_scale));
}

// g (k = 0, low half) and h (k = 1, high half) of the lane's words.
template <int D>
struct PairAcc {
    uint32_t* w;
    const Physics& ph;
    template <int K, int I>
    __device__ __forceinline__ float get() const {
        return half_of<K == 1>(w[I], ph.wf[kVelSet<D>.v[I].group]);
    }
    template <int K, int I>
    __device__ __forceinline__ void set(float v) const {
        set_half<K == 1>(w[I], v, ph.inv_wf[kVelSet<D>.v[I].group]);
    }
};

// Pull, collide and store one cell in the lane layout: F64 and F32Dev as
// g[] and h[] arrays, half storage as g/h words.
template <int D, class P>
__device__ __forceinline__ void step_lane_cell(const char* src, char* dst, uint32_t plane,
                                               const RowOffsets<typename P::S>& o,
                                               const Physics& ph) {
    using T = typename P::T;
    constexpr int Q = VelSet<D>::Q;
    if constexpr (P::kScaled) {
        constexpr VelSet<D> V = kVelSet<D>;
        uint32_t w[Q];
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr Vel v = V.v[i];
            const char* base = src + (size_t)(2 * i) * plane + o.yo[v.y + 3] + o.zo[v.z + 3];
            w[i] = load_at<uint32_t>(base, o.xo[v.x + 3]);
        });
        collide_lane_acc<D, P, false, true>(PairAcc<D>{w, ph}, ph);
        char* row = dst + o.row;
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            store_at(row + (size_t)(2 * i) * plane, o.own, w[i]);
        });
    } else {
        T g[Q], h[Q];
        load_lane<D, P>(src, plane, o, g, h, ph);
        collide_lane<D, P>(g, h, ph);
        store_lane<D, P>(dst, plane, o, g, h, ph);
    }
}

// ---------------------------------------------------------------------------
// The finite-difference form (Sec. III): after the collision (which already
// took the centre term), each population loses the neighbour terms of its
// third-order upwind-biased convection, read from the time-n state:
//   dt xi_a d(p)/dx_a = (dt r / 6) |e_a| [p(x - 2s) - 6 p(x - s) + 3 p(x) + 2 p(x + s)],
// s = sign(e_a), per axis with e_a != 0 (the stencil leans against the
// flow).  Neighbour x + d along an axis is offset index 3 - d (offsets hold
// x - e for e = -3..3, wrapped or clamped like the pull).

// Neighbour part  sum_a |e_a| [p(x - 2s) - 6 p(x - s) + 2 p(x + s)]  of
// population V at the plane starting at `sp`.
template <int D, class P, int I>
__device__ __forceinline__ typename P::T fd_neighbours(const char* sp,
                                                       const RowOffsets<typename P::S>& o,
                                                       const Physics& ph) {
    using T = typename P::T;
    using S = typename P::S;
    constexpr Vel v = kVelSet<D>.v[I];
    T nb = T(0);
    static_for<0, D>([&](auto A) {
        constexpr int a = decltype(A)::value;
        constexpr int e = a == 0 ? v.x : (a == 1 ? v.y : v.z);
        if constexpr (e != 0) {
            constexpr int s = e > 0 ? 1 : -1;
            constexpr int m = e > 0 ? e : -e;
            auto at = [&](auto Dd) {
                constexpr int d = decltype(Dd)::value;
                const uint32_t xo = a == 0 ? o.xo[3 - d] : o.xo[3];
                const uint32_t yo = a == 1 ? o.yo[3 - d] : o.yo[3];
                const uint32_t zo = a == 2 ? o.zo[3 - d] : o.zo[3];
                return from_store<P>(load_at<S>(sp + yo + zo, xo), ph, v.group);
            };
            const T far = at(std::integral_constant<int, -2 * s>{});
            const T near = at(std::integral_constant<int, -s>{});
            const T ahead = at(std::integral_constant<int, s>{});
            nb += T(m) * ((far - T(6) * near) + T(2) * ahead);
        }
    });
    return nb;
}

template <int D, class P>
__device__ __forceinline__ void convect_store_split(const char* src, char* dst, uint32_t plane,
                                                    const RowOffsets<typename P::S>& o,
                                                    const typename P::T* p, const Physics& ph) {
    using T = typename P::T;
    constexpr VelSet<D> V = kVelSet<D>;
    const T cs = fd_scale<T>(ph);
    char* row = dst + o.row;
    static_for<0, VelSet<D>::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const char* sp = src + (size_t)(2 * i) * plane;
        const T nb = fd_neighbours<D, P, i>(sp, o, ph);
        store_at(row + (size_t)(2 * i) * plane, o.own,
                 to_store<P>(p[i] - cs * nb, ph, V.v[i].group));
    });
}

template <int D, class P>
__device__ __forceinline__ void convect_store_lane(const char* src, char* dst, uint32_t plane,
                                                   const RowOffsets<typename P::S>& o,
                                                   const typename P::T* g,
                                                   const typename P::T* h, const Physics& ph) {
    using T = typename P::T;
    constexpr VelSet<D> V = kVelSet<D>;
    const T cs = fd_scale<T>(ph);
    char* row = dst + o.row;
    static_for<0, VelSet<D>::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int grp = V.v[i].group;
        const char* sp = src + (size_t)(2 * i) * plane;
        const T nbg = fd_neighbours<D, P, i>(sp, o, ph);
        const T nbh = fd_neighbours<D, P, i>(sp + h_offset(sizeof(typename P::S), plane), o, ph);
        char* base = row + (size_t)(2 * i) * plane;
        store_at(base, o.own, to_store<P>(g[i] - cs * nbg, ph, grp));
        store_at(base + h_offset(sizeof(typename P::S), plane), o.own,
                 to_store<P>(h[i] - cs * nbh, ph, grp));
    });
}

}  // namespace core
}  // namespace lbm

// The finite-difference form of Sec. III in two passes per step.
//
// The fused kernel (k_fd_step in kernels.hip) reads each population's
// upwind neighbours from cache.  At D3Q107 the rows around the cells in
// flight on one XCD, over all 214 planes, exceed its L2, so neighbour rows
// are fetched from HBM again and again.  Here a step is split:
//
//   moments pass  one lane per cell streams the 2Q centre values once,
//                 keeping only running sums, and writes a per-cell record:
//                 the macroscopic state, kappa rho of the energy-conserving
//                 collision, and (FP32 deviation storage) the residuals of
//                 the exact-moment correction of the targets;
//   update passes one lane per cell, a chunk of populations per launch:
//                 the chunk's targets from the record, relaxation with
//                 rates dt / tau and the upwind convection, whose neighbour
//                 rows -- a chunk's planes only -- stay in the L2.  Where
//                 rows are whole 256-cell tiles, a workgroup stages each
//                 population's stencil rows in LDS with 16-byte loads
//                 (k_fd_update_lds); otherwise each lane reads its stencil
//                 from global memory (k_fd_update).  Each pass also adds its
//                 new populations' moment sums into a per-cell accumulator,
//                 and the last one turns the totals into the next step's
//                 record, so the moments pass runs only after the state
//                 was set from outside (init) or by a fused step.
//
// The arithmetic is that of the fused kernel: the same equilibrium, the
// same target sums for the correction (accumulated in the same order), the
// same relaxation and convection terms.
#include <type_traits>

#include "lbm_internal.h"
#include "step_core.h"

namespace lbm {
namespace {

using namespace core;

// Record fields, each a plane (stride P, the population planes' stride) of
// values in the arithmetic type:
//   0 drho (deviation storage) or rho; 1..D u; D+1 t = T - 1; D+2 kappa rho;
//   deviation storage only: D+3 dm_g, D+4 .. 2D+3 dj_g, 2D+4 de_g, 2D+5 dm_h.
template <int D, bool DEV>
constexpr int kRecFields = DEV ? 2 * D + 6 : D + 3;
// After the record: the running moment sums of the new state, s0, sj (D),
// se and sh (sum of h), accumulated chunk by chunk.  Its read-modify-write
// per chunk (48 B per cell in FP64) costs less than the moments pass it
// saves, a read of every population: D3Q107 256^3 FP64 19.7 ms against 23.3
// ms per step with the six chunks below (with 8 narrower chunks and the
// one-lane update kernel it was the other way round, 32.0 against 30.4).
template <int D>
constexpr int kAccFields = D + 3;

// Population chunks of the update passes: the rest and axis populations
// (which take the correction) with the first pairs, then 21 at a time in 3D
// (6 launches) and the other 24 in 2D (2 launches).  Wider chunks read the
// record and the accumulator fewer times; 28 in 3D was slower again
// (measured at 256^3).
template <int D>
constexpr int kChunk0 = D == 2 ? 13 : 15;
template <int D>
constexpr int kChunkW = D == 2 ? 24 : 21;
template <int D>
constexpr int chunk_count() {
    constexpr int Q = VelSet<D>::Q;
    return 1 + (Q - kChunk0<D> + kChunkW<D> - 1) / kChunkW<D>;
}
template <int D>
constexpr int chunk_begin(int c) { return c == 0 ? 0 : kChunk0<D> + (c - 1) * kChunkW<D>; }
template <int D>
constexpr int chunk_end(int c) {
    constexpr int Q = VelSet<D>::Q;
    const int e = kChunk0<D> + c * kChunkW<D>;
    return c == 0 ? kChunk0<D> : (e < Q ? e : Q);
}

// Uncorrected targets' moment sums and the residuals of the exact-moment
// correction (as relax<…, DEV> forms them: per +- pair, group by group,
// then the rest population).
template <int D, typename T>
__device__ __forceinline__ void target_residuals(const Equilibrium<D, T, true>& eq,
                                                 const Physics& a, T arho, T beta, T want_m,
                                                 const T* want_j, T want_e, T je_on, T& dm,
                                                 T* dj, T& de) {
#pragma clang fp contract(off)
    constexpr VelSet<D> V = kVelSet<D>;
    constexpr int G = VelSet<D>::G;
    T sm = 0, sjx = 0, sjy = 0, sjz = 0, se = 0;
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
            T tp, tm;
            pair_targets(A0, A1, A2, c, w, arho, beta, tp, tm);
            const T sum = tp + tm;
            const T dif = tp - tm;
            sm += sum;
            if constexpr (v.x != 0) sjx = fmadd(T(v.x), dif, sjx);
            if constexpr (v.y != 0) sjy = fmadd(T(v.y), dif, sjy);
            if constexpr (D == 3 && v.z != 0) sjz = fmadd(T(v.z), dif, sjz);
            se = fmadd(T(V.qn[g]), sum, se);
        });
    });
    T A0, A1, A2;
    eq.template coef<0>(A0, A1, A2);
    sm += rest_target(A0, weight<T>(a, 0), arho, beta);
    dm = want_m - sm;
    de = je_on * (want_e - se);
    dj[0] = je_on * (want_j[0] - sjx);
    dj[1] = je_on * (want_j[1] - sjy);
    if constexpr (D == 3) dj[2] = je_on * (want_j[2] - sjz);
}

// The record of one cell from its moment sums (g: s0, sj, se; h: sh).
template <int D, class P>
__device__ __forceinline__ void write_record(typename P::T s0, typename P::T sx,
                                             typename P::T sy, typename P::T sz,
                                             typename P::T se, typename P::T sh,
                                             typename P::T* __restrict__ rec, int64_t N,
                                             int64_t cell, const Physics& ph) {
    using T = typename P::T;
    constexpr bool DEV = P::kDev;
    T sj[3] = {sx, sy, sz};
    T rho, drho, u[3] = {0, 0, 0}, t;
    macro<D, T, DEV>(s0, sj, se, sh, T(ph.r), ph.inv_dof, ph.half_delta, rho, drho, u, t);
    Equilibrium<D, T, DEV> eq;
    eq.setup(u, t, T(ph.r));
    const T want_e = (rho * eq.U + T(D) * (drho + rho * t)) / eq.r2;
    const T kr = energy_fix_kr<D, T, DEV>(ph, rho, eq, want_e, se);
    rec[cell] = DEV ? drho : rho;
#pragma unroll
    for (int k = 0; k < D; ++k) rec[(size_t)(1 + k) * N + cell] = u[k];
    rec[(size_t)(D + 1) * N + cell] = t;
    rec[(size_t)(D + 2) * N + cell] = kr;
    if constexpr (DEV) {
        const T hd = T(ph.half_delta);
        const T hdT = hd * (T(1) + t);
        T dm, dj[3] = {0, 0, 0}, de;
        target_residuals<D, T>(eq, ph, rho, drho, drho, sj, want_e, T(1), dm, dj, de);
        rec[(size_t)(D + 3) * N + cell] = dm;
#pragma unroll
        for (int k = 0; k < D; ++k) rec[(size_t)(D + 4 + k) * N + cell] = dj[k];
        rec[(size_t)(2 * D + 4) * N + cell] = de;
        T dmh, djh[3] = {0, 0, 0}, deh;
        target_residuals<D, T>(eq, ph, hdT * rho + kr, hdT * drho + hd * t + kr,
                               hd * (drho + rho * t) + kr, sj, T(0), T(0), dmh, djh, deh);
        rec[(size_t)(2 * D + 5) * N + cell] = dmh;
    }
}

template <int D, class P>
__global__ __launch_bounds__(256) void k_fd_moments(const void* __restrict__ src_v,
                                                    typename P::T* __restrict__ rec,
                                                    int64_t cells, int64_t N,
                                                    const Physics ph) {
    using T = typename P::T;
    using S = typename P::S;
    constexpr VelSet<D> V = kVelSet<D>;
    constexpr int Q = VelSet<D>::Q;
    const int64_t cell = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (cell >= cells) return;  // lanes are independent here (N: the plane stride)
    const S* src = static_cast<const S*>(src_v);
    // running sums over the centre values (moment_sums, streamed)
    T s0 = 0, sx = 0, sy = 0, sz = 0, se = 0, sh = 0;
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr Vel v = V.v[i];
        const T x = from_store<P>(src[(size_t)(2 * i) * N + cell], ph, v.group);
        const T y = from_store<P>(src[(size_t)(2 * i + 1) * N + cell], ph, v.group);
        s0 += x;
        if constexpr (v.x != 0) sx += T(v.x) * x;
        if constexpr (v.y != 0) sy += T(v.y) * x;
        if constexpr (D == 3 && v.z != 0) sz += T(v.z) * x;
        if constexpr (V.qn[v.group] != 0) se += T(V.qn[v.group]) * x;
        sh += y;
    });
    write_record<D, P>(s0, sx, sy, sz, se, sh, rec, N, cell, ph);
}

// Sweep order of the update passes (2.5D blocking).  A tile is 256 cells of
// one x-row.  The rows are cut into y sub-bands of fd_yb rows, dealt to the
// XCDs round-robin (sub-band s to XCD s % 8, which is workgroup b % 8); an
// XCD sweeps each of its sub-bands x-chunk (fd_w tiles) by x-chunk, and
// within a chunk z-slab by z-slab, row by row.  The planes a stencil reads
// at y +- 1, 2 and z +- 1, 2 were then fetched by the same XCD within the
// last few sub-band slabs, which the host sizes to stay in its L2.  Returns
// false for the padding workgroups of the last round.
__device__ __forceinline__ bool sweep_tile(const StepArgs& a, int b, int& xt, int& cy, int& cz) {
    const int W = a.fd_w, YB = a.fd_yb;
    const int chunks = (a.tiles_per_row + W - 1) / W;
    const int per_chunk = W * YB * a.nz;
    const int per_sub = chunks * per_chunk;
    const int j = b >> 3;
    const int round = j / per_sub;
    const int in_sub = j - round * per_sub;
    const int chunk = in_sub / per_chunk;
    const int in_chunk = in_sub - chunk * per_chunk;
    cz = in_chunk / (YB * W);
    const int in_slab = in_chunk - cz * (YB * W);
    cy = (round * 8 + (b & 7)) * YB + in_slab / W;
    xt = chunk * W + in_slab % W;
    return xt < a.tiles_per_row && cy < a.ny;
}

// One cell of an update pass over populations [C0, C1): the record's
// macroscopic state and equilibrium, the correction residuals (first chunk
// only: it holds the rest and axis populations that take them), and the
// running moment sums of the new populations.  Both update kernels run
// these steps in this order; they differ only in where a stencil's stored
// values come from.
template <int D, class P, int C0, int C1>
struct FdCell {
    using T = typename P::T;
    using S = typename P::S;
    static constexpr bool DEV = P::kDev;
    Equilibrium<D, T, DEV> eq;
    T rho, arho_h, beta_g, beta_h, omf, omg, cs;
    T dm = 0, de = 0, dmh = 0, dj[3] = {0, 0, 0};
    T a0 = 0, ax = 0, ay = 0, az = 0, ae = 0, ah = 0;

    __device__ __forceinline__ void load(const T* __restrict__ rec, int64_t N, int64_t cell,
                                         const Physics& ph) {
        const T m0 = rec[cell];
        T u[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < D; ++k) u[k] = rec[(size_t)(1 + k) * N + cell];
        const T t = rec[(size_t)(D + 1) * N + cell];
        // kappa rho is zero unless the energy-conserving collision is on
        const T kr = ph.ec != 0 ? rec[(size_t)(D + 2) * N + cell] : T(0);
        rho = DEV ? T(1) + m0 : m0;
        const T drho = DEV ? m0 : m0 - T(1);
        eq.setup(u, t, T(ph.r));
        const T hd = T(ph.half_delta);
        const T hdT = hd * (T(1) + t);
        arho_h = hdT * rho + kr;
        beta_g = DEV ? drho : T(0);
        beta_h = DEV ? hdT * drho + hd * t + kr : T(0);
        if constexpr (DEV && C0 == 0) {
            dm = rec[(size_t)(D + 3) * N + cell];
#pragma unroll
            for (int k = 0; k < D; ++k) dj[k] = rec[(size_t)(D + 4 + k) * N + cell];
            de = rec[(size_t)(2 * D + 4) * N + cell];
            dmh = rec[(size_t)(2 * D + 5) * N + cell];
        }
        omf = T(ph.omega_f);
        omg = T(ph.omega_g);
        cs = fd_scale<T>(ph);
    }

    // Population i: target (uncorrected w (arho P~(c) + beta), +- pair
    // arithmetic, plus the correction on the rest and axis populations),
    // relaxation with the convection centre term (relax<..., FD>), neighbour
    // terms (fd_neighbours), store.  at(dist, axis, d) is the stored value
    // of distribution dist (0: g, 1: h) at the neighbour x + d along axis
    // (d = 0: the cell itself).
    template <int i, class At>
    __device__ __forceinline__ void update(const Physics& ph, At&& at, S* __restrict__ dst,
                                           int64_t N, int64_t cell) {
        constexpr VelSet<D> V = kVelSet<D>;
        constexpr Vel v = V.v[i];
        constexpr int g = v.group;
        T A0, A1, A2;
        eq.template coef<V.qn[g]>(A0, A1, A2);
        const T w = weight<T>(ph, g);
        // the targets exactly as relax<...> and target_residuals form them
        T tg, th;
        if constexpr (i == 0) {
            tg = rest_target(A0, w, rho, beta_g);
            th = rest_target(A0, w, arho_h, beta_h);
        } else {
            constexpr int first = (i - group_start<D>(g)) % 2 == 0 ? i : i - 1;
            constexpr Vel vf = V.v[first];
            const T c = eq.template dot<vf.x, vf.y, vf.z>();
            T gp, gm, hp, hm;
            pair_targets(A0, A1, A2, c, w, rho, beta_g, gp, gm);
            pair_targets(A0, A1, A2, c, w, arho_h, beta_h, hp, hm);
            tg = i == first ? gp : gm;
            th = i == first ? hp : hm;
        }
        if constexpr (DEV && i == 0) {
            tg += dm - de;
            th += dmh;
        }
        if constexpr (DEV && i >= 1 && i <= 2 * D) {
            constexpr int axis = v.x != 0 ? 0 : (v.y != 0 ? 1 : 2);
            constexpr int s = (v.x + v.y + v.z) > 0 ? 1 : -1;
            const T half = T(0.5) * dj[axis];
            tg += s > 0 ? de * T(1.0 / (2 * D)) + half : de * T(1.0 / (2 * D)) - half;
        }
        using Z = std::integral_constant<int, 0>;
        using G = std::integral_constant<int, 0>;
        using H = std::integral_constant<int, 1>;
        T xg = from_store<P>(at(G{}, Z{}, Z{}), ph, g);
        T xh = from_store<P>(at(H{}, Z{}, Z{}), ph, g);
        if constexpr (l1_of(v) != 0) {
            const T kc = T(3 * l1_of(v)) * cs;
            xg = relax_value(xg, tg, omf, kc);
            xh = relax_value(xh, th, omg, kc);
        } else {
            xg = relax_value(xg, tg, omf);
            xh = relax_value(xh, th, omg);
        }
        T nbg = T(0), nbh = T(0);
        static_for<0, D>([&](auto A) {
            constexpr int ax_ = decltype(A)::value;
            constexpr int e = ax_ == 0 ? v.x : (ax_ == 1 ? v.y : v.z);
            if constexpr (e != 0) {
                constexpr int s = e > 0 ? 1 : -1;
                constexpr int m = e > 0 ? e : -e;
                using M2 = std::integral_constant<int, -2 * s>;
                using M1 = std::integral_constant<int, -s>;
                using P1 = std::integral_constant<int, s>;
                nbg += T(m) * ((from_store<P>(at(G{}, A, M2{}), ph, g) -
                                T(6) * from_store<P>(at(G{}, A, M1{}), ph, g)) +
                               T(2) * from_store<P>(at(G{}, A, P1{}), ph, g));
                nbh += T(m) * ((from_store<P>(at(H{}, A, M2{}), ph, g) -
                                T(6) * from_store<P>(at(H{}, A, M1{}), ph, g)) +
                               T(2) * from_store<P>(at(H{}, A, P1{}), ph, g));
            }
        });
        const T ng = xg - cs * nbg;
        const T nh = xh - cs * nbh;
        const size_t pg_off = (size_t)(2 * i) * N, ph_off = pg_off + N;
        store_at(reinterpret_cast<char*>(dst + pg_off), (uint32_t)(cell * sizeof(S)),
                 to_store<P>(ng, ph, g));
        store_at(reinterpret_cast<char*>(dst + ph_off), (uint32_t)(cell * sizeof(S)),
                 to_store<P>(nh, ph, g));
        {
            a0 += ng;
            if constexpr (v.x != 0) ax += T(v.x) * ng;
            if constexpr (v.y != 0) ay += T(v.y) * ng;
            if constexpr (D == 3 && v.z != 0) az += T(v.z) * ng;
            if constexpr (V.qn[g] != 0) ae += T(V.qn[g]) * ng;
            ah += nh;
        }
    }

    // Running sums: the first chunk starts them, the last turns the totals
    // into the next step's record (this lane has read its cell's record).
    __device__ __forceinline__ void finish(T* __restrict__ rec, int64_t N, int64_t cell,
                                           const Physics& ph) {
        {
            T* acc = rec + (size_t)kRecFields<D, DEV> * N;
            T sums[6] = {a0, ax, ay, az, ae, ah};
            constexpr int kSlots[6] = {0, 1, 2, D == 3 ? 3 : -1, D + 1, D + 2};
            if constexpr (C0 != 0) {
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    if (kSlots[k] >= 0) sums[k] += acc[(size_t)kSlots[k] * N + cell];
            }
            if constexpr (C1 == VelSet<D>::Q) {
                write_record<D, P>(sums[0], sums[1], sums[2], sums[3], sums[4], sums[5], rec, N,
                                   cell, ph);
            } else {
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    if (kSlots[k] >= 0) acc[(size_t)kSlots[k] * N + cell] = sums[k];
            }
        }
    }
};

// Update of populations [C0, C1) of every cell, one lane per cell, the
// stencil values read straight from global memory (through L1/L2).
template <int D, class P, int C0, int C1>
__global__ __launch_bounds__(256) void k_fd_update(const void* __restrict__ src_v,
                                                   void* __restrict__ dst_v,
                                                   typename P::T* __restrict__ rec,
                                                   const StepArgs a) {
    using S = typename P::S;
    const int64_t N = a.P;  // plane stride (record and populations)
    int xt, cy, cz;
    if (!sweep_tile(a, (int)blockIdx.x, xt, cy, cz)) return;
    const int cx = xt * 256 + (int)threadIdx.x;
    if (cx >= a.nx) return;
    const int64_t cell = (int64_t)cx + (int64_t)a.nx * cy + (int64_t)a.nxy * cz;
    const Physics& ph = a.ph;
    PullTable<D> pt;  // pt.src for shift e gives the cell at x - e (wrapped or clamped)
    pt.fill(cx, cy, cz, a.nx, a.ny, a.nz, a.nxy, a.open_end, true);
    const S* src = static_cast<const S*>(src_v);
    S* dst = static_cast<S*>(dst_v);
    FdCell<D, P, C0, C1> c;
    c.load(rec, N, cell, ph);
    static_for<C0, C1>([&](auto I) {
        constexpr int i = decltype(I)::value;
        // offset of the neighbour x + d along axis ax of this cell
        auto at = [&](auto Dist, auto Ax, auto Dd) {
            constexpr int ax = decltype(Ax)::value;
            constexpr int d = decltype(Dd)::value;
            constexpr int dist = decltype(Dist)::value;
            int o = ax == 0 ? pt.x[3 - d] : pt.x[3];
            o += ax == 1 ? pt.y[3 - d] : pt.y[3];
            if constexpr (D == 3) o += ax == 2 ? pt.z[3 - d] : pt.z[3];
            return src[(size_t)(2 * i + dist) * N + o];
        };
        c.template update<i>(ph, at, dst, N, cell);
    });
    c.finish(rec, N, cell, ph);
}

// LDS-staged update, for rows of whole tiles (nx a multiple of 256).  The
// one-lane-per-cell kernel issues a 4-byte load per stencil point, about
// eight per population and cell; its counters show the vector memory
// address unit busy 80-98% of the time while HBM is not saturated.  Here a
// workgroup serves one 256-cell tile and, per phase of kFdPhase
// populations, loads the rows their stencils read -- the tile's own row
// with two cells of halo either side, and the three upwind-biased rows
// along y and along z where a population moves along them -- four cells a
// lane (one 16-byte load per row and wave in FP32), stages them in LDS, and
// each lane takes its cell's stencil values from there.  The arithmetic is
// FdCell's, as in k_fd_update.
//
// LDS per population: the centre rows of g and h (264 slots each: two
// unused, two halo, 256 cells, two halo, two unused, so the cells start at a
// 16-byte boundary), then up to 12 neighbour rows of 256 (3 per moving axis
// y, z and per distribution).
template <int D>
constexpr int kLdsCentre = 264;
template <int D>
constexpr int kLdsSlots = 2 * kLdsCentre<D> + (D == 3 ? 12 : 6) * 256;
// Populations staged per barrier phase: two for D3Q107 in FP32 (2% faster at
// 256^3), one otherwise (two were 1-3.5% slower: FP64 needs twice the LDS and
// 190-209 VGPRs, and D2Q37 rows are fewer).
template <int D, class P>
constexpr int kFdPhase = (D == 3 && sizeof(typename P::S) == 4) ? 2 : 1;

// Stencil rows of population i staged per phase: the g and h centre rows,
// then per moving axis (y first) and distribution the rows at -2s, -s, +s.
template <int D>
constexpr int fd_rows(int i) {
    const Vel v = kVelSet<D>.v[i];
    return 2 + 6 * ((v.y != 0 ? 1 : 0) + (D == 3 && v.z != 0 ? 1 : 0));
}

template <int D, class P, int C0, int C1, int PB>
__global__ __launch_bounds__(256) void k_fd_update_lds(const void* __restrict__ src_v,
                                                       void* __restrict__ dst_v,
                                                       typename P::T* __restrict__ rec,
                                                       const StepArgs a) {
    using S = typename P::S;
    typedef S S4 __attribute__((ext_vector_type(4)));
    constexpr VelSet<D> V = kVelSet<D>;
    constexpr int CW = kLdsCentre<D>;
    constexpr int SL = kLdsSlots<D>;  // LDS slots of one population
    static_assert(PB == 1 || PB == 2, "one or two populations per phase");
    __shared__ __attribute__((aligned(16))) S lds[PB * SL];
    const int64_t N = a.P;  // plane stride (record and populations)
    int xt, cy, cz;
    // the whole workgroup leaves together (it meets at barriers below)
    if (!sweep_tile(a, (int)blockIdx.x, xt, cy, cz)) return;
    const int tid = (int)threadIdx.x;
    // wave-uniform, in a scalar register: the row loads below branch on it
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int x0 = xt * 256;
    const int64_t cell = (int64_t)(x0 + tid) + (int64_t)a.nx * cy + (int64_t)a.nxy * cz;
    const Physics& ph = a.ph;
    const bool open_x = a.open_end & 1u, open_y = a.open_end & 2u, open_z = a.open_end & 4u;
    // starts (cells) of the tile's part of its own row and of rows y + d and
    // z + d, d = -2, -1, 1, 2: wave-uniform, computed once
    const int64_t own = (int64_t)a.nx * cy + (int64_t)a.nxy * cz + x0;
    int64_t ys[4], zs[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int d = k < 2 ? k - 2 : k - 1;
        ys[k] = own + (int64_t)(pull_coord(cy, -d, a.ny, open_y) - cy) * a.nx;
        zs[k] = D == 3 ? own + (int64_t)(pull_coord(cz, -d, a.nz, open_z) - cz) * a.nxy : own;
    }
    // halo cells x0 - 2, x0 - 1, x0 + 256, x0 + 257 of the tile's row (lanes 0..3)
    const int hsh = lane < 2 ? 2 - lane : -254 - lane;  // pull shift e: source x0 - e
    const int64_t halo_src = (int64_t)pull_coord(x0, hsh, a.nx, open_x) - x0;
    const int halo_slot = lane < 2 ? 2 + lane : 258 + lane;  // slots 2, 3, 260, 261
    const S* src = static_cast<const S*>(src_v);
    S* dst = static_cast<S*>(dst_v);
    // A phase stages PB populations.  Its rows, population by population, are
    // numbered R = 0, 1, ...; wave w loads rows w, w + 4, ..., picked branch-
    // free.  The next phase's loads are issued before this one is computed
    // and land in LDS after the barrier that ends this phase's reads.  The
    // halo of population j's distribution d is loaded by wave 2 j + d.
    constexpr int kMaxSets = (14 * PB + 3) / 4;
    S4 q[kMaxSets];
    int slot[kMaxSets];
    bool has[kMaxSets];
    S hv = S(0);
    bool halo = false;
    int halo_at = 0;
    auto issue = [&](auto Ph) {
        constexpr int i0 = C0 + PB * decltype(Ph)::value;
        constexpr int np = (C1 - i0) < PB ? (C1 - i0) : PB;
        constexpr int nr0 = fd_rows<D>(i0);
        constexpr int nrows = nr0 + (np > 1 ? fd_rows<D>(i0 + 1) : 0);
        // phase row R: its start in global memory and its LDS slot
        auto row_of = [&](auto RR, const S*& ptr, int& sl) {
            constexpr int R = decltype(RR)::value;
            constexpr int j = R < nr0 ? 0 : 1;
            constexpr int i = i0 + j;
            constexpr int r = R - (j ? nr0 : 0);
            constexpr Vel v = V.v[i];
            constexpr bool my = v.y != 0;
            constexpr int sy = v.y > 0 ? 1 : -1, sz = v.z > 0 ? 1 : -1;
            if constexpr (r < 2) {
                ptr = src + (size_t)(2 * i + r) * N + own;
                sl = j * SL + r * CW + 4;
            } else {
                constexpr int k = (r - 2) % 3;         // -2s, -s, +s
                constexpr int dist = ((r - 2) / 3) % 2;
                constexpr bool along_y = my && (r - 2) < 6;
                constexpr int sg = along_y ? sy : sz;
                constexpr int d = k == 0 ? -2 * sg : (k == 1 ? -sg : sg);
                constexpr int kk = d < 0 ? d + 2 : d + 1;  // index in ys / zs
                ptr = src + (size_t)(2 * i + dist) * N + (along_y ? ys[kk] : zs[kk]);
                sl = j * SL + 2 * CW + (r - 2) * 256;
            }
        };
        static_for<0, kMaxSets>([&](auto M) {
            constexpr int m = decltype(M)::value;
            const S* ptr = nullptr;
            int sl = 0;
            static_for<0, 4>([&](auto W) {
                constexpr int R = 4 * m + decltype(W)::value;
                if constexpr (R < nrows) {
                    const S* pr;
                    int sr;
                    row_of(std::integral_constant<int, R>{}, pr, sr);
                    ptr = wave == decltype(W)::value ? pr : ptr;
                    sl = wave == decltype(W)::value ? sr : sl;
                }
            });
            has[m] = 4 * m + 3 < nrows || ptr != nullptr;
            slot[m] = sl;
            if (has[m]) q[m] = *reinterpret_cast<const S4*>(ptr + 4 * lane);
        });
        // halo: population j = wave / 2, distribution wave % 2
        const int j = wave >> 1, dist = wave & 1;
        constexpr bool hx0 = V.v[i0].x != 0;
        constexpr bool hx1 = np > 1 && V.v[np > 1 ? i0 + 1 : i0].x != 0;
        const bool need = j == 0 ? hx0 : (j == 1 ? hx1 : false);
        halo = need && lane < 4;
        halo_at = j * SL + dist * CW + halo_slot;
        if (halo) hv = src[(size_t)(2 * (i0 + j) + dist) * N + own + halo_src];
    };
    FdCell<D, P, C0, C1> c;
    c.load(rec, N, cell, ph);
    constexpr int kPhases = (C1 - C0 + PB - 1) / PB;
    issue(std::integral_constant<int, 0>{});
    static_for<0, kPhases>([&](auto Ph) {
        constexpr int phz = decltype(Ph)::value;
        constexpr int i0 = C0 + PB * phz;
        constexpr int np = (C1 - i0) < PB ? (C1 - i0) : PB;
        if constexpr (phz != 0) __syncthreads();  // the previous phase's reads are done
#pragma unroll
        for (int m = 0; m < kMaxSets; ++m)
            if (has[m]) *reinterpret_cast<S4*>(lds + slot[m] + 4 * lane) = q[m];
        if (halo) lds[halo_at] = hv;
        __syncthreads();
        if constexpr (phz + 1 < kPhases) issue(std::integral_constant<int, phz + 1>{});
        static_for<0, np>([&](auto J) {
            constexpr int j = decltype(J)::value;
            constexpr int i = i0 + j;
            constexpr Vel v = V.v[i];
            constexpr bool my = v.y != 0;
            constexpr int sy = v.y > 0 ? 1 : -1, sz = v.z > 0 ? 1 : -1;
            const S* base = lds + j * SL;
            auto at = [&](auto Dist, auto Ax, auto Dd) {
                constexpr int dist = decltype(Dist)::value;
                constexpr int ax = decltype(Ax)::value;
                constexpr int d = decltype(Dd)::value;
                if constexpr (d == 0 || ax == 0) {
                    return base[dist * CW + 4 + tid + d];
                } else {
                    constexpr int s = ax == 1 ? sy : sz;
                    constexpr int k = d == -2 * s ? 0 : (d == -s ? 1 : 2);
                    constexpr int blk = (ax == 2 && my) ? 2 : 0;  // y's rows come first
                    return base[2 * CW + (3 * (blk + dist) + k) * 256 + tid];
                }
            };
            c.template update<i>(ph, at, dst, N, cell);
        });
    });
    c.finish(rec, N, cell, ph);
}

template <int D, class P, int C>
hipError_t launch_chunks(const StepArgs& a, typename P::T* rec, int grid, hipStream_t s) {
    if constexpr (C == chunk_count<D>()) {
        return hipSuccess;
    } else {
        // rows of whole tiles: the LDS-staged kernel (its 16-byte row loads
        // need every row to start on a tile boundary)
        constexpr int c0 = chunk_begin<D>(C), c1 = chunk_end<D>(C);
        hipError_t e =
            a.nx % 256 == 0
                ? launch_kernel(&k_fd_update_lds<D, P, c0, c1, kFdPhase<D, P>>, dim3(grid),
                                dim3(256), s, a.src, a.dst, rec, a)
                : launch_kernel(&k_fd_update<D, P, c0, c1>, dim3(grid), dim3(256), s, a.src,
                                a.dst, rec, a);
        if (e != hipSuccess) return e;
        return launch_chunks<D, P, C + 1>(a, rec, grid, s);
    }
}

// Bytes of the planes that one update chunk's stencils keep live: the
// reuse window (the slabs z-2 .. z+2 of a sub-band's x-chunk in 3D, the rows
// y-2 .. y+2 of an x-chunk in 2D) is held within this much of an XCD's L2.
constexpr int64_t kFdWindowBytes = 2 << 20;

template <int D, class P>
hipError_t fd_two_pass_impl(const StepArgs& a0, void* rec_v, bool record_valid, hipStream_t s) {
    using T = typename P::T;
    StepArgs a = a0;
    T* rec = static_cast<T*>(rec_v);
    const int tiles = (int)((a.N + 255) / 256);
    if (!record_valid) {
        hipError_t e = launch_kernel(&k_fd_moments<D, P>, dim3(tiles), dim3(256), s, a.src, rec,
                                     a.N, a.P, a.ph);
        if (e != hipSuccess) return e;
    }
    // one x-row tile of one chunk's planes (at most 14 populations, g and h)
    const int64_t tile_bytes = 256LL * 2 * kChunkW<D> * (int64_t)sizeof(typename P::S);
    a.tiles_per_row = (a.nx + 255) / 256;
    // tiles in a reuse window; D3Q107 FP64 gets twice the bytes (3% faster
    // at 256^3; D2Q37 FP64 was 5% slower with it, and 1.5x was slower in 3D)
    const int64_t window = (D == 3 && sizeof(typename P::S) == 8) ? 2 * kFdWindowBytes
                                                                   : kFdWindowBytes;
    int64_t budget = window / (5 * tile_bytes);
    if (budget < 1) budget = 1;
    if (D == 3) {
        // x-chunks of whole rows when they fit, sub-bands of YB rows: the
        // window is 5 slabs of YB x W tiles
        a.fd_w = (int)(a.tiles_per_row < budget ? a.tiles_per_row : budget);
        // the tallest sub-band within the window that splits y into k
        // rounds of eight (every XCD takes the same number of sub-bands)
        const int64_t max_yb = budget / a.fd_w;
        int k = 1;
        while ((a.ny + 8 * k - 1) / (8 * k) > max_yb && 8 * k < a.ny) ++k;
        a.fd_yb = (a.ny + 8 * k - 1) / (8 * k);
    } else {
        // one sub-band per XCD; the window is 5 rows of a W-tile chunk
        a.fd_w = (int)(a.tiles_per_row < budget ? a.tiles_per_row : budget);
        a.fd_yb = (a.ny + 7) / 8;
    }
    const int chunks = (a.tiles_per_row + a.fd_w - 1) / a.fd_w;
    const int subs = (a.ny + a.fd_yb - 1) / a.fd_yb;
    const int rounds = (subs + 7) / 8;
    const int64_t grid = 8LL * rounds * chunks * a.fd_w * a.fd_yb * a.nz;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    return launch_chunks<D, P, 0>(a, rec, (int)grid, s);
}

}  // namespace

size_t fd_record_bytes(int dim, int precision, int64_t P) {
    const bool dev = precision != LBM_FP64;  // record (deviation storage: residuals too)
    const int fields = dim == 2 ? (dev ? kRecFields<2, true> : kRecFields<2, false>) + kAccFields<2>
                                : (dev ? kRecFields<3, true> : kRecFields<3, false>) + kAccFields<3>;
    return (size_t)fields * (size_t)P * (precision == LBM_FP64 ? 8 : 4);
}

hipError_t launch_fd_two_pass(int dim, int precision, const StepArgs& a, void* record,
                              bool record_valid, hipStream_t s) {
    if (precision == LBM_FP64)
        return dim == 2 ? fd_two_pass_impl<2, F64>(a, record, record_valid, s)
                        : fd_two_pass_impl<3, F64>(a, record, record_valid, s);
    if (precision == LBM_FP32_DEV)
        return dim == 2 ? fd_two_pass_impl<2, F32Dev>(a, record, record_valid, s)
                        : fd_two_pass_impl<3, F32Dev>(a, record, record_valid, s);
    return hipErrorInvalidValue;
}

}  // namespace lbm

// HIP kernels for gfx950: initialisation, the fused collide-and-stream step,
// and the FP64 readout / conservation reductions.
//
// Data layout in HBM (one ping-pong side): [Q][2][N] -- for population i the
// g plane (N values, x fastest) and then the h plane.  Every plane is read
// once and written once per step: one HBM read and one HBM write per
// population per cell.
//
// The step (Sec. II reduced BGK equations, Sec. IV equilibrium, lattice time
// step of Sec. V) at cell x:
//   1. pull   g_i(x) <- g_i'(x - e_i), h_i likewise (periodic wrap, or clamp
//             at a zero-gradient end), straight from the other ping-pong side;
//   2. moments rho = sum g_i, rho u = r sum e_i g_i,
//             rho E = r^2/2 sum |e_i|^2 g_i + sum h_i, T from
//             E = u^2/2 + (D + delta) T / 2;
//   3. equilibrium F_i = w_i rho P(c_i), c_i = xi_i . u, P the 4th-order
//             Hermite polynomial, evaluated as even/odd parts per +/- pair;
//   4. relax  g_i' = g_i + (F_i - g_i)/tau_f,
//             h_i' = h_i + ((delta/2) T F_i - h_i)/tau_g;
//   5. store  g_i', h_i' at x (coalesced).
#include <tuple>
#include <type_traits>
#include <utility>

#include "lbm_internal.h"

namespace lbm {
namespace {

// Launch with the launch's own status (hipLaunchKernel), so that an error
// left behind by unrelated work in the process is not taken for ours.
template <typename... KArgs, typename... Args>
hipError_t launch_kernel(void (*kernel)(KArgs...), dim3 grid, dim3 block, hipStream_t s,
                         Args&&... args) {
    std::tuple<std::decay_t<KArgs>...> vals(std::forward<Args>(args)...);
    void* ptrs[sizeof...(KArgs) > 0 ? sizeof...(KArgs) : 1];
    std::apply([&](auto&... v) {
        int i = 0;
        ((ptrs[i++] = static_cast<void*>(&v)), ...);
    }, vals);
    return hipLaunchKernel(reinterpret_cast<const void*>(kernel), grid, block, ptrs, 0, s);
}

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

// First velocity index of group g (velocities are ordered group by group).
template <int D>
constexpr int group_start(int g) {
    int s = 0;
    for (int k = 0; k < g; ++k) s += kVelSet<D>.count[k];
    return s;
}

// Group weight in the arithmetic type (kernel arguments carry both).
template <typename T>
__device__ __forceinline__ T weight(const StepArgs& a, int g);
template <>
__device__ __forceinline__ double weight<double>(const StepArgs& a, int g) { return a.w[g]; }
template <>
__device__ __forceinline__ float weight<float>(const StepArgs& a, int g) { return a.wf[g]; }

// Moment sums over one set of Q populations p (scaled lattice units):
// s0 = sum p, sj = sum e p, se = sum |e|^2 p.
template <int D, typename T>
__device__ __forceinline__ void moment_sums(const T* p, T& s0, T* sj, T& se) {
    constexpr VelSet<D> V = kVelSet<D>;
    constexpr int Q = VelSet<D>::Q;
    T a0 = 0, ax = 0, ay = 0, az = 0, ae = 0;
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr Vel v = V.v[i];
        const T x = p[i];
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
template <int D, typename T, bool DEV>
__device__ __forceinline__ void relax(T* p, const Equilibrium<D, T, DEV>& eq,
                                      const StepArgs& a, T arho, T beta, T omega, T want_m,
                                      const T* want_j, T want_e, T je_on) {
    constexpr VelSet<D> V = kVelSet<D>;
    constexpr int G = VelSet<D>::G;
    static_assert(V.v[1].group == 1 && V.v[2 * D].group == 1 && V.v[2 * D + 1].group == 2,
                  "the axis populations must follow the rest population");
    T sm = 0, sjx = 0, sjy = 0, sjz = 0, se = 0;
    T t1[2 * D];  // targets of the axis populations, corrected below
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
            const T c2 = c * c;
            const T even = A0 + c2 * (A2 + c2 * T(1.0 / 24.0));
            const T odd = c * (A1 + c2 * T(1.0 / 6.0));
            const T tp = w * (arho * (even + odd) + beta);
            const T tm = w * (arho * (even - odd) + beta);
            if constexpr (DEV) {
                const T sum = tp + tm;
                const T dif = tp - tm;
                sm += sum;
                if constexpr (v.x != 0) sjx += T(v.x) * dif;
                if constexpr (v.y != 0) sjy += T(v.y) * dif;
                if constexpr (D == 3 && v.z != 0) sjz += T(v.z) * dif;
                se += T(V.qn[g]) * sum;
            }
            if constexpr (DEV && g == 1) {
                t1[i - 1] = tp;
                t1[i] = tm;
            } else {
                p[i] = p[i] + omega * (tp - p[i]);
                p[i + 1] = p[i + 1] + omega * (tm - p[i + 1]);
            }
        });
    });
    T A0, A1, A2;
    eq.template coef<0>(A0, A1, A2);
    T t0 = weight<T>(a, 0) * (arho * A0 + beta);
    if constexpr (DEV) {
        sm += t0;
        const T dm = want_m - sm;
        const T de = je_on * (want_e - se);
        const T dj[3] = {je_on * (want_j[0] - sjx), je_on * (want_j[1] - sjy),
                         D == 3 ? je_on * (want_j[2] - sjz) : T(0)};
        t0 += dm - de;
        const T de_axis = de * T(1.0 / (2 * D));
        static_for<0, D>([&](auto I) {
            constexpr int k = decltype(I)::value;
            constexpr Vel v = V.v[1 + 2 * k];  // +e_axis (first of its pair)
            constexpr int axis = v.x != 0 ? 0 : (v.y != 0 ? 1 : 2);
            const T half = T(0.5) * dj[axis];
            const T tp = t1[2 * k] + de_axis + half;
            const T tm = t1[2 * k + 1] + de_axis - half;
            p[1 + 2 * k] = p[1 + 2 * k] + omega * (tp - p[1 + 2 * k]);
            p[2 + 2 * k] = p[2 + 2 * k] + omega * (tm - p[2 + 2 * k]);
        });
    }
    p[0] = p[0] + omega * (t0 - p[0]);
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
// Work item of one wave: a segment of L consecutive cells of one grid row
// (fixed y and z).  y, z and every pull offset along them are therefore
// wave-uniform and live in scalar registers; per lane only the seven x
// offsets (shifts -3..3, wrapped or clamped) are held.  Each population
// load is then one scalar base plus one of those seven lane offsets.

template <typename T>
struct RowOffsets {
    uint32_t xo[7];  // per lane
    uint32_t yo[7];  // wave-uniform
    uint32_t zo[7];  // wave-uniform
    uint32_t own;    // per lane: byte offset of the lane's own cell in its row
    uint32_t row;    // wave-uniform: byte offset of the row start
};

// Decode the wave's row segment; returns false if the wave has no work.
template <int D, typename T, int L>
__device__ __forceinline__ bool row_item(const StepArgs& a, int lane_cell, uint32_t role_off,
                                         RowOffsets<T>& o, bool& active) {
    // Which row segment this wave serves.  The hardware deals workgroups to
    // the eight XCDs round-robin by id.  With xcd_rows set, workgroup b runs
    // turn j = b / 8 on XCD b % 8, and the turns of one XCD walk whole rows
    // (row = 8 (j / tiles_per_row) + b % 8): all segments of a row share one
    // L2, so the cache lines that x-shifted pulls share between neighbouring
    // segments are fetched from HBM once, while the eight XCDs together still
    // sweep one compact band of rows.  Without it (few rows), segments go
    // out in plain launch order.
    const int wave = (int)(threadIdx.x >> 6);
    int seg, row;
    if (a.xcd_rows) {
        const int b = (int)blockIdx.x;
        const int j = b >> 3;
        row = (j / a.tiles_per_row) * 8 + (b & 7);
        seg = (j % a.tiles_per_row) * 4 + wave;
        if (row >= a.rows || seg >= a.segs) return false;
    } else {
        const int item = (int)blockIdx.x * 4 + wave;
        if (item >= a.items) return false;
        seg = item % a.segs;
        row = item / a.segs;
    }
    seg = __builtin_amdgcn_readfirstlane(seg);
    row = __builtin_amdgcn_readfirstlane(row);
    const int y = row % a.ny;
    const int z = row / a.ny;
    const int xr = seg * L + lane_cell;
    active = xr < a.nx;
    const int x = active ? xr : a.nx - 1;
    const bool stream = a.stream != 0;
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        const int e = stream ? k - 3 : 0;
        o.xo[k] = (uint32_t)pull_coord(x, e, a.nx, a.open_end & 1u) * (uint32_t)sizeof(T) + role_off;
        o.yo[k] = (uint32_t)(pull_coord(y, e, a.ny, a.open_end & 2u) * a.nx) * (uint32_t)sizeof(T);
        if constexpr (D == 3)
            o.zo[k] = (uint32_t)(pull_coord(z, e, a.nz, a.open_end & 4u) * a.nxy) *
                      (uint32_t)sizeof(T);
        else
            o.zo[k] = 0;
    }
    o.own = (uint32_t)x * (uint32_t)sizeof(T) + role_off;
    o.row = (uint32_t)(y * a.nx + z * a.nxy) * (uint32_t)sizeof(T);
    return true;
}

// Fused step, one lane per cell: the lane holds all 2Q populations.  A wave
// serves 64 cells of one row.
template <int D, typename T, bool DEV, int WAVES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES, 8)))
void k_step(const StepArgs a) {
    constexpr VelSet<D> V = kVelSet<D>;
    constexpr int Q = VelSet<D>::Q;
    RowOffsets<T> o;
    bool active;
    if (!row_item<D, T, 64>(a, (int)threadIdx.x & 63, 0u, o, active)) return;

    const uint32_t plane = (uint32_t)a.N * (uint32_t)sizeof(T);
    const char* src = static_cast<const char*>(a.src);
    T g[Q], h[Q];
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr Vel v = V.v[i];
        const char* base = src + (size_t)(2 * i) * plane + o.yo[v.y + 3] + o.zo[v.z + 3];
        g[i] = load_at<T>(base, o.xo[v.x + 3]);
        h[i] = load_at<T>(base + plane, o.xo[v.x + 3]);
    });

    T s0, sj[3] = {0, 0, 0}, se, sh, dummy_j[3], dummy_e;
    moment_sums<D, T>(g, s0, sj, se);
    moment_sums<D, T>(h, sh, dummy_j, dummy_e);
    T rho, drho, u[3] = {0, 0, 0}, t;
    macro<D, T, DEV>(s0, sj, se, sh, T(a.r), a.inv_dof, a.half_delta, rho, drho, u, t);
    Equilibrium<D, T, DEV> eq;
    eq.setup(u, t, T(a.r));
    const T hd = T(a.half_delta);
    const T hdT = hd * (T(1) + t);
    // BGK targets: F for g; (delta/2) T F for h (shifted by the rest state in
    // deviation storage); exact target moments for the correction
    const T beta_g = DEV ? drho : T(0);
    const T beta_h = DEV ? hdT * drho + hd * t : T(0);
    const T want_e = (rho * eq.U + T(D) * (drho + rho * t)) / eq.r2;
    relax<D, T, DEV>(g, eq, a, rho, beta_g, T(a.omega_f), drho, sj, want_e, T(1));
    relax<D, T, DEV>(h, eq, a, hdT * rho, beta_h, T(a.omega_g), hd * (drho + rho * t), sj,
                     T(0), T(0));

    // Lanes past the end of a ragged row hold the row's last cell (clamped),
    // loaded and updated exactly like the lane that owns it, so they store
    // the same bits to the same place.  No branch: a branch here lets the
    // compiler sink the whole relaxation into the store block and keep every
    // target and population live at once.
    (void)active;
    char* dst = static_cast<char*>(a.dst) + o.row;
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        char* base = dst + (size_t)(2 * i) * plane;
        store_at<T>(base, o.own, g[i]);
        store_at<T>(base + plane, o.own, h[i]);
    });
}

// Fused step, split layout: a wave serves 32 cells of one row; lane l < 32
// holds the g populations of cell l, lane l + 32 the h populations of the
// same cell.  The moment sums are exchanged between the two halves
// (lane ^ 32), both halves evaluate the same equilibrium, each relaxes its own
// distribution.  This halves the registers a lane needs (Q instead of 2Q
// values).
template <int D, typename T, bool DEV, int WAVES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES, 8)))
void k_step_split(const StepArgs a) {
    constexpr VelSet<D> V = kVelSet<D>;
    constexpr int Q = VelSet<D>::Q;
    const int lane = (int)threadIdx.x & 63;
    const int role = lane >> 5;  // 0: g, 1: h
    const uint32_t plane = (uint32_t)a.N * (uint32_t)sizeof(T);
    RowOffsets<T> o;
    bool active;
    if (!row_item<D, T, 32>(a, lane & 31, role ? plane : 0u, o, active)) return;

    const char* src = static_cast<const char*>(a.src);
    T p[Q];
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr Vel v = V.v[i];
        const char* base = src + (size_t)(2 * i) * plane + o.yo[v.y + 3] + o.zo[v.z + 3];
        p[i] = load_at<T>(base, o.xo[v.x + 3]);
    });

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
    macro<D, T, DEV>(g0, gj, ge, sh, T(a.r), a.inv_dof, a.half_delta, rho, drho, u, t);
    Equilibrium<D, T, DEV> eq;
    eq.setup(u, t, T(a.r));
    const T hd = T(a.half_delta);
    const T hdT = hd * (T(1) + t);
    const T arho = role ? hdT * rho : rho;
    const T beta = DEV ? (role ? hdT * drho + hd * t : drho) : T(0);
    const T want_e = (rho * eq.U + T(D) * (drho + rho * t)) / eq.r2;
    const T want_m = role ? hd * (drho + rho * t) : drho;
    relax<D, T, DEV>(p, eq, a, arho, beta, role ? T(a.omega_g) : T(a.omega_f), want_m, gj,
                     want_e, role ? T(0) : T(1));

    // tail lanes store their clamped cell's identical update (see k_step)
    (void)active;
    char* dst = static_cast<char*>(a.dst) + o.row;
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        store_at<T>(dst + (size_t)(2 * i) * plane, o.own, p[i]);
    });
}

// ---------------------------------------------------------------------------
// Initial state S_0 = equilibrium of (rho, u, T), evaluated in double and
// stored in the storage precision (deviation from the rest equilibrium in
// FP32_DEV: g_i - w_i, h_i - (delta/2) w_i).
template <int D, typename T, bool DEV>
__global__ __launch_bounds__(256) void k_init(char* dst, const double* __restrict__ rho_in,
                                              const double* __restrict__ u_in,
                                              const double* __restrict__ T_in, int64_t N,
                                              double half_delta, double r, const WGroups wg) {
    constexpr VelSet<D> V = kVelSet<D>;
    constexpr int Q = VelSet<D>::Q;
    const int64_t cell = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (cell >= N) return;
    const double rho = rho_in[cell];
    const double temp = T_in[cell];
    double u[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < D; ++k) u[k] = u_in[k * N + cell];
    Equilibrium<D, double, true> eq;  // deviation form, in double
    eq.setup(u, temp - 1.0, r);
    const double hdT = half_delta * temp;
    const size_t plane = (size_t)N * sizeof(T);
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr Vel v = V.v[i];
        double A0, A1, A2;  // A0 is A0 - 1 (deviation form)
        eq.template coef<V.qn[v.group]>(A0, A1, A2);
        const double c = eq.template dot<v.x, v.y, v.z>();
        const double pm1 = A0 + c * (A1 + c * (A2 + c * (1.0 / 6.0 + c * (1.0 / 24.0))));
        const double w = wg.w[v.group];
        const double Fdev = w * (rho * pm1 + (rho - 1.0));  // F_i - w_i
        double gv, hv;
        if constexpr (DEV) {
            gv = Fdev;
            hv = hdT * Fdev + half_delta * w * (temp - 1.0);  // H_i - (delta/2) w_i
        } else {
            gv = Fdev + w;
            hv = hdT * (Fdev + w);
        }
        char* base = dst + (size_t)(2 * i) * plane;
        reinterpret_cast<T*>(base)[cell] = T(gv);
        reinterpret_cast<T*>(base + plane)[cell] = T(hv);
    });
}

// ---------------------------------------------------------------------------
// Readout of S_n in double: per-cell rho, u, E and/or per-workgroup partial
// totals (rho, rho u, rho E), reduced across the wave and the workgroup in a
// fixed order.
template <int D, typename T, bool DEV>
__global__ __launch_bounds__(kReadBlock) void k_readout(const ReadArgs a) {
    constexpr VelSet<D> V = kVelSet<D>;
    constexpr int Q = VelSet<D>::Q;
    constexpr int NT = D + 2;
    const int64_t cell = (int64_t)blockIdx.x * kReadBlock + threadIdx.x;
    double tot[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) tot[k] = 0.0;
    if (cell < a.N) {
        int x, y, z;
        coords((int)cell, a.nx, a.nxy, x, y, z);
        PullTable<D> pt;
        pt.fill(x, y, z, a.nx, a.ny, a.nz, a.nxy, a.open_end, a.stream != 0);
        const uint32_t plane = (uint32_t)a.N * (uint32_t)sizeof(T);
        const char* src = static_cast<const char*>(a.src);
        double s0 = 0, sj[3] = {0, 0, 0}, se = 0, sh = 0;
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr Vel v = V.v[i];
            const uint32_t off = (uint32_t)pt.template src<v.x, v.y, v.z>() * (uint32_t)sizeof(T);
            const char* base = src + (size_t)(2 * i) * plane;
            const double gv = (double)load_at<T>(base, off);
            const double hv = (double)load_at<T>(base, off + plane);
            s0 += gv;
            if constexpr (v.x != 0) sj[0] += double(v.x) * gv;
            if constexpr (v.y != 0) sj[1] += double(v.y) * gv;
            if constexpr (D == 3 && v.z != 0) sj[2] += double(v.z) * gv;
            se += double(V.qn[v.group]) * gv;
            sh += hv;
        });
        const double rho = DEV ? 1.0 + s0 : s0;
        const double rhoE = 0.5 * a.r * a.r * se + sh + (DEV ? a.rest_energy : 0.0);
        tot[0] = rho;
#pragma unroll
        for (int k = 0; k < D; ++k) tot[1 + k] = a.r * sj[k];
        tot[D + 1] = rhoE;
        if (a.rho) a.rho[cell] = rho;
        if (a.u) {
#pragma unroll
            for (int k = 0; k < D; ++k) a.u[k * a.N + cell] = tot[1 + k] / rho;
        }
        if (a.E) a.E[cell] = rhoE / rho;
    }
    if (!a.partials) return;
    // wave reduction (fixed butterfly), then across the 4 waves in order
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        double v = tot[k];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
        tot[k] = v;
    }
    __shared__ double wsum[kReadBlock / 64][NT];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < NT; ++k) wsum[wave][k] = tot[k];
    }
    __syncthreads();
    if (threadIdx.x < NT) {
        double v = 0.0;
        for (int w = 0; w < kReadBlock / 64; ++w) v += wsum[w][threadIdx.x];
        a.partials[(int64_t)blockIdx.x * NT + threadIdx.x] = v;
    }
}

// Final pass: one workgroup sums the partials in a fixed order.
template <int NT>
__global__ __launch_bounds__(256) void k_final_reduce(const double* __restrict__ partials,
                                                      int blocks, double* out) {
    __shared__ double sm[256][NT];
    double acc[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < blocks; b += 256) {
#pragma unroll
        for (int k = 0; k < NT; ++k) acc[k] += partials[(int64_t)b * NT + k];
    }
#pragma unroll
    for (int k = 0; k < NT; ++k) sm[threadIdx.x][k] = acc[k];
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int k = 0; k < NT; ++k) sm[threadIdx.x][k] += sm[threadIdx.x + s][k];
        }
        __syncthreads();
    }
    if (threadIdx.x < NT) out[threadIdx.x] = sm[0][threadIdx.x];
}

template <int D, typename T, bool DEV>
hipError_t step_impl(bool split, const StepArgs& a0, hipStream_t s) {
    StepArgs a = a0;
    const int L = split ? 32 : 64;  // cells per wave
    a.segs = (a.nx + L - 1) / L;
    a.rows = a.ny * a.nz;
    a.items = a.segs * a.rows;
    a.tiles_per_row = (a.segs + 3) / 4;  // four waves (segments) per workgroup
    // whole rows per XCD once there are enough rows to keep all eight busy
    a.xcd_rows = a.rows >= 64 ? 1 : 0;
    const int grid = a.xcd_rows ? 8 * a.tiles_per_row * ((a.rows + 7) / 8) : (a.items + 3) / 4;
    // Occupancy hint for the split D3Q107 FP32 kernel: asking for at least
    // two waves per SIMD gave 4% more bandwidth than the compiler's own
    // choice (three waves at 162 VGPRs); the other kernels run best as
    // compiled.
    constexpr int kSplitWaves = (D == 3 && sizeof(T) == 4) ? 2 : 1;
    if (split)
        return launch_kernel(&k_step_split<D, T, DEV, kSplitWaves>, dim3(grid), dim3(256), s, a);
    else
        return launch_kernel(&k_step<D, T, DEV, 1>, dim3(grid), dim3(256), s, a);
}

}  // namespace

hipError_t launch_init(int dim, int precision, void* dst, const double* rho,
                       const double* u, const double* T, int64_t N, double half_delta,
                       double r, const double* w_group, hipStream_t s) {
    WGroups wg;
    for (int k = 0; k < 10; ++k) wg.w[k] = w_group[k];
    const int grid = (int)((N + 255) / 256);
    char* d = static_cast<char*>(dst);
    if (dim == 2 && precision == LBM_FP64)
        return launch_kernel(&k_init<2, double, false>, dim3(grid), dim3(256), s, d, rho, u, T, N, half_delta, r, wg);
    else if (dim == 2)
        return launch_kernel(&k_init<2, float, true>, dim3(grid), dim3(256), s, d, rho, u, T, N, half_delta, r, wg);
    else if (precision == LBM_FP64)
        return launch_kernel(&k_init<3, double, false>, dim3(grid), dim3(256), s, d, rho, u, T, N, half_delta, r, wg);
    else
        return launch_kernel(&k_init<3, float, true>, dim3(grid), dim3(256), s, d, rho, u, T, N, half_delta, r, wg);
}

hipError_t launch_step(int dim, int precision, bool split, const StepArgs& a, hipStream_t s) {
    if (dim == 2 && precision == LBM_FP64) return step_impl<2, double, false>(split, a, s);
    if (dim == 2) return step_impl<2, float, true>(split, a, s);
    if (precision == LBM_FP64) return step_impl<3, double, false>(split, a, s);
    return step_impl<3, float, true>(split, a, s);
}

int step_block_cells(int, int, bool split) { return split ? 128 : 256; }

hipError_t launch_readout(int dim, int precision, const ReadArgs& a, int blocks, hipStream_t s) {
    if (dim == 2 && precision == LBM_FP64)
        return launch_kernel(&k_readout<2, double, false>, dim3(blocks), dim3(kReadBlock), s, a);
    else if (dim == 2)
        return launch_kernel(&k_readout<2, float, true>, dim3(blocks), dim3(kReadBlock), s, a);
    else if (precision == LBM_FP64)
        return launch_kernel(&k_readout<3, double, false>, dim3(blocks), dim3(kReadBlock), s, a);
    else
        return launch_kernel(&k_readout<3, float, true>, dim3(blocks), dim3(kReadBlock), s, a);
}

hipError_t launch_final_reduce(int dim, const double* partials, int blocks, double* out,
                               hipStream_t s) {
    if (dim == 2)
        return launch_kernel(&k_final_reduce<4>, dim3(1), dim3(256), s, partials, blocks, out);
    else
        return launch_kernel(&k_final_reduce<5>, dim3(1), dim3(256), s, partials, blocks, out);
}

}  // namespace lbm

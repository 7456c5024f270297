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
#include <type_traits>

#include "lbm_internal.h"

namespace lbm {
namespace {

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

template <typename T>
__device__ __forceinline__ void store_at(char* base, uint32_t byte_off, T v) {
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

// Logical tile of this workgroup.  Workgroups are dispatched to the eight
// XCDs round-robin by id; this gives each XCD one contiguous range of tiles,
// so the x-neighbour lines that shifted reads share land in the same L2.
__device__ __forceinline__ int logical_tile(int tiles_per_xcd) {
    const int b = blockIdx.x;
    return (b & 7) * tiles_per_xcd + (b >> 3);
}

// Cell -> (x, y, z).
__device__ __forceinline__ void coords(int cell, int nx, int nxy, int& x, int& y,
                                       int& z) {
    z = cell / nxy;
    const int rem = cell - z * nxy;
    y = rem / nx;
    x = rem - y * nx;
}

// Shell coefficients of the 4th-order equilibrium polynomial for one cell.
//   P(c) = A0 + A1 c + A2 c^2 + c^3/6 + c^4/24  with, for |xi|^2 = q,
//   A0 - 1 = (-U + t(q-D))/2 + (3U^2 + 6t(D+2-q)U + 3t^2(q^2-2(D+2)q+D(D+2)))/24
//   A1 = 1 - U/2 + t(q-D-2)/2,  A2 = 1/2 - U/4 + t(q-D-4)/4,
// U = |u|^2, t = T - 1.  F_i = a_g P~ + b_g and H_i = hdT F_i + c_g, where
// P~ = P (FP64) or P - 1 (deviation storage, so that the rest part w_i is
// never formed in float).
template <int D, typename T, bool DEV>
struct Equilibrium {
    static constexpr int G = VelSet<D>::G;
    T A0[G], A1[G], A2[G], a[G], b[G], c[G];
    T ru[3];
    T hdT;

    __device__ __forceinline__ void setup(T rho, T drho, const T* u, T t, T r,
                                          T half_delta, const double* wg) {
        constexpr VelSet<D> V = kVelSet<D>;
        const T U = D == 3 ? u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
                           : u[0] * u[0] + u[1] * u[1];
        const T r2 = r * r;
#pragma unroll
        for (int k = 0; k < D; ++k) ru[k] = r * u[k];
        hdT = half_delta * (T(1) + t);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const T q = r2 * T(V.qn[g]);
            const T Dd = T(D);
            const T a0m1 = T(0.5) * (t * (q - Dd) - U) +
                           T(1.0 / 24.0) * (T(3) * U * U + T(6) * t * (Dd + T(2) - q) * U +
                                            T(3) * t * t * (q * q - T(2) * (Dd + T(2)) * q +
                                                            Dd * (Dd + T(2))));
            A0[g] = DEV ? a0m1 : T(1) + a0m1;
            A1[g] = T(1) - T(0.5) * U + T(0.5) * t * (q - Dd - T(2));
            A2[g] = T(0.5) - T(0.25) * U + T(0.25) * t * (q - Dd - T(4));
            const T w = T(wg[g]);
            a[g] = w * rho;
            b[g] = DEV ? w * drho : T(0);
            c[g] = DEV ? half_delta * w * t : T(0);
        }
    }
};

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

// Relax one set of populations toward alpha F_i + beta_g with rate omega.
// For g: alpha = 1, beta = b; for h: alpha = hdT, beta = hdT b + c.
template <int D, typename T, bool DEV>
__device__ __forceinline__ void relax(T* p, const Equilibrium<D, T, DEV>& eq,
                                      T alpha, const T* beta, T omega) {
    constexpr VelSet<D> V = kVelSet<D>;
    constexpr int Q = VelSet<D>::Q;
    {  // rest population: c = 0
        const T F = eq.a[0] * eq.A0[0];
        p[0] = p[0] + omega * (alpha * F + beta[0] - p[0]);
    }
    static_for<0, (Q - 1) / 2>([&](auto I) {
        constexpr int i = 1 + 2 * decltype(I)::value;
        constexpr Vel v = V.v[i];
        constexpr int g = v.group;
        T c = T(0);
        if constexpr (v.x != 0) c += T(v.x) * eq.ru[0];
        if constexpr (v.y != 0) c += T(v.y) * eq.ru[1];
        if constexpr (D == 3 && v.z != 0) c += T(v.z) * eq.ru[2];
        const T c2 = c * c;
        const T even = eq.A0[g] + c2 * (eq.A2[g] + c2 * T(1.0 / 24.0));
        const T odd = c * (eq.A1[g] + c2 * T(1.0 / 6.0));
        const T Fp = eq.a[g] * (even + odd);
        const T Fm = eq.a[g] * (even - odd);
        p[i] = p[i] + omega * (alpha * Fp + beta[g] - p[i]);
        p[i + 1] = p[i + 1] + omega * (alpha * Fm + beta[g] - p[i + 1]);
    });
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
// Fused step, one lane per cell: the lane holds all 2Q populations.
template <int D, typename T, bool DEV>
__global__ __launch_bounds__(256) void k_step(const StepArgs a) {
    constexpr VelSet<D> V = kVelSet<D>;
    constexpr int Q = VelSet<D>::Q;
    constexpr int G = VelSet<D>::G;
    const int tile = logical_tile(a.tiles_per_xcd);
    if (tile >= a.tiles) return;
    const int cell = tile * 256 + (int)threadIdx.x;
    if (cell >= a.N) return;
    int x, y, z;
    coords(cell, a.nx, a.nxy, x, y, z);
    PullTable<D> pt;
    pt.fill(x, y, z, a.nx, a.ny, a.nz, a.nxy, a.open_end, a.stream != 0);

    const uint32_t plane = (uint32_t)a.N * (uint32_t)sizeof(T);
    const char* src = static_cast<const char*>(a.src);
    T g[Q], h[Q];
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr Vel v = V.v[i];
        const uint32_t off = (uint32_t)pt.template src<v.x, v.y, v.z>() * (uint32_t)sizeof(T);
        const char* base = src + (size_t)(2 * i) * plane;
        g[i] = load_at<T>(base, off);
        h[i] = load_at<T>(base, off + plane);
    });

    T s0, sj[3] = {0, 0, 0}, se, sh, dummy_j[3], dummy_e;
    moment_sums<D, T>(g, s0, sj, se);
    moment_sums<D, T>(h, sh, dummy_j, dummy_e);
    T rho, drho, u[3] = {0, 0, 0}, t;
    macro<D, T, DEV>(s0, sj, se, sh, T(a.r), a.inv_dof, a.half_delta, rho, drho, u, t);
    Equilibrium<D, T, DEV> eq;
    eq.setup(rho, drho, u, t, T(a.r), T(a.half_delta), a.w);

    T beta_g[G], beta_h[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
        beta_g[k] = eq.b[k];
        beta_h[k] = eq.hdT * eq.b[k] + eq.c[k];
    }
    relax<D, T, DEV>(g, eq, T(1), beta_g, T(a.omega_f));
    relax<D, T, DEV>(h, eq, eq.hdT, beta_h, T(a.omega_g));

    char* dst = static_cast<char*>(a.dst);
    const uint32_t own = (uint32_t)cell * (uint32_t)sizeof(T);
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        char* base = dst + (size_t)(2 * i) * plane;
        store_at<T>(base, own, g[i]);
        store_at<T>(base, own + plane, h[i]);
    });
}

// Fused step, split layout: a wave serves 32 cells; lane l < 32 holds the g
// populations of cell l, lane l + 32 the h populations of the same cell.
// The moment sums are exchanged between the two halves (lane ^ 32), both
// halves evaluate the same equilibrium, each relaxes its own distribution.
// This halves the registers a lane needs (Q instead of 2Q values).
template <int D, typename T, bool DEV>
__global__ __launch_bounds__(256) void k_step_split(const StepArgs a) {
    constexpr VelSet<D> V = kVelSet<D>;
    constexpr int Q = VelSet<D>::Q;
    constexpr int G = VelSet<D>::G;
    const int tile = logical_tile(a.tiles_per_xcd);
    if (tile >= a.tiles) return;  // whole workgroup leaves together
    const int lane = (int)threadIdx.x & 63;
    const int role = lane >> 5;  // 0: g, 1: h
    const int cell_raw = tile * 128 + ((int)threadIdx.x >> 6) * 32 + (lane & 31);
    const bool active = cell_raw < a.N;
    const int cell = active ? cell_raw : (int)a.N - 1;  // keep tail lanes in the exchange
    int x, y, z;
    coords(cell, a.nx, a.nxy, x, y, z);
    PullTable<D> pt;
    pt.fill(x, y, z, a.nx, a.ny, a.nz, a.nxy, a.open_end, a.stream != 0);

    const uint32_t plane = (uint32_t)a.N * (uint32_t)sizeof(T);
    const uint32_t role_off = role ? plane : 0u;
    const char* src = static_cast<const char*>(a.src);
    T p[Q];
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr Vel v = V.v[i];
        const uint32_t off = (uint32_t)pt.template src<v.x, v.y, v.z>() * (uint32_t)sizeof(T) + role_off;
        p[i] = load_at<T>(src + (size_t)(2 * i) * plane, off);
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
    eq.setup(rho, drho, u, t, T(a.r), T(a.half_delta), a.w);
    const T alpha = role ? eq.hdT : T(1);
    T beta[G];
#pragma unroll
    for (int k = 0; k < G; ++k) beta[k] = role ? eq.hdT * eq.b[k] + eq.c[k] : eq.b[k];
    relax<D, T, DEV>(p, eq, alpha, beta, role ? T(a.omega_g) : T(a.omega_f));

    if (!active) return;
    char* dst = static_cast<char*>(a.dst);
    const uint32_t own = (uint32_t)cell * (uint32_t)sizeof(T) + role_off;
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        store_at<T>(dst + (size_t)(2 * i) * plane, own, p[i]);
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
    eq.setup(rho, rho - 1.0, u, temp - 1.0, r, half_delta, wg.w);
    const size_t plane = (size_t)N * sizeof(T);
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr Vel v = V.v[i];
        constexpr int g = v.group;
        double c = 0.0;
        if constexpr (v.x != 0) c += double(v.x) * eq.ru[0];
        if constexpr (v.y != 0) c += double(v.y) * eq.ru[1];
        if constexpr (D == 3 && v.z != 0) c += double(v.z) * eq.ru[2];
        const double pm1 = eq.A0[g] + c * (eq.A1[g] + c * (eq.A2[g] + c * (1.0 / 6.0 + c * (1.0 / 24.0))));
        const double Fdev = eq.a[g] * pm1 + eq.b[g];      // F_i - w_i
        const double w = wg.w[g];
        const double F = Fdev + w;
        const double H = half_delta * temp * F;
        double gv, hv;
        if constexpr (DEV) {
            gv = Fdev;
            hv = eq.hdT * Fdev + eq.c[g];                 // H_i - (delta/2) w_i
        } else {
            gv = F;
            hv = H;
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
    const int cells_per_tile = split ? 128 : 256;
    a.tiles = (int)((a.N + cells_per_tile - 1) / cells_per_tile);
    a.tiles_per_xcd = (a.tiles + 7) / 8;
    const int grid = a.tiles_per_xcd * 8;
    if (split)
        hipLaunchKernelGGL((k_step_split<D, T, DEV>), dim3(grid), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_step<D, T, DEV>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
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
        hipLaunchKernelGGL((k_init<2, double, false>), dim3(grid), dim3(256), 0, s, d, rho, u, T, N, half_delta, r, wg);
    else if (dim == 2)
        hipLaunchKernelGGL((k_init<2, float, true>), dim3(grid), dim3(256), 0, s, d, rho, u, T, N, half_delta, r, wg);
    else if (precision == LBM_FP64)
        hipLaunchKernelGGL((k_init<3, double, false>), dim3(grid), dim3(256), 0, s, d, rho, u, T, N, half_delta, r, wg);
    else
        hipLaunchKernelGGL((k_init<3, float, true>), dim3(grid), dim3(256), 0, s, d, rho, u, T, N, half_delta, r, wg);
    return hipGetLastError();
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
        hipLaunchKernelGGL((k_readout<2, double, false>), dim3(blocks), dim3(kReadBlock), 0, s, a);
    else if (dim == 2)
        hipLaunchKernelGGL((k_readout<2, float, true>), dim3(blocks), dim3(kReadBlock), 0, s, a);
    else if (precision == LBM_FP64)
        hipLaunchKernelGGL((k_readout<3, double, false>), dim3(blocks), dim3(kReadBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_readout<3, float, true>), dim3(blocks), dim3(kReadBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_final_reduce(int dim, const double* partials, int blocks, double* out,
                               hipStream_t s) {
    if (dim == 2)
        hipLaunchKernelGGL((k_final_reduce<4>), dim3(1), dim3(256), 0, s, partials, blocks, out);
    else
        hipLaunchKernelGGL((k_final_reduce<5>), dim3(1), dim3(256), 0, s, partials, blocks, out);
    return hipGetLastError();
}

}  // namespace lbm

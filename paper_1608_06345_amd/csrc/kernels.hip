// HIP kernels for gfx950: initialisation, the fused collide-and-stream step,
// the fused finite-difference step (Sec. III; its two-pass form is in
// fd.hip), and the FP64 readout / conservation reductions.
//
// Data layout in HBM (one ping-pong side): population i owns a slab of 2 P
// values (P >= N, x fastest).  FP64 and FP32: the g plane, then the h plane
// ([Q][2][P]); half storage: the g and h halves of a cell side by side in
// one 32-bit word ([Q][P][2]; cell_bytes, h_offset).  Every value is read
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
// The D3Q107 step also comes with its pulled rows staged in LDS
// (k_step_split_lds, variant SPLIT_LDS): same results, measured slower.
#include <tuple>
#include <type_traits>
#include <utility>

#include "lbm_internal.h"
#include "step_core.h"

namespace lbm {
namespace {

using namespace core;

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
    fill_row_offsets<D, T>(o, x, y, z, a.nx, a.ny, a.nz, a.nxy, a.open_end, a.stream != 0,
                           role_off);
    return true;
}

// Fused step, one lane per cell: the lane holds all 2Q populations.  A wave
// serves 64 cells of one row.  P is the storage precision (F64, F32Dev,
// F16Dev).
template <int D, class P, int WAVES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES, 8)))
void k_step(const StepArgs a) {
    using T = typename P::T;
    using S = typename P::S;
    constexpr int Q = VelSet<D>::Q;
    RowOffsets<S> o;
    bool active;
    if (!row_item<D, S, 64>(a, (int)threadIdx.x & 63, 0u, o, active)) return;
    const uint32_t plane = (uint32_t)a.P * (uint32_t)sizeof(S);
    // Lanes past the end of a ragged row hold the row's last cell (clamped),
    // loaded and updated exactly like the lane that owns it, so they store
    // the same bits to the same place.  No branch: a branch here lets the
    // compiler sink the whole relaxation into the store block and keep every
    // target and population live at once.
    (void)active;
    step_lane_cell<D, P>(static_cast<const char*>(a.src), static_cast<char*>(a.dst), plane, o,
                         a.ph);
}

// Fused step, split layout (see collide_split): a wave serves 32 cells of
// one row.  This halves the registers a lane needs (Q instead of 2Q values).
template <int D, class P, int WAVES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES, 8)))
void k_step_split(const StepArgs a) {
    using T = typename P::T;
    using S = typename P::S;
    constexpr int Q = VelSet<D>::Q;
    const int lane = (int)threadIdx.x & 63;
    const int role = lane >> 5;  // 0: g, 1: h
    const uint32_t plane = (uint32_t)a.P * (uint32_t)sizeof(S);
    RowOffsets<S> o;
    bool active;
    if (!row_item<D, S, 32>(a, lane & 31, role ? h_offset(sizeof(S), plane) : 0u, o, active))
        return;
    T p[Q];
    load_split<D, P>(static_cast<const char*>(a.src), plane, o, p, a.ph);
    collide_split<D, P>(p, role, a.ph);
    // tail lanes store their clamped cell's identical update (see k_step)
    (void)active;
    store_split<D, P>(static_cast<char*>(a.dst), plane, o, p, a.ph);
}

// Fused step, split layout, with the pulled rows staged in LDS (D3Q107;
// rows of whole 128-cell tiles).  A workgroup serves one 128-cell tile of a
// row, its four waves 32 cells each as in k_step_split.  The pull of
// population i reads the tile's row shifted by e_i: row (y - e_y, z - e_z),
// cells x0 - e_x .. x0 - e_x + 127.  Instead of one 4-byte (or 2-byte) load
// per lane and population, the workgroup loads that row once with 4-cell
// loads per lane -- lanes 0..31 the g row, lanes 32..63 the h row, one
// instruction per population -- plus up to three halo cells either side,
// stages it in LDS, and each lane takes its cell's pulled value from there.
// Populations go through LDS in batches of kLdsBatch; the next batch's loads
// are issued before the current one is read back.  Collision and store are
// k_step_split's.
constexpr int kLdsBatch = 16;
constexpr int kLdsRow = 136;  // slots per staged row: 4 (3 halo), 128 cells, 4 (3 halo)

template <class P, int WAVES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES, 8)))
void k_step_split_lds(const StepArgs a) {
    constexpr int D = 3;
    using T = typename P::T;
    using S = typename P::S;
    typedef S S4 __attribute__((ext_vector_type(4)));
    typedef S S8 __attribute__((ext_vector_type(8)));
    // half storage: g/h words, two elements per cell (see cell_bytes)
    constexpr bool kPaired = sizeof(S) == 2;
    constexpr int64_t kCellElems = kPaired ? 2 : 1;
    constexpr VelSet<D> V = kVelSet<D>;
    constexpr int Q = VelSet<D>::Q;
    __shared__ __attribute__((aligned(16))) S lds[kLdsBatch * 2 * kLdsRow];
    // workgroup b: turn j = b / 8 on XCD b % 8 walks whole rows (as row_item)
    const int b = (int)blockIdx.x;
    const int j = b >> 3;
    const int row = (j / a.tiles_per_row) * 8 + (b & 7);
    if (row >= a.rows) return;  // the whole workgroup
    const int tile = j % a.tiles_per_row;
    const int y = row % a.ny, z = row / a.ny;
    const int x0 = tile * 128;
    const int tid = (int)threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int role = lane >> 5;  // 0: g, 1: h
    const int c = wave * 32 + (lane & 31);  // the lane's cell in the tile
    const bool open_x = a.open_end & 1u, open_y = a.open_end & 2u, open_z = a.open_end & 4u;
    const int64_t N = a.P;  // plane stride
    const S* src = static_cast<const S*>(a.src);
    // halo lanes (k = lane & 31 < 6): cells x0 - 3 .. x0 - 1, x0 + 128 .. x0 + 130
    const int hk = lane & 31;
    const int hshift = hk < 3 ? 3 - hk : -125 - hk;  // pull shift e: source x0 - e
    const int hx = pull_coord(x0, hshift, a.nx, open_x);
    const int hslot = hk < 3 ? 1 + hk : 129 + hk;  // slots 1..3, 132..134
    // Batch loads: wave w takes the batch's populations w, w + 4, ...
    S4 q[kLdsBatch / 4];
    S hv[kLdsBatch / 4];
    auto issue = [&](auto Bt) {
        constexpr int b0 = decltype(Bt)::value * kLdsBatch;
        static_for<0, kLdsBatch / 4>([&](auto M) {
            constexpr int m = decltype(M)::value;
            // population of this slot for each wave, picked branch-free
            int64_t start = 0;
            bool has = false, hx_need = false;
            static_for<0, 4>([&](auto W) {
                constexpr int i = b0 + 4 * m + decltype(W)::value;
                if constexpr (i < Q) {
                    constexpr Vel v = V.v[i];
                    const int64_t st =
                        (int64_t)(2 * i) * N +
                        kCellElems * ((int64_t)pull_coord(y, v.y, a.ny, open_y) * a.nx +
                                      (int64_t)pull_coord(z, v.z, a.nz, open_z) * a.nxy);
                    const bool w = wave == decltype(W)::value;
                    start = w ? st : start;
                    has = w ? true : has;
                    hx_need = w ? (v.x != 0) : hx_need;
                }
            });
            hv[m] = S(0);
            if (has) {
                if constexpr (kPaired) {
                    // four cells' g/h words (16 bytes); keep this lane's halves
                    const S* rowp = src + start;
                    const S8 pw = *reinterpret_cast<const S8*>(rowp + 2 * (x0 + 4 * (lane & 31)));
                    q[m] = role ? __builtin_shufflevector(pw, pw, 1, 3, 5, 7)
                                : __builtin_shufflevector(pw, pw, 0, 2, 4, 6);
                    if (hx_need && hk < 6) hv[m] = rowp[2 * hx + role];
                } else {
                    const S* rowp = src + start + (role ? N : 0);
                    q[m] = *reinterpret_cast<const S4*>(rowp + x0 + 4 * (lane & 31));
                    if (hx_need && hk < 6) hv[m] = rowp[hx];
                }
            }
        });
    };
    T p[Q];
    constexpr int kBatches = (Q + kLdsBatch - 1) / kLdsBatch;
    issue(std::integral_constant<int, 0>{});
    static_for<0, kBatches>([&](auto Bt) {
        constexpr int bt = decltype(Bt)::value;
        constexpr int b0 = bt * kLdsBatch;
        if constexpr (bt != 0) __syncthreads();  // the previous batch's reads are done
        static_for<0, kLdsBatch / 4>([&](auto M) {
            constexpr int m = decltype(M)::value;
            // slot of population b0 + 4 m + wave
            const int pi = 4 * m + wave;
            if (b0 + pi < Q) {
                S* slot = lds + (pi * 2 + role) * kLdsRow;
                *reinterpret_cast<S4*>(slot + 4 + 4 * (lane & 31)) = q[m];
                if (hk < 6) slot[hslot] = hv[m];
            }
        });
        __syncthreads();
        if constexpr (bt + 1 < kBatches) issue(std::integral_constant<int, bt + 1>{});
        static_for<0, kLdsBatch>([&](auto K) {
            constexpr int i = b0 + decltype(K)::value;
            if constexpr (i < Q) {
                constexpr Vel v = V.v[i];
                const S x = lds[(decltype(K)::value * 2 + role) * kLdsRow + 4 + c - v.x];
                p[i] = from_store<P>(x, a.ph, v.group);
            }
        });
    });
    collide_split<D, P>(p, role, a.ph);
    const uint32_t plane = (uint32_t)N * (uint32_t)sizeof(S);
    RowOffsets<S> o;
    o.row = (uint32_t)(y * a.nx + z * a.nxy) * cell_bytes(sizeof(S));
    o.own = (uint32_t)(x0 + c) * cell_bytes(sizeof(S)) + (role ? h_offset(sizeof(S), plane) : 0u);
    store_split<D, P>(static_cast<char*>(a.dst), plane, o, p, a.ph);
}

// ---------------------------------------------------------------------------
// Initial state S_0 = equilibrium of (rho, u, T), evaluated in double and
// stored in the storage precision (deviation from the rest equilibrium in
// FP32_DEV: g_i - w_i, h_i - (delta/2) w_i).
template <int D, class P>
__global__ __launch_bounds__(256) void k_init(char* dst, const double* __restrict__ rho_in,
                                              const double* __restrict__ u_in,
                                              const double* __restrict__ T_in, int64_t N,
                                              int64_t stride, double half_delta, double r,
                                              const WGroups wg) {
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
    using S = typename P::S;
    const size_t plane = (size_t)stride * sizeof(S);
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
        if constexpr (P::kDev) {
            gv = Fdev;
            hv = hdT * Fdev + half_delta * w * (temp - 1.0);  // H_i - (delta/2) w_i
        } else {
            gv = Fdev + w;
            hv = hdT * (Fdev + w);
        }
        char* base = dst + (size_t)(2 * i) * plane;
        if constexpr (P::kScaled) {  // stored divided by w (see F16Dev)
            gv /= w;
            hv /= w;
        }
        // rounded once, from double, to the storage type (via float for half)
        using Mid = std::conditional_t<sizeof(S) < 4, float, S>;
        char* at = base + (size_t)cell * cell_bytes(sizeof(S));
        *reinterpret_cast<S*>(at) = S(Mid(gv));
        *reinterpret_cast<S*>(at + h_offset(sizeof(S), (uint32_t)plane)) = S(Mid(hv));
    });
}

// ---------------------------------------------------------------------------
// The finite-difference form (Sec. III): explicit Euler in time, third-order
// upwind-biased convection per axis, BGK with rates dt / tau.  A wave loads
// the centre values of its cells, collides them in registers (taking the
// convection centre term with them), then reads each population's upwind
// neighbours from the time-n state and stores the new value.  The
// neighbour reads come from cache.  Waves go out in launch order (row by
// row).  Ordering them in per-XCD y bands, whole or in x-chunks, was
// measured: at most 5% faster in 3D, 9% slower in 2D.  The rows around the
// cells in flight on one XCD, over all 2Q planes, exceed its L2 either way.
template <int D, typename S, int L>
__device__ __forceinline__ bool fd_item(const StepArgs& a, int lane_cell, uint32_t role_off,
                                        RowOffsets<S>& o) {
    const int item = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (item >= a.items) return false;
    int seg = item % a.segs;
    const int row = item / a.segs;
    int y = row % a.ny;
    int z = row / a.ny;
    seg = __builtin_amdgcn_readfirstlane(seg);
    y = __builtin_amdgcn_readfirstlane(y);
    z = __builtin_amdgcn_readfirstlane(z);
    const int xr = seg * L + lane_cell;
    const int x = xr < a.nx ? xr : a.nx - 1;  // tail lanes repeat the last cell
    fill_row_offsets<D, S>(o, x, y, z, a.nx, a.ny, a.nz, a.nxy, a.open_end, true, role_off);
    return true;
}

template <int D, class P, bool SPLIT, int WAVES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES, 8)))
void k_fd_step(const StepArgs a) {
    using T = typename P::T;
    using S = typename P::S;
    constexpr int Q = VelSet<D>::Q;
    const int lane = (int)threadIdx.x & 63;
    const uint32_t plane = (uint32_t)a.P * (uint32_t)sizeof(S);
    const char* src = static_cast<const char*>(a.src);
    char* dst = static_cast<char*>(a.dst);
    RowOffsets<S> o;
    if constexpr (SPLIT) {
        const int role = lane >> 5;  // 0: g, 1: h (see collide_split)
        if (!fd_item<D, S, 32>(a, lane & 31, role ? h_offset(sizeof(S), plane) : 0u, o)) return;
        T p[Q];
        load_split<D, P, false>(src, plane, o, p, a.ph);
        collide_split<D, P, true>(p, role, a.ph);
        convect_store_split<D, P>(src, dst, plane, o, p, a.ph);
    } else {
        if (!fd_item<D, S, 64>(a, lane, 0u, o)) return;
        T g[Q], h[Q];
        load_lane<D, P, false>(src, plane, o, g, h, a.ph);
        collide_lane<D, P, true>(g, h, a.ph);
        convect_store_lane<D, P>(src, dst, plane, o, g, h, a.ph);
    }
}

// ---------------------------------------------------------------------------
// Readout of S_n in double (Sec. II moments): per-cell rho, u, E, T and/or
// per-workgroup partial totals (rho, rho u, rho E), reduced across the wave
// and the workgroup in a fixed order.
template <int D, class P>
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
        using S = typename P::S;
        constexpr bool DEV = P::kDev;
        const uint32_t plane = (uint32_t)a.P * (uint32_t)sizeof(S);
        const char* src = static_cast<const char*>(a.src);
        double s0 = 0, sj[3] = {0, 0, 0}, se = 0, sh = 0;
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr Vel v = V.v[i];
            const uint32_t off =
                (uint32_t)pt.template src<v.x, v.y, v.z>() * cell_bytes(sizeof(S));
            const char* base = src + (size_t)(2 * i) * plane;
            const double scale = P::kScaled ? a.w[v.group] : 1.0;
            const double gv = (double)load_at<S>(base, off) * scale;
            const double hv = (double)load_at<S>(base, off + h_offset(sizeof(S), plane)) * scale;
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
        if (a.T) {
            // Sec. II: E = |u|^2 / 2 + (D + delta) T / 2
            double uu = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) uu += (tot[1 + k] / rho) * (tot[1 + k] / rho);
            a.T[cell] = (2.0 * (rhoE / rho) - uu) * a.inv_dof;
        }
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

template <int D, class P>
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
    // Occupancy hint for the split D3Q107 float kernels: asking for at least
    // two waves per SIMD gave 4% more bandwidth than the compiler's own
    // choice (three waves at 162 VGPRs).  In double, two waves (256 VGPRs,
    // 30 values spilled to scratch, against one wave at 256 + 28 AGPRs) ran
    // 2.4% faster in isolated timings but not in the benchmark, and the
    // spills added 13% to the HBM bytes; it keeps one.  The other kernels
    // run best as compiled.
    constexpr int kSplitWaves = (D == 3 && sizeof(typename P::T) == 4) ? 2 : 1;
    if (split)
        return launch_kernel(&k_step_split<D, P, kSplitWaves>, dim3(grid), dim3(256), s, a);
    else
        return launch_kernel(&k_step<D, P, 1>, dim3(grid), dim3(256), s, a);
}

template <int D, class P>
hipError_t fd_step_impl(bool split, const StepArgs& a0, hipStream_t s) {
    StepArgs a = a0;
    const int L = split ? 32 : 64;
    a.segs = (a.nx + L - 1) / L;
    a.rows = a.ny * a.nz;
    a.items = a.segs * a.rows;
    a.tiles_per_row = (a.segs + 3) / 4;
    a.xcd_rows = 0;
    const int grid = (a.items + 3) / 4;
    if (split) return launch_kernel(&k_fd_step<D, P, true, 1>, dim3(grid), dim3(256), s, a);
    return launch_kernel(&k_fd_step<D, P, false, 1>, dim3(grid), dim3(256), s, a);
}

}  // namespace

// Run `f` with the storage policy of `precision`.
template <class F>
hipError_t with_policy(int precision, F&& f) {
    if (precision == LBM_FP64) return f(F64{});
    if (precision == LBM_FP16_SCALED) return f(F16Dev{});
    return f(F32Dev{});
}

hipError_t launch_init(int dim, int precision, void* dst, const double* rho,
                       const double* u, const double* T, int64_t N, int64_t stride,
                       double half_delta, double r, const double* w_group, hipStream_t s) {
    WGroups wg;
    for (int k = 0; k < 10; ++k) wg.w[k] = w_group[k];
    const int grid = (int)((N + 255) / 256);
    char* d = static_cast<char*>(dst);
    return with_policy(precision, [&](auto pol) {
        using P = decltype(pol);
        if (dim == 2)
            return launch_kernel(&k_init<2, P>, dim3(grid), dim3(256), s, d, rho, u, T, N, stride, half_delta, r, wg);
        return launch_kernel(&k_init<3, P>, dim3(grid), dim3(256), s, d, rho, u, T, N, stride, half_delta, r, wg);
    });
}

hipError_t launch_step_lds(int precision, const StepArgs& a0, hipStream_t s) {
    StepArgs a = a0;
    if (a.nx % 128 != 0 || !a.stream) return hipErrorInvalidValue;
    a.rows = a.ny * a.nz;
    a.tiles_per_row = a.nx / 128;
    const int grid = 8 * a.tiles_per_row * ((a.rows + 7) / 8);
    return with_policy(precision, [&](auto pol) {
        using P = decltype(pol);
        constexpr int kWaves = sizeof(typename P::T) == 4 ? 2 : 1;
        return launch_kernel(&k_step_split_lds<P, kWaves>, dim3(grid), dim3(256), s, a);
    });
}

hipError_t launch_step(int dim, int precision, bool split, const StepArgs& a, hipStream_t s) {
    return with_policy(precision, [&](auto pol) {
        using P = decltype(pol);
        return dim == 2 ? step_impl<2, P>(split, a, s) : step_impl<3, P>(split, a, s);
    });
}

int step_block_cells(int, int, bool split) { return split ? 128 : 256; }

hipError_t launch_fd_step(int dim, int precision, bool split, const StepArgs& a, hipStream_t s) {
    // no half storage in the finite-difference form (lbm_create_fd refuses it)
    if (precision == LBM_FP16_SCALED) return hipErrorInvalidValue;
    if (precision == LBM_FP64)
        return dim == 2 ? fd_step_impl<2, F64>(split, a, s) : fd_step_impl<3, F64>(split, a, s);
    return dim == 2 ? fd_step_impl<2, F32Dev>(split, a, s) : fd_step_impl<3, F32Dev>(split, a, s);
}

hipError_t launch_readout(int dim, int precision, const ReadArgs& a, int blocks, hipStream_t s) {
    return with_policy(precision, [&](auto pol) {
        using P = decltype(pol);
        if (dim == 2) return launch_kernel(&k_readout<2, P>, dim3(blocks), dim3(kReadBlock), s, a);
        return launch_kernel(&k_readout<3, P>, dim3(blocks), dim3(kReadBlock), s, a);
    });
}

hipError_t launch_final_reduce(int dim, const double* partials, int blocks, double* out,
                               hipStream_t s) {
    if (dim == 2)
        return launch_kernel(&k_final_reduce<4>, dim3(1), dim3(256), s, partials, blocks, out);
    else
        return launch_kernel(&k_final_reduce<5>, dim3(1), dim3(256), s, partials, blocks, out);
}

}  // namespace lbm

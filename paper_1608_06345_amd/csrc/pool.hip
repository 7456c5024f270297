// Batched multi-solve runtime: many independent solves (different grids,
// gamma, tau, step counts) resident in one device arena and advanced
// together, one launch per velocity set per step, replayed from hipGraphs.
//
// Device state
//   arena      one allocation; each resident solve owns a contiguous region
//              of two ping-pong sides laid out exactly as a single solve's
//              (see cell_bytes, h_offset).
//   table      static per-slot parameters (geometry, physics, step budget),
//              written by the host when membership changes.
//   steps_done per-slot step counters, advanced on the device by k_advance
//              after every step; the host only resets a slot's counter on
//              admission and reads them to find finished solves.
//   directory  per velocity set: the first tile of each resident solve and
//              its slot, in ascending tile order, plus the total tile count.
//
// A step launch has one workgroup per tile of its velocity set.  Each tile
// belongs to one solve (binary search in the directory) and
// covers four row segments, exactly as in a single-solve launch, including
// the whole-rows-per-XCD order (tile starts are multiples of 8, so tile t
// runs on XCD t % 8 as in a single launch).  Ping-pong parity
// comes from the solve's own counter: it reads side steps_done & 1 and
// writes the other.  Solves that have used up their steps are skipped.
//
// Because the kernels read all of this from device memory, a captured graph
// of K steps keeps its topology for good: admissions and releases rewrite the
// table and the directory between replays, and only the grid sizes of the
// graph's step launches are updated in place when the tile count changes
// (continuous batching without re-capture).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "lbm_internal.h"
#include "step_core.h"

namespace lbm {

struct SolveEntry {
    uint64_t base;        // byte address of side 0 (side 1 follows)
    uint64_t side_bytes;
    int32_t N, P, nx, ny, nz, nxy;  // P: plane stride in cells (plane_stride)
    uint32_t open_end;
    int32_t segs, rows, items, tiles_per_row, xcd_rows, tiles;
    int32_t dim, active;
    int64_t steps_total;
    double omega_f, omega_g, half_delta, inv_dof;
};

struct TileDir {
    int32_t count;        // resident solves of this velocity set
    int32_t total_tiles;
    int32_t pad[2];
    // followed in memory by int32 begin[max_slots] and int32 slot[max_slots]
};

struct PoolArgs {
    const SolveEntry* table;
    const int64_t* steps_done;
    const TileDir* dir;
    const int32_t* begin;
    const int32_t* slot;
    Physics ph;  // lattice weights and scale (per-solve rates come from the table)
};

namespace {

using namespace core;


template <int L>
__device__ __forceinline__ bool pool_item(const SolveEntry& e, int local, int wave, int& seg,
                                          int& row) {
    if (e.xcd_rows) {
        const int j = local >> 3;
        row = (j / e.tiles_per_row) * 8 + (local & 7);
        seg = (j % e.tiles_per_row) * 4 + wave;
        return row < e.rows && seg < e.segs;
    }
    const int item = local * 4 + wave;
    seg = item % e.segs;
    row = item / e.segs;
    return item < e.items;
}

// One workgroup per tile: the grid of each launch is exactly the tile count
// of the resident solves (a loop over tiles would keep loop state live
// across the whole body and cost a wave per SIMD of occupancy).
template <int D, class P, bool SPLIT, int WAVES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES, 8)))
void k_pool_step(const PoolArgs pa) {
    using T = typename P::T;
    using S = typename P::S;
    constexpr int Q = VelSet<D>::Q;
    constexpr int L = SPLIT ? 32 : 64;
    const int tile = (int)blockIdx.x;
    if (tile >= pa.dir->total_tiles) return;
    const int count = pa.dir->count;
    const int lane = (int)threadIdx.x & 63;
    const int wave = (int)(threadIdx.x >> 6);
    const int role = SPLIT ? lane >> 5 : 0;
    // the resident solve that owns this tile: last begin <= tile
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pa.begin[mid] <= tile) lo = mid;
        else hi = mid - 1;
    }
    const int s = __builtin_amdgcn_readfirstlane(pa.slot[lo]);
    const int local = tile - pa.begin[lo];
    const SolveEntry& e = pa.table[s];
    const int64_t done = pa.steps_done[s];
    if (!e.active || done >= e.steps_total || local >= e.tiles) return;
    int seg, row;
    if (!pool_item<L>(e, local, wave, seg, row)) return;
    seg = __builtin_amdgcn_readfirstlane(seg);
    row = __builtin_amdgcn_readfirstlane(row);
    const int y = row % e.ny;
    const int z = row / e.ny;
    const int xr = seg * L + (SPLIT ? (lane & 31) : lane);
    const int x = xr < e.nx ? xr : e.nx - 1;  // tail lanes redo the last cell
    const uint32_t plane = (uint32_t)e.P * (uint32_t)sizeof(S);
    RowOffsets<S> o;
    fill_row_offsets<D, S>(o, x, y, z, e.nx, e.ny, e.nz, e.nxy, e.open_end, true,
                           role ? h_offset(sizeof(S), plane) : 0u);
    const int par = (int)(done & 1);
    const char* src = reinterpret_cast<const char*>(e.base + (par ? e.side_bytes : 0));
    char* dst = reinterpret_cast<char*>(e.base + (par ? 0 : e.side_bytes));
    Physics ph = pa.ph;
    ph.omega_f = e.omega_f;
    ph.omega_g = e.omega_g;
    ph.half_delta = e.half_delta;
    ph.inv_dof = e.inv_dof;
    if constexpr (SPLIT) {
        T p[Q];
        load_split<D, P>(src, plane, o, p, ph);
        collide_split<D, P>(p, role, ph);
        store_split<D, P>(dst, plane, o, p, ph);
    } else {
        step_lane_cell<D, P>(src, dst, plane, o, ph);
    }
}

// One step done for every resident solve that still had steps to run.
__global__ __launch_bounds__(256) void k_advance(const SolveEntry* table, int64_t* steps_done,
                                                 int max_slots) {
    const int s = (int)(blockIdx.x * 256 + threadIdx.x);
    if (s < max_slots && table[s].active && steps_done[s] < table[s].steps_total)
        steps_done[s] = steps_done[s] + 1;
}

// The step kernel of a velocity set, in the pool's precision: the same
// layouts as the single-solve launches (default_split: one lane per cell for
// D2Q37 and for half storage, the g/h lane-pair split for D3Q107 in float
// and double).
template <class P>
const void* pool_step_kernel_p(int dim) {
    if (dim == 2) return reinterpret_cast<const void*>(&k_pool_step<2, P, false, 1>);
    if constexpr (P::kScaled) {
        return reinterpret_cast<const void*>(&k_pool_step<3, P, false, 1>);
    } else {
        constexpr int w = sizeof(typename P::T) == 4 ? 2 : 1;
        return reinterpret_cast<const void*>(&k_pool_step<3, P, true, w>);
    }
}

const void* pool_step_kernel(int precision, int dim) {
    if (precision == LBM_FP64) return pool_step_kernel_p<F64>(dim);
    if (precision == LBM_FP16_SCALED) return pool_step_kernel_p<F16Dev>(dim);
    return pool_step_kernel_p<F32Dev>(dim);
}

template <class P>
hipError_t launch_pool_step_p(int dim, const PoolArgs& a, int grid, hipStream_t s) {
    if (dim == 2) return launch_kernel(&k_pool_step<2, P, false, 1>, dim3(grid), dim3(256), s, a);
    if constexpr (P::kScaled) {
        return launch_kernel(&k_pool_step<3, P, false, 1>, dim3(grid), dim3(256), s, a);
    } else {
        constexpr int w = sizeof(typename P::T) == 4 ? 2 : 1;
        return launch_kernel(&k_pool_step<3, P, true, w>, dim3(grid), dim3(256), s, a);
    }
}

hipError_t launch_pool_step(int precision, int dim, const PoolArgs& a, int grid, hipStream_t s) {
    if (precision == LBM_FP64) return launch_pool_step_p<F64>(dim, a, grid, s);
    if (precision == LBM_FP16_SCALED) return launch_pool_step_p<F16Dev>(dim, a, grid, s);
    return launch_pool_step_p<F32Dev>(dim, a, grid, s);
}

struct Slot {
    bool used = false;
    int dim = 0;
    int64_t nx = 0, ny = 0, nz = 0, N = 0, P = 0;
    uint32_t bc = 0;
    double gamma = 0, delta = 0, tau_f = 0, tau_g = 0;
    int64_t steps_total = 0;
    size_t offset = 0, bytes = 0;
    bool reported = false;
};

int err_of(hipError_t e) {
    if (e == hipSuccess) return LBM_OK;
    if (e == hipErrorOutOfMemory) return LBM_ENOMEM;
    return LBM_EDEVICE;
}

#define POOL_HIP(call)                            \
    do {                                          \
        const hipError_t e_ = (call);             \
        if (e_ != hipSuccess) return lbm::err_of(e_);  \
    } while (0)

}  // namespace
}  // namespace lbm

using lbm::Slot;
using lbm::SolveEntry;
using lbm::TileDir;

struct lbm_pool {
    int precision = 0;
    size_t elem = 4;
    size_t budget = 0;
    int max_slots = 0;
    char* arena = nullptr;
    std::map<size_t, size_t> free_list;  // offset -> bytes, coalesced
    size_t used_bytes = 0;
    std::vector<Slot> slots;
    std::vector<SolveEntry> table;
    // device
    SolveEntry* d_table = nullptr;
    int64_t* d_steps = nullptr;
    char* d_dir[2] = {nullptr, nullptr};  // TileDir + begin[] + slot[] per velocity set
    double* d_stage = nullptr;            // initial fields of an admission
    size_t stage_cells = 0;
    double* d_partials = nullptr;
    size_t partial_blocks = 0;
    double* d_totals = nullptr;
    // host staging of table/directories (pinned; reused once the last upload completed)
    char* h_upload = nullptr;
    size_t upload_bytes = 0;
    hipEvent_t upload_done = nullptr;
    int64_t* h_steps = nullptr;  // pinned copy of the counters
    bool dirty = true;
    int resident[2] = {0, 0};
    hipStream_t stream = nullptr, own_stream = nullptr;
    int tiles_total[2] = {0, 0};  // tiles of the resident solves, per velocity set
    struct Graph {
        hipGraph_t def = nullptr;
        hipGraphExec_t exec = nullptr;
        std::vector<hipGraphNode_t> step_nodes[2];  // kernel nodes per velocity set
        int grid[2] = {0, 0};                        // their current grid size
    };
    std::map<int, Graph> graphs;  // key: ticks * 4 + velocity-set mask
};

namespace {

size_t dir_bytes(int max_slots) { return sizeof(TileDir) + 2 * sizeof(int32_t) * max_slots; }

// first-fit allocation in the arena, 256-byte granules
bool arena_alloc(lbm_pool* p, size_t bytes, size_t* off) {
    bytes = (bytes + 255) & ~(size_t)255;
    for (auto it = p->free_list.begin(); it != p->free_list.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            p->free_list.erase(it);
            if (rest) p->free_list[at] = rest;
            p->used_bytes += bytes;
            return true;
        }
    }
    return false;
}

void arena_free(lbm_pool* p, size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    p->used_bytes -= bytes;
    auto it = p->free_list.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != p->free_list.end() && it->first + it->second == next->first) {
        it->second += next->second;
        p->free_list.erase(next);
    }
    if (it != p->free_list.begin()) {
        auto prev = std::prev(it);
        if (prev->first + prev->second == it->first) {
            prev->second += it->second;
            p->free_list.erase(it);
        }
    }
}

int tiles_of(int dim, int precision, int64_t nx, int64_t ny, int64_t nz, SolveEntry& e) {
    const int L = lbm::default_split(dim, precision) ? 32 : 64;  // cells per wave
    e.segs = (int)((nx + L - 1) / L);
    e.rows = (int)(ny * nz);
    e.items = e.segs * e.rows;
    e.tiles_per_row = (e.segs + 3) / 4;
    e.xcd_rows = e.rows >= 64 ? 1 : 0;
    const int t = e.xcd_rows ? 8 * e.tiles_per_row * ((e.rows + 7) / 8) : (e.items + 3) / 4;
    return (t + 7) & ~7;  // tile starts stay multiples of 8
}

// Upload the table and both directories (before the next step launch).
int upload(lbm_pool* p) {
    if (!p->dirty) return LBM_OK;
    POOL_HIP(hipEventSynchronize(p->upload_done));  // the staging block is free again
    const size_t tb = sizeof(SolveEntry) * p->max_slots;
    std::memcpy(p->h_upload, p->table.data(), tb);
    for (int d = 0; d < 2; ++d) {
        char* blk = p->h_upload + tb + d * dir_bytes(p->max_slots);
        TileDir* dir = reinterpret_cast<TileDir*>(blk);
        int32_t* begin = reinterpret_cast<int32_t*>(blk + sizeof(TileDir));
        int32_t* slot = begin + p->max_slots;
        int count = 0, total = 0;
        for (int s = 0; s < p->max_slots; ++s) {
            const SolveEntry& e = p->table[s];
            if (!e.active || e.dim != d + 2) continue;
            begin[count] = total;
            slot[count] = s;
            total += e.tiles;
            ++count;
        }
        dir->count = count;
        dir->total_tiles = total;
        p->resident[d] = count;
        p->tiles_total[d] = total;
    }
    POOL_HIP(hipMemcpyAsync(p->d_table, p->h_upload, tb, hipMemcpyHostToDevice, p->stream));
    for (int d = 0; d < 2; ++d)
        POOL_HIP(hipMemcpyAsync(p->d_dir[d], p->h_upload + tb + d * dir_bytes(p->max_slots),
                                dir_bytes(p->max_slots), hipMemcpyHostToDevice, p->stream));
    POOL_HIP(hipEventRecord(p->upload_done, p->stream));
    p->dirty = false;
    return LBM_OK;
}

lbm::PoolArgs pool_args(lbm_pool* p, int d) {
    lbm::PoolArgs a;
    std::memset(&a, 0, sizeof(a));
    a.table = p->d_table;
    a.steps_done = p->d_steps;
    a.dir = reinterpret_cast<const TileDir*>(p->d_dir[d]);
    a.begin = reinterpret_cast<const int32_t*>(p->d_dir[d] + sizeof(TileDir));
    a.slot = a.begin + p->max_slots;
    a.ph = lbm::physics_of(d + 2, 0.0, 1.0, 1.0);  // weights and r; rates per solve
    return a;
}

// Enqueue `ticks` steps for the velocity sets in `mask` (bit 0: D2Q37, bit 1: D3Q107).
int enqueue_steps(lbm_pool* p, int ticks, int mask, hipStream_t s) {
    for (int t = 0; t < ticks; ++t) {
        for (int d = 0; d < 2; ++d) {
            if (!(mask & (1 << d))) continue;
            const lbm::PoolArgs a = pool_args(p, d);
            const int grid = p->tiles_total[d] > 0 ? p->tiles_total[d] : 1;
            hipError_t e = lbm::launch_pool_step(p->precision, d + 2, a, grid, s);
            POOL_HIP(e);
        }
        POOL_HIP(lbm::launch_kernel(&lbm::k_advance, dim3((p->max_slots + 255) / 256), dim3(256),
                                    s, (const SolveEntry*)p->d_table, p->d_steps, p->max_slots));
    }
    return LBM_OK;
}

int check_slot(lbm_pool* p, int slot) {
    if (!p || slot < 0 || slot >= p->max_slots || !p->slots[slot].used) return LBM_EINVAL;
    return LBM_OK;
}

int ensure_partials(lbm_pool* p, int64_t N) {
    const size_t blocks = (size_t)((N + lbm::kReadBlock - 1) / lbm::kReadBlock);
    if (blocks <= p->partial_blocks) return LBM_OK;
    if (p->d_partials) POOL_HIP(hipFree(p->d_partials));
    p->d_partials = nullptr;
    p->partial_blocks = 0;
    POOL_HIP(hipMalloc((void**)&p->d_partials, blocks * 5 * sizeof(double)));
    p->partial_blocks = blocks;
    return LBM_OK;
}

// Readout of a slot's S_n (n = its steps done), like a single solve's.
int pool_readout(lbm_pool* p, int slot, double* rho, double* u, double* E, double* T,
                 bool totals) {
    const Slot& sl = p->slots[slot];
    POOL_HIP(hipMemcpyAsync(p->h_steps + slot, p->d_steps + slot, sizeof(int64_t),
                            hipMemcpyDeviceToHost, p->stream));
    POOL_HIP(hipStreamSynchronize(p->stream));
    const int64_t n = p->h_steps[slot];
    const SolveEntry& e = p->table[slot];
    lbm::ReadArgs a;
    std::memset(&a, 0, sizeof(a));
    // S_0 sits unstreamed in side 1; later P_{n-1} is in side (n - 1) & 1
    const int side = n == 0 ? 1 : (int)((n - 1) & 1);
    a.src = reinterpret_cast<const void*>(e.base + (side ? e.side_bytes : 0));
    a.stream = n == 0 ? 0 : 1;
    a.N = sl.N;
    a.P = sl.P;
    a.nx = (int32_t)sl.nx;
    a.ny = (int32_t)sl.ny;
    a.nz = (int32_t)sl.nz;
    a.nxy = (int32_t)(sl.nx * sl.ny);
    a.open_end = e.open_end;
    a.r = lbm::lattice_tables(sl.dim).r;
    a.rest_energy = 0.5 * (sl.dim + sl.delta);
    a.inv_dof = 1.0 / (sl.dim + sl.delta);
    for (int g = 0; g < lbm::lattice_tables(sl.dim).groups; ++g)
        a.w[g] = lbm::lattice_tables(sl.dim).w_group[g];
    a.rho = rho;
    a.u = u;
    a.E = E;
    a.T = T;
    const int blocks = (int)((sl.N + lbm::kReadBlock - 1) / lbm::kReadBlock);
    if (totals) {
        int rc = ensure_partials(p, sl.N);
        if (rc != LBM_OK) return rc;
        a.partials = p->d_partials;
    }
    POOL_HIP(lbm::launch_readout(sl.dim, p->precision, a, blocks, p->stream));
    if (totals)
        POOL_HIP(lbm::launch_final_reduce(sl.dim, p->d_partials, blocks, p->d_totals, p->stream));
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_pool_create(size_t budget_bytes, int max_slots, int precision, lbm_pool_handle* out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    if (max_slots < 1 || max_slots > 65536 || budget_bytes < 4096) return LBM_EINVAL;
    if (precision != LBM_FP64 && precision != LBM_FP32_DEV && precision != LBM_FP16_SCALED)
        return LBM_EINVAL;
    lbm_pool* p = new (std::nothrow) lbm_pool;
    if (!p) return LBM_ENOMEM;
    p->precision = precision;
    p->elem = precision == LBM_FP64 ? 8 : (precision == LBM_FP32_DEV ? 4 : 2);
    p->budget = budget_bytes & ~(size_t)255;
    p->max_slots = max_slots;
    p->slots.resize(max_slots);
    p->table.assign(max_slots, SolveEntry{});
    p->upload_bytes = sizeof(SolveEntry) * max_slots + 2 * dir_bytes(max_slots);
    hipError_t e = hipMalloc((void**)&p->arena, p->budget);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_table, sizeof(SolveEntry) * max_slots);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_steps, sizeof(int64_t) * max_slots);
    for (int d = 0; d < 2 && e == hipSuccess; ++d) e = hipMalloc((void**)&p->d_dir[d], dir_bytes(max_slots));
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_totals, 8 * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_upload, p->upload_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_steps, sizeof(int64_t) * max_slots, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->upload_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->own_stream, hipStreamNonBlocking);
    if (e == hipSuccess) {
        p->stream = p->own_stream;
        // counters start at zero: copied from the (zeroed) pinned block, not
        // memset, so nothing of the kind can end up inside a captured graph
        std::memset(p->h_steps, 0, sizeof(int64_t) * max_slots);
        e = hipMemcpyAsync(p->d_steps, p->h_steps, sizeof(int64_t) * max_slots,
                           hipMemcpyHostToDevice, p->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    }
    if (e != hipSuccess) {
        lbm_pool_destroy(p);
        return lbm::err_of(e);
    }
    p->free_list[0] = p->budget;
    *out = p;
    return LBM_OK;
}

int lbm_pool_destroy(lbm_pool_handle p) {
    if (!p) return LBM_OK;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    for (auto& kv : p->graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.def) (void)hipGraphDestroy(kv.second.def);
    }
    if (p->arena) (void)hipFree(p->arena);
    if (p->d_table) (void)hipFree(p->d_table);
    if (p->d_steps) (void)hipFree(p->d_steps);
    for (int d = 0; d < 2; ++d)
        if (p->d_dir[d]) (void)hipFree(p->d_dir[d]);
    if (p->d_stage) (void)hipFree(p->d_stage);
    if (p->d_partials) (void)hipFree(p->d_partials);
    if (p->d_totals) (void)hipFree(p->d_totals);
    if (p->h_upload) (void)hipHostFree(p->h_upload);
    if (p->h_steps) (void)hipHostFree(p->h_steps);
    if (p->upload_done) (void)hipEventDestroy(p->upload_done);
    if (p->own_stream) (void)hipStreamDestroy(p->own_stream);
    delete p;
    return LBM_OK;
}

int lbm_pool_set_stream(lbm_pool_handle p, void* stream) {
    if (!p) return LBM_EINVAL;
    p->stream = static_cast<hipStream_t>(stream);
    return LBM_OK;
}

// Every check of a request that admission makes before looking at the pool's
// state: shape, gamma (delta = 2/(gamma - 1) - D of Sec. II, snapped to 0
// within 1e-9, must not be negative), rates, step count and boundary codes.
static bool request_valid(const lbm_request* r, int precision, double* delta_out) {
    if (!r || (precision != LBM_FP64 && precision != LBM_FP32_DEV &&
               precision != LBM_FP16_SCALED))
        return false;
    if (r->dim != 2 && r->dim != 3) return false;
    if (r->nx < 1 || r->ny < 1 || r->nz < 1 || (r->dim == 2 && r->nz != 1)) return false;
    const double N = (double)r->nx * (double)r->ny * (double)r->nz;
    const size_t elem = precision == LBM_FP64 ? 8 : (precision == LBM_FP32_DEV ? 4 : 2);
    if (N * (double)elem > 2147483647.0) return false;
    const int64_t P = lbm::plane_stride(r->nx * r->ny * r->nz, elem, r->dim);
    if ((double)P * (double)elem > 2147483647.0) return false;
    if (!(r->gamma > 1.0) || !std::isfinite(r->gamma)) return false;
    double delta = 2.0 / (r->gamma - 1.0) - r->dim;
    if (std::fabs(delta) < 1e-9) delta = 0.0;
    if (delta < 0.0) return false;
    if (!(r->tau_f > 0.5) || !(r->tau_g > 0.5) || !std::isfinite(r->tau_f) ||
        !std::isfinite(r->tau_g))
        return false;
    if (r->steps < 0 || (r->bc & ~0x3Fu)) return false;
    for (int k = 0; k < 3; ++k)
        if (((r->bc >> (2 * k)) & 3u) > LBM_BC_ZERO_GRADIENT) return false;
    if (r->dim == 2 && ((r->bc >> 4) & 3u) != LBM_BC_PERIODIC) return false;
    if (delta_out) *delta_out = delta;
    return true;
}

size_t lbm_pool_request_bytes(const lbm_request* r, int precision) {
    if (!request_valid(r, precision, nullptr)) return 0;
    const size_t elem = precision == LBM_FP64 ? 8 : (precision == LBM_FP32_DEV ? 4 : 2);
    const size_t P = (size_t)lbm::plane_stride(r->nx * r->ny * r->nz, elem, r->dim);
    const int q = r->dim == 2 ? LBM_D2Q37 : LBM_D3Q107;
    const size_t bytes = 2 * 2 * (size_t)q * P * elem;
    return (bytes + 255) & ~(size_t)255;
}

static int pool_admit(lbm_pool_handle p, const lbm_request* r, const double* rho,
                      const double* u, const double* T, bool device, int* slot_out) {
    if (!p || !r || !rho || !u || !T || !slot_out) return LBM_EINVAL;
    *slot_out = -1;
    double delta = 0.0;
    if (!request_valid(r, p->precision, &delta)) return LBM_EINVAL;
    const size_t bytes = lbm_pool_request_bytes(r, p->precision);
    if (bytes > p->budget) return LBM_ENOMEM;  // can never fit
    int slot = -1;
    for (int s = 0; s < p->max_slots; ++s)
        if (!p->slots[s].used) {
            slot = s;
            break;
        }
    size_t off = 0;
    if (slot < 0 || !arena_alloc(p, bytes, &off)) return LBM_EBUSY;

    Slot& sl = p->slots[slot];
    sl.used = true;
    sl.dim = r->dim;
    sl.nx = r->nx;
    sl.ny = r->ny;
    sl.nz = r->nz;
    sl.N = r->nx * r->ny * r->nz;
    sl.P = lbm::plane_stride(sl.N, p->precision == LBM_FP64 ? 8 : (p->precision == LBM_FP32_DEV ? 4 : 2),
                             r->dim);
    sl.bc = r->bc;
    sl.gamma = r->gamma;
    sl.delta = delta;
    sl.tau_f = r->tau_f;
    sl.tau_g = r->tau_g;
    sl.steps_total = r->steps;
    sl.offset = off;
    sl.bytes = bytes;
    sl.reported = false;

    SolveEntry e{};
    e.base = reinterpret_cast<uint64_t>(p->arena + off);
    e.side_bytes = bytes / 2;
    e.N = (int32_t)sl.N;
    e.P = (int32_t)sl.P;
    e.nx = (int32_t)r->nx;
    e.ny = (int32_t)r->ny;
    e.nz = (int32_t)r->nz;
    e.nxy = (int32_t)(r->nx * r->ny);
    e.open_end = (r->bc & 3u) | (((r->bc >> 2) & 3u) << 1) | (((r->bc >> 4) & 3u) << 2);
    e.tiles = tiles_of(r->dim, p->precision, r->nx, r->ny, r->nz, e);
    e.dim = r->dim;
    e.active = 1;
    e.steps_total = r->steps;
    const lbm::Physics ph = lbm::physics_of(r->dim, delta, r->tau_f, r->tau_g);
    e.omega_f = ph.omega_f;
    e.omega_g = ph.omega_g;
    e.half_delta = ph.half_delta;
    e.inv_dof = ph.inv_dof;
    p->table[slot] = e;
    p->dirty = true;

    // fields -> S_0 into side 1 -> P_0 = Collide(S_0) into side 0
    const double* drho = rho;
    const double* du = u;
    const double* dT = T;
    auto fail = [&](int rc) {
        sl.used = false;
        p->table[slot].active = 0;
        arena_free(p, off, bytes);
        return rc;
    };
    if (!device) {
        const size_t need = (size_t)sl.N * (2 + r->dim);
        if (need > p->stage_cells) {
            if (p->d_stage) {
                hipError_t e2 = hipStreamSynchronize(p->stream);
                if (e2 == hipSuccess) e2 = hipFree(p->d_stage);
                if (e2 != hipSuccess) return fail(lbm::err_of(e2));
            }
            p->d_stage = nullptr;
            p->stage_cells = 0;
            hipError_t e2 = hipMalloc((void**)&p->d_stage, need * sizeof(double));
            if (e2 != hipSuccess) return fail(lbm::err_of(e2));
            p->stage_cells = need;
        }
        const size_t nb = (size_t)sl.N * sizeof(double);
        hipError_t e2 = hipMemcpyAsync(p->d_stage, rho, nb, hipMemcpyHostToDevice, p->stream);
        if (e2 == hipSuccess)
            e2 = hipMemcpyAsync(p->d_stage + sl.N, T, nb, hipMemcpyHostToDevice, p->stream);
        if (e2 == hipSuccess)
            e2 = hipMemcpyAsync(p->d_stage + 2 * sl.N, u, nb * r->dim, hipMemcpyHostToDevice,
                                p->stream);
        if (e2 != hipSuccess) return fail(lbm::err_of(e2));
        drho = p->d_stage;
        dT = p->d_stage + sl.N;
        du = p->d_stage + 2 * sl.N;
    }
    char* side0 = p->arena + off;
    char* side1 = side0 + bytes / 2;
    hipError_t e2 = lbm::launch_init(r->dim, p->precision, side1, drho, du, dT, sl.N, sl.P,
                                     0.5 * delta, ph.r, ph.w, p->stream);
    if (e2 == hipSuccess) {
        lbm::StepArgs a;
        std::memset(&a, 0, sizeof(a));
        a.src = side1;
        a.dst = side0;
        a.N = sl.N;
        a.P = sl.P;
        a.nx = e.nx;
        a.ny = e.ny;
        a.nz = e.nz;
        a.nxy = e.nxy;
        a.open_end = e.open_end;
        a.stream = 0;
        a.ph = ph;
        e2 = lbm::launch_step(r->dim, p->precision, lbm::default_split(r->dim, p->precision), a,
                              p->stream);
    }
    if (e2 == hipSuccess) {
        p->h_steps[slot] = 0;
        e2 = hipMemcpyAsync(p->d_steps + slot, p->h_steps + slot, sizeof(int64_t),
                            hipMemcpyHostToDevice, p->stream);
        // the pinned word must not change before the copy ran
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(p->stream);
    }
    if (e2 != hipSuccess) return fail(lbm::err_of(e2));
    *slot_out = slot;
    return LBM_OK;
}

int lbm_pool_admit(lbm_pool_handle p, const lbm_request* r, const double* rho, const double* u,
                   const double* T, int* slot_out) {
    return pool_admit(p, r, rho, u, T, false, slot_out);
}

int lbm_pool_admit_dev(lbm_pool_handle p, const lbm_request* r, const double* rho,
                       const double* u, const double* T, int* slot_out) {
    return pool_admit(p, r, rho, u, T, true, slot_out);
}

int lbm_pool_run(lbm_pool_handle p, int ticks) {
    if (!p || ticks < 0 || ticks > 4096) return LBM_EINVAL;
    if (ticks == 0) return LBM_OK;
    int rc = upload(p);
    if (rc != LBM_OK) return rc;
    const int mask = (p->resident[0] ? 1 : 0) | (p->resident[1] ? 2 : 0);
    if (!mask) return LBM_OK;
    const int key = ticks * 4 + mask;
    auto it = p->graphs.find(key);
    if (it == p->graphs.end()) {
        // capture once on a private stream, replay on the pool's stream
        hipStream_t cap;
        POOL_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        int rc2 = LBM_OK;
        if (e == hipSuccess) rc2 = enqueue_steps(p, ticks, mask, cap);
        hipGraph_t g = nullptr;
        const hipError_t e_end = hipStreamEndCapture(cap, &g);
        hipGraphExec_t exec = nullptr;
        if (e == hipSuccess && rc2 == LBM_OK && e_end == hipSuccess)
            e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipStreamDestroy(cap);
        if (e != hipSuccess || rc2 != LBM_OK || e_end != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return rc2 != LBM_OK ? rc2 : lbm::err_of(e != hipSuccess ? e : e_end);
        }
        lbm_pool::Graph gr;
        gr.def = g;
        gr.exec = exec;
        // remember the step-kernel nodes, to resize their grids later
        size_t n = 0;
        POOL_HIP(hipGraphGetNodes(g, nullptr, &n));
        std::vector<hipGraphNode_t> nodes(n);
        POOL_HIP(hipGraphGetNodes(g, nodes.data(), &n));
        for (int d = 0; d < 2; ++d) {
            const void* fn = lbm::pool_step_kernel(p->precision, d + 2);
            for (auto node : nodes) {
                hipGraphNodeType type;
                POOL_HIP(hipGraphNodeGetType(node, &type));
                if (type != hipGraphNodeTypeKernel) continue;
                hipKernelNodeParams kp;
                POOL_HIP(hipGraphKernelNodeGetParams(node, &kp));
                if (kp.func == fn) gr.step_nodes[d].push_back(node);
            }
            gr.grid[d] = p->tiles_total[d] > 0 ? p->tiles_total[d] : 1;
        }
        it = p->graphs.emplace(key, gr).first;
    }
    // membership changed since this graph last ran: resize its step launches
    // in place (the topology stays, nothing is re-captured)
    lbm_pool::Graph& gr = it->second;
    for (int d = 0; d < 2; ++d) {
        const int grid = p->tiles_total[d] > 0 ? p->tiles_total[d] : 1;
        if (grid == gr.grid[d] || gr.step_nodes[d].empty()) continue;
        POOL_HIP(hipStreamSynchronize(p->stream));  // no replay in flight
        for (auto node : gr.step_nodes[d]) {
            hipKernelNodeParams kp;
            POOL_HIP(hipGraphKernelNodeGetParams(node, &kp));
            kp.gridDim = dim3(grid);
            POOL_HIP(hipGraphExecKernelNodeSetParams(gr.exec, node, &kp));
        }
        gr.grid[d] = grid;
    }
    POOL_HIP(hipGraphLaunch(gr.exec, p->stream));
    return LBM_OK;
}

int lbm_pool_run_eager(lbm_pool_handle p, int ticks) {
    if (!p || ticks < 0) return LBM_EINVAL;
    int rc = upload(p);
    if (rc != LBM_OK) return rc;
    const int mask = (p->resident[0] ? 1 : 0) | (p->resident[1] ? 2 : 0);
    if (!mask) return LBM_OK;
    return enqueue_steps(p, ticks, mask, p->stream);
}

int lbm_pool_poll(lbm_pool_handle p, int* finished, int max_finished, int* n_finished) {
    if (!p || !n_finished || (max_finished > 0 && !finished)) return LBM_EINVAL;
    *n_finished = 0;
    POOL_HIP(hipMemcpyAsync(p->h_steps, p->d_steps, sizeof(int64_t) * p->max_slots,
                            hipMemcpyDeviceToHost, p->stream));
    POOL_HIP(hipStreamSynchronize(p->stream));
    for (int s = 0; s < p->max_slots; ++s) {
        Slot& sl = p->slots[s];
        if (!sl.used || sl.reported || p->h_steps[s] < sl.steps_total) continue;
        if (*n_finished >= max_finished) break;
        finished[(*n_finished)++] = s;
        sl.reported = true;
    }
    return LBM_OK;
}

int lbm_pool_slot_steps(lbm_pool_handle p, int slot, int64_t* steps_done) {
    int rc = check_slot(p, slot);
    if (rc != LBM_OK || !steps_done) return rc != LBM_OK ? rc : LBM_EINVAL;
    POOL_HIP(hipMemcpyAsync(p->h_steps + slot, p->d_steps + slot, sizeof(int64_t),
                            hipMemcpyDeviceToHost, p->stream));
    POOL_HIP(hipStreamSynchronize(p->stream));
    *steps_done = p->h_steps[slot];
    return LBM_OK;
}

int lbm_pool_moments(lbm_pool_handle p, int slot, double* rho, double* u, double* E) {
    int rc = check_slot(p, slot);
    if (rc != LBM_OK) return rc;
    if (!rho || !u || !E) return LBM_EINVAL;
    const Slot& sl = p->slots[slot];
    const size_t n = (size_t)sl.N * sizeof(double);
    double* d = nullptr;
    POOL_HIP(hipMalloc((void**)&d, n * (2 + sl.dim)));
    rc = pool_readout(p, slot, d, d + 2 * sl.N, d + sl.N, nullptr, false);
    hipError_t e = hipSuccess;
    if (rc == LBM_OK) e = hipMemcpyAsync(rho, d, n, hipMemcpyDeviceToHost, p->stream);
    if (rc == LBM_OK && e == hipSuccess)
        e = hipMemcpyAsync(E, d + sl.N, n, hipMemcpyDeviceToHost, p->stream);
    if (rc == LBM_OK && e == hipSuccess)
        e = hipMemcpyAsync(u, d + 2 * sl.N, n * sl.dim, hipMemcpyDeviceToHost, p->stream);
    const hipError_t es = hipStreamSynchronize(p->stream);
    (void)hipFree(d);
    if (rc != LBM_OK) return rc;
    if (e != hipSuccess) return lbm::err_of(e);
    return lbm::err_of(es);
}

int lbm_pool_moments_dev(lbm_pool_handle p, int slot, double* rho, double* u, double* E) {
    int rc = check_slot(p, slot);
    if (rc != LBM_OK) return rc;
    if (!rho || !u || !E) return LBM_EINVAL;
    return pool_readout(p, slot, rho, u, E, nullptr, false);
}

int lbm_pool_temperature(lbm_pool_handle p, int slot, double* T) {
    int rc = check_slot(p, slot);
    if (rc != LBM_OK) return rc;
    if (!T) return LBM_EINVAL;
    const size_t n = (size_t)p->slots[slot].N * sizeof(double);
    double* d = nullptr;
    POOL_HIP(hipMalloc((void**)&d, n));
    rc = pool_readout(p, slot, nullptr, nullptr, nullptr, d, false);
    hipError_t e = hipSuccess;
    if (rc == LBM_OK) e = hipMemcpyAsync(T, d, n, hipMemcpyDeviceToHost, p->stream);
    const hipError_t es = hipStreamSynchronize(p->stream);
    (void)hipFree(d);
    if (rc != LBM_OK) return rc;
    if (e != hipSuccess) return lbm::err_of(e);
    return lbm::err_of(es);
}

int lbm_pool_totals(lbm_pool_handle p, int slot, double* mass, double* mom, double* energy) {
    int rc = check_slot(p, slot);
    if (rc != LBM_OK) return rc;
    if (!mass || !mom || !energy) return LBM_EINVAL;
    rc = pool_readout(p, slot, nullptr, nullptr, nullptr, nullptr, true);
    if (rc != LBM_OK) return rc;
    const int dim = p->slots[slot].dim;
    double t[8];
    POOL_HIP(hipMemcpyAsync(t, p->d_totals, (dim + 2) * sizeof(double), hipMemcpyDeviceToHost,
                            p->stream));
    POOL_HIP(hipStreamSynchronize(p->stream));
    *mass = t[0];
    for (int k = 0; k < dim; ++k) mom[k] = t[1 + k];
    *energy = t[dim + 1];
    for (int k = 0; k < dim + 2; ++k)
        if (!std::isfinite(t[k])) return LBM_ENONFINITE;
    return LBM_OK;
}

int lbm_pool_release(lbm_pool_handle p, int slot) {
    int rc = check_slot(p, slot);
    if (rc != LBM_OK) return rc;
    // queued work that still reads the slot must finish before its memory is reused
    POOL_HIP(hipStreamSynchronize(p->stream));
    Slot& sl = p->slots[slot];
    arena_free(p, sl.offset, sl.bytes);
    sl.used = false;
    p->table[slot] = SolveEntry{};
    p->dirty = true;
    return LBM_OK;
}

int lbm_pool_get_info(lbm_pool_handle p, lbm_pool_info* info) {
    if (!p || !info) return LBM_EINVAL;
    info->budget_bytes = p->budget;
    info->used_bytes = p->used_bytes;
    size_t largest = 0;
    for (auto& kv : p->free_list) largest = std::max(largest, kv.second);
    info->largest_free_bytes = largest;
    info->max_slots = p->max_slots;
    int n = 0;
    for (auto& s : p->slots) n += s.used ? 1 : 0;
    info->resident = n;
    info->graphs = (int)p->graphs.size();
    return LBM_OK;
}

}  // extern "C"

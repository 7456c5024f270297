// Internal declarations shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <tuple>
#include <type_traits>
#include <utility>

#include "lbm.h"
#include "velocity_set.h"

namespace lbm {

// Lattice constants derived on the host (lattice.cpp).
struct LatticeTables {
    int dim, q, groups;
    double r;
    double w_group[10];
    double w[107];
    int8_t e[107][3];
    int group[107];
};
const LatticeTables& lattice_tables(int dim);

// Group weights by value (kernel argument).
struct WGroups {
    double w[10];
};

// Physical parameters of one solve as the collision uses them.
struct Physics {
    double omega_f, omega_g;  // 1 / tau (lattice scheme), dt / tau (finite differences)
    double half_delta;        // delta / 2
    double inv_dof;           // 1 / (D + delta)
    double r;                 // lattice scale, xi = r e
    double w[10];             // group weights
    float wf[10];             // the same, rounded to float
    float inv_wf[10];         // 1 / w (scaling of half-precision storage)
    double fd_cs;             // finite differences: dt r / 6 (0 for the lattice scheme)
    float fd_csf;             // the same, rounded to float
    double ec;                // energy-conserving collision: 1 - tau_g / tau_f, else 0
    float ecf;                // the same, rounded to float
};

// Arguments of the fused step kernel (passed by value in the kernarg
// segment, so every field is wave-uniform and lives in SGPRs).
struct StepArgs {
    const void* src;      // one ping-pong side (layout: cell_bytes, h_offset)
    void* dst;            // same layout
    int64_t N;            // cells
    int64_t P;            // plane stride in cells (>= N; see plane_stride)
    int32_t nx, ny, nz;
    int32_t nxy;          // nx * ny
    uint32_t open_end;    // bit k: axis k is zero-gradient, else periodic
    int32_t stream;       // 1: pull-stream then collide; 0: collide in place
    int32_t segs;         // row segments per row (one wave each)
    int32_t rows;         // ny * nz
    int32_t items;        // row segments in the grid
    int32_t tiles_per_row;  // workgroups (four segments each) per row
    int32_t xcd_rows;     // 1: each XCD serves whole rows (see kernels.hip)
    int32_t fd_w;         // finite-difference update sweep: tiles per x-chunk
    int32_t fd_yb;        // finite-difference update sweep: rows per y sub-band
    Physics ph;
};

// Plane stride (cells) of a solve's population planes for N cells of elem
// bytes each in dim dimensions (lattice.cpp): N rounded up to 128 bytes, and
// for large planes moved off a large power of two bytes apart.
int64_t plane_stride(int64_t N, size_t elem, int dim);

// Storage layout of one ping-pong side.  Population i owns the slab of
// 2 P elem bytes that starts at byte 2 i P elem.  In FP64 and FP32 the slab
// holds the g plane and then the h plane.  In half storage the g and h
// values of a cell share one 32-bit word, g in the low half, so that one
// 4-byte access moves both populations of the cell.  cell_bytes: distance
// from one cell to the next; h_offset: where h sits relative to g.
constexpr uint32_t cell_bytes(size_t elem) { return elem == 2 ? 4u : (uint32_t)elem; }
constexpr uint32_t h_offset(size_t elem, uint32_t plane_bytes) {
    return elem == 2 ? 2u : plane_bytes;
}

// Register layout the lattice step takes by default.  D3Q107 in float or
// double splits g and h over lane pairs (214 values do not fit one lane);
// half storage keeps one cell per lane in both velocity sets, its 214 halves
// held as 107 g/h words.
constexpr bool default_split(int dim, int precision) {
    return dim == 3 && precision != LBM_FP16_SCALED;
}

// Collision parameters of a solve (lattice.cpp).  dt > 0 selects the
// finite-difference form: relaxation rates dt / tau, convection scale dt r / 6.
// energy_fix selects the energy-conserving collision (see collide_*).
Physics physics_of(int dim, double delta, double tau_f, double tau_g, double dt = 0.0,
                   bool energy_fix = false);

// Arguments of the readout kernel (moments and conservation partials).
struct ReadArgs {
    const void* src;
    int64_t N;
    int64_t P;                // plane stride of src in cells
    int32_t nx, ny, nz, nxy;
    uint32_t open_end;
    int32_t stream;           // 1: the source holds P_{n-1}; pull to get S_n
    double r;
    double rest_energy;       // (D + delta) / 2, added back in deviation storage
    double inv_dof;           // 1 / (D + delta): T = (2E - |u|^2) / (D + delta)
    double w[10];             // group weights (scaled storage is divided by them)
    double* rho;              // [N] or null
    double* u;                // [D][N] or null
    double* E;                // [N] or null
    double* T;                // [N] or null
    double* partials;         // [blocks][D + 2] or null
};

// Launch with the launch's own status (hipLaunchKernel), so that an error
// left behind by unrelated work in the process is not taken for ours.
template <typename... KArgs, typename... Args>
inline hipError_t launch_kernel(void (*kernel)(KArgs...), dim3 grid, dim3 block, hipStream_t s,
                         Args&&... args) {
    std::tuple<std::decay_t<KArgs>...> vals(std::forward<Args>(args)...);
    void* ptrs[sizeof...(KArgs) > 0 ? sizeof...(KArgs) : 1];
    std::apply([&](auto&... v) {
        int i = 0;
        ((ptrs[i++] = static_cast<void*>(&v)), ...);
    }, vals);
    return hipLaunchKernel(reinterpret_cast<const void*>(kernel), grid, block, ptrs, 0, s);
}

// Kernel launchers (kernels.hip).  `split` selects the layout in which one
// lane holds the g populations of a cell and its partner lane (lane ^ 32)
// the h populations.
hipError_t launch_init(int dim, int precision, void* dst, const double* rho,
                       const double* u, const double* T, int64_t N, int64_t stride,
                       double half_delta, double r, const double* w_group,
                       hipStream_t s);
// D3Q107 lattice step with the pulled rows staged in LDS (nx a multiple of
// 128, streaming steps only; hipErrorInvalidValue otherwise).
hipError_t launch_step_lds(int precision, const StepArgs& a, hipStream_t s);
hipError_t launch_step(int dim, int precision, bool split, const StepArgs& a,
                       hipStream_t s);
// One explicit finite-difference step (Sec. III); sets the wave mapping
// fields of a copy of `a`.
hipError_t launch_fd_step(int dim, int precision, bool split, const StepArgs& a,
                          hipStream_t s);
// The same step in two passes (fd.hip): a moments pass writing a per-cell
// record, then update passes over chunks of populations, which also leave
// the next step's record behind (record_valid: skip the moments pass).
// FP64 and FP32 deviation storage.
size_t fd_record_bytes(int dim, int precision, int64_t P);
hipError_t launch_fd_two_pass(int dim, int precision, const StepArgs& a, void* record,
                              bool record_valid, hipStream_t s);
int step_block_cells(int dim, int precision, bool split);
hipError_t launch_readout(int dim, int precision, const ReadArgs& a,
                          int blocks, hipStream_t s);
hipError_t launch_final_reduce(int dim, const double* partials, int blocks,
                               double* out, hipStream_t s);
constexpr int kReadBlock = 256;

}  // namespace lbm

struct lbm_solver;
namespace lbm {
// Readout of a solve's S_n into device outputs (any may be null), with the
// FP64 totals into the solve's own buffer when `totals` (api.hip).
int solver_readout(lbm_solver* h, double* rho, double* u, double* E, double* T, bool totals);
}  // namespace lbm

// The opaque handle.
struct lbm_solver {
    int dim, q, precision;
    int64_t nx, ny, nz, N;
    int64_t P;            // plane stride in cells (lbm::plane_stride)
    uint32_t bc;
    double gamma, delta, tau_f, tau_g;
    const lbm::LatticeTables* lat;
    size_t elem;          // bytes per stored value
    size_t buf_bytes;     // bytes of one ping-pong side (2 Q P elem)
    void* buf[2];         // ping-pong sides
    int cur;              // side holding the latest post-collision state
    bool have_state;
    bool initial;         // buf[cur ^ 1] holds S_0 itself (no step yet)
    int64_t steps;
    int scheme;           // 0: lattice (collide, stream), 1: finite differences
    int collision;        // LBM_COLLISION_PAPER or LBM_COLLISION_ENERGY_CONSERVING
    double dt;            // finite-difference time step (grid step 1, speeds r e)
    double* partials;     // readout block partials
    double* totals;       // [D + 2] final totals (device)
    int read_blocks;
    hipStream_t stream;
    hipStream_t own_stream;
    int device;
    bool split;
    bool lds;             // D3Q107 lattice step: pulled rows staged in LDS
    bool fd_fused;        // finite differences: one fused kernel (LANE / SPLIT variants)
    void* fd_record;      // finite differences, two passes: per-cell record
    bool fd_record_valid; // the record describes the current state
    size_t device_bytes;
};

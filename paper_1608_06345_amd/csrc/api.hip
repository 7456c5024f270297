// C ABI of liblbm: solve lifetime, initial fields, stepping and readouts.
// Every entry point validates its arguments on the host, checks every HIP
// call, and returns an lbm_status code; no exception crosses the boundary.
#include <cmath>
#include <cstring>
#include <new>

#include "lbm_internal.h"

using lbm::LatticeTables;

namespace {

int dev_err(hipError_t e) {
    if (e == hipSuccess) return LBM_OK;
    if (e == hipErrorOutOfMemory) return LBM_ENOMEM;
    return LBM_EDEVICE;
}

#define LBM_HIP(call)                          \
    do {                                       \
        const hipError_t e_ = (call);          \
        if (e_ != hipSuccess) return dev_err(e_); \
    } while (0)

// delta from gamma (Sec. II: gamma = (delta + D + 2) / (delta + D)).
bool delta_of(double gamma, int dim, double* delta) {
    if (!(gamma > 1.0) || !std::isfinite(gamma)) return false;
    double d = 2.0 / (gamma - 1.0) - dim;
    if (std::fabs(d) < 1e-9) d = 0.0;
    if (d < 0.0) return false;
    *delta = d;
    return true;
}

struct Shape {
    int dim, q, precision;
    int64_t nx, ny, nz, N, P;  // P: plane stride in cells
    size_t elem;
};

int check_shape(int dim, int velocity_set, int precision, int64_t nx, int64_t ny,
                int64_t nz, Shape* s) {
    if (dim == 2 && velocity_set != LBM_D2Q37) return LBM_EINVAL;
    if (dim == 3 && velocity_set != LBM_D3Q107) return LBM_EINVAL;
    if (dim != 2 && dim != 3) return LBM_EINVAL;
    if (precision != LBM_FP64 && precision != LBM_FP32_DEV && precision != LBM_FP16_SCALED)
        return LBM_EINVAL;
    if (nx < 1 || ny < 1 || nz < 1) return LBM_EINVAL;
    if (dim == 2 && nz != 1) return LBM_EINVAL;
    const size_t elem = precision == LBM_FP64 ? 8 : (precision == LBM_FP32_DEV ? 4 : 2);
    // one population plane (its stride included) must stay addressable with
    // 32-bit byte offsets: the kernels add a plane offset to a cell offset in
    // 32 bits
    if (nx > (1LL << 31) || ny > (1LL << 31) || nz > (1LL << 31)) return LBM_EINVAL;
    const double N = (double)nx * (double)ny * (double)nz;
    if (N * (double)elem > 2147483647.0) return LBM_EINVAL;
    const int64_t P = lbm::plane_stride(nx * ny * nz, elem, dim);
    if ((double)P * (double)elem > 2147483647.0) return LBM_EINVAL;
    s->dim = dim;
    s->q = velocity_set;
    s->precision = precision;
    s->nx = nx;
    s->ny = ny;
    s->nz = nz;
    s->N = nx * ny * nz;
    s->P = P;
    s->elem = elem;
    return LBM_OK;
}

int read_blocks_of(int64_t N) { return (int)((N + lbm::kReadBlock - 1) / lbm::kReadBlock); }

size_t footprint(const Shape& s) {
    const size_t side = 2 * (size_t)s.q * (size_t)s.P * s.elem;
    const size_t partial = (size_t)read_blocks_of(s.N) * (s.dim + 2) * sizeof(double);
    return 2 * side + partial + 8 * sizeof(double);
}

lbm::StepArgs step_args(const lbm_solver* h, const void* src, void* dst, bool stream) {
    lbm::StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.src = src;
    a.dst = dst;
    a.N = h->N;
    a.P = h->P;
    a.nx = (int32_t)h->nx;
    a.ny = (int32_t)h->ny;
    a.nz = (int32_t)h->nz;
    a.nxy = (int32_t)(h->nx * h->ny);
    a.open_end = (h->bc & 3u) | (((h->bc >> 2) & 3u) << 1) | (((h->bc >> 4) & 3u) << 2);
    a.stream = stream ? 1 : 0;
    a.ph = lbm::physics_of(h->dim, h->delta, h->tau_f, h->tau_g, h->scheme ? h->dt : 0.0,
                           h->collision == LBM_COLLISION_ENERGY_CONSERVING);
    return a;
}

// Readout of S_n into the given device outputs (any may be null).
int readout(lbm_solver* h, double* rho, double* u, double* E, double* T, bool totals) {
    lbm::ReadArgs a;
    std::memset(&a, 0, sizeof(a));
    // Lattice scheme: S_0 sits unstreamed in the idle side; later
    // S_n = Stream(P_{n-1}).  Finite differences: S_n itself is current.
    if (h->scheme) {
        a.src = h->buf[h->cur];
        a.stream = 0;
    } else {
        a.src = h->buf[h->cur ^ 1];
        a.stream = h->initial ? 0 : 1;
    }
    a.N = h->N;
    a.P = h->P;
    a.nx = (int32_t)h->nx;
    a.ny = (int32_t)h->ny;
    a.nz = (int32_t)h->nz;
    a.nxy = (int32_t)(h->nx * h->ny);
    a.open_end = (h->bc & 3u) | (((h->bc >> 2) & 3u) << 1) | (((h->bc >> 4) & 3u) << 2);
    a.r = h->lat->r;
    a.rest_energy = 0.5 * (h->dim + h->delta);
    a.inv_dof = 1.0 / (h->dim + h->delta);
    for (int g = 0; g < h->lat->groups; ++g) a.w[g] = h->lat->w_group[g];
    a.rho = rho;
    a.u = u;
    a.E = E;
    a.T = T;
    a.partials = totals ? h->partials : nullptr;
    LBM_HIP(lbm::launch_readout(h->dim, h->precision, a, h->read_blocks, h->stream));
    if (totals)
        LBM_HIP(lbm::launch_final_reduce(h->dim, h->partials, h->read_blocks, h->totals,
                                         h->stream));
    return LBM_OK;
}

int create_solver(int dim, int velocity_set, double gamma, double tau_f, double tau_g, double dt,
                  int64_t nx, int64_t ny, int64_t nz, uint32_t bc, int precision,
                  lbm_handle* out);

}  // namespace

int lbm::solver_readout(lbm_solver* h, double* rho, double* u, double* E, double* T,
                        bool totals) {
    return readout(h, rho, u, E, T, totals);
}

namespace {

// Finite differences, AUTO variant: the two-pass step, except for D2Q37 in
// FP64 on rows that are not whole 256-cell tiles.  There the fused kernel's
// neighbour rows still fit the L2 and it streams faster than the two-pass
// step with its one-lane update kernel (measured on 4096^2: 5.9 ms fused,
// 8.7 ms two-pass with that kernel); with the LDS-staged update the
// two-pass step is faster (5.4-5.6 ms).  D3Q107 FP32 256^3: 31.7 ms fused,
// 10.2 ms two-pass.
bool fd_fused_by_default(int dim, int precision, int64_t nx) {
    return dim == 2 && precision == LBM_FP64 && nx % 256 != 0;
}

}  // namespace

extern "C" {

const char* lbm_strerror(int code) {
    switch (code) {
        case LBM_OK: return "success";
        case LBM_EINVAL: return "invalid argument";
        case LBM_ENOMEM: return "out of device memory";
        case LBM_EDEVICE: return "HIP runtime error";
        case LBM_ESTATE: return "call out of order (no initial fields)";
        case LBM_ENONFINITE: return "non-finite conservation total";
        case LBM_EBUSY: return "no free pool slot or arena space now";
        case LBM_ESCRATCH: return "grid exceeds the no-allocation readout's 64 MiB scratch";
        default: return "unknown status";
    }
}

int lbm_lattice(int velocity_set, int8_t* e, double* w, double* r) {
    int dim;
    if (velocity_set == LBM_D2Q37) dim = 2;
    else if (velocity_set == LBM_D3Q107) dim = 3;
    else return LBM_EINVAL;
    const LatticeTables& t = lbm::lattice_tables(dim);
    for (int i = 0; i < t.q; ++i) {
        if (e) {
            e[3 * i + 0] = t.e[i][0];
            e[3 * i + 1] = t.e[i][1];
            e[3 * i + 2] = t.e[i][2];
        }
        if (w) w[i] = t.w[i];
    }
    if (r) *r = t.r;
    return t.q;
}

size_t lbm_footprint_bytes(int dim, int velocity_set, int precision, int64_t nx, int64_t ny,
                           int64_t nz) {
    Shape s;
    if (check_shape(dim, velocity_set, precision, nx, ny, nz, &s) != LBM_OK) return 0;
    return footprint(s);
}

int lbm_create_ex(int dim, int velocity_set, double gamma, double tau_f, double tau_g,
                  int64_t nx, int64_t ny, int64_t nz, uint32_t bc, int precision,
                  lbm_handle* out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    if (!(tau_f > 0.5) || !(tau_g > 0.5) || !std::isfinite(tau_f) || !std::isfinite(tau_g))
        return LBM_EINVAL;
    return create_solver(dim, velocity_set, gamma, tau_f, tau_g, 0.0, nx, ny, nz, bc, precision,
                         out);
}

int lbm_create_fd(int dim, int velocity_set, double gamma, double tau_f, double tau_g, double dt,
                  int64_t nx, int64_t ny, int64_t nz, uint32_t bc, int precision,
                  lbm_handle* out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    if (dim != 2 && dim != 3) return LBM_EINVAL;
    const double r = lbm::lattice_tables(dim).r;
    if (!std::isfinite(dt) || !(dt > 0.0) || dt * 3.0 * r > 1.0 + 1e-12) return LBM_EINVAL;
    if (!std::isfinite(tau_f) || !std::isfinite(tau_g) || !(tau_f > 0.0) || !(tau_g > 0.0) ||
        dt > tau_f || dt > tau_g)
        return LBM_EINVAL;
    // Half storage re-rounds every value each step, and the stable time step
    // of this form is ~10x shorter than a lattice step: the rounding, then
    // differenced with weights up to 6, costs percents of the velocity.
    if (precision == LBM_FP16_SCALED) return LBM_EINVAL;
    return create_solver(dim, velocity_set, gamma, tau_f, tau_g, dt, nx, ny, nz, bc, precision,
                         out);
}

}  // extern "C"

namespace {

int create_solver(int dim, int velocity_set, double gamma, double tau_f, double tau_g, double dt,
                  int64_t nx, int64_t ny, int64_t nz, uint32_t bc, int precision,
                  lbm_handle* out) {
    Shape s;
    int rc = check_shape(dim, velocity_set, precision, nx, ny, nz, &s);
    if (rc != LBM_OK) return rc;
    double delta;
    if (!delta_of(gamma, dim, &delta)) return LBM_EINVAL;
    if (bc & ~0x3Fu) return LBM_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (((bc >> (2 * k)) & 3u) > LBM_BC_ZERO_GRADIENT) return LBM_EINVAL;
    if (dim == 2 && ((bc >> 4) & 3u) != LBM_BC_PERIODIC) return LBM_EINVAL;

    lbm_solver* h = new (std::nothrow) lbm_solver;
    if (!h) return LBM_ENOMEM;
    std::memset(h, 0, sizeof(*h));
    h->dim = dim;
    h->q = velocity_set;
    h->precision = precision;
    h->nx = nx;
    h->ny = ny;
    h->nz = nz;
    h->N = s.N;
    h->P = s.P;
    h->bc = bc;
    h->gamma = gamma;
    h->delta = delta;
    h->tau_f = tau_f;
    h->tau_g = tau_g;
    h->scheme = dt > 0.0 ? 1 : 0;
    h->dt = dt;
    h->lat = &lbm::lattice_tables(dim);
    h->elem = s.elem;
    h->buf_bytes = 2 * (size_t)s.q * (size_t)s.P * s.elem;
    h->read_blocks = read_blocks_of(s.N);
    // one lane per cell keeps all 2Q populations in registers; for D3Q107
    // in float or double that is 214 values, so those kernels split g and h
    // across lane pairs (half storage holds them as 107 g/h words)
    h->split = lbm::default_split(dim, precision);
    h->lds = false;
    h->fd_fused = fd_fused_by_default(dim, precision, nx);
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        delete h;
        return dev_err(e);
    }
    e = hipMalloc(&h->buf[0], h->buf_bytes);
    if (e == hipSuccess) e = hipMalloc(&h->buf[1], h->buf_bytes);
    if (e == hipSuccess && h->scheme)
        e = hipMalloc(&h->fd_record, lbm::fd_record_bytes(dim, precision, s.P));
    if (e == hipSuccess)
        e = hipMalloc((void**)&h->partials, (size_t)h->read_blocks * (dim + 2) * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&h->totals, 8 * sizeof(double));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        lbm_destroy(h);
        return dev_err(e);
    }
    h->stream = h->own_stream;
    h->device_bytes = footprint(s) + (h->scheme ? lbm::fd_record_bytes(dim, precision, s.P) : 0);
    *out = h;
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_create(int dim, int velocity_set, double gamma, double tau_f, double tau_g, int64_t nx,
               int64_t ny, int64_t nz, uint32_t bc, lbm_handle* out) {
    return lbm_create_ex(dim, velocity_set, gamma, tau_f, tau_g, nx, ny, nz, bc, LBM_FP64, out);
}

int lbm_destroy(lbm_handle h) {
    if (!h) return LBM_OK;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->buf[0]) (void)hipFree(h->buf[0]);
    if (h->buf[1]) (void)hipFree(h->buf[1]);
    if (h->partials) (void)hipFree(h->partials);
    if (h->totals) (void)hipFree(h->totals);
    if (h->fd_record) (void)hipFree(h->fd_record);
    if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
    delete h;
    return LBM_OK;
}

int lbm_set_stream(lbm_handle h, void* stream) {
    if (!h) return LBM_EINVAL;
    h->stream = static_cast<hipStream_t>(stream);
    return LBM_OK;
}

int lbm_set_variant(lbm_handle h, int variant) {
    if (!h) return LBM_EINVAL;
    switch (variant) {
        case LBM_VARIANT_AUTO:
            h->split = lbm::default_split(h->dim, h->precision);
            h->fd_fused = fd_fused_by_default(h->dim, h->precision, h->nx);
            h->lds = false;
            return LBM_OK;
        case LBM_VARIANT_LANE:
            h->split = false;
            h->fd_fused = true;
            h->lds = false;
            return LBM_OK;
        case LBM_VARIANT_SPLIT:
            h->split = true;
            h->fd_fused = true;
            h->lds = false;
            return LBM_OK;
        case LBM_VARIANT_TWO_PASS:
            if (!h->scheme) return LBM_EINVAL;
            h->fd_fused = false;
            h->lds = false;
            return LBM_OK;
        case LBM_VARIANT_SPLIT_LDS:
            if (h->scheme || h->dim != 3 || h->nx % 128 != 0) return LBM_EINVAL;
            h->split = true;
            h->lds = true;
            return LBM_OK;
        default: return LBM_EINVAL;
    }
}

int lbm_set_collision(lbm_handle h, int mode) {
    if (!h) return LBM_EINVAL;
    if (mode != LBM_COLLISION_PAPER && mode != LBM_COLLISION_ENERGY_CONSERVING)
        return LBM_EINVAL;
    // the lattice scheme stores post-collision states: a state collided in
    // one mode cannot continue in the other
    if (h->have_state) return LBM_ESTATE;
    h->collision = mode;
    return LBM_OK;
}

int lbm_synchronize(lbm_handle h) {
    if (!h) return LBM_EINVAL;
    LBM_HIP(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

int lbm_init_fields_dev(lbm_handle h, const double* rho, const double* u, const double* T) {
    if (!h || !rho || !u || !T) return LBM_EINVAL;
    // S_0 into side 0; P_0 = Collide(S_0) into side 1 (same collision code as
    // every step, with the pull switched off).
    LBM_HIP(lbm::launch_init(h->dim, h->precision, h->buf[0], rho, u, T, h->N, h->P,
                             0.5 * h->delta, h->lat->r, h->lat->w_group, h->stream));
    if (h->scheme) {  // finite differences keep S_n itself
        h->fd_record_valid = false;
        h->cur = 0;
        h->initial = true;
        h->have_state = true;
        h->steps = 0;
        return LBM_OK;
    }
    const lbm::StepArgs a = step_args(h, h->buf[0], h->buf[1], false);
    LBM_HIP(lbm::launch_step(h->dim, h->precision, h->split, a, h->stream));
    h->cur = 1;
    h->initial = true;
    h->have_state = true;
    h->steps = 0;
    return LBM_OK;
}

int lbm_init_fields(lbm_handle h, const double* rho, const double* u, const double* T) {
    if (!h || !rho || !u || !T) return LBM_EINVAL;
    const size_t n = (size_t)h->N * sizeof(double);
    double* d = nullptr;
    LBM_HIP(hipMalloc((void**)&d, n * (2 + h->dim)));
    hipError_t e = hipMemcpyAsync(d, rho, n, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d + h->N, T, n, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d + 2 * h->N, u, n * h->dim, hipMemcpyHostToDevice, h->stream);
    int rc = dev_err(e);
    if (rc == LBM_OK) rc = lbm_init_fields_dev(h, d, d + 2 * h->N, d + h->N);
    const hipError_t es = hipStreamSynchronize(h->stream);
    (void)hipFree(d);
    if (rc != LBM_OK) return rc;
    return dev_err(es);
}

int lbm_step(lbm_handle h, int64_t n) {
    if (!h || n < 0) return LBM_EINVAL;
    if (!h->have_state) return LBM_ESTATE;
    for (int64_t k = 0; k < n; ++k) {
        const lbm::StepArgs a = step_args(h, h->buf[h->cur], h->buf[h->cur ^ 1], true);
        if (h->scheme && h->fd_fused) {
            LBM_HIP(lbm::launch_fd_step(h->dim, h->precision, h->split, a, h->stream));
            h->fd_record_valid = false;
        } else if (h->scheme) {
            LBM_HIP(lbm::launch_fd_two_pass(h->dim, h->precision, a, h->fd_record,
                                            h->fd_record_valid, h->stream));
            h->fd_record_valid = true;
        } else if (h->lds)
            LBM_HIP(lbm::launch_step_lds(h->precision, a, h->stream));
        else
            LBM_HIP(lbm::launch_step(h->dim, h->precision, h->split, a, h->stream));
        h->cur ^= 1;
        h->initial = false;
        ++h->steps;
    }
    return LBM_OK;
}

int lbm_moments_dev(lbm_handle h, double* rho, double* u, double* E) {
    if (!h || !rho || !u || !E) return LBM_EINVAL;
    if (!h->have_state) return LBM_ESTATE;
    return readout(h, rho, u, E, nullptr, false);
}

int lbm_moments(lbm_handle h, double* rho, double* u, double* E) {
    if (!h || !rho || !u || !E) return LBM_EINVAL;
    if (!h->have_state) return LBM_ESTATE;
    const size_t n = (size_t)h->N * sizeof(double);
    double* d = nullptr;
    LBM_HIP(hipMalloc((void**)&d, n * (2 + h->dim)));
    int rc = readout(h, d, d + 2 * h->N, d + h->N, nullptr, false);
    hipError_t e = hipSuccess;
    if (rc == LBM_OK) e = hipMemcpyAsync(rho, d, n, hipMemcpyDeviceToHost, h->stream);
    if (rc == LBM_OK && e == hipSuccess)
        e = hipMemcpyAsync(E, d + h->N, n, hipMemcpyDeviceToHost, h->stream);
    if (rc == LBM_OK && e == hipSuccess)
        e = hipMemcpyAsync(u, d + 2 * h->N, n * h->dim, hipMemcpyDeviceToHost, h->stream);
    const hipError_t es = hipStreamSynchronize(h->stream);
    (void)hipFree(d);
    if (rc != LBM_OK) return rc;
    if (e != hipSuccess) return dev_err(e);
    return dev_err(es);
}

int lbm_temperature_dev(lbm_handle h, double* T) {
    if (!h || !T) return LBM_EINVAL;
    if (!h->have_state) return LBM_ESTATE;
    return readout(h, nullptr, nullptr, nullptr, T, false);
}

int lbm_temperature(lbm_handle h, double* T) {
    if (!h || !T) return LBM_EINVAL;
    if (!h->have_state) return LBM_ESTATE;
    const size_t n = (size_t)h->N * sizeof(double);
    double* d = nullptr;
    LBM_HIP(hipMalloc((void**)&d, n));
    int rc = readout(h, nullptr, nullptr, nullptr, d, false);
    hipError_t e = hipSuccess;
    if (rc == LBM_OK) e = hipMemcpyAsync(T, d, n, hipMemcpyDeviceToHost, h->stream);
    const hipError_t es = hipStreamSynchronize(h->stream);
    (void)hipFree(d);
    if (rc != LBM_OK) return rc;
    if (e != hipSuccess) return dev_err(e);
    return dev_err(es);
}

int lbm_totals(lbm_handle h, double* mass, double* mom, double* energy) {
    if (!h || !mass || !mom || !energy) return LBM_EINVAL;
    if (!h->have_state) return LBM_ESTATE;
    int rc = readout(h, nullptr, nullptr, nullptr, nullptr, true);
    if (rc != LBM_OK) return rc;
    double t[8];
    LBM_HIP(hipMemcpyAsync(t, h->totals, (h->dim + 2) * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream));
    LBM_HIP(hipStreamSynchronize(h->stream));
    *mass = t[0];
    for (int k = 0; k < h->dim; ++k) mom[k] = t[1 + k];
    *energy = t[h->dim + 1];
    for (int k = 0; k < h->dim + 2; ++k)
        if (!std::isfinite(t[k])) return LBM_ENONFINITE;
    return LBM_OK;
}

int lbm_get_info(lbm_handle h, lbm_info* info) {
    if (!h || !info) return LBM_EINVAL;
    info->dim = h->dim;
    info->q = h->q;
    info->precision = h->precision;
    info->nx = h->nx;
    info->ny = h->ny;
    info->nz = h->nz;
    info->bc = h->bc;
    info->gamma = h->gamma;
    info->delta = h->delta;
    info->tau_f = h->tau_f;
    info->tau_g = h->tau_g;
    info->r = h->lat->r;
    info->steps = h->steps;
    info->device_bytes = h->device_bytes;
    info->scheme = h->scheme;
    info->dt = h->dt;
    info->collision = h->collision;
    return LBM_OK;
}

}  // extern "C"

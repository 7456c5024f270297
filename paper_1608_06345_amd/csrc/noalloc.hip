// lbm_moments_noalloc: lbm_moments without any device allocation.
//
// lbm_moments stages rho, u and E of the whole grid in a device buffer it
// allocates and frees on every call.  This variant stages them in a
// file-scope device array instead, whose device address is looked up once
// per device (hipGetSymbolAddress, with that device current) and kept; the
// readout kernel is lbm_moments' own, so the results are bit for bit the
// same.  Every call on one device shares that device's array: calls that
// overlap on one device (two host threads, two streams) race.
#include <cstring>
#include <mutex>

#include "lbm_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // (2 + D) doubles per cell
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int status_of(hipError_t e) {
    if (e == hipSuccess) return LBM_OK;
    if (e == hipErrorOutOfMemory) return LBM_ENOMEM;
    return LBM_EDEVICE;
}

// Device address of `scratch` on the current device `dev` (looked up on the
// first call there).  The array's name is a host-side stand-in; only this
// address may reach a kernel or a copy.
int scratch_address(int dev, double** out) {
    if (dev < 0 || dev >= kMaxDevices) return LBM_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return e != hipSuccess ? status_of(e) : LBM_EDEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<double*>(g_scratch_ptr[dev]);
    return LBM_OK;
}

int moments_noalloc(lbm_solver* h, double* rho, double* u, double* E) {
    double* d = nullptr;
    int rc = scratch_address(h->device, &d);
    if (rc != LBM_OK) return rc;
    const int64_t N = h->N;
    const size_t n = (size_t)N * sizeof(double);
    // layout of the staged fields: rho [N], E [N], u [dim][N]
    rc = lbm::solver_readout(h, d, d + 2 * N, d + N, nullptr, false);
    hipError_t e = hipSuccess;
    if (rc == LBM_OK) e = hipMemcpyAsync(rho, d, n, hipMemcpyDeviceToHost, h->stream);
    if (rc == LBM_OK && e == hipSuccess)
        e = hipMemcpyAsync(E, d + N, n, hipMemcpyDeviceToHost, h->stream);
    if (rc == LBM_OK && e == hipSuccess)
        e = hipMemcpyAsync(u, d + 2 * N, n * h->dim, hipMemcpyDeviceToHost, h->stream);
    const hipError_t es = hipStreamSynchronize(h->stream);
    if (rc != LBM_OK) return rc;
    if (e != hipSuccess) return status_of(e);
    return status_of(es);
}

}  // namespace

extern "C" int lbm_moments_noalloc(lbm_handle h, double* rho, double* u, double* E) {
    if (!h || !rho || !u || !E) return LBM_EINVAL;
    if (!h->have_state) return LBM_ESTATE;
    if ((size_t)h->N * (size_t)(2 + h->dim) * sizeof(double) > kScratchBytes)
        return LBM_ESCRATCH;
    // the solve's device is current for the lookup and the work, then the
    // caller's device is restored
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return status_of(e);
    if (cur != h->device) {
        e = hipSetDevice(h->device);
        if (e != hipSuccess) return status_of(e);
    }
    const int rc = moments_noalloc(h, rho, u, E);
    if (cur != h->device) {
        e = hipSetDevice(cur);
        if (rc == LBM_OK && e != hipSuccess) return status_of(e);
    }
    return rc;
}

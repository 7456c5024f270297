// HBM ceiling probes (include/hbm_probe.h): a streaming copy and a read-only
// sweep, 16 bytes per lane access, in a few launch shapes; and the D3Q107
// step's own memory access shape with no arithmetic.  Workgroup b
// covers U * 256 consecutive 16-byte elements, lane t the elements
// b U 256 + k 256 + t (k < U): every wave access is one contiguous 1 KiB, and
// a lane has U loads in flight before its first store.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "hbm_probe.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

template <int U, bool NT>
__global__ __launch_bounds__(256) void k_probe_copy(f4* __restrict__ dst,
                                                     const f4* __restrict__ src, int64_t n) {
    const int64_t base = (int64_t)blockIdx.x * (U * 256) + threadIdx.x;
    f4 v[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const int64_t i = base + (int64_t)k * 256;
        if (i < n) v[k] = NT ? __builtin_nontemporal_load(src + i) : src[i];
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const int64_t i = base + (int64_t)k * 256;
        if (i < n) {
            if constexpr (NT)
                __builtin_nontemporal_store(v[k], dst + i);
            else
                dst[i] = v[k];
        }
    }
}

template <int U, bool NT>
__global__ __launch_bounds__(256) void k_probe_read(const f4* __restrict__ src, int64_t n,
                                                     float* sink) {
    const int64_t base = (int64_t)blockIdx.x * (U * 256) + threadIdx.x;
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const int64_t i = base + (int64_t)k * 256;
        if (i < n) {
            const f4 v = NT ? __builtin_nontemporal_load(src + i) : src[i];
            acc += (v.x + v.y) + (v.z + v.w);
        }
    }
    // -0x1.fffffep127 is reached by no sum of ordinary data
    if (acc == -3.40282347e38f) sink[threadIdx.x] = acc;
}

// The memory access shape of the D3Q107 split step kernel with no
// arithmetic: a workgroup of four waves serves 128 cells of one x-row, a
// wave 32 of them, lanes 0..31 reading plane 2i and lanes 32..63 plane 2i+1
// of each of the 107 population pairs (one 4-byte value per lane and
// plane), all loads issued before the stores; workgroup b runs on XCD b % 8,
// whose turns walk whole rows.  Each value is written back to the same
// place in the other buffer.
constexpr int kPatternPlanes = 214;

__global__ __launch_bounds__(256) void k_probe_planes(const float* __restrict__ src,
                                                      float* __restrict__ dst, int64_t stride,
                                                      int rows, int tiles_per_row, int nx) {
    const int b = (int)blockIdx.x, j = b >> 3;
    const int row = (j / tiles_per_row) * 8 + (b & 7);
    if (row >= rows) return;
    const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int x = (j % tiles_per_row) * 128 + wave * 32 + (lane & 31);
    const int64_t cell = (int64_t)row * nx + x;
    const int role = lane >> 5;
    float v[kPatternPlanes / 2];
#pragma unroll
    for (int i = 0; i < kPatternPlanes / 2; ++i) v[i] = src[(int64_t)(2 * i + role) * stride + cell];
    // a data-dependent factor of one keeps every store a computed value
    const float one = v[0] == -3.40282347e38f ? 0.5f : 1.0f;
#pragma unroll
    for (int i = 0; i < kPatternPlanes / 2; ++i)
        __builtin_nontemporal_store(v[i] * one, dst + (int64_t)(2 * i + role) * stride + cell);
}

struct Variant {
    const char* name;
    int unroll;
    bool nt;
};
constexpr Variant kVariants[] = {
    {"u1", 1, false}, {"u4", 4, false}, {"u4_nt", 4, true}, {"u8_nt", 8, true}, {"u16_nt", 16, true}};
constexpr int kNumVariants = (int)(sizeof(kVariants) / sizeof(kVariants[0]));

// Launch with the launch's own status; the arguments have the kernel's
// parameter types exactly.
template <typename... A>
hipError_t launch(const void* kernel, dim3 grid, hipStream_t s, A... args) {
    void* ptrs[] = {static_cast<void*>(&args)...};
    return hipLaunchKernel(kernel, grid, dim3(256), ptrs, 0, s);
}

hipError_t launch_copy(int variant, f4* dst, const f4* src, int64_t n, hipStream_t s) {
    const Variant v = kVariants[variant];
    const int64_t per = (int64_t)v.unroll * 256;
    const int64_t grid = (n + per - 1) / per;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 g((unsigned)grid);
    const void* k;
    switch (variant) {
        case 0: k = reinterpret_cast<const void*>(&k_probe_copy<1, false>); break;
        case 1: k = reinterpret_cast<const void*>(&k_probe_copy<4, false>); break;
        case 2: k = reinterpret_cast<const void*>(&k_probe_copy<4, true>); break;
        case 3: k = reinterpret_cast<const void*>(&k_probe_copy<8, true>); break;
        default: k = reinterpret_cast<const void*>(&k_probe_copy<16, true>); break;
    }
    return launch(k, g, s, dst, src, n);
}

hipError_t launch_read(int variant, const f4* src, int64_t n, float* sink, hipStream_t s) {
    const Variant v = kVariants[variant];
    const int64_t per = (int64_t)v.unroll * 256;
    const int64_t grid = (n + per - 1) / per;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 g((unsigned)grid);
    const void* k;
    switch (variant) {
        case 0: k = reinterpret_cast<const void*>(&k_probe_read<1, false>); break;
        case 1: k = reinterpret_cast<const void*>(&k_probe_read<4, false>); break;
        case 2: k = reinterpret_cast<const void*>(&k_probe_read<4, true>); break;
        case 3: k = reinterpret_cast<const void*>(&k_probe_read<8, true>); break;
        default: k = reinterpret_cast<const void*>(&k_probe_read<16, true>); break;
    }
    return launch(k, g, s, src, n, sink);
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

extern "C" {

int hbm_probe_variants(int kind) { return kind == 0 || kind == 1 ? kNumVariants : -1; }

const char* hbm_probe_variant_name(int kind, int variant) {
    if ((kind != 0 && kind != 1) || variant < 0 || variant >= kNumVariants) return nullptr;
    return kVariants[variant].name;
}

int hbm_probe_copy(void* dst, const void* src, size_t bytes, int variant, void* stream) {
    if (!dst || !src || bytes == 0 || bytes % 16 || !aligned16(dst) || !aligned16(src))
        return -1;
    if (variant < 0 || variant >= kNumVariants) return -1;
    const char* d = static_cast<const char*>(dst);
    const char* s = static_cast<const char*>(src);
    if (d < s + bytes && s < d + bytes) return -1;  // overlapping ranges
    const hipError_t e = launch_copy(variant, static_cast<f4*>(dst), static_cast<const f4*>(src),
                                     (int64_t)(bytes / 16), static_cast<hipStream_t>(stream));
    return e == hipSuccess ? 0 : -3;
}

int hbm_probe_planes(void* dst, const void* src, int64_t cells, int64_t stride, int nx,
                     void* stream) {
    if (!dst || !src || cells < 1 || nx < 128 || nx % 128 || cells % nx || stride < cells)
        return -1;
    if (!aligned16(dst) || !aligned16(src)) return -1;
    const size_t bytes = (size_t)kPatternPlanes * (size_t)stride * sizeof(float);
    const char* d = static_cast<const char*>(dst);
    const char* sp = static_cast<const char*>(src);
    if (d < sp + bytes && sp < d + bytes) return -1;
    const int64_t rows = cells / nx;
    const int tiles = nx / 128;
    const int64_t grid = 8 * (int64_t)tiles * ((rows + 7) / 8);
    if (grid > 0x7fffffff || rows > 0x7fffffff) return -1;
    const hipError_t e = launch(reinterpret_cast<const void*>(&k_probe_planes), dim3((unsigned)grid),
                                static_cast<hipStream_t>(stream), static_cast<const float*>(src),
                                static_cast<float*>(dst), stride, (int)rows, tiles, nx);
    return e == hipSuccess ? 0 : -3;
}

int hbm_probe_read(const void* src, size_t bytes, int variant, float* sink, void* stream) {
    if (!src || !sink || bytes == 0 || bytes % 16 || !aligned16(src)) return -1;
    if (variant < 0 || variant >= kNumVariants) return -1;
    const hipError_t e = launch_read(variant, static_cast<const f4*>(src), (int64_t)(bytes / 16),
                                     sink, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? 0 : -3;
}

}  // extern "C"

/*
 * libhbmprobe -- HBM ceiling probes used by the benchmark beside the
 * solver's own kernels: a streaming copy and a read-only sweep of a device
 * buffer of known size, 16 bytes per lane access.  They measure what plain
 * data movement reaches on the device, the practical ceiling against which
 * the bandwidth-bound step kernels of liblbm are read.  Not part of the
 * solver: liblbm neither links nor calls them.
 *
 * Every call returns 0 on success, -1 (invalid argument) or -3 (a HIP call
 * failed); launches are asynchronous on `stream` (a hipStream_t, NULL for the
 * null stream).  Buffers are device memory owned by the caller.
 */
#ifndef HBM_PROBE_H
#define HBM_PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Number of copy / read kernel variants (launch shapes); variant ids run
 * from 0 to this number minus one.  kind: 0 copy, 1 read. */
int hbm_probe_variants(int kind);

/* Short name of a variant (static string), NULL for an unknown one. */
const char *hbm_probe_variant_name(int kind, int variant);

/* dst[0 .. bytes) = src[0 .. bytes).  bytes a positive multiple of 16, both
 * pointers 16-byte aligned, the ranges disjoint.  HBM traffic: 2 * bytes. */
int hbm_probe_copy(void *dst, const void *src, size_t bytes, int variant,
                   void *stream);

/* Read src[0 .. bytes) as floats and sum them per lane; `sink` (device, at
 * least 256 floats) receives a lane's sum only if it equals a value no sum
 * of ordinary data reaches, so the loads cannot be dropped and nothing is
 * written in practice.  HBM traffic: bytes. */
int hbm_probe_read(const void *src, size_t bytes, int variant, float *sink,
                   void *stream);

/* The memory access shape of the D3Q107 split step kernel, with no
 * arithmetic: 214 planes of `cells` floats, plane k starting at
 * src + k * stride floats, are read and written to the same places of dst.
 * A wave serves 32 cells of one x-row of nx cells (lanes 0..31 plane 2i,
 * lanes 32..63 plane 2i + 1 of each pair, one 4-byte value per lane and
 * plane), loading all 214 values before storing them; workgroups of four
 * waves are dealt to the XCDs by whole rows, as the step does.  nx a
 * multiple of 128, cells a multiple of nx, stride >= cells, both buffers
 * 16-byte aligned, 214 * stride floats each and disjoint.  HBM traffic:
 * 2 * 214 * cells * 4 bytes, the step's algorithmic bytes. */
int hbm_probe_planes(void *dst, const void *src, int64_t cells, int64_t stride,
                     int nx, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HBM_PROBE_H */

/*
 * yoro_measure.h -- a kernel that measures the machine rather than the
 * method: the practical HBM ceiling for the warp's access pattern.
 *
 * The plain warp + fill moves 4 B of depth and 4 B of RGBA in and 4 B of
 * RGBA out per pixel.  yoro_measure_stream moves the same bytes with no
 * computation in between, so its bandwidth is what a kernel with that
 * pattern can reach on this GPU; the warp kernel's bandwidth divided by it is
 * its fraction of that practical ceiling (beside its fraction of the vendor
 * figure).
 *
 * Conventions as in yoro.h: caller-owned device pointers, no allocation or
 * synchronisation, work queued on the given stream, YORO_ERR_INVALID_ARG
 * before anything is queued, YORO_ERR_DEVICE on a failed launch.
 */
#ifndef YORO_MEASURE_H
#define YORO_MEASURE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* c[i] = a[i] ^ b[i] for i < n (u32 words): two 4-byte reads and one 4-byte
 * write per element, as 16-byte non-temporal loads and stores, one group of
 * four elements per thread over a grid that covers the buffers once.
 * a, b, c: device, 16-byte aligned, c not overlapping a or b;
 * 1 <= n < 2^41. */
int32_t yoro_measure_stream(const uint32_t* a, const uint32_t* b, uint32_t* c, int64_t n, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* YORO_MEASURE_H */

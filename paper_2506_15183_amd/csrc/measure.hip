// The streaming kernel of include/yoro_measure.h: the warp's access pattern
// (two 4-byte reads, one 4-byte write per element) with nothing in between.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "yoro.h"
#include "yoro_internal.h"
#include "yoro_measure.h"

namespace {

typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));

// One 16-byte group per thread over a grid that covers the buffers once: the
// workgroups run in launch order, so the addresses in flight stay in one
// window of memory.  (A persistent grid-stride loop measured 10-25 % slower:
// its workgroups drift apart over the buffers.)
__global__ __launch_bounds__(256) void stream_kernel(const u32x4v* __restrict__ a, const u32x4v* __restrict__ b,
                                                     u32x4v* __restrict__ c, int64_t groups) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < groups) __builtin_nontemporal_store(__builtin_nontemporal_load(a + g) ^ __builtin_nontemporal_load(b + g), c + g);
}

__global__ __launch_bounds__(64) void stream_tail_kernel(const uint32_t* a, const uint32_t* b, uint32_t* c, int64_t first,
                                                         int64_t n) {
  const int64_t i = first + threadIdx.x;
  if (i < n) c[i] = a[i] ^ b[i];
}

bool al16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

extern "C" int32_t yoro_measure_stream(const uint32_t* a, const uint32_t* b, uint32_t* c, int64_t n,
                                       void* hip_stream) {
  if (!a || !b || !c || n <= 0 || !al16(a) || !al16(b) || !al16(c)) {
    yoro::set_last_error("yoro_measure_stream: null or misaligned pointer, or n < 1");
    return YORO_ERR_INVALID_ARG;
  }
  const uintptr_t lo = (uintptr_t)c, hi = lo + 4 * (uintptr_t)n;
  auto over = [&](const void* p) { return (uintptr_t)p < hi && lo < (uintptr_t)p + 4 * (uintptr_t)n; };
  if (over(a) || over(b)) {
    yoro::set_last_error("yoro_measure_stream: c overlaps an input");
    return YORO_ERR_INVALID_ARG;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t groups = n / 4;
  if ((groups + 255) / 256 > 0x7FFFFFFFLL) {
    yoro::set_last_error("yoro_measure_stream: n too large");
    return YORO_ERR_INVALID_ARG;
  }
  if (groups > 0) {
    const int grid = (int)((groups + 255) / 256);
    hipLaunchKernelGGL(stream_kernel, dim3(grid), dim3(256), 0, s, reinterpret_cast<const u32x4v*>(a),
                       reinterpret_cast<const u32x4v*>(b), reinterpret_cast<u32x4v*>(c), groups);
  }
  if (n % 4) hipLaunchKernelGGL(stream_tail_kernel, dim3(1), dim3(64), 0, s, a, b, c, groups * 4, n);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    yoro::set_last_error("yoro_measure_stream: launch failed");
    return YORO_ERR_DEVICE;
  }
  return YORO_OK;
}

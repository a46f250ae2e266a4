// Reprojection through a general pose (Section 6: the rotation matrix of a
// unit quaternion, the view and projection matrices, and the reprojection
// M = (VP_src)^-1 VP_tgt), for eyes that are rotated or moved along any axis
// (toed-in stereo, head motion).  The shift is no longer one-signed along a
// row, so the depth test spans the whole frame:
//   1  fill the caller's key buffer (one u64 per target pixel) with EMPTY;
//   2  scatter: per source pixel, the pinhole point of its planar depth,
//      X_t = A X + b with A = R^T, b = -R^T t (the target eye's pose in the
//      source eye's frame), the perspective divide, roundf of both
//      coordinates, and a global 64-bit atomicMin of
//      (target depth bits << 32) | source index;
//   3  resolve + fill per target row in LDS: a reached key gathers its
//      source pixel's RGBA, then the direct path's row fill (row_common.h).
// FP32 with each operation rounded once, in the order the oracle states.
//
// HBM traffic per pixel: 4 B depth read + 8 B key atomic (read-modify-write
// in the L2 / memory) in the scatter, 8 B key read + 4 B RGBA gathered +
// 4 B RGBA written (+4 B depth, +1 B mask) in the resolve, and 8 B written
// by the clear.
#include <algorithm>

#include "row_common.h"

namespace yoro {
namespace {

__global__ __launch_bounds__(kThreads) void pose_clear_kernel(uint64_t* keys, size_t n) {
  const size_t n2 = n / 2;
  ulonglong2* k2 = reinterpret_cast<ulonglong2*>(keys);  // the buffer is 16-byte aligned
  const ulonglong2 e = make_ulonglong2(kEmpty, kEmpty);
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < n2; i += (size_t)gridDim.x * kThreads) k2[i] = e;
  if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) keys[n - 1] = kEmpty;
}

__global__ __launch_bounds__(kThreads) void pose_scatter_kernel(const float* __restrict__ src_depth, PoseGeom g,
                                                                 uint64_t* keys) {
  const size_t n = (size_t)g.width * (size_t)g.height;
  const float Wf = (float)g.width, Hf = (float)g.height;
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads) {
    const int y = (int)(i / (size_t)g.width);
    const int x = (int)(i - (size_t)y * (size_t)g.width);
    const float z = __builtin_nontemporal_load(&src_depth[i]);
    const float a = ((float)x - g.cx) / g.f;
    const float c = ((float)y - g.cy) / g.f;
    float Xt, Yt, Zt, depth;
    bool ok;
    if (z == __builtin_inff()) {  // a point at infinity: the rotation alone moves it
      Xt = (g.A[0] * a + g.A[1] * c) + g.A[2];
      Yt = (g.A[3] * a + g.A[4] * c) + g.A[5];
      Zt = (g.A[6] * a + g.A[7] * c) + g.A[8];
      depth = __builtin_inff();
      ok = true;
    } else {
      const float X = a * z, Y = c * z;
      Xt = ((g.A[0] * X + g.A[1] * Y) + g.A[2] * z) + g.b[0];
      Yt = ((g.A[3] * X + g.A[4] * Y) + g.A[5] * z) + g.b[1];
      Zt = ((g.A[6] * X + g.A[7] * Y) + g.A[8] * z) + g.b[2];
      depth = Zt;
      ok = z > 0.0f;  // NaN and non-positive depths carry no geometry
    }
    ok = ok && (Zt > 0.0f);
    const float xf = g.f * (Xt / Zt) + g.cx;
    const float yf = g.f * (Yt / Zt) + g.cy;
    const float rx = roundf(xf), ry = roundf(yf);
    ok = ok && (rx >= 0.0f) && (rx < Wf) && (ry >= 0.0f) && (ry < Hf);
    if (ok) {
      const size_t o = (size_t)(int)ry * (size_t)g.width + (size_t)(int)rx;
      atomicMin(reinterpret_cast<unsigned long long*>(&keys[o]),
                (unsigned long long)(((uint64_t)__float_as_uint(depth) << 32) | (uint32_t)i));
    }
  }
}

// One target row per workgroup at a time: keys in, the source colour
// gathered for every reached pixel, then the row fill.
template <int PPT>
__global__ __launch_bounds__(kThreads) void pose_resolve_kernel(const uint64_t* __restrict__ keys,
                                                                 const uint32_t* __restrict__ src_rgba, int W, int H,
                                                                 int fill, int target_right, uint32_t* dst_rgba,
                                                                 float* dst_depth, uint8_t* dst_mask, int wl) {
  extern __shared__ __align__(16) unsigned char smem[];
  RowLds s(smem, wl);
  for (int y = blockIdx.x; y < H; y += gridDim.x) {
    const size_t row = (size_t)y * (size_t)W;
    YORO_GLOBAL uint32_t* orow = gmem(dst_rgba) + row;
    YORO_GLOBAL float* zrow = dst_depth ? gmem(dst_depth) + row : nullptr;
    YORO_GLOBAL uint8_t* mrow = dst_mask ? gmem(dst_mask) + row : nullptr;
    uint64_t k[PPT];
    uint32_t col[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      k[i] = kEmpty;
      col[i] = 0u;
    }
    for_cols<PPT>(W, [&](int i, int x) { k[i] = __builtin_nontemporal_load(&keys[row + x]); });
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      // Every reached key names a source pixel of the frame.
      if ((uint32_t)(k[i] >> 32) != 0xFFFFFFFFu) col[i] = src_rgba[(uint32_t)k[i]];
    }
    for_cols<PPT>(W, [&](int i, int x) {
      s.key[x] = ((uint32_t)(k[i] >> 32) != 0xFFFFFFFFu) ? ((k[i] & 0xFFFFFFFF00000000ull) | col[i]) : kEmpty;
    });
    __syncthreads();
    resolve_fill_row<PPT>(s, W, target_right != 0, fill != 0, [&](int x, uint32_t c, uint32_t zb, uint8_t mk) {
      orow[x] = c;
      if (zrow) zrow[x] = __uint_as_float(zb);
      if (mrow) mrow[x] = mk;
    });
    __syncthreads();  // the next row reuses the LDS
  }
}

hipError_t set_lds_limit(const void* fn, size_t bytes) {
  if (bytes > 65536) return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  return hipSuccess;
}

#define YORO_PPT_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(12) X(16) X(20) X(24) X(28) X(32)

}  // namespace

hipError_t launch_pose(const uint32_t* src_rgba, const float* src_depth, const PoseGeom& g, int fill_mode,
                       int target_right, uint32_t* dst_rgba, float* dst_depth, uint8_t* dst_mask, uint64_t* keys,
                       int cus, hipStream_t stream) {
  const int ppt = ppt_for(g.width);
  if (ppt < 0) return hipErrorInvalidValue;
  const size_t n = (size_t)g.width * (size_t)g.height;
  const long long blocks = ((long long)n + kThreads - 1) / kThreads;
  const int grid_px = (int)std::min<long long>(blocks, (long long)cus * 16);
  hipLaunchKernelGGL(pose_clear_kernel, dim3(std::max(1, grid_px)), dim3(kThreads), 0, stream, keys, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pose_scatter_kernel, dim3(std::max(1, grid_px)), dim3(kThreads), 0, stream, src_depth, g, keys);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int wl = lds_width(g.width);
  const size_t lds = warp_lds_bytes(wl);
  const int grid_rows = std::max(1, std::min(g.height, cus * 8));
  switch (ppt) {
#define X(P)                                                                                                      \
  case P: {                                                                                                       \
    e = set_lds_limit((const void*)pose_resolve_kernel<P>, lds);                                                  \
    if (e != hipSuccess) return e;                                                                                \
    hipLaunchKernelGGL(pose_resolve_kernel<P>, dim3(grid_rows), dim3(kThreads), lds, stream, keys, src_rgba,       \
                       g.width, g.height, fill_mode != 0 ? 1 : 0, target_right, dst_rgba, dst_depth, dst_mask, wl); \
    return hipGetLastError();                                                                                     \
  }
    YORO_PPT_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace yoro

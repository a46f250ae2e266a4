// The near-object hybrid's device side (include/yoro_hybrid.h): the near
// layer of a box-and-sphere scene drawn for one eye (the conventional
// rendering the hybrid leaves the nearest objects to), and the composite of
// a near layer over the warped and filled far field.  The far field itself
// is the single-frame warp kernel with its near pixels skipped
// (warp_fill.hip).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "yoro_hybrid.h"
#include "yoro_internal.h"

namespace yoro {
namespace {

static_assert(sizeof(yoro_object) == 88, "yoro_object layout");

constexpr int kSphere = 0;

// The SplitMix64 finaliser and the two-word hash of the scene generator's
// texture noise (Steele, Lea and Flood, 2014; constants of SplitMix64).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t hash64(uint64_t a, uint64_t b) {
  return mix64(a * 0x9E3779B97F4A7C15ull ^ mix64(b + 0x632BE59BD9B4E019ull));
}

// Ray o + t d (d.z = 1): the smallest t > 1e-9, or +inf.  FP64, each
// operation in the written order.
__device__ __forceinline__ double hit_sphere(const yoro_object& s, const double o[3], const double d[3]) {
  const double oc[3] = {o[0] - s.c[0], o[1] - s.c[1], o[2] - s.c[2]};
  const double a = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  const double b = oc[0] * d[0] + oc[1] * d[1] + oc[2] * d[2];
  const double c = oc[0] * oc[0] + oc[1] * oc[1] + oc[2] * oc[2] - s.h[0] * s.h[0];
  const double disc = b * b - a * c;
  if (disc < 0.0) return INFINITY;
  const double sq = sqrt(disc);
  const double t0 = (-b - sq) / a;
  if (t0 > 1e-9) return t0;
  const double t1 = (-b + sq) / a;
  if (t1 > 1e-9) return t1;
  return INFINITY;
}

__device__ __forceinline__ double hit_box(const yoro_object& bx, const double o[3], const double d[3]) {
  double tn = -INFINITY, tf = INFINITY;
  for (int k = 0; k < 3; ++k) {
    const double lo = bx.c[k] - bx.h[k], hi = bx.c[k] + bx.h[k];
    if (d[k] == 0.0) {
      if (o[k] < lo || o[k] > hi) return INFINITY;
      continue;
    }
    double t1 = (lo - o[k]) / d[k], t2 = (hi - o[k]) / d[k];
    if (t1 > t2) {
      const double tmp = t1;
      t1 = t2;
      t2 = tmp;
    }
    if (t1 > tn) tn = t1;
    if (t2 < tf) tf = t2;
  }
  if (tn > tf) return INFINITY;
  if (tn > 1e-9) return tn;
  if (tf > 1e-9) return tf;
  return INFINITY;
}

__device__ __forceinline__ int32_t clamp255(int32_t v) { return v < 0 ? 0 : (v > 255 ? 255 : v); }

// The object's colour at surface point p (object-space texel noise and
// checker, so both eyes see one colour for one point).
__device__ __forceinline__ uint32_t shade(const yoro_object& o, const double p[3]) {
  const double q[3] = {p[0] - o.c[0], p[1] - o.c[1], p[2] - o.c[2]};
  int64_t t[3];
  for (int k = 0; k < 3; ++k) t[k] = (int64_t)floor(q[k] / o.texel);
  int32_t base[3] = {o.rgb[0], o.rgb[1], o.rgb[2]};
  if (o.cell > 0.0) {
    int64_t par = 0;
    for (int k = 0; k < 3; ++k) par += (int64_t)floor(q[k] / o.cell);
    if (par & 1)
      for (int k = 0; k < 3; ++k) base[k] /= 2;
  }
  const uint64_t h = hash64(o.id, hash64((uint64_t)t[0], hash64((uint64_t)t[1], (uint64_t)t[2])));
  const int32_t span = 2 * o.noise + 1;
  uint32_t out = 255u << 24;
  for (int k = 0; k < 3; ++k) {
    const int32_t nz = o.noise > 0 ? (int32_t)((h >> (16 * k)) & 0xFFFF) % span - o.noise : 0;
    out |= (uint32_t)clamp255(base[k] + nz) << (8 * k);
  }
  return out;
}

// One thread per output pixel (16 x 16 pixels per workgroup).  Objects whose
// nearest possible point lies past near_m (with a margin far above FP64
// rounding) cannot give a near pixel and are passed over; the rest are
// tested in index order, the first of equal t kept.
__global__ __launch_bounds__(256) void render_near_kernel(const yoro_object* __restrict__ objs, int n, int W, int H,
                                                          int x_off, int y_off, double f, double cx, double cy,
                                                          double eye_x, float near_m, uint32_t* __restrict__ rgba,
                                                          float* __restrict__ depth) {
  const int px = blockIdx.x * 16 + (threadIdx.x & 15);
  const int py = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (px >= W || py >= H) return;
  const double o[3] = {eye_x, 0.0, 0.0};
  const double d[3] = {((double)(px + x_off) + 0.5 - cx) / f, ((double)(py + y_off) + 0.5 - cy) / f, 1.0};
  const double nearest_allowed = (double)near_m * (1.0 + 1e-9) + 1e-9;
  double tbest = INFINITY;
  int best = -1;
  for (int i = 0; i < n; ++i) {
    const yoro_object ob = objs[i];
    const double zmin = ob.c[2] - (ob.kind == kSphere ? ob.h[0] : ob.h[2]);
    if (zmin > nearest_allowed) continue;
    const double t = ob.kind == kSphere ? hit_sphere(ob, o, d) : hit_box(ob, o, d);
    if (t < tbest) {
      tbest = t;
      best = i;
    }
  }
  const size_t pix = (size_t)py * (size_t)W + (size_t)px;
  uint32_t c = 0u;
  float z = INFINITY;
  if (best >= 0 && tbest < (double)near_m && (float)tbest < near_m) {
    const double p[3] = {o[0] + tbest * d[0], o[1] + tbest * d[1], o[2] + tbest * d[2]};
    c = shade(objs[best], p);
    z = (float)tbest;
  }
  rgba[pix] = c;
  depth[pix] = z;
}

// The near layer over the far field: near pixels win outright.
__global__ __launch_bounds__(256) void composite_near_kernel(const uint32_t* __restrict__ near_rgba,
                                                             const float* __restrict__ near_depth, float near_m,
                                                             int64_t n, uint32_t* __restrict__ rgba,
                                                             float* __restrict__ depth, uint8_t* __restrict__ mask) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float z = near_depth[i];
    if (z < near_m) {
      rgba[i] = near_rgba[i];
      if (depth) depth[i] = z;
      if (mask) mask[i] = YORO_MASK_NEAR;
    }
  }
}

}  // namespace

hipError_t launch_render_near(const yoro_object* objs, int n, int W, int H, int x_off, int y_off, double f, double cx,
                              double cy, double eye_x, float near_m, uint32_t* rgba, float* depth,
                              hipStream_t stream) {
  hipLaunchKernelGGL(render_near_kernel, dim3((W + 15) / 16, (H + 15) / 16), dim3(256), 0, stream, objs, n, W, H,
                     x_off, y_off, f, cx, cy, eye_x, near_m, rgba, depth);
  return hipGetLastError();
}

hipError_t launch_composite_near(const uint32_t* near_rgba, const float* near_depth, float near_m, int64_t n,
                                 uint32_t* rgba, float* depth, uint8_t* mask, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(composite_near_kernel, dim3(grid), dim3(256), 0, stream, near_rgba, near_depth, near_m, n, rgba,
                     depth, mask);
  return hipGetLastError();
}

}  // namespace yoro

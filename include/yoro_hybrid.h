/*
 * yoro_hybrid.h -- the near-object hybrid (Section 11.4, Impact of Object
 * Distance): nearer than a minimum distance, objects lose too much to the
 * reprojection, so they are rendered conventionally for the second eye and
 * the method synthesises the rest.
 *
 * The scene is split at depth near_m along the view axis.  The far field,
 * every source pixel with depth >= near_m, is warped and filled exactly as
 * yoro_reproject does (the nearer pixels take no part, as if they had no
 * geometry).  The near field, every surface point nearer than near_m, is
 * rendered for the target eye by the caller (yoro_render_near draws it for
 * the box-and-sphere scenes of this library's tests and benchmarks) and lies
 * in front of all far-field content: each target pixel whose near layer
 * depth is below near_m takes the layer's colour and depth (mask 3), every
 * other pixel the warped and filled far field.
 *
 * Conventions as in yoro.h: caller-owned device pointers, no allocation or
 * synchronisation, work queued on the given stream, YORO_ERR_INVALID_ARG
 * before anything is queued, YORO_ERR_DEVICE on a failed launch.
 */
#ifndef YORO_HYBRID_H
#define YORO_HYBRID_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define YORO_MASK_NEAR 3 /* mask value of a pixel taken from the near layer */

/*
 * yoro_reproject_hybrid -- yoro_reproject of the far field (source depth >=
 * near_m) with fill_mode, then the near layer over it.  near_rgba (H x W x 4
 * u8) and near_depth (H x W FP32): the target eye's near field; a depth that
 * is not below near_m (+inf, NaN) means no near surface at that pixel.
 * near_m: finite, > 0.  dst_depth and dst_mask are optional except with
 * YORO_FILL_PATCHER (as in yoro_reproject).  Outputs must not overlap any
 * input or each other.  YORO_FILL_LEARNED is YORO_ERR_UNSUPPORTED (apply it
 * with yoro_fill_holes to the result's far-field holes, mask 1).
 */
int32_t yoro_reproject_hybrid(const uint8_t* src_rgba, const float* src_depth, int32_t width, int32_t height,
                              float baseline_m, float focal_px, int32_t target_eye, int32_t fill_mode, float near_m,
                              const uint8_t* near_rgba, const float* near_depth, uint8_t* dst_rgba, float* dst_depth,
                              uint8_t* dst_mask, void* hip_stream);

/*
 * An analytic scene object: a sphere (kind 0, radius h[0]) or an axis-aligned
 * box (kind 1, half extents h) centred at c, in the left eye's camera frame
 * (metres, x right, y down, z forward).  Its colour at a surface point p is
 * rgb, halved on odd cells of an object-space checker of edge `cell` (0: no
 * checker), plus per-channel noise in [-noise, noise] hashed from id and the
 * object-space texel of p (edge `texel`), clamped to [0, 255]; alpha 255.
 * The layout of the scene generator's objects (88 bytes).
 */
typedef struct yoro_object {
  int32_t kind;
  uint32_t id;
  double c[3];
  double h[3];
  double texel;
  double cell;
  int32_t rgb[3];
  int32_t noise;
} yoro_object;

/*
 * yoro_render_near -- the near layer of one eye for a scene of n objects
 * (device array): a pinhole camera at (eye_x, 0, 0) looking along +z, focal
 * focal_px, principal point (cx, cy); output pixel (px, py) is camera pixel
 * (px + x_off, py + y_off) with its centre at +0.5.  Per pixel, in FP64: the
 * nearest intersection t over all objects (equal t: the lower index); when
 * t < near_m and (float)t < near_m the pixel gets that object's colour and
 * depth (float)t, otherwise RGBA 0 and depth +inf.  rgba: H x W x 4 u8,
 * depth: H x W FP32, both overwritten.  n: 0..65536; near_m > 0 (+inf
 * renders every surface).
 */
int32_t yoro_render_near(const yoro_object* objects, int32_t n, int32_t width, int32_t height, int32_t x_off,
                         int32_t y_off, double focal_px, double cx, double cy, double eye_x, float near_m,
                         uint8_t* rgba, float* depth, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* YORO_HYBRID_H */

/*
 * ORACLE -- test infrastructure only.  Plain, slow, obviously correct CPU
 * reference for the stereo reprojection hot path.  Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the product path
 * never does.  It shares no code with the GPU path.
 *
 * What it computes (parallel stereo, linear FP32 eye-space depth):
 *
 *   Reprojector (Section 6; reprojection equation M = (VP_left)^-1 VP_right,
 *   Algorithm 1): for two pinhole eyes that differ only by a shift B along x,
 *   the matrix transform of a pixel at depth z moves it along its row by the
 *   disparity B*f/z pixels and leaves y and z unchanged.  Observation O1
 *   (Section 5): the shift is horizontal and has one sign, so every row is
 *   independent.  The target column is the source column minus the rounded
 *   disparity when the right eye is synthesised from the left, plus it when
 *   the left eye is synthesised from the right.
 *
 *   Algorithm 2 (per-row scatter): each source pixel is written to its target
 *   column; when several land on one column the one with the lowest depth is
 *   kept (the text after Algorithm 2; the listing's comparison sign reads the
 *   other way and is taken as a typo).  Here the kept value is the minimum of
 *   the 64-bit key (float bits of z) << 32 | source index.  Equal depths in
 *   one row have equal disparity and so never collide: the index never
 *   decides, it only names the source.
 *
 *   Resolve (Algorithm 3, non-disocclusion branch): a hit takes the source
 *   pixel's RGBA (all four bytes) and depth.  A target column nobody reached
 *   is a disocclusion (hole).
 *
 *   Fill (Section 7; Observation O2 and the Patcher figure): a hole is filled
 *   from background, never foreground.  Nearest-background reading used here:
 *   take the nearest hit to the left and the nearest hit to the right in the
 *   resolved row (never an already filled pixel), keep the one with the
 *   larger depth; on equal depth keep the one on the side opposite the shift
 *   (right when the right eye is synthesised, left otherwise); with one
 *   neighbour take it; with none leave the hole (RGBA 0, depth +inf,
 *   mask 2).  Mask values: 0 hit, 1 hole (filled, or left empty when no
 *   fill is asked for), 2 hole with no hit in its row.
 *
 *   Patcher fill (Section 7, Algorithm 3 with its weight function,
 *   Equation 7), mode OR_FILL_PATCHER.  The listing mixes coordinate spaces
 *   (intermediate-buffer records and colour samples at the same index, a uv
 *   coordinate against pixel widths) and is one-dimensional although the
 *   kernel is said to be h = 3 rows high, so it is taken as follows.  For a
 *   hole at (x, y) with nearest row hits L and R (as above, L = -1 or R = W
 *   when absent) the kernel starts at the nearest-background hit e chosen as
 *   above, with depth ze, and runs outward from the hole, away from it, over
 *   n = R - L - 1 columns (the kernel is as wide as the disocclusion in the
 *   hole's row, Section 7, text before Equation 7; no cap), stopping at the
 *   frame's edge, and, per column, rows y, y - 1, y + 1 (h = 3).  A sample
 *   is used only if it lies in the frame, is a hit (mask 0, never a filled
 *   hole) and is not nearer than the edge
 *   (depth >= ze: the foreground skip).  With t = |x - e| / (R - L - 1),
 *   the position in the disocclusion (u - r_x) / r_z measured from the
 *   background edge (in the paper's own orientation, the left eye made
 *   from the right with the background on the left, r_x is that edge; the
 *   distance from e keeps the two eyes mirror images), each used sample takes
 *   w = w_rem / 2 + (0.3 w_rem) t of the remaining weight w_rem (which
 *   starts at 1): c_acc += C w, w_rem -= w.  The hole gets
 *   clamp(rint(c_acc / (1 - w_rem))) per RGB channel, the edge's alpha and
 *   depth, mask 1; a hole with no hit in its row stays empty (mask 2).  All
 *   of it in FP32 in exactly this order (it decides 8-bit values).  The
 *   edge itself is always the first sample, so the division is never by 0.
 *
 *   Near-object hybrid (Section 11.4, Impact of Object Distance: objects
 *   nearer than a minimum distance are rendered conventionally and the
 *   method handles the rest), oracle_reproject_hybrid.  Reading: the scene
 *   is split at depth D along the view axis.  The far field is every source
 *   pixel with depth z >= D: it is warped and filled exactly as above, the
 *   pixels with z < D taking no part (as if they had no geometry).  The
 *   near field is every surface point nearer than D, rendered for the
 *   target eye by the caller's renderer and handed in as a layer (colour and
 *   depth; a depth that is not below D, NaN included, means no near surface
 *   there).  It lies in front of all far-field content, so the target pixel
 *   takes the near layer's colour and depth wherever its depth is below D
 *   (mask 3), and the warped and filled far field elsewhere.
 *
 * Rounding reading: d = roundf(q), halfway cases away from zero, with
 * q = (B*f)/z, one FP32 multiply then one correctly rounded FP32 division.
 * Depths that are NaN, zero or negative carry no geometry and are skipped; a
 * disparity that is not below the frame width always lands off-frame and is
 * skipped before the integer conversion.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math (no FMA contraction, so
 * every FP32 operation rounds once, as written).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_TARGET_RIGHT = 0, OR_TARGET_LEFT = 1 };
enum { OR_FILL_NONE = 0, OR_FILL_NEAREST_BG = 1, OR_FILL_PATCHER = 3, OR_FILL_SIDE_ONLY = 101 };
enum { OR_MASK_NEAR = 3 }; /* hybrid: the pixel is the near layer's */

#define OR_EMPTY 0xFFFFFFFFFFFFFFFFull

static uint32_t float_bits(float v) {
  uint32_t u;
  memcpy(&u, &v, sizeof(u));
  return u;
}

static float bits_float(uint32_t u) {
  float v;
  memcpy(&v, &u, sizeof(v));
  return v;
}

/* Disparity of one source pixel.  Returns 0 and sets *d when the pixel is
 * splatted, -1 when it is skipped. */
int oracle_disparity(float z, float bf, int32_t width, int32_t* d) {
  if (!(z > 0.0f)) return -1;          /* NaN, +-0, negative: no geometry */
  float q = bf / z;                    /* +inf depth gives 0 */
  if (!(q < (float)width)) return -1;  /* a shift of a full row is always off-frame */
  *d = (int32_t)roundf(q);             /* halfway cases away from zero */
  return 0;
}

/* Nearest-background choice for the hole at column xt of one resolved row.
 * hit[x] != 0 marks resolved hits; zr[x] is their depth.  Returns the chosen
 * column or -1. */
static int32_t pick_neighbour(const uint8_t* hit, const float* zr, int32_t width, int32_t xt, int32_t s,
                              int32_t mode) {
  int32_t L = -1, R = -1;
  for (int32_t x = xt - 1; x >= 0; --x)
    if (hit[x]) { L = x; break; }
  for (int32_t x = xt + 1; x < width; ++x)
    if (hit[x]) { R = x; break; }
  if (L < 0 && R < 0) return -1;
  if (L < 0) return R;
  if (R < 0) return L;
  int32_t bg_side = (s < 0) ? R : L; /* side opposite the shift */
  if (mode == OR_FILL_SIDE_ONLY) return bg_side;
  if (zr[L] > zr[R]) return L;
  if (zr[R] > zr[L]) return R;
  return bg_side; /* bitwise-equal depth */
}

/* Fill one resolved row in place.  hit/zr describe the resolved row before
 * any fill; rgba/depth/mask are the outputs of that row. */
static void fill_row(uint8_t* rgba, float* depth, uint8_t* mask, const uint8_t* hit, const float* zr,
                     const uint8_t* col, int32_t width, int32_t s, int32_t mode) {
  for (int32_t xt = 0; xt < width; ++xt) {
    if (hit[xt]) continue;
    int32_t p = pick_neighbour(hit, zr, width, xt, s, mode);
    if (p < 0) {
      memset(&rgba[4 * xt], 0, 4);
      depth[xt] = INFINITY;
      mask[xt] = 2;
    } else {
      memcpy(&rgba[4 * xt], &col[4 * p], 4);
      depth[xt] = zr[p];
      mask[xt] = 1;
    }
  }
}

/* Patcher value of the hole at (x, y) of a frame whose hits have mask 0. */
static void patcher_pixel(const uint8_t* rgba, const float* depth, const uint8_t* mask, int32_t width,
                          int32_t height, int32_t x, int32_t y, int32_t s, uint8_t* out_rgba, float* out_z,
                          uint8_t* out_m) {
  const size_t row = (size_t)y * (size_t)width;
  int32_t L = x - 1, R = x + 1;
  while (L >= 0 && mask[row + L] != 0) --L;
  while (R < width && mask[row + R] != 0) ++R;
  if (L < 0 && R >= width) {
    memset(out_rgba, 0, 4);
    *out_z = INFINITY;
    *out_m = 2;
    return;
  }
  int32_t e;
  if (L < 0) e = R;
  else if (R >= width) e = L;
  else if (depth[row + L] > depth[row + R]) e = L;
  else if (depth[row + R] > depth[row + L]) e = R;
  else e = (s < 0) ? R : L;
  const float ze = depth[row + e];
  const int32_t rz = R - L - 1;
  const float t = (float)abs(x - e) / (float)rz;
  const int32_t dir = (e == R) ? 1 : -1;
  const int32_t n = rz; /* the disocclusion's width */
  static const int32_t dys[3] = {0, -1, 1};
  float w_rem = 1.0f, acc[3] = {0.0f, 0.0f, 0.0f};
  for (int32_t k = 0; k < n; ++k) {
    const int32_t cx = e + dir * k;
    if (cx < 0 || cx >= width) break;
    for (int32_t j = 0; j < 3; ++j) {
      const int32_t cy = y + dys[j];
      if (cy < 0 || cy >= height) continue;
      const size_t p = (size_t)cy * (size_t)width + (size_t)cx;
      if (mask[p] != 0) continue;    /* only resolved hits */
      if (depth[p] < ze) continue;   /* skip foreground */
      const float a = w_rem * 0.5f;
      const float b = 0.3f * w_rem;
      const float w = a + b * t;
      for (int c = 0; c < 3; ++c) acc[c] = acc[c] + (float)rgba[4 * p + c] * w;
      w_rem = w_rem - w;
    }
  }
  const float norm = 1.0f - w_rem;
  for (int c = 0; c < 3; ++c) {
    float v = rintf(acc[c] / norm);
    v = v < 0.0f ? 0.0f : (v > 255.0f ? 255.0f : v);
    out_rgba[c] = (uint8_t)v;
  }
  out_rgba[3] = rgba[4 * (row + (size_t)e) + 3];
  *out_z = ze;
  *out_m = 1;
}

/* Patcher over a whole frame, in place: holes (mask != 0) are refilled from
 * hits only, so the order does not matter. */
static void patcher_frame(uint8_t* rgba, float* depth, uint8_t* mask, int32_t width, int32_t height, int32_t s) {
  for (int32_t y = 0; y < height; ++y)
    for (int32_t x = 0; x < width; ++x) {
      const size_t i = (size_t)y * (size_t)width + (size_t)x;
      if (mask[i] == 0) continue;
      uint8_t c[4];
      float z;
      uint8_t m;
      patcher_pixel(rgba, depth, mask, width, height, x, y, s, c, &z, &m);
      /* Written after all reads of this pixel; other holes read hits only. */
      memcpy(&rgba[4 * i], c, 4);
      depth[i] = z;
      mask[i] = m;
    }
}

/*
 * Reproject one frame.  src_rgba: H*W*4 bytes; src_depth: H*W floats;
 * dst_rgba: H*W*4; dst_depth and dst_mask may be NULL.  Returns 0, or -1 on
 * bad arguments.
 */
int oracle_reproject(const uint8_t* src_rgba, const float* src_depth, int32_t width, int32_t height,
                     float baseline_m, float focal_px, int32_t target_eye, int32_t fill_mode,
                     uint8_t* dst_rgba, float* dst_depth, uint8_t* dst_mask, int32_t nthreads) {
  if (width <= 0 || height <= 0 || !src_rgba || !src_depth || !dst_rgba) return -1;
  if (target_eye != OR_TARGET_RIGHT && target_eye != OR_TARGET_LEFT) return -1;
  if (fill_mode == OR_FILL_PATCHER) {
    /* The Patcher reads neighbouring rows: warp every row first, then fill. */
    const size_t n = (size_t)width * (size_t)height;
    float* z = dst_depth ? dst_depth : (float*)malloc(sizeof(float) * n);
    uint8_t* m = dst_mask ? dst_mask : (uint8_t*)malloc(n);
    int rc = oracle_reproject(src_rgba, src_depth, width, height, baseline_m, focal_px, target_eye, OR_FILL_NONE,
                              dst_rgba, z, m, nthreads);
    if (rc == 0) patcher_frame(dst_rgba, z, m, width, height, target_eye == OR_TARGET_RIGHT ? -1 : +1);
    if (!dst_depth) free(z);
    if (!dst_mask) free(m);
    return rc;
  }
  const float bf = baseline_m * focal_px;
  const int32_t s = (target_eye == OR_TARGET_RIGHT) ? -1 : +1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel
  {
    uint64_t* K = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)width);
    uint8_t* hit = (uint8_t*)malloc((size_t)width);
    float* zr = (float*)malloc(sizeof(float) * (size_t)width);
    uint8_t* col = (uint8_t*)malloc(4 * (size_t)width);
    float* dz = (float*)malloc(sizeof(float) * (size_t)width);
    uint8_t* mk = (uint8_t*)malloc((size_t)width);
#pragma omp for schedule(static)
    for (int32_t y = 0; y < height; ++y) {
      /* Scatter with the depth test (Algorithm 2). */
      for (int32_t x = 0; x < width; ++x) K[x] = OR_EMPTY;
      for (int32_t x = 0; x < width; ++x) {
        size_t i = (size_t)y * (size_t)width + (size_t)x;
        float z = src_depth[i];
        int32_t d;
        if (oracle_disparity(z, bf, width, &d) != 0) continue;
        int32_t xt = x + s * d;
        if (xt < 0 || xt >= width) continue;
        uint64_t key = ((uint64_t)float_bits(z) << 32) | (uint64_t)(uint32_t)i;
        if (key < K[xt]) K[xt] = key;
      }
      /* Resolve. */
      for (int32_t xt = 0; xt < width; ++xt) {
        if (K[xt] == OR_EMPTY) {
          hit[xt] = 0;
          zr[xt] = INFINITY;
          memset(&col[4 * xt], 0, 4);
          dz[xt] = INFINITY;
          mk[xt] = 1;
        } else {
          size_t i = (size_t)(uint32_t)K[xt];
          hit[xt] = 1;
          zr[xt] = bits_float((uint32_t)(K[xt] >> 32));
          memcpy(&col[4 * xt], &src_rgba[4 * i], 4);
          dz[xt] = src_depth[i];
          mk[xt] = 0;
        }
      }
      uint8_t* orow = &dst_rgba[4 * (size_t)y * (size_t)width];
      memcpy(orow, col, 4 * (size_t)width);
      float* zrow = dz;
      uint8_t* mrow = mk;
      if (fill_mode != OR_FILL_NONE) fill_row(orow, zrow, mrow, hit, zr, col, width, s, fill_mode);
      if (dst_depth) memcpy(&dst_depth[(size_t)y * (size_t)width], zrow, sizeof(float) * (size_t)width);
      if (dst_mask) memcpy(&dst_mask[(size_t)y * (size_t)width], mrow, (size_t)width);
    }
    free(K);
    free(hit);
    free(zr);
    free(col);
    free(dz);
    free(mk);
  }
  return 0;
}

/*
 * Stand-alone fill of an already warped frame, in place.  Pixels with
 * mask == 0 are hits; every other pixel is a hole and is refilled from the
 * hits of its row (never from another hole).  Returns 0 or -1.
 */
int oracle_fill_holes(uint8_t* rgba, float* depth, uint8_t* mask, int32_t width, int32_t height,
                      int32_t target_eye, int32_t fill_mode) {
  if (width <= 0 || height <= 0 || !rgba || !depth || !mask) return -1;
  if (target_eye != OR_TARGET_RIGHT && target_eye != OR_TARGET_LEFT) return -1;
  if (fill_mode == OR_FILL_NONE) return 0;
  const int32_t s = (target_eye == OR_TARGET_RIGHT) ? -1 : +1;
  if (fill_mode == OR_FILL_PATCHER) {
    patcher_frame(rgba, depth, mask, width, height, s);
    return 0;
  }
  uint8_t* hit = (uint8_t*)malloc((size_t)width);
  float* zr = (float*)malloc(sizeof(float) * (size_t)width);
  uint8_t* col = (uint8_t*)malloc(4 * (size_t)width);
  for (int32_t y = 0; y < height; ++y) {
    uint8_t* r = &rgba[4 * (size_t)y * (size_t)width];
    float* z = &depth[(size_t)y * (size_t)width];
    uint8_t* m = &mask[(size_t)y * (size_t)width];
    for (int32_t x = 0; x < width; ++x) {
      hit[x] = (m[x] == 0);
      zr[x] = z[x];
    }
    memcpy(col, r, 4 * (size_t)width);
    fill_row(r, z, m, hit, zr, col, width, s, fill_mode);
  }
  free(hit);
  free(zr);
  free(col);
  return 0;
}

/*
 * Resolution-independent intermediate buffer (Section 6 (c) and (d)):
 * the reprojection runs on a buffer of ceil(W/k) x ceil(H/k) texels
 * (k = 1, 2, 4, 8, 16), one per k x k block of pixels (the last row and
 * column of blocks may be cut by the frame's edge), that holds, per texel,
 * how far its pixel moves; the full-resolution image is then sampled
 * through it.  Readings:
 *   texel (i, j) takes the depth z of the full-resolution source pixel at
 *   its block's centre, (k i + c, k j + c) with c = k / 2 (c = 0 for
 *   k = 1), each coordinate clamped to the frame;
 *   q = (B f) / z with the direct path's skip rule (z > 0, q < W); the
 *   texel moves by the rounded texel disparity dk = roundf(q / k) to
 *   it = i - dk (right eye; i + dk for the left), skipped unless
 *   0 <= it < ceil(W/k); the nearest depth wins (key: depth bits, then texel
 *   index); the winner's record is its shift q, in full-resolution pixels,
 *   and its depth z;
 *   full-resolution pixel (x, y) reads buffer row y / k at
 *   u = (x - c) / k, i0 = floor(u), f = u - i0, the nearest texel
 *   n = f < 0.5 ? i0 : i0 + 1 (clamped to the row; it is always the texel
 *   whose k x k block holds the pixel): a hole there is a hole here;
 *   otherwise the shift is n's, or, with linear interpolation along the
 *   row (Section 6 (d)), when i0 and i0 + 1 are both in the row, both hits
 *   and their shifts within one pixel of each other (one surface),
 *   s = s0 + f (s1 - s0);
 *   the source column is x + roundf(s) (right eye; x - roundf(s) for the
 *   left), a hole if off the row; a hit takes that source pixel's RGBA and
 *   the depth of texel n; the nearest-background fill then runs on the
 *   full-resolution row as in the direct path.
 * FP32 throughout, in exactly this order.  With k = 1 every pixel is a
 * texel, s = q, roundf(s) is the direct path's disparity and the result is
 * the direct path's (pinned).
 */
int oracle_reproject_lowres(const uint8_t* src_rgba, const float* src_depth, int32_t width, int32_t height,
                            float baseline_m, float focal_px, int32_t target_eye, int32_t fill_mode, int32_t k,
                            int32_t linear, uint8_t* dst_rgba, float* dst_depth, uint8_t* dst_mask) {
  if (width <= 0 || height <= 0 || !src_rgba || !src_depth || !dst_rgba) return -1;
  if (target_eye != OR_TARGET_RIGHT && target_eye != OR_TARGET_LEFT) return -1;
  if (!(k == 1 || k == 2 || k == 4 || k == 8 || k == 16)) return -1;
  if (fill_mode != OR_FILL_NONE && fill_mode != OR_FILL_NEAREST_BG) return -1;
  const float bf = baseline_m * focal_px;
  const int32_t s = (target_eye == OR_TARGET_RIGHT) ? -1 : +1;
  const int32_t wk = (width + k - 1) / k, hk = (height + k - 1) / k, c = k / 2;
  uint64_t* K = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)wk);
  float* sh = (float*)malloc(sizeof(float) * (size_t)wk);
  float* zt = (float*)malloc(sizeof(float) * (size_t)wk);
  uint8_t* hit = (uint8_t*)malloc((size_t)width);
  float* zr = (float*)malloc(sizeof(float) * (size_t)width);
  uint8_t* col = (uint8_t*)malloc(4 * (size_t)width);
  float* dz = (float*)malloc(sizeof(float) * (size_t)width);
  uint8_t* mk = (uint8_t*)malloc((size_t)width);
  for (int32_t j = 0; j < hk; ++j) {
    /* Stage 1: scatter the buffer row. */
    const int32_t yc = k * j + c < height ? k * j + c : height - 1;
    const size_t srow = (size_t)yc * (size_t)width;
    for (int32_t i = 0; i < wk; ++i) K[i] = OR_EMPTY;
    for (int32_t i = 0; i < wk; ++i) {
      const int32_t xc = k * i + c < width ? k * i + c : width - 1;
      const float z = src_depth[srow + (size_t)xc];
      if (!(z > 0.0f)) continue;
      const float q = bf / z;
      if (!(q < (float)width)) continue;
      const int32_t dk = (int32_t)roundf(q / (float)k);
      const int32_t it = i + s * dk;
      if (it < 0 || it >= wk) continue;
      const uint64_t key = ((uint64_t)float_bits(z) << 32) | (uint64_t)(uint32_t)i;
      if (key < K[it]) K[it] = key;
    }
    for (int32_t i = 0; i < wk; ++i) {
      if (K[i] == OR_EMPTY) continue;
      const float z = bits_float((uint32_t)(K[i] >> 32));
      sh[i] = bf / z;
      zt[i] = z;
    }
    /* Stage 2: the k full-resolution rows that read this buffer row. */
    for (int32_t y = k * j; y < k * j + k && y < height; ++y) {
      const size_t row = (size_t)y * (size_t)width;
      for (int32_t x = 0; x < width; ++x) {
        const float u = ((float)x - (float)c) / (float)k;
        const float i0f = floorf(u);
        const float f = u - i0f;
        int32_t i0 = (int32_t)i0f, i1 = i0 + 1;
        int32_t n = f < 0.5f ? i0 : i1;
        n = n < 0 ? 0 : (n >= wk ? wk - 1 : n);
        int ok = K[n] != OR_EMPTY;
        int32_t xs = -1;
        if (ok) {
          float sv = sh[n];
          if (linear && i0 >= 0 && i1 < wk && K[i0] != OR_EMPTY && K[i1] != OR_EMPTY &&
              fabsf(sh[i1] - sh[i0]) <= 1.0f) {
            const float dsh = sh[i1] - sh[i0];
            const float m = f * dsh;
            sv = sh[i0] + m;
          }
          const int32_t r = (int32_t)roundf(sv);
          xs = (s < 0) ? x + r : x - r;
          ok = xs >= 0 && xs < width;
        }
        if (ok) {
          hit[x] = 1;
          zr[x] = zt[n];
          memcpy(&col[4 * x], &src_rgba[4 * (row + (size_t)xs)], 4);
          dz[x] = zt[n];
          mk[x] = 0;
        } else {
          hit[x] = 0;
          zr[x] = INFINITY;
          memset(&col[4 * x], 0, 4);
          dz[x] = INFINITY;
          mk[x] = 1;
        }
      }
      uint8_t* orow = &dst_rgba[4 * row];
      memcpy(orow, col, 4 * (size_t)width);
      if (fill_mode != OR_FILL_NONE) fill_row(orow, dz, mk, hit, zr, col, width, s, fill_mode);
      if (dst_depth) memcpy(&dst_depth[row], dz, sizeof(float) * (size_t)width);
      if (dst_mask) memcpy(&dst_mask[row], mk, (size_t)width);
    }
  }
  free(K);
  free(sh);
  free(zt);
  free(hit);
  free(zr);
  free(col);
  free(dz);
  free(mk);
  return 0;
}

/*
 * Reprojection through a general pose (Section 6: the rotation matrix of a
 * unit quaternion, Equation rmatrix; the view and projection matrices; the
 * reprojection M = (VP_src)^-1 VP_tgt).  The printed view matrix has a zero
 * bottom row and the printed projection has no perspective divide, so the
 * cameras are taken as the pinholes the rest of the method assumes.
 * Readings:
 *   cameras: x right, y down, z forward; focal length f px, principal point
 *   (cx, cy); pixel (x, y) with planar depth z is the point
 *   ((x - cx) z / f, (y - cy) z / f, z) of its eye's camera;
 *   the pose (q, t): the target eye's orientation (unit quaternion,
 *   q[0] = r_x the scalar part, as Equation rmatrix places it) and position,
 *   both in the source eye's camera frame; a source-camera point X is
 *   X_t = R^T (X - t) in the target camera (for parallel stereo the right
 *   eye is q = (1, 0, 0, 0), t = (B, 0, 0), and this is the direct path);
 *   A = R^T and b = -(R^T t) are formed in double from Equation rmatrix, in
 *   the order written below, and rounded to FP32;
 *   per source pixel, in FP32 with each operation rounded once:
 *     a = (x - cx) / f, c = (y - cy) / f;
 *     finite z > 0:  X = a z, Y = c z,
 *                    X_t = ((A00 X + A01 Y) + A02 z) + b0 (Y_t, Z_t alike),
 *                    target depth Z_t;
 *     z = +inf (a point at infinity: only the rotation moves it):
 *                    X_t = (A00 a + A01 c) + A02 (Y_t, Z_t alike),
 *                    target depth +inf;
 *     any other z (NaN, <= 0) is not splatted;
 *     skipped unless Z_t > 0; xf = f (X_t / Z_t) + cx, yf = f (Y_t / Z_t) + cy,
 *     the target pixel (roundf(xf), roundf(yf)), skipped unless inside the
 *     frame;
 *   two-dimensional depth test over the whole frame: the least key
 *   (target depth bits << 32) | source index wins (equal depths can meet
 *   here, and the lower source index then wins);
 *   resolve as the direct path (the source pixel's RGBA, the target depth);
 *   fill per target row as the direct path, the tie side opposite the shift
 *   read from the translation: right when t_x >= 0, else left.
 */
static void pose_matrix(const float* q, const float* t, float* A, float* b) {
  const double rx = q[0], ry = q[1], rz = q[2], rw = q[3];
  double R[3][3];
  R[0][0] = 1.0 - 2.0 * rz * rz - 2.0 * rw * rw;
  R[0][1] = 2.0 * ry * rz - 2.0 * rx * rw;
  R[0][2] = 2.0 * ry * rw + 2.0 * rx * rz;
  R[1][0] = 2.0 * ry * rz + 2.0 * rx * rw;
  R[1][1] = 1.0 - 2.0 * ry * ry - 2.0 * rw * rw;
  R[1][2] = 2.0 * rz * rw - 2.0 * rx * ry;
  R[2][0] = 2.0 * ry * rw - 2.0 * rx * rz;
  R[2][1] = 2.0 * rz * rw + 2.0 * rx * ry;
  R[2][2] = 1.0 - 2.0 * ry * ry - 2.0 * rz * rz;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) A[3 * i + j] = (float)R[j][i];
    b[i] = (float)(-((R[0][i] * (double)t[0] + R[1][i] * (double)t[1]) + R[2][i] * (double)t[2]));
  }
}

/* Target pixel and depth of one source pixel; returns 0 when it is splatted. */
int oracle_project_pose(float z, int32_t x, int32_t y, int32_t width, int32_t height, float focal_px, float cx,
                        float cy, const float* q, const float* t, int32_t* xt, int32_t* yt, float* zt) {
  float A[9], b[3];
  pose_matrix(q, t, A, b);
  const float a = ((float)x - cx) / focal_px;
  const float c = ((float)y - cy) / focal_px;
  float Xt, Yt, Zt, depth;
  if (z == INFINITY) {
    Xt = (A[0] * a + A[1] * c) + A[2];
    Yt = (A[3] * a + A[4] * c) + A[5];
    Zt = (A[6] * a + A[7] * c) + A[8];
    depth = INFINITY;
  } else if (z > 0.0f) {
    const float X = a * z, Y = c * z;
    Xt = ((A[0] * X + A[1] * Y) + A[2] * z) + b[0];
    Yt = ((A[3] * X + A[4] * Y) + A[5] * z) + b[1];
    Zt = ((A[6] * X + A[7] * Y) + A[8] * z) + b[2];
    depth = Zt;
  } else {
    return -1;
  }
  if (!(Zt > 0.0f)) return -1;
  const float xf = focal_px * (Xt / Zt) + cx;
  const float yf = focal_px * (Yt / Zt) + cy;
  const float rxf = roundf(xf), ryf = roundf(yf);
  if (!(rxf >= 0.0f && rxf < (float)width && ryf >= 0.0f && ryf < (float)height)) return -1;
  *xt = (int32_t)rxf;
  *yt = (int32_t)ryf;
  *zt = depth;
  return 0;
}

int oracle_reproject_pose(const uint8_t* src_rgba, const float* src_depth, int32_t width, int32_t height,
                          float focal_px, float cx, float cy, const float* q, const float* t, int32_t fill_mode,
                          uint8_t* dst_rgba, float* dst_depth, uint8_t* dst_mask) {
  if (width <= 0 || height <= 0 || !src_rgba || !src_depth || !dst_rgba || !q || !t) return -1;
  if (fill_mode != OR_FILL_NONE && fill_mode != OR_FILL_NEAREST_BG) return -1;
  const size_t n = (size_t)width * (size_t)height;
  uint64_t* K = (uint64_t*)malloc(sizeof(uint64_t) * n);
  for (size_t i = 0; i < n; ++i) K[i] = OR_EMPTY;
  /* Scatter with the depth test over the whole frame. */
  for (int32_t y = 0; y < height; ++y)
    for (int32_t x = 0; x < width; ++x) {
      const size_t i = (size_t)y * (size_t)width + (size_t)x;
      int32_t xt, yt;
      float zt;
      if (oracle_project_pose(src_depth[i], x, y, width, height, focal_px, cx, cy, q, t, &xt, &yt, &zt) != 0)
        continue;
      const size_t o = (size_t)yt * (size_t)width + (size_t)xt;
      const uint64_t key = ((uint64_t)float_bits(zt) << 32) | (uint64_t)(uint32_t)i;
      if (key < K[o]) K[o] = key;
    }
  /* Resolve and fill, row by row of the target. */
  const int32_t s = (t[0] >= 0.0f) ? -1 : +1;
  uint8_t* hit = (uint8_t*)malloc((size_t)width);
  float* zr = (float*)malloc(sizeof(float) * (size_t)width);
  uint8_t* col = (uint8_t*)malloc(4 * (size_t)width);
  float* dz = (float*)malloc(sizeof(float) * (size_t)width);
  uint8_t* mk = (uint8_t*)malloc((size_t)width);
  for (int32_t y = 0; y < height; ++y) {
    const size_t row = (size_t)y * (size_t)width;
    for (int32_t x = 0; x < width; ++x) {
      const uint64_t k = K[row + (size_t)x];
      if (k == OR_EMPTY) {
        hit[x] = 0;
        zr[x] = INFINITY;
        memset(&col[4 * x], 0, 4);
        dz[x] = INFINITY;
        mk[x] = 1;
      } else {
        const size_t i = (size_t)(uint32_t)k;
        hit[x] = 1;
        zr[x] = bits_float((uint32_t)(k >> 32));
        memcpy(&col[4 * x], &src_rgba[4 * i], 4);
        dz[x] = zr[x];
        mk[x] = 0;
      }
    }
    uint8_t* orow = &dst_rgba[4 * row];
    memcpy(orow, col, 4 * (size_t)width);
    if (fill_mode != OR_FILL_NONE) fill_row(orow, dz, mk, hit, zr, col, width, s, fill_mode);
    if (dst_depth) memcpy(&dst_depth[row], dz, sizeof(float) * (size_t)width);
    if (dst_mask) memcpy(&dst_mask[row], mk, (size_t)width);
  }
  free(K);
  free(hit);
  free(zr);
  free(col);
  free(dz);
  free(mk);
  return 0;
}

/*
 * Hole error against a reference image (Section 9, PSNR): the sum of squared
 * RGB differences over pixels with mask != 0, and the number of such pixels.
 * Integer arithmetic, so the sum is exact.
 */
/*
 * Near-object hybrid (see the header): the far field (source depth >= near_m)
 * warped and filled per fill_mode, then the near layer (near_rgba, near_depth:
 * the target eye's near field, H*W*4 bytes and H*W floats) wherever its depth
 * is below near_m.  Outputs as oracle_reproject; dst_depth and dst_mask may
 * be NULL.  Returns 0, or -1 on bad arguments.
 */
int oracle_reproject_hybrid(const uint8_t* src_rgba, const float* src_depth, int32_t width, int32_t height,
                            float baseline_m, float focal_px, int32_t target_eye, int32_t fill_mode, float near_m,
                            const uint8_t* near_rgba, const float* near_depth, uint8_t* dst_rgba, float* dst_depth,
                            uint8_t* dst_mask, int32_t nthreads) {
  if (width <= 0 || height <= 0 || !src_rgba || !src_depth || !near_rgba || !near_depth || !dst_rgba) return -1;
  const size_t n = (size_t)width * (size_t)height;
  /* The far field: source pixels nearer than near_m carry no geometry. */
  float* far_depth = (float*)malloc(sizeof(float) * n);
  for (size_t i = 0; i < n; ++i) far_depth[i] = src_depth[i] < near_m ? NAN : src_depth[i];
  float* z = dst_depth ? dst_depth : (float*)malloc(sizeof(float) * n);
  uint8_t* m = dst_mask ? dst_mask : (uint8_t*)malloc(n);
  int rc = oracle_reproject(src_rgba, far_depth, width, height, baseline_m, focal_px, target_eye, fill_mode,
                            dst_rgba, z, m, nthreads);
  /* The near field lies in front of everything warped: it wins outright. */
  if (rc == 0) {
    for (size_t i = 0; i < n; ++i) {
      if (near_depth[i] < near_m) {
        memcpy(&dst_rgba[4 * i], &near_rgba[4 * i], 4);
        z[i] = near_depth[i];
        m[i] = OR_MASK_NEAR;
      }
    }
  }
  free(far_depth);
  if (!dst_depth) free(z);
  if (!dst_mask) free(m);
  return rc;
}

void oracle_hole_sse(const uint8_t* rgba, const uint8_t* ref, const uint8_t* mask, int64_t n_pixels,
                     uint64_t* sse, uint64_t* count) {
  uint64_t acc = 0, cnt = 0;
  for (int64_t i = 0; i < n_pixels; ++i) {
    if (mask && mask[i] == 0) continue;
    for (int c = 0; c < 3; ++c) {
      int32_t e = (int32_t)rgba[4 * i + c] - (int32_t)ref[4 * i + c];
      acc += (uint64_t)(e * e);
    }
    cnt += 1;
  }
  *sse = acc;
  *count = cnt;
}

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
enum { OR_FILL_NONE = 0, OR_FILL_NEAREST_BG = 1, OR_FILL_SIDE_ONLY = 101 };

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
 * Hole error against a reference image (Section 9, PSNR): the sum of squared
 * RGB differences over pixels with mask != 0, and the number of such pixels.
 * Integer arithmetic, so the sum is exact.
 */
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

/*
 * Seeded synthetic scenes and an analytic ray-caster (boxes and spheres).
 *
 * This is the input generator shared by the tests, the benchmark and the
 * learned-fill training loop.  It holds none of the reprojection method's
 * arithmetic: it only produces, for a pinhole camera placed at either eye,
 * the colour and the linear eye-space depth of the nearest surface, i.e. the
 * G-buffer that the rendered (dominant) eye hands to the reprojector
 * (Section 3.2, G-buffer; Section 4, system overview), and the true second
 * eye that the synthesised one is compared against (Section 9, PSNR).
 *
 * Camera model (parallel stereo): both eyes share focal length f (pixels)
 * and principal point (cx, cy); pixel (px, py) has its centre at px + 0.5,
 * y points down, the view direction is +z.  The left eye sits at the origin
 * and the right eye at (+B, 0, 0).  Depth is the planar eye-space z of the
 * hit (the ray direction has z = 1, so z equals the ray parameter t).
 *
 * Random numbers: SplitMix64 seeds xoshiro256** (Blackman and Vigna, 2018);
 * uniform doubles take the top 53 bits.  No std:: or libc distribution is
 * used, so a seed gives the same scene on every compiler and libc.
 *
 * All geometry is FP64; only the stored depth is rounded to FP32.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define YS_SPHERE 0
#define YS_BOX 1

typedef struct ys_object {
  int32_t kind;      /* YS_SPHERE or YS_BOX */
  uint32_t id;       /* hashed into the texture noise */
  double c[3];       /* centre, left-eye camera coordinates, metres */
  double h[3];       /* sphere: radius in h[0]; box: half extents */
  double texel;      /* object-space texel edge (metres), about 1 px at its depth */
  double cell;       /* checker cell edge (metres); 0 disables the checker */
  int32_t rgb[3];    /* base colour */
  int32_t noise;     /* noise amplitude: each channel gets U{-noise..noise} */
} ys_object;

/* ---------------------------------------------------------------- PRNG --- */

static uint64_t splitmix64(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* SplitMix64 finaliser used as a stateless hash. */
static uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

typedef struct { uint64_t s[4]; } xoshiro;

static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t xo_next(xoshiro* g) {
  uint64_t* s = g->s;
  uint64_t result = rotl(s[1] * 5, 7) * 9;
  uint64_t t = s[1] << 17;
  s[2] ^= s[0];
  s[3] ^= s[1];
  s[1] ^= s[2];
  s[0] ^= s[3];
  s[2] ^= t;
  s[3] = rotl(s[3], 45);
  return result;
}

static void xo_seed(xoshiro* g, uint64_t seed) {
  uint64_t s = seed;
  for (int i = 0; i < 4; ++i) g->s[i] = splitmix64(&s);
}

static double xo_unit(xoshiro* g) { return (double)(xo_next(g) >> 11) * 0x1.0p-53; }
static double xo_uniform(xoshiro* g, double a, double b) { return a + (b - a) * xo_unit(g); }
static int64_t xo_int(xoshiro* g, int64_t lo, int64_t hi) { /* inclusive */
  uint64_t span = (uint64_t)(hi - lo) + 1u;
  return lo + (int64_t)(xo_next(g) % span);
}

/* Exported so that Python-side generators can draw from the same stream. */
uint64_t ys_hash64(uint64_t a, uint64_t b) { return mix64(a * 0x9E3779B97F4A7C15ull ^ mix64(b + 0x632BE59BD9B4E019ull)); }

void ys_uniform_fill(uint64_t seed, double* out, int64_t n) {
  xoshiro g;
  xo_seed(&g, seed);
  for (int64_t i = 0; i < n; ++i) out[i] = xo_unit(&g);
}

/* ------------------------------------------------------- scene recipe --- */

/*
 * Generate n objects for a virtual frame of width W, height H, focal f,
 * principal point at the frame centre.  Depth of each centre is uniform on
 * [zmin, zmax] (log_uniform = 0) or log-uniform (log_uniform = 1).  Screen
 * position is uniform over the frame widened by a 10 % margin and
 * back-projected at that depth.  The apparent half size is a*W pixels with
 * a ~ U[0.02, 0.15]; the object shrinks until its nearest point is at least
 * 0.25 m from the eye plane.  Half the objects are spheres, half boxes.
 * checker_lo..checker_hi > 0 enables a checker of cell U{lo..hi} px at depth.
 * Returns the number of objects written.
 */
int ys_generate(uint64_t seed, int32_t W, int32_t H, double f, int32_t n, double zmin, double zmax,
                int32_t log_uniform, int32_t checker_lo, int32_t checker_hi, int32_t noise,
                ys_object* out) {
  xoshiro g;
  xo_seed(&g, seed);
  for (int i = 0; i < n; ++i) {
    ys_object* o = &out[i];
    memset(o, 0, sizeof(*o));
    o->kind = (xo_next(&g) >> 63) ? YS_BOX : YS_SPHERE;
    o->id = (uint32_t)i + 1u;
    double zc = log_uniform ? exp(xo_uniform(&g, log(zmin), log(zmax))) : xo_uniform(&g, zmin, zmax);
    double u = xo_uniform(&g, -0.1 * W, 1.1 * W);
    double v = xo_uniform(&g, -0.1 * H, 1.1 * H);
    double a = xo_uniform(&g, 0.02, 0.15);
    double s = a * W * zc / f;
    double e[3] = {1.0, 1.0, 1.0};
    if (o->kind == YS_BOX) {
      for (int k = 0; k < 3; ++k) e[k] = xo_uniform(&g, 0.5, 1.0);
    }
    double rad = (o->kind == YS_BOX) ? s * sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]) : s;
    if (zc - rad < 0.25) s *= (zc - 0.25) / rad;
    o->c[0] = (u - 0.5 * W) / f * zc;
    o->c[1] = (v - 0.5 * H) / f * zc;
    o->c[2] = zc;
    for (int k = 0; k < 3; ++k) o->h[k] = s * e[k];
    o->texel = zc / f;
    o->cell = 0.0;
    if (checker_hi > 0) o->cell = (double)xo_int(&g, checker_lo, checker_hi) * zc / f;
    for (int k = 0; k < 3; ++k) o->rgb[k] = (int32_t)xo_int(&g, 24, 232);
    o->noise = noise;
  }
  return n;
}

/* ----------------------------------------------------------- shading --- */

static int32_t clamp255(int32_t v) { return v < 0 ? 0 : (v > 255 ? 255 : v); }

static void shade(const ys_object* o, const double p[3], uint8_t rgba[4]) {
  /* Object-space point: both eyes see the same colour for the same point. */
  double q[3] = {p[0] - o->c[0], p[1] - o->c[1], p[2] - o->c[2]};
  int64_t t[3];
  for (int k = 0; k < 3; ++k) t[k] = (int64_t)floor(q[k] / o->texel);
  int32_t base[3] = {o->rgb[0], o->rgb[1], o->rgb[2]};
  if (o->cell > 0.0) {
    int64_t par = 0;
    for (int k = 0; k < 3; ++k) par += (int64_t)floor(q[k] / o->cell);
    if (par & 1) {
      for (int k = 0; k < 3; ++k) base[k] /= 2;
    }
  }
  uint64_t hsh = ys_hash64(o->id, ys_hash64((uint64_t)t[0], ys_hash64((uint64_t)t[1], (uint64_t)t[2])));
  int32_t span = 2 * o->noise + 1;
  for (int k = 0; k < 3; ++k) {
    int32_t nz = o->noise > 0 ? (int32_t)((hsh >> (16 * k)) & 0xFFFF) % span - o->noise : 0;
    rgba[k] = (uint8_t)clamp255(base[k] + nz);
  }
  rgba[3] = 255;
}

/* Background: a per-row colour (depends on the virtual row only), so both
 * eyes agree on it; depth is a fixed far value. */
static void background(uint64_t seed, int64_t row, int32_t Hv, uint8_t rgba[4]) {
  uint64_t h = ys_hash64(seed ^ 0xB6C0F00Dull, (uint64_t)row);
  double tnorm = Hv > 1 ? (double)row / (double)(Hv - 1) : 0.0;
  int32_t r = 70 + (int32_t)(90.0 * tnorm) + (int32_t)(h & 15) - 8;
  int32_t gg = 110 + (int32_t)(60.0 * tnorm) + (int32_t)((h >> 8) & 15) - 8;
  int32_t b = 200 - (int32_t)(80.0 * tnorm) + (int32_t)((h >> 16) & 15) - 8;
  rgba[0] = (uint8_t)clamp255(r);
  rgba[1] = (uint8_t)clamp255(gg);
  rgba[2] = (uint8_t)clamp255(b);
  rgba[3] = 255;
}

/* ------------------------------------------------------- intersection --- */

/* Ray o + t*d (d.z = 1).  Returns the smallest t > tmin, or INFINITY. */
static double hit_sphere(const ys_object* s, const double o[3], const double d[3]) {
  double oc[3] = {o[0] - s->c[0], o[1] - s->c[1], o[2] - s->c[2]};
  double a = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  double b = oc[0] * d[0] + oc[1] * d[1] + oc[2] * d[2];
  double c = oc[0] * oc[0] + oc[1] * oc[1] + oc[2] * oc[2] - s->h[0] * s->h[0];
  double disc = b * b - a * c;
  if (disc < 0.0) return INFINITY;
  double sq = sqrt(disc);
  double t0 = (-b - sq) / a;
  if (t0 > 1e-9) return t0;
  double t1 = (-b + sq) / a;
  if (t1 > 1e-9) return t1;
  return INFINITY;
}

static double hit_box(const ys_object* bx, const double o[3], const double d[3]) {
  double tn = -INFINITY, tf = INFINITY;
  for (int k = 0; k < 3; ++k) {
    double lo = bx->c[k] - bx->h[k], hi = bx->c[k] + bx->h[k];
    if (d[k] == 0.0) {
      if (o[k] < lo || o[k] > hi) return INFINITY;
      continue;
    }
    double t1 = (lo - o[k]) / d[k], t2 = (hi - o[k]) / d[k];
    if (t1 > t2) { double tmp = t1; t1 = t2; t2 = tmp; }
    if (t1 > tn) tn = t1;
    if (t2 < tf) tf = t2;
  }
  if (tn > tf) return INFINITY;
  if (tn > 1e-9) return tn;
  if (tf > 1e-9) return tf;
  return INFINITY;
}

/* Conservative pixel rectangle covered by object o seen from eye_x. */
static int obj_rect(const ys_object* o, double f, double cx, double cy, double eye_x, int32_t W,
                    int32_t H, int32_t r[4]) {
  double rad = o->kind == YS_SPHERE ? o->h[0] : sqrt(o->h[0] * o->h[0] + o->h[1] * o->h[1] + o->h[2] * o->h[2]);
  double zn = o->c[2] - rad, zf = o->c[2] + rad;
  if (zf <= 0.0) return 0;
  if (zn <= 1e-6) { r[0] = 0; r[1] = W - 1; r[2] = 0; r[3] = H - 1; return 1; }
  double X[2] = {o->c[0] - eye_x - rad, o->c[0] - eye_x + rad};
  double Y[2] = {o->c[1] - rad, o->c[1] + rad};
  double Z[2] = {zn, zf};
  double xmn = INFINITY, xmx = -INFINITY, ymn = INFINITY, ymx = -INFINITY;
  for (int i = 0; i < 2; ++i)
    for (int k = 0; k < 2; ++k) {
      double px = f * X[i] / Z[k] + cx, py = f * Y[i] / Z[k] + cy;
      if (px < xmn) xmn = px;
      if (px > xmx) xmx = px;
      if (py < ymn) ymn = py;
      if (py > ymx) ymx = py;
    }
  double x0 = floor(xmn - 0.5) - 1.0, x1 = ceil(xmx - 0.5) + 1.0;
  double y0 = floor(ymn - 0.5) - 1.0, y1 = ceil(ymx - 0.5) + 1.0;
  if (x1 < 0.0 || y1 < 0.0 || x0 > W - 1 || y0 > H - 1) return 0;
  r[0] = x0 < 0.0 ? 0 : (int32_t)x0;
  r[1] = x1 > W - 1 ? W - 1 : (int32_t)x1;
  r[2] = y0 < 0.0 ? 0 : (int32_t)y0;
  r[3] = y1 > H - 1 ? H - 1 : (int32_t)y1;
  return 1;
}

/*
 * Render an eye.  The output window is W x H pixels; window pixel (px, py)
 * is virtual pixel (px + x_off, py + y_off) of a camera with principal point
 * (cx, cy) given in virtual pixels.  eye_x is the eye position on the x axis
 * (0 for the left eye, B for the right).  bg_seed and Hv pick the background
 * (per virtual row).  Nearest hit wins; equal t keeps the lower object index.
 * rgba: W*H*4 bytes, depth: W*H floats.  nthreads <= 0 uses OpenMP's default.
 */
void ys_render(const ys_object* objs, int32_t n, int32_t W, int32_t H, int32_t x_off, int32_t y_off,
               double f, double cx, double cy, double eye_x, uint64_t bg_seed, int32_t Hv,
               double bg_depth, uint8_t* rgba, float* depth, int32_t nthreads) {
  /* Rectangles in window coordinates. */
  int32_t(*rect)[4] = (int32_t(*)[4])malloc(sizeof(int32_t[4]) * (size_t)(n > 0 ? n : 1));
  int32_t* vis = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  for (int i = 0; i < n; ++i) vis[i] = obj_rect(&objs[i], f, cx - x_off, cy - y_off, eye_x, W, H, rect[i]);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel
  {
    double* tbest = (double*)malloc(sizeof(double) * (size_t)W);
    int32_t* best = (int32_t*)malloc(sizeof(int32_t) * (size_t)W);
#pragma omp for schedule(dynamic, 4)
    for (int32_t py = 0; py < H; ++py) {
      for (int32_t px = 0; px < W; ++px) {
        tbest[px] = INFINITY;
        best[px] = -1;
      }
      const double o[3] = {eye_x, 0.0, 0.0};
      const double dy = ((double)(py + y_off) + 0.5 - cy) / f;
      /* Objects in index order with a strict test: equal t keeps the lower index. */
      for (int32_t i = 0; i < n; ++i) {
        if (!vis[i] || py < rect[i][2] || py > rect[i][3]) continue;
        for (int32_t px = rect[i][0]; px <= rect[i][1]; ++px) {
          const double d[3] = {((double)(px + x_off) + 0.5 - cx) / f, dy, 1.0};
          double t = objs[i].kind == YS_SPHERE ? hit_sphere(&objs[i], o, d) : hit_box(&objs[i], o, d);
          if (t < tbest[px]) {
            tbest[px] = t;
            best[px] = i;
          }
        }
      }
      for (int32_t px = 0; px < W; ++px) {
        size_t pix = (size_t)py * (size_t)W + (size_t)px;
        if (best[px] >= 0 && tbest[px] < bg_depth) {
          const double d[3] = {((double)(px + x_off) + 0.5 - cx) / f, dy, 1.0};
          double p[3] = {o[0] + tbest[px] * d[0], o[1] + tbest[px] * d[1], o[2] + tbest[px] * d[2]};
          shade(&objs[best[px]], p, &rgba[4 * pix]);
          depth[pix] = (float)tbest[px];
        } else {
          background(bg_seed, (int64_t)py + y_off, Hv, &rgba[4 * pix]);
          depth[pix] = (float)bg_depth;
        }
      }
    }
    free(tbest);
    free(best);
  }
  free(rect);
  free(vis);
}

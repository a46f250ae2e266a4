// Inference of the learned hole filler as single calls (include/yoro_model.h):
// the forward sequence of the encoder-decoder over the layer kernels of
// nn.hip, its activation buffers carved from a caller workspace, and the
// hole-tile driver (gather all crops, run them in chunks, composite blocks).
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdint>
#include <functional>

#include "yoro.h"
#include "yoro_internal.h"
#include "yoro_model.h"
#include "yoro_nn.h"

namespace {

struct Layer {
  int cin, cout;  // kernel channel counts (multiples of 32)
};
// e0a e0b e1a e1b e2a e2b e3a e3b d2a d2b d2c d1a d1b d1c d0a d0b d0c head; the
// 5-channel input and the 3-channel head are padded to 32.
constexpr Layer kLayers[YORO_MODEL_LAYERS] = {
    {32, 32},   {32, 32},   {32, 64},   {64, 64},   {64, 128},  {128, 128}, {128, 256}, {256, 256}, {256, 128},
    {256, 128}, {128, 128}, {128, 64},  {128, 64},  {64, 64},   {64, 32},   {64, 32},   {32, 32},   {32, 32}};

long long layer_offset(int i) {
  long long o = 0;
  for (int j = 0; j < i; ++j) o += 9LL * kLayers[j].cin * kLayers[j].cout;
  return o;
}

int32_t model_fail(int32_t status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  yoro::set_last_error(buf);
  return status;
}

bool al16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
bool al4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

// Activation buffers of one forward pass (bf16 NHWC; res FP32 [P0][3]),
// except c0, the full-resolution concatenation, which holds its two
// 32-channel halves as planes ([2][P0][32]: d0a, then e0b): its writers
// then store whole 64-byte pixel records, and its reader takes the second
// input chunk from the second plane.
struct Acts {
  uint16_t *e0a, *c0, *d0b, *d0c;
  uint16_t *p1, *e1a, *c1, *d1b, *d1c;
  uint16_t *p2, *e2a, *c2, *d2b, *d2c;
  uint16_t *p3, *e3a, *e3b;
  float* res;
};

// Lays the buffers out from base (NULL: only measures); returns the bytes used.
size_t carve(char* base, long long n, int h, int w, Acts* a) {
  size_t off = 0;
  auto take = [&](long long elems, size_t esize) -> char* {
    char* p = base ? base + off : nullptr;
    off += ((size_t)elems * esize + 255) & ~(size_t)255;
    return p;
  };
  long long P[4];
  for (int l = 0; l < 4; ++l) P[l] = n * (long long)(h >> l) * (w >> l);
  auto bf = [&](long long p, int c) { return reinterpret_cast<uint16_t*>(take(p * c, 2)); };
  Acts t;
  t.e0a = bf(P[0], 32), t.c0 = bf(P[0], 64), t.d0b = bf(P[0], 32), t.d0c = bf(P[0], 32);
  t.p1 = bf(P[1], 32), t.e1a = bf(P[1], 64), t.c1 = bf(P[1], 128), t.d1b = bf(P[1], 64), t.d1c = bf(P[1], 64);
  t.p2 = bf(P[2], 64), t.e2a = bf(P[2], 128), t.c2 = bf(P[2], 256), t.d2b = bf(P[2], 128), t.d2c = bf(P[2], 128);
  t.p3 = bf(P[3], 128), t.e3a = bf(P[3], 256), t.e3b = bf(P[3], 256);
  t.res = reinterpret_cast<float*>(take(P[0] * 3, 4));
  if (a) *a = t;
  return off;
}

// The forward pass; every step is a layer kernel of nn.hip.
hipError_t forward(const uint16_t* wts, const uint8_t* rgba, const float* depth, const uint8_t* mask, int n, int h,
                   int w, const Acts& a, hipStream_t s, const std::function<hipError_t()>* pace = nullptr) {
  using namespace yoro;
  hipError_t e = hipSuccess;
  // Every layer is one launch; the pacing call follows each.  A paced pass
  // shares the GPU with latency-critical work: its convolutions run one
  // workgroup per tile.
  const bool persistent = !(pace && *pace);
  auto ok = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
    if (e == hipSuccess && pace && *pace) e = (*pace)();
  };
  auto conv = [&](int i, const uint16_t* x, int ldx, int lev, uint16_t* y, int ldy, long long xcs = 32) {
    const Layer L = kLayers[i];
    ok(nn_conv3x3(x, ldx, n, h >> lev, w >> lev, L.cin, wts + layer_offset(i), L.cout, y, ldy, 0, L.cout, 1, nullptr,
                  0, s, persistent, xcs));
  };
  const long long plane0 = (long long)n * h * w * 32;  // one 32-channel plane of c0
  // The first convolution packs the frame's channels itself (no packed copy).
  // The encoders' second convolutions also write the 2x2 average pool of
  // their output (the next level's input) in the same pass.
  auto conv_pool = [&](int i, const uint16_t* x, int ldx, int lev, uint16_t* y, int ldy, uint16_t* pool, int ldp) {
    const Layer L = kLayers[i];
    ok(nn_conv3x3_pool(x, ldx, n, h >> lev, w >> lev, L.cin, wts + layer_offset(i), L.cout, y, ldy, 1, pool, ldp, s,
                       persistent));
  };
  ok(nn_conv3x3_input(reinterpret_cast<const uint32_t*>(rgba), depth, mask, n, h, w, wts + layer_offset(0),
                      kLayers[0].cout, a.e0a, 32, 1, s, persistent));
  conv_pool(1, a.e0a, 32, 0, a.c0 + plane0, 32, a.p1, 32);  // e0b -> the skip plane of c0, and its pool
  conv(2, a.p1, 32, 1, a.e1a, 64);
  conv_pool(3, a.e1a, 64, 1, a.c1 + 64, 128, a.p2, 64);  // e1b
  conv(4, a.p2, 64, 2, a.e2a, 128);
  conv_pool(5, a.e2a, 128, 2, a.c2 + 128, 256, a.p3, 128);  // e2b
  conv(6, a.p3, 128, 3, a.e3a, 256);
  conv(7, a.e3a, 256, 3, a.e3b, 256);
  // The decoders' first convolutions read the lower level's output through
  // a nearest x2 upsampling done in their input loads (no upsampled copy).
  auto conv_up = [&](int i, const uint16_t* xlo, int ldx, int lev, uint16_t* y, int ldy) {
    const Layer L = kLayers[i];
    ok(nn_conv3x3_up(xlo, ldx, n, h >> lev, w >> lev, L.cin, wts + layer_offset(i), L.cout, y, ldy, 0, L.cout, 1,
                     nullptr, 0, s, persistent));
  };
  conv_up(8, a.e3b, 256, 2, a.c2, 256);  // d2a -> the decoder half of c2
  conv(9, a.c2, 256, 2, a.d2b, 128);
  conv(10, a.d2b, 128, 2, a.d2c, 128);
  conv_up(11, a.d2c, 128, 1, a.c1, 128);  // d1a
  conv(12, a.c1, 128, 1, a.d1b, 64);
  conv(13, a.d1b, 64, 1, a.d1c, 64);
  conv_up(14, a.d1c, 64, 0, a.c0, 32);  // d0a -> the decoder plane of c0
  conv(15, a.c0, 32, 0, a.d0b, 32, plane0);
  conv(16, a.d0b, 32, 0, a.d0c, 32);
  // Head: FP32 residual, the first 3 of its 32 padded outputs, no activation.
  ok(nn_conv3x3(a.d0c, 32, n, h, w, 32, wts + layer_offset(17), 32, a.res, 3, 1, 3, 0, nullptr, 0, s, persistent));
  return e;
}

int32_t launched(hipError_t e, const char* who) {
  if (e != hipSuccess) return model_fail(YORO_ERR_DEVICE, "%s: launch failed: %s", who, hipGetErrorString(e));
  return YORO_OK;
}

bool shape_ok(long long n, int h, int w) {
  return n > 0 && h > 0 && w > 0 && h % 8 == 0 && w % 8 == 0 && n * h * w < (1LL << 31);
}

size_t crop_input_bytes(long long k, int crop) {
  const long long px = k * crop * crop;
  return (((size_t)px * 4 + 255) & ~(size_t)255) * 2 + (((size_t)px + 255) & ~(size_t)255);
}

}  // namespace

extern "C" {

int32_t yoro_model_layout(int32_t* cin_pad, int32_t* cout_pad, int64_t* offset) {
  for (int i = 0; i < YORO_MODEL_LAYERS; ++i) {
    if (cin_pad) cin_pad[i] = kLayers[i].cin;
    if (cout_pad) cout_pad[i] = kLayers[i].cout;
  }
  if (offset)
    for (int i = 0; i <= YORO_MODEL_LAYERS; ++i) offset[i] = layer_offset(i);
  return YORO_OK;
}

size_t yoro_model_weights_bytes(void) { return (size_t)layer_offset(YORO_MODEL_LAYERS) * 2; }

int32_t yoro_model_pack(const float* master, void* weights, void* hip_stream) {
  return yoro_model_pack_train(master, weights, nullptr, hip_stream);
}

int32_t yoro_model_pack_train(const float* master, void* weights, void* weights_bwd, void* hip_stream) {
  const char* who = "yoro_model_pack";
  if (!master || !weights || !al4(master) || !al16(weights) || (weights_bwd && !al16(weights_bwd)))
    return model_fail(YORO_ERR_INVALID_ARG, "%s: null or misaligned pointer", who);
  long long off[YORO_MODEL_LAYERS + 1];
  int cin[YORO_MODEL_LAYERS], cout[YORO_MODEL_LAYERS];
  for (int i = 0; i < YORO_MODEL_LAYERS; ++i) cin[i] = kLayers[i].cin, cout[i] = kLayers[i].cout;
  for (int i = 0; i <= YORO_MODEL_LAYERS; ++i) off[i] = layer_offset(i);
  return launched(yoro::nn_pack_model(master, off, cin, cout, YORO_MODEL_LAYERS, static_cast<uint16_t*>(weights),
                                      static_cast<uint16_t*>(weights_bwd), (hipStream_t)hip_stream),
                  who);
}

size_t yoro_model_workspace_bytes(int32_t n, int32_t h, int32_t w) {
  if (!shape_ok(n, h, w)) return 0;
  return carve(nullptr, n, h, w, nullptr);
}

int32_t yoro_model_workspace_layout(int32_t n, int32_t h, int32_t w, int64_t* offsets) {
  if (!offsets || !shape_ok(n, h, w))
    return model_fail(YORO_ERR_INVALID_ARG, "yoro_model_workspace_layout: bad shape or null offsets");
  char* const base = reinterpret_cast<char*>(256);  // any aligned non-null base: offsets are relative to it
  Acts a;
  carve(base, n, h, w, &a);
  const void* order[YORO_MODEL_ACTIVATIONS] = {a.e0a, a.c0,  a.d0b, a.d0c, a.p1,  a.e1a, a.c1,  a.d1b, a.d1c,
                                               a.p2,  a.e2a, a.c2,  a.d2b, a.d2c, a.p3,  a.e3a, a.e3b, a.res};
  for (int i = 0; i < YORO_MODEL_ACTIVATIONS; ++i)
    offsets[i] = (int64_t)(reinterpret_cast<const char*>(order[i]) - base);
  return YORO_OK;
}

int32_t yoro_model_residual(const void* weights, const uint8_t* rgba, const float* depth, const uint8_t* mask,
                            int32_t n, int32_t h, int32_t w, float* res, void* workspace, size_t workspace_bytes,
                            void* hip_stream) {
  const char* who = "yoro_model_residual";
  if (!weights || !rgba || !depth || !mask || !res || !workspace)
    return model_fail(YORO_ERR_INVALID_ARG, "%s: null pointer", who);
  if (!shape_ok(n, h, w)) return model_fail(YORO_ERR_INVALID_ARG, "%s: bad shape %d x %d x %d", who, n, h, w);
  if (!al16(weights) || !al4(rgba) || !al4(depth) || !al4(res) || !al16(workspace))
    return model_fail(YORO_ERR_INVALID_ARG, "%s: misaligned pointer", who);
  Acts a;
  if (workspace_bytes < carve(static_cast<char*>(workspace), n, h, w, &a))
    return model_fail(YORO_ERR_WORKSPACE_TOO_SMALL, "%s: workspace too small", who);
  a.res = res;
  return launched(forward(static_cast<const uint16_t*>(weights), rgba, depth, mask, n, h, w, a, (hipStream_t)hip_stream),
                  who);
}

int32_t yoro_model_fill(const void* weights, const uint8_t* rgba, const float* depth, const uint8_t* mask, int32_t n,
                        int32_t h, int32_t w, uint8_t* out, void* workspace, size_t workspace_bytes,
                        void* hip_stream) {
  const char* who = "yoro_model_fill";
  if (!weights || !rgba || !depth || !mask || !out || !workspace)
    return model_fail(YORO_ERR_INVALID_ARG, "%s: null pointer", who);
  if (!shape_ok(n, h, w)) return model_fail(YORO_ERR_INVALID_ARG, "%s: bad shape %d x %d x %d", who, n, h, w);
  if (!al16(weights) || !al4(rgba) || !al4(depth) || !al4(out) || !al16(workspace))
    return model_fail(YORO_ERR_INVALID_ARG, "%s: misaligned pointer", who);
  Acts a;
  if (workspace_bytes < carve(static_cast<char*>(workspace), n, h, w, &a))
    return model_fail(YORO_ERR_WORKSPACE_TOO_SMALL, "%s: workspace too small", who);
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e = forward(static_cast<const uint16_t*>(weights), rgba, depth, mask, n, h, w, a, s);
  if (e == hipSuccess)
    e = yoro::nn_composite(a.res, reinterpret_cast<const uint32_t*>(rgba), mask, (long long)n * h * w,
                           reinterpret_cast<uint32_t*>(out), s);
  return launched(e, who);
}

size_t yoro_model_bands_workspace_bytes(int32_t w, int32_t h, int32_t band, int32_t halo) {
  if (w <= 0 || h <= 0 || w % 8 || h % 8 || band <= 0 || band % 8 || halo < 0 || halo % 8 || 2 * halo > band)
    return 0;
  const int ch = band + 2 * halo < h ? band + 2 * halo : h;
  if (!shape_ok(1, ch, w)) return 0;
  // The activations of one band crop (their residual buffer is the first of
  // three residual buffers) and two more residual buffers.
  return carve(nullptr, 1, ch, w, nullptr) + 2 * (((size_t)ch * w * 3 * 4 + 255) & ~(size_t)255);
}

int32_t yoro_model_fill_bands(const void* weights, const uint8_t* rgba, const float* depth, const uint8_t* mask,
                              int32_t w, int32_t h, int32_t band, int32_t halo, const uint8_t* band_has_holes,
                              uint8_t* out, void* workspace, size_t workspace_bytes, void* hip_stream) {
  return yoro::model_fill_bands_paced(weights, rgba, depth, mask, w, h, band, halo, band_has_holes, out, workspace,
                                      workspace_bytes, hip_stream, std::function<hipError_t()>());
}

size_t yoro_model_tiles_workspace_bytes(int32_t k, int32_t chunk, int32_t tile, int32_t halo) {
  if (k <= 0 || chunk <= 0 || tile <= 0 || halo < 0 || k > 65535) return 0;
  const int crop = tile + 2 * halo;
  if (!shape_ok(chunk < k ? chunk : k, crop, crop)) return 0;
  return crop_input_bytes(k, crop) + carve(nullptr, chunk < k ? chunk : k, crop, crop, nullptr);
}

int32_t yoro_model_fill_tiles(const void* weights, const uint8_t* rgba, const float* depth, const uint8_t* mask,
                              int32_t w, int32_t h, const int32_t* plan, int32_t k, int32_t tile, int32_t halo,
                              int32_t chunk, uint8_t* out, void* workspace, size_t workspace_bytes,
                              void* hip_stream) {
  return yoro::model_fill_tiles_paced(weights, rgba, depth, mask, w, h, plan, k, tile, halo, chunk, out, workspace,
                                      workspace_bytes, hip_stream, std::function<hipError_t()>());
}

}  // extern "C"

namespace yoro {

// Bands of `band` rows, each run on the crop of rows [y0 - halo, y0 + band +
// halo) clamped inward to the frame (full width: a contiguous row range of
// the frame, read in place).  A band's composite writes `out`, which may be
// `rgba`, so it is queued only once no later band's crop reaches its rows
// (crops only move down, so that is when the next crop starts below it).
// With halo <= band / 2 at most two bands wait at a time (the last crop,
// shifted up at a short last band, can reach two bands back): three
// residual buffers in turn.
int32_t model_fill_bands_paced(const void* weights, const uint8_t* rgba, const float* depth, const uint8_t* mask,
                               int32_t w, int32_t h, int32_t band, int32_t halo, const uint8_t* band_has_holes,
                               uint8_t* out, void* workspace, size_t workspace_bytes, void* hip_stream,
                               const std::function<hipError_t()>& pace) {
  const char* who = "yoro_model_fill_bands";
  if (!weights || !rgba || !depth || !mask || !out || !workspace)
    return model_fail(YORO_ERR_INVALID_ARG, "%s: null pointer", who);
  const size_t need = yoro_model_bands_workspace_bytes(w, h, band, halo);
  if (need == 0)
    return model_fail(YORO_ERR_INVALID_ARG, "%s: bad frame %d x %d, band %d or halo %d (multiples of 8, halo <= band/2)",
                      who, w, h, band, halo);
  if (!al16(weights) || !al4(rgba) || !al4(depth) || !al4(out) || !al16(workspace))
    return model_fail(YORO_ERR_INVALID_ARG, "%s: misaligned pointer", who);
  if (workspace_bytes < need) return model_fail(YORO_ERR_WORKSPACE_TOO_SMALL, "%s: workspace too small", who);
  const int ch = band + 2 * halo < h ? band + 2 * halo : h;
  Acts a;
  const size_t used = carve(static_cast<char*>(workspace), 1, ch, w, &a);
  const size_t rbytes = ((size_t)ch * w * 3 * 4 + 255) & ~(size_t)255;
  float* res[3] = {a.res, reinterpret_cast<float*>(static_cast<char*>(workspace) + used),
                   reinterpret_cast<float*>(static_cast<char*>(workspace) + used + rbytes)};
  hipStream_t s = (hipStream_t)hip_stream;
  const int nb = (h + band - 1) / band;
  auto crop_of = [&](int b) {
    int oy = b * band - halo;
    return oy < 0 ? 0 : (oy > h - ch ? h - ch : oy);
  };
  struct Pending {
    int b, oy;
  };
  Pending q[3];
  int nq = 0;
  hipError_t e = hipSuccess;
  auto composite = [&](const Pending& p) {
    const int y0 = p.b * band, rows = (y0 + band < h ? band : h - y0);
    const long long off = (long long)y0 * w;
    return yoro::nn_composite(res[p.b % 3] + (long long)(y0 - p.oy) * w * 3,
                              reinterpret_cast<const uint32_t*>(rgba) + off, mask + off, (long long)rows * w,
                              reinterpret_cast<uint32_t*>(out) + off, s);
  };
  for (int b = 0; b < nb && e == hipSuccess; ++b) {
    if (band_has_holes && !band_has_holes[b]) continue;
    const int oy = crop_of(b);
    // Bands whose rows this crop (and every later one) no longer reaches.
    while (nq > 0 && e == hipSuccess && (q[0].b + 1) * band <= oy) {
      e = composite(q[0]);
      q[0] = q[1], q[1] = q[2], --nq;
    }
    if (e != hipSuccess) break;
    const long long off = (long long)oy * w;
    Acts ab = a;
    ab.res = res[b % 3];
    e = forward(static_cast<const uint16_t*>(weights), rgba + 4 * off, depth + off, mask + off, 1, ch, w, ab, s,
                &pace);
    q[nq++] = Pending{b, oy};
  }
  for (int i = 0; i < nq && e == hipSuccess; ++i) e = composite(q[i]);
  return launched(e, who);
}

int32_t model_fill_tiles_paced(const void* weights, const uint8_t* rgba, const float* depth, const uint8_t* mask,
                               int32_t w, int32_t h, const int32_t* plan, int32_t k, int32_t tile, int32_t halo,
                               int32_t chunk, uint8_t* out, void* workspace, size_t workspace_bytes,
                               void* hip_stream, const std::function<hipError_t()>& pace) {
  const char* who = "yoro_model_fill_tiles";
  if (!weights || !rgba || !depth || !mask || !plan || !out || !workspace)
    return model_fail(YORO_ERR_INVALID_ARG, "%s: null pointer", who);
  const int crop = tile + 2 * halo;
  if (w <= 0 || h <= 0 || k <= 0 || k > 65535 || chunk <= 0 || tile <= 0 || tile % 8 || halo < 0 || halo % 8 ||
      crop > w || crop > h || w % 8 || h % 8)
    return model_fail(YORO_ERR_INVALID_ARG, "%s: bad frame %d x %d, k %d, chunk %d, tile %d or halo %d", who, w, h, k,
                      chunk, tile, halo);
  if (!al16(weights) || !al4(rgba) || !al4(depth) || !al4(out) || !al4(plan) || !al16(workspace))
    return model_fail(YORO_ERR_INVALID_ARG, "%s: misaligned pointer", who);
  const size_t need = yoro_model_tiles_workspace_bytes(k, chunk, tile, halo);
  if (need == 0) return model_fail(YORO_ERR_INVALID_ARG, "%s: chunk of crops too large", who);
  if (workspace_bytes < need) return model_fail(YORO_ERR_WORKSPACE_TOO_SMALL, "%s: workspace too small", who);
  const long long cpx = (long long)crop * crop;
  char* ws = static_cast<char*>(workspace);
  uint32_t* crgba = reinterpret_cast<uint32_t*>(ws);
  float* cdepth = reinterpret_cast<float*>(ws + (((size_t)k * cpx * 4 + 255) & ~(size_t)255));
  uint8_t* cmask = reinterpret_cast<uint8_t*>(ws + 2 * (((size_t)k * cpx * 4 + 255) & ~(size_t)255));
  const int cmax = chunk < k ? chunk : k;
  Acts a;
  carve(ws + crop_input_bytes(k, crop), cmax, crop, crop, &a);
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e = yoro::nn_gather_crops(reinterpret_cast<const uint32_t*>(rgba), depth, mask, w, plan, k, crop, crgba,
                                       cdepth, cmask, s);
  for (int c0 = 0; c0 < k && e == hipSuccess; c0 += cmax) {
    const int kc = k - c0 < cmax ? k - c0 : cmax;
    e = forward(static_cast<const uint16_t*>(weights), reinterpret_cast<const uint8_t*>(crgba + c0 * cpx),
                cdepth + c0 * cpx, cmask + c0 * cpx, kc, crop, crop, a, s, &pace);
    if (e == hipSuccess)
      e = yoro::nn_composite_tiles(a.res, plan + 4 * c0, kc, crop, tile, w, h, reinterpret_cast<const uint32_t*>(rgba),
                                   mask, reinterpret_cast<uint32_t*>(out), s);
  }
  return launched(e, who);
}

}  // namespace yoro

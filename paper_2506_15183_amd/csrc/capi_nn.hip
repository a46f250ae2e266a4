// C-ABI of the learned-fill layers (declared in include/yoro_nn.h): host
// validation and launch.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdint>

#include "yoro.h"
#include "yoro_internal.h"
#include "yoro_nn.h"

namespace {

int32_t nn_fail(int32_t status, const char* fmt, ...) {
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

bool shape_ok(int32_t n, int32_t h, int32_t w) {
  return n > 0 && h > 0 && w > 0 && (int64_t)n * h * w < (int64_t)1 << 40;
}

int32_t launched(hipError_t e, const char* who) {
  if (e != hipSuccess) return nn_fail(YORO_ERR_DEVICE, "%s: launch failed: %s", who, hipGetErrorString(e));
  return YORO_OK;
}

}  // namespace

extern "C" {

int32_t yoro_nn_conv3x3(const void* x, int32_t ldx, int32_t n, int32_t h, int32_t w, int32_t cin, const void* wgt,
                        int32_t cout, void* y, int32_t ldy, int32_t y_fp32, int32_t cout_store, int32_t epilogue,
                        const void* msrc, int32_t ldm, void* hip_stream) {
  const char* who = "yoro_nn_conv3x3";
  if (!x || !wgt || !y) return nn_fail(YORO_ERR_INVALID_ARG, "%s: null pointer", who);
  if (!shape_ok(n, h, w)) return nn_fail(YORO_ERR_INVALID_ARG, "%s: bad shape", who);
  if (cin <= 0 || cin % 32 || cout <= 0 || cout % 32)
    return nn_fail(YORO_ERR_INVALID_ARG, "%s: cin %d and cout %d must be positive multiples of 32", who, cin, cout);
  if (ldx < cin || ldx % 8 || !al16(x) || !al16(wgt))
    return nn_fail(YORO_ERR_INVALID_ARG, "%s: x/w must be 16-byte aligned with ldx >= cin, ldx %% 8 == 0", who);
  if (cout_store <= 0 || cout_store > cout || ldy < cout_store)
    return nn_fail(YORO_ERR_INVALID_ARG, "%s: bad cout_store %d or ldy %d", who, cout_store, ldy);
  if (y_fp32 ? !al4(y) : ((reinterpret_cast<uintptr_t>(y) & 1u) != 0))
    return nn_fail(YORO_ERR_INVALID_ARG, "%s: misaligned y", who);
  if (epilogue < YORO_NN_EPI_NONE || epilogue > YORO_NN_EPI_RELU_GRAD)
    return nn_fail(YORO_ERR_INVALID_ARG, "%s: unknown epilogue %d", who, epilogue);
  if (epilogue == YORO_NN_EPI_RELU_GRAD && (!msrc || ldm < cout_store))
    return nn_fail(YORO_ERR_INVALID_ARG, "%s: the ReLU-derivative epilogue needs msrc with ldm >= cout_store", who);
  return launched(yoro::nn_conv3x3(static_cast<const uint16_t*>(x), ldx, n, h, w, cin,
                                   static_cast<const uint16_t*>(wgt), cout, y, ldy, y_fp32 ? 1 : 0, cout_store,
                                   epilogue, static_cast<const uint16_t*>(msrc), ldm, (hipStream_t)hip_stream),
                  who);
}

size_t yoro_nn_conv3x3_wgrad_workspace(int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout) {
  if (!shape_ok(n, h, w) || cin <= 0 || cout <= 0) return 0;
  if (cin % 32 || cout % 32) return 0;
  return yoro::nn_wgrad_chunks(n, h, w, cin, cout) * 9 * (size_t)cin * (size_t)cout * sizeof(float);
}

int32_t yoro_nn_conv3x3_wgrad(const void* x, int32_t ldx, const void* dy, int32_t lddy, int32_t n, int32_t h,
                              int32_t w, int32_t cin, int32_t cout, float* dw, void* workspace, size_t workspace_bytes,
                              void* hip_stream) {
  const char* who = "yoro_nn_conv3x3_wgrad";
  if (!x || !dy || !dw || !workspace) return nn_fail(YORO_ERR_INVALID_ARG, "%s: null pointer", who);
  if (!shape_ok(n, h, w)) return nn_fail(YORO_ERR_INVALID_ARG, "%s: bad shape", who);
  if (cin <= 0 || cin % 32 || cout <= 0 || cout % 32)
    return nn_fail(YORO_ERR_INVALID_ARG, "%s: cin %d and cout %d must be positive multiples of 32", who, cin, cout);
  if (ldx < cin || ldx % 8 || lddy < cout || lddy % 8 || !al16(x) || !al16(dy) || !al16(workspace) || !al4(dw))
    return nn_fail(YORO_ERR_INVALID_ARG, "%s: misaligned pointer or stride", who);
  if (workspace_bytes < yoro_nn_conv3x3_wgrad_workspace(n, h, w, cin, cout))
    return nn_fail(YORO_ERR_WORKSPACE_TOO_SMALL, "%s: workspace too small", who);
  return launched(yoro::nn_conv3x3_wgrad(static_cast<const uint16_t*>(x), ldx, static_cast<const uint16_t*>(dy), lddy,
                                         n, h, w, cin, cout, dw, static_cast<float*>(workspace),
                                         (hipStream_t)hip_stream),
                  who);
}

int32_t yoro_nn_pack_weights(const float* w, int32_t cin, int32_t cout, void* w_fwd, void* w_bwd, void* hip_stream) {
  const char* who = "yoro_nn_pack_weights";
  if (!w || !w_fwd || cin <= 0 || cout <= 0) return nn_fail(YORO_ERR_INVALID_ARG, "%s: bad argument", who);
  return launched(yoro::nn_pack_weights(w, cin, cout, static_cast<uint16_t*>(w_fwd), static_cast<uint16_t*>(w_bwd),
                                        (hipStream_t)hip_stream),
                  who);
}

int32_t yoro_nn_avgpool2(const void* x, int32_t ldx, int32_t n, int32_t h, int32_t w, int32_t c, void* y, int32_t ldy,
                         void* hip_stream) {
  const char* who = "yoro_nn_avgpool2";
  if (!x || !y || !shape_ok(n, h, w) || h % 2 || w % 2 || c <= 0 || ldx < c || ldy < c)
    return nn_fail(YORO_ERR_INVALID_ARG, "%s: bad argument", who);
  return launched(yoro::nn_avgpool2(static_cast<const uint16_t*>(x), ldx, n, h, w, c, static_cast<uint16_t*>(y), ldy,
                                    (hipStream_t)hip_stream),
                  who);
}

int32_t yoro_nn_avgpool2_grad(const void* g, int32_t ldg, const void* addend, int32_t lda, const void* msrc,
                              int32_t ldm, int32_t n, int32_t h, int32_t w, int32_t c, void* dx, int32_t lddx,
                              void* hip_stream) {
  const char* who = "yoro_nn_avgpool2_grad";
  if (!g || !dx || !shape_ok(n, h, w) || h % 2 || w % 2 || c <= 0 || ldg < c || lddx < c ||
      (addend && lda < c) || (msrc && ldm < c))
    return nn_fail(YORO_ERR_INVALID_ARG, "%s: bad argument", who);
  return launched(yoro::nn_avgpool2_grad(static_cast<const uint16_t*>(g), ldg, static_cast<const uint16_t*>(addend),
                                         lda, static_cast<const uint16_t*>(msrc), ldm, n, h, w, c,
                                         static_cast<uint16_t*>(dx), lddx, (hipStream_t)hip_stream),
                  who);
}

int32_t yoro_nn_upsample2(const void* x, int32_t ldx, int32_t n, int32_t h, int32_t w, int32_t c, void* y, int32_t ldy,
                          void* hip_stream) {
  const char* who = "yoro_nn_upsample2";
  if (!x || !y || !shape_ok(n, h, w) || c <= 0 || ldx < c || ldy < c)
    return nn_fail(YORO_ERR_INVALID_ARG, "%s: bad argument", who);
  return launched(yoro::nn_upsample2(static_cast<const uint16_t*>(x), ldx, n, h, w, c, static_cast<uint16_t*>(y), ldy,
                                     (hipStream_t)hip_stream),
                  who);
}

int32_t yoro_nn_upsample2_grad(const void* g, int32_t ldg, int32_t n, int32_t h, int32_t w, int32_t c, void* dx,
                               int32_t lddx, void* hip_stream) {
  const char* who = "yoro_nn_upsample2_grad";
  if (!g || !dx || !shape_ok(n, h, w) || c <= 0 || ldg < c || lddx < c)
    return nn_fail(YORO_ERR_INVALID_ARG, "%s: bad argument", who);
  return launched(yoro::nn_upsample2_grad(static_cast<const uint16_t*>(g), ldg, n, h, w, c,
                                          static_cast<uint16_t*>(dx), lddx, (hipStream_t)hip_stream),
                  who);
}

int32_t yoro_nn_input(const uint8_t* rgba, const float* depth, const uint8_t* mask, int64_t npix, void* x,
                      void* hip_stream) {
  const char* who = "yoro_nn_input";
  if (!rgba || !depth || !mask || !x || npix <= 0 || !al4(rgba) || !al4(depth) || !al16(x))
    return nn_fail(YORO_ERR_INVALID_ARG, "%s: bad argument", who);
  return launched(yoro::nn_input(reinterpret_cast<const uint32_t*>(rgba), depth, mask, npix, static_cast<uint16_t*>(x),
                                 (hipStream_t)hip_stream),
                  who);
}

int32_t yoro_nn_l1_grad(const float* res, const uint8_t* rgba, const uint8_t* mask, const uint8_t* target_rgba,
                        int64_t npix, void* g_res, float* loss, void* workspace, void* hip_stream) {
  const char* who = "yoro_nn_l1_grad";
  if (!res || !rgba || !mask || !target_rgba || !g_res || !loss || !workspace || npix <= 0 || !al4(rgba) ||
      !al4(target_rgba) || !al16(g_res) || !al4(workspace))
    return nn_fail(YORO_ERR_INVALID_ARG, "%s: bad argument", who);
  return launched(yoro::nn_l1_grad(res, reinterpret_cast<const uint32_t*>(rgba), mask,
                                   reinterpret_cast<const uint32_t*>(target_rgba), npix, static_cast<uint16_t*>(g_res),
                                   loss, static_cast<float*>(workspace), (hipStream_t)hip_stream),
                  who);
}

int32_t yoro_nn_composite(const float* res, const uint8_t* rgba, const uint8_t* mask, int64_t npix, uint8_t* out,
                          void* hip_stream) {
  const char* who = "yoro_nn_composite";
  if (!res || !rgba || !mask || !out || npix <= 0 || !al4(rgba) || !al4(out))
    return nn_fail(YORO_ERR_INVALID_ARG, "%s: bad argument", who);
  return launched(yoro::nn_composite(res, reinterpret_cast<const uint32_t*>(rgba), mask, npix,
                                     reinterpret_cast<uint32_t*>(out), (hipStream_t)hip_stream),
                  who);
}

int32_t yoro_nn_adamw(float* w, float* m, float* v, const float* g, int64_t n, float lr, float beta1, float beta2,
                      float eps, float weight_decay, int32_t step, void* hip_stream) {
  const char* who = "yoro_nn_adamw";
  if (!w || !m || !v || !g || n <= 0 || step < 1) return nn_fail(YORO_ERR_INVALID_ARG, "%s: bad argument", who);
  return launched(yoro::nn_adamw(w, m, v, g, n, lr, beta1, beta2, eps, weight_decay, step, (hipStream_t)hip_stream),
                  who);
}

int32_t yoro_nn_tile_holes(const uint8_t* mask, int32_t w, int32_t h, int32_t tile, uint32_t* counts,
                           void* hip_stream) {
  const char* who = "yoro_nn_tile_holes";
  if (!mask || !counts || w <= 0 || h <= 0 || tile <= 0 || !al4(counts))
    return nn_fail(YORO_ERR_INVALID_ARG, "%s: bad argument", who);
  return launched(yoro::nn_tile_holes(mask, w, h, tile, counts, (hipStream_t)hip_stream), who);
}

int32_t yoro_nn_gather_crops(const uint8_t* rgba, const float* depth, const uint8_t* mask, int32_t w, int32_t h,
                             const int32_t* plan, int32_t k, int32_t crop, uint8_t* crop_rgba, float* crop_depth,
                             uint8_t* crop_mask, void* hip_stream) {
  const char* who = "yoro_nn_gather_crops";
  if (!rgba || !depth || !mask || !plan || !crop_rgba || !crop_depth || !crop_mask || w <= 0 || h <= 0 || k <= 0 ||
      k > 65535 || crop <= 0 || crop > w || crop > h || !al4(rgba) || !al4(depth) || !al4(crop_rgba) ||
      !al4(crop_depth) || !al4(plan))
    return nn_fail(YORO_ERR_INVALID_ARG, "%s: bad argument", who);
  return launched(yoro::nn_gather_crops(reinterpret_cast<const uint32_t*>(rgba), depth, mask, w, plan, k, crop,
                                        reinterpret_cast<uint32_t*>(crop_rgba), crop_depth, crop_mask,
                                        (hipStream_t)hip_stream),
                  who);
}

int32_t yoro_nn_composite_tiles(const float* res, const int32_t* plan, int32_t k, int32_t crop, int32_t tile,
                                const uint8_t* rgba, const uint8_t* mask, int32_t w, int32_t h, uint8_t* out,
                                void* hip_stream) {
  const char* who = "yoro_nn_composite_tiles";
  if (!res || !plan || !rgba || !mask || !out || k <= 0 || k > 65535 || crop <= 0 || tile <= 0 || tile > crop ||
      w <= 0 || h <= 0 || !al4(rgba) || !al4(out) || !al4(plan))
    return nn_fail(YORO_ERR_INVALID_ARG, "%s: bad argument", who);
  return launched(yoro::nn_composite_tiles(res, plan, k, crop, tile, w, h, reinterpret_cast<const uint32_t*>(rgba),
                                           mask, reinterpret_cast<uint32_t*>(out), (hipStream_t)hip_stream),
                  who);
}

}  // extern "C"

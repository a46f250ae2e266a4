/*
 * yoro_nn.h -- C-ABI of the learned hole filler in libyoro.so.
 *
 * The paper fills disocclusions with a filter (Section 7, Algorithm 3) and
 * names data-driven inpainting as the costly alternative it rejects for
 * mobile GPUs (Section 7; the GAN baseline of Section 8, evaluated in Section 11, Table 4).  This
 * library adds such a filler as an option on a data-centre GPU: a 4-level
 * convolutional encoder-decoder (3x3 convolutions, 32 base channels, 2x2
 * average pooling, nearest x2 upsampling, skip concatenations) whose output
 * is a residual added to the plain nearest-background fill on hole pixels
 * (Section 5, Observation O2, gives that fill).  These entry points are the
 * layers it is built from; the network is sequenced by the caller.
 *
 * Conventions
 * -----------
 * - Device pointers, caller-owned; no allocation or synchronisation inside;
 *   work is queued on the stream passed (void* hipStream_t, NULL = null
 *   stream).  Host validation returns YORO_ERR_INVALID_ARG (yoro.h) before
 *   anything is queued; launch failures return YORO_ERR_DEVICE.
 * - Tensors are NHWC: n images of h x w pixels, a pixel's channels
 *   contiguous.  ld is the element stride between consecutive pixels
 *   (>= channels; lets a layer read or write a channel slice of a wider
 *   concatenation buffer: pass the slice's first element and the buffer's ld).
 * - Activations, activation gradients and weight copies are bfloat16, passed
 *   as raw 16-bit words; they are rounded to nearest, ties to even, when
 *   written.  Master weights, weight gradients and the network output
 *   (residual) are FP32.  Products accumulate in FP32 on the matrix cores.
 * - bf16 pointers must be 16-byte aligned and ld a multiple of 8.
 * - Weights: [9][cout][cin], tap t = 3*ky + kx applied to input pixel
 *   (y + ky - 1, x + kx - 1); zero padding outside the image.
 */
#ifndef YORO_NN_H
#define YORO_NN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum yoro_nn_epilogue {
  YORO_NN_EPI_NONE = 0,
  YORO_NN_EPI_RELU = 1,
  /* multiply by (msrc > 0): the ReLU derivative at the same position of a
   * stored forward activation (input-gradient convolutions) */
  YORO_NN_EPI_RELU_GRAD = 2
} yoro_nn_epilogue;

/*
 * 3x3 convolution, stride 1, zero padding 1:
 *   y[p][co] = epi( sum_t sum_ci x[p + off(t)][ci] * w[t][co][ci] ),
 * for co < cout_store (the rest of the output is not written).
 * cin, cout: multiples of 32.  y is bf16 (y_fp32 = 0) or FP32 (y_fp32 = 1).
 * The input gradient of a convolution is this same operation applied to the
 * output gradient with the backward weight copy of yoro_nn_pack_weights.
 */
int32_t yoro_nn_conv3x3(const void* x, int32_t ldx, int32_t n, int32_t h, int32_t w, int32_t cin, const void* wgt,
                        int32_t cout, void* y, int32_t ldy, int32_t y_fp32, int32_t cout_store, int32_t epilogue,
                        const void* msrc, int32_t ldm, void* hip_stream);

/*
 * Weight gradient of the 3x3 convolution:
 *   dw[t][co][ci] = sum_p dy[p][co] * x[p + off(t)][ci]   (FP32 out).
 * Summed in fixed-size pixel chunks whose partial sums (in workspace) are
 * added in chunk order, so the result is deterministic.  workspace: device,
 * >= yoro_nn_conv3x3_wgrad_workspace(...) bytes, 16-byte aligned.
 */
size_t yoro_nn_conv3x3_wgrad_workspace(int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout);
int32_t yoro_nn_conv3x3_wgrad(const void* x, int32_t ldx, const void* dy, int32_t lddy, int32_t n, int32_t h,
                              int32_t w, int32_t cin, int32_t cout, float* dw, void* workspace, size_t workspace_bytes,
                              void* hip_stream);

/* FP32 master [9][cout][cin] -> bf16 forward copy [9][cout][cin] and backward
 * copy [9][cin][cout] with taps flipped (t -> 8 - t); w_bwd may be NULL
 * (inference needs only the forward copy). */
int32_t yoro_nn_pack_weights(const float* w, int32_t cin, int32_t cout, void* w_fwd, void* w_bwd, void* hip_stream);

/* 2x2 average pool: x is n x h x w (h, w even), y is n x h/2 x w/2. */
int32_t yoro_nn_avgpool2(const void* x, int32_t ldx, int32_t n, int32_t h, int32_t w, int32_t c, void* y, int32_t ldy,
                         void* hip_stream);
/* Its gradient at full resolution h x w, plus an optional addend (the skip
 * connection's gradient), times an optional ReLU derivative (msrc > 0):
 *   dx[p] = (g[parent(p)] / 4 + addend[p]) * (msrc[p] > 0). */
int32_t yoro_nn_avgpool2_grad(const void* g, int32_t ldg, const void* addend, int32_t lda, const void* msrc,
                              int32_t ldm, int32_t n, int32_t h, int32_t w, int32_t c, void* dx, int32_t lddx,
                              void* hip_stream);
/* Nearest x2 upsampling: x is n x h x w, y is n x 2h x 2w; and its gradient
 * (the sum of the four children) back to n x h x w. */
int32_t yoro_nn_upsample2(const void* x, int32_t ldx, int32_t n, int32_t h, int32_t w, int32_t c, void* y, int32_t ldy,
                          void* hip_stream);
int32_t yoro_nn_upsample2_grad(const void* g, int32_t ldg, int32_t n, int32_t h, int32_t w, int32_t c, void* dx,
                               int32_t lddx, void* hip_stream);

/* Network input from a plain-filled warp (yoro_reproject outputs): 32 bf16
 * channels per pixel: R/255, G/255, B/255, hole (mask != 0), log-depth mapped
 * from [log 0.3 m, log 50 m] to [0, 1] and clamped, then zeros.  x: npix x 32. */
int32_t yoro_nn_input(const uint8_t* rgba, const float* depth, const uint8_t* mask, int64_t npix, void* x,
                      void* hip_stream);

/* Masked L1 against a target image: loss = mean over hole pixels (mask != 0)
 * and R, G, B of |plain/255 + res - target/255|, and its gradient w.r.t. the
 * residual (bf16, npix x 32, channels >= 3 zero).  res: npix x 3 FP32.
 * loss: one FP32 on the device.  workspace >= YORO_NN_L1_WORKSPACE bytes. */
#define YORO_NN_L1_WORKSPACE ((size_t)(16 + 512) * 4)
int32_t yoro_nn_l1_grad(const float* res, const uint8_t* rgba, const uint8_t* mask, const uint8_t* target_rgba,
                        int64_t npix, void* g_res, float* loss, void* workspace, void* hip_stream);

/* Output: hole pixels get clamp(rint(255 * (plain/255 + res)), 0, 255) in
 * R, G, B and keep their alpha; other pixels are copied. */
int32_t yoro_nn_composite(const float* res, const uint8_t* rgba, const uint8_t* mask, int64_t npix, uint8_t* out,
                          void* hip_stream);

/*
 * Hole-tile inference.  A w x h frame is cut into tile x tile blocks; only
 * blocks with a hole need the network, each run inside a crop of
 * crop x crop pixels (the block plus a halo on every side at least as wide
 * as the network's boundary reach, 54 px) placed inside the frame on the
 * 8-pixel pooling grid.  Each crop edge is then a frame edge or a halo away
 * from the block, so the block's result equals the whole frame's.
 *
 * A plan is a device int32 array [k][4]: (crop x, crop y, block x, block y)
 * per crop, the crop inside the frame and the block inside the crop.
 *
 * yoro_nn_tile_holes: counts[ty * ntx + tx] = number of pixels with
 *   mask != 0 in block (tx, ty), ntx = ceil(w / tile); device u32 array.
 * yoro_nn_gather_crops: copy the k planned crops of a frame's RGBA, depth and
 *   mask into contiguous crop batches (k x crop x crop).
 * yoro_nn_composite_tiles: for each planned crop, write the learned composite
 *   of the hole pixels of its block into out (a frame, normally a copy of
 *   the plain fill); res is the network's residual over the crop batch.
 * The plan is read on the device and trusted: the caller keeps every crop
 * inside the frame.
 */
int32_t yoro_nn_tile_holes(const uint8_t* mask, int32_t w, int32_t h, int32_t tile, uint32_t* counts,
                           void* hip_stream);
int32_t yoro_nn_gather_crops(const uint8_t* rgba, const float* depth, const uint8_t* mask, int32_t w, int32_t h,
                             const int32_t* plan, int32_t k, int32_t crop, uint8_t* crop_rgba, float* crop_depth,
                             uint8_t* crop_mask, void* hip_stream);
int32_t yoro_nn_composite_tiles(const float* res, const int32_t* plan, int32_t k, int32_t crop, int32_t tile,
                                const uint8_t* rgba, const uint8_t* mask, int32_t w, int32_t h, uint8_t* out,
                                void* hip_stream);

/* One AdamW step on n FP32 parameters (decoupled weight decay, bias-corrected
 * moments; step counts from 1). */
int32_t yoro_nn_adamw(float* w, float* m, float* v, const float* g, int64_t n, float lr, float beta1, float beta2,
                      float eps, float weight_decay, int32_t step, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* YORO_NN_H */

/*
 * yoro_model.h -- inference of the learned hole filler as single calls.
 *
 * The network is the encoder-decoder whose layers yoro_nn.h exposes (the
 * paper's own disocclusion fill is the filter of Section 7; a learned filler
 * stands in for the data-driven inpainting that section sets aside as too
 * heavy for a phone, and refines the nearest-background fill of Section 5,
 * Observation O2).  These calls run its whole forward pass and composite on
 * the device, so a serving loop can use it without a host-side sequencer.
 *
 * Weights: "model weights" are the bf16 forward copies of all 18 layers,
 * packed back to back; layer i occupies elements [offset[i], offset[i+1])
 * as [9][cout_pad][cin_pad] (yoro_model_layout).  yoro_model_pack makes
 * them from FP32 masters laid out the same way.
 *
 * Conventions as in yoro.h: caller-owned device pointers, no allocation or
 * synchronisation, work queued on the given stream, YORO_ERR_INVALID_ARG
 * before anything is queued, YORO_ERR_WORKSPACE_TOO_SMALL when the
 * workspace is short, YORO_ERR_DEVICE on a failed launch.
 */
#ifndef YORO_MODEL_H
#define YORO_MODEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define YORO_MODEL_LAYERS 18

/* Host arrays: cin_pad[18], cout_pad[18] (the kernels' channel counts, each
 * a multiple of 32) and offset[19] (elements).  Any pointer may be NULL. */
int32_t yoro_model_layout(int32_t* cin_pad, int32_t* cout_pad, int64_t* offset);
size_t yoro_model_weights_bytes(void);

/* FP32 masters (offset[18] floats, same layout) -> bf16 model weights
 * (round to nearest, ties to even), all layers in one launch. */
int32_t yoro_model_pack(const float* master, void* weights, void* hip_stream);

/* The same, and, if weights_bwd is not NULL, the backward copies that the
 * input gradient runs on: layer i at the same offsets as [9][cin_pad]
 * [cout_pad] with the taps flipped (tap 8 - t), as yoro_nn_pack_weights
 * writes them.  For training, which refreshes both copies after each
 * update. */
int32_t yoro_model_pack_train(const float* master, void* weights, void* weights_bwd, void* hip_stream);

/* Workspace for n images of h x w (h, w multiples of 8, n*h*w < 2^31). */
size_t yoro_model_workspace_bytes(int32_t n, int32_t h, int32_t w);

/* Where a forward pass over n images of h x w leaves its stored activations
 * in the workspace (read them after the call, e.g. to check each layer):
 * offsets[18] in bytes from the workspace's start, of NHWC bf16 buffers in
 * this order, with their channels per pixel (level l has (h >> l) x (w >> l)
 * pixels per image): e0a 32; c0 64 (d0a, then e0b; held as two planes, all
 * pixels' 32 channels of d0a, then all pixels' 32 channels of e0b); d0b 32;
 * d0c 32; p1 32; e1a 64; c1 128 (d1a, e1b); d1b 64; d1c 64; p2 64; e2a 128;
 * c2 256 (d2a, e2b); d2b 128; d2c 128; p3 128; e3a 256; e3b 256; and the
 * FP32 residual, 3 per pixel (yoro_model_residual writes the caller's res
 * instead). */
#define YORO_MODEL_ACTIVATIONS 18
int32_t yoro_model_workspace_layout(int32_t n, int32_t h, int32_t w, int64_t* offsets);

/* Residual (FP32 [n*h*w][3]) of the network on n plain-filled images
 * (rgba u8 [n][h][w][4], depth f32 [n][h][w], mask u8 [n][h][w]). */
int32_t yoro_model_residual(const void* weights, const uint8_t* rgba, const float* depth, const uint8_t* mask,
                            int32_t n, int32_t h, int32_t w, float* res, void* workspace, size_t workspace_bytes,
                            void* hip_stream);

/* Learned fill of n whole frames: out = rgba except on hole pixels
 * (mask != 0), which get clamp(rint(255 * (plain / 255 + residual))) with
 * alpha kept.  out may equal rgba. */
int32_t yoro_model_fill(const void* weights, const uint8_t* rgba, const float* depth, const uint8_t* mask, int32_t n,
                        int32_t h, int32_t w, uint8_t* out, void* workspace, size_t workspace_bytes,
                        void* hip_stream);

/* Learned fill of the planned blocks of one w x h frame (plan: device int32
 * [k][4] as in yoro_nn.h; crop = tile + 2 * halo; the plan is trusted to
 * keep crops inside the frame).  All k crops are gathered first, then run
 * `chunk` at a time, so out may equal rgba.  Pixels outside the planned
 * blocks, and non-hole pixels, are not written. */
size_t yoro_model_tiles_workspace_bytes(int32_t k, int32_t chunk, int32_t tile, int32_t halo);
int32_t yoro_model_fill_tiles(const void* weights, const uint8_t* rgba, const float* depth, const uint8_t* mask,
                              int32_t w, int32_t h, const int32_t* plan, int32_t k, int32_t tile, int32_t halo,
                              int32_t chunk, uint8_t* out, void* workspace, size_t workspace_bytes,
                              void* hip_stream);

/* Learned fill of one w x h frame in bands of `band` full-width rows: band
 * b covers rows [b band, b band + band) and runs on the crop of rows
 * [b band - halo, b band + band + halo), shifted inward at the frame's top
 * and bottom (band, halo, w, h multiples of 8, halo <= band / 2).  With halo
 * at or above the network's reach (54 pixels) the result equals
 * yoro_model_fill bit for bit, at about (band + 2 halo) / band of its work
 * and with the workspace of one crop.  band_has_holes: host, one byte per
 * band (NULL: every band); a band without holes is skipped (its pixels are
 * not written).  out may equal rgba: a band is written only after every
 * band pass that reads its rows. */
size_t yoro_model_bands_workspace_bytes(int32_t w, int32_t h, int32_t band, int32_t halo);
int32_t yoro_model_fill_bands(const void* weights, const uint8_t* rgba, const float* depth, const uint8_t* mask,
                              int32_t w, int32_t h, int32_t band, int32_t halo, const uint8_t* band_has_holes,
                              uint8_t* out, void* workspace, size_t workspace_bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* YORO_MODEL_H */

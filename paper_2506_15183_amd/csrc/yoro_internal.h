// Internal definitions shared by the HIP kernels and the C-ABI host code.
#pragma once

#include <functional>

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace yoro {

// One frame of work as the kernels see it.  RGBA8 pixels are moved as one
// 32-bit word each (byte order preserved).
struct DevJob {
  const uint32_t* src_rgba;
  const float* src_depth;
  uint32_t* dst_rgba;
  float* dst_depth;  // nullable
  uint8_t* dst_mask; // nullable
  int32_t width;
  int32_t height;
  float baseline_m;
  float focal_px;
  int32_t target_eye;  // 0: target right (x_t = x - d); 1: target left (x_t = x + d)
  int32_t fill_mode;   // 0: none; 1: nearest background
  uint32_t row_start;  // first row of this job in the batch's flat row space
  uint32_t pad_;
};
static_assert(sizeof(DevJob) == 72, "DevJob layout");

// Header at the start of a batch workspace.
struct BatchHeader {
  uint32_t n_jobs;
  uint32_t total_rows;
  uint32_t max_width;
  uint32_t errors;  // rows skipped because they did not fit the launch's LDS
  uint32_t pad_[12];
};
static_assert(sizeof(BatchHeader) == 64, "BatchHeader layout");

// Jobs carried in one upload kernel's arguments.
constexpr int kUploadChunk = 24;
struct UploadChunk {
  DevJob jobs[kUploadChunk];
  uint32_t first;
  uint32_t count;
};

constexpr int kThreads = 256;      // threads per workgroup (4 waves of 64)
constexpr int kFillPatcher = 3;    // YORO_FILL_PATCHER
constexpr int kMaxPPT = 32;        // pixels per thread: width <= kThreads * kMaxPPT = 8192

// Pixels per thread for rows up to max_width columns: the smallest
// instantiated value with kThreads * ppt >= max_width (-1 if too wide).
inline int ppt_for(int max_width) {
  static const int kPPT[] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 16, 20, 24, 28, 32};
  const int need = (max_width + kThreads - 1) / kThreads;
  for (int p : kPPT)
    if (p >= need) return p;
  return -1;
}
// Width the row kernel's LDS is laid out for: max_width rounded up to 64.
inline int lds_width(int max_width) { return (max_width + 63) & ~63; }
// Dynamic LDS bytes of the warp kernel laid out for wl columns: 64-bit keys
// (plus 64 sinks), hit masks, 16 bytes of padding and the u16 hole list (four
// per-wave segments of 64 entries per kThreads columns).
inline size_t warp_lds_bytes(int wl) {
  const size_t w = (size_t)wl;
  const size_t hl = (w + kThreads - 1) / kThreads * kThreads;
  return (w + 64) * 8 + (w / 64) * 8 + 16 + hl * 2;
}
// Dynamic LDS bytes of the stand-alone fill kernel: colours, depths, masks.
inline size_t fill_lds_bytes(int wl) {
  const size_t w = (size_t)wl;
  return w * 4 + w * 4 + (w / 64) * 8;
}

// Texel slots the low-resolution kernel keeps in LDS for rows up to
// max_width columns at k = 1 << lg: ceil(max_width / k) rounded up to 64.
inline int lowres_texel_slots(int max_width, int lg) {
  const int wk = (max_width + (1 << lg) - 1) >> lg;
  return (wk + 63) & ~63;
}

// Launchers (defined in warp_fill.hip).  They return hipSuccess or the launch error.
// near: the near-object hybrid's far field (source depth < near_m skipped).
// grid >= the frame's height: one workgroup per row (the one-row kernel);
// otherwise a persistent grid of `grid` workgroups.  table: null, or a batch
// workspace to receive the frame as a one-job batch (header, job record).
hipError_t launch_warp_single(const DevJob& job, int ppt, int grid, hipStream_t stream, bool near = false,
                              float near_m = 0.0f, BatchHeader* table = nullptr);
// The batch kernel's grid covers the flat row space once, `rows`
// consecutive rows per workgroup, 1 <= rows <= kBatchRows (total_rows: the
// rows the grid is sized for).
constexpr int kBatchRows = 3;
hipError_t launch_warp_batch(const BatchHeader* hdr, const DevJob* jobs, int max_width, uint32_t total_rows, int rows,
                             hipStream_t stream);
// Writes chunk.count job records at dst + chunk.first and, if hdst is not
// null, hdr at hdst, from the kernel's arguments.
hipError_t launch_upload(const UploadChunk& chunk, DevJob* dst, const BatchHeader& hdr, BatchHeader* hdst,
                         hipStream_t stream);
hipError_t launch_fill(uint32_t* rgba, float* depth, uint8_t* mask, int32_t width, int32_t height,
                       int32_t target_eye, int32_t fill_mode, int ppt, int grid, hipStream_t stream);
hipError_t launch_hole_sse(const uint32_t* rgba, const uint32_t* ref, const uint8_t* mask, int64_t n,
                           unsigned long long* out, int grid, hipStream_t stream);
// This thread's message for yoro_last_error() (defined in capi.hip).
void set_last_error(const char* msg);

// Learned-fill kernels (defined in nn.hip).  bf16 tensors are raw uint16_t.
constexpr int kWgradGroups = 512;     // workgroups the weight gradient's split-K grid aims for
constexpr int kWgradMaxChunks = 512;  // at most this many chunk partial sums
constexpr int kLossBlocks = 512;      // blocks (and partial sums) of the L1 loss
constexpr int kPackMaxLayers = 32;    // layers one nn_pack_model launch takes
// FP32 masters of `layers` layers, layer l at elements [off[l], off[l + 1])
// as [9][cout[l]][cin[l]], to bf16 copies: forward (same layout) and, if wb
// is not null, backward ([9][cin][cout], taps flipped), in one launch.
hipError_t nn_pack_model(const float* w, const long long* off, const int* cin, const int* cout, int layers,
                         uint16_t* wf, uint16_t* wb, hipStream_t s);
size_t nn_wgrad_chunks(long long N, int H, int W, int Cin, int Cout);
// The convolutions below launch a persistent grid (the workgroups that fit,
// each looping over output tiles) unless persistent is false: then one
// workgroup per tile, which lets kernels on other queues take compute units
// between tiles (for work that shares the GPU with latency-critical
// launches).
// xcs: elements from one 32-channel input chunk to the next (32 for NHWC
// x; larger when x keeps its channel chunks in separate planes, each
// [pixels][ldx]).
hipError_t nn_conv3x3(const uint16_t* x, int ldx, int N, int H, int W, int Cin, const uint16_t* wgt, int Cout, void* y,
                      int ldy, int y_fp32, int cout_store, int epi, const uint16_t* msrc, int ldm, hipStream_t s,
                      bool persistent = true, long long xcs = 32);
// yoro_model_fill_tiles with a host call after each layer of the network is
// enqueued (each chunk of crops runs the 18 layers in turn): the caller may
// wait there, e.g. for the layer before, so that work queued behind the fill
// on the same hardware queue waits for a layer or two at most.  With a pace,
// the convolutions launch one workgroup per tile (not persistent), so work
// on other queues also gets compute units within a tile's time.  Same
// arguments, results and errors as yoro_model_fill_tiles otherwise; an empty
// pace is that call.
int32_t model_fill_tiles_paced(const void* weights, const uint8_t* rgba, const float* depth, const uint8_t* mask,
                               int32_t w, int32_t h, const int32_t* plan, int32_t k, int32_t tile, int32_t halo,
                               int32_t chunk, uint8_t* out, void* workspace, size_t workspace_bytes,
                               void* hip_stream, const std::function<hipError_t()>& pace);

// yoro_model_fill_bands with the same host call after each layer.
int32_t model_fill_bands_paced(const void* weights, const uint8_t* rgba, const float* depth, const uint8_t* mask,
                               int32_t w, int32_t h, int32_t band, int32_t halo, const uint8_t* band_has_holes,
                               uint8_t* out, void* workspace, size_t workspace_bytes, void* hip_stream,
                               const std::function<hipError_t()>& pace);

// The first convolution (Cin 32, bf16 output, optional ReLU) reading the
// frame's RGBA, depth and mask and packing them as nn_input does, in one
// pass; equal to nn_input then nn_conv3x3.
hipError_t nn_conv3x3_input(const uint32_t* rgba, const float* depth, const uint8_t* mask, int N, int H, int W,
                            const uint16_t* wgt, int Cout, uint16_t* y, int ldy, int relu, hipStream_t s,
                            bool persistent = true);
// The convolution (bf16 output, optional ReLU) followed by a 2x2 average
// pool of its stored output into `pool` (H, W even), in one pass; equal to
// nn_conv3x3 then nn_avgpool2.
hipError_t nn_conv3x3_pool(const uint16_t* x, int ldx, int N, int H, int W, int Cin, const uint16_t* wgt, int Cout,
                           uint16_t* y, int ldy, int relu, uint16_t* pool, int ldp, hipStream_t s,
                           bool persistent = true);
// The same convolution applied to the nearest x2 upsampling of x (x is
// N x H/2 x W/2; H, W even), read in place.
hipError_t nn_conv3x3_up(const uint16_t* x, int ldx, int N, int H, int W, int Cin, const uint16_t* wgt, int Cout,
                         void* y, int ldy, int y_fp32, int cout_store, int epi, const uint16_t* msrc, int ldm,
                         hipStream_t s, bool persistent = true);
hipError_t nn_conv3x3_wgrad(const uint16_t* x, int ldx, const uint16_t* dy, int lddy, int N, int H, int W, int Cin,
                            int Cout, float* dw, float* ws, hipStream_t s);
hipError_t nn_pack_weights(const float* w, int cin, int cout, uint16_t* wf, uint16_t* wb, hipStream_t s);
hipError_t nn_avgpool2(const uint16_t* x, int ldx, int N, int h, int w, int c, uint16_t* y, int ldy, hipStream_t s);
hipError_t nn_avgpool2_grad(const uint16_t* g, int ldg, const uint16_t* add, int lda, const uint16_t* msrc, int ldm,
                            int N, int h, int w, int c, uint16_t* dx, int lddx, hipStream_t s);
hipError_t nn_upsample2(const uint16_t* x, int ldx, int N, int h, int w, int c, uint16_t* y, int ldy, hipStream_t s);
hipError_t nn_upsample2_grad(const uint16_t* g, int ldg, int N, int h, int w, int c, uint16_t* dx, int lddx,
                             hipStream_t s);
hipError_t nn_input(const uint32_t* rgba, const float* depth, const uint8_t* mask, long long npix, uint16_t* x,
                    hipStream_t s);
hipError_t nn_l1_grad(const float* res, const uint32_t* rgba, const uint8_t* mask, const uint32_t* target,
                      long long npix, uint16_t* g, float* loss, float* ws, hipStream_t s);
hipError_t nn_composite(const float* res, const uint32_t* rgba, const uint8_t* mask, long long npix, uint32_t* out,
                        hipStream_t s);
hipError_t nn_adamw(float* w, float* m, float* v, const float* g, long long n, float lr, float b1, float b2, float eps,
                    float wd, int step, hipStream_t s);
hipError_t nn_tile_holes(const uint8_t* mask, int w, int h, int tile, uint32_t* counts, hipStream_t s);
hipError_t nn_gather_crops(const uint32_t* rgba, const float* depth, const uint8_t* mask, int w, const int* plan, int k,
                           int crop, uint32_t* crgba, float* cdepth, uint8_t* cmask, hipStream_t s);
hipError_t nn_composite_tiles(const float* res, const int* plan, int k, int crop, int tile, int w, int h,
                              const uint32_t* rgba, const uint8_t* mask, uint32_t* out, hipStream_t s);

// Occupancy-derived workgroups per CU for the row kernels.
// Resident workgroups per CU of a warp kernel laid out for max_width columns:
// the single-frame kernel, the batch kernel, or their one-row-per-workgroup
// instantiations.
enum { kWarpSingle = 0, kWarpBatch = 1, kWarpBatchOneRow = 2, kWarpSingleOneRow = 3 };
int warp_blocks_per_cu(int max_width, int kind);
int fill_blocks_per_cu(int width, int fill_mode);

// The near-object hybrid (hybrid.hip): the near layer of a box-and-sphere
// scene for one eye, and its composite over the far field.
}  // namespace yoro
struct yoro_object;
namespace yoro {
hipError_t launch_render_near(const ::yoro_object* objs, int n, int W, int H, int x_off, int y_off, double f,
                              double cx, double cy, double eye_x, float near_m, uint32_t* rgba, float* depth,
                              hipStream_t stream);
hipError_t launch_composite_near(const uint32_t* near_rgba, const float* near_depth, float near_m, int64_t n,
                                 uint32_t* rgba, float* depth, uint8_t* mask, int grid, hipStream_t stream);

// Reprojection through a general pose (pose.hip): X_t = A X + b per pinhole
// point, A = R^T and b = -R^T t of the target eye's pose in the source eye's
// frame, rounded to FP32 by the host.
struct PoseGeom {
  float A[9];
  float b[3];
  float f, cx, cy;
  int32_t width, height;
};
// keys: the caller's workspace, width * height u64, 16-byte aligned.
hipError_t launch_pose(const uint32_t* src_rgba, const float* src_depth, const PoseGeom& g, int fill_mode,
                       int target_right, uint32_t* dst_rgba, float* dst_depth, uint8_t* dst_mask, uint64_t* keys,
                       int cus, hipStream_t stream);

// Reprojection through a downsampled intermediate buffer (lowres.hip):
// k = 1 << lg (lg 0..4), units of G = 1 << glg rows (glg <= lg).  one != NULL
// launches that single frame; otherwise the batch table (hdr, jobs).
size_t lowres_lds_bytes(int max_width, int lg);
int lowres_blocks_per_cu(int max_width, int lg, bool batch);
hipError_t launch_lowres(const DevJob* one, const BatchHeader* hdr, const DevJob* jobs, int max_width, int lg,
                         int glg, int linear, int grid, hipStream_t stream);

}  // namespace yoro

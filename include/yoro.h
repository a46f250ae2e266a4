/*
 * yoro.h -- C-ABI of libyoro.so: synthesise the second eye of a stereo pair
 * from one rendered eye (colour + per-pixel depth) on an AMD Instinct
 * MI355X (gfx950).
 *
 * Method: "You Only Render Once" (arXiv 2506.15183).  The rendered
 * (dominant) eye's G-buffer (Section 3.2) is reprojected to the other eye
 * (Section 6: reprojection equation M = (VP_left)^-1 VP_right, Algorithms 1
 * and 2) and its disocclusions are filled from the background (Section 5
 * Observation O2, Section 7 Patcher).  For two pinhole eyes that differ only
 * by a shift B along x (parallel stereo) the matrix transform reduces to a
 * per-pixel horizontal shift of d = round(B*f/z) pixels, one-signed by
 * Observation O1, so every row is independent.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All image pointers are caller-owned DEVICE pointers.  The library never
 *   allocates, frees or synchronises inside these calls and launches only on
 *   the stream passed (hipStream_t given as void*; NULL = the null stream).
 *   Every call returns as soon as its kernels are queued.
 * - RGBA8: row-major H x W x 4 bytes, byte order R, G, B, A, contiguous,
 *   4-byte aligned.  Depth: row-major H x W FP32, linear eye-space depth in
 *   metres (planar z, not ray length), 4-byte aligned.  Depth > 0 is
 *   geometry (+inf is "at infinity"); NaN, +-0 and negative depths carry no
 *   geometry and are not splatted (not an error).
 * - Mask: u8 per pixel, 0 = hit, 1 = disocclusion (filled, or left empty
 *   with YORO_FILL_NONE), 2 = disocclusion with no hit anywhere in its row
 *   (left as RGBA 0, depth +inf).
 * - Sizes: 1 <= width <= YORO_MAX_WIDTH, 1 <= height <= YORO_MAX_HEIGHT.
 * - Errors: arguments are checked on the host before anything is queued; a
 *   bad argument returns YORO_ERR_INVALID_ARG (or YORO_ERR_UNSUPPORTED) and
 *   queues nothing.  A failed launch returns YORO_ERR_DEVICE.  Faults inside
 *   kernels surface at the caller's next synchronisation of the stream.
 *   yoro_last_error() returns this thread's message for the last non-OK
 *   status.  No C++ exception crosses this interface.
 * - Determinism: collisions are resolved by a 64-bit atomicMin on
 *   (depth bits << 32 | source RGBA word).  Two sources of one row with
 *   bitwise-equal depth have equal disparity and so never reach the same
 *   target column: every collision is decided by the depth bits alone, the
 *   low word only carries the winner's colour, and every output bit is
 *   independent of thread order.  (The general-pose call, whose depth test
 *   spans the frame, keys on (target depth bits << 32 | source index).)
 */
#ifndef YORO_H
#define YORO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define YORO_VERSION 1
#define YORO_MAX_WIDTH 8192
#define YORO_MAX_HEIGHT 16384

typedef enum yoro_target_eye {
  /* Source = left eye, target = right eye (right camera at +B on x):
   * target column = source column - d. */
  YORO_TARGET_RIGHT = 0,
  /* Source = right eye, target = left eye: target column = source column + d. */
  YORO_TARGET_LEFT = 1
} yoro_target_eye;

typedef enum yoro_fill_mode {
  /* Leave disocclusions empty: RGBA 0, depth +inf, mask 1. */
  YORO_FILL_NONE = 0,
  /* Row-wise nearest background: of the nearest hit to the left and the
   * nearest hit to the right (in the resolved row, never a filled pixel),
   * take the one with the larger depth; on equal depth the one on the side
   * opposite the shift (right for YORO_TARGET_RIGHT, left for
   * YORO_TARGET_LEFT); with one neighbour take it (Section 5 O2; Section 7,
   * Patcher figure). */
  YORO_FILL_NEAREST_BG = 1,
  /* Learned fill: the nearest-background fill above, then the learned
   * filler of yoro_model.h refines the hole pixels (mask != 0) of the whole
   * frame (non-hole pixels are left bit for bit).  Section 7 sets
   * data-driven inpainting aside as too heavy for a phone; the network is
   * this library's extension.  Needs a yoro_model, so only yoro_fill_holes
   * and yoro_stereo_batch take it (elsewhere YORO_ERR_UNSUPPORTED), and only
   * for frames whose width and height are multiples of 8. */
  YORO_FILL_LEARNED = 2,
  /* The weighted Patcher (Section 7, Algorithm 3 with Equation 7): from the
   * nearest-background hit e of a hole at x (chosen as above, nearest hits L
   * and R), samples outward from e over R - L - 1 columns (the
   * disocclusion's width, no cap; stopping at the frame's edge) and rows
   * y, y-1, y+1 that are hits not nearer than e; each takes
   * w_rem/2 + 0.3 w_rem |x - e| / (R - L - 1) of the remaining weight w_rem
   * (starting at 1); the hole gets rint(sum(C w) / (1 - w_rem)) per RGB
   * channel in FP32, e's alpha and depth, mask 1.  Reads neighbouring rows,
   * so yoro_reproject needs dst_depth and dst_mask for it and the batched
   * call does not take it (YORO_ERR_UNSUPPORTED). */
  YORO_FILL_PATCHER = 3
} yoro_fill_mode;

/*
 * The learned filler as the fill calls take it.  weights: device, the bf16
 * model weights of yoro_model.h (yoro_model_weights_bytes(), 16-byte
 * aligned).  workspace: device, 16-byte aligned, at least
 * yoro_model_workspace_bytes(1, h, w) bytes for the largest frame it fills
 * (the network's activations; overwritten by every learned fill, so calls
 * that share one workspace must be ordered on one stream).  Caller-owned;
 * the library only reads the struct during the call.
 */
typedef struct yoro_model {
  const void* weights;
  void* workspace;
  size_t workspace_bytes;
} yoro_model;

typedef enum yoro_status {
  YORO_OK = 0,
  YORO_ERR_INVALID_ARG = 1,
  YORO_ERR_UNSUPPORTED = 2,
  YORO_ERR_WORKSPACE_TOO_SMALL = 3,
  YORO_ERR_DEVICE = 4
} yoro_status;

/*
 * yoro_reproject -- warp one frame to the other eye and (optionally) fill
 * its disocclusions (Section 6, Algorithms 1-2; Section 7).
 *
 * Per source pixel (x, y) with depth z > 0:
 *   bf = baseline_m * focal_px              (one FP32 multiply)
 *   q  = bf / z                             (correctly rounded FP32 division)
 *   skip unless q < width; d = roundf(q)    (halfway away from zero)
 *   xt = x - d (TARGET_RIGHT) or x + d (TARGET_LEFT); skip unless 0 <= xt < W
 *   the nearest depth wins target (xt, y).
 * Hit targets take the winning source pixel's RGBA (all four bytes) and
 * depth; the rest are disocclusions, handled per fill_mode.
 *
 * src_rgba, src_depth: inputs (not modified).  dst_rgba: output, required.
 * dst_depth, dst_mask: optional outputs (NULL to skip).  Outputs must not
 * overlap the inputs or each other.  baseline_m and focal_px: finite, > 0.
 */
int32_t yoro_reproject(const uint8_t* src_rgba, const float* src_depth, int32_t width, int32_t height,
                       float baseline_m, float focal_px, int32_t target_eye, int32_t fill_mode,
                       uint8_t* dst_rgba, float* dst_depth, uint8_t* dst_mask, void* hip_stream);

/*
 * yoro_fill_holes -- fill the disocclusions of an already warped frame in
 * place (Section 7; Section 5 O2).  Pixels with mask == 0 are hits and are
 * left unchanged; every other pixel is a hole and is refilled per fill_mode
 * from the hits of its row only (so the result does not depend on order),
 * and with YORO_FILL_LEARNED then refined by the network, which reads the
 * whole plain-filled frame.  rgba, depth, mask: in/out, all required.
 * model: required for YORO_FILL_LEARNED (YORO_ERR_INVALID_ARG if NULL,
 * YORO_ERR_WORKSPACE_TOO_SMALL if its workspace is short), ignored
 * otherwise.  YORO_FILL_NONE is a no-op.
 */
int32_t yoro_fill_holes(uint8_t* rgba, float* depth, uint8_t* mask, int32_t width, int32_t height,
                        int32_t target_eye, int32_t fill_mode, const yoro_model* model, void* hip_stream);

/*
 * Batched stereo synthesis: many frames of mixed sizes in one persistent
 * launch.  Each job is one yoro_reproject call.  Rows of all jobs form one
 * flat index space that the workgroups stride over.
 */
typedef struct yoro_job {
  const uint8_t* src_rgba;
  const float* src_depth;
  uint8_t* dst_rgba;
  float* dst_depth; /* nullable */
  uint8_t* dst_mask; /* nullable */
  int32_t width;
  int32_t height;
  float baseline_m;
  float focal_px;
  int32_t target_eye;
  int32_t fill_mode;
} yoro_job;

/* Device workspace bytes needed for n_jobs jobs (a header plus one record
 * per job).  Returns 0 for n_jobs <= 0 or n_jobs > YORO_MAX_BATCH_JOBS. */
#define YORO_MAX_BATCH_JOBS 65536
size_t yoro_stereo_batch_workspace_bytes(int32_t n_jobs);

/*
 * yoro_stereo_batch_prepare -- validate jobs_host[0..n_jobs) on the host
 * (same rules as yoro_reproject, plus: no job's outputs may overlap any
 * job's inputs or outputs) and queue the upload of the job table into
 * dev_workspace (device memory, >= yoro_stereo_batch_workspace_bytes,
 * 16-byte aligned) on hip_stream.  The upload is done by small kernels that
 * carry the table in their arguments, so jobs_host may be freed on return
 * and the call may be captured into a HIP graph.  YORO_FILL_LEARNED jobs
 * need the model and so go through yoro_stereo_batch
 * (YORO_ERR_UNSUPPORTED here).
 */
int32_t yoro_stereo_batch_prepare(const yoro_job* jobs_host, int32_t n_jobs, void* dev_workspace,
                                  size_t workspace_bytes, void* hip_stream);

/*
 * yoro_stereo_batch_launch -- run the jobs that the last prepare on this
 * workspace uploaded, as one kernel whose grid covers the rows of all jobs
 * once (a few consecutive rows per workgroup).  max_width must be >= every
 * job's width (it sizes the per-row scratch in LDS); rows of a wider job are
 * skipped and counted in the workspace's error counter (see
 * yoro_stereo_batch_errors).  total_rows: the sum of the prepared jobs'
 * heights (1 .. 2^32 - 1), which sizes the grid; rows past a smaller value
 * are skipped and counted the same way.  Capture-safe: no allocation, copy
 * or sync.
 */
int32_t yoro_stereo_batch_launch(const void* dev_workspace, int32_t max_width, int64_t total_rows,
                                 void* hip_stream);

/*
 * yoro_stereo_batch -- prepare + launch, then the learned fill of the jobs
 * whose fill_mode is YORO_FILL_LEARNED.  Those jobs are warped with the
 * nearest-background fill in the batched launch, so plain and learned jobs
 * share it; each learned job then runs yoro_fill_holes's network pass on
 * its output, in job order on hip_stream.  A learned job needs dst_depth
 * and dst_mask (the network's inputs) and width and height that are
 * multiples of 8; model is required when any job is learned (its
 * workspace sized for the largest learned job) and ignored otherwise.
 * Capture-safe like prepare and launch.
 */
int32_t yoro_stereo_batch(const yoro_job* jobs_host, int32_t n_jobs, void* dev_workspace,
                          size_t workspace_bytes, const yoro_model* model, void* hip_stream);

/* Device address of the workspace's u32 error counter (rows skipped by the
 * last launch because max_width was too small); reset by prepare. */
const uint32_t* yoro_stereo_batch_errors(const void* dev_workspace);

/*
 * yoro_stereo_batch_static -- yoro_stereo_batch for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, hosts that forbid hipMalloc): the same prepare + launch of the
 * same kernels, with the job table in a fixed device array inside the
 * library (64 + 72 * YORO_STATIC_MAX_JOBS bytes per GPU, held until the
 * process ends) instead of a caller workspace.  It allocates and frees no
 * device memory.  Plain jobs only: YORO_FILL_LEARNED and
 * YORO_FILL_PATCHER are YORO_ERR_UNSUPPORTED; more than
 * YORO_STATIC_MAX_JOBS jobs is YORO_ERR_INVALID_ARG.  Every call on one GPU
 * shares that GPU's array, which keeps the last call's table (each call
 * rewrites the header and every record it uses, error counter included):
 * calls that overlap on one GPU (on different streams, or not yet finished
 * when another is queued on another stream) race, so order them on one
 * stream.  Outputs and other errors as yoro_stereo_batch.
 */
#define YORO_STATIC_MAX_JOBS 1024
int32_t yoro_stereo_batch_static(const yoro_job* jobs_host, int32_t n_jobs, void* hip_stream);

/*
 * yoro_reproject_lowres -- yoro_reproject through a downsampled intermediate
 * buffer (Section 6 (c), resolution-independent intermediate buffers, and
 * (d), linear interpolation along the row).  The warp runs on one texel per
 * scale x scale block of the frame and the full-resolution image is then
 * sampled through it:
 *   k = scale (1, 2, 4, 8 or 16), c = k / 2 (0 for k = 1);
 *   texel (i, j) takes the depth z of pixel (k i + c, k j + c), each
 *   coordinate clamped to the frame (the last block row and column may be
 *   cut by the frame's edge); q = bf / z with yoro_reproject's skip rule;
 *   it moves to texel column i -+ roundf(q / k) (skipped unless inside the
 *   buffer row, ceil(width / k) texels); the nearest depth wins and the
 *   texel keeps q (full-resolution pixels) and z;
 *   pixel (x, y) reads texel n = its own block's: none reached it -> hole;
 *   else s = q of n, or with linear != 0, when the texels i0 = floor(u) and
 *   i0 + 1 around u = (x - c) / k are both in the row, both reached and
 *   their q differ by at most 1, s = q0 + f (q1 - q0) with f = u - i0;
 *   the source column is x + roundf(s) (TARGET_RIGHT) or x - roundf(s)
 *   (TARGET_LEFT); off the row -> hole; else the pixel takes that source
 *   pixel's RGBA (its own row) and the depth z of texel n, mask 0.
 * All FP32, each operation rounded once.  Holes are then filled per
 * fill_mode exactly as yoro_reproject fills them.  With scale 1 the result
 * is yoro_reproject's, bit for bit, and the call runs yoro_reproject's
 * kernels.  Arguments, ownership, outputs and
 * errors as yoro_reproject; scale outside {1, 2, 4, 8, 16} or linear
 * outside {0, 1} is YORO_ERR_INVALID_ARG.
 */
int32_t yoro_reproject_lowres(const uint8_t* src_rgba, const float* src_depth, int32_t width, int32_t height,
                              float baseline_m, float focal_px, int32_t target_eye, int32_t fill_mode,
                              int32_t scale, int32_t linear, uint8_t* dst_rgba, float* dst_depth,
                              uint8_t* dst_mask, void* hip_stream);

/*
 * yoro_stereo_batch_launch_lowres -- run the jobs that the last prepare on
 * this workspace uploaded, each as yoro_reproject_lowres with the given
 * scale and linear flag, as one persistent kernel.  A workgroup takes
 * scale rows of one block row at a time; scale 1 runs
 * yoro_stereo_batch_launch's kernel.  max_width, total_rows and the error
 * counter as in yoro_stereo_batch_launch (the persistent kernel of scales
 * 2-16 checks total_rows but needs it for no grid).  Capture-safe: no
 * allocation, copy or sync.
 */
int32_t yoro_stereo_batch_launch_lowres(const void* dev_workspace, int32_t max_width, int64_t total_rows,
                                        int32_t scale, int32_t linear, void* hip_stream);

/*
 * yoro_reproject_pose -- warp one frame to an eye at a general pose (Section
 * 6: the rotation matrix of a unit quaternion, the view and projection
 * matrices and the reprojection M = (VP_src)^-1 VP_tgt), for rotated or
 * toed-in eyes and head motion, and fill its disocclusions.
 *
 * Cameras are pinholes: focal_px, principal point (cx, cy), x right, y
 * down, z forward; pixel (x, y) with planar depth z is the point
 * ((x - cx) z / f, (y - cy) z / f, z) of its eye.  rotation (host, 4 floats:
 * r_x the scalar part, then r_y, r_z, r_w, as Equation rmatrix places them;
 * |q| within 1e-4 of 1) and translation (host, 3 floats, metres) are the
 * target eye's orientation and position in the source eye's camera frame,
 * so a point X maps to X_t = R^T (X - t); parallel stereo's right eye is
 * rotation (1, 0, 0, 0), translation (B, 0, 0).  The library forms
 * A = R^T and b = -R^T t in double and rounds them to FP32; then per source
 * pixel, in FP32 with each operation rounded once:
 *   a = (x - cx) / f, c = (y - cy) / f;
 *   finite z > 0: X = a z, Y = c z, X_t = ((A00 X + A01 Y) + A02 z) + b0
 *                 (Y_t, Z_t alike), target depth Z_t;
 *   z = +inf:     X_t = (A00 a + A01 c) + A02 (alike), target depth +inf;
 *   other z:      not splatted;
 *   skipped unless Z_t > 0; xf = f (X_t / Z_t) + cx, yf = f (Y_t / Z_t) + cy;
 *   target (roundf(xf), roundf(yf)), skipped unless inside the frame;
 *   over the whole frame the least (target depth bits << 32 | source index)
 *   wins.
 * Hits take the source pixel's RGBA and the target depth; holes are filled
 * per fill_mode along target rows as yoro_reproject fills them, with the
 * tie side (and the Patcher's orientation) of YORO_TARGET_RIGHT when
 * translation[0] >= 0 and of YORO_TARGET_LEFT otherwise.
 *
 * workspace: device, >= yoro_reproject_pose_workspace_bytes(width, height)
 * (one u64 per pixel), 16-byte aligned, not overlapping any other buffer;
 * overwritten.  Other arguments, ownership, outputs and errors as
 * yoro_reproject.
 */
size_t yoro_reproject_pose_workspace_bytes(int32_t width, int32_t height);
int32_t yoro_reproject_pose(const uint8_t* src_rgba, const float* src_depth, int32_t width, int32_t height,
                            float focal_px, float cx, float cy, const float* rotation, const float* translation,
                            int32_t fill_mode, uint8_t* dst_rgba, float* dst_depth, uint8_t* dst_mask,
                            void* workspace, size_t workspace_bytes, void* hip_stream);

/*
 * yoro_hole_sse -- hole error of a synthesised eye against a reference image
 * (Section 9, PSNR = 10 log10(255^2 / MSE)).  Writes to dev_out[0] the sum
 * of squared R, G, B differences over pixels with mask != 0 (over all
 * pixels if mask is NULL) and to dev_out[1] the number of such pixels; both
 * u64, exact.  dev_out: device, 2 x u64, 8-byte aligned; overwritten.
 */
int32_t yoro_hole_sse(const uint8_t* rgba, const uint8_t* ref_rgba, const uint8_t* mask, int32_t width,
                      int32_t height, uint64_t* dev_out, void* hip_stream);

/* This thread's message for the last non-OK status ("" if none). */
const char* yoro_last_error(void);

/* YORO_VERSION of the built library. */
int32_t yoro_version(void);

#ifdef __cplusplus
}
#endif

#endif /* YORO_H */

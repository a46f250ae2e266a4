/*
 * yoro_serve.h -- a real-time serving loop for many headsets on one GPU.
 *
 * Each headset renders one eye and needs the other at its display rate (the
 * paper targets 90-120 frames per second per eye pair, Sections 1 and 12).
 * Frames arrive on the host clock; the loop launches every frame that has
 * arrived as soon as it may (continuous batching: one persistent batched
 * launch of yoro.h per batch, up to max_batch frames, at most max_in_flight
 * batches queued), and records when each frame's result is final.
 *
 * Optional learned refinement (policy YORO_SERVE_LEARNED): once a batch's
 * warp is seen done, the loop counts each frame's holes per tile on the
 * device (on a stream of its own that the call creates and destroys, so
 * neither the plain stream nor a refinement delays it) and reads the counts
 * back; a frame whose hole fraction is at most
 * learned_max_hole_fraction is refined on the learned stream (in place, on
 * the frame's output) by yoro_model_fill_tiles over its hole tiles, or, with
 * band > 0, by yoro_model_fill_bands over the full-width bands that hold
 * holes; the others keep the plain fill.  A frame whose headset's previous counted frame was above the
 * threshold is released as soon as its warp is done (fallback predicted, no
 * wait for its own count), and while a headset falls back its holes are
 * counted on every 8th frame only, every 64th while its last count was above
 * twice the threshold (holes = -1 in the results of the others).
 * Refinements start at least learned_min_interval_ns apart (a GPU-time
 * budget); a frame that comes sooner, or while a refinement runs, keeps the
 * plain fill (path BUSY) and is released as soon as its warp is done.  One refinement runs at a time; a frame that
 * finds it busy, or whose output set has already been handed to a newer
 * frame of its headset, keeps the plain fill.  A batch that reuses the
 * output set under refinement waits for it on the device.
 *
 * Memory: every buffer is the caller's.  Headsets own a pool of source
 * frames and n_outputs output sets each (outputs are used round-robin); the
 * loop needs a device workspace and a pinned host staging area of the sizes
 * given below.  yoro_serve_admit picks the headsets that fit an HBM budget.
 *
 * Streams: the plain work runs on hip_stream, the refinement on
 * options->learned_stream (both of default priority).  A worker thread of
 * the call enqueues each refinement one layer of the network at a time and
 * keeps at most two layers queued, so a warp that shares a hardware queue
 * with the refinement waits for two layers' kernels at most; the
 * refinement's convolutions run one workgroup per output tile, so a warp on
 * another queue gets compute units within a tile's time.  The call returns
 * when every admitted frame is final; it synchronises both streams at the
 * end.
 */
#ifndef YORO_SERVE_H
#define YORO_SERVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define YORO_SERVE_MAX_OUTPUTS 4

typedef enum yoro_serve_policy { YORO_SERVE_PLAIN = 0, YORO_SERVE_LEARNED = 1 } yoro_serve_policy;
typedef enum yoro_serve_path {
  YORO_PATH_PLAIN = 0,        /* plain nearest-background fill */
  YORO_PATH_LEARNED = 1,      /* refined by the learned filler */
  YORO_PATH_FALLBACK = 2,     /* learned policy, too many holes: plain fill */
  YORO_PATH_BUSY = 3,         /* learned policy, refinement busy: plain fill */
  YORO_PATH_REJECTED = 4      /* headset not admitted: not processed */
} yoro_serve_path;

typedef struct yoro_serve_source {   /* one rendered source-eye frame */
  const uint8_t* rgba;               /* device RGBA8 [h][w][4] */
  const float* depth;                /* device FP32 [h][w] */
} yoro_serve_source;

typedef struct yoro_serve_headset {
  int32_t width, height;
  float baseline_m, focal_px;
  int32_t target_eye;                /* YORO_TARGET_* */
  int32_t first_source, n_sources;   /* its pool: sources[first_source + i] */
  int32_t admitted;                  /* 0: its frames are rejected */
  int32_t n_outputs;                 /* 1..YORO_SERVE_MAX_OUTPUTS */
  uint8_t* dst_rgba[YORO_SERVE_MAX_OUTPUTS];
  float* dst_depth[YORO_SERVE_MAX_OUTPUTS];    /* nullable */
  uint8_t* dst_mask[YORO_SERVE_MAX_OUTPUTS];   /* required by the learned policy */
} yoro_serve_headset;

typedef struct yoro_serve_arrival {  /* sorted by t_ns */
  int64_t t_ns;                      /* since the start of the run */
  int32_t headset;
  int32_t source;                    /* index into the headset's pool */
} yoro_serve_arrival;

typedef struct yoro_serve_options {
  int32_t max_batch;                 /* frames per launch, >= 1 */
  int32_t max_in_flight;             /* batches queued at once, >= 1 */
  int32_t policy;                    /* yoro_serve_policy */
  float learned_max_hole_fraction;   /* refine only at or below this */
  const void* model_weights;         /* yoro_model.h weights (learned policy) */
  void* learned_workspace;           /* tiles: yoro_model_tiles_workspace_bytes(max tiles, chunk, tile,
                                        halo); bands: the largest yoro_model_bands_workspace_bytes(w, h,
                                        band, halo) of the admitted headsets */
  size_t learned_workspace_bytes;
  int32_t tile, halo, chunk;         /* hole-tile inference (yoro_model.h) */
  void* learned_stream;              /* hipStream_t for the refinement */
  int64_t learned_min_interval_ns;   /* refinements start at least this far apart */
  int32_t progressive;               /* learned policy: 0 holds a frame to be refined until the
                                        refinement is done; 1 releases every frame at its warp (plain
                                        fill, done_ns) and refines it afterwards in place, a hole tile
                                        at a time (refined_ns) */
  int32_t band;                      /* learned policy: 0 refines hole tiles; > 0 refines the bands of
                                        `band` full-width rows that hold holes (a multiple of tile,
                                        2 halo <= band; headsets' sizes multiples of 8) */
} yoro_serve_options;

typedef struct yoro_serve_result {   /* one per arrival */
  int64_t launch_ns;                 /* plain batch queued */
  int64_t done_ns;                   /* result final (host observed) */
  int32_t path;                      /* yoro_serve_path */
  int32_t batch_frames;              /* frames in its plain batch */
  int64_t holes;                     /* hole pixels (learned policy), else -1 */
  int64_t refined_ns;                /* progressive: its refinement done (host observed), else -1 */
} yoro_serve_result;

/* Sizes for the largest headset frame max_w x max_h. */
size_t yoro_serve_workspace_bytes(const yoro_serve_options* options, int32_t max_w, int32_t max_h);
size_t yoro_serve_host_bytes(const yoro_serve_options* options, int32_t max_w, int32_t max_h);

/* Admission: headsets in order, each admitted while the running total of
 * bytes[i] stays within budget - reserved; admitted[i] = 1 or 0.  Returns
 * the number admitted (or -1 on a bad argument).  Host only. */
int32_t yoro_serve_admit(const int64_t* bytes, int32_t n, int64_t budget, int64_t reserved, int32_t* admitted);

/* Runs the arrivals in real time.  workspace: device, host_staging: pinned
 * host memory (hipHostMalloc or a pinned torch tensor). */
int32_t yoro_serve_run(const yoro_serve_headset* headsets, int32_t n_headsets, const yoro_serve_source* sources,
                       int32_t n_sources, const yoro_serve_arrival* arrivals, int64_t n_arrivals,
                       const yoro_serve_options* options, void* workspace, size_t workspace_bytes,
                       void* host_staging, size_t host_bytes, void* hip_stream, yoro_serve_result* results);

#ifdef __cplusplus
}
#endif

#endif /* YORO_SERVE_H */

// C-ABI of libyoro.so (declared in include/yoro.h): host-side validation,
// launch geometry, and the batch job table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "yoro.h"
#include "yoro_hybrid.h"
#include "yoro_internal.h"
#include "yoro_model.h"

namespace {

thread_local std::string g_err;

int32_t fail(int32_t status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return status;
}

int32_t ok() { return YORO_OK; }

// Per-device facts, queried once per device.
struct DeviceFacts {
  int cus = 0;
  bool valid = false;
};
std::mutex g_dev_mu;
std::vector<DeviceFacts> g_dev;

bool device_facts(DeviceFacts* out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  std::lock_guard<std::mutex> lk(g_dev_mu);
  if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
  if (!g_dev[dev].valid) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return false;
    g_dev[dev].cus = p.multiProcessorCount;
    g_dev[dev].valid = true;
  }
  *out = g_dev[dev];
  return true;
}

int pick_ppt(int width) { return yoro::ppt_for(width); }

// A = R^T and b = -R^T t for the target eye's pose (q, t) in the source
// eye's frame, R the rotation matrix of the unit quaternion q with q[0] the
// scalar part (Section 6, Equation rmatrix), formed in double and rounded
// to FP32 once.
void pose_affine(const float* q, const float* t, float* A, float* b) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  double R[3][3];
  R[0][0] = 1.0 - 2.0 * y * y - 2.0 * z * z;
  R[0][1] = 2.0 * x * y - 2.0 * w * z;
  R[0][2] = 2.0 * x * z + 2.0 * w * y;
  R[1][0] = 2.0 * x * y + 2.0 * w * z;
  R[1][1] = 1.0 - 2.0 * x * x - 2.0 * z * z;
  R[1][2] = 2.0 * y * z - 2.0 * w * x;
  R[2][0] = 2.0 * x * z - 2.0 * w * y;
  R[2][1] = 2.0 * y * z + 2.0 * w * x;
  R[2][2] = 1.0 - 2.0 * x * x - 2.0 * y * y;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) A[3 * r + c] = (float)R[c][r];
    b[r] = (float)(-((R[0][r] * (double)t[0] + R[1][r] * (double)t[1]) + R[2][r] * (double)t[2]));
  }
}

// log2 of an intermediate-buffer scale of 1, 2, 4, 8 or 16; -1 otherwise.
int scale_log2(int32_t scale) {
  for (int lg = 0; lg <= 4; ++lg)
    if (scale == (1 << lg)) return lg;
  return -1;
}

bool aligned4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

bool known_mode(int32_t m) {
  return m == YORO_FILL_NONE || m == YORO_FILL_NEAREST_BG || m == YORO_FILL_LEARNED || m == YORO_FILL_PATCHER;
}

// The entry points without a model argument cannot run the learned fill.
int32_t reject_learned(int32_t fill_mode, const char* who) {
  if (fill_mode == YORO_FILL_LEARNED)
    return fail(YORO_ERR_UNSUPPORTED, "%s: the learned fill needs a model; use yoro_fill_holes or yoro_stereo_batch",
                who);
  return YORO_OK;
}

struct Range {
  uintptr_t lo, hi;  // [lo, hi)
  bool out;
};

bool overlaps(const Range& a, const Range& b) { return a.lo < b.hi && b.lo < a.hi; }

int32_t check_frame(const void* src_rgba, const void* src_depth, int32_t width, int32_t height, float baseline_m,
                    float focal_px, int32_t target_eye, int32_t fill_mode, const void* dst_rgba,
                    const void* dst_depth, const void* dst_mask, const char* who) {
  if (!src_rgba || !src_depth || !dst_rgba)
    return fail(YORO_ERR_INVALID_ARG, "%s: src_rgba, src_depth and dst_rgba are required", who);
  if (width <= 0 || height <= 0)
    return fail(YORO_ERR_INVALID_ARG, "%s: width %d and height %d must be positive", who, width, height);
  if (width > YORO_MAX_WIDTH || height > YORO_MAX_HEIGHT)
    return fail(YORO_ERR_UNSUPPORTED, "%s: %dx%d exceeds the supported %dx%d", who, width, height, YORO_MAX_WIDTH,
                YORO_MAX_HEIGHT);
  if (!std::isfinite(baseline_m) || !(baseline_m > 0.0f) || !std::isfinite(focal_px) || !(focal_px > 0.0f))
    return fail(YORO_ERR_INVALID_ARG, "%s: baseline %g and focal %g must be finite and positive", who,
                (double)baseline_m, (double)focal_px);
  if (target_eye != YORO_TARGET_RIGHT && target_eye != YORO_TARGET_LEFT)
    return fail(YORO_ERR_INVALID_ARG, "%s: unknown target eye %d", who, target_eye);
  if (!known_mode(fill_mode)) return fail(YORO_ERR_INVALID_ARG, "%s: unknown fill mode %d", who, fill_mode);
  if (!aligned4(src_rgba) || !aligned4(src_depth) || !aligned4(dst_rgba) || (dst_depth && !aligned4(dst_depth)))
    return fail(YORO_ERR_INVALID_ARG, "%s: RGBA and depth pointers must be 4-byte aligned", who);
  const uintptr_t n = (uintptr_t)width * (uintptr_t)height;
  std::vector<Range> r = {{(uintptr_t)src_rgba, (uintptr_t)src_rgba + 4 * n, false},
                          {(uintptr_t)src_depth, (uintptr_t)src_depth + 4 * n, false},
                          {(uintptr_t)dst_rgba, (uintptr_t)dst_rgba + 4 * n, true}};
  if (dst_depth) r.push_back({(uintptr_t)dst_depth, (uintptr_t)dst_depth + 4 * n, true});
  if (dst_mask) r.push_back({(uintptr_t)dst_mask, (uintptr_t)dst_mask + n, true});
  for (size_t i = 0; i < r.size(); ++i)
    for (size_t j = i + 1; j < r.size(); ++j)
      if ((r[i].out || r[j].out) && overlaps(r[i], r[j]))
        return fail(YORO_ERR_INVALID_ARG, "%s: an output buffer overlaps another buffer", who);
  return YORO_OK;
}

// A model for the learned fill of frames up to w x h: weights and workspace
// present and 16-byte aligned, sizes multiples of 8, the workspace large
// enough and clear of every buffer in `frames`.
int32_t check_model(const yoro_model* m, int32_t w, int32_t h, const std::vector<Range>& frames, const char* who) {
  if (!m || !m->weights || !m->workspace)
    return fail(YORO_ERR_INVALID_ARG, "%s: the learned fill needs a model with weights and a workspace", who);
  if ((reinterpret_cast<uintptr_t>(m->weights) & 15u) || (reinterpret_cast<uintptr_t>(m->workspace) & 15u))
    return fail(YORO_ERR_INVALID_ARG, "%s: model weights and workspace must be 16-byte aligned", who);
  if (w % 8 || h % 8)
    return fail(YORO_ERR_UNSUPPORTED, "%s: the learned fill needs width and height multiples of 8 (got %dx%d)", who,
                w, h);
  const size_t need = yoro_model_workspace_bytes(1, h, w);
  if (need == 0) return fail(YORO_ERR_UNSUPPORTED, "%s: frame %dx%d too large for the learned fill", who, w, h);
  if (m->workspace_bytes < need)
    return fail(YORO_ERR_WORKSPACE_TOO_SMALL, "%s: model workspace %zu < %zu bytes", who, m->workspace_bytes, need);
  const Range ws{(uintptr_t)m->workspace, (uintptr_t)m->workspace + m->workspace_bytes, true};
  const Range wt{(uintptr_t)m->weights, (uintptr_t)m->weights + yoro_model_weights_bytes(), false};
  if (overlaps(ws, wt)) return fail(YORO_ERR_INVALID_ARG, "%s: the model workspace overlaps its weights", who);
  for (const Range& r : frames)
    if (r.hi > r.lo && (overlaps(ws, r) || (r.out && overlaps(wt, r))))
      return fail(YORO_ERR_INVALID_ARG, "%s: the model's buffers overlap a frame buffer", who);
  return YORO_OK;
}

yoro::DevJob make_job(const yoro_job& j, uint32_t row_start) {
  yoro::DevJob d;
  d.src_rgba = reinterpret_cast<const uint32_t*>(j.src_rgba);
  d.src_depth = j.src_depth;
  d.dst_rgba = reinterpret_cast<uint32_t*>(j.dst_rgba);
  d.dst_depth = j.dst_depth;
  d.dst_mask = j.dst_mask;
  d.width = j.width;
  d.height = j.height;
  d.baseline_m = j.baseline_m;
  d.focal_px = j.focal_px;
  d.target_eye = j.target_eye;
  d.fill_mode = j.fill_mode;
  d.row_start = row_start;
  d.pad_ = 0;
  return d;
}

// Grid of the single-frame warp: one workgroup per row when the rows fit
// the one-row kernel's resident workgroups (10 % over still pays), else a
// persistent grid.
int warp_grid(int width, int height) {
  DeviceFacts f;
  const long long cus = device_facts(&f) ? f.cus : 256;
  const long long one = cus * yoro::warp_blocks_per_cu(width, yoro::kWarpSingleOneRow);
  if ((long long)height * 10 <= one * 11) return height;
  return (int)std::max<long long>(1, std::min<long long>(height, cus * yoro::warp_blocks_per_cu(width, yoro::kWarpSingle)));
}

int grid_for(int rows, int blocks_per_cu) {
  DeviceFacts f;
  const int cus = device_facts(&f) ? f.cus : 256;
  const long long g = (long long)cus * blocks_per_cu;
  return (int)std::max<long long>(1, std::min<long long>(rows, g));
}

// yoro_stereo_batch_prepare, and the first half of yoro_stereo_batch, which
// alone accepts learned jobs (it has the model).  queue = false only checks.
int32_t prepare_batch(const yoro_job* jobs, int32_t n_jobs, void* dev_workspace, size_t workspace_bytes,
                      void* hip_stream, bool allow_learned, bool queue = true) {
  try {
    if (!jobs || n_jobs <= 0 || n_jobs > YORO_MAX_BATCH_JOBS)
      return fail(YORO_ERR_INVALID_ARG, "yoro_stereo_batch_prepare: need 1..%d jobs", YORO_MAX_BATCH_JOBS);
    if (!dev_workspace || (reinterpret_cast<uintptr_t>(dev_workspace) & 15u))
      return fail(YORO_ERR_INVALID_ARG, "yoro_stereo_batch_prepare: workspace must be non-null and 16-byte aligned");
    if (workspace_bytes < yoro_stereo_batch_workspace_bytes(n_jobs))
      return fail(YORO_ERR_WORKSPACE_TOO_SMALL, "yoro_stereo_batch_prepare: workspace %zu < %zu bytes",
                  workspace_bytes, yoro_stereo_batch_workspace_bytes(n_jobs));
    std::vector<Range> ranges;
    ranges.reserve((size_t)n_jobs * 5);
    uint64_t rows = 0;
    int32_t max_w = 0;
    for (int32_t i = 0; i < n_jobs; ++i) {
      const yoro_job& j = jobs[i];
      char who[64];
      snprintf(who, sizeof(who), "yoro_stereo_batch_prepare: job %d", i);
      int32_t st = check_frame(j.src_rgba, j.src_depth, j.width, j.height, j.baseline_m, j.focal_px, j.target_eye,
                               j.fill_mode, j.dst_rgba, j.dst_depth, j.dst_mask, who);
      if (st != YORO_OK) return st;
      if (j.fill_mode == YORO_FILL_PATCHER)
        return fail(YORO_ERR_UNSUPPORTED, "%s: the Patcher fill reads neighbouring rows; use yoro_reproject", who);
      if (j.fill_mode == YORO_FILL_LEARNED && !allow_learned)
        return fail(YORO_ERR_UNSUPPORTED, "%s: the learned fill needs a model; use yoro_stereo_batch", who);
      const uintptr_t n = (uintptr_t)j.width * (uintptr_t)j.height;
      ranges.push_back({(uintptr_t)j.src_rgba, (uintptr_t)j.src_rgba + 4 * n, false});
      ranges.push_back({(uintptr_t)j.src_depth, (uintptr_t)j.src_depth + 4 * n, false});
      ranges.push_back({(uintptr_t)j.dst_rgba, (uintptr_t)j.dst_rgba + 4 * n, true});
      if (j.dst_depth) ranges.push_back({(uintptr_t)j.dst_depth, (uintptr_t)j.dst_depth + 4 * n, true});
      if (j.dst_mask) ranges.push_back({(uintptr_t)j.dst_mask, (uintptr_t)j.dst_mask + n, true});
      rows += (uint64_t)j.height;
      max_w = std::max(max_w, j.width);
    }
    if (rows > 0xFFFFFFFFull) return fail(YORO_ERR_UNSUPPORTED, "yoro_stereo_batch_prepare: too many rows");
    // No output may overlap anything else: sort by start; an output must not
    // overlap its sorted neighbours' spans (track the furthest end so far).
    std::sort(ranges.begin(), ranges.end(), [](const Range& a, const Range& b) { return a.lo < b.lo; });
    uintptr_t far_hi = 0;
    bool far_out = false;
    for (size_t i = 0; i < ranges.size(); ++i) {
      if (i > 0 && ranges[i].lo < far_hi && (ranges[i].out || far_out))
        return fail(YORO_ERR_INVALID_ARG, "yoro_stereo_batch_prepare: an output buffer overlaps another buffer");
      if (ranges[i].hi > far_hi) {
        far_hi = ranges[i].hi;
        far_out = ranges[i].out;
      } else if (ranges[i].out) {
        far_out = true;
      }
    }
    if (!queue) return ok();
    hipStream_t s = (hipStream_t)hip_stream;
    auto* hdr = reinterpret_cast<yoro::BatchHeader*>(dev_workspace);
    auto* dj = reinterpret_cast<yoro::DevJob*>(hdr + 1);
    yoro::BatchHeader h{};
    h.n_jobs = (uint32_t)n_jobs;
    h.total_rows = (uint32_t)rows;
    h.max_width = (uint32_t)max_w;
    h.errors = 0;
    hipError_t e = hipSuccess;
    uint32_t row = 0;
    for (int32_t first = 0; e == hipSuccess && first < n_jobs; first += yoro::kUploadChunk) {
      yoro::UploadChunk c{};
      c.first = (uint32_t)first;
      c.count = (uint32_t)std::min(yoro::kUploadChunk, n_jobs - first);
      for (uint32_t k = 0; k < c.count; ++k) {
        c.jobs[k] = make_job(jobs[first + k], row);
        row += (uint32_t)jobs[first + k].height;
      }
      e = yoro::launch_upload(c, dj, h, first == 0 ? hdr : nullptr, s);  // the first launch writes the header too
    }
    if (e != hipSuccess)
      return fail(YORO_ERR_DEVICE, "yoro_stereo_batch_prepare: upload failed: %s", hipGetErrorString(e));
    return ok();
  } catch (...) {
    return fail(YORO_ERR_DEVICE, "yoro_stereo_batch_prepare: internal error");
  }
}

int32_t launch_batch(const void* dev_workspace, int32_t max_width, int64_t total_rows, void* hip_stream,
                     const char* who) {
  try {
    if (!dev_workspace) return fail(YORO_ERR_INVALID_ARG, "%s: null workspace", who);
    if (max_width <= 0 || max_width > YORO_MAX_WIDTH)
      return fail(YORO_ERR_INVALID_ARG, "%s: max_width %d out of range", who, max_width);
    if (total_rows <= 0 || total_rows > 0xFFFFFFFFll)
      return fail(YORO_ERR_INVALID_ARG, "%s: total_rows %lld out of range", who, (long long)total_rows);
    const auto* hdr = reinterpret_cast<const yoro::BatchHeader*>(dev_workspace);
    const auto* dj = reinterpret_cast<const yoro::DevJob*>(hdr + 1);
    // The grid covers the rows once.  A batch that fills the resident
    // workgroups several times over takes kBatchRows rows per workgroup (the
    // next row's loads in flight while one finishes).  A small batch's time
    // is the length of its workgroups' row chains: one row per workgroup
    // while the rows fit the one-row kernel's resident workgroups (10 % over
    // still pays: the short second wave costs less than two-row chains), two
    // while they fit twice the multi-row kernel's.  One 1832 x 1920 frame:
    // 21.5 us with three rows per workgroup, 15.4 with one.
    DeviceFacts f;
    const long long cus = device_facts(&f) ? f.cus : 256;
    const long long one = cus * yoro::warp_blocks_per_cu(max_width, yoro::kWarpBatchOneRow);
    const long long multi = cus * yoro::warp_blocks_per_cu(max_width, yoro::kWarpBatch);
    const int rows = total_rows * 10 <= one * 11 ? 1 : (total_rows * 10 <= multi * 22 ? 2 : yoro::kBatchRows);
    hipError_t e = yoro::launch_warp_batch(hdr, dj, max_width, (uint32_t)total_rows, rows, (hipStream_t)hip_stream);
    if (e != hipSuccess)
      return fail(YORO_ERR_DEVICE, "%s: launch failed: %s", who, hipGetErrorString(e));
    return ok();
  } catch (...) {
    return fail(YORO_ERR_DEVICE, "%s: internal error", who);
  }
}

// The job table of yoro_stereo_batch_static: a header and YORO_STATIC_MAX_JOBS
// records in a device array of the library's own.  In host code `scratch`
// names a host-side stand-in, never the device memory: every host use goes
// through the address hipGetSymbolAddress returns for the current device.
constexpr size_t kStaticTableBytes = sizeof(yoro::BatchHeader) + (size_t)YORO_STATIC_MAX_JOBS * sizeof(yoro::DevJob);
static __device__ __align__(256) unsigned char scratch[kStaticTableBytes];

std::mutex g_static_mu;
std::vector<void*> g_static_ptr;  // per device: the device address of scratch

// The device address of this device's table (looked up once per device).
int32_t static_table(void** out, const char* who) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(YORO_ERR_DEVICE, "%s: hipGetDevice failed: %s", who, hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(g_static_mu);
  if ((int)g_static_ptr.size() <= dev) g_static_ptr.resize(dev + 1, nullptr);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(YORO_ERR_DEVICE, "%s: no device address for the job table: %s", who, hipGetErrorString(e));
    g_static_ptr[dev] = p;
  }
  *out = g_static_ptr[dev];
  return YORO_OK;
}

}  // namespace

namespace yoro {
void set_last_error(const char* msg) { g_err = msg; }
}  // namespace yoro

extern "C" {

int32_t yoro_version(void) { return YORO_VERSION; }

const char* yoro_last_error(void) { return g_err.c_str(); }

int32_t yoro_reproject(const uint8_t* src_rgba, const float* src_depth, int32_t width, int32_t height,
                       float baseline_m, float focal_px, int32_t target_eye, int32_t fill_mode, uint8_t* dst_rgba,
                       float* dst_depth, uint8_t* dst_mask, void* hip_stream) {
  try {
    int32_t st = check_frame(src_rgba, src_depth, width, height, baseline_m, focal_px, target_eye, fill_mode,
                             dst_rgba, dst_depth, dst_mask, "yoro_reproject");
    if (st == YORO_OK) st = reject_learned(fill_mode, "yoro_reproject");
    if (st != YORO_OK) return st;
    const bool patcher = fill_mode == YORO_FILL_PATCHER;
    if (patcher && (!dst_depth || !dst_mask))
      return fail(YORO_ERR_INVALID_ARG, "yoro_reproject: the Patcher fill needs dst_depth and dst_mask");
    // The Patcher reads neighbouring rows: warp every row first, then fill.
    yoro_job j{src_rgba, src_depth, dst_rgba, dst_depth, dst_mask, width, height, baseline_m, focal_px,
               target_eye, patcher ? (int32_t)YORO_FILL_NONE : fill_mode};
    const int ppt = pick_ppt(width);
    if (ppt < 0) return fail(YORO_ERR_UNSUPPORTED, "yoro_reproject: width %d too wide", width);
    hipError_t e = yoro::launch_warp_single(make_job(j, 0), ppt, warp_grid(width, height), (hipStream_t)hip_stream);
    if (e == hipSuccess && patcher)
      e = yoro::launch_fill(reinterpret_cast<uint32_t*>(dst_rgba), dst_depth, dst_mask, width, height, target_eye,
                            fill_mode, ppt, grid_for(height, yoro::fill_blocks_per_cu(width, fill_mode)),
                            (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(YORO_ERR_DEVICE, "yoro_reproject: launch failed: %s", hipGetErrorString(e));
    return ok();
  } catch (...) {
    return fail(YORO_ERR_DEVICE, "yoro_reproject: internal error");
  }
}

int32_t yoro_reproject_lowres(const uint8_t* src_rgba, const float* src_depth, int32_t width, int32_t height,
                              float baseline_m, float focal_px, int32_t target_eye, int32_t fill_mode,
                              int32_t scale, int32_t linear, uint8_t* dst_rgba, float* dst_depth,
                              uint8_t* dst_mask, void* hip_stream) {
  try {
    int32_t st = check_frame(src_rgba, src_depth, width, height, baseline_m, focal_px, target_eye, fill_mode,
                             dst_rgba, dst_depth, dst_mask, "yoro_reproject_lowres");
    if (st == YORO_OK) st = reject_learned(fill_mode, "yoro_reproject_lowres");
    if (st != YORO_OK) return st;
    const int lg = scale_log2(scale);
    if (lg < 0) return fail(YORO_ERR_INVALID_ARG, "yoro_reproject_lowres: scale %d is not 1, 2, 4, 8 or 16", scale);
    if (linear != 0 && linear != 1)
      return fail(YORO_ERR_INVALID_ARG, "yoro_reproject_lowres: linear must be 0 or 1, got %d", linear);
    const bool patcher = fill_mode == YORO_FILL_PATCHER;
    if (patcher && (!dst_depth || !dst_mask))
      return fail(YORO_ERR_INVALID_ARG, "yoro_reproject_lowres: the Patcher fill needs dst_depth and dst_mask");
    const int ppt = pick_ppt(width);
    if (ppt < 0) return fail(YORO_ERR_UNSUPPORTED, "yoro_reproject_lowres: width %d too wide", width);
    yoro_job j{src_rgba, src_depth, dst_rgba, dst_depth, dst_mask, width, height, baseline_m, focal_px,
               target_eye, patcher ? (int32_t)YORO_FILL_NONE : fill_mode};
    if (lg == 0) {
      // One texel per pixel samples its own shift: the direct path, with or
      // without interpolation (the shift is read at the texel itself).
      hipError_t e = yoro::launch_warp_single(make_job(j, 0), ppt, warp_grid(width, height), (hipStream_t)hip_stream);
      if (e == hipSuccess && patcher)
        e = yoro::launch_fill(reinterpret_cast<uint32_t*>(dst_rgba), dst_depth, dst_mask, width, height, target_eye,
                              fill_mode, ppt, grid_for(height, yoro::fill_blocks_per_cu(width, fill_mode)),
                              (hipStream_t)hip_stream);
      if (e != hipSuccess)
        return fail(YORO_ERR_DEVICE, "yoro_reproject_lowres: launch failed: %s", hipGetErrorString(e));
      return ok();
    }
    const yoro::DevJob dj = make_job(j, 0);
    // Units of G rows: as many rows per unit as still leave two units per
    // resident workgroup.
    DeviceFacts f;
    const int cus = device_facts(&f) ? f.cus : 256;
    const long long full = (long long)cus * yoro::lowres_blocks_per_cu(width, lg, false);
    const long long blocks = ((long long)height + (1 << lg) - 1) >> lg;
    int glg = lg;
    while (glg > 0 && blocks * (1ll << (lg - glg)) < 2 * full) --glg;
    const long long units = blocks << (lg - glg);
    const int grid = (int)std::max<long long>(1, std::min(units, full));
    hipError_t e = yoro::launch_lowres(&dj, nullptr, nullptr, width, lg, glg, linear, grid, (hipStream_t)hip_stream);
    if (e == hipSuccess && patcher)
      e = yoro::launch_fill(reinterpret_cast<uint32_t*>(dst_rgba), dst_depth, dst_mask, width, height, target_eye,
                            fill_mode, ppt, grid_for(height, yoro::fill_blocks_per_cu(width, fill_mode)),
                            (hipStream_t)hip_stream);
    if (e != hipSuccess)
      return fail(YORO_ERR_DEVICE, "yoro_reproject_lowres: launch failed: %s", hipGetErrorString(e));
    return ok();
  } catch (...) {
    return fail(YORO_ERR_DEVICE, "yoro_reproject_lowres: internal error");
  }
}

size_t yoro_reproject_pose_workspace_bytes(int32_t width, int32_t height) {
  if (width <= 0 || height <= 0 || width > YORO_MAX_WIDTH || height > YORO_MAX_HEIGHT) return 0;
  return (size_t)width * (size_t)height * sizeof(uint64_t);
}

int32_t yoro_reproject_pose(const uint8_t* src_rgba, const float* src_depth, int32_t width, int32_t height,
                            float focal_px, float cx, float cy, const float* rotation, const float* translation,
                            int32_t fill_mode, uint8_t* dst_rgba, float* dst_depth, uint8_t* dst_mask,
                            void* workspace, size_t workspace_bytes, void* hip_stream) {
  try {
    const char* who = "yoro_reproject_pose";
    // The frame checks of yoro_reproject (baseline and eye do not apply here).
    int32_t st = check_frame(src_rgba, src_depth, width, height, 1.0f, focal_px, YORO_TARGET_RIGHT, fill_mode,
                             dst_rgba, dst_depth, dst_mask, who);
    if (st == YORO_OK) st = reject_learned(fill_mode, who);
    if (st != YORO_OK) return st;
    if (!std::isfinite(cx) || !std::isfinite(cy))
      return fail(YORO_ERR_INVALID_ARG, "%s: principal point (%g, %g) must be finite", who, (double)cx, (double)cy);
    if (!rotation || !translation) return fail(YORO_ERR_INVALID_ARG, "%s: rotation and translation are required", who);
    double n2 = 0.0;
    for (int i = 0; i < 4; ++i) {
      if (!std::isfinite(rotation[i])) return fail(YORO_ERR_INVALID_ARG, "%s: rotation must be finite", who);
      n2 += (double)rotation[i] * (double)rotation[i];
    }
    if (std::fabs(n2 - 1.0) > 1e-4)
      return fail(YORO_ERR_INVALID_ARG, "%s: rotation must be a unit quaternion (|q|^2 = %g)", who, n2);
    for (int i = 0; i < 3; ++i)
      if (!std::isfinite(translation[i])) return fail(YORO_ERR_INVALID_ARG, "%s: translation must be finite", who);
    const size_t need = yoro_reproject_pose_workspace_bytes(width, height);
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 15u))
      return fail(YORO_ERR_INVALID_ARG, "%s: workspace must be non-null and 16-byte aligned", who);
    if (workspace_bytes < need)
      return fail(YORO_ERR_WORKSPACE_TOO_SMALL, "%s: workspace %zu < %zu bytes", who, workspace_bytes, need);
    const uintptr_t n = (uintptr_t)width * (uintptr_t)height;
    const Range ws{(uintptr_t)workspace, (uintptr_t)workspace + need, true};
    const Range others[] = {{(uintptr_t)src_rgba, (uintptr_t)src_rgba + 4 * n, false},
                            {(uintptr_t)src_depth, (uintptr_t)src_depth + 4 * n, false},
                            {(uintptr_t)dst_rgba, (uintptr_t)dst_rgba + 4 * n, true},
                            {(uintptr_t)dst_depth, dst_depth ? (uintptr_t)dst_depth + 4 * n : 0, true},
                            {(uintptr_t)dst_mask, dst_mask ? (uintptr_t)dst_mask + n : 0, true}};
    for (const Range& r : others)
      if (r.hi > r.lo && overlaps(ws, r)) return fail(YORO_ERR_INVALID_ARG, "%s: the workspace overlaps a buffer", who);
    const bool patcher = fill_mode == YORO_FILL_PATCHER;
    if (patcher && (!dst_depth || !dst_mask))
      return fail(YORO_ERR_INVALID_ARG, "%s: the Patcher fill needs dst_depth and dst_mask", who);
    yoro::PoseGeom g{};
    pose_affine(rotation, translation, g.A, g.b);
    g.f = focal_px;
    g.cx = cx;
    g.cy = cy;
    g.width = width;
    g.height = height;
    // The fill's tie side (and the Patcher's orientation) follows the
    // translation: the side opposite a shift to the right is the right.
    const int32_t eye = translation[0] >= 0.0f ? YORO_TARGET_RIGHT : YORO_TARGET_LEFT;
    DeviceFacts f;
    const int cus = device_facts(&f) ? f.cus : 256;
    hipError_t e = yoro::launch_pose(reinterpret_cast<const uint32_t*>(src_rgba), src_depth, g,
                                     patcher ? (int)YORO_FILL_NONE : fill_mode, eye == YORO_TARGET_RIGHT ? 1 : 0,
                                     reinterpret_cast<uint32_t*>(dst_rgba), dst_depth, dst_mask,
                                     reinterpret_cast<uint64_t*>(workspace), cus, (hipStream_t)hip_stream);
    if (e == hipSuccess && patcher)
      e = yoro::launch_fill(reinterpret_cast<uint32_t*>(dst_rgba), dst_depth, dst_mask, width, height, eye, fill_mode,
                            pick_ppt(width), grid_for(height, yoro::fill_blocks_per_cu(width, fill_mode)),
                            (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(YORO_ERR_DEVICE, "%s: launch failed: %s", who, hipGetErrorString(e));
    return ok();
  } catch (...) {
    return fail(YORO_ERR_DEVICE, "yoro_reproject_pose: internal error");
  }
}

int32_t yoro_reproject_hybrid(const uint8_t* src_rgba, const float* src_depth, int32_t width, int32_t height,
                              float baseline_m, float focal_px, int32_t target_eye, int32_t fill_mode, float near_m,
                              const uint8_t* near_rgba, const float* near_depth, uint8_t* dst_rgba, float* dst_depth,
                              uint8_t* dst_mask, void* hip_stream) {
  const char* who = "yoro_reproject_hybrid";
  try {
    int32_t st = check_frame(src_rgba, src_depth, width, height, baseline_m, focal_px, target_eye, fill_mode,
                             dst_rgba, dst_depth, dst_mask, who);
    if (st == YORO_OK) st = reject_learned(fill_mode, who);
    if (st != YORO_OK) return st;
    if (!std::isfinite(near_m) || !(near_m > 0.0f))
      return fail(YORO_ERR_INVALID_ARG, "%s: near_m %g must be finite and positive", who, (double)near_m);
    if (!near_rgba || !near_depth || !aligned4(near_rgba) || !aligned4(near_depth))
      return fail(YORO_ERR_INVALID_ARG, "%s: near_rgba and near_depth are required, 4-byte aligned", who);
    const uintptr_t n = (uintptr_t)width * (uintptr_t)height;
    const Range ins[] = {{(uintptr_t)near_rgba, (uintptr_t)near_rgba + 4 * n, false},
                         {(uintptr_t)near_depth, (uintptr_t)near_depth + 4 * n, false}};
    const Range outs[] = {{(uintptr_t)dst_rgba, (uintptr_t)dst_rgba + 4 * n, true},
                          {(uintptr_t)dst_depth, dst_depth ? (uintptr_t)dst_depth + 4 * n : 0, true},
                          {(uintptr_t)dst_mask, dst_mask ? (uintptr_t)dst_mask + n : 0, true}};
    for (const Range& a : ins)
      for (const Range& b : outs)
        if (b.hi > b.lo && overlaps(a, b)) return fail(YORO_ERR_INVALID_ARG, "%s: an output overlaps the near layer", who);
    const bool patcher = fill_mode == YORO_FILL_PATCHER;
    if (patcher && (!dst_depth || !dst_mask))
      return fail(YORO_ERR_INVALID_ARG, "%s: the Patcher fill needs dst_depth and dst_mask", who);
    const int ppt = pick_ppt(width);
    if (ppt < 0) return fail(YORO_ERR_UNSUPPORTED, "%s: width %d too wide", who, width);
    // The far field: warped (near pixels skipped) and filled; the Patcher
    // reads neighbouring rows, so it runs after every row is warped; the
    // near layer goes over the finished far field.
    yoro_job j{src_rgba, src_depth, dst_rgba, dst_depth, dst_mask, width, height, baseline_m, focal_px,
               target_eye, patcher ? (int32_t)YORO_FILL_NONE : fill_mode};
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = yoro::launch_warp_single(make_job(j, 0), ppt, warp_grid(width, height), s, true, near_m);
    if (e == hipSuccess && patcher)
      e = yoro::launch_fill(reinterpret_cast<uint32_t*>(dst_rgba), dst_depth, dst_mask, width, height, target_eye,
                            fill_mode, ppt, grid_for(height, yoro::fill_blocks_per_cu(width, fill_mode)), s);
    if (e == hipSuccess) {
      DeviceFacts f;
      const int cus = device_facts(&f) ? f.cus : 256;
      const int64_t want = ((int64_t)n + 255) / 256;
      const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)cus * 8));
      e = yoro::launch_composite_near(reinterpret_cast<const uint32_t*>(near_rgba), near_depth, near_m, (int64_t)n,
                                      reinterpret_cast<uint32_t*>(dst_rgba), dst_depth, dst_mask, grid, s);
    }
    if (e != hipSuccess) return fail(YORO_ERR_DEVICE, "%s: launch failed: %s", who, hipGetErrorString(e));
    return ok();
  } catch (...) {
    return fail(YORO_ERR_DEVICE, "%s: internal error", who);
  }
}

int32_t yoro_render_near(const yoro_object* objects, int32_t n, int32_t width, int32_t height, int32_t x_off,
                         int32_t y_off, double focal_px, double cx, double cy, double eye_x, float near_m,
                         uint8_t* rgba, float* depth, void* hip_stream) {
  const char* who = "yoro_render_near";
  try {
    if (!rgba || !depth || (n > 0 && !objects))
      return fail(YORO_ERR_INVALID_ARG, "%s: rgba, depth and (for n > 0) objects are required", who);
    if (n < 0 || n > 65536) return fail(YORO_ERR_INVALID_ARG, "%s: n %d out of range", who, n);
    if (width <= 0 || height <= 0 || width > YORO_MAX_WIDTH || height > YORO_MAX_HEIGHT)
      return fail(YORO_ERR_INVALID_ARG, "%s: bad size %dx%d", who, width, height);
    if (!std::isfinite(focal_px) || !(focal_px > 0.0) || !std::isfinite(cx) || !std::isfinite(cy) ||
        !std::isfinite(eye_x))
      return fail(YORO_ERR_INVALID_ARG, "%s: camera parameters must be finite (focal > 0)", who);
    if (std::isnan(near_m) || !(near_m > 0.0f)) return fail(YORO_ERR_INVALID_ARG, "%s: near_m must be > 0", who);
    if (!aligned4(rgba) || !aligned4(depth) || (objects && (reinterpret_cast<uintptr_t>(objects) & 7u)))
      return fail(YORO_ERR_INVALID_ARG, "%s: misaligned pointer", who);
    const uintptr_t np = (uintptr_t)width * (uintptr_t)height;
    const Range a{(uintptr_t)rgba, (uintptr_t)rgba + 4 * np, true}, b{(uintptr_t)depth, (uintptr_t)depth + 4 * np, true};
    const Range o{(uintptr_t)objects, (uintptr_t)objects + sizeof(yoro_object) * (uintptr_t)n, false};
    if (overlaps(a, b) || (n > 0 && (overlaps(a, o) || overlaps(b, o))))
      return fail(YORO_ERR_INVALID_ARG, "%s: buffers overlap", who);
    hipError_t e = yoro::launch_render_near(objects, n, width, height, x_off, y_off, focal_px, cx, cy, eye_x, near_m,
                                            reinterpret_cast<uint32_t*>(rgba), depth, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(YORO_ERR_DEVICE, "%s: launch failed: %s", who, hipGetErrorString(e));
    return ok();
  } catch (...) {
    return fail(YORO_ERR_DEVICE, "%s: internal error", who);
  }
}

int32_t yoro_fill_holes(uint8_t* rgba, float* depth, uint8_t* mask, int32_t width, int32_t height,
                        int32_t target_eye, int32_t fill_mode, const yoro_model* model, void* hip_stream) {
  try {
    if (!rgba || !depth || !mask) return fail(YORO_ERR_INVALID_ARG, "yoro_fill_holes: rgba, depth, mask required");
    if (width <= 0 || height <= 0)
      return fail(YORO_ERR_INVALID_ARG, "yoro_fill_holes: width %d and height %d must be positive", width, height);
    if (width > YORO_MAX_WIDTH || height > YORO_MAX_HEIGHT)
      return fail(YORO_ERR_UNSUPPORTED, "yoro_fill_holes: %dx%d exceeds the supported size", width, height);
    if (target_eye != YORO_TARGET_RIGHT && target_eye != YORO_TARGET_LEFT)
      return fail(YORO_ERR_INVALID_ARG, "yoro_fill_holes: unknown target eye %d", target_eye);
    if (!known_mode(fill_mode)) return fail(YORO_ERR_INVALID_ARG, "yoro_fill_holes: unknown fill mode %d", fill_mode);
    if (!aligned4(rgba) || !aligned4(depth))
      return fail(YORO_ERR_INVALID_ARG, "yoro_fill_holes: rgba and depth must be 4-byte aligned");
    const uintptr_t n = (uintptr_t)width * (uintptr_t)height;
    Range a{(uintptr_t)rgba, (uintptr_t)rgba + 4 * n, true}, b{(uintptr_t)depth, (uintptr_t)depth + 4 * n, true},
        c{(uintptr_t)mask, (uintptr_t)mask + n, true};
    if (overlaps(a, b) || overlaps(a, c) || overlaps(b, c))
      return fail(YORO_ERR_INVALID_ARG, "yoro_fill_holes: buffers overlap");
    const bool learned = fill_mode == YORO_FILL_LEARNED;
    if (learned) {
      const int32_t st = check_model(model, width, height, {a, b, c}, "yoro_fill_holes");
      if (st != YORO_OK) return st;
    }
    if (fill_mode == YORO_FILL_NONE) return ok();
    // The learned fill refines the plain nearest-background fill.
    const int32_t row_mode = learned ? (int32_t)YORO_FILL_NEAREST_BG : fill_mode;
    const int ppt = pick_ppt(width);
    const int grid = grid_for(height, yoro::fill_blocks_per_cu(width, row_mode));
    hipError_t e = yoro::launch_fill(reinterpret_cast<uint32_t*>(rgba), depth, mask, width, height, target_eye,
                                     row_mode, ppt, grid, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(YORO_ERR_DEVICE, "yoro_fill_holes: launch failed: %s", hipGetErrorString(e));
    if (learned)
      return yoro_model_fill(model->weights, rgba, depth, mask, 1, height, width, rgba, model->workspace,
                             model->workspace_bytes, hip_stream);
    return ok();
  } catch (...) {
    return fail(YORO_ERR_DEVICE, "yoro_fill_holes: internal error");
  }
}

size_t yoro_stereo_batch_workspace_bytes(int32_t n_jobs) {
  if (n_jobs <= 0 || n_jobs > YORO_MAX_BATCH_JOBS) return 0;
  return sizeof(yoro::BatchHeader) + (size_t)n_jobs * sizeof(yoro::DevJob);
}

int32_t yoro_stereo_batch_prepare(const yoro_job* jobs, int32_t n_jobs, void* dev_workspace, size_t workspace_bytes,
                                  void* hip_stream) {
  return prepare_batch(jobs, n_jobs, dev_workspace, workspace_bytes, hip_stream, false);
}

int32_t yoro_stereo_batch_launch(const void* dev_workspace, int32_t max_width, int64_t total_rows, void* hip_stream) {
  return launch_batch(dev_workspace, max_width, total_rows, hip_stream, "yoro_stereo_batch_launch");
}

int32_t yoro_stereo_batch_launch_lowres(const void* dev_workspace, int32_t max_width, int64_t total_rows,
                                        int32_t scale, int32_t linear, void* hip_stream) {
  try {
    if (!dev_workspace) return fail(YORO_ERR_INVALID_ARG, "yoro_stereo_batch_launch_lowres: null workspace");
    if (max_width <= 0 || max_width > YORO_MAX_WIDTH)
      return fail(YORO_ERR_INVALID_ARG, "yoro_stereo_batch_launch_lowres: max_width %d out of range", max_width);
    const int lg = scale_log2(scale);
    if (lg < 0)
      return fail(YORO_ERR_INVALID_ARG, "yoro_stereo_batch_launch_lowres: scale %d is not 1, 2, 4, 8 or 16", scale);
    if (linear != 0 && linear != 1)
      return fail(YORO_ERR_INVALID_ARG, "yoro_stereo_batch_launch_lowres: linear must be 0 or 1, got %d", linear);
    if (total_rows <= 0 || total_rows > 0xFFFFFFFFll)
      return fail(YORO_ERR_INVALID_ARG, "yoro_stereo_batch_launch_lowres: total_rows %lld out of range",
                  (long long)total_rows);
    const auto* hdr = reinterpret_cast<const yoro::BatchHeader*>(dev_workspace);
    const auto* dj = reinterpret_cast<const yoro::DevJob*>(hdr + 1);
    DeviceFacts f;
    const int cus = device_facts(&f) ? f.cus : 256;
    if (lg == 0)  // scale 1 is the direct path
      return launch_batch(dev_workspace, max_width, total_rows, hip_stream, "yoro_stereo_batch_launch_lowres");
    const int grid = cus * yoro::lowres_blocks_per_cu(max_width, lg, true);
    hipError_t e = yoro::launch_lowres(nullptr, hdr, dj, max_width, lg, lg, linear, grid, (hipStream_t)hip_stream);
    if (e != hipSuccess)
      return fail(YORO_ERR_DEVICE, "yoro_stereo_batch_launch_lowres: launch failed: %s", hipGetErrorString(e));
    return ok();
  } catch (...) {
    return fail(YORO_ERR_DEVICE, "yoro_stereo_batch_launch_lowres: internal error");
  }
}

int32_t yoro_stereo_batch(const yoro_job* jobs, int32_t n_jobs, void* dev_workspace, size_t workspace_bytes,
                          const yoro_model* model, void* hip_stream) {
  const char* who = "yoro_stereo_batch";
  try {
    // prepare's checks, then the learned jobs', all before anything is
    // queued.
    int32_t st = prepare_batch(jobs, n_jobs, dev_workspace, workspace_bytes, hip_stream, true, false);
    if (st != YORO_OK) return st;
    int32_t max_w = 0, lw = 0, lh = 0;
    int64_t rows = 0;
    bool any_learned = false;
    std::vector<Range> frames;
    frames.push_back({(uintptr_t)dev_workspace, (uintptr_t)dev_workspace + workspace_bytes, true});
    for (int32_t i = 0; i < n_jobs; ++i) {
      const yoro_job& j = jobs[i];
      max_w = std::max(max_w, j.width);
      rows += j.height;
      const uintptr_t n = (uintptr_t)j.width * (uintptr_t)j.height;
      frames.push_back({(uintptr_t)j.src_rgba, (uintptr_t)j.src_rgba + 4 * n, false});
      frames.push_back({(uintptr_t)j.src_depth, (uintptr_t)j.src_depth + 4 * n, false});
      frames.push_back({(uintptr_t)j.dst_rgba, (uintptr_t)j.dst_rgba + 4 * n, true});
      if (j.dst_depth) frames.push_back({(uintptr_t)j.dst_depth, (uintptr_t)j.dst_depth + 4 * n, true});
      if (j.dst_mask) frames.push_back({(uintptr_t)j.dst_mask, (uintptr_t)j.dst_mask + n, true});
      if (j.fill_mode != YORO_FILL_LEARNED) continue;
      if (!j.dst_depth || !j.dst_mask)
        return fail(YORO_ERR_INVALID_ARG, "%s: job %d: the learned fill needs dst_depth and dst_mask", who, i);
      if (j.width % 8 || j.height % 8)
        return fail(YORO_ERR_UNSUPPORTED, "%s: job %d: the learned fill needs width and height multiples of 8", who, i);
      any_learned = true;
      if ((int64_t)j.width * j.height > (int64_t)lw * lh) lw = j.width, lh = j.height;
    }
    if (any_learned) {
      // The workspace must hold the largest learned frame's activations.
      st = check_model(model, lw, lh, frames, who);
      if (st != YORO_OK) return st;
      for (int32_t i = 0; i < n_jobs; ++i)
        if (jobs[i].fill_mode == YORO_FILL_LEARNED &&
            model->workspace_bytes < yoro_model_workspace_bytes(1, jobs[i].height, jobs[i].width))
          return fail(YORO_ERR_WORKSPACE_TOO_SMALL, "%s: job %d: model workspace too small", who, i);
    }
    if (n_jobs == 1) {
      // One frame: the single-frame kernel warps it and writes the batch
      // table itself (one launch instead of an upload and a batch launch);
      // the workspace then holds the same one-job batch as after prepare.
      const hipError_t e = yoro::launch_warp_single(make_job(jobs[0], 0), pick_ppt(jobs[0].width),
                                                    warp_grid(jobs[0].width, jobs[0].height),
                                                    (hipStream_t)hip_stream, false, 0.0f,
                                                    reinterpret_cast<yoro::BatchHeader*>(dev_workspace));
      st = e == hipSuccess ? YORO_OK : fail(YORO_ERR_DEVICE, "%s: launch failed: %s", who, hipGetErrorString(e));
    } else {
      st = prepare_batch(jobs, n_jobs, dev_workspace, workspace_bytes, hip_stream, true);
      if (st == YORO_OK) st = launch_batch(dev_workspace, max_w, rows, hip_stream, who);
    }
    if (st != YORO_OK || !any_learned) return st;
    for (int32_t i = 0; i < n_jobs && st == YORO_OK; ++i) {
      const yoro_job& j = jobs[i];
      if (j.fill_mode != YORO_FILL_LEARNED) continue;
      st = yoro_model_fill(model->weights, j.dst_rgba, j.dst_depth, j.dst_mask, 1, j.height, j.width, j.dst_rgba,
                           model->workspace, model->workspace_bytes, hip_stream);
    }
    return st;
  } catch (...) {
    return fail(YORO_ERR_DEVICE, "%s: internal error", who);
  }
}

int32_t yoro_stereo_batch_static(const yoro_job* jobs, int32_t n_jobs, void* hip_stream) {
  const char* who = "yoro_stereo_batch_static";
  try {
    if (!jobs || n_jobs <= 0 || n_jobs > YORO_STATIC_MAX_JOBS)
      return fail(YORO_ERR_INVALID_ARG, "%s: need 1..%d jobs (the fixed table's size), got %d", who,
                  YORO_STATIC_MAX_JOBS, n_jobs);
    for (int32_t i = 0; i < n_jobs; ++i)
      if (jobs[i].fill_mode == YORO_FILL_LEARNED)
        return fail(YORO_ERR_UNSUPPORTED, "%s: job %d: the learned fill needs a model workspace; use "
                    "yoro_stereo_batch", who, i);
    void* table = nullptr;
    int32_t st = static_table(&table, who);
    if (st != YORO_OK) return st;
    st = prepare_batch(jobs, n_jobs, table, kStaticTableBytes, hip_stream, false);
    if (st != YORO_OK) return st;
    int32_t max_w = 0;
    int64_t rows = 0;
    for (int32_t i = 0; i < n_jobs; ++i) max_w = std::max(max_w, jobs[i].width), rows += jobs[i].height;
    return launch_batch(table, max_w, rows, hip_stream, who);
  } catch (...) {
    return fail(YORO_ERR_DEVICE, "%s: internal error", who);
  }
}

const uint32_t* yoro_stereo_batch_errors(const void* dev_workspace) {
  if (!dev_workspace) return nullptr;
  return &reinterpret_cast<const yoro::BatchHeader*>(dev_workspace)->errors;
}

int32_t yoro_hole_sse(const uint8_t* rgba, const uint8_t* ref_rgba, const uint8_t* mask, int32_t width,
                      int32_t height, uint64_t* dev_out, void* hip_stream) {
  try {
    if (!rgba || !ref_rgba || !dev_out) return fail(YORO_ERR_INVALID_ARG, "yoro_hole_sse: null pointer");
    if (width <= 0 || height <= 0) return fail(YORO_ERR_INVALID_ARG, "yoro_hole_sse: bad size");
    if (!aligned4(rgba) || !aligned4(ref_rgba) || (reinterpret_cast<uintptr_t>(dev_out) & 7u))
      return fail(YORO_ERR_INVALID_ARG, "yoro_hole_sse: misaligned pointer");
    const int64_t n = (int64_t)width * (int64_t)height;
    DeviceFacts f;
    const int cus = device_facts(&f) ? f.cus : 256;
    const int64_t want = (n + yoro::kThreads - 1) / yoro::kThreads;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)cus * 8));
    hipError_t e = yoro::launch_hole_sse(reinterpret_cast<const uint32_t*>(rgba),
                                         reinterpret_cast<const uint32_t*>(ref_rgba), mask, n,
                                         reinterpret_cast<unsigned long long*>(dev_out), grid,
                                         (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(YORO_ERR_DEVICE, "yoro_hole_sse: launch failed: %s", hipGetErrorString(e));
    return ok();
  } catch (...) {
    return fail(YORO_ERR_DEVICE, "yoro_hole_sse: internal error");
  }
}

}  // extern "C"

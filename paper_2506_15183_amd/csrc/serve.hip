// The real-time serving loop of include/yoro_serve.h: continuous batching of
// arriving frames onto the persistent batched warp, completion tracking with
// events, and the optional hole-tile learned refinement with its fallback.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdint>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "yoro.h"
#include "yoro_internal.h"
#include "yoro_model.h"
#include "yoro_serve.h"

namespace {

using Clock = std::chrono::steady_clock;

int32_t serve_fail(int32_t status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  yoro::set_last_error(buf);
  return status;
}

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

int tiles_of(int w, int h, int tile) { return tile > 0 ? ((w + tile - 1) / tile) * ((h + tile - 1) / tile) : 0; }

bool learned(const yoro_serve_options* o) { return o->policy == YORO_SERVE_LEARNED; }

// Device workspace: max_in_flight job-table slots (held until a batch's warp
// is done), then 2 * max_in_flight hole-count slots (held until its counts
// are on the host), then the crop plan.  Host staging: the count slots'
// copies, then the plan.
struct Layout {
  size_t table;   // per-slot job table bytes
  size_t counts;  // per-slot tile counts bytes (device and host)
  int count_slots;
  size_t plan;    // plan bytes (device and host)
  int tiles;      // tiles of the largest frame
};

Layout layout(const yoro_serve_options* o, int max_w, int max_h) {
  Layout L{};
  L.table = up256(yoro_stereo_batch_workspace_bytes(o->max_batch));
  L.tiles = learned(o) ? tiles_of(max_w, max_h, o->tile) : 0;
  L.counts = up256((size_t)o->max_batch * L.tiles * 4);
  L.count_slots = learned(o) ? 2 * o->max_in_flight : 0;
  L.plan = up256((size_t)L.tiles * 16);
  return L;
}

bool options_ok(const yoro_serve_options* o) {
  if (!o || o->max_batch < 1 || o->max_batch > YORO_MAX_BATCH_JOBS || o->max_in_flight < 1 || o->max_in_flight > 64)
    return false;
  if (o->policy != YORO_SERVE_PLAIN && o->policy != YORO_SERVE_LEARNED) return false;
  if (learned(o) && (o->tile <= 0 || o->tile % 8 || o->halo < 0 || o->halo % 8 || o->chunk < 1 ||
                     !o->model_weights || !o->learned_workspace || !o->learned_stream ||
                     !(o->learned_max_hole_fraction >= 0.0f) || o->learned_min_interval_ns < 0 ||
                     (o->progressive != 0 && o->progressive != 1) || o->band < 0 ||
                     (o->band > 0 && (o->band % o->tile || 2 * o->halo > o->band))))
    return false;
  return true;
}

// In-flight plain batch.
struct Batch {
  int slot;             // job-table slot (and its warp event)
  int cslot = -1;       // hole-count slot (and its event), learned policy
  std::vector<int64_t> frames;
  std::vector<char> counted;  // frames whose holes are counted
  bool warped = false;  // its warp event has been seen
  bool counting = false;  // hole counts were queued
};

// While a headset's frames fall back, its hole fraction is re-counted on
// every kRecount-th frame only, every kRecountFar-th while its last count was
// above twice the threshold (a frame that may be refined is always counted).
constexpr int kRecount = 8;
constexpr int kRecountFar = 64;

}  // namespace

// Two-deep pacing of a refinement on its stream: after each layer is
// enqueued, record an event and wait for the one recorded after the layer
// before.  At most two layers of the refinement are queued at a time, and
// the device does not wait for the host between layers.  (An event still
// pending when the pacer is destroyed is released once it completes.)
class Pacer {
 public:
  explicit Pacer(hipStream_t s) : s_(s) {
    for (hipEvent_t& e : ev_)
      if (err_ == hipSuccess) err_ = hipEventCreateWithFlags(&e, hipEventDisableTiming);
  }
  ~Pacer() {
    for (hipEvent_t e : ev_)
      if (e) (void)hipEventDestroy(e);
  }
  hipError_t error() const { return err_; }
  hipError_t operator()() {
    hipError_t r = hipEventRecord(ev_[n_ & 1], s_);
    if (r == hipSuccess && n_ > 0) r = hipEventSynchronize(ev_[(n_ - 1) & 1]);
    ++n_;
    return r;
  }

 private:
  hipStream_t s_;
  hipEvent_t ev_[2] = {nullptr, nullptr};
  hipError_t err_ = hipSuccess;
  int n_ = 0;
};

// Enqueues refinements from a thread of its own: a tile fill is hundreds of
// kernel launches (about a millisecond of host time), during which the
// serving thread keeps taking arrivals and completions.  One job at a time;
// `issued` turns 1 once the job's completion event is recorded (-1 if the
// enqueueing failed, with the message in `err`), and only then may the
// serving thread query or wait on that event.
class Refiner {
 public:
  explicit Refiner(int device) : th_([this, device] { loop(device); }) {}
  ~Refiner() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_one();
    th_.join();  // a job being enqueued is finished first
  }
  void submit(std::function<int32_t(std::string*)> job) {
    issued.store(0, std::memory_order_release);
    {
      std::lock_guard<std::mutex> lk(mu_);
      job_ = std::move(job);
    }
    cv_.notify_one();
  }
  std::atomic<int> issued{1};
  std::string err;  // valid once issued == -1

 private:
  void loop(int device) {
    const hipError_t e = hipSetDevice(device);
    for (;;) {
      std::function<int32_t(std::string*)> job;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [this] { return stop_ || job_; });
        if (!job_) return;  // stop, nothing queued
        job.swap(job_);
      }
      int32_t st = YORO_OK;
      if (e != hipSuccess) {
        err = std::string("refinement thread: ") + hipGetErrorString(e);
        st = YORO_ERR_DEVICE;
      } else {
        st = job(&err);
      }
      issued.store(st == YORO_OK ? 1 : -1, std::memory_order_release);
    }
  }
  std::mutex mu_;
  std::condition_variable cv_;
  bool stop_ = false;
  std::function<int32_t(std::string*)> job_;
  std::thread th_;
};

extern "C" {

size_t yoro_serve_workspace_bytes(const yoro_serve_options* options, int32_t max_w, int32_t max_h) {
  if (!options_ok(options) || max_w <= 0 || max_h <= 0) return 0;
  const Layout L = layout(options, max_w, max_h);
  return L.table * options->max_in_flight + L.counts * L.count_slots + L.plan;
}

size_t yoro_serve_host_bytes(const yoro_serve_options* options, int32_t max_w, int32_t max_h) {
  if (!options_ok(options) || max_w <= 0 || max_h <= 0) return 0;
  const Layout L = layout(options, max_w, max_h);
  return L.counts * L.count_slots + L.plan;
}

int32_t yoro_serve_admit(const int64_t* bytes, int32_t n, int64_t budget, int64_t reserved, int32_t* admitted) {
  if (!bytes || !admitted || n < 0 || budget < 0 || reserved < 0) return -1;
  int64_t left = budget - reserved;
  int32_t count = 0;
  for (int32_t i = 0; i < n; ++i) {
    const bool fits = bytes[i] >= 0 && bytes[i] <= left;
    admitted[i] = fits ? 1 : 0;
    if (fits) {
      left -= bytes[i];
      ++count;
    }
  }
  return count;
}

int32_t yoro_serve_run(const yoro_serve_headset* headsets, int32_t n_headsets, const yoro_serve_source* sources,
                       int32_t n_sources, const yoro_serve_arrival* arrivals, int64_t n_arrivals,
                       const yoro_serve_options* options, void* workspace, size_t workspace_bytes,
                       void* host_staging, size_t host_bytes, void* hip_stream, yoro_serve_result* results) {
  const char* who = "yoro_serve_run";
  if (!headsets || n_headsets <= 0 || !sources || n_sources <= 0 || (!arrivals && n_arrivals) || n_arrivals < 0 ||
      !results || !workspace || !host_staging)
    return serve_fail(YORO_ERR_INVALID_ARG, "%s: null pointer or empty input", who);
  if (!options_ok(options)) return serve_fail(YORO_ERR_INVALID_ARG, "%s: bad options", who);
  const yoro_serve_options& O = *options;
  const bool L_on = learned(&O);
  int max_w = 0, max_h = 0;
  for (int i = 0; i < n_headsets; ++i) {
    const yoro_serve_headset& H = headsets[i];
    if (H.n_sources < 1) return serve_fail(YORO_ERR_INVALID_ARG, "%s: headset %d: empty pool", who, i);
    if (!H.admitted) continue;  // its arrivals are only marked rejected
    if (H.n_outputs < 1 || H.n_outputs > YORO_SERVE_MAX_OUTPUTS || H.first_source < 0 ||
        H.first_source + H.n_sources > n_sources || H.width <= 0 || H.height <= 0)
      return serve_fail(YORO_ERR_INVALID_ARG, "%s: headset %d: bad pool or outputs", who, i);
    for (int o = 0; o < H.n_outputs; ++o)
      if (!H.dst_rgba[o] || (L_on && (!H.dst_mask[o] || !H.dst_depth[o])))
        return serve_fail(YORO_ERR_INVALID_ARG, "%s: headset %d: missing output %d", who, i, o);
    if (L_on) {
      const int crop = O.band > 0 ? 0 : O.tile + 2 * O.halo;
      if (H.width % 8 || H.height % 8 || H.width < crop || H.height < crop)
        return serve_fail(YORO_ERR_INVALID_ARG, "%s: headset %d: %d x %d does not take %d-pixel crops", who, i,
                          H.width, H.height, crop);
    }
    max_w = H.width > max_w ? H.width : max_w;
    max_h = H.height > max_h ? H.height : max_h;
  }
  for (int64_t k = 0; k < n_arrivals; ++k) {
    const yoro_serve_arrival& A = arrivals[k];
    if (A.headset < 0 || A.headset >= n_headsets || A.source < 0 || A.source >= headsets[A.headset].n_sources ||
        (k > 0 && A.t_ns < arrivals[k - 1].t_ns))
      return serve_fail(YORO_ERR_INVALID_ARG, "%s: arrival %lld: bad headset, source or order", who, (long long)k);
  }
  const Layout Lay = layout(&O, max_w, max_h);
  if (workspace_bytes < yoro_serve_workspace_bytes(&O, max_w, max_h) ||
      host_bytes < yoro_serve_host_bytes(&O, max_w, max_h))
    return serve_fail(YORO_ERR_WORKSPACE_TOO_SMALL, "%s: workspace or host staging too small", who);
  size_t l_need = 0;
  if (L_on && O.band > 0) {
    for (int i = 0; i < n_headsets; ++i) {
      if (!headsets[i].admitted) continue;
      const size_t b = yoro_model_bands_workspace_bytes(headsets[i].width, headsets[i].height, O.band, O.halo);
      if (b == 0) return serve_fail(YORO_ERR_INVALID_ARG, "%s: headset %d: too large for bands", who, i);
      l_need = b > l_need ? b : l_need;
    }
  } else if (L_on) {
    l_need = yoro_model_tiles_workspace_bytes(Lay.tiles, O.chunk, O.tile, O.halo);
  }
  if (L_on && O.learned_workspace_bytes < l_need)
    return serve_fail(YORO_ERR_WORKSPACE_TOO_SMALL, "%s: learned workspace too small", who);

  hipStream_t s = (hipStream_t)hip_stream;
  hipStream_t ls = (hipStream_t)O.learned_stream;
  char* ws = static_cast<char*>(workspace);
  char* hs = static_cast<char*>(host_staging);
  char* counts_dev = ws + Lay.table * O.max_in_flight;
  int32_t* plan_dev = reinterpret_cast<int32_t*>(counts_dev + Lay.counts * Lay.count_slots);
  int32_t* plan_host = reinterpret_cast<int32_t*>(hs + Lay.counts * Lay.count_slots);

  // ev: a batch's warp is done; cev: its hole counts are on the host.
  std::vector<hipEvent_t> ev(O.max_in_flight, nullptr), cev(Lay.count_slots, nullptr);
  hipEvent_t lev = nullptr;
  hipError_t he = hipSuccess;
  for (int i = 0; i < O.max_in_flight && he == hipSuccess; ++i) he = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
  for (int i = 0; i < Lay.count_slots && he == hipSuccess; ++i)
    he = hipEventCreateWithFlags(&cev[i], hipEventDisableTiming);
  if (he == hipSuccess) he = hipEventCreateWithFlags(&lev, hipEventDisableTiming);
  // Hole counts get a stream of their own (default priority), so a frame's
  // decision never queues behind a refinement.
  hipStream_t cs = nullptr;
  if (he == hipSuccess && L_on) he = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);

  std::vector<int> next_out(n_headsets, 0);
  // Hole fraction of each headset's latest counted frame (-1: none yet).  A
  // frame whose headset was last above the threshold is released as soon as
  // its warp is done (fallback predicted); the others wait for their counts.
  std::vector<double> last_frac(n_headsets, -1.0);
  std::vector<int> since_count(n_headsets, 0);
  // Last arrival written into each headset's output set: a finished frame is
  // refined only while its output still holds it.
  std::vector<int64_t> last_in(n_headsets * YORO_SERVE_MAX_OUTPUTS, -1);
  std::vector<int> out_of(n_arrivals, 0);
  std::vector<int> free_slots, free_cslots;
  for (int i = O.max_in_flight - 1; i >= 0; --i) free_slots.push_back(i);
  for (int i = Lay.count_slots - 1; i >= 0; --i) free_cslots.push_back(i);
  std::deque<int64_t> pending;
  std::deque<Batch> inflight;
  std::vector<int64_t> in_batch(n_headsets, -1);
  int64_t batch_no = 0;
  std::vector<yoro_job> jobs;
  jobs.reserve(O.max_batch);
  int device = 0;
  (void)hipGetDevice(&device);
  std::unique_ptr<Refiner> refiner;
  if (L_on) refiner.reset(new Refiner(device));
  bool l_active = false;
  int64_t l_frame = -1;
  int64_t l_started = -1;  // start of the last refinement (ns), -1: none yet
  int l_headset = -1, l_out = -1;
  int32_t status = he == hipSuccess ? YORO_OK : serve_fail(YORO_ERR_DEVICE, "%s: event: %s", who, hipGetErrorString(he));

  const Clock::time_point t0 = Clock::now();
  auto now_ns = [&]() { return (int64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count(); };
  int64_t next = 0;

  // Learned stage for frame k whose counts are in counts_host; returns its path.
  auto refine = [&](int64_t k, const uint32_t* counts) -> int32_t {
    const yoro_serve_headset& H = headsets[arrivals[k].headset];
    const int nt = tiles_of(H.width, H.height, O.tile);
    int64_t holes = 0;
    for (int t = 0; t < nt; ++t) holes += counts[t];
    results[k].holes = holes;
    if ((double)holes > (double)O.learned_max_hole_fraction * (double)H.width * H.height) return YORO_PATH_FALLBACK;
    if (holes == 0) return YORO_PATH_LEARNED;  // nothing to refine
    if (l_active || last_in[arrivals[k].headset * YORO_SERVE_MAX_OUTPUTS + out_of[k]] != k) return YORO_PATH_BUSY;
    const int64_t t_start = now_ns();
    if (l_started >= 0 && t_start - l_started < O.learned_min_interval_ns) return YORO_PATH_BUSY;
    const int o = out_of[k];
    if (O.band > 0) {
      // Bands of `band` rows cover whole rows of tiles.
      const int ntx = (H.width + O.tile - 1) / O.tile, per = O.band / O.tile;
      std::vector<uint8_t> flags((H.height + O.band - 1) / O.band, 0);
      for (int t = 0; t < nt; ++t)
        if (counts[t]) flags[(t / ntx) / per] = 1;
      refiner->submit([&O, &H, o, flags, ls, lev](std::string* err) -> int32_t {
        Pacer pace(ls);
        hipError_t e = pace.error();
        if (e != hipSuccess) {
          *err = std::string("pacing event: ") + hipGetErrorString(e);
          return YORO_ERR_DEVICE;
        }
        const int32_t st = yoro::model_fill_bands_paced(
            O.model_weights, H.dst_rgba[o], H.dst_depth[o], H.dst_mask[o], H.width, H.height, O.band, O.halo,
            flags.data(), H.dst_rgba[o], O.learned_workspace, O.learned_workspace_bytes, ls,
            [&pace]() { return pace(); });
        if (st != YORO_OK) {
          *err = std::string("band fill: ") + yoro_last_error();
          return st;
        }
        e = hipEventRecord(lev, ls);
        if (e != hipSuccess) {
          *err = std::string("event record: ") + hipGetErrorString(e);
          return YORO_ERR_DEVICE;
        }
        return YORO_OK;
      });
      l_active = true, l_frame = k, l_headset = arrivals[k].headset, l_out = o;
      l_started = t_start;
      return YORO_PATH_LEARNED;
    }
    const int crop = O.tile + 2 * O.halo, ntx = (H.width + O.tile - 1) / O.tile;
    int kc = 0;
    for (int t = 0; t < nt; ++t) {
      if (!counts[t]) continue;
      const int tx = (t % ntx) * O.tile, ty = (t / ntx) * O.tile;
      int ox = tx - O.halo, oy = ty - O.halo;
      ox = ox < 0 ? 0 : (ox > H.width - crop ? H.width - crop : ox);
      oy = oy < 0 ? 0 : (oy > H.height - crop ? H.height - crop : oy);
      plan_host[4 * kc] = ox, plan_host[4 * kc + 1] = oy, plan_host[4 * kc + 2] = tx, plan_host[4 * kc + 3] = ty;
      ++kc;
    }
    // The plan buffer is not touched again before this refinement completes.
    refiner->submit([&O, &H, o, kc, plan_dev, plan_host, ls, lev](std::string* err) -> int32_t {
      hipError_t e = hipMemcpyAsync(plan_dev, plan_host, (size_t)kc * 16, hipMemcpyHostToDevice, ls);
      if (e != hipSuccess) {
        *err = std::string("plan upload: ") + hipGetErrorString(e);
        return YORO_ERR_DEVICE;
      }
      // Two layers in flight at a time: streams can share a hardware queue,
      // and a warp batch queued behind the refinement then waits for those
      // layers, not for the whole refinement.
      Pacer pace(ls);
      e = pace.error();
      if (e != hipSuccess) {
        *err = std::string("pacing event: ") + hipGetErrorString(e);
        return YORO_ERR_DEVICE;
      }
      const int32_t st = yoro::model_fill_tiles_paced(
          O.model_weights, H.dst_rgba[o], H.dst_depth[o], H.dst_mask[o], H.width, H.height, plan_dev, kc, O.tile,
          O.halo, O.chunk, H.dst_rgba[o], O.learned_workspace, O.learned_workspace_bytes, ls,
          [&pace]() { return pace(); });
      if (st != YORO_OK) {
        *err = std::string("tile fill: ") + yoro_last_error();
        return st;
      }
      e = hipEventRecord(lev, ls);
      if (e != hipSuccess) {
        *err = std::string("event record: ") + hipGetErrorString(e);
        return YORO_ERR_DEVICE;
      }
      return YORO_OK;
    });
    l_active = true, l_frame = k, l_headset = arrivals[k].headset, l_out = o;
    l_started = t_start;
    return YORO_PATH_LEARNED;
  };

  while (status == YORO_OK) {
    // Arrivals that are due.
    const int64_t t = now_ns();
    while (next < n_arrivals && arrivals[next].t_ns <= t) {
      yoro_serve_result& R = results[next];
      R.launch_ns = -1, R.done_ns = -1, R.batch_frames = 0, R.holes = -1, R.refined_ns = -1;
      if (!headsets[arrivals[next].headset].admitted) {
        R.path = YORO_PATH_REJECTED;
      } else {
        R.path = YORO_PATH_PLAIN;
        pending.push_back(next);
      }
      ++next;
    }
    // Warps done (one stream: they finish in order).  A batch's job-table
    // slot is free as soon as its warp is; under the plain policy, and for
    // frames whose headset predicts a fallback, the result is final then.
    for (Batch& B : inflight) {
      if (B.warped) continue;
      const hipError_t q = hipEventQuery(ev[B.slot]);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) {
        status = serve_fail(YORO_ERR_DEVICE, "%s: batch: %s", who, hipGetErrorString(q));
        break;
      }
      const int64_t tn = now_ns();
      B.counted.assign(B.frames.size(), 0);
      for (size_t i = 0; i < B.frames.size(); ++i) {
        const int64_t k = B.frames[i];
        const int h = arrivals[k].headset;
        if (!L_on) {
          results[k].path = YORO_PATH_PLAIN, results[k].done_ns = tn;
        } else if (last_frac[h] > (double)O.learned_max_hole_fraction) {
          results[k].path = YORO_PATH_FALLBACK, results[k].done_ns = tn;
          const int every = last_frac[h] > 2.0 * (double)O.learned_max_hole_fraction ? kRecountFar : kRecount;
          if (++since_count[h] >= every) B.counted[i] = 1, since_count[h] = 0;
        } else if (l_active || (l_started >= 0 && tn - l_started < O.learned_min_interval_ns)) {
          // No refinement could start now: the plain fill is final.
          results[k].path = YORO_PATH_BUSY, results[k].done_ns = tn;
          if (++since_count[h] >= kRecount) B.counted[i] = 1, since_count[h] = 0;
        } else {
          // A candidate for refinement (2): held until then, or, progressive,
          // released now with the plain fill and refined in place later.
          B.counted[i] = 2, since_count[h] = 0;
          if (O.progressive) results[k].path = YORO_PATH_BUSY, results[k].done_ns = tn;
        }
      }
      B.warped = true;
      free_slots.push_back(B.slot);
      bool any = false;
      for (char c : B.counted) any |= c != 0;
      if (L_on && any) {
        // Count the holes (on the count stream) only now that the frames'
        // completion has been taken, so issuing the work delays no one.
        uint32_t* cd = reinterpret_cast<uint32_t*>(counts_dev + Lay.counts * B.cslot);
        hipError_t e = hipSuccess;
        for (size_t i = 0; i < B.frames.size() && e == hipSuccess; ++i) {
          if (!B.counted[i]) continue;
          const int64_t k = B.frames[i];
          const yoro_serve_headset& H = headsets[arrivals[k].headset];
          e = yoro::nn_tile_holes(H.dst_mask[out_of[k]], H.width, H.height, O.tile, cd + i * Lay.tiles, cs);
        }
        if (e == hipSuccess)
          e = hipMemcpyAsync(hs + Lay.counts * B.cslot, cd, B.frames.size() * Lay.tiles * 4, hipMemcpyDeviceToHost,
                             cs);
        if (e == hipSuccess) e = hipEventRecord(cev[B.cslot], cs);
        if (e != hipSuccess) {
          status = serve_fail(YORO_ERR_DEVICE, "%s: hole counts: %s", who, hipGetErrorString(e));
          break;
        }
        B.counting = true;
      }
    }
    // Hole counts on the host (learned stream: in order too).
    while (!inflight.empty() && status == YORO_OK && inflight.front().warped) {
      Batch& B = inflight.front();
      if (L_on && B.counting) {
        const hipError_t q = hipEventQuery(cev[B.cslot]);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) {
          status = serve_fail(YORO_ERR_DEVICE, "%s: hole counts: %s", who, hipGetErrorString(q));
          break;
        }
        const int64_t tn = now_ns();
        const uint32_t* counts = reinterpret_cast<const uint32_t*>(hs + Lay.counts * B.cslot);
        for (size_t i = 0; i < B.frames.size(); ++i) {
          const int64_t k = B.frames[i];
          const yoro_serve_headset& H = headsets[arrivals[k].headset];
          if (!B.counted[i]) continue;
          if (B.counted[i] != 2) {  // a recount of a released frame: keep the statistics only
            int64_t holes = 0;
            for (int t = 0, nt = tiles_of(H.width, H.height, O.tile); t < nt; ++t) holes += counts[i * Lay.tiles + t];
            results[k].holes = holes;
          } else {
            const int32_t p = refine(k, counts + i * Lay.tiles);
            if (p < 0) break;
            results[k].path = p;
            const bool pending_refine = p == YORO_PATH_LEARNED && l_active && l_frame == k;
            if (!O.progressive) {
              if (!pending_refine) results[k].done_ns = tn;
            } else if (p == YORO_PATH_LEARNED && !pending_refine) {
              results[k].refined_ns = tn;  // no holes: nothing to refine
            }
          }
          last_frac[arrivals[k].headset] = (double)results[k].holes / ((double)H.width * H.height);
        }
      }
      if (L_on) free_cslots.push_back(B.cslot);
      inflight.pop_front();
    }
    // The refinement in flight.
    if (l_active && status == YORO_OK) {
      const int is = refiner->issued.load(std::memory_order_acquire);
      if (is < 0) {
        status = serve_fail(YORO_ERR_DEVICE, "%s: refinement: %s", who, refiner->err.c_str());
      } else if (is > 0) {
        const hipError_t q = hipEventQuery(lev);
        if (q == hipSuccess) {
          if (O.progressive)
            results[l_frame].refined_ns = now_ns();
          else
            results[l_frame].done_ns = now_ns();
          l_active = false;
        } else if (q != hipErrorNotReady) {
          status = serve_fail(YORO_ERR_DEVICE, "%s: refinement: %s", who, hipGetErrorString(q));
        }
      }
    }
    // Launch what has arrived.
    while (status == YORO_OK && !pending.empty() && !free_slots.empty() && (!L_on || !free_cslots.empty())) {
      Batch B;
      B.slot = free_slots.back();
      free_slots.pop_back();
      if (L_on) {
        B.cslot = free_cslots.back();
        free_cslots.pop_back();
      }
      jobs.clear();
      bool wait_learned = false;
      // At most one frame per headset per batch (its outputs rotate, so two
      // would collide); the others keep their place in the queue.
      std::deque<int64_t> later;
      while (!pending.empty() && (int)jobs.size() < O.max_batch) {
        const int64_t k = pending.front();
        pending.pop_front();
        const yoro_serve_arrival& A = arrivals[k];
        if (in_batch[A.headset] == batch_no) {
          later.push_back(k);
          continue;
        }
        in_batch[A.headset] = batch_no;
        const yoro_serve_headset& H = headsets[A.headset];
        const yoro_serve_source& S = sources[H.first_source + A.source];
        const int o = next_out[A.headset];
        next_out[A.headset] = (o + 1) % H.n_outputs;
        out_of[k] = o;
        last_in[A.headset * YORO_SERVE_MAX_OUTPUTS + o] = k;
        if (l_active && A.headset == l_headset && o == l_out) wait_learned = true;
        yoro_job j;
        j.src_rgba = S.rgba, j.src_depth = S.depth;
        j.dst_rgba = H.dst_rgba[o], j.dst_depth = H.dst_depth[o], j.dst_mask = H.dst_mask[o];
        j.width = H.width, j.height = H.height, j.baseline_m = H.baseline_m, j.focal_px = H.focal_px;
        j.target_eye = H.target_eye, j.fill_mode = YORO_FILL_NEAREST_BG;
        jobs.push_back(j);
        B.frames.push_back(k);
      }
      while (!later.empty()) {
        pending.push_front(later.back());
        later.pop_back();
      }
      ++batch_no;
      // The event must be recorded before a wait on it means anything.
      while (wait_learned && refiner->issued.load(std::memory_order_acquire) == 0) std::this_thread::yield();
      if (wait_learned && refiner->issued.load(std::memory_order_acquire) < 0) {
        status = serve_fail(YORO_ERR_DEVICE, "%s: refinement: %s", who, refiner->err.c_str());
        break;
      }
      hipError_t e = wait_learned ? hipStreamWaitEvent(s, lev, 0) : hipSuccess;
      if (e != hipSuccess) {
        status = serve_fail(YORO_ERR_DEVICE, "%s: wait: %s", who, hipGetErrorString(e));
        break;
      }
      const int32_t st = yoro_stereo_batch(jobs.data(), (int32_t)jobs.size(), ws + Lay.table * B.slot, Lay.table, nullptr, s);
      if (st != YORO_OK) {
        status = st;
        break;
      }
      e = hipEventRecord(ev[B.slot], s);
      if (e != hipSuccess) {
        status = serve_fail(YORO_ERR_DEVICE, "%s: batch launch: %s", who, hipGetErrorString(e));
        break;
      }
      const int64_t tl = now_ns();
      for (int64_t k : B.frames) results[k].launch_ns = tl, results[k].batch_frames = (int32_t)B.frames.size();
      inflight.push_back(std::move(B));
    }
    if (next == n_arrivals && pending.empty() && inflight.empty() && !l_active) break;
  }
  // Drain whatever is queued (after an error too) before the events go away;
  // the refinement thread first finishes enqueueing its job, if any.
  refiner.reset();
  (void)hipStreamSynchronize(s);
  if (L_on) (void)hipStreamSynchronize(ls);
  if (cs) {
    (void)hipStreamSynchronize(cs);
    (void)hipStreamDestroy(cs);
  }
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : cev)
    if (e) (void)hipEventDestroy(e);
  if (lev) (void)hipEventDestroy(lev);
  return status;
}

}  // extern "C"

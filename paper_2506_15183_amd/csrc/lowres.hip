// Reprojection through a downsampled intermediate buffer (Section 6 (c),
// resolution-independent intermediate buffers; (d), linear interpolation
// along the row), fused with the resolve and the nearest-background fill.
//
// The buffer has one texel per k x k block of the frame (k = 2^lg, 1..16).
// A workgroup (256 threads) takes one unit at a time: G consecutive rows
// (G = 2^glg <= k) of one block row j of one frame.  Per unit:
//   1  scatter texel row j in LDS: texel i takes the depth z of its block's
//      centre pixel (k i + k/2, k j + k/2, clamped to the frame), shifts by
//      dk = roundf(q / k), q = (B f) / z (FP32, the direct path's skip rule
//      q < W), and a 64-bit atomicMin of (z bits << 32 | i) keeps the
//      nearest; each reached texel is then rewritten in place as
//      (q bits << 32 | z bits) -- the buffer records how far its pixel moves;
//   2  every pixel x reads its own block's texel n: a hole there is a hole;
//      otherwise its shift s (or, with interpolation, s0 + f (s1 - s0)
//      between the texels around u = (x - k/2) / k when both are reached and
//      their shifts differ by at most one pixel) names the source column
//      x -+ roundf(s) (a hole if off the row), and the pixel takes the
//      texel's depth;
//   3  the direct path's resolve and fill (row_common.h) over those source
//      columns and depths.  None of this depends on the row within the
//      block, so stages 2 and 3 run once per unit and leave a per-column
//      map (source column, depth, mask) in LDS;
//   4  each row of the unit is then a gather through the map from its own
//      source row, and the stores.
// FP32 in exactly the order above, with the products exact (k is a power of
// two), so the result is bit-exact against the plain definition.
//
// Launch geometry is XCD-aware: gfx950 hands workgroups to its 8 XCDs in
// turn, each with its own L2, so the units of one block row (which share the
// block's centre depth row) are given to workgroups of one XCD.
//
// HBM traffic per pixel: 4 B RGBA gathered + 4/k^2 .. 4/k B of depth (the
// centre row is read in whole cache lines) + 4 B RGBA written (+4 B depth,
// +1 B mask when asked for), against 8 B read by the direct path.
#include "row_common.h"

namespace yoro {
namespace {

// Launch geometry shared by every unit of a launch.
struct LowresGeom {
  int32_t lg;      // k = 1 << lg
  int32_t glg;     // G = 1 << glg rows per unit, glg <= lg
  int32_t linear;  // interpolate the shift along the row
  int32_t wkl;     // texel slots in LDS (>= ceil(max width / k))
  int32_t tko;     // byte offset of the texel slots in LDS (after the row's)
};

// Texel row j of job J into tk[0, wk): after the call (and a barrier) tk[i]
// is kEmpty or (q bits << 32 | z bits) of the texel that reached i.
__device__ __forceinline__ void scatter_texel_row(const DevJob& J, int j, int lg, uint64_t* tk) {
  const int W = J.width, H = J.height;
  const int k = 1 << lg, c = k >> 1;
  const int wk = (W + k - 1) >> lg;
  const float bf = J.baseline_m * J.focal_px;
  const float Wf = (float)W;
  const float invk = 1.0f / (float)k;  // exact
  const int m = J.target_eye == 0 ? -1 : 0;  // it = i -+ dk, as i + ((dk ^ m) - m)
  const int yc = min(j * k + c, H - 1);
  YORO_GLOBAL const float* zp = gmem(J.src_depth) + (size_t)yc * (size_t)W;
  for (int i = threadIdx.x; i < wk; i += kThreads) tk[i] = kEmpty;
  __syncthreads();
  for (int i = threadIdx.x; i < wk; i += kThreads) {
    const float z = zp[min(i * k + c, W - 1)];
    const float q = bf / z;
    const int dk = round_half_away(q * invk);
    const int it = i + ((dk ^ m) - m);
    if ((z > 0.0f) & (q < Wf) & ((unsigned)it < (unsigned)wk))
      atomicMin(&tk[it], ((uint64_t)__float_as_uint(z) << 32) | (uint32_t)i);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < wk; i += kThreads) {
    const uint64_t key = tk[i];
    if ((uint32_t)(key >> 32) != 0xFFFFFFFFu) {
      const uint32_t zb = (uint32_t)(key >> 32);
      const float q = bf / __uint_as_float(zb);  // the winner's own q, recomputed bit for bit
      tk[i] = ((uint64_t)__float_as_uint(q) << 32) | zb;
    }
  }
  __syncthreads();
}

// Stages 2 and 3 for one block row, whose texel row is in tk: every column
// of the block's rows shares its texel, its source column, its depth and so
// its fill choice; only the colours differ from row to row.  So the block's
// map is built once, in place in s.key: column x ends as
//   (depth bits << 32) | (mask << 16) | (source column + 1)
// with source column + 1 = 0 for a pixel that stays empty (RGBA 0).
template <int PPT>
__device__ __forceinline__ void block_map(const DevJob& J, int lg, bool linear, const uint64_t* tk, const RowLds& s) {
  const int W = J.width;
  const int k = 1 << lg, c = k >> 1;
  const int wk = (W + k - 1) >> lg;
  const float invk = 1.0f / (float)k;
  const bool target_right = J.target_eye == 0;
  const int ms = target_right ? 0 : -1;  // xs = x +- r, as x + ((r ^ ms) - ms)

  for_cols<PPT>(W, [&](int, int x) {
    const int t = x - c;
    const int i0 = t >> lg;  // floor((x - c) / k): arithmetic shift
    const int rem = t & (k - 1);
    // The nearest texel n = i0 or i0 + 1, clamped to the row, is one of the
    // two (clamped) neighbours read here.
    const uint64_t k0 = tk[max(i0, 0)], k1 = tk[min(i0 + 1, wk - 1)];
    const uint64_t kn = (2 * rem < k) ? k0 : k1;
    const bool reached = (uint32_t)(kn >> 32) != 0xFFFFFFFFu;
    float sv = __uint_as_float((uint32_t)(kn >> 32));
    if (linear) {
      const float s0 = __uint_as_float((uint32_t)(k0 >> 32));
      const float s1 = __uint_as_float((uint32_t)(k1 >> 32));
      if ((i0 >= 0) & (i0 + 1 < wk) & ((uint32_t)(k0 >> 32) != 0xFFFFFFFFu) &
          ((uint32_t)(k1 >> 32) != 0xFFFFFFFFu) & (fabsf(s1 - s0) <= 1.0f)) {
        const float f = (float)rem * invk;  // exact
        const float dsh = s1 - s0;
        const float mf = f * dsh;
        sv = s0 + mf;
      }
    }
    // A reached texel's shift is in [0, W), where round_half_away is exact.
    const int r = round_half_away(reached ? sv : 0.0f);
    const int xs = x + ((r ^ ms) - ms);
    const bool hit = reached & ((unsigned)xs < (unsigned)W);
    s.key[x] = hit ? (((uint64_t)(uint32_t)kn << 32) | (uint32_t)(xs + 1)) : kEmpty;
  });
  __syncthreads();
  uint64_t* key = s.key;
  resolve_fill_row<PPT>(s, W, target_right, J.fill_mode != 0, [&](int x, uint32_t c1, uint32_t zb, uint8_t mk) {
    key[x] = ((uint64_t)zb << 32) | ((uint32_t)mk << 16) | c1;
  });
  __syncthreads();
}

// The rows [y0, y1) of a block through its map: per pixel one gather from
// its own row and the stores.
template <int PPT>
__device__ __forceinline__ void block_rows(const DevJob& J, int y0, int y1, const RowLds& s) {
  const int W = J.width;
  const int tid = threadIdx.x;
  uint32_t mlo[PPT], mhi[PPT];
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    mlo[i] = 0u;
    mhi[i] = 0u;
  }
  for_cols<PPT>(W, [&](int i, int x) {
    const uint64_t m = s.key[x];
    mlo[i] = (uint32_t)m;
    mhi[i] = (uint32_t)(m >> 32);
  });
  for (int y = y0; y < y1; ++y) {
    const size_t row = (size_t)y * (size_t)W;
    YORO_GLOBAL const uint32_t* src = gmem(J.src_rgba) + row;
    YORO_GLOBAL uint32_t* orow = gmem(J.dst_rgba) + row;
    uint32_t col[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      // An empty pixel loads its own column (clamped into the row) and drops it.
      const int c1 = (int)(mlo[i] & 0xFFFFu);
      col[i] = 0u;
      if (i * kThreads < W) col[i] = src[c1 ? c1 - 1 : min(tid + i * kThreads, W - 1)];
    }
    for_cols<PPT>(W, [&](int i, int x) { orow[x] = (mlo[i] & 0xFFFFu) ? col[i] : 0u; });
    if (J.dst_depth) {
      YORO_GLOBAL float* zrow = gmem(J.dst_depth) + row;
      for_cols<PPT>(W, [&](int i, int x) { zrow[x] = __uint_as_float(mhi[i]); });
    }
    if (J.dst_mask) {
      YORO_GLOBAL uint8_t* mrow = gmem(J.dst_mask) + row;
      for_cols<PPT>(W, [&](int i, int x) { mrow[x] = (uint8_t)(mlo[i] >> 16); });
    }
  }
}

// Units of one launch, walked in the order that keeps a block row's units
// on one XCD: workgroup w belongs to XCD class w % nx (nx = min(8, grid))
// and takes that class's units m = w / nx, w / nx + (workgroups in the
// class), ...; unit m of a class is sub-unit m % U of block row
// (m / U) * nx + class, U = k / G units per block row.  Block rows number
// the jobs' rows in job order, ceil(H / k) per job.  Every workgroup leaves
// its loop once its block row passes the last job.
template <int PPT, bool BATCH>
__device__ __forceinline__ void lowres_units(const DevJob& one, const BatchHeader* hdr, const DevJob* jobs,
                                             const LowresGeom& g, int wl, unsigned char* smem) {
  RowLds s(smem, wl);
  uint64_t* tk = reinterpret_cast<uint64_t*>(smem + g.tko);
  const int grid = (int)gridDim.x, w = (int)blockIdx.x;
  const int nx = min(8, grid);
  const int cls = w % nx;
  const int nslot = (grid - cls + nx - 1) / nx;
  const int k = 1 << g.lg, G = 1 << g.glg;
  const uint32_t U = (uint32_t)(k / G);
  const uint32_t n_jobs = BATCH ? hdr->n_jobs : 1u;
  if (n_jobs == 0) return;
  uint32_t ji = 0, jfirst = 0;  // current job and its first block row
  for (uint32_t m = (uint32_t)(w / nx);; m += (uint32_t)nslot) {
    const uint32_t b = (m / U) * (uint32_t)nx + (uint32_t)cls;
    const uint32_t sub = m % U;
    // Advance to the job holding block row b (block rows only grow).
    bool done = false;
    for (;;) {
      const int H = BATCH ? jobs[ji].height : one.height;
      const uint32_t nb = (uint32_t)((H + k - 1) >> g.lg);
      if (b < jfirst + nb) break;
      jfirst += nb;
      if (++ji >= n_jobs) {
        done = true;
        break;
      }
    }
    if (done) break;
    const DevJob J = BATCH ? jobs[ji] : one;
    const int j = (int)(b - jfirst);
    const int y0 = j * k + (int)sub * G;
    if (y0 >= J.height) continue;  // uniform: a cut last block row
    const int y1 = min(y0 + G, J.height);
    if (J.width > wl || ((J.width + k - 1) >> g.lg) > g.wkl) {
      // Rows wider than the launch's LDS layout are skipped and counted.
      if (BATCH && threadIdx.x == 0) atomicAdd(&const_cast<BatchHeader*>(hdr)->errors, (uint32_t)(y1 - y0));
      continue;
    }
    // Wave priorities: the texel row's loads and scatter first (3), the
    // gathers of the unit's rows next (2), the map's resolve last (1; its
    // fill runs at 0), so a unit's memory requests leave early.
    __builtin_amdgcn_s_setprio(3);
    scatter_texel_row(J, j, g.lg, tk);
    __builtin_amdgcn_s_setprio(1);
    block_map<PPT>(J, g.lg, g.linear != 0, tk, s);
    __builtin_amdgcn_s_setprio(2);
    block_rows<PPT>(J, y0, y1, s);
    __builtin_amdgcn_s_setprio(0);
  }
}

template <int PPT>
__global__ __launch_bounds__(kThreads) void lowres_single_kernel(DevJob J, LowresGeom g, int wl) {
  extern __shared__ __align__(16) unsigned char smem[];
  lowres_units<PPT, false>(J, nullptr, nullptr, g, wl, smem);
}

template <int PPT>
__global__ __launch_bounds__(kThreads) void lowres_batch_kernel(BatchHeader* hdr, const DevJob* __restrict__ jobs,
                                                                LowresGeom g, int wl) {
  extern __shared__ __align__(16) unsigned char smem[];
  lowres_units<PPT, true>(DevJob{}, hdr, jobs, g, wl, smem);
}

hipError_t set_lds_limit(const void* fn, size_t bytes) {
  if (bytes > 65536) return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  return hipSuccess;
}

#define YORO_PPT_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(12) X(16) X(20) X(24) X(28) X(32)

const void* lowres_fn(int ppt, bool batch) {
  switch (ppt) {
#define X(P) \
  case P:    \
    return batch ? (const void*)lowres_batch_kernel<P> : (const void*)lowres_single_kernel<P>;
    YORO_PPT_CASES(X)
#undef X
    default:
      return nullptr;
  }
}

}  // namespace

size_t lowres_lds_bytes(int max_width, int lg) {
  return warp_lds_bytes(lds_width(max_width)) + (size_t)lowres_texel_slots(max_width, lg) * 8;
}

int lowres_blocks_per_cu(int max_width, int lg, bool batch) {
  const void* fn = lowres_fn(ppt_for(max_width), batch);
  if (!fn) return 1;
  const size_t lds = lowres_lds_bytes(max_width, lg);
  (void)set_lds_limit(fn, lds);
  int nb = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kThreads, lds);
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_lowres(const DevJob* one, const BatchHeader* hdr, const DevJob* jobs, int max_width, int lg,
                         int glg, int linear, int grid, hipStream_t stream) {
  const int ppt = ppt_for(max_width);
  const bool batch = one == nullptr;
  const void* fn = lowres_fn(ppt, batch);
  if (!fn || lg < 0 || lg > 4 || glg < 0 || glg > lg || grid <= 0) return hipErrorInvalidValue;
  const int wl = lds_width(max_width);
  const LowresGeom g{lg, glg, linear, lowres_texel_slots(max_width, lg), (int32_t)warp_lds_bytes(wl)};
  const size_t lds = lowres_lds_bytes(max_width, lg);
  hipError_t e = set_lds_limit(fn, lds);
  if (e != hipSuccess) return e;
  switch (ppt) {
#define X(P)                                                                                                      \
  case P:                                                                                                         \
    if (batch)                                                                                                    \
      hipLaunchKernelGGL(lowres_batch_kernel<P>, dim3(grid), dim3(kThreads), lds, stream,                         \
                         const_cast<BatchHeader*>(hdr), jobs, g, wl);                                             \
    else                                                                                                          \
      hipLaunchKernelGGL(lowres_single_kernel<P>, dim3(grid), dim3(kThreads), lds, stream, *one, g, wl);          \
    return hipGetLastError();
    YORO_PPT_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace yoro

// Fused per-row warp + resolve + nearest-background fill for gfx950.
//
// One workgroup (256 threads, 4 wave64s) owns one image row at a time
// (Observation O1, Section 5: the shift is horizontal and one-signed, so
// rows are independent) and strides over the rows of the frame, or of every
// job of a batch, as a persistent grid.
//
// Per row, all in LDS (the row's 64-bit target keys start EMPTY):
//   B  scatter with the depth test (Section 6, reprojection equation and
//      Algorithms 1-2; the lowest depth is kept): per source pixel
//      d = roundf((B*f)/z) in FP32, target column x -+ d, and an LDS
//      atomicMin of (float bits of z) << 32 | source RGBA.  Equal depths in
//      one row have equal disparity and so never meet on one target: the
//      minimum is decided by the depth alone, and the low word simply
//      carries the winner's colour (Algorithm 3's gather of the source
//      colour, done by the scatter itself).  The loads of the workgroup's
//      next row are issued right after the scatter, into the same registers,
//      so they are in flight during C-F;
//   C  per wave64 a ballot of "target reached" gives one 64-bit hit mask per
//      64 columns, and each wave lists its holes;
//   E  each listed hole walks the hit masks from its own word to its
//      nearest hit on either side and takes the farther one (Section 5 O2;
//      Section 7 Patcher figure: on equal depth, the side opposite the
//      shift): the hole's key becomes that hit's key;
//   F  every column is stored from its key (an empty key: RGBA 0, depth
//      +inf), four consecutive columns per lane with one 16-byte
//      non-temporal store, and the keys are cleared for the next row.
// C and E touch only LDS, so each row issues a fixed number of global
// stores, all in F, after the next row's loads: the wait for those loads
// at the next scatter does not have to wait for this row's stores.
//
// The code avoids divergent branches where it can: on CDNA the scalar unit
// issues at the same per-SIMD rate as the vector ALU, so exec-mask juggling
// costs as much as arithmetic.
//
// Wave priorities step through a row: next-row loads 3, scatter 2, C and E
// 1 (the hole walk 0), stores 3.  A workgroup's memory requests get out
// ahead of the phases that wait only on LDS.
//
// HBM traffic per target pixel: 4 B depth + 4 B RGBA read, 4 B RGBA written
// (+4 B depth, +1 B mask when asked for).
#include <atomic>

#include "row_common.h"
#include "yoro.h"

namespace yoro {
namespace {

typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));

// One row's inputs held in registers: thread t owns columns t + i*kThreads.
template <int PPT>
struct RowIn {
  float z[PPT];
  uint32_t c[PPT];
};

// Lanes past the row's end load nothing and keep stale registers: the
// scatter tests x < W in the one ragged chunk.  (Zeroing the registers
// first would make the next row's loads wait for every outstanding store.)
template <int PPT>
__device__ __forceinline__ void load_row(const DevJob& J, int y, RowIn<PPT>& in) {
  const int W = J.width;
  const size_t row = (size_t)y * (size_t)W;
  YORO_GLOBAL const float* zp = gmem(J.src_depth) + row;
  YORO_GLOBAL const uint32_t* cp = gmem(J.src_rgba) + row;
  for_cols<PPT>(W, [&](int i, int x) {
    in.z[i] = __builtin_nontemporal_load(&zp[x]);
    in.c[i] = __builtin_nontemporal_load(&cp[x]);
  });
}

// B: scatter with the depth test into keys that are EMPTY.  Lanes with
// nothing to splat (no geometry, a shift of a full row or more, a target off
// the row, a column past the row's end) hit their own sink slot instead of
// branching.
// NEAR (the near-object hybrid's far field): source pixels nearer than
// near_m take no part.
template <int PPT, bool NEAR = false>
__device__ __forceinline__ void scatter_row(const DevJob& J, const RowIn<PPT>& in, const RowLds& s, int wl,
                                            float near_m = 0.0f) {
  const int W = J.width;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const float bf = J.baseline_m * J.focal_px;
  const uint32_t Wbits = __float_as_uint((float)W);
  // x_t = x - d (target right) or x + d (target left), as x + ((d ^ m) - m).
  const int m = J.target_eye == 0 ? -1 : 0;
  const int nfull = W / kThreads;
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    if (i <= nfull && i * kThreads < W) {
      const int x = tid + i * kThreads;
      const float z = in.z[i];
      const float q = bf / z;
      const int d = round_half_away(q);
      const int xt = x + ((d ^ m) - m);
      // z > 0 and q < W together are q in [+0, W): as bf > 0, any other z
      // (<= 0, NaN) gives a negative, -0, infinite or NaN q, whose bits
      // compare above W's.
      bool ok = (__float_as_uint(q) < Wbits) & ((unsigned)xt < (unsigned)W);
      if (i == nfull) ok &= x < W;
      if (NEAR) ok &= z >= near_m;
      atomicMin(&s.key[ok ? xt : wl + lane], ((uint64_t)__float_as_uint(z) << 32) | in.c[i]);
    }
  }
}

// C and E, in LDS only.  C: per wave64 a ballot of "target reached" (a hit's
// high word holds the bits of a depth in (0, +inf], never the all-ones of
// EMPTY) gives one hit mask per 64 columns; each wave appends its holes to
// its own segment of the hole list.  E (with fill): each listed hole walks
// the hit masks to its nearest hits and its key becomes the chosen hit's
// key.  E reads only hits' keys and writes only holes' keys.
template <int PPT>
__device__ __forceinline__ void mark_and_fill_row(const RowLds& s, int W, bool target_right, bool fill) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int nw = (W + 63) >> 6;
  uint16_t* holes = s.holes + wave * s.seg;  // this wave's segment
  uint32_t run = 0;    // holes listed by this wave so far (wave-uniform)
  uint64_t mword = 0;  // lane i: hit mask of chunk i's 64 columns of this wave
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    if (i * kThreads < W) {
      const int x = tid + i * kThreads;
      const uint64_t k = s.key[min(x, W - 1)];
      const bool inrow = x < W;
      const bool hit = inrow & ((uint32_t)(k >> 32) != 0xFFFFFFFFu);
      const uint64_t hm = __ballot(hit);
      if (fill) {
        const uint64_t om = __ballot(inrow) & ~hm;
        if ((om >> lane) & 1ull) {
          const uint32_t below =
              __builtin_amdgcn_mbcnt_hi((uint32_t)(om >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)om, 0u));
          holes[run + below] = (uint16_t)x;
        }
        run += (uint32_t)__popcll(om);
      }
      // Park this chunk's mask in lane i for one store below.
      mword = (lane == i) ? hm : mword;
    }
  }
  // One LDS store per lane that parked a mask: word (i*4 + wave) holds
  // chunk i's columns of this wave.
  const int nchunks = (W + kThreads - 1) / kThreads;
  const int word = lane * (kThreads / 64) + wave;
  if (lane < nchunks && word < nw) s.mask[word] = mword;
  __syncthreads();
  if (!fill) return;
  __builtin_amdgcn_s_setprio(0);
  for (uint32_t h0 = 0; h0 < run; h0 += 64) {
    const uint32_t h = h0 + lane;
    int x = h < run ? (int)holes[h] : 0;
    const bool act = (h < run) & (x < W);  // every listed column is < W; guard anyway
    x = act ? x : 0;
    int L, R;
    nearest_hits_walk(s.mask, nw, W, x, L, R);
    const uint32_t zl = (uint32_t)(s.key[max(L, 0)] >> 32);
    const uint32_t zr = (uint32_t)(s.key[min(R, W - 1)] >> 32);
    const int p = pick_side(L, R, W, zl, zr, target_right);
    if (act && p >= 0) s.key[x] = s.key[p];
  }
}

// F: store every column from its key and leave the keys EMPTY.  A hit or a
// filled hole carries its key's colour and depth; a key still EMPTY is a
// hole left unfilled: RGBA 0, depth +inf, mask 1 (2 when the fill found no
// hit in the row).  Without depth or mask outputs: four consecutive columns
// per lane, one 16-byte non-temporal store when the row is 16-byte aligned.
template <int PPT, bool EXTRA>
__device__ __forceinline__ void store_row(const DevJob& J, int y, const RowLds& s) {
  const int W = J.width;
  const size_t row = (size_t)y * (size_t)W;
  YORO_GLOBAL uint32_t* orow = gmem(J.dst_rgba) + row;
  if (!EXTRA) {
    constexpr int NF = (PPT + 3) / 4;  // chunks of 4 * kThreads columns
    const bool vec = (reinterpret_cast<uintptr_t>(orow) & 15u) == 0;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int x0 = f * 4 * kThreads + 4 * (int)threadIdx.x;
      if (f * 4 * kThreads < W && x0 < W) {
        // x0 + 3 < W rounded up to 4 <= wl: inside the key row.
        const ulonglong2 k01 = *reinterpret_cast<const ulonglong2*>(&s.key[x0]);
        const ulonglong2 k23 = *reinterpret_cast<const ulonglong2*>(&s.key[x0 + 2]);
        *reinterpret_cast<ulonglong2*>(&s.key[x0]) = make_ulonglong2(kEmpty, kEmpty);
        *reinterpret_cast<ulonglong2*>(&s.key[x0 + 2]) = make_ulonglong2(kEmpty, kEmpty);
        auto col = [](uint64_t k) { return (uint32_t)(k >> 32) == 0xFFFFFFFFu ? 0u : (uint32_t)k; };
        const u32x4v c = u32x4v{col(k01.x), col(k01.y), col(k23.x), col(k23.y)};
        if (vec && x0 + 3 < W) {
          __builtin_nontemporal_store(c, reinterpret_cast<YORO_GLOBAL u32x4v*>(orow + x0));
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (x0 + j < W) orow[x0 + j] = c[j];
        }
      }
    }
    return;
  }
  YORO_GLOBAL float* zrow = J.dst_depth ? gmem(J.dst_depth) + row : nullptr;
  YORO_GLOBAL uint8_t* mrow = J.dst_mask ? gmem(J.dst_mask) + row : nullptr;
  const uint8_t unfilled = J.fill_mode != 0 ? 2 : 1;
  for_cols<PPT>(W, [&](int, int x) {
    const uint64_t k = s.key[x];
    s.key[x] = kEmpty;
    const bool empty = (uint32_t)(k >> 32) == 0xFFFFFFFFu;
    orow[x] = empty ? 0u : (uint32_t)k;
    if (zrow) zrow[x] = __uint_as_float(empty ? kInfBits : (uint32_t)(k >> 32));
    if (mrow) mrow[x] = ((s.mask[x >> 6] >> (x & 63)) & 1ull) ? 0 : (empty ? unfilled : 1);
  });
}

// C, E and F of row y of job J, whose scatter is done (the caller's barrier
// separates them from it).
template <int PPT>
__device__ __forceinline__ void finish_row(const DevJob& J, int y, const RowLds& s) {
  __builtin_amdgcn_s_setprio(1);
  mark_and_fill_row<PPT>(s, J.width, J.target_eye == 0, J.fill_mode != 0);
  __syncthreads();
  __builtin_amdgcn_s_setprio(3);
  if (J.dst_depth || J.dst_mask)
    store_row<PPT, true>(J, y, s);
  else
    store_row<PPT, false>(J, y, s);
}

__device__ __forceinline__ void clear_keys(const RowLds& s, int wl) {
  for (int e = threadIdx.x; e < wl / 2; e += kThreads)
    reinterpret_cast<ulonglong2*>(s.key)[e] = make_ulonglong2(kEmpty, kEmpty);
}

// Waves per SIMD the kernels ask the compiler for, i.e. their VGPR budget.
// The single-frame kernel (persistent, the registers of the prefetched row
// live through C-F): 6, which measured faster than 7 and 5.  The batch
// kernel: 7 (72 VGPRs, no spills), faster than 6.  Both fewer when the LDS
// of the widest row of an instantiation (one workgroup = one wave per SIMD)
// allows fewer, so wide rows get the registers that occupancy leaves free.
constexpr int warp_waves(int ppt, int cap) {
  const int w = kThreads * ppt;
  const int lds = (w + 64) * 8 + (w / 64) * 8 + 16 + w * 2;  // warp_lds_bytes of that width
  const int fit = 160 * 1024 / lds;
  return ppt <= 9 ? cap : (fit < 1 ? 1 : (fit < cap ? fit : cap));
}

// ONE: one row per workgroup (the grid is the frame's height), no next row
// held in registers, 8 waves per SIMD; otherwise a persistent grid.  table:
// null, or a batch workspace that receives this frame as a one-job batch
// (header and job record, written by one thread; no row is ever skipped).
template <int PPT, bool NEAR, bool ONE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(warp_waves(PPT, ONE ? 8 : 6)))) void
warp_single_kernel(DevJob J, int wl, float near_m, BatchHeader* table) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (table && blockIdx.x == 0 && threadIdx.x == 0) {
    BatchHeader h{};
    h.n_jobs = 1;
    h.total_rows = (uint32_t)J.height;
    h.max_width = (uint32_t)J.width;
    *table = h;
    *reinterpret_cast<DevJob*>(table + 1) = J;
  }
  RowLds s(smem, wl);
  clear_keys(s, wl);
  RowIn<PPT> cur;
  int y = blockIdx.x;
  if (y < J.height) load_row<PPT>(J, y, cur);
  __syncthreads();
  for (; y < J.height; y += gridDim.x) {
    // An opaque copy of the width per row keeps the compiler from hoisting
    // every per-chunk predicate out of the loop (they spill otherwise).
    DevJob Jr = J;
    asm volatile("" : "+s"(Jr.width));
    __builtin_amdgcn_s_setprio(2);
    scatter_row<PPT, NEAR>(Jr, cur, s, wl, near_m);
    const int yn = y + gridDim.x;
    __builtin_amdgcn_s_setprio(3);
    if (!ONE && yn < Jr.height) load_row<PPT>(Jr, yn, cur);
    __syncthreads();
    finish_row<PPT>(Jr, y, s);
    if (ONE) break;
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();  // the next row reuses the LDS
  }
}

// The batch kernel covers the batch's flat row space once: workgroup b takes
// the `rows` consecutive rows from b * rows (1 <= rows <= kBatchRows), the
// next row's loads in flight while the current one finishes.  Workgroups
// start in launch order, so the rows in flight stay in one window of memory
// (a persistent grid-stride loop measured 7 % slower: its workgroups drift
// apart).  ONE: the instantiation for one row per workgroup, which holds no
// next row (38 registers instead of 66-72, 8 waves per SIMD).
template <int PPT, bool ONE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(warp_waves(PPT, ONE ? 8 : 7)))) void
warp_batch_kernel(BatchHeader* hdr, const DevJob* __restrict__ jobs, int wl, uint32_t rows_arg) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t rows = ONE ? 1u : rows_arg;
  const uint32_t n = hdr->n_jobs, total = hdr->total_rows;
  const uint64_t first = (uint64_t)blockIdx.x * rows;
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    const uint64_t covered = (uint64_t)gridDim.x * rows;
    if (total > covered) atomicAdd(&hdr->errors, (uint32_t)(total - covered));  // rows the grid does not reach
  }
  if (first >= total) return;  // uniform per workgroup, before any barrier
  uint32_t r = (uint32_t)first;
  const uint32_t rend = total - r < rows ? total : r + rows;
  // The job of row r: the last whose row_start <= r (binary search).
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (jobs[mid].row_start <= r) lo = mid; else hi = mid;
  }
  uint32_t j = lo;
  RowLds s(smem, wl);
  clear_keys(s, wl);
  RowIn<PPT> cur;
  {
    const DevJob J = jobs[j];
    if (J.width <= wl) load_row<PPT>(J, (int)(r - J.row_start), cur);
  }
  __syncthreads();
  for (; r < rend; ++r) {
    const uint32_t rn = r + 1;
    const uint32_t jn = (rn < rend && j + 1 < n && jobs[j + 1].row_start <= rn) ? j + 1 : j;
    {
      const DevJob J = jobs[j];
      if (J.width <= wl) {
        __builtin_amdgcn_s_setprio(2);
        scatter_row<PPT>(J, cur, s, wl);
      } else if (threadIdx.x == 0) {
        atomicAdd(&hdr->errors, 1u);  // rows wider than the LDS layout are skipped
      }
    }
    if (rn < rend) {
      const DevJob Jn = jobs[jn];
      __builtin_amdgcn_s_setprio(3);
      if (Jn.width <= wl) load_row<PPT>(Jn, (int)(rn - Jn.row_start), cur);
    }
    __syncthreads();
    {
      const DevJob J = jobs[j];
      if (J.width <= wl) finish_row<PPT>(J, (int)(r - J.row_start), s);
    }
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();  // the next row reuses the LDS
    j = jn;
  }
}

// ---------------------------------------------------------------------------
// Stand-alone fill of a warped frame, in place.  Hits (mask == 0) are read,
// never written; holes read only hits, so in-place is safe.
template <int PPT>
__global__ __launch_bounds__(kThreads) void fill_kernel(uint32_t* rgba, float* depth, uint8_t* mask, int W, int H,
                                                        int target_eye, int wl) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t* col = reinterpret_cast<uint32_t*>(smem);
  uint32_t* zs = col + wl;  // depth bits
  uint64_t* hm = reinterpret_cast<uint64_t*>(zs + wl);
  const int tid = threadIdx.x;
  const bool target_right = target_eye == 0;
  const int nw = (W + 63) >> 6;
  for (int y = blockIdx.x; y < H; y += gridDim.x) {
    const size_t row = (size_t)y * (size_t)W;
    uint8_t m8[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int x = tid + i * kThreads;
      m8[i] = 1;
      if (x < W) {
        m8[i] = mask[row + x];
        col[x] = rgba[row + x];
        zs[x] = __float_as_uint(depth[row + x]);
      }
    }
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int x = tid + i * kThreads;
      const uint64_t m = __ballot(x < W && m8[i] == 0);
      if ((tid & 63) == 0 && x < W) hm[x >> 6] = m;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int x = tid + i * kThreads;
      if (x < W && m8[i] != 0) {
        int L, R;
        nearest_hits_walk(hm, nw, W, x, L, R);
        const int p = pick_side(L, R, W, L >= 0 ? zs[L] : 0u, R < W ? zs[R] : 0u, target_right);
        rgba[row + x] = p >= 0 ? col[p] : 0u;
        depth[row + x] = p >= 0 ? __uint_as_float(zs[p]) : __builtin_inff();
        mask[row + x] = p >= 0 ? 1 : 2;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Patcher fill of a warped frame, in place (Section 7, Algorithm 3 with the
// weight function of Equation 7).  For a hole at (x, y): the nearest hits L
// and R of its row and the nearest-background edge e among them (as in the
// plain fill), then samples outward from e, away from the hole, over
// n = R - L - 1 columns (the kernel is as wide as the disocclusion) and rows
// y, y - 1, y + 1; a sample counts if it is a hit not nearer than the edge.
// Each counted sample takes
// w = w_rem/2 + 0.3 w_rem t of the remaining weight, t = |x - e| / (R - L - 1)
// the hole's position measured from the edge, and the hole becomes
// rint(sum(C w) / (1 - w_rem)) per channel, with the edge's alpha and depth.
// FP32 in exactly that order (the arithmetic decides 8-bit values).  Row y
// is staged in LDS; rows y +- 1 are read from memory, hits only (a hole's
// mask stays nonzero when it is filled, so in place is safe).  The walk stops
// early at the first counted sample whose weight rounds to exactly zero (the
// remaining weight shrinks by a factor in [0.2, 0.5] per counted sample, down
// through the subnormals, which this code keeps, so this happens within about
// 150 counted samples): a zero weight leaves w_rem unchanged, so every later
// weight is zero as well and adds exactly nothing; the sums and the result
// are those of the full-width walk, bit for bit.

template <int PPT>
__global__ __launch_bounds__(kThreads) void patcher_kernel(uint32_t* rgba, float* depth, uint8_t* mask, int W, int H,
                                                           int target_eye, int wl) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t* col = reinterpret_cast<uint32_t*>(smem);
  uint32_t* zs = col + wl;  // depth bits
  uint64_t* hm = reinterpret_cast<uint64_t*>(zs + wl);
  const int tid = threadIdx.x;
  const bool target_right = target_eye == 0;
  const int nw = (W + 63) >> 6;
  for (int y = blockIdx.x; y < H; y += gridDim.x) {
    const size_t row = (size_t)y * (size_t)W;
    uint8_t m8[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int x = tid + i * kThreads;
      m8[i] = 1;
      if (x < W) {
        m8[i] = mask[row + x];
        col[x] = rgba[row + x];
        zs[x] = __float_as_uint(depth[row + x]);
      }
    }
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int x = tid + i * kThreads;
      const uint64_t m = __ballot(x < W && m8[i] == 0);
      if ((tid & 63) == 0 && x < W) hm[x >> 6] = m;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int x = tid + i * kThreads;
      if (x < W && m8[i] != 0) {
        int L, R;
        nearest_hits_walk(hm, nw, W, x, L, R);
        const int e = pick_side(L, R, W, L >= 0 ? zs[L] : 0u, R < W ? zs[R] : 0u, target_right);
        if (e < 0) {
          rgba[row + x] = 0u;
          depth[row + x] = __builtin_inff();
          mask[row + x] = 2;
          continue;
        }
        const float ze = __uint_as_float(zs[e]);
        const int rz = R - L - 1;
        const float t = (float)abs(x - e) / (float)rz;
        const int dir = e == R ? 1 : -1;
        const int n = rz;
        float w_rem = 1.0f, a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
        bool spent = false;  // a counted sample had weight exactly zero
        for (int k = 0; k < n && !spent; ++k) {
          const int cx = e + dir * k;
          if (cx < 0 || cx >= W) break;
          for (int j = 0; j < 3; ++j) {
            const int cy = y + (j == 0 ? 0 : (j == 1 ? -1 : 1));
            if (cy < 0 || cy >= H) continue;
            uint32_t c;
            float z;
            if (j == 0) {
              if (!((hm[cx >> 6] >> (cx & 63)) & 1ull)) continue;
              c = col[cx];
              z = __uint_as_float(zs[cx]);
            } else {
              const size_t q = (size_t)cy * (size_t)W + (size_t)cx;
              if (mask[q] != 0) continue;
              c = rgba[q];
              z = depth[q];
            }
            if (z < ze) continue;  // foreground
            const float wa = w_rem * 0.5f;
            const float wb = 0.3f * w_rem;
            const float w = wa + wb * t;
            if (w == 0.0f) {
              spent = true;
              break;
            }
            a0 = a0 + (float)(c & 255u) * w;
            a1 = a1 + (float)((c >> 8) & 255u) * w;
            a2 = a2 + (float)((c >> 16) & 255u) * w;
            w_rem = w_rem - w;
          }
        }
        const float norm = 1.0f - w_rem;
        const float v0 = fminf(fmaxf(rintf(a0 / norm), 0.0f), 255.0f);
        const float v1 = fminf(fmaxf(rintf(a1 / norm), 0.0f), 255.0f);
        const float v2 = fminf(fmaxf(rintf(a2 / norm), 0.0f), 255.0f);
        rgba[row + x] = (uint32_t)v0 | ((uint32_t)v1 << 8) | ((uint32_t)v2 << 16) | (col[e] & 0xFF000000u);
        depth[row + x] = ze;
        mask[row + x] = 1;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Hole error: integer sum of squared RGB differences over mask != 0.
__global__ __launch_bounds__(kThreads) void zero2_kernel(unsigned long long* out) {
  if (threadIdx.x < 2) out[threadIdx.x] = 0ull;
}

__global__ __launch_bounds__(kThreads) void hole_sse_kernel(const uint32_t* __restrict__ a,
                                                            const uint32_t* __restrict__ b,
                                                            const uint8_t* __restrict__ mask, int64_t n,
                                                            unsigned long long* out) {
  unsigned long long sse = 0, cnt = 0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    if (mask && mask[i] == 0) continue;
    const uint32_t u = a[i], v = b[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int e = (int)((u >> (8 * c)) & 255u) - (int)((v >> (8 * c)) & 255u);
      sse += (unsigned long long)(e * e);
    }
    cnt += 1;
  }
  // Wave reduction, then one atomic per wave (integer: order does not matter).
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sse += __shfl_down(sse, off);
    cnt += __shfl_down(cnt, off);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&out[0], sse);
    atomicAdd(&out[1], cnt);
  }
}

// ---------------------------------------------------------------------------
// Job records (and, with hdst, the batch header) carried in the kernel
// arguments, written to the device table: a prepare takes one launch per 24
// jobs and no host-to-device copy.
__global__ void upload_kernel(UploadChunk chunk, DevJob* dst, BatchHeader h, BatchHeader* hdst) {
  const uint32_t t = threadIdx.x;
  if (t < chunk.count) dst[chunk.first + t] = chunk.jobs[t];
  if (hdst && t == 0) *hdst = h;
}

// ---------------------------------------------------------------------------
hipError_t set_lds_limit(const void* fn, size_t bytes) {
  if (bytes > 65536) return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  return hipSuccess;
}

#define YORO_PPT_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(12) X(16) X(20) X(24) X(28) X(32)

}  // namespace

hipError_t launch_warp_single(const DevJob& job, int ppt, int grid, hipStream_t stream, bool near, float near_m,
                              BatchHeader* table) {
  const int wl = lds_width(job.width);
  const size_t lds = warp_lds_bytes(wl);
  // A grid of one workgroup per row runs the one-row instantiation.
  const bool one = grid >= job.height;
  switch (ppt) {
#define X(P)                                                                                                 \
  case P: {                                                                                                  \
    const void* k = near ? (one ? (const void*)warp_single_kernel<P, true, true>                             \
                                : (const void*)warp_single_kernel<P, true, false>)                           \
                         : (one ? (const void*)warp_single_kernel<P, false, true>                            \
                                : (const void*)warp_single_kernel<P, false, false>);                         \
    hipError_t e = set_lds_limit(k, lds);                                                                    \
    if (e != hipSuccess) return e;                                                                           \
    if (near && one)                                                                                         \
      hipLaunchKernelGGL((warp_single_kernel<P, true, true>), dim3(job.height), dim3(kThreads), lds, stream, \
                         job, wl, near_m, table);                                                            \
    else if (near)                                                                                           \
      hipLaunchKernelGGL((warp_single_kernel<P, true, false>), dim3(grid), dim3(kThreads), lds, stream, job, \
                         wl, near_m, table);                                                                 \
    else if (one)                                                                                            \
      hipLaunchKernelGGL((warp_single_kernel<P, false, true>), dim3(job.height), dim3(kThreads), lds, stream, \
                         job, wl, 0.0f, table);                                                              \
    else                                                                                                     \
      hipLaunchKernelGGL((warp_single_kernel<P, false, false>), dim3(grid), dim3(kThreads), lds, stream, job, \
                         wl, 0.0f, table);                                                                   \
    return hipGetLastError();                                                                                \
  }
    YORO_PPT_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_warp_batch(const BatchHeader* hdr, const DevJob* jobs, int max_width, uint32_t total_rows, int rows,
                             hipStream_t stream) {
  if (rows < 1 || rows > kBatchRows) return hipErrorInvalidValue;
  const uint64_t groups = ((uint64_t)total_rows + rows - 1) / rows;
  const int grid = (int)(groups > 0 ? groups : 1);
  const int ppt = ppt_for(max_width);
  const int wl = lds_width(max_width);
  const size_t lds = warp_lds_bytes(wl);
  BatchHeader* h = const_cast<BatchHeader*>(hdr);
  switch (ppt) {
#define X(P)                                                                                              \
  case P: {                                                                                               \
    const void* k = rows == 1 ? (const void*)warp_batch_kernel<P, true> : (const void*)warp_batch_kernel<P, false>; \
    hipError_t e = set_lds_limit(k, lds);                                                                 \
    if (e != hipSuccess) return e;                                                                        \
    if (rows == 1)                                                                                        \
      hipLaunchKernelGGL((warp_batch_kernel<P, true>), dim3(grid), dim3(kThreads), lds, stream, h, jobs, wl, 1u); \
    else                                                                                                  \
      hipLaunchKernelGGL((warp_batch_kernel<P, false>), dim3(grid), dim3(kThreads), lds, stream, h, jobs, wl,    \
                         (uint32_t)rows);                                                                 \
    return hipGetLastError();                                                                             \
  }
    YORO_PPT_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_fill(uint32_t* rgba, float* depth, uint8_t* mask, int32_t width, int32_t height, int32_t target_eye,
                       int32_t fill_mode, int ppt, int grid, hipStream_t stream) {
  const int wl = lds_width(width);
  const size_t lds = fill_lds_bytes(wl);
  const bool patcher = fill_mode == kFillPatcher;
  switch (ppt) {
#define X(P)                                                                                                  \
  case P: {                                                                                                   \
    const void* k = patcher ? (const void*)patcher_kernel<P> : (const void*)fill_kernel<P>;                   \
    hipError_t e = set_lds_limit(k, lds);                                                                     \
    if (e != hipSuccess) return e;                                                                            \
    if (patcher)                                                                                              \
      hipLaunchKernelGGL(patcher_kernel<P>, dim3(grid), dim3(kThreads), lds, stream, rgba, depth, mask, width, \
                         height, target_eye, wl);                                                             \
    else                                                                                                      \
      hipLaunchKernelGGL(fill_kernel<P>, dim3(grid), dim3(kThreads), lds, stream, rgba, depth, mask, width,    \
                         height, target_eye, wl);                                                             \
    return hipGetLastError();                                                                                 \
  }
    YORO_PPT_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_hole_sse(const uint32_t* rgba, const uint32_t* ref, const uint8_t* mask, int64_t n,
                           unsigned long long* out, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(zero2_kernel, dim3(1), dim3(kThreads), 0, stream, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(hole_sse_kernel, dim3(grid), dim3(kThreads), 0, stream, rgba, ref, mask, n, out);
  return hipGetLastError();
}

hipError_t launch_upload(const UploadChunk& chunk, DevJob* dst, const BatchHeader& hdr, BatchHeader* hdst,
                         hipStream_t stream) {
  hipLaunchKernelGGL(upload_kernel, dim3(1), dim3(64), 0, stream, chunk, dst, hdr, hdst);
  return hipGetLastError();
}

namespace {
// Resident workgroups per CU of the warp kernels, by kernel and LDS row
// width (a property of the kernel, queried once per combination).
std::atomic<int> g_warp_occupancy[4][YORO_MAX_WIDTH / 64 + 1];
}  // namespace

int warp_blocks_per_cu(int max_width, int kind) {
  const int wl = lds_width(max_width);
  if (wl / 64 > YORO_MAX_WIDTH / 64 || kind < 0 || kind > 3) return 1;
  std::atomic<int>& slot = g_warp_occupancy[kind][wl / 64];
  const int cached = slot.load(std::memory_order_relaxed);
  if (cached > 0) return cached;
  int nb = 0;
  const int ppt = ppt_for(max_width);
  const size_t lds = warp_lds_bytes(lds_width(max_width));
  hipError_t e = hipErrorInvalidValue;
  switch (ppt) {
#define X(P)                                                                                                      \
  case P:                                                                                                         \
    if (kind == kWarpSingle) {                                                                                    \
      (void)set_lds_limit((const void*)warp_single_kernel<P, false, false>, lds);                                  \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, warp_single_kernel<P, false, false>, kThreads, lds);   \
    } else if (kind == kWarpSingleOneRow) {                                                                       \
      (void)set_lds_limit((const void*)warp_single_kernel<P, false, true>, lds);                                   \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, warp_single_kernel<P, false, true>, kThreads, lds);    \
    } else if (kind == kWarpBatch) {                                                                              \
      (void)set_lds_limit((const void*)warp_batch_kernel<P, false>, lds);                                          \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, warp_batch_kernel<P, false>, kThreads, lds);           \
    } else {                                                                                                      \
      (void)set_lds_limit((const void*)warp_batch_kernel<P, true>, lds);                                           \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, warp_batch_kernel<P, true>, kThreads, lds);            \
    }                                                                                                             \
    break;
    YORO_PPT_CASES(X)
#undef X
    default:
      break;
  }
  if (e != hipSuccess || nb <= 0) return 1;
  slot.store(nb, std::memory_order_relaxed);
  return nb;
}

int fill_blocks_per_cu(int width, int fill_mode) {
  int nb = 0;
  const int ppt = ppt_for(width);
  const size_t lds = fill_lds_bytes(lds_width(width));
  const bool patcher = fill_mode == kFillPatcher;
  hipError_t e = hipErrorInvalidValue;
  switch (ppt) {
#define X(P)                                                                                       \
  case P:                                                                                          \
    (void)set_lds_limit(patcher ? (const void*)patcher_kernel<P> : (const void*)fill_kernel<P>, lds); \
    e = patcher ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, patcher_kernel<P>, kThreads, lds)  \
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fill_kernel<P>, kThreads, lds);    \
    break;
    YORO_PPT_CASES(X)
#undef X
    default:
      break;
  }
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

}  // namespace yoro

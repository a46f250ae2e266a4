// Fused per-row warp + resolve + nearest-background fill for gfx950.
//
// One workgroup (256 threads, 4 wave64s) owns one image row at a time
// (Observation O1, Section 5: the shift is horizontal, so rows are
// independent).  A row goes through five phases, all in LDS:
//
//   A  coalesced loads: the row's depth into registers, its RGBA into LDS,
//      and the row's 64-bit target keys set to EMPTY;
//   B  scatter with the depth test (Section 6, Algorithms 1-2; the lowest
//      depth is kept): per source pixel d = roundf((B*f)/z) in FP32,
//      target column x -+ d, and an LDS atomicMin of
//      (float bits of z) << 32 | source column;
//   C  per wave64 a ballot of "target reached" -> one 64-bit mask per 64
//      columns;
//   D  wave 0 scans the masks: for every 64-column word the last hit at or
//      before it and the first hit at or after it;
//   E  resolve (Algorithm 3, non-disocclusion branch: gather the source
//      colour) and, for holes, the nearest hit on each side from the masks
//      plus the word scan, keeping the farther one (Section 5 O2), ties to
//      the side opposite the shift; coalesced stores.
//
// HBM traffic per target pixel: 4 B depth + 4 B RGBA read, 4 B RGBA written
// (+4 B depth, +1 B mask when asked for).  Everything else stays in LDS.
#include "yoro_internal.h"

namespace yoro {
namespace {

constexpr uint64_t kEmpty = ~0ull;
constexpr int kNone = 0x7fffffff;

template <int PPT>
struct RowLds {
  uint64_t* key;   // [wcap]   target keys
  uint32_t* col;   // [wcap]   source RGBA of the row
  uint64_t* mask;  // [words]  hit masks, one per 64 columns
  int32_t* lastc;  // [words]  last hit column in words <= w, or -1
  int32_t* firstc; // [words]  first hit column in words >= w, or kNone
  __device__ explicit RowLds(unsigned char* base) {
    constexpr int wcap = kThreads * PPT;
    constexpr int words = (wcap + 63) / 64;
    key = reinterpret_cast<uint64_t*>(base);
    mask = key + wcap;
    col = reinterpret_cast<uint32_t*>(mask + words);
    lastc = reinterpret_cast<int32_t*>(col + wcap);
    firstc = lastc + words;
  }
};

// Phase D: for every word w < nw, lastc[w] = the largest hit column in words
// 0..w (or -1) and firstc[w] = the smallest hit column in words w..nw-1 (or
// kNone).  Run by wave 0 only; each lane takes a contiguous block of words.
template <int PPT>
__device__ __forceinline__ void scan_words(const uint64_t* mask, int32_t* lastc, int32_t* firstc, int nw) {
  constexpr int kWordsMax = (kThreads * PPT + 63) / 64;
  constexpr int kPer = (kWordsMax + 63) / 64;  // words per lane (1 or 2)
  const int lane = threadIdx.x;
  const int w0 = lane * kPer;
  int fwd[kPer], bwd[kPer];
  int run = -1;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int w = w0 + j;
    int v = -1;
    if (w < nw) {
      const uint64_t m = mask[w];
      if (m) v = w * 64 + 63 - __clzll((long long)m);
    }
    run = max(run, v);
    fwd[j] = run;
  }
  int run_b = kNone;
#pragma unroll
  for (int j = kPer - 1; j >= 0; --j) {
    const int w = w0 + j;
    int v = kNone;
    if (w < nw) {
      const uint64_t m = mask[w];
      if (m) v = w * 64 + __ffsll((long long)m) - 1;
    }
    run_b = min(run_b, v);
    bwd[j] = run_b;
  }
  // Exclusive scans across lanes: max from the left, min from the right.
  int inc = run;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(inc, off);
    if (lane >= off) inc = max(inc, t);
  }
  int exc = __shfl_up(inc, 1);
  if (lane == 0) exc = -1;
  int incb = run_b;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_down(incb, off);
    if (lane + off < 64) incb = min(incb, t);
  }
  int excb = __shfl_down(incb, 1);
  if (lane == 63) excb = kNone;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int w = w0 + j;
    if (w < nw) {
      lastc[w] = max(fwd[j], exc);
      firstc[w] = min(bwd[j], excb);
    }
  }
}

// Nearest hit strictly left (L) and strictly right (R) of column x.
__device__ __forceinline__ void neighbours(const uint64_t* mask, const int32_t* lastc, const int32_t* firstc,
                                           int nw, int x, int& L, int& R) {
  const int w = x >> 6, b = x & 63;
  const uint64_t m = mask[w];
  const uint64_t lo = m & ((1ull << b) - 1ull);
  const uint64_t hi = (b == 63) ? 0ull : (m >> (b + 1));
  L = lo ? (w * 64 + 63 - __clzll((long long)lo)) : (w > 0 ? lastc[w - 1] : -1);
  R = hi ? (x + __ffsll((long long)hi)) : (w + 1 < nw ? firstc[w + 1] : kNone);
}

template <int PPT>
__device__ __forceinline__ void warp_fill_row(const DevJob& J, int y, unsigned char* smem) {
  RowLds<PPT> s(smem);
  const int W = J.width;
  const int tid = threadIdx.x;
  const size_t row = (size_t)y * (size_t)W;
  const float bf = J.baseline_m * J.focal_px;
  const int sgn = (J.target_eye == 0) ? -1 : 1;
  const int nw = (W + 63) >> 6;

  // A: loads.
  float z[PPT];
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int x = tid + i * kThreads;
    if (x < W) {
      z[i] = __builtin_nontemporal_load(&J.src_depth[row + x]);
      s.col[x] = __builtin_nontemporal_load(&J.src_rgba[row + x]);
      s.key[x] = kEmpty;
    }
  }
  __syncthreads();

  // B: scatter with the depth test.
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int x = tid + i * kThreads;
    if (x < W) {
      const float zz = z[i];
      if (zz > 0.0f) {
        const float q = bf / zz;
        if (q < (float)W) {
          const int d = (int)roundf(q);
          const int xt = x + sgn * d;
          if ((unsigned)xt < (unsigned)W)
            atomicMin(&s.key[xt], ((uint64_t)__float_as_uint(zz) << 32) | (uint32_t)x);
        }
      }
    }
  }
  __syncthreads();

  // C: hit masks.
  if (J.fill_mode != 0) {
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int x = tid + i * kThreads;
      const bool hit = (x < W) && (s.key[x] != kEmpty);
      const uint64_t m = __ballot(hit);
      if ((tid & 63) == 0 && x < W) s.mask[x >> 6] = m;
    }
    __syncthreads();
    // D: word scan.
    if (tid < 64) scan_words<PPT>(s.mask, s.lastc, s.firstc, nw);
    __syncthreads();
  }

  // E: resolve + fill + store.
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int x = tid + i * kThreads;
    if (x < W) {
      uint64_t k = s.key[x];
      uint8_t mk = 0;
      if (k == kEmpty) {
        mk = 1;
        if (J.fill_mode != 0) {
          int L, R;
          neighbours(s.mask, s.lastc, s.firstc, nw, x, L, R);
          int p;
          if (L < 0 && R >= W) {
            p = -1;
          } else if (L < 0) {
            p = R;
          } else if (R >= W) {
            p = L;
          } else {
            const uint32_t zl = (uint32_t)(s.key[L] >> 32), zr = (uint32_t)(s.key[R] >> 32);
            p = zl > zr ? L : (zr > zl ? R : (sgn < 0 ? R : L));
          }
          if (p >= 0) {
            k = s.key[p];
          } else {
            mk = 2;
          }
        }
      }
      uint32_t c = 0;
      float zo = __builtin_inff();
      if (k != kEmpty) {
        c = s.col[(uint32_t)k];
        zo = __uint_as_float((uint32_t)(k >> 32));
      }
      __builtin_nontemporal_store(c, &J.dst_rgba[row + x]);
      if (J.dst_depth) __builtin_nontemporal_store(zo, &J.dst_depth[row + x]);
      if (J.dst_mask) J.dst_mask[row + x] = mk;
    }
  }
  __syncthreads();  // the next row reuses the LDS
}

template <int PPT>
__global__ __launch_bounds__(kThreads) void warp_single_kernel(DevJob J) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int y = blockIdx.x; y < J.height; y += gridDim.x) warp_fill_row<PPT>(J, y, smem);
}

template <int PPT>
__global__ __launch_bounds__(kThreads) void warp_batch_kernel(BatchHeader* hdr, const DevJob* __restrict__ jobs) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t n = hdr->n_jobs, total = hdr->total_rows;
  uint32_t j = 0;
  for (uint32_t r = blockIdx.x; r < total; r += gridDim.x) {
    // Rows only grow, so the job index only moves forward.
    while (j + 1 < n && jobs[j + 1].row_start <= r) ++j;
    const DevJob J = jobs[j];
    if (J.width > kThreads * PPT) {
      if (threadIdx.x == 0) atomicAdd(&hdr->errors, 1u);
      continue;
    }
    warp_fill_row<PPT>(J, (int)(r - J.row_start), smem);
  }
}

// ---------------------------------------------------------------------------
// Stand-alone fill of a warped frame, in place.  Hits (mask == 0) are read,
// never written; holes read only hits, so in-place is safe.
template <int PPT>
__global__ __launch_bounds__(kThreads) void fill_kernel(uint32_t* rgba, float* depth, uint8_t* mask, int W, int H,
                                                        int target_eye) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int wcap = kThreads * PPT;
  constexpr int words = (wcap + 63) / 64;
  uint32_t* col = reinterpret_cast<uint32_t*>(smem);
  float* zs = reinterpret_cast<float*>(col + wcap);
  uint64_t* hm = reinterpret_cast<uint64_t*>(zs + wcap);
  int32_t* lastc = reinterpret_cast<int32_t*>(hm + words);
  int32_t* firstc = lastc + words;
  const int tid = threadIdx.x;
  const int sgn = (target_eye == 0) ? -1 : 1;
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
        zs[x] = depth[row + x];
      }
    }
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int x = tid + i * kThreads;
      const uint64_t m = __ballot(x < W && m8[i] == 0);
      if ((tid & 63) == 0 && x < W) hm[x >> 6] = m;
    }
    __syncthreads();
    if (tid < 64) scan_words<PPT>(hm, lastc, firstc, nw);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int x = tid + i * kThreads;
      if (x < W && m8[i] != 0) {
        int L, R;
        neighbours(hm, lastc, firstc, nw, x, L, R);
        int p;
        if (L < 0 && R >= W) {
          p = -1;
        } else if (L < 0) {
          p = R;
        } else if (R >= W) {
          p = L;
        } else {
          const uint32_t zl = __float_as_uint(zs[L]), zr = __float_as_uint(zs[R]);
          // Hits carry depth > 0 or +inf, so the bit patterns order like the values.
          p = zl > zr ? L : (zr > zl ? R : (sgn < 0 ? R : L));
        }
        if (p >= 0) {
          rgba[row + x] = col[p];
          depth[row + x] = zs[p];
          mask[row + x] = 1;
        } else {
          rgba[row + x] = 0u;
          depth[row + x] = __builtin_inff();
          mask[row + x] = 2;
        }
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
__global__ void upload_kernel(UploadChunk chunk, DevJob* dst) {
  const uint32_t t = threadIdx.x;
  if (t < chunk.count) dst[chunk.first + t] = chunk.jobs[t];
}

__global__ void header_kernel(BatchHeader h, BatchHeader* dst) {
  if (threadIdx.x == 0) *dst = h;
}

// ---------------------------------------------------------------------------
template <int PPT>
hipError_t set_lds_limit(const void* fn, size_t bytes) {
  if (bytes > 65536) return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  return hipSuccess;
}

#define YORO_PPT_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(12) X(16) X(20) X(24) X(28) X(32)

}  // namespace

hipError_t launch_warp_single(const DevJob& job, int ppt, int grid, hipStream_t stream) {
  const size_t lds = warp_lds_bytes(ppt);
  switch (ppt) {
#define X(P)                                                                                   \
  case P: {                                                                                    \
    hipError_t e = set_lds_limit<P>((const void*)warp_single_kernel<P>, lds);                  \
    if (e != hipSuccess) return e;                                                             \
    hipLaunchKernelGGL(warp_single_kernel<P>, dim3(grid), dim3(kThreads), lds, stream, job);   \
    return hipGetLastError();                                                                  \
  }
    YORO_PPT_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_warp_batch(const BatchHeader* hdr, const DevJob* jobs, int ppt, int grid, hipStream_t stream) {
  const size_t lds = warp_lds_bytes(ppt);
  BatchHeader* h = const_cast<BatchHeader*>(hdr);
  switch (ppt) {
#define X(P)                                                                                      \
  case P: {                                                                                       \
    hipError_t e = set_lds_limit<P>((const void*)warp_batch_kernel<P>, lds);                      \
    if (e != hipSuccess) return e;                                                                \
    hipLaunchKernelGGL(warp_batch_kernel<P>, dim3(grid), dim3(kThreads), lds, stream, h, jobs);   \
    return hipGetLastError();                                                                     \
  }
    YORO_PPT_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_fill(uint32_t* rgba, float* depth, uint8_t* mask, int32_t width, int32_t height, int32_t target_eye,
                       int32_t fill_mode, int ppt, int grid, hipStream_t stream) {
  (void)fill_mode;
  const size_t lds = fill_lds_bytes(ppt);
  switch (ppt) {
#define X(P)                                                                                            \
  case P: {                                                                                             \
    hipError_t e = set_lds_limit<P>((const void*)fill_kernel<P>, lds);                                  \
    if (e != hipSuccess) return e;                                                                      \
    hipLaunchKernelGGL(fill_kernel<P>, dim3(grid), dim3(kThreads), lds, stream, rgba, depth, mask, width, \
                       height, target_eye);                                                             \
    return hipGetLastError();                                                                           \
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

hipError_t launch_upload(const UploadChunk& chunk, DevJob* dst, hipStream_t stream) {
  hipLaunchKernelGGL(upload_kernel, dim3(1), dim3(64), 0, stream, chunk, dst);
  return hipGetLastError();
}

hipError_t launch_header(BatchHeader hdr, BatchHeader* dst, hipStream_t stream) {
  hipLaunchKernelGGL(header_kernel, dim3(1), dim3(64), 0, stream, hdr, dst);
  return hipGetLastError();
}

int warp_blocks_per_cu(int ppt, bool batch) {
  int nb = 0;
  const size_t lds = warp_lds_bytes(ppt);
  hipError_t e = hipErrorInvalidValue;
  switch (ppt) {
#define X(P)                                                                                                       \
  case P:                                                                                                          \
    (void)set_lds_limit<P>(batch ? (const void*)warp_batch_kernel<P> : (const void*)warp_single_kernel<P>, lds);          \
    e = batch ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, warp_batch_kernel<P>, kThreads, lds)             \
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, warp_single_kernel<P>, kThreads, lds);           \
    break;
    YORO_PPT_CASES(X)
#undef X
    default:
      break;
  }
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

int fill_blocks_per_cu(int ppt) {
  int nb = 0;
  const size_t lds = fill_lds_bytes(ppt);
  hipError_t e = hipErrorInvalidValue;
  switch (ppt) {
#define X(P)                                                                              \
  case P:                                                                                 \
    (void)set_lds_limit<P>((const void*)fill_kernel<P>, lds);                                   \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fill_kernel<P>, kThreads, lds); \
    break;
    YORO_PPT_CASES(X)
#undef X
    default:
      break;
  }
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

}  // namespace yoro

// Row machinery shared by the row kernels (device code only): the per-row
// LDS layout, column iteration, the hit-mask walk, the nearest-background
// choice, the rounding of a shift, and the resolve + fill phases that turn
// a row of 64-bit target keys into output pixels.
#pragma once

#include "yoro_internal.h"

namespace yoro {
namespace {

constexpr uint64_t kEmpty = ~0ull;
constexpr uint32_t kInfBits = 0x7F800000u;  // bits of +inf

#define YORO_GLOBAL __attribute__((address_space(1)))

template <class T>
__device__ __forceinline__ YORO_GLOBAL T* gmem(T* p) {
  return (YORO_GLOBAL T*)p;
}

// Per-row LDS of the warp kernel, laid out for rows up to wl columns (wl: a
// multiple of 64, uniform for the launch).
struct RowLds {
  uint64_t* key;     // [wl + 64] target keys: depth bits << 32 | RGBA; the
                     //           last 64 are per-lane sinks for lanes with
                     //           nothing to splat
  uint64_t* mask;    // [wl/64]   hit masks, one per 64 columns
  uint32_t* pad;     // [4]
  uint16_t* holes;   // [4 seg]   columns of the row's holes, one segment per
                     //           wave (a wave owns one 64-column block per
                     //           kThreads columns, so seg = 64 per chunk)
  int seg;
  __device__ RowLds(unsigned char* base, int wl) {
    key = reinterpret_cast<uint64_t*>(base);
    mask = key + wl + 64;
    pad = reinterpret_cast<uint32_t*>(mask + (wl >> 6));
    holes = reinterpret_cast<uint16_t*>(pad + 4);
    seg = ((wl + kThreads - 1) / kThreads) * 64;
  }
};

// Runs body(i, x) for every column x = threadIdx.x + i*kThreads < W.  Chunks
// that lie wholly inside the row take a uniform (scalar) branch with no
// per-lane test; only the one ragged chunk tests x < W per lane.
template <int PPT, class F>
__device__ __forceinline__ void for_cols(int W, F&& body) {
  const int nfull = W / kThreads;
  const int x0 = threadIdx.x;
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    if (i < nfull) {
      body(i, x0 + i * kThreads);
    } else if (i == nfull) {
      if (x0 + i * kThreads < W) body(i, x0 + i * kThreads);
    }
  }
}

// Nearest hits strictly left (L, or -1) and strictly right (R, or W) of
// column x, walking the hit masks word by word from x's own word (hole runs
// are short: most walks end in the first or second word).
__device__ __forceinline__ void nearest_hits_walk(const uint64_t* mask, int nw, int W, int x, int& L, int& R) {
  const int w0 = x >> 6, b = x & 63;
  int w = w0;
  uint64_t m = mask[w] & ((1ull << b) - 1ull);
  while (m == 0 && w > 0) m = mask[--w];
  L = m ? (w * 64 + 63 - __clzll((long long)m)) : -1;
  w = w0;
  m = (b == 63) ? 0ull : (mask[w] >> (b + 1)) << (b + 1);
  while (m == 0 && w + 1 < nw) m = mask[++w];
  R = m ? (w * 64 + __ffsll((long long)m) - 1) : W;
}

// Which of the nearest hits fills a hole: the farther one; on equal depth
// the one opposite the shift (right when synthesising the right eye).
// zl, zr: depth bits of the hits (depths in (0, +inf] order like their bits).
__device__ __forceinline__ int pick_side(int L, int R, int W, uint32_t zl, uint32_t zr, bool target_right) {
  if (L < 0) return R < W ? R : -1;
  if (R >= W) return L;
  return zl > zr ? L : (zr > zl ? R : (target_right ? R : L));
}

// roundf(q) for 0 <= q < 2^23 without a float-to-int conversion (whose result
// is undefined for the lanes that do not splat): adding 2^23 rounds q to the
// nearest integer, ties to even, in the low mantissa bits; a tie that went
// down (q - r == 0.5 exactly) is then moved up, giving ties away from zero.
// Any other q gives an unspecified but harmless value.
__device__ __forceinline__ int round_half_away(float q) {
  const float y = q + 0x1p23f;
  const float r = y - 0x1p23f;
  return (__float_as_int(y) - 0x4B000000) + ((q - r) == 0.5f ? 1 : 0);
}

// Phases C-E of a row whose target keys (depth bits << 32 | RGBA, kEmpty
// for a target nobody reached) are in s.key[0, W):
//   C  every column is stored (a hole provisionally as RGBA 0, depth +inf,
//      mask 1); per wave64 a ballot of "target reached" gives one 64-bit hit
//      mask per 64 columns, and each wave appends its holes to its own
//      segment of the hole list as it goes;
//   E  each wave's listed holes walk the hit masks (all waves') from their
//      own word to their nearest hit on either side and take the farther
//      one (Section 5 O2; Section 7 Patcher figure: on equal depth, the side
//      opposite the shift), overwriting their provisional values.
// Every column's result goes to emit(x, low word, depth bits, mask): a hit
// (mask 0) and a filled hole (mask 1) carry their key's low word and depth,
// an unfilled hole gives 0, +inf and 1 (2 when its row has no hit at all).
// emit runs once per column in C and again for each hole in E; E reads only
// hits' keys, so emit may overwrite a hole's own key.  The caller
// synchronises before the LDS is reused.
template <int PPT, class Emit>
__device__ __forceinline__ void resolve_fill_row(const RowLds& s, int W, bool target_right, bool fill,
                                                 Emit&& emit) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int nw = (W + 63) >> 6;
  const int nfull = W / kThreads;
  uint16_t* holes = s.holes + wave * s.seg;  // this wave's segment

  // C: store every column (holes get RGBA 0 / +inf / mask 1 for now), build
  // the hit masks, list the holes.  A hit's high word holds the bits of a
  // depth in (0, +inf], never the all-ones of EMPTY.
  uint32_t run = 0;    // holes listed by this wave so far (wave-uniform)
  uint64_t mword = 0;  // lane i: hit mask of chunk i's 64 columns of this wave
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    if (i * kThreads < W) {
      const int x = tid + i * kThreads;
      const uint64_t k = s.key[min(x, W - 1)];
      const bool inrow = x < W;
      const bool hit = inrow & ((uint32_t)(k >> 32) != 0xFFFFFFFFu);
      const uint32_t c = hit ? (uint32_t)k : 0u;
      const uint32_t zo = hit ? (uint32_t)(k >> 32) : kInfBits;
      if (i < nfull) {
        emit(x, c, zo, hit ? 0 : 1);
      } else if (inrow) {
        emit(x, c, zo, hit ? 0 : 1);
      }
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
      // Park this chunk's mask in lane i (lo/hi halves) for one store below.
      mword = (lane == i) ? hm : mword;
    }
  }
  if (fill) {
    // One LDS store per lane that parked a mask: word (i*4 + wave) holds
    // chunk i's columns of this wave.
    const int nchunks = (W + kThreads - 1) / kThreads;
    const int word = lane * (kThreads / 64) + wave;
    if (lane < nchunks && word < nw) s.mask[word] = mword;
    __syncthreads();
    // E (at the lowest wave priority): this wave fills the holes it listed.
    // Only hits are read, only holes written.
    __builtin_amdgcn_s_setprio(0);
    for (uint32_t h0 = 0; h0 < run; h0 += 64) {
      const uint32_t h = h0 + lane;
      int x = h < run ? (int)holes[h] : 0;
      const bool act = (h < run) & (x < W);  // every listed column is < W; guard the store anyway
      x = act ? x : 0;
      int L, R;
      nearest_hits_walk(s.mask, nw, W, x, L, R);
      const uint32_t zl = (uint32_t)(s.key[max(L, 0)] >> 32);
      const uint32_t zr = (uint32_t)(s.key[min(R, W - 1)] >> 32);
      const int p = pick_side(L, R, W, zl, zr, target_right);
      const uint64_t k = s.key[max(p, 0)];
      if (act) emit(x, p >= 0 ? (uint32_t)k : 0u, p >= 0 ? (uint32_t)(k >> 32) : kInfBits, p >= 0 ? 1 : 2);
    }
  }
}

}  // namespace
}  // namespace yoro

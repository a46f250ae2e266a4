// Kernels of the learned hole filler (a 4-level convolutional
// encoder-decoder, BF16 storage, FP32 accumulation on the MFMA units).
//
// Tensors are NHWC: a pixel's channels are contiguous; "ld" is the element
// stride between consecutive pixels (>= the channel count, so a convolution
// can read or write a channel slice of a wider concatenation buffer).
// Activations and weight copies are bfloat16 (raw 16-bit words here), master
// weights, their gradients and the network's residual output are FP32.
//
// conv3x3: implicit GEMM.  M = pixels, N = output channels, K = 9 taps x
// input channels, on v_mfma_f32_16x16x32_bf16 (A: 16 pixels x 32 channels,
// B: 32 channels x 16 outputs, D: 16 x 16 FP32).  Lane l of a wave holds A
// row (l % 16) with k = 8*(l/16) .. +7, B column (l % 16) with the same k,
// and D column (l % 16) with rows 4*(l/16) .. +3.  Input patches are staged
// in LDS and shared by the nine taps.  The same kernel computes the input
// gradient with the weights flipped and transposed.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "yoro_internal.h"

namespace yoro {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;
typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;

// float -> bfloat16 bits, round to nearest, ties to even (no NaN inputs here).
// Round to nearest, ties to even (gfx950 converts in hardware:
// v_cvt_pk_bf16_f32, two values per instruction).
__device__ __forceinline__ uint16_t to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ uint32_t to_bf16x2(float lo, float hi) {
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  const bf16x2_t v = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// Signed 16-bit max of two packed bf16 values with the halves of `lo`
// (one v_pk_max_i16).
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t v, uint32_t lo) {
  typedef short short2_t __attribute__((ext_vector_type(2)));
  // (Opaque to the compiler: otherwise it splits a packed conversion that
  // feeds this max into two single ones and a permute.)
  asm("" : "+v"(v));
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(short2_t, v),
                                                                __builtin_bit_cast(short2_t, lo)));
}

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

constexpr int kConvThreads = 256;  // 4 waves

// ----------------------------------------------------------- conv3x3, tiled --
// Output tile: 8 rows x 32 pixels of one image x CT channels per 256-thread
// workgroup.  Per 32-channel input chunk the (8+2) x (32+2) input patch and
// the chunk's weights for all nine taps are staged once in LDS; wave w
// computes rows 2w and 2w+1 (four 16-pixel M tiles) x CT channels, so each
// B fragment feeds four MFMAs and each A fragment CT/16.
// The LDS pixel stride is 40 bf16 (32 channels + 8 pad = 80 bytes) so the 16
// lanes reading one k group of 16 consecutive pixels hit distinct banks.
constexpr int kTileH = 8, kTileW = 32;
constexpr int kPatchH = kTileH + 2, kPatchW = kTileW + 2;
constexpr int kPatchStride = 40;
constexpr int kPatchLoads = (kPatchH * kPatchW * 4 + kConvThreads - 1) / kConvThreads;  // 16-byte loads per thread
constexpr int kRawLoads = (kPatchH * kPatchW + kConvThreads - 1) / kConvThreads;  // first layer: pixels per thread

constexpr float kLogZmin = -1.2039728043259361f;  // log(0.3)
constexpr float kLogZmax = 3.912023005428146f;    // log(50)

// The network's first eight input channels of one pixel as bf16 (R, G, B
// in [0, 1], the hole mask, log depth scaled to [0, 1] with NaN -> 1, three
// zeros); the other 24 channels are zero.
__device__ __forceinline__ u32x4 input_channels(uint32_t c, float z, uint8_t m) {
  float ld = (logf(z) - kLogZmin) / (kLogZmax - kLogZmin);
  ld = (ld >= 0.0f) ? (ld <= 1.0f ? ld : 1.0f) : (ld < 0.0f ? 0.0f : 1.0f);  // NaN -> 1
  uint16_t v[5];
  v[0] = to_bf16((float)(c & 255u) / 255.0f);
  v[1] = to_bf16((float)((c >> 8) & 255u) / 255.0f);
  v[2] = to_bf16((float)((c >> 16) & 255u) / 255.0f);
  v[3] = to_bf16(m != 0 ? 1.0f : 0.0f);
  v[4] = to_bf16(ld);
  return u32x4{(uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16), (uint32_t)v[4], 0u};
}

// Waves per SIMD (the VGPR budget) for a CT-wide output tile: what the LDS
// of one workgroup (patch + CT channels of weights) lets fit, and no more
// than the registers of the prefetched patch leave room for without spills.
constexpr int conv_waves(int ct) { return ct <= 32 ? 3 : 2; }

// RAW: the first layer, whose input is the frame itself (raw_rgba, ...).
// NW: input chunks whose weights stay in LDS for every item (1, or 2 for the
// 64-input-channel layers of a 32-channel tile, which then stage no weights
// per item).
template <int CT, bool RAW, int NW = 1>
__global__ __launch_bounds__(kConvThreads) __attribute__((amdgpu_waves_per_eu(NW > 1 ? 2 : conv_waves(CT)))) void
conv3x3_tiled_kernel(const uint16_t* __restrict__ x, int ldx, long long xcs, int N,
                                                                     int H, int W, int Cin,
                                                                     const uint16_t* __restrict__ wgt, int Cout,
                                                                     void* __restrict__ y, int ldy, int y_fp32,
                                                                     int cout_store, int epi,
                                                                     const uint16_t* __restrict__ msrc, int ldm,
                                                                     int ups, int ntiles, uint16_t* __restrict__ pool,
                                                                     int ldp, const uint32_t* __restrict__ raw_rgba,
                                                                     const float* __restrict__ raw_depth,
                                                                     const uint8_t* __restrict__ raw_mask) {
  constexpr int NB = CT / 16;
  // 8-byte output stores: bf16 output, channel groups of 4 whole, and 8-byte
  // aligned rows (the launcher checks the base pointers).
  // Offsets inside a tile's rows of every buffer fit 32 bits (the usual
  // case): interior tiles then load their patch, and the 8-byte path stores
  // its outputs, through one base address per tile and 32-bit per-lane byte
  // offsets (no 64-bit address arithmetic per lane).
  const long long ld_max = max(max(ldx, ldy), max(ldm, ldp));
  const bool small = 4LL * (kPatchH + 1) * W * ld_max < (1LL << 31);
  const bool wide = small && !y_fp32 && (cout_store & 3) == 0 && (ldy & 3) == 0 && (epi != 2 || (ldm & 3) == 0) &&
                    ((reinterpret_cast<uintptr_t>(y) | reinterpret_cast<uintptr_t>(msrc)) & 7u) == 0;
  // ReLU on two packed bf16 values: a signed 16-bit max with 0 zeroes the
  // negative ones (as max(v, 0) before rounding would); with -32768 it
  // changes nothing.
  const uint32_t relu_floor = epi == 1 ? 0u : 0x80008000u;
  __shared__ __align__(16) uint16_t patch[kPatchH * kPatchW * kPatchStride];
  // The chunk's weights for all nine taps: [tap][output channel][32 + 8 pad].
  __shared__ __align__(16) uint16_t wlds[NW * 9 * CT * kPatchStride];
  const int tiles_x = (W + kTileW - 1) / kTileW, tiles_y = (H + kTileH - 1) / kTileH;
  const int co0 = blockIdx.y * CT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kg = (lane >> 4) * 8;
  // Chunk ci0's weights go to slot (ci0 / 32) % NW.
  auto stage_weights = [&](int ci0) {
    uint16_t* slot = wlds + ((ci0 >> 5) % NW) * (9 * CT * kPatchStride);
    for (int e = threadIdx.x; e < 9 * CT * 4; e += kConvThreads) {
      const int tc = e >> 2, part = e & 3;  // tc = tap * CT + output channel
      const int t = tc / CT, co = tc - t * CT;
      *reinterpret_cast<u32x4*>(slot + tc * kPatchStride + part * 8) =
          *reinterpret_cast<const u32x4*>(wgt + ((long long)t * Cout + co0 + co) * Cin + ci0 + part * 8);
    }
  };
  // 64-channel tiles: the next item's chunk weights (nine 16-byte pieces
  // per thread) are loaded into registers with its patch and written to LDS
  // at its start, so their load overlaps this item's MFMAs like the patch's.
  // Narrower tiles load and stage them at the item's start.
  constexpr bool kPreW = CT == 64;
  constexpr int kWLoads = 9 * CT * 4 / kConvThreads;
  u32x4 wpre[kPreW ? kWLoads : 1];
  auto load_weights = [&](int ci0) {
    int tid = threadIdx.x;  // (recomputed per item rather than held across the loop)
    asm volatile("" : "+v"(tid));
#pragma unroll
    for (int k = 0; k < kWLoads; ++k) {
      const int e = tid + k * kConvThreads;
      const int tc = e >> 2, part = e & 3;
      const int t = tc / CT, co = tc - t * CT;
      wpre[k] = *reinterpret_cast<const u32x4*>(wgt + ((long long)t * Cout + co0 + co) * Cin + ci0 + part * 8);
    }
  };
  auto store_weights = [&](int ci0) {
    uint16_t* slot = wlds + ((ci0 >> 5) % NW) * (9 * CT * kPatchStride);
#pragma unroll
    for (int k = 0; k < kWLoads; ++k) {
      const int e = threadIdx.x + k * kConvThreads;
      *reinterpret_cast<u32x4*>(slot + (e >> 2) * kPatchStride + (e & 3) * 8) = wpre[k];
    }
  };
  // When every input chunk's weights fit (Cin = 32 NW) they stay in LDS for
  // every tile this workgroup takes; otherwise each chunk of each tile
  // stages its own.
  const bool one_chunk = Cin == 32 * NW;
  if (one_chunk)
    for (int c = 0; c < NW; ++c) stage_weights(32 * c);
  // Tiles v = blockIdx.x, + gridDim.x, ... in an XCD-aware order: workgroup
  // w runs on XCD w % 8 (gridDim.x is a multiple of 8 or the whole tile
  // count), and each XCD takes one contiguous range of tiles, so tiles that
  // share halo rows share an L2.
  const int q8 = ntiles >> 3, r8 = ntiles & 7;
  auto origin = [&](int v, int& x0, int& y0, int& n) {
    const int xc = v & 7;
    int b = xc * q8 + min(xc, r8) + (v >> 3);
    const int tx = b % tiles_x;
    b /= tiles_x;
    const int ty = b % tiles_y;
    n = b / tiles_y;
    x0 = tx * kTileW;
    y0 = ty * kTileH;
  };
  // The workgroup's items are (tile, 32-channel input chunk) in order.  The
  // next item's patch is loaded into registers before this item's MFMAs and
  // stores go out, and written to LDS at the next item's start, so the loads
  // are in flight while this item computes.  Every lane loads (coordinates
  // clamped into the frame, no branches, so no load has to land before the
  // next is issued); which lanes lie outside the frame is kept as a bit mask
  // and their values are zeroed when written to LDS.  The first layer's
  // frame values are held raw (colour, depth bits, mask) and packed then.
  u32x4 pre[kPatchLoads];
  uint32_t inside_bits = 0;
  auto load_patch = [&](int v, int ci0) {
    int x0, y0, n;
    origin(v, x0, y0, n);
    const long long img = (long long)n * H * W;
    if (small && x0 >= 1 && y0 >= 1 && x0 + kPatchW - 1 <= W && y0 + kPatchH - 1 <= H) {
      // An interior tile: the patch lies inside the frame, so no clamping,
      // and every element sits at a fixed offset from the patch's top-left
      // pixel (y0 - 1, x0 - 1); an upsampled input reads the
      // half-resolution pixel under it, (y0 / 2 - 1, x0 / 2 - 1) on.
      const long long base = ups ? (img >> 2) + (long long)((y0 >> 1) - 1) * (W >> 1) + ((x0 >> 1) - 1)
                                 : img + (long long)(y0 - 1) * W + (x0 - 1);
      inside_bits = ~0u;
      // The per-lane offsets are recomputed for each tile (a few
      // instructions) rather than held in registers across the loop.
      int tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      if (RAW) {  // one lane per pixel
        const char* rb = reinterpret_cast<const char*>(raw_rgba + base);
        const char* db = reinterpret_cast<const char*>(raw_depth + base);
#pragma unroll
        for (int k = 0; k < kRawLoads; ++k) {
          const int e = tid + k * kConvThreads;
          const int pix = e < kPatchH * kPatchW ? e : 0;
          const int py = pix / kPatchW, px = pix - py * kPatchW;
          const uint32_t rel = (uint32_t)(py * W + px);
          pre[k] = u32x4{*reinterpret_cast<const uint32_t*>(rb + rel * 4u),
                         *reinterpret_cast<const uint32_t*>(db + rel * 4u), (uint32_t)(raw_mask + base)[rel], 0u};
        }
        return;
      }
#pragma unroll
      for (int k = 0; k < kPatchLoads; ++k) {
        const int e = tid + k * kConvThreads;
        // Entries past the patch (skipped when stored) read its first pixel.
        const int pix = e < kPatchH * kPatchW * 4 ? e >> 2 : 0;
        const int py = pix / kPatchW, px = pix - py * kPatchW;
        const uint32_t rel = ups ? (uint32_t)(((py + 1) >> 1) * (W >> 1) + ((px + 1) >> 1)) : (uint32_t)(py * W + px);
        const char* xb = reinterpret_cast<const char*>(x + (base * ldx + (ci0 >> 5) * xcs));
        pre[k] = *reinterpret_cast<const u32x4*>(xb + (rel * (uint32_t)ldx + (uint32_t)(e & 3) * 8u) * 2u);
      }
      return;
    }
    inside_bits = 0;
    if (RAW) {  // one lane per pixel, clamped into the frame
#pragma unroll
      for (int k = 0; k < kRawLoads; ++k) {
        const int e = threadIdx.x + k * kConvThreads;
        const int py = e / kPatchW, px = e - py * kPatchW;
        const int gy = y0 + py - 1, gx = x0 + px - 1;
        const bool inside = e < kPatchH * kPatchW && gy >= 0 && gy < H && gx >= 0 && gx < W;
        inside_bits |= (uint32_t)inside << k;
        const long long q = img + (long long)min(max(gy, 0), H - 1) * W + min(max(gx, 0), W - 1);
        pre[k] = u32x4{raw_rgba[q], __float_as_uint(raw_depth[q]), (uint32_t)raw_mask[q], 0u};
      }
      return;
    }
#pragma unroll
    for (int k = 0; k < kPatchLoads; ++k) {
      const int e = threadIdx.x + k * kConvThreads;
      const int pix = e >> 2, part = e & 3;
      const int py = pix / kPatchW, px = pix - py * kPatchW;
      const int gy = y0 + py - 1, gx = x0 + px - 1;
      const bool inside = e < kPatchH * kPatchW * 4 && gy >= 0 && gy < H && gx >= 0 && gx < W;
      inside_bits |= (uint32_t)inside << k;
      const int cy = min(max(gy, 0), H - 1), cx = min(max(gx, 0), W - 1);
      // ups: x is the half-resolution image and the input is its nearest x2
      // upsampling, read in place.
      const long long src = ups ? (img >> 2) + (long long)(cy >> 1) * (W >> 1) + (cx >> 1)
                                : img + (long long)cy * W + cx;
      pre[k] = *reinterpret_cast<const u32x4*>(x + src * ldx + (ci0 >> 5) * xcs + part * 8);
    }
  };
  auto store_patch = [&]() {
    if (RAW) {
      // The first layer: each pixel's packed input (built channel by channel
      // as the input-packing kernel does) in its first 8 channels; the other
      // 24 stay zero from the start.
#pragma unroll
      for (int k = 0; k < kRawLoads; ++k) {
        const int e = threadIdx.x + k * kConvThreads;
        const u32x4 v = pre[k];
        asm volatile("" : : "v"(v));  // (as below)
        if (e >= kPatchH * kPatchW) continue;
        const u32x4 c = ((inside_bits >> k) & 1u) ? input_channels(v[0], __uint_as_float(v[1]), (uint8_t)v[2])
                                                  : u32x4{0u, 0u, 0u, 0u};
        *reinterpret_cast<u32x4*>(patch + e * kPatchStride) = c;
      }
      return;
    }
#pragma unroll
    for (int k = 0; k < kPatchLoads; ++k) {
      const int e = threadIdx.x + k * kConvThreads;
      u32x4 v = pre[k];
      // Every lane takes its loaded value here, also where it stores none,
      // so the wait for the load is not left pending on one branch (a
      // pending load makes the compiler wait for every outstanding memory
      // operation, the previous tile's stores included, before the next
      // loads).
      asm volatile("" : : "v"(v));
      if (e >= kPatchH * kPatchW * 4) continue;
      const bool inside = (inside_bits >> k) & 1u;
      if (!inside) v = u32x4{0u, 0u, 0u, 0u};
      *reinterpret_cast<u32x4*>(patch + (e >> 2) * kPatchStride + (e & 3) * 8) = v;
    }
  };
  floatx4 acc[4][NB];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[m][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
  if (RAW)  // channels 8..31 of the first layer's patch stay zero
    for (int e = threadIdx.x; e < kPatchH * kPatchW * 4; e += kConvThreads)
      *reinterpret_cast<u32x4*>(patch + (e >> 2) * kPatchStride + (e & 3) * 8) = u32x4{0u, 0u, 0u, 0u};
  int v = blockIdx.x, ci0 = 0;
  if (v < ntiles) {
    load_patch(v, 0);
    if (kPreW && !one_chunk) load_weights(0);
  }
  while (v < ntiles) {
    __syncthreads();  // the previous item's readers are done with the patch (and the weights)
    store_patch();
    if (!one_chunk) {
      if (kPreW)
        store_weights(ci0);
      else
        stage_weights(ci0);
    }
    int vn = v, cn = ci0 + 32;
    if (cn == Cin) {
      vn = v + gridDim.x;
      cn = 0;
    }
    __syncthreads();
    if (vn < ntiles) {
      load_patch(vn, cn);
      if (kPreW && !one_chunk) load_weights(cn);
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      u32x4 bcur[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        bcur[nb] = *reinterpret_cast<const u32x4*>(wlds + ((ci0 >> 5) % NW) * (9 * CT * kPatchStride) +
                                                   (t * CT + nb * 16 + (lane & 15)) * kPatchStride + kg);
      const int ky = t / 3, kx = t % 3;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int r = 2 * wave + (m >> 1), c = (m & 1) * 16 + (lane & 15);
        const u32x4 av =
            *reinterpret_cast<const u32x4*>(patch + ((r + ky) * kPatchW + (c + kx)) * kPatchStride + kg);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(av), as_bf16x8(bcur[nb]), acc[m][nb], 0, 0,
                                                               0);
      }
    }
    if (cn != 0) {  // more input chunks of this tile to come
      v = vn;
      ci0 = cn;
      continue;
    }
  int x0, y0, n;
  origin(v, x0, y0, n);
  const long long img = (long long)n * H * W;
  // Epilogue: lane holds channel co0 + 16nb + lane%16 of pixels 4*(lane/16)+r
  // of M tile m, i.e. row 2*wave + m/2, column 16*(m%2) + 4*(lane/16) + r.
  if (wide) {
    // bf16 outputs: the four lanes 4q..4q+3 of a 16-lane group hold four
    // channels of the same four pixels; a 4 x 4 transpose between them (two
    // DPP exchanges) gives lane j = lane%4 pixel 4*(lane/16) + j's four
    // channels 4q..4q+3, stored as one 8-byte write instead of four 2-byte
    // ones.  The values are those of the per-element path below.
    // Per-lane offsets and selectors are recomputed for each tile rather
    // than held in registers across the loop (the opaque copy of the lane
    // index keeps the compiler from hoisting them).
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const int j = ln & 3, q = (ln >> 2) & 3, g = ln >> 4;
    // v_perm byte selectors (result byte i = byte sel[i] of the pair
    // {first operand: bytes 4..7, second: bytes 0..3}).
    const uint32_t sel_s = (j & 1) ? 0x05040100u : 0x07060302u;
    const uint32_t sel_lo = j == 0 ? 0x05040100u : j == 1 ? 0x03020504u : j == 2 ? 0x07060100u : 0x03020706u;
    const uint32_t sel_hi = j == 0 ? 0x07060100u : j == 1 ? 0x03020706u : j == 2 ? 0x05040100u : 0x03020504u;
    char* yb = reinterpret_cast<char*>(y) + 2 * ((img + (long long)y0 * W + x0) * ldy + co0);
    const char* mb =
        epi == 2 ? reinterpret_cast<const char*>(msrc) + 2 * ((img + (long long)y0 * W + x0) * ldm + co0) : nullptr;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int row = 2 * wave + (m >> 1), col = (m & 1) * 16 + g * 4 + j;
      const bool in = y0 + row < H && x0 + col < W;
      const uint32_t po = (uint32_t)(row * W + col);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        // A: pixels 4g, 4g + 1 of channel 4q + j; B: pixels 4g + 2, 4g + 3.
        const uint32_t A = relu_bf16x2(to_bf16x2(acc[m][nb][0], acc[m][nb][1]), relu_floor);
        const uint32_t B = relu_bf16x2(to_bf16x2(acc[m][nb][2], acc[m][nb][3]), relu_floor);
        // Lanes j and j ^ 2 swap pixel pairs: own is the pair holding pixel
        // 4g + j in channel j, recv the same pair in channel j ^ 2.
        const uint32_t own = (j & 2) ? B : A;
        const uint32_t recv = (uint32_t)__builtin_amdgcn_mov_dpp((int)((j & 2) ? A : B), 0x4E, 0xF, 0xF, true);
        // Lanes j and j ^ 1 swap the pair's other pixel in both channels: R
        // holds pixel 4g + j in channels j ^ 1 (low half) and j ^ 3 (high).
        const uint32_t S = __builtin_amdgcn_perm(recv, own, sel_s);
        const uint32_t R = (uint32_t)__builtin_amdgcn_mov_dpp((int)S, 0xB1, 0xF, 0xF, true);
        // Channels 4q, 4q + 1 from R and the word holding the even channel
        // of j's pair {j, j ^ 2}; channels 4q + 2, 4q + 3 from R and the other.
        const uint32_t even = (j & 2) ? recv : own, odd = (j & 2) ? own : recv;
        uint32_t w01 = __builtin_amdgcn_perm(R, even, sel_lo);
        uint32_t w23 = __builtin_amdgcn_perm(R, odd, sel_hi);
        const int co = nb * 16 + 4 * q;
        if (!in || co0 + co >= cout_store) continue;
        const uint32_t off = (po * (uint32_t)ldy + (uint32_t)co) * 2u;
        if (epi == 2) {  // ReLU derivative: zero where the forward activation was not positive
          const uint2 mk = *reinterpret_cast<const uint2*>(mb + (po * (uint32_t)ldm + (uint32_t)co) * 2u);
          const uint32_t mw[2] = {mk.x, mk.y};
          uint32_t* ww[2] = {&w01, &w23};
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            if (!(from_bf16((uint16_t)(mw[u] & 0xFFFFu)) > 0.0f)) *ww[u] &= 0xFFFF0000u;
            if (!(from_bf16((uint16_t)(mw[u] >> 16)) > 0.0f)) *ww[u] &= 0x0000FFFFu;
          }
        }
        *reinterpret_cast<uint2*>(yb + off) = uint2{w01, w23};
      }
    }
  } else if (y_fp32 && small && epi != 2) {
    // FP32 outputs (the head's residual): the per-element stores below, at
    // 32-bit offsets from the tile's first output.
    int ln = lane;
    asm volatile("" : "+v"(ln));
    char* yb = reinterpret_cast<char*>(y) + 4 * ((img + (long long)y0 * W + x0) * ldy + co0);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int row = 2 * wave + (m >> 1);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int co = nb * 16 + (ln & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = (m & 1) * 16 + (ln >> 4) * 4 + r;
          if (y0 + row >= H || x0 + col >= W || co0 + co >= cout_store) continue;
          const float v = epi == 1 ? fmaxf(acc[m][nb][r], 0.0f) : acc[m][nb][r];
          *reinterpret_cast<float*>(yb + ((uint32_t)(row * W + col) * (uint32_t)ldy + (uint32_t)co) * 4u) = v;
        }
      }
    }
  } else {
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int gy = y0 + 2 * wave + (m >> 1);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int co = co0 + nb * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gx = x0 + (m & 1) * 16 + (lane >> 4) * 4 + r;
        if (gy >= H || gx >= W || co >= cout_store) continue;
        const long long p = img + (long long)gy * W + gx;
        float v = acc[m][nb][r];
        if (epi == 1) v = fmaxf(v, 0.0f);
        if (epi == 2) v = (from_bf16(msrc[p * ldm + co]) > 0.0f) ? v : 0.0f;
        if (y_fp32)
          reinterpret_cast<float*>(y)[p * ldy + co] = v;
        else
          reinterpret_cast<uint16_t*>(y)[p * ldy + co] = to_bf16(v);
      }
    }
  }
  }
  // Optional 2x2 average pool of the stored bf16 outputs (H, W even): a
  // window is rows 2*wave, 2*wave + 1 (M tiles m and m + 2) and columns
  // r, r + 1 (r even) of one lane, summed as the pooling kernel sums them.
  if (pool && small) {
    // The same sums from the rounded, rectified values as packed words, at
    // 32-bit offsets from the tile's first pooled pixel.
    const int Ho = H >> 1, Wo = W >> 1;
    const long long imgo = (long long)n * Ho * Wo;
    const int yo = (y0 >> 1) + wave;
    char* pb = reinterpret_cast<char*>(pool) + 2 * ((imgo + (long long)(y0 >> 1) * Wo + (x0 >> 1)) * ldp + co0);
    // (Recomputed rather than kept from the stores above: holding those
    // words until here would cost registers.)
    uint32_t lo = relu_floor;
    asm volatile("" : "+s"(lo));
    int ln = lane;
    asm volatile("" : "+v"(ln));
#pragma unroll
    for (int m = 0; m < 2; ++m) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int co = nb * 16 + (ln & 15);
#pragma unroll
        for (int r = 0; r < 4; r += 2) {
          const int xr = ((m & 1) * 16 + (ln >> 4) * 4 + r) >> 1;
          if (yo >= Ho || (x0 >> 1) + xr >= Wo || co0 + co >= cout_store) continue;
          const uint32_t T = relu_bf16x2(to_bf16x2(acc[m][nb][r], acc[m][nb][r + 1]), lo);
          const uint32_t U = relu_bf16x2(to_bf16x2(acc[m + 2][nb][r], acc[m + 2][nb][r + 1]), lo);
          const float sum = (__uint_as_float(T << 16) + __uint_as_float(T & 0xFFFF0000u)) +
                            (__uint_as_float(U << 16) + __uint_as_float(U & 0xFFFF0000u));
          const uint32_t off = ((uint32_t)(wave * Wo + xr) * (uint32_t)ldp + (uint32_t)co) * 2u;
          *reinterpret_cast<uint16_t*>(pb + off) = to_bf16(sum * 0.25f);
        }
      }
    }
  } else if (pool) {
    const int Ho = H >> 1, Wo = W >> 1;
    const long long imgo = (long long)n * Ho * Wo;
    const int yo = (y0 >> 1) + wave;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int co = co0 + nb * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; r += 2) {
          const int xo = (x0 + (m & 1) * 16 + (lane >> 4) * 4 + r) >> 1;
          if (yo >= Ho || xo >= Wo || co >= cout_store) continue;
          float q[4];
          const float src[4] = {acc[m][nb][r], acc[m][nb][r + 1], acc[m + 2][nb][r], acc[m + 2][nb][r + 1]};
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            float v = src[u];
            if (epi == 1) v = fmaxf(v, 0.0f);  // (a pooled launch has no masked epilogue)
            q[u] = from_bf16(to_bf16(v));
          }
          const float sum = (q[0] + q[1]) + (q[2] + q[3]);
          pool[(imgo + (long long)yo * Wo + xo) * ldp + co] = to_bf16(sum * 0.25f);
        }
      }
    }
  }
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[m][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
  v = vn;
  ci0 = cn;
  }  // items
}

// ---------------------------------------------------------- weight grad --
// dW[t][co][ci] = sum_p dy[p][co] * x[p + off(t)][ci]: per tap a GEMM with
// M = co, N = ci, K = pixels.  A workgroup owns a TCO x 32 block of (co, ci)
// and all nine taps, and walks the tiles of kWgRows x kWgCols pixels of its
// chunk.  Per tile, dy (TCO channels) and the x patch with its one-pixel
// halo (32 channels) are staged in LDS channel-major; the patch is stored
// three times, shifted by 0, 1 and 2 columns, so that each tap's operand is
// an aligned 16-byte read.  Each tile row is one K step of 32 pixels for all
// nine taps, which share the step's dy fragments.  Wave w owns ci rows
// 16 (w & 1) .. +15 and TCO / 32 of the 16-row co tiles: 9 TCO / 32
// accumulators.  Partial sums go to ws[chunk][t][co][ci]; a second kernel
// adds the chunks in order, so the result does not depend on scheduling.
constexpr int kWgRows = 4;                                        // tile rows = K steps per tile
constexpr int kWgCols = 32;                                       // pixels per K step
constexpr int kWgTci = 32;                                        // input channels per workgroup
constexpr int kWgRowStride = 40;                                  // bf16 per staged row: 32 + 8 pad
constexpr int kWgDyStride = kWgRows * kWgRowStride + 8;           // bf16 per dy channel
constexpr int kWgXStride = (kWgRows + 2) * kWgRowStride + 8;      // bf16 per x channel and shift
// The channel strides (84 and 124 dwords) put the 16 channels that one
// fragment read touches on distinct 4-dword bank groups.

template <int TCO>
__global__ __launch_bounds__(256) void conv3x3_wgrad_kernel(const uint16_t* __restrict__ x, int ldx,
                                                            const uint16_t* __restrict__ dy, int lddy, int H, int W,
                                                            int Cin, int Cout, long long tiles, int nchunks,
                                                            float* __restrict__ ws) {
  __shared__ __align__(16) uint16_t sdy[TCO * kWgDyStride];
  __shared__ __align__(16) uint16_t sx[3 * kWgTci * kWgXStride];
  constexpr int CPW = TCO / 32;  // co tiles per wave
  const int nci = Cin / kWgTci;
  const int co0 = (blockIdx.x / nci) * TCO, ci0 = (blockIdx.x % nci) * kWgTci;
  const int chunk = blockIdx.y;
  const long long t0 = tiles * chunk / nchunks, t1 = tiles * (chunk + 1) / nchunks;
  const int tiles_x = (W + kWgCols - 1) / kWgCols, tiles_y = (H + kWgRows - 1) / kWgRows;
  const long long per_img = (long long)tiles_x * tiles_y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kg = (lane >> 4) * 8;
  const int cit = wave & 1, cog = wave >> 1;
  floatx4 acc[CPW][9];
#pragma unroll
  for (int i = 0; i < CPW; ++i)
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[i][t] = floatx4{0.f, 0.f, 0.f, 0.f};

  // Staging: thread e of a tile loads dy items e, e + 256, ... and x items
  // likewise (item = 8 channels of one pixel).  The next tile's items are
  // loaded into registers while the current tile's MFMAs run; addresses are
  // clamped into the tensors and items outside the image are zeroed when
  // they are written to LDS (branch-free loads keep them all in flight).
  constexpr int kDyItems = kWgRows * kWgCols * (TCO / 8);
  constexpr int kXPix = (kWgRows + 2) * (kWgCols + 2);
  constexpr int kXItems = kXPix * (kWgTci / 8);
  constexpr int kDyPer = (kDyItems + 255) / 256, kXPer = (kXItems + 255) / 256;
  u32x4 vdy[kDyPer], vx[kXPer];
  unsigned okdy = 0, okx = 0;
  auto load_tile = [&](long long tile) {
    const long long n = tile / per_img;
    const int rem = (int)(tile - n * per_img);
    const int y0 = (rem / tiles_x) * kWgRows, x0 = (rem % tiles_x) * kWgCols;
    okdy = 0, okx = 0;
#pragma unroll
    for (int k = 0; k < kDyPer; ++k) {
      const int e = threadIdx.x + 256 * k;
      const int px = e % (kWgRows * kWgCols), c8 = (e / (kWgRows * kWgCols)) * 8;
      const int yy = y0 + px / kWgCols, xx = x0 + px % kWgCols;
      const bool ok = e < kDyItems && yy < H && xx < W;
      const long long pix = ok ? (n * H + yy) * W + xx : 0;
      vdy[k] = *reinterpret_cast<const u32x4*>(dy + pix * lddy + co0 + (ok ? c8 : 0));
      okdy |= (ok ? 1u : 0u) << k;
    }
#pragma unroll
    for (int k = 0; k < kXPer; ++k) {
      const int e = threadIdx.x + 256 * k;
      const int px = e % kXPix, c8 = (e / kXPix) * 8;
      const int yy = y0 - 1 + px / (kWgCols + 2), xx = x0 - 1 + px % (kWgCols + 2);
      const bool ok = e < kXItems && yy >= 0 && yy < H && xx >= 0 && xx < W;
      const long long pix = ok ? (n * H + yy) * W + xx : 0;
      vx[k] = *reinterpret_cast<const u32x4*>(x + pix * ldx + ci0 + (ok ? c8 : 0));
      okx |= (ok ? 1u : 0u) << k;
    }
  };
  // dy[y0 + r][x0 + c][co0 + ch] -> sdy[ch][r][c]; x[y0 - 1 + rr][x0 - 1 + pc]
  // [ci0 + ch] -> sx[s][ch][rr][pc - s] for the shifts s = 0, 1, 2 whose
  // column pc - s lies in [0, 32).  Lanes 2i and 2i + 1 hold two neighbouring
  // pixels of one row (the rows' widths are even) with the same 8 channels;
  // they swap half their channels (one DPP exchange per 2 words) so that
  // each holds 4 channels of both pixels, written as 4-byte pixel pairs
  // (shifts 0 and 2, whose pairs start on even columns; shift 1 keeps
  // 2-byte stores of the lane's own pixel).
  static_assert(kDyItems % 256 == 0, "every dy item of a tile is in use");
  const int odd = threadIdx.x & 1;
  auto pair_up = [&](const u32x4& v, bool ok, uint32_t (&o)[4]) {
    // o[i]: channel 4 * odd + i of the pixel pair (even pixel in the low half)
    const uint32_t w0 = ok ? v[0] : 0u, w1 = ok ? v[1] : 0u, w2 = ok ? v[2] : 0u, w3 = ok ? v[3] : 0u;
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_mov_dpp((int)(odd ? w0 : w2), 0xB1, 0xF, 0xF, true);
    const uint32_t r1 = (uint32_t)__builtin_amdgcn_mov_dpp((int)(odd ? w1 : w3), 0xB1, 0xF, 0xF, true);
    const uint32_t a0 = odd ? r0 : w0, b0 = odd ? w2 : r0, a1 = odd ? r1 : w1, b1 = odd ? w3 : r1;
    o[0] = __builtin_amdgcn_perm(b0, a0, 0x05040100u);
    o[1] = __builtin_amdgcn_perm(b0, a0, 0x07060302u);
    o[2] = __builtin_amdgcn_perm(b1, a1, 0x05040100u);
    o[3] = __builtin_amdgcn_perm(b1, a1, 0x07060302u);
  };
  auto store_tile = [&]() {
#pragma unroll
    for (int k = 0; k < kDyPer; ++k) {
      const int e = threadIdx.x + 256 * k;
      const int px = e % (kWgRows * kWgCols), c8 = (e / (kWgRows * kWgCols)) * 8;
      uint32_t o[4];
      pair_up(vdy[k], (okdy >> k) & 1u, o);
      const int pe = px & ~1;
      uint16_t* d = sdy + (c8 + 4 * odd) * kWgDyStride + (pe / kWgCols) * kWgRowStride + pe % kWgCols;
#pragma unroll
      for (int i = 0; i < 4; ++i) *reinterpret_cast<uint32_t*>(d + i * kWgDyStride) = o[i];
    }
#pragma unroll
    for (int k = 0; k < kXPer; ++k) {
      const int e = threadIdx.x + 256 * k;
      const int px = e % kXPix, c8 = (e / kXPix) * 8;
      const int rr = px / (kWgCols + 2), pc = px % (kWgCols + 2);
      const bool ok = (okx >> k) & 1u;
      uint32_t o[4];
      pair_up(vx[k], ok, o);  // (all lanes, before any skip)
      if (e >= kXItems) continue;
      const int pe = pc & ~1;
#pragma unroll
      for (int sh = 0; sh < 3; sh += 2) {
        const int c = pe - sh;
        if (c < 0 || c >= kWgCols) continue;
        uint16_t* d = sx + (sh * kWgTci + c8 + 4 * odd) * kWgXStride + rr * kWgRowStride + c;
#pragma unroll
        for (int i = 0; i < 4; ++i) *reinterpret_cast<uint32_t*>(d + i * kWgXStride) = o[i];
      }
      const int c = pc - 1;
      if (c < 0 || c >= kWgCols) continue;
      uint16_t* d = sx + (kWgTci + c8) * kWgXStride + rr * kWgRowStride + c;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t w = ok ? vx[k][j] : 0u;
        d[(2 * j) * kWgXStride] = (uint16_t)(w & 0xFFFFu);
        d[(2 * j + 1) * kWgXStride] = (uint16_t)(w >> 16);
      }
    }
  };

  if (t0 < t1) load_tile(t0);
  for (long long tile = t0; tile < t1; ++tile) {
    __syncthreads();  // the previous tile's fragments have been read
    store_tile();
    __syncthreads();
    if (tile + 1 < t1) load_tile(tile + 1);
#pragma unroll
    for (int r = 0; r < kWgRows; ++r) {
      u32x4 a[CPW];
#pragma unroll
      for (int i = 0; i < CPW; ++i)
        a[i] = *reinterpret_cast<const u32x4*>(&sdy[((cog * CPW + i) * 16 + (lane & 15)) * kWgDyStride +
                                                    r * kWgRowStride + kg]);
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const int ty = t / 3, tx = t % 3;
        const u32x4 b = *reinterpret_cast<const u32x4*>(
            &sx[(tx * kWgTci + cit * 16 + (lane & 15)) * kWgXStride + (r + ty) * kWgRowStride + kg]);
#pragma unroll
        for (int i = 0; i < CPW; ++i)
          acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a[i]), as_bf16x8(b), acc[i][t], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    float* out = ws + ((long long)chunk * 9 + t) * Cout * Cin;
#pragma unroll
    for (int i = 0; i < CPW; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int co = co0 + (cog * CPW + i) * 16 + (lane >> 4) * 4 + r;
        const int ci = ci0 + cit * 16 + (lane & 15);
        out[(long long)co * Cin + ci] = acc[i][t][r];
      }
  }
}

// The chunk partial sums ws[c][i] (c < nchunks, i < n) added in a fixed
// order in two steps, so the result does not depend on scheduling: first
// each group of kSumGroup consecutive chunks into the group's first slot (in
// place), then the groups' sums in order.  The first step's loads are
// independent, so they are in flight together.
constexpr int kSumGroup = 16;

__global__ void sum_chunk_groups_kernel(float* __restrict__ ws, int nchunks, long long n) {
  const int ngroups = (nchunks + kSumGroup - 1) / kSumGroup;
  for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < n * ngroups;
       j += (long long)gridDim.x * blockDim.x) {
    const int g = (int)(j / n);
    const long long i = j - (long long)g * n;
    const int c0 = g * kSumGroup, cn = nchunks - c0 < kSumGroup ? nchunks - c0 : kSumGroup;
    float v[kSumGroup];
#pragma unroll
    for (int c = 0; c < kSumGroup; ++c) v[c] = c < cn ? ws[(long long)(c0 + c) * n + i] : 0.0f;
    float s = v[0];
#pragma unroll
    for (int c = 1; c < kSumGroup; ++c)
      if (c < cn) s += v[c];
    ws[(long long)c0 * n + i] = s;
  }
}

__global__ void sum_chunks_kernel(const float* __restrict__ ws, int nchunks, long long n, float* __restrict__ out) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int c = 0; c < nchunks; c += kSumGroup) s += ws[(long long)c * n + i];  // fixed order: deterministic
    out[i] = s;
  }
}

// --------------------------------------------------------------- weights --
// Master [9][cout][cin] FP32 -> bf16 forward copy (same layout) and backward
// copy [9][cin][cout] with the taps flipped (tap 8 - t), which turns the input
// gradient into a plain 3x3 convolution of the output gradient.
__global__ void pack_weights_kernel(const float* __restrict__ w, int cin, int cout, uint16_t* __restrict__ wf,
                                    uint16_t* __restrict__ wb) {
  const long long n = 9LL * cin * cout;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int t = (int)(i / ((long long)cin * cout));
    const int rem = (int)(i - (long long)t * cin * cout);
    const int co = rem / cin, ci = rem % cin;
    const uint16_t h = to_bf16(w[i]);
    wf[i] = h;
    if (wb) wb[((long long)(8 - t) * cin + ci) * cout + co] = h;
  }
}

// All layers of a model in one launch: element i of the concatenated FP32
// masters belongs to the layer whose [off[l], off[l + 1]) holds it, and is
// packed as pack_weights_kernel packs it.
struct PackTable {
  long long off[kPackMaxLayers + 1];
  int cin[kPackMaxLayers], cout[kPackMaxLayers];
  int layers;
};

__global__ void pack_model_kernel(const float* __restrict__ w, PackTable tab, uint16_t* __restrict__ wf,
                                  uint16_t* __restrict__ wb) {
  const long long n = tab.off[tab.layers];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    int l = 0;
    while (l + 1 < tab.layers && tab.off[l + 1] <= i) ++l;
    const int cin = tab.cin[l], cout = tab.cout[l];
    const long long j = i - tab.off[l];
    const int t = (int)(j / ((long long)cin * cout));
    const int rem = (int)(j - (long long)t * cin * cout);
    const int co = rem / cin, ci = rem % cin;
    const uint16_t h = to_bf16(w[i]);
    wf[i] = h;
    if (wb) wb[tab.off[l] + ((long long)(8 - t) * cin + ci) * cout + co] = h;
  }
}

// ------------------------------------------------------- pool / upsample --
// h, w: the full-resolution size (pool input / upsample output).
__global__ void avgpool2_kernel(const uint16_t* __restrict__ x, int ldx, int N, int h, int w, int c,
                                uint16_t* __restrict__ y, int ldy) {
  const int ho = h / 2, wo = w / 2;
  const long long n = (long long)N * ho * wo * c;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % c);
    long long q = i / c;
    const int j = (int)(q % wo);
    q /= wo;
    const int ii = (int)(q % ho);
    const int nn = (int)(q / ho);
    const long long b = ((long long)nn * h + 2 * ii) * w + 2 * j;
    const float s = (from_bf16(x[b * ldx + ch]) + from_bf16(x[(b + 1) * ldx + ch])) +
                    (from_bf16(x[(b + w) * ldx + ch]) + from_bf16(x[(b + w + 1) * ldx + ch]));
    y[(((long long)nn * ho + ii) * wo + j) * ldy + ch] = to_bf16(s * 0.25f);
  }
}

// dx = (pool-gradient of g + addend) * (msrc > 0), at full resolution h x w.
__global__ void avgpool2_grad_kernel(const uint16_t* __restrict__ g, int ldg, const uint16_t* __restrict__ add, int lda,
                                     const uint16_t* __restrict__ msrc, int ldm, int N, int h, int w, int c,
                                     uint16_t* __restrict__ dx, int lddx) {
  const long long n = (long long)N * h * w * c;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % c);
    const long long p = i / c;
    const int xx = (int)(p % w);
    const long long q = p / w;
    const int yy = (int)(q % h);
    const int nn = (int)(q / h);
    const long long pg = ((long long)nn * (h / 2) + yy / 2) * (w / 2) + xx / 2;
    float v = from_bf16(g[pg * ldg + ch]) * 0.25f;
    if (add) v += from_bf16(add[p * lda + ch]);
    if (msrc && !(from_bf16(msrc[p * ldm + ch]) > 0.0f)) v = 0.0f;
    dx[p * lddx + ch] = to_bf16(v);
  }
}

// h, w: the half-resolution size (upsample input / gradient output).
__global__ void upsample2_kernel(const uint16_t* __restrict__ x, int ldx, int N, int h, int w, int c,
                                 uint16_t* __restrict__ y, int ldy) {
  const long long n = (long long)N * 4 * h * w * c;
  const int W2 = 2 * w;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % c);
    const long long p = i / c;
    const int xx = (int)(p % W2);
    const long long q = p / W2;
    const int yy = (int)(q % (2 * h));
    const int nn = (int)(q / (2 * h));
    y[p * ldy + ch] = x[(((long long)nn * h + yy / 2) * w + xx / 2) * ldx + ch];
  }
}

__global__ void upsample2_grad_kernel(const uint16_t* __restrict__ g, int ldg, int N, int h, int w, int c,
                                      uint16_t* __restrict__ dx, int lddx) {
  const long long n = (long long)N * h * w * c;
  const int W2 = 2 * w;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % c);
    const long long p = i / c;
    const int xx = (int)(p % w);
    const long long q = p / w;
    const int yy = (int)(q % h);
    const int nn = (int)(q / h);
    const long long b = ((long long)nn * 2 * h + 2 * yy) * W2 + 2 * xx;
    const float s = (from_bf16(g[b * ldg + ch]) + from_bf16(g[(b + 1) * ldg + ch])) +
                    (from_bf16(g[(b + W2) * ldg + ch]) + from_bf16(g[(b + W2 + 1) * ldg + ch]));
    dx[p * lddx + ch] = to_bf16(s);
  }
}

// Eight channels (16 bytes) per thread: the same arithmetic per element as
// the kernels above, used when channel counts and strides are multiples of 8.
__device__ __forceinline__ float lo_bf(uint32_t v) { return __uint_as_float(v << 16); }
__device__ __forceinline__ float hi_bf(uint32_t v) { return __uint_as_float(v & 0xFFFF0000u); }
__device__ __forceinline__ uint32_t pack_bf(float a, float b) { return to_bf16x2(a, b); }

__global__ void avgpool2_v8_kernel(const uint16_t* __restrict__ x, int ldx, int N, int h, int w, int c,
                                   uint16_t* __restrict__ y, int ldy) {
  const int ho = h / 2, wo = w / 2, c8 = c / 8;
  const long long n = (long long)N * ho * wo * c8;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % c8) * 8;
    long long q = i / c8;
    const int j = (int)(q % wo);
    q /= wo;
    const int ii = (int)(q % ho);
    const int nn = (int)(q / ho);
    const long long b = ((long long)nn * h + 2 * ii) * w + 2 * j;
    const u32x4 a = *reinterpret_cast<const u32x4*>(x + b * ldx + ch);
    const u32x4 bb = *reinterpret_cast<const u32x4*>(x + (b + 1) * ldx + ch);
    const u32x4 cc = *reinterpret_cast<const u32x4*>(x + (b + w) * ldx + ch);
    const u32x4 d = *reinterpret_cast<const u32x4*>(x + (b + w + 1) * ldx + ch);
    u32x4 o;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float sl = (lo_bf(a[k]) + lo_bf(bb[k])) + (lo_bf(cc[k]) + lo_bf(d[k]));
      const float sh = (hi_bf(a[k]) + hi_bf(bb[k])) + (hi_bf(cc[k]) + hi_bf(d[k]));
      o[k] = pack_bf(sl * 0.25f, sh * 0.25f);
    }
    *reinterpret_cast<u32x4*>(y + (((long long)nn * ho + ii) * wo + j) * ldy + ch) = o;
  }
}

__global__ void avgpool2_grad_v8_kernel(const uint16_t* __restrict__ g, int ldg, const uint16_t* __restrict__ add,
                                        int lda, const uint16_t* __restrict__ msrc, int ldm, int N, int h, int w, int c,
                                        uint16_t* __restrict__ dx, int lddx) {
  const int c8 = c / 8;
  const long long n = (long long)N * h * w * c8;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % c8) * 8;
    const long long p = i / c8;
    const int xx = (int)(p % w);
    const long long q = p / w;
    const int yy = (int)(q % h);
    const int nn = (int)(q / h);
    const long long pg = ((long long)nn * (h / 2) + yy / 2) * (w / 2) + xx / 2;
    const u32x4 gv = *reinterpret_cast<const u32x4*>(g + pg * ldg + ch);
    u32x4 av = {0u, 0u, 0u, 0u}, mv = {0u, 0u, 0u, 0u};
    if (add) av = *reinterpret_cast<const u32x4*>(add + p * lda + ch);
    if (msrc) mv = *reinterpret_cast<const u32x4*>(msrc + p * ldm + ch);
    u32x4 o;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float vl = lo_bf(gv[k]) * 0.25f, vh = hi_bf(gv[k]) * 0.25f;
      if (add) {
        vl += lo_bf(av[k]);
        vh += hi_bf(av[k]);
      }
      if (msrc) {
        if (!(lo_bf(mv[k]) > 0.0f)) vl = 0.0f;
        if (!(hi_bf(mv[k]) > 0.0f)) vh = 0.0f;
      }
      o[k] = pack_bf(vl, vh);
    }
    *reinterpret_cast<u32x4*>(dx + p * lddx + ch) = o;
  }
}

__global__ void upsample2_v8_kernel(const uint16_t* __restrict__ x, int ldx, int N, int h, int w, int c,
                                    uint16_t* __restrict__ y, int ldy) {
  const int c8 = c / 8, W2 = 2 * w;
  const long long n = (long long)N * 4 * h * w * c8;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % c8) * 8;
    const long long p = i / c8;
    const int xx = (int)(p % W2);
    const long long q = p / W2;
    const int yy = (int)(q % (2 * h));
    const int nn = (int)(q / (2 * h));
    *reinterpret_cast<u32x4*>(y + p * ldy + ch) =
        *reinterpret_cast<const u32x4*>(x + (((long long)nn * h + yy / 2) * w + xx / 2) * ldx + ch);
  }
}

__global__ void upsample2_grad_v8_kernel(const uint16_t* __restrict__ g, int ldg, int N, int h, int w, int c,
                                         uint16_t* __restrict__ dx, int lddx) {
  const int c8 = c / 8, W2 = 2 * w;
  const long long n = (long long)N * h * w * c8;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % c8) * 8;
    const long long p = i / c8;
    const int xx = (int)(p % w);
    const long long q = p / w;
    const int yy = (int)(q % h);
    const int nn = (int)(q / h);
    const long long b = ((long long)nn * 2 * h + 2 * yy) * W2 + 2 * xx;
    const u32x4 a = *reinterpret_cast<const u32x4*>(g + b * ldg + ch);
    const u32x4 bb = *reinterpret_cast<const u32x4*>(g + (b + 1) * ldg + ch);
    const u32x4 cc = *reinterpret_cast<const u32x4*>(g + (b + W2) * ldg + ch);
    const u32x4 d = *reinterpret_cast<const u32x4*>(g + (b + W2 + 1) * ldg + ch);
    u32x4 o;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float sl = (lo_bf(a[k]) + lo_bf(bb[k])) + (lo_bf(cc[k]) + lo_bf(d[k]));
      const float sh = (hi_bf(a[k]) + hi_bf(bb[k])) + (hi_bf(cc[k]) + hi_bf(d[k]));
      o[k] = pack_bf(sl, sh);
    }
    *reinterpret_cast<u32x4*>(dx + p * lddx + ch) = o;
  }
}

// --------------------------------------------------- input, loss, output --

// Network input, 32 channels: R, G, B / 255, hole (mask != 0), log-depth in
// [log 0.3, log 50] -> [0, 1] (clamped; +inf and NaN -> 1), then zeros.
__global__ void unet_input_kernel(const uint32_t* __restrict__ rgba, const float* __restrict__ depth,
                                  const uint8_t* __restrict__ mask, long long npix, uint16_t* __restrict__ x) {
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (long long)gridDim.x * blockDim.x) {
    const u32x4 w0 = input_channels(rgba[p], depth[p], mask[p]);
    u32x4 zero = {0u, 0u, 0u, 0u};
    u32x4* dst = reinterpret_cast<u32x4*>(x + p * 32);
    dst[0] = w0;
    dst[1] = zero;
    dst[2] = zero;
    dst[3] = zero;
  }
}

// Hole pixels (mask != 0): 16 mask bytes per load (VEC, mask 16-byte
// aligned), a block-wide sum, one atomic per block (integer: the order does
// not matter).
template <bool VEC>
__global__ __launch_bounds__(256) void count_holes_kernel(const uint8_t* __restrict__ mask, long long npix,
                                                          unsigned int* __restrict__ out) {
  __shared__ unsigned int part[4];
  unsigned int c = 0;
  const long long nv = VEC ? npix >> 4 : 0;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (long long)gridDim.x * blockDim.x) {
    const u32x4 q = *reinterpret_cast<const u32x4*>(mask + (v << 4));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t w = q[k];
      c += ((w & 0xFFu) != 0) + ((w & 0xFF00u) != 0) + ((w & 0xFF0000u) != 0) + ((w >> 24) != 0);
    }
  }
  if (VEC) {
    if (blockIdx.x == 0)
      for (long long p = (nv << 4) + threadIdx.x; p < npix; p += blockDim.x) c += mask[p] != 0;
  } else {
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (long long)gridDim.x * blockDim.x)
      c += mask[p] != 0;
  }
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, part[0] + part[1] + part[2] + part[3]);
}

__global__ void zero_u32_kernel(unsigned int* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// Masked L1: per-block partial sums of |plain/255 + res - target/255| over
// hole pixels and RGB, and the gradient d(loss)/d(res) (bf16, 32 channels:
// the head convolution is padded to 32 outputs).
constexpr int kLossThreads = 256;
__global__ __launch_bounds__(kLossThreads) void l1_grad_kernel(const float* __restrict__ res,
                                                               const uint32_t* __restrict__ rgba,
                                                               const uint8_t* __restrict__ mask,
                                                               const uint32_t* __restrict__ target, long long npix,
                                                               const unsigned int* __restrict__ nholes,
                                                               uint16_t* __restrict__ g, float* __restrict__ partial) {
  __shared__ float red[kLossThreads];
  const unsigned int nh = *nholes;
  const float scale = nh ? 1.0f / (3.0f * (float)nh) : 0.0f;
  float acc = 0.0f;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (long long)gridDim.x * blockDim.x) {
    uint16_t gv[3] = {0, 0, 0};
    if (mask[p] != 0) {
      const uint32_t c = rgba[p], tg = target[p];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float pred = (float)((c >> (8 * k)) & 255u) / 255.0f + res[p * 3 + k];
        const float d = pred - (float)((tg >> (8 * k)) & 255u) / 255.0f;
        acc += fabsf(d);
        gv[k] = to_bf16(d > 0.0f ? scale : (d < 0.0f ? -scale : 0.0f));
      }
    }
    u32x4 w0 = {(uint32_t)gv[0] | ((uint32_t)gv[1] << 16), (uint32_t)gv[2], 0u, 0u};
    u32x4 zero = {0u, 0u, 0u, 0u};
    u32x4* dst = reinterpret_cast<u32x4*>(g + p * 32);
    dst[0] = w0;
    dst[1] = zero;
    dst[2] = zero;
    dst[3] = zero;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kLossThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void l1_finish_kernel(const float* __restrict__ partial, int nblocks, const unsigned int* __restrict__ nholes,
                                 float* __restrict__ loss) {
  if (threadIdx.x == 0) {
    float s = 0.0f;
    for (int b = 0; b < nblocks; ++b) s += partial[b];  // fixed order
    const unsigned int nh = *nholes;
    *loss = nh ? s / (3.0f * (float)nh) : 0.0f;
  }
}

// Hole pixels: u8 = clamp(rint(255 * (plain/255 + res))); others copied.
__global__ void composite_kernel(const float* __restrict__ res, const uint32_t* __restrict__ rgba,
                                 const uint8_t* __restrict__ mask, long long npix, uint32_t* __restrict__ out) {
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (long long)gridDim.x * blockDim.x) {
    const uint32_t c = rgba[p];
    uint32_t o = c;
    if (mask[p] != 0) {
      o = c & 0xFF000000u;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float pred = (float)((c >> (8 * k)) & 255u) / 255.0f + res[p * 3 + k];
        float q = rintf(255.0f * pred);
        q = q < 0.0f ? 0.0f : (q > 255.0f ? 255.0f : q);
        o |= (uint32_t)q << (8 * k);
      }
    }
    out[p] = o;
  }
}

// AdamW (decoupled weight decay, bias-corrected moments), FP32, elementwise.
__global__ void adamw_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                             const float* __restrict__ g, long long n, float lr, float b1, float b2, float eps, float wd,
                             float c1, float c2) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    float wi = w[i] * (1.0f - lr * wd);
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    wi -= lr * mh / (sqrtf(vh) + eps);
    w[i] = wi;
  }
}

// ------------------------------------------------------------ hole tiles --
// counts[ty * ntx + tx] = number of pixels with mask != 0 in the tile x tile
// block at (tx, ty) (clipped to the frame).
__global__ __launch_bounds__(256) void tile_holes_kernel(const uint8_t* __restrict__ mask, int w, int h, int tile,
                                                         int ntx, uint32_t* __restrict__ counts) {
  __shared__ uint32_t part[4];
  const int tx = blockIdx.x % ntx, ty = blockIdx.x / ntx;
  const int x0 = tx * tile, y0 = ty * tile;
  const int x1 = min(x0 + tile, w), y1 = min(y0 + tile, h);
  uint32_t c = 0;
  for (int y = y0 + (int)threadIdx.y; y < y1; y += blockDim.y)
    for (int x = x0 + (int)threadIdx.x; x < x1; x += blockDim.x) c += mask[(long long)y * w + x] != 0;
  // blockDim = (64, 4): one wave per threadIdx.y.
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if (threadIdx.x == 0) part[threadIdx.y] = c;
  __syncthreads();
  if (threadIdx.x == 0 && threadIdx.y == 0) counts[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// plan[4k .. 4k+3] = (crop x, crop y, tile x, tile y) of crop k.  Copies crop k
// (crop x crop pixels) of a frame into the crop batch.
__global__ void gather_crops_kernel(const uint32_t* __restrict__ rgba, const float* __restrict__ depth,
                                    const uint8_t* __restrict__ mask, int w, const int* __restrict__ plan, int crop,
                                    uint32_t* __restrict__ crgba, float* __restrict__ cdepth,
                                    uint8_t* __restrict__ cmask) {
  const int k = blockIdx.y;
  const int ox = plan[4 * k], oy = plan[4 * k + 1];
  const long long n = (long long)crop * crop;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int cy = (int)(i / crop), cx = (int)(i % crop);
    const long long src = (long long)(oy + cy) * w + (ox + cx);
    const long long dst = (long long)k * n + i;
    crgba[dst] = rgba[src];
    cdepth[dst] = depth[src];
    cmask[dst] = mask[src];
  }
}

// Writes the tile part of each crop's learned composite into the frame: hole
// pixels of tile k become clamp(rint(255 * (plain/255 + res))), alpha kept;
// other pixels are left as they are.
__global__ void composite_tiles_kernel(const float* __restrict__ res, const int* __restrict__ plan, int crop, int tile,
                                       int w, int h, const uint32_t* __restrict__ rgba,
                                       const uint8_t* __restrict__ mask, uint32_t* __restrict__ out) {
  const int k = blockIdx.y;
  const int ox = plan[4 * k], oy = plan[4 * k + 1];
  const int tx = plan[4 * k + 2], ty = plan[4 * k + 3];
  const long long n = (long long)tile * tile;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int x = tx + (int)(i % tile), y = ty + (int)(i / tile);
    if (x >= w || y >= h) continue;
    const long long p = (long long)y * w + x;
    if (mask[p] == 0) continue;
    const long long q = ((long long)k * crop + (y - oy)) * crop + (x - ox);
    const uint32_t c = rgba[p];
    uint32_t o = c & 0xFF000000u;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float pred = (float)((c >> (8 * ch)) & 255u) / 255.0f + res[q * 3 + ch];
      float v = rintf(255.0f * pred);
      v = v < 0.0f ? 0.0f : (v > 255.0f ? 255.0f : v);
      o |= (uint32_t)v << (8 * ch);
    }
    out[p] = o;
  }
}

int grid_1d(long long n, int threads) {
  const long long g = (n + threads - 1) / threads;
  return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

}  // namespace

// ------------------------------------------------------------- launchers --
namespace {
// Compute units of the current device and resident convolution workgroups
// per CU, queried once.
int device_cus() {
  static const int c = [] {
    int d = 0, v = 0;
    if (hipGetDevice(&d) != hipSuccess || hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess)
      v = 0;
    return v > 0 ? v : 256;
  }();
  return c;
}

template <int CT, bool RAW, int NW = 1>
int conv_blocks_per_cu() {
  static const int nb = [] {
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, conv3x3_tiled_kernel<CT, RAW, NW>, kConvThreads, 0) != hipSuccess)
      v = 0;
    return v > 0 ? v : 1;
  }();
  return nb;
}

hipError_t conv3x3_launch(const uint16_t* x, int ldx, int N, int H, int W, int Cin, const uint16_t* wgt, int Cout,
                          void* y, int ldy, int y_fp32, int cout_store, int epi, const uint16_t* msrc, int ldm, int ups,
                          hipStream_t s, bool persistent, uint16_t* pool = nullptr, int ldp = 0,
                          const uint32_t* raw_rgba = nullptr, const float* raw_depth = nullptr,
                          const uint8_t* raw_mask = nullptr, long long xcs = 32) {
  const long long tiles = (long long)N * ((H + kTileH - 1) / kTileH) * ((W + kTileW - 1) / kTileW);
  if (tiles > 0x7FFFFFFFLL) return hipErrorInvalidValue;
  const int nt = (int)tiles;
  // A persistent grid: the workgroups that fit at once (over the ny blocks of
  // output channels), a multiple of 8, each looping over tiles; its next
  // item's patch loads overlap the current item's MFMAs across tiles too.
  // Otherwise one workgroup per tile: compute units then free up tile by
  // tile, so kernels on other queues get them within a tile's time rather
  // than at the end of the layer.
  auto grid_x = [&](int per_cu, int ny) -> unsigned {
    if (!persistent) return (unsigned)nt;
    const long long g = ((long long)device_cus() * per_cu / ny) & ~7LL;
    return (unsigned)(g >= 8 && g < nt ? g : nt);
  };
  if (raw_rgba) {  // the first layer (Cin 32, Cout a multiple of 32)
    if (Cin != 32 || Cout % 32 != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL((conv3x3_tiled_kernel<32, true>), dim3(grid_x(conv_blocks_per_cu<32, true>(), Cout / 32), Cout / 32),
                       dim3(kConvThreads), 0, s, x, ldx, xcs, N, H, W, Cin, wgt, Cout, y, ldy, y_fp32, cout_store, epi,
                       msrc, ldm, ups, nt, pool, ldp, raw_rgba, raw_depth, raw_mask);
  } else if (cout_store <= 16) {  // e.g. the 3-channel head: only the first 16 outputs are computed
    hipLaunchKernelGGL((conv3x3_tiled_kernel<16, false>), dim3(grid_x(conv_blocks_per_cu<16, false>(), 1), 1),
                       dim3(kConvThreads), 0, s, x, ldx, xcs, N, H, W, Cin, wgt, Cout, y, ldy, y_fp32, cout_store, epi,
                       msrc, ldm, ups, nt, pool, ldp, raw_rgba, raw_depth, raw_mask);
  } else if (Cout % 64 == 0) {
    hipLaunchKernelGGL((conv3x3_tiled_kernel<64, false>), dim3(grid_x(conv_blocks_per_cu<64, false>(), Cout / 64), Cout / 64),
                       dim3(kConvThreads), 0, s, x, ldx, xcs, N, H, W, Cin, wgt, Cout, y, ldy, y_fp32, cout_store, epi,
                       msrc, ldm, ups, nt, pool, ldp, raw_rgba, raw_depth, raw_mask);
  } else if (Cin == 64) {  // both input chunks' weights resident
    hipLaunchKernelGGL((conv3x3_tiled_kernel<32, false, 2>),
                       dim3(grid_x(conv_blocks_per_cu<32, false, 2>(), Cout / 32), Cout / 32), dim3(kConvThreads), 0,
                       s, x, ldx, xcs, N, H, W, Cin, wgt, Cout, y, ldy, y_fp32, cout_store, epi, msrc, ldm, ups, nt, pool,
                       ldp, raw_rgba, raw_depth, raw_mask);
  } else {
    hipLaunchKernelGGL((conv3x3_tiled_kernel<32, false>), dim3(grid_x(conv_blocks_per_cu<32, false>(), Cout / 32), Cout / 32),
                       dim3(kConvThreads), 0, s, x, ldx, xcs, N, H, W, Cin, wgt, Cout, y, ldy, y_fp32, cout_store, epi,
                       msrc, ldm, ups, nt, pool, ldp, raw_rgba, raw_depth, raw_mask);
  }
  return hipGetLastError();
}
}  // namespace

hipError_t nn_conv3x3(const uint16_t* x, int ldx, int N, int H, int W, int Cin, const uint16_t* wgt, int Cout, void* y,
                      int ldy, int y_fp32, int cout_store, int epi, const uint16_t* msrc, int ldm, hipStream_t s,
                      bool persistent, long long xcs) {
  if (xcs < 32 || xcs % 8 != 0) return hipErrorInvalidValue;
  return conv3x3_launch(x, ldx, N, H, W, Cin, wgt, Cout, y, ldy, y_fp32, cout_store, epi, msrc, ldm, 0, s, persistent,
                        nullptr, 0, nullptr, nullptr, nullptr, xcs);
}

hipError_t nn_conv3x3_input(const uint32_t* rgba, const float* depth, const uint8_t* mask, int N, int H, int W,
                            const uint16_t* wgt, int Cout, uint16_t* y, int ldy, int relu, hipStream_t s,
                            bool persistent) {
  if (!rgba || !depth || !mask) return hipErrorInvalidValue;
  return conv3x3_launch(nullptr, 32, N, H, W, 32, wgt, Cout, y, ldy, 0, Cout, relu ? 1 : 0, nullptr, 0, 0, s,
                        persistent, nullptr, 0, rgba, depth, mask);
}

hipError_t nn_conv3x3_pool(const uint16_t* x, int ldx, int N, int H, int W, int Cin, const uint16_t* wgt, int Cout,
                           uint16_t* y, int ldy, int relu, uint16_t* pool, int ldp, hipStream_t s, bool persistent) {
  if (H % 2 || W % 2 || !pool) return hipErrorInvalidValue;
  return conv3x3_launch(x, ldx, N, H, W, Cin, wgt, Cout, y, ldy, 0, Cout, relu ? 1 : 0, nullptr, 0, 0, s, persistent,
                        pool, ldp);
}

hipError_t nn_conv3x3_up(const uint16_t* x, int ldx, int N, int H, int W, int Cin, const uint16_t* wgt, int Cout,
                         void* y, int ldy, int y_fp32, int cout_store, int epi, const uint16_t* msrc, int ldm,
                         hipStream_t s, bool persistent) {
  if (H % 2 || W % 2) return hipErrorInvalidValue;
  return conv3x3_launch(x, ldx, N, H, W, Cin, wgt, Cout, y, ldy, y_fp32, cout_store, epi, msrc, ldm, 1, s, persistent);
}

int wgrad_tco(int Cout) { return Cout % 64 == 0 ? 64 : 32; }

long long wgrad_tiles(long long N, int H, int W) {
  return N * ((H + kWgRows - 1) / kWgRows) * ((W + kWgCols - 1) / kWgCols);
}

// Split-K chunks: enough that the grid holds about kWgradGroups workgroups,
// at most one per tile and at most kWgradMaxChunks.
size_t nn_wgrad_chunks(long long N, int H, int W, int Cin, int Cout) {
  const long long tiles = wgrad_tiles(N, H, W);
  const long long blocks = (long long)(Cout / wgrad_tco(Cout)) * (Cin / kWgTci);
  if (tiles <= 0 || blocks <= 0) return 0;
  long long c = (kWgradGroups + blocks - 1) / blocks;
  if (c > tiles) c = tiles;
  if (c > kWgradMaxChunks) c = kWgradMaxChunks;
  return (size_t)(c > 0 ? c : 1);
}

hipError_t nn_conv3x3_wgrad(const uint16_t* x, int ldx, const uint16_t* dy, int lddy, int N, int H, int W, int Cin,
                            int Cout, float* dw, float* ws, hipStream_t s) {
  if (Cin % kWgTci || Cout % 32) return hipErrorInvalidValue;
  const long long tiles = wgrad_tiles(N, H, W);
  const int nchunks = (int)nn_wgrad_chunks(N, H, W, Cin, Cout);
  const int tco = wgrad_tco(Cout);
  const dim3 grid((Cout / tco) * (Cin / kWgTci), nchunks);
  if (tco == 64)
    hipLaunchKernelGGL((conv3x3_wgrad_kernel<64>), grid, dim3(256), 0, s, x, ldx, dy, lddy, H, W, Cin, Cout, tiles,
                       nchunks, ws);
  else
    hipLaunchKernelGGL((conv3x3_wgrad_kernel<32>), grid, dim3(256), 0, s, x, ldx, dy, lddy, H, W, Cin, Cout, tiles,
                       nchunks, ws);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long n = 9LL * Cout * Cin;
  if (nchunks > 1) {
    const long long groups = (nchunks + kSumGroup - 1) / kSumGroup;
    hipLaunchKernelGGL(sum_chunk_groups_kernel, dim3(grid_1d(n * groups, 256)), dim3(256), 0, s, ws, nchunks, n);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(sum_chunks_kernel, dim3(grid_1d(n, 256)), dim3(256), 0, s, ws, nchunks, n, dw);
  return hipGetLastError();
}

hipError_t nn_pack_weights(const float* w, int cin, int cout, uint16_t* wf, uint16_t* wb, hipStream_t s) {
  hipLaunchKernelGGL(pack_weights_kernel, dim3(grid_1d(9LL * cin * cout, 256)), dim3(256), 0, s, w, cin, cout, wf, wb);
  return hipGetLastError();
}

hipError_t nn_pack_model(const float* w, const long long* off, const int* cin, const int* cout, int layers,
                         uint16_t* wf, uint16_t* wb, hipStream_t s) {
  if (layers < 1 || layers > kPackMaxLayers) return hipErrorInvalidValue;
  PackTable tab{};
  for (int l = 0; l < layers; ++l) tab.cin[l] = cin[l], tab.cout[l] = cout[l];
  for (int l = 0; l <= layers; ++l) tab.off[l] = off[l];
  tab.layers = layers;
  hipLaunchKernelGGL(pack_model_kernel, dim3(grid_1d(off[layers], 256)), dim3(256), 0, s, w, tab, wf, wb);
  return hipGetLastError();
}

static bool v8(int c, const void* a, int lda, const void* b, int ldb) {
  return c % 8 == 0 && lda % 8 == 0 && ldb % 8 == 0 && ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15u) == 0;
}

hipError_t nn_avgpool2(const uint16_t* x, int ldx, int N, int h, int w, int c, uint16_t* y, int ldy, hipStream_t s) {
  if (v8(c, x, ldx, y, ldy)) {
    hipLaunchKernelGGL(avgpool2_v8_kernel, dim3(grid_1d((long long)N * (h / 2) * (w / 2) * (c / 8), 256)), dim3(256), 0,
                       s, x, ldx, N, h, w, c, y, ldy);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(avgpool2_kernel, dim3(grid_1d((long long)N * (h / 2) * (w / 2) * c, 256)), dim3(256), 0, s, x, ldx,
                     N, h, w, c, y, ldy);
  return hipGetLastError();
}

hipError_t nn_avgpool2_grad(const uint16_t* g, int ldg, const uint16_t* add, int lda, const uint16_t* msrc, int ldm,
                            int N, int h, int w, int c, uint16_t* dx, int lddx, hipStream_t s) {
  if (v8(c, g, ldg, dx, lddx) && (!add || v8(c, add, lda, add, lda)) && (!msrc || v8(c, msrc, ldm, msrc, ldm))) {
    hipLaunchKernelGGL(avgpool2_grad_v8_kernel, dim3(grid_1d((long long)N * h * w * (c / 8), 256)), dim3(256), 0, s, g,
                       ldg, add, lda, msrc, ldm, N, h, w, c, dx, lddx);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(avgpool2_grad_kernel, dim3(grid_1d((long long)N * h * w * c, 256)), dim3(256), 0, s, g, ldg, add,
                     lda, msrc, ldm, N, h, w, c, dx, lddx);
  return hipGetLastError();
}

hipError_t nn_upsample2(const uint16_t* x, int ldx, int N, int h, int w, int c, uint16_t* y, int ldy, hipStream_t s) {
  if (v8(c, x, ldx, y, ldy)) {
    hipLaunchKernelGGL(upsample2_v8_kernel, dim3(grid_1d((long long)N * 4 * h * w * (c / 8), 256)), dim3(256), 0, s, x,
                       ldx, N, h, w, c, y, ldy);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(upsample2_kernel, dim3(grid_1d((long long)N * 4 * h * w * c, 256)), dim3(256), 0, s, x, ldx, N, h,
                     w, c, y, ldy);
  return hipGetLastError();
}

hipError_t nn_upsample2_grad(const uint16_t* g, int ldg, int N, int h, int w, int c, uint16_t* dx, int lddx,
                             hipStream_t s) {
  if (v8(c, g, ldg, dx, lddx)) {
    hipLaunchKernelGGL(upsample2_grad_v8_kernel, dim3(grid_1d((long long)N * h * w * (c / 8), 256)), dim3(256), 0, s, g,
                       ldg, N, h, w, c, dx, lddx);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(upsample2_grad_kernel, dim3(grid_1d((long long)N * h * w * c, 256)), dim3(256), 0, s, g, ldg, N, h,
                     w, c, dx, lddx);
  return hipGetLastError();
}

hipError_t nn_input(const uint32_t* rgba, const float* depth, const uint8_t* mask, long long npix, uint16_t* x,
                    hipStream_t s) {
  hipLaunchKernelGGL(unet_input_kernel, dim3(grid_1d(npix, 256)), dim3(256), 0, s, rgba, depth, mask, npix, x);
  return hipGetLastError();
}

hipError_t nn_l1_grad(const float* res, const uint32_t* rgba, const uint8_t* mask, const uint32_t* target,
                      long long npix, uint16_t* g, float* loss, float* ws, hipStream_t s) {
  // ws layout: [0] hole count (u32), [16 ..] per-block partial sums.
  unsigned int* cnt = reinterpret_cast<unsigned int*>(ws);
  float* partial = ws + 16;
  hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, s, cnt, 1);
  if ((reinterpret_cast<uintptr_t>(mask) & 15u) == 0) {
    const int cb = grid_1d((npix >> 4) > 0 ? (npix >> 4) : 1, 256);
    hipLaunchKernelGGL(count_holes_kernel<true>, dim3(cb < 256 ? cb : 256), dim3(256), 0, s, mask, npix, cnt);
  } else {
    const int cb = grid_1d(npix, 256);
    hipLaunchKernelGGL(count_holes_kernel<false>, dim3(cb < 256 ? cb : 256), dim3(256), 0, s, mask, npix, cnt);
  }
  const int nb = kLossBlocks;
  hipLaunchKernelGGL(l1_grad_kernel, dim3(nb), dim3(kLossThreads), 0, s, res, rgba, mask, target, npix, cnt, g,
                     partial);
  hipLaunchKernelGGL(l1_finish_kernel, dim3(1), dim3(64), 0, s, partial, nb, cnt, loss);
  return hipGetLastError();
}

hipError_t nn_composite(const float* res, const uint32_t* rgba, const uint8_t* mask, long long npix, uint32_t* out,
                        hipStream_t s) {
  hipLaunchKernelGGL(composite_kernel, dim3(grid_1d(npix, 256)), dim3(256), 0, s, res, rgba, mask, npix, out);
  return hipGetLastError();
}

hipError_t nn_adamw(float* w, float* m, float* v, const float* g, long long n, float lr, float b1, float b2, float eps,
                    float wd, int step, hipStream_t s) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(adamw_kernel, dim3(grid_1d(n, 256)), dim3(256), 0, s, w, m, v, g, n, lr, b1, b2, eps, wd, c1, c2);
  return hipGetLastError();
}

hipError_t nn_tile_holes(const uint8_t* mask, int w, int h, int tile, uint32_t* counts, hipStream_t s) {
  const int ntx = (w + tile - 1) / tile, nty = (h + tile - 1) / tile;
  hipLaunchKernelGGL(tile_holes_kernel, dim3(ntx * nty), dim3(64, 4), 0, s, mask, w, h, tile, ntx, counts);
  return hipGetLastError();
}

hipError_t nn_gather_crops(const uint32_t* rgba, const float* depth, const uint8_t* mask, int w, const int* plan, int k,
                           int crop, uint32_t* crgba, float* cdepth, uint8_t* cmask, hipStream_t s) {
  const long long n = (long long)crop * crop;
  const long long blocks = (n + 255) / 256;
  hipLaunchKernelGGL(gather_crops_kernel, dim3((unsigned)(blocks < 1024 ? blocks : 1024), k), dim3(256), 0, s, rgba,
                     depth, mask, w, plan, crop, crgba, cdepth, cmask);
  return hipGetLastError();
}

hipError_t nn_composite_tiles(const float* res, const int* plan, int k, int crop, int tile, int w, int h,
                              const uint32_t* rgba, const uint8_t* mask, uint32_t* out, hipStream_t s) {
  const long long n = (long long)tile * tile;
  hipLaunchKernelGGL(composite_tiles_kernel, dim3((unsigned)((n + 255) / 256), k), dim3(256), 0, s, res, plan, crop,
                     tile, w, h, rgba, mask, out);
  return hipGetLastError();
}

}  // namespace yoro

// FP64 local energies of the one-hot SiLU model (108 -> 128 -> 128 -> 1) on the FP64 matrix
// cores, 16 rows (sites, each given by its 27 slot species) per half of a 512-thread block.
// Used by the re-decision of near-threshold trials and by the FP64 site energies.
//
// Arithmetic of each row energy:
//   z0[u] = b0[u] + the W0 column of slot m's species, added for m = 0..26 (species 4: none);
//   z1[u] = b1[u] + sum over k = 0..127 of W1[u][k] silu(z0[k]), in 32 steps of 4 inputs;
//   E = b2 + sum over chunks c = 0..7 of (sum over i = 0..15 of W2[16c+i] silu(z1[16c+i])).
// Layout of the 16x16x4 FP64 products: wave v of a half owns units 32v .. 32v + 31 as two
// 16-unit tiles; the 16 rows are the other dimension.  Lane l supplies the weight of unit
// 16T + l % 16 and input 4s + l / 16 and the activation of that input in row l % 16, and
// receives units 16T + l / 16 + 4j, j = 0..3, of row l % 16.
#pragma once
#include "scalar_eval.hpp"

namespace smc {

constexpr int kR64Hid = 128;
constexpr int kR64Rows = 16;                  // rows per half block
constexpr int kR64Threads = 512;              // two halves of four waves
constexpr int kR64Half = kR64Threads / 2;
constexpr int kR64HStride = kR64Hid + 1;      // padded row stride of the activation buffer
constexpr int kR64SpStride = 32;              // bytes per row of slot species (27 used)
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Weights in LDS: W0 and W1 as their FP32 values ([input][unit]; FP64 arithmetic takes them
// exactly), b0, b1 and W2 as FP64.
struct Rows64W {
  float w0[108 * kR64Hid];
  float w1[kR64Hid * kR64Hid];
  double b0[kR64Hid], b1[kR64Hid], w2[kR64Hid];
};

// Per-half buffers in LDS.
struct Rows64Half {
  uint8_t sp[kR64Rows * kR64SpStride];        // slot species of the 16 rows (16-byte aligned)
  double h[kR64Rows * kR64HStride];           // silu(z0), then the W2-weighted silu(z1)
  double part[kR64Rows * 8];                  // chunk sums of the output
};

// Stage the weights (every thread of the block).  w32t: W0, b0, W1, ... in the [input][unit]
// layout as FP32; w64t: the same as FP64 (b0, b1, W2 come from it).  Every load is issued before
// the first LDS store (one memory round trip); mid() runs between the loads and the stores, so
// that a caller's own loads go out with them.
template <typename Mid>
__device__ __forceinline__ void rows64_stage(Rows64W &S, const float *w32t, const double *w64t, Mid mid) {
  constexpr int n0 = 108 * kR64Hid / 4, nw = n0 + kR64Hid * kR64Hid / 4;
  constexpr int per = (nw + kR64Threads - 1) / kR64Threads;
  const int tid = threadIdx.x;
  const double *b0 = w64t + kR64Hid * 108, *b1 = b0 + kR64Hid + kR64Hid * kR64Hid, *W2 = b1 + kR64Hid;
  const float4 *w0 = (const float4 *)w32t;
  const float4 *w1 = (const float4 *)(w32t + kR64Hid * 108 + kR64Hid);
  float4 t[per];
#pragma unroll
  for (int i = 0; i < per; ++i) {
    const int q = tid + i * kR64Threads;
    t[i] = q < n0 ? w0[q] : (q < nw ? w1[q - n0] : make_float4(0.0f, 0.0f, 0.0f, 0.0f));
  }
  const int ub = tid % kR64Hid;
  const double bb = (tid < kR64Hid ? b0 : (tid < 2 * kR64Hid ? b1 : W2))[ub];  // threads past 3 H load W2 unused
  mid();
#pragma unroll
  for (int i = 0; i < per; ++i) {
    const int q = tid + i * kR64Threads;
    if (q < n0) ((float4 *)S.w0)[q] = t[i];
    else if (q < nw) ((float4 *)S.w1)[q - n0] = t[i];
  }
  if (tid < kR64Hid) S.b0[tid] = bb;
  else if (tid < 2 * kR64Hid) S.b1[tid - kR64Hid] = bb;
  else if (tid < 3 * kR64Hid) S.w2[tid - 2 * kR64Hid] = bb;
}

// Energies of the 16 rows of this thread's half (slot species in B.sp, written and ordered by a
// barrier before the call).  Every thread of the block calls it (block-wide barriers); a half
// with live == false computes nothing.  mid() runs after layer 0 (a caller's loads for its next
// item).  Returns row lt's energy in threads lt < 16 of a live half (lt: thread index in the half).
template <typename Mid>
__device__ __forceinline__ double rows64_half(const Rows64W &S, double b2, bool live, int lt, Rows64Half &B,
                                              Mid mid) {
  const int wv = lt >> 6, li = lt & 15, lk = (lt >> 4) & 3;
  double *h = B.h;
  // Layer 0 + activation: the one-hot input of slot m is K-step m (its four channels); a row has
  // at most one non-zero product per K-step (none for species 4) and the others are exact zeros,
  // so every sum is the sequence b0 + the selected W0 columns in slot order, each addition
  // rounded once.
  if (live) {
    const uint4 lo = *(const uint4 *)(B.sp + li * kR64SpStride);
    const uint4 hi = *(const uint4 *)(B.sp + li * kR64SpStride + 16);
    const uint32_t sw[7] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z};
    f64x4 acc[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[t][j] = S.b0[32 * wv + 16 * t + lk + 4 * j];
#pragma unroll
    for (int m = 0; m < 27; ++m) {
      const uint32_t sp = (sw[m >> 2] >> (8 * (m & 3))) & 255u;
      const double b = sp == (uint32_t)lk ? 1.0 : 0.0;
      const float *wr = S.w0 + (4 * m + lk) * kR64Hid + 32 * wv + li;
      acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)wr[0], b, acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)wr[16], b, acc[1], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) h[li * kR64HStride + 32 * wv + 16 * t + lk + 4 * j] = silu<double>(acc[t][j]);
  }
  __syncthreads();
  mid();
  // Layer 1, times W2 after the activation.
  {
    f64x4 acc[2];
    if (live) {
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[t][j] = S.b1[32 * wv + 16 * t + lk + 4 * j];
#pragma unroll 8
      for (int s = 0; s < kR64Hid / 4; ++s) {
        const double b = h[li * kR64HStride + 4 * s + lk];
        const float *wr = S.w1 + (4 * s + lk) * kR64Hid + 32 * wv + li;
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)wr[0], b, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)wr[16], b, acc[1], 0, 0, 0);
      }
    }
    __syncthreads();
    if (live) {
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int u = 32 * wv + 16 * t + lk + 4 * j;
          h[li * kR64HStride + u] = S.w2[u] * silu<double>(acc[t][j]);
        }
    }
  }
  __syncthreads();
  // E = b2 + sum over units in a fixed order: 8 consecutive chunks of 16, then the chunks
  if (live && lt < kR64Rows * 8) {
    const int lr = lt / 8, c = lt % 8;
    double sm = 0.0;
#pragma unroll
    for (int i = 0; i < kR64Hid / 8; ++i) sm += h[lr * kR64HStride + c * (kR64Hid / 8) + i];
    B.part[lt] = sm;
  }
  __syncthreads();
  double E = 0.0;
  if (live && lt < kR64Rows) {
    E = b2;
#pragma unroll
    for (int c = 0; c < 8; ++c) E += B.part[lt * 8 + c];
  }
  return E;
}

}  // namespace smc

// Matrix-core evaluation of the local-energy MLP (108 one-hot inputs -> 128 -> 128 -> 1,
// SiLU) for 32 sites at a time, in FP32, BF16, split BF16 (hi+lo, three products) or
// OCP FP8 E4M3.
//
// Layout.  Every layer is computed transposed, H^T = W . X^T, with the MFMA 32x32xK
// instructions: the A operand holds 32 hidden units of a weight tile (from LDS), the B
// operand holds the activations of 32 sites, one site per lane (mod 32).  The output
// registers of a layer (lane = site, 16 hidden units per lane) are exactly the B operand
// of the next layer once the next layer's weights are packed with the matching K order,
// so activations never leave registers.  A output register v of lane group g = lane/32
// in M-tile T holds hidden unit 32T + 8(v/4) + 4g + (v%4).
//
// SiLU.  With y = -log2(e) z, silu(z) = -ln(2) * y / (1 + 2^y).  The factor -log2(e)
// is folded into W0 and the biases, -ln(2) into the next layer (it cancels against the
// -log2(e) of that layer, log2(e) ln(2) = 1) and into W2, so each activation costs one
// exp2, one add, one reciprocal and one multiply.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smc {

enum { kP32 = 0, kPBF16 = 1, kPBF16X3 = 2, kPFP8 = 3 };

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

constexpr int kHid = 128;
constexpr int kMT = 4;  // M-tiles of 32 hidden units

// Bytes of the packed weights of each precision in LDS (layer 0 then layer 1), followed by
// c0[128], c1[128], w2[128] (floats) and two words of FP8 scale exponents.
template <int P>
struct PackSize;
template <>
struct PackSize<kP32> {
  static constexpr int kL0 = kMT * 14 * 64 * 16;  // 56 K-steps of 2, four per 16-byte read
  static constexpr int kL1 = kMT * 16 * 64 * 16;  // 64 K-steps of 2
};
template <>
struct PackSize<kPBF16> {
  static constexpr int kL0 = kMT * 7 * 64 * 16;   // 7 K-steps of 16 (108 -> 112)
  static constexpr int kL1 = kMT * 8 * 64 * 16;   // 8 K-steps of 16
};
template <>
struct PackSize<kPBF16X3> {
  static constexpr int kL0 = 2 * PackSize<kPBF16>::kL0;  // hi then lo
  static constexpr int kL1 = 2 * PackSize<kPBF16>::kL1;
};
template <>
struct PackSize<kPFP8> {
  static constexpr int kL0 = kMT * 2 * 64 * 32;   // 2 K-steps of 64 (108 -> 128)
  static constexpr int kL1 = kMT * 2 * 64 * 32;
};
template <int P>
constexpr int pack_bytes() {
  return PackSize<P>::kL0 + PackSize<P>::kL1 + 3 * kHid * 4 + 16;
}

// Activation: h' = y / ((1 + 2^y) s); s = 1, or the FP8 activation scale 2^kh so that the
// quantised value is h'/2^kh (folded into the add).
__device__ __forceinline__ float act(float y, float s) {
  const float e = __builtin_amdgcn_exp2f(y);
  return y * __builtin_amdgcn_rcpf(fmaf(e, s, s));
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two floats to two BF16 (round to nearest even) in one packed conversion.
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  const f32x2 v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

__device__ __forceinline__ float bf16_lo_f32(uint32_t w) { return __builtin_bit_cast(float, w << 16); }
__device__ __forceinline__ float bf16_hi_f32(uint32_t w) { return __builtin_bit_cast(float, w & 0xffff0000u); }

// Two activations (folded SiLU, s = 1) split into BF16 hi and lo parts for the split-BF16
// products: x = y * r with r = 1 / (1 + 2^y); hi = bf16(x); lo = bf16(y * r - hi) with the
// product unrounded (one fma).
__device__ __forceinline__ void act_split(float y0, float y1, uint32_t &hi, uint32_t &lo) {
  const float r0 = __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(y0) + 1.0f);
  const float r1 = __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(y1) + 1.0f);
  hi = pack_bf16x2(y0 * r0, y1 * r1);
  lo = pack_bf16x2(fmaf(y0, r0, -bf16_lo_f32(hi)), fmaf(y1, r1, -bf16_hi_f32(hi)));
}

// One-hot of a species id (0..3; 4 and above: no channel) as 4 BF16 values in 2 dwords: BF16 1.0
// shifted to channel p by two 64-bit shifts of 8p bits each (p = 4 shifts it out entirely, where
// a single shift by 64 would not; larger ids count as 4).
__device__ __forceinline__ void onehot_bf16(uint32_t p, uint32_t &lo, uint32_t &hi) {
  const uint32_t sh = (p < 4u ? p : 4u) << 3;
  const uint64_t v = ((uint64_t)0x3F80u << sh) << sh;
  lo = (uint32_t)v;
  hi = (uint32_t)(v >> 32);
}

// One-hot of a species id as 4 FP8 E4M3 bytes in one dword (1.0 = 0x38).
__device__ __forceinline__ uint32_t onehot_fp8(uint32_t p) {
  return (uint32_t)((uint64_t)0x38u << (p << 3));  // p = 4 shifts the byte out
}

struct EvalSmem {
  const uint8_t *w;     // packed weights of the precision
  const float *c0, *c1, *w2;
  float b2;
  int k_scale_a0, k_scale_a1, k_scale_h;  // FP8 E8M0 scale exponents (biased)
  float sh;                                // FP8 activation scale 2^kh
};

// Scheduling hint for one region: kM matrix products, each preceded by up to kD/kM LDS
// reads and followed by up to kV/kM vector ALU instructions, so that one wave's activation
// work issues while its own products run.
template <int kM, int kV, int kD>
__device__ __forceinline__ void interleave() {
  constexpr int v = (kV + kM - 1) / kM, d = (kD + kM - 1) / kM;
  __builtin_amdgcn_sched_group_barrier(0x100, d, 0);
#pragma unroll
  for (int i = 0; i < kM; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x402, v, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, d, 0);
  }
}

// BF16 evaluation, software-pipelined over the four M-tiles of hidden units: while half of
// the activations of layer-0 tile T are turned into the B operands of one layer-1 K-step
// (vector ALU), the wave issues half of the layer-0 products of tile T+1 and the layer-1
// products of the previous K-step (matrix cores); the last-layer activation of output tile
// To - 1 runs while the final layer-1 products of tile To are in flight.  Each accumulator receives its products
// in the same order as in the layer-by-layer evaluation, so the result is identical.  (Split
// BF16 keeps the layer-by-layer order: the pipeline's extra live registers spill in the colour
// kernel and cost more than the overlap gains.)
template <typename GetSlot>
__device__ __forceinline__ float eval_tile_bf16_pipe(const EvalSmem &S, GetSlot get) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 5;
  const i32x4 *A0h = (const i32x4 *)S.w;
  const i32x4 *A1h = (const i32x4 *)(S.w + PackSize<kPBF16>::kL0);

  // layer-0 B operands: K-step s covers features 16s..16s+15; lane group g supplies slots
  // 4s+2g and 4s+2g+1 (slot 27: the constant-one bias input)
  bf16x8 b0[7];
#pragma unroll
  for (int s = 0; s < 7; ++s) {
    const int m0 = 4 * s + 2 * g;
    const uint32_t p0 = (uint32_t)get(m0);
    const uint32_t p1 = (m0 + 1 < 27) ? (uint32_t)get(m0 + 1) : 0u;
    i32x4 bw;
    uint32_t l0, h0, l1, h1;
    onehot_bf16(p0, l0, h0);
    onehot_bf16(p1, l1, h1);
    bw[0] = (int)l0; bw[1] = (int)h0; bw[2] = (int)l1; bw[3] = (int)h1;
    b0[s] = __builtin_bit_cast(bf16x8, bw);
  }
  // layer-0 products of tile T over K-steps s0 <= s < s1
  auto layer0 = [&](int T, int s0, int s1, f32x16 &a) {
#pragma unroll
    for (int s = s0; s < s1; ++s)
      a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, A0h[(T * 7 + s) * 64 + lane]), b0[s], a,
                                                  0, 0, 0);
  };
  // layer-1 B operands of K-step 2T + hh: registers 8hh..8hh+7 of layer-0 tile T
  auto build = [&](const f32x16 &a, int hh, i32x4 &bh) {
#pragma unroll
    for (int q = 0; q < 4; ++q) bh[q] = (int)pack_bf16x2(act(a[8 * hh + 2 * q], 1.0f), act(a[8 * hh + 2 * q + 1], 1.0f));
  };
  f32x16 acc1[kMT];
#pragma unroll
  for (int T = 0; T < kMT; ++T)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const f32x4 b = *(const f32x4 *)(S.c1 + 32 * T + 8 * j + 4 * g);
#pragma unroll
      for (int i = 0; i < 4; ++i) acc1[T][4 * j + i] = b[i];
    }
  // layer-1 K-step s into every output tile
  auto layer1 = [&](int s, const i32x4 &bh) {
    const bf16x8 Bh = __builtin_bit_cast(bf16x8, bh);
#pragma unroll
    for (int To = 0; To < kMT; ++To)
      acc1[To] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, A1h[(To * 8 + s) * 64 + lane]), Bh,
                                                         acc1[To], 0, 0, 0);
  };
  constexpr int kL0H = 4;      // layer-0 products in the first half of a tile
  constexpr int kL1M = 4;      // products (and weight reads) of one layer-1 K-step
  constexpr int kBuildV = 36;  // vector ALU of one build

  // region k = 2T + hh builds the B operands of layer-1 K-step k, issues half of the layer-0
  // products of tile T+1 and the layer-1 products of K-step k-1
  f32x16 a0[2];
#pragma unroll
  for (int v = 0; v < 16; ++v) a0[0][v] = 0.0f;
  layer0(0, 0, 7, a0[0]);
  __builtin_amdgcn_sched_barrier(0);
  i32x4 bh[2];
#pragma unroll
  for (int k = 0; k < 2 * kMT; ++k) {
    const int T = k >> 1, hh = k & 1;
    build(a0[T & 1], hh, bh[k & 1]);
    if (T + 1 < kMT) {
      if (hh == 0) {
#pragma unroll
        for (int v = 0; v < 16; ++v) a0[(T + 1) & 1][v] = 0.0f;
      }
      layer0(T + 1, hh ? 4 : 0, hh ? 7 : 4, a0[(T + 1) & 1]);
    }
    if (k >= 1) layer1(k - 1, bh[(k - 1) & 1]);
    if (k == 0) interleave<kL0H, kBuildV, kL0H>();
    else if (T + 1 < kMT) interleave<kL0H + kL1M, kBuildV, kL0H + kL1M>();
    else interleave<kL1M, kBuildV, kL1M>();
    __builtin_amdgcn_sched_barrier(0);
  }
  // last layer-1 K-step one output tile at a time; activation and output dot product of
  // tile To - 1 alongside
  const bf16x8 Bh7 = __builtin_bit_cast(bf16x8, bh[1]);
  float part = 0.0f;
  auto out_dot = [&](int T) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const f32x4 w = *(const f32x4 *)(S.w2 + 32 * T + 8 * j + 4 * g);
#pragma unroll
      for (int i = 0; i < 4; ++i) part = fmaf(w[i], act(acc1[T][4 * j + i], 1.0f), part);
    }
  };
#pragma unroll
  for (int To = 0; To < kMT; ++To) {
    acc1[To] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, A1h[(To * 8 + 7) * 64 + lane]), Bh7,
                                                       acc1[To], 0, 0, 0);
    if (To >= 1) {
      out_dot(To - 1);
      interleave<1, 16 * 5, 1>();
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  out_dot(kMT - 1);
  const float other = __shfl_xor(part, 32);
  const float p0 = g == 0 ? part : other, p1 = g == 0 ? other : part;
  return S.b2 + (p0 + p1);
}

// Energy of the site held by this lane (lane % 32) of a 32-site tile.  get(m) returns the
// species of feature slot m (0 = centre, 1 + k = neighbour k) of the lane's site; only the
// slots the lane's operands need are requested.  Both lane groups return the same value.
template <int P, typename GetSlot>
__device__ __forceinline__ float eval_tile(const EvalSmem &S, GetSlot get) {
  if constexpr (P == kPBF16) return eval_tile_bf16_pipe(S, get);
  const int lane = threadIdx.x & 63;
  const int g = lane >> 5;
  f32x16 acc[kMT];
  // Layer-0 bias.  FP32/BF16: a weight column fed by a constant-one input in the padding
  // slot 27 (feature 108), so it rides on the matrix cores.  FP8: accumulator
  // initialisation (register v of M-tile T holds hidden 32T + 8(v/4) + 4g + v%4), keeping
  // the bias out of the 3-bit mantissa.
#pragma unroll
  for (int T = 0; T < kMT; ++T)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (P == kPFP8) {
        const f32x4 b = *(const f32x4 *)(S.c0 + 32 * T + 8 * j + 4 * g);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[T][4 * j + i] = b[i];
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[T][4 * j + i] = 0.0f;
      }
    }

  // ---------------------------------------------------------------- layer 0
  if constexpr (P == kP32) {
    // K-step s covers features 2s, 2s+1; lane group g supplies feature 2s + g = slot s/2,
    // channel 2(s%2) + g.
    const f32x4 *A = (const f32x4 *)S.w;
#pragma unroll
    for (int m = 0; m < 28; ++m) {
      const uint32_t p = m < 27 ? (uint32_t)get(m) : 0u;  // slot 27: constant one (bias)
      const float b0 = (p == (uint32_t)g) ? 1.0f : 0.0f;
      const float b1 = (p == (uint32_t)(2 + g)) ? 1.0f : 0.0f;
#pragma unroll
      for (int T = 0; T < kMT; ++T) {
        const f32x4 a = A[(T * 14 + m / 2) * 64 + lane];
        const int o = (m & 1) * 2;
        acc[T] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[o], b0, acc[T], 0, 0, 0);
        acc[T] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[o + 1], b1, acc[T], 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  } else if constexpr (P == kPBF16 || P == kPBF16X3) {
    // K-step s covers features 16s..16s+15; lane group g supplies slots 4s+2g, 4s+2g+1.
    const i32x4 *Ahi = (const i32x4 *)S.w;
    const i32x4 *Alo = (const i32x4 *)(S.w + PackSize<kPBF16>::kL0);
#pragma unroll
    for (int s = 0; s < 7; ++s) {
      const int m0 = 4 * s + 2 * g;
      const uint32_t p0 = (uint32_t)get(m0);
      const uint32_t p1 = (m0 + 1 < 27) ? (uint32_t)get(m0 + 1) : 0u;  // slot 27: bias input
      i32x4 bw;
      uint32_t l0, h0, l1, h1;
      onehot_bf16(p0, l0, h0);
      onehot_bf16(p1, l1, h1);
      bw[0] = (int)l0; bw[1] = (int)h0; bw[2] = (int)l1; bw[3] = (int)h1;
      const bf16x8 b = __builtin_bit_cast(bf16x8, bw);
#pragma unroll
      for (int T = 0; T < kMT; ++T) {
        const bf16x8 ah = __builtin_bit_cast(bf16x8, Ahi[(T * 7 + s) * 64 + lane]);
        acc[T] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, b, acc[T], 0, 0, 0);
        if constexpr (P == kPBF16X3) {
          const bf16x8 al = __builtin_bit_cast(bf16x8, Alo[(T * 7 + s) * 64 + lane]);
          acc[T] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, b, acc[T], 0, 0, 0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
    // FP8: K-step s covers features 64s..64s+63; lane group g supplies slots 16s+8g..+7.
    const i32x8 *A = (const i32x8 *)S.w;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      i32x8 b;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int m = 16 * s + 8 * g + j;
        b[j] = (m < 27) ? (int)onehot_fp8((uint32_t)get(m)) : 0;
      }
#pragma unroll
      for (int T = 0; T < kMT; ++T)
        acc[T] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[(T * 2 + s) * 64 + lane], b, acc[T], 0, 0,
                                                                   0, S.k_scale_a0, 0, 127);
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  // ---------------------------------------------------------------- activation 0
  // and the B operands of layer 1 built from the output registers.
  f32x16 acc1[kMT];
#pragma unroll
  for (int T = 0; T < kMT; ++T)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const f32x4 b = *(const f32x4 *)(S.c1 + 32 * T + 8 * j + 4 * g);
#pragma unroll
      for (int i = 0; i < 4; ++i) acc1[T][4 * j + i] = b[i];
    }

  if constexpr (P == kP32) {
    f32x16 h[kMT];
#pragma unroll
    for (int T = 0; T < kMT; ++T)
#pragma unroll
      for (int v = 0; v < 16; ++v) h[T][v] = act(acc[T][v], 1.0f);
    // K-step s = 16T + v: lane group g supplies its own register v of M-tile T.
    const f32x4 *A = (const f32x4 *)(S.w + PackSize<kP32>::kL0);
#pragma unroll
    for (int T = 0; T < kMT; ++T)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int To = 0; To < kMT; ++To) {
          const f32x4 a = A[(To * 16 + T * 4 + q) * 64 + lane];
#pragma unroll
          for (int i = 0; i < 4; ++i)
            acc1[To] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], h[T][4 * q + i], acc1[To], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
  } else if constexpr (P == kPBF16 || P == kPBF16X3) {
    // K-step s' = 2T + hh takes registers 8hh..8hh+7 of M-tile T.  The B operands of step
    // s'+1 are built before the products of step s' are issued, so that the wave's activation
    // work sits between its matrix products instead of waiting behind them.
    const i32x4 *Ahi = (const i32x4 *)(S.w + (P == kPBF16 ? PackSize<kPBF16>::kL0 : PackSize<kPBF16X3>::kL0));
    const i32x4 *Alo = (const i32x4 *)(S.w + PackSize<kPBF16X3>::kL0 + PackSize<kPBF16>::kL1);
    auto build = [&](int T, int hh, i32x4 &bh, i32x4 &bl) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if constexpr (P == kPBF16X3) {
          uint32_t h, l;
          act_split(acc[T][8 * hh + 2 * q], acc[T][8 * hh + 2 * q + 1], h, l);
          bh[q] = (int)h;
          bl[q] = (int)l;
        } else {
          bh[q] = (int)pack_bf16x2(act(acc[T][8 * hh + 2 * q], 1.0f), act(acc[T][8 * hh + 2 * q + 1], 1.0f));
        }
      }
    };
    i32x4 bh[2], bl[2], bh7, bl7;
    build(0, 0, bh[0], bl[0]);
#pragma unroll
    for (int s = 0; s < 2 * kMT - 2; ++s) {
      const int cur = s & 1;
      build((s + 1) >> 1, (s + 1) & 1, bh[cur ^ 1], bl[cur ^ 1]);
      if (s + 3 == 2 * kMT) build(kMT - 1, 1, bh7, bl7);  // the last K-step too
      const bf16x8 Bh = __builtin_bit_cast(bf16x8, bh[cur]);
      bf16x8 ah[kMT];
#pragma unroll
      for (int To = 0; To < kMT; ++To) {
        ah[To] = __builtin_bit_cast(bf16x8, Ahi[(To * 8 + s) * 64 + lane]);
        acc1[To] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[To], Bh, acc1[To], 0, 0, 0);
      }
      if constexpr (P == kPBF16X3) {
        const bf16x8 Bl = __builtin_bit_cast(bf16x8, bl[cur]);
#pragma unroll
        for (int To = 0; To < kMT; ++To) {
          const bf16x8 al = __builtin_bit_cast(bf16x8, Alo[(To * 8 + s) * 64 + lane]);
          acc1[To] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, Bh, acc1[To], 0, 0, 0);
        }
#pragma unroll
        for (int To = 0; To < kMT; ++To)
          acc1[To] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[To], Bl, acc1[To], 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // the last two K-steps one output tile at a time, with the activation and output dot
    // product of the previous tile alongside (each accumulator keeps its product order)
    const bf16x8 Bh6 = __builtin_bit_cast(bf16x8, bh[0]), Bl6 = __builtin_bit_cast(bf16x8, bl[0]);
    const bf16x8 Bh7 = __builtin_bit_cast(bf16x8, bh7), Bl7 = __builtin_bit_cast(bf16x8, bl7);
    float part = 0.0f;
    auto out_dot = [&](int T) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const f32x4 w = *(const f32x4 *)(S.w2 + 32 * T + 8 * j + 4 * g);
#pragma unroll
        for (int i = 0; i < 4; ++i) part = fmaf(w[i], act(acc1[T][4 * j + i], 1.0f), part);
      }
    };
#pragma unroll
    for (int To = 0; To < kMT; ++To) {
#pragma unroll
      for (int s = 2 * kMT - 2; s < 2 * kMT; ++s) {
        const bf16x8 Bh = s == 2 * kMT - 2 ? Bh6 : Bh7;
        const bf16x8 ah = __builtin_bit_cast(bf16x8, Ahi[(To * 8 + s) * 64 + lane]);
        acc1[To] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, Bh, acc1[To], 0, 0, 0);
        if constexpr (P == kPBF16X3) {
          const bf16x8 al = __builtin_bit_cast(bf16x8, Alo[(To * 8 + s) * 64 + lane]);
          acc1[To] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, Bh, acc1[To], 0, 0, 0);
          acc1[To] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, s == 2 * kMT - 2 ? Bl6 : Bl7, acc1[To], 0, 0, 0);
        }
      }
      if (To >= 1) {
        out_dot(To - 1);
        interleave<P == kPBF16X3 ? 6 : 2, 16 * 5, P == kPBF16X3 ? 4 : 2>();
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    out_dot(kMT - 1);
    const float other = __shfl_xor(part, 32);
    const float q0 = g == 0 ? part : other, q1 = g == 0 ? other : part;
    return S.b2 + (q0 + q1);
  } else {
    // FP8: K-step s' takes M-tiles 2s' and 2s'+1 (16 registers each) of this lane group.
    const i32x8 *A = (const i32x8 *)(S.w + PackSize<kPFP8>::kL0);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      i32x8 b;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int T = 2 * s + j / 4;
        const int v = 4 * (j % 4);
        int w = 0;
        w = __builtin_amdgcn_cvt_pk_fp8_f32(act(acc[T][v], S.sh), act(acc[T][v + 1], S.sh), w, false);
        w = __builtin_amdgcn_cvt_pk_fp8_f32(act(acc[T][v + 2], S.sh), act(acc[T][v + 3], S.sh), w, true);
        b[j] = w;
      }
#pragma unroll
      for (int To = 0; To < kMT; ++To)
        acc1[To] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[(To * 2 + s) * 64 + lane], b, acc1[To], 0, 0,
                                                                     0, S.k_scale_a1, 0, S.k_scale_h);
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  // ---------------------------------------------------------------- activation 1, layer 2
  float part = 0.0f;
#pragma unroll
  for (int T = 0; T < kMT; ++T)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const f32x4 w = *(const f32x4 *)(S.w2 + 32 * T + 8 * j + 4 * g);
#pragma unroll
      for (int i = 0; i < 4; ++i) part = fmaf(w[i], act(acc1[T][4 * j + i], 1.0f), part);
    }
  const float other = __shfl_xor(part, 32);
  const float p0 = g == 0 ? part : other, p1 = g == 0 ? other : part;
  return S.b2 + (p0 + p1);
}

}  // namespace smc

// FCC lattice path: geometry, the MLPNet evaluator on the matrix cores and the per-colour
// phase kernels of a sweep.
//
// Geometry.  Cell (x,y,z) holds four basis sites at doubled coordinates (2x,2y,2z) +
// {(0,0,0), (0,1,1), (1,0,1), (1,1,0)} for b = 0..3; site index s = ((z*Ly + y)*Lx + x)*4 + b;
// periodic modulo 2L per axis.  Neighbour slots: shell 1 (12 vectors, permutations of
// (+-1,+-1,0), distance a/sqrt2), shell 2 (6, (+-2,0,0)), shell 3 (24, permutations of
// (+-2,+-1,+-1)), each shell in lexicographic order of (dx,dy,dz).  The MLPNet reads shells
// 1-2 (the site and 18 neighbours, 76 one-hot inputs); qSRO reads shells 1-3.
//
// MLPNet (Eqs. (4)-(6)): E = W3 . relu(W2 relu(W1 relu(W0 x + b0) + b1) + b2) + b3 with
// 96 units per hidden layer.  Evaluated transposed, 32 sites per tile, exactly like the BCC
// evaluator: three M-tiles of 32 hidden units, the output registers of one layer are the B
// operand of the next, and the layer-0 bias rides on a constant-one input (slot 19,
// feature 76).  ReLU needs no folding of constants.
//
// A sweep runs, per replica and colour: k_propose (Philox proposals, same-species trials
// set aside, active trials appended to a list), k_rows_net / k_rows_qsro (post-swap local
// energies of every zone site of every active trial), k_decide (zone sums against the energy
// cache, Metropolis decision or a place in the FP64 queue, apply) and k_recheck (FP64 zone
// energies before and after for queued trials, decide, apply).
#pragma once
#include "mfma_eval.hpp"
#include "scalar_eval.hpp"
#include "sweep_scalar.hpp"

namespace smc {
namespace fcc {

constexpr int kNbr = 42;        // shells 1-3
constexpr int kNbrMlp = 18;     // shells 1-2
constexpr int kDirs = 12;       // nearest neighbours = swap partners
constexpr int kOmMlp = 28;      // |Omega| with shells 1-2
constexpr int kOmQsro = 60;     // |Omega| with shells 1-3
constexpr int kOmMax = 60;
constexpr int kRegQ = 304;      // read region of a qSRO trial: the zone and its shells 1-3
constexpr int kHid = 96;
constexpr int kMT = 3;          // M-tiles of 32 hidden units
constexpr int kIn = 76;         // 19 slots x 4 channels
constexpr int kSlots = 19;

__host__ __device__ constexpr int8_t dx(int k) {
  constexpr int8_t t[kNbr] = {-1, -1, -1, -1, 0,  0,  0,  0,  1,  1,  1,  1,  -2, 0,
                              0,  0,  0,  2,  -2, -2, -2, -2, -1, -1, -1, -1, -1, -1,
                              -1, -1, 1,  1,  1,  1,  1,  1,  1,  1,  2,  2,  2,  2};
  return t[k];
}
__host__ __device__ constexpr int8_t dy(int k) {
  constexpr int8_t t[kNbr] = {-1, 0,  0,  1,  -1, -1, 1,  1,  -1, 0,  0,  1,  0,  -2,
                              0,  0,  2,  0,  -1, -1, 1,  1,  -2, -2, -1, -1, 1,  1,
                              2,  2,  -2, -2, -1, -1, 1,  1,  2,  2,  -1, -1, 1,  1};
  return t[k];
}
__host__ __device__ constexpr int8_t dz(int k) {
  constexpr int8_t t[kNbr] = {0,  -1, 1,  0,  -1, 1,  -1, 1,  0,  -1, 1,  0,  0,  0,
                              -2, 2,  0,  0,  -1, 1,  -1, 1,  -1, 1,  -2, 2,  -2, 2,
                              -1, 1,  -1, 1,  -2, 2,  -2, 2,  -1, 1,  -1, 1,  -1, 1};
  return t[k];
}
__host__ __device__ constexpr int shell_of(int k) { return k < 12 ? 1 : (k < 18 ? 2 : 3); }

// Replica-local site indices stay below 2^31 (checked when a context is made), so positions
// and indices use 32-bit arithmetic.
__host__ __device__ inline Pos pos(int64_t s64, int32_t lx, int32_t ly) {
  const uint32_t s = (uint32_t)s64;
  const int32_t b = (int32_t)(s & 3u);
  const uint32_t c = s >> 2;
  const int32_t x = (int32_t)(c % (uint32_t)lx);
  const uint32_t r = c / (uint32_t)lx;
  const int32_t y = (int32_t)(r % (uint32_t)ly);
  const int32_t z = (int32_t)(r / (uint32_t)ly);
  // basis offsets (0,0,0), (0,1,1), (1,0,1), (1,1,0): x parity is bit 1 of b, y parity bit 0
  const int32_t bx = b >> 1, by = b & 1, bz = bx ^ by;
  return Pos{2 * x + bx, 2 * y + by, 2 * z + bz};
}

__host__ __device__ inline int32_t index(Pos p, int32_t lx, int32_t ly) {
  const int32_t b = ((p.x & 1) << 1) | (p.y & 1);
  return (((p.z >> 1) * ly + (p.y >> 1)) * lx + (p.x >> 1)) * 4 + b;
}

__host__ __device__ inline int32_t at(Pos p, int ddx, int ddy, int ddz, int32_t lx, int32_t ly, int32_t lz) {
  Pos q{wrap1(p.x + ddx, 2 * lx), wrap1(p.y + ddy, 2 * ly), wrap1(p.z + ddz, 2 * lz)};
  return index(q, lx, ly);
}

// Partner slot from the first Philox word: floor((r0 >> 32) * 12 / 2^32).
__host__ __device__ inline int dir_of(uint64_t r0) { return (int)(((r0 >> 32) * 12ull) >> 32); }

// Trial site of (colour, link cell t) of a replica with four basis sites, or -1 where that
// link cell is too short to hold the colour's offset.
__device__ inline int64_t trial_site(const Replica &R, int32_t colour, int64_t t) {
  const int32_t b = colour & 3;
  int32_t rest = colour >> 2;
  const int32_t ox = rest % R.ax[0].big;
  rest /= R.ax[0].big;
  const int32_t oy = rest % R.ax[1].big;
  const int32_t oz = rest / R.ax[1].big;
  // link-cell and site indices stay below 2^31: 32-bit arithmetic
  const uint32_t tu = (uint32_t)t, q0 = (uint32_t)R.ax[0].q, q1 = (uint32_t)R.ax[1].q;
  const int32_t cx = (int32_t)(tu % q0);
  const uint32_t t1 = tu / q0;
  const int32_t cy = (int32_t)(t1 % q1);
  const int32_t cz = (int32_t)(t1 / q1);
  if (ox >= axis_len(R.ax[0], cx) || oy >= axis_len(R.ax[1], cy) || oz >= axis_len(R.ax[2], cz)) return -1;
  const int32_t x = axis_start(R.ax[0], cx) + ox, y = axis_start(R.ax[1], cy) + oy, z = axis_start(R.ax[2], cz) + oz;
  return ((z * R.L[1] + y) * R.L[0] + x) * 4 + b;
}

// ------------------------------------------------------------------ MLPNet on matrix cores

template <int P>
struct NetSize;
template <>
struct NetSize<kP32> {
  static constexpr int kL0 = kMT * 10 * 64 * 16;  // 40 K-steps of 2 (80 features), four per read
  static constexpr int kL1 = kMT * 12 * 64 * 16;  // 48 K-steps of 2
};
template <>
struct NetSize<kPBF16> {
  static constexpr int kL0 = kMT * 5 * 64 * 16;   // 5 K-steps of 16
  static constexpr int kL1 = kMT * 6 * 64 * 16;   // 6 K-steps of 16
};
template <>
struct NetSize<kPBF16X3> {
  static constexpr int kL0 = 2 * NetSize<kPBF16>::kL0;  // hi then lo
  static constexpr int kL1 = 2 * NetSize<kPBF16>::kL1;
};
template <>
struct NetSize<kPFP8> {
  static constexpr int kL0 = kMT * 2 * 64 * 32;  // 2 K-steps of 64 (80 features, zero padded)
  static constexpr int kL1 = kMT * 2 * 64 * 32;  // 2 K-steps of 64 (96 units, zero padded)
};
// Image: layer 0, layer 1, layer 2, then c1[96], c2[96], w3[96] (floats) and 16 bytes.  FP8
// also holds c0[96] (after w3): its layer 0 takes the bias in the accumulator, and the 16
// bytes hold the E8M0 scale exponents of the products.
template <int P>
constexpr int net_bytes() {
  return NetSize<P>::kL0 + 2 * NetSize<P>::kL1 + (P == kPFP8 ? 4 : 3) * kHid * 4 + 16;
}

struct NetSmem {
  const uint8_t *w;
  const float *c1, *c2, *w3;
  float b3;
  // FP8: accumulator start of layer 0, and the biased scale exponents of the A (weight) and B
  // (activation) operands of layers 0, 1, 2 (layer 0's B is the exact one-hot, scale 1)
  const float *c0;
  int sa0, sa1, sa2, sb1, sb2;
};

// max(x, 0) as one median-of-three instruction (fmaxf also quiets signalling NaNs first, which
// costs a second instruction); activations are finite.
__device__ __forceinline__ float relu(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 3.402823466e38f); }

// One hidden layer: acc_out = c + W . relu(acc_in), weights at A (hi, and lo for split BF16;
// FP8: scaled products with the biased exponents sa, sb of the weight and activation operands).
template <int P>
__device__ __forceinline__ void net_hidden(const uint8_t *A0, const float *c, const f32x16 (&in)[kMT],
                                           f32x16 (&out)[kMT], int sa = 127, int sb = 127) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 5;
#pragma unroll
  for (int T = 0; T < kMT; ++T)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const f32x4 b = *(const f32x4 *)(c + 32 * T + 8 * j + 4 * g);
#pragma unroll
      for (int i = 0; i < 4; ++i) out[T][4 * j + i] = b[i];
    }
  if constexpr (P == kPFP8) {
    // K-step s takes M-tiles 2s and 2s + 1 (tile 3 is zero) of this lane group: 16 registers
    // each, relu'd and converted to E4M3 (the accumulators are already in the units of this
    // layer's activation scale)
    const i32x8 *A = (const i32x8 *)A0;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      i32x8 b;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int T = 2 * s + t;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          int w = 0;
          if (T < kMT) {
            w = __builtin_amdgcn_cvt_pk_fp8_f32(relu(in[T][4 * q]), relu(in[T][4 * q + 1]), w, false);
            w = __builtin_amdgcn_cvt_pk_fp8_f32(relu(in[T][4 * q + 2]), relu(in[T][4 * q + 3]), w, true);
          }
          b[4 * t + q] = w;
        }
      }
#pragma unroll
      for (int To = 0; To < kMT; ++To)
        out[To] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[(To * 2 + s) * 64 + lane], b, out[To], 0, 0, 0,
                                                                  sa, 0, sb);
      __builtin_amdgcn_sched_barrier(0);
    }
  } else if constexpr (P == kP32) {
    f32x16 h[kMT];
#pragma unroll
    for (int T = 0; T < kMT; ++T)
#pragma unroll
      for (int v = 0; v < 16; ++v) h[T][v] = relu(in[T][v]);
    // K-step s = 16T + v: lane group g supplies its own register v of M-tile T
    const f32x4 *A = (const f32x4 *)A0;
#pragma unroll
    for (int T = 0; T < kMT; ++T)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int To = 0; To < kMT; ++To) {
          const f32x4 a = A[(To * 12 + T * 4 + q) * 64 + lane];
#pragma unroll
          for (int i = 0; i < 4; ++i)
            out[To] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], h[T][4 * q + i], out[To], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
  } else {
    // K-step s = 2T + hh takes registers 8hh..8hh+7 of M-tile T; the B operands of step s + 1
    // are built before the products of step s are issued
    const i32x4 *Ahi = (const i32x4 *)A0;
    const i32x4 *Alo = (const i32x4 *)(A0 + NetSize<kPBF16>::kL1);
    auto build = [&](int T, int hh, i32x4 &bh, i32x4 &bl) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float x0 = relu(in[T][8 * hh + 2 * q]);
        const float x1 = relu(in[T][8 * hh + 2 * q + 1]);
        const uint32_t w = pack_bf16x2(x0, x1);
        bh[q] = (int)w;
        if constexpr (P == kPBF16X3) bl[q] = (int)pack_bf16x2(x0 - bf16_lo_f32(w), x1 - bf16_hi_f32(w));
      }
    };
    i32x4 bh[2], bl[2];
    build(0, 0, bh[0], bl[0]);
#pragma unroll
    for (int s = 0; s < 2 * kMT; ++s) {
      const int cur = s & 1;
      if (s + 1 < 2 * kMT) build((s + 1) >> 1, (s + 1) & 1, bh[cur ^ 1], bl[cur ^ 1]);
      const bf16x8 Bh = __builtin_bit_cast(bf16x8, bh[cur]);
#pragma unroll
      for (int To = 0; To < kMT; ++To) {
        const bf16x8 ah = __builtin_bit_cast(bf16x8, Ahi[(To * 6 + s) * 64 + lane]);
        out[To] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, Bh, out[To], 0, 0, 0);
        if constexpr (P == kPBF16X3) {
          const bf16x8 Bl = __builtin_bit_cast(bf16x8, bl[cur]);
          const bf16x8 al = __builtin_bit_cast(bf16x8, Alo[(To * 6 + s) * 64 + lane]);
          out[To] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, Bl, out[To], 0, 0, 0);
          out[To] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, Bh, out[To], 0, 0, 0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// Slots a lane gathers for layer 0: all 20 for FP32 (both lane groups build the same B
// operand), 10 for BF16 (lane group g takes slots 4s + 2g and 4s + 2g + 1 of K-step s), 16 for
// FP8 (lane group g takes slots 16s + 8g .. + 7 of K-step s; slots 20 and up are padding).
// Slot 0 is the site, 1 + k neighbour k (k < 18) and slot 19 the constant-one input.
template <int P>
constexpr int kGath = P == kP32 ? 20 : (P == kPFP8 ? 16 : 10);
template <int P>
__device__ __forceinline__ int gath_slot(int q, int g) {
  return P == kP32 ? q : (P == kPFP8 ? 16 * (q >> 3) + 8 * g + (q & 7) : 4 * (q >> 1) + 2 * g + (q & 1));
}

// Index offsets of slot m (0: the site, 1 + k: neighbour k, k < kUsed; further slots 0) from
// a site of basis b, valid for every site whose doubled coordinates lie two or more steps
// inside each face (no wrap): off[kStride b + m].  Index arithmetic is linear in the cell
// coordinates, so one interior site per basis gives the table.
template <int kStride, int kUsed>
__device__ inline void fill_offsets(int32_t *s_off, const Replica &R) {
  for (int v = threadIdx.x; v < 4 * kStride; v += blockDim.x) {
    const int b = v / kStride, m = v - kStride * (v / kStride);
    const int bx = b >> 1, by = b & 1;
    const Pos p{4 + bx, 4 + by, 4 + (bx ^ by)};
    int32_t o = 0;
    if (m >= 1 && m <= kUsed)
      o = index(Pos{p.x + dx(m - 1), p.y + dy(m - 1), p.z + dz(m - 1)}, R.L[0], R.L[1]) - index(p, R.L[0], R.L[1]);
    s_off[v] = o;
  }
}

// Interior test of the offset tables: every neighbour of shells 1-3 lies within the box
// (signed bounds, so that a short axis has no interior rather than a wrapped bound).
__device__ __forceinline__ bool interior(Pos p, const Replica &R) {
  return p.x >= 2 && p.x <= 2 * R.L[0] - 3 && p.y >= 2 && p.y <= 2 * R.L[1] - 3 && p.z >= 2 && p.z <= 2 * R.L[2] - 3;
}

// Species of this lane's gathered slots of the site at p; load(s) returns the species at
// replica-local index s.  When every lane of the wave holds an interior site the indices come
// from the offset table, otherwise each one is wrapped per axis.
template <int P, typename Load>
__device__ __forceinline__ void gather_slots(Pos p, const Replica &R, const int32_t *s_off, Load load,
                                             uint32_t (&sp)[kGath<P>]) {
  const int g = (threadIdx.x >> 5) & 1;
  const int32_t lx = R.L[0], ly = R.L[1], lz = R.L[2];
  const int32_t base = index(p, lx, ly);
  if (__all(interior(p, R))) {
    const int32_t *o = s_off + 20 * (((p.x & 1) << 1) | (p.y & 1));
#pragma unroll
    for (int q = 0; q < kGath<P>; ++q) {
      const int m = gath_slot<P>(q, g);
      const uint32_t v = load(base + o[m < kSlots ? m : 0]);
      sp[q] = m < kSlots ? v : 0u;
    }
  } else {
#pragma unroll
    for (int q = 0; q < kGath<P>; ++q) {
      const int m = gath_slot<P>(q, g);
      const int k = (m > 0 && m < kSlots) ? m - 1 : 0;
      const uint32_t v = load((m == 0 || m >= kSlots) ? base : at(p, dx(k), dy(k), dz(k), lx, ly, lz));
      sp[q] = m < kSlots ? v : 0u;
    }
  }
}

// Energy of the site held by this lane (lane % 32) of a 32-site tile from the species of its
// gathered slots.  Both lane groups return the same value.
template <int P>
__device__ __forceinline__ float eval_net(const NetSmem &S, const uint32_t (&sp)[kGath<P>]) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 5;
  f32x16 acc[kMT];
#pragma unroll
  for (int T = 0; T < kMT; ++T)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[T][v] = 0.0f;
  if constexpr (P == kPFP8) {
    // the bias starts the accumulators; K-step s covers features 64s..64s+63: lane group g
    // supplies slots 16s + 8g .. + 7 as E4M3 one-hot dwords (slot 19, the constant-one input,
    // and the padding slots give zero)
#pragma unroll
    for (int T = 0; T < kMT; ++T)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const f32x4 b = *(const f32x4 *)(S.c0 + 32 * T + 8 * j + 4 * g);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[T][4 * j + i] = b[i];
      }
    const i32x8 *A = (const i32x8 *)S.w;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      i32x8 b;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int m = 16 * s + 8 * g + j;
        b[j] = m < kSlots ? (int)onehot_fp8(sp[8 * s + j]) : 0;
      }
#pragma unroll
      for (int T = 0; T < kMT; ++T)
        acc[T] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[(T * 2 + s) * 64 + lane], b, acc[T], 0, 0, 0, S.sa0,
                                                                 0, 127);
      __builtin_amdgcn_sched_barrier(0);
    }
  } else if constexpr (P == kP32) {
    // K-steps 2m, 2m+1 hold slot m: lane group g supplies channel g, then channel 2 + g
    const f32x4 *A = (const f32x4 *)S.w;
#pragma unroll
    for (int m = 0; m < 20; ++m) {
      const uint32_t p = sp[m];
      const float b0 = (p == (uint32_t)g) ? 1.0f : 0.0f;
      const float b1 = (p == (uint32_t)(2 + g)) ? 1.0f : 0.0f;
#pragma unroll
      for (int T = 0; T < kMT; ++T) {
        const f32x4 a = A[(T * 10 + m / 2) * 64 + lane];
        const int o = (m & 1) * 2;
        acc[T] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[o], b0, acc[T], 0, 0, 0);
        acc[T] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[o + 1], b1, acc[T], 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
    // K-step s covers slots 4s..4s+3: lane group g supplies slots 4s + 2g and 4s + 2g + 1
    const i32x4 *Ahi = (const i32x4 *)S.w;
    const i32x4 *Alo = (const i32x4 *)(S.w + NetSize<kPBF16>::kL0);
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      const uint32_t p0 = sp[2 * s], p1 = sp[2 * s + 1];
      i32x4 bw;
      uint32_t l0, h0, l1, h1;
      onehot_bf16(p0, l0, h0);
      onehot_bf16(p1, l1, h1);
      bw[0] = (int)l0; bw[1] = (int)h0; bw[2] = (int)l1; bw[3] = (int)h1;
      const bf16x8 b = __builtin_bit_cast(bf16x8, bw);
#pragma unroll
      for (int T = 0; T < kMT; ++T) {
        const bf16x8 ah = __builtin_bit_cast(bf16x8, Ahi[(T * 5 + s) * 64 + lane]);
        acc[T] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, b, acc[T], 0, 0, 0);
        if constexpr (P == kPBF16X3) {
          const bf16x8 al = __builtin_bit_cast(bf16x8, Alo[(T * 5 + s) * 64 + lane]);
          acc[T] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, b, acc[T], 0, 0, 0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  f32x16 acc1[kMT], acc2[kMT];
  net_hidden<P>(S.w + NetSize<P>::kL0, S.c1, acc, acc1, S.sa1, S.sb1);
  net_hidden<P>(S.w + NetSize<P>::kL0 + NetSize<P>::kL1, S.c2, acc1, acc2, S.sa2, S.sb2);
  float part = 0.0f;
#pragma unroll
  for (int T = 0; T < kMT; ++T)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const f32x4 w = *(const f32x4 *)(S.w3 + 32 * T + 8 * j + 4 * g);
#pragma unroll
      for (int i = 0; i < 4; ++i) part = fmaf(w[i], relu(acc2[T][4 * j + i]), part);
    }
  const float other = __shfl_xor(part, 32);
  const float q0 = g == 0 ? part : other, q1 = g == 0 ? other : part;
  return S.b3 + (q0 + q1);
}

template <int P>
__device__ inline NetSmem net_smem(const uint8_t *s_w, float b3) {
  NetSmem S;
  S.w = s_w;
  S.c1 = (const float *)(s_w + NetSize<P>::kL0 + 2 * NetSize<P>::kL1);
  S.c2 = S.c1 + kHid;
  S.w3 = S.c2 + kHid;
  S.b3 = b3;
  S.c0 = S.w3 + kHid;
  S.sa0 = S.sa1 = S.sa2 = S.sb1 = S.sb2 = 127;
  if constexpr (P == kPFP8) {
    const uint32_t e0 = *(const uint32_t *)(S.c0 + kHid), e1 = *(const uint32_t *)(S.c0 + kHid + 1);
    S.sa0 = (int)(e0 & 255u);
    S.sa1 = (int)((e0 >> 8) & 255u);
    S.sa2 = (int)((e0 >> 16) & 255u);
    S.sb1 = (int)(e1 & 255u);
    S.sb2 = (int)((e1 >> 8) & 255u);
  }
  return S;
}

constexpr int kNetThreads = 512;

// ------------------------------------------------------------------ per-lane evaluators

// qSRO local energy (Eq. 2) over FCC shells 1-3 with the host-folded coefficients (as on
// BCC: Vf[m][c][q] = V_m^{max,min} / z_m, Wf[m][c] = W_m^c / z_m^2, K = C + lambda sum W^2).
template <typename T, typename GetSpecies>
__device__ inline T qsro_site(GetSpecies sp, const T *F) {
  const T *Vf = F, *Wf = F + 75;
  const int c = sp(-1);
  // per-shell species counts as 6-bit fields of one integer (at most 24 neighbours per
  // shell); species 5 and above count nowhere
  uint32_t packed[3] = {0u, 0u, 0u};
#pragma unroll
  for (int k = 0; k < kNbr; ++k) {
    const uint32_t q = (uint32_t)sp(k);
    packed[shell_of(k) - 1] += q < 5u ? 1u << (6u * q) : 0u;
  }
  T cnt[3][5];
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int q = 0; q < 5; ++q) cnt[m][q] = T((packed[m] >> (6 * q)) & 63u);
  T e = F[90];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    T acc = T(0);
#pragma unroll
    for (int q = 0; q < 5; ++q) acc = fma(Vf[(m * 5 + c) * 5 + q], cnt[m][q], acc);
    T self = T(0);
#pragma unroll
    for (int p = 0; p < 5; ++p) self += (p == c) ? cnt[m][p] : T(0);
    e += acc + Wf[m * 5 + c] * self * self;
  }
  return e;
}

// ------------------------------------------------------------------ sweep phases

struct Trial {
  int32_t site;     // replica-local trial site, -1: the link cell has no site of this colour
  int32_t partner;
  double theta;
  int32_t dir;
  int16_t same;
  int16_t px, py, pz;  // doubled coordinates of the trial site (each below 2 * 4096)
  int16_t pad_;
};

__device__ __forceinline__ Pos trial_pos(const Trial &t) { return Pos{t.px, t.py, t.pz}; }

// Position of zone entry k of a trial at pi (offsets from the zone table, wrapped).
__device__ __forceinline__ Pos zone_pos(Pos pi, const int8_t *o, const Replica &R) {
  return Pos{wrap1(pi.x + o[0], 2 * R.L[0]), wrap1(pi.y + o[1], 2 * R.L[1]), wrap1(pi.z + o[2], 2 * R.L[2])};
}

struct QEntry {     // FP64 re-decision queue entry: index into the active list
  int32_t slot;
  float dE_fast;
};

struct Args {
  const Replica *reps;
  int32_t r, colour;
  const uint64_t *sweep;
  uint64_t seed;
  uint8_t *occ;            // all replicas
  float *ecache;
  Trial *trials;           // [n_trials of the colour]
  int32_t *active;         // [n_trials]: trial indices of different-species trials
  uint32_t *n_active;      // device count of active trials (reset before each colour)
  float *e1;               // [active slot][om_n] post-swap energies of the sweep precision
  const int8_t *om;        // [12][kOmMax][3] zone offsets
  int32_t om_n;            // 28 (MLPNet) or 60 (qSRO)
  double guard;
  uint32_t *q_count;       // device count of queued trials (reset before each colour)
  QEntry *queue;           // [n_trials]
  unsigned long long *e_fixed;
  uint64_t *counters;      // [4][n_replicas]
  int32_t n_replicas;
  uint64_t attempts;       // trials of this colour that have a site (counted on the host)
  unsigned long long *dpart;  // MLPNet: [2][k_decide blocks] per-block accepted dE (fixed point)
                              // and accepts; null: k_decide adds them with atomics
  int32_t dpart_n;            // k_decide blocks
  double *trace_dE, *trace_dE_fast;
  uint8_t *trace_flags;
  double *probe_dE;        // non-null: the re-decision kernels write dE of queue entry q to
                           // probe_dE[q] and change nothing
};

constexpr int kPhaseThreads = 512;  // threads of the propose and decide kernels (256: 0.6-1.8 % slower sweeps)
constexpr int kPhaseWaves = kPhaseThreads / 64;

// Block-aggregated append: one atomic per block; slots in (wave, lane) order within the block.
// Every thread of the block must call it.
__device__ __forceinline__ uint32_t block_append(uint32_t *count, bool want, uint32_t *s_wave) {
  const unsigned long long m = __ballot(want);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) s_wave[wave] = (uint32_t)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t total = 0;
    for (int w = 0; w < kPhaseWaves; ++w) {
      const uint32_t c = s_wave[w];
      s_wave[w] = total;
      total += c;
    }
    s_wave[kPhaseWaves] = total ? atomicAdd(count, total) : 0u;
  }
  __syncthreads();
  return s_wave[kPhaseWaves] + s_wave[wave] + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

// Block sum of a 64-bit integer per thread (every thread must call it); valid in thread 0.
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v, unsigned long long *s_part) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) s_part[wave] = v;
  __syncthreads();
  unsigned long long t = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kPhaseWaves; ++w) t += s_part[w];
  return t;
}

__global__ __launch_bounds__(kPhaseThreads) void k_propose(Args a) {
  __shared__ uint32_t s_wave[kPhaseWaves + 1];
  const Replica R = a.reps[a.r];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = t < R.n_trials;
  Trial tr{-1, 0, 0.0, 0, 1, 0, 0, 0, 0};
  const int64_t i = live ? fcc::trial_site(R, a.colour, t) : -1;
  if (i >= 0) {
    const U64x4 x = philox4x64_10((uint64_t)i, *a.sweep, (uint64_t)a.r, 0, a.seed, 0);
    const int d = dir_of(x.v[0]);
    const double u = (double)((x.v[1] >> 11) + 1) * 0x1.0p-53;
    const Pos pi = pos(i, R.L[0], R.L[1]);
    const int64_t n = at(pi, dx(d), dy(d), dz(d), R.L[0], R.L[1], R.L[2]);
    const uint8_t *occ = a.occ + R.site0;
    tr.site = (int32_t)i;
    tr.partner = (int32_t)n;
    tr.theta = isinf(R.temperature) ? (double)INFINITY : -kBoltzmannEvPerK * R.temperature * log(u);
    tr.dir = d;
    tr.same = occ[i] == occ[n];
    tr.px = (int16_t)pi.x;
    tr.py = (int16_t)pi.y;
    tr.pz = (int16_t)pi.z;
    if (tr.same) {
      if (a.trace_flags) a.trace_flags[R.site0 + i] = kFlagSame;
      if (a.trace_dE) a.trace_dE[R.site0 + i] = 0.0;
      if (a.trace_dE_fast) a.trace_dE_fast[R.site0 + i] = 0.0;
    }
  }
  if (live) a.trials[t] = tr;
  const bool active = i >= 0 && !tr.same;
  const uint32_t slot = block_append(a.n_active, active, s_wave);
  if (active) a.active[slot] = (int32_t)t;
  // the attempt and different-species counters are added once per colour by k_decide (the
  // host's count and n_active): per-block atomics on the same two addresses cost 3-5 % of a
  // BF16 or FP8 sweep
}

// Species of site s of a replica as seen with sites i and n exchanged.
__device__ __forceinline__ uint32_t swapped(const uint8_t *occ, int32_t s, int32_t i, int32_t n, uint32_t si,
                                            uint32_t sn) {
  return s == i ? sn : (s == n ? si : (uint32_t)occ[s]);
}

// Post-swap MLPNet energies of the zone sites of every active trial: row = active slot x
// zone position, 32 rows per wave tile.
// Threads of the row kernels: the BF16 (52 KB) and FP8 (38 KB) images let three 256-thread
// blocks share a CU; the FP32 and split-BF16 images (103 KB) one 512-thread block.
template <int P>
constexpr int net_threads() {
  return (P == kPBF16 || P == kPFP8) ? 256 : kNetThreads;
}

// At least two waves per SIMD: the register budget is then the architectural VGPRs alone, so
// the accumulators stay in VGPRs (with a 256-thread block the compiler otherwise places them
// in AGPRs and copies every activation out first).
template <int P>
__global__ __launch_bounds__(net_threads<P>(), 2) void k_rows_net(Args a, const uint8_t *wpack, float b3) {
  constexpr int kW = net_bytes<P>();
  constexpr int kThreads = net_threads<P>();
  __shared__ __attribute__((aligned(16))) uint8_t s_w[kW];
  __shared__ int32_t s_off[80];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const Replica R = a.reps[a.r];
  for (int q = tid; q < kW / 16; q += kThreads) ((int4 *)s_w)[q] = ((const int4 *)wpack)[q];
  fill_offsets<20, kNbrMlp>(s_off, R);
  __syncthreads();
  const NetSmem S = net_smem<P>(s_w, b3);
  const uint8_t *occ = a.occ + R.site0;
  const int32_t rows = (int32_t)(*a.n_active) * kOmMlp;  // below 2^31: trials x 28 of one colour
  const int32_t tiles = (rows + 31) / 32;
  constexpr int kWaves = kThreads / 64;
  for (int32_t tile = blockIdx.x * kWaves + wave; tile < tiles; tile += gridDim.x * kWaves) {
    const int32_t row = tile * 32 + (lane & 31);
    const bool valid = row < rows;
    const int32_t slot = valid ? row / kOmMlp : 0;
    const int k = valid ? row - slot * kOmMlp : 0;
    const Trial tr = a.trials[a.active[slot]];
    const int64_t i = tr.site, n = tr.partner;
    const uint32_t si = occ[i], sn = occ[n];
    const Pos pj = zone_pos(trial_pos(tr), a.om + (tr.dir * kOmMax + k) * 3, R);
    uint32_t sp[kGath<P>];
    gather_slots<P>(pj, R, s_off, [&](int32_t s) { return swapped(occ, s, (int32_t)i, (int32_t)n, si, sn); }, sp);
    const float E = eval_net<P>(S, sp);
    if (valid && lane < 32) a.e1[row] = E;
  }
}

// Post-swap qSRO energies (FP32): a block stages the read regions of kRqTrials active trials in
// LDS (304 sites each, the swapped pair exchanged, one byte load per site instead of one per
// zone row and slot), then evaluates their 60 zone rows from LDS, one row per thread, with the
// per-lane arithmetic.  The region tables (offsets per partner slot, and the region position of
// every zone row's slot) stay in LDS for the whole launch.
constexpr int kRqTrials = 16;
constexpr int kRqThreads = 1024;  // 960 rows per pass, one per thread (measured: 256 threads 3.8e8,
                                  // 512 threads 4.8e8, 1024 threads 5.3e8 attempts/s on 200^3)
__global__ __launch_bounds__(kRqThreads) void k_rows_qsro(Args a, const float *F, const uint16_t *roff,
                                                          const uint16_t *ridx, const uint16_t *rpos) {
  __shared__ __attribute__((aligned(16))) uint16_t s_idx[kDirs * kOmQsro * (kNbr + 1)];
  __shared__ uint16_t s_roff[kDirs * kRegQ];
  __shared__ uint16_t s_rpos[2 * kDirs];
  __shared__ uint8_t s_reg[kRqTrials * kRegQ];
  __shared__ float s_F[kQsroPacked];
  __shared__ int32_t s_site[kRqTrials], s_part[kRqTrials];
  __shared__ int16_t s_px[kRqTrials], s_py[kRqTrials], s_pz[kRqTrials];
  __shared__ uint8_t s_dir[kRqTrials];
  const Replica R = a.reps[a.r];
  const uint8_t *occ = a.occ + R.site0;
  const int tid = threadIdx.x;
  const int32_t ntr = (int32_t)(*a.n_active);
  if ((int32_t)blockIdx.x * kRqTrials >= ntr) return;  // no trial for this block
  static_assert((kDirs * kOmQsro * (kNbr + 1)) % 2 == 0, "idx table in 4-byte words");
  for (int q = tid; q < kDirs * kOmQsro * (kNbr + 1) / 2; q += kRqThreads)
    ((uint32_t *)s_idx)[q] = ((const uint32_t *)ridx)[q];
  for (int q = tid; q < kDirs * kRegQ; q += kRqThreads) s_roff[q] = roff[q];
  if (tid < 2 * kDirs) s_rpos[tid] = rpos[tid];
  for (int q = tid; q < kQsroPacked; q += kRqThreads) s_F[q] = F[q];
  for (int32_t b0 = (int32_t)blockIdx.x * kRqTrials; b0 < ntr; b0 += (int32_t)gridDim.x * kRqTrials) {
    if (tid < kRqTrials && b0 + tid < ntr) {
      const Trial tr = a.trials[a.active[b0 + tid]];
      s_site[tid] = tr.site;
      s_part[tid] = tr.partner;
      s_px[tid] = tr.px;
      s_py[tid] = tr.py;
      s_pz[tid] = tr.pz;
      s_dir[tid] = (uint8_t)tr.dir;
    }
    __syncthreads();
    // regions: the trial site holds the partner's species and the partner the site's
    for (int v = tid; v < kRqTrials * kRegQ; v += kRqThreads) {
      const int tt = v / kRegQ, p = v - tt * kRegQ;
      if (b0 + tt < ntr) {
        const int d = s_dir[tt];
        const uint32_t o = s_roff[d * kRegQ + p];
        const Pos pi{s_px[tt], s_py[tt], s_pz[tt]};
        int32_t s = at(pi, (int)(o & 15u) - 8, (int)((o >> 4) & 15u) - 8, (int)((o >> 8) & 15u) - 8, R.L[0], R.L[1],
                       R.L[2]);
        if (p == s_rpos[2 * d]) s = s_part[tt];
        else if (p == s_rpos[2 * d + 1]) s = s_site[tt];
        s_reg[v] = occ[s];
      }
    }
    __syncthreads();
    for (int r = tid; r < kRqTrials * kOmQsro; r += kRqThreads) {
      const int tt = r / kOmQsro, k = r - tt * kOmQsro;
      if (b0 + tt < ntr) {
        const uint16_t *ir = s_idx + (s_dir[tt] * kOmQsro + k) * (kNbr + 1);
        const uint8_t *reg = s_reg + tt * kRegQ;
        a.e1[(int64_t)(b0 + tt) * kOmQsro + k] = qsro_site<float>([&](int k2) -> int { return reg[ir[k2 + 1]]; }, s_F);
      }
    }
    __syncthreads();
  }
}

// Zone sums against the cache (fixed order), then the Metropolis decision or the FP64 queue.
// The zone energies of a trial are contiguous (OM is a multiple of four): 16-byte loads, all
// of them and the cache gathers in flight at once.
// Lanes per trial in k_decide: each sums a contiguous quarter of the zone.
constexpr int kDecideLanes = 4;

template <int OM>
__global__ __launch_bounds__(kPhaseThreads) void k_decide(Args a) {
  static_assert(OM % kDecideLanes == 0, "zone size");
  constexpr int kPer = OM / kDecideLanes;
  __shared__ unsigned long long s_part[kPhaseWaves];
  const Replica R = a.reps[a.r];
  const int sub = threadIdx.x & (kDecideLanes - 1);
  const int32_t slot = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) / kDecideLanes);
  const uint32_t n_act = *a.n_active;
  const bool live = slot < (int32_t)n_act;  // the four lanes of a trial agree
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int Rn = a.n_replicas;
    atomicAdd((unsigned long long *)&a.counters[0 * Rn + a.r], (unsigned long long)a.attempts);
    atomicAdd((unsigned long long *)&a.counters[1 * Rn + a.r], (unsigned long long)n_act);
  }
  bool accept = false;
  long long fixed = 0;
  if (live) {
    const Trial tr = a.trials[a.active[slot]];
    uint8_t *occ = a.occ + R.site0;
    float *ec = a.ecache + R.site0;
    const Pos pi = trial_pos(tr);
    const float *e1 = a.e1 + (int64_t)slot * OM + sub * kPer;
    const int8_t *o = a.om + (tr.dir * kOmMax + sub * kPer) * 3;
    int32_t idx[kPer];
    float part = 0.0f;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      idx[j] = at(pi, o[3 * j], o[3 * j + 1], o[3 * j + 2], R.L[0], R.L[1], R.L[2]);
      part += e1[j] - ec[idx[j]];
    }
    // (q0 + q1) + (q2 + q3) on every lane: float addition is commutative, so the four lanes
    // hold the same dE and take the same decision
    const float pair = part + __shfl_xor(part, 1);
    const float dE = pair + __shfl_xor(pair, 2);
    const double dEd = (double)dE;
    const bool lead = sub == 0;
    if (lead && a.trace_dE_fast) a.trace_dE_fast[R.site0 + tr.site] = dEd;
    if (fabs(dEd - tr.theta) < a.guard) {
      if (lead) {
        const uint32_t q = atomicAdd(a.q_count, 1u);
        a.queue[q] = QEntry{slot, dE};
      }
    } else {
      accept = dEd <= tr.theta;
      if (accept) {
        if (lead) {
          const uint8_t si = occ[tr.site];
          occ[tr.site] = occ[tr.partner];
          occ[tr.partner] = si;
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) ec[idx[j]] = e1[j];
        fixed = lead ? to_fixed(dEd) : 0;
      }
      if (lead && a.trace_flags) a.trace_flags[R.site0 + tr.site] = accept ? kFlagAccept : 0;
      if (lead && a.trace_dE) a.trace_dE[R.site0 + tr.site] = dEd;
    }
  }
  // the block's accepted dE (2^-32 eV units) and accept count: with dpart, partials summed by
  // decide_totals in k_recheck_net_decide (MLPNet: per-block atomics on the same two addresses cost 3-7 % of a BF16
  // or FP8 sweep), else one atomic each (qSRO, whose longer decide spreads them out: the extra
  // launch measured 1.4 % slower)
  const unsigned long long esum = block_sum_u64((unsigned long long)fixed, s_part);
  __syncthreads();
  const unsigned long long nacc = block_sum_u64(accept && sub == 0 ? 1ull : 0ull, s_part);
  if (threadIdx.x == 0) {
    if (a.dpart) {
      a.dpart[blockIdx.x] = esum;
      a.dpart[gridDim.x + blockIdx.x] = nacc;
    } else {
      if (esum) atomicAdd(&a.e_fixed[a.r], esum);
      if (nacc) atomicAdd((unsigned long long *)&a.counters[2 * a.n_replicas + a.r], nacc);
    }
  }
}

// Adds the a.dpart_n partials of k_decide to the replica's running total and accept counter
// (exact integer sums).  Every thread of a kPhaseThreads block calls it.
__device__ __forceinline__ void decide_totals(const Args &a, unsigned long long *s_part) {
  const int nb = a.dpart_n;
  unsigned long long e = 0, n = 0;
  for (int b = threadIdx.x; b < nb; b += kPhaseThreads) {
    e += a.dpart[b];
    n += a.dpart[nb + b];
  }
  e = block_sum_u64(e, s_part);
  __syncthreads();
  n = block_sum_u64(n, s_part);
  if (threadIdx.x == 0) {
    if (e) atomicAdd(&a.e_fixed[a.r], e);
    if (n) atomicAdd((unsigned long long *)&a.counters[2 * a.n_replicas + a.r], n);
  }
}

// ------------------------------------------------------------------ FP64 evaluation

// FP64 MLPNet blob with every weight matrix stored [input][unit]: W0t[76][96], b0, W1t[96][96],
// b1, W2t[96][96], b2, W3[96], b3.  The FP64 kernels read its values from an FP32 copy (every
// entry is an FP32 parameter) staged in LDS.
constexpr int kR64Threads = 384;  // six waves: one 16-unit tile of the 96 units each
constexpr int kNetParamsDev = kHid * kIn + kHid + 2 * (kHid * kHid + kHid) + kHid + 1;  // 26,113
constexpr int kHS = kHid + 1;     // padded activation row stride

// FP64 energies of up to 16 rows (slot species in s_sp[row][19]) on the FP64 matrix cores, for
// the re-decision and the FP64 site energies: wave v (of 6) owns units 16v .. 16v + 15 in every
// layer, the rows are the other dimension of the 16x16x4 products.  W: the blob's values as FP32
// numbers (exact).  Layer 0 takes slot m as K-step m (lane l: channel l / 16 of row l % 16); a
// row has at most one non-zero product per K-step, so its sums are b0 plus the selected W0
// columns in slot order.  The hidden layers sum 4 products per step; the output layer is one
// fma per unit in order.  Rows past nrows are computed from empty slots and not written.
typedef double f64x4_fcc __attribute__((ext_vector_type(4)));
__device__ void net64_rows16(const float *W, const uint8_t *s_sp, int nrows, double *s_h, double *s_out) {
  const int tid = threadIdx.x, wv = tid >> 6, li = tid & 15, lk = (tid >> 4) & 3, u0 = 16 * wv;
  const float *W0 = W, *b0 = W0 + kIn * kHid, *W1 = b0 + kHid, *b1 = W1 + kHid * kHid, *W2 = b1 + kHid,
              *b2 = W2 + kHid * kHid, *W3 = b2 + kHid, *b3 = W3 + kHid;
  const bool rv = li < nrows;
  f64x4_fcc acc;
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = (double)b0[u0 + lk + 4 * j];
#pragma unroll
  for (int m = 0; m < kSlots; ++m) {
    const uint32_t sp = rv ? s_sp[li * kSlots + m] : 4u;
    const double b = sp == (uint32_t)lk ? 1.0 : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)W0[(4 * m + lk) * kHid + u0 + li], b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) s_h[li * kHS + u0 + lk + 4 * j] = acc[j] > 0.0 ? acc[j] : 0.0;
  __syncthreads();
  for (int layer = 0; layer < 2; ++layer) {
    const float *Wl = layer == 0 ? W1 : W2, *bl = layer == 0 ? b1 : b2;
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = (double)bl[u0 + lk + 4 * j];
#pragma unroll 8
    for (int st = 0; st < kHid / 4; ++st)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)Wl[(4 * st + lk) * kHid + u0 + li],
                                                 s_h[li * kHS + 4 * st + lk], acc, 0, 0, 0);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) s_h[li * kHS + u0 + lk + 4 * j] = acc[j] > 0.0 ? acc[j] : 0.0;
    __syncthreads();
  }
  // E_r = b3 + sum_o W3[o] h3[r][o], units in order
  if (tid < nrows) {
    double e = (double)b3[0];
    for (int k = 0; k < kHid; ++k) e = fma((double)W3[k], s_h[tid * kHS + k], e);
    s_out[tid] = e;
  }
  __syncthreads();
}

// The network's values as FP32 numbers (exact: the FP64 blob rounded to FP32 changes nothing) into
// LDS, in one batch of 16-byte loads (every thread of the block).
__device__ __forceinline__ void net64_stage(float *s_w, const float *W32) {
  constexpr int n4 = kNetParamsDev / 4, per = (n4 + kR64Threads - 1) / kR64Threads;
  const int tid = threadIdx.x;
  const float4 *w4 = (const float4 *)W32;
  float4 t[per];
#pragma unroll
  for (int k = 0; k < per; ++k) {
    const int q = tid + k * kR64Threads;
    t[k] = q < n4 ? w4[q] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
  const float tail = tid < kNetParamsDev - 4 * n4 ? W32[4 * n4 + tid] : 0.0f;
#pragma unroll
  for (int k = 0; k < per; ++k) {
    const int q = tid + k * kR64Threads;
    if (q < n4) ((float4 *)s_w)[q] = t[k];
  }
  if (tid < kNetParamsDev - 4 * n4) s_w[4 * n4 + tid] = tail;
}

// FP64 local energies of every site of one replica (MLPNet) with the re-decision's row evaluator
// (net64_rows16), 16 sites per pass and one block per CU (the weights in LDS); each thread loads
// its slot species of the next pass while the current one is evaluated.
constexpr int kS64NetRows = 16;
__global__ __launch_bounds__(kR64Threads) void k_site_energies_net64(const Replica *reps, int32_t r,
                                                                     const uint8_t *occ_all, const float *W32,
                                                                     double *out) {
  __shared__ __attribute__((aligned(16))) float s_w[kNetParamsDev];
  __shared__ double s_h[kS64NetRows * kHS];
  __shared__ double s_out[kS64NetRows];
  __shared__ uint8_t s_sp[kS64NetRows * kSlots];
  static_assert(kS64NetRows * kSlots <= kR64Threads, "one slot species per thread");
  const Replica R = reps[r];
  const uint8_t *occ = occ_all + R.site0;
  const int64_t passes = (R.n_sites + kS64NetRows - 1) / kS64NetRows;
  if ((int64_t)blockIdx.x >= passes) return;
  const int tid = threadIdx.x;
  auto fetch = [&](int64_t pass) -> uint8_t {
    if (tid >= kS64NetRows * kSlots || pass >= passes) return 4;
    const int lr = tid / kSlots, m = tid - lr * kSlots;
    const int64_t j = pass * kS64NetRows + lr;
    if (j >= R.n_sites) return 4;
    if (m == 0) return occ[j];
    const Pos p = pos(j, R.L[0], R.L[1]);
    return occ[at(p, dx(m - 1), dy(m - 1), dz(m - 1), R.L[0], R.L[1], R.L[2])];
  };
  uint8_t cur = fetch(blockIdx.x);
  net64_stage(s_w, W32);
  for (int64_t pass = blockIdx.x; pass < passes; pass += gridDim.x) {
    const int64_t j0 = pass * kS64NetRows;
    const int nrows = R.n_sites - j0 < kS64NetRows ? (int)(R.n_sites - j0) : kS64NetRows;
    if (tid < kS64NetRows * kSlots) s_sp[tid] = cur;
    __syncthreads();
    cur = fetch(pass + gridDim.x);
    net64_rows16(s_w, s_sp, nrows, s_h, s_out);
    if (tid < nrows) out[R.site0 + j0 + tid] = s_out[tid];
  }
}

// Local energies of every site of one replica with the matrix-core MLPNet evaluator.
template <int P>
__global__ __launch_bounds__(kNetThreads) void k_site_energies_net(const Replica *reps, int32_t r,
                                                                   const uint8_t *occ_all, const uint8_t *wpack,
                                                                   float b3, float *out) {
  constexpr int kW = net_bytes<P>();
  __shared__ __attribute__((aligned(16))) uint8_t s_w[kW];
  __shared__ int32_t s_off[80];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const Replica R = reps[r];
  for (int q = tid; q < kW / 16; q += kNetThreads) ((int4 *)s_w)[q] = ((const int4 *)wpack)[q];
  fill_offsets<20, kNbrMlp>(s_off, R);
  __syncthreads();
  const NetSmem S = net_smem<P>(s_w, b3);
  const uint8_t *occ = occ_all + R.site0;
  const int64_t tiles = (R.n_sites + 31) / 32;
  constexpr int kWaves = kNetThreads / 64;
  for (int64_t tile = (int64_t)blockIdx.x * kWaves + wave; tile < tiles; tile += (int64_t)gridDim.x * kWaves) {
    const int64_t j = tile * 32 + (lane & 31);
    const bool valid = j < R.n_sites;
    const Pos p = pos(valid ? j : 0, R.L[0], R.L[1]);
    uint32_t sp[kGath<P>];
    gather_slots<P>(p, R, s_off, [&](int32_t s) { return (uint32_t)occ[s]; }, sp);
    const float E = eval_net<P>(S, sp);
    if (valid && lane < 32) out[R.site0 + j] = E;
  }
}

// Per-lane qSRO local energies of every site (FP32 or FP64).
template <typename T>
__global__ void k_site_energies_qsro(const Replica *reps, int32_t r, const uint8_t *occ_all, const T *F, T *out) {
  const Replica R = reps[r];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= R.n_sites) return;
  const uint8_t *occ = occ_all + R.site0;
  const Pos p = pos(j, R.L[0], R.L[1]);
  out[R.site0 + j] = qsro_site<T>(
      [&](int k) -> int { return k < 0 ? occ[j] : occ[at(p, dx(k), dy(k), dz(k), R.L[0], R.L[1], R.L[2])]; }, F);
}

// FP64 re-decision of queued trials (MLPNet), first launch: the zone's 28 local energies after
// and 28 before the swap, split over kRcSplit work items of 14 rows (one 16-row matrix-product
// tile) so that a short queue still spreads over the chip; each writes its rows to row_e.
// k_recheck_net_decide sums, decides and applies.
constexpr int kRcSplit = 4;
constexpr int kRcRows = 2 * kOmMlp / kRcSplit;  // 14
static_assert(kRcRows <= 16 && (kR64Threads / 64) * 16 == kHid, "one 16-row tile; one 16-unit tile per wave");
static_assert(kRcRows * kRcSplit == 2 * kOmMlp, "row split");

__global__ __launch_bounds__(kR64Threads) void k_recheck_net(Args a, const float *W32, double *row_e) {
  // the blob's values in LDS (FP32 numbers, exact: W32 is the FP64 blob rounded to FP32, which
  // changes nothing), loaded in one batch of 16-byte loads: the queue is short, so each block's
  // latency is the kernel's time and weight reads must not go to L2 per layer
  __shared__ __attribute__((aligned(16))) float s_w[kNetParamsDev];
  __shared__ double s_h[16 * kHS];
  __shared__ double s_out[16];
  __shared__ uint8_t s_sp[kRcRows * kSlots];
  const Replica R = a.reps[a.r];
  uint8_t *occ = a.occ + R.site0;
  const uint32_t nq = *a.q_count;
  const int tid = threadIdx.x;
  if (blockIdx.x >= nq * kRcSplit) return;  // no work item for this block
  net64_stage(s_w, W32);
  __syncthreads();
  for (uint32_t w = blockIdx.x; w < nq * kRcSplit; w += gridDim.x) {
    const uint32_t q = w / kRcSplit;
    const int r0 = (int)(w - q * kRcSplit) * kRcRows;
    const QEntry qe = a.queue[q];
    const Trial tr = a.trials[a.active[qe.slot]];
    const int64_t i = tr.site, n = tr.partner;
    const uint32_t si = occ[i], sn = occ[n];
    const Pos pi = trial_pos(tr);
    const int8_t *o = a.om + tr.dir * kOmMax * 3;
    // rows 0..27 after the swap, 28..55 before
    for (int v = tid; v < kRcRows * kSlots; v += kR64Threads) {
      const int row = r0 + v / kSlots, m = v % kSlots;
      const bool post = row < kOmMlp;
      const int k = post ? row : row - kOmMlp;
      const Pos pj = zone_pos(pi, o + 3 * k, R);
      const int32_t s = m == 0 ? index(pj, R.L[0], R.L[1]) : at(pj, dx(m - 1), dy(m - 1), dz(m - 1), R.L[0], R.L[1], R.L[2]);
      s_sp[v] = (uint8_t)(post ? swapped(occ, s, (int32_t)i, (int32_t)n, si, sn) : (uint32_t)occ[s]);
    }
    __syncthreads();
    net64_rows16(s_w, s_sp, kRcRows, s_h, s_out);
    if (tid < kRcRows) row_e[(size_t)q * 2 * kOmMlp + r0 + tid] = s_out[tid];
    __syncthreads();
  }
}

// Decision of the queued MLPNet trials after k_recheck_net (the kernel boundary orders the rows),
// one wave per trial: the 56 row energies loaded by 56 lanes and summed in row order (rows
// 0..27 after the swap, 28..55 before), the Metropolis decision and the apply (or, for a probe,
// dE only).
__global__ __launch_bounds__(kPhaseThreads) void k_recheck_net_decide(Args a, const double *row_e) {
  // the last block, which usually has no queued trial, adds k_decide's partials (a sweep's
  // launch; probes pass none)
  if (a.dpart && blockIdx.x == gridDim.x - 1) {
    __shared__ unsigned long long s_part[kPhaseWaves];
    decide_totals(a, s_part);
  }
  const Replica R = a.reps[a.r];
  uint8_t *occ = a.occ + R.site0;
  const uint32_t nq = *a.q_count;
  const int lane = threadIdx.x & 63;
  const uint32_t waves = gridDim.x * (blockDim.x / 64);
  for (uint32_t q = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); q < nq; q += waves) {
    const QEntry qe = a.queue[q];
    const Trial tr = a.trials[a.active[qe.slot]];
    const double *re = row_e + (size_t)q * 2 * kOmMlp;
    const double v1 = lane < kOmMlp ? re[lane] : 0.0, v0 = lane < kOmMlp ? re[kOmMlp + lane] : 0.0;
    double e1 = 0.0, e0 = 0.0;
#pragma unroll
    for (int k = 0; k < kOmMlp; ++k) e1 += __shfl(v1, k);
#pragma unroll
    for (int k = 0; k < kOmMlp; ++k) e0 += __shfl(v0, k);
    const double dE = e1 - e0;
    if (a.probe_dE) {
      if (lane == 0) a.probe_dE[q] = dE;
      continue;
    }
    const bool accept = dE <= tr.theta;
    const int Rn = a.n_replicas;
    if (lane == 0) {
      const int64_t i = tr.site, n = tr.partner;
      if (accept) {
        const uint8_t si = occ[i], sn = occ[n];
        occ[i] = sn;
        occ[n] = si;
        atomicAdd(&a.e_fixed[a.r], (unsigned long long)to_fixed(dE));
        atomicAdd((unsigned long long *)&a.counters[2 * Rn + a.r], 1ull);
      }
      atomicAdd((unsigned long long *)&a.counters[3 * Rn + a.r], 1ull);
      if (a.trace_flags) a.trace_flags[R.site0 + i] = kFlagFp64 | (accept ? kFlagAccept : 0);
      if (a.trace_dE) a.trace_dE[R.site0 + i] = dE;
    }
    if (accept && lane < kOmMlp) {
      // the cache keeps the sweep precision's post-swap energies
      const Pos pi = trial_pos(tr);
      const int8_t *o = a.om + tr.dir * kOmMax * 3;
      a.ecache[R.site0 + at(pi, o[3 * lane], o[3 * lane + 1], o[3 * lane + 2], R.L[0], R.L[1], R.L[2])] =
          a.e1[(int64_t)qe.slot * kOmMlp + lane];
    }
  }
}

// FP64 re-decision of queued trials (qSRO): one row per thread, one trial per block.
constexpr int kRcQsroThreads = 128;
__global__ __launch_bounds__(kRcQsroThreads) void k_recheck_qsro(Args a, const double *W) {
  __shared__ double s_out[2 * kOmQsro];
  __shared__ int s_accept;
  const Replica R = a.reps[a.r];
  uint8_t *occ = a.occ + R.site0;
  const uint32_t nq = *a.q_count;
  const int tid = threadIdx.x;
  for (uint32_t q = blockIdx.x; q < nq; q += gridDim.x) {
    const QEntry qe = a.queue[q];
    const Trial tr = a.trials[a.active[qe.slot]];
    const int64_t i = tr.site, n = tr.partner;
    const uint32_t si = occ[i], sn = occ[n];
    const Pos pi = trial_pos(tr);
    const int8_t *o = a.om + tr.dir * kOmMax * 3;
    if (tid < 2 * kOmQsro) {
      const bool post = tid < kOmQsro;
      const int k = post ? tid : tid - kOmQsro;
      const Pos pj = zone_pos(pi, o + 3 * k, R);
      s_out[tid] = qsro_site<double>(
          [&](int k2) -> int {
            const int32_t s = k2 < 0 ? index(pj, R.L[0], R.L[1]) : at(pj, dx(k2), dy(k2), dz(k2), R.L[0], R.L[1], R.L[2]);
            return (int)(post ? swapped(occ, s, (int32_t)i, (int32_t)n, si, sn) : (uint32_t)occ[s]);
          },
          W);
    }
    __syncthreads();
    if (tid == 0) {
      double e1 = 0.0, e0 = 0.0;
      for (int k = 0; k < kOmQsro; ++k) e1 += s_out[k];
      for (int k = 0; k < kOmQsro; ++k) e0 += s_out[kOmQsro + k];
      const double dE = e1 - e0;
      bool accept = false;
      if (a.probe_dE) {
        a.probe_dE[q] = dE;
      } else {
        accept = dE <= tr.theta;
        const int Rn = a.n_replicas;
        if (accept) {
          occ[i] = (uint8_t)sn;
          occ[n] = (uint8_t)si;
          atomicAdd(&a.e_fixed[a.r], (unsigned long long)to_fixed(dE));
          atomicAdd((unsigned long long *)&a.counters[2 * Rn + a.r], 1ull);
        }
        atomicAdd((unsigned long long *)&a.counters[3 * Rn + a.r], 1ull);
        if (a.trace_flags) a.trace_flags[R.site0 + i] = kFlagFp64 | (accept ? kFlagAccept : 0);
        if (a.trace_dE) a.trace_dE[R.site0 + i] = dE;
      }
      s_accept = accept;
    }
    __syncthreads();
    if (tid < kOmQsro && s_accept)
      a.ecache[R.site0 + at(pi, o[3 * tid], o[3 * tid + 1], o[3 * tid + 2], R.L[0], R.L[1], R.L[2])] =
          a.e1[(int64_t)qe.slot * kOmQsro + tid];
    __syncthreads();
  }
}

// Pair counts per shell (1-3) and ordered species pair, and species counts, of one replica.
__global__ void k_pair_counts(const Replica *reps, int32_t r, const uint8_t *occ_all, int32_t S,
                              unsigned long long *cnt, unsigned long long *nsp) {
  __shared__ unsigned int s_cnt[3 * 5 * 5 + 5];
  for (int q = threadIdx.x; q < 3 * 25 + 5; q += blockDim.x) s_cnt[q] = 0u;
  __syncthreads();
  const Replica R = reps[r];
  const uint8_t *occ = occ_all + R.site0;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < R.n_sites; j += (int64_t)gridDim.x * blockDim.x) {
    const int p = occ[j];
    if (p >= S) continue;  // occupancies are validated on entry; never index past the histogram
    atomicAdd(&s_cnt[75 + p], 1u);
    const Pos ps = pos(j, R.L[0], R.L[1]);
    for (int k = 0; k < kNbr; ++k) {
      const int q = occ[at(ps, dx(k), dy(k), dz(k), R.L[0], R.L[1], R.L[2])];
      if (q < S) atomicAdd(&s_cnt[((shell_of(k) - 1) * 5 + p) * 5 + q], 1u);
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < 3 * 25 + 5; q += blockDim.x) {
    if (!s_cnt[q]) continue;
    if (q < 75) {
      const int m = q / 25, p = (q / 5) % 5, qq = q % 5;
      if (p < S && qq < S) atomicAdd(&cnt[(m * S + p) * S + qq], (unsigned long long)s_cnt[q]);
    } else if (q - 75 < S) {
      atomicAdd(&nsp[q - 75], (unsigned long long)s_cnt[q]);
    }
  }
}

}  // namespace fcc
}  // namespace smc

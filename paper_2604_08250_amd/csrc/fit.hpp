// Kernels of the differentiation pattern: energies of whole snapshots, their gradient with
// respect to the MLP parameters, the fit objective, Adam, and the cluster-expansion labels.
//
// Rows.  Row r of a batch is site j = r mod N of snapshot b = r / N (N = 2 L^3 sites per
// snapshot); its local energy is the MLP of Eqs. (4)-(6) on the one-hot features of the
// site and its 26 shell-1..3 neighbours, and S_b sums the rows of snapshot b.
//
// BF16 path (matrix cores, FP32 accumulation).  Forward: the sweep's tile evaluator.
// Backward, fused per chunk of 128 rows in a block of four waves, each wave owning 32 rows:
//   forward again, keeping y1 = -log2(e) z1 and y2 = -log2(e) z2 in registers;
//   gz2 = gE W2 silu'(z2);  gh1 = W1^T gz2 (matrix cores, W1^T image in LDS);
//   gz1 = gh1 silu'(z1);
// then the weight gradients, which sum over rows, are matrix-core products with the rows as
// the K dimension: the per-row vectors are staged in LDS as [unit][row] BF16 tiles (the
// transposition that puts rows into K), and each wave owns one quarter of dW1 and of dW0:
//   phase A: dW1 = sum_r gz2 (x) h1  and  db1 = sum_r gz2;
//   phase B: dW0 = sum_r gz1 (x) x  (x built from 4-bit species codes in LDS; feature 108 is
//            the constant one, so db0 comes out of the same product)  and  dW2 = sum_r gE h2.
// Each block accumulates its chunks in registers and writes one partial gradient; a second
// kernel adds the partials in block order, so the result does not depend on timing.
//
// Reference path (FP32 or FP64): one thread per (row, unit) per layer with the per-row
// values in global scratch, and one thread per parameter summing the rows in order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"
#include "mfma_eval.hpp"

namespace smc {

constexpr int kFitF = 108;
constexpr int kFitThreads = 256;  // backward block: four waves
constexpr int kFitRows = 128;     // rows per backward chunk
constexpr int kFitFwdThreads = 512;
constexpr int kFitW0 = PackSize<kPBF16>::kL0;
constexpr int kFitW1 = PackSize<kPBF16>::kL1;
constexpr int kFitPack = kFitW0 + kFitW1 + 2 * kHid * 4;  // layer 0, layer 1, c1, w2 (scaled)
constexpr int kOffB0 = kHid * kFitF;
constexpr int kOffW1 = kOffB0 + kHid;
constexpr int kOffB1 = kOffW1 + kHid * kHid;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid;
constexpr int kFitParams = kOffB2 + 1;
constexpr float kFitLog2e = 1.44269504088896340736f;
constexpr float kFitLn2 = 0.69314718055994530942f;

__device__ __forceinline__ int fit_hid(int T, int v, int g) { return 32 * T + 8 * (v >> 2) + 4 * g + (v & 3); }

// ---------------------------------------------------------------------------- packing

__device__ __forceinline__ uint16_t fit_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// BF16 images from the FP32 blob: layer 0 (-log2(e) W0, bias in feature 108), layer 1 (W1)
// in the operand orders of the tile evaluator, c1 = -log2(e) b1, w2 = -ln(2) W2, and W1^T
// as the A operand of the backward product (element (T, s, lane, e): W1[o][i] with
// i = 32T + lane%32 and o the hidden unit that register 8(s%2)+e of M-tile s/2 holds).
__global__ void k_fit_pack_bf16(const float *p, uint8_t *pack, uint8_t *w1t) {
  const int n0 = kFitW0 / 2, n1 = kFitW1 / 2;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const float *W0 = p, *b0 = p + kOffB0, *W1 = p + kOffW1, *b1 = p + kOffB1, *W2 = p + kOffW2;
  uint16_t *L0 = (uint16_t *)pack, *L1 = L0 + n0, *LT = (uint16_t *)w1t;
  float *c1 = (float *)(pack + kFitW0 + kFitW1), *w2 = c1 + kHid;
  if (t < n0) {
    const int e = t & 7, l = (t >> 3) & 63, s = (t >> 9) % 7, T = (t >> 9) / 7;
    const int o = 32 * T + (l & 31), f = 16 * s + 8 * (l >> 5) + e;
    const float w = f < kFitF ? -kFitLog2e * W0[o * kFitF + f] : (f == kFitF ? -kFitLog2e * b0[o] : 0.0f);
    L0[t] = fit_bf16(w);
  } else if (t < n0 + n1) {
    const int u = t - n0;
    const int e = u & 7, l = (u >> 3) & 63, s = (u >> 9) & 7, To = u >> 12;
    const int o = 32 * To + (l & 31), i = fit_hid(s >> 1, 8 * (s & 1) + e, l >> 5);
    L1[u] = fit_bf16(W1[o * kHid + i]);
  } else if (t < n0 + 2 * n1) {
    const int u = t - n0 - n1;
    const int e = u & 7, l = (u >> 3) & 63, s = (u >> 9) & 7, T = u >> 12;
    const int i = 32 * T + (l & 31), o = fit_hid(s >> 1, 8 * (s & 1) + e, l >> 5);
    LT[u] = fit_bf16(W1[o * kHid + i]);
  } else if (t < n0 + 2 * n1 + kHid) {
    const int o = t - n0 - 2 * n1;
    c1[o] = -kFitLog2e * b1[o];
    w2[o] = -kFitLn2 * W2[o];
  }
}

// ---------------------------------------------------------------------------- gathers

// Species of the 14 layer-0 slots a lane group feeds: slots 4s + 2g + e (s = 0..6, e = 0, 1);
// slot 27 is the constant-one bias input and reads as species 0.
__device__ __forceinline__ void fit_gather(const uint8_t *occ, Pos p, int32_t L, int g, uint32_t sp[14]) {
#pragma unroll
  for (int s = 0; s < 7; ++s)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int m0 = 4 * s + e, m1 = 4 * s + 2 + e;
      const int dx0 = m0 ? shell_dx(m0 - 1) : 0, dy0 = m0 ? shell_dy(m0 - 1) : 0, dz0 = m0 ? shell_dz(m0 - 1) : 0;
      const int dx1 = m1 <= 26 ? shell_dx(m1 - 1) : 0, dy1 = m1 <= 26 ? shell_dy(m1 - 1) : 0,
                dz1 = m1 <= 26 ? shell_dz(m1 - 1) : 0;
      const int dx = g ? dx1 : dx0, dy = g ? dy1 : dy0, dz = g ? dz1 : dz0;
      const uint32_t v = occ[site_at(p, dx, dy, dz, L, L, L)];
      sp[2 * s + e] = (g && m1 == 27) ? 0u : v;
    }
}

struct FitArgs {
  const uint8_t *snap;  // [batch][n_sites]
  int32_t L;
  int64_t n_sites, n_rows;
  const uint8_t *pack, *w1t;
  const float *b2;      // forward: the output bias in the FP32 blob
  const double *gE;     // backward: [batch] upstream gradient per snapshot
  float *partial;       // backward: [gridDim.x][kFitParams]
  double *row_e;        // forward: [n_rows]
};

// ---------------------------------------------------------------------------- forward

__global__ __launch_bounds__(kFitFwdThreads) void k_fit_fwd_bf16(FitArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t s_w[kFitPack];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 5;
  for (int q = tid; q < kFitPack / 16; q += kFitFwdThreads) ((int4 *)s_w)[q] = ((const int4 *)a.pack)[q];
  __syncthreads();
  EvalSmem S;
  S.w = s_w;
  S.c1 = (const float *)(s_w + kFitW0 + kFitW1);
  S.c0 = S.c1;
  S.w2 = S.c1 + kHid;
  S.b2 = *a.b2;
  S.k_scale_a0 = S.k_scale_a1 = S.k_scale_h = 127;
  S.sh = 1.0f;
  const int64_t n_tiles = (a.n_rows + 31) / 32;
  for (int64_t tile = (int64_t)blockIdx.x * 8 + wave; tile < n_tiles; tile += (int64_t)gridDim.x * 8) {
    const int64_t row = tile * 32 + (lane & 31);
    const bool valid = row < a.n_rows;
    const int64_t r = valid ? row : 0;
    const int64_t b = r / a.n_sites, j = r - b * a.n_sites;
    uint32_t sp[14];
    fit_gather(a.snap + b * a.n_sites, site_pos(j, a.L, a.L), a.L, g, sp);
    const float E = eval_tile<kPBF16>(S, [&](int m) -> uint32_t { return sp[(m >> 2) * 2 + (m & 1)]; });
    if (valid && lane < 32) a.row_e[row] = (double)E;
  }
}

// S[b] = sum of the rows of snapshot b, in a fixed order (one block per snapshot).
__global__ void k_fit_snap_sum(const double *row_e, int64_t n_sites, double *S) {
  __shared__ double s_p[256];
  const int b = blockIdx.x, t = threadIdx.x;
  double acc = 0.0;
  for (int64_t j = t; j < n_sites; j += 256) acc += row_e[(int64_t)b * n_sites + j];
  s_p[t] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) s_p[t] += s_p[t + w];
    __syncthreads();
  }
  if (t == 0) S[b] = s_p[0];
}

// Fit objective (one block): loss = mean_b ((S_b - E_b)/N)^2 and gs_b = dloss/dS_b.
__global__ void k_fit_loss(const double *S, const double *label, int32_t batch, double n_sites, double *gs,
                           double *loss) {
  __shared__ double s_p[256];
  const int t = threadIdx.x;
  double acc = 0.0;
  for (int b = t; b < batch; b += 256) {
    const double d = S[b] - label[b];
    acc += (d / n_sites) * (d / n_sites);
    gs[b] = 2.0 * d / (n_sites * n_sites * (double)batch);
  }
  s_p[t] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) s_p[t] += s_p[t + w];
    __syncthreads();
  }
  if (t == 0) *loss = s_p[0] / batch;
}

// ---------------------------------------------------------------------------- backward

__device__ __forceinline__ bf16x8 fit_ld8(const uint16_t *p) { return __builtin_bit_cast(bf16x8, *(const i32x4 *)p); }

// Offset of (unit u, row r) in a [unit][row] BF16 staging tile.  Rows come in 16-byte chunks
// of 8; the chunk index is XOR-ed with the unit so that lanes reading the same chunk of
// consecutive units (the matrix-core operand reads) hit different LDS banks instead of the
// same four (a 256-byte row stride maps every unit to the same banks).
__device__ __forceinline__ int fit_off(int u, int r) { return u * kFitRows + ((((r >> 3) ^ u) & 15) << 3) + (r & 7); }

__device__ __forceinline__ float fit_sum8(const uint16_t *p) {
  const i32x4 w = *(const i32x4 *)p;
  float s = 0.0f;
#pragma unroll
  for (int q = 0; q < 4; ++q) s += bf16_lo_f32((uint32_t)w[q]) + bf16_hi_f32((uint32_t)w[q]);
  return s;
}

// silu'(z) from y = -log2(e) z:  sigma = 1/(1 + 2^y),  silu'(z) = sigma (1 + z (1 - sigma)).
__device__ __forceinline__ float fit_dsilu(float y) {
  const float sg = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(y));
  const float z = -kFitLn2 * y;
  return sg * fmaf(z, 1.0f - sg, 1.0f);
}

// Sum of v over the 32 lanes of this lane group: a butterfly on the 16 values of one
// M-tile.  Afterwards the lane with bits (b4 b3 b2 b1 b0) of lane % 32 holds the sum of
// value 8 b4 + 4 b3 + 2 b2 + b1 (lanes 2k and 2k+1 hold the same sum).
__device__ __forceinline__ float fit_rowsum16(const float (&v)[16], int lane) {
  float x[8];
  const bool b4 = lane & 16, b3 = lane & 8, b2 = lane & 4, b1 = lane & 2;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float keep = b4 ? v[i + 8] : v[i], send = b4 ? v[i] : v[i + 8];
    x[i] = keep + __shfl_xor(send, 16);
  }
  float y[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float keep = b3 ? x[i + 4] : x[i], send = b3 ? x[i] : x[i + 4];
    y[i] = keep + __shfl_xor(send, 8);
  }
  float z[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float keep = b2 ? y[i + 2] : y[i], send = b2 ? y[i] : y[i + 2];
    z[i] = keep + __shfl_xor(send, 4);
  }
  const float keep = b1 ? z[1] : z[0], send = b1 ? z[0] : z[1];
  const float w = keep + __shfl_xor(send, 2);
  return w + __shfl_xor(w, 1);
}

__global__ __launch_bounds__(kFitThreads) void k_fit_bwd_bf16(FitArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t s_pack[kFitPack];
  __shared__ __attribute__((aligned(16))) uint8_t s_w1t[kFitW1];
  __shared__ __attribute__((aligned(16))) uint16_t s_a[kHid * kFitRows];  // h1 (scaled), then gz1
  __shared__ __attribute__((aligned(16))) uint16_t s_b[kHid * kFitRows];  // gz2
  __shared__ uint32_t s_sp[27 * (kFitRows / 8)];                          // 4-bit species [slot][row/8]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 5, l32 = lane & 31;
  for (int q = tid; q < kFitPack / 16; q += kFitThreads) ((int4 *)s_pack)[q] = ((const int4 *)a.pack)[q];
  for (int q = tid; q < kFitW1 / 16; q += kFitThreads) ((int4 *)s_w1t)[q] = ((const int4 *)a.w1t)[q];
  const i32x4 *A0 = (const i32x4 *)s_pack;
  const i32x4 *A1 = (const i32x4 *)(s_pack + kFitW0);
  const i32x4 *AT = (const i32x4 *)s_w1t;
  const float *c1v = (const float *)(s_pack + kFitW0 + kFitW1), *w2v = c1v + kHid;

  f32x16 accW1[kMT], accW0[kMT];  // this wave's quarter of dW1 (o tile = wave) and dW0 (f tile = wave)
#pragma unroll
  for (int T = 0; T < kMT; ++T)
#pragma unroll
    for (int v = 0; v < 16; ++v) accW1[T][v] = accW0[T][v] = 0.0f;
  float db1 = 0.0f, dw2[kMT] = {0.0f, 0.0f, 0.0f, 0.0f};

  const int64_t n_chunks = (a.n_rows + kFitRows - 1) / kFitRows;
  const int rl = 32 * wave + l32;  // row within the chunk
  // Stage one BF16 value per (unit, row): register pair q of (T, hh) holds units
  // u = 32T + 8j + 4g + i with j = 2hh + q/2, i = 2(q%2) + e.  In fit_off the swizzle term
  // (row chunk) ^ (u & 15) splits into a per-lane part (chunk ^ 4g) and K = 8(j%2) + i, which
  // takes eight values; their offsets are computed once, so each write is base + constant.
  int sbase[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int K = 8 * (k >> 2) + (k & 3);
    sbase[k] = 128 * (4 * g) + 8 * (((rl >> 3) ^ (4 * g) ^ K) & 15) + (rl & 7);
  }
  auto stage = [&](uint16_t *dst, int T, int hh, const i32x4 &p) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int j = 2 * hh + (q >> 1), i = 2 * (q & 1) + e;
        const int k = 4 * (j & 1) + i;  // K = 8 (j % 2) + i
        dst[sbase[k] + kFitRows * (32 * T + 8 * j + i)] = (uint16_t)((uint32_t)p[q] >> (16 * e));
      }
  };
  for (int64_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
    for (int q = tid; q < 27 * (kFitRows / 8); q += kFitThreads) s_sp[q] = 0u;
    const int64_t row = chunk * kFitRows + rl;
    const bool valid = row < a.n_rows;
    const int64_t r = valid ? row : 0;
    const int64_t b = r / a.n_sites, j = r - b * a.n_sites;
    const float gs = valid ? (float)a.gE[b] : 0.0f;
    uint32_t sp[14];
    fit_gather(a.snap + b * a.n_sites, site_pos(j, a.L, a.L), a.L, g, sp);
    __syncthreads();  // weights loaded (first chunk); s_sp cleared; previous chunk's reads done
#pragma unroll
    for (int s = 0; s < 7; ++s)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int m = 4 * s + 2 * g + e;
        if (m < 27) atomicOr(&s_sp[m * (kFitRows / 8) + (rl >> 3)], sp[2 * s + e] << (4 * (rl & 7)));
      }

    // ---------------------------------------------------------------- layer 0: y1
    f32x16 acc0[kMT];
#pragma unroll
    for (int T = 0; T < kMT; ++T)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc0[T][v] = 0.0f;
#pragma unroll
    for (int s = 0; s < 7; ++s) {
      uint32_t l0, h0, l1, h1;
      onehot_bf16(sp[2 * s], l0, h0);
      onehot_bf16(sp[2 * s + 1], l1, h1);
      i32x4 bw;
      bw[0] = (int)l0; bw[1] = (int)h0; bw[2] = (int)l1; bw[3] = (int)h1;
      const bf16x8 B = __builtin_bit_cast(bf16x8, bw);
#pragma unroll
      for (int T = 0; T < kMT; ++T)
        acc0[T] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, A0[(T * 7 + s) * 64 + lane]), B,
                                                          acc0[T], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
    // ---------------------------------------------------------------- layer 1: y2 (h1 staged)
    f32x16 acc1[kMT];
#pragma unroll
    for (int T = 0; T < kMT; ++T)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const f32x4 c = *(const f32x4 *)(c1v + 32 * T + 8 * jj + 4 * g);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc1[T][4 * jj + i] = c[i];
      }
#pragma unroll
    for (int T = 0; T < kMT; ++T)
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        i32x4 a1p;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          a1p[q] = (int)pack_bf16x2(act(acc0[T][8 * hh + 2 * q], 1.0f), act(acc0[T][8 * hh + 2 * q + 1], 1.0f));
        const bf16x8 B = __builtin_bit_cast(bf16x8, a1p);
#pragma unroll
        for (int To = 0; To < kMT; ++To)
          acc1[To] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              __builtin_bit_cast(bf16x8, A1[(To * 8 + 2 * T + hh) * 64 + lane]), B, acc1[To], 0, 0, 0);
        stage(s_a, T, hh, a1p);
        __builtin_amdgcn_sched_barrier(0);
      }
    // ---------------------------------------------------------------- dW2 += sum_r gE h2; gz2 (staged)
    i32x4 g2p[kMT][2];
#pragma unroll
    for (int T = 0; T < kMT; ++T) {
      float hg[16];
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const f32x4 wa = *(const f32x4 *)(w2v + 32 * T + 8 * (2 * hh) + 4 * g);
        const f32x4 wb = *(const f32x4 *)(w2v + 32 * T + 8 * (2 * hh + 1) + 4 * g);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float gz[2];
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const int v = 8 * hh + 2 * q + e;
            const float y = acc1[T][v];
            const float w2s = (2 * q + e) < 4 ? wa[2 * q + e] : wb[2 * q + e - 4];  // -ln2 W2[o]
            const float sg = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(y));
            const float z = -kFitLn2 * y;
            gz[e] = gs * (-kFitLog2e * w2s) * (sg * fmaf(z, 1.0f - sg, 1.0f));
            hg[v] = gs * (z * sg);  // gE silu(z2)
          }
          g2p[T][hh][q] = (int)pack_bf16x2(gz[0], gz[1]);
        }
        stage(s_b, T, hh, g2p[T][hh]);
      }
      dw2[T] += fit_rowsum16(hg, lane);
    }
    // ---------------------------------------------------------------- gh1 = W1^T gz2, gz1
    f32x16 accg[kMT];
#pragma unroll
    for (int T = 0; T < kMT; ++T)
#pragma unroll
      for (int v = 0; v < 16; ++v) accg[T][v] = 0.0f;
#pragma unroll
    for (int T = 0; T < kMT; ++T)
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const bf16x8 B = __builtin_bit_cast(bf16x8, g2p[T][hh]);
#pragma unroll
        for (int Ti = 0; Ti < kMT; ++Ti)
          accg[Ti] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              __builtin_bit_cast(bf16x8, AT[(Ti * 8 + 2 * T + hh) * 64 + lane]), B, accg[Ti], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
    i32x4 g1p[kMT][2];
#pragma unroll
    for (int T = 0; T < kMT; ++T)
#pragma unroll
      for (int hh = 0; hh < 2; ++hh)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int v = 8 * hh + 2 * q;
          g1p[T][hh][q] = (int)pack_bf16x2(accg[T][v] * fit_dsilu(acc0[T][v]), accg[T][v + 1] * fit_dsilu(acc0[T][v + 1]));
        }

    // ---------------------------------------------------------------- phase A: dW1, db1
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kFitRows / 16; ++k) {
      const bf16x8 A = fit_ld8(s_b + fit_off(32 * wave + l32, 16 * k + 8 * g));
#pragma unroll
      for (int nt = 0; nt < kMT; ++nt)
        accW1[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, fit_ld8(s_a + fit_off(32 * nt + l32, 16 * k + 8 * g)),
                                                            accW1[nt], 0, 0, 0);
    }
    {
      const int o = tid >> 1, half = tid & 1;
#pragma unroll
      for (int q = 0; q < 8; ++q) db1 += fit_sum8(s_b + fit_off(o, 64 * half + 8 * q));
    }
    __syncthreads();
    // ---------------------------------------------------------------- phase B: dW0 (+db0)
#pragma unroll
    for (int T = 0; T < kMT; ++T)
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) stage(s_a, T, hh, g1p[T][hh]);
    __syncthreads();
    {
      const int f = 32 * wave + l32, m = f >> 2, c = f & 3;
#pragma unroll
      for (int k = 0; k < kFitRows / 16; ++k) {
        const uint32_t word = m < 27 ? s_sp[m * (kFitRows / 8) + 2 * k + g] : 0u;
        i32x4 bw;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          uint32_t d = 0;
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const uint32_t nib = (word >> (4 * (2 * q + e))) & 15u;
            const bool one = m < 27 ? nib == (uint32_t)c : (m == 27 && c == 0);
            d |= (one ? 0x3F80u : 0u) << (16 * e);
          }
          bw[q] = (int)d;
        }
        const bf16x8 B = __builtin_bit_cast(bf16x8, bw);
#pragma unroll
        for (int mt = 0; mt < kMT; ++mt)
          accW0[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fit_ld8(s_a + fit_off(32 * mt + l32, 16 * k + 8 * g)),
                                                              B, accW0[mt], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // ------------------------------------------------------------------ this block's partial
  float *P = a.partial + (int64_t)blockIdx.x * kFitParams;
#pragma unroll
  for (int nt = 0; nt < kMT; ++nt)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int o = fit_hid(wave, v, g), i = 32 * nt + l32;
      P[kOffW1 + o * kHid + i] = -kFitLn2 * accW1[nt][v];  // staged h1 carried -log2(e)
    }
#pragma unroll
  for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = fit_hid(mt, v, g), f = 32 * wave + l32;
      if (f < kFitF) P[i * kFitF + f] = accW0[mt][v];
      else if (f == kFitF) P[kOffB0 + i] = accW0[mt][v];
    }
  // dW2: every wave summed its own rows; even lanes of each group hold register
  // 8 b4 + 4 b3 + 2 b2 + b1 (lane bits 4..1) of every M-tile.  The per-wave sums meet in s_b
  // (free after the last chunk's barrier) and are added in wave order.
  float(*s_w2)[kHid] = (float(*)[kHid])s_b;
  if (!(l32 & 1)) {
    const int v = 8 * ((l32 >> 4) & 1) + 4 * ((l32 >> 3) & 1) + 2 * ((l32 >> 2) & 1) + ((l32 >> 1) & 1);
#pragma unroll
    for (int T = 0; T < kMT; ++T) s_w2[wave][fit_hid(T, v, g)] = dw2[T];
  }
  __syncthreads();
  if (tid < kHid) P[kOffW2 + tid] = (s_w2[0][tid] + s_w2[1][tid]) + (s_w2[2][tid] + s_w2[3][tid]);
  const float d1 = db1 + __shfl_xor(db1, 1);
  if (!(tid & 1)) P[kOffB1 + (tid >> 1)] = d1;
  if (tid == 0) P[kOffB2] = 0.0f;
}

// grad[p] = sum of the block partials in block order; the output bias gets sum_b gE_b N.
__global__ void k_fit_reduce(const float *partial, int32_t n_blocks, const double *gE, int32_t batch, double n_sites,
                             float *grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kFitParams) return;
  double acc = 0.0;
  if (p == kOffB2) {
    for (int b = 0; b < batch; ++b) acc += gE[b] * n_sites;
  } else {
    for (int k = 0; k < n_blocks; ++k) acc += (double)partial[(int64_t)k * kFitParams + p];
  }
  grad[p] = (float)acc;
}

// ---------------------------------------------------------------------------- Adam

// Adam (Kingma and Ba) on FP32 master weights, in the bias-corrected form
// p -= (lr / (1 - b1^t)) m / (sqrt(v) / sqrt(1 - b2^t) + eps).
__global__ void k_adam(float *p, float *m, float *v, const float *grad, int32_t n, float lr, float beta1, float beta2,
                       float eps, float bc1, float bc2_sqrt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gr = grad[i];
  const float mi = beta1 * m[i] + (1.0f - beta1) * gr;
  const float vi = beta2 * v[i] + (1.0f - beta2) * gr * gr;
  m[i] = mi;
  v[i] = vi;
  p[i] -= (lr / bc1) * (mi / (sqrtf(vi) / bc2_sqrt + eps));
}

// ---------------------------------------------------------------------------- reference path

template <typename T>
__device__ __forceinline__ T fit_silu(T z) {
  return z / (T(1) + exp(-z));
}
template <typename T>
__device__ __forceinline__ T fit_dsilu_ref(T z) {
  const T s = T(1) / (T(1) + exp(-z));
  return s * (T(1) + z * (T(1) - s));
}

struct FitRefArgs {
  const uint8_t *snap;
  int32_t L;
  int64_t n_sites;
  int64_t r0;     // first row of this chunk
  int32_t rc;     // rows in this chunk
  const double *gE;
  uint8_t *sp;    // [rc][27]
};

__global__ void k_ref_species(FitRefArgs a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)a.rc * 27) return;
  const int64_t rr = t / 27;
  const int m = (int)(t - rr * 27);
  const int64_t r = a.r0 + rr, b = r / a.n_sites, j = r - b * a.n_sites;
  const Pos p = site_pos(j, a.L, a.L);
  const int k = m - 1;
  const int dx = m ? shell_dx(k) : 0, dy = m ? shell_dy(k) : 0, dz = m ? shell_dz(k) : 0;
  a.sp[t] = a.snap[b * a.n_sites + site_at(p, dx, dy, dz, a.L, a.L, a.L)];
}

template <typename T>
__global__ void k_ref_l0(FitRefArgs a, const T *W, T *Z1) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)a.rc * kHid) return;
  const int64_t r = t / kHid;
  const int o = (int)(t - r * kHid);
  T z = W[kOffB0 + o];
  for (int m = 0; m < 27; ++m) {
    const int s = a.sp[r * 27 + m];
    if (s < 4) z += W[o * kFitF + 4 * m + s];
  }
  Z1[t] = z;
}

template <typename T>
__global__ void k_ref_l1(FitRefArgs a, const T *W, const T *Z1, T *Z2) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)a.rc * kHid) return;
  const int64_t r = t / kHid;
  const int o = (int)(t - r * kHid);
  T z = W[kOffB1 + o];
  for (int i = 0; i < kHid; ++i) z += W[kOffW1 + o * kHid + i] * fit_silu(Z1[r * kHid + i]);
  Z2[t] = z;
}

template <typename T>
__global__ void k_ref_out(FitRefArgs a, const T *W, const T *Z2, double *row_e) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.rc) return;
  T e = W[kOffB2];
  for (int o = 0; o < kHid; ++o) e += W[kOffW2 + o] * fit_silu(Z2[r * kHid + o]);
  row_e[a.r0 + r] = (double)e;
}

template <typename T>
__global__ void k_ref_g2(FitRefArgs a, const T *W, const T *Z2, T *G2) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)a.rc * kHid) return;
  const int64_t r = t / kHid;
  const int o = (int)(t - r * kHid);
  const T g = (T)a.gE[(a.r0 + r) / a.n_sites];
  G2[t] = g * W[kOffW2 + o] * fit_dsilu_ref(Z2[t]);
}

template <typename T>
__global__ void k_ref_g1(FitRefArgs a, const T *W, const T *Z1, const T *G2, T *G1) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)a.rc * kHid) return;
  const int64_t r = t / kHid;
  const int i = (int)(t - r * kHid);
  T s = 0;
  for (int o = 0; o < kHid; ++o) s += W[kOffW1 + o * kHid + i] * G2[r * kHid + o];
  G1[t] = s * fit_dsilu_ref(Z1[t]);
}

// One thread per parameter: this chunk's rows summed in order, added to acc[p].
template <typename T>
__global__ void k_ref_wgrad(FitRefArgs a, const T *Z1, const T *Z2, const T *G1, const T *G2, double *acc) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kFitParams) return;
  double s = 0.0;
  if (p < kOffB0) {
    const int o = p / kFitF, f = p - o * kFitF, m = f >> 2, c = f & 3;
    for (int r = 0; r < a.rc; ++r)
      if (a.sp[(int64_t)r * 27 + m] == c) s += (double)G1[(int64_t)r * kHid + o];
  } else if (p < kOffW1) {
    const int o = p - kOffB0;
    for (int r = 0; r < a.rc; ++r) s += (double)G1[(int64_t)r * kHid + o];
  } else if (p < kOffB1) {
    const int o = (p - kOffW1) / kHid, i = (p - kOffW1) % kHid;
    for (int r = 0; r < a.rc; ++r) s += (double)(G2[(int64_t)r * kHid + o] * fit_silu(Z1[(int64_t)r * kHid + i]));
  } else if (p < kOffW2) {
    const int o = p - kOffB1;
    for (int r = 0; r < a.rc; ++r) s += (double)G2[(int64_t)r * kHid + o];
  } else if (p < kOffB2) {
    const int o = p - kOffW2;
    for (int r = 0; r < a.rc; ++r)
      s += a.gE[(a.r0 + r) / a.n_sites] * (double)fit_silu(Z2[(int64_t)r * kHid + o]);
  } else {
    for (int r = 0; r < a.rc; ++r) s += a.gE[(a.r0 + r) / a.n_sites];
  }
  acc[p] += s;
}

template <typename T>
__global__ void k_fit_convert(const float *in, T *out, int32_t n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (T)in[i];
}

__global__ void k_fit_to_f32(const double *in, float *out, int32_t n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

__global__ void k_fit_zero_f64(double *p, int32_t n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// ---------------------------------------------------------------------------- CE labels

// Per snapshot (one block): sum over sites of the site-local CE energy, half of every pair
// term with the 26 shell-1..3 neighbours plus the cluster table entry of every triangle shape
// anchored at the site.  tab: pair[3][S][S] then J[n_tri][S][S][S] (eV); tri: [n_tri][6].
__global__ void k_ce_energy(const uint8_t *snap, int32_t L, int64_t n_sites, int32_t S, int32_t n_tri,
                            const double *tab, const int8_t *tri, double *out) {
  extern __shared__ double s_tab[];
  const int t = threadIdx.x;
  const int n_tab = 3 * S * S + n_tri * S * S * S;
  for (int q = t; q < n_tab; q += blockDim.x) s_tab[q] = tab[q];
  __shared__ double s_p[256];
  __syncthreads();
  const uint8_t *occ = snap + (int64_t)blockIdx.x * n_sites;
  const double *J = s_tab + 3 * S * S;
  double acc = 0.0;
  for (int64_t s = t; s < n_sites; s += blockDim.x) {
    const Pos p = site_pos(s, L, L);
    const int c = occ[s];
    double e = 0.0;
    for (int k = 0; k < kNbr; ++k) {
      const int q = occ[site_at(p, shell_dx(k), shell_dy(k), shell_dz(k), L, L, L)];
      e += 0.5 * s_tab[((shell_of(k) - 1) * S + c) * S + q];
    }
    for (int u = 0; u < n_tri; ++u) {
      const int8_t *o = tri + 6 * u;
      const int qa = occ[site_at(p, o[0], o[1], o[2], L, L, L)];
      const int qb = occ[site_at(p, o[3], o[4], o[5], L, L, L)];
      e += J[((u * S + c) * S + qa) * S + qb];
    }
    acc += e;
  }
  s_p[t] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) s_p[t] += s_p[t + w];
    __syncthreads();
  }
  if (t == 0) out[blockIdx.x] = s_p[0];
}

}  // namespace smc

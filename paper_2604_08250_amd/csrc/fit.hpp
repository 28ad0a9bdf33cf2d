// Kernels of the differentiation pattern: energies of whole snapshots, their gradient with
// respect to the MLP parameters, the fit objective, Adam, and the cluster-expansion labels.
//
// Rows.  Row r of a batch is site j = r mod N of snapshot b = r / N (N = 2 L^3 sites per
// snapshot); its local energy is the MLP of Eqs. (4)-(6) on the one-hot features of the
// site and its 26 shell-1..3 neighbours, and S_b sums the rows of snapshot b.
//
// BF16 path (matrix cores, FP32 accumulation).  Forward: the sweep's tile evaluator.
// Backward: the gradient of the energy sum of each segment of a snapshot (a range of its
// chunks; one segment per snapshot when there are at least as many snapshots as CUs) with a
// unit upstream gradient, and that energy sum; a second kernel weights the segment gradients
// by the upstream gradient of their snapshot.  The loss gradient needs the snapshot energies
// first, so this order lets one pass serve both: the fit step runs no separate forward.
// Per chunk of 128 rows of one snapshot, in a block of eight waves, each wave owning 16 rows
// (16x16 matrix-core tiles: two waves per SIMD fit in the register file):
//   forward again, keeping silu'(z1) from the same exponential and reciprocal as h1;
//   E = W2 . silu(z2) + b2;  gz2 = W2 silu'(z2);  gh1 = W1^T gz2 (matrix cores, W1^T image in LDS);
//   gz1 = gh1 silu'(z1);
// then the weight gradients, which sum over rows, are matrix-core products with the rows as
// the K dimension: the per-row vectors are staged in LDS as [unit][row] BF16 tiles (the
// transposition that puts rows into K), and each wave owns one eighth of dW1 and of dW0:
//   phase A: dW1 = sum_r gz2 (x) h1  and  db1 = sum_r gz2;
//   phase B: dW0 = sum_r gz1 (x) x  (x built from 4-bit species codes in LDS; feature 108 is
//            the constant one, so db0 comes out of the same product).
// dW2 = sum_r h2 is a butterfly over the lanes of each wave.  Each block accumulates the
// chunks of a segment in registers and writes the segment's gradient and energy sum; the
// combination adds them in segment order, so the result does not depend on timing.
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
constexpr int kFitThreads = 512;  // backward block: eight waves of 16 rows
constexpr int kFitRows = 128;     // rows per backward chunk
constexpr int kFitFwdThreads = 512;
constexpr int kFitW0 = PackSize<kPBF16>::kL0;
constexpr int kFitW1 = PackSize<kPBF16>::kL1;
constexpr int kFitPack = kFitW0 + kFitW1 + 2 * kHid * 4;  // layer 0, layer 1, c1, w2 (scaled)
// Backward images (16x16 tiles): layer 0 as 3 K-steps of 32 and one of 16 (112 features),
// layer 1, W1^T, then c1 and w2 as in the forward pack.
constexpr int kBwdW0a = 8 * 3 * 64 * 8;  // BF16 elements of the 16x16x32 steps
constexpr int kBwdW0 = 2 * (kBwdW0a + 8 * 64 * 4);
constexpr int kBwdW1 = 2 * kHid * kHid;
constexpr int kBwdPack = kBwdW0 + 2 * kBwdW1 + 2 * kHid * 4;
constexpr int kOffB0 = kHid * kFitF;
constexpr int kOffW1 = kOffB0 + kHid;
constexpr int kOffB1 = kOffW1 + kHid * kHid;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid;
constexpr int kFitParams = kOffB2 + 1;
constexpr float kFitLog2e = 1.44269504088896340736f;
constexpr float kFitLn2 = 0.69314718055994530942f;

__device__ __forceinline__ int fit_hid(int T, int v, int g) { return 32 * T + 8 * (v >> 2) + 4 * g + (v & 3); }
// Hidden unit behind K slot (lane group g4, element j) of K-step s in a 16x16x32 product whose
// B operand is built from the accumulators of 16-unit tiles 2s and 2s + 1: a lane holds units
// 4 g4 .. 4 g4 + 3 of each tile for its row.
__device__ __forceinline__ int fit_hid16(int s, int g4, int j) { return 16 * (2 * s + (j >> 2)) + 4 * g4 + (j & 3); }

// ---------------------------------------------------------------------------- packing

__device__ __forceinline__ uint16_t fit_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// BF16 images from the FP32 blob.  Forward pack (operand orders of the sweep's tile
// evaluator): layer 0 (-log2(e) W0, bias in feature 108), layer 1 (W1), c1 = -log2(e) b1,
// w2 = -ln(2) W2.  Backward pack (16x16 tiles, A operands; lane l holds row l % 16 and K
// slots 8 (l / 16) .. + 7 of a 16x16x32 step, or 4 (l / 16) .. + 3 of a 16x16x16 step):
// layer 0 (features 32 s + 8 (l / 16) + j, then 96 + 4 (l / 16) + j), layer 1 (W1[o][i]
// with i = fit_hid16(s, l / 16, j)), W1^T (W1[o][i] with o = fit_hid16(s, l / 16, j)), c1, W2.
__device__ __forceinline__ float fit_w0s(const float *W0, const float *b0, int o, int f) {
  return f < kFitF ? -kFitLog2e * W0[o * kFitF + f] : (f == kFitF ? -kFitLog2e * b0[o] : 0.0f);
}

constexpr int kFitPackThreads = kFitW0 / 2 + kFitW1 / 2 + kBwdW0 / 2 + kBwdW1 + kHid;

__global__ void k_fit_pack_bf16(const float *p, uint8_t *pack, uint8_t *bwd) {
  const int n0 = kFitW0 / 2, n1 = kFitW1 / 2, m0 = kBwdW0 / 2, m1 = kBwdW1 / 2;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  const float *W0 = p, *b0 = p + kOffB0, *W1 = p + kOffW1, *b1 = p + kOffB1, *W2 = p + kOffW2;
  uint16_t *L0 = (uint16_t *)pack, *L1 = L0 + n0;
  float *c1 = (float *)(pack + kFitW0 + kFitW1), *w2 = c1 + kHid;
  uint16_t *B0 = (uint16_t *)bwd, *B1 = B0 + m0, *BT = B1 + m1;
  float *bc1 = (float *)(bwd + kBwdW0 + 2 * kBwdW1), *bw2 = bc1 + kHid;
  if (t < n0) {
    const int e = t & 7, l = (t >> 3) & 63, s = (t >> 9) % 7, T = (t >> 9) / 7;
    L0[t] = fit_bf16(fit_w0s(W0, b0, 32 * T + (l & 31), 16 * s + 8 * (l >> 5) + e));
    return;
  }
  t -= n0;
  if (t < n1) {
    const int e = t & 7, l = (t >> 3) & 63, s = (t >> 9) & 7, To = t >> 12;
    const int o = 32 * To + (l & 31), i = fit_hid(s >> 1, 8 * (s & 1) + e, l >> 5);
    L1[t] = fit_bf16(W1[o * kHid + i]);
    return;
  }
  t -= n1;
  if (t < m0) {
    if (t < kBwdW0a) {
      const int j = t & 7, l = (t >> 3) & 63, s = (t >> 9) % 3, T = (t >> 9) / 3;
      B0[t] = fit_bf16(fit_w0s(W0, b0, 16 * T + (l & 15), 32 * s + 8 * (l >> 4) + j));
    } else {
      const int u = t - kBwdW0a, j = u & 3, l = (u >> 2) & 63, T = u >> 8;
      B0[t] = fit_bf16(fit_w0s(W0, b0, 16 * T + (l & 15), 96 + 4 * (l >> 4) + j));
    }
    return;
  }
  t -= m0;
  if (t < 2 * m1) {
    const bool tr = t >= m1;
    const int u = tr ? t - m1 : t;
    const int j = u & 7, l = (u >> 3) & 63, s = (u >> 9) & 3, T = u >> 11;
    const int a = 16 * T + (l & 15), k = fit_hid16(s, l >> 4, j);
    if (tr) BT[u] = fit_bf16(W1[k * kHid + a]);  // A[i = a][o = k]
    else B1[u] = fit_bf16(W1[a * kHid + k]);     // A[o = a][i = k]
    return;
  }
  t -= 2 * m1;
  if (t < kHid) {
    c1[t] = bc1[t] = -kFitLog2e * b1[t];
    w2[t] = -kFitLn2 * W2[t];
    bw2[t] = W2[t];
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

// Species of the 7 layer-0 slots a lane feeds in the backward's 16x16 tiles: slots
// 8 s + 2 g4 + e (s = 0..2, e = 0, 1), then slot 24 + g4 (slot 27, the constant-one input,
// reads the site itself; the caller replaces it by species 0).
__device__ __forceinline__ void fit_gather16(const uint8_t *occ, Pos p, int32_t L, int g4, uint32_t sp[7]) {
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    int dx = 0, dy = 0, dz = 0;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int m = q < 6 ? 8 * (q >> 1) + 2 * g + (q & 1) : 24 + g;
      const int ex = (m && m < 27) ? shell_dx(m - 1) : 0, ey = (m && m < 27) ? shell_dy(m - 1) : 0,
                ez = (m && m < 27) ? shell_dz(m - 1) : 0;
      if (g == g4) { dx = ex; dy = ey; dz = ez; }
    }
    sp[q] = occ[site_at(p, dx, dy, dz, L, L, L)];
  }
}

struct FitArgs {
  const uint8_t *snap;  // [batch][n_sites]
  int32_t L;
  int64_t n_sites, n_rows;
  const uint8_t *pack, *bwd;  // forward and backward BF16 images
  const float *b2;            // forward: the output bias in the FP32 blob
  float *partial;       // backward: [n_seg][kFitParams] gradient of each segment's row energies
  double *row_e;        // forward: [n_rows]; backward: [n_seg] sum of each segment's row energies
  // backward segments: snapshot s / nps, chunks (s % nps) cps .. + cps of its chunks_snap
  int32_t n_seg, nps, cps, chunks_snap;
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

// Fit objective (one block): loss = mean_b ((S_b - E_b)/N)^2 and gs_b = dloss/dS_b, with
// S_b the sum of the nps segment sums S[nps b .. nps b + nps - 1] in order.
__global__ void k_fit_loss(const double *S, int32_t nps, const double *label, int32_t batch, double n_sites,
                           double *gs, double *loss) {
  __shared__ double s_p[256];
  const int t = threadIdx.x;
  double acc = 0.0;
  for (int b = t; b < batch; b += 256) {
    double Sb = 0.0;
    for (int k = 0; k < nps; ++k) Sb += S[(int64_t)b * nps + k];
    const double d = Sb - label[b];
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

// Sum of v over the 16 lanes of this lane group (lane bits 0..3), as a butterfly on the 16
// values.  Afterwards the lane with low bits (b3 b2 b1 b0) holds the sum of value
// 8 b3 + 4 b2 + 2 b1 + b0.
__device__ __forceinline__ float fit_lanesum16(const float (&v)[16], int lane) {
  float x[8];
  const bool b3 = lane & 8, b2 = lane & 4, b1 = lane & 2, b0 = lane & 1;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float keep = b3 ? v[i + 8] : v[i], send = b3 ? v[i] : v[i + 8];
    x[i] = keep + __shfl_xor(send, 8);
  }
  float y[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float keep = b2 ? x[i + 4] : x[i], send = b2 ? x[i] : x[i + 4];
    y[i] = keep + __shfl_xor(send, 4);
  }
  float z[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float keep = b1 ? y[i + 2] : y[i], send = b1 ? y[i] : y[i + 2];
    z[i] = keep + __shfl_xor(send, 2);
  }
  const float keep = b0 ? z[1] : z[0], send = b0 ? z[0] : z[1];
  return keep + __shfl_xor(send, 1);
}

typedef short s16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 fit_mfma16(const i32x4 &a, const i32x4 &b, const f32x4 &c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

// B operand of a 16x16x32 step from the accumulators of 16-unit tiles 2s and 2s + 1: K slot
// (g4, j) holds unit fit_hid16(s, g4, j) of the lane's row.
__device__ __forceinline__ i32x4 fit_bpack(const float (&x)[8][4], int s) {
  i32x4 r;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int T = 2 * s + (q >> 1), v = 2 * (q & 1);
    r[q] = (int)pack_bf16x2(x[T][v], x[T][v + 1]);
  }
  return r;
}

__global__ __launch_bounds__(kFitThreads) void k_fit_bwd_bf16(FitArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t s_pack[kBwdPack];
  __shared__ __attribute__((aligned(16))) uint16_t s_a[kHid * kFitRows];  // h1 (scaled), then gz1
  __shared__ __attribute__((aligned(16))) uint16_t s_b[kHid * kFitRows];  // gz2
  __shared__ uint32_t s_sp[27 * (kFitRows / 8)];                          // 4-bit species [slot][row/8]
  __shared__ __attribute__((aligned(16))) float s_big[kHid];               // layer-1 start of rows past the end
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g4 = lane >> 4, l16 = lane & 15;  // 16x16 roles: lane group, row
  if (tid < kHid) s_big[tid] = 1e30f;
  const int g = lane >> 5, l32 = lane & 31;   // 32x32 roles in the weight-gradient products
  for (int q = tid; q < kBwdPack / 16; q += kFitThreads) ((int4 *)s_pack)[q] = ((const int4 *)a.bwd)[q];
  const i32x4 *A0 = (const i32x4 *)s_pack;                                  // [T][s < 3][lane]
  const s16x4 *A0t = (const s16x4 *)(s_pack + 2 * kBwdW0a);                // [T][lane]: the K = 16 step
  const i32x4 *A1 = (const i32x4 *)(s_pack + kBwdW0);                       // [To][s][lane]
  const i32x4 *AT = (const i32x4 *)(s_pack + kBwdW0 + kBwdW1);              // [Ti][s][lane]
  const float *c1v = (const float *)(s_pack + kBwdW0 + 2 * kBwdW1), *w2v = c1v + kHid;

  // this wave's eighth of dW1 (o tile wave / 2, i tiles 2 (wave % 2) + n) and of dW0
  // (feature tile wave / 2, unit tiles 2 (wave % 2) + n), in 32x32 tiles
  const int t_hi = wave >> 1, t_lo = 2 * (wave & 1);
  f32x16 accW1[2], accW0[2];
#pragma unroll
  for (int n = 0; n < 2; ++n)
#pragma unroll
    for (int v = 0; v < 16; ++v) accW1[n][v] = accW0[n][v] = 0.0f;
  float db1 = 0.0f, dw2[2] = {0.0f, 0.0f};
  double es = 0.0;  // energy sum of this lane's row position over the segment's chunks
  const float b2 = *a.b2;
  const uint32_t N = (uint32_t)a.n_sites;

  const int rl = 16 * wave + l16;  // row within the chunk
  // Staging of one BF16 value per (unit, row): the lane holds units 16 T + 4 g4 + v of its
  // row; in fit_off the swizzle term (row chunk) ^ (u & 15) depends on v only, so the four
  // offsets are computed once and each write is base + 2048 T.
  int sbase[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) sbase[v] = fit_off(4 * g4 + v, rl);
  auto stage = [&](uint16_t *dst, const i32x4 (&b)[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int T = 2 * s + (q >> 1), v = 2 * (q & 1) + e;
          dst[sbase[v] + kFitRows * 16 * T] = (uint16_t)((uint32_t)b[s][q] >> (16 * e));
        }
  };
  // the block walks (segment, chunk) items: segments blockIdx.x + k gridDim.x, each over its
  // chunk range; the species of the next item are loaded one item ahead (consumed only in the
  // next iteration, so the loads overlap this chunk's work)
  auto c_begin = [&](int seg) { return (seg % a.nps) * a.cps; };
  auto c_end = [&](int seg) { return min(a.chunks_snap, (seg % a.nps + 1) * a.cps); };
  uint32_t spn[7];
  auto fetch = [&](int seg, int c) {
    const uint32_t j = (uint32_t)c * kFitRows + rl;
    const uint32_t jj = j < N ? j : 0u;
    fit_gather16(a.snap + (int64_t)(seg / a.nps) * a.n_sites, site_pos32((int32_t)jj, a.L, a.L), a.L, g4, spn);
  };
  int seg = blockIdx.x, c = seg < a.n_seg ? c_begin(seg) : 0;
  if (seg < a.n_seg) fetch(seg, c);
  while (seg < a.n_seg) {
    uint32_t sp[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) sp[q] = spn[q];
    if (g4 == 3) sp[6] = 0u;  // slot 27: the constant-one input, species 0
    const bool valid = (uint32_t)c * kFitRows + rl < N;
    int nseg = seg, nc = c + 1;
    if (nc >= c_end(seg)) {
      nseg = seg + gridDim.x;
      nc = nseg < a.n_seg ? c_begin(nseg) : 0;
    }
    __syncthreads();  // weights loaded (first chunk); the previous chunk's LDS reads done
    if (nseg < a.n_seg) fetch(nseg, nc);
    // species words for phase B: row 8 c + i of a slot goes to nibble 2 (i % 4) + i / 4 of
    // word c (byte i % 4 holds rows i and i + 4).  The eight lanes of a row octet OR their
    // nibbles together with row shifts, and the last of them writes the word (every word of
    // every slot below 27 is written).
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      const int m = q < 6 ? 8 * (q >> 1) + 2 * g4 + (q & 1) : 24 + g4;
      uint32_t w = sp[q] << (8 * (l16 & 3) + 4 * ((l16 >> 2) & 1));
      w |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0x111, 0xf, 0xf, true);  // row_shr:1
      w |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0x112, 0xf, 0xf, true);  // row_shr:2
      w |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0x114, 0xf, 0xf, true);  // row_shr:4
      if (m < 27 && (l16 & 7) == 7) s_sp[m * (kFitRows / 8) + (rl >> 3)] = w;
    }

    // ---------------------------------------------------------------- layer 0: y1
    f32x4 acc[8];
#pragma unroll
    for (int T = 0; T < 8; ++T) acc[T] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      uint32_t l0, h0, l1, h1;
      onehot_bf16(sp[2 * s], l0, h0);
      onehot_bf16(sp[2 * s + 1], l1, h1);
      const i32x4 B = {(int)l0, (int)h0, (int)l1, (int)h1};
#pragma unroll
      for (int T = 0; T < 8; ++T) acc[T] = fit_mfma16(A0[(T * 3 + s) * 64 + lane], B, acc[T]);
    }
    {
      uint32_t l0, h0;
      onehot_bf16(sp[6], l0, h0);
      const s16x4 B = __builtin_bit_cast(s16x4, (uint64_t)l0 | ((uint64_t)h0 << 32));
#pragma unroll
      for (int T = 0; T < 8; ++T) acc[T] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A0t[T * 64 + lane], B, acc[T], 0, 0, 0);
    }
    // h1 = silu(z1) (times -log2(e)) and silu'(z1) from one exponential and reciprocal
    float h[8][4], ds1[8][4];
#pragma unroll
    for (int T = 0; T < 8; ++T)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float y = acc[T][v];
        const float sg = __builtin_amdgcn_rcpf(fmaf(__builtin_amdgcn_exp2f(y), 1.0f, 1.0f));
        h[T][v] = y * sg;
        ds1[T][v] = sg * fmaf(-kFitLn2 * y, 1.0f - sg, 1.0f);
      }
    i32x4 hb[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) hb[s] = fit_bpack(h, s);
    stage(s_a, hb);
    // ---------------------------------------------------------------- layer 1: y2
    // rows past the snapshot's last site start from a huge pre-activation: silu(z2) and
    // silu'(z2) are then zero, so they add nothing to any gradient or energy
    const float *c1r = valid ? c1v : s_big;
#pragma unroll
    for (int T = 0; T < 8; ++T) acc[T] = *(const f32x4 *)(c1r + 16 * T + 4 * g4);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int T = 0; T < 8; ++T) acc[T] = fit_mfma16(A1[(T * 4 + s) * 64 + lane], hb[s], acc[T]);
    // ---------------------------------------------------------------- E, gz2, dW2 += sum_r h2
    float gz[8][4], hg[2][16], ep = 0.0f;
#pragma unroll
    for (int T = 0; T < 8; ++T) {
      const f32x4 w2 = *(const f32x4 *)(w2v + 16 * T + 4 * g4);  // W2[o]
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float y = acc[T][v];
        const float sg = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(y));
        const float z = -kFitLn2 * y, zs = z * sg;  // silu(z2)
        gz[T][v] = w2[v] * (sg * fmaf(z, 1.0f - sg, 1.0f));
        hg[T >> 2][4 * (T & 3) + v] = zs;
        ep = fmaf(w2[v], zs, ep);
      }
    }
    dw2[0] += fit_lanesum16(hg[0], lane);
    dw2[1] += fit_lanesum16(hg[1], lane);
    // row energy: the four lane groups of the row hold disjoint units
    ep += __shfl_xor(ep, 16);
    ep += __shfl_xor(ep, 32);
    if (valid) es += (double)(ep + b2);
    i32x4 gb[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) gb[s] = fit_bpack(gz, s);
    stage(s_b, gb);
    // ---------------------------------------------------------------- gh1 = W1^T gz2, gz1
#pragma unroll
    for (int T = 0; T < 8; ++T) acc[T] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int T = 0; T < 8; ++T) acc[T] = fit_mfma16(AT[(T * 4 + s) * 64 + lane], gb[s], acc[T]);
#pragma unroll
    for (int T = 0; T < 8; ++T)
#pragma unroll
      for (int v = 0; v < 4; ++v) gz[T][v] = acc[T][v] * ds1[T][v];
    i32x4 g1b[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) g1b[s] = fit_bpack(gz, s);

    // ---------------------------------------------------------------- phase A: dW1, db1
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kFitRows / 16; ++k) {
      const bf16x8 A = fit_ld8(s_b + fit_off(32 * t_hi + l32, 16 * k + 8 * g));
#pragma unroll
      for (int n = 0; n < 2; ++n)
        accW1[n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
            A, fit_ld8(s_a + fit_off(32 * (t_lo + n) + l32, 16 * k + 8 * g)), accW1[n], 0, 0, 0);
    }
    {
      const int o = tid >> 2, part = tid & 3;
#pragma unroll
      for (int q = 0; q < 4; ++q) db1 += fit_sum8(s_b + fit_off(o, 32 * part + 8 * q));
    }
    __syncthreads();
    // ---------------------------------------------------------------- phase B: dW0 (+db0)
    stage(s_a, g1b);
    __syncthreads();
    {
      // x[row][f] as BF16 one-hot values by byte permutes: with the species of four rows as
      // bytes b, the selector (b | 4, b, ...) picks byte b of K80 = 0x80 << 8c and of
      // K3F = 0x3F << 8c, giving 0x3F80 (one) where b == c and zero elsewhere; the byte 0x0C
      // selects the constant zero (features past the bias; the bias slot reads species 0)
      const int f = 32 * t_hi + l32, m = f >> 2, cc = f & 3;
      const uint32_t k80 = 0x80u << (8 * cc), k3f = 0x3Fu << (8 * cc);
      auto onehot2 = [&](uint32_t sb, uint32_t sel) -> int {
        return (int)__builtin_amdgcn_perm(k80, k3f, __builtin_amdgcn_perm(sb | 0x04040404u, sb, sel));
      };
#pragma unroll
      for (int k = 0; k < kFitRows / 16; ++k) {
        const uint32_t word = m < 27 ? s_sp[m * (kFitRows / 8) + 2 * k + g] : (m == 27 ? 0u : 0xCCCCCCCCu);
        const uint32_t r03 = word & 0x0F0F0F0Fu, r47 = (word >> 4) & 0x0F0F0F0Fu;
        const i32x4 bw = {onehot2(r03, 0x01050004u), onehot2(r03, 0x03070206u), onehot2(r47, 0x01050004u),
                          onehot2(r47, 0x03070206u)};
        const bf16x8 B = __builtin_bit_cast(bf16x8, bw);
#pragma unroll
        for (int n = 0; n < 2; ++n)
          accW0[n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fit_ld8(s_a + fit_off(32 * (t_lo + n) + l32, 16 * k + 8 * g)),
                                                             B, accW0[n], 0, 0, 0);
      }
    }
    if (nseg != seg) {
      // ---------------------------------------------------------------- segment done: flush
      __syncthreads();  // every wave's phase A (s_b reads) and phase B are done
      float *P = a.partial + (int64_t)seg * kFitParams;
      {
        // dW1[o][i]: o = fit_hid(t_hi, v, g), i = 32 (t_lo + n) + l32
        float *pw = P + kOffW1 + (32 * t_hi + 4 * g) * kHid + 32 * t_lo + l32;
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            pw[(8 * (v >> 2) + (v & 3)) * kHid + 32 * n] = -kFitLn2 * accW1[n][v];  // staged h1 carried -log2(e)
            accW1[n][v] = 0.0f;
          }
        // dW0[i][f] (f < 108) and db0[i] (f = 108): i = fit_hid(t_lo + n, v, g), f = 32 t_hi + l32
        const int f = 32 * t_hi + l32;
        float *pb = f < kFitF ? P + (32 * t_lo + 4 * g) * kFitF + f : P + kOffB0 + 32 * t_lo + 4 * g;
        const int stride = f < kFitF ? kFitF : 1;
        if (f <= kFitF) {
#pragma unroll
          for (int n = 0; n < 2; ++n)
#pragma unroll
            for (int v = 0; v < 16; ++v) pb[(32 * n + 8 * (v >> 2) + (v & 3)) * stride] = accW0[n][v];
        }
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
          for (int v = 0; v < 16; ++v) accW0[n][v] = 0.0f;
      }
      // dW2 and the energy sum meet in s_b: lane (g4, l16) holds unit 16 (4 h + l16 / 4) +
      // 4 g4 + l16 % 4 of half h; lanes of lane group 0 hold the row sums
      float(*s_w2)[kHid] = (float(*)[kHid])s_b;
      double *s_e = (double *)(s_b + 8 * kHid * 2);
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) s_w2[wave][16 * (4 * hf + (l16 >> 2)) + 4 * g4 + (l16 & 3)] = dw2[hf];
      if (g4 == 0) s_e[rl] = es;
      dw2[0] = dw2[1] = 0.0f;
      es = 0.0;
      __syncthreads();
      if (tid < kHid) {
        float sum = 0.0f;
#pragma unroll
        for (int w = 0; w < 8; ++w) sum += s_w2[w][tid];
        P[kOffW2 + tid] = sum;
      } else if (tid == kHid) {
        double e = 0.0;
        for (int r = 0; r < kFitRows; ++r) e += s_e[r];
        a.row_e[seg] = e;
      }
      const float d1 = (db1 + __shfl_xor(db1, 1)) + (__shfl_xor(db1, 2) + __shfl_xor(db1, 3));
      if (!(tid & 3)) P[kOffB1 + (tid >> 2)] = d1;
      db1 = 0.0f;
      if (tid == 0) P[kOffB2] = (float)(min(N, (uint32_t)c_end(seg) * kFitRows) - (uint32_t)c_begin(seg) * kFitRows);
    }
    seg = nseg;
    c = nc;
  }
}

// grad[p] = sum over segments s of ge[s / nps] * partial[s][p] in segment order: wave w of the
// block sums segments w, w + 8, ... and the eight sums are added in wave order.  The output
// bias entry of a segment holds its row count, so that entry becomes sum_b ge_b N.
__global__ __launch_bounds__(512) void k_fit_combine(const float *partial, int32_t n_seg, int32_t nps,
                                                     const double *ge, float *grad) {
  __shared__ double s_acc[8][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int p = blockIdx.x * 64 + lane;
  double acc = 0.0;
  if (p < kFitParams) {
#pragma unroll 4
    for (int s = w; s < n_seg; s += 8) acc += ge[s / nps] * (double)partial[(int64_t)s * kFitParams + p];
  }
  s_acc[w][lane] = acc;
  __syncthreads();
  if (w == 0 && p < kFitParams) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) t += s_acc[k][lane];
    grad[p] = (float)t;
  }
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

// Host side of the FCC lattice path: MLPNet weight images, zone tables, context set-up, local
// energies and the enqueue of one sweep.  Included once, by the translation unit of the C ABI
// (the generic kernels it launches are defined there).
#pragma once
#include <math.h>

#include <algorithm>
#include <array>
#include <vector>

#include "context.hpp"
#include "fcc.hpp"
#include "pack.hpp"
#include "reduce.hpp"
#include "sweep_mfma.hpp"

namespace smc {
namespace fcc {

constexpr int kNetParams = kHid * kIn + kHid + 2 * (kHid * kHid + kHid) + kHid + 1;  // 26,113

// Hidden unit held in output register v by lane group g of M-tile T.
inline int unit_of(int T, int v, int g) { return 32 * T + 8 * (v / 4) + 4 * g + (v % 4); }

// Smallest k with x <= 2^k (0 for x <= 0).
inline int pow2_at_least(double x) { return x > 0.0 ? (int)ceil(log2(x)) : 0; }

// FP8 image: E4M3 weights with a power-of-two scale per layer (k0, k1, k2: the largest |W|
// maps to at most 448).  The activation entering layer l + 1 is relu(z_l) / 2^kh_l, with
// kh_l from a bound of relu(z_l) that follows from the weights: z_0 <= b0 + the sum over
// slots of the largest positive weight of the slot, z_1 <= b1 + sum_k max(W1, 0) hmax_0.
// Layers 0 and 1 accumulate in units of the next activation scale (their bias is divided by
// 2^kh), so relu of the accumulator converts to E4M3 as it is; layer 2 accumulates in eV.
// The scaled products take A scale 2^(k - kh_next) or 2^k and B scale 2^(kh_in - kh_next).
inline void pack_net_fp8(const float *p, uint8_t *B) {
  constexpr int L0 = NetSize<kPFP8>::kL0, L1 = NetSize<kPFP8>::kL1;
  const float *W0 = p, *b0 = W0 + kHid * kIn, *W1 = b0 + kHid, *b1 = W1 + kHid * kHid, *W2 = b1 + kHid,
              *b2 = W2 + kHid * kHid, *W3 = b2 + kHid;
  double a0 = 0, a1 = 0, a2 = 0;
  for (int i = 0; i < kHid * kIn; ++i) a0 = std::max(a0, (double)fabsf(W0[i]));
  for (int i = 0; i < kHid * kHid; ++i) {
    a1 = std::max(a1, (double)fabsf(W1[i]));
    a2 = std::max(a2, (double)fabsf(W2[i]));
  }
  const int k0 = pow2_at_least(a0 / 448.0), k1 = pow2_at_least(a1 / 448.0), k2 = pow2_at_least(a2 / 448.0);
  double h0 = 0.0, h1 = 0.0;
  for (int o = 0; o < kHid; ++o) {
    double z = b0[o];
    for (int m = 0; m < kSlots; ++m) {
      double best = 0.0;
      for (int c = 0; c < 4; ++c) best = std::max(best, (double)W0[o * kIn + 4 * m + c]);
      z += best;
    }
    h0 = std::max(h0, z);
  }
  for (int o = 0; o < kHid; ++o) {
    double z = b1[o];
    for (int k = 0; k < kHid; ++k) z += std::max(0.0, (double)W1[o * kHid + k]) * h0;
    h1 = std::max(h1, z);
  }
  const int kh0 = pow2_at_least(h0 / 448.0), kh1 = pow2_at_least(h1 / 448.0);
  auto e8 = [](int v) { return (uint32_t)std::min(254, std::max(0, v)); };
  const uint32_t sa0 = e8(127 + k0 - kh0), sa1 = e8(127 + k1), sa2 = e8(127 + k2), sb1 = e8(127 + kh0 - kh1),
                 sb2 = e8(127 + kh1);
  const float i0 = ldexpf(1.0f, -k0), i1 = ldexpf(1.0f, -k1), i2 = ldexpf(1.0f, -k2);
  uint8_t *A0 = B, *A1 = B + L0, *A2 = B + L0 + L1;
  for (int T = 0; T < kMT; ++T)
    for (int s = 0; s < 2; ++s)
      for (int l = 0; l < 64; ++l)
        for (int e = 0; e < 32; ++e) {
          const int o = 32 * T + (l & 31), f = 64 * s + 32 * (l >> 5) + e;
          const size_t idx = ((size_t)(T * 2 + s) * 64 + l) * 32 + e;
          A0[idx] = f < kIn ? f32_to_e4m3_rne(W0[o * kIn + f] * i0) : 0;
          const int Ti = 2 * s + e / 16;
          const int k = Ti < kMT ? unit_of(Ti, e % 16, l >> 5) : -1;
          A1[idx] = k >= 0 ? f32_to_e4m3_rne(W1[o * kHid + k] * i1) : 0;
          A2[idx] = k >= 0 ? f32_to_e4m3_rne(W2[o * kHid + k] * i2) : 0;
        }
  float *vec = (float *)(B + L0 + 2 * L1);
  const float s0 = ldexpf(1.0f, -kh0), s1 = ldexpf(1.0f, -kh1);
  for (int h = 0; h < kHid; ++h) {
    vec[h] = b1[h] * s1;
    vec[kHid + h] = b2[h];
    vec[2 * kHid + h] = W3[h];
    vec[3 * kHid + h] = b0[h] * s0;
  }
  uint32_t *ex = (uint32_t *)(vec + 4 * kHid);
  ex[0] = sa0 | (sa1 << 8) | (sa2 << 16);
  ex[1] = sb1 | (sb2 << 8);
}

// Image of the MLPNet weights in the operand order of eval_net<P> (P: 0 FP32, 1 BF16, 2 split
// BF16, 3 FP8).  Layer 0 takes 80 features: the 76 inputs, the bias on feature 76, zeros.
inline std::vector<uint8_t> pack_net(int P, const float *p) {
  constexpr int L0[4] = {NetSize<kP32>::kL0, NetSize<kPBF16>::kL0, NetSize<kPBF16X3>::kL0, NetSize<kPFP8>::kL0};
  constexpr int L1[4] = {NetSize<kP32>::kL1, NetSize<kPBF16>::kL1, NetSize<kPBF16X3>::kL1, NetSize<kPFP8>::kL1};
  const float *W0 = p, *b0 = W0 + kHid * kIn, *W1 = b0 + kHid, *b1 = W1 + kHid * kHid, *W2 = b1 + kHid,
              *b2 = W2 + kHid * kHid, *W3 = b2 + kHid;
  std::vector<uint8_t> out((size_t)L0[P] + 2 * L1[P] + (P == 3 ? 4 : 3) * kHid * 4 + 16, 0);
  uint8_t *B = out.data();
  if (P == 3) {
    pack_net_fp8(p, B);
    return out;
  }
  for (int layer = 0; layer < 3; ++layer) {
    uint8_t *dst = layer == 0 ? B : B + L0[P] + (layer - 1) * L1[P];
    const float *W = layer == 1 ? W1 : W2;
    auto w = [&](int o, int k) -> float {
      if (layer > 0) return W[o * kHid + k];
      return k < kIn ? W0[o * kIn + k] : (k == kIn ? b0[o] : 0.0f);
    };
    if (P == 0) {
      // K-step s covers two inputs: layer 0 feature 2s + g, later layers unit_of(s/16, s%16, g)
      float *F = (float *)dst;
      const int nread = layer == 0 ? 10 : 12;
      for (int T = 0; T < kMT; ++T)
        for (int s4 = 0; s4 < nread; ++s4)
          for (int l = 0; l < 64; ++l)
            for (int i = 0; i < 4; ++i) {
              const int s = 4 * s4 + i, g = l >> 5;
              const int k = layer == 0 ? 2 * s + g : unit_of(s / 16, s % 16, g);
              F[((T * nread + s4) * 64 + l) * 4 + i] = w(32 * T + (l & 31), k);
            }
    } else {
      // K-step s covers 16 inputs, lane group g holds eight: layer 0 features 16s + 8g + e,
      // later layers unit_of(s/2, 8(s%2) + e, g)
      const int nstep = layer == 0 ? 5 : 6;
      const int n = kMT * nstep * 64 * 8;
      uint16_t *hi = (uint16_t *)dst, *lo = hi + n;
      for (int T = 0; T < kMT; ++T)
        for (int s = 0; s < nstep; ++s)
          for (int l = 0; l < 64; ++l)
            for (int e = 0; e < 8; ++e) {
              const int g = l >> 5;
              const int k = layer == 0 ? 16 * s + 8 * g + e : unit_of(s / 2, 8 * (s % 2) + e, g);
              const float x = w(32 * T + (l & 31), k);
              const int idx = ((T * nstep + s) * 64 + l) * 8 + e;
              const uint16_t h = f32_to_bf16_rne(x);
              hi[idx] = h;
              if (P == 2) lo[idx] = f32_to_bf16_rne(x - bf16_to_f32(h));
            }
    }
  }
  float *vec = (float *)(B + L0[P] + 2 * L1[P]);
  for (int h = 0; h < kHid; ++h) {
    vec[h] = b1[h];
    vec[kHid + h] = b2[h];
    vec[2 * kHid + h] = W3[h];
  }
  return out;
}

// FP64 MLPNet blob with every weight matrix stored [input][unit].
inline std::vector<double> net_fp64(const float *p) {
  std::vector<double> t(kNetParams);
  const float *W0 = p, *b0 = W0 + kHid * kIn, *W1 = b0 + kHid, *b1 = W1 + kHid * kHid, *W2 = b1 + kHid,
              *b2 = W2 + kHid * kHid, *W3 = b2 + kHid, *b3 = W3 + kHid;
  double *T0 = t.data(), *c0 = T0 + kIn * kHid, *T1 = c0 + kHid, *c1 = T1 + kHid * kHid, *T2 = c1 + kHid,
         *c2 = T2 + kHid * kHid, *T3 = c2 + kHid, *c3 = T3 + kHid;
  for (int o = 0; o < kHid; ++o) {
    for (int f = 0; f < kIn; ++f) T0[f * kHid + o] = W0[o * kIn + f];
    for (int k = 0; k < kHid; ++k) {
      T1[k * kHid + o] = W1[o * kHid + k];
      T2[k * kHid + o] = W2[o * kHid + k];
    }
    c0[o] = b0[o];
    c1[o] = b1[o];
    c2[o] = b2[o];
    T3[o] = W3[o];
  }
  c3[0] = b3[0];
  return t;
}

// Zone of a swap with partner slot d, for every d: the origin, the partner and the
// neighbours (first n_nbr slots) of either; sorted, duplicates removed.  Returns |Omega|.
inline int zone_table(int n_nbr, std::vector<int8_t> &out) {
  out.assign((size_t)kDirs * kOmMax * 3, 0);
  int count = 0;
  for (int d = 0; d < kDirs; ++d) {
    using V = std::array<int, 3>;
    const V pd = {dx(d), dy(d), dz(d)};
    std::vector<V> v = {{0, 0, 0}, pd};
    for (int k = 0; k < n_nbr; ++k) {
      v.push_back({dx(k), dy(k), dz(k)});
      v.push_back({pd[0] + dx(k), pd[1] + dy(k), pd[2] + dz(k)});
    }
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    if ((int)v.size() > kOmMax) return -1;
    count = (int)v.size();
    for (int k = 0; k < count; ++k)
      for (int a = 0; a < 3; ++a) out[((size_t)d * kOmMax + k) * 3 + a] = (int8_t)v[k][a];
  }
  return count;
}

// Read region of a trial with partner slot d: every zone site and its first n_nbr neighbours, in
// the order first met walking the zone (om, the table above: n_om sites) and each site's slots
// (centre, then neighbours 0..n_nbr-1).  off: [12][n_reg] offsets packed as (dx + 8) |
// (dy + 8) << 4 | (dz + 8) << 8; idx: [12][n_om][n_nbr + 1] region position of zone row k's
// slot m; pos: [12][2] positions of the trial site (offset 0) and the partner (offset of slot
// d).  Returns false if a region size differs from n_reg.
inline bool region_tables(const std::vector<int8_t> &om, int n_om, int n_nbr, int n_reg, std::vector<uint16_t> &off,
                          std::vector<uint16_t> &idx, std::vector<uint16_t> &pos) {
  off.assign((size_t)kDirs * n_reg, 0);
  idx.assign((size_t)kDirs * n_om * (n_nbr + 1), 0);
  pos.assign((size_t)kDirs * 2, 0);
  for (int d = 0; d < kDirs; ++d) {
    std::vector<std::array<int, 3>> reg;
    auto find = [&](const std::array<int, 3> &v) -> int {
      for (size_t q = 0; q < reg.size(); ++q)
        if (reg[q] == v) return (int)q;
      reg.push_back(v);
      return (int)reg.size() - 1;
    };
    for (int k = 0; k < n_om; ++k) {
      const int8_t *o = &om[((size_t)d * kOmMax + k) * 3];
      for (int m = 0; m <= n_nbr; ++m) {
        const std::array<int, 3> v = {o[0] + (m ? dx(m - 1) : 0), o[1] + (m ? dy(m - 1) : 0), o[2] + (m ? dz(m - 1) : 0)};
        idx[((size_t)d * n_om + k) * (n_nbr + 1) + m] = (uint16_t)find(v);
      }
    }
    pos[2 * d] = (uint16_t)find({0, 0, 0});            // zone sites: already present
    pos[2 * d + 1] = (uint16_t)find({dx(d), dy(d), dz(d)});
    if ((int)reg.size() != n_reg) return false;
    for (int q = 0; q < n_reg; ++q)
      off[(size_t)d * n_reg + q] = (uint16_t)((reg[q][0] + 8) | ((reg[q][1] + 8) << 4) | ((reg[q][2] + 8) << 8));
  }
  return true;
}

inline int ensure_pack(smc_ctx *c, int P) {
  FccState &f = c->fcc;
  if (f.pack_ready[P]) return SMC_OK;
  const std::vector<uint8_t> img = pack_net(P, c->host_params.data());
  if (!f.d_pack[P]) HIPC(c, hipMalloc(&f.d_pack[P], img.size()));
  HIPC(c, hipMemcpyAsync(f.d_pack[P], img.data(), img.size(), hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));  // img is freed on return
  f.pack_ready[P] = true;
  return SMC_OK;
}

inline int load_params(smc_ctx *c, const float *params_dev) {
  FccState &f = c->fcc;
  const int64_t P = c->n_params;
  c->host_params.resize(P);
  HIPC(c, hipMemcpyAsync(c->host_params.data(), params_dev, sizeof(float) * P, hipMemcpyDeviceToHost, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  for (bool &r : f.pack_ready) r = false;
  const float *p = c->host_params.data();
  if (f.model == 0) {
    f.b3 = p[kNetParams - 1];
    const std::vector<double> t = net_fp64(p);
    const std::vector<float> t32(t.begin(), t.end());  // exact: every entry is an FP32 parameter
    HIPC(c, hipMemcpyAsync(c->d_w64, t.data(), sizeof(double) * t.size(), hipMemcpyHostToDevice, c->stream));
    HIPC(c, hipMemcpyAsync(c->d_w32, t32.data(), sizeof(float) * t32.size(), hipMemcpyHostToDevice, c->stream));
  } else {
    // folded qSRO coefficients with the FCC shell sizes
    const double z[3] = {12.0, 6.0, 24.0};
    std::vector<double> F(kQsroPacked, 0.0);
    std::vector<float> F32(kQsroPacked);
    for (int m = 0; m < 3; ++m)
      for (int cc = 0; cc < 5; ++cc) {
        for (int q = 0; q < 5; ++q)
          if (q != cc) F[(m * 5 + cc) * 5 + q] = (double)p[(m * 5 + std::max(cc, q)) * 5 + std::min(cc, q)] / z[m];
        F[75 + m * 5 + cc] = (double)p[75 + m * 5 + cc] / (z[m] * z[m]);
      }
    double K = (double)p[91];
    for (int q = 0; q < 15; ++q) K += (double)p[90] * (double)p[75 + q] * (double)p[75 + q];
    F[90] = K;
    for (int q = 0; q < kQsroPacked; ++q) F32[q] = (float)F[q];
    HIPC(c, hipMemcpyAsync(c->d_w64, F.data(), sizeof(double) * kQsroPacked, hipMemcpyHostToDevice, c->stream));
    HIPC(c, hipMemcpyAsync(c->d_w32, F32.data(), sizeof(float) * kQsroPacked, hipMemcpyHostToDevice, c->stream));
  }
  HIPC(c, hipStreamSynchronize(c->stream));
  return SMC_OK;
}

// Blocks of the matrix-core kernels: LDS holds one weight image per block.
// Trials of colour col of a replica that have a site: the link cells long enough to hold the
// colour's offset along every axis (fcc::trial_site gives -1 for the others).
inline uint64_t colour_attempts(const Replica &R, int32_t col) {
  int32_t rest = col >> 2;
  const int32_t ox = rest % R.ax[0].big;
  rest /= R.ax[0].big;
  const int32_t oy = rest % R.ax[1].big, oz = rest / R.ax[1].big;
  return (uint64_t)axis_cells_holding(R.ax[0], ox) * (uint64_t)axis_cells_holding(R.ax[1], oy) *
         (uint64_t)axis_cells_holding(R.ax[2], oz);
}

// k_recheck_net_decide: one wave per queued trial (at most n of them), kPhaseWaves waves per
// block, at most one block per CU (the waves loop over the queue)
inline unsigned net_decide_grid(const smc_ctx *c, int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kPhaseWaves - 1) / kPhaseWaves, c->n_cu));
}

inline int net_blocks(const smc_ctx *c, int P) { return (P == SMC_FP8_E4M3 ? 4 : (P == SMC_BF16 ? 3 : 1)) * c->n_cu; }

template <int P>
void launch_site_energies_net(smc_ctx *c, float *out) {
  for (size_t r = 0; r < c->reps.size(); ++r) {
    const int64_t tiles = (c->reps[r].n_sites + 31) / 32;
    const unsigned grid = (unsigned)std::min<int64_t>((tiles + 7) / 8, net_blocks(c, P));
    hipLaunchKernelGGL((k_site_energies_net<P>), dim3(grid), dim3(kNetThreads), 0, c->stream, c->d_reps, (int32_t)r,
                       c->occ, c->fcc.d_pack[P], c->fcc.b3, out);
  }
}

// Local energies with the sweep-precision evaluator (float out).
inline int site_energies_fast(smc_ctx *c, int P, float *out) {
  if (c->fcc.model == 1) {
    if (P != SMC_FP32) return fail(c, SMC_E_UNSUPPORTED, "qSRO on FCC runs in FP32 or FP64");
    for (size_t r = 0; r < c->reps.size(); ++r)
      hipLaunchKernelGGL(k_site_energies_qsro<float>, dim3(grid_for(c->reps[r].n_sites, 256)), dim3(256), 0,
                         c->stream, c->d_reps, (int32_t)r, c->occ, c->d_w32, out);
    HIPC(c, hipGetLastError());
    return SMC_OK;
  }
  if (P != SMC_FP32 && P != SMC_BF16 && P != SMC_BF16X3 && P != SMC_FP8_E4M3)
    return fail(c, SMC_E_UNSUPPORTED, "the FCC MLPNet runs in FP32, BF16, split BF16, FP8 or FP64");
  int rc = ensure_pack(c, P);
  if (rc) return rc;
  if (P == SMC_FP32) launch_site_energies_net<kP32>(c, out);
  else if (P == SMC_BF16) launch_site_energies_net<kPBF16>(c, out);
  else if (P == SMC_BF16X3) launch_site_energies_net<kPBF16X3>(c, out);
  else launch_site_energies_net<kPFP8>(c, out);
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

inline int site_energies64(smc_ctx *c, double *out) {
  for (size_t r = 0; r < c->reps.size(); ++r) {
    const int64_t n = c->reps[r].n_sites;
    if (c->fcc.model == 0) {
      const unsigned grid = (unsigned)std::min<int64_t>((n + kS64NetRows - 1) / kS64NetRows, c->n_cu);  // LDS: one per CU
      hipLaunchKernelGGL(k_site_energies_net64, dim3(grid), dim3(kR64Threads), 0, c->stream, c->d_reps, (int32_t)r,
                         c->occ, (const float *)c->d_w32, out);
    } else {
      hipLaunchKernelGGL(k_site_energies_qsro<double>, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, c->d_reps,
                         (int32_t)r, c->occ, c->d_w64, out);
    }
  }
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

// FP64 from-scratch totals per replica into d_escratch.
inline int scratch_totals(smc_ctx *c) {
  if (!c->d_site64) HIPC(c, hipMalloc(&c->d_site64, sizeof(double) * c->n_total));
  if (!c->d_psum) HIPC(c, hipMalloc(&c->d_psum, sizeof(double) * kSumChunks));
  int rc = site_energies64(c, c->d_site64);
  if (rc) return rc;
  for (size_t r = 0; r < c->reps.size(); ++r)
    sum_doubles(c->stream, c->d_site64 + c->reps[r].site0, c->reps[r].n_sites, c->d_psum, c->d_escratch + r);
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

inline int refresh(smc_ctx *c) {
  int rc = scratch_totals(c);
  if (rc) return rc;
  if (c->cfg.precision == SMC_FP64)
    hipLaunchKernelGGL(k_narrow, dim3(grid_for(c->n_total, 256)), dim3(256), 0, c->stream, c->d_site64, c->ecache,
                       c->n_total);
  else if ((rc = site_energies_fast(c, c->cfg.precision, c->ecache)))
    return rc;
  const int R = (int)c->reps.size();
  HIPC(c, hipMemcpyAsync(c->d_ebase, c->d_escratch, sizeof(double) * R, hipMemcpyDeviceToDevice, c->stream));
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(R, 256)), dim3(256), 0, c->stream, (uint64_t *)c->d_efixed, (int64_t)R,
                     (uint64_t)0);
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

template <int P>
void launch_rows_net(smc_ctx *c, const Args &a, int64_t n_trials) {
  const int64_t tiles = (n_trials * kOmMlp + 31) / 32;
  constexpr int kWaves = net_threads<P>() / 64;
  const unsigned grid =
      (unsigned)std::max<int64_t>(1, std::min<int64_t>((tiles + kWaves - 1) / kWaves, net_blocks(c, P)));
  hipLaunchKernelGGL((k_rows_net<P>), dim3(grid), dim3(net_threads<P>()), 0, c->stream, a, c->fcc.d_pack[P],
                     c->fcc.b3);
}

// Enqueue one sweep on c->stream (also under graph capture): per replica and colour the
// counter reset, proposals, zone rows, decisions and FP64 re-decisions; then the device
// sweep counter advances.
inline int enqueue_sweep(smc_ctx *c, const smc_stats *st, bool trace) {
  FccState &f = c->fcc;
  const int R = (int)c->reps.size();
  const bool fp64 = c->cfg.precision == SMC_FP64;
  const int P = fp64 ? SMC_FP32 : c->cfg.precision;
  // one pair of counters (active, queued) per replica colour, all cleared here, so that no
  // colour waits on a clearing launch of its own
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(c->colours_total, 256)), dim3(256), 0, c->stream,
                     (uint64_t *)f.d_counts, (int64_t)c->colours_total, (uint64_t)0);
  int slot = 0;
  for (int r = 0; r < R; ++r) {
    const Replica &rep = c->reps[r];
    const int64_t nt = std::max<int64_t>(1, rep.n_trials);
    for (int col = 0; col < rep.n_colours; ++col, ++slot) {
      Args a{};
      a.reps = c->d_reps;
      a.r = r;
      a.colour = col;
      a.sweep = c->d_sweep;
      a.seed = c->cfg.seed;
      a.occ = c->occ;
      a.ecache = c->ecache;
      a.trials = f.d_trials;
      a.active = f.d_active;
      a.n_active = f.d_counts + 2 * slot;
      a.e1 = f.d_e1;
      a.om = f.d_om;
      a.om_n = f.om_n;
      a.guard = fp64 ? (double)INFINITY : c->guard;
      a.q_count = f.d_counts + 2 * slot + 1;
      a.queue = f.d_queue;
      a.e_fixed = c->d_efixed;
      a.counters = c->d_counters;
      a.n_replicas = R;
      a.attempts = colour_attempts(rep, col);
      a.dpart = f.model == 0 ? (unsigned long long *)f.d_dpart : nullptr;
      if (trace) {
        a.trace_dE = st->trace_dE;
        a.trace_dE_fast = st->trace_dE_fast;
        a.trace_flags = st->trace_flags;
      }
      hipLaunchKernelGGL(k_propose, dim3(grid_for(nt, kPhaseThreads)), dim3(kPhaseThreads), 0, c->stream, a);
      const int ev = prof_begin(c);
      if (f.model == 1) {
        // 75 KB of LDS per block: at most two blocks per CU
        const unsigned g = (unsigned)std::min<int64_t>((nt + kRqTrials - 1) / kRqTrials, 2 * (int64_t)c->n_cu);
        hipLaunchKernelGGL(k_rows_qsro, dim3(g), dim3(kRqThreads), 0, c->stream, a, (const float *)c->d_w32, f.d_rq_off,
                           f.d_rq_idx, f.d_rq_pos);
      } else if (P == SMC_FP32) {
        launch_rows_net<kP32>(c, a, nt);
      } else if (P == SMC_BF16) {
        launch_rows_net<kPBF16>(c, a, nt);
      } else if (P == SMC_BF16X3) {
        launch_rows_net<kPBF16X3>(c, a, nt);
      } else {
        launch_rows_net<kPFP8>(c, a, nt);
      }
      prof_end(c, ev, 0);
      const dim3 dg(grid_for(nt * kDecideLanes, kPhaseThreads));
      a.dpart_n = (int32_t)dg.x;
      if (f.model == 0)
        hipLaunchKernelGGL(k_decide<kOmMlp>, dg, dim3(kPhaseThreads), 0, c->stream, a);
      else
        hipLaunchKernelGGL(k_decide<kOmQsro>, dg, dim3(kPhaseThreads), 0, c->stream, a);
      // blocks loop over the queue (usually short): a few per CU
      const int ev2 = prof_begin(c);
      if (f.model == 0) {
        const unsigned rg = (unsigned)std::min<int64_t>(c->n_cu, nt * kRcSplit);  // LDS: one block per CU
        hipLaunchKernelGGL(k_recheck_net, dim3(rg), dim3(kR64Threads), 0, c->stream, a, (const float *)c->d_w32,
                           f.d_rowe);
        hipLaunchKernelGGL(k_recheck_net_decide, dim3(net_decide_grid(c, nt)), dim3(kPhaseThreads), 0, c->stream,
                           a, (const double *)f.d_rowe);
      } else {
        const unsigned rg = (unsigned)std::min<int64_t>(2 * (int64_t)c->n_cu, nt);
        hipLaunchKernelGGL(k_recheck_qsro, dim3(rg), dim3(kRcQsroThreads), 0, c->stream, a,
                           (const double *)c->d_w64);
      }
      prof_end(c, ev2, 1);
    }
  }
  hipLaunchKernelGGL(k_next_sweep, dim3(1), dim3(64), 0, c->stream, c->d_sweep);
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

// FP64 dE of the swaps that the given trial sites propose at `sweep` (Philox as in a sweep), on
// the current lattice, with the re-decision kernels in probe mode (nothing changes).
inline int delta_e64(smc_ctx *c, int32_t replica, uint64_t sweep, const int64_t *sites, int32_t n,
                     int64_t *partner_out, double *dE_out) {
  FccState &f = c->fcc;
  const Replica &R = c->reps[replica];
  std::vector<Trial> tr(n);
  std::vector<int32_t> act(n);
  std::vector<QEntry> qe(n);
  for (int32_t k = 0; k < n; ++k) {
    if (sites[k] < 0 || sites[k] >= R.n_sites) return fail(c, SMC_E_INVALID, "site out of range");
    const U64x4 x = philox4x64_10((uint64_t)sites[k], sweep, (uint64_t)replica, 0, c->cfg.seed, 0);
    const int d = dir_of(x.v[0]);
    const Pos p = pos(sites[k], R.L[0], R.L[1]);
    const int64_t nb = at(p, dx(d), dy(d), dz(d), R.L[0], R.L[1], R.L[2]);
    tr[k] = Trial{(int32_t)sites[k], (int32_t)nb, 0.0, d, 0, (int16_t)p.x, (int16_t)p.y, (int16_t)p.z, 0};
    act[k] = k;
    qe[k] = QEntry{k, 0.0f};
    if (partner_out) partner_out[k] = nb;
  }
  Trial *d_tr = nullptr;
  int32_t *d_act = nullptr;
  QEntry *d_q = nullptr;
  uint32_t *d_n = nullptr;
  double *d_out = nullptr, *d_rowe = nullptr;
  const uint32_t nn = (uint32_t)n;
  int rc = SMC_OK;
  if (hipMalloc(&d_tr, sizeof(Trial) * n) || hipMalloc(&d_act, sizeof(int32_t) * n) ||
      hipMalloc(&d_q, sizeof(QEntry) * n) || hipMalloc(&d_n, sizeof(uint32_t)) ||
      hipMalloc(&d_out, sizeof(double) * n) || hipMalloc(&d_rowe, sizeof(double) * 2 * kOmMlp * n))
    rc = fail(c, SMC_E_NOMEM, "probe buffers");
  if (!rc && (hipMemcpyAsync(d_tr, tr.data(), sizeof(Trial) * n, hipMemcpyHostToDevice, c->stream) ||
              hipMemcpyAsync(d_act, act.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, c->stream) ||
              hipMemcpyAsync(d_q, qe.data(), sizeof(QEntry) * n, hipMemcpyHostToDevice, c->stream) ||
              hipMemcpyAsync(d_n, &nn, sizeof(uint32_t), hipMemcpyHostToDevice, c->stream)))
    rc = fail(c, SMC_E_DEVICE, "probe upload");
  if (!rc) {
    Args a{};
    a.reps = c->d_reps;
    a.r = replica;
    a.occ = c->occ;
    a.ecache = c->ecache;
    a.trials = d_tr;
    a.active = d_act;
    a.e1 = f.d_e1;
    a.om = f.d_om;
    a.om_n = f.om_n;
    a.q_count = d_n;
    a.queue = d_q;
    a.e_fixed = c->d_efixed;
    a.counters = c->d_counters;
    a.n_replicas = (int32_t)c->reps.size();
    a.probe_dE = d_out;
    if (f.model == 0) {
      hipLaunchKernelGGL(k_recheck_net, dim3((unsigned)std::min<int64_t>((int64_t)n * kRcSplit, c->n_cu)),
                         dim3(kR64Threads), 0, c->stream, a, (const float *)c->d_w32, d_rowe);
      hipLaunchKernelGGL(k_recheck_net_decide, dim3(net_decide_grid(c, n)), dim3(kPhaseThreads), 0, c->stream, a,
                         (const double *)d_rowe);
    } else
      hipLaunchKernelGGL(k_recheck_qsro, dim3((unsigned)std::min<int64_t>(n, 2 * (int64_t)c->n_cu)),
                         dim3(kRcQsroThreads), 0, c->stream, a, (const double *)c->d_w64);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(dE_out, d_out, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream) ||
        hipStreamSynchronize(c->stream))
      rc = fail(c, SMC_E_DEVICE, "probe kernel");
  }
  void *bufs[] = {d_tr, d_act, d_q, d_n, d_out, d_rowe};
  for (void *p : bufs)
    if (p) (void)hipFree(p);
  return rc;
}

inline void release(smc_ctx *c) {
  FccState &f = c->fcc;
  void *bufs[] = {f.d_om,     f.d_trials, f.d_active,  f.d_e1,      f.d_queue,  f.d_counts, f.d_dpart,
                  f.d_rowe,   f.d_pack[0], f.d_pack[1], f.d_pack[2], f.d_pack[3],
                  f.d_rq_off, f.d_rq_idx, f.d_rq_pos};
  for (void *p : bufs)
    if (p) (void)hipFree(p);
}

// A context on the FCC lattice (MLPNet or qSRO); the caller has checked the pointers.
inline int create(const smc_config *cfg, uint8_t *occ_dev, const float *params_dev, float *ecache_dev,
                  void *hip_stream, double guard, smc_ctx **out) {
  int model;
  if (cfg->feature == SMC_FEAT_MLPNET_S12) {
    model = 0;
    if (cfg->hidden != kHid) return SMC_E_UNSUPPORTED;
  } else if (cfg->feature == SMC_FEAT_QSRO_S123) {
    model = 1;
    if (cfg->precision != SMC_FP32 && cfg->precision != SMC_FP64) return SMC_E_UNSUPPORTED;
  } else {
    return SMC_E_UNSUPPORTED;
  }
  int64_t total = 0;
  for (int r = 0; r < cfg->n_replicas; ++r) {
    for (int a = 0; a < 3; ++a)
      if (cfg->cells[3 * r + a] < 4 || cfg->cells[3 * r + a] > 4096) return SMC_E_INVALID;
    if (!(cfg->temperature_K[r] >= 0.0)) return SMC_E_INVALID;
    total += 4LL * cfg->cells[3 * r] * cfg->cells[3 * r + 1] * cfg->cells[3 * r + 2];
  }
  if (total >= (1LL << 31)) return SMC_E_UNSUPPORTED;
  smc_ctx *c = new (std::nothrow) smc_ctx();
  if (!c) return SMC_E_NOMEM;
  c->cfg = *cfg;
  c->cells.assign(cfg->cells, cfg->cells + 3 * cfg->n_replicas);
  c->temps.assign(cfg->temperature_K, cfg->temperature_K + cfg->n_replicas);
  c->cfg.cells = c->cells.data();
  c->cfg.temperature_K = c->temps.data();
  c->stream = (hipStream_t)hip_stream;
  c->occ = occ_dev;
  c->ecache = ecache_dev;
  c->guard = guard;
  FccState &f = c->fcc;
  f.on = true;
  f.model = model;
  c->hidden = model == 0 ? kHid : 0;
  c->n_in = model == 0 ? kIn : 0;
  c->n_params = model == 0 ? kNetParams : 92;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0) c->n_cu = n;
  }
  int64_t site0 = 0;
  for (int r = 0; r < cfg->n_replicas; ++r) {
    c->reps.push_back(make_replica(&c->cells[3 * r], site0, c->temps[r], 4));
    site0 += c->reps.back().n_sites;
    f.cap = std::max(f.cap, c->reps.back().n_trials);
    c->colours_total += c->reps.back().n_colours;
    c->max_colours = std::max(c->max_colours, c->reps.back().n_colours);
  }
  c->n_total = site0;
  std::vector<int8_t> om;
  f.om_n = zone_table(model == 0 ? kNbrMlp : kNbr, om);
  const int R = cfg->n_replicas;
  auto cleanup = [&](int code) {
    smc_destroy(c);
    return code;
  };
  if (f.om_n != (model == 0 ? kOmMlp : kOmQsro)) return cleanup(SMC_E_DEVICE);
  const int64_t nw = model == 0 ? kNetParams : kQsroPacked;
  bool ok = hipMalloc(&c->d_reps, sizeof(Replica) * R) == hipSuccess &&
            hipMalloc(&c->d_w32, sizeof(float) * nw) == hipSuccess &&
            hipMalloc(&c->d_w64, sizeof(double) * nw) == hipSuccess &&
            hipMalloc(&c->d_ebase, sizeof(double) * R) == hipSuccess &&
            hipMalloc(&c->d_efixed, sizeof(unsigned long long) * R) == hipSuccess &&
            hipMalloc(&c->d_escratch, sizeof(double) * R) == hipSuccess &&
            hipMalloc(&c->d_counters, sizeof(uint64_t) * 4 * R) == hipSuccess &&
            hipMalloc(&c->d_sweep, sizeof(uint64_t)) == hipSuccess &&
            hipMalloc(&f.d_om, om.size()) == hipSuccess &&
            hipMalloc(&f.d_trials, sizeof(Trial) * f.cap) == hipSuccess &&
            hipMalloc(&f.d_active, sizeof(int32_t) * f.cap) == hipSuccess &&
            hipMalloc(&f.d_e1, sizeof(float) * f.cap * f.om_n) == hipSuccess &&
            hipMalloc(&f.d_queue, sizeof(QEntry) * f.cap) == hipSuccess &&
            hipMalloc(&f.d_counts, sizeof(uint64_t) * c->colours_total) == hipSuccess &&
            hipMalloc(&f.d_dpart, sizeof(uint64_t) * 2 * grid_for(f.cap * kDecideLanes, kPhaseThreads)) ==
                hipSuccess &&
            (model != 0 || hipMalloc(&f.d_rowe, sizeof(double) * 2 * kOmMlp * f.cap) == hipSuccess);
  if (!ok) return cleanup(SMC_E_NOMEM);
  const uint64_t zero = 0;
  if (hipMemcpyAsync(c->d_sweep, &zero, sizeof(uint64_t), hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(c->d_reps, c->reps.data(), sizeof(Replica) * R, hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(f.d_om, om.data(), om.size(), hipMemcpyHostToDevice, c->stream) ||
      hipStreamSynchronize(c->stream))
    return cleanup(SMC_E_DEVICE);
  if (model == 1) {
    std::vector<uint16_t> roff, ridx, rpos;
    if (!region_tables(om, kOmQsro, kNbr, kRegQ, roff, ridx, rpos)) return cleanup(SMC_E_DEVICE);
    if (hipMalloc(&f.d_rq_off, sizeof(uint16_t) * roff.size()) != hipSuccess ||
        hipMalloc(&f.d_rq_idx, sizeof(uint16_t) * ridx.size()) != hipSuccess ||
        hipMalloc(&f.d_rq_pos, sizeof(uint16_t) * rpos.size()) != hipSuccess)
      return cleanup(SMC_E_NOMEM);
    if (hipMemcpy(f.d_rq_off, roff.data(), sizeof(uint16_t) * roff.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(f.d_rq_idx, ridx.data(), sizeof(uint16_t) * ridx.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(f.d_rq_pos, rpos.data(), sizeof(uint16_t) * rpos.size(), hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(SMC_E_DEVICE);
  }
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(4 * R, 256)), dim3(256), 0, c->stream, c->d_counters, (int64_t)4 * R,
                     (uint64_t)0);
  int rc = load_params(c, params_dev);
  if (!rc) rc = refresh(c);
  if (!rc && hipStreamSynchronize(c->stream) != hipSuccess) rc = SMC_E_DEVICE;
  if (rc) return cleanup(rc);
  *out = c;
  return SMC_OK;
}

}  // namespace fcc
}  // namespace smc

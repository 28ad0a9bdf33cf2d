// Host-side packing of MLP weights for the matrix-core evaluator and read-region tables.
// The packed orders mirror the operand layouts documented in mfma_eval.hpp.
#include "pack.hpp"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <array>

#include "lattice.hpp"

namespace smc {

namespace {

constexpr int kH = 128, kF = 108;
constexpr float kLog2e = 1.44269504088896340736f;
constexpr float kLn2 = 0.69314718055994530942f;

// Sizes in bytes of layer 0 / layer 1 images (must equal PackSize<> in mfma_eval.hpp).
constexpr int kL0[4] = {4 * 14 * 64 * 16, 4 * 7 * 64 * 16, 2 * 4 * 7 * 64 * 16, 4 * 2 * 64 * 32};
constexpr int kL1[4] = {4 * 16 * 64 * 16, 4 * 8 * 64 * 16, 2 * 4 * 8 * 64 * 16, 4 * 2 * 64 * 32};

// Hidden unit held in output register v by lane group g of M-tile T.
inline int hidden_of(int T, int v, int g) { return 32 * T + 8 * (v / 4) + 4 * g + (v % 4); }

int pow2_exponent_at_least(double x) {
  if (!(x > 0.0)) return 0;
  return (int)ceil(log2(x));
}

}  // namespace

uint16_t f32_to_bf16_rne(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

float bf16_to_f32(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

uint8_t f32_to_e4m3_rne(float x) {
  const uint8_t s = signbit(x) ? 0x80 : 0x00;
  const float a = fabsf(x);
  if (isnan(x)) return 0x7f;
  if (a >= 448.0f) return s | 0x7e;  // saturate
  int e;
  const float m = frexpf(a, &e);  // a = m 2^e, m in [0.5, 1)
  if (a == 0.0f) return s;
  int E = e - 1;                  // a = (2m) 2^E
  if (E < -6) {                   // subnormal: q 2^-9, q in 0..7 (8 rounds up to the min normal)
    const float q = rintf(a * 512.0f);
    return s | (uint8_t)q;
  }
  float r = rintf((2.0f * m - 1.0f) * 8.0f);
  if (r >= 8.0f) {
    r = 0.0f;
    ++E;
  }
  if (E > 8 || (E == 8 && r > 6.0f)) return s | 0x7e;
  return s | (uint8_t)(((E + 7) << 3) | (int)r);
}

float e4m3_to_f32(uint8_t v) {
  const int s = v >> 7, E = (v >> 3) & 15, m = v & 7;
  float a;
  if (E == 15 && m == 7) return NAN;
  if (E == 0) a = ldexpf((float)m, -9);
  else a = ldexpf(1.0f + m / 8.0f, E - 7);
  return s ? -a : a;
}

PackedModel pack_model(int P, const float *p) {
  PackedModel out;
  const float *W0 = p, *b0 = W0 + kH * kF, *W1 = b0 + kH, *b1 = W1 + kH * kH, *W2 = b1 + kH, *b2 = W2 + kH;
  std::vector<float> W0s(kH * kF), c0(kH), c1(kH), w2s(kH);
  for (int i = 0; i < kH * kF; ++i) W0s[i] = -kLog2e * W0[i];
  for (int h = 0; h < kH; ++h) {
    c0[h] = -kLog2e * b0[h];
    c1[h] = -kLog2e * b1[h];
    w2s[h] = -kLn2 * W2[h];
  }
  out.b2 = b2[0];
  // feature 108 (padding slot 27, constant-one input) carries the bias except in FP8, where
  // the bias initialises the accumulators instead
  auto w0 = [&](int h, int f) { return f < kF ? W0s[h * kF + f] : (f == kF && P != 3 ? c0[h] : 0.0f); };
  auto w1 = [&](int o, int k) { return W1[o * kH + k]; };
  const int total = kL0[P] + kL1[P] + 3 * kH * 4 + 16;
  out.bytes.assign(total, 0);
  uint8_t *B = out.bytes.data();
  if (P == 0) {
    float *L0 = (float *)B, *L1 = (float *)(B + kL0[0]);
    for (int T = 0; T < 4; ++T)
      for (int s4 = 0; s4 < 14; ++s4)
        for (int l = 0; l < 64; ++l)
          for (int i = 0; i < 4; ++i) {
            const int s = 4 * s4 + i, f = 2 * s + (l >> 5);
            L0[((T * 14 + s4) * 64 + l) * 4 + i] = w0(32 * T + (l & 31), f);
          }
    for (int To = 0; To < 4; ++To)
      for (int s4 = 0; s4 < 16; ++s4)
        for (int l = 0; l < 64; ++l)
          for (int i = 0; i < 4; ++i) {
            const int s = 4 * s4 + i;
            L1[((To * 16 + s4) * 64 + l) * 4 + i] = w1(32 * To + (l & 31), hidden_of(s / 16, s % 16, l >> 5));
          }
  } else if (P == 1 || P == 2) {
    const int nL0 = 4 * 7 * 64 * 8, nL1 = 4 * 8 * 64 * 8;  // bf16 elements per (hi or lo) image
    uint16_t *L0h = (uint16_t *)B, *L0l = L0h + nL0;
    uint16_t *L1h = (uint16_t *)(B + kL0[P]), *L1l = L1h + nL1;
    auto put = [&](uint16_t *hi, uint16_t *lo, int idx, float w) {
      const uint16_t h = f32_to_bf16_rne(w);
      hi[idx] = h;
      if (P == 2) lo[idx] = f32_to_bf16_rne(w - bf16_to_f32(h));
    };
    for (int T = 0; T < 4; ++T)
      for (int s = 0; s < 7; ++s)
        for (int l = 0; l < 64; ++l)
          for (int e = 0; e < 8; ++e)
            put(L0h, L0l, ((T * 7 + s) * 64 + l) * 8 + e, w0(32 * T + (l & 31), 16 * s + 8 * (l >> 5) + e));
    for (int To = 0; To < 4; ++To)
      for (int s = 0; s < 8; ++s)
        for (int l = 0; l < 64; ++l)
          for (int e = 0; e < 8; ++e)
            put(L1h, L1l, ((To * 8 + s) * 64 + l) * 8 + e,
                w1(32 * To + (l & 31), hidden_of(s / 2, 8 * (s % 2) + e, l >> 5)));
  } else {
    // FP8: power-of-two per-layer scales (applied by the scaled MFMA)
    double a0 = 0, a1 = 0;
    for (float w : W0s) a0 = std::max(a0, (double)fabsf(w));
    for (int i = 0; i < kH * kH; ++i) a1 = std::max(a1, (double)fabsf(W1[i]));
    const int k0 = pow2_exponent_at_least(a0 / 448.0), k1 = pow2_exponent_at_least(a1 / 448.0);
    // activation bound from the weights: z = b0 + sum over slots of one column per slot,
    // so z <= b0 + sum_m max(0, max_p W0[., 4m+p]); |silu(z)| <= max(z, 0.2785)
    double hmax = 0;
    for (int h = 0; h < kH; ++h) {
      double zmax = b0[h];
      for (int m = 0; m < 27; ++m) {
        double best = 0.0;
        for (int q = 0; q < 4; ++q) best = std::max(best, (double)W0[h * kF + 4 * m + q]);
        zmax += best;
      }
      hmax = std::max(hmax, 1.4426950408889634 * std::max(zmax, 0.2785));
    }
    const int kh = pow2_exponent_at_least(hmax / 448.0);
    out.k_scale_a0 = 127 + k0;
    out.k_scale_a1 = 127 + k1;
    out.k_scale_h = 127 + kh;
    out.sh = ldexpf(1.0f, kh);
    const float i0 = ldexpf(1.0f, -k0), i1 = ldexpf(1.0f, -k1);
    uint8_t *L0 = B, *L1 = B + kL0[3];
    for (int T = 0; T < 4; ++T)
      for (int s = 0; s < 2; ++s)
        for (int l = 0; l < 64; ++l)
          for (int e = 0; e < 32; ++e)
            L0[((T * 2 + s) * 64 + l) * 32 + e] =
                f32_to_e4m3_rne(w0(32 * T + (l & 31), 64 * s + 32 * (l >> 5) + e) * i0);
    for (int To = 0; To < 4; ++To)
      for (int s = 0; s < 2; ++s)
        for (int l = 0; l < 64; ++l)
          for (int e = 0; e < 32; ++e)
            L1[((To * 2 + s) * 64 + l) * 32 + e] =
                f32_to_e4m3_rne(w1(32 * To + (l & 31), hidden_of(2 * s + e / 16, e % 16, l >> 5)) * i1);
  }
  float *vec = (float *)(B + kL0[P] + kL1[P]);
  for (int h = 0; h < kH; ++h) {
    vec[h] = c0[h];
    vec[kH + h] = c1[h];
    vec[2 * kH + h] = w2s[h];
  }
  return out;
}

RegionTables build_region_tables() {
  RegionTables t;
  t.reg_off.assign(8 * kRegion, 0);
  t.om_off.assign(8 * kOmegaOneHot, 0);
  t.idx.assign(8 * kOmegaOneHot * 28, 0);
  t.reg_pos.assign(16, 0);
  using V = std::array<int, 3>;
  auto pack = [](const V &v) { return (uint16_t)((v[0] + 8) | ((v[1] + 8) << 4) | ((v[2] + 8) << 8)); };
  std::vector<V> slot = {{0, 0, 0}};
  for (int k = 0; k < kNbr; ++k) slot.push_back({shell_dx(k), shell_dy(k), shell_dz(k)});
  for (int d = 0; d < 8; ++d) {
    const V pd = {shell_dx(d), shell_dy(d), shell_dz(d)};
    std::vector<V> om = {{0, 0, 0}, pd};
    for (int k = 0; k < kNbr; ++k) {
      om.push_back(slot[k + 1]);
      om.push_back({pd[0] + slot[k + 1][0], pd[1] + slot[k + 1][1], pd[2] + slot[k + 1][2]});
    }
    std::sort(om.begin(), om.end());
    om.erase(std::unique(om.begin(), om.end()), om.end());
    std::vector<V> reg;
    for (const V &o : om)
      for (const V &s : slot) reg.push_back({o[0] + s[0], o[1] + s[1], o[2] + s[2]});
    std::sort(reg.begin(), reg.end());
    reg.erase(std::unique(reg.begin(), reg.end()), reg.end());
    if ((int)om.size() != kOmegaOneHot || (int)reg.size() != kRegion) return RegionTables{};
    auto pos = [&](const V &v) { return (int)(std::lower_bound(reg.begin(), reg.end(), v) - reg.begin()); };
    for (int p = 0; p < kRegion; ++p) t.reg_off[d * kRegion + p] = pack(reg[p]);
    for (int k = 0; k < kOmegaOneHot; ++k) {
      t.om_off[d * kOmegaOneHot + k] = pack(om[k]);
      for (int m = 0; m < kSlotsOneHot; ++m)
        t.idx[(d * kOmegaOneHot + k) * 28 + m] =
            (uint8_t)pos({om[k][0] + slot[m][0], om[k][1] + slot[m][1], om[k][2] + slot[m][2]});
    }
    t.reg_pos[2 * d] = (uint8_t)pos({0, 0, 0});
    t.reg_pos[2 * d + 1] = (uint8_t)pos(pd);
  }
  return t;
}

}  // namespace smc

// Per-lane local-energy evaluator (one site per lane).  Used for the FP64 re-decision
// of near-threshold trials and for the FP64 reference mode; the sweep precisions use the
// matrix-core evaluator.
#pragma once
#include "lattice.hpp"

namespace smc {

constexpr int kSlots = 27;  // centre + 26 neighbours

template <typename T>
__device__ inline T silu(T z);

template <>
__device__ inline double silu<double>(double z) {
  return z / (1.0 + exp(-z));
}

template <>
__device__ inline float silu<float>(float z) {
  // z * sigmoid(z) with the hardware exp2 and reciprocal (about 1 ulp each)
  const float e = __builtin_amdgcn_exp2f(-z * 1.44269504088896341f);
  return z * __builtin_amdgcn_rcpf(1.0f + e);
}

// Species of the 27 slots of site j (replica-local index) at position p, seen with the
// species of the sites i and n exchanged when swap is true.
// Replica-local site indices are below 2^31 (enforced when a context is made), so the
// neighbour indices are formed in 32-bit arithmetic.
__device__ inline void gather_slots_at(const uint8_t *occ, Pos p, int64_t j, int32_t lx, int32_t ly, int32_t lz,
                                       int n_slots, bool swap, int64_t i, int64_t n, uint8_t si, uint8_t sn,
                                       uint8_t *slot) {
  const int32_t i32 = (int32_t)i, n32 = (int32_t)n;  // -1 when unused (no swap)
  auto get = [&](int32_t s) -> uint8_t {
    if (swap) {
      if (s == i32) return sn;
      if (s == n32) return si;
    }
    return occ[s];
  };
  auto at32 = [&](int k) -> int32_t {
    const int32_t x = wrap1(p.x + shell_dx(k), 2 * lx), y = wrap1(p.y + shell_dy(k), 2 * ly),
                  z = wrap1(p.z + shell_dz(k), 2 * lz);
    return (((z >> 1) * ly + (y >> 1)) * lx + (x >> 1)) * 2 + (x & 1);
  };
  slot[0] = get((int32_t)j);
#pragma unroll
  for (int k = 0; k < kNbr; ++k)
    if (k + 1 < n_slots) slot[k + 1] = get(at32(k));
}

__device__ inline void gather_slots(const uint8_t *occ, int64_t j, int32_t lx, int32_t ly, int32_t lz,
                                    int n_slots, bool swap, int64_t i, int64_t n, uint8_t si,
                                    uint8_t sn, uint8_t *slot) {
  gather_slots_at(occ, site_pos(j, lx, ly), j, lx, ly, lz, n_slots, swap, i, n, si, sn, slot);
}

// E = W2 . silu(W1 . silu(W0 x + b0) + b1) + b2 with x built from the slot species.
// FEAT 0: x = [onehot(centre), shell-1 counts, shell-2 counts] (12 inputs, 15 slots);
// FEAT 1: x = one-hot of the 27 slots (108 inputs).  Species >= 4 have no channel.
template <int FEAT, int H, typename T>
__device__ inline T mlp_scalar(const uint8_t *slot, const T *W) {
  constexpr int F = FEAT == 0 ? 12 : 108;
  const T *W0 = W, *b0 = W0 + H * F, *W1 = b0 + H, *b1 = W1 + H * H, *W2 = b1 + H, *b2 = W2 + H;
  T h0[H];
  if (FEAT == 0) {
    T x[12];
#pragma unroll
    for (int f = 0; f < 12; ++f) x[f] = T(0);
#pragma unroll
    for (int m = 0; m < 15; ++m) {
      const int p = slot[m];
      const int base = m == 0 ? 0 : (m <= 8 ? 4 : 8);
#pragma unroll
      for (int c = 0; c < 4; ++c) x[base + c] += (p == c) ? T(1) : T(0);
    }
#pragma unroll
    for (int o = 0; o < H; ++o) {
      T acc = b0[o];
#pragma unroll
      for (int f = 0; f < 12; ++f) acc = fma(W0[o * F + f], x[f], acc);
      h0[o] = silu<T>(acc);
    }
  } else {
#pragma unroll
    for (int o = 0; o < H; ++o) {
      T acc = b0[o];
      for (int m = 0; m < kSlots; ++m) {
        const int p = slot[m];
        if (p < 4) acc += W0[o * F + 4 * m + p];
      }
      h0[o] = silu<T>(acc);
    }
  }
  T e = b2[0];
  for (int o = 0; o < H; ++o) {
    T acc = b1[o];
#pragma unroll
    for (int k = 0; k < H; ++k) acc = fma(W1[o * H + k], h0[k], acc);
    e = fma(W2[o], silu<T>(acc), e);
  }
  return e;
}

// qSRO local energy (Eq. 2) from the slot species (centre + shells 1..3), with the host-folded
// coefficients Vf[m][c][q] = V_m^{max(c,q) min(c,q)} / z_m (0 for q = c), Wf[m][c] =
// W_m^c / z_m^2 and K = C + lambda sum W^2:  E = K + sum_m (sum_q Vf[m][c][q] n_m[q] +
// Wf[m][c] n_m[c]^2), n_m[q] the number of shell-m neighbours of species q.
constexpr int kQsroPacked = 3 * 25 + 15 + 1;

template <typename T>
__device__ inline T qsro_scalar(const uint8_t *slot, const T *F) {
  const T *Vf = F, *Wf = F + 75;
  const int c = slot[0];
  // per-shell species counts as 6-bit fields of one integer (at most 24 neighbours per
  // shell); species 5 and above count nowhere
  uint32_t packed[3] = {0u, 0u, 0u};
#pragma unroll
  for (int k = 0; k < kNbr; ++k) {
    const uint32_t q = (uint32_t)slot[k + 1];
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

}  // namespace smc

// Swap kernels of the matrix-core path (one-hot features over shells 1-3, 128 hidden).
//
// One launch per colour (mini-step).  A persistent block of 512 threads keeps the packed
// weights and the slot->region table in LDS and walks groups of 32 link cells:
//   1. proposal: Philox block per trial, partner, species, threshold theta (FP64);
//      same-species trials are finished here; the others are compacted;
//   2. gather: the 192 sites read by each trial (the affected zone and its neighbours) are
//      loaded into LDS with the two swapped species exchanged, and the cached energies of
//      the 40 affected sites;
//   3. energy: the post-swap local energies of all affected sites of the group, 32 sites per
//      matrix-core tile (mfma_eval.hpp);
//   4. decide: dE = sum over the zone of (new - cached) in a fixed order; trials with
//      |dE - theta| below the guard band go to a queue re-decided in FP64, the others are
//      accepted iff dE <= theta;
//   5. apply: accepted swaps write the two species and the new energies of their zone.
#pragma once
#include "mfma_eval.hpp"
#include "sweep_scalar.hpp"

namespace smc {

constexpr int kGroup = 32;
constexpr int kMfmaThreads = 512;
constexpr int kReg = 192;
constexpr int kOm = 40;
constexpr int kIdxRow = 28;

struct RecheckEntry {
  int64_t site;      // replica-local trial site
  int64_t partner;   // replica-local partner
  double theta;
  float dE_fast;
  int32_t replica;
  int32_t dir;
  float e1[kOm];     // new energies of the zone from the sweep precision (cache values)
};

struct MfmaArgs {
  const Replica *reps;
  uint8_t *occ;
  float *ecache;
  const uint8_t *wpack;     // pack_bytes<P>() bytes
  const int32_t *reg_off;   // [8][192]
  const int32_t *om_off;    // [8][40]
  const uint8_t *idx;       // [8][40][28]
  const uint8_t *reg_pos;   // [8][2]
  float b2;
  int32_t k_a0, k_a1, k_h;
  float sh;
  int32_t replica, colour;
  uint64_t seed, sweep;
  double guard;
  uint32_t *q_count;        // queue length of this colour
  RecheckEntry *queue;
  unsigned long long *e_fixed;  // [R] accepted dE in units of 2^-32 eV
  uint64_t *counters;           // [4][R]
  int32_t n_replicas;
  int32_t n_groups;
  double *trace_dE;
  double *trace_dE_fast;
  uint8_t *trace_flags;
};

__device__ __forceinline__ void unpack_off(int32_t v, int &dx, int &dy, int &dz) {
  dx = (v & 0xff) - 16;
  dy = ((v >> 8) & 0xff) - 16;
  dz = ((v >> 16) & 0xff) - 16;
}

template <int P>
__global__ __launch_bounds__(kMfmaThreads) void k_sweep_colour_mfma(MfmaArgs a) {
  constexpr int kW = pack_bytes<P>();
  __shared__ __attribute__((aligned(16))) uint8_t s_w[kW];
  __shared__ __attribute__((aligned(16))) uint8_t s_idx[8 * kOm * kIdxRow];
  __shared__ uint8_t s_reg[kGroup * kReg];
  __shared__ float s_e[kGroup * kOm];
  __shared__ float s_ec[kGroup * kOm];
  __shared__ int32_t s_site[kGroup], s_part[kGroup], s_px[kGroup], s_py[kGroup], s_pz[kGroup];
  __shared__ double s_theta[kGroup];
  __shared__ uint8_t s_dir[kGroup], s_si[kGroup], s_sn[kGroup], s_acc[kGroup];
  __shared__ int s_nact;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const Replica R = a.reps[a.replica];
  uint8_t *occ = a.occ + R.site0;
  float *ec = a.ecache + R.site0;

  // weights and slot table into LDS, once per block
  for (int q = tid; q < kW / 16; q += kMfmaThreads) ((int4 *)s_w)[q] = ((const int4 *)a.wpack)[q];
  for (int q = tid; q < 8 * kOm * kIdxRow / 4; q += kMfmaThreads) ((int *)s_idx)[q] = ((const int *)a.idx)[q];
  __syncthreads();
  EvalSmem S;
  S.w = s_w;
  S.c0 = (const float *)(s_w + PackSize<P>::kL0 + PackSize<P>::kL1);
  S.c1 = S.c0 + kHid;
  S.w2 = S.c1 + kHid;
  S.b2 = a.b2;
  S.k_scale_a0 = a.k_a0;
  S.k_scale_a1 = a.k_a1;
  S.k_scale_h = a.k_h;
  S.sh = a.sh;

  // XCD-aware group order: blocks b and b+8k share an XCD (round-robin dispatch), so each
  // XCD walks one contiguous eighth of the colour's link cells.
  const int G = gridDim.x;
  int gstart = blockIdx.x, gstep = G, gend = a.n_groups;
  if (G % 8 == 0 && G >= 8) {
    const int x = blockIdx.x & 7, j = blockIdx.x >> 3, per = (a.n_groups + 7) / 8;
    gstart = x * per + j;
    gstep = G / 8;
    gend = min(a.n_groups, (x + 1) * per);
  }
  uint32_t cnt_att = 0, cnt_diff = 0, cnt_acc = 0;
  long long fixed_sum = 0;

  for (int grp = gstart; grp < gend; grp += gstep) {
    // ------------------------------------------------------------ 1. proposal
    if (wave == 0) {
      const int64_t t = (int64_t)grp * kGroup + lane;
      const int64_t i = (lane < kGroup && t < R.n_trials) ? trial_site(R, a.colour, t) : -1;
      bool active = false;
      int d = 0;
      double theta = 0.0;
      Pos pi{0, 0, 0};
      int64_t n = 0;
      uint8_t si = 0, sn = 0;
      if (i >= 0) {
        const U64x4 r = philox4x64_10((uint64_t)i, a.sweep, (uint64_t)a.replica, 0, a.seed, 0);
        d = (int)(r.v[0] >> 61);
        const double u = (double)((r.v[1] >> 11) + 1) * 0x1.0p-53;
        theta = isinf(R.temperature) ? (double)INFINITY : -kBoltzmannEvPerK * R.temperature * log(u);
        pi = site_pos(i, R.L[0], R.L[1]);
        n = site_at(pi, shell_dx(d), shell_dy(d), shell_dz(d), R.L[0], R.L[1], R.L[2]);
        si = occ[i];
        sn = occ[n];
        active = si != sn;
        if (!active) {
          if (a.trace_flags) a.trace_flags[R.site0 + i] = kFlagSame;
          if (a.trace_dE) a.trace_dE[R.site0 + i] = 0.0;
          if (a.trace_dE_fast) a.trace_dE_fast[R.site0 + i] = 0.0;
        }
      }
      const unsigned long long valid = __ballot(i >= 0);
      const unsigned long long act_mask = __ballot(active);
      const int ca = __popcll(act_mask & ((1ull << lane) - 1ull));
      if (active) {
        s_site[ca] = (int32_t)i;
        s_part[ca] = (int32_t)n;
        s_px[ca] = pi.x;
        s_py[ca] = pi.y;
        s_pz[ca] = pi.z;
        s_theta[ca] = theta;
        s_dir[ca] = (uint8_t)d;
        s_si[ca] = si;
        s_sn[ca] = sn;
      }
      if (lane == 0) {
        s_nact = __popcll(act_mask);
        cnt_att += __popcll(valid);
        cnt_diff += __popcll(act_mask);
      }
    }
    __syncthreads();
    const int nact = s_nact;

    // ------------------------------------------------------------ 2. gather
    for (int q = tid; q < nact * kReg; q += kMfmaThreads) {
      const int t = q / kReg, p = q - t * kReg;
      const int d = s_dir[t];
      int dx, dy, dz;
      unpack_off(a.reg_off[d * kReg + p], dx, dy, dz);
      const Pos pi{s_px[t], s_py[t], s_pz[t]};
      const int64_t j = site_at(pi, dx, dy, dz, R.L[0], R.L[1], R.L[2]);
      uint8_t v = occ[j];
      if (p == a.reg_pos[2 * d]) v = s_sn[t];
      if (p == a.reg_pos[2 * d + 1]) v = s_si[t];
      s_reg[q] = v;
    }
    for (int q = tid; q < nact * kOm; q += kMfmaThreads) {
      const int t = q / kOm, k = q - t * kOm;
      int dx, dy, dz;
      unpack_off(a.om_off[s_dir[t] * kOm + k], dx, dy, dz);
      const Pos pi{s_px[t], s_py[t], s_pz[t]};
      s_ec[q] = ec[site_at(pi, dx, dy, dz, R.L[0], R.L[1], R.L[2])];
    }
    __syncthreads();

    // ------------------------------------------------------------ 3. energies
    const int rows = nact * kOm;
    for (int tile = wave; tile * 32 < rows; tile += kMfmaThreads / 64) {
      const int row = tile * 32 + (lane & 31);
      const bool valid = row < rows;
      const int t = valid ? row / kOm : 0;
      const int k = valid ? row - t * kOm : 0;
      const uint8_t *irow = s_idx + (s_dir[t] * kOm + k) * kIdxRow;
      const uint8_t *reg = s_reg + t * kReg;
      const float E = eval_tile<P>(S, [&](int m) -> uint32_t { return reg[irow[m]]; });
      if (valid && lane < 32) s_e[row] = E;
    }
    __syncthreads();

    // ------------------------------------------------------------ 4. decide
    if (wave == 0) {
      bool accept = false;
      double dEd = 0.0;
      if (lane < nact) {
        float dE = 0.0f;
        for (int k = 0; k < kOm; ++k) dE += s_e[lane * kOm + k] - s_ec[lane * kOm + k];
        dEd = (double)dE;
        const double theta = s_theta[lane];
        const int64_t i = s_site[lane];
        if (fabs(dEd - theta) < a.guard) {
          const uint32_t slot = atomicAdd(a.q_count, 1u);
          RecheckEntry &e = a.queue[slot];
          e.site = i;
          e.partner = s_part[lane];
          e.theta = theta;
          e.dE_fast = dE;
          e.replica = a.replica;
          e.dir = s_dir[lane];
          for (int k = 0; k < kOm; ++k) e.e1[k] = s_e[lane * kOm + k];
          if (a.trace_dE_fast) a.trace_dE_fast[R.site0 + i] = dEd;
        } else {
          accept = dEd <= theta;
          if (accept) {
            occ[i] = s_sn[lane];
            occ[s_part[lane]] = s_si[lane];
          }
          if (a.trace_flags) a.trace_flags[R.site0 + i] = accept ? kFlagAccept : 0;
          if (a.trace_dE) a.trace_dE[R.site0 + i] = dEd;
          if (a.trace_dE_fast) a.trace_dE_fast[R.site0 + i] = dEd;
        }
        s_acc[lane] = accept;
      }
      // fixed-order sum of the accepted dE of this group
      const unsigned long long acc_mask = __ballot(accept);
      double v = accept ? dEd : 0.0;
      for (int off = 1; off < 32; off <<= 1) {
        const double o = __shfl_down(v, off);
        v += (lane + off < 32) ? o : 0.0;
      }
      if (lane == 0) {
        fixed_sum += to_fixed(v);
        cnt_acc += __popcll(acc_mask);
      }
    }
    __syncthreads();

    // ------------------------------------------------------------ 5. apply the cache
    for (int q = tid; q < nact * kOm; q += kMfmaThreads) {
      const int t = q / kOm, k = q - t * kOm;
      if (!s_acc[t]) continue;
      int dx, dy, dz;
      unpack_off(a.om_off[s_dir[t] * kOm + k], dx, dy, dz);
      const Pos pi{s_px[t], s_py[t], s_pz[t]};
      ec[site_at(pi, dx, dy, dz, R.L[0], R.L[1], R.L[2])] = s_e[q];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const int Rn = a.n_replicas;
    atomicAdd(&a.e_fixed[a.replica], (unsigned long long)fixed_sum);
    atomicAdd((unsigned long long *)&a.counters[0 * Rn + a.replica], (unsigned long long)cnt_att);
    atomicAdd((unsigned long long *)&a.counters[1 * Rn + a.replica], (unsigned long long)cnt_diff);
    atomicAdd((unsigned long long *)&a.counters[2 * Rn + a.replica], (unsigned long long)cnt_acc);
  }
}

// FP64 re-decision of queued near-threshold trials: 80 lanes evaluate the 40 affected
// sites after and before the swap in FP64 (per-lane evaluator), one trial per block step.
struct RecheckArgs {
  const Replica *reps;
  uint8_t *occ;
  float *ecache;
  const double *w64;
  const int32_t *om_off;  // [8][40]
  const uint32_t *q_count;
  const RecheckEntry *queue;
  unsigned long long *e_fixed;
  uint64_t *counters;
  int32_t n_replicas;
  double *trace_dE;
  uint8_t *trace_flags;
};

__global__ __launch_bounds__(128) void k_recheck(RecheckArgs a) {
  __shared__ double s_e[2 * kOm];
  __shared__ int s_accept;
  const uint32_t n = *a.q_count;
  const int tid = threadIdx.x;
  for (uint32_t q = blockIdx.x; q < n; q += gridDim.x) {
    const RecheckEntry &e = a.queue[q];
    const Replica R = a.reps[e.replica];
    uint8_t *occ = a.occ + R.site0;
    const Pos pi = site_pos(e.site, R.L[0], R.L[1]);
    const int d = e.dir;
    const uint8_t si = occ[e.site], sn = occ[e.partner];
    if (tid < 2 * kOm) {
      const int k = tid % kOm;
      int dx, dy, dz;
      unpack_off(a.om_off[d * kOm + k], dx, dy, dz);
      const int64_t j = site_at(pi, dx, dy, dz, R.L[0], R.L[1], R.L[2]);
      s_e[tid] = site_energy<1, 128, double>(occ, R, j, tid < kOm, e.site, e.partner, si, sn, a.w64);
    }
    __syncthreads();
    if (tid == 0) {
      double e1 = 0.0, e0 = 0.0;
      for (int k = 0; k < kOm; ++k) e1 += s_e[k];
      for (int k = 0; k < kOm; ++k) e0 += s_e[kOm + k];
      const double dE = e1 - e0;
      const bool accept = dE <= e.theta;
      const int Rn = a.n_replicas;
      if (accept) {
        occ[e.site] = sn;
        occ[e.partner] = si;
        atomicAdd(&a.e_fixed[e.replica], (unsigned long long)to_fixed(dE));
        atomicAdd((unsigned long long *)&a.counters[2 * Rn + e.replica], 1ull);
      }
      atomicAdd((unsigned long long *)&a.counters[3 * Rn + e.replica], 1ull);
      if (a.trace_flags) a.trace_flags[R.site0 + e.site] = kFlagFp64 | (accept ? kFlagAccept : 0);
      if (a.trace_dE) a.trace_dE[R.site0 + e.site] = dE;
      s_accept = accept;
    }
    __syncthreads();
    if (tid < kOm && s_accept) {
      // the cache keeps the sweep precision's energies of the zone
      int dx, dy, dz;
      unpack_off(a.om_off[d * kOm + tid], dx, dy, dz);
      a.ecache[R.site0 + site_at(pi, dx, dy, dz, R.L[0], R.L[1], R.L[2])] = e.e1[tid];
    }
    __syncthreads();
  }
}

// Local energy of every site of one replica with the matrix-core evaluator (fills the cache).
template <int P>
__global__ __launch_bounds__(256) void k_site_energies_mfma(const Replica *reps, int32_t r, const uint8_t *occ_all,
                                                           const uint8_t *wpack, float b2, int32_t k_a0,
                                                           int32_t k_a1, int32_t k_h, float sh, float *out) {
  constexpr int kW = pack_bytes<P>();
  __shared__ __attribute__((aligned(16))) uint8_t s_w[kW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int q = tid; q < kW / 16; q += 256) ((int4 *)s_w)[q] = ((const int4 *)wpack)[q];
  __syncthreads();
  const Replica R = reps[r];
  const uint8_t *occ = occ_all + R.site0;
  EvalSmem S;
  S.w = s_w;
  S.c0 = (const float *)(s_w + PackSize<P>::kL0 + PackSize<P>::kL1);
  S.c1 = S.c0 + kHid;
  S.w2 = S.c1 + kHid;
  S.b2 = b2;
  S.k_scale_a0 = k_a0;
  S.k_scale_a1 = k_a1;
  S.k_scale_h = k_h;
  S.sh = sh;
  const int64_t tiles = (R.n_sites + 31) / 32;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < tiles; tile += (int64_t)gridDim.x * 4) {
    const int64_t j = tile * 32 + (lane & 31);
    const bool valid = j < R.n_sites;
    const Pos p = site_pos(valid ? j : 0, R.L[0], R.L[1]);
    const float E = eval_tile<P>(S, [&](int m) -> uint32_t {
      if (m == 0) return occ[valid ? j : 0];
      const int k = m - 1;
      return occ[site_at(p, shell_dx(k), shell_dy(k), shell_dz(k), R.L[0], R.L[1], R.L[2])];
    });
    if (valid && lane < 32) out[R.site0 + j] = E;
  }
}

}  // namespace smc

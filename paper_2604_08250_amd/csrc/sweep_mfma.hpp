// Swap kernels of the matrix-core path (one-hot features over shells 1-3, 128 hidden).
//
// One launch per colour index (mini-step) processes that colour of every replica whose
// schedule has it (replicas of uneven size are independent and share the launch).  A
// persistent block of 512 threads keeps the packed weights and the lookup tables in LDS and
// walks its groups of GROUP link cells as a pipeline over trial buffers (buffer b: the next
// kFill different-species trials of the block's groups in order, or one group's):
//   proposal (buffer b+2, by the first wave to run out of tiles of buffer b): Philox block per
//      trial, partner, species, threshold theta (FP64); same-species trials are finished here,
//      the others compacted into the buffer;
//   gather (buffer b+1, issued before the energies of buffer b and consumed after them): the
//      192 sites read by each trial (its affected zone Omega and their neighbours) and the
//      cached energies of the 40 zone sites, into registers, then into LDS with the two
//      swapped species exchanged;
//   energy (buffer b): the post-swap local energies of every zone site, 32 sites per
//      matrix-core tile (mfma_eval.hpp), tiles claimed dynamically by the eight waves; for the
//      qSRO model (Eq. 2, P = kPQsro) 64 sites per wave tile, one per lane, each counting its
//      neighbours' species from the staged region (the per-lane evaluator's arithmetic);
//   decide (buffer b): dE = sum over the zone of (new - cached) in a fixed order; trials with
//      |dE - theta| inside the guard band go to a queue re-decided in FP64, the others are
//      accepted iff dE <= theta;
//   apply (buffer b): accepted swaps write the two species and the new zone energies.
// Trials of one colour never read what another trial of the colour writes (link cells of
// at least four cells), so reads may run ahead of writes across buffers.
#pragma once
#include "mfma_eval.hpp"
#include "sweep_scalar.hpp"

namespace smc {

constexpr int kMfmaThreads = 512;
constexpr int kReg = 192;
constexpr int kOm = 40;
constexpr int kIdxRow = 28;
constexpr int kPart = 8;  // dE partial sums per trial
constexpr int kPQsro = 4; // the qSRO model's evaluation in place of the MLP's precisions

// Bytes of the evaluator's parameters in LDS: the packed MLP weights of a precision, or the
// folded qSRO coefficients (kQsroPacked floats, padded to 16 bytes).
template <int P>
constexpr int smem_weight_bytes() {
  if constexpr (P == kPQsro) return (kQsroPacked * 4 + 15) / 16 * 16;
  else return pack_bytes<P>();
}

// Different-species trials per trial buffer of the colour kernel (MLP): the count n <= CAP (the
// buffer capacity) that gives the most trials per energy-phase step, a step being one 32-row
// tile on each of the block's kMfmaThreads / 64 waves (40 rows per trial).  The wave that runs
// out of tiles first makes the next proposals: where tiles are short (BF16, FP8) one tile slot
// is kept for it (capacity 64: 63 trials, 79 tiles, 10 steps; capacity 32: 31, 39, 5), where
// they are long (split BF16, FP32) the buffer is full (32 trials, 40 tiles, 5 steps).  Measured
// on 256^3 against one buffer per group of 32 proposals (about 25.6 trials): split BF16 +1.5 % at
// 32 (+1.1 % at 31), FP8 +4.0 % at 31 (+0.6 % at 32), both -2 % at 24; capacity 64 then gave
// BF16 +5.8 % and FP8 +1.9 % over 31.
template <int P, int CAP>
constexpr int fill_target() {
  const int tile_rows = 32, waves = kMfmaThreads / 64, slot = (P == kPBF16 || P == kPFP8) ? 1 : 0;
  int best = 1, best_steps = 1;
  for (int n = 1; n <= CAP; ++n) {
    const int tiles = (n * kOm + tile_rows - 1) / tile_rows;
    const int steps = (tiles + slot + waves - 1) / waves;
    if (n * best_steps >= best * steps) {
      best = n;
      best_steps = steps;
    }
  }
  return best;
}
static_assert(fill_target<kPBF16X3, 32>() == 32 && fill_target<kPFP8, 64>() == 63 &&
                  fill_target<kPBF16, 16>() == 12 && fill_target<kPBF16X3, 16>() == 12,
              "trial buffer fill");

struct RecheckEntry {
  int64_t site;      // replica-local trial site
  int64_t partner;   // replica-local partner
  double theta;
  float dE_fast;
  int32_t replica;
  int32_t dir;
  float e1[kOm];     // new energies of the zone from the sweep precision (cache values)
  uint8_t reg[kReg]; // species of the read region after the swap (when has_reg)
  int32_t has_reg;   // 0: the FP64 evaluation gathers the region from the lattice itself
};

struct MfmaArgs {
  const Replica *reps;
  uint8_t *occ;
  float *ecache;
  const uint8_t *wpack;     // pack_bytes<P>() bytes
  const uint16_t *reg_off;  // [8][192]
  const uint16_t *om_off;   // [8][40]
  const uint8_t *idx;       // [8][40][28]
  const uint8_t *reg_pos;   // [8][2]
  float b2;
  int32_t k_a0, k_a1, k_h;
  float sh;
  int32_t colour;           // colour index of this launch
  const int32_t *seg_rep;   // [nseg] replicas that have this colour
  const int32_t *seg_start; // [nseg + 1] first flattened group of each replica
  int32_t nseg;
  int32_t xcd_order;        // 1: each XCD walks a contiguous range of groups
  uint64_t seed;
  const uint64_t *sweep;    // device sweep counter (graph replays advance it)
  double guard;
  uint32_t *q_count;        // queue length of this colour
  RecheckEntry *queue;
  unsigned long long *e_fixed;  // [R] accepted dE in units of 2^-32 eV
  uint64_t *counters;           // [4][R]
  int32_t n_replicas;
  double *trace_dE;
  double *trace_dE_fast;
  uint8_t *trace_flags;
};

__device__ __forceinline__ void unpack_off(uint32_t v, int &dx, int &dy, int &dz) {
  dx = (int)(v & 15u) - 8;
  dy = (int)((v >> 4) & 15u) - 8;
  dz = (int)((v >> 8) & 15u) - 8;
}

// Per-trial data of one group (three groups in flight).
template <int GROUP>
struct TrialBuf {
  int32_t site[GROUP], part[GROUP], px[GROUP], py[GROUP], pz[GROUP];
  double theta[GROUP];
  uint8_t dir[GROUP], si[GROUP], sn[GROUP];
  int32_t nact, nvalid, rep;
};

template <int P, int GROUP>
// qSRO: four waves per SIMD (two blocks per CU), which holds it to 128 VGPRs
__global__ __launch_bounds__(kMfmaThreads, P == kPQsro ? 4 : 2) void k_sweep_colour_mfma(MfmaArgs a) {
  constexpr int kW = smem_weight_bytes<P>();
  __shared__ __attribute__((aligned(16))) uint8_t s_w[kW];
  __shared__ __attribute__((aligned(16))) uint8_t s_idx[8 * kOm * kIdxRow];
  __shared__ uint16_t s_roff[8 * kReg];
  __shared__ uint16_t s_ooff[8 * kOm];
  __shared__ uint8_t s_rpos[16];
  // FP32: one buffer per group of GROUP proposals (1.8 % slower with packed buffers of 32)
  constexpr bool kPack = P != kP32;
  // buffer capacity: BF16, FP8 (short tiles, small weights) and qSRO (no weights) take 64
  // trials per buffer, so that the per-buffer phases count once per 63 or 64 trials; split BF16
  // has no LDS left for it
  constexpr int kCap = (P == kPBF16 || P == kPFP8 || P == kPQsro) && GROUP == 32 ? 64 : GROUP;
  // qSRO fills its buffers: its short evaluation leaves the per-buffer phases as the larger cost
  // (64 trials, 40 tiles of 64 rows; buffers of 32 and 25 trials measured 0.5 % and 6 % slower
  // than one buffer per group, 64 trials 6 % faster)
  constexpr int kFill = P == kPQsro ? kCap : (kPack ? fill_target<P, kCap>() : GROUP);
  __shared__ uint8_t s_reg[kCap * kReg];
  __shared__ float s_e[kCap * kOm];
  __shared__ float s_ec[kCap * kOm];
  __shared__ float s_psum[kCap * kPart];
  __shared__ TrialBuf<kCap> s_tb[3];
  __shared__ TrialBuf<kCap> s_carry;  // proposed trials that did not fit the last buffer
  __shared__ int s_pgrp;              // the block's next group to propose
  __shared__ uint8_t s_acc[kCap];
  __shared__ int s_tile, s_prop;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  if constexpr (P == kPQsro) {
    for (int q = tid; q < kQsroPacked; q += kMfmaThreads) ((float *)s_w)[q] = ((const float *)a.wpack)[q];
  } else {
    for (int q = tid; q < kW / 16; q += kMfmaThreads) ((int4 *)s_w)[q] = ((const int4 *)a.wpack)[q];
  }
  for (int q = tid; q < 8 * kOm * kIdxRow / 4; q += kMfmaThreads) ((int *)s_idx)[q] = ((const int *)a.idx)[q];
  for (int q = tid; q < 8 * kReg; q += kMfmaThreads) s_roff[q] = a.reg_off[q];
  for (int q = tid; q < 8 * kOm; q += kMfmaThreads) s_ooff[q] = a.om_off[q];
  if (tid < 16) s_rpos[tid] = a.reg_pos[tid];
  EvalSmem S{};
  if constexpr (P != kPQsro) {
    S.w = s_w;
    S.c0 = (const float *)(s_w + PackSize<P>::kL0 + PackSize<P>::kL1);
    S.c1 = S.c0 + kHid;
    S.w2 = S.c1 + kHid;
    S.b2 = a.b2;
    S.k_scale_a0 = a.k_a0;
    S.k_scale_a1 = a.k_a1;
    S.k_scale_h = a.k_h;
    S.sh = a.sh;
  }
  const uint64_t sweep = *a.sweep;

  // Flattened groups of all participating replicas.  XCD-aware order: blocks b and b+8k
  // share an XCD (round-robin dispatch), so each XCD walks one contiguous eighth.
  const int n_groups = a.seg_start[a.nseg];
  const int G = gridDim.x;
  int gstart = blockIdx.x, gstep = G, gend = n_groups;
  if (a.xcd_order && G % 8 == 0 && G >= 8) {
    const int x = blockIdx.x & 7, j = blockIdx.x >> 3, per = (n_groups + 7) / 8;
    gstart = x * per + j;
    gstep = G / 8;
    gend = min(n_groups, (x + 1) * per);
  }
  // per-replica statistics, flushed when the block moves to another replica
  int stat_rep = -1;
  uint32_t cnt_att = 0, cnt_diff = 0, cnt_acc = 0;
  long long fixed_sum = 0;
  auto flush = [&]() {
    if (tid == 0 && stat_rep >= 0) {
      const int Rn = a.n_replicas;
      atomicAdd(&a.e_fixed[stat_rep], (unsigned long long)fixed_sum);
      atomicAdd((unsigned long long *)&a.counters[0 * Rn + stat_rep], (unsigned long long)cnt_att);
      atomicAdd((unsigned long long *)&a.counters[1 * Rn + stat_rep], (unsigned long long)cnt_diff);
      atomicAdd((unsigned long long *)&a.counters[2 * Rn + stat_rep], (unsigned long long)cnt_acc);
    }
    cnt_att = cnt_diff = cnt_acc = 0;
    fixed_sum = 0;
  };

  // replica and replica-local group of a flattened group (binary search over the segments)
  auto locate = [&](int grp, int &rep, int &lgrp) {
    int lo = 0, hi = a.nseg - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.seg_start[mid] <= grp) lo = mid;
      else hi = mid - 1;
    }
    rep = a.seg_rep[lo];
    lgrp = grp - a.seg_start[lo];
  };

  // Proposals (one wave).  The block walks its groups in order and packs their different-species
  // trials into trial buffers of kFill trials (fewer at a change of replica and at the end), so
  // that the energy phases have the same number of tiles instead of one that varies with each
  // group's count; trials past kFill wait in s_carry and open the next buffer.  Without kPack a
  // buffer takes one group's trials.  The trials of a
  // colour are independent, so the buffer a trial lands in changes nothing in its result.
  // Stream position p of a buffer (carried trials first) goes to tb[p] below kFill, else to
  // s_carry[p - kFill]; a wave's LDS loads precede its stores, so moving the carried trials
  // within s_carry is safe.  Lane 0 writes s_carry's count and replica and s_pgrp at the end;
  // a barrier separates two calls, so that no lane reads them before that write.
  auto place = [&](TrialBuf<kCap> &tb, int p, int32_t i, int32_t n, int x, int y, int z, double theta, uint8_t d,
                   uint8_t si, uint8_t sn) {
    TrialBuf<kCap> &dst = p < kFill ? tb : s_carry;
    const int q = p < kFill ? p : p - kFill;
    dst.site[q] = i;
    dst.part[q] = n;
    dst.px[q] = x;
    dst.py[q] = y;
    dst.pz[q] = z;
    dst.theta[q] = theta;
    dst.dir[q] = d;
    dst.si[q] = si;
    dst.sn[q] = sn;
  };
  // g0: the group of this buffer without kPack
  auto fill = [&](TrialBuf<kCap> &tb, int g0) {
    int cnt = 0, rep = 0, natt = 0, g = g0;
    if constexpr (kPack) {
      cnt = s_carry.nact;
      rep = s_carry.rep;
      g = s_pgrp;
      if (lane < cnt) {
        const int32_t ci = s_carry.site[lane], cn = s_carry.part[lane];
        const int x = s_carry.px[lane], y = s_carry.py[lane], z = s_carry.pz[lane];
        const double th = s_carry.theta[lane];
        const uint8_t d = s_carry.dir[lane], si = s_carry.si[lane], sn = s_carry.sn[lane];
        place(tb, lane, ci, cn, x, y, z, th, d, si, sn);
      }
    }
    while (cnt < kFill && g < gend) {
      int grep = 0, lgrp = 0;
      locate(g, grep, lgrp);
      if ((cnt > 0 || natt > 0) && grep != rep) break;  // a buffer holds one replica
      rep = grep;
      const Replica &R = a.reps[rep];
      const uint8_t *occ = a.occ + R.site0;
      const int64_t t = (int64_t)lgrp * GROUP + lane;
      const int64_t i = (lane < GROUP && t < R.n_trials) ? trial_site(R, a.colour, t) : -1;
      bool active = false;
      int d = 0;
      double theta = 0.0;
      Pos pi{0, 0, 0};
      int64_t n = 0;
      uint8_t si = 0, sn = 0;
      if (i >= 0) {
        const U64x4 r = philox4x64_10((uint64_t)i, sweep, (uint64_t)rep, 0, a.seed, 0);
        d = (int)(r.v[0] >> 61);
        const double u = (double)((r.v[1] >> 11) + 1) * 0x1.0p-53;
        theta = isinf(R.temperature) ? (double)INFINITY : -kBoltzmannEvPerK * R.temperature * log(u);
        pi = site_pos32((int32_t)i, R.L[0], R.L[1]);
        n = site_at32(pi, shell_dx(d), shell_dy(d), shell_dz(d), R.L[0], R.L[1], R.L[2]);
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
      if (active) {
        const int p = cnt + __popcll(act_mask & ((1ull << lane) - 1ull));
        if constexpr (kPack) place(tb, p, (int32_t)i, (int32_t)n, pi.x, pi.y, pi.z, theta, (uint8_t)d, si, sn);
        else {
          tb.site[p] = (int32_t)i;
          tb.part[p] = (int32_t)n;
          tb.px[p] = pi.x;
          tb.py[p] = pi.y;
          tb.pz[p] = pi.z;
          tb.theta[p] = theta;
          tb.dir[p] = (uint8_t)d;
          tb.si[p] = si;
          tb.sn[p] = sn;
        }
      }
      cnt += __popcll(act_mask);
      natt += __popcll(valid);
      g += gstep;
      if (!kPack) break;  // one group (every group holds at least one trial)
    }
    // every lane has read s_carry's count and replica above; lane 0 alone writes them
    if (lane == 0) {
      tb.nact = cnt < kFill ? cnt : kFill;
      tb.nvalid = natt;
      tb.rep = rep;
      if constexpr (kPack) {
        s_carry.nact = cnt > kFill ? cnt - kFill : 0;
        s_carry.rep = rep;
        s_pgrp = g;
      }
    }
  };

  // gather loads of one group into registers (the loads stay in flight until used).  Sixteen
  // threads serve one trial: thread tid reads region positions p = tid % 16 + 16k (k < 12),
  // packed four bytes to a register, and the cached energies of zone sites tid % 16 + 16m
  // (m < 3, below 40) of trial tid / 16, so the trial's position and partner slot are read
  // once per thread.
  static_assert(kMfmaThreads % kCap == 0 && kReg % (kMfmaThreads / kCap) == 0, "threads per trial");
  constexpr int kTpt = kMfmaThreads / kCap;  // threads per trial: 8, 16 or 32 (kCap 64, 32, 16)
  constexpr int kPfReg = kReg / kTpt;         // region bytes per thread: 12 or 6
  constexpr int kPfOm = (kOm + kTpt - 1) / kTpt;  // cached energies per thread: 3 or 2
  // the loaded bytes stay unpacked until gather_store, so that issuing the loads never waits
  // for them
  uint32_t pf_reg[kPfReg];
  float pf_om[kPfOm];
  const int g_t = tid / kTpt, g_l = tid % kTpt;
  auto gather_issue = [&](const TrialBuf<kCap> &tb) {
    const Replica &R = a.reps[tb.rep];
    const uint8_t *occ = a.occ + R.site0;
    const float *ec = a.ecache + R.site0;
    if (g_t < tb.nact) {
      const Pos pt{tb.px[g_t], tb.py[g_t], tb.pz[g_t]};
      const int d = tb.dir[g_t];
#pragma unroll
      for (int k = 0; k < kPfReg; ++k) {
        int dx, dy, dz;
        unpack_off(s_roff[d * kReg + g_l + kTpt * k], dx, dy, dz);
        pf_reg[k] = occ[site_at32(pt, dx, dy, dz, R.L[0], R.L[1], R.L[2])];
      }
#pragma unroll
      for (int m = 0; m < kPfOm; ++m) {
        const int k = g_l + kTpt * m;
        if (k < kOm) {
          int dx, dy, dz;
          unpack_off(s_ooff[d * kOm + k], dx, dy, dz);
          pf_om[m] = ec[site_at32(pt, dx, dy, dz, R.L[0], R.L[1], R.L[2])];
        }
      }
    }
  };
  auto gather_store = [&](const TrialBuf<kCap> &tb) {
    if (g_t < tb.nact) {
      const int d = tb.dir[g_t];
      const int pi = s_rpos[2 * d], pn = s_rpos[2 * d + 1];
#pragma unroll
      for (int k = 0; k < kPfReg; ++k) {
        const int p = g_l + kTpt * k;
        uint8_t v = (uint8_t)pf_reg[k];
        if (p == pi) v = tb.sn[g_t];
        if (p == pn) v = tb.si[g_t];
        s_reg[g_t * kReg + p] = v;
      }
#pragma unroll
      for (int m = 0; m < kPfOm; ++m) {
        const int k = g_l + kTpt * m;
        if (k < kOm) s_ec[g_t * kOm + k] = pf_om[m];
      }
    }
  };

  // prologue: the first two trial buffers, gather of the first
  if (tid == 0) {
    s_carry.nact = 0;
    s_carry.rep = 0;
    s_pgrp = gstart;
  }
  __syncthreads();
  if (wave == 0) fill(s_tb[0], gstart);
  __syncthreads();
  if (wave == 0) fill(s_tb[1], gstart + gstep);
  __syncthreads();
  gather_issue(s_tb[0]);

  int it = 0;
  for (int grp = gstart;; grp += gstep, ++it) {
    if constexpr (!kPack) {
      if (grp >= gend) break;
    }
    TrialBuf<kCap> &cur = s_tb[it % 3];
    TrialBuf<kCap> &nxt = s_tb[(it + 1) % 3];
    TrialBuf<kCap> &nxt2 = s_tb[(it + 2) % 3];
    // ------------------------------------------------------------ gather (g) into LDS
    gather_store(cur);
    if (tid == 0) s_tile = s_prop = 0;
    __syncthreads();
    const int nact = cur.nact;
    // packed: a buffer with neither trials nor attempts (nothing gathered above) means that the
    // block's groups are all done (filled two steps ago, barriers since; the same value in every
    // thread)
    if constexpr (kPack) {
      if (nact == 0 && cur.nvalid == 0) break;
    }
    const Replica &R = a.reps[cur.rep];
    uint8_t *occ = a.occ + R.site0;
    float *ec = a.ecache + R.site0;
    // ------------------------------------------------------------ gather (g+1) in flight
    if (kPack || grp + gstep < gend) gather_issue(nxt);  // nothing for an empty buffer
    // ------------------------------------------------------------ energies (g)
    const int rows = nact * kOm;
    constexpr int kTileRows = P == kPQsro ? 64 : 32;
    const int ntiles = (rows + kTileRows - 1) / kTileRows;
    for (;;) {
      int tile = 0;
      if (lane == 0) tile = atomicAdd(&s_tile, 1);
      tile = __shfl(tile, 0);
      if (tile >= ntiles) break;
      const int row = tile * kTileRows + (lane & (kTileRows - 1));
      const bool valid = row < rows;
      const int t = valid ? row / kOm : 0;
      const int k = valid ? row - t * kOm : 0;
      const uint8_t *irow = s_idx + (cur.dir[t] * kOm + k) * kIdxRow;
      const uint8_t *reg = s_reg + t * kReg;
      if constexpr (P == kPQsro) {
        uint8_t slot[kSlots];
#pragma unroll
        for (int m = 0; m < kSlots; ++m) slot[m] = reg[irow[m]];
        const float E = qsro_scalar<float>(slot, (const float *)s_w);
        if (valid) s_e[row] = E;
      } else {
        const float E = eval_tile<P>(S, [&](int m) -> uint32_t { return reg[irow[m]]; });
        if (valid && lane < 32) s_e[row] = E;
      }
    }
    // ------------------------------------------------------------ proposal (g+2)
    // by the first wave that runs out of tiles (the others still finish theirs)
    {
      int first = 0;
      if (lane == 0) first = atomicAdd(&s_prop, 1) == 0;
      if (__shfl(first, 0)) fill(nxt2, grp + 2 * gstep);
    }
    __syncthreads();
    // ------------------------------------------------------------ decide (g)
    if (tid < nact * kPart) {
      const int t = tid / kPart, part = tid - t * kPart;
      float s = 0.0f;
#pragma unroll
      for (int k = 0; k < kOm / kPart; ++k) {
        const int q = t * kOm + part * (kOm / kPart) + k;
        s += s_e[q] - s_ec[q];
      }
      s_psum[tid] = s;
    }
    __syncthreads();
    if (wave == 0) {
      bool accept = false;
      double dEd = 0.0;
      if (lane < nact) {
        float dE = 0.0f;
#pragma unroll
        for (int part = 0; part < kPart; ++part) dE += s_psum[lane * kPart + part];
        dEd = (double)dE;
        const double theta = cur.theta[lane];
        const int64_t i = cur.site[lane];
        if (fabs(dEd - theta) < a.guard) {
          const uint32_t slot = atomicAdd(a.q_count, 1u);
          RecheckEntry &e = a.queue[slot];
          e.site = i;
          e.partner = cur.part[lane];
          e.theta = theta;
          e.dE_fast = dE;
          e.replica = cur.rep;
          e.dir = cur.dir[lane];
          for (int k = 0; k < kOm; ++k) e.e1[k] = s_e[lane * kOm + k];
          // the gathered region (swap applied) travels with the entry
          for (int k = 0; k < kReg / 4; ++k) ((uint32_t *)e.reg)[k] = ((const uint32_t *)(s_reg + lane * kReg))[k];
          e.has_reg = 1;
          if (a.trace_dE_fast) a.trace_dE_fast[R.site0 + i] = dEd;
        } else {
          accept = dEd <= theta;
          if (accept) {
            occ[i] = cur.sn[lane];
            occ[cur.part[lane]] = cur.si[lane];
          }
          if (a.trace_flags) a.trace_flags[R.site0 + i] = accept ? kFlagAccept : 0;
          if (a.trace_dE) a.trace_dE[R.site0 + i] = dEd;
          if (a.trace_dE_fast) a.trace_dE_fast[R.site0 + i] = dEd;
        }
        s_acc[lane] = accept;
      }
      // the accepted dE in fixed point: packed, converted per trial (an integer sum, the same
      // whichever buffer holds a trial); else the group's fixed-order sum, converted once
      const unsigned long long acc_mask = __ballot(accept);
      long long fx = 0;
      constexpr int kRed = kCap > 32 ? 64 : 32;  // lanes holding a buffer's trials
      if constexpr (kPack) {
        fx = accept ? to_fixed(dEd) : 0;
        for (int off = 1; off < kRed; off <<= 1) {
          const long long o = __shfl_down(fx, off);
          fx += (lane + off < kRed) ? o : 0;
        }
      } else {
        double v = accept ? dEd : 0.0;
        for (int off = 1; off < kRed; off <<= 1) {
          const double o = __shfl_down(v, off);
          v += (lane + off < kRed) ? o : 0.0;
        }
        if (lane == 0) fx = to_fixed(v);
      }
      if (lane == 0) {
        if (cur.rep != stat_rep) {
          flush();
          stat_rep = cur.rep;
        }
        fixed_sum += fx;
        cnt_att += cur.nvalid;
        cnt_diff += nact;
        cnt_acc += __popcll(acc_mask);
      }
    }
    __syncthreads();
    // ------------------------------------------------------------ apply (g)
    // The threads of trial g_t write its new zone energies if it was accepted.  No barrier
    // follows: the next group's gather_store writes only s_reg and s_ec, which this phase
    // does not read, and the next barrier orders everything after it.
    if (g_t < nact && s_acc[g_t]) {
      const Pos pt{cur.px[g_t], cur.py[g_t], cur.pz[g_t]};
      const int d = cur.dir[g_t];
#pragma unroll
      for (int m = 0; m < kPfOm; ++m) {
        const int k = g_l + kTpt * m;
        if (k < kOm) {
          int dx, dy, dz;
          unpack_off(s_ooff[d * kOm + k], dx, dy, dz);
          ec[site_at32(pt, dx, dy, dz, R.L[0], R.L[1], R.L[2])] = s_e[g_t * kOm + k];
        }
      }
    }
  }
  flush();
}

// Advance the device sweep counter (last node of a sweep).
__global__ void k_next_sweep(uint64_t *sweep) {
  if (threadIdx.x == 0) *sweep += 1;
}

// Local energy of every site of one replica with the matrix-core evaluator (fills the cache).
// Eight waves per block, like the colour kernel: two per SIMD with one block per CU.
constexpr int kSeThreads = 512;
template <int P>
__global__ __launch_bounds__(kSeThreads) void k_site_energies_mfma(const Replica *reps, int32_t r,
                                                                  const uint8_t *occ_all, const uint8_t *wpack,
                                                                  float b2, int32_t k_a0, int32_t k_a1, int32_t k_h,
                                                                  float sh, float *out) {
  constexpr int kW = pack_bytes<P>();
  constexpr int kWaves = kSeThreads / 64;
  __shared__ __attribute__((aligned(16))) uint8_t s_w[kW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int q = tid; q < kW / 16; q += kSeThreads) ((int4 *)s_w)[q] = ((const int4 *)wpack)[q];
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
  for (int64_t tile = (int64_t)blockIdx.x * kWaves + wave; tile < tiles; tile += (int64_t)gridDim.x * kWaves) {
    const int64_t j = tile * 32 + (lane & 31);
    const bool valid = j < R.n_sites;
    const Pos p = site_pos32(valid ? (int32_t)j : 0, R.L[0], R.L[1]);
    const float E = eval_tile<P>(S, [&](int m) -> uint32_t {
      if (m == 0) return occ[valid ? j : 0];
      const int k = m - 1;
      return occ[site_at32(p, shell_dx(k), shell_dy(k), shell_dz(k), R.L[0], R.L[1], R.L[2])];
    });
    if (valid && lane < 32) out[R.site0 + j] = E;
  }
}

}  // namespace smc

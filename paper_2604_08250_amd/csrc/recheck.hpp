// FP64 re-decision of the near-threshold trials queued by the matrix-core colour kernel (and
// of the double-lattice strategy, and the FP64 probes): the local energies of the zone before
// and after the swap in FP64, their difference reduced in zone order, the Metropolis decision
// and the apply.
//
// Two launches per colour.  k_recheck_rows evaluates the 80 FP64 local energies of every
// queued trial (rows 0..39: the zone after the swap, 40..79: before) on the FP64 matrix cores,
// 16 rows per half block, so that even a short queue spreads over the whole GPU (for the qSRO
// model, k_recheck_rows_qsro: one row per thread); k_recheck_decide then reduces each trial's
// rows in zone order, decides and applies.  The kernel boundary between them orders the row
// energies before their use, with no device-scope fence.
#pragma once
#include <algorithm>

#include "rows64.hpp"
#include "sweep_mfma.hpp"

namespace smc {

struct RecheckArgs {
  const Replica *reps;
  uint8_t *occ;
  float *ecache;
  const double *w64;        // FP64 blob with W0 and W1 transposed ([input][unit]) for coalescing
  const float *w32t;        // the same layout in FP32 (the model's own values), staged in LDS
  const uint16_t *reg_off;  // [8][192]
  const uint16_t *om_off;   // [8][40]
  const uint8_t *idx;       // [8][40][28]
  const uint8_t *reg_pos;   // [8][2]
  const uint32_t *q_count;
  const RecheckEntry *queue;
  unsigned long long *e_fixed;
  uint64_t *counters;
  int32_t n_replicas;
  double *trace_dE;
  uint8_t *trace_flags;
  double *probe_dE;   // non-null: write dE of queue entry q to probe_dE[q] and change nothing
  double *row_e;      // [queue capacity][80] FP64 local energies
};

constexpr int kRows64 = 2 * kOm;              // rows 0..39 after the swap, 40..79 before
constexpr int kRcRowsB = kR64Rows;            // rows per work item of k_recheck_rows
constexpr int kRcBlocksPerTrial = kRows64 / kRcRowsB;  // 5 work items per queued trial
constexpr int kRcThreads = kR64Threads;
static_assert(kRcRowsB * kRcBlocksPerTrial == kRows64, "row split");

// Work item w: queued trial q = w / 5 and its rows r0 = 16 (w % 5) .. r0 + 15, evaluated by
// rows64_half (the arithmetic every FP64 evaluation of a zone uses).  Persistent blocks, one per
// CU: each stages W0 and W1 in LDS once and then walks work items with no weight traffic, two at
// a time (one per half block), so that the LDS round trips of two items overlap; each item's
// global loads are issued during the previous item's layers.
constexpr int kRcHalf = kR64Half;
__global__ __launch_bounds__(kRcThreads) void k_recheck_rows(RecheckArgs a) {
  __shared__ __attribute__((aligned(16))) Rows64W s_wt;
  __shared__ __attribute__((aligned(16))) Rows64Half s_half[2];
  __shared__ uint8_t s_reg[2][kReg];
  const uint32_t n = *a.q_count;
  const uint32_t items = n * kRcBlocksPerTrial;
  if (blockIdx.x >= items) return;  // no work item for this block
  const int tid = threadIdx.x, hf = tid / kRcHalf, lt = tid % kRcHalf;
  const double b2 = a.w64[kR64Hid * 108 + kR64Hid + kR64Hid * kR64Hid + 2 * kR64Hid];
  // The loads of an item come in two stages, each issued while the previous item is computed:
  // the queue entry (stage 1), then the tables its direction selects (stage 2).
  struct Item {
    uint32_t q;
    int r0, d, has_reg, rep, pos_i, pos_n;
    bool in_range, live;
    int64_t site;
    uint32_t regw;          // word lt of the queued region (threads lt < 48)
    int pslot[2];           // zone-region positions of this thread's two slot-species entries
  };
  auto stage1 = [&](uint32_t w, Item &it) {
    it.q = w / kRcBlocksPerTrial;
    it.r0 = (int)(w - it.q * kRcBlocksPerTrial) * kRcRowsB;
    it.in_range = w < items;
    it.site = -1;
    it.d = it.has_reg = it.rep = 0;
    it.regw = 0u;
    if (it.in_range) {
      const RecheckEntry &e = a.queue[it.q];
      it.site = e.site;
      it.d = e.dir;
      it.has_reg = e.has_reg;
      it.rep = e.replica;
      if (lt < kReg / 4) it.regw = ((const uint32_t *)e.reg)[lt];
    }
  };
  auto stage2 = [&](Item &it) {
    it.live = it.in_range && it.site >= 0;
    it.pos_i = it.pos_n = 0;
    it.pslot[0] = it.pslot[1] = 0;
    if (it.live) {
      const int d = it.d;
      it.pos_i = a.reg_pos[2 * d];
      it.pos_n = a.reg_pos[2 * d + 1];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int v = lt + k * kRcHalf;
        if (v < kRcRowsB * 27) {
          const int lr = v / 27, m = v - lr * 27, gr = it.r0 + lr;
          it.pslot[k] = a.idx[(d * kOm + (gr < kOm ? gr : gr - kOm)) * kIdxRow + m];
        }
      }
    }
  };
  // item w of pass p: half 0 takes blockIdx.x + 2 G p, half 1 the item G further (G blocks), so
  // that a last pass with fewer items than halves leaves whole blocks to one half (whose waves
  // then have the SIMDs to themselves) and a short queue spreads over every block
  Item cur, nxt;
  stage1(blockIdx.x + hf * gridDim.x, cur);
  rows64_stage(s_wt, a.w32t, a.w64, [&] { stage2(cur); });
  for (uint32_t base = blockIdx.x; base < items; base += 2 * gridDim.x) {
    // every thread reaches every barrier; a half without a valid item computes nothing
    const bool live = cur.live;
    const int r0 = cur.r0, d = cur.d, has_reg = cur.has_reg, pos_i = cur.pos_i, pos_n = cur.pos_n;
    const uint32_t q = cur.q;
    if (live) {
      if (has_reg) {
        // the colour kernel queued the region with the trial (swap applied)
        if (lt < kReg / 4) ((uint32_t *)s_reg[hf])[lt] = cur.regw;
      } else if (lt < kReg) {
        const Replica R = a.reps[cur.rep];
        const Pos pi = site_pos(cur.site, R.L[0], R.L[1]);
        int dx, dy, dz;
        unpack_off(a.reg_off[d * kReg + lt], dx, dy, dz);
        s_reg[hf][lt] = a.occ[R.site0 + site_at(pi, dx, dy, dz, R.L[0], R.L[1], R.L[2])];
      }
    }
    __syncthreads();
    // slot species of this item's rows: the rows after the swap see i and n exchanged relative
    // to the rows before (s_reg holds the lattice after the swap when has_reg, else before)
    if (live) {
      const uint8_t at_i = s_reg[hf][pos_i], at_n = s_reg[hf][pos_n];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int v = lt + k * kRcHalf;
        if (v < kRcRowsB * 27) {
          const int lr = v / 27, gr = r0 + lr, p = cur.pslot[k];
          const bool exch = (gr < kOm) != (has_reg != 0);
          s_half[hf].sp[lr * kR64SpStride + (v - lr * 27)] =
              exch ? (p == pos_i ? at_n : (p == pos_n ? at_i : s_reg[hf][p])) : s_reg[hf][p];
        }
      }
    }
    __syncthreads();
    // the next item's queue entry in flight during layer 0, its tables during layer 1
    stage1(base + 2 * gridDim.x + hf * gridDim.x, nxt);
    const double E = rows64_half(s_wt, b2, live, lt, s_half[hf], [&] { stage2(nxt); });
    if (live && lt < kRcRowsB) a.row_e[(size_t)q * kRows64 + r0 + lt] = E;
    __syncthreads();
    cur = nxt;
  }
}

// One wave per queued trial: dE = (sum of the 40 rows after) - (sum of the 40 before), each
// summed in zone order (the rows are loaded by 40 lanes at once and added in order from lane
// registers); decide and apply (or, for a probe, only report dE).  Everything the apply needs
// (the replica, the two species, the zone positions, the cache values) is loaded with the rows,
// so that a trial costs two dependent memory round trips (entry, then the rest) before its
// writes.
__global__ __launch_bounds__(256) void k_recheck_decide(RecheckArgs a) {
  const uint32_t n = *a.q_count;
  const int lane = threadIdx.x & 63;
  const uint32_t waves = gridDim.x * (blockDim.x / 64);
  for (uint32_t q = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); q < n; q += waves) {
    const RecheckEntry &e = a.queue[q];
    const int64_t site = e.site, partner = e.partner;
    if (site < 0) continue;
    const int32_t rep = e.replica, dir = e.dir;
    const double theta = e.theta;
    const double *re = a.row_e + (size_t)q * kRows64;
    const double v1 = lane < kOm ? re[lane] : 0.0, v0 = lane < kOm ? re[kOm + lane] : 0.0;
    const bool probe = a.probe_dE != nullptr;
    const Replica R = a.reps[rep];
    uint8_t *occ = a.occ + R.site0;
    int32_t cpos = 0;
    float ce = 0.0f;
    uint8_t si = 0, sn = 0;
    if (!probe) {
      if (lane < kOm) {
        const Pos pi = site_pos(site, R.L[0], R.L[1]);
        int dx, dy, dz;
        unpack_off(a.om_off[dir * kOm + lane], dx, dy, dz);
        cpos = (int32_t)site_at(pi, dx, dy, dz, R.L[0], R.L[1], R.L[2]);
        ce = e.e1[lane];
      }
      if (lane == 0) {
        si = occ[site];
        sn = occ[partner];
      }
    }
    double e1 = 0.0, e0 = 0.0;
#pragma unroll
    for (int k = 0; k < kOm; ++k) e1 += __shfl(v1, k);
#pragma unroll
    for (int k = 0; k < kOm; ++k) e0 += __shfl(v0, k);
    const double dE = e1 - e0;
    if (probe) {
      if (lane == 0) a.probe_dE[q] = dE;
      continue;
    }
    const bool accept = dE <= theta;
    const int Rn = a.n_replicas;
    if (lane == 0) {
      if (accept) {
        occ[site] = sn;
        occ[partner] = si;
        atomicAdd(&a.e_fixed[rep], (unsigned long long)to_fixed(dE));
        atomicAdd((unsigned long long *)&a.counters[2 * Rn + rep], 1ull);
      }
      atomicAdd((unsigned long long *)&a.counters[3 * Rn + rep], 1ull);
      if (a.trace_flags) a.trace_flags[R.site0 + site] = kFlagFp64 | (accept ? kFlagAccept : 0);
      if (a.trace_dE) a.trace_dE[R.site0 + site] = dE;
    }
    // the cache keeps the sweep precision's energies of the zone
    if (accept && lane < kOm) a.ecache[R.site0 + cpos] = ce;
  }
}

// FP64 rows of the qSRO model (Eq. 2) for the queue of the matrix-core path: one block per
// queued trial (grid-stride), the region in LDS, one row per thread (rows 0..39 after the swap,
// 40..79 before), each counted and evaluated by the per-lane evaluator in FP64.  Its decisions
// are k_recheck_decide's, as for the MLP.
constexpr int kRqThreads = 128;
__global__ __launch_bounds__(kRqThreads) void k_recheck_rows_qsro(RecheckArgs a, const double *F) {
  __shared__ uint8_t s_reg[kReg];
  const uint32_t n = *a.q_count;
  const int tid = threadIdx.x;
  for (uint32_t q = blockIdx.x; q < n; q += gridDim.x) {
    const RecheckEntry &e = a.queue[q];
    const bool live = e.site >= 0;  // uniform over the block
    const int d = e.dir, has_reg = e.has_reg;
    if (live) {
      if (has_reg) {
        // the colour kernel queued the region with the trial (swap applied)
        if (tid < kReg / 4) ((uint32_t *)s_reg)[tid] = ((const uint32_t *)e.reg)[tid];
      } else {
        const Replica R = a.reps[e.replica];
        const Pos pi = site_pos(e.site, R.L[0], R.L[1]);
        for (int v = tid; v < kReg; v += kRqThreads) {
          int dx, dy, dz;
          unpack_off(a.reg_off[d * kReg + v], dx, dy, dz);
          s_reg[v] = a.occ[R.site0 + site_at(pi, dx, dy, dz, R.L[0], R.L[1], R.L[2])];
        }
      }
    }
    __syncthreads();
    if (live && tid < kRows64) {
      // the rows after the swap see i and n exchanged relative to the rows before (s_reg holds
      // the lattice after the swap when has_reg, else before)
      const int pos_i = a.reg_pos[2 * d], pos_n = a.reg_pos[2 * d + 1];
      const uint8_t at_i = s_reg[pos_i], at_n = s_reg[pos_n];
      const bool exch = (tid < kOm) != (has_reg != 0);
      const uint8_t *irow = a.idx + (d * kOm + (tid < kOm ? tid : tid - kOm)) * kIdxRow;
      uint8_t slot[kSlots];
#pragma unroll
      for (int m = 0; m < kSlots; ++m) {
        const int p = irow[m];
        slot[m] = exch ? (p == pos_i ? at_n : (p == pos_n ? at_i : s_reg[p])) : s_reg[p];
      }
      a.row_e[(size_t)q * kRows64 + tid] = qsro_scalar<double>(slot, F);
    }
    __syncthreads();
  }
}

// Enqueue both kernels for a queue of at most max_entries trials (the length itself is read
// on the device).
inline void launch_recheck(const RecheckArgs &ra, int64_t max_entries, int n_cu, hipStream_t stream) {
  const int64_t items = std::max<int64_t>(1, max_entries) * kRcBlocksPerTrial;
  const unsigned rows_grid = (unsigned)std::min<int64_t>(items, n_cu);  // one block per CU (LDS)
  hipLaunchKernelGGL(k_recheck_rows, dim3(rows_grid), dim3(kRcThreads), 0, stream, ra);
  const unsigned dec_grid = (unsigned)std::min<int64_t>((std::max<int64_t>(1, max_entries) + 3) / 4, (int64_t)n_cu);
  hipLaunchKernelGGL(k_recheck_decide, dim3(dec_grid), dim3(256), 0, stream, ra);
}

// The same for the qSRO model: FP64 qSRO rows (F: the folded FP64 coefficients), then the
// decisions.
inline void launch_recheck_qsro(const RecheckArgs &ra, const double *F, int64_t max_entries, int n_cu,
                                hipStream_t stream) {
  const unsigned rows_grid = (unsigned)std::min<int64_t>(std::max<int64_t>(1, max_entries), 4 * (int64_t)n_cu);
  hipLaunchKernelGGL(k_recheck_rows_qsro, dim3(rows_grid), dim3(kRqThreads), 0, stream, ra, F);
  const unsigned dec_grid = (unsigned)std::min<int64_t>((std::max<int64_t>(1, max_entries) + 3) / 4, (int64_t)n_cu);
  hipLaunchKernelGGL(k_recheck_decide, dim3(dec_grid), dim3(256), 0, stream, ra);
}

}  // namespace smc

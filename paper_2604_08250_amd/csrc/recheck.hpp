// FP64 re-decision of the near-threshold trials queued by the matrix-core colour kernel (and
// of the double-lattice strategy): the local energies of the zone before and after the swap in
// FP64, their difference reduced in zone order, the Metropolis decision and the apply.
#pragma once
#include "sweep_mfma.hpp"

namespace smc {

struct RecheckArgs {
  const Replica *reps;
  uint8_t *occ;
  float *ecache;
  const double *w64;        // FP64 blob with W0 and W1 transposed ([input][unit]) for coalescing
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
  uint32_t *done;     // [queue capacity] blocks finished per entry, zero between uses
};

constexpr int kRcThreads = 1024;
constexpr int kRows64 = 2 * kOm;              // rows 0..39 after the swap, 40..79 before
constexpr int kRcSplit = 1;                   // blocks sharing one queued trial
constexpr int kRcRowsB = kRows64 / kRcSplit;  // rows per block: all 80
constexpr int kRcParts = kRcThreads / kHid;   // 8 threads per hidden unit
constexpr int kRcRows = kRcRowsB / kRcParts;  // rows per thread: 10
constexpr int kHStride = kHid + 1;            // padded row stride of the activation buffer

// One block per (queued trial, block of kRcRowsB rows); with kRcSplit = 1 a block holds all
// 80 rows of its trial and reduces them from LDS.  With a split, each block writes its rows to
// row_e and the block that completes a trial (per-trial counter) reduces the 80 energies; the
// reduction is in a fixed order either way, then the decision and the apply.  No block ever
// waits for another.  A split was measured several times slower: every block's device-scope
// fence writes back the L2 that the colour kernel has just dirtied.  The layer-0 slot loop
// stays rolled: at 1024 threads (128 VGPRs) unrolling it by three already spills.
__global__ __launch_bounds__(kRcThreads) void k_recheck(RecheckArgs a) {
  __shared__ double s_h[kRcRowsB * kHStride];  // activations, then per-unit terms of layer 2
  __shared__ double s_part[kRcRowsB * kRcParts];
  __shared__ uint8_t s_reg[kReg];
  __shared__ uint8_t s_sp[kRcRowsB * 27];
  __shared__ double s_e[kRows64];
  __shared__ int s_last, s_accept;
  const uint32_t n = *a.q_count;
  const int tid = threadIdx.x;
  const int o = tid % kHid, part = tid / kHid;  // thread owns unit o for local rows part + 8j
  const double *W0 = a.w64, *b0 = W0 + kHid * 108, *W1 = b0 + kHid, *b1 = W1 + kHid * kHid, *W2 = b1 + kHid,
               *b2 = W2 + kHid;
  for (uint32_t w = blockIdx.x; w < n * kRcSplit; w += gridDim.x) {
    const uint32_t q = w / kRcSplit;
    const int r0 = (int)(w % kRcSplit) * kRcRowsB;
    const RecheckEntry &e = a.queue[q];
    if (e.site < 0) continue;  // probe entry without a valid site (uniform across the block)
    const Replica R = a.reps[e.replica];
    uint8_t *occ = a.occ + R.site0;
    const Pos pi = site_pos(e.site, R.L[0], R.L[1]);
    const int d = e.dir;
    const uint8_t si = occ[e.site], sn = occ[e.partner];
    const int pos_i = a.reg_pos[2 * d], pos_n = a.reg_pos[2 * d + 1];
    if (tid < kReg) {
      int dx, dy, dz;
      unpack_off(a.reg_off[d * kReg + tid], dx, dy, dz);
      s_reg[tid] = occ[site_at(pi, dx, dy, dz, R.L[0], R.L[1], R.L[2])];
    }
    __syncthreads();
    // slot species of this block's rows (post-swap rows see i and n exchanged)
    for (int v = tid; v < kRcRowsB * 27; v += kRcThreads) {
      const int lr = v / 27, m = v - lr * 27, gr = r0 + lr;
      const bool post = gr < kOm;
      const int p = a.idx[(d * kOm + (post ? gr : gr - kOm)) * kIdxRow + m];
      s_sp[v] = post ? (p == pos_i ? sn : (p == pos_n ? si : s_reg[p])) : s_reg[p];
    }
    __syncthreads();
    // layer 0 + activation: the selected W0 column of each slot, added in slot order
    {
      double acc[kRcRows];
#pragma unroll
      for (int j = 0; j < kRcRows; ++j) acc[j] = b0[o];
#pragma unroll 1
      for (int m = 0; m < 27; ++m) {
        const double w0 = W0[(4 * m) * kHid + o], w1 = W0[(4 * m + 1) * kHid + o],
                     w2 = W0[(4 * m + 2) * kHid + o], w3 = W0[(4 * m + 3) * kHid + o];
#pragma unroll
        for (int j = 0; j < kRcRows; ++j) {
          const int sp = s_sp[(part + kRcParts * j) * 27 + m];
          const double wv = sp == 0 ? w0 : (sp == 1 ? w1 : (sp == 2 ? w2 : w3));
          if (sp < 4) acc[j] += wv;
        }
      }
#pragma unroll
      for (int j = 0; j < kRcRows; ++j) s_h[(part + kRcParts * j) * kHStride + o] = silu<double>(acc[j]);
    }
    __syncthreads();
    // layer 1 + activation, times W2
    {
      double acc[kRcRows];
#pragma unroll
      for (int j = 0; j < kRcRows; ++j) acc[j] = b1[o];
#pragma unroll 16
      for (int k = 0; k < kHid; ++k) {
        const double wk = W1[k * kHid + o];
#pragma unroll
        for (int j = 0; j < kRcRows; ++j) acc[j] = fma(wk, s_h[(part + kRcParts * j) * kHStride + k], acc[j]);
      }
      __syncthreads();
      const double w2 = W2[o];
#pragma unroll
      for (int j = 0; j < kRcRows; ++j) s_h[(part + kRcParts * j) * kHStride + o] = w2 * silu<double>(acc[j]);
    }
    __syncthreads();
    // E_r = b2 + sum over units in a fixed order: 8 consecutive chunks of 16, then the chunks
    if (tid < kRcRowsB * kRcParts) {
      const int lr = tid / kRcParts, c = tid % kRcParts;
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < kHid / kRcParts; ++i) s += s_h[lr * kHStride + c * (kHid / kRcParts) + i];
      s_part[tid] = s;
    }
    __syncthreads();
    if (tid < kRcRowsB) {
      double E = b2[0];
#pragma unroll
      for (int c = 0; c < kRcParts; ++c) E += s_part[tid * kRcParts + c];
      if constexpr (kRcSplit == 1) s_e[tid] = E;
      else a.row_e[(size_t)q * kRows64 + r0 + tid] = E;
    }
    if constexpr (kRcSplit > 1) {
      __threadfence();
      __syncthreads();
      if (tid == 0) s_last = atomicAdd(&a.done[q], 1u) == kRcSplit - 1;
      __syncthreads();
    } else {
      if (tid == 0) s_last = 1;
      __syncthreads();
    }
    if (s_last) {
      if constexpr (kRcSplit > 1) __threadfence();
      if (tid == 0) {
        double e1 = 0.0, e0 = 0.0;
        if constexpr (kRcSplit == 1) {
          for (int k = 0; k < kOm; ++k) e1 += s_e[k];
          for (int k = 0; k < kOm; ++k) e0 += s_e[kOm + k];
        } else {
          const double *re = a.row_e + (size_t)q * kRows64;
          for (int k = 0; k < kOm; ++k) e1 += __hip_atomic_load(re + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          for (int k = 0; k < kOm; ++k)
            e0 += __hip_atomic_load(re + kOm + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          a.done[q] = 0;  // ready for the next use of this queue slot
        }
        const double dE = e1 - e0;
        const bool probe = a.probe_dE != nullptr;
        const bool accept = !probe && dE <= e.theta;
        const int Rn = a.n_replicas;
        if (probe) a.probe_dE[q] = dE;
        if (accept) {
          occ[e.site] = sn;
          occ[e.partner] = si;
          atomicAdd(&a.e_fixed[e.replica], (unsigned long long)to_fixed(dE));
          atomicAdd((unsigned long long *)&a.counters[2 * Rn + e.replica], 1ull);
        }
        if (!probe) atomicAdd((unsigned long long *)&a.counters[3 * Rn + e.replica], 1ull);
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
    }
    __syncthreads();
  }
}

}  // namespace smc

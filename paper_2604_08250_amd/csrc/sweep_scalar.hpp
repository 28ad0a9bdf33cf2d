// Sweep, energy and bookkeeping kernels of the per-lane path: one trial per lane.
#pragma once
#include "scalar_eval.hpp"
#include "tables.hpp"

namespace smc {

// Flags written to the per-site trace.
constexpr uint8_t kFlagAccept = 1, kFlagSame = 2, kFlagFp64 = 4;

struct SweepArgs {
  const Replica *reps;
  uint8_t *occ;
  float *ecache;
  const float *w32;
  const double *w64;
  const int8_t *omega;     // [8][kOmegaMax][3]
  int32_t omega_n;
  int32_t replica;          // the replica, when seg_start is null
  int32_t colour;
  // batched: the replicas that have this colour (seg_rep[nseg]) and the first block of each
  // (seg_start[nseg + 1], in blocks of kScalarBlock trials); block -> (replica, trial block)
  const int32_t *seg_rep;
  const int32_t *seg_start;
  int32_t nseg;
  int32_t fp64_mode;       // decide every trial with FP64 energies, no cache
  uint64_t seed;
  uint64_t sweep;
  double guard;
  unsigned long long *e_fixed;  // [n_replicas] accepted dE in units of 2^-32 eV
  uint64_t *counters;      // [4][n_replicas]: attempts, diff, accepts, rechecks
  int32_t n_replicas;
  double *trace_dE;
  double *trace_dE_fast;
  uint8_t *trace_flags;
};

// Accepted energy changes are summed per block in a fixed order and added to an integer
// accumulator in units of 2^-32 eV, so the running total does not depend on block order.
__device__ __forceinline__ long long to_fixed(double x) { return __double2ll_rn(x * 4294967296.0); }

// Trial site of (colour, trial) inside a replica, or -1 past the colour's last trial.  The
// trials of a colour run over the link cells long enough to hold its offset (the long cells
// come first on each axis), x fastest, so no trial index of a colour is spent on a cell that
// cannot hold it.  Link-cell indices stay below 2^31: 32-bit arithmetic.
__device__ inline int64_t trial_site(const Replica &R, int32_t colour, int64_t t) {
  int32_t o[3];
  colour_offsets(R, colour, o);
  const uint32_t nx = (uint32_t)axis_cells_holding(R.ax[0], o[0]),
                 ny = (uint32_t)axis_cells_holding(R.ax[1], o[1]),
                 nz = (uint32_t)axis_cells_holding(R.ax[2], o[2]);
  const uint32_t tu = (uint32_t)t;
  const uint32_t t1 = tu / nx, cz = t1 / ny;
  if (t < 0 || cz >= nz) return -1;
  const int32_t x = axis_start(R.ax[0], (int32_t)(tu - t1 * nx)) + o[0],
                y = axis_start(R.ax[1], (int32_t)(t1 - cz * ny)) + o[1],
                z = axis_start(R.ax[2], (int32_t)cz) + o[2];
  return (((int64_t)z * R.L[1] + y) * R.L[0] + x) * 2 + (colour & 1);
}

// Local energy of site j at position p.
template <int FEAT, int H, typename T>
__device__ inline T site_energy_at(const uint8_t *occ, const Replica &R, Pos p, int64_t j, bool swap, int64_t i,
                                   int64_t n, uint8_t si, uint8_t sn, const T *W) {
  uint8_t slot[kSlots];
  gather_slots_at(occ, p, j, R.L[0], R.L[1], R.L[2], FEAT == 0 ? 15 : kSlots, swap, i, n, si, sn, slot);
  if constexpr (FEAT == 2) return qsro_scalar<T>(slot, W);
  else return mlp_scalar<FEAT, H, T>(slot, W);
}

template <int FEAT, int H, typename T>
__device__ inline T site_energy(const uint8_t *occ, const Replica &R, int64_t j, bool swap, int64_t i,
                                int64_t n, uint8_t si, uint8_t sn, const T *W) {
  return site_energy_at<FEAT, H, T>(occ, R, site_pos(j, R.L[0], R.L[1]), j, swap, i, n, si, sn, W);
}

// Zone site k of a trial at pi: its position (wrapped per axis) and replica-local index.
__device__ inline int64_t zone_site(const Replica &R, Pos pi, const int8_t *om, int k, Pos &pj) {
  pj = Pos{wrap1(pi.x + om[3 * k], 2 * R.L[0]), wrap1(pi.y + om[3 * k + 1], 2 * R.L[1]),
           wrap1(pi.z + om[3 * k + 2], 2 * R.L[2])};
  return site_index(pj, R.L[0], R.L[1]);
}

// Local energy of every site of one replica (FP32 into the cache, or FP64).
template <int FEAT, int H, typename T>
__global__ void k_site_energies(const Replica *reps, int32_t r, const uint8_t *occ, const T *W, T *out) {
  const Replica R = reps[r];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= R.n_sites) return;
  const uint8_t *o = occ + R.site0;
  out[R.site0 + j] = site_energy<FEAT, H, T>(o, R, j, false, -1, -1, 0, 0, W);
}

constexpr int kScalarBlock = 64;

// One colour (mini-step) of one replica, or of every replica that has it (each block serves
// one replica); one lane per link cell.
template <int FEAT, int H>
__global__ __launch_bounds__(kScalarBlock) void k_sweep_colour_scalar(SweepArgs a) {
  __shared__ float s_e1[kScalarBlock][kOmegaMax];
  __shared__ double s_de[kScalarBlock];
  __shared__ uint32_t s_cnt[3];
  // XCD-aware order: blocks b and b + 8k run on one XCD (round-robin dispatch), so logical
  // block (b % 8) per + b / 8 gives each XCD one contiguous run of link-cell rows, whose read
  // regions overlap and stay in that XCD's L2 (the tail past a multiple of 8 keeps its index)
  int blk = (int)blockIdx.x;
  {
    const int nb = (int)gridDim.x, full = nb - nb % 8;
    if (blk < full) blk = (blk % 8) * (full / 8) + blk / 8;
  }
  int rep = a.replica;
  if (a.seg_start) {
    int lo = 0, hi = a.nseg;  // last segment whose first block is <= blockIdx.x
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (a.seg_start[mid] <= blk) lo = mid;
      else hi = mid;
    }
    rep = a.seg_rep[lo];
    blk -= a.seg_start[lo];
  }
  const Replica R = a.reps[rep];
  const int tid = threadIdx.x;
  const int64_t t = (int64_t)blk * kScalarBlock + tid;
  if (tid < 3) s_cnt[tid] = 0;
  __syncthreads();
  double applied = 0.0;
  const int64_t i = t < R.n_trials ? trial_site(R, a.colour, t) : -1;
  if (i >= 0) {
    uint8_t *occ = a.occ + R.site0;
    float *ec = a.ecache + R.site0;
    const U64x4 r = philox4x64_10((uint64_t)i, a.sweep, (uint64_t)rep, 0, a.seed, 0);
    const int d = (int)(r.v[0] >> 61);
    const double u = (double)((r.v[1] >> 11) + 1) * 0x1.0p-53;
    const double theta = isinf(R.temperature) ? (double)INFINITY
                                              : -kBoltzmannEvPerK * R.temperature * log(u);
    const Pos pi = site_pos(i, R.L[0], R.L[1]);
    const int64_t n = site_at(pi, shell_dx(d), shell_dy(d), shell_dz(d), R.L[0], R.L[1], R.L[2]);
    const uint8_t si = occ[i], sn = occ[n];
    uint8_t flags = 0;
    double dE = 0.0, dE_fast = 0.0;
    if (si == sn) {
      flags = kFlagSame;
    } else {
      atomicAdd(&s_cnt[0], 1u);
      const int8_t *om = a.omega + d * kOmegaMax * 3;
      bool exact = a.fp64_mode != 0;
      if (!exact) {
        float acc = 0.0f;
        for (int k = 0; k < a.omega_n; ++k) {
          Pos pj;
          const int64_t j = zone_site(R, pi, om, k, pj);
          const float e1 = site_energy_at<FEAT, H, float>(occ, R, pj, j, true, i, n, si, sn, a.w32);
          s_e1[tid][k] = e1;
          acc += e1 - ec[j];
        }
        dE_fast = (double)acc;
        dE = dE_fast;
        if (fabs(dE_fast - theta) < a.guard) exact = true;
      }
      if (exact) {
        double e1 = 0.0, e0 = 0.0;
        for (int k = 0; k < a.omega_n; ++k) {
          Pos pj;
          const int64_t j = zone_site(R, pi, om, k, pj);
          e1 += site_energy_at<FEAT, H, double>(occ, R, pj, j, true, i, n, si, sn, a.w64);
          e0 += site_energy_at<FEAT, H, double>(occ, R, pj, j, false, i, n, si, sn, a.w64);
        }
        dE = e1 - e0;
        flags |= kFlagFp64;
        atomicAdd(&s_cnt[2], 1u);
        if (a.fp64_mode) dE_fast = dE;
      }
      if (dE <= theta) {
        flags |= kFlagAccept;
        atomicAdd(&s_cnt[1], 1u);
        applied = dE;
        occ[i] = sn;
        occ[n] = si;
        for (int k = 0; k < a.omega_n; ++k) {
          const int64_t j = site_at(pi, om[3 * k], om[3 * k + 1], om[3 * k + 2], R.L[0], R.L[1], R.L[2]);
          if (!a.fp64_mode) ec[j] = s_e1[tid][k];
        }
      }
    }
    if (a.trace_flags) a.trace_flags[R.site0 + i] = flags;
    if (a.trace_dE) a.trace_dE[R.site0 + i] = dE;
    if (a.trace_dE_fast) a.trace_dE_fast[R.site0 + i] = dE_fast;
  }
  s_de[tid] = applied;
  const unsigned long long valid = __ballot(i >= 0);
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int k = 0; k < kScalarBlock; ++k) s += s_de[k];
    atomicAdd(&a.e_fixed[rep], (unsigned long long)to_fixed(s));
    const int R_ = a.n_replicas;
    atomicAdd((unsigned long long *)&a.counters[0 * R_ + rep], (unsigned long long)__popcll(valid));
    atomicAdd((unsigned long long *)&a.counters[1 * R_ + rep], (unsigned long long)s_cnt[0]);
    atomicAdd((unsigned long long *)&a.counters[2 * R_ + rep], (unsigned long long)s_cnt[1]);
    atomicAdd((unsigned long long *)&a.counters[3 * R_ + rep], (unsigned long long)s_cnt[2]);
  }
}

// Deterministic sum of n doubles (fixed per-thread strides, fixed tree); out += sum.
__global__ void k_sum_into(const double *v, int64_t n, double *out, int accumulate) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += 256) acc += v[k];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = accumulate ? *out + s[0] : s[0];
}

// Pair counts for short-range order: per coordination shell m (1..3) and ordered species pair
// (p, q), the number of (site, shell-m neighbour) pairs with those species, and the number of
// sites of each species; per-block LDS histograms, then one global add per counter.
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
    const Pos pos = site_pos(j, R.L[0], R.L[1]);
    for (int k = 0; k < kNbr; ++k) {
      const int q = occ[site_at(pos, shell_dx(k), shell_dy(k), shell_dz(k), R.L[0], R.L[1], R.L[2])];
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

// Fill n words with v (grid-stride, so any launch shape covers all of them).
__global__ void k_fill_u64(uint64_t *p, int64_t n, uint64_t v) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    p[k] = v;
}

__global__ void k_widen(const float *in, double *out, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = (double)in[k];
}

__global__ void k_copy_f32(const float *in, float *out, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = in[k];
}

__global__ void k_narrow(const double *in, float *out, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = (float)in[k];
}

}  // namespace smc

// Double-lattice sweep strategy: Algorithm 1 of the paper as written (Sec. III-A).  Per
// mini-step (colour) the whole lattice is evaluated twice, E0 from sigma0 and E1 from sigma1,
// the auxiliary lattice in which every trial of the colour has swapped its pair; each link
// cell then reduces E1 - E0 over its affected zone Omega, decides by the Metropolis criterion,
// and accepted pairs are copied from sigma1 to sigma0.  Rejected pairs are copied back from
// sigma0 to sigma1, so the two lattices agree again at the end of the mini-step.
//
// The evaluators are the zone strategy's (the same tile evaluator over whole lattices), and
// the zone sums use the zone strategy's order (eight partial sums of five sites, added in
// order), so both strategies follow the same trajectory bit for bit; the double lattice
// evaluates every site twice per mini-step instead of the 40 zone sites of each trial once.
#pragma once
#include "sweep_mfma.hpp"

namespace smc {

struct DlTrial {
  int32_t site;     // replica-local trial site, -1 where the link cell has no site of this colour
  int32_t partner;
  double theta;
  int32_t dir;
  int32_t same;
};

struct DlArgs {
  const Replica *reps;
  int32_t r, colour;
  const uint64_t *sweep;
  uint64_t seed;
  uint8_t *occ;       // sigma0 (all replicas)
  uint8_t *sigma1;    // sigma1 (all replicas)
  DlTrial *trials;    // [n_trials of the colour]
  const float *E0, *E1;  // [N_total]
  float *ecache;
  const uint16_t *om_off;  // [8][40]
  double guard;
  uint32_t *q_count;
  RecheckEntry *queue;
  unsigned long long *e_fixed;
  uint64_t *counters;
  int32_t n_replicas;
  double *trace_dE, *trace_dE_fast;
  uint8_t *trace_flags;
};

// Proposals of the colour (Philox stream as in the zone strategy); different-species trials
// swap their pair in sigma1.
__global__ void k_dl_propose(DlArgs a) {
  const Replica R = a.reps[a.r];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= R.n_trials) return;
  DlTrial tr{-1, 0, 0.0, 0, 1};
  const int64_t i = trial_site(R, a.colour, t);
  if (i >= 0) {
    const U64x4 x = philox4x64_10((uint64_t)i, *a.sweep, (uint64_t)a.r, 0, a.seed, 0);
    const int d = (int)(x.v[0] >> 61);
    const double u = (double)((x.v[1] >> 11) + 1) * 0x1.0p-53;
    const Pos pi = site_pos(i, R.L[0], R.L[1]);
    const int64_t n = site_at(pi, shell_dx(d), shell_dy(d), shell_dz(d), R.L[0], R.L[1], R.L[2]);
    const uint8_t si = a.occ[R.site0 + i], sn = a.occ[R.site0 + n];
    tr.site = (int32_t)i;
    tr.partner = (int32_t)n;
    tr.theta = isinf(R.temperature) ? (double)INFINITY : -kBoltzmannEvPerK * R.temperature * log(u);
    tr.dir = d;
    tr.same = si == sn;
    if (!tr.same) {
      a.sigma1[R.site0 + i] = sn;
      a.sigma1[R.site0 + n] = si;
    }
  }
  a.trials[t] = tr;
}

// Zone reductions of E1 - E0, decision and copy-back, one trial per lane.  Lanes 0-31 and
// 32-63 of a wave hold the trials of two groups of 32 link cells, whose accepted dE are summed
// as in the zone strategy before entering the running total.
__global__ __launch_bounds__(256) void k_dl_decide(DlArgs a) {
  const Replica R = a.reps[a.r];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool live = t < R.n_trials;
  DlTrial tr{-1, 0, 0.0, 0, 1};
  if (live) tr = a.trials[t];
  const bool valid = tr.site >= 0;
  const bool active = valid && !tr.same;
  bool accept = false;
  double dEd = 0.0;
  const int64_t i = tr.site, n = tr.partner;
  if (valid && tr.same) {
    if (a.trace_flags) a.trace_flags[R.site0 + i] = kFlagSame;
    if (a.trace_dE) a.trace_dE[R.site0 + i] = 0.0;
    if (a.trace_dE_fast) a.trace_dE_fast[R.site0 + i] = 0.0;
  }
  if (active) {
    const Pos pi = site_pos(i, R.L[0], R.L[1]);
    float dE = 0.0f;
    for (int part = 0; part < kPart; ++part) {
      float s = 0.0f;
      for (int k = 0; k < kOm / kPart; ++k) {
        int dx, dy, dz;
        unpack_off(a.om_off[tr.dir * kOm + part * (kOm / kPart) + k], dx, dy, dz);
        const int64_t j = R.site0 + site_at(pi, dx, dy, dz, R.L[0], R.L[1], R.L[2]);
        s += a.E1[j] - a.E0[j];
      }
      dE += s;
    }
    dEd = (double)dE;
    if (fabs(dEd - tr.theta) < a.guard) {
      const uint32_t slot = atomicAdd(a.q_count, 1u);
      RecheckEntry &e = a.queue[slot];
      e.has_reg = 0;
      e.site = i;
      e.partner = n;
      e.theta = tr.theta;
      e.dE_fast = dE;
      e.replica = a.r;
      e.dir = tr.dir;
      for (int k = 0; k < kOm; ++k) {
        int dx, dy, dz;
        unpack_off(a.om_off[tr.dir * kOm + k], dx, dy, dz);
        e.e1[k] = a.E1[R.site0 + site_at(pi, dx, dy, dz, R.L[0], R.L[1], R.L[2])];
      }
      if (a.trace_dE_fast) a.trace_dE_fast[R.site0 + i] = dEd;
    } else {
      accept = dEd <= tr.theta;
      if (accept) {
        a.occ[R.site0 + i] = a.sigma1[R.site0 + i];
        a.occ[R.site0 + n] = a.sigma1[R.site0 + n];
        for (int k = 0; k < kOm; ++k) {
          int dx, dy, dz;
          unpack_off(a.om_off[tr.dir * kOm + k], dx, dy, dz);
          const int64_t j = R.site0 + site_at(pi, dx, dy, dz, R.L[0], R.L[1], R.L[2]);
          a.ecache[j] = a.E1[j];
        }
      }
      if (a.trace_flags) a.trace_flags[R.site0 + i] = accept ? kFlagAccept : 0;
      if (a.trace_dE) a.trace_dE[R.site0 + i] = dEd;
      if (a.trace_dE_fast) a.trace_dE_fast[R.site0 + i] = dEd;
    }
  }
  // group sums of accepted dE (32 lanes, the zone strategy's order) and counters
  double v = accept ? dEd : 0.0;
  const int l32 = lane & 31;
  for (int off = 1; off < 32; off <<= 1) {
    const double o = __shfl_down(v, off, 32);
    v += (l32 + off < 32) ? o : 0.0;
  }
  const unsigned long long vmask = __ballot(valid), amask = __ballot(active), cmask = __ballot(accept);
  if (l32 == 0 && v != 0.0) atomicAdd(&a.e_fixed[a.r], (unsigned long long)to_fixed(v));
  if (lane == 0) {
    const int Rn = a.n_replicas;
    atomicAdd((unsigned long long *)&a.counters[0 * Rn + a.r], (unsigned long long)__popcll(vmask));
    atomicAdd((unsigned long long *)&a.counters[1 * Rn + a.r], (unsigned long long)__popcll(amask));
    atomicAdd((unsigned long long *)&a.counters[2 * Rn + a.r], (unsigned long long)__popcll(cmask));
  }
}

// After the FP64 re-decisions: sigma1 takes sigma0's species at every trial pair again.
__global__ void k_dl_sync(DlArgs a) {
  const Replica R = a.reps[a.r];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= R.n_trials) return;
  const DlTrial tr = a.trials[t];
  if (tr.site < 0 || tr.same) return;
  a.sigma1[R.site0 + tr.site] = a.occ[R.site0 + tr.site];
  a.sigma1[R.site0 + tr.partner] = a.occ[R.site0 + tr.partner];
}

}  // namespace smc

// FP64 local energies of every site for the one-hot model with 128 hidden units, on the FP64
// matrix cores with the re-decision's row evaluator (rows64_half), so that a site's FP64 energy
// here and in a re-decided zone is the same number.  Persistent blocks of 512 threads, one per
// CU: the weights are staged in LDS once, then each half block takes 16 consecutive sites at a
// time (half 1 G items after half 0, G blocks), gathers their 27 slot species and evaluates them;
// each thread loads its species of the next item while the current one is evaluated.
#pragma once
#include "rows64.hpp"
#include "tables.hpp"

namespace smc {

constexpr int kS64Rows = kR64Rows;
constexpr int kS64Threads = kR64Threads;

// w32t / w64t: the blob with W0 and W1 stored [input][unit] in FP32 and FP64:
// W0t[108][128], b0, W1t[128][128], b1, W2, b2.
__global__ __launch_bounds__(kS64Threads) void k_site_energies64_onehot(const Replica *reps, int32_t r,
                                                                       const uint8_t *occ_all, const float *w32t,
                                                                       const double *w64t, double *out) {
  __shared__ __attribute__((aligned(16))) Rows64W s_wt;
  __shared__ __attribute__((aligned(16))) Rows64Half s_half[2];
  const Replica R = reps[r];
  const uint8_t *occ = occ_all + R.site0;
  const int64_t items = (R.n_sites + kS64Rows - 1) / kS64Rows;
  if ((int64_t)blockIdx.x >= items) return;  // no work item for this block
  const int tid = threadIdx.x, hf = tid / kR64Half, lt = tid % kR64Half;
  const double b2 = w64t[kR64Hid * 108 + kR64Hid + kR64Hid * kR64Hid + 2 * kR64Hid];
  // the two slot species of this thread for item w (16 rows x 27 slots over the half's 256
  // threads); rows past the end get species 4 (no channel) and are not written
  auto fetch = [&](int64_t w, uint8_t (&sp)[2]) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int v = lt + k * kR64Half;
      sp[k] = 4;
      if (w < items && v < kS64Rows * kSlots) {
        const int lr = v / kSlots, m = v - lr * kSlots;
        const int64_t j = w * kS64Rows + lr;
        if (j < R.n_sites) {
          if (m == 0) {
            sp[k] = occ[j];
          } else {
            const Pos p = site_pos32((int32_t)j, R.L[0], R.L[1]);
            sp[k] = occ[site_at32(p, shell_dx(m - 1), shell_dy(m - 1), shell_dz(m - 1), R.L[0], R.L[1], R.L[2])];
          }
        }
      }
    }
  };
  uint8_t cur[2], nxt[2];
  fetch(blockIdx.x + hf * (int64_t)gridDim.x, cur);
  rows64_stage(s_wt, w32t, w64t, [] {});
  for (int64_t base = blockIdx.x; base < items; base += 2 * (int64_t)gridDim.x) {
    const int64_t w = base + hf * (int64_t)gridDim.x;
    const bool live = w < items;
    const int64_t j0 = w * kS64Rows;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int v = lt + k * kR64Half;
      if (live && v < kS64Rows * kSlots) {
        const int lr = v / kSlots;
        s_half[hf].sp[lr * kR64SpStride + (v - lr * kSlots)] = cur[k];
      }
    }
    __syncthreads();
    fetch(w + 2 * (int64_t)gridDim.x, nxt);  // in flight during the evaluation
    const double E = rows64_half(s_wt, b2, live, lt, s_half[hf], [] {});
    if (live && lt < kS64Rows && j0 + lt < R.n_sites) out[R.site0 + j0 + lt] = E;
    __syncthreads();
    cur[0] = nxt[0];
    cur[1] = nxt[1];
  }
}

}  // namespace smc

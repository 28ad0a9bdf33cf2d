// FP64 local energies of every site for the one-hot model with 128 hidden units, one block per
// 64 sites at a time: thread (unit o, part p) owns rows p + 8 j.  Every output is accumulated in
// the same order as the per-lane evaluator (layer-0 columns in slot order, layer-1 products in
// unit order, the output sum in unit order); this kernel shares the weight loads of a unit
// across the rows of a block instead of reloading them per site.
#pragma once
#include "scalar_eval.hpp"
#include "tables.hpp"

namespace smc {

constexpr int kS64Rows = 64;
constexpr int kS64Threads = 1024;
constexpr int kS64Hid = 128;
constexpr int kS64Parts = kS64Threads / kS64Hid;      // 8
constexpr int kS64PerThread = kS64Rows / kS64Parts;   // 8
constexpr int kS64Stride = kS64Hid + 1;

// W: FP64 blob with W0 and W1 stored [input][unit]: W0t[108][128], b0, W1t[128][128], b1, W2, b2.
__global__ __launch_bounds__(kS64Threads) void k_site_energies64_onehot(const Replica *reps, int32_t r,
                                                                       const uint8_t *occ_all, const double *W,
                                                                       double *out) {
  __shared__ double s_h[kS64Rows * kS64Stride];
  __shared__ uint8_t s_sp[kS64Rows * kSlots];
  const Replica R = reps[r];
  const uint8_t *occ = occ_all + R.site0;
  const int tid = threadIdx.x;
  const int o = tid % kS64Hid, part = tid / kS64Hid;
  const double *W0 = W, *b0 = W0 + 108 * kS64Hid, *W1 = b0 + kS64Hid, *b1 = W1 + kS64Hid * kS64Hid,
               *W2 = b1 + kS64Hid, *b2 = W2 + kS64Hid;
  const int64_t passes = (R.n_sites + kS64Rows - 1) / kS64Rows;
  for (int64_t pass = blockIdx.x; pass < passes; pass += gridDim.x) {
    const int64_t j0 = pass * kS64Rows;
    const int nrows = R.n_sites - j0 < kS64Rows ? (int)(R.n_sites - j0) : kS64Rows;
    for (int v = tid; v < kS64Rows * kSlots; v += kS64Threads) {
      const int lr = v / kSlots, m = v - lr * kSlots;
      uint8_t sp = 4;  // rows past the end: no channel
      if (lr < nrows) {
        const int64_t j = j0 + lr;
        if (m == 0) {
          sp = occ[j];
        } else {
          const Pos p = site_pos(j, R.L[0], R.L[1]);
          sp = occ[site_at(p, shell_dx(m - 1), shell_dy(m - 1), shell_dz(m - 1), R.L[0], R.L[1], R.L[2])];
        }
      }
      s_sp[v] = sp;
    }
    __syncthreads();
    double acc[kS64PerThread];
#pragma unroll
    for (int q = 0; q < kS64PerThread; ++q) acc[q] = b0[o];
#pragma unroll 1
    for (int m = 0; m < kSlots; ++m) {
      const double w0 = W0[(4 * m) * kS64Hid + o], w1 = W0[(4 * m + 1) * kS64Hid + o],
                   w2 = W0[(4 * m + 2) * kS64Hid + o], w3 = W0[(4 * m + 3) * kS64Hid + o];
#pragma unroll
      for (int q = 0; q < kS64PerThread; ++q) {
        // no branch: species 4 adds +0.0, which leaves the sum as it is
        const int sp = s_sp[(part + kS64Parts * q) * kSlots + m];
        const double wv = sp == 0 ? w0 : (sp == 1 ? w1 : (sp == 2 ? w2 : w3));
        acc[q] += sp < 4 ? wv : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < kS64PerThread; ++q) s_h[(part + kS64Parts * q) * kS64Stride + o] = silu<double>(acc[q]);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kS64PerThread; ++q) acc[q] = b1[o];
#pragma unroll 16
    for (int k = 0; k < kS64Hid; ++k) {
      const double wk = W1[k * kS64Hid + o];
#pragma unroll
      for (int q = 0; q < kS64PerThread; ++q) acc[q] = fma(wk, s_h[(part + kS64Parts * q) * kS64Stride + k], acc[q]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kS64PerThread; ++q) s_h[(part + kS64Parts * q) * kS64Stride + o] = silu<double>(acc[q]);
    __syncthreads();
    if (tid < nrows) {
      double e = b2[0];
      for (int k = 0; k < kS64Hid; ++k) e = fma(W2[k], s_h[tid * kS64Stride + k], e);
      out[R.site0 + j0 + tid] = e;
    }
    __syncthreads();
  }
}

}  // namespace smc

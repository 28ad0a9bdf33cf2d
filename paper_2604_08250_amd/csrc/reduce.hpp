// Two-stage deterministic sum of a long array of doubles (the FP64 from-scratch totals).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sweep_scalar.hpp"

namespace smc {

// Partial sums of n doubles over gridDim.x contiguous chunks (a fixed partition of [0, n)),
// each in the order of k_sum_into, into part[block].
__global__ void k_sum_chunks(const double *v, int64_t n, double *part) {
  __shared__ double s[256];
  const int64_t G = gridDim.x, b = blockIdx.x;
  const int64_t lo = n * b / G, hi = n * (b + 1) / G;
  double acc = 0.0;
  for (int64_t k = lo + threadIdx.x; k < hi; k += 256) acc += v[k];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[b] = s[0];
}

// Chunks of the two-stage sum: at most kSumChunks blocks of at least 2^16 values each.
constexpr int kSumChunks = 1024;

// out = sum of n device doubles in an order fixed by n alone: one block for short arrays,
// else chunk partials (part: device scratch of kSumChunks doubles) and their sum.
inline void sum_doubles(hipStream_t stream, const double *v, int64_t n, double *part, double *out) {
  const int64_t G = std::min<int64_t>(kSumChunks, n >> 16);
  if (G < 2) {
    hipLaunchKernelGGL(k_sum_into, dim3(1), dim3(256), 0, stream, v, n, out, 0);
    return;
  }
  hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)G), dim3(256), 0, stream, v, n, part);
  hipLaunchKernelGGL(k_sum_into, dim3(1), dim3(256), 0, stream, (const double *)part, G, out, 0);
}

}  // namespace smc

// Norms and relative error of Eq. (8): ||A||_F^2, ||G||_F^2 and
// RE = sqrt((||A||^2 - ||G||^2) / ||A||^2), which is ||A - A^|| / ||A|| for
// orthonormal factors (A^ is then the orthogonal projection of A onto the
// tensor product of the factors' ranges, so ||A - A^||^2 = ||A||^2 - ||G||^2).
// Sums run in float64 over fixed partitions in a fixed order, so the results
// are reproducible run to run.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace trk {

constexpr int kNormNT = 256;
constexpr int kNormMaxParts = 1024;

// parts[b] = sum over the elements e = b*256 + t + k * gridDim*256 of x[e]
// (SQ: x[e]^2), each thread in increasing k, then a fixed tree per block.
template <typename T, bool SQ>
__global__ void __launch_bounds__(kNormNT)
k_partial_sum(const T* __restrict__ x, int64_t n, double* __restrict__ parts) {
  __shared__ double red[kNormNT];
  const int64_t stride = (int64_t)gridDim.x * kNormNT;
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kNormNT + threadIdx.x; e < n; e += stride) {
    const double v = (double)x[e];
    acc = SQ ? fma(v, v, acc) : acc + v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kNormNT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) parts[blockIdx.x] = red[0];
}

// out[0] = ||A||^2 = sum of the nparts partials (in order), out[1] = ||G||^2
// over the float64 core, out[2] = RE.  One workgroup.
static __global__ void __launch_bounds__(kNormNT)
k_norms_re(const double* __restrict__ parts, int nparts, const double* __restrict__ core,
           int64_t ncore, double* __restrict__ out) {
  __shared__ double red[kNormNT];
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < ncore; e += kNormNT) acc = fma(core[e], core[e], acc);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kNormNT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double a2 = 0.0;
    for (int b = 0; b < nparts; ++b) a2 += parts[b];
    const double g2 = red[0];
    out[0] = a2;
    out[1] = g2;
    out[2] = a2 > 0.0 ? sqrt(fmax(a2 - g2, 0.0) / a2) : 0.0;
  }
}

}  // namespace trk

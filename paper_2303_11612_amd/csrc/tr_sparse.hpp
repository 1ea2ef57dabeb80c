// Sparse input for the first mode of the ST-HOSVD with sampled products
// (Alg. 5 on the sparse tensors of Section 6.1 / 6.5): the mode-1 unfolding
// X_(1) (I_1 x J_1) in compressed sparse columns -- column j's nonzeros are
// entries colptr[j] .. colptr[j+1]-1 of rowidx / vals, rows in increasing
// order.  Only the first mode reads the sparse tensor: its column norms
// (nearly-optimal probabilities), the gather of the sampled columns and the
// shrink Q_1^T X_(1); the shrunk tensor is dense.  A row index outside
// [0, I_1) is skipped and flags kDevBadIndex.
#pragma once

#include "tr_colnorms.hpp"
#include "tr_kernels.hpp"

namespace trk {

// Squared norm of every column: the nonzeros in row order with the same
// square-and-add as the dense kernels (adding the zeros they also visit
// changes nothing), so the norms -- and the draws -- are those of the dense
// tensor bit for bit.
template <typename T>
__global__ void __launch_bounds__(kNT)
k_colnorms_csc(const int64_t* __restrict__ colptr, const T* __restrict__ vals, int64_t J,
               double* __restrict__ norms, unsigned long long* __restrict__ max_bits) {
  __shared__ unsigned long long scr[kNT / kWave];
  const int64_t j = (int64_t)blockIdx.x * kNT + threadIdx.x;
  double acc = 0.0;
  if (j < J) {
    const int64_t e1 = colptr[j + 1];
    for (int64_t e = colptr[j]; e < e1; ++e) acc = sq_add(acc, (double)vals[e]);
    norms[j] = acc;
  }
  if (max_bits) block_max_bits(j < J ? acc : 0.0, max_bits, scr);
}

// C'(:, t) = X_(1)(:, idx[t]) at the input's dtype (unscaled, as k_gather):
// workgroup t clears its column, then scatters the column's nonzeros.
template <typename T>
__global__ void __launch_bounds__(kNT)
k_gather_csc(const int64_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
             const T* __restrict__ vals, int64_t I, const int64_t* __restrict__ idx,
             T* __restrict__ Cp, uint32_t* __restrict__ status) {
  const int64_t t = blockIdx.x;
  T* col = Cp + I * t;
  for (int64_t i = threadIdx.x; i < I; i += kNT) col[i] = T(0);
  __syncthreads();
  const int64_t j = idx[t];
  const int64_t e1 = colptr[j + 1];
  for (int64_t e = colptr[j] + threadIdx.x; e < e1; e += kNT) {
    const int64_t r = rowidx[e];
    if (r >= 0 && r < I) col[r] = vals[e];
    else if (status) atomicOr(status, kDevBadIndex);
  }
}

// The first shrink Y = Q_1^T X_(1) (mu x J, float64, Y[k + kout j]): one
// thread per column, its nonzeros in row order; Qt is I x MU row-major (zero
// padded past kout).
template <typename T, int MU>
__global__ void __launch_bounds__(kNT)
k_ttm_csc(const int64_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
          const T* __restrict__ vals, int64_t I, int64_t J, const double* __restrict__ Qt,
          int kout, double* __restrict__ Y, uint32_t* __restrict__ status) {
  const int64_t j = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (j >= J) return;
  double acc[MU];
#pragma unroll
  for (int k = 0; k < MU; ++k) acc[k] = 0.0;
  const int64_t e1 = colptr[j + 1];
  for (int64_t e = colptr[j]; e < e1; ++e) {
    const int64_t r = rowidx[e];
    if (r < 0 || r >= I) {
      if (status) atomicOr(status, kDevBadIndex);
      continue;
    }
    const double v = (double)vals[e];
    const double* q = Qt + r * MU;
#pragma unroll
    for (int k = 0; k < MU; ++k) acc[k] = fma(q[k], v, acc[k]);
  }
#pragma unroll
  for (int k = 0; k < MU; ++k)
    if (k < kout) Y[k + (int64_t)kout * j] = acc[k];
}

}  // namespace trk

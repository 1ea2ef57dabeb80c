// Column norms n_j = ||A_(n)(:, j)||^2 of a mode-n view (Remark after
// Alg. 3: the nearly-optimal sampling probabilities are proportional to them)
// and the running maximum of their bit patterns, which the sampler's integer
// weights are scaled by.  Norms of the caller's tensor sum each column's rows
// in increasing order, one thread per column, so they are bit-exact.
#pragma once

#include "tr_consts.hpp"
#include "tr_device.hpp"

namespace trk {

// Square-and-add with two roundings (no fused multiply-add), the order the
// column norms are defined with.
__device__ __forceinline__ double sq_add(double acc, double x) {
#pragma clang fp contract(off)
  const double sq = x * x;
  return acc + sq;
}

// Largest IEEE bit pattern over the workgroup (non-negative doubles compare
// like their bit patterns; a NaN norm wins, which flags it downstream).
__device__ __forceinline__ void block_max_bits(double v, unsigned long long* out,
                                               unsigned long long* scratch) {
  unsigned long long b = (unsigned long long)__double_as_longlong(v);
#pragma unroll
  for (int m = 1; m < kWave; m <<= 1) {
    const unsigned long long o = __shfl_xor(b, m, kWave);
    b = o > b ? o : b;
  }
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) scratch[wid] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) m = scratch[w] > m ? scratch[w] : m;
    atomicMax(out, m);
  }
}

// Loads rows [i0, i0 + TI) of the kNT consecutive columns starting at `base`
// (an L == 1 view: column c is contiguous, length I) into registers, and
// stores them to tile[ii][c].  All TI loads of a thread are issued before any
// is consumed (out-of-range elements read a clamped in-range address and are
// not stored).
template <typename T, int TI>
__device__ __forceinline__ void load_fiber_chunk(const T* __restrict__ base, int64_t I,
                                                 int64_t i0, int ncol, T (&v)[TI],
                                                 bool (&ok)[TI]) {
#pragma unroll
  for (int m = 0; m < TI; ++m) {
    const int e = threadIdx.x + kNT * m;
    const int cc = e / TI, ii = e % TI;
    ok[m] = cc < ncol && i0 + ii < I;
    v[m] = base[ok[m] ? (int64_t)cc * I + i0 + ii : 0];
  }
}
template <typename T, int TI>
__device__ __forceinline__ void store_fiber_chunk(const T (&v)[TI], const bool (&ok)[TI],
                                                  T (*tile)[kNT + 1]) {
#pragma unroll
  for (int m = 0; m < TI; ++m) {
    const int e = threadIdx.x + kNT * m;
    if (ok[m]) tile[e % TI][e / TI] = v[m];
  }
}
template <typename T, int TI>
__device__ __forceinline__ void stage_fiber_chunk(const T* __restrict__ base, int64_t I,
                                                  int64_t i0, int ncol, T (*tile)[kNT + 1]) {
  T v[TI];
  bool ok[TI];
  load_fiber_chunk<T, TI>(base, I, i0, ncol, v, ok);
  store_fiber_chunk<T, TI>(v, ok, tile);
}

// The same chunk with 16-byte loads (VW consecutive rows of one column per
// load); needs I a multiple of VW and a 16-byte aligned base.
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int W = 4;
};
template <>
struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int W = 2;
};
template <typename T, int TI>
struct FiberChunkV {
  static constexpr int VW = Vec16<T>::W, NV = TI / VW;  // vectors per column chunk
  typename Vec16<T>::type v[NV];                           // NV = loads per thread
  bool ok[NV];
  __device__ __forceinline__ void load(const T* __restrict__ base, int64_t I, int64_t i0,
                                       int ncol) {
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      const int e = threadIdx.x + kNT * m;
      const int cc = e / NV, q = e % NV;
      ok[m] = cc < ncol && i0 + VW * q < I;
      v[m] = *reinterpret_cast<const typename Vec16<T>::type*>(
          base + (ok[m] ? (int64_t)cc * I + i0 + VW * q : 0));
    }
  }
  __device__ __forceinline__ void store(T (*tile)[kNT + 1]) const {
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      const int e = threadIdx.x + kNT * m;
      const int cc = e / NV, q = e % NV;
      if (ok[m]) {
#pragma unroll
        for (int t = 0; t < VW; ++t) tile[VW * q + t][cc] = v[m][t];
      }
    }
  }
};

// ---------------------------------------------------------------------------
// K3  Column norms n_j = ||A_(n)(:, j)||^2, rows summed in increasing order.
// VEC: the chunks are loaded 16 bytes at a time (I a multiple of 16/sizeof(T),
// X 16-byte aligned).
// ---------------------------------------------------------------------------
// Columns [256 blk, 256 blk + 256) of the view, by the calling workgroup
// (tile and scr: its LDS buffers).
template <typename T, bool VEC>
__device__ __forceinline__ void colnorms_l1_block(
    const T* __restrict__ X, int64_t I, int64_t J, double* __restrict__ norms,
    unsigned long long* __restrict__ max_bits, int64_t blk,
    T (*tile)[kNT + 1], unsigned long long* scr) {
  constexpr int TI = RowsPerChunk<T>::value;
  const int c = threadIdx.x;
  const int64_t j0 = blk * kNT;
  const int ncol = (int)min((int64_t)kNT, J - j0);
  const T* base = X + j0 * I;
  double acc = 0.0;
  // the next chunk's loads are in flight while this one is summed from LDS
  T v[VEC ? 1 : TI];
  bool ok[VEC ? 1 : TI];
  FiberChunkV<T, TI> cv;
  if constexpr (VEC) cv.load(base, I, 0, ncol);
  else load_fiber_chunk<T, TI>(base, I, 0, ncol, v, ok);
  for (int64_t i0 = 0; i0 < I; i0 += TI) {
    if constexpr (VEC) cv.store(tile);
    else store_fiber_chunk<T, TI>(v, ok, tile);
    __syncthreads();
    if (i0 + TI < I) {
      if constexpr (VEC) cv.load(base, I, i0 + TI, ncol);
      else load_fiber_chunk<T, TI>(base, I, i0 + TI, ncol, v, ok);
    }
    const int ti = (int)min((int64_t)TI, I - i0);
    if (c < ncol)
      for (int ii = 0; ii < ti; ++ii) acc = sq_add(acc, (double)tile[ii][c]);
    __syncthreads();
  }
  if (c < ncol) norms[j0 + c] = acc;
  if (max_bits) block_max_bits(c < ncol ? acc : 0.0, max_bits, scr);
}

template <typename T, bool VEC>
__global__ void __launch_bounds__(kNT)
k_colnorms_l1(const T* __restrict__ X, int64_t I, int64_t J,
              double* __restrict__ norms, unsigned long long* __restrict__ max_bits) {
  __shared__ T tile[RowsPerChunk<T>::value][kNT + 1];
  __shared__ unsigned long long scr[kNT / kWave];
  colnorms_l1_block<T, VEC>(X, I, J, norms, max_bits, blockIdx.x, tile, scr);
}

template <typename T>
__global__ void __launch_bounds__(kNT)
k_colnorms_ln(const T* __restrict__ X, int64_t L, int64_t I, int64_t R,
              double* __restrict__ norms, unsigned long long* __restrict__ max_bits) {
  __shared__ unsigned long long scr[kNT / kWave];
  const int64_t J = L * R;
  const int64_t j = (int64_t)blockIdx.x * kNT + threadIdx.x;
  double acc = 0.0;
  if (j < J) {
    const int64_t r = j / L, l = j - r * L;
    const T* p = X + l + L * I * r;
    constexpr int B = 16;  // loads in flight per thread; the sum stays in row order
    for (int64_t i0 = 0; i0 < I; i0 += B) {
      T v[B];
#pragma unroll
      for (int b = 0; b < B; ++b) v[b] = p[L * min(i0 + b, I - 1)];
#pragma unroll
      for (int b = 0; b < B; ++b)
        if (i0 + b < I) acc = sq_add(acc, (double)v[b]);
    }
    norms[j] = acc;
  }
  if (max_bits) block_max_bits(acc, max_bits, scr);
}

// Column norms of a tensor the library produced itself (ST-HOSVD's shrunk
// tensors, whose last bits differ from any other computation's anyway), for
// views with too few columns to fill the device one thread per column: S
// threads per column each sum a contiguous segment of ceil(I/S) rows in row
// order, and the segment sums are added in segment order (deterministic).
template <typename T, int S>
__global__ void __launch_bounds__(kNT)
k_colnorms_seg(const T* __restrict__ X, int64_t L, int64_t I, int64_t R,
               double* __restrict__ norms, unsigned long long* __restrict__ max_bits) {
  constexpr int CPB = kNT / S;  // columns per workgroup
  __shared__ double part[S][CPB + 1];
  __shared__ unsigned long long scr[kNT / kWave];
  const int cl = threadIdx.x % CPB, sg = threadIdx.x / CPB;
  const int64_t J = L * R;
  const int64_t j = (int64_t)blockIdx.x * CPB + cl;
  const int64_t seg = (I + S - 1) / S;
  const int64_t i0 = sg * seg, i1 = min(I, i0 + seg);
  double acc = 0.0;
  if (j < J) {
    const int64_t r = j / L, l = j - r * L;
    const T* p = X + l + L * I * r;
    constexpr int B = 16;
    for (int64_t a = i0; a < i1; a += B) {
      T v[B];
#pragma unroll
      for (int b = 0; b < B; ++b) v[b] = p[L * min(a + b, i1 - 1)];
#pragma unroll
      for (int b = 0; b < B; ++b)
        if (a + b < i1) acc = sq_add(acc, (double)v[b]);
    }
  }
  part[sg][cl] = acc;
  __syncthreads();
  double tot = 0.0;
  if (sg == 0 && j < J) {
    tot = part[0][cl];
#pragma unroll
    for (int g = 1; g < S; ++g) tot += part[g][cl];
    norms[j] = tot;
  }
  if (max_bits) block_max_bits(tot, max_bits, scr);
}

// Atomic maximum of the IEEE bit patterns of v[0..n) (used when the norms are
// supplied by the caller rather than produced by the column-norm kernel).
static __global__ void __launch_bounds__(kNT)
k_max_bits(const double* __restrict__ v, int64_t n, unsigned long long* __restrict__ out) {
  __shared__ unsigned long long scr[kNT / kWave];
  const int64_t j = (int64_t)blockIdx.x * kNT + threadIdx.x;
  block_max_bits(j < n ? v[j] : 0.0, out, scr);
}

}  // namespace trk

// Device helpers shared by the gfx950 kernels: the Philox4x64-10 generator and
// wave64 / workgroup reductions with a fixed (deterministic) combination order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trk {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 256-bit counter, 128-bit
// key, ten rounds.  Each round forms the 128-bit products of counter words 0
// and 2 with two odd multipliers and recombines them with words 1, 3 and the
// key; the key advances by two Weyl increments between rounds.
// ---------------------------------------------------------------------------
struct U64x4 {
  uint64_t w[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1,
                                               uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
  constexpr uint64_t kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
  constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t hi0 = __umul64hi(kM0, c0), lo0 = kM0 * c0;
    const uint64_t hi1 = __umul64hi(kM1, c2), lo1 = kM1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return U64x4{{c0, c1, c2, c3}};
}

// Counter word 2 ("tag") separates the two random streams of the method.
constexpr uint64_t kTagGauss = 0;
constexpr uint64_t kTagSample = 1;

// ---------------------------------------------------------------------------
// Reductions.  All combine in a fixed pattern, so results are bitwise
// reproducible run to run.
// ---------------------------------------------------------------------------

// Lane permutations through DPP (no LDS round trip).  A double moves as two
// 32-bit halves with the same control word.  Every pattern used here reads a
// valid lane for every lane in ROW_MASK; lanes outside ROW_MASK get an
// unspecified value, which callers select away.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Reciprocal and reciprocal square root for arguments in a moderate range
// (callers scale by powers of two first): the hardware estimate refined by
// two Newton-Raphson steps, r <- r + r (1 - x r) and y <- y + y (1 - x y^2) / 2,
// each of which squares the relative error.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}
// sqrt(x) = x / sqrt(x), with one Newton correction s <- s + (x - s^2) / (2 s).
__device__ __forceinline__ double sqrt_nr(double x) {
  const double y = rsqrt_nr(x);
  const double s = x * y;
  return fma(fma(-s, s, x), 0.5 * y, s);
}

// DPP control words (GFX9 encoding).
constexpr int kDppQuadXor1 = 0xb1;      // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4e;      // quad_perm [2,3,0,1]
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;

// Sum over the 64 lanes; every lane gets the total.  Quad, half-row and row
// stages by DPP, the two cross-row stages by row broadcasts, then the total
// (complete in lane 63) is read back to all lanes.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<kDppQuadXor1>(v);
  v += dpp_f64<kDppQuadXor2>(v);
  v += dpp_f64<kDppRowHalfMirror>(v);
  v += dpp_f64<kDppRowMirror>(v);
  // rows 1 and 3 add lane 15 of rows 0 and 2; rows 2 and 3 then add lane 31
  const double b15 = dpp_f64<kDppRowBcast15, 0xa>(v);
  v += ((threadIdx.x >> 4) & 1) ? b15 : 0.0;
  const double b31 = dpp_f64<kDppRowBcast31, 0xc>(v);
  v += ((threadIdx.x >> 5) & 1) ? b31 : 0.0;
  const long long t = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(t & 0xffffffff), 63);
  const int hi = __builtin_amdgcn_readlane((int)(t >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int m = 1; m < kWave; m <<= 1) v = fmax(v, __shfl_xor(v, m, kWave));
  return v;
}

// Sum over the workgroup of one double per thread; every thread gets the
// result.  `scratch` holds at least blockDim.x/64 + 1 doubles.  Contains two
// barriers; the caller must not reuse `scratch` before all threads returned.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  v = wave_sum(v);
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < nw; ++w) t += scratch[w];
  __syncthreads();
  return t;
}

// Transpose-reduce of M values (M a power of two <= 64) across one wave: on
// return lane l holds the wave-wide sum of value index wave_vec_index<M>(l).
// Uses M-1 + (6 - log2 M) shuffles instead of 6*M.  Every index is a
// compile-time constant (the halving stages are unrolled by recursion).
template <int M>
__device__ __forceinline__ int wave_vec_index(int lane) {
  int idx = 0;
  int half = M / 2;
#pragma unroll
  for (int b = 0; (1 << b) < M; ++b, half /= 2)
    if ((lane >> b) & 1) idx += half;
  return idx;
}

template <int M, int HALF, int B>
__device__ __forceinline__ void wave_vec_stage(double (&v)[M], int lane) {
  if constexpr (HALF >= 1) {
    const bool up = ((lane >> B) & 1) != 0;
#pragma unroll
    for (int q = 0; q < HALF; ++q) {
      const double send = up ? v[q] : v[q + HALF];
      const double keep = up ? v[q + HALF] : v[q];
      v[q] = keep + __shfl_xor(send, 1 << B, kWave);
    }
    wave_vec_stage<M, HALF / 2, B + 1>(v, lane);
  }
}

template <int M>
__device__ __forceinline__ double wave_vec_sum(double (&v)[M], int lane) {
  static_assert(M >= 1 && M <= kWave && (M & (M - 1)) == 0, "M power of 2");
  wave_vec_stage<M, M / 2, 0>(v, lane);
  double r = v[0];
#pragma unroll
  for (int mask = M; mask < kWave; mask <<= 1) r += __shfl_xor(r, mask, kWave);
  return r;
}

}  // namespace trk

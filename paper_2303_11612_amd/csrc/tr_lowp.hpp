// Low-precision power-scheme products: BF16 or FP8 (OCP e4m3, max 448)
// operands on the matrix cores with FP32 accumulation.  Everything that
// decides the factor stays float64: the Gaussian start, the sum of the
// per-block partial products, the QR and SVD of the sketch, the sampling
// probabilities and the shrink.
//
// One power step C <- M D M^T C (M an I x J unfolding or the gathered C'_n,
// D a diagonal column weight) is one fused kernel: a block takes 32 columns
// of M at a time, forms the 32 x s slab W = D M_blk^T C with the columns of
// M in registers, and then adds M_blk W into its own I x s partial sum from
// the same data (staged transposed in LDS).  M is read from HBM once per
// step, and W never leaves the block.
//
// Lane layout of v_mfma_f32_16x16x32_{bf16,fp8_fp8} (lane l = 16 g + h):
//   A (16 x 32): lane l holds A[h][8g .. 8g + 7];
//   B (32 x 16): lane l holds B[8g .. 8g + 7][h];
//   D (16 x 16): lane l, item v holds D[4g + v][h].
// The first product M_blk^T C takes both operands in the chosen format (C
// rounded once per step).  The second, M_blk W, takes M-hat as bfloat16
// (every bfloat16 and every e4m3 value is one exactly) and W as a bfloat16
// pair hi + lo = W to about 16 bits: rounding W itself would bury every
// direction whose singular value is below 2^-8 (bfloat16) or 2^-4 (e4m3)
// of the largest under the rounding error of the largest.
// FP8 operands carry scales: C per column (tau_k, from its max |entry|), the
// gathered C' per sampled column (sigma_t, folded into D) and a tensor read
// in FP8 one scale for the whole tensor (alpha, folded into D).  Values
// beyond 448 after scaling saturate to +-448; NaN stays NaN.
#pragma once

#include <type_traits>

#include "tr_kernels.hpp"
#include "tr_power.hpp"

namespace trk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr float kFp8Max = 448.0f;

struct OpBf16 {
  using stor = uint16_t;  // one element in memory
  using vec = bf16x8;     // one MFMA operand: 8 elements
  static constexpr bool kScaled = false;
  static __device__ __forceinline__ vec pack(const float (&x)[8]) {
    vec v;
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = (__bf16)x[t];  // round to nearest even
    return v;
  }
  static __device__ __forceinline__ stor cvt1(float x) {
    const __bf16 b = (__bf16)x;
    return __builtin_bit_cast(uint16_t, b);
  }
  template <int T>
  static __device__ __forceinline__ float elem(vec v) {
    return (float)v[T];
  }
  static __device__ __forceinline__ vec load8(const stor* p) {
    return *reinterpret_cast<const vec*>(p);
  }
  static __device__ __forceinline__ f32x4 mfma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

struct OpFp8 {
  using stor = uint8_t;
  using vec = long;  // element t in byte t
  static constexpr bool kScaled = true;
  static __device__ __forceinline__ float sat(float x) {
    return fabsf(x) > kFp8Max ? copysignf(kFp8Max, x) : x;
  }
  static __device__ __forceinline__ vec pack(const float (&x)[8]) {
    unsigned lo = 0, hi = 0;
    lo = __builtin_amdgcn_cvt_pk_fp8_f32(sat(x[0]), sat(x[1]), lo, false);
    lo = __builtin_amdgcn_cvt_pk_fp8_f32(sat(x[2]), sat(x[3]), lo, true);
    hi = __builtin_amdgcn_cvt_pk_fp8_f32(sat(x[4]), sat(x[5]), hi, false);
    hi = __builtin_amdgcn_cvt_pk_fp8_f32(sat(x[6]), sat(x[7]), hi, true);
    return (long)(((unsigned long)hi << 32) | lo);
  }
  static __device__ __forceinline__ stor cvt1(float x) {
    return (stor)(__builtin_amdgcn_cvt_pk_fp8_f32(sat(x), 0.0f, 0, false) & 0xffu);
  }
  template <int T>
  static __device__ __forceinline__ float elem(vec v) {
    const int w = (int)((unsigned long)v >> (T < 4 ? 0 : 32));
    return __builtin_amdgcn_cvt_f32_fp8(w, T & 3);
  }
  static __device__ __forceinline__ vec load8(const stor* p) {
    return *reinterpret_cast<const long*>(p);
  }
  static __device__ __forceinline__ f32x4 mfma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
  }
};

template <int T, int END>
struct LpFor {
  template <typename F>
  static __device__ __forceinline__ void run(F&& f) {
    f(std::integral_constant<int, T>{});
    LpFor<T + 1, END>::run(f);
  }
};
template <int END>
struct LpFor<END, END> {
  template <typename F>
  static __device__ __forceinline__ void run(F&&) {}
};

__device__ __forceinline__ float block_max_f32(float v, float* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  float m = red[0];
  for (int w = 1; w < (int)(blockDim.x / kWave); ++w) m = fmaxf(m, red[w]);
  return m;
}

// Operand form of the sketch C (I x s, float64, column-major): Cq[k][i]
// (k < SP, i < Ip, zero outside I x s) in the operand type, and tau[k], the
// scale of column k (1 for BF16).  One block of 256 threads per k < SP; Ip <= 512.
// (Column k's workgroup; the whole workgroup calls it.)
template <typename OP>
__device__ __forceinline__ void quant_y_col(const double* __restrict__ C, int64_t I, int s,
                                            int Ip, typename OP::stor* __restrict__ Cq,
                                            float* __restrict__ tau, int k, float* red) {
  float v[2];
  float mx = 0.0f;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int64_t i = threadIdx.x + kNT * u;
    v[u] = (k < s && i < I) ? (float)C[i + I * k] : 0.0f;
    mx = fmaxf(mx, fabsf(v[u]));
  }
  float sc = 1.0f;
  if (OP::kScaled) {
    mx = block_max_f32(mx, red);
    sc = mx > 0.0f ? mx / kFp8Max : 1.0f;
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = threadIdx.x + kNT * u;
    if (i < Ip) Cq[(int64_t)k * Ip + i] = OP::cvt1(v[u] / sc);
  }
  if (threadIdx.x == 0) tau[k] = sc;
}

template <typename OP>
__global__ void __launch_bounds__(kNT)
k_quant_y(const double* __restrict__ C, int64_t I, int s, int Ip,
          typename OP::stor* __restrict__ Cq, float* __restrict__ tau) {
  __shared__ float red[kNT / kWave];
  quant_y_col<OP>(C, I, s, Ip, Cq, tau, blockIdx.x, red);
}

// Gathered sample matrix in operand form: column t of Cq (rows 0 .. Ip - 1,
// zero beyond I) is column idx[t] of the unfolding of the L x I x R view X,
// divided by its scale sigma_t (FP8: max |entry| / 448; BF16: 1), and
// omega[t] = scale2[t] sigma_t^2, so that C' diag(scale2) C'^T =
// Cq diag(omega) Cq^T.  One block of 256 threads per sampled column; Ip <= 512.
template <typename Tin, typename OP>
__global__ void __launch_bounds__(kNT)
k_gather_lp(const Tin* __restrict__ X, int64_t L, int64_t I, const int64_t* __restrict__ idx,
            int Ip, const double* __restrict__ scale2, typename OP::stor* __restrict__ Cq,
            float* __restrict__ omega, const int* __restrict__ perm, int64_t Tn) {
  __shared__ float red[kNT / kWave];
  // perm: the samples in slab order, as for k_gather (the whole workgroup
  // leaves together when its place is past T)
  const int64_t t = gather_sample(perm, Tn);
  if (t < 0) return;
  const int64_t j = idx[t];
  const int64_t r = j / L, l = j - r * L;
  const Tin* col = X + l + L * I * r;
  float v[2];
  float mx = 0.0f;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int64_t i = threadIdx.x + kNT * u;
    v[u] = i < I ? (float)col[L * i] : 0.0f;
    mx = fmaxf(mx, fabsf(v[u]));
  }
  float sc = 1.0f;
  if (OP::kScaled) {
    mx = block_max_f32(mx, red);
    sc = mx > 0.0f ? mx / kFp8Max : 1.0f;
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = threadIdx.x + kNT * u;
    if (i < Ip) Cq[t * Ip + i] = OP::cvt1(v[u] / sc);
  }
  if (threadIdx.x == 0) omega[t] = (float)(scale2[t] * (double)sc * (double)sc);
}

// max |x| over n entries, as the bit pattern of a non-negative float (so an
// integer max combines the blocks in any order with the same result).  The
// caller zeroes *out.
template <typename Tin>
__global__ void __launch_bounds__(kNT)
k_maxabs(const Tin* __restrict__ X, int64_t n, unsigned* __restrict__ out) {
  float m = 0.0f;
  for (int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kNT)
    m = fmaxf(m, fabsf((float)X[e]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x % kWave) == 0) atomicMax(out, __float_as_uint(m));
}

template <typename Tin, typename OP, int MI,
          bool kStored = std::is_same<Tin, typename OP::stor>::value>
struct LpXBuf {
  // tensor form: raw values, converted after arrival
  Tin v[2][MI][8];
  float om[8];
};
template <typename Tin, typename OP, int MI>
struct LpXBuf<Tin, OP, MI, true> {
  // operand form: the loaded bytes are the MFMA operand
  typename OP::vec v[2][MI];
  float om[8];
};

// Workgroup barrier for LDS traffic only: global loads in flight stay in
// flight (the barrier of the language waits for them as well).
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Fused power step on the matrix cores.  M is the unfolding of the L x I x R
// view X (element (i, j) at X[l + L (i + ldi r)], j = l + L r, J = L R) in
// tensor form (Tin float or double: converted on load, times 1/alpha for FP8)
// or the gathered C' in operand form (Tin == OP::stor, L == 1, ldi == Ip,
// rows I .. Ip - 1 zero).  Cq, tau: the operand form of C (k_quant_y).
// omega: column weights of the operand form (ignored in tensor form, where
// every weight is 1); xmax: max |M| for the FP8 tensor form (NULL: alpha =
// 1).  Tensor form requires J < 2^32.
//   part[b][k][i] (b = block, k < 16 NKT, i < Ip = 128 MI) =
//     sum over the column blocks of b of Mhat(i, blk) W_blk(:, k),
//   W_blk = diag(omega_blk) Mhat_blk^T Chat diag(tau),
// in float32 (rows i >= I and columns k >= s hold garbage or zero).  Block:
// 4 waves; wave w owns rows [32 MI w, 32 MI (w + 1)) of both products.  The
// waves' partial slabs of W are added in LDS in wave order, so the result
// does not depend on timing.
template <typename Tin, typename OP, int MI, int NKT, bool V4 = false>
__global__ void __launch_bounds__(kPwWaves * kWave, 1)
k_pw_lp(const Tin* __restrict__ X, int64_t L, int64_t I, int64_t R, int64_t ldi,
        const typename OP::stor* __restrict__ Cq, const float* __restrict__ tau,
        const float* __restrict__ omega, const unsigned* __restrict__ xmax,
        float* __restrict__ part) {
  using vec = typename OP::vec;
  constexpr bool kStored = std::is_same<Tin, typename OP::stor>::value;
  constexpr int SP = 16 * NKT, Ip = 128 * MI, RW = 32 * MI;
  constexpr int XS = 36;  // row stride (floats) of the LDS tiles: rows stay 16-byte aligned
  extern __shared__ float lds[];
  float* xs = lds + (threadIdx.x / kWave) * RW * XS;  // this wave's rows x 32 columns
  float* wsb = lds + 4 * RW * XS;                      // [2][4 waves][SP][XS]
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int h = lane & 15, g = lane >> 4;
  const int rw0 = wid * RW;
  const int64_t J = L * R;
  float inv_alpha = 1.0f, omega0 = 1.0f;
  if (xmax) {
    const float mx = __uint_as_float(*xmax);
    if (mx > 0.0f) {
      const float a = mx / kFp8Max;
      inv_alpha = kFp8Max / mx;
      omega0 = a * a;
    }
  }
  // A operand of the first product, fixed for the whole kernel: lane (h, g)
  // holds C(rw0 + 32 m + 8 g + t, 16 kt + h), t < 8.
  vec ya[NKT][MI];
  float tk[NKT];
#pragma unroll
  for (int kt = 0; kt < NKT; ++kt) {
#pragma unroll
    for (int m = 0; m < MI; ++m)
      ya[kt][m] = OP::load8(Cq + (int64_t)(16 * kt + h) * Ip + rw0 + 32 * m + 8 * g);
    tk[kt] = tau[16 * kt + h];
  }
  f32x4 acc[2 * MI][NKT];
#pragma unroll
  for (int it = 0; it < 2 * MI; ++it)
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt) acc[it][kt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

  const int64_t ncb = (J + 31) / 32;
  int64_t cb = blockIdx.x;
  int buf = 0;
  using Buf = LpXBuf<Tin, OP, MI>;
  // loads of column block c: lane (h, g) takes columns 32 c + 16 jt + h, rows
  // rw0 + 32 m + 8 g + t (clamped to valid addresses; see the masks below)
  auto load = [&](int64_t c, Buf& B) __attribute__((always_inline)) {
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) {
      const int64_t j = 32 * c + 16 * jt + h;
      const int64_t jc = j < J ? j : J - 1;
      if constexpr (kStored) {
        const auto* colp = X + jc * ldi + rw0 + 8 * g;
#pragma unroll
        for (int m = 0; m < MI; ++m) B.v[jt][m] = OP::load8(colp + 32 * m);
      } else if constexpr (V4) {
        // L == 1, float, I and ldi multiples of 4, X 16-byte aligned: a
        // lane's 8 rows as two 16-byte loads; a group of 4 rows at or past I
        // reads rows I - 4 .. I - 1 instead (those rows of M meet zero rows
        // of C in the first product, and the second product's rows past I
        // are not used)
        static_assert(sizeof(Tin) == 4, "16-byte loads of four rows");
        const Tin* colp = X + jc * ldi;
#pragma unroll
        for (int m = 0; m < MI; ++m)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int64_t r0 = rw0 + 32 * m + 8 * g + 4 * q;
            const f32x4 v = *reinterpret_cast<const f32x4*>(colp + (r0 + 4 <= I ? r0 : I - 4));
#pragma unroll
            for (int t = 0; t < 4; ++t) B.v[jt][m][4 * q + t] = v[t];
          }
      } else {
        // 32-bit division (the host guarantees J < 2^32): no divergent
        // 64-bit path, whose branches would make every wait conservative
        const uint32_t r = (uint32_t)jc / (uint32_t)L;
        const Tin* colp = X + (jc - (int64_t)r * L) + L * ldi * (int64_t)r;
#pragma unroll
        for (int m = 0; m < MI; ++m)
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int64_t i = rw0 + 32 * m + 8 * g + t;
            B.v[jt][m][t] = colp[L * (i < I ? i : I - 1)];
          }
      }
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t j = 32 * c + 8 * g + t;
      B.om[t] = kStored ? omega[j < J ? j : J - 1] : 1.0f;
    }
  };
  auto process = [&](int64_t c, Buf& B) __attribute__((always_inline)) {
    // operands of the first product; their values (as float) go to LDS for
    // the second
    vec b1[2][MI];
#pragma unroll
    for (int jt = 0; jt < 2; ++jt)
#pragma unroll
      for (int m = 0; m < MI; ++m) {
        float f[8];
        if constexpr (kStored) {
          b1[jt][m] = B.v[jt][m];
        } else {
#pragma unroll
          for (int t = 0; t < 8; ++t) f[t] = (float)B.v[jt][m][t] * inv_alpha;
          b1[jt][m] = OP::pack(f);
        }
        // the rounded values: the same M-hat in both products
        LpFor<0, 8>::run([&](auto T) {
          f[decltype(T)::value] = OP::template elem<decltype(T)::value>(b1[jt][m]);
        });
#pragma unroll
        for (int t = 0; t < 8; ++t) xs[(32 * m + 8 * g + t) * XS + 16 * jt + h] = f[t];
      }
    // first product: this wave's rows of M_blk^T C, per 16-column tile jt
    float* wsw = wsb + (buf * 4 + wid) * SP * XS;
#pragma unroll
    for (int jt = 0; jt < 2; ++jt)
#pragma unroll
      for (int kt = 0; kt < NKT; ++kt) {
        f32x4 p = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int m = 0; m < MI; ++m) p = OP::mfma(ya[kt][m], b1[jt][m], p);
#pragma unroll
        for (int v = 0; v < 4; ++v) wsw[(16 * kt + 4 * g + v) * XS + 16 * jt + h] = p[v];
      }
    lds_barrier();
    // W_blk^T as the A operand of the second product: lane (h, g) takes
    // k = 16 kt + h and columns 8 g .. 8 g + 7 of the block, summed over the
    // four waves in order, times tau_k and the column weights, split into a
    // bfloat16 pair hi + lo (about 16 significant bits)
    bool jok[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) jok[t] = 32 * c + 8 * g + t < J;
    bf16x8 whi[NKT], wlo[NKT];
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt) {
      float w[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) w[t] = 0.0f;
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) {
        const float* src = wsb + ((buf * 4 + ww) * SP + 16 * kt + h) * XS + 8 * g;
        const f32x4 lo = *reinterpret_cast<const f32x4*>(src);
        const f32x4 hi = *reinterpret_cast<const f32x4*>(src + 4);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          w[t] += lo[t];
          w[t + 4] += hi[t];
        }
      }
      const float sk = tk[kt] * omega0;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const float x = jok[t] ? w[t] * sk * B.om[t] : 0.0f;
        const __bf16 xh = (__bf16)x;
        whi[kt][t] = xh;
        wlo[kt][t] = (__bf16)(x - (float)xh);
      }
    }
    // second product (bfloat16 operands: every M-hat value is one exactly):
    // this wave's rows i (16 per tile it) of M_blk W_blk
#pragma unroll
    for (int it = 0; it < 2 * MI; ++it) {
      const float* src = xs + (16 * it + h) * XS + 8 * g;
      const f32x4 lo = *reinterpret_cast<const f32x4*>(src);
      const f32x4 hi = *reinterpret_cast<const f32x4*>(src + 4);
      const float f[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
      const bf16x8 b2 = OpBf16::pack(f);
#pragma unroll
      for (int kt = 0; kt < NKT; ++kt) {
        acc[it][kt] = OpBf16::mfma(whi[kt], b2, acc[it][kt]);
        acc[it][kt] = OpBf16::mfma(wlo[kt], b2, acc[it][kt]);
      }
    }
    buf ^= 1;
  };
  // Column blocks blockIdx.x, + gridDim.x, ...: counted triples over three
  // register buffers (pairs over two with MI = 4), each item prefetching the
  // columns two items ahead (one) while it multiplies out its own, so that
  // two column blocks' loads are in flight behind the products (one was not
  // enough to cover the load latency with two workgroups per compute unit).
  // A counted loop keeps every
  // prefetch in the loop body (an early exit between the items would let the
  // compiler sink them behind the products); prefetches past the last block
  // read clamped, valid addresses and go unused.
  // With 512 rows (MI = 4) the third buffer would spill: two buffers there.
  const int64_t G = gridDim.x;
  const int64_t nit = cb < ncb ? (ncb - cb + G - 1) / G : 0;
  if constexpr (MI <= 2) {
    Buf xa, xb, xc;
    if (nit > 0) {
      load(cb, xa);
      load(cb + G, xb);
    }
    int64_t k = 0;
    for (; k + 3 <= nit; k += 3) {
      load(cb + 2 * G, xc);
      __builtin_amdgcn_sched_barrier(0);
      process(cb, xa);
      cb += G;
      load(cb + 2 * G, xa);
      __builtin_amdgcn_sched_barrier(0);
      process(cb, xb);
      cb += G;
      load(cb + 2 * G, xb);
      __builtin_amdgcn_sched_barrier(0);
      process(cb, xc);
      cb += G;
    }
    if (k < nit) process(cb, xa);
    if (k + 1 < nit) process(cb + G, xb);
  } else {
    Buf xa, xb;
    if (nit > 0) load(cb, xa);
    int64_t k = 0;
    for (; k + 2 <= nit; k += 2) {
      load(cb + G, xb);
      __builtin_amdgcn_sched_barrier(0);
      process(cb, xa);
      cb += G;
      load(cb + G, xa);
      __builtin_amdgcn_sched_barrier(0);
      process(cb, xb);
      cb += G;
    }
    if (k < nit) process(cb, xa);
  }
  float* out = part + (int64_t)blockIdx.x * SP * Ip;
#pragma unroll
  for (int it = 0; it < 2 * MI; ++it)
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        out[(16 * kt + 4 * g + v) * Ip + rw0 + 16 * it + h] = acc[it][kt][v];
}

// C(i, k) = sum over b (in increasing order, float64) of part[b][k][i], for
// i < I, k < s; C column-major I x s.  Block: 32 entries x 8 groups of
// blocks b (group q takes b = q, q + 8, ...); the 8 group sums are added in
// order.
// (Workgroup blk of cdiv(I s, 32); the whole workgroup calls it.)
__device__ __forceinline__ void reduce_parts_lp_blk(const float* __restrict__ part,
                                                    int64_t nparts, int64_t I, int s, int SP,
                                                    int Ip, double* __restrict__ C,
                                                    uint32_t* __restrict__ status, int64_t blk,
                                                    double (*red)[33]) {
  const int el = threadIdx.x & 31, q = threadIdx.x >> 5;
  const int64_t n = I * s;
  const int64_t e = blk * 32 + el;
  const int64_t ec = e < n ? e : n - 1;
  const int64_t i = ec % I, k = ec / I;
  const float* src = part + k * Ip + i;
  const int64_t stride = (int64_t)SP * Ip;
  double acc = 0.0;
  constexpr int B = 8;
  for (int64_t b0 = q; b0 < nparts; b0 += 8 * B) {
    float v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int64_t b = b0 + 8 * u;
      v[u] = src[(b < nparts ? b : q) * stride];
    }
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (b0 + 8 * u < nparts) acc += (double)v[u];
  }
  red[q][el] = acc;
  __syncthreads();
  if (q == 0 && e < n) {
    double s8 = red[0][el];
#pragma unroll
    for (int u = 1; u < 8; ++u) s8 += red[u][el];
    C[e] = s8;
    if (!isfinite(s8) && status) atomicOr(status, kDevNonFinite);
  }
}

static __global__ void __launch_bounds__(kNT)
k_reduce_parts_lp(const float* __restrict__ part, int64_t nparts, int64_t I, int s, int SP,
                  int Ip, double* __restrict__ C, uint32_t* __restrict__ status) {
  __shared__ double red[8][33];
  reduce_parts_lp_blk(part, nparts, I, s, SP, Ip, C, status, blockIdx.x, red);
}

// One mode's k_reduce_parts_lp (workgroups 0 .. nred - 1) and the next mode's
// k_quant_y (workgroups nred .., one per operand column) in one launch: the
// two share no buffer (the product that read the operand buffers and wrote
// the partial sums has finished).
template <typename OP>
__global__ void __launch_bounds__(kNT)
k_reduce_quant(const float* __restrict__ part, int64_t nparts, int64_t I, int s, int SP, int Ip,
               double* __restrict__ C, uint32_t* __restrict__ status, int64_t nred,
               const double* __restrict__ Y2, int64_t I2, int s2, int Ip2,
               typename OP::stor* __restrict__ Cq, float* __restrict__ tau) {
  __shared__ double rred[8][33];
  __shared__ float qred[kNT / kWave];
  if ((int64_t)blockIdx.x < nred)
    reduce_parts_lp_blk(part, nparts, I, s, SP, Ip, C, status, blockIdx.x, rred);
  else
    quant_y_col<OP>(Y2, I2, s2, Ip2, Cq, tau, (int)(blockIdx.x - nred), qred);
}

}  // namespace trk

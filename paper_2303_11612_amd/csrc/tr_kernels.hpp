// gfx950 kernels of the per-mode randomized range finder.
//
// Every kernel addresses a tensor through its mode-n 3-D view L x I x R
// (element (l, i, r) at l + L*(i + I*r); unfolding column j = l + L*r).  Two
// streaming shapes cover all modes with coalesced HBM reads:
//   * column-streaming (one thread per unfolding column, rows in increasing
//     order): for L == 1 the fibers are contiguous, so a workgroup stages a
//     chunk of rows of 256 columns through LDS (coalesced along the fiber) and
//     each thread reads its column back from LDS; for L > 1 neighbouring
//     threads own neighbouring l and read global memory directly.
//   * row-streaming (one thread per row i, columns in increasing order): for
//     L == 1 neighbouring threads read neighbouring rows directly; for L > 1 a
//     workgroup stages 32 consecutive l of 256 rows through LDS.
// Wave-uniform operands (a row of Q^T, a row of the sketch) are indexed by
// loop counters only, so they are fetched through the scalar cache.
#pragma once

#include "tr_device.hpp"

namespace trk {

constexpr int kNT = 256;            // threads of the streaming kernels
constexpr double kTwoPi = 6.283185307179586;
constexpr uint32_t kDevNonFinite = 0x1u;
constexpr uint32_t kDevZeroDist = 0x2u;

template <typename T>
struct RowsPerChunk {
  static constexpr int value = sizeof(T) == 4 ? 32 : 16;  // 128 B per fiber chunk
};

// ---------------------------------------------------------------------------
// K1  Gaussian test matrix (Alg. 1 step 2 / Alg. 4 step 5).  One thread per
// Philox block of four outputs; Box-Muller on words (0,1) and (2,3).  Writes
// G (I x s column-major) and Gt (row-major copy, row i = G(i, :)).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kNT)
k_gaussian(double* __restrict__ G, double* __restrict__ Gt, int64_t I, int64_t s,
           uint64_t mode, uint64_t seed) {
  const int64_t total = I * s;
  const int64_t b = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (4 * b >= total) return;
  const U64x4 r = philox4x64_10((uint64_t)b, mode, kTagGauss, 0, seed, 0);
#pragma unroll
  for (int pair = 0; pair < 2; ++pair) {
    const uint64_t ra = r.w[2 * pair], rb = r.w[2 * pair + 1];
    const double u1 = (double)((ra >> 11) + 1) * 0x1p-53;
    const double u2 = (double)(rb >> 11) * 0x1p-53;
    const double rho = sqrt(-2.0 * log(u1));
    const double th = kTwoPi * u2;
    const double z[2] = {rho * cos(th), rho * sin(th)};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t e = 4 * b + 2 * pair + h;
      if (e < total) {
        G[e] = z[h];
        if (Gt) {
          const int64_t i = e % I, c = e / I;
          Gt[i * s + c] = z[h];
        }
      }
    }
  }
}

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

// ---------------------------------------------------------------------------
// K3  Column norms n_j = ||A_(n)(:, j)||^2, rows summed in increasing order.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kNT)
k_colnorms_l1(const T* __restrict__ X, int64_t I, int64_t J,
              double* __restrict__ norms, unsigned long long* __restrict__ max_bits) {
  constexpr int TI = RowsPerChunk<T>::value;
  __shared__ T tile[TI][kNT + 1];
  __shared__ unsigned long long scr[kNT / kWave];
  const int c = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * kNT;
  const int ncol = (int)min((int64_t)kNT, J - j0);
  const T* base = X + j0 * I;
  double acc = 0.0;
  for (int64_t i0 = 0; i0 < I; i0 += TI) {
#pragma unroll
    for (int m = 0; m < TI; ++m) {
      const int e = c + kNT * m;
      const int cc = e / TI, ii = e % TI;
      if (cc < ncol && i0 + ii < I) tile[ii][cc] = base[(int64_t)cc * I + i0 + ii];
    }
    __syncthreads();
    const int ti = (int)min((int64_t)TI, I - i0);
    if (c < ncol)
      for (int ii = 0; ii < ti; ++ii) acc = sq_add(acc, (double)tile[ii][c]);
    __syncthreads();
  }
  if (c < ncol) norms[j0 + c] = acc;
  if (max_bits) block_max_bits(c < ncol ? acc : 0.0, max_bits, scr);
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
    for (int64_t i = 0; i < I; ++i) acc = sq_add(acc, (double)p[L * i]);
    norms[j] = acc;
  }
  if (max_bits) block_max_bits(acc, max_bits, scr);
}

// Atomic maximum of the IEEE bit patterns of v[0..n) (used when the norms are
// supplied by the caller rather than produced by the column-norm kernel).
__global__ void __launch_bounds__(kNT)
k_max_bits(const double* __restrict__ v, int64_t n, unsigned long long* __restrict__ out) {
  __shared__ unsigned long long scr[kNT / kWave];
  const int64_t j = (int64_t)blockIdx.x * kNT + threadIdx.x;
  block_max_bits(j < n ? v[j] : 0.0, out, scr);
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}

// ---------------------------------------------------------------------------
// K4  Sampler: integer weights, exact prefix sums, Philox draws.
// ---------------------------------------------------------------------------
constexpr int kScanChunk = 1024;  // elements per scan block (256 threads x 4)

__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v,
                                                            unsigned long long* scr) {
#pragma unroll
  for (int m = 1; m < kWave; m <<= 1) v += __shfl_xor(v, m, kWave);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) scr[wid] = v;
  __syncthreads();
  unsigned long long t = 0;
  for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += scr[w];
  __syncthreads();
  return t;
}

// Exclusive scan over the workgroup; returns this thread's exclusive prefix
// and the block total in *total.
__device__ __forceinline__ unsigned long long block_exscan_u64(
    unsigned long long v, unsigned long long* scr, unsigned long long* total) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  unsigned long long inc = v;
#pragma unroll
  for (int m = 1; m < kWave; m <<= 1) {
    const unsigned long long o = __shfl_up(inc, m, kWave);
    if (lane >= m) inc += o;
  }
  if (lane == kWave - 1) scr[wid] = inc;
  __syncthreads();
  unsigned long long before = 0, all = 0;
  for (int w = 0; w < nw; ++w) {
    if (w < wid) before += scr[w];
    all += scr[w];
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
}

__global__ void __launch_bounds__(kNT)
k_weights(const double* __restrict__ norms, int64_t J,
          const unsigned long long* __restrict__ max_bits, int kexp, int uniform,
          unsigned long long* __restrict__ w, unsigned long long* __restrict__ bsum,
          uint32_t* __restrict__ status) {
  __shared__ unsigned long long scr[kNT / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  double M = 0.0;
  bool bad = false;
  if (!uniform) {
    M = __longlong_as_double((long long)*max_bits);
    bad = !(M > 0.0) || !isfinite(M);
  }
  const double scale = ldexp(1.0, kexp);
  unsigned long long local = 0;
#pragma unroll
  for (int m = 0; m < kScanChunk / kNT; ++m) {
    const int64_t j = base + threadIdx.x + (int64_t)kNT * m;
    if (j < J) {
      unsigned long long wj = 1;
      if (!uniform) {
        const double n = norms[j];
        if (bad || n == 0.0) {
          wj = 0;
        } else {
          const double q = n / M;
          const double f = floor(q * scale);
          wj = (unsigned long long)f;
          if (wj < 1) wj = 1;
        }
      }
      w[j] = wj;
      local += wj;
    }
  }
  const unsigned long long t = block_sum_u64(local, scr);
  if (threadIdx.x == 0) bsum[blockIdx.x] = t;
  if (bad && status && blockIdx.x == 0 && threadIdx.x == 0)
    atomicOr(status, isfinite(M) ? kDevZeroDist : (kDevNonFinite | kDevZeroDist));
}

// In-place exclusive scan of the block sums (one workgroup of 1024 threads).
__global__ void __launch_bounds__(1024)
k_scan_bsum(unsigned long long* __restrict__ bsum, int64_t nb) {
  __shared__ unsigned long long scr[1024 / kWave];
  const int t = threadIdx.x;
  const int64_t per = (nb + 1023) / 1024;
  const int64_t a = t * per, b = min(nb, a + per);
  unsigned long long local = 0;
  for (int64_t k = a; k < b; ++k) local += bsum[k];
  unsigned long long total;
  unsigned long long run = block_exscan_u64(local, scr, &total);
  for (int64_t k = a; k < b; ++k) {
    const unsigned long long v = bsum[k];
    bsum[k] = run;
    run += v;
  }
}

// Inclusive prefix sums cdf_j = w_0 + ... + w_j.
__global__ void __launch_bounds__(kNT)
k_cdf(const unsigned long long* __restrict__ w, const unsigned long long* __restrict__ boff,
      int64_t J, unsigned long long* __restrict__ cdf) {
  __shared__ unsigned long long scr[kNT / kWave];
  constexpr int E = kScanChunk / kNT;
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * E;
  unsigned long long v[E];
  unsigned long long local = 0;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    v[m] = (base + m < J) ? w[base + m] : 0ull;
    local += v[m];
  }
  unsigned long long total;
  unsigned long long run = boff[blockIdx.x] + block_exscan_u64(local, scr, &total);
#pragma unroll
  for (int m = 0; m < E; ++m) {
    run += v[m];
    if (base + m < J) cdf[base + m] = run;
  }
}

// One thread per draw t: x = floor((h 2^64 + l) W / 2^128) exactly, then the
// first j with cdf_j > x, and the rescale sqrt((W / w_j) / T).  Also stores
// scale^2 (the column weight of C' C'^T).
__global__ void __launch_bounds__(kNT)
k_draw(const unsigned long long* __restrict__ cdf, int64_t J, int64_t T, uint64_t seed,
       uint64_t mode, int uniform, int64_t* __restrict__ idx, double* __restrict__ scale,
       double* __restrict__ scale2) {
  const int64_t t = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (t >= T) return;
  const unsigned long long W = uniform ? (unsigned long long)J : cdf[J - 1];
  const U64x4 r = philox4x64_10((uint64_t)(t / 2), mode, kTagSample, 0, seed, 0);
  const uint64_t h = r.w[2 * (t & 1)], l = r.w[2 * (t & 1) + 1];
  const uint64_t a1 = __umul64hi(W, l);
  const uint64_t b0 = W * h, b1 = __umul64hi(W, h);
  const uint64_t sum = b0 + a1;
  const uint64_t x = b1 + (sum < b0 ? 1u : 0u);
  int64_t j;
  unsigned long long wj;
  if (uniform) {
    j = (int64_t)x;
    wj = 1;
  } else if (W == 0) {
    j = 0;
    wj = 0;
  } else {
    int64_t lo = 0, hi = J - 1;
    while (lo < hi) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      if (cdf[mid] > x) hi = mid; else lo = mid + 1;
    }
    j = lo;
    wj = cdf[j] - (j > 0 ? cdf[j - 1] : 0ull);
  }
  double sc = 0.0;
  if (wj > 0) sc = sqrt(((double)W / (double)wj) / (double)T);
  idx[t] = j;
  scale[t] = sc;
  if (scale2) scale2[t] = sc * sc;
}

// ---------------------------------------------------------------------------
// K5  Gather C'(:, t) = A_(n)(:, idx[t]) (unscaled; the rescale enters the
// products as the column weight scale^2).  grid = (T, ceil(I / 256)).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kNT)
k_gather(const T* __restrict__ X, int64_t L, int64_t I, const int64_t* __restrict__ idx,
         T* __restrict__ Cp) {
  const int64_t t = blockIdx.x;
  const int64_t i = (int64_t)blockIdx.y * kNT + threadIdx.x;
  if (i >= I) return;
  const int64_t j = idx[t];
  const int64_t r = j / L, l = j - r * L;
  Cp[i + I * t] = X[l + L * (i + I * r)];
}

// ---------------------------------------------------------------------------
// K9 (and the first half of each power step)  Y = X x_n Q^T, column-streaming:
// Y(l, k, r) = colscale_j * sum_i Qt[i*mu + k] X(l, i, r), float64 accumulation.
// MU is a compile-time bound on mu (accumulators live in registers).
// ---------------------------------------------------------------------------
template <typename Tin, typename Tout, int MU>
__global__ void __launch_bounds__(kNT)
k_ttm_l1(const Tin* __restrict__ X, int64_t I, int64_t R, const double* __restrict__ Qt,
         int mu, const double* __restrict__ colscale, Tout* __restrict__ Y) {
  constexpr int TI = RowsPerChunk<Tin>::value;
  __shared__ Tin tile[TI][kNT + 1];
  const int c = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * kNT;
  const int ncol = (int)min((int64_t)kNT, R - j0);
  const Tin* base = X + j0 * I;
  double acc[MU];
#pragma unroll
  for (int k = 0; k < MU; ++k) acc[k] = 0.0;
  for (int64_t i0 = 0; i0 < I; i0 += TI) {
#pragma unroll
    for (int m = 0; m < TI; ++m) {
      const int e = c + kNT * m;
      const int cc = e / TI, ii = e % TI;
      if (cc < ncol && i0 + ii < I) tile[ii][cc] = base[(int64_t)cc * I + i0 + ii];
    }
    __syncthreads();
    const int ti = (int)min((int64_t)TI, I - i0);
    for (int ii = 0; ii < ti; ++ii) {
      const double x = (double)tile[ii][c];
      const double* q = Qt + (i0 + ii) * mu;
#pragma unroll
      for (int k = 0; k < MU; ++k)
        if (k < mu) acc[k] = fma(q[k], x, acc[k]);
    }
    __syncthreads();
  }
  if (c < ncol) {
    const int64_t j = j0 + c;
    const double d = colscale ? colscale[j] : 1.0;
#pragma unroll
    for (int k = 0; k < MU; ++k)
      if (k < mu) Y[k + (int64_t)mu * j] = (Tout)(acc[k] * d);
  }
}

template <typename Tin, typename Tout, int MU>
__global__ void __launch_bounds__(kNT)
k_ttm_ln(const Tin* __restrict__ X, int64_t L, int64_t I, int64_t R,
         const double* __restrict__ Qt, int mu, const double* __restrict__ colscale,
         Tout* __restrict__ Y) {
  const int64_t J = L * R;
  const int64_t j = (int64_t)blockIdx.x * kNT + threadIdx.x;
  const bool act = j < J;
  const int64_t jj = act ? j : 0;
  const int64_t r = jj / L, l = jj - r * L;
  const Tin* p = X + l + L * I * r;
  double acc[MU];
#pragma unroll
  for (int k = 0; k < MU; ++k) acc[k] = 0.0;
  for (int64_t i = 0; i < I; ++i) {
    const double x = act ? (double)p[L * i] : 0.0;
    const double* q = Qt + i * mu;
#pragma unroll
    for (int k = 0; k < MU; ++k)
      if (k < mu) acc[k] = fma(q[k], x, acc[k]);
  }
  if (act) {
    const double d = colscale ? colscale[j] : 1.0;
#pragma unroll
    for (int k = 0; k < MU; ++k)
      if (k < mu) Y[l + L * (k + (int64_t)mu * r)] = (Tout)(acc[k] * d);
  }
}

// ---------------------------------------------------------------------------
// Second half of a power step, row-streaming: part_b(i, k) = sum over the
// columns j of block b of X(i, j) Z(j, k), where Z is the L x s x R output of
// the first half (Z(j, k) at l + L*(k + s*r)).  Partials are reduced in a
// fixed order by k_reduce_parts, so the result is reproducible.
// ---------------------------------------------------------------------------
template <typename Tin, int SM>
__global__ void __launch_bounds__(kNT)
k_gramb_l1(const Tin* __restrict__ X, int64_t I, int64_t R, const double* __restrict__ Z,
           int s, int64_t chunk, double* __restrict__ part) {
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = min(R, r0 + chunk);
  double* out = part + (int64_t)blockIdx.x * I * s;
  for (int64_t ib = 0; ib < I; ib += kNT) {
    const int64_t i = ib + threadIdx.x;
    const bool act = i < I;
    double acc[SM];
#pragma unroll
    for (int k = 0; k < SM; ++k) acc[k] = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
      const double x = act ? (double)X[i + I * r] : 0.0;
      const double* z = Z + (int64_t)s * r;
#pragma unroll
      for (int k = 0; k < SM; ++k)
        if (k < s) acc[k] = fma(x, z[k], acc[k]);
    }
    if (act) {
#pragma unroll
      for (int k = 0; k < SM; ++k)
        if (k < s) out[i + I * k] = acc[k];
    }
  }
}

template <typename Tin, int SM>
__global__ void __launch_bounds__(kNT)
k_gramb_ln(const Tin* __restrict__ X, int64_t L, int64_t I, int64_t R,
           const double* __restrict__ Z, int s, int64_t chunk, double* __restrict__ part) {
  constexpr int TL = 32;
  __shared__ Tin tile[TL][kNT + 1];
  const int64_t J = L * R;
  const int64_t ja = (int64_t)blockIdx.x * chunk;
  const int64_t jb = min(J, ja + chunk);
  double* out = part + (int64_t)blockIdx.x * I * s;
  for (int64_t ib = 0; ib < I; ib += kNT) {
    const int64_t i = ib + threadIdx.x;
    double acc[SM];
#pragma unroll
    for (int k = 0; k < SM; ++k) acc[k] = 0.0;
    for (int64_t j = ja; j < jb;) {
      const int64_t r = j / L, l0 = j - r * L;
      const int tl = (int)min((int64_t)TL, min(L - l0, jb - j));
#pragma unroll
      for (int m = 0; m < TL; ++m) {
        const int e = threadIdx.x + kNT * m;
        const int ll = e % TL, ii = e / TL;
        if (ll < tl && ib + ii < I) tile[ll][ii] = X[l0 + ll + L * (ib + ii + I * r)];
      }
      __syncthreads();
      for (int ll = 0; ll < tl; ++ll) {
        const double x = (double)tile[ll][threadIdx.x];
        const double* z = Z + (l0 + ll) + L * (int64_t)s * r;
#pragma unroll
        for (int k = 0; k < SM; ++k)
          if (k < s) acc[k] = fma(x, z[L * k], acc[k]);
      }
      __syncthreads();
      j += tl;
    }
    if (i < I) {
#pragma unroll
      for (int k = 0; k < SM; ++k)
        if (k < s) out[i + I * k] = acc[k];
    }
  }
}

// Y(e) = sum_b part_b(e) in increasing b; also the row-major copy Yt.
__global__ void __launch_bounds__(kNT)
k_reduce_parts(const double* __restrict__ part, int64_t nparts, int64_t I, int s,
               double* __restrict__ Y, double* __restrict__ Yt, uint32_t* __restrict__ status) {
  const int64_t n = I * s;
  const int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (e >= n) return;
  double acc = 0.0;
  for (int64_t b = 0; b < nparts; ++b) acc += part[b * n + e];
  Y[e] = acc;
  const int64_t i = e % I, k = e / I;
  Yt[i * s + k] = acc;
  if (!isfinite(acc) && status) atomicOr(status, kDevNonFinite);
}

// ---------------------------------------------------------------------------
// K7 + K8  Factor of a sketch on one workgroup of 512 threads: Householder QR
// C = P R, one-sided Jacobi SVD of R (columns rotated until orthogonal), sort,
// P formed in place of the reflectors, Q = P U_R(:, 1:mu), canonical signs.
// Thread t holds rows t + 512 p (p < RPT) of C in registers; SM >= s.
// ---------------------------------------------------------------------------
constexpr int kFactorNT = 512;

template <int SM>
__device__ __forceinline__ double pick(const double (&a)[SM], int k) {
  double r = 0.0;
#pragma unroll
  for (int j = 0; j < SM; ++j) r = (j == k) ? a[j] : r;
  return r;
}

template <int SM>
__device__ __forceinline__ void put(double (&a)[SM], int k, double v) {
#pragma unroll
  for (int j = 0; j < SM; ++j) a[j] = (j == k) ? v : a[j];
}

// Workgroup sum of the vector part(j), j in [jlo, s), computed by `f(j)` per
// thread; the result lands in vec[j].  Chunks of 16 values go through the
// wave transpose-reduce.  Two barriers.
template <int SM, typename F>
__device__ __forceinline__ void block_vec_sum(F f, double* scr, double* vec) {
  constexpr int NW = kFactorNT / kWave;
  constexpr int CH = SM < 16 ? SM : 16;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
  for (int c0 = 0; c0 < SM; c0 += CH) {
    double v[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) v[q] = f(c0 + q);
    const double r = wave_vec_sum<CH>(v, lane);
    if (lane < CH) scr[wid * SM + c0 + wave_vec_index<CH>(lane)] = r;
  }
  __syncthreads();
  if (threadIdx.x < SM) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += scr[w * SM + threadIdx.x];
    vec[threadIdx.x] = t;
  }
  __syncthreads();
}

template <int RPT, int SM>
__global__ void __launch_bounds__(kFactorNT)
k_factor(const double* __restrict__ C, int I, int s, int mu, double* __restrict__ Q,
         double* __restrict__ Qt, double* __restrict__ sig_out, void* __restrict__ Qcast,
         int cast_f32, uint32_t* __restrict__ status) {
  constexpr int NT = kFactorNT, NW = NT / kWave, LD = SM + 1;
  __shared__ double s_scr[NW * SM];
  __shared__ double s_vec[SM];
  __shared__ double s_R[SM * LD];   // R, then the rotated R; column c at s_R[c*LD]
  __shared__ double s_U[SM * LD];   // leading left singular vectors of R
  __shared__ double s_tau[SM];
  __shared__ double s_sig[SM];
  __shared__ int s_perm[SM];
  __shared__ int s_flag;
  __shared__ double s_bval[NW * SM];
  __shared__ double s_babs[NW * SM];
  __shared__ int s_bidx[NW * SM];
  __shared__ double s_sign[SM];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;

  double a[RPT][SM];
#pragma unroll
  for (int p = 0; p < RPT; ++p) {
    const int i = tid + NT * p;
#pragma unroll
    for (int j = 0; j < SM; ++j) a[p][j] = (i < I && j < s) ? C[i + (int64_t)I * j] : 0.0;
  }
  for (int e = tid; e < SM * LD; e += NT) {
    s_R[e] = 0.0;
    s_U[e] = 0.0;
  }
  __syncthreads();

  // ---- Householder QR (LAPACK dgeqr2 conventions: H = I - tau v v^T) ----
  for (int k = 0; k < s; ++k) {
    double part = 0.0, al = 0.0;
#pragma unroll
    for (int p = 0; p < RPT; ++p) {
      const int i = tid + NT * p;
      const double x = pick<SM>(a[p], k);
      if (i > k && i < I) part += x * x;
      if (i == k) al = x;
    }
    block_vec_sum<2>([&](int j) { return j == 0 ? part : al; }, s_scr, s_vec);
    const double sum2 = s_vec[0], alpha = s_vec[1];
    double beta, tk, inv;
    if (sum2 == 0.0) {
      beta = alpha;
      tk = 0.0;
      inv = 0.0;
    } else {
      beta = -copysign(sqrt(alpha * alpha + sum2), alpha);
      tk = (beta - alpha) / beta;
      inv = 1.0 / (alpha - beta);
    }
    double v[RPT];
#pragma unroll
    for (int p = 0; p < RPT; ++p) {
      const int i = tid + NT * p;
      const double x = pick<SM>(a[p], k);
      v[p] = (i == k) ? 1.0 : ((i > k && i < I) ? x * inv : 0.0);
    }
    block_vec_sum<SM>(
        [&](int j) {
          double t = 0.0;
          if (j > k && j < s) {
#pragma unroll
            for (int p = 0; p < RPT; ++p) t += v[p] * a[p][j];
          }
          return t;
        },
        s_scr, s_vec);
#pragma unroll
    for (int p = 0; p < RPT; ++p) {
#pragma unroll
      for (int j = 0; j < SM; ++j)
        if (j > k && j < s) a[p][j] -= tk * v[p] * s_vec[j];
    }
#pragma unroll
    for (int p = 0; p < RPT; ++p) {
      const int i = tid + NT * p;
      if (i == k) {
        s_R[k * LD + k] = beta;
#pragma unroll
        for (int j = 0; j < SM; ++j)
          if (j > k && j < s) s_R[j * LD + k] = a[p][j];
      }
      put<SM>(a[p], k, v[p]);
    }
    if (tid == 0) s_tau[k] = tk;
  }
  __syncthreads();

  // ---- one-sided Jacobi on the columns of R (circle-method pair order) ----
  const int se = s + (s & 1);
  const int np = se / 2;
  const int G = np <= NT / 64 ? 64 : (np <= NT / 32 ? 32 : 16);
  const int g = tid / G, gl = tid % G;
  for (int sweep = 0; sweep < 40 && se > 1; ++sweep) {
    if (tid == 0) s_flag = 0;
    __syncthreads();
    for (int step = 0; step < se - 1; ++step) {
      if (g < np) {
        const int x0 = g, x1 = se - 1 - g;
        int p = (x0 == 0) ? 0 : ((x0 - 1 + step) % (se - 1)) + 1;
        int q = ((x1 - 1 + step) % (se - 1)) + 1;
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double aa = 0.0, bb = 0.0, cc = 0.0;
        for (int i = gl; i < s; i += G) {
          const double x = s_R[p * LD + i], y = s_R[q * LD + i];
          aa += x * x;
          bb += y * y;
          cc += x * y;
        }
        for (int m = 1; m < G; m <<= 1) {
          aa += __shfl_xor(aa, m, kWave);
          bb += __shfl_xor(bb, m, kWave);
          cc += __shfl_xor(cc, m, kWave);
        }
        if (cc != 0.0 && fabs(cc) > 1e-15 * sqrt(aa) * sqrt(bb)) {
          const double zeta = (bb - aa) / (2.0 * cc);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
          const double cs = 1.0 / sqrt(1.0 + t * t);
          const double sn = cs * t;
          for (int i = gl; i < s; i += G) {
            const double x = s_R[p * LD + i], y = s_R[q * LD + i];
            s_R[p * LD + i] = cs * x - sn * y;
            s_R[q * LD + i] = sn * x + cs * y;
          }
          if (gl == 0) s_flag = 1;
        }
      }
      __syncthreads();
    }
    const int more = s_flag;
    __syncthreads();
    if (!more) break;
  }

  // ---- singular values, descending order, U_R = normalised columns ----
  if (tid < s) {
    double n2 = 0.0;
    for (int i = 0; i < s; ++i) n2 += s_R[tid * LD + i] * s_R[tid * LD + i];
    s_sig[tid] = sqrt(n2);
  }
  __syncthreads();
  if (tid < s) {
    const double me = s_sig[tid];
    int rank = 0;
    for (int q = 0; q < s; ++q) {
      const double o = s_sig[q];
      if (o > me || (o == me && q < tid)) ++rank;
    }
    s_perm[rank] = tid;
    if (sig_out) sig_out[rank] = me;
    if (!isfinite(me) && status) atomicOr(status, kDevNonFinite);
  }
  __syncthreads();
  for (int e = tid; e < mu * s; e += NT) {
    const int c = e / s, i = e % s;
    const int pc = s_perm[c];
    const double sg = s_sig[pc];
    s_U[c * LD + i] = sg > 0.0 ? s_R[pc * LD + i] / sg : (i == pc ? 1.0 : 0.0);
  }
  __syncthreads();

  // ---- P = H_0 ... H_{s-1} [I_s; 0] in place of the reflectors (dorg2r) ----
  for (int k = s - 1; k >= 0; --k) {
    const double tk = s_tau[k];
    double vk[RPT];
#pragma unroll
    for (int p = 0; p < RPT; ++p) vk[p] = pick<SM>(a[p], k);
    if (k < s - 1) {
      block_vec_sum<SM>(
          [&](int j) {
            double t = 0.0;
            if (j > k && j < s) {
#pragma unroll
              for (int p = 0; p < RPT; ++p) t += vk[p] * a[p][j];
            }
            return t;
          },
          s_scr, s_vec);
#pragma unroll
      for (int p = 0; p < RPT; ++p) {
#pragma unroll
        for (int j = 0; j < SM; ++j)
          if (j > k && j < s) a[p][j] -= tk * vk[p] * s_vec[j];
      }
    }
#pragma unroll
    for (int p = 0; p < RPT; ++p) {
      const int i = tid + NT * p;
      const double nv = (i == k) ? 1.0 - tk : ((i > k) ? -tk * vk[p] : 0.0);
      put<SM>(a[p], k, nv);
    }
  }

  // ---- Q = P U_R(:, 1:mu); per column, the largest |entry| (lowest row) ----
  for (int c = 0; c < mu; ++c) {
    double best = -1.0, bval = 0.0;
    int bidx = 0x7fffffff;
#pragma unroll
    for (int p = 0; p < RPT; ++p) {
      const int i = tid + NT * p;
      double z = 0.0;
#pragma unroll
      for (int j = 0; j < SM; ++j)
        if (j < s) z += a[p][j] * s_U[c * LD + j];
      if (i < I && (fabs(z) > best)) {
        best = fabs(z);
        bval = z;
        bidx = i;
      }
    }
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) {
      const double ob = __shfl_xor(best, m, kWave);
      const double ov = __shfl_xor(bval, m, kWave);
      const int oi = __shfl_xor(bidx, m, kWave);
      if (ob > best || (ob == best && oi < bidx)) {
        best = ob;
        bval = ov;
        bidx = oi;
      }
    }
    if (lane == 0) {
      s_babs[wid * SM + c] = best;
      s_bval[wid * SM + c] = bval;
      s_bidx[wid * SM + c] = bidx;
    }
  }
  __syncthreads();
  if (tid < mu) {
    double best = -1.0, bval = 0.0;
    int bidx = 0x7fffffff;
    for (int w = 0; w < NW; ++w) {
      const double ob = s_babs[w * SM + tid];
      const int oi = s_bidx[w * SM + tid];
      if (ob > best || (ob == best && oi < bidx)) {
        best = ob;
        bval = s_bval[w * SM + tid];
        bidx = oi;
      }
    }
    s_sign[tid] = bval < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  for (int c = 0; c < mu; ++c) {
    const double sg = s_sign[c];
#pragma unroll
    for (int p = 0; p < RPT; ++p) {
      const int i = tid + NT * p;
      if (i < I) {
        double z = 0.0;
#pragma unroll
        for (int j = 0; j < SM; ++j)
          if (j < s) z += a[p][j] * s_U[c * LD + j];
        z *= sg;
        Q[i + (int64_t)I * c] = z;
        if (Qt) Qt[(int64_t)i * mu + c] = z;
        if (Qcast) {
          if (cast_f32) ((float*)Qcast)[i + (int64_t)I * c] = (float)z;
          else ((double*)Qcast)[i + (int64_t)I * c] = z;
        }
      }
    }
  }
}

// Row-major copy Qt of a column-major I x mu matrix Q.
__global__ void k_transpose(const double* __restrict__ Q, int64_t I, int64_t mu,
                            double* __restrict__ Qt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= I * mu) return;
  const int64_t i = e % I, k = e / I;
  Qt[i * mu + k] = Q[e];
}

template <typename Tout>
__global__ void k_cast(const double* __restrict__ src, int64_t n, Tout* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dst[e] = (Tout)src[e];
}

}  // namespace trk

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

#include "tr_colnorms.hpp"
#include "tr_consts.hpp"
#include "tr_device.hpp"

namespace trk {

// ---------------------------------------------------------------------------
// K1  Gaussian test matrix (Alg. 1 step 2 / Alg. 4 step 5).  One thread per
// Philox block of four outputs; Box-Muller on words (0,1) and (2,3).  Writes
// G (I x s column-major) and Gt (row-major copy, row i = G(i, :), stride
// ldgt).
// ---------------------------------------------------------------------------
// The four normals of Philox block b of a mode: entries 4b .. 4b + 3 of G.
__device__ __forceinline__ void gauss_block(uint64_t b, uint64_t mode, uint64_t seed,
                                            double (&z)[4]) {
  const U64x4 r = philox4x64_10(b, mode, kTagGauss, 0, seed, 0);
#pragma unroll
  for (int pair = 0; pair < 2; ++pair) {
    const uint64_t ra = r.w[2 * pair], rb = r.w[2 * pair + 1];
    const double u1 = (double)((ra >> 11) + 1) * 0x1p-53;
    const double u2 = (double)(rb >> 11) * 0x1p-53;
    const double rho = sqrt(-2.0 * log(u1));
    const double th = kTwoPi * u2;
    z[2 * pair] = rho * cos(th);
    z[2 * pair + 1] = rho * sin(th);
  }
}

static __global__ void __launch_bounds__(kNT)
k_gaussian(double* __restrict__ G, double* __restrict__ Gt, int64_t I, int64_t s,
           int64_t ldgt, uint64_t mode, uint64_t seed) {
  const int64_t total = I * s;
  const int64_t b = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (4 * b >= total) return;
  double z[4];
  gauss_block((uint64_t)b, mode, seed, z);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t e = 4 * b + q;
    if (e < total) {
      G[e] = z[q];
      if (Gt) {
        const int64_t i = e % I, c = e / I;
        Gt[i * ldgt + c] = z[q];
      }
    }
  }
}

// Every mode's Gaussian test matrix in one launch (the decompositions draw
// all of them up front): mode m takes threads [t0, t0 + cdiv(I s, 4)) for its
// entries, drawn exactly as k_gaussian draws them for that mode, then
// I (ldgt - s) threads that zero the padding columns of its row-major copy;
// threads 0 .. nzero - 1 also clear zero[0 .. nzero - 1].
struct GaussMode {
  double* G;
  double* Gt;
  int64_t I, s, ldgt, t0;
};
struct GaussModes {
  GaussMode m[8];
  int n;
  int nzero;
  unsigned long long* zero;
};

static __global__ void __launch_bounds__(kNT)
k_gaussian_modes(GaussModes gm, uint64_t seed) {
  const int64_t f = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (gm.zero && f < gm.nzero) gm.zero[f] = 0ull;
  int md = -1;
  for (int q = 0; q < gm.n; ++q)
    if (f >= gm.m[q].t0) md = q;
  if (md < 0) return;
  const GaussMode M = gm.m[md];
  const int64_t total = M.I * M.s, ng = (total + 3) / 4;
  const int64_t b = f - M.t0;
  if (b >= ng) {
    const int64_t pw = M.ldgt - M.s, p = b - ng;
    if (pw > 0 && p < M.I * pw) {
      const int64_t i = p / pw;
      M.Gt[i * M.ldgt + M.s + (p - i * pw)] = 0.0;
    }
    return;
  }
  double z[4];
  gauss_block((uint64_t)b, (uint64_t)md, seed, z);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t e = 4 * b + q;
    if (e < total) {
      M.G[e] = z[q];
      const int64_t i = e % M.I, c = e / M.I;
      M.Gt[i * M.ldgt + c] = z[q];
    }
  }
}

static __global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
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

// Chunk `blk` of the weights (the calling workgroup; every thread calls).
__device__ __forceinline__ void weights_block(const double* __restrict__ norms, int64_t J,
                                              const unsigned long long* __restrict__ max_bits,
                                              int kexp, int uniform,
                                              unsigned long long* __restrict__ w,
                                              unsigned long long* __restrict__ bsum,
                                              uint32_t* __restrict__ status, int64_t blk) {
  __shared__ unsigned long long scr[kNT / kWave];
  const int64_t base = blk * kScanChunk;
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
  if (threadIdx.x == 0) bsum[blk] = t;
  if (bad && status && blk == 0 && threadIdx.x == 0)
    atomicOr(status, isfinite(M) ? kDevZeroDist : (kDevNonFinite | kDevZeroDist));
}

static __global__ void __launch_bounds__(kNT)
k_weights(const double* __restrict__ norms, int64_t J,
          const unsigned long long* __restrict__ max_bits, int kexp, int uniform,
          unsigned long long* __restrict__ w, unsigned long long* __restrict__ bsum,
          uint32_t* __restrict__ status) {
  weights_block(norms, J, max_bits, kexp, uniform, w, bsum, status, blockIdx.x);
}

// In-place exclusive scan of the block sums (one workgroup of 1024 threads).
static __global__ void __launch_bounds__(1024)
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

// Inclusive prefix sums cdf_j = w_0 + ... + w_j.  boff holds each block's
// offset (the scanned block sums), or with `raw` the block sums themselves:
// block b then adds up those of blocks 0 .. b-1 itself (exact integer sums;
// used for a few blocks, where it saves the scan launch).
// Chunk `blk` of the inclusive prefix sums (the calling workgroup).
__device__ __forceinline__ void cdf_block(const unsigned long long* __restrict__ w,
                                          const unsigned long long* __restrict__ boff, int raw,
                                          int64_t J, unsigned long long* __restrict__ cdf,
                                          int64_t blk) {
  __shared__ unsigned long long scr[kNT / kWave];
  constexpr int E = kScanChunk / kNT;
  const int64_t base = blk * kScanChunk + (int64_t)threadIdx.x * E;
  unsigned long long v[E];
  unsigned long long local = 0;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    v[m] = (base + m < J) ? w[base + m] : 0ull;
    local += v[m];
  }
  unsigned long long off;
  if (raw) {
    unsigned long long part = 0;
    for (int64_t k = threadIdx.x; k < blk; k += kNT) part += boff[k];
    off = block_sum_u64(part, scr);
  } else {
    off = boff[blk];
  }
  unsigned long long total;
  unsigned long long run = off + block_exscan_u64(local, scr, &total);
#pragma unroll
  for (int m = 0; m < E; ++m) {
    run += v[m];
    if (base + m < J) cdf[base + m] = run;
  }
}

static __global__ void __launch_bounds__(kNT)
k_cdf(const unsigned long long* __restrict__ w, const unsigned long long* __restrict__ boff,
      int raw, int64_t J, unsigned long long* __restrict__ cdf) {
  cdf_block(w, boff, raw, J, cdf, blockIdx.x);
}

// One thread per draw t: x = floor((h 2^64 + l) W / 2^128) exactly, then the
// first j with cdf_j > x, and the rescale sqrt((W / w_j) / T).  Also stores
// scale^2 (the column weight of C' C'^T).
__device__ __forceinline__ void draw_one(const unsigned long long* __restrict__ cdf, int64_t J,
                                         int64_t T, uint64_t seed, uint64_t mode, int uniform,
                                         int64_t* __restrict__ idx, double* __restrict__ scale,
                                         double* __restrict__ scale2, int64_t t) {
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
    // the first j with cdf_j > x lies in [lo, hi] (cdf_{J-1} = W > x).  An
    // 8-ary step probes seven positions with independent loads (one round
    // trip instead of three dependent ones of a binary step): if c probes
    // have cdf <= x, j lies between probe c and probe c + 1.
    int64_t lo = 0, hi = J - 1;
    while (hi - lo >= 8) {
      const int64_t len = hi - lo + 1;
      unsigned long long v[7];
#pragma unroll
      for (int k = 0; k < 7; ++k) v[k] = cdf[lo + len * (k + 1) / 8];
      int c = 0;
#pragma unroll
      for (int k = 0; k < 7; ++k) c += v[k] <= x ? 1 : 0;
      const int64_t nlo = c == 0 ? lo : lo + len * c / 8 + 1;
      hi = c == 7 ? hi : lo + len * (c + 1) / 8;
      lo = nlo;
    }
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
  if (scale) scale[t] = sc;
  if (scale2) scale2[t] = sc * sc;
}

static __global__ void __launch_bounds__(kNT)
k_draw(const unsigned long long* __restrict__ cdf, int64_t J, int64_t T, uint64_t seed,
       uint64_t mode, int uniform, int64_t* __restrict__ idx, double* __restrict__ scale,
       double* __restrict__ scale2) {
  const int64_t t = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (t < T) draw_one(cdf, J, T, seed, mode, uniform, idx, scale, scale2, t);
}

// The nearly-optimal sampler of a mode with J <= kSmallSampleJ columns in one
// launch: every workgroup computes the integer weights of k_weights and their
// inclusive prefix sums (thread t sums a contiguous chunk, then one block
// scan) into LDS -- workgroup 0 also writes them to w and cdf -- and then
// draws t = 256 b + thread as k_draw does, searching the LDS copy.  The same
// integers, hence the same indices and scales, as the three launches it
// replaces (grid: ceil(T / 256)).
constexpr int kSmallSampleJ = 6144;
static __global__ void __launch_bounds__(kNT)
k_sample_small(const double* __restrict__ norms, int64_t J,
               const unsigned long long* __restrict__ max_bits, int kexp, int64_t T,
               uint64_t seed, uint64_t mode, unsigned long long* __restrict__ w,
               unsigned long long* __restrict__ cdf, int64_t* __restrict__ idx,
               double* __restrict__ scale, double* __restrict__ scale2,
               uint32_t* __restrict__ status) {
  __shared__ unsigned long long cl[kSmallSampleJ];
  __shared__ unsigned long long scr[kNT / kWave];
  const double M = __longlong_as_double((long long)*max_bits);
  const bool bad = !(M > 0.0) || !isfinite(M);
  const double sc = ldexp(1.0, kexp);
  const int Ji = (int)J;
  const int E = (Ji + kNT - 1) / kNT;
  const int a = min(Ji, (int)threadIdx.x * E), b = min(Ji, a + E);
  unsigned long long local = 0;
  for (int j = a; j < b; ++j) {
    unsigned long long wj = 0;
    const double n = norms[j];
    if (!bad && n != 0.0) {
      wj = (unsigned long long)floor((n / M) * sc);
      if (wj < 1) wj = 1;
    }
    if (blockIdx.x == 0) w[j] = wj;
    cl[j] = wj;
    local += wj;
  }
  unsigned long long total;
  unsigned long long run = block_exscan_u64(local, scr, &total);
  for (int j = a; j < b; ++j) {
    run += cl[j];
    cl[j] = run;
    if (blockIdx.x == 0) cdf[j] = run;
  }
  if (bad && status && blockIdx.x == 0 && threadIdx.x == 0)
    atomicOr(status, isfinite(M) ? kDevZeroDist : (kDevNonFinite | kDevZeroDist));
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (t < T) draw_one(cl, J, T, seed, mode, 0, idx, scale, scale2, t);
}

// ---------------------------------------------------------------------------
// K5  Gather C'(:, t) = A_(n)(:, idx[t]) (unscaled; the rescale enters the
// products as the column weight scale^2).  grid = (T, ceil(I / 256)).
// ---------------------------------------------------------------------------
// perm (optional): the samples in slab order (k_bucket_samples); workgroup b
// then copies sample perm[(b mod 8) ceil(T/8) + b / 8], so that the samples
// of a slab, whose elements share lines, run on one XCD (workgroups go to the
// eight XCDs in turn) and meet those lines in its L2 (grid: 8 ceil(T/8)).
__device__ __forceinline__ int64_t gather_sample(const int* __restrict__ perm, int64_t Tn) {
  if (!perm) return blockIdx.x;
  const int64_t pos = (int64_t)(blockIdx.x % 8) * ((Tn + 7) / 8) + blockIdx.x / 8;
  return pos < Tn ? perm[pos] : -1;
}

template <typename T>
__global__ void __launch_bounds__(kNT)
k_gather(const T* __restrict__ X, int64_t L, int64_t I, const int64_t* __restrict__ idx,
         T* __restrict__ Cp, const int* __restrict__ perm, int64_t Tn) {
  const int64_t t = gather_sample(perm, Tn);
  if (t < 0) return;
  const int64_t i = (int64_t)blockIdx.y * kNT + threadIdx.x;
  if (i >= I) return;
  const int64_t j = idx[t];
  const int64_t r = j / L, l = j - r * L;
  Cp[i + I * t] = X[l + L * (i + I * r)];
}

// The samples of an L x I x R view in slab order (slab r = columns
// l + L r): perm lists the sample indices t slab by slab, in any order within
// a slab (a counting sort: bin counts, their exclusive scan, then each sample
// takes the next place of its bin).  One workgroup of 1024 threads; R <=
// kBucketR, T <= kBucketT, L R < 2^32; every idx in [0, L R).
constexpr int kBucketR = 8192, kBucketT = 16384;
static __global__ void __launch_bounds__(1024)
k_bucket_samples(const int64_t* __restrict__ idx, int64_t Tn, int64_t L, int64_t R,
                 int* __restrict__ perm) {
  constexpr int PT = kBucketT / 1024;  // samples per thread, their slabs kept in registers
  __shared__ int cnt[kBucketR];
  __shared__ unsigned long long scr[1024 / kWave];
  const int Ri = (int)R;
  for (int b = threadIdx.x; b < Ri; b += 1024) cnt[b] = 0;
  int rs[PT];
#pragma unroll
  for (int m = 0; m < PT; ++m) {
    const int64_t t = threadIdx.x + 1024 * m;
    // L R < 2^32 (host): a 32-bit division
    rs[m] = t < Tn ? (int)((uint32_t)idx[t] / (uint32_t)L) : -1;
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < PT; ++m)
    if (rs[m] >= 0) atomicAdd(&cnt[rs[m]], 1);
  __syncthreads();
  const int per = (Ri + 1023) / 1024;
  const int a = min(Ri, (int)threadIdx.x * per), b = min(Ri, a + per);
  unsigned long long local = 0;
  for (int k = a; k < b; ++k) local += (unsigned)cnt[k];
  unsigned long long total;
  unsigned long long run = block_exscan_u64(local, scr, &total);
  for (int k = a; k < b; ++k) {
    const int c = cnt[k];
    cnt[k] = (int)run;
    run += (unsigned)c;
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < PT; ++m)
    if (rs[m] >= 0) perm[atomicAdd(&cnt[rs[m]], 1)] = (int)threadIdx.x + 1024 * m;
}

// ---------------------------------------------------------------------------
// K9 (and the first half of a power step on an L > 1 view)  Y = X x_n Q^T,
// column-streaming: Y(l, k, r) = colscale_j * sum_i Qt[i*MU + k] X(l, i, r),
// float64 accumulation.  Qt rows are padded to the compile-time stride MU with
// zeros, so each row is one batched scalar load and the inner loop has no
// branches.  Outputs k < kout are written with row stride kout (kout = mu for
// a mode product; kout = MU keeps the zero padding for the power steps).
// ---------------------------------------------------------------------------
// Columns [256 blk, 256 blk + 256) by the calling workgroup (tile: its LDS).
template <typename Tin, int MU, typename Tout = double>
__device__ __forceinline__ void ttm_l1_block(const Tin* __restrict__ X, int64_t I, int64_t R,
                                             const double* __restrict__ Qt, int kout,
                                             const double* __restrict__ colscale,
                                             Tout* __restrict__ Y, int64_t blk,
                                             Tin (*tile)[kNT + 1]) {
  constexpr int TI = RowsPerChunk<Tin>::value;
  const int c = threadIdx.x;
  const int64_t j0 = blk * kNT;
  const int ncol = (int)min((int64_t)kNT, R - j0);
  const Tin* base = X + j0 * I;
  double acc[MU];
#pragma unroll
  for (int k = 0; k < MU; ++k) acc[k] = 0.0;
  for (int64_t i0 = 0; i0 < I; i0 += TI) {
    stage_fiber_chunk<Tin, TI>(base, I, i0, ncol, tile);
    __syncthreads();
    const int ti = (int)min((int64_t)TI, I - i0);
    for (int ii = 0; ii < ti; ++ii) {
      const double x = (double)tile[ii][c];
      const double* q = Qt + (i0 + ii) * MU;
#pragma unroll
      for (int k = 0; k < MU; ++k) acc[k] = fma(q[k], x, acc[k]);
    }
    __syncthreads();
  }
  if (c < ncol) {
    const int64_t j = j0 + c;
    const double d = colscale ? colscale[j] : 1.0;
#pragma unroll
    for (int k = 0; k < MU; ++k)
      if (k < kout) Y[k + (int64_t)kout * j] = (Tout)(acc[k] * d);
  }
}

template <typename Tin, int MU>
__global__ void __launch_bounds__(kNT)
k_ttm_l1(const Tin* __restrict__ X, int64_t I, int64_t R, const double* __restrict__ Qt,
         int kout, const double* __restrict__ colscale, double* __restrict__ Y) {
  __shared__ Tin tile[RowsPerChunk<Tin>::value][kNT + 1];
  ttm_l1_block<Tin, MU>(X, I, R, Qt, kout, colscale, Y, blockIdx.x, tile);
}

template <typename Tin, int MU>
__global__ void __launch_bounds__(kNT)
k_ttm_ln(const Tin* __restrict__ X, int64_t L, int64_t I, int64_t R,
         const double* __restrict__ Qt, int kout, const double* __restrict__ colscale,
         double* __restrict__ Y) {
  const int64_t J = L * R;
  const int64_t j = (int64_t)blockIdx.x * kNT + threadIdx.x;
  const bool act = j < J;
  const int64_t jj = act ? j : 0;
  const int64_t r = jj / L, l = jj - r * L;
  const Tin* p = X + l + L * I * r;
  double acc[MU];
#pragma unroll
  for (int k = 0; k < MU; ++k) acc[k] = 0.0;
  constexpr int B = 8;  // loads in flight per thread
  for (int64_t i0 = 0; i0 < I; i0 += B) {
    Tin v[B];
#pragma unroll
    for (int b = 0; b < B; ++b) v[b] = p[L * min(i0 + b, I - 1)];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      if (i0 + b < I) {
        const double x = act ? (double)v[b] : 0.0;
        const double* q = Qt + (i0 + b) * MU;
#pragma unroll
        for (int k = 0; k < MU; ++k) acc[k] = fma(q[k], x, acc[k]);
      }
    }
  }
  if (act) {
    const double d = colscale ? colscale[j] : 1.0;
#pragma unroll
    for (int k = 0; k < MU; ++k)
      if (k < kout) Y[l + L * (k + (int64_t)kout * r)] = acc[k] * d;
  }
}

// Y = X x_n Q^T for a view with few columns (one launch): S threads per
// column each take a contiguous segment of ceil(I/S) rows (MU accumulators,
// rows in increasing order), and the segment sums are added in segment order
// in LDS; colscale (optional) multiplies column j's outputs.  Qt is row-major
// with row stride MU.  Yc (optional): a second copy of Y in float32 (yc_f32)
// or float64 (the caller's core, written by the last shrink).
template <typename Tin, int MU, int S>
__global__ void __launch_bounds__(kNT)
k_ttm_seg(const Tin* __restrict__ X, int64_t L, int64_t I, int64_t R,
          const double* __restrict__ Qt, int kout, const double* __restrict__ colscale,
          double* __restrict__ Y, void* __restrict__ Yc, int yc_f32) {
  constexpr int CPB = kNT / S;  // columns per workgroup
  __shared__ double part[S][CPB][MU];
  const int cl = threadIdx.x % CPB, sg = threadIdx.x / CPB;
  const int64_t J = L * R;
  const int64_t j = (int64_t)blockIdx.x * CPB + cl;
  const bool act = j < J;
  const int64_t jj = act ? j : 0;
  const int64_t r = jj / L, l = jj - r * L;
  const Tin* p = X + l + L * I * r;
  const int64_t seg = (I + S - 1) / S;
  const int64_t ia = sg * seg, ib = min(I, ia + seg);
  double acc[MU];
#pragma unroll
  for (int k = 0; k < MU; ++k) acc[k] = 0.0;
  constexpr int B = 8;
  for (int64_t i0 = ia; i0 < ib; i0 += B) {
    Tin v[B];
#pragma unroll
    for (int b = 0; b < B; ++b) v[b] = p[L * min(i0 + b, ib - 1)];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      if (i0 + b < ib) {
        const double x = act ? (double)v[b] : 0.0;
        const double* q = Qt + (i0 + b) * MU;
#pragma unroll
        for (int k = 0; k < MU; ++k) acc[k] = fma(q[k], x, acc[k]);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < MU; ++k) part[sg][cl][k] = acc[k];
  __syncthreads();
  for (int e = threadIdx.x; e < CPB * kout; e += kNT) {
    const int c = e / kout, k = e - c * kout;
    const int64_t jc = (int64_t)blockIdx.x * CPB + c;
    if (jc < J) {
      double t = part[0][c][k];
#pragma unroll
      for (int g = 1; g < S; ++g) t += part[g][c][k];
      if (colscale) t *= colscale[jc];
      const int64_t rc = jc / L, lc = jc - rc * L;
      const int64_t o = lc + L * (k + (int64_t)kout * rc);
      Y[o] = t;
      if (Yc) {
        if (yc_f32) static_cast<float*>(Yc)[o] = (float)t;
        else static_cast<double*>(Yc)[o] = t;
      }
    }
  }
}

// Mode product for views with few columns: block (x, y) covers kNT columns
// and the rows [y*ich, (y+1)*ich); partial sums over its rows go to
// part[y][j*MU + k] and are added in increasing y by k_sum_splits.
template <typename Tin, int MU>
__global__ void __launch_bounds__(kNT)
k_ttm_split(const Tin* __restrict__ X, int64_t L, int64_t I, int64_t R,
            const double* __restrict__ Qt, int64_t ich, double* __restrict__ part) {
  const int64_t J = L * R;
  const int64_t j = (int64_t)blockIdx.x * kNT + threadIdx.x;
  const bool act = j < J;
  const int64_t jj = act ? j : 0;
  const int64_t r = jj / L, l = jj - r * L;
  const Tin* p = X + l + L * I * r;
  const int64_t ia = (int64_t)blockIdx.y * ich, ib = min(I, ia + ich);
  double acc[MU];
#pragma unroll
  for (int k = 0; k < MU; ++k) acc[k] = 0.0;
  constexpr int B = 8;
  for (int64_t i0 = ia; i0 < ib; i0 += B) {
    Tin v[B];
#pragma unroll
    for (int b = 0; b < B; ++b) v[b] = p[L * min(i0 + b, ib - 1)];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      if (i0 + b < ib) {
        const double x = act ? (double)v[b] : 0.0;
        const double* q = Qt + (i0 + b) * MU;
#pragma unroll
        for (int k = 0; k < MU; ++k) acc[k] = fma(q[k], x, acc[k]);
      }
    }
  }
  if (act) {
    double* out = part + ((int64_t)blockIdx.y * J + j) * MU;
#pragma unroll
    for (int k = 0; k < MU; ++k) out[k] = acc[k];
  }
}

// Y(l, k, r) = colscale_j * sum_y part[y][j*MU + k] for k < kout, row stride kout.
static __global__ void __launch_bounds__(kNT)
k_sum_splits(const double* __restrict__ part, int64_t nsplit, int64_t L, int64_t R, int MU,
             int kout, const double* __restrict__ colscale, double* __restrict__ Y) {
  const int64_t J = L * R;
  const int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (e >= J * kout) return;
  const int64_t j = e / kout, k = e - j * kout;
  double acc = 0.0;
  constexpr int B = 8;
  for (int64_t y0 = 0; y0 < nsplit; y0 += B) {
    double v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) v[u] = part[(min(y0 + u, nsplit - 1) * J + j) * MU + k];
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (y0 + u < nsplit) acc += v[u];
  }
  if (colscale) acc *= colscale[j];
  const int64_t r = j / L, l = j - r * L;
  Y[l + L * (k + (int64_t)kout * r)] = acc;
}

// Y(e) = sum_b part_b(e) in increasing b; also the row-major copy Yt (stride
// ldyt >= s; its padding columns are left untouched, i.e. zero).
static __global__ void __launch_bounds__(kNT)
k_reduce_parts(const double* __restrict__ part, int64_t nparts, int64_t I, int s, int ldyt,
               double* __restrict__ Y, double* __restrict__ Yt, uint32_t* __restrict__ status) {
  const int64_t n = I * s;
  const int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (e >= n) return;
  double acc = 0.0;
  constexpr int B = 16;  // loads in flight; the sum stays in increasing b
  for (int64_t b0 = 0; b0 < nparts; b0 += B) {
    double v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) v[u] = part[min(b0 + u, nparts - 1) * n + e];
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (b0 + u < nparts) acc += v[u];
  }
  Y[e] = acc;
  const int64_t i = e % I, k = e / I;
  Yt[i * ldyt + k] = acc;
  if (!isfinite(acc) && status) atomicOr(status, kDevNonFinite);
}

static __global__ void k_fill_f64(double* __restrict__ p, int64_t n, double v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}

// Row-major copy Qt (row stride ldqt >= mu, padding zero) of a column-major
// I x mu matrix Q.
static __global__ void k_transpose(const double* __restrict__ Q, int64_t I, int64_t mu, int64_t ldqt,
                            double* __restrict__ Qt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= I * ldqt) return;
  const int64_t i = e / ldqt, k = e % ldqt;
  Qt[e] = k < mu ? Q[i + I * k] : 0.0;
}

template <typename Tout>
__global__ void k_cast(const double* __restrict__ src, int64_t n, Tout* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dst[e] = (Tout)src[e];
}

}  // namespace trk

// Grouped kernels of the batched ST-HOSVD driver (tucker_rand_sthosvd_batch):
// one launch runs one stage of the range finder (Alg. 5) for every request of
// a batch.  Each request's mode is described by a BMode in device memory; a
// grouped launch gives request r the blocks [start[r], start[r + 1]), so
// every block works for exactly one request and every request's arithmetic
// is the same whatever else is in the batch (results are bitwise independent
// of the batch's composition).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "tr_kernels.hpp"

namespace trk {

// One request's view of mode n and its buffers.
struct BMode {
  const void* X;       // the mode's tensor: the caller's (first mode) or float64
  int64_t L, I, R, J;  // its mode-n view L x I x R, J = L R columns
  int64_t T;           // draws of the sampled product (sampled modes)
  int64_t Tp;          // columns of the power matrix: T, or J when T > J
  int s, mu, ldq;      // sketch width, rank, row stride of Q^T
  int sampled;         // 1: draw T columns; 0: every column once, weight 1
  int nearly;          // nearly-optimal probabilities (else uniform)
  int kexp;            // 60 - ceil(log2 J)
  int64_t nchunk;      // ceil(J / kScanChunk)
  int q;               // power steps
  int mode;            // n (Philox counter word)
  uint64_t seed;
  double* norms;
  unsigned long long* maxb;
  unsigned long long* w;
  unsigned long long* cdf;
  unsigned long long* bsum;
  int64_t* idx;
  double* scale2;      // column weights of C' C'^T
  double* Cp;          // I x Tp float64: the gathered columns
  double* G;           // I x s Gaussian start
  double* Y;           // I x s sketch
  double* W;           // Tp x s
  double* Qt;          // I x ldq row-major Q^T (the factor's output)
  double* out;         // float64 shrink output (modes before the last)
  void* core;          // the caller's core (last mode)
  uint32_t* status;
};

// The request owning block b of a grouped launch (start[0] = 0, nondecreasing;
// the batch is small, so a linear walk).
__device__ __forceinline__ int breq(const int64_t* __restrict__ start, int nreq, int64_t b) {
  int r = 0;
  while (r + 1 < nreq && start[r + 1] <= b) ++r;
  return r;
}

// Gaussian starts of every (request, mode): job q owns Philox blocks
// [t0_q, t0_q + ceil(I s / 4)) of the flat thread index; the same counters as
// k_gaussian, so G_n is the one a lone decomposition draws.  The first thread
// of a job also clears that mode's running maximum of the column norms.
struct BGauss {
  double* G;
  int64_t I, s, t0;
  int mode;
  uint64_t seed;
  unsigned long long* maxb;
};

static __global__ void __launch_bounds__(kNT)
kb_gauss(const BGauss* __restrict__ jobs, int njob) {
  const int64_t f = (int64_t)blockIdx.x * kNT + threadIdx.x;
  int lo = 0, hi = njob - 1;  // last job with t0 <= f
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].t0 <= f) lo = mid; else hi = mid - 1;
  }
  const BGauss jb = jobs[lo];
  const int64_t b = f - jb.t0;
  const int64_t total = jb.I * jb.s;
  if (b < 0 || b >= (total + 3) / 4) return;
  if (b == 0 && jb.maxb) *jb.maxb = 0ull;
  double z[4];
  gauss_block((uint64_t)b, (uint64_t)jb.mode, jb.seed, z);
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (4 * b + u < total) jb.G[4 * b + u] = z[u];
}

// Squared column norms, one thread per column, rows in increasing order (the
// order that defines them), and the running maximum of their bit patterns.
template <typename Tin>
__global__ void __launch_bounds__(kNT)
kb_colnorms(const BMode* __restrict__ md, const int64_t* __restrict__ start, int nreq) {
  __shared__ unsigned long long scr[kNT / kWave];
  const int r = breq(start, nreq, blockIdx.x);
  const BMode& d = md[r];
  const int64_t j = (blockIdx.x - start[r]) * kNT + threadIdx.x;
  const bool ok = j < d.J;
  double acc = 0.0;
  if (ok) {
    const Tin* X = static_cast<const Tin*>(d.X);
    const int64_t rr = j / d.L, l = j - rr * d.L;
    const Tin* col = X + l + d.L * d.I * rr;
    for (int64_t i = 0; i < d.I; ++i) acc = sq_add(acc, (double)col[d.L * i]);
    d.norms[j] = acc;
  }
  block_max_bits(ok ? acc : 0.0, d.maxb, scr);
}

// Integer weights and their chunk totals, chunk by chunk (nearly-optimal).
static __global__ void __launch_bounds__(kNT)
kb_weights(const BMode* __restrict__ md, const int64_t* __restrict__ start, int nreq) {
  const int r = breq(start, nreq, blockIdx.x);
  const BMode& d = md[r];
  weights_block(d.norms, d.J, d.maxb, d.kexp, 0, d.w, d.bsum, d.status,
                (int64_t)blockIdx.x - start[r]);
}

// Inclusive prefix sums: each chunk adds the chunk totals before it.
static __global__ void __launch_bounds__(kNT)
kb_cdf(const BMode* __restrict__ md, const int64_t* __restrict__ start, int nreq) {
  const int r = breq(start, nreq, blockIdx.x);
  const BMode& d = md[r];
  cdf_block(d.w, d.bsum, 1, d.J, d.cdf, (int64_t)blockIdx.x - start[r]);
}

// The columns of the power matrix: Philox draws with binary search and
// rescale (sampled modes), or every column once with weight 1 (exact modes).
static __global__ void __launch_bounds__(kNT)
kb_draw(const BMode* __restrict__ md, const int64_t* __restrict__ start, int nreq) {
  const int r = breq(start, nreq, blockIdx.x);
  const BMode& d = md[r];
  const int64_t t = (blockIdx.x - start[r]) * kNT + threadIdx.x;
  if (t >= d.Tp) return;
  if (d.sampled) {
    draw_one(d.cdf, d.J, d.T, d.seed, (uint64_t)d.mode, d.nearly ? 0 : 1, d.idx, nullptr,
             d.scale2, t);
  } else {
    d.idx[t] = t;
    d.scale2[t] = 1.0;
  }
}

// Cp(:, t) = A_(n)(:, idx[t]) widened to float64: block (t, row chunk) of a
// request owns rows [256 c, 256 c + 256) of column t.
template <typename Tin>
__global__ void __launch_bounds__(kNT)
kb_gather(const BMode* __restrict__ md, const int64_t* __restrict__ start, int nreq) {
  const int r = breq(start, nreq, blockIdx.x);
  const BMode& d = md[r];
  const int64_t rc = (d.I + kNT - 1) / kNT;
  const int64_t lb = blockIdx.x - start[r];
  const int64_t t = lb / rc, i = (lb - t * rc) * kNT + threadIdx.x;
  if (i >= d.I) return;
  const int64_t j = d.idx[t];
  const int64_t rr = j / d.L, l = j - rr * d.L;
  d.Cp[i + d.I * t] = (double)static_cast<const Tin*>(d.X)[l + d.L * (i + d.I * rr)];
}

// The power products C = (Cp D Cp^T)^q G of one request on one workgroup
// (Strategy A: W = D Cp^T Y, then Y = Cp W), every sum in increasing index
// order; the power matrices of a batch are small (Tp <= 8192 columns).
static __global__ void __launch_bounds__(kNT)
kb_power(const BMode* __restrict__ md) {
  const BMode& d = md[blockIdx.x];
  const int64_t I = d.I, Tp = d.Tp, s = d.s;
  for (int64_t e = threadIdx.x; e < I * s; e += kNT) d.Y[e] = d.G[e];
  __syncthreads();
  for (int step = 0; step < d.q; ++step) {
    for (int64_t e = threadIdx.x; e < Tp * s; e += kNT) {
      const int64_t t = e % Tp, k = e / Tp;
      const double* c = d.Cp + I * t;
      const double* y = d.Y + I * k;
      double acc = 0.0;
      for (int64_t i = 0; i < I; ++i) acc = fma(c[i], y[i], acc);
      d.W[e] = acc * d.scale2[t];
    }
    __syncthreads();
    for (int64_t e = threadIdx.x; e < I * s; e += kNT) {
      const int64_t i = e % I, k = e / I;
      const double* wk = d.W + Tp * k;
      double acc = 0.0;
      for (int64_t t = 0; t < Tp; ++t) acc = fma(d.Cp[i + I * t], wk[t], acc);
      d.Y[e] = acc;
      if (!isfinite(acc) && d.status) atomicOr(d.status, kDevNonFinite);
    }
    __syncthreads();
  }
}

// The shrink Y = X x_n Q_n^T, one thread per column of the mode-n view (rows
// in increasing order), into the float64 intermediate or, for the last mode,
// the caller's core (Tout).
template <typename Tin, typename Tout, int MU>
__global__ void __launch_bounds__(kNT)
kb_shrink(const BMode* __restrict__ md, const int64_t* __restrict__ start, int nreq, int last) {
  const int r = breq(start, nreq, blockIdx.x);
  const BMode& d = md[r];
  const int64_t j = (blockIdx.x - start[r]) * kNT + threadIdx.x;
  if (j >= d.J) return;
  const Tin* X = static_cast<const Tin*>(d.X);
  const int64_t rr = j / d.L, l = j - rr * d.L;
  const Tin* col = X + l + d.L * d.I * rr;
  double acc[MU];
#pragma unroll
  for (int k = 0; k < MU; ++k) acc[k] = 0.0;
  for (int64_t i = 0; i < d.I; ++i) {
    const double x = (double)col[d.L * i];
    const double* qr = d.Qt + i * d.ldq;
#pragma unroll
    for (int k = 0; k < MU; ++k)
      if (k < d.mu) acc[k] = fma(qr[k], x, acc[k]);
  }
  const int64_t base = l + d.L * d.mu * rr;  // (l, k, r) of the L x mu x R output
#pragma unroll
  for (int k = 0; k < MU; ++k) {
    if (k >= d.mu) break;
    if (last) static_cast<Tout*>(d.core)[base + d.L * k] = (Tout)acc[k];
    else d.out[base + d.L * k] = acc[k];
  }
}

}  // namespace trk

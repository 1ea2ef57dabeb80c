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

#include "tr_colnorms.hpp"
#include "tr_kernels.hpp"
#include "tr_power.hpp"

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

// The request owning block b of a grouped launch (start[0] = 0, nondecreasing,
// start[nreq] > b; a request with no blocks has start[r] == start[r + 1]):
// the largest r with start[r] <= b, i.e. the number of r in [1, nreq) with
// start[r] <= b, counted by the whole wave (one load per lane and a ballot
// per 64 requests).  Every lane of the wave calls it with the same b.
__device__ __forceinline__ int breq(const int64_t* __restrict__ start, int nreq, int64_t b) {
  const int lane = threadIdx.x & (kWave - 1);
  int cnt = 0;
  for (int base = 1; base < nreq; base += kWave) {
    const int rr = base + lane;
    cnt += __popcll(__ballot(rr < nreq && start[rr] <= b));
  }
  return cnt;
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

// The same norms for the first mode (L = 1, contiguous columns): 256 columns
// per workgroup staged through LDS so the loads are coalesced, each column's
// rows still summed in increasing order (the same values).
template <typename Tin>
__global__ void __launch_bounds__(kNT)
kb_colnorms_l1(const BMode* __restrict__ md, const int64_t* __restrict__ start, int nreq) {
  __shared__ Tin tile[RowsPerChunk<Tin>::value][kNT + 1];
  __shared__ unsigned long long scr[kNT / kWave];
  const int r = breq(start, nreq, blockIdx.x);
  const BMode& d = md[r];
  const Tin* X = static_cast<const Tin*>(d.X);
  const int64_t blk = blockIdx.x - start[r];
  if (d.I % Vec16<Tin>::W == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0)
    colnorms_l1_block<Tin, true>(X, d.I, d.J, d.norms, d.maxb, blk, tile, scr);
  else
    colnorms_l1_block<Tin, false>(X, d.I, d.J, d.norms, d.maxb, blk, tile, scr);
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

// One power step (Strategy A) of C = (Cp D Cp^T)^q G, in two grouped launches:
//   kb_pw_w: W(t, k) = D_t sum_i Cp(i, t) Y(i, k), one wave per column t of Cp,
//            lanes over rows (each lane's rows in increasing order, then a
//            fixed butterfly over the lanes), Y = G in the first step;
//   kb_pw_y: Y(i, k) = sum_t Cp(i, t) W(t, k), one thread per entry, t in
//            increasing order.
// A request with fewer power steps than the batch's most skips the rest.
constexpr int kPwCols = kNT / kWave;  // columns t per kb_pw_w workgroup

template <int SM>
__global__ void __launch_bounds__(kNT)
kb_pw_w(const BMode* __restrict__ md, const int64_t* __restrict__ start, int nreq, int step) {
  const int r = breq(start, nreq, blockIdx.x);
  const BMode& d = md[r];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int64_t t = (blockIdx.x - start[r]) * kPwCols + wv;
  if (step >= d.q || t >= d.Tp) return;  // wave-uniform, no barrier follows
  const int64_t I = d.I;
  const int s = d.s;
  const double* __restrict__ Yin = step == 0 ? d.G : d.Y;
  const double* __restrict__ c = d.Cp + I * t;
  double acc[SM];
#pragma unroll
  for (int k = 0; k < SM; ++k) acc[k] = 0.0;
  for (int64_t i = lane; i < I; i += kWave) {
    const double ci = c[i];
#pragma unroll
    for (int k = 0; k < SM; ++k)
      if (k < s) acc[k] = fma(ci, Yin[i + I * k], acc[k]);
  }
  const double w = d.scale2[t];
#pragma unroll
  for (int k = 0; k < SM; ++k) {
    if (k < s) {
      double v = acc[k];
#pragma unroll
      for (int m = kWave / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
      if (lane == 0) d.W[t + d.Tp * k] = v * w;
    }
  }
}

static __global__ void __launch_bounds__(kNT)
kb_pw_y(const BMode* __restrict__ md, const int64_t* __restrict__ start, int nreq, int step) {
  const int r = breq(start, nreq, blockIdx.x);
  const BMode& d = md[r];
  const int64_t e = (blockIdx.x - start[r]) * kNT + threadIdx.x;
  if (step >= d.q || e >= d.I * d.s) return;
  const int64_t I = d.I, Tp = d.Tp;
  const int64_t i = e % I, k = e / I;
  const double* __restrict__ wk = d.W + Tp * k;
  const double* __restrict__ ci = d.Cp + i;
  double acc = 0.0;
  for (int64_t t = 0; t < Tp; ++t) acc = fma(ci[I * t], wk[t], acc);
  d.Y[e] = acc;
  if (!isfinite(acc) && d.status) atomicOr(d.status, kDevNonFinite);
}

// The shrink Y = X x_n Q_n^T, one thread per column of the mode-n view (rows
// in increasing order), into the float64 intermediate or, for the last mode,
// the caller's core (Tout).  Rows of Q^T are staged 32 at a time in LDS (zero
// beyond the request's ldq), and a thread issues its loads of 8 rows before
// it uses them.  MU >= every request's ldq.
constexpr int kShrinkRows = 32, kShrinkBatch = 8;

template <typename Tin, typename Tout, int MU>
__global__ void __launch_bounds__(kNT)
kb_shrink(const BMode* __restrict__ md, const int64_t* __restrict__ start, int nreq, int last) {
  __shared__ double qs[kShrinkRows][MU];
  const int r = breq(start, nreq, blockIdx.x);
  const BMode& d = md[r];
  const int64_t j = (blockIdx.x - start[r]) * kNT + threadIdx.x;
  const bool ok = j < d.J;
  const int64_t I = d.I, L = d.L;
  const int ldq = d.ldq;
  const Tin* __restrict__ X = static_cast<const Tin*>(d.X);
  const int64_t rr = ok ? j / L : 0, l = ok ? j - rr * L : 0;
  const Tin* __restrict__ col = X + l + L * I * rr;
  double acc[MU];
#pragma unroll
  for (int k = 0; k < MU; ++k) acc[k] = 0.0;
  for (int64_t i0 = 0; i0 < I; i0 += kShrinkRows) {
    const int ti = (int)min((int64_t)kShrinkRows, I - i0);
    for (int e = threadIdx.x; e < kShrinkRows * MU; e += kNT) {
      const int ii = e / MU, k = e - ii * MU;
      qs[ii][k] = (ii < ti && k < ldq) ? d.Qt[(i0 + ii) * ldq + k] : 0.0;
    }
    __syncthreads();
    if (ok) {
#pragma unroll 1
      for (int h = 0; h < ti; h += kShrinkBatch) {
        Tin v[kShrinkBatch];
#pragma unroll
        for (int b = 0; b < kShrinkBatch; ++b) v[b] = col[L * min(i0 + h + b, I - 1)];
#pragma unroll
        for (int b = 0; b < kShrinkBatch; ++b) {
          if (h + b < ti) {
            const double x = (double)v[b];
#pragma unroll
            for (int k = 0; k < MU; ++k) acc[k] = fma(qs[h + b][k], x, acc[k]);
          }
        }
      }
    }
    __syncthreads();
  }
  if (!ok) return;
  const int64_t base = l + L * d.mu * rr;  // (l, k, r) of the L x mu x R output
#pragma unroll
  for (int k = 0; k < MU; ++k) {
    if (k < d.mu) {
      if (last) static_cast<Tout*>(d.core)[base + L * k] = (Tout)acc[k];
      else d.out[base + L * k] = acc[k];
    }
  }
}

// The shrink of the first mode (L = 1) on the FP64 matrix cores:
// Y(k, j) = sum_i Q(i, k) X(i, j).  A workgroup takes kSmCols columns of one
// request (kSmTiles tiles of 16 columns per wave) and walks the rows in
// chunks of CR: each chunk of X is loaded with consecutive threads on
// consecutive rows of a column (coalesced for any I; rows past I and columns
// past J read a clamped valid address), stored to an LDS tile, and multiplied
// out from there with the chunk's rows of Q^T (staged beside it, zero beyond
// I and beyond the request's ldq, so clamped rows add exactly 0); the next
// chunk's loads are in flight during the products.  Lane layout of the MFMA
// as in tr_power.hpp: in each 16-row step lane (h, g) supplies rows
// 4g .. 4g + 3 of column h of a tile, four MFMAs per 16 outputs k.
constexpr int kSmTiles = 2, kSmCols = 16 * kSmTiles * (kNT / kWave);

template <typename Tin, typename Tout, int NKT>
__global__ void __launch_bounds__(kNT)
kb_shrink_mfma(const BMode* __restrict__ md, const int64_t* __restrict__ start, int nreq,
               int last) {
  constexpr int SP = 16 * NKT;
  constexpr int CR = sizeof(Tin) == 4 ? 64 : 32;   // rows per chunk
  constexpr int LDT = kSmCols + 1;                 // tile row stride (odd: no conflicts)
  constexpr int NL = CR * kSmCols / kNT;           // X loads per thread per chunk
  constexpr int NQ = CR * SP / kNT;                // Q^T loads per thread per chunk
  __shared__ Tin tile[CR][LDT];
  __shared__ double qs[CR][SP];
  const int r = breq(start, nreq, blockIdx.x);
  const BMode& d = md[r];
  const int64_t I = d.I, J = d.J;
  const int ldq = d.ldq;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wv = tid / kWave;
  const int h = lane & 15, g = lane >> 4;
  const int64_t jb = (blockIdx.x - start[r]) * kSmCols;
  const Tin* __restrict__ X = static_cast<const Tin*>(d.X);
  const double* __restrict__ Qt = d.Qt;
  Tin xv[NL];
  double qv[NQ];
  auto load = [&](int64_t i0) __attribute__((always_inline)) {
#pragma unroll
    for (int m = 0; m < NL; ++m) {
      const int e = tid + kNT * m;
      const int cc = e / CR, ii = e - cc * CR;
      xv[m] = X[min(jb + cc, J - 1) * I + min(i0 + ii, I - 1)];
    }
#pragma unroll
    for (int m = 0; m < NQ; ++m) {
      const int e = tid + kNT * m;
      const int ii = e / SP, k = e - ii * SP;
      const int64_t i = min(i0 + ii, I - 1);
      qv[m] = Qt[i * ldq + min(k, ldq - 1)];
    }
  };
  f64x4 acc[kSmTiles][NKT];
#pragma unroll
  for (int tl = 0; tl < kSmTiles; ++tl)
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt) acc[tl][kt] = f64x4{0.0, 0.0, 0.0, 0.0};
  load(0);
  for (int64_t i0 = 0; i0 < I; i0 += CR) {
#pragma unroll
    for (int m = 0; m < NL; ++m) {
      const int e = tid + kNT * m;
      const int cc = e / CR, ii = e - cc * CR;
      tile[ii][cc] = xv[m];
    }
#pragma unroll
    for (int m = 0; m < NQ; ++m) {
      const int e = tid + kNT * m;
      const int ii = e / SP, k = e - ii * SP;
      qs[ii][k] = (i0 + ii < I && k < ldq) ? qv[m] : 0.0;
    }
    __syncthreads();
    if (i0 + CR < I) load(i0 + CR);
#pragma unroll
    for (int u = 0; u < CR / 16; ++u)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int row = 16 * u + 4 * g + t;
#pragma unroll
        for (int tl = 0; tl < kSmTiles; ++tl) {
          const double b = (double)tile[row][16 * (kSmTiles * wv + tl) + h];
#pragma unroll
          for (int kt = 0; kt < NKT; ++kt)
            acc[tl][kt] = mfma_f64(qs[row][16 * kt + h], b, acc[tl][kt]);
        }
      }
    __syncthreads();
  }
  const int mu = d.mu;
#pragma unroll
  for (int tl = 0; tl < kSmTiles; ++tl) {
    const int64_t j = jb + 16 * (kSmTiles * wv + tl) + h;
    if (j >= J) continue;
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = 16 * kt + g + 4 * q;
        if (k < mu) {
          if (last) static_cast<Tout*>(d.core)[k + (int64_t)mu * j] = (Tout)acc[tl][kt][q];
          else d.out[k + (int64_t)mu * j] = acc[tl][kt][q];
        }
      }
  }
}

}  // namespace trk

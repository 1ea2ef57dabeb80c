// Register-resident factor kernel: Q_n = the mu leading left singular vectors
// of the sketch C (I x s, float64), with the same decomposition as k_factor
// (Householder QR of C, QR of R1^T, one-sided Jacobi on X = R2^T, Q_n =
// Q1 [U_X(:, 1:mu); 0]) but laid out for instruction count rather than for
// generality.  Thread t of the 256-thread workgroup keeps rows t and t + 256
// of C (and later of Q_n) in VGPRs; every column index is a compile-time
// constant (the column loops are instantiated per step), so nothing is
// indexed dynamically.  Workgroup sums go through one LDS tile of per-thread
// partials read back by 256/SM lanes per value and finished with DPP.
// Supports s <= SM (16, 24, 32, 40 or 48), I <= 256 R (mu <= MU).  The code is
// straight-line per step, so a smaller SM also means fewer instructions to
// fetch: a call after a large sweep fetches them from beyond the L2.
#pragma once

#include <type_traits>

#include "tr_device.hpp"
#include "tr_factor.hpp"
#include "tr_power.hpp"

namespace trk {

template <int SM>
struct RfShape {
  static constexpr int NT = 256;
  // reducer lanes per value (a power of two, SEG * SM <= NT)
  static constexpr int SEG = SM <= 16 ? 16 : (SM <= 32 ? 8 : 4);
  static constexpr int SEGLEN = NT / SEG;  // partial rows summed by one reducer lane
  static constexpr int PS = SM + 2;        // partial row stride (16-byte aligned rows)
  static constexpr int JW = kWave / SEG;   // values covered by one wave of reducers
  static constexpr int LDX = SM + 2;       // column stride of X and U (16-byte aligned)
  // Segment g starts JW doubles after the end of segment g-1: the reducers of
  // one wave (JW values x SEG segments) then spread over all 32 banks, and
  // segments never overlap.
  __host__ __device__ static constexpr int poff(int g) { return g * JW; }
  // Q formation: each wave stages 64 rows of V (the Householder vectors) in
  // its own LDS block of row stride LDV (16 TT columns, zero beyond SM)
  static constexpr int TT = (SM + 15) / 16;   // 16-wide tiles of V^T V per dimension
  static constexpr int LDV = 16 * TT + 2;
  static constexpr int kVB = NT * LDV;
  static constexpr int kP = NT * PS + SEG * JW > kVB ? NT * PS + SEG * JW : kVB;
  static constexpr int kTotal = kP + 2 * SM * LDX + 6 * SM + 16;  // doubles
  static constexpr size_t lds_bytes() { return 8 * (size_t)kTotal; }
};

template <int K, int END>
struct StaticFor {
  template <class F>
  __device__ __forceinline__ static void run(F& f) {
    if constexpr (K < END) {
      f(std::integral_constant<int, K>{});
      StaticFor<K + 1, END>::run(f);
    }
  }
};

struct RfSum {
  static constexpr double kId = 0.0;
  __device__ static double f(double a, double b) { return a + b; }
};
struct RfMax {
  static constexpr double kId = 0.0;  // operands are magnitudes
  __device__ static double f(double a, double b) { return fmax(a, b); }
};
struct RfMin {
  static constexpr double kId = 1.0e300;
  __device__ static double f(double a, double b) { return fmin(a, b); }
};

// Combine over SEG consecutive lanes (SEG in {4, 8, 16}); every lane of the
// group ends with the same value.  Must run with the whole wave active.
template <int SEG, class Op>
__device__ __forceinline__ double seg_reduce(double v) {
  v = Op::f(v, dpp_f64<kDppQuadXor1>(v));
  v = Op::f(v, dpp_f64<kDppQuadXor2>(v));
  if constexpr (SEG >= 8) v = Op::f(v, dpp_f64<kDppRowHalfMirror>(v));
  if constexpr (SEG >= 16) v = Op::f(v, dpp_f64<kDppRowMirror>(v));
  return v;
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// vec[j] = Op over the 256 threads of p[j], for J0 <= j < jend (jend <= N).
// Every thread must call it (two barriers).  Entries p[j] with j < J0 are not
// read; the caller keeps them initialised.
template <int SM, int N, int J0, class Op>
__device__ __forceinline__ void rf_reduce(const double (&p)[N], int jend, double* P,
                                          double* vec, int tid) {
  using S = RfShape<SM>;
  static_assert(N % 2 == 0 && N <= SM, "partials per thread");
  const int prow = tid * S::PS + S::poff(tid / S::SEGLEN);
  constexpr int JA = J0 & ~1;
#pragma unroll
  for (int j = JA; j < N; j += 2) {
    if (j < jend) {
      double2 v;
      v.x = p[j];
      v.y = p[j + 1];
      *reinterpret_cast<double2*>(P + prow + j) = v;
    }
  }
  __syncthreads();
  const int rj = tid / S::SEG, rg = tid % S::SEG;
  const bool mine = rj >= J0 && rj < jend;
  double acc = Op::kId;
  if (mine) {
    // every load of a batch is issued before the first add (one LDS round
    // trip per batch), then the batch is summed as a binary tree
    const double* src = P + rg * S::SEGLEN * S::PS + S::poff(rg) + rj;
    constexpr int BT = S::SEGLEN < 32 ? S::SEGLEN : 32;
#pragma unroll
    for (int b0 = 0; b0 < S::SEGLEN; b0 += BT) {
      double t[BT];
#pragma unroll
      for (int i = 0; i < BT; ++i) t[i] = src[(b0 + i) * S::PS];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int w = BT / 2; w >= 1; w /= 2) {
#pragma unroll
        for (int i = 0; i < w; ++i) t[i] = Op::f(t[i], t[i + w]);
      }
      acc = b0 == 0 ? t[0] : Op::f(acc, t[0]);
    }
  }
  acc = seg_reduce<S::SEG, Op>(acc);
  if (mine && rg == 0) vec[rj] = acc;
  __syncthreads();
}

// Householder reflector for (alpha, sum of squares below): beta, tau and the
// scale inv = 1 / (alpha - beta) of the vector below the unit entry.
__device__ __forceinline__ void householder(double alpha, double sum2, double* beta,
                                            double* tau, double* inv) {
  if (sum2 == 0.0) {
    *beta = alpha;
    *tau = 0.0;
    *inv = 0.0;
  } else {
    const double b = -copysign(sqrt(alpha * alpha + sum2), alpha);
    *beta = b;
    *tau = (b - alpha) / b;
    *inv = 1.0 / (alpha - b);
  }
}

// The kernel is straight-line code of 60-430 KB, run once per call, and the
// tensor sweeps before a call evict it from the caches, so each 64-byte
// instruction line would otherwise be fetched from HBM on demand.  A launch
// touches every 128-byte line of its own code once, with ordinary loads from
// all threads at the start: [this instruction's line, the end recorded by an
// earlier launch of the same kernel).  Returns the folded words (the caller
// consumes them so that the loads stay); no range recorded yet: no loads.
template <int NT, int M>
__device__ __forceinline__ unsigned touch_code(unsigned long long end) {
  const unsigned long long pc = __builtin_amdgcn_s_getpc() & ~127ull;
  unsigned acc = 0;
  if (end > pc && end - pc <= 128ull * NT * M) {
    const unsigned n = (unsigned)((end - pc) >> 7);
    unsigned v[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const unsigned l = threadIdx.x + NT * m;
      v[m] = l < n ? *reinterpret_cast<const unsigned*>(pc + 128ull * l) : 0u;
    }
#pragma unroll
    for (int m = 0; m < M; ++m) acc ^= v[m];
  }
  return acc;
}

// Where each factor kernel's code ends (written by its launches, read by the
// next ones); KIND tells the job-list and the job-table kernels apart.
template <int SM, int R, int MU, int KIND>
__device__ unsigned long long g_rf_code_end = 0;

// One factorization by the calling workgroup.
template <int SM, int R, int MU>
__device__ __forceinline__ void factor_rf_body(const FactorJob& jb, int cast_f32,
                                               uint32_t* __restrict__ status,
                                               unsigned long long code_end) {
  const double* __restrict__ C = jb.C;
  const int I = jb.I, s = jb.s, mu = jb.mu, ldqt = jb.ldqt;
  const bool qr_only = jb.qr_only != 0;  // Q1's leading columns, no SVD
  const bool tri_in = jb.tri_in != 0 && I == s;  // R1 = C: no QR
  double* __restrict__ Q = jb.Q;
  double* __restrict__ Qt = jb.Qt;
  double* __restrict__ sig_out = jb.sig;
  void* __restrict__ Qcast = jb.Qcast;
  using S = RfShape<SM>;
  constexpr int NT = S::NT, NW = NT / kWave, LDX = S::LDX;
  static_assert(MU <= SM && MU % 8 == 0, "column bound");
  extern __shared__ double smem[];
  double* P = smem;
  double* X = P + S::kP;         // Jacobi matrix, column c at X[c * LDX]
  double* U = X + SM * LDX;      // U_X(:, 1:mu)
  double* vec = U + SM * LDX;    // reduced values
  double* rowk = vec + SM;       // row k of the current step, double-buffered
  double* tau = rowk + 2 * SM;
  double* sig = tau + SM;
  int* perm = reinterpret_cast<int*>(sig + SM);
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int s1 = s - 1, I1 = I - 1;

  // all loads first from clamped addresses, then the masks (a select on a
  // loaded value would let the compiler branch around, and wait on, each load)
  double a[R][SM];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int ic = min(tid + NT * r, I1);
#pragma unroll
    for (int j = 0; j < SM; ++j) a[r][j] = C[(size_t)min(j, s1) * I + ic];
  }
  __builtin_amdgcn_sched_barrier(0);
  // the code lines' loads go out behind the sketch's, and both are waited
  // for together (vec[0] is cleared below in any case)
  const unsigned touched = touch_code<NT, 16>(code_end);
  if (touched == 0x5bd1e995u) vec[0] = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = tid + NT * r;
#pragma unroll
    for (int j = 0; j < SM; ++j)
      a[r][j] *= (i < I && j < s && (!tri_in || i <= j)) ? 1.0 : 0.0;
  }
  for (int e = tid; e < SM * LDX; e += NT) X[e] = 0.0;
  if (tid < SM) vec[tid] = 0.0;
  __syncthreads();

  // ---- 1. Householder QR of C; v_k (unit entry implied) overwrites column k
  //         below the diagonal, R1 stays on and above it ----
  auto qr_step = [&](auto kc) __attribute__((always_inline)) {
    constexpr int k = decltype(kc)::value;
    if (k >= s) return;
    double* rk = rowk + (k & 1) * SM;
    if (tid == k) {
#pragma unroll
      for (int j = k; j < SM; ++j) rk[j] = a[0][j];
    }
    double x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = tid + NT * r > k ? a[r][k] : 0.0;
    double p[SM];
#pragma unroll
    for (int j = 0; j < SM; ++j) {
      double t = 0.0;
      if (j >= k) {
#pragma unroll
        for (int r = 0; r < R; ++r) t = fma(x[r], a[r][j], t);
      }
      p[j] = t;
    }
    rf_reduce<SM, SM, k, RfSum>(p, s, P, vec, tid);
    double beta, tk, inv;
    householder(rk[k], vec[k], &beta, &tk, &inv);
    double tv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + NT * r;
      tv[r] = tk * (i > k ? inv * a[r][k] : (i == k ? 1.0 : 0.0));
    }
#pragma unroll
    for (int c0 = 0; c0 < SM; c0 += 8) {
      if (c0 + 8 > k + 1 && c0 < s) {
#pragma unroll
        for (int j = c0 > k ? c0 : k + 1; j < (c0 + 8 < SM ? c0 + 8 : SM); ++j) {
          const double w = rk[j] + inv * vec[j];
#pragma unroll
          for (int r = 0; r < R; ++r) a[r][j] = fma(-tv[r], w, a[r][j]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + NT * r;
      a[r][k] = i > k ? inv * a[r][k] : (i == k ? beta : a[r][k]);
    }
    if (tid == 0) tau[k] = tk;
  };
  // an upper-triangular square input is its own R1 (Q1 = I: every tau zero,
  // so the Q formation below returns U itself)
  if (tri_in) {
    if (tid < SM) tau[tid] = 0.0;
  } else {
    StaticFor<0, SM>::run(qr_step);
  }

  // ---- 2. QR of M = R1^T by wave 0: lane j holds column j of M (row j of
  //         R1, in thread j's registers); column k is broadcast by readlane ----
  if (wid == 0 && !qr_only) {
    double m[SM];
#pragma unroll
    for (int i = 0; i < SM; ++i) m[i] = (i >= lane && i < s) ? a[0][i] : 0.0;
    auto lq_step = [&](auto kc) __attribute__((always_inline)) {
      constexpr int k = decltype(kc)::value;
      if (k >= s) return;
      double xs[SM];
      double pj = 0.0;
#pragma unroll
      for (int c0 = 0; c0 < SM; c0 += 8) {
        if (c0 + 8 > k + 1 && c0 < s) {
#pragma unroll
          for (int i = c0 > k ? c0 : k + 1; i < (c0 + 8 < SM ? c0 + 8 : SM); ++i) {
            xs[i] = readlane_f64(m[i], k);
            pj = fma(xs[i], m[i], pj);
          }
        }
      }
      const double alpha = readlane_f64(m[k], k);
      const double sum2 = readlane_f64(pj, k);
      double beta, tk, inv;
      householder(alpha, sum2, &beta, &tk, &inv);
      const double w = m[k] + inv * pj;
      const double tw = tk * w;
#pragma unroll
      for (int c0 = 0; c0 < SM; c0 += 8) {
        if (c0 + 8 > k + 1 && c0 < s) {
#pragma unroll
          for (int i = c0 > k ? c0 : k + 1; i < (c0 + 8 < SM ? c0 + 8 : SM); ++i)
            m[i] = fma(-(inv * xs[i]), tw, m[i]);
        }
      }
      m[k] = lane == k ? beta : m[k] - tw;
    };
    StaticFor<0, SM>::run(lq_step);
    // X(j, c) = R2(c, j) for c <= j: lane j writes row j
    if (lane < SM) {
#pragma unroll
      for (int c = 0; c < SM; ++c) X[c * LDX + lane] = (c <= lane && lane < s) ? m[c] : 0.0;
    }
  }
  __syncthreads();

  // ---- 3. one-sided Jacobi on the columns of X.  SM <= 32: wave 0 alone
  //         (no barrier between steps: one wave's LDS accesses complete in
  //         order), pair g on lanes LP g .. LP g + LP - 1 (LP = 8 for
  //         SM == 16, 4 for 24 and 32).  SM == 40, 48: all four waves, 8 lanes
  //         per pair, pair g on lanes 8 (g / 4) .. + 7 of wave g % 4.  Each
  //         lane holds RU
  //         consecutive rows of the pair's two columns.  Column norms are
  //         recomputed at the start of each sweep and then updated with each
  //         rotation (a' = a - t c, b' = b + t c).  The sweeps end after one
  //         without a rotation larger than tol_big (see below). ----
  if (!qr_only) {
    // one wave up to 32 columns (no barrier between steps: measured 12 %
    // faster at SM = 24 than four waves with one); two lanes per pair would
    // be needed to fit 40 or 48 columns in one wave, which is slower
    constexpr bool kOneWave = SM <= 32;
    // lanes per pair; four waves give 64 / LP * 4 pair slots >= SM / 2
    constexpr int LP = SM == 16 ? 8 : (SM <= 32 ? 4 : 8);
    constexpr int RU = SM / LP;            // rows per lane
    static_assert(RU * LP == SM && (kOneWave ? kWave / LP : NW * (kWave / LP)) >= SM / 2,
                  "Jacobi pair layout");
    const int se = s + (s & 1), np = se / 2, sm1 = se - 1;
    const int lq = lane % LP;
    const int slot = kOneWave ? lane / LP : (lane / LP) * NW + wid;
    const bool gact = slot < np;
    const int gg = gact ? slot : 0;
    const double tol = 2.0 * s * 2.220446049250313e-16;
    // Cyclic Jacobi converges quadratically: after a sweep whose rotations
    // all had |x.y| / (|x| |y|) <= tol_big = sqrt(tol) / 10, every pair is
    // below tol, so the sweep that would only confirm it is skipped.
    const double tol_big = 0.1 * sqrt(tol);
    double* jn = sig;  // column norms^2 during the sweeps
    if (!kOneWave || wid == 0) {
      for (int sweep = 0; sweep < 40 && se > 1; ++sweep) {
        if (tid < se) {
          double t = 0.0;
#pragma unroll
          for (int i = 0; i < SM; ++i) t = fma(X[tid * LDX + i], X[tid * LDX + i], t);
          jn[tid] = t;
        }
        if (!kOneWave) __syncthreads();
        int rot = 0;
        // circle method: position 0 fixed, positions 1..se-1 advance each step
        int pp = gg == 0 ? -1 : gg - 1;  // -1: the fixed position
        int qq = se - 2 - gg;
        for (int step = 0; step < sm1; ++step) {
          const int p0 = pp < 0 ? 0 : pp + 1, q0 = qq + 1;
          const int p = min(p0, q0), q = max(p0, q0);
          double* xp = X + p * LDX + lq * RU;
          double* xq = X + q * LDX + lq * RU;
          double xv[RU], yv[RU];
#pragma unroll
          for (int u = 0; u < RU; ++u) {
            xv[u] = xp[u];
            yv[u] = xq[u];
          }
          const double aa = jn[p], bb = jn[q];
          double cc = 0.0;
#pragma unroll
          for (int u = 0; u < RU; ++u) cc = fma(xv[u], yv[u], cc);
          cc = seg_reduce<LP, RfSum>(cc);
          // Rotate when |x.y| / (|x| |y|) > tol (an estimate of the norms
          // suffices).  tan(theta) = sign(d) e / (|d| + hypot(d, e)) with
          // d = |y|^2 - |x|^2, e = 2 x.y, after scaling d and e by a common
          // power of two into [1/2, 1) so that every operand below is of
          // moderate size; cos = 1 / sqrt(1 + t^2), sin = t cos.  Late sweeps
          // rotate few pairs, and a wave with none skips the arithmetic.
          const double rel = fabs(cc) * __builtin_amdgcn_rsq(aa) * __builtin_amdgcn_rsq(bb);
          if (gact && cc != 0.0 && rel > tol) {
            const double dd = bb - aa;
            const int exe = __builtin_amdgcn_frexp_exp(cc) + 1;
            const int ex = dd == 0.0 ? exe : max(__builtin_amdgcn_frexp_exp(dd), exe);
            const double d = ldexp(dd, -ex), e = ldexp(2.0 * cc, -ex);
            const double t = copysign(1.0, d) * e * rcp_nr(fabs(d) + sqrt_nr(fma(d, d, e * e)));
            const double cs = rsqrt_nr(fma(t, t, 1.0));
            const double sn = cs * t;
#pragma unroll
            for (int u = 0; u < RU; ++u) {
              xp[u] = cs * xv[u] - sn * yv[u];
              xq[u] = sn * xv[u] + cs * yv[u];
            }
            if (lq == 0) {
              jn[p] = fma(-t, cc, aa);
              jn[q] = fma(t, cc, bb);
            }
            rot |= rel > tol_big ? 1 : 0;
          }
          if (!kOneWave) __syncthreads();
          if (pp >= 0) pp = pp + 1 == sm1 ? 0 : pp + 1;
          qq = qq + 1 == sm1 ? 0 : qq + 1;
        }
        if (kOneWave ? !__any(rot) : !__syncthreads_or(rot)) break;
      }
    }
  }
  __syncthreads();

  // ---- 4. singular values, descending (ties: lower column first); for an
  //         orthonormal basis only, U = I (Q1's columns in their order) ----
  if (tid < s && !qr_only) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < SM; ++i) t = fma(X[tid * LDX + i], X[tid * LDX + i], t);
    sig[tid] = sqrt(t);
  }
  __syncthreads();
  if (tid < s && !qr_only) {
    const double me = sig[tid];
    int rank = 0;
    for (int q = 0; q < s; ++q) {
      const double o = sig[q];
      rank += (o > me || (o == me && q < tid)) ? 1 : 0;
    }
    perm[rank] = tid;
    if (sig_out) sig_out[rank] = me;
    if (!isfinite(me) && status) atomicOr(status, kDevNonFinite);
  }
  if (tid < SM) vec[tid] = 0.0;
  __syncthreads();
  for (int e = tid; e < mu * SM; e += NT) {
    const int c = e / SM, i = e % SM;
    if (qr_only) {
      U[c * LDX + i] = (i < s && i == c) ? 1.0 : 0.0;
      continue;
    }
    const int pc = perm[c];
    const double sg = sig[pc];
    const double xv = X[pc * LDX + i];
    U[c * LDX + i] = i >= s ? 0.0 : (sg > 0.0 ? xv / sg : (i == pc ? 1.0 : 0.0));
  }
  __syncthreads();

  // ---- 5. Z = H_0 ... H_{s-1} [U; 0] in compact form.  With
  //         Z_{k+1} = H_{k+1} ... H_{s-1} [U; 0] and w_k = tau_k v_k^T Z_{k+1},
  //         Z = [U; 0] - sum_k v_k w_k, and since [U; 0] is zero below row s,
  //         w_k = tau_k (y_k - sum_{m > k} (v_k^T v_m) w_m), y = V(0:s, :)^T U.
  //         So one product G = V^T V (matrix cores), a short recurrence for
  //         the rows w_k, and one local update of every row replace the s
  //         dependent reflector applications. ----
  {
    constexpr int TT = S::TT, LDV = S::LDV, NTL = TT * (TT + 1) / 2;
    double* Vb = P + wid * kWave * LDV;  // this wave's 64 rows of V
    const int h = lane & 15, g = lane >> 4;
    f64x4 gacc[NTL];
#pragma unroll
    for (int t = 0; t < NTL; ++t) gacc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
    // rows tid + NT r, r descending: the last pass leaves rows 0 .. 63 (with
    // the top s rows of V) in wave 0's block
#pragma unroll
    for (int r = R - 1; r >= 0; --r) {
      const int i = tid + NT * r;
      wave_lds_order();
#pragma unroll
      for (int j = 0; j < 16 * TT; ++j) {
        double v = 0.0;
        if (j < SM) v = j < s ? (i > j ? a[r][j] : (i == j ? 1.0 : 0.0)) : 0.0;
        Vb[lane * LDV + j] = v;
      }
      wave_lds_order();
#pragma unroll
      for (int kk = 0; kk < kWave / 4; ++kk) {
        const double* row = Vb + (4 * kk + g) * LDV + h;
        int t = 0;
#pragma unroll
        for (int ta = 0; ta < TT; ++ta)
#pragma unroll
          for (int tb = ta; tb < TT; ++tb, ++t) gacc[t] = mfma_f64(row[16 * ta], row[16 * tb], gacc[t]);
      }
    }
    // the waves' partial tiles in the blocks of waves 1..3, summed in wave
    // order into G (row-major, stride LDX, in the Jacobi buffer, free now)
    double* Gp = P + kWave * LDV;
    double* G = X;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NTL; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) Gp[((wid * NTL + t) * 4 + q) * kWave + lane] = gacc[t][q];
    __syncthreads();
    for (int e = tid; e < NTL * 4 * kWave; e += NT) {
      const int t = e / (4 * kWave), q = (e / kWave) % 4, ln = e % kWave;
      int ta = 0, tb = 0, c = 0;
      for (int x = 0; x < TT; ++x)
        for (int y = x; y < TT; ++y, ++c)
          if (c == t) {
            ta = x;
            tb = y;
          }
      const int m = 16 * ta + (ln >> 4) + 4 * q, k = 16 * tb + (ln & 15);
      double sum = Gp[((0 * NTL + t) * 4 + q) * kWave + ln];
#pragma unroll
      for (int w = 1; w < NW; ++w) sum += Gp[((w * NTL + t) * 4 + q) * kWave + ln];
      if (m < SM && k < SM) G[m * LDX + k] = sum;
    }
    __syncthreads();
    // y(k, c) = sum_i V(i, k) U(i, c) over i < SM (V is zero above its unit
    // diagonal and U below row s), zero for c >= mu
    double* Ys = Gp;
    double* Ws = Gp + SM * MU;
    for (int e = tid; e < SM * MU; e += NT) {
      const int k = e / MU, c = e % MU;
      const int cc = c < mu ? c : 0;
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < SM; ++i) t = fma(P[i * LDV + k], U[cc * LDX + i], t);
      Ys[e] = c < mu ? t : 0.0;
    }
    __syncthreads();
    // w_k, k = s-1 .. 0, lane c of wave 0; G, y and w are zero past s, so
    // every step runs unmasked (the dot product in two alternating partial
    // sums, added at the end)
    if (wid == 0) {
      const int c = lane < MU ? lane : MU - 1;
      double w[SM];
      auto w_step = [&](auto kc) __attribute__((always_inline)) {
        constexpr int k = SM - 1 - decltype(kc)::value;
        double acc0 = Ys[k * MU + c], acc1 = 0.0;
#pragma unroll
        for (int m = k + 1; m < SM; ++m) {
          const double gkm = G[k * LDX + m];
          if ((m - k) & 1) acc0 = fma(-gkm, w[m], acc0);
          else acc1 = fma(-gkm, w[m], acc1);
        }
        w[k] = k < s ? tau[k] * (acc0 + acc1) : 0.0;
      };
      StaticFor<0, SM>::run(w_step);
      if (lane < MU) {
#pragma unroll
        for (int k = 0; k < SM; ++k) Ws[k * MU + lane] = w[k];
      }
    }
    __syncthreads();
  }
  double z[R][MU];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = tid + NT * r;
#pragma unroll
    for (int c = 0; c < MU; ++c) {
      const double u = U[min(c, mu - 1) * LDX + min(i, SM - 1)];
      z[r][c] = (i < s && c < mu) ? u : 0.0;
    }
  }
  {
    const double* Ws = P + kWave * S::LDV + SM * MU;
    // (rows k >= s of W are zero, so the loop runs unmasked)
#pragma unroll
    for (int k = 0; k < SM; ++k) {
      double v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = tid + NT * r;
        v[r] = i > k ? a[r][k] : (i == k ? 1.0 : 0.0);
      }
#pragma unroll
      for (int c = 0; c < MU; ++c) {
        const double wk = Ws[k * MU + c];
#pragma unroll
        for (int r = 0; r < R; ++r) z[r][c] = fma(-v[r], wk, z[r][c]);
      }
    }
  }
  __syncthreads();  // W (in P) is read until here; the sign step reuses P

  // ---- 6. sign: the largest-magnitude entry of each column (lowest row on
  //         ties) becomes positive ----
  {
    double pm[MU];
#pragma unroll
    for (int c = 0; c < MU; ++c) {
      double t = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) t = fmax(t, fabs(z[r][c]));
      pm[c] = t;
    }
    rf_reduce<SM, MU, 0, RfMax>(pm, mu, P, vec, tid);
#pragma unroll
    for (int c = 0; c < MU; ++c) {
      const double mx = vec[c];
      double t = RfMin::kId;
#pragma unroll
      for (int r = R - 1; r >= 0; --r) {
        const int i = tid + NT * r;
        if (i < I && fabs(z[r][c]) == mx) t = 2.0 * i + (z[r][c] < 0.0 ? 1.0 : 0.0);
      }
      pm[c] = t;
    }
    rf_reduce<SM, MU, 0, RfMin>(pm, mu, P, vec, tid);
  }
  double sg[MU];
#pragma unroll
  for (int c = 0; c < MU; ++c) {
    const double key = vec[c];
    sg[c] = (key - 2.0 * floor(0.5 * key)) != 0.0 ? -1.0 : 1.0;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = tid + NT * r;
    if (i < I) {
#pragma unroll
      for (int c = 0; c < MU; ++c) {
        if (c < mu) {
          const double zz = z[r][c] * sg[c];
          Q[i + (int64_t)I * c] = zz;
          if (Qcast) {
            if (cast_f32) ((float*)Qcast)[i + (int64_t)I * c] = (float)zz;
            else ((double*)Qcast)[i + (int64_t)I * c] = zz;
          }
          if (Qt) Qt[(int64_t)i * ldqt + c] = zz;
        }
      }
      if (Qt)
        for (int c = mu; c < ldqt; ++c) Qt[(int64_t)i * ldqt + c] = 0.0;
    }
  }
}

// Workgroup b factors jobs.j[b] (several independent sketches per launch).
template <int SM, int R, int MU>
__global__ void __launch_bounds__(256)
k_factor_rf(FactorJobs jobs, int cast_f32, uint32_t* __restrict__ status) {
  factor_rf_body<SM, R, MU>(jobs.j[blockIdx.x], cast_f32, status, g_rf_code_end<SM, R, MU, 0>);
  if (threadIdx.x == 0 && blockIdx.x == 0)
    g_rf_code_end<SM, R, MU, 0> = __builtin_amdgcn_s_getpc();
}

// Jobs from a device table (the batched driver, whose batches outnumber the
// kernel-argument job list): workgroup b factors tab[b] and reports to
// status_tab[b] (no status when status_tab is null).
template <int SM, int R, int MU>
__global__ void __launch_bounds__(256)
k_factor_rf_tab(const FactorJob* __restrict__ tab, int cast_f32, uint32_t* const* status_tab) {
  factor_rf_body<SM, R, MU>(tab[blockIdx.x], cast_f32,
                            status_tab ? status_tab[blockIdx.x] : nullptr,
                            g_rf_code_end<SM, R, MU, 1>);
  if (threadIdx.x == 0 && blockIdx.x == 0)
    g_rf_code_end<SM, R, MU, 1> = __builtin_amdgcn_s_getpc();
}

}  // namespace trk

// Factor kernel of the range finder with its working matrices in LDS or in
// global scratch (any s <= 64): the sketch's mu leading left singular vectors
// by Householder QR, a second QR, one-sided Jacobi and the reflectors applied
// back (Alg. 1 and 4, the SVD step that yields Q_n).
#pragma once

#include "tr_device.hpp"
#include "tr_kernels.hpp"

namespace trk {

// ---------------------------------------------------------------------------
// K7 + K8  Factor of a sketch C (I x s, float64) on one workgroup of 256
// threads: Q = the mu leading left singular vectors of C.
//   1. Householder QR  C = H_0 ... H_{s-1} [R1; 0]          (block-wide)
//   2. QR of R1^T = Q2 R2                                    (one wave)
//   3. one-sided Jacobi on the columns of X = R2^T           (four waves)
//      C = Q1 R1 = Q1 X Q2^T, so the left singular vectors of C are
//      Q1 U_X with U_X the normalised rotated columns of X; the second QR
//      makes the Jacobi sweeps converge about twice as fast.
//   4. sort by singular value, U = U_X(:, 1:mu)
//   5. Q = H_0 ... H_{s-1} [U; 0]                            (block-wide)
//   6. sign of each column: largest |entry| (lowest row on ties) positive.
// The I x s and I x mu working matrices live in LDS, or (kGlobal) in global
// scratch supplied by the caller when they do not fit.  Thread t owns rows
// t + 256 m throughout, so only reductions cross threads.
// ---------------------------------------------------------------------------
constexpr int kFactorNT = 256;

// SM > 64 (the wide variant, s <= 128): M = R1 (the second QR is skipped;
// R1's left singular vectors are those C's Q1 rotates) stays in LDS, U lives
// in global scratch (FactorJob::gW, SM LDR doubles) as do the I x s and
// I x mu working matrices, and the Jacobi gives each column pair four lanes
// (all pairs of a step at once; the pair of a step is computed, not tabled).
template <int SM>
struct FactorShape {
  static constexpr int NT = kFactorNT, NW = NT / kWave, LDR = SM + 1;
  static constexpr bool kWide = SM > 64;
  // always-LDS part (doubles): M/X, U, scratch, vec and small vectors
  static constexpr int kSmall =
      (kWide ? 1 : 2) * SM * LDR + NW * SM + 11 * SM + 16 + (kWide ? 0 : SM * SM / 2);
  static size_t lds_bytes(int I, int s, int mu, bool global_mats) {
    return 8 * ((global_mats ? 0 : (size_t)I * (s + mu)) + kSmall);
  }
  static size_t wide_scratch_bytes() { return kWide ? 8 * (size_t)(SM * LDR) : 0; }
};

__device__ __forceinline__ void lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// Circle-method pairing: at step t of a sweep over se (even) columns, pair g
// joins positions g and se-1-g; position 0 is fixed, the others rotate.
__device__ __forceinline__ void jacobi_pair(int g, int step, int se, int* pp, int* qq) {
  const int x1 = se - 1 - g;
  const int p = g == 0 ? 0 : ((g - 1 + step) % (se - 1)) + 1;
  const int q = ((x1 - 1 + step) % (se - 1)) + 1;
  *pp = p < q ? p : q;
  *qq = p < q ? q : p;
}

// One factorization of a batch: the sketch C (I x s), its outputs Q (I x mu),
// Qt (row stride ldqt), sigma and the optional cast copy of Q, and (global
// variant) the I x s scratch gA; Q doubles as the I x mu scratch there.
struct FactorJob {
  const double* C;
  double* Q;
  double* Qt;
  double* sig;
  void* Qcast;
  double* gA;
  int I, s, mu, ldqt;
  double* gW;  // wide variant (s > 64): scratch for the two s x s matrices
  // orthonormal basis only (the register-resident kernel): Q = the first mu
  // columns of the Householder QR's Q1 with canonical signs, no SVD (the
  // power scheme's orthonormalisation between steps); sig is not written
  int qr_only;
  // (the register-resident kernel) C is s x s (I == s) and upper triangular:
  // the Householder QR is skipped and entries below the diagonal are ignored
  int tri_in;
};
constexpr int kMaxFactorJobs = 8;
// Independent factorizations launched together, one workgroup each (by value
// in the kernel arguments; workgroup b takes j[b]).
struct FactorJobs {
  FactorJob j[kMaxFactorJobs];
};

template <int SM, bool kGlobal>
__global__ void __launch_bounds__(kFactorNT)
k_factor(FactorJobs jobs, int cast_f32, uint32_t* __restrict__ status) {
  const FactorJob& jb = jobs.j[blockIdx.x];
  const double* __restrict__ C = jb.C;
  const int I = jb.I, s = jb.s, mu = jb.mu, ldqt = jb.ldqt;
  double* __restrict__ Q = jb.Q;
  double* __restrict__ Qt = jb.Qt;
  double* __restrict__ sig_out = jb.sig;
  void* __restrict__ Qcast = jb.Qcast;
  double* __restrict__ gA = jb.gA;
  double* __restrict__ gZ = jb.Q;
  using F = FactorShape<SM>;
  constexpr int NT = F::NT, NW = F::NW, LDR = F::LDR, H = SM / 2, HW = (H + NW - 1) / NW;
  constexpr int CH = SM < 16 ? SM : 16;  // columns per register chunk
  extern __shared__ double smem[];
  double* sp = smem;
  constexpr bool kWide = F::kWide;
  static_assert(!kWide || kGlobal, "the wide variant keeps its matrices in global memory");
  double* A = kGlobal ? gA : sp;                    // I x s, column-major
  double* Z = kGlobal ? gZ : sp + (size_t)I * s;    // I x mu, column-major
  if (!kGlobal) sp += (size_t)I * (s + mu);
  // R1^T, then X = R2^T (column c at M[c*LDR]); wide: R1 itself
  double* M = sp;
  // R2^T while it is built, then U_X(:, 1:mu); wide: in global scratch
  double* U = kWide ? jb.gW : M + SM * LDR;
  sp += (kWide ? 1 : 2) * SM * LDR;
  double* scr = sp;                // NW x SM reduction scratch
  double* vec = scr + NW * SM;     // reduced vector
  double* tau = vec + SM;
  double* rowk = tau + SM;
  double* vec2 = rowk + SM;        // single-wave reductions
  double* sig = vec2 + SM;
  double* sgn = sig + SM;
  double* jn = sgn + SM;           // Jacobi column norms^2
  int* perm = reinterpret_cast<int*>(jn + SM);
  int* flag = reinterpret_cast<int*>(jn + 2 * SM);
  int* pairs = reinterpret_cast<int*>(jn + 2 * SM + 8);  // p | q << 8 per (step, g)
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int s1 = s - 1, I1 = I - 1, mu1 = mu - 1;

  for (int e = tid; e < I * s; e += NT) A[e] = C[e];
  for (int e = tid; e < SM * LDR; e += NT) {
    M[e] = 0.0;
    U[e] = 0.0;
  }
  for (int e = tid; e < (NW + 4) * SM; e += NT) scr[e] = 0.0;  // scr, vec, tau, rowk, vec2
  __syncthreads();

  // Chunk c0 of a workgroup vector sum: lane-wise partials part[q] (values
  // c0 + q) go through the wave transpose-reduce into scr.
  auto chunk_to_scr = [&](double (&part)[CH], int c0) {
    const double r = wave_vec_sum<CH>(part, lane);
    if (lane < CH) scr[wid * SM + c0 + wave_vec_index<CH>(lane)] = r;
  };
  auto finish_sum = [&]() {  // scr -> vec, two barriers
    __syncthreads();
    if (tid < SM) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) t += scr[w * SM + tid];
      vec[tid] = t;
    }
    __syncthreads();
  };

  // ---- 1. Householder QR of C: v_k = 1, H_k = I - tau_k v v^T ----
  for (int k = 0; k < s; ++k) {
    const double alpha = A[(size_t)k * I + k];
    if (tid < SM) rowk[tid] = A[(size_t)min(tid, s1) * I + k];
    // pass 1: part[k] = sum_{i>k} x_i^2, part[j] = sum_{i>k} x_i a_ij (j > k);
    // chunks holding only columns j < k or j >= s are skipped
#pragma unroll
    for (int c0 = 0; c0 < SM; c0 += CH) {
      if (c0 + CH <= k || c0 >= s) continue;
      double part[CH];
#pragma unroll
      for (int q = 0; q < CH; ++q) part[q] = 0.0;
      for (int i = tid; i < I; i += NT) {
        const double x = A[(size_t)k * I + i] * (i > k ? 1.0 : 0.0);
        double av[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) av[q] = A[(size_t)min(c0 + q, s1) * I + i];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          const int j = c0 + q;
          part[q] += x * (j == k ? x : (j > k && j < s ? av[q] : 0.0));
        }
      }
      chunk_to_scr(part, c0);
    }
    finish_sum();
    const double sum2 = vec[k];
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
    // pass 2: a_ij -= tau v_i w_j with w_j = a_kj + inv * vec[j]; v_i into column k
#pragma unroll
    for (int c0 = 0; c0 < SM; c0 += CH) {
      if (c0 + CH <= k + 1 || c0 >= s) continue;
      double w[CH];
#pragma unroll
      for (int q = 0; q < CH; ++q) w[q] = rowk[c0 + q] + inv * vec[c0 + q];
      for (int i = tid; i < I; i += NT) {
        const double v = A[(size_t)k * I + i] * inv;
        double av[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) av[q] = A[(size_t)min(c0 + q, s1) * I + i];
        if (i > k) {
#pragma unroll
          for (int q = 0; q < CH; ++q) {
            const int j = c0 + q;
            if (j > k && j < s) A[(size_t)j * I + i] = av[q] - tk * v * w[q];
          }
        }
      }
    }
    for (int i = tid; i < I; i += NT)
      if (i > k) A[(size_t)k * I + i] *= inv;
    // R1 row k -> column k of M = R1^T (wide: row k of M = R1)
    if (tid < s) {
      const double r1 = tid == k ? beta
                        : (tid > k ? rowk[tid] - tk * (rowk[tid] + inv * vec[tid]) : 0.0);
      if constexpr (kWide) M[tid * LDR + k] = r1;
      else M[k * LDR + tid] = r1;
    }
    if (tid == 0) tau[k] = tk;
    __syncthreads();
  }

  // ---- 2. QR of M = R1^T (s x s) by wave 0, lane = row; U = R2^T ----
  if (!kWide && wid == 0) {
    const int ln = min(lane, s1);
    for (int k = 0; k < s; ++k) {
      const double alpha = M[k * LDR + k];
      const double mk = M[k * LDR + ln] * (lane > k && lane < s ? 1.0 : 0.0);
#pragma unroll
      for (int c0 = 0; c0 < SM; c0 += CH) {
        if (c0 + CH <= k || c0 >= s) continue;
        double part[CH];
        double mv[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) mv[q] = M[min(c0 + q, s1) * LDR + ln];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          const int j = c0 + q;
          part[q] = mk * (j == k ? mk : (j > k && j < s ? mv[q] : 0.0));
        }
        const double r = wave_vec_sum<CH>(part, lane);
        if (lane < CH) vec2[c0 + wave_vec_index<CH>(lane)] = r;
      }
      lds_fence();
      const double sum2 = vec2[k];
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
      // R2 row k (lane j holds entry j), read before rows > k change
      const double mkj = M[ln * LDR + k];
      const double r2 = lane == k ? beta
                        : (lane > k && lane < s ? mkj - tk * (mkj + inv * vec2[ln]) : 0.0);
      // rows i > k: M(i, j) -= tau v_i w_j, w_j = M(k, j) + inv vec2[j]
      const double v = mk * inv;
#pragma unroll
      for (int c0 = 0; c0 < SM; c0 += CH) {
        if (c0 + CH <= k + 1 || c0 >= s) continue;
        double mv[CH], wk[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          mv[q] = M[min(c0 + q, s1) * LDR + ln];
          wk[q] = M[min(c0 + q, s1) * LDR + k] + inv * vec2[c0 + q];
        }
        if (lane > k && lane < s) {
#pragma unroll
          for (int q = 0; q < CH; ++q) {
            const int j = c0 + q;
            if (j > k && j < s) M[j * LDR + lane] = mv[q] - tk * v * wk[q];
          }
        }
      }
      if (lane < s) U[k * LDR + lane] = r2;   // X(j, k) = R2(k, j)
      lds_fence();
    }
    // X = R2^T becomes the Jacobi matrix
    for (int e = lane; e < SM * LDR; e += kWave) {
      M[e] = U[e];
      U[e] = 0.0;
    }
  }
  __syncthreads();

  // ---- 3. one-sided Jacobi on the columns of X; pair g on wave g % NW ----
  if constexpr (kWide) {
    // wide: pair g on lanes 4g .. 4g + 3, lane lq holding rows lq + 4u of the
    // pair's two columns (rows past s are zero and stay zero); every pair of
    // a step rotates at once, one barrier per step
    constexpr int LP = NT / (SM / 2), RU = SM / LP;
    static_assert(LP == 4, "four lanes per pair");
    const int se = s + (s & 1), np = se / 2;
    const int g = tid / LP, lq = tid % LP;
    const bool gact = g < np;
    const double tol = 2.0 * s * 2.220446049250313e-16;
    const double tol_big = 0.1 * sqrt(tol);
    for (int sweep = 0; sweep < 40 && se > 1; ++sweep) {
      if (tid < se) {
        double a = 0.0;
        for (int i = 0; i < s; ++i) a += M[tid * LDR + i] * M[tid * LDR + i];
        jn[tid] = a;
      }
      __syncthreads();
      int rot = 0;
      for (int step = 0; step < se - 1; ++step) {
        int p = 0, q = 1;
        if (gact) jacobi_pair(g, step, se, &p, &q);
        double* xp = M + p * LDR;
        double* xq = M + q * LDR;
        double xv[RU], yv[RU];
        double c = 0.0;
#pragma unroll
        for (int u = 0; u < RU; ++u) {
          xv[u] = xp[lq + LP * u];
          yv[u] = xq[lq + LP * u];
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) c = fma(xv[u], yv[u], c);
        c += dpp_f64<kDppQuadXor1>(c);
        c += dpp_f64<kDppQuadXor2>(c);
        const double a = jn[p], b = jn[q];
        if (gact && c != 0.0 && fabs(c) > tol * sqrt(a) * sqrt(b)) {
          const double zeta = (b - a) / (2.0 * c);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + t * t);
          const double sn = cs * t;
#pragma unroll
          for (int u = 0; u < RU; ++u) {
            xp[lq + LP * u] = cs * xv[u] - sn * yv[u];
            xq[lq + LP * u] = sn * xv[u] + cs * yv[u];
          }
          if (lq == 0) {
            jn[p] = a - t * c;
            jn[q] = b + t * c;
          }
          rot |= fabs(c) > tol_big * sqrt(a) * sqrt(b) ? 1 : 0;
        }
        __syncthreads();
      }
      if (!__syncthreads_or(rot)) break;
    }
  } else {
    const int se = s + (s & 1);
    const int np = se / 2;
    const int np1 = np - 1;
    const int ln = min(lane, s1);
    const double tol = 2.0 * s * 2.220446049250313e-16;
    // Cyclic Jacobi converges quadratically: after a sweep whose rotations
    // all had |x.y| / (|x| |y|) <= tol_big = sqrt(tol) / 10, every pair is
    // below tol, so the sweep that would only confirm it is skipped.
    const double tol_big = 0.1 * sqrt(tol);
    for (int e = tid; e < (se - 1) * np; e += NT) {
      int pp, qq;
      jacobi_pair(e % np, e / np, se, &pp, &qq);
      pairs[(e / np) * H + (e % np)] = pp | (qq << 8);
    }
    for (int sweep = 0; sweep < 40 && se > 1; ++sweep) {
      if (tid < se) {  // exact column norms at the start of every sweep
        double a = 0.0;
        for (int i = 0; i < s; ++i) a += M[tid * LDR + i] * M[tid * LDR + i];
        jn[tid] = a;
      }
      if (tid == 0) *flag = 0;
      __syncthreads();
      for (int step = 0; step < se - 1; ++step) {
        double xs[HW], ys[HW], cc[HW], aa[HW], bb[HW];
        int ps[HW], qs[HW];
#pragma unroll
        for (int h = 0; h < HW; ++h) {
          const int g = wid + NW * h;
          const int pq = pairs[step * H + min(g, np1)];
          ps[h] = pq & 0xff;
          qs[h] = pq >> 8;
        }
#pragma unroll
        for (int h = 0; h < HW; ++h) {
          xs[h] = M[ps[h] * LDR + ln];
          ys[h] = M[qs[h] * LDR + ln];
          aa[h] = jn[ps[h]];
          bb[h] = jn[qs[h]];
        }
#pragma unroll
        for (int h = 0; h < HW; ++h) cc[h] = wave_sum(lane < s ? xs[h] * ys[h] : 0.0);
#pragma unroll
        for (int h = 0; h < HW; ++h) {
          const int g = wid + NW * h;
          const double a = aa[h], b = bb[h], c = cc[h];
          if (g < np && c != 0.0 && fabs(c) > tol * sqrt(a) * sqrt(b)) {
            const double zeta = (b - a) / (2.0 * c);
            const double t =
                (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double cs = 1.0 / sqrt(1.0 + t * t);
            const double sn = cs * t;
            if (lane < s) {
              M[ps[h] * LDR + lane] = cs * xs[h] - sn * ys[h];
              M[qs[h] * LDR + lane] = sn * xs[h] + cs * ys[h];
            }
            if (lane == 0) {
              jn[ps[h]] = a - t * c;
              jn[qs[h]] = b + t * c;
              if (fabs(c) > tol_big * sqrt(a) * sqrt(b)) *flag = 1;
            }
          }
        }
        __syncthreads();
      }
      const int more = *flag;
      __syncthreads();
      if (!more) break;
    }
  }

  // ---- 4. singular values, descending order (ties: lower column first) ----
  if (tid < s) {
    double a = 0.0;
    for (int i = 0; i < s; ++i) a += M[tid * LDR + i] * M[tid * LDR + i];
    sig[tid] = sqrt(a);
  }
  __syncthreads();
  if (tid < s) {
    const double me = sig[tid];
    int rank = 0;
    for (int q = 0; q < s; ++q) {
      const double o = sig[q];
      if (o > me || (o == me && q < tid)) ++rank;
    }
    perm[rank] = tid;
    if (sig_out) sig_out[rank] = me;
    if (!isfinite(me) && status) atomicOr(status, kDevNonFinite);
  }
  __syncthreads();
  for (int e = tid; e < mu * s; e += NT) {
    const int c = e / s, i = e % s;
    const int pc = perm[c];
    const double sg = sig[pc];
    U[c * LDR + i] = sg > 0.0 ? M[pc * LDR + i] / sg : (i == pc ? 1.0 : 0.0);
  }
  __syncthreads();

  // ---- 5. Z = H_0 ... H_{s-1} [U; 0] ----
  for (int e = tid; e < I * mu; e += NT) {
    const int c = e / I, i = e % I;
    Z[e] = i < s ? U[c * LDR + min(i, s1)] : 0.0;
  }
  __syncthreads();
  for (int k = s - 1; k >= 0; --k) {
    const double tk = tau[k];
#pragma unroll
    for (int c0 = 0; c0 < SM; c0 += CH) {
      if (c0 >= mu) continue;
      double part[CH];
#pragma unroll
      for (int q = 0; q < CH; ++q) part[q] = 0.0;
      for (int i = tid; i < I; i += NT) {
        const double v = i == k ? 1.0 : A[(size_t)k * I + i] * (i > k ? 1.0 : 0.0);
        double zv[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) zv[q] = Z[(size_t)min(c0 + q, mu1) * I + i];
#pragma unroll
        for (int q = 0; q < CH; ++q) part[q] += v * (c0 + q < mu ? zv[q] : 0.0);
      }
      chunk_to_scr(part, c0);
    }
    finish_sum();
#pragma unroll
    for (int c0 = 0; c0 < SM; c0 += CH) {
      if (c0 >= mu) continue;
      double w[CH];
#pragma unroll
      for (int q = 0; q < CH; ++q) w[q] = tk * vec[c0 + q];
      for (int i = tid; i < I; i += NT) {
        const double v = i == k ? 1.0 : A[(size_t)k * I + i] * (i > k ? 1.0 : 0.0);
        double zv[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) zv[q] = Z[(size_t)min(c0 + q, mu1) * I + i];
        if (i >= k) {
#pragma unroll
          for (int q = 0; q < CH; ++q)
            if (c0 + q < mu) Z[(size_t)(c0 + q) * I + i] = zv[q] - v * w[q];
        }
      }
    }
  }
  __syncthreads();

  // ---- 6. signs and outputs ----
  for (int c = wid; c < mu; c += NW) {
    double best = -1.0, bval = 0.0;
    for (int i0 = 0; i0 < I; i0 += kWave) {
      const int i = i0 + lane;
      const double z = Z[(size_t)c * I + min(i, I1)];
      const double az = i < I ? fabs(z) : -1.0;
      const double m = wave_max(az);
      if (m > best) {
        const unsigned long long hit = __ballot(az == m);
        const int l = __ffsll((long long)hit) - 1;
        best = m;
        bval = __shfl(z, l, kWave);
      }
    }
    if (lane == 0) sgn[c] = bval < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  // Q's mu columns, and with Qt its padding columns up to ldqt too
  const int lq = Qt ? ldqt : mu;
  for (int e = tid; e < I * lq; e += NT) {
    const int i = e / lq, c = e % lq;
    const double zz = Z[(size_t)min(c, mu1) * I + i] * sgn[min(c, mu1)];
    const double z = c < mu ? zz : 0.0;
    if (c < mu) {
      Q[i + (int64_t)I * c] = z;
      if (Qcast) {
        if (cast_f32) ((float*)Qcast)[i + (int64_t)I * c] = (float)z;
        else ((double*)Qcast)[i + (int64_t)I * c] = z;
      }
    }
    if (Qt) Qt[(int64_t)i * ldqt + c] = z;  // padding columns are zero
  }
}

}  // namespace trk

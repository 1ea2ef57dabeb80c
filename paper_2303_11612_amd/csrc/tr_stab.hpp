// Power scheme with an orthonormalisation after every step and the triangular
// factors accumulated (the numerically safer form of the power products,
// equal to them in exact arithmetic):
//   Z_0 R_0 = G,  Z_i R_i = M D M^T Z_{i-1}  (i = 1..q),  Rbar = R_q ... R_0,
// so (M D M^T)^q G = Z_q Rbar and its leading left singular vectors are
// Z_q U'(:, 1:mu) with Rbar = U' S V'^T.  Each Z_i is an orthonormal basis of
// the iterate's range from the factor kernel, and R_i = Z_i^T Y_i.  The
// kernels here form R_i, accumulate Rbar and apply the small factor U' (with
// the canonical signs) to produce Q_n, for several modes per launch: job y of
// a launch is mode y's (blockIdx.y), and a mode's arithmetic does not depend
// on the others.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace trk {

constexpr int kStabNT = 256;
constexpr int kStabMaxJobs = 8;  // modes per launch

// One mode's step: R = Z^T Y (Z, Y column-major I x s, R column-major s x s),
// then Rbar <- R Rbar (first: Rbar <- R), s <= 64.
struct StabStep {
  const double* Z;
  const double* Y;
  double* R;
  double* Rbar;
  int64_t I;
  int s, first;
};
struct StabSteps {
  StabStep j[kStabMaxJobs];
};

// R(a, b) = sum_i Z(i, a) Y(i, b) for a, b < s.  Grid (smax^2, jobs), smax the
// largest s: workgroup x of job y takes entry (x % smax, x / smax) if both are
// below the job's s; thread t sums rows t, t + 256, ... in order, the partial
// sums are added by a fixed tree.
static __global__ void __launch_bounds__(kStabNT)
k_small_tn(StabSteps jobs, int smax) {
  __shared__ double red[kStabNT];
  const StabStep& jb = jobs.j[blockIdx.y];
  const int s = jb.s;
  const int64_t I = jb.I;
  const int a = (int)(blockIdx.x % smax), b = (int)(blockIdx.x / smax);
  if (a >= s || b >= s) return;  // the whole workgroup
  const double* __restrict__ Z = jb.Z;
  const double* __restrict__ Y = jb.Y;
  const double* za = Z + (int64_t)a * I;
  const double* yb = Y + (int64_t)b * I;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < I; i += kStabNT) acc = fma(za[i], yb[i], acc);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kStabNT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) jb.R[a + (int64_t)s * b] = red[0];
}

// Rbar <- R Rbar (first: Rbar <- R); s x s column-major, s <= 64.  One
// workgroup per job; the old Rbar is staged in LDS, each entry summed in
// increasing c.
static __global__ void __launch_bounds__(kStabNT)
k_rbar_update(StabSteps jobs) {
  __shared__ double old[64 * 64];
  const StabStep& jb = jobs.j[blockIdx.x];
  const double* __restrict__ R = jb.R;
  double* __restrict__ Rbar = jb.Rbar;
  const int s = jb.s, first = jb.first;
  const int n = s * s;
  if (first) {
    for (int e = threadIdx.x; e < n; e += kStabNT) Rbar[e] = R[e];
    return;
  }
  for (int e = threadIdx.x; e < n; e += kStabNT) old[e] = Rbar[e];
  __syncthreads();
  for (int e = threadIdx.x; e < n; e += kStabNT) {
    const int a = e % s, b = e / s;
    double acc = 0.0;
    for (int c = 0; c < s; ++c) acc = fma(R[a + s * c], old[c + s * b], acc);
    Rbar[e] = acc;
  }
}

// One mode's Q = Z U(:, 1:mu) (Z: I x s, U: s x mu, both column-major, ld I
// and s) with each column's largest-magnitude entry made positive (lowest row
// on ties), written as Q64 (I x mu), Qt (row stride ldqt, columns mu..ldqt-1
// zero; may be null) and Qcast (caller dtype; may be null); with Cd (may be
// null) also the sketch Z Rbar (I x s).  nb = (Qt ? ldqt : mu) + (Cd ? s : 0).
struct StabFinal {
  const double* Z;
  const double* U;
  const double* Rbar;
  double* Q64;
  double* Qt;
  void* Qcast;
  double* Cd;
  int64_t I;
  int s, mu, ldqt, nb;
};
struct StabFinals {
  StabFinal j[kStabMaxJobs];
};

// Grid (max nb, jobs).  Workgroups k < mu of job y produce its column k,
// mu <= k < ldqt clear Qt's padding column k, and (with Cd) ldqt + c write
// column c of the sketch; k >= nb have nothing to do.
static __global__ void __launch_bounds__(kStabNT)
k_stab_final(StabFinals jobs, int cast_f32) {
  __shared__ double babs[kStabNT], bval[kStabNT];
  __shared__ int64_t bidx[kStabNT];
  const StabFinal& jb = jobs.j[blockIdx.y];
  const int k = blockIdx.x;
  if (k >= jb.nb) return;  // the whole workgroup
  const double* __restrict__ Z = jb.Z;
  const double* __restrict__ U = jb.U;
  const double* __restrict__ Rbar = jb.Rbar;
  double* __restrict__ Q64 = jb.Q64;
  double* __restrict__ Qt = jb.Qt;
  void* __restrict__ Qcast = jb.Qcast;
  double* __restrict__ Cd = jb.Cd;
  const int64_t I = jb.I;
  const int s = jb.s, mu = jb.mu, ldqt = jb.ldqt;
  const int t = threadIdx.x;
  const int lq = Qt ? ldqt : mu;
  if (k >= lq) {  // a column of the sketch Z Rbar
    const int c = k - lq;
    for (int64_t i = t; i < I; i += kStabNT) {
      double acc = 0.0;
      for (int e = 0; e < s; ++e) acc = fma(Z[i + I * e], Rbar[e + (int64_t)s * c], acc);
      Cd[i + I * c] = acc;
    }
    return;
  }
  if (k >= mu) {
    for (int64_t i = t; i < I; i += kStabNT) Qt[i * ldqt + k] = 0.0;
    return;
  }
  auto entry = [&](int64_t i) {
    double acc = 0.0;
    for (int e = 0; e < s; ++e) acc = fma(Z[i + I * e], U[e + (int64_t)s * k], acc);
    return acc;
  };
  double ba = -1.0, bv = 0.0;
  int64_t bi = 0;
  for (int64_t i = t; i < I; i += kStabNT) {
    const double v = entry(i);
    if (fabs(v) > ba) {  // rows visited in increasing order: ties keep the lowest
      ba = fabs(v);
      bv = v;
      bi = i;
    }
  }
  babs[t] = ba;
  bval[t] = bv;
  bidx[t] = bi;
  __syncthreads();
  for (int w = kStabNT / 2; w > 0; w >>= 1) {
    if (t < w) {
      const double oa = babs[t + w];
      const int64_t oi = bidx[t + w];
      if (oa > babs[t] || (oa == babs[t] && oi < bidx[t])) {
        babs[t] = oa;
        bval[t] = bval[t + w];
        bidx[t] = oi;
      }
    }
    __syncthreads();
  }
  const double sg = bval[0] < 0.0 ? -1.0 : 1.0;
  for (int64_t i = t; i < I; i += kStabNT) {
    const double v = sg * entry(i);
    Q64[i + I * k] = v;
    if (Qt) Qt[i * ldqt + k] = v;
    if (Qcast) {
      if (cast_f32) static_cast<float*>(Qcast)[i + I * k] = (float)v;
      else static_cast<double*>(Qcast)[i + I * k] = v;
    }
  }
}

}  // namespace trk

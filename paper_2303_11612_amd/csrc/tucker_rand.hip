// Host side of the library: argument validation, workspace planning, the
// per-mode launch sequences of randomized T-HOSVD (Alg. 1 / Alg. 4) and
// ST-HOSVD (Alg. 2 / Alg. 5), and the exported C ABI of tucker_rand.h.
//
// Nothing here allocates device memory; every buffer comes from the caller's
// workspace.  All launches go to the caller's stream and no call waits on the
// device, so a whole decomposition can be enqueued (or captured) at once.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "tr_factor.hpp"
#include "tr_kernels.hpp"
#include "tr_factor_rf.hpp"
#include "tr_power.hpp"
#include "tr_lowp.hpp"
#include "tr_sparse.hpp"
#include "tr_stab.hpp"
#include "tr_norms.hpp"
#include "tr_host.hpp"
#include "tucker_rand.h"

namespace {

using namespace trh;
using trk::kNT;

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// ---------------------------------------------------------------------------
// Kernel timer: a pool of event pairs recorded around selected launches.
// ---------------------------------------------------------------------------
struct TimedLaunch {
  int cls;
  int mode;
  hipEvent_t start, stop;
};

}  // namespace

struct tr_timer {
  uint32_t mask = 0;
  std::vector<hipEvent_t> pool;  // 2 * capacity events
  std::vector<TimedLaunch> used;
};

namespace {

struct TimeScope {
  tr_timer* t = nullptr;
  hipStream_t st = nullptr;
  int idx = -1;
  TimeScope(tr_timer* timer, int cls, int mode, hipStream_t stream) : st(stream) {
    if (!timer || !(timer->mask & (1u << cls))) return;
    const size_t k = timer->used.size();
    if (2 * k + 1 >= timer->pool.size()) return;
    t = timer;
    idx = (int)k;
    TimedLaunch tl{cls, mode, timer->pool[2 * k], timer->pool[2 * k + 1]};
    timer->used.push_back(tl);
    (void)hipEventRecord(tl.start, st);
  }
  ~TimeScope() {
    if (t) (void)hipEventRecord(t->used[idx].stop, st);
  }
};

// ---------------------------------------------------------------------------
// Compile-time widths: a row of Q^T or of the sketch is padded with zeros to
// the next width in this list, which the kernels are instantiated for.
// ---------------------------------------------------------------------------
constexpr int kWidths[] = {4, 8, 12, 16, 20, 24, 32, 40, 48, 64, 80, 96, 112, 128};
inline int pad_width(int64_t m) {
  for (int w : kWidths)
    if (m <= w) return w;
  return 0;
}

// Power steps: k_pw_w (one block per 16 columns) then k_pw_y over row tiles
// of 32 and pw_splits(I, J) column ranges, whose partial sketches
// k_reduce_parts adds.  W is J x pw_width(s), row-major.
inline int pw_nkt(int64_t s) { return (int)cdiv(s, 16); }
inline int64_t pw_width(int64_t s) { return 16 * cdiv(s, 16); }
constexpr int kPwMT = 2;
inline int64_t pw_itiles(int64_t I) { return cdiv(I, 16 * kPwMT); }
inline int64_t pw_splits(int64_t I, int64_t J) {
  // about four blocks per compute unit, at least 64 columns per range; one
  // range up to 128 columns (the product then writes the sketch itself and
  // the step needs no reduction launch)
  if (J <= 128) return 1;
  return std::max<int64_t>(1, std::min<int64_t>(cdiv(1024, pw_itiles(I)), cdiv(J, 64)));
}
// Number of partial sketches a power step on this source produces (at most).
inline int64_t power_parts(int64_t I, int64_t J, int64_t s) {
  const int64_t ns = pw_splits(I, J);
  const int64_t two = cdiv(J, cdiv(J, ns));
  return pw_fused_ok(I, J, s) ? std::max(two, pw_fused_blocks(J)) : two;
}

// Views with few columns split their rows over blocks (k_ttm_split) so that
// about 512 blocks run; 1 means the one-pass kernels.
inline int64_t ttm_splits(int64_t J, int64_t I) {
  const int64_t bx = cdiv(J, kNT);
  if (bx >= 256 || I < 32) return 1;
  return std::max<int64_t>(1, std::min<int64_t>(cdiv(512, bx), I / 16));
}

inline int factor_sm(int64_t s) {
  return s <= 16 ? 16 : (s <= 32 ? 32 : (s <= 64 ? 64 : 128));
}
// sketch widths above 64 (up to 128): plain power scheme in native precision
// only, factor kernel kGlb128 with its s x s matrices in global scratch
constexpr int64_t kMaxSketch = 128;
inline bool wide_sketch(int64_t s) { return s > 64; }
constexpr size_t kMaxLds = 163840;

// LDS bytes of the factor kernel; `global_mats` keeps the I x s and I x mu
// working matrices in global scratch instead.
inline size_t factor_lds_bytes(int64_t I, int64_t s, int64_t mu, bool global_mats) {
  switch (factor_sm(s)) {
    case 16: return trk::FactorShape<16>::lds_bytes((int)I, (int)s, (int)mu, global_mats);
    case 32: return trk::FactorShape<32>::lds_bytes((int)I, (int)s, (int)mu, global_mats);
    case 64: return trk::FactorShape<64>::lds_bytes((int)I, (int)s, (int)mu, global_mats);
    default: return trk::FactorShape<128>::lds_bytes((int)I, (int)s, (int)mu, true);
  }
}
inline bool factor_in_lds(int64_t I, int64_t s, int64_t mu) {
  return !wide_sketch(s) && factor_lds_bytes(I, s, mu, false) <= kMaxLds;
}
inline bool factor_supported(int64_t I, int64_t s) {
  return s >= 1 && s <= kMaxSketch && I <= (1 << 24);
}
// global scratch of the wide factor variant (its two s x s matrices)
inline size_t factor_wide_bytes(int64_t s) {
  return wide_sketch(s) ? trk::FactorShape<128>::wide_scratch_bytes() : 0;
}

inline size_t lp_esz(int prec) { return prec == TR_PREC_FP8E4M3 ? 1 : 2; }

// ---------------------------------------------------------------------------
// Plan: per-mode shapes and the workspace layout.
// ---------------------------------------------------------------------------
struct ModePlan {
  int64_t L, I, R, J;   // 3-D view of the tensor the mode is computed from
  int64_t s, mu, T;     // sketch width, rank, samples (T = 0: exact)
  int sw, muw;          // padded widths of the sketch rows and of Q^T rows
  size_t oFw = 0;       // wide factor scratch (s > 64)
  bool sampled;
  bool src_f64;         // the tensor of this mode is float64
  bool intermediate;    // ... and the library's own shrunk tensor (ST-HOSVD, n > 0)
  bool lp;              // power products in the low-precision format (the
                        // caller's tensor or samples of it; never an intermediate)
};

struct Plan {
  int N = 0;
  bool sthosvd = false;
  int dtype = TR_F64;
  int prob = TR_PROB_NONE;
  int q = 1;
  uint64_t seed = 0;
  int64_t dims[TR_MAX_ORDER];
  ModePlan m[TR_MAX_ORDER];
  // workspace offsets (bytes)
  size_t oY, oYt, oZ, oPart, oNorms, oW, oCdf, oBsum, oIdx, oScale, oScale2, oCp,
      oMax, oSig, oX0, oX1, oCore, oSplit, total;
  // low-precision power steps
  int prec = TR_PREC_NATIVE;
  size_t oYq = 0, oTau = 0, oPartLp = 0, oCq = 0, oOmega = 0, oXmax = 0;
  size_t oQ[TR_MAX_ORDER], oQt[TR_MAX_ORDER];
  // T-HOSVD: every mode's sketch and singular values are kept until the
  // factorizations of all modes run in one launch
  size_t oYn[TR_MAX_ORDER] = {}, oSign[TR_MAX_ORDER] = {};
  // every mode's Gaussian G_n (I x s) and its zero-padded row-major copy
  // (I x sw), drawn in one launch before the first mode
  size_t oGs[TR_MAX_ORDER] = {}, oYts[TR_MAX_ORDER] = {};
  // power scheme with the triangular factors accumulated (tr_stab.hpp):
  // TR_FLAG_STABILIZED_POWER, and always for low precision with q > 1
  bool racc = false;
  bool fused = true;  // one-sweep power steps allowed (TR_FLAG_UNFUSED_POWER clears it)
  // related forms (Alg. 6 / Alg. 7): Q_n = P_n U_n with U_n from P_n^T A_(n)
  bool related = false;
  // per mode: orthonormal iterate Z (I x s), factor scratch (I x s), R_i and
  // Rbar (s x s), the factor U' of Rbar (s x mu), singular-value scratch (s)
  size_t oZn[TR_MAX_ORDER] = {}, oGA[TR_MAX_ORDER] = {}, oRst[TR_MAX_ORDER] = {},
         oRbar[TR_MAX_ORDER] = {}, oUp[TR_MAX_ORDER] = {}, oSgs[TR_MAX_ORDER] = {};
  // partial sums of ||A||^2 for the norms / RE diagnostics, and a small
  // output slot (||A||^2 read back by the fixed-precision driver)
  size_t oNparts = 0, oNout = 0;
  size_t splitBytes = 0;  // capacity of the split-rows scratch
};

// Validates and fills the plan; returns TR_OK or an error code.
int make_plan(const tr_params* p, int dtype, bool sthosvd, Plan* P) {
  if (!p || !P) return TR_EINVAL;
  if (dtype != TR_F64 && dtype != TR_F32) return TR_EINVAL;
  if (p->order < 1 || p->order > TR_MAX_ORDER || !p->dims || !p->ranks) return TR_EINVAL;
  if (p->oversample < 0 || p->power < 1) return TR_EINVAL;
  if (p->prob != TR_PROB_NONE && p->prob != TR_PROB_NEARLY_OPTIMAL &&
      p->prob != TR_PROB_UNIFORM)
    return TR_EINVAL;
  if (p->prob != TR_PROB_NONE && !p->samples) return TR_EINVAL;
  if (p->flags & ~(uint32_t)(TR_FLAG_STABILIZED_POWER | TR_FLAG_UNFUSED_POWER |
                             TR_FLAG_RELATED_FORM))
    return TR_EINVAL;
  if (p->precision != TR_PREC_NATIVE && p->precision != TR_PREC_BF16 &&
      p->precision != TR_PREC_FP8E4M3)
    return TR_EINVAL;
  const bool lp = p->precision != TR_PREC_NATIVE;
  P->prec = p->precision;
  P->racc = (p->flags & TR_FLAG_STABILIZED_POWER) != 0 || (lp && p->power > 1);
  P->fused = (p->flags & TR_FLAG_UNFUSED_POWER) == 0;
  P->related = (p->flags & TR_FLAG_RELATED_FORM) != 0;
  const int N = p->order;
  P->N = N;
  P->sthosvd = sthosvd;
  P->dtype = dtype;
  P->prob = p->prob;
  P->q = p->power;
  P->seed = p->seed;
  int64_t cur[TR_MAX_ORDER];
  for (int n = 0; n < N; ++n) {
    if (p->dims[n] < 1 || p->dims[n] > (int64_t)1 << 31) return TR_EINVAL;
    P->dims[n] = cur[n] = p->dims[n];
  }
  double total_el = 1.0;
  for (int n = 0; n < N; ++n) total_el *= (double)cur[n];
  if (total_el > 9.0e15) return TR_EINVAL;

  size_t maxIs = 0, maxZ = 0, maxPart = 0, maxJs = 0, maxT = 0, maxCp = 0, maxInter = 0,
         maxSplit = 0, maxYq = 0, maxPartLp = 0, maxCq = 0;
  bool any_lp = false, any_f64 = false;
  int64_t maxS = 0;
  for (int n = 0; n < N; ++n) {
    ModePlan& M = P->m[n];
    M.L = 1;
    M.R = 1;
    for (int k = 0; k < n; ++k) M.L *= cur[k];
    for (int k = n + 1; k < N; ++k) M.R *= cur[k];
    M.I = cur[n];
    M.J = M.L * M.R;
    M.mu = p->ranks[n];
    if (M.mu < 1 || M.mu > M.I || M.mu > M.J) return TR_EINVAL;
    M.s = std::min<int64_t>(M.mu + p->oversample, M.I);
    M.src_f64 = (dtype == TR_F64) || (sthosvd && n > 0);
    M.intermediate = sthosvd && n > 0;
    M.T = 0;
    M.sampled = false;
    if (p->prob != TR_PROB_NONE) {
      if (p->samples[n] < 1) return TR_EINVAL;
      if (p->samples[n] <= M.J) {
        M.sampled = true;
        M.T = p->samples[n];
      }
    }
    if (!factor_supported(M.I, M.s)) return TR_ENOTSUP;
    if (wide_sketch(M.s) && (lp || P->racc || P->related)) return TR_ENOTSUP;
    // low precision rounds the caller's data only: an ST-HOSVD intermediate
    // (float64, at most mu_1/I_1 of the input) keeps its energy in few
    // columns, so rounding it would turn the format's roundoff directly into
    // subspace error, for little traffic saved
    M.lp = lp && !M.intermediate;
    any_lp = any_lp || M.lp;
    any_f64 = any_f64 || !M.lp;
    if (M.lp) {
      if (!lp_supported(M.I, M.s)) return TR_ENOTSUP;
      const int64_t jl = M.sampled ? M.T : M.J;
      if (!M.sampled && M.J >= ((int64_t)1 << 32)) return TR_ENOTSUP;
      const int64_t Ip = lp_ip(M.I), SP = 16 * lp_nkt(M.s);
      maxYq = std::max(maxYq, (size_t)(SP * Ip));
      maxPartLp = std::max(maxPartLp, (size_t)(lp_blocks(M.I, M.s, jl) * SP * Ip));
      if (M.sampled) maxCq = std::max(maxCq, (size_t)(Ip * M.T));
    }
    M.sw = pad_width(M.s);
    M.muw = pad_width(M.mu);
    if (M.sw == 0 || M.muw == 0) return TR_ENOTSUP;
    const int64_t jsrc = M.sampled ? M.T : M.J;
    const int64_t lsrc = M.sampled ? 1 : M.L;
    const bool fsrc = M.src_f64;
    maxIs = std::max(maxIs, (size_t)(M.I * M.sw));
    (void)lsrc;
    (void)fsrc;
    maxZ = std::max(maxZ, (size_t)(jsrc * pw_width(M.s)));
    // the shrink of this mode reads the tensor the mode is computed from
    maxSplit = std::max(maxSplit, (size_t)(ttm_splits(M.J, M.I) * M.J * M.muw));
    maxPart = std::max(maxPart, (size_t)(power_parts(M.I, jsrc, M.s) * M.I * M.s));
    maxS = std::max(maxS, M.s);
    if (M.sampled) {
      maxJs = std::max(maxJs, (size_t)M.J);
      maxT = std::max(maxT, (size_t)M.T);
      maxCp = std::max(maxCp, (size_t)(M.I * M.T));
    }
    if (sthosvd) cur[n] = M.mu;  // the next mode sees the shrunk tensor
  }
  // intermediate tensors: after each shrink of the chain (the last one is the
  // core, kept in float64 before the cast to the caller's dtype)
  size_t core_el = 1;
  {
    int64_t shp[TR_MAX_ORDER];
    for (int n = 0; n < N; ++n) shp[n] = P->dims[n];
    for (int n = 0; n < N; ++n) {
      int64_t Jc = 1;
      for (int k2 = 0; k2 < N; ++k2)
        if (k2 != n) Jc *= shp[k2];
      maxSplit = std::max(maxSplit, (size_t)(ttm_splits(Jc, shp[n]) * Jc * P->m[n].muw));
      shp[n] = P->m[n].mu;
      size_t e = 1;
      for (int k = 0; k < N; ++k) e *= (size_t)shp[k];
      if (n + 1 < N) maxInter = std::max(maxInter, e);
      else core_el = e;
    }
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(std::max<size_t>(bytes, 8));
    return o;
  };
  P->oY = take(8 * maxIs);
  P->oYt = take(8 * maxIs);
  // the float64 power steps' W and partial sketches (unused in low precision)
  // (the related forms' Gram step is a float64 power step on the mode's tensor)
  if (P->related) {
    any_f64 = true;
    for (int n = 0; n < N; ++n) {
      const ModePlan& M = P->m[n];
      maxZ = std::max(maxZ, (size_t)(M.J * pw_width(M.s)));
      maxPart = std::max(maxPart, (size_t)(power_parts(M.I, M.J, M.s) * M.I * M.s));
    }
  }
  P->oZ = take(any_f64 ? 8 * maxZ : 8);
  P->oPart = take(any_f64 ? 8 * maxPart : 8);
  P->oNorms = take(8 * maxJs);
  P->oW = take(8 * maxJs);
  P->oCdf = take(8 * maxJs);
  P->oBsum = take(8 * (size_t)(cdiv((int64_t)maxJs, trk::kScanChunk) + 1));
  P->oIdx = take(8 * maxT);
  P->oScale = take(8 * maxT);
  P->oScale2 = take(8 * maxT);
  P->oCp = take(any_f64 ? 8 * maxCp : 8);
  P->oMax = take(8 * (size_t)N);  // one running maximum per mode
  for (int n = 0; n < N; ++n) {
    P->oGs[n] = take(8 * (size_t)(P->m[n].I * P->m[n].s));
    P->oYts[n] = take(8 * (size_t)(P->m[n].I * P->m[n].sw));
  }
  P->oSig = take(8 * (size_t)maxS);
  for (int n = 0; n < N; ++n) {
    P->oQ[n] = take(8 * (size_t)(P->m[n].I * P->m[n].mu));
    P->oQt[n] = take(8 * (size_t)(P->m[n].I * P->m[n].muw));
  }
  if (!sthosvd)
    for (int n = 0; n < N; ++n) {
      P->oYn[n] = take(8 * (size_t)(P->m[n].I * P->m[n].s));
      P->oSign[n] = take(8 * (size_t)P->m[n].s);
    }
  for (int n = 0; n < N; ++n)
    if (wide_sketch(P->m[n].s)) P->m[n].oFw = take(factor_wide_bytes(P->m[n].s));
  if (P->racc || P->related)
    for (int n = 0; n < N; ++n) {
      const size_t Is = (size_t)(P->m[n].I * P->m[n].s), ss = (size_t)(P->m[n].s * P->m[n].s);
      P->oZn[n] = take(8 * Is);
      P->oGA[n] = take(8 * Is);
      P->oRst[n] = take(8 * ss);
      P->oRbar[n] = take(8 * ss);
      P->oUp[n] = take(8 * (size_t)(P->m[n].s * P->m[n].mu));
      P->oSgs[n] = take(8 * (size_t)P->m[n].s);
    }
  P->oX0 = take(8 * maxInter);
  P->oX1 = take(8 * maxInter);
  P->oCore = take(8 * core_el);
  P->oSplit = take(8 * maxSplit);
  P->splitBytes = 8 * maxSplit;
  P->oNparts = take(8 * (size_t)trk::kNormMaxParts);
  P->oNout = take(8 * 4);
  if (any_lp) {
    P->oYq = take(2 * maxYq);
    P->oTau = take(4 * 64);
    P->oPartLp = take(4 * maxPartLp);
    P->oCq = take(lp_esz(P->prec) * maxCq);
    P->oOmega = take(4 * maxT);
    P->oXmax = take(4);
  }
  P->total = off;
  return TR_OK;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// ---------------------------------------------------------------------------
// Launchers (all asynchronous on `st`).
// ---------------------------------------------------------------------------
int launch_fill_f64(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return TR_OK;
  hipLaunchKernelGGL(trk::k_fill_f64, dim3((unsigned)cdiv(n, kNT)), dim3(kNT), 0, st, p, n, v);
  return check_launch();
}

// G (I x s) and its row-major copy Gt (optional) with zero padding to stride
// ldgt.
int launch_gaussian(double* G, double* Gt, int64_t I, int64_t s, int64_t ldgt, int mode,
                    uint64_t seed, hipStream_t st) {
  if (Gt && ldgt > s) TR_TRY(launch_fill_f64(Gt, I * ldgt, 0.0, st));
  const int64_t blocks4 = cdiv(I * s, 4);
  hipLaunchKernelGGL(trk::k_gaussian, dim3((unsigned)cdiv(blocks4, kNT)), dim3(kNT), 0, st,
                     G, Gt, I, s, ldgt, (uint64_t)mode, seed);
  return check_launch();
}

// Norms of the caller's tensor sum each column's rows in order (one thread
// per column), which makes them bit-exact; `seg_ok` (the library's own shrunk
// tensor) lets a view with few columns split each column over 8 threads.
template <typename T>
int launch_colnorms_t(const T* X, int64_t L, int64_t I, int64_t R, double* norms,
                      unsigned long long* maxb, hipStream_t st, bool seg_ok) {
  const int64_t J = L * R;
  const dim3 grid((unsigned)cdiv(J, kNT));
  constexpr int kSeg = 8;
  if (seg_ok && J < 64 * (int64_t)kNT && I >= 4 * kSeg)
    hipLaunchKernelGGL((trk::k_colnorms_seg<T, kSeg>), dim3((unsigned)cdiv(J, kNT / kSeg)),
                       dim3(kNT), 0, st, X, L, I, R, norms, maxb);
  else if (L == 1 && (I * (int64_t)sizeof(T)) % 16 == 0 &&
           reinterpret_cast<uintptr_t>(X) % 16 == 0)
    hipLaunchKernelGGL((trk::k_colnorms_l1<T, true>), grid, dim3(kNT), 0, st, X, I, J, norms,
                       maxb);
  else if (L == 1)
    hipLaunchKernelGGL((trk::k_colnorms_l1<T, false>), grid, dim3(kNT), 0, st, X, I, J, norms,
                       maxb);
  else
    hipLaunchKernelGGL(trk::k_colnorms_ln<T>, grid, dim3(kNT), 0, st, X, L, I, R, norms, maxb);
  return check_launch();
}

int launch_colnorms(bool f64, const void* X, int64_t L, int64_t I, int64_t R, double* norms,
                    unsigned long long* maxb, hipStream_t st, bool seg_ok = false) {
  return f64 ? launch_colnorms_t((const double*)X, L, I, R, norms, maxb, st, seg_ok)
             : launch_colnorms_t((const float*)X, L, I, R, norms, maxb, st, seg_ok);
}

int launch_fill(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t st) {
  hipLaunchKernelGGL(trk::k_fill_u64, dim3((unsigned)cdiv(n, kNT)), dim3(kNT), 0, st, p, n, v);
  return check_launch();
}

size_t sample_ws_bytes(int64_t J) {
  return align_up(8 * (size_t)J) * 2 + align_up(8 * (size_t)(cdiv(J, trk::kScanChunk) + 1)) +
         align_up(8);
}

// w, cdf: [J] u64; bsum: [ceil(J/1024)+1] u64.  norms/max_bits only for
// nearly-optimal probabilities.
int launch_sample(const double* norms, const unsigned long long* maxb, int64_t J, int64_t T,
                  int prob, uint64_t seed, int mode, unsigned long long* w,
                  unsigned long long* cdf, unsigned long long* bsum, int64_t* idx,
                  double* scale, double* scale2, uint32_t* status, hipStream_t st) {
  const int uniform = prob == TR_PROB_UNIFORM;
  if (!uniform) {
    int cl2 = 0;
    while (((int64_t)1 << cl2) < J) ++cl2;
    const int kexp = 60 - cl2;
    if (J <= trk::kSmallSampleJ) {
      hipLaunchKernelGGL(trk::k_sample_small, dim3((unsigned)cdiv(T, kNT)), dim3(kNT), 0, st,
                         norms, J, maxb, kexp, T, seed, (uint64_t)mode, w, cdf, idx, scale,
                         scale2, status);
      return check_launch();
    }
    const int64_t nb = cdiv(J, trk::kScanChunk);
    hipLaunchKernelGGL(trk::k_weights, dim3((unsigned)nb), dim3(kNT), 0, st, norms, J, maxb,
                       kexp, 0, w, bsum, status);
    TR_TRY(check_launch());
    // up to 1024 blocks, each block of k_cdf sums the block totals before it
    // (at most 2^20 loads in all); beyond that one workgroup scans them first
    const int raw = nb <= 1024 ? 1 : 0;
    if (!raw) {
      hipLaunchKernelGGL(trk::k_scan_bsum, dim3(1), dim3(1024), 0, st, bsum, nb);
      TR_TRY(check_launch());
    }
    hipLaunchKernelGGL(trk::k_cdf, dim3((unsigned)nb), dim3(kNT), 0, st, w, bsum, raw, J, cdf);
    TR_TRY(check_launch());
  }
  hipLaunchKernelGGL(trk::k_draw, dim3((unsigned)cdiv(T, kNT)), dim3(kNT), 0, st, cdf, J, T,
                     seed, (uint64_t)mode, uniform, idx, scale, scale2);
  return check_launch();
}

// perm_ws (optional, 4 T bytes): with it an inner mode of 64..8192 slabs
// whose slab rows span 512 bytes or more gathers its samples in slab order, a
// slab's samples on one XCD (the 512x512x256 bumps tensor's mode 2: 77.3 ->
// 39.2 us plus 12 us for the ordering; with shorter rows, as the 80-byte rows
// of the 400^3 benchmark's mode 2, the samples already share their lines and
// the ordering costs more than it saves: 12.7 against 9.1 + 7.3 us).
int slab_order(bool f64, int64_t L, int64_t R, const int64_t* idx, int64_t T, int* perm_ws,
               int** perm, hipStream_t st) {
  *perm = nullptr;
  const int64_t row_bytes = L * (f64 ? 8 : 4);
  if (perm_ws && row_bytes >= 512 && R >= 64 && R <= trk::kBucketR && T <= trk::kBucketT &&
      L * R < ((int64_t)1 << 32)) {
    hipLaunchKernelGGL(trk::k_bucket_samples, dim3(1), dim3(1024), 0, st, idx, T, L, R, perm_ws);
    TR_TRY(check_launch());
    *perm = perm_ws;
  }
  return TR_OK;
}

int launch_gather(bool f64, const void* X, int64_t L, int64_t I, const int64_t* idx, int64_t T,
                  void* Cp, hipStream_t st, int64_t R = 0, int* perm_ws = nullptr) {
  int* perm = nullptr;
  TR_TRY(slab_order(f64, L, R, idx, T, perm_ws, &perm, st));
  const dim3 grid((unsigned)(perm ? 8 * cdiv(T, 8) : T), (unsigned)cdiv(I, kNT));
  if (f64)
    hipLaunchKernelGGL(trk::k_gather<double>, grid, dim3(kNT), 0, st, (const double*)X, L, I,
                       idx, (double*)Cp, perm, T);
  else
    hipLaunchKernelGGL(trk::k_gather<float>, grid, dim3(kNT), 0, st, (const float*)X, L, I,
                       idx, (float*)Cp, perm, T);
  return check_launch();
}

// Mode-1 shrink on the matrix cores (mu <= 32, I a multiple of 4, 16-byte
// aligned source, padded Q^T within LDS); false otherwise (the caller then
// uses the vector kernels).  The batch B of 16-row steps is the one of
// 4, 5, 6, 8 that pads the row count least.
inline int ttm1_batch(int64_t I) {
  const int64_t ns = cdiv(I, 16);
  int best = 8;
  int64_t bestpad = cdiv(ns, 8) * 8;
  for (int b : {6, 5, 4}) {
    const int64_t pad = cdiv(ns, b) * b;
    if (pad < bestpad) {
      best = b;
      bestpad = pad;
    }
  }
  return best;
}

// bytes of the Q^T tile a block of the mode-1 MFMA shrink stages in LDS
inline size_t ttm1_lds(int64_t I, int B, int NKT) {
  return 8 * (size_t)(cdiv(cdiv(I, 16), B) * B * 16) * 16 * NKT;
}

template <typename Tin, int NKT, int B, bool STR, int kW>
void ttm1_mfma_k(const Tin* X, int64_t L, int64_t I, int64_t R, const double* Qt, int width,
                 int kout, double* Y, hipStream_t st) {
  // kW waves share one Q^T tile: the LDS allows at most three tiles per
  // compute unit, and twice the waves keep twice the loads in flight (16
  // where a tile leaves room for one block per compute unit)
  const size_t lds = ttm1_lds(I, B, NKT);
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)&trk::k_ttm1_mfma<Tin, NKT, B, STR, kW>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  const int64_t ntile = cdiv(R, 16);
  // persistent blocks: as many as fit three to a compute unit (by the Q^T
  // tile in LDS), capped by the tiles there are
  // and by the registers (a block that is not resident from the start would
  // run its share of tiles after the others)
  static const int64_t reg_cu = [] {
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, (const void*)&trk::k_ttm1_mfma<Tin, NKT, B, STR, kW>) !=
            hipSuccess ||
        fa.numRegs <= 0)
      return (int64_t)1;
    const int64_t per_simd = 512 / (8 * cdiv(fa.numRegs, 8));
    return std::max<int64_t>(1, 4 * per_simd / kW);
  }();
  const int64_t per_cu = std::min<int64_t>(reg_cu, lds <= 53248 ? 3 : (lds <= 81920 ? 2 : 1));
  const int64_t nblk = std::max<int64_t>(1, std::min<int64_t>(256 * per_cu, cdiv(ntile, kW)));
  hipLaunchKernelGGL((trk::k_ttm1_mfma<Tin, NKT, B, STR, kW>), dim3((unsigned)nblk),
                     dim3(kW * trk::kWave), lds, st, X, L, I, R, Qt, width, kout, Y);
}

template <typename Tin, int NKT, bool STR, int kW>
void ttm1_mfma_w(const Tin* X, int64_t L, int64_t I, int64_t R, const double* Qt, int width,
                 int kout, double* Y, hipStream_t st) {
  switch (ttm1_batch(I)) {
    case 4: ttm1_mfma_k<Tin, NKT, 4, STR, kW>(X, L, I, R, Qt, width, kout, Y, st); break;
    case 5: ttm1_mfma_k<Tin, NKT, 5, STR, kW>(X, L, I, R, Qt, width, kout, Y, st); break;
    case 6: ttm1_mfma_k<Tin, NKT, 6, STR, kW>(X, L, I, R, Qt, width, kout, Y, st); break;
    default: ttm1_mfma_k<Tin, NKT, 8, STR, kW>(X, L, I, R, Qt, width, kout, Y, st); break;
  }
}

template <typename Tin, int NKT, bool STR>
void ttm1_mfma_b(const Tin* X, int64_t L, int64_t I, int64_t R, const double* Qt, int width,
                 int kout, double* Y, hipStream_t st) {
  // a 32-wide tile of more than 80 KB fits once per compute unit: sixteen
  // waves then share it (four per SIMD rather than two, for the matrix
  // instructions' latency; measured on 512 x 131072 float32, mu = 30)
  if constexpr (NKT == 2) {
    if (ttm1_lds(I, ttm1_batch(I), NKT) > 81920) {
      ttm1_mfma_w<Tin, NKT, STR, 16>(X, L, I, R, Qt, width, kout, Y, st);
      return;
    }
  }
  ttm1_mfma_w<Tin, NKT, STR, 8>(X, L, I, R, Qt, width, kout, Y, st);
}

// Y[k + kout j] = sum_i Qt[i width + k] X_(n)(i, j) on the matrix cores, for
// the columns j < J of a plain I x J matrix (L == 1: 16-byte loads, I a
// multiple of 4, X 16-byte aligned) or of an L x I x R view (strided loads;
// the caller must want the outputs in this layout).  False if not applicable.
template <typename Tin>
bool ttm1_mfma(const Tin* X, int64_t L, int64_t I, int64_t J, const double* Qt, int width,
               int kout, double* Y, hipStream_t st) {
  const bool str = L > 1;
  if (kout > 32) return false;
  if (!str && (I % 4 != 0 || (reinterpret_cast<uintptr_t>(X) % 16) != 0)) return false;
  if (I < 4) return false;
  const int nkt = (int)cdiv(kout, 16);
  const int b = ttm1_batch(I);
  if (ttm1_lds(I, b, nkt) > 131072) return false;
  if (str) {
    if (nkt == 1) ttm1_mfma_b<Tin, 1, true>(X, L, I, J, Qt, width, kout, Y, st);
    else ttm1_mfma_b<Tin, 2, true>(X, L, I, J, Qt, width, kout, Y, st);
  } else {
    if (nkt == 1) ttm1_mfma_b<Tin, 1, false>(X, 1, I, J, Qt, width, kout, Y, st);
    else ttm1_mfma_b<Tin, 2, false>(X, 1, I, J, Qt, width, kout, Y, st);
  }
  return true;
}

// Returns true when the kernel it ran also wrote the copy yc (k_ttm_seg).
template <typename Tin, int MU>
bool ttm_w(const Tin* X, int64_t L, int64_t I, int64_t R, const double* Qt, int kout,
           const double* colscale, double* Y, double* split, void* yc, int yc_f32,
           hipStream_t st) {
  const int64_t J = L * R;
  const dim3 grid((unsigned)cdiv(J, kNT));
  const int64_t ns = ttm_splits(J, I);
  if constexpr (MU <= 24) {
    if (ns > 1) {
      // segments combined inside the workgroup: one launch, no partials; the
      // fewer the columns, the more (and shorter) segments per column, so that
      // a view of a few hundred columns still spreads over the chip
      if (J < 1024 && I >= 256)
        hipLaunchKernelGGL((trk::k_ttm_seg<Tin, MU, 64>), dim3((unsigned)cdiv(J, kNT / 64)),
                           dim3(kNT), 0, st, X, L, I, R, Qt, kout, colscale, Y, yc, yc_f32);
      else if (J < 8192 && I >= 128)
        hipLaunchKernelGGL((trk::k_ttm_seg<Tin, MU, 32>), dim3((unsigned)cdiv(J, kNT / 32)),
                           dim3(kNT), 0, st, X, L, I, R, Qt, kout, colscale, Y, yc, yc_f32);
      else
        hipLaunchKernelGGL((trk::k_ttm_seg<Tin, MU, 16>), dim3((unsigned)cdiv(J, kNT / 16)),
                           dim3(kNT), 0, st, X, L, I, R, Qt, kout, colscale, Y, yc, yc_f32);
      return yc != nullptr;
    }
  }
  if (ns > 1 && split) {
    const int64_t ich = cdiv(I, ns);
    const int64_t nsu = cdiv(I, ich);
    hipLaunchKernelGGL((trk::k_ttm_split<Tin, MU>), dim3((unsigned)cdiv(J, kNT), (unsigned)nsu),
                       dim3(kNT), 0, st, X, L, I, R, Qt, ich, split);
    hipLaunchKernelGGL(trk::k_sum_splits, dim3((unsigned)cdiv(J * kout, kNT)), dim3(kNT), 0, st,
                       split, nsu, L, R, MU, kout, colscale, Y);
    return false;
  }
  if (L == 1 && !colscale && ttm1_mfma(X, 1, I, R, Qt, MU, kout, Y, st)) return false;
  if (L == 1)
    hipLaunchKernelGGL((trk::k_ttm_l1<Tin, MU>), grid, dim3(kNT), 0, st, X, I, R, Qt, kout,
                       colscale, Y);
  else
    hipLaunchKernelGGL((trk::k_ttm_ln<Tin, MU>), grid, dim3(kNT), 0, st, X, L, I, R, Qt, kout,
                       colscale, Y);
  return false;
}

// Y = X x_n Q^T with Qt of row stride `width` (zero-padded); outputs k < kout.
// yc (optional): where a copy of Y is wanted (float32 if yc_f32); *yc_done
// tells whether the kernel wrote it (else the caller casts Y).
template <typename Tin>
int ttm_t(const Tin* X, int64_t L, int64_t I, int64_t R, const double* Qt, int width, int kout,
          const double* colscale, double* Y, double* split, hipStream_t st,
          void* yc = nullptr, int yc_f32 = 0, bool* yc_done = nullptr) {
  bool done = false;
  // one instance per padded row width
  auto run = [&](auto w) -> bool {
    return ttm_w<Tin, decltype(w)::value>(X, L, I, R, Qt, kout, colscale, Y, split, yc, yc_f32,
                                          st);
  };
  switch (width) {
    case 4: done = run(std::integral_constant<int, 4>{}); break;
    case 8: done = run(std::integral_constant<int, 8>{}); break;
    case 12: done = run(std::integral_constant<int, 12>{}); break;
    case 16: done = run(std::integral_constant<int, 16>{}); break;
    case 20: done = run(std::integral_constant<int, 20>{}); break;
    case 24: done = run(std::integral_constant<int, 24>{}); break;
    case 32: done = run(std::integral_constant<int, 32>{}); break;
    case 40: done = run(std::integral_constant<int, 40>{}); break;
    case 48: done = run(std::integral_constant<int, 48>{}); break;
    case 64: done = run(std::integral_constant<int, 64>{}); break;
    case 80: done = run(std::integral_constant<int, 80>{}); break;
    case 96: done = run(std::integral_constant<int, 96>{}); break;
    case 112: done = run(std::integral_constant<int, 112>{}); break;
    case 128: done = run(std::integral_constant<int, 128>{}); break;
    default: return TR_ENOTSUP;
  }
  if (yc_done) *yc_done = done;
  return check_launch();
}

// split: scratch for the split-rows form (ttm_splits(J, I) * J * width
// doubles), or NULL to always use the one-pass kernels.
int launch_ttm(bool in_f64, const void* X, int64_t L, int64_t I, int64_t R, const double* Qt,
               int width, int kout, const double* colscale, double* Y, double* split,
               hipStream_t st, void* yc = nullptr, int yc_f32 = 0, bool* yc_done = nullptr) {
  if (in_f64)
    return ttm_t((const double*)X, L, I, R, Qt, width, kout, colscale, Y, split, st, yc, yc_f32,
                 yc_done);
  return ttm_t((const float*)X, L, I, R, Qt, width, kout, colscale, Y, split, st, yc, yc_f32,
               yc_done);
}

int launch_cast(const double* src, int64_t n, bool to_f32, void* dst, hipStream_t st) {
  if (to_f32)
    hipLaunchKernelGGL(trk::k_cast<float>, dim3((unsigned)cdiv(n, kNT)), dim3(kNT), 0, st, src,
                       n, (float*)dst);
  else
    hipLaunchKernelGGL(trk::k_cast<double>, dim3((unsigned)cdiv(n, kNT)), dim3(kNT), 0, st, src,
                       n, (double*)dst);
  return check_launch();
}

// gidx (optional, L == 1): column j of the product is column gidx[j] of X,
// which then has at least max gidx + 1 columns (the sampled C' read in place).
// With one column range the product writes Y, Yt (row stride sw; Yt's reads
// are done by then) and the status itself and *nparts is 0: no reduction.
template <typename Tin, int NKT>
int pw_step(const Tin* X, int64_t L, int64_t I, int64_t R, const double* colw, double* Yt,
            int sw, int s, double* W, double* part, int64_t* nparts, hipStream_t st,
            const int64_t* gidx, double* Y, uint32_t* status) {
  const int64_t J = L * R;
  // W = X^T Y has the shape of the mode-1 shrink with Q^T = Yt: the
  // persistent MFMA kernel (Yt staged in LDS, next tile in flight) when there
  // are no column weights and enough columns to occupy it (with few columns
  // k_pw_w's one-tile blocks, rows split over four waves, are faster)
  const bool many = cdiv(J, 16 * trk::kPwWaves) >= 1024;
  if (!gidx && !colw && many && ttm1_mfma(X, L, I, J, Yt, sw, 16 * NKT, W, st)) {
    TR_TRY(check_launch());
  } else if (many)
    // many columns: a tile per wave (no reduction across waves) still gives
    // at least four workgroups per compute unit
    hipLaunchKernelGGL((trk::k_pw_w<Tin, NKT, true>), dim3((unsigned)cdiv(J, 16 * trk::kPwWaves)),
                       dim3(trk::kPwWaves * trk::kWave), 0, st, X, L, I, R, colw, Yt, sw, W,
                       gidx);
  else
    hipLaunchKernelGGL((trk::k_pw_w<Tin, NKT>), dim3((unsigned)cdiv(J, 16)),
                       dim3(trk::kPwWaves * trk::kWave), 0, st, X, L, I, R, colw, Yt, sw, W,
                       gidx);
  TR_TRY(check_launch());
  const int64_t jper = cdiv(J, pw_splits(I, J));
  const int64_t ny = cdiv(J, jper);
  const bool direct = ny == 1;
  hipLaunchKernelGGL((trk::k_pw_y<Tin, NKT, kPwMT>), dim3((unsigned)pw_itiles(I), (unsigned)ny),
                     dim3(trk::kPwWaves * trk::kWave), 0, st, X, L, I, R, W, s, jper, part,
                     gidx, direct ? Y : nullptr, direct ? Yt : nullptr, sw,
                     direct ? status : nullptr);
  *nparts = direct ? 0 : ny;
  return check_launch();
}

template <typename Tin>
int pw_step_t(const Tin* X, int64_t L, int64_t I, int64_t R, const double* colw, double* Yt,
              int sw, int64_t s, double* W, double* part, int64_t* nparts, hipStream_t st,
              const int64_t* gidx, double* Y, uint32_t* status) {
  const int si = (int)s;
#define TR_PW_CASE(n)                                                                    \
  case n:                                                                                \
    return pw_step<Tin, n>(X, L, I, R, colw, Yt, sw, si, W, part, nparts, st, gidx, Y, \
                           status);
  switch (pw_nkt(s)) {
    TR_PW_CASE(1)
    TR_PW_CASE(2)
    TR_PW_CASE(3)
    TR_PW_CASE(4)
    TR_PW_CASE(5)
    TR_PW_CASE(6)
    TR_PW_CASE(7)
    TR_PW_CASE(8)
    default: return TR_ENOTSUP;
  }
#undef TR_PW_CASE
}

size_t power_ws_bytes(int64_t L, int64_t I, int64_t R, int64_t s, bool f64) {
  (void)f64;
  const int64_t J = L * R;
  const int sw = pad_width(s);
  return align_up(8 * (size_t)(J * pw_width(s))) + align_up(8 * (size_t)(power_parts(I, J, s) * I * s)) +
         align_up(8 * (size_t)(I * sw));
}

// C = (X_(n) D X_(n)^T)^q G by the two halves of Strategy A, starting from
// Yt = G^T (row stride sw, zero-padded).  Z, part: scratch.
// gidx (optional, L == 1): the product's column j is column gidx[j] of X
// (sampled columns read in place; not with the one-sweep kernel).
int run_power(bool f64, const void* X, int64_t L, int64_t I, int64_t R, const double* colw,
              int q, int64_t s, int sw, double* Y, double* Yt, double* Z, double* part,
              uint32_t* status, hipStream_t st, bool fused = true,
              const int64_t* gidx = nullptr) {
  for (int step = 0; step < q; ++step) {
    int64_t nused = 0;
    // one sweep with W kept on chip when the rows and the sketch are narrow
    const int rc = fused && !gidx
                       ? launch_pw_fused(f64, X, L, I, R, colw, Yt, sw, s, part, &nused, st)
                       : TR_ENOTSUP;
    if (rc != TR_OK && rc != TR_ENOTSUP) return rc;
    if (rc == TR_ENOTSUP) {
      if (f64)
        TR_TRY(pw_step_t((const double*)X, L, I, R, colw, Yt, sw, s, Z, part, &nused, st, gidx,
                         Y, status));
      else
        TR_TRY(pw_step_t((const float*)X, L, I, R, colw, Yt, sw, s, Z, part, &nused, st, gidx,
                         Y, status));
      if (nused == 0) continue;  // the product wrote Y and Yt
    }
    hipLaunchKernelGGL(trk::k_reduce_parts, dim3((unsigned)cdiv(I * s, kNT)), dim3(kNT), 0, st,
                       part, nused, I, (int)s, sw, Y, Yt, status);
    TR_TRY(check_launch());
  }
  return TR_OK;
}

// ---------------------------------------------------------------------------
// Low-precision power steps.
// ---------------------------------------------------------------------------
int launch_quant_y(int prec, const double* C, int64_t I, int64_t s, void* Cq, float* tau,
                   hipStream_t st) {
  const int Ip = (int)lp_ip(I), SP = 16 * lp_nkt(s);
  if (prec == TR_PREC_FP8E4M3)
    hipLaunchKernelGGL(trk::k_quant_y<trk::OpFp8>, dim3(SP), dim3(kNT), 0, st, C, I, (int)s, Ip,
                       (uint8_t*)Cq, tau);
  else
    hipLaunchKernelGGL(trk::k_quant_y<trk::OpBf16>, dim3(SP), dim3(kNT), 0, st, C, I, (int)s,
                       Ip, (uint16_t*)Cq, tau);
  return check_launch();
}

template <typename Tin>
int gather_lp_t(int prec, const Tin* X, int64_t L, int64_t I, const int64_t* idx, int64_t T,
                const double* scale2, void* Cq, float* omega, const int* perm, hipStream_t st) {
  const int Ip = (int)lp_ip(I);
  const dim3 grid((unsigned)(perm ? 8 * cdiv(T, 8) : T));
  if (prec == TR_PREC_FP8E4M3)
    hipLaunchKernelGGL((trk::k_gather_lp<Tin, trk::OpFp8>), grid, dim3(kNT), 0, st, X, L, I,
                       idx, Ip, scale2, (uint8_t*)Cq, omega, perm, T);
  else
    hipLaunchKernelGGL((trk::k_gather_lp<Tin, trk::OpBf16>), grid, dim3(kNT), 0, st, X, L, I,
                       idx, Ip, scale2, (uint16_t*)Cq, omega, perm, T);
  return check_launch();
}

int launch_gather_lp(int prec, bool f64, const void* X, int64_t L, int64_t I, const int64_t* idx,
                     int64_t T, const double* scale2, void* Cq, float* omega, hipStream_t st,
                     int64_t R = 0, int* perm_ws = nullptr) {
  int* perm = nullptr;
  TR_TRY(slab_order(f64, L, R, idx, T, perm_ws, &perm, st));
  return f64 ? gather_lp_t(prec, (const double*)X, L, I, idx, T, scale2, Cq, omega, perm, st)
             : gather_lp_t(prec, (const float*)X, L, I, idx, T, scale2, Cq, omega, perm, st);
}

int launch_maxabs(bool f64, const void* X, int64_t n, unsigned* out, hipStream_t st) {
  // the slot is 8-byte aligned and at least 8 bytes long (workspace layout)
  TR_TRY(launch_fill(reinterpret_cast<unsigned long long*>(out), 1, 0ull, st));
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, cdiv(n, kNT * 8)));
  if (f64)
    hipLaunchKernelGGL(trk::k_maxabs<double>, dim3(nb), dim3(kNT), 0, st, (const double*)X, n,
                       out);
  else
    hipLaunchKernelGGL(trk::k_maxabs<float>, dim3(nb), dim3(kNT), 0, st, (const float*)X, n, out);
  return check_launch();
}

int launch_factor(const double* C, int64_t I, int64_t s, int64_t mu, double* Q, double* Qt,
                  int ldqt, double* sig, void* Qcast, int cast_f32, uint32_t* status,
                  double* gA, hipStream_t st);

// The power scheme in low precision (k_quant_y, k_pw_lp, k_reduce_parts_lp
// per step), C and G float64 I x s column-major.  M: a tensor view (kind
// kLpF32 / kLpF64, ldi = I, omega unused) or the operand-form sample matrix
// (kLpStored, L = 1, ldi = Ip, omega = its column weights).  q = 1:
// C = M D M^T G.  q > 1: subspace iteration -- between steps the sketch is
// replaced by an orthonormal basis of its range (its s left singular vectors,
// float64), because rounding the raw iterate (AA^T)^i G to the operand format
// would erase every direction below the format's precision relative to the
// leading one; C = M D M^T Y_{q-1} has the range of (M D M^T)^q G.
// G is overwritten for q > 1.
// One low-precision power step C = M D M^T Y (Y and C float64 I x s).
int power_lp_step(const Plan& P, int kind, const void* M, int64_t L, int64_t I, int64_t R,
                  int64_t ldi, const float* omega, const unsigned* xmax, int64_t s,
                  const double* Y, double* C, void* ws, uint32_t* status, hipStream_t st) {
  void* Cq = static_cast<char*>(ws) + P.oYq;
  float* tau = reinterpret_cast<float*>(static_cast<char*>(ws) + P.oTau);
  float* part = reinterpret_cast<float*>(static_cast<char*>(ws) + P.oPartLp);
  const int64_t nblk = lp_blocks(I, s, L * R);
  const int64_t Ip = lp_ip(I), SP = 16 * lp_nkt(s);
  TR_TRY(launch_quant_y(P.prec, Y, I, s, Cq, tau, st));
  TR_TRY(launch_pw_lp(P.prec, kind, s, M, L, I, R, ldi, Cq, tau, omega, xmax, part, nblk, st));
  hipLaunchKernelGGL(trk::k_reduce_parts_lp, dim3((unsigned)cdiv(I * s, 32)), dim3(kNT), 0, st,
                     part, nblk, I, (int)s, (int)SP, (int)Ip, C, status);
  return check_launch();
}

// One low-precision power step for k modes of the same tensor M (tensor
// form, ldi = I_n): C_b = M D M^T Y_b for mode modes[b], as power_lp_step for
// each in turn, with each mode's reduction and the next mode's operand
// quantisation in one launch (they share no buffer), 2k launches in all.
int power_lp_step_modes(const Plan& P, const int* modes, int k, const void* M,
                        const unsigned* xmax, const double* const* Y, double* const* C,
                        void* ws, uint32_t* status, hipStream_t st) {
  void* Cq = static_cast<char*>(ws) + P.oYq;
  float* tau = reinterpret_cast<float*>(static_cast<char*>(ws) + P.oTau);
  float* part = reinterpret_cast<float*>(static_cast<char*>(ws) + P.oPartLp);
  {
    const ModePlan& M0 = P.m[modes[0]];
    TR_TRY(launch_quant_y(P.prec, Y[0], M0.I, M0.s, Cq, tau, st));
  }
  for (int b = 0; b < k; ++b) {
    const ModePlan& Mb = P.m[modes[b]];
    const int kind = Mb.src_f64 ? kLpF64 : kLpF32;
    const int64_t I = Mb.I, s = Mb.s;
    const int64_t nblk = lp_blocks(I, s, Mb.L * Mb.R);
    const int Ip = (int)lp_ip(I), SP = (int)(16 * lp_nkt(s));
    TR_TRY(launch_pw_lp(P.prec, kind, s, M, Mb.L, I, Mb.R, I, Cq, tau, nullptr, xmax, part,
                        nblk, st));
    const int64_t nred = cdiv(I * s, 32);
    if (b + 1 == k) {
      hipLaunchKernelGGL(trk::k_reduce_parts_lp, dim3((unsigned)nred), dim3(kNT), 0, st, part,
                         nblk, I, (int)s, SP, Ip, C[b], status);
      TR_TRY(check_launch());
      break;
    }
    const ModePlan& Mn = P.m[modes[b + 1]];
    const int Ip2 = (int)lp_ip(Mn.I), SP2 = (int)(16 * lp_nkt(Mn.s));
    const dim3 grid((unsigned)(nred + SP2));
    if (P.prec == TR_PREC_FP8E4M3)
      hipLaunchKernelGGL(trk::k_reduce_quant<trk::OpFp8>, grid, dim3(kNT), 0, st, part, nblk, I,
                         (int)s, SP, Ip, C[b], status, nred, Y[b + 1], Mn.I, (int)Mn.s, Ip2,
                         (uint8_t*)Cq, tau);
    else
      hipLaunchKernelGGL(trk::k_reduce_quant<trk::OpBf16>, grid, dim3(kNT), 0, st, part, nblk,
                         I, (int)s, SP, Ip, C[b], status, nred, Y[b + 1], Mn.I, (int)Mn.s, Ip2,
                         (uint16_t*)Cq, tau);
    TR_TRY(check_launch());
  }
  return TR_OK;
}

int launch_factor_jobs(const trk::FactorJob* job, int n, int cast_f32, uint32_t* status,
                       hipStream_t st);

// Orthonormalisation steps of the R-accumulated power scheme for k modes at
// once: Z_n = an orthonormal basis of C_n's range (one factor launch for
// all), Zt_n its zero-padded row-major copy (row stride ldzt; skipped when
// null), then Rbar_n <- (Z_n^T C_n) Rbar_n (first: the product alone).  C_n is
// left intact (the factor's scratch is its own).
int stab_orth(const Plan& P, const int* modes, int k, double* const* C, double* const* Zt,
              bool first, void* ws, uint32_t* status, hipStream_t st) {
  trk::FactorJob jobs[TR_MAX_ORDER];
  for (int b = 0; b < k; ++b) {
    const int n = modes[b];
    const ModePlan& M = P.m[n];
    // an orthonormal basis of C only: the Householder QR's Q1 (no SVD) where
    // the register-resident kernel runs; the wider kernels' SVD basis spans
    // the same space
    jobs[b] = trk::FactorJob{C[b], at<double>(ws, P.oZn[n]), Zt[b], at<double>(ws, P.oSgs[n]),
                             nullptr, at<double>(ws, P.oGA[n]), (int)M.I, (int)M.s, (int)M.s,
                             Zt[b] ? M.sw : 0, nullptr, 1};
  }
  TR_TRY(launch_factor_jobs(jobs, k, 0, status, st));
  // R_n = Z_n^T C_n and the Rbar_n update: one launch each for all k modes
  static_assert(trk::kStabMaxJobs >= TR_MAX_ORDER, "one stabilised job per mode");
  trk::StabSteps steps{};
  int64_t smax = 1;
  for (int b = 0; b < k; ++b) {
    const int n = modes[b];
    const ModePlan& M = P.m[n];
    steps.j[b] = trk::StabStep{at<double>(ws, P.oZn[n]), C[b], at<double>(ws, P.oRst[n]),
                               at<double>(ws, P.oRbar[n]), M.I, (int)M.s, first ? 1 : 0};
    smax = std::max<int64_t>(smax, M.s);
  }
  hipLaunchKernelGGL(trk::k_small_tn, dim3((unsigned)(smax * smax), (unsigned)k),
                     dim3(trk::kStabNT), 0, st, steps, (int)smax);
  TR_TRY(check_launch());
  hipLaunchKernelGGL(trk::k_rbar_update, dim3((unsigned)k), dim3(trk::kStabNT), 0, st, steps);
  return check_launch();
}

// Whether the R-accumulated low-precision scheme starts from G itself
// (Z_0 = G, R_0 = I) rather than from an orthonormal basis of it: with
// s <= I / 2 the Gaussian G is well conditioned (kappa about
// (1 + sqrt(s/I)) / (1 - sqrt(s/I)) <= 6), so rounding it to the operand
// format keeps every direction, and the first orthonormalisation is skipped.
inline bool lp_raw_start(int64_t I, int64_t s) { return 2 * s <= I; }

// Low-precision power products of mode n from G (float64 I x s): without
// R-accumulation (q = 1) C = M D M^T G; with it, Z_0 Rbar = G (Z_0 = G and
// Rbar = I when lp_raw_start), then per step C = M D M^T Z_{i-1} in the
// operand format and Z_i, Rbar updated (the iterate that is rounded is
// orthonormal or a well-conditioned G, which keeps directions far below the
// leading one; C_n = Z_q Rbar is left to the final factor).
int run_power_lp(const Plan& P, int n, int kind, const void* M, int64_t L, int64_t I, int64_t R,
                 int64_t ldi, const float* omega, const unsigned* xmax, int64_t s,
                 double* G, double* C, void* ws, uint32_t* status, hipStream_t st) {
  if (!P.racc)
    return power_lp_step(P, kind, M, L, I, R, ldi, omega, xmax, s, G, C, ws, status, st);
  double* const none[1] = {nullptr};
  double* Zn = at<double>(ws, P.oZn[n]);
  const bool raw = lp_raw_start(I, s);
  double* cs[1] = {G};
  if (!raw) TR_TRY(stab_orth(P, &n, 1, cs, none, true, ws, status, st));
  cs[0] = C;
  for (int step = 0; step < P.q; ++step) {
    double* Z = raw && step == 0 ? G : Zn;
    TR_TRY(power_lp_step(P, kind, M, L, I, R, ldi, omega, xmax, s, Z, C, ws, status, st));
    TR_TRY(stab_orth(P, &n, 1, cs, none, raw && step == 0, ws, status, st));
  }
  return TR_OK;
}

// TUCKER_RAND_FACTOR=lds selects the LDS-resident factor kernel for every
// shape (both variants are then testable on the same inputs).
inline bool force_lds_factor() {
  const char* v = std::getenv("TUCKER_RAND_FACTOR");
  return v != nullptr && std::strcmp(v, "lds") == 0;
}

static_assert(trk::kMaxFactorJobs >= TR_MAX_ORDER, "one factorization job per mode");

// The smallest register-resident instance covering (I, s, mu), or -1.
inline int factor_rf_variant(int64_t I, int64_t s, int64_t mu) {
  if (I > 512 || s > 48) return -1;
  const bool r1 = I <= 256;
  if (s <= 16) return r1 ? kRf16x1 : kRf16x2;
  if (s <= 24 && r1) return kRf24x1;
  if (s <= 24 && mu <= 16) return kRf24x2;
  if (s <= 32 && r1) return kRf32x1;
  if (s <= 32 && mu <= 16) return kRf32x2;
  if (s <= 40 && r1) return kRf40x1;
  if (s <= 40 && mu <= 32) return kRf40x2;
  if (r1) return kRf48x1;
  return mu <= 32 ? kRf48x2 : -1;
}

int factor_variant(int64_t I, int64_t s, int64_t mu, bool has_scratch, bool has_wide,
                   int* var) {
  if (!factor_supported(I, s) || mu < 1 || mu > s) return TR_ENOTSUP;
  if (wide_sketch(s)) {
    if (!has_scratch || !has_wide) return TR_ENOMEM;
    *var = kGlb128;
    return TR_OK;
  }
  const int rf = factor_rf_variant(I, s, mu);
  if (rf >= 0 && !force_lds_factor()) {
    *var = rf;
    return TR_OK;
  }
  const int sm = factor_sm(s);
  const int k = sm == 16 ? 0 : (sm == 32 ? 1 : 2);
  if (factor_in_lds(I, s, mu)) {
    *var = kLds16 + k;
    return TR_OK;
  }
  if (!has_scratch) return TR_ENOMEM;
  *var = kGlb16 + k;
  return TR_OK;
}

// Independent factorizations (n <= kMaxFactorJobs): one launch per kernel
// instance, one workgroup per job, so jobs of the same instance run side by
// side.  Each job: Q (I x mu, float64), Qt (row stride ldqt, zero padding),
// sigma, optional cast copy of Q in the caller's dtype; gA: I x s float64
// scratch, needed only when the working matrices do not fit in LDS (may
// equal C).
// Bounds of the register-resident instances: s <= SM, I <= 256 R, mu <= MU.
struct RfBounds {
  int var, sm, r, mu;
};
constexpr RfBounds kRfBounds[] = {
    {kRf16x1, 16, 1, 16}, {kRf16x2, 16, 2, 16}, {kRf24x1, 24, 1, 24}, {kRf24x2, 24, 2, 16},
    {kRf32x1, 32, 1, 32}, {kRf32x2, 32, 2, 16}, {kRf40x1, 40, 1, 40}, {kRf40x2, 40, 2, 32},
    {kRf48x1, 48, 1, 48}, {kRf48x2, 48, 2, 32}};

inline bool is_rf_variant(int var) {
  for (const RfBounds& b : kRfBounds)
    if (b.var == var) return true;
  return false;
}

int launch_factor_jobs(const trk::FactorJob* job, int n, int cast_f32, uint32_t* status,
                       hipStream_t st) {
  if (n < 1 || n > trk::kMaxFactorJobs) return TR_EINVAL;
  int var[trk::kMaxFactorJobs];
  for (int b = 0; b < n; ++b)
    TR_TRY(factor_variant(job[b].I, job[b].s, job[b].mu, job[b].gA != nullptr,
                          job[b].gW != nullptr, &var[b]));
  // Jobs of different register-resident instances would run one launch after
  // another; when one instance covers them all (the narrowest such), a single
  // launch runs them side by side and takes about as long as its widest job.
  bool all_rf = true, mixed = false;
  for (int b = 0; b < n; ++b) {
    all_rf = all_rf && is_rf_variant(var[b]);
    mixed = mixed || var[b] != var[0];
  }
  if (all_rf && mixed) {
    for (const RfBounds& c : kRfBounds) {
      bool fits = true;
      for (int b = 0; b < n; ++b)
        fits = fits && job[b].s <= c.sm && job[b].I <= 256 * c.r && job[b].mu <= c.mu;
      if (fits) {
        for (int b = 0; b < n; ++b) var[b] = c.var;
        break;
      }
    }
  }
  bool done[trk::kMaxFactorJobs] = {};
  for (int b = 0; b < n; ++b) {
    if (done[b]) continue;
    trk::FactorJobs group{};
    int m = 0;
    for (int c = b; c < n; ++c)
      if (!done[c] && var[c] == var[b]) {
        group.j[m++] = job[c];
        done[c] = true;
      }
    TR_TRY(launch_factor_group(var[b], group, m, cast_f32, status, st));
  }
  return TR_OK;
}

int launch_factor(const double* C, int64_t I, int64_t s, int64_t mu, double* Q, double* Qt,
                  int ldqt, double* sig, void* Qcast, int cast_f32, uint32_t* status,
                  double* gA, hipStream_t st) {
  trk::FactorJob jb{C, Q, Qt, sig, Qcast, gA, (int)I, (int)s, (int)mu, ldqt};
  return launch_factor_jobs(&jb, 1, cast_f32, status, st);
}

// ---------------------------------------------------------------------------
// Drivers
// ---------------------------------------------------------------------------
int copy_d2d(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (!dst || bytes == 0) return TR_OK;
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st) == hipSuccess
             ? TR_OK
             : TR_EDEVICE;
}

// Every mode's G_n and its padded row-major copy into the plan's buffers,
// and every mode's running maximum of the column norms cleared, in one launch.
int launch_gaussian_modes(const Plan& P, void* ws, hipStream_t st) {
  static_assert(TR_MAX_ORDER <= 8, "GaussModes holds at most 8 modes");
  trk::GaussModes gm{};
  int64_t t = 0;
  for (int n = 0; n < P.N; ++n) {
    const ModePlan& M = P.m[n];
    gm.m[n] = trk::GaussMode{at<double>(ws, P.oGs[n]), at<double>(ws, P.oYts[n]), M.I, M.s,
                             M.sw, t};
    t += cdiv(M.I * M.s, 4) + M.I * (M.sw - M.s);
  }
  gm.n = P.N;
  gm.nzero = P.N;
  gm.zero = at<unsigned long long>(ws, P.oMax);
  t = std::max<int64_t>(t, P.N);
  hipLaunchKernelGGL(trk::k_gaussian_modes, dim3((unsigned)cdiv(t, kNT)), dim3(kNT), 0, st, gm,
                     P.seed);
  return check_launch();
}

// Partial sums (SQ: of squares) of n elements of x (float64, or float32 when
// !f64) into kNormMaxParts or fewer partials; returns their count.
int norm_parts(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(trk::kNormMaxParts, cdiv(n, 4 * trk::kNormNT)));
}
int launch_partial_sum(const void* x, bool f32, bool sq, int64_t n, double* parts,
                       hipStream_t st) {
  const dim3 g((unsigned)norm_parts(n)), b(trk::kNormNT);
  if (f32 && sq)
    hipLaunchKernelGGL((trk::k_partial_sum<float, true>), g, b, 0, st, (const float*)x, n, parts);
  else if (sq)
    hipLaunchKernelGGL((trk::k_partial_sum<double, true>), g, b, 0, st, (const double*)x, n,
                       parts);
  else
    hipLaunchKernelGGL((trk::k_partial_sum<double, false>), g, b, 0, st, (const double*)x, n,
                       parts);
  return check_launch();
}

// The first mode's unfolding in compressed sparse columns (tr_sparse.hpp).
struct CscView {
  const int64_t* colptr;  // [J_1 + 1]
  const int32_t* rowidx;  // [nnz]
  const void* vals;       // [nnz], the decomposition's dtype
  int64_t nnz;
};

int launch_colnorms_csc(bool f64, const CscView& sp, int64_t J, double* norms,
                        unsigned long long* maxb, hipStream_t st) {
  const dim3 grid((unsigned)cdiv(J, kNT));
  if (f64)
    hipLaunchKernelGGL(trk::k_colnorms_csc<double>, grid, dim3(kNT), 0, st, sp.colptr,
                       (const double*)sp.vals, J, norms, maxb);
  else
    hipLaunchKernelGGL(trk::k_colnorms_csc<float>, grid, dim3(kNT), 0, st, sp.colptr,
                       (const float*)sp.vals, J, norms, maxb);
  return check_launch();
}

int launch_gather_csc(bool f64, const CscView& sp, int64_t I, const int64_t* idx, int64_t T,
                      void* Cp, uint32_t* status, hipStream_t st) {
  if (f64)
    hipLaunchKernelGGL(trk::k_gather_csc<double>, dim3((unsigned)T), dim3(kNT), 0, st, sp.colptr,
                       sp.rowidx, (const double*)sp.vals, I, idx, (double*)Cp, status);
  else
    hipLaunchKernelGGL(trk::k_gather_csc<float>, dim3((unsigned)T), dim3(kNT), 0, st, sp.colptr,
                       sp.rowidx, (const float*)sp.vals, I, idx, (float*)Cp, status);
  return check_launch();
}

template <typename T, int MU>
void ttm_csc_w(const CscView& sp, int64_t I, int64_t J, const double* Qt, int kout, double* Y,
               uint32_t* status, hipStream_t st) {
  hipLaunchKernelGGL((trk::k_ttm_csc<T, MU>), dim3((unsigned)cdiv(J, kNT)), dim3(kNT), 0, st,
                     sp.colptr, sp.rowidx, (const T*)sp.vals, I, J, Qt, kout, Y, status);
}

template <typename T>
int ttm_csc_t(const CscView& sp, int64_t I, int64_t J, const double* Qt, int width, int kout,
              double* Y, uint32_t* status, hipStream_t st) {
  switch (width) {
    case 4: ttm_csc_w<T, 4>(sp, I, J, Qt, kout, Y, status, st); break;
    case 8: ttm_csc_w<T, 8>(sp, I, J, Qt, kout, Y, status, st); break;
    case 12: ttm_csc_w<T, 12>(sp, I, J, Qt, kout, Y, status, st); break;
    case 16: ttm_csc_w<T, 16>(sp, I, J, Qt, kout, Y, status, st); break;
    case 20: ttm_csc_w<T, 20>(sp, I, J, Qt, kout, Y, status, st); break;
    case 24: ttm_csc_w<T, 24>(sp, I, J, Qt, kout, Y, status, st); break;
    case 32: ttm_csc_w<T, 32>(sp, I, J, Qt, kout, Y, status, st); break;
    case 40: ttm_csc_w<T, 40>(sp, I, J, Qt, kout, Y, status, st); break;
    case 48: ttm_csc_w<T, 48>(sp, I, J, Qt, kout, Y, status, st); break;
    case 64: ttm_csc_w<T, 64>(sp, I, J, Qt, kout, Y, status, st); break;
    case 80: ttm_csc_w<T, 80>(sp, I, J, Qt, kout, Y, status, st); break;
    case 96: ttm_csc_w<T, 96>(sp, I, J, Qt, kout, Y, status, st); break;
    case 112: ttm_csc_w<T, 112>(sp, I, J, Qt, kout, Y, status, st); break;
    case 128: ttm_csc_w<T, 128>(sp, I, J, Qt, kout, Y, status, st); break;
    default: return TR_ENOTSUP;
  }
  return check_launch();
}

// ||A||^2, ||G||^2 and RE (Eq. (8)) into diag->norms after a decomposition:
// ||A||^2 from the partials of mode 1's column norms when they were taken,
// else from one sum-of-squares sweep of A (of a sparse A's stored values);
// ||G||^2 from the float64 core.
int launch_norms_re(const Plan& P, const void* A, void* ws, const tr_diag* diag,
                    hipStream_t st, const CscView* sp = nullptr) {
  if (!diag || !diag->norms) return TR_OK;
  const ModePlan& M0 = P.m[0];
  // a sparse tensor's squares are those of its stored values
  const int64_t numel = sp ? sp->nnz : M0.L * M0.I * M0.R;
  double* parts = at<double>(ws, P.oNparts);
  const bool have = M0.sampled && P.prob == TR_PROB_NEARLY_OPTIMAL;
  const int np = norm_parts(have ? M0.J : numel);
  if (!have)
    TR_TRY(launch_partial_sum(sp ? sp->vals : A, P.dtype == TR_F32, true, numel, parts, st));
  int64_t ncore = 1;
  for (int n = 0; n < P.N; ++n) ncore *= P.m[n].mu;
  hipLaunchKernelGGL(trk::k_norms_re, dim3(1), dim3(trk::kNormNT), 0, st, parts, np,
                     at<double>(ws, P.oCore), ncore, diag->norms);
  return check_launch();
}

// Range finder of mode n on tensor X (3-D view from the plan): fills Q64 / Qt
// of the mode in the workspace and the caller's Q (cast to dtype).
// Sketch of mode n of tensor X (3-D view from the plan): C_n = (M M^T)^q G_n
// into Y (I x s, float64).
int range_sketch(const Plan& P, int n, const void* X, void* ws, const tr_diag* diag,
                 bool need_xmax, double* Y, hipStream_t st, const CscView* sp = nullptr) {
  const ModePlan& M = P.m[n];
  tr_timer* tm = diag ? diag->timer : nullptr;
  uint32_t* status = diag ? diag->status : nullptr;
  // G_n, its row-major copy and the cleared running maximum of the column
  // norms come from launch_gaussian_modes, earlier on the stream
  double* G = at<double>(ws, P.oGs[n]);
  double* Yt = at<double>(ws, P.oYts[n]);
  double* Z = at<double>(ws, P.oZ);
  double* part = at<double>(ws, P.oPart);
  const bool norms_needed = M.sampled && P.prob == TR_PROB_NEARLY_OPTIMAL;
  const void* src = X;
  bool src_f64 = M.src_f64;
  int64_t L = M.L, R = M.R;
  const double* colw = nullptr;
  const int64_t* gidx = nullptr;  // sampled columns read in place (contiguous fibers)
  const bool lp = M.lp;
  if (M.sampled) {
    double* norms = at<double>(ws, P.oNorms);
    auto* maxb = at<unsigned long long>(ws, P.oMax) + n;
    int64_t* idx = at<int64_t>(ws, P.oIdx);
    double* scale = at<double>(ws, P.oScale);
    double* scale2 = at<double>(ws, P.oScale2);
    if (norms_needed) {
      TimeScope ts(tm, TR_KC_COLNORMS, n, st);
      if (sp)
        TR_TRY(launch_colnorms_csc(M.src_f64, *sp, M.J, norms, maxb, st));
      else
        TR_TRY(launch_colnorms(M.src_f64, X, M.L, M.I, M.R, norms, maxb, st, M.intermediate));
    }
    // ||A||^2 for the diagnostics: the column norms of mode 1 add up to it
    if (norms_needed && n == 0 && diag && diag->norms)
      TR_TRY(launch_partial_sum(norms, false, false, M.J, at<double>(ws, P.oNparts), st));
    {
      TimeScope ts(tm, TR_KC_SAMPLE, n, st);
      TR_TRY(launch_sample(norms, maxb, M.J, M.T, P.prob, P.seed, n,
                           at<unsigned long long>(ws, P.oW), at<unsigned long long>(ws, P.oCdf),
                           at<unsigned long long>(ws, P.oBsum), idx, scale, scale2, status, st));
    }
    {
      TimeScope ts(tm, TR_KC_GATHER, n, st);
      if (sp)
        TR_TRY(launch_gather_csc(M.src_f64, *sp, M.I, idx, M.T, at<void>(ws, P.oCp), status,
                                 st));
      else if (lp)
        TR_TRY(launch_gather_lp(P.prec, M.src_f64, X, M.L, M.I, idx, M.T, scale2,
                                at<void>(ws, P.oCq), at<float>(ws, P.oOmega), st, M.R,
                                at<int>(ws, P.oW)));
      else if (M.L == 1 && !(P.fused && pw_fused_ok(M.I, M.T, M.s)))
        // contiguous columns, and the products are the two-kernel ones:
        // they read C' = X(:, idx) in place, without the gathered copy
        gidx = idx;
      else
        TR_TRY(launch_gather(M.src_f64, X, M.L, M.I, idx, M.T, at<void>(ws, P.oCp), st, M.R,
                             at<int>(ws, P.oW)));  // the weights are spent by now
    }
    if (diag && diag->indices && diag->indices[n])
      TR_TRY(copy_d2d(diag->indices[n], idx, 8 * (size_t)M.T, st));
    if (diag && diag->scales && diag->scales[n])
      TR_TRY(copy_d2d(diag->scales[n], scale, 8 * (size_t)M.T, st));
    if (!gidx) src = at<void>(ws, P.oCp);
    L = 1;
    R = M.T;
    colw = scale2;
  }
  // C_n = (M M^T)^q G_n, starting from Yt = G_n^T.
  if (lp) {
    unsigned* xmax = nullptr;
    if (!M.sampled && P.prec == TR_PREC_FP8E4M3) {
      xmax = at<unsigned>(ws, P.oXmax);
      if (need_xmax) TR_TRY(launch_maxabs(M.src_f64, X, M.L * M.I * M.R, xmax, st));
    }
    TimeScope ts(tm, TR_KC_POWER, n, st);
    if (M.sampled)
      TR_TRY(run_power_lp(P, n, kLpStored, at<void>(ws, P.oCq), 1, M.I, M.T, lp_ip(M.I),
                          at<float>(ws, P.oOmega), nullptr, M.s, G, Y, ws, status, st));
    else
      TR_TRY(run_power_lp(P, n, M.src_f64 ? kLpF64 : kLpF32, X, M.L, M.I, M.R, M.I, nullptr,
                          xmax, M.s, G, Y, ws, status, st));
  } else if (P.racc) {
    // Z_0 Rbar = G (Yt = Z_0^T, padded), then per step Y = M D M^T Z_{i-1}
    // and Z_i, Rbar updated
    TimeScope ts(tm, TR_KC_POWER, n, st);
    double* Gs[1] = {G};
    double* Zts[1] = {Yt};
    TR_TRY(stab_orth(P, &n, 1, Gs, Zts, true, ws, status, st));
    double* Ys[1] = {Y};
    for (int step = 0; step < P.q; ++step) {
      TR_TRY(run_power(src_f64, src, L, M.I, R, colw, 1, M.s, M.sw, Y, Yt, Z, part, status, st,
                       P.fused, gidx));
      TR_TRY(stab_orth(P, &n, 1, Ys, Zts, false, ws, status, st));
    }
  } else {
    TimeScope ts(tm, TR_KC_POWER, n, st);
    TR_TRY(run_power(src_f64, src, L, M.I, R, colw, P.q, M.s, M.sw, Y, Yt, Z, part, status, st,
                     P.fused, gidx));
  }
  // (with R-accumulation the sketch Z_q Rbar is written by the final factor step)
  if (!P.racc && diag && diag->sketch && diag->sketch[n])
    TR_TRY(copy_d2d(diag->sketch[n], Y, 8 * (size_t)(M.I * M.s), st));
  return TR_OK;
}

// The factorization of mode n's sketch Y: Q64 / Qt of the mode in the
// workspace and the caller's Q (cast to dtype).  Y is dead afterwards (it
// doubles as the factor's scratch).
trk::FactorJob factor_job(const Plan& P, int n, double* Y, double* sig, void* ws, void* Qout) {
  const ModePlan& M = P.m[n];
  return trk::FactorJob{Y, at<double>(ws, P.oQ[n]), at<double>(ws, P.oQt[n]), sig, Qout, Y,
                        (int)M.I, (int)M.s, (int)M.mu, M.muw,
                        wide_sketch(M.s) ? at<double>(ws, M.oFw) : nullptr};
}

double* mode_sigma(const Plan& P, int n, const tr_diag* diag, void* ws, size_t off) {
  return (diag && diag->sigma && diag->sigma[n]) ? diag->sigma[n] : at<double>(ws, off);
}

// R-accumulated form: the factor of Rbar_n (s x s) into U'_n (s x mu); its
// singular values are those of C_n = Z_n Rbar_n.  When the mode's
// orthonormalisations run in the register-resident kernel (Z_i = Q_1 of the
// Householder QR with canonical signs, so each R_i = Z_i^T C_i and R_0 are
// upper triangular up to rounding) Rbar_n is upper triangular and its factor
// skips the QR.
trk::FactorJob rbar_job(const Plan& P, int n, double* sig, void* ws) {
  const ModePlan& M = P.m[n];
  int var = -1;
  const bool tri = factor_variant(M.I, M.s, M.s, true, false, &var) == TR_OK &&
                   is_rf_variant(var);
  return trk::FactorJob{at<double>(ws, P.oRbar[n]), at<double>(ws, P.oUp[n]), nullptr, sig,
                        nullptr, at<double>(ws, P.oGA[n]), (int)M.s, (int)M.s, (int)M.mu, 0,
                        nullptr, 0, tri ? 1 : 0};
}

// R-accumulated form, after rbar_job, for k modes in one launch: Q_n = Z_n
// U'_n(:, 1:mu) with canonical signs into the mode's Q64 / Qt and the caller's
// Q (Qout[b] for modes[b]); the sketch Z_n Rbar_n into the diagnostics when
// asked for.
int stab_final(const Plan& P, const int* modes, int k, void* ws, void* const* Qout,
               const tr_diag* diag, hipStream_t st) {
  trk::StabFinals fin{};
  int nbmax = 1;
  for (int b = 0; b < k; ++b) {
    const int n = modes[b];
    const ModePlan& M = P.m[n];
    // (without R-accumulation the sketch was copied out when it was formed)
    double* Cd =
        (P.racc && diag && diag->sketch && diag->sketch[n]) ? diag->sketch[n] : nullptr;
    const int nb = (int)(M.muw + (Cd ? M.s : 0));
    fin.j[b] = trk::StabFinal{at<double>(ws, P.oZn[n]), at<double>(ws, P.oUp[n]),
                              at<double>(ws, P.oRbar[n]), at<double>(ws, P.oQ[n]),
                              at<double>(ws, P.oQt[n]), Qout[b], Cd, M.I, (int)M.s,
                              (int)M.mu, M.muw, nb};
    nbmax = std::max(nbmax, nb);
  }
  hipLaunchKernelGGL(trk::k_stab_final, dim3((unsigned)nbmax, (unsigned)k), dim3(trk::kStabNT),
                     0, st, fin, P.dtype == TR_F32 ? 1 : 0);
  return check_launch();
}

int stab_final(const Plan& P, int n, void* ws, void* Qout, const tr_diag* diag,
               hipStream_t st) {
  void* const qo[1] = {Qout};
  return stab_final(P, &n, 1, ws, qo, diag, st);
}

// Related forms (Alg. 6 / Alg. 7), for k modes at once.  Step 1: P_n, an
// orthonormal basis of range(C_n), into the mode's Z buffer and its padded
// row-major copy into the mode's Yt (the start of the Gram's power step).
// Without R-accumulation P_n is the s left singular vectors of the sketch
// Y_n (one factor launch; their singular values, C_n's, go to sig); with it
// P_n = Z_q, and the factor of Rbar gives C_n's singular values.
int related_basis(const Plan& P, const int* modes, int k, double* const* Y, double* const* sig,
                  void* ws, uint32_t* status, hipStream_t st) {
  trk::FactorJob jobs[TR_MAX_ORDER];
  for (int b = 0; b < k; ++b) {
    const int n = modes[b];
    const ModePlan& M = P.m[n];
    jobs[b] = P.racc ? rbar_job(P, n, sig[b], ws)
                     : trk::FactorJob{Y[b], at<double>(ws, P.oZn[n]), at<double>(ws, P.oYts[n]),
                                      sig[b], nullptr, at<double>(ws, P.oGA[n]), (int)M.I,
                                      (int)M.s, (int)M.s, M.sw};
  }
  TR_TRY(launch_factor_jobs(jobs, k, 0, status, st));
  if (P.racc)
    for (int b = 0; b < k; ++b) {
      const ModePlan& M = P.m[modes[b]];
      hipLaunchKernelGGL(trk::k_transpose, dim3((unsigned)cdiv(M.I * M.sw, kNT)), dim3(kNT), 0,
                         st, at<double>(ws, P.oZn[modes[b]]), M.I, M.s, (int64_t)M.sw,
                         at<double>(ws, P.oYts[modes[b]]));
      TR_TRY(check_launch());
    }
  return TR_OK;
}

// Step 2 for mode n: the Gram matrix P_n^T A_(n) A_(n)^T P_n (s x s, into the
// mode's R_i buffer) by one exact float64 power step over the mode's tensor X
// (the full unfolding, also for sampled modes) and P_n^T times its result;
// Y (I x s) is scratch.
int related_gram(const Plan& P, int n, const void* X, double* Y, void* ws, uint32_t* status,
                 hipStream_t st) {
  const ModePlan& M = P.m[n];
  TR_TRY(run_power(M.src_f64, X, M.L, M.I, M.R, nullptr, 1, M.s, M.sw, Y,
                   at<double>(ws, P.oYts[n]), at<double>(ws, P.oZ), at<double>(ws, P.oPart),
                   status, st, P.fused));
  trk::StabSteps one{};
  one.j[0] = trk::StabStep{at<double>(ws, P.oZn[n]), Y, at<double>(ws, P.oRst[n]), nullptr, M.I,
                           (int)M.s, 0};
  hipLaunchKernelGGL(trk::k_small_tn, dim3((unsigned)(M.s * M.s), 1u), dim3(trk::kStabNT), 0, st,
                     one, (int)M.s);
  return check_launch();
}

// Step 3 for k modes: U_n = the mu leading eigenvectors of the Gram matrix
// (its left singular vectors: it is symmetric positive semidefinite), one
// factor launch; then step 4 per mode: Q_n = P_n U_n with canonical signs.
// (the eigenvalues, descending, are left in the mode's singular-value
// scratch: the fixed-precision driver reads them)
int related_eig(const Plan& P, const int* modes, int k, void* ws, uint32_t* status,
                hipStream_t st) {
  trk::FactorJob jobs[TR_MAX_ORDER];
  for (int b = 0; b < k; ++b) {
    const int n = modes[b];
    const ModePlan& M = P.m[n];
    jobs[b] = trk::FactorJob{at<double>(ws, P.oRst[n]), at<double>(ws, P.oUp[n]), nullptr,
                             at<double>(ws, P.oSgs[n]), nullptr, at<double>(ws, P.oGA[n]),
                             (int)M.s, (int)M.s, (int)M.mu, 0};
  }
  return launch_factor_jobs(jobs, k, 0, status, st);
}

int related_finish(const Plan& P, const int* modes, int k, void* ws, void* const* Qout,
                   const tr_diag* diag, uint32_t* status, hipStream_t st) {
  TR_TRY(related_eig(P, modes, k, ws, status, st));
  return stab_final(P, modes, k, ws, Qout, diag, st);
}

// Range finder of mode n (ST-HOSVD: sketch, then factor).
int range_finder(const Plan& P, int n, const void* X, void* ws, void* Qout,
                 const tr_diag* diag, bool need_xmax, hipStream_t st,
                 const CscView* sp = nullptr) {
  double* Y = at<double>(ws, P.oY);
  TR_TRY(range_sketch(P, n, X, ws, diag, need_xmax, Y, st, sp));
  tr_timer* tm = diag ? diag->timer : nullptr;
  uint32_t* status = diag ? diag->status : nullptr;
  TimeScope ts(tm, TR_KC_FACTOR, n, st);
  double* sig = mode_sigma(P, n, diag, ws, P.oSig);
  if (P.related) {  // Alg. 7: Q_n = P_n U_n, U_n from P_n^T A_(n)
    double* Ys[1] = {Y};
    double* sigs[1] = {sig};
    TR_TRY(related_basis(P, &n, 1, Ys, sigs, ws, status, st));
    TR_TRY(related_gram(P, n, X, Y, ws, status, st));
    void* qo[1] = {Qout};
    return related_finish(P, &n, 1, ws, qo, diag, status, st);
  }
  if (P.racc) {
    const trk::FactorJob jb = rbar_job(P, n, sig, ws);
    TR_TRY(launch_factor_jobs(&jb, 1, 0, status, st));
    return stab_final(P, n, ws, Qout, diag, st);
  }
  const trk::FactorJob jb = factor_job(P, n, Y, sig, ws, Qout);
  return launch_factor_jobs(&jb, 1, P.dtype == TR_F32, status, st);
}

int check_buffers(const Plan& P, const void* A, void* const* Q, const void* core, void* ws,
                  size_t ws_bytes) {
  if (!A || !Q || !core) return TR_EINVAL;
  for (int n = 0; n < P.N; ++n)
    if (!Q[n]) return TR_EINVAL;
  if (P.total > 0 && !ws) return TR_EINVAL;
  if (ws_bytes < P.total) return TR_ENOMEM;
  return TR_OK;
}

// One shrink X x_n Q_n^T of the chain; the last one goes through the float64
// core buffer and is cast into the caller's core.
int shrink(const Plan& P, int n, int step, const void* cur, bool cur_f64, int64_t L,
           int64_t I, int64_t R, void* ws, void* core, tr_timer* tm, void** out,
           hipStream_t st, const CscView* sp = nullptr, uint32_t* status = nullptr) {
  const ModePlan& M = P.m[n];
  const bool last = n == P.N - 1;
  double* dst = at<double>(ws, last ? P.oCore : ((step % 2 == 0) ? P.oX0 : P.oX1));
  bool cast_done = false;  // the last shrink's kernel wrote the caller's core too
  {
    TimeScope ts(tm, TR_KC_TTM, n, st);
    // (the fixed-precision driver shrinks views its plan did not size the
    // split-rows scratch for; those run the one-pass kernels)
    const size_t need = 8 * (size_t)(ttm_splits(L * R, I) * L * R * M.muw);
    double* split = need <= P.splitBytes ? at<double>(ws, P.oSplit) : nullptr;
    if (sp && cur_f64)
      TR_TRY(ttm_csc_t<double>(*sp, I, L * R, at<double>(ws, P.oQt[n]), M.muw, (int)M.mu, dst,
                               status, st));
    else if (sp)
      TR_TRY(ttm_csc_t<float>(*sp, I, L * R, at<double>(ws, P.oQt[n]), M.muw, (int)M.mu, dst,
                              status, st));
    else
      TR_TRY(launch_ttm(cur_f64, cur, L, I, R, at<double>(ws, P.oQt[n]), M.muw, (int)M.mu,
                        nullptr, dst, split, st, last ? core : nullptr, P.dtype == TR_F32,
                        &cast_done));
  }
  if (last && !cast_done) TR_TRY(launch_cast(dst, L * M.mu * R, P.dtype == TR_F32, core, st));
  *out = dst;
  return TR_OK;
}

int run_thosvd(const tr_params* p, int dtype, const void* A, void* const* Q, void* core,
               void* ws, size_t ws_bytes, const tr_diag* diag, hipStream_t st) {
  Plan P;
  TR_TRY(make_plan(p, dtype, false, &P));
  TR_TRY(check_buffers(P, A, Q, core, ws, ws_bytes));
  // the modes are independent: all sketches first (every mode reads the same
  // tensor, so its max |entry| -- the FP8 scale -- is taken once), then all
  // factorizations in one launch per kernel instance
  trk::FactorJob jobs[TR_MAX_ORDER];
  tr_timer* tm0 = diag ? diag->timer : nullptr;
  uint32_t* status = diag ? diag->status : nullptr;
  // low precision with q > 1: the unsampled modes advance one power step at
  // a time together, so that each round of orthonormalisation between steps
  // is one factor launch for all of them
  bool together[TR_MAX_ORDER] = {};
  int ntog = 0;
  for (int n = 0; n < P.N; ++n) {
    together[n] = P.prec != TR_PREC_NATIVE && P.q > 1 && !P.m[n].sampled;
    ntog += together[n] ? 1 : 0;
  }
  bool xmax_ready = false;
  {
    TimeScope ts(tm0, TR_KC_GAUSSIAN, 0, st);
    TR_TRY(launch_gaussian_modes(P, ws, st));
  }
  for (int n = 0; n < P.N; ++n) {
    if (together[n]) continue;
    TR_TRY(range_sketch(P, n, A, ws, diag, !xmax_ready, at<double>(ws, P.oYn[n]), st));
    // an unsampled mode in FP8 has taken the tensor's max |entry| (every mode
    // reads the same tensor)
    if (!P.m[n].sampled) xmax_ready = true;
  }
  if (ntog > 0) {
    // R-accumulated power steps (low precision, q > 1), all these modes per
    // step: Z_0 Rbar = G_n, then C_n = A_(n) A_(n)^T Z_{i-1} in the operand
    // format and Z_i, Rbar updated -- one factor launch per round for all
    unsigned* xmax = nullptr;
    if (P.prec == TR_PREC_FP8E4M3) {
      xmax = at<unsigned>(ws, P.oXmax);
      const ModePlan& M0 = P.m[0];
      if (!xmax_ready) TR_TRY(launch_maxabs(M0.src_f64, A, M0.L * M0.I * M0.R, xmax, st));
    }
    int modes[TR_MAX_ORDER];
    double* Cs[TR_MAX_ORDER];
    double* const nozt[TR_MAX_ORDER] = {};
    int k = 0;
    // modes whose G is first orthonormalised (the rest start from G itself,
    // as run_power_lp does) and their first R-accumulation step
    int k0 = 0;
    int modes0[TR_MAX_ORDER];
    double* Cs0[TR_MAX_ORDER];
    bool raw[TR_MAX_ORDER] = {};
    for (int n = 0; n < P.N; ++n)
      if (together[n]) {
        modes[k] = n;
        Cs[k++] = at<double>(ws, P.oYn[n]);
        raw[n] = lp_raw_start(P.m[n].I, P.m[n].s);
        if (!raw[n]) {
          modes0[k0] = n;
          Cs0[k0++] = at<double>(ws, P.oGs[n]);
        }
      }
    if (k0 > 0) {
      TimeScope ts(tm0, TR_KC_POWER, 0, st);
      TR_TRY(stab_orth(P, modes0, k0, Cs0, nozt, true, ws, status, st));
    }
    for (int step = 0; step < P.q; ++step) {
      {
        const double* Zs[TR_MAX_ORDER];
        for (int b = 0; b < k; ++b) {
          const int n = modes[b];
          Zs[b] = raw[n] && step == 0 ? at<double>(ws, P.oGs[n]) : at<double>(ws, P.oZn[n]);
        }
        TimeScope ts(tm0, TR_KC_POWER, 0, st);
        TR_TRY(power_lp_step_modes(P, modes, k, A, xmax, Zs, Cs, ws, status, st));
      }
      TimeScope ts(tm0, TR_KC_POWER, 0, st);
      if (step > 0 || k0 == k) {
        TR_TRY(stab_orth(P, modes, k, Cs, nozt, false, ws, status, st));
      } else {
        // the first step: the raw-start modes begin their Rbar here, the
        // others extend theirs (two groups, one factor launch each)
        int m1[TR_MAX_ORDER], m2[TR_MAX_ORDER];
        double* c1[TR_MAX_ORDER];
        double* c2[TR_MAX_ORDER];
        int n1 = 0, n2 = 0;
        for (int b = 0; b < k; ++b) {
          if (raw[modes[b]]) {
            m1[n1] = modes[b];
            c1[n1++] = Cs[b];
          } else {
            m2[n2] = modes[b];
            c2[n2++] = Cs[b];
          }
        }
        TR_TRY(stab_orth(P, m1, n1, c1, nozt, true, ws, status, st));
        if (n2 > 0) TR_TRY(stab_orth(P, m2, n2, c2, nozt, false, ws, status, st));
      }
    }
  }
  if (P.related) {
    // Alg. 6: every mode's P_n (one launch), its Gram matrix (a power step
    // over A each), then every mode's U_n (one launch) and Q_n = P_n U_n
    TimeScope ts(diag ? diag->timer : nullptr, TR_KC_FACTOR, 0, st);
    int modes[TR_MAX_ORDER];
    double* Ys[TR_MAX_ORDER];
    double* sigs[TR_MAX_ORDER];
    for (int n = 0; n < P.N; ++n) {
      modes[n] = n;
      Ys[n] = at<double>(ws, P.oYn[n]);
      sigs[n] = mode_sigma(P, n, diag, ws, P.oSign[n]);
    }
    TR_TRY(related_basis(P, modes, P.N, Ys, sigs, ws, status, st));
    for (int n = 0; n < P.N; ++n) TR_TRY(related_gram(P, n, A, Ys[n], ws, status, st));
    TR_TRY(related_finish(P, modes, P.N, ws, Q, diag, status, st));
  }
  for (int n = 0; n < P.N && !P.related; ++n) {
    double* sig = mode_sigma(P, n, diag, ws, P.oSign[n]);
    jobs[n] = P.racc ? rbar_job(P, n, sig, ws)
                     : factor_job(P, n, at<double>(ws, P.oYn[n]), sig, ws, Q[n]);
  }
  if (!P.related) {
    TimeScope ts(diag ? diag->timer : nullptr, TR_KC_FACTOR, 0, st);
    TR_TRY(launch_factor_jobs(jobs, P.N, P.dtype == TR_F32, diag ? diag->status : nullptr, st));
    if (P.racc) {
      int all[TR_MAX_ORDER];
      for (int n = 0; n < P.N; ++n) all[n] = n;
      TR_TRY(stab_final(P, all, P.N, ws, Q, diag, st));
    }
  }
  int64_t shp[TR_MAX_ORDER];
  for (int k = 0; k < P.N; ++k) shp[k] = P.dims[k];
  const void* cur = A;
  bool cur_f64 = dtype == TR_F64;
  tr_timer* tm = diag ? diag->timer : nullptr;
  for (int n = 0; n < P.N; ++n) {
    int64_t L = 1, R = 1;
    for (int k = 0; k < n; ++k) L *= shp[k];
    for (int k = n + 1; k < P.N; ++k) R *= shp[k];
    void* out = nullptr;
    TR_TRY(shrink(P, n, n, cur, cur_f64, L, shp[n], R, ws, core, tm, &out, st));
    shp[n] = P.m[n].mu;
    cur = out;
    cur_f64 = true;
  }
  return launch_norms_re(P, A, ws, diag, st);
}

// ---------------------------------------------------------------------------
// Fixed-precision problem (Problem 2): ranks chosen for a tolerance.
// ---------------------------------------------------------------------------

// The core chain of T-HOSVD over the plan's (possibly patched) ranks.
int core_chain(const Plan& P, const void* A, void* ws, void* core, tr_timer* tm,
               hipStream_t st) {
  int64_t shp[TR_MAX_ORDER];
  for (int k = 0; k < P.N; ++k) shp[k] = P.dims[k];
  const void* cur = A;
  bool cur_f64 = P.dtype == TR_F64;
  for (int n = 0; n < P.N; ++n) {
    int64_t L = 1, R = 1;
    for (int k = 0; k < n; ++k) L *= shp[k];
    for (int k = n + 1; k < P.N; ++k) R *= shp[k];
    void* out = nullptr;
    TR_TRY(shrink(P, n, n, cur, cur_f64, L, shp[n], R, ws, core, tm, &out, st));
    shp[n] = P.m[n].mu;
    cur = out;
    cur_f64 = true;
  }
  return TR_OK;
}

// Reads `count` doubles from the device (synchronising the stream).
int read_back(const double* dev, double* host, int count, hipStream_t st) {
  if (hipMemcpyAsync(host, dev, 8 * (size_t)count, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return TR_EDEVICE;
  return TR_OK;
}

// Smallest mu in [1, cap] with x2 - sum_{k <= mu} lam_k <= budget (cap when
// none is); *resid receives that residual (clamped at 0).
int64_t choose_rank(const double* lam, int64_t cap, double x2, double budget, double* resid) {
  double acc = 0.0;
  for (int64_t mu = 1; mu <= cap; ++mu) {
    acc += lam[mu - 1];
    if (x2 - acc <= budget || mu == cap) {
      *resid = std::max(x2 - acc, 0.0);
      return mu;
    }
  }
  *resid = x2;
  return cap;
}

// After the ranks of modes 0..done are chosen, the views of the later modes
// (ST-HOSVD) follow the shrunk tensor; a sampled mode whose columns no
// longer outnumber its samples becomes exact.
void repatch_views(Plan& P, int done, int64_t T_of_mode(const tr_params*, int),
                   const tr_params* p) {
  int64_t cur[TR_MAX_ORDER];
  for (int k = 0; k < P.N; ++k) cur[k] = k <= done ? P.m[k].mu : P.dims[k];
  for (int n = done + 1; n < P.N; ++n) {
    ModePlan& M = P.m[n];
    M.L = 1;
    M.R = 1;
    for (int k = 0; k < n; ++k) M.L *= cur[k];
    for (int k = n + 1; k < P.N; ++k) M.R *= cur[k];
    M.J = M.L * M.R;
    const int64_t T = T_of_mode(p, n);
    M.sampled = P.prob != TR_PROB_NONE && T >= 1 && T <= M.J;
    M.T = M.sampled ? T : 0;
  }
}

int64_t samples_of(const tr_params* p, int n) {
  return (p->prob != TR_PROB_NONE && p->samples) ? p->samples[n] : 0;
}

int run_adaptive(const tr_params* p0, int dtype, bool sthosvd, double tol, int relative,
                 const void* A, void* const* Q, void* core, void* ws, size_t ws_bytes,
                 int64_t* ranks_out, double* bound_out, const tr_diag* diag, hipStream_t st) {
  if (!(tol > 0.0) || (relative != 0 && relative != 1) || !ranks_out || !bound_out)
    return TR_EINVAL;
  if (!p0) return TR_EINVAL;
  tr_params p = *p0;
  p.flags |= TR_FLAG_RELATED_FORM;
  Plan P;
  TR_TRY(make_plan(&p, dtype, sthosvd, &P));
  TR_TRY(check_buffers(P, A, Q, core, ws, ws_bytes));
  uint32_t* status = diag ? diag->status : nullptr;
  tr_timer* tm = diag ? diag->timer : nullptr;
  const int N = P.N;
  int64_t mumax[TR_MAX_ORDER];
  for (int n = 0; n < N; ++n) mumax[n] = P.m[n].mu;
  // ||A||^2 (one sum-of-squares sweep), read back
  const ModePlan& M0 = P.m[0];
  const int64_t numel = M0.L * M0.I * M0.R;
  double* out3 = at<double>(ws, P.oNout);
  TR_TRY(launch_partial_sum(A, dtype == TR_F32, true, numel, at<double>(ws, P.oNparts), st));
  hipLaunchKernelGGL(trk::k_norms_re, dim3(1), dim3(trk::kNormNT), 0, st,
                     at<double>(ws, P.oNparts), norm_parts(numel), at<double>(ws, P.oCore),
                     (int64_t)0, out3);
  TR_TRY(check_launch());
  double h3[3];
  TR_TRY(read_back(out3, h3, 3, st));
  const double a2 = h3[0];
  const double eps2 = relative ? tol * tol * a2 : tol * tol;
  {
    TimeScope ts(tm, TR_KC_GAUSSIAN, 0, st);
    TR_TRY(launch_gaussian_modes(P, ws, st));
  }
  double lam[64];
  double used = 0.0;
  if (!sthosvd) {
    // every mode from A: sketches, bases, Gram matrices and their
    // eigenvalues for all modes, one read-back, then the chosen factors
    int modes[TR_MAX_ORDER];
    double* Ys[TR_MAX_ORDER];
    double* sigs[TR_MAX_ORDER];
    bool xmax_ready = false;
    for (int n = 0; n < N; ++n) {
      TR_TRY(range_sketch(P, n, A, ws, diag, !xmax_ready, at<double>(ws, P.oYn[n]), st));
      // an unsampled mode in FP8 has taken the tensor's max |entry|
      if (!P.m[n].sampled) xmax_ready = true;
      modes[n] = n;
      Ys[n] = at<double>(ws, P.oYn[n]);
      sigs[n] = mode_sigma(P, n, diag, ws, P.oSign[n]);
    }
    TimeScope ts(tm, TR_KC_FACTOR, 0, st);
    TR_TRY(related_basis(P, modes, N, Ys, sigs, ws, status, st));
    for (int n = 0; n < N; ++n) TR_TRY(related_gram(P, n, A, Ys[n], ws, status, st));
    TR_TRY(related_eig(P, modes, N, ws, status, st));
    for (int n = 0; n < N; ++n) {
      ModePlan& M = P.m[n];
      TR_TRY(read_back(at<double>(ws, P.oSgs[n]), lam, (int)M.s, st));
      double r2 = 0.0;
      const int64_t cap = std::min<int64_t>(std::min<int64_t>(mumax[n], M.J), M.s);
      M.mu = choose_rank(lam, cap, a2, eps2 / N, &r2);
      M.muw = pad_width(M.mu);
      used += r2;
      TR_TRY(stab_final(P, n, ws, Q[n], diag, st));
    }
    TR_TRY(core_chain(P, A, ws, core, tm, st));
  } else {
    const void* cur = A;
    bool cur_f64 = dtype == TR_F64;
    double x2 = a2;  // ||current tensor||^2
    for (int n = 0; n < N; ++n) {
      ModePlan& M = P.m[n];
      double* Y = at<double>(ws, P.oY);
      TR_TRY(range_sketch(P, n, cur, ws, diag, true, Y, st));
      {
        TimeScope ts(tm, TR_KC_FACTOR, n, st);
        double* Ys[1] = {Y};
        double* sigs[1] = {mode_sigma(P, n, diag, ws, P.oSig)};
        TR_TRY(related_basis(P, &n, 1, Ys, sigs, ws, status, st));
        TR_TRY(related_gram(P, n, cur, Y, ws, status, st));
        TR_TRY(related_eig(P, &n, 1, ws, status, st));
      }
      TR_TRY(read_back(at<double>(ws, P.oSgs[n]), lam, (int)M.s, st));
      double r2 = 0.0;
      const int64_t cap = std::min<int64_t>(std::min<int64_t>(mumax[n], M.J), M.s);
      M.mu = choose_rank(lam, cap, x2, (eps2 - used) / (N - n), &r2);
      M.muw = pad_width(M.mu);
      used += r2;
      double kept = 0.0;
      for (int64_t k = 0; k < M.mu; ++k) kept += lam[k];
      x2 = kept;
      TR_TRY(stab_final(P, n, ws, Q[n], diag, st));
      void* out = nullptr;
      TR_TRY(shrink(P, n, n, cur, cur_f64, M.L, M.I, M.R, ws, core, tm, &out, st));
      cur = out;
      cur_f64 = true;
      repatch_views(P, n, samples_of, &p);
    }
  }
  for (int n = 0; n < N; ++n) ranks_out[n] = P.m[n].mu;
  *bound_out = std::sqrt(used);
  return launch_norms_re(P, A, ws, diag, st);
}

// ---------------------------------------------------------------------------
// Fixed device scratch for callers that cannot allocate (tucker_rand_sthosvd_
// noalloc).  Each device that loads the library holds one copy of the array
// for the life of the process; its device address is looked up once per
// device (with that device current) and kept, because the array's name in
// host code is only a host-side stand-in.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[TR_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, which must be the
// device of `st` (the null stream belongs to the current device).
int scratch_address(hipStream_t st, void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return TR_EDEVICE;
  if (dev < 0 || dev >= kMaxDevices) return TR_ENOTSUP;
  if (st) {
    hipDevice_t sdev = -1;
    if (hipStreamGetDevice(st, &sdev) != hipSuccess) return TR_EDEVICE;
    if (sdev != dev) return TR_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TR_EDEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TR_OK;
}

// sp: the first mode's unfolding in compressed sparse columns (A unused then;
// the first mode must be sampled, in native precision, without flags).
int run_sthosvd(const tr_params* p, int dtype, const void* A, void* const* Q, void* core,
                void* ws, size_t ws_bytes, const tr_diag* diag, hipStream_t st,
                const CscView* sp = nullptr) {
  Plan P;
  TR_TRY(make_plan(p, dtype, true, &P));
  if (sp) {
    if (!P.m[0].sampled || P.prec != TR_PREC_NATIVE || P.racc || P.related) return TR_ENOTSUP;
    if (P.m[0].I > 2147483647LL) return TR_ENOTSUP;
    A = sp->vals;
  }
  TR_TRY(check_buffers(P, A, Q, core, ws, ws_bytes));
  const void* cur = A;
  bool cur_f64 = dtype == TR_F64;
  tr_timer* tm = diag ? diag->timer : nullptr;
  {
    TimeScope ts(tm, TR_KC_GAUSSIAN, 0, st);
    TR_TRY(launch_gaussian_modes(P, ws, st));
  }
  for (int n = 0; n < P.N; ++n) {
    const CscView* spn = n == 0 ? sp : nullptr;
    TR_TRY(range_finder(P, n, cur, ws, Q[n], diag, true, st, spn));
    const ModePlan& M = P.m[n];
    void* out = nullptr;
    TR_TRY(shrink(P, n, n, cur, cur_f64, M.L, M.I, M.R, ws, core, tm, &out, st, spn,
                  diag ? diag->status : nullptr));
    cur = out;
    cur_f64 = true;
  }
  return launch_norms_re(P, A, ws, diag, st, sp);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* tucker_rand_status_string(int status) {
  switch (status) {
    case TR_OK: return "ok";
    case TR_EINVAL: return "invalid argument";
    case TR_ENOMEM: return "workspace too small";
    case TR_EDEVICE: return "HIP device error";
    case TR_ENOTSUP: return "not supported by this library";
    case TR_ENUMERIC: return "numeric failure";
    default: return "unknown status";
  }
}

int tucker_rand_workspace_size(const tr_params* p, int dtype, int sthosvd, size_t* bytes) {
  if (!bytes) return TR_EINVAL;
  Plan P;
  const int rc = make_plan(p, dtype, sthosvd != 0, &P);
  if (rc != TR_OK) return rc;
  *bytes = P.total;
  return TR_OK;
}

int tucker_rand_thosvd(const tr_params* p, int dtype, const void* A, void* const* Q, void* core,
                       void* workspace, size_t workspace_bytes, const tr_diag* diag,
                       void* stream) {
  return run_thosvd(p, dtype, A, Q, core, workspace, workspace_bytes, diag, (hipStream_t)stream);
}

int tucker_rand_sthosvd(const tr_params* p, int dtype, const void* A, void* const* Q, void* core,
                        void* workspace, size_t workspace_bytes, const tr_diag* diag,
                        void* stream) {
  return run_sthosvd(p, dtype, A, Q, core, workspace, workspace_bytes, diag,
                     (hipStream_t)stream);
}

int tucker_rand_sthosvd_csc(const tr_params* p, int dtype, int64_t nnz, const int64_t* colptr,
                            const int32_t* rowidx, const void* vals, void* const* Q, void* core,
                            void* workspace, size_t workspace_bytes, const tr_diag* diag,
                            void* stream) {
  if (nnz < 0 || !colptr || (nnz > 0 && (!rowidx || !vals))) return TR_EINVAL;
  static const double kNoValues = 0.0;  // a host stand-in when nnz == 0 (never read)
  const CscView sp{colptr, rowidx, nnz > 0 ? vals : (const void*)&kNoValues, nnz};
  return run_sthosvd(p, dtype, nullptr, Q, core, workspace, workspace_bytes, diag,
                     (hipStream_t)stream, &sp);
}

int tucker_rand_sthosvd_noalloc(const tr_params* p, int dtype, const void* A, void* const* Q,
                                void* core, const tr_diag* diag, void* stream) {
  Plan P;
  TR_TRY(make_plan(p, dtype, true, &P));
  if (P.total > (size_t)TR_NOALLOC_SCRATCH_BYTES) return TR_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  void* ws = nullptr;
  TR_TRY(scratch_address(st, &ws));
  return run_sthosvd(p, dtype, A, Q, core, ws, (size_t)TR_NOALLOC_SCRATCH_BYTES, diag, st);
}

int tucker_rand_adaptive(const tr_params* p, int dtype, int sthosvd, double tol, int relative,
                         const void* A, void* const* Q, void* core, void* workspace,
                         size_t workspace_bytes, int64_t* ranks_out, double* bound_out,
                         const tr_diag* diag, void* stream) {
  return run_adaptive(p, dtype, sthosvd != 0, tol, relative, A, Q, core, workspace,
                      workspace_bytes, ranks_out, bound_out, diag, (hipStream_t)stream);
}

int tucker_rand_gaussian(int64_t I, int64_t s, int32_t mode, uint64_t seed, double* G,
                         void* stream) {
  if (I < 1 || s < 1 || !G || mode < 0) return TR_EINVAL;
  return launch_gaussian(G, nullptr, I, s, s, mode, seed, (hipStream_t)stream);
}

int tucker_rand_colnorms(int dtype, const void* X, int64_t L, int64_t I, int64_t R,
                         double* norms, uint64_t* max_bits, void* stream) {
  if ((dtype != TR_F64 && dtype != TR_F32) || !X || !norms || L < 1 || I < 1 || R < 1)
    return TR_EINVAL;
  return launch_colnorms(dtype == TR_F64, X, L, I, R, norms, (unsigned long long*)max_bits,
                         (hipStream_t)stream);
}

size_t tucker_rand_sample_workspace_size(int64_t J) { return J < 1 ? 0 : sample_ws_bytes(J); }

int tucker_rand_sample(const double* norms, int64_t J, int64_t T, int prob, uint64_t seed,
                       int32_t mode, int64_t* idx, double* scale, void* workspace,
                       size_t workspace_bytes, uint32_t* status, void* stream) {
  if (J < 1 || T < 1 || !idx || !scale || mode < 0) return TR_EINVAL;
  if (prob != TR_PROB_NEARLY_OPTIMAL && prob != TR_PROB_UNIFORM) return TR_EINVAL;
  if (prob == TR_PROB_NEARLY_OPTIMAL && !norms) return TR_EINVAL;
  if (!workspace || workspace_bytes < sample_ws_bytes(J)) return TR_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  auto* w = (unsigned long long*)ws;
  auto* cdf = (unsigned long long*)(ws + align_up(8 * (size_t)J));
  auto* bsum = (unsigned long long*)(ws + 2 * align_up(8 * (size_t)J));
  auto* maxb = (unsigned long long*)(ws + 2 * align_up(8 * (size_t)J) +
                                     align_up(8 * (size_t)(cdiv(J, trk::kScanChunk) + 1)));
  if (prob == TR_PROB_NEARLY_OPTIMAL) {
    // max over the given norms (order-free: integer max of the bit patterns)
    TR_TRY(launch_fill(maxb, 1, 0ull, st));
    hipLaunchKernelGGL(trk::k_max_bits, dim3((unsigned)cdiv(J, kNT)), dim3(kNT), 0, st, norms,
                       J, maxb);
    TR_TRY(check_launch());
  }
  return launch_sample(norms, maxb, J, T, prob, seed, mode, w, cdf, bsum, idx, scale, nullptr,
                       status, st);
}

int tucker_rand_gather(int dtype, const void* X, int64_t L, int64_t I, int64_t R,
                       const int64_t* idx, int64_t T, void* Cp, void* stream) {
  if ((dtype != TR_F64 && dtype != TR_F32) || !X || !idx || !Cp || L < 1 || I < 1 || R < 1 ||
      T < 1)
    return TR_EINVAL;
  return launch_gather(dtype == TR_F64, X, L, I, idx, T, Cp, (hipStream_t)stream);
}

size_t tucker_rand_power_workspace_size(int dtype, int64_t L, int64_t I, int64_t R,
                                        int64_t s) {
  if (L < 1 || I < 1 || R < 1 || s < 1 || s > kMaxSketch) return 0;
  return power_ws_bytes(L, I, R, s, dtype == TR_F64);
}

int tucker_rand_power(int dtype, const void* X, int64_t L, int64_t I, int64_t R,
                      const double* colweight, int32_t q, const double* G, int64_t s, double* C,
                      void* workspace, size_t workspace_bytes, void* stream) {
  if ((dtype != TR_F64 && dtype != TR_F32) || !X || !G || !C || L < 1 || I < 1 || R < 1 ||
      s < 1 || q < 1)
    return TR_EINVAL;
  if (s > kMaxSketch) return TR_ENOTSUP;
  const bool f64 = dtype == TR_F64;
  if (!workspace || workspace_bytes < power_ws_bytes(L, I, R, s, f64)) return TR_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  const int64_t J = L * R;
  const int sw = pad_width(s);
  char* ws = (char*)workspace;
  double* Z = (double*)ws;
  double* part = (double*)(ws + align_up(8 * (size_t)(J * pw_width(s))));
  double* Yt = (double*)(ws + align_up(8 * (size_t)(J * pw_width(s))) +
                         align_up(8 * (size_t)(power_parts(I, J, s) * I * s)));
  hipLaunchKernelGGL(trk::k_transpose, dim3((unsigned)cdiv(I * sw, kNT)), dim3(kNT), 0, st, G, I,
                     s, (int64_t)sw, Yt);
  TR_TRY(check_launch());
  return run_power(f64, X, L, I, R, colweight, q, s, sw, C, Yt, Z, part, nullptr, st);
}

size_t tucker_rand_factor_workspace_size(int64_t I, int64_t s, int64_t mu) {
  if (I < 1 || s < 1 || s > kMaxSketch || mu < 1 || mu > s) return 0;
  if (factor_in_lds(I, s, mu)) return 0;
  return align_up(8 * (size_t)(I * s)) + factor_wide_bytes(s);
}

int tucker_rand_factor(const double* C, int64_t I, int64_t s, int64_t mu, double* Q,
                       double* sigma, void* workspace, size_t workspace_bytes, void* stream) {
  if (!C || !Q || I < 1 || s < 1 || s > I || mu < 1 || mu > s) return TR_EINVAL;
  if (s > kMaxSketch) return TR_ENOTSUP;
  const size_t need = tucker_rand_factor_workspace_size(I, s, mu);
  if (need > 0 && (!workspace || workspace_bytes < need)) return TR_ENOMEM;
  trk::FactorJob jb{C, Q, nullptr, sigma, nullptr, (double*)workspace, (int)I, (int)s, (int)mu,
                    (int)mu, nullptr};
  if (wide_sketch(s))
    jb.gW = (double*)((char*)workspace + align_up(8 * (size_t)(I * s)));
  return launch_factor_jobs(&jb, 1, 0, nullptr, (hipStream_t)stream);
}

size_t tucker_rand_ttm_workspace_size(int64_t L, int64_t I, int64_t R, int64_t mu) {
  if (L < 1 || I < 1 || R < 1 || mu < 1 || mu > kMaxSketch) return 0;
  return align_up(8 * (size_t)(I * pad_width(mu))) + align_up(8 * (size_t)(L * mu * R));
}

int tucker_rand_ttm(int in_dtype, const void* X, int64_t L, int64_t I, int64_t R,
                    const double* Q, int64_t mu, int out_dtype, void* Y, void* workspace,
                    size_t workspace_bytes, void* stream) {
  if ((in_dtype != TR_F64 && in_dtype != TR_F32) || (out_dtype != TR_F64 && out_dtype != TR_F32))
    return TR_EINVAL;
  if (!X || !Q || !Y || L < 1 || I < 1 || R < 1 || mu < 1) return TR_EINVAL;
  if (mu > kMaxSketch) return TR_ENOTSUP;
  if (!workspace || workspace_bytes < tucker_rand_ttm_workspace_size(L, I, R, mu)) return TR_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  const int w = pad_width(mu);
  double* Qt = (double*)workspace;
  double* Y64 = (double*)((char*)workspace + align_up(8 * (size_t)(I * w)));
  hipLaunchKernelGGL(trk::k_transpose, dim3((unsigned)cdiv(I * w, kNT)), dim3(kNT), 0, st, Q, I,
                     mu, (int64_t)w, Qt);
  TR_TRY(check_launch());
  TR_TRY(launch_ttm(in_dtype == TR_F64, X, L, I, R, Qt, w, (int)mu, nullptr, Y64, nullptr, st));
  return launch_cast(Y64, L * mu * R, out_dtype == TR_F32, Y, st);
}

int tucker_rand_timer_create(int capacity, uint32_t class_mask, tr_timer** out) {
  if (!out || capacity < 1) return TR_EINVAL;
  tr_timer* t = new (std::nothrow) tr_timer();
  if (!t) return TR_EINVAL;
  t->mask = class_mask;
  t->pool.resize(2 * (size_t)capacity);
  // recording a launch never grows the list (no host allocation inside a call)
  t->used.reserve((size_t)capacity);
  for (auto& e : t->pool) {
    if (hipEventCreate(&e) != hipSuccess) {
      delete t;
      return TR_EDEVICE;
    }
  }
  *out = t;
  return TR_OK;
}

int tucker_rand_timer_destroy(tr_timer* t) {
  if (!t) return TR_EINVAL;
  for (auto& e : t->pool) (void)hipEventDestroy(e);
  delete t;
  return TR_OK;
}

int tucker_rand_timer_reset(tr_timer* t) {
  if (!t) return TR_EINVAL;
  t->used.clear();
  return TR_OK;
}

int tucker_rand_timer_read(tr_timer* t, int kernel_class, double* total_ms, int64_t* launches,
                           double* mode0_ms, int64_t* mode0_launches) {
  if (!t || kernel_class < 0 || kernel_class >= TR_KC_COUNT) return TR_EINVAL;
  double tot = 0.0, tot0 = 0.0;
  int64_t cnt = 0, cnt0 = 0;
  for (const auto& u : t->used) {
    if (u.cls != kernel_class) continue;
    if (hipEventSynchronize(u.stop) != hipSuccess) return TR_EDEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, u.start, u.stop) != hipSuccess) return TR_EDEVICE;
    tot += ms;
    ++cnt;
    if (u.mode == 0) {
      tot0 += ms;
      ++cnt0;
    }
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = cnt;
  if (mode0_ms) *mode0_ms = tot0;
  if (mode0_launches) *mode0_launches = cnt0;
  return TR_OK;
}

}  // extern "C"

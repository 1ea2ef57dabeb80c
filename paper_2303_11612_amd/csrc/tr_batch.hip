// Batched randomized ST-HOSVD with sampled products (Alg. 5) for a group of
// requests of different sizes and ranks: the requests advance through the
// modes together and every stage of a mode is one grouped launch over all of
// them (tr_batch.hpp), driven by a table of per-request descriptors in the
// workspace.  A batch of any size costs about eight launches per mode.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "tr_batch.hpp"
#include "tr_factor_rf.hpp"
#include "tr_host.hpp"
#include "tucker_rand.h"

namespace trh {
namespace {

constexpr size_t kAl = 256;
inline size_t al(size_t x) { return (x + kAl - 1) / kAl * kAl; }
constexpr int64_t kMaxTp = 8192;   // columns of a power matrix
constexpr int kMaxMu = 32;         // rank (shrink accumulators, factor instance)
constexpr int kMaxS = 48;          // sketch width (factor instance)
constexpr int64_t kMaxI = 512;     // mode size (factor instance)

struct MPlan {
  int64_t L, I, R, J, T, Tp;
  int s, mu, ldq, sampled;
};

struct RPlan {
  int N;
  MPlan m[TR_MAX_ORDER];
  // offsets inside the request's region
  size_t oNorms, oW, oCdf, oBsum, oMax, oIdx, oS2, oCp, oG[TR_MAX_ORDER], oY, oWs, oQ64,
      oQt[TR_MAX_ORDER], oSig, oX0, oX1, total;
};

int ceil_log2(int64_t J) {
  int c = 0;
  while (((int64_t)1 << c) < J) ++c;
  return c;
}

int plan_request(const tr_params* p, int N, RPlan* P) {
  if (!p || p->order != N || N < 1 || N > TR_MAX_ORDER || !p->dims || !p->ranks) return TR_EINVAL;
  if (p->oversample < 0 || p->power < 1 || p->flags != 0) return TR_EINVAL;
  if (p->precision != TR_PREC_NATIVE) return TR_ENOTSUP;
  if (p->prob != TR_PROB_NEARLY_OPTIMAL && p->prob != TR_PROB_UNIFORM) return TR_ENOTSUP;
  if (!p->samples) return TR_EINVAL;
  int64_t cur[TR_MAX_ORDER];
  for (int n = 0; n < N; ++n) {
    if (p->dims[n] < 1 || p->dims[n] > ((int64_t)1 << 31)) return TR_EINVAL;
    cur[n] = p->dims[n];
  }
  P->N = N;
  size_t maxJ = 0, maxT = 0, maxCp = 0, maxIs = 0, maxTs = 0, maxSig = 0, maxInter = 0;
  for (int n = 0; n < N; ++n) {
    MPlan& M = P->m[n];
    M.L = 1;
    M.R = 1;
    for (int k = 0; k < n; ++k) M.L *= cur[k];
    for (int k = n + 1; k < N; ++k) M.R *= cur[k];
    M.I = cur[n];
    M.J = M.L * M.R;
    M.mu = (int)p->ranks[n];
    if (p->ranks[n] < 1 || p->ranks[n] > M.I || p->ranks[n] > M.J) return TR_EINVAL;
    if (p->samples[n] < 1) return TR_EINVAL;
    M.s = (int)std::min<int64_t>(p->ranks[n] + p->oversample, M.I);
    if (M.I > kMaxI || M.s > kMaxS || M.mu > kMaxMu) return TR_ENOTSUP;
    M.sampled = p->samples[n] <= M.J;
    M.T = M.sampled ? p->samples[n] : 0;
    M.Tp = M.sampled ? M.T : M.J;
    if (M.Tp > kMaxTp) return TR_ENOTSUP;
    if ((M.J + trk::kScanChunk - 1) / trk::kScanChunk > 1024) return TR_ENOTSUP;
    M.ldq = M.mu <= 8 ? 8 : (M.mu <= 16 ? 16 : (M.mu <= 24 ? 24 : 32));
    maxJ = std::max(maxJ, (size_t)M.J);
    maxT = std::max(maxT, (size_t)M.Tp);
    maxCp = std::max(maxCp, (size_t)(M.I * M.Tp));
    maxIs = std::max(maxIs, (size_t)(M.I * M.s));
    maxTs = std::max(maxTs, (size_t)(M.Tp * M.s));
    maxSig = std::max(maxSig, (size_t)M.s);
    cur[n] = M.mu;
    size_t e = 1;
    for (int k = 0; k < N; ++k) e *= (size_t)cur[k];
    if (n + 1 < N) maxInter = std::max(maxInter, e);
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += al(std::max<size_t>(bytes, 8));
    return o;
  };
  P->oNorms = take(8 * maxJ);
  P->oW = take(8 * maxJ);
  P->oCdf = take(8 * maxJ);
  P->oBsum = take(8 * ((maxJ + trk::kScanChunk - 1) / trk::kScanChunk + 1));
  P->oMax = take(8 * (size_t)N);
  P->oIdx = take(8 * maxT);
  P->oS2 = take(8 * maxT);
  P->oCp = take(8 * maxCp);
  for (int n = 0; n < N; ++n) P->oG[n] = take(8 * (size_t)(P->m[n].I * P->m[n].s));
  P->oY = take(8 * maxIs);
  P->oWs = take(8 * maxTs);
  size_t maxIm = 0;
  for (int n = 0; n < N; ++n) maxIm = std::max(maxIm, (size_t)(P->m[n].I * P->m[n].mu));
  P->oQ64 = take(8 * maxIm);
  for (int n = 0; n < N; ++n) P->oQt[n] = take(8 * (size_t)(P->m[n].I * P->m[n].ldq));
  P->oSig = take(8 * maxSig);
  P->oX0 = take(8 * maxInter);
  P->oX1 = take(8 * maxInter);
  P->total = off;
  return TR_OK;
}

// Kernels of a mode whose block maps are kept: colnorms, weights / cdf
// (chunks), draw, gather, shrink.
// kMapM16, kMapM32: the first mode's shrink on the matrix cores, for Q^T rows
// of stride <= 16 and <= 32.
enum { kMapNorm = 0, kMapChunk, kMapDraw, kMapGather, kMapPwW, kMapPwY, kMapShrink, kMapM16,
       kMapM32, kMaps };

struct Layout {
  size_t oMd, oGj, oFj, oSt, oMaps, descBytes, reqBase, total;
  std::vector<size_t> reqOff;
};

Layout layout(int nreq, int N, const std::vector<RPlan>& P) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += al(std::max<size_t>(bytes, 8));
    return o;
  };
  L.oMd = take(sizeof(trk::BMode) * (size_t)N * nreq);
  L.oGj = take(sizeof(trk::BGauss) * (size_t)N * nreq);
  L.oFj = take(sizeof(trk::FactorJob) * (size_t)N * nreq);
  L.oSt = take(sizeof(uint32_t*) * (size_t)nreq);
  L.oMaps = take(sizeof(int64_t) * (size_t)N * kMaps * (nreq + 1));
  L.descBytes = off;
  L.reqBase = off;
  L.reqOff.resize(nreq);
  for (int r = 0; r < nreq; ++r) L.reqOff[r] = take(P[r].total);
  L.total = off;
  return L;
}

int validate(int nreq, const tr_params* const* p, int dtype, std::vector<RPlan>* P, int* N) {
  if (nreq < 1 || !p || !p[0]) return TR_EINVAL;
  if (dtype != TR_F64 && dtype != TR_F32) return TR_EINVAL;
  *N = p[0]->order;
  P->resize(nreq);
  for (int r = 0; r < nreq; ++r) TR_TRY(plan_request(p[r], *N, &(*P)[r]));
  return TR_OK;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// The narrowest register-resident factor instance for every job of a mode.
int factor_tab(const std::vector<RPlan>& P, int n, const trk::FactorJob* tab, int nreq,
               int cast_f32, uint32_t* const* sttab, hipStream_t st) {
  int smax = 0, mumax = 0;
  for (const RPlan& R : P) {
    smax = std::max(smax, R.m[n].s);
    mumax = std::max(mumax, R.m[n].mu);
  }
  if (smax <= 24 && mumax <= 16) return launch_factor_tab_kRf24x2(tab, nreq, cast_f32, sttab, st);
  if (smax <= 40) return launch_factor_tab_kRf40x2(tab, nreq, cast_f32, sttab, st);
  return launch_factor_tab_kRf48x2(tab, nreq, cast_f32, sttab, st);
}

template <int SM>
void power_steps(int nreq, const trk::BMode* md, const int64_t* mw, int64_t bw,
                 const int64_t* my, int64_t by, int qmax, hipStream_t st) {
  for (int step = 0; step < qmax; ++step) {
    hipLaunchKernelGGL(trk::kb_pw_w<SM>, dim3((unsigned)bw), dim3(trk::kNT), 0, st, md, mw,
                       nreq, step);
    hipLaunchKernelGGL(trk::kb_pw_y, dim3((unsigned)by), dim3(trk::kNT), 0, st, md, my, nreq,
                       step);
  }
}

template <typename Tin>
void launch_mode(int n, int nreq, const trk::BMode* md, const int64_t* maps,
                 const std::vector<int64_t> (&nb)[kMaps], int any_nearly, int smax, int qmax,
                 hipStream_t st) {
  const int64_t* mp = maps + (size_t)n * kMaps * (nreq + 1);
  auto mapk = [&](int k) { return mp + (size_t)k * (nreq + 1); };
  if (any_nearly) {
    if (nb[kMapNorm].back() > 0) {
      if (n == 0)
        hipLaunchKernelGGL(trk::kb_colnorms_l1<Tin>, dim3((unsigned)nb[kMapNorm].back()),
                           dim3(trk::kNT), 0, st, md, mapk(kMapNorm), nreq);
      else
        hipLaunchKernelGGL(trk::kb_colnorms<Tin>, dim3((unsigned)nb[kMapNorm].back()),
                           dim3(trk::kNT), 0, st, md, mapk(kMapNorm), nreq);
    }
    if (nb[kMapChunk].back() > 0) {
      hipLaunchKernelGGL(trk::kb_weights, dim3((unsigned)nb[kMapChunk].back()), dim3(trk::kNT),
                         0, st, md, mapk(kMapChunk), nreq);
      hipLaunchKernelGGL(trk::kb_cdf, dim3((unsigned)nb[kMapChunk].back()), dim3(trk::kNT), 0,
                         st, md, mapk(kMapChunk), nreq);
    }
  }
  hipLaunchKernelGGL(trk::kb_draw, dim3((unsigned)nb[kMapDraw].back()), dim3(trk::kNT), 0, st,
                     md, mapk(kMapDraw), nreq);
  hipLaunchKernelGGL(trk::kb_gather<Tin>, dim3((unsigned)nb[kMapGather].back()), dim3(trk::kNT),
                     0, st, md, mapk(kMapGather), nreq);
  const int64_t bw = nb[kMapPwW].back(), by = nb[kMapPwY].back();
  if (smax <= 16)
    power_steps<16>(nreq, md, mapk(kMapPwW), bw, mapk(kMapPwY), by, qmax, st);
  else if (smax <= 32)
    power_steps<32>(nreq, md, mapk(kMapPwW), bw, mapk(kMapPwY), by, qmax, st);
  else
    power_steps<48>(nreq, md, mapk(kMapPwW), bw, mapk(kMapPwY), by, qmax, st);
}

template <typename Tin, typename Tout, int MU>
void shrink_k(int nreq, const trk::BMode* md, const int64_t* map, int64_t blocks, int last,
              hipStream_t st) {
  hipLaunchKernelGGL((trk::kb_shrink<Tin, Tout, MU>), dim3((unsigned)blocks), dim3(trk::kNT), 0,
                     st, md, map, nreq, last);
}

// The first mode: one launch per output tile count (16 or 32 rows of Q^T).
template <typename Tin, typename Tout>
void shrink_first(int nreq, const trk::BMode* md, const int64_t* maps,
                  const std::vector<int64_t> (&nb)[kMaps], int last, hipStream_t st) {
  const dim3 b(trk::kNT);
  if (nb[kMapM16].back() > 0)
    hipLaunchKernelGGL((trk::kb_shrink_mfma<Tin, Tout, 1>), dim3((unsigned)nb[kMapM16].back()),
                       b, 0, st, md, maps + (size_t)kMapM16 * (nreq + 1), nreq, last);
  if (nb[kMapM32].back() > 0)
    hipLaunchKernelGGL((trk::kb_shrink_mfma<Tin, Tout, 2>), dim3((unsigned)nb[kMapM32].back()),
                       b, 0, st, md, maps + (size_t)kMapM32 * (nreq + 1), nreq, last);
}

template <typename Tin, typename Tout>
void shrink_mu(int mumax, int nreq, const trk::BMode* md, const int64_t* map, int64_t blocks,
               int last, hipStream_t st) {
  if (mumax <= 8) shrink_k<Tin, Tout, 8>(nreq, md, map, blocks, last, st);
  else if (mumax <= 16) shrink_k<Tin, Tout, 16>(nreq, md, map, blocks, last, st);
  else if (mumax <= 24) shrink_k<Tin, Tout, 24>(nreq, md, map, blocks, last, st);
  else shrink_k<Tin, Tout, 32>(nreq, md, map, blocks, last, st);
}

int run_batch(int nreq, const tr_params* const* p, int dtype, const void* const* A,
              void* const* const* Q, void* const* core, void* ws, size_t ws_bytes,
              uint32_t* status, hipStream_t st) {
  std::vector<RPlan> P;
  int N = 0;
  TR_TRY(validate(nreq, p, dtype, &P, &N));
  if (!A || !Q || !core) return TR_EINVAL;
  for (int r = 0; r < nreq; ++r) {
    if (!A[r] || !Q[r] || !core[r]) return TR_EINVAL;
    for (int n = 0; n < N; ++n)
      if (!Q[r][n]) return TR_EINVAL;
  }
  const Layout Lo = layout(nreq, N, P);
  if (!ws) return TR_EINVAL;
  if (ws_bytes < Lo.total) return TR_ENOMEM;
  // host copies of the descriptor tables, written to the workspace at once
  std::vector<unsigned char> desc(Lo.descBytes, 0);
  auto hd = [&](size_t off) { return desc.data() + off; };
  trk::BMode* md = reinterpret_cast<trk::BMode*>(hd(Lo.oMd));
  trk::BGauss* gj = reinterpret_cast<trk::BGauss*>(hd(Lo.oGj));
  trk::FactorJob* fj = reinterpret_cast<trk::FactorJob*>(hd(Lo.oFj));
  uint32_t** stt = reinterpret_cast<uint32_t**>(hd(Lo.oSt));
  int64_t* maps = reinterpret_cast<int64_t*>(hd(Lo.oMaps));
  int64_t gt = 0;
  int any_nearly = 0, mumax[TR_MAX_ORDER] = {}, smax[TR_MAX_ORDER] = {}, qmax = 0;
  std::vector<int64_t> nb[TR_MAX_ORDER][kMaps];
  for (int r = 0; r < nreq; ++r) stt[r] = status ? status + r : nullptr;
  for (int n = 0; n < N; ++n) {
    for (int k = 0; k < kMaps; ++k) nb[n][k].assign(nreq + 1, 0);
    for (int r = 0; r < nreq; ++r) {
      const RPlan& R = P[r];
      const MPlan& M = R.m[n];
      void* base = static_cast<char*>(ws) + Lo.reqOff[r];
      const bool nearly = p[r]->prob == TR_PROB_NEARLY_OPTIMAL && M.sampled;
      any_nearly |= nearly ? 1 : 0;
      mumax[n] = std::max(mumax[n], M.mu);
      smax[n] = std::max(smax[n], M.s);
      qmax = std::max(qmax, p[r]->power);
      trk::BMode& d = md[(size_t)n * nreq + r];
      d.X = n == 0 ? A[r] : at<double>(base, (n % 2 == 1) ? R.oX0 : R.oX1);
      d.L = M.L;
      d.I = M.I;
      d.R = M.R;
      d.J = M.J;
      d.T = M.T;
      d.Tp = M.Tp;
      d.s = M.s;
      d.mu = M.mu;
      d.ldq = M.ldq;
      d.sampled = M.sampled;
      d.nearly = nearly;
      d.kexp = 60 - ceil_log2(M.J);
      d.nchunk = (M.J + trk::kScanChunk - 1) / trk::kScanChunk;
      d.q = p[r]->power;
      d.mode = n;
      d.seed = p[r]->seed;
      d.norms = at<double>(base, R.oNorms);
      d.maxb = at<unsigned long long>(base, R.oMax) + n;
      d.w = at<unsigned long long>(base, R.oW);
      d.cdf = at<unsigned long long>(base, R.oCdf);
      d.bsum = at<unsigned long long>(base, R.oBsum);
      d.idx = at<int64_t>(base, R.oIdx);
      d.scale2 = at<double>(base, R.oS2);
      d.Cp = at<double>(base, R.oCp);
      d.G = at<double>(base, R.oG[n]);
      d.Y = at<double>(base, R.oY);
      d.W = at<double>(base, R.oWs);
      d.Qt = at<double>(base, R.oQt[n]);
      d.out = n + 1 < N ? at<double>(base, (n % 2 == 0) ? R.oX0 : R.oX1) : nullptr;
      d.core = n + 1 < N ? nullptr : core[r];
      d.status = stt[r];
      trk::BGauss& g = gj[(size_t)n * nreq + r];
      g = trk::BGauss{d.G, M.I, M.s, gt, n, p[r]->seed, nearly ? d.maxb : nullptr};
      gt += (M.I * M.s + 3) / 4;
      fj[(size_t)n * nreq + r] =
          trk::FactorJob{d.Y, at<double>(base, R.oQ64), d.Qt, at<double>(base, R.oSig),
                         Q[r][n], nullptr, (int)M.I, M.s, M.mu, M.ldq};
      const int64_t rc = (M.I + trk::kNT - 1) / trk::kNT;
      nb[n][kMapNorm][r + 1] = nearly ? cdiv(M.J, trk::kNT) : 0;
      nb[n][kMapChunk][r + 1] = nearly ? d.nchunk : 0;
      nb[n][kMapDraw][r + 1] = cdiv(M.Tp, trk::kNT);
      nb[n][kMapGather][r + 1] = M.Tp * rc;
      nb[n][kMapPwW][r + 1] = cdiv(M.Tp, trk::kPwCols);
      nb[n][kMapPwY][r + 1] = cdiv(M.I * M.s, trk::kNT);
      nb[n][kMapShrink][r + 1] = n == 0 ? 0 : cdiv(M.J, trk::kNT);
      if (n == 0) nb[n][M.ldq <= 16 ? kMapM16 : kMapM32][r + 1] = cdiv(M.J, trk::kSmCols);
    }
    for (int k = 0; k < kMaps; ++k) {
      int64_t* mp = maps + ((size_t)n * kMaps + k) * (nreq + 1);
      mp[0] = 0;
      for (int r = 0; r < nreq; ++r) nb[n][k][r + 1] += nb[n][k][r];
      for (int r = 0; r <= nreq; ++r) mp[r] = nb[n][k][r];
    }
  }
  // device addresses of the tables
  trk::BMode* dmd = at<trk::BMode>(ws, Lo.oMd);
  trk::BGauss* dgj = at<trk::BGauss>(ws, Lo.oGj);
  trk::FactorJob* dfj = at<trk::FactorJob>(ws, Lo.oFj);
  uint32_t* const* dst = at<uint32_t*>(ws, Lo.oSt);
  int64_t* dmaps = at<int64_t>(ws, Lo.oMaps);
  // the host copy of the tables lives only during this call: a copy that has
  // completed when it returns (ordered after the stream's earlier work)
  if (hipMemcpyWithStream(ws, desc.data(), Lo.descBytes, hipMemcpyHostToDevice, st) !=
      hipSuccess)
    return TR_EDEVICE;
  // every request's every Gaussian start, and the norm maxima cleared
  hipLaunchKernelGGL(trk::kb_gauss, dim3((unsigned)cdiv(gt, trk::kNT)), dim3(trk::kNT), 0, st,
                     dgj, N * nreq);
  TR_TRY(check_launch());
  const bool f32 = dtype == TR_F32;
  for (int n = 0; n < N; ++n) {
    const trk::BMode* mdn = dmd + (size_t)n * nreq;
    if (n == 0 && f32)
      launch_mode<float>(n, nreq, mdn, dmaps, nb[n], any_nearly, smax[n], qmax, st);
    else
      launch_mode<double>(n, nreq, mdn, dmaps, nb[n], any_nearly, smax[n], qmax, st);
    TR_TRY(check_launch());
    TR_TRY(factor_tab(P, n, dfj + (size_t)n * nreq, nreq, f32 ? 1 : 0,
                      status ? dst : nullptr, st));
    const int64_t* smap = dmaps + ((size_t)n * kMaps + kMapShrink) * (nreq + 1);
    const int64_t* fmaps = dmaps + (size_t)n * kMaps * (nreq + 1);
    const int64_t blocks = nb[n][kMapShrink].back();
    const int last = n + 1 == N;
    if (n == 0 && f32) {
      if (last) shrink_first<float, float>(nreq, mdn, fmaps, nb[n], 1, st);
      else shrink_first<float, double>(nreq, mdn, fmaps, nb[n], 0, st);
    } else if (n == 0) {
      shrink_first<double, double>(nreq, mdn, fmaps, nb[n], last, st);
    } else if (f32) {
      if (last) shrink_mu<double, float>(mumax[n], nreq, mdn, smap, blocks, 1, st);
      else shrink_mu<double, double>(mumax[n], nreq, mdn, smap, blocks, 0, st);
    } else {
      shrink_mu<double, double>(mumax[n], nreq, mdn, smap, blocks, last, st);
    }
    TR_TRY(check_launch());
  }
  return TR_OK;
}

}  // namespace
}  // namespace trh

extern "C" {

int tucker_rand_batch_workspace_size(int nreq, const tr_params* const* p, int dtype,
                                     size_t* bytes) {
  if (!bytes) return TR_EINVAL;
  std::vector<trh::RPlan> P;
  int N = 0;
  const int rc = trh::validate(nreq, p, dtype, &P, &N);
  if (rc != TR_OK) return rc;
  *bytes = trh::layout(nreq, N, P).total;
  return TR_OK;
}

int tucker_rand_sthosvd_batch(int nreq, const tr_params* const* p, int dtype,
                              const void* const* A, void* const* const* Q, void* const* core,
                              void* workspace, size_t workspace_bytes, uint32_t* status,
                              void* stream) {
  return trh::run_batch(nreq, p, dtype, A, Q, core, workspace, workspace_bytes, status,
                        (hipStream_t)stream);
}

}  // extern "C"

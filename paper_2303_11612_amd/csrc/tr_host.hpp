// Host-side pieces shared by the library's translation units: launch status
// helpers, the shapes of the low-precision power steps and of the factor
// kernel instances, and the launchers compiled in their own units (so that
// their many kernel instances build in parallel).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "tr_factor.hpp"
#include "tucker_rand.h"

namespace trh {

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline int check_launch() { return hipGetLastError() == hipSuccess ? TR_OK : TR_EDEVICE; }

#define TR_TRY(expr)              \
  do {                            \
    const int _rc = (expr);       \
    if (_rc != TR_OK) return _rc; \
  } while (0)


// Low-precision power steps (k_pw_lp): rows padded to Ip = 128 MI (MI in
// {1, 2, 4}, so I <= 512), sketch columns to 16 NKT (NKT <= 3, so s <= 48).
inline int lp_mi(int64_t I) { return I <= 128 ? 1 : (I <= 256 ? 2 : 4); }
inline int64_t lp_ip(int64_t I) { return 128 * lp_mi(I); }
inline int lp_nkt(int64_t s) { return (int)cdiv(s, 16); }
inline bool lp_supported(int64_t I, int64_t s) { return I <= 512 && s >= 1 && s <= 48; }
inline size_t lp_lds_bytes(int mi, int nkt) {
  return 4 * (size_t)(4 * 32 * mi * 36 + 2 * 4 * 16 * nkt * 36);
}
// Blocks of one power step over J columns: at most the resident blocks of
// the chip, at least two column blocks of 32 each.
inline int64_t lp_blocks(int64_t I, int64_t s, int64_t J) {
  const int64_t per_cu = lp_lds_bytes(lp_mi(I), lp_nkt(s)) <= 80 * 1024 ? 2 : 1;
  return std::max<int64_t>(1, std::min<int64_t>(256 * per_cu, cdiv(cdiv(J, 32), 2)));
}

// Source of a low-precision power step: a float32 / float64 tensor view, or
// the gathered sample matrix already in operand form.
enum LpSrc { kLpF32 = 0, kLpF64 = 1, kLpStored = 2 };

// One low-precision power step (k_pw_lp) in the format `prec` (tr_prec) on a
// source of kind LpSrc; part receives nblk partial sketches.  In
// tr_lowp_launch.hip.
int launch_pw_lp(int prec, int kind, int64_t s, const void* X, int64_t L, int64_t I, int64_t R,
                 int64_t ldi, const void* Cq, const float* tau, const float* omega,
                 const unsigned* xmax, float* part, int64_t nblk, hipStream_t st);

// Kernel instance a factorization runs in: the register-resident kernel
// (<SM, R, MU>: s <= SM, I <= 256 R, mu <= MU), else the LDS-resident one,
// else the one with its working matrices in global scratch.
enum FactorVariant {
  kRf16x1, kRf16x2, kRf32x1, kRf32x2, kRf48x1, kRf48x2,
  kLds16, kLds32, kLds64, kGlb16, kGlb32, kGlb64, kRf24x1, kRf24x2, kRf40x1, kRf40x2,
  kGlb128,  // 64 < s <= 128: matrices in global scratch, FactorJob::gW set
  kNumFactorVariants
};

// Fused exact power step (k_pw_fused): I <= 128 rows and sketch width
// s <= 32; one partial sketch per block, pw_fused_blocks(J) blocks.  In
// tr_pw_fused.hip; TR_ENOTSUP (nothing launched) when not applicable.
inline bool pw_fused_ok(int64_t I, int64_t J, int64_t s) {
  return I >= 1 && I <= 128 && s >= 1 && s <= 32 && J >= 1;
}
inline int64_t pw_fused_blocks(int64_t J) {
  // one block per compute unit: the wider instances hold one wave per SIMD
  return std::max<int64_t>(1, std::min<int64_t>(256, cdiv(cdiv(J, 16), 4)));
}
int launch_pw_fused(bool f64, const void* X, int64_t L, int64_t I, int64_t R,
                    const double* colw, const double* Yt, int sw, int64_t s, double* part,
                    int64_t* nparts, hipStream_t st);

// One launch of the factor kernel instance `var` over n jobs (one workgroup
// each).  In tr_factor_launch.hip.
int launch_factor_group(int var, const trk::FactorJobs& jobs, int n, int cast_f32,
                        uint32_t* status, hipStream_t st);

// Factorizations whose jobs sit in a device table (n workgroups), in the
// register-resident instances for up to 512 rows: kRf24x2, kRf40x2, kRf48x2.
// status_tab (device, may be null): one status word pointer per job.  In
// tr_factor_inst.hip (those instances' units).
int launch_factor_tab_kRf24x2(const trk::FactorJob* tab, int n, int cast_f32,
                              uint32_t* const* status_tab, hipStream_t st);
int launch_factor_tab_kRf40x2(const trk::FactorJob* tab, int n, int cast_f32,
                              uint32_t* const* status_tab, hipStream_t st);
int launch_factor_tab_kRf48x2(const trk::FactorJob* tab, int n, int cast_f32,
                              uint32_t* const* status_tab, hipStream_t st);

}  // namespace trh

// One factor kernel instance per compilation: TR_FACTOR_INST (a
// FactorVariant) selects it, and the build compiles this file once per
// instance so that they build in parallel.
#include <hip/hip_runtime.h>

#include "tr_factor_rf.hpp"
#include "tr_host.hpp"
#include "tr_factor.hpp"
#include "tr_kernels.hpp"

#ifndef TR_FACTOR_INST
#error "TR_FACTOR_INST selects the factor kernel instance of this unit"
#endif

namespace trh {
namespace {

template <int SM, int R, int MU>
int factor_rf_jobs(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                   hipStream_t st) {
  const size_t lds = trk::RfShape<SM>::lds_bytes();
  if (lds > 65536 &&
      hipFuncSetAttribute((const void*)&trk::k_factor_rf<SM, R, MU>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return TR_EDEVICE;
  hipLaunchKernelGGL((trk::k_factor_rf<SM, R, MU>), dim3((unsigned)n), dim3(trk::RfShape<SM>::NT),
                     lds, st, jobs, cast_f32, status);
  return check_launch();
}

template <int SM, int R, int MU>
int factor_rf_tab(const trk::FactorJob* tab, int n, int cast_f32, uint32_t* const* status_tab,
                  hipStream_t st) {
  const size_t lds = trk::RfShape<SM>::lds_bytes();
  if (lds > 65536 &&
      hipFuncSetAttribute((const void*)&trk::k_factor_rf_tab<SM, R, MU>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return TR_EDEVICE;
  hipLaunchKernelGGL((trk::k_factor_rf_tab<SM, R, MU>), dim3((unsigned)n),
                     dim3(trk::RfShape<SM>::NT), lds, st, tab, cast_f32, status_tab);
  return check_launch();
}

template <int SM, bool G>
int factor_k_jobs(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                  hipStream_t st) {
  size_t lds = 0;
  for (int b = 0; b < n; ++b)
    lds = std::max(lds, trk::FactorShape<SM>::lds_bytes(jobs.j[b].I, jobs.j[b].s, jobs.j[b].mu, G));
  if (lds > 65536 &&
      hipFuncSetAttribute((const void*)&trk::k_factor<SM, G>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return TR_EDEVICE;
  hipLaunchKernelGGL((trk::k_factor<SM, G>), dim3((unsigned)n), dim3(trk::kFactorNT), lds, st,
                     jobs, cast_f32, status);
  return check_launch();
}

}  // namespace

#if TR_FACTOR_INST == 0
static_assert(kRf16x1 == 0, "instance numbering");
int launch_factor_kRf16x1(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st) {
  return factor_rf_jobs<16, 1, 16>(jobs, n, cast_f32, status, st);
}
#endif
#if TR_FACTOR_INST == 1
static_assert(kRf16x2 == 1, "instance numbering");
int launch_factor_kRf16x2(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st) {
  return factor_rf_jobs<16, 2, 16>(jobs, n, cast_f32, status, st);
}
#endif
#if TR_FACTOR_INST == 2
static_assert(kRf32x1 == 2, "instance numbering");
int launch_factor_kRf32x1(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st) {
  return factor_rf_jobs<32, 1, 32>(jobs, n, cast_f32, status, st);
}
#endif
#if TR_FACTOR_INST == 3
static_assert(kRf32x2 == 3, "instance numbering");
int launch_factor_kRf32x2(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st) {
  return factor_rf_jobs<32, 2, 16>(jobs, n, cast_f32, status, st);
}
#endif
#if TR_FACTOR_INST == 4
static_assert(kRf48x1 == 4, "instance numbering");
int launch_factor_kRf48x1(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st) {
  return factor_rf_jobs<48, 1, 48>(jobs, n, cast_f32, status, st);
}
#endif
#if TR_FACTOR_INST == 5
static_assert(kRf48x2 == 5, "instance numbering");
int launch_factor_kRf48x2(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st) {
  return factor_rf_jobs<48, 2, 32>(jobs, n, cast_f32, status, st);
}
int launch_factor_tab_kRf48x2(const trk::FactorJob* tab, int n, int cast_f32,
                         uint32_t* const* status_tab, hipStream_t st) {
  return factor_rf_tab<48, 2, 32>(tab, n, cast_f32, status_tab, st);
}
#endif
#if TR_FACTOR_INST == 6
static_assert(kLds16 == 6, "instance numbering");
int launch_factor_kLds16(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st) {
  return factor_k_jobs<16, false>(jobs, n, cast_f32, status, st);
}
#endif
#if TR_FACTOR_INST == 7
static_assert(kLds32 == 7, "instance numbering");
int launch_factor_kLds32(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st) {
  return factor_k_jobs<32, false>(jobs, n, cast_f32, status, st);
}
#endif
#if TR_FACTOR_INST == 8
static_assert(kLds64 == 8, "instance numbering");
int launch_factor_kLds64(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st) {
  return factor_k_jobs<64, false>(jobs, n, cast_f32, status, st);
}
#endif
#if TR_FACTOR_INST == 9
static_assert(kGlb16 == 9, "instance numbering");
int launch_factor_kGlb16(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st) {
  return factor_k_jobs<16, true>(jobs, n, cast_f32, status, st);
}
#endif
#if TR_FACTOR_INST == 10
static_assert(kGlb32 == 10, "instance numbering");
int launch_factor_kGlb32(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st) {
  return factor_k_jobs<32, true>(jobs, n, cast_f32, status, st);
}
#endif
#if TR_FACTOR_INST == 11
static_assert(kGlb64 == 11, "instance numbering");
int launch_factor_kGlb64(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st) {
  return factor_k_jobs<64, true>(jobs, n, cast_f32, status, st);
}
#endif
#if TR_FACTOR_INST == 12
static_assert(kRf24x1 == 12, "instance numbering");
int launch_factor_kRf24x1(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st) {
  return factor_rf_jobs<24, 1, 24>(jobs, n, cast_f32, status, st);
}
#endif
#if TR_FACTOR_INST == 13
static_assert(kRf24x2 == 13, "instance numbering");
int launch_factor_kRf24x2(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st) {
  return factor_rf_jobs<24, 2, 16>(jobs, n, cast_f32, status, st);
}
int launch_factor_tab_kRf24x2(const trk::FactorJob* tab, int n, int cast_f32,
                         uint32_t* const* status_tab, hipStream_t st) {
  return factor_rf_tab<24, 2, 16>(tab, n, cast_f32, status_tab, st);
}
#endif
#if TR_FACTOR_INST == 14
static_assert(kRf40x1 == 14, "instance numbering");
int launch_factor_kRf40x1(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st) {
  return factor_rf_jobs<40, 1, 40>(jobs, n, cast_f32, status, st);
}
#endif
#if TR_FACTOR_INST == 15
static_assert(kRf40x2 == 15, "instance numbering");
int launch_factor_kRf40x2(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st) {
  return factor_rf_jobs<40, 2, 32>(jobs, n, cast_f32, status, st);
}
int launch_factor_tab_kRf40x2(const trk::FactorJob* tab, int n, int cast_f32,
                         uint32_t* const* status_tab, hipStream_t st) {
  return factor_rf_tab<40, 2, 32>(tab, n, cast_f32, status_tab, st);
}
#endif
#if TR_FACTOR_INST == 16
static_assert(kGlb128 == 16, "instance numbering");
int launch_factor_kGlb128(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                          hipStream_t st) {
  return factor_k_jobs<128, true>(jobs, n, cast_f32, status, st);
}
#endif

}  // namespace trh

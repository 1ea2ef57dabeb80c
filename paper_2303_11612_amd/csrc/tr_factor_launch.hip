// Dispatch of a batch of factorization jobs to its kernel instance (each
// instance is compiled in its own unit from tr_factor_inst.hip).
#include <hip/hip_runtime.h>

#include "tr_host.hpp"

namespace trh {

int launch_factor_kRf16x1(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st);
int launch_factor_kRf16x2(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st);
int launch_factor_kRf32x1(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st);
int launch_factor_kRf32x2(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st);
int launch_factor_kRf48x1(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st);
int launch_factor_kRf48x2(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st);
int launch_factor_kLds16(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st);
int launch_factor_kLds32(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st);
int launch_factor_kLds64(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st);
int launch_factor_kGlb16(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st);
int launch_factor_kGlb32(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st);
int launch_factor_kGlb64(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st);
int launch_factor_kRf24x1(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st);
int launch_factor_kRf24x2(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st);
int launch_factor_kRf40x1(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st);
int launch_factor_kRf40x2(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                      hipStream_t st);

int launch_factor_kGlb128(const trk::FactorJobs& jobs, int n, int cast_f32, uint32_t* status,
                          hipStream_t st);

int launch_factor_group(int var, const trk::FactorJobs& jobs, int n, int cast_f32,
                        uint32_t* status, hipStream_t st) {
  switch (var) {
    case kRf16x1: return launch_factor_kRf16x1(jobs, n, cast_f32, status, st);
    case kRf16x2: return launch_factor_kRf16x2(jobs, n, cast_f32, status, st);
    case kRf32x1: return launch_factor_kRf32x1(jobs, n, cast_f32, status, st);
    case kRf32x2: return launch_factor_kRf32x2(jobs, n, cast_f32, status, st);
    case kRf48x1: return launch_factor_kRf48x1(jobs, n, cast_f32, status, st);
    case kRf48x2: return launch_factor_kRf48x2(jobs, n, cast_f32, status, st);
    case kLds16: return launch_factor_kLds16(jobs, n, cast_f32, status, st);
    case kLds32: return launch_factor_kLds32(jobs, n, cast_f32, status, st);
    case kLds64: return launch_factor_kLds64(jobs, n, cast_f32, status, st);
    case kGlb16: return launch_factor_kGlb16(jobs, n, cast_f32, status, st);
    case kGlb32: return launch_factor_kGlb32(jobs, n, cast_f32, status, st);
    case kGlb64: return launch_factor_kGlb64(jobs, n, cast_f32, status, st);
    case kRf24x1: return launch_factor_kRf24x1(jobs, n, cast_f32, status, st);
    case kRf24x2: return launch_factor_kRf24x2(jobs, n, cast_f32, status, st);
    case kRf40x1: return launch_factor_kRf40x1(jobs, n, cast_f32, status, st);
    case kRf40x2: return launch_factor_kRf40x2(jobs, n, cast_f32, status, st);
    case kGlb128: return launch_factor_kGlb128(jobs, n, cast_f32, status, st);
    default: return TR_EINVAL;
  }
}

}  // namespace trh

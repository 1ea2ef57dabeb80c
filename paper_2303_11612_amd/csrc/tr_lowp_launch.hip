// Launchers of the fused low-precision power step: one kernel instance per
// source type, operand format, row tiling (MI) and sketch width (NKT).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "tr_host.hpp"
#include "tr_lowp.hpp"

namespace trh {
namespace {

template <typename Tin, typename OP, int MI, int NKT>
int pw_lp_k(const void* X, int64_t L, int64_t I, int64_t R, int64_t ldi, const void* Cq,
            const float* tau, const float* omega, const unsigned* xmax, float* part,
            int64_t nblk, hipStream_t st) {
  const size_t lds = lp_lds_bytes(MI, NKT);
  // float tensor form with contiguous columns: 16-byte row loads
  const bool v4 = std::is_same<Tin, float>::value && L == 1 && I % 4 == 0 && ldi % 4 == 0 &&
                  reinterpret_cast<uintptr_t>(X) % 16 == 0;
  auto* fn = v4 ? &trk::k_pw_lp<Tin, OP, MI, NKT, std::is_same<Tin, float>::value>
                : &trk::k_pw_lp<Tin, OP, MI, NKT>;
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  hipLaunchKernelGGL(fn, dim3((unsigned)nblk), dim3(trk::kPwWaves * trk::kWave), lds, st,
                     (const Tin*)X, L, I, R, ldi, (const typename OP::stor*)Cq, tau, omega,
                     xmax, part);
  return check_launch();
}

template <typename Tin, typename OP, int MI>
int pw_lp_n(int nkt, const void* X, int64_t L, int64_t I, int64_t R, int64_t ldi,
            const void* Cq, const float* tau, const float* omega, const unsigned* xmax,
            float* part, int64_t nblk, hipStream_t st) {
  switch (nkt) {
    case 1: return pw_lp_k<Tin, OP, MI, 1>(X, L, I, R, ldi, Cq, tau, omega, xmax, part, nblk, st);
    case 2: return pw_lp_k<Tin, OP, MI, 2>(X, L, I, R, ldi, Cq, tau, omega, xmax, part, nblk, st);
    case 3: return pw_lp_k<Tin, OP, MI, 3>(X, L, I, R, ldi, Cq, tau, omega, xmax, part, nblk, st);
    default: return TR_ENOTSUP;
  }
}

template <typename Tin, typename OP>
int pw_lp_m(int64_t s, const void* X, int64_t L, int64_t I, int64_t R, int64_t ldi,
            const void* Cq, const float* tau, const float* omega, const unsigned* xmax,
            float* part, int64_t nblk, hipStream_t st) {
  const int nkt = lp_nkt(s);
  switch (lp_mi(I)) {
    case 1: return pw_lp_n<Tin, OP, 1>(nkt, X, L, I, R, ldi, Cq, tau, omega, xmax, part, nblk, st);
    case 2: return pw_lp_n<Tin, OP, 2>(nkt, X, L, I, R, ldi, Cq, tau, omega, xmax, part, nblk, st);
    default: return pw_lp_n<Tin, OP, 4>(nkt, X, L, I, R, ldi, Cq, tau, omega, xmax, part, nblk, st);
  }
}

template <typename OP>
int pw_lp_src(int kind, int64_t s, const void* X, int64_t L, int64_t I, int64_t R, int64_t ldi,
              const void* Cq, const float* tau, const float* omega, const unsigned* xmax,
              float* part, int64_t nblk, hipStream_t st) {
  switch (kind) {
    case kLpF32:
      return pw_lp_m<float, OP>(s, X, L, I, R, ldi, Cq, tau, omega, xmax, part, nblk, st);
    case kLpF64:
      return pw_lp_m<double, OP>(s, X, L, I, R, ldi, Cq, tau, omega, xmax, part, nblk, st);
    default:
      return pw_lp_m<typename OP::stor, OP>(s, X, L, I, R, ldi, Cq, tau, omega, xmax, part,
                                             nblk, st);
  }
}

}  // namespace

int launch_pw_lp(int prec, int kind, int64_t s, const void* X, int64_t L, int64_t I, int64_t R,
                 int64_t ldi, const void* Cq, const float* tau, const float* omega,
                 const unsigned* xmax, float* part, int64_t nblk, hipStream_t st) {
  if (prec == TR_PREC_FP8E4M3)
    return pw_lp_src<trk::OpFp8>(kind, s, X, L, I, R, ldi, Cq, tau, omega, xmax, part, nblk, st);
  return pw_lp_src<trk::OpBf16>(kind, s, X, L, I, R, ldi, Cq, tau, omega, xmax, part, nblk, st);
}

}  // namespace trh

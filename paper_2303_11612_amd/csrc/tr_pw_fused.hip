// Launch of the fused exact power step (k_pw_fused), in a unit of its own so
// that its instances build in parallel with the rest.
#include <hip/hip_runtime.h>

#include "tr_host.hpp"
#include "tr_power.hpp"

namespace trh {
namespace {

template <typename Tin, int NKT, int NCH>
void pw_fused_k(const Tin* X, int64_t L, int64_t I, int64_t R, const double* colw,
                const double* Yt, int sw, int s, double* part, int64_t nblk, hipStream_t st) {
  hipLaunchKernelGGL((trk::k_pw_fused<Tin, NKT, NCH>), dim3((unsigned)nblk),
                     dim3(trk::kPwWaves * trk::kWave), 0, st, X, L, I, R, colw, Yt, sw, s, part);
}

template <typename Tin, int NKT>
int pw_fused_n(const Tin* X, int64_t L, int64_t I, int64_t R, const double* colw,
               const double* Yt, int sw, int s, double* part, int64_t nblk, hipStream_t st) {
  switch (cdiv(I, 16)) {
    case 1: pw_fused_k<Tin, NKT, 1>(X, L, I, R, colw, Yt, sw, s, part, nblk, st); break;
    case 2: pw_fused_k<Tin, NKT, 2>(X, L, I, R, colw, Yt, sw, s, part, nblk, st); break;
    case 3: pw_fused_k<Tin, NKT, 3>(X, L, I, R, colw, Yt, sw, s, part, nblk, st); break;
    case 4: pw_fused_k<Tin, NKT, 4>(X, L, I, R, colw, Yt, sw, s, part, nblk, st); break;
    case 5: pw_fused_k<Tin, NKT, 5>(X, L, I, R, colw, Yt, sw, s, part, nblk, st); break;
    case 6: pw_fused_k<Tin, NKT, 6>(X, L, I, R, colw, Yt, sw, s, part, nblk, st); break;
    case 7: pw_fused_k<Tin, NKT, 7>(X, L, I, R, colw, Yt, sw, s, part, nblk, st); break;
    case 8: pw_fused_k<Tin, NKT, 8>(X, L, I, R, colw, Yt, sw, s, part, nblk, st); break;
    default: return TR_ENOTSUP;
  }
  return check_launch();
}

}  // namespace

int launch_pw_fused(bool f64, const void* X, int64_t L, int64_t I, int64_t R,
                    const double* colw, const double* Yt, int sw, int64_t s, double* part,
                    int64_t* nparts, hipStream_t st) {
  if (!pw_fused_ok(I, L * R, s)) return TR_ENOTSUP;
  // float64 input, 8 row chunks and two column groups would spill registers
  if (f64 && s > 16 && cdiv(I, 16) == 8) return TR_ENOTSUP;
  const int64_t nblk = pw_fused_blocks(L * R);
  const int si = (int)s;
  int rc;
  if (s <= 16)
    rc = f64 ? pw_fused_n<double, 1>((const double*)X, L, I, R, colw, Yt, sw, si, part, nblk, st)
             : pw_fused_n<float, 1>((const float*)X, L, I, R, colw, Yt, sw, si, part, nblk, st);
  else
    rc = f64 ? pw_fused_n<double, 2>((const double*)X, L, I, R, colw, Yt, sw, si, part, nblk, st)
             : pw_fused_n<float, 2>((const float*)X, L, I, R, colw, Yt, sw, si, part, nblk, st);
  if (rc == TR_OK) *nparts = nblk;
  return rc;
}

}  // namespace trh

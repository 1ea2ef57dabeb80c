// Dense contractions on the FP64 matrix cores: the power-scheme products
// C <- X_(n) D X_(n)^T C (Strategy A: two skinny products per step) and the
// mode-1 shrink Y = X x_1 Q^T.  v_mfma_f64_16x16x4f64 lane
// layout (lane l = 16 * g + h, h = l % 16, g = l / 16):
//   A (16 x 4): lane l holds A[h][g];  B (4 x 16): lane l holds B[g][h];
//   D (16 x 16): lane l, item v holds D[g + 4 v][h].
// The source is the L x I x R column-major view of a mode-n unfolding,
// X_(n)(i, j) = X[l + L (i + I r)], j = l + L r (L == 1: a plain I x J
// matrix such as the gathered C'_n).  Inputs in float32 are widened to
// float64 on load; every product and sum is float64.  Sums run in a fixed
// order, so results are bitwise reproducible.  Out-of-range operands are
// loaded from a clamped (valid, finite) address and multiplied by 0, which
// keeps every load unconditional: a select on a loaded value would let the
// compiler turn the load into a branch that waits for it on its own.
#pragma once

#include "tr_device.hpp"

namespace trk {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kPwWaves = 4;
constexpr int kPwBatch = 4;  // loop iterations whose loads are issued together

// W(j, k) = d_j sum_i X_(n)(i, j) Y(i, k) for j < J, k < 16 NKT (row-major,
// row stride 16 NKT; columns k >= s come out zero).  Y is read from its
// row-major copy Yt (row stride sw >= s, zero padding).  Block: one tile of
// 16 columns j; its four waves take interleaved quarters of the rows i and
// their partial tiles are added in LDS (wave order 0..3).  WPT (few rows):
// each wave takes a tile of its own (64 columns per block) and all its rows,
// in order, with no reduction across waves.
template <typename Tin, int NKT, bool WPT = false>
__global__ void __launch_bounds__(kPwWaves * kWave)
k_pw_w(const Tin* __restrict__ X, int64_t L, int64_t I, int64_t R,
       const double* __restrict__ colw, const double* __restrict__ Yt, int sw,
       double* __restrict__ W, const int64_t* __restrict__ gidx = nullptr) {
  constexpr int SP = 16 * NKT;
  constexpr int kSplit = WPT ? 1 : kPwWaves;  // waves sharing a tile's rows
  __shared__ f64x4 red[WPT ? 1 : kPwWaves - 1][NKT][kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int h = lane & 15, g = lane >> 4;
  const int64_t J = L * R;
  const int64_t tile = WPT ? (int64_t)blockIdx.x * kPwWaves + wid : (int64_t)blockIdx.x;
  const int rw = WPT ? 0 : wid;  // this wave's first chunk
  const int64_t j = tile * 16 + h;
  const bool jok = j < J;
  const int64_t jc = jok ? j : J - 1;
  const int64_t js = gidx ? gidx[jc] : jc;  // gathered through the index (L == 1)
  const int64_t r = js / L;
  const Tin* xc = X + (js - r * L) + L * I * r;  // X_(n)(i, js) = xc[L i]
  const int64_t nch = (I + 15) / 16;             // chunks of 16 rows
  f64x4 acc[NKT];
#pragma unroll
  for (int kt = 0; kt < NKT; ++kt) acc[kt] = f64x4{0.0, 0.0, 0.0, 0.0};
  // chunks rw, rw + kSplit, ...; kPwBatch of them have their loads in flight together
  for (int64_t c0 = rw; c0 < nch; c0 += kSplit * kPwBatch) {
    // all loads of the batch first (raw values), then masks and products
    Tin xr[kPwBatch][4];
    double yr[kPwBatch][4][NKT];
#pragma unroll
    for (int u = 0; u < kPwBatch; ++u) {
      const int64_t c = c0 + kSplit * u;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        // rows 16c + 4g + t feed the t-th product of chunk c
        const int64_t i = 16 * c + 4 * g + t;
        const int64_t ic = i < I ? i : I - 1;
        xr[u][t] = xc[L * ic];
#pragma unroll
        for (int kt = 0; kt < NKT; ++kt) {
          const int k = 16 * kt + h;
          yr[u][t][kt] = Yt[ic * sw + (k < sw ? k : sw - 1)];
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < kPwBatch; ++u)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bool iok = 16 * (c0 + kSplit * u) + 4 * g + t < I;
        const double b = (double)xr[u][t] * ((jok && iok) ? 1.0 : 0.0);
#pragma unroll
        for (int kt = 0; kt < NKT; ++kt) {
          const double a = yr[u][t][kt] * ((iok && 16 * kt + h < sw) ? 1.0 : 0.0);
          acc[kt] = mfma_f64(a, b, acc[kt]);
        }
      }
  }
  if constexpr (!WPT) {
    if (wid > 0) {
#pragma unroll
      for (int kt = 0; kt < NKT; ++kt) red[wid - 1][kt][lane] = acc[kt];
    }
    __syncthreads();
  }
  if ((WPT || wid == 0) && jok) {
    const double d = colw ? colw[j] : 1.0;
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt) {
      f64x4 v = acc[kt];
      if constexpr (!WPT) {
#pragma unroll
        for (int w = 0; w < kPwWaves - 1; ++w) v += red[w][kt][lane];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) W[j * SP + 16 * kt + g + 4 * q] = v[q] * d;
    }
  }
}

// part_b(i, k) = sum over the columns j of range b of X_(n)(i, j) W(j, k),
// for i < I, k < s (column-major I x s per range).  Block (x, y): rows
// 16 MT x .. 16 MT (x + 1), column range [y jper, (y + 1) jper); its four
// waves take consecutive quarters of the range (multiples of 4 columns) and
// their tiles are added in LDS (wave order 0..3).  The partial sums of the
// ranges are added by k_reduce_parts in increasing b.  With one range and Y
// set, the block writes what k_reduce_parts would instead: Y (column-major
// I x s), its row-major copy Yt (row stride ldyt) and the non-finite flag.
template <typename Tin, int NKT, int MT>
__global__ void __launch_bounds__(kPwWaves * kWave)
k_pw_y(const Tin* __restrict__ X, int64_t L, int64_t I, int64_t R,
       const double* __restrict__ W, int s, int64_t jper, double* __restrict__ part,
       const int64_t* __restrict__ gidx = nullptr, double* __restrict__ Y = nullptr,
       double* __restrict__ Yt = nullptr, int ldyt = 0, uint32_t* __restrict__ status = nullptr) {
  constexpr int SP = 16 * NKT;
  __shared__ f64x4 red[kPwWaves - 1][MT][NKT][kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int h = lane & 15, g = lane >> 4;
  const int64_t J = L * R, LI = L * I, nX = L * I * R;
  const int64_t ib = (int64_t)blockIdx.x * 16 * MT;
  const int64_t jb = (int64_t)blockIdx.y * jper, je = min(J, jb + jper);
  const int64_t wq = ((je - jb + 4 * kPwWaves - 1) / (4 * kPwWaves)) * 4;
  const int64_t ja = jb + wid * wq, jz = min(je, ja + wq);
  int64_t roff[MT];
  bool rok[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int64_t i = ib + 16 * mt + h;
    rok[mt] = i < I;
    roff[mt] = L * (rok[mt] ? i : I - 1);
  }
  f64x4 acc[MT][NKT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt) acc[mt][kt] = f64x4{0.0, 0.0, 0.0, 0.0};
  if (ja < jz) {
    // this lane's column j = j0 + g, tracked as (l, r) without dividing;
    // kPwBatch groups of 4 columns have their loads in flight together
    int64_t r = (ja + g) / L, l = ja + g - r * L;
    for (int64_t j0 = ja; j0 < jz; j0 += 4 * kPwBatch) {
      // all loads of the batch first (raw values), then masks and products
      Tin xr[kPwBatch][MT];
      double wr[kPwBatch][NKT];
#pragma unroll
      for (int u = 0; u < kPwBatch; ++u) {
        const int64_t j = j0 + 4 * u + g;
        const int64_t jw = j < jz ? j : jz - 1;
        // through the index (L == 1): column gidx[j] of the source, whose
        // rows are all in range
        const int64_t base = gidx ? I * gidx[jw] : l + LI * r;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int64_t e = base + roff[mt];
          xr[u][mt] = X[gidx ? e : (e < nX ? e : nX - 1)];
        }
#pragma unroll
        for (int kt = 0; kt < NKT; ++kt) wr[u][kt] = W[jw * SP + 16 * kt + h];
        l += 4;
        while (l >= L) {
          l -= L;
          ++r;
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < kPwBatch; ++u) {
        const bool jok = j0 + 4 * u + g < jz;
        double a[MT], b[NKT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) a[mt] = (double)xr[u][mt] * ((jok && rok[mt]) ? 1.0 : 0.0);
#pragma unroll
        for (int kt = 0; kt < NKT; ++kt) b[kt] = wr[u][kt] * (jok ? 1.0 : 0.0);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int kt = 0; kt < NKT; ++kt) acc[mt][kt] = mfma_f64(a[mt], b[kt], acc[mt][kt]);
      }
    }
  }
  if (wid > 0) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int kt = 0; kt < NKT; ++kt) red[wid - 1][mt][kt][lane] = acc[mt][kt];
  }
  __syncthreads();
  if (wid == 0) {
    double* out = part + (int64_t)blockIdx.y * I * s;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int kt = 0; kt < NKT; ++kt) {
        f64x4 v = acc[mt][kt];
#pragma unroll
        for (int w = 0; w < kPwWaves - 1; ++w) v += red[w][mt][kt][lane];
        const int k = 16 * kt + h;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t i = ib + 16 * mt + g + 4 * q;
          if (i < I && k < s) {
            if (Y) {
              Y[i + I * k] = v[q];
              Yt[i * ldyt + k] = v[q];
              if (!isfinite(v[q]) && status) atomicOr(status, kDevNonFinite);
            } else {
              out[i + I * k] = v[q];
            }
          }
        }
      }
  }
}


// Mode-1 shrink on the matrix cores: Y(k, j) = sum_i Q(i, k) X(i, j) for the
// L == 1 view (X is I x R, column-major, I a multiple of 4 and 16-byte
// aligned), k < kout, written as Y[k + kout j] in float64.  Q^T is staged once
// per block in LDS as rows of 16 NKT (zero beyond `width`) and zero rows up
// to a whole number of batches, so rows beyond I contribute exactly 0 and no
// product needs a mask.  Blocks of WAVES waves loop over tiles of 16 columns,
// one tile per wave at a time.  A 16-row step gives each lane group g rows 4g .. 4g + 3 of
// its column as one 16-byte vector load (a group beyond the column reads the
// last group again; a column beyond R reads column R - 1, and its outputs are
// not stored).  Work items are (tile, B steps); the loads of the next item
// are in flight while the current one is multiplied out, from two
// alternating register buffers.  STR: the columns are those of an L x I x R
// view (column j = l + L r at X + l + L I r, rows at stride L, one scalar
// load per row clamped to row I - 1; any I); the outputs keep the layout
// Y[k + kout j] (the first product of a power step, W = X^T Y).
template <typename Tin, int B, bool STR = false>
__device__ __forceinline__ void ttm1_load(const Tin* __restrict__ col, int64_t L, int64_t I,
                                          int64_t s0, int g, Tin (&xr)[B][4]) {
#pragma unroll
  for (int u = 0; u < B; ++u) {
    const int64_t i0 = 16 * (s0 + u) + 4 * g;
    const int64_t ic = i0 + 4 <= I ? i0 : I - 4;
    if constexpr (STR) {
#pragma unroll
      for (int t = 0; t < 4; ++t) xr[u][t] = col[L * (i0 + t < I ? i0 + t : I - 1)];
    } else if constexpr (sizeof(Tin) == 4) {
      const f32x4 v = *reinterpret_cast<const f32x4*>(col + ic);
#pragma unroll
      for (int t = 0; t < 4; ++t) xr[u][t] = v[t];
    } else {
      const f64x2 v0 = *reinterpret_cast<const f64x2*>(col + ic);
      const f64x2 v1 = *reinterpret_cast<const f64x2*>(col + ic + 2);
      xr[u][0] = v0[0];
      xr[u][1] = v0[1];
      xr[u][2] = v1[0];
      xr[u][3] = v1[1];
    }
  }
}

template <typename Tin, int NKT, int B, bool STR = false, int WAVES = kPwWaves>
__global__ void __launch_bounds__(WAVES * kWave)
k_ttm1_mfma(const Tin* __restrict__ X, int64_t L, int64_t I, int64_t R,
            const double* __restrict__ Qt, int width, int kout, double* __restrict__ Y) {
  constexpr int SP = 16 * NKT;
  extern __shared__ double qs[];  // qs[i * SP + k] = Q(i, k), zero rows i >= I
  const int64_t nsteps = (I + 15) / 16;
  const int64_t nitem = (nsteps + B - 1) / B;  // items per tile
  const int64_t ipad = nitem * B * 16;
  for (int64_t e = threadIdx.x; e < ipad * SP; e += WAVES * kWave) {
    const int64_t i = e / SP;
    const int k = (int)(e - i * SP);
    qs[e] = (i < I && k < width) ? Qt[(i < I ? i : 0) * width + (k < width ? k : 0)] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int h = lane & 15, g = lane >> 4;
  const int64_t ntile = (R + 15) / 16;
  const int64_t stride = (int64_t)gridDim.x * WAVES;
  int64_t tile = (int64_t)blockIdx.x * WAVES + wid, s0 = 0;
  if (tile >= ntile) return;
  auto colp = [&](int64_t tl) {
    const int64_t j0 = tl * 16 + h;
    const int64_t j = j0 < R ? j0 : R - 1;
    if constexpr (STR) {
      const int64_t r = j / L;
      return X + (j - r * L) + L * I * r;
    } else {
      return X + j * I;
    }
  };
  Tin xa[B][4], xb[B][4];
  ttm1_load<Tin, B, STR>(colp(tile), L, I, s0, g, xa);
  f64x4 acc[NKT];
#pragma unroll
  for (int kt = 0; kt < NKT; ++kt) acc[kt] = f64x4{0.0, 0.0, 0.0, 0.0};
  // one work item: prefetch the next into `nxt`, multiply out `cur`
  auto item = [&](Tin (&cur)[B][4], Tin (&nxt)[B][4]) __attribute__((always_inline)) -> bool {
    int64_t ntl = tile, ns = s0 + B;
    if (ns >= nsteps) {
      ns = 0;
      ntl += stride;
    }
    const bool more = ntl < ntile;
    // unconditional (the last item reloads its own rows): a conditional
    // prefetch would make every wait below count as if it had not been issued
    ttm1_load<Tin, B, STR>(colp(more ? ntl : tile), L, I, more ? ns : s0, g, nxt);
    __builtin_amdgcn_sched_barrier(0);
    const double* qb = qs + (16 * s0 + 4 * g) * SP + h;
#pragma unroll
    for (int u = 0; u < B; ++u)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double b = (double)cur[u][t];
#pragma unroll
        for (int kt = 0; kt < NKT; ++kt)
          acc[kt] = mfma_f64(qb[(16 * u + t) * SP + 16 * kt], b, acc[kt]);
      }
    if (s0 + B >= nsteps) {  // tile complete
      const int64_t j = tile * 16 + h;
      if (j < R) {
#pragma unroll
        for (int kt = 0; kt < NKT; ++kt)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int k = 16 * kt + g + 4 * q;
            if (k < kout) Y[k + (int64_t)kout * j] = acc[kt][q];
          }
      }
#pragma unroll
      for (int kt = 0; kt < NKT; ++kt) acc[kt] = f64x4{0.0, 0.0, 0.0, 0.0};
    }
    tile = ntl;
    s0 = ns;
    return more;
  };
  while (item(xa, xb) && item(xb, xa)) {
  }
}

// One exact power step in a single sweep, for I <= 16 NCH (NCH <= 8) rows and
// sketch width s <= 16 NKT (NKT <= 2): for each 16-column tile J_t of
// X_(n) (one wave per tile at a time, persistent),
//   W_t = D_t X_(n)(:, J_t)^T Y      (16 x 16 NKT, on the matrix cores,
//                                      Y staged in LDS, zero beyond I and s)
//   P  += X_(n)(:, J_t) W_t          (I x 16 NKT, accumulated in registers)
// so W never leaves the compute unit and X is read from HBM once.  W_t goes
// through a per-wave LDS tile to change operand layout (row j = column of the
// tile, scaled by the column weight d_j, zero for columns past J).  X is
// loaded twice per tile, in the two operand layouts (the second load hits
// the caches).  A block adds its four waves' P in wave order and writes
// part[block] (column-major I x s); k_reduce_parts adds the blocks in order.
__device__ __forceinline__ void wave_lds_order() {
  // LDS operations of one wave complete in issue order; this keeps the
  // compiler from moving LDS reads and writes across it
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

template <typename Tin, int NKT, int NCH>
__global__ void __launch_bounds__(kPwWaves * kWave)
k_pw_fused(const Tin* __restrict__ X, int64_t L, int64_t I, int64_t R,
           const double* __restrict__ colw, const double* __restrict__ Yt, int sw, int s,
           double* __restrict__ part) {
  constexpr int SP = 16 * NKT, IP = 16 * NCH;
  __shared__ double ys[IP * SP];               // Y(i, k), zero for i >= I or k >= sw
  __shared__ double wl[kPwWaves][16 * SP];     // per wave: W(j, k) of its tile, row j
  __shared__ f64x4 red[kPwWaves - 1][NKT][kWave];
  for (int e = threadIdx.x; e < IP * SP; e += kPwWaves * kWave) {
    const int i = e / SP, k = e - i * SP;
    ys[e] = (i < I && k < sw) ? Yt[(int64_t)(i < I ? i : 0) * sw + (k < sw ? k : 0)] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int h = lane & 15, g = lane >> 4;
  const int64_t J = L * R, ntile = (J + 15) / 16;
  const int64_t stride = (int64_t)gridDim.x * kPwWaves;
  auto colp = [&](int64_t j) {
    const int64_t jc = j < J ? j : J - 1;
    const int64_t r = jc / L;
    return X + (jc - r * L) + L * I * r;
  };
  f64x4 acc[NCH][NKT];
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt) acc[c][kt] = f64x4{0.0, 0.0, 0.0, 0.0};
  double* w = wl[wid];
  // B layout of the first product: rows 16c + 4g + t of column 16 tile + h;
  // A layout of the second: row 16c + h of columns 16 tile + 4q + g.  Loads
  // overlap the products: a tile's A operands are issued before its first
  // product, the next tile's B operands before its second product (past the
  // last tile a wave reloads its own tile).
  auto load_b = [&](int64_t tl, Tin (&xb)[NCH][4]) __attribute__((always_inline)) {
    const Tin* pb = colp(tl * 16 + h);
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t i = 16 * c + 4 * g + t;
        xb[c][t] = pb[L * (i < I ? i : I - 1)];
      }
  };
  auto load_a = [&](int64_t tl, Tin (&xa)[NCH][4]) __attribute__((always_inline)) {
    const Tin* pa[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) pa[q] = colp(tl * 16 + 4 * q + g);
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int64_t i = 16 * c + h;
#pragma unroll
      for (int q = 0; q < 4; ++q) xa[c][q] = pa[q][L * (i < I ? i : I - 1)];
    }
  };
  int64_t tile = (int64_t)blockIdx.x * kPwWaves + wid;
  if (tile < ntile) {
    Tin xb[NCH][4], xa[NCH][4];
    load_b(tile, xb);
    for (; tile < ntile; tile += stride) {
      load_a(tile, xa);
      __builtin_amdgcn_sched_barrier(0);
      // W^T(k, j) = sum_i Y(i, k) X(i, j): lane (g, h), item v holds k = 16 kt + g + 4 v, j = h
      f64x4 aw[NKT];
#pragma unroll
      for (int kt = 0; kt < NKT; ++kt) aw[kt] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const double b = (double)xb[c][t];
          const double* yr = ys + (16 * c + 4 * g + t) * SP + h;
#pragma unroll
          for (int kt = 0; kt < NKT; ++kt) aw[kt] = mfma_f64(yr[16 * kt], b, aw[kt]);
        }
      __builtin_amdgcn_sched_barrier(0);
      load_b(tile + stride < ntile ? tile + stride : tile, xb);
      __builtin_amdgcn_sched_barrier(0);
      const int64_t jb = tile * 16 + h;
      double d = 0.0;
      if (jb < J) d = colw ? colw[jb] : 1.0;
#pragma unroll
      for (int kt = 0; kt < NKT; ++kt)
#pragma unroll
        for (int v = 0; v < 4; ++v) w[h * SP + 16 * kt + g + 4 * v] = aw[kt][v] * d;
      wave_lds_order();
      // P(i, k) += sum_j X(i, j) W(j, k): A = X(16c + h, 4q + g), B = W(4q + g, 16 kt + h)
      double wb[4][NKT];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int kt = 0; kt < NKT; ++kt) wb[q][kt] = w[(4 * q + g) * SP + 16 * kt + h];
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double a = (double)xa[c][q];
#pragma unroll
          for (int kt = 0; kt < NKT; ++kt) acc[c][kt] = mfma_f64(a, wb[q][kt], acc[c][kt]);
        }
      wave_lds_order();
    }
  }
  // lane (g, h), item v of acc[c][kt]: row 16c + g + 4v, column k = 16 kt + h
  double* out = part + (int64_t)blockIdx.x * I * s;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    if (wid > 0) {
#pragma unroll
      for (int kt = 0; kt < NKT; ++kt) red[wid - 1][kt][lane] = acc[c][kt];
    }
    __syncthreads();
    if (wid == 0) {
#pragma unroll
      for (int kt = 0; kt < NKT; ++kt) {
        f64x4 v = acc[c][kt];
#pragma unroll
        for (int ww = 0; ww < kPwWaves - 1; ++ww) v += red[ww][kt][lane];
        const int k = 16 * kt + h;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t i = 16 * c + g + 4 * q;
          if (i < I && k < s) out[i + I * k] = v[q];
        }
      }
    }
    __syncthreads();
  }
}

}  // namespace trk

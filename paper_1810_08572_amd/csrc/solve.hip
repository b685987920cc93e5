// Solve phase: sparse matrix-vector kernels with fused epilogues, the
// Chebyshev smoother, the V-cycle and preconditioned conjugate gradients
// (the multigrid-preconditioned Krylov solve of section 2.5).
//
// Layout: the finest operator is applied from a slot-major ELL copy of its
// off-diagonal part (one thread per row, every slot load coalesced) plus the
// diagonal; coarse operators, P and R are CSR, applied by groups of LPR
// lanes per row with a shuffle reduction inside the group.  Reductions are
// deterministic and fence-free: producers write one partial per block,
// consumers add the partials in a fixed order.
#include <hip/hip_ext.h>

#include "common.h"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace ppe {
namespace {

enum Epi : int {
  E_SPMV = 0,   // y = A x
  E_RESID = 1,  // y = b - A x
  E_CHEB = 2,   // r = (b - A x)/diag; d = c1 d + c2 r; y = x + d
  E_DOT = 3,    // y = A x, partial sums of x.y
  E_POWER = 4,  // y = (A x)/diag / ||x||, partial sums of y.y
  E_CHEB0 = 5,  // the first two Chebyshev steps from a zero guess in one
                // pass: x = c0 b/diag is formed on the fly (for the row and
                // its neighbours), then the E_CHEB step from d = x
};

// partial-sum slots (each kRedBlocks doubles) in s->partial: power iteration
enum Slot : int { P_POW = 0 /* 0, 1 */, P_NSLOTS = 2 };
// device scalars in s->scal
enum Scal : int { S_POW = 0, S_N = 2 };

// Matrix values come in type M (FP64, or the FP32 copy of the mixed mode);
// vectors and all arithmetic are FP64 in both modes, so the V-cycle is one
// fixed linear operator of the (rounded) hierarchy either way.
//
// The smoothing steps scale the residual by a diagonal sd: the matrix
// diagonal for the Chebyshev smoother, the row l1 norms for l1-Jacobi.  One
// step is r = (b - A x)/sd; d = c1 d + c2 r; y = x + d, which with c1 = 0,
// c2 = 1 is an l1-Jacobi sweep.  `diag` is always the matrix diagonal (the
// finest level's product and the power steps read it).


// Operand of the matrix product: x_j, or for E_CHEB0 the first Chebyshev
// iterate c0 b_j / diag_j (the same expression the unfused first step stores).
template <int EPI, class M>
__device__ __forceinline__ double operand(int j, const double* __restrict__ x,
                                          const double* __restrict__ b,
                                          const M* __restrict__ sd, double c0) {
  if (EPI == E_CHEB0) return c0 * (b[j] / (double)sd[j]);
  return x[j];
}

template <int EPI, class M>
__device__ __forceinline__ double epilogue(int i, double ax, const double* __restrict__ x,
                                           const double* __restrict__ b,
                                           const M* __restrict__ diag,
                                           const M* __restrict__ sd, double* __restrict__ d,
                                           double c1, double c2, double scale,
                                           double* __restrict__ y, double c0 = 0.0) {
  if (EPI == E_CHEB0) {
    const double di = (double)sd[i];
    const double x1 = c0 * (b[i] / di);
    const double r = (b[i] - ax) / di;
    const double dn = c1 * x1 + c2 * r;
    d[i] = dn;
    y[i] = x1 + dn;
    return 0.0;
  } else if (EPI == E_SPMV) {
    y[i] = ax;
    return 0.0;
  } else if (EPI == E_RESID) {
    y[i] = b[i] - ax;
    return 0.0;
  } else if (EPI == E_CHEB) {
    const double r = (b[i] - ax) / (double)sd[i];
    const double dn = (c1 == 0.0 ? 0.0 : c1 * d[i]) + c2 * r;
    d[i] = dn;
    y[i] = x[i] + dn;
    return 0.0;
  } else if (EPI == E_DOT) {
    y[i] = ax;
    return x[i] * ax;
  } else {
    const double v = (ax / (double)diag[i]) * scale;
    y[i] = v;
    return v * v;
  }
}

// Off-diagonal part of row i of an ELL matrix (slot-major, n rows) added to
// s in slot order.  With WM > 0 (W <= WM) the slot loop is unrolled, so every
// column index, and then every gathered operand, is requested before the
// first one is used.
template <int EPI, int WM, class M>
__device__ __forceinline__ double ell_row(double s, int i, int n, int W,
                                          const int* __restrict__ ecol,
                                          const M* __restrict__ eval,
                                          const double* __restrict__ x,
                                          const double* __restrict__ b,
                                          const M* __restrict__ sd, double c0) {
  if (WM > 0) {
    int col[WM > 0 ? WM : 1];
    M v[WM > 0 ? WM : 1];
    if (W == WM) {
      // every slot stored (the hexahedral case): no condition at all, so the
      // loads issue back to back whatever the value type
#pragma unroll
      for (int k = 0; k < WM; ++k) {
        const size_t e = (size_t)k * n + i;
        col[k] = ecol[e];
        v[k] = eval[e];
      }
    } else {
#pragma unroll
      for (int k = 0; k < WM; ++k) {
        const size_t e = (size_t)k * n + i;
        col[k] = k < W ? ecol[e] : i;
        v[k] = k < W ? eval[e] : M(0);
      }
    }
    double g[WM > 0 ? WM : 1];
#pragma unroll
    for (int k = 0; k < WM; ++k) g[k] = operand<EPI, M>(col[k], x, b, sd, c0);
#pragma unroll
    for (int k = 0; k < WM; ++k)
      if (k < W) s = s + (double)v[k] * g[k];
    return s;
  }
  for (int k = 0; k < W; ++k) {
    const size_t e = (size_t)k * n + i;
    s = s + (double)eval[e] * operand<EPI, M>(ecol[e], x, b, sd, c0);
  }
  return s;
}

// ---- finest level: ELL, one thread per row (grid-stride)
template <int EPI, class M, int WM>
__global__ void __launch_bounds__(kBlock) k_ell(int n, int W, const int* __restrict__ ecol,
                                                const M* __restrict__ eval,
                                                const M* __restrict__ diag,
                                                const M* __restrict__ sd,
                                                const double* __restrict__ x,
                                                const double* __restrict__ b,
                                                double* __restrict__ d, double c1, double c2,
                                                double* __restrict__ y,
                                                double* __restrict__ partials, double c0) {
  double dot = 0.0;
  for (int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; i < n;
       i += gridDim.x * kBlock) {
    double s = (double)diag[i] * operand<EPI, M>(i, x, b, sd, c0);
    s = ell_row<EPI, WM, M>(s, i, n, W, ecol, eval, x, b, sd, c0);
    dot += epilogue<EPI, M>(i, s, x, b, diag, sd, d, c1, c2, 1.0, y, c0);
  }
  if (EPI == E_DOT) {
    double v[1] = {dot};
    write_partials<kBlock, 1>(v, partials);
  }
}

// ---- CSR, LPR lanes per row; every lane runs the same trip count so the
// group shuffles always see all lanes.

// s + the sum over the entries k0 + lane, k0 + lane + LPR, ... (< k1) of a
// CSR row of v[k] op(ci[k]), added in that order; the loads of U entries are
// requested before the first is used (the order of the sum is that of the
// plain loop).
// FP32 values (the mixed V-cycle) are loaded unconditionally, from the
// lane's first entry past the row's end: loaded behind a branch, each was
// converted to double inside it and so waited for one at a time.  Column
// indices, gathers and FP64 values stay behind the branch, where the loads
// already issue back to back (loading them unconditionally cost the FP64
// V-cycle 9%).
template <int LPR, int U, class M, class Op>
__device__ __forceinline__ double row_sum(double s, int k0, int k1, int lane,
                                          const int* __restrict__ ci, const M* __restrict__ v,
                                          Op op) {
  for (int k = k0 + lane; k < k1; k += LPR * U) {
    int c[U];
    M w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int kk = k + u * LPR;
      c[u] = kk < k1 ? ci[kk] : -1;
      if constexpr (sizeof(M) == 4)
        w[u] = v[kk < k1 ? kk : k];
      else
        w[u] = kk < k1 ? v[kk] : M(0);
    }
    double g[U];
#pragma unroll
    for (int u = 0; u < U; ++u) g[u] = c[u] >= 0 ? op(c[u]) : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (c[u] >= 0) s = s + (double)w[u] * g[u];
  }
  return s;
}
constexpr int kRowU = 8;

// A row's own values that the epilogue reads, loaded by the row's first lane
// before the row's entries (so they are not a dependent load after the
// group's shuffles), and the epilogue on them: the same arithmetic as
// epilogue().  `diag` holds the smoothing diagonal for the smoothing steps
// and the matrix diagonal for the power steps.
struct RowOwn {
  double x, b, diag, d;
};

template <int EPI, class M>
__device__ __forceinline__ RowOwn row_own(int i, const double* __restrict__ x,
                                          const double* __restrict__ b,
                                          const M* __restrict__ diag, const M* __restrict__ sd,
                                          const double* __restrict__ d, double c1) {
  RowOwn o{0.0, 0.0, 1.0, 0.0};
  if (EPI == E_CHEB0) {
    o.b = b[i];
    o.diag = (double)sd[i];
  } else if (EPI == E_RESID) {
    o.b = b[i];
  } else if (EPI == E_CHEB) {
    o.b = b[i];
    o.diag = (double)sd[i];
    o.x = x[i];
    if (c1 != 0.0) o.d = d[i];
  } else if (EPI == E_DOT) {
    o.x = x[i];
  } else if (EPI == E_POWER) {
    o.diag = (double)diag[i];
  }
  return o;
}

template <int EPI>
__device__ __forceinline__ double epilogue_own(int i, double ax, const RowOwn& o,
                                               double* __restrict__ d, double c1, double c2,
                                               double scale, double* __restrict__ y, double c0) {
  if (EPI == E_CHEB0) {
    const double x1 = c0 * (o.b / o.diag);
    const double r = (o.b - ax) / o.diag;
    const double dn = c1 * x1 + c2 * r;
    d[i] = dn;
    y[i] = x1 + dn;
    return 0.0;
  } else if (EPI == E_SPMV) {
    y[i] = ax;
    return 0.0;
  } else if (EPI == E_RESID) {
    y[i] = o.b - ax;
    return 0.0;
  } else if (EPI == E_CHEB) {
    const double r = (o.b - ax) / o.diag;
    const double dn = (c1 == 0.0 ? 0.0 : c1 * o.d) + c2 * r;
    d[i] = dn;
    y[i] = o.x + dn;
    return 0.0;
  } else if (EPI == E_DOT) {
    y[i] = ax;
    return o.x * ax;
  } else {
    const double v = (ax / o.diag) * scale;
    y[i] = v;
    return v * v;
  }
}
template <int EPI, int LPR, class M>
__global__ void __launch_bounds__(kBlock) k_csr(int n, const int* __restrict__ rp,
                                                const int* __restrict__ ci,
                                                const M* __restrict__ v, const M* __restrict__ diag,
                                                const M* __restrict__ sd,
                                                const double* __restrict__ x,
                                                const double* __restrict__ b,
                                                double* __restrict__ d, double c1, double c2,
                                                double* __restrict__ y,
                                                const double* __restrict__ prevp, int gprev,
                                                double* __restrict__ partials, double c0) {
  double scale = 1.0;
  if (EPI == E_POWER) scale = 1.0 / sqrt(sum_partials<kBlock>(prevp, gprev));
  const int lane = threadIdx.x % LPR;
  const int groups = gridDim.x * (kBlock / LPR);
  const int my = (blockIdx.x * kBlock + threadIdx.x) / LPR;
  const int trips = (n + groups - 1) / groups;
  double dot = 0.0;
  for (int t = 0; t < trips; ++t) {
    const int g = t * groups + my;
    double s = 0.0;
    RowOwn own{0.0, 0.0, 1.0, 0.0};
    if (g < n) {
      if (lane == 0) own = row_own<EPI, M>(g, x, b, diag, sd, d, c1);
      s = row_sum<LPR, kRowU, M>(s, rp[g], rp[g + 1], lane, ci, v,
                                 [&](int j) { return operand<EPI, M>(j, x, b, sd, c0); });
    }
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) s += __shfl_down(s, o, LPR);
    if (g < n && lane == 0) dot += epilogue_own<EPI>(g, s, own, d, c1, c2, scale, y, c0);
  }
  if (EPI == E_DOT || EPI == E_POWER) {
    double vv[1] = {dot};
    write_partials<kBlock, 1>(vv, partials);
  }
}

// y (+)= P x for a rectangular CSR (prolongation adds into y).  With FIRST
// (restriction only) the pass also takes the coarse level's first smoothing
// step from a zero guess on the row it has just formed: d1 = x1 =
// inv_theta y / sd, the arithmetic of k_cheb_first.
template <int LPR, bool ADD, class M, bool FIRST>
__global__ void __launch_bounds__(kBlock) k_csr_rect(int n, const int* __restrict__ rp,
                                                     const int* __restrict__ ci,
                                                     const M* __restrict__ v,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ y,
                                                     const M* __restrict__ sd, double inv_theta,
                                                     double* __restrict__ d1,
                                                     double* __restrict__ x1) {
  static_assert(!(ADD && FIRST), "the first smoothing step follows a restriction");
  const int g = (blockIdx.x * kBlock + threadIdx.x) / LPR;
  const int lane = threadIdx.x % LPR;
  double s = 0.0, y0 = 0.0, sdi = 1.0;
  if (g < n) {
    // the row's own operands are requested before its entries
    if (ADD && lane == 0) y0 = y[g];
    if (FIRST && lane == 0) sdi = (double)sd[g];
    s = row_sum<LPR, kRowU, M>(s, rp[g], rp[g + 1], lane, ci, v, [&](int j) { return x[j]; });
  }
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) s += __shfl_down(s, o, LPR);
  if (g < n && lane == 0) {
    y[g] = ADD ? y0 + s : s;
    if (FIRST) {
      const double w = inv_theta * (s / sdi);
      d1[g] = w;
      x1[g] = w;
    }
  }
}

// ---- prolongation fused with the first post-smoothing step
// After the coarse correction e the V-cycle forms x = x1 + P e and takes a
// Chebyshev step from it (c1 = 0: r = (b - A x)/diag, d = c2 r, y = x + d).
// Row i needs x at its neighbours, so one pass uses the product AP = A P
// kept from the Galerkin product: (A x)_i = (A x1)_i + (AP e)_i, exact up to
// the order of the sums.  That saves the separate prolongation pass and its
// write and re-read of x.
constexpr int kFuseU = 4;  // CSR entries per lane requested before any is used

// Entries k0 + lane + u LPR (u < U) of a CSR row ending at k1: columns (-1
// past the end) and values (FP32 values loaded unconditionally, as in
// row_sum; an empty row loads none).
template <int LPR, int U, class M>
__device__ __forceinline__ void chunk_load(int k0, int k1, int lane, const int* __restrict__ ci,
                                           const M* __restrict__ v, int (&c)[U], M (&w)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = k0 + lane + u * LPR;
    c[u] = k < k1 ? ci[k] : -1;
    if constexpr (sizeof(M) == 4)
      w[u] = k1 > k0 ? v[k < k1 ? k : k0] : M(0);
    else
      w[u] = k < k1 ? v[k] : M(0);
  }
}

// s + sum of w[u] x[c[u]] over the loaded entries, every gather requested
// before the first product.
template <int U, class M>
__device__ __forceinline__ double chunk_sum(double s, const int (&c)[U], const M (&w)[U],
                                            const double* __restrict__ x) {
  double g[U];
#pragma unroll
  for (int u = 0; u < U; ++u) g[u] = c[u] >= 0 ? x[c[u]] : 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (c[u] >= 0) s = s + (double)w[u] * g[u];
  return s;
}

// The lane's entries of a row past its first chunk (rows longer than LPR U).
template <int LPR, int U, class M>
__device__ __forceinline__ double row_rest(double s, int k0, int k1, int lane,
                                           const int* __restrict__ ci, const M* __restrict__ v,
                                           const double* __restrict__ x) {
  for (int k = k0 + lane + LPR * U; k < k1; k += LPR) s = s + (double)v[k] * x[ci[k]];
  return s;
}

// Sums of the LPR lanes of a row group, left in lane 0.
template <int LPR>
__device__ __forceinline__ void group_sum2(double& a, double& b) {
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) {
    a += __shfl_down(a, o, LPR);
    b += __shfl_down(b, o, LPR);
  }
}

// A, P and AP all CSR (A's rows hold the diagonal); LPR lanes per row.
template <class M, int LPR>
__global__ void __launch_bounds__(kBlock) k_csr_prolong_cheb(
    int n, const int* __restrict__ rp, const int* __restrict__ ci, const M* __restrict__ v,
    const M* __restrict__ sd, const int* __restrict__ prp, const int* __restrict__ pci,
    const M* __restrict__ pv, const int* __restrict__ arp, const int* __restrict__ aci,
    const M* __restrict__ av, const double* __restrict__ e, const double* __restrict__ x1,
    const double* __restrict__ b, double* __restrict__ d, double c2, double* __restrict__ y) {
  const int i = (blockIdx.x * kBlock + threadIdx.x) / LPR;
  const int lane = threadIdx.x % LPR;
  double ax = 0.0, pe = 0.0, bi = 0.0, di = 1.0, xi = 0.0;
  if (i < n) {
    if (lane == 0) {
      bi = b[i];
      di = (double)sd[i];
      xi = x1[i];
    }
    const int r0 = rp[i], r1 = rp[i + 1], p0 = prp[i], p1 = prp[i + 1], a0 = arp[i],
              a1 = arp[i + 1];
    int cc[kFuseU], pc[kFuseU], ac[kFuseU];
    M cw[kFuseU], pw[kFuseU], aw[kFuseU];
    chunk_load<LPR, kFuseU, M>(r0, r1, lane, ci, v, cc, cw);
    chunk_load<LPR, kFuseU, M>(p0, p1, lane, pci, pv, pc, pw);
    chunk_load<LPR, kFuseU, M>(a0, a1, lane, aci, av, ac, aw);
    ax = chunk_sum<kFuseU, M>(ax, cc, cw, x1);
    ax = chunk_sum<kFuseU, M>(ax, ac, aw, e);
    pe = chunk_sum<kFuseU, M>(pe, pc, pw, e);
    ax = row_rest<LPR, kFuseU, M>(ax, r0, r1, lane, ci, v, x1);
    ax = row_rest<LPR, kFuseU, M>(ax, a0, a1, lane, aci, av, e);
    pe = row_rest<LPR, kFuseU, M>(pe, p0, p1, lane, pci, pv, e);
  }
  group_sum2<LPR>(ax, pe);
  if (i < n && lane == 0) {
    const double r = (bi - ax) / di;
    const double dn = c2 * r;
    d[i] = dn;
    y[i] = (xi + pe) + dn;
  }
}
// ---- end of the fused prolongation

// First smoothing step from a zero guess: d = b / (theta sd); x = d.
template <class M>
__global__ void k_cheb_first(int n, const double* __restrict__ b, const M* __restrict__ sd,
                             double inv_theta, double* __restrict__ d, double* __restrict__ x) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double v = inv_theta * (b[i] / (double)sd[i]);
  d[i] = v;
  x[i] = v;
}

// Dense coarsest solve x = Ainv b (FP64 in both modes): one wave per row,
// lanes over columns.
__global__ void __launch_bounds__(kBlock) k_dense_gemv(int n, const double* __restrict__ Ainv,
                                                       const double* __restrict__ b,
                                                       double* __restrict__ x) {
  const int i = (blockIdx.x * kBlock + threadIdx.x) / kWave;
  const int lane = threadIdx.x % kWave;
  double s = 0.0;
  if (i < n)
    for (int j = lane; j < n; j += kWave) s = s + Ainv[(size_t)i * n + j] * b[j];
  s = wave_sum(s);
  if (i < n && lane == 0) x[i] = s;
}

// Row l1 norms sum_j |a_ij| of the finest level (ELL off-diagonal slots,
// padding 0, plus the diagonal), in slot order after the diagonal.
__global__ void k_l1_ell(int n, int W, const double* __restrict__ eval,
                         const double* __restrict__ diag, double* __restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double s = fabs(diag[i]);
  for (int k = 0; k < W; ++k) s += fabs(eval[(size_t)k * n + i]);
  out[i] = s;
}

// Row l1 norms of a CSR level (its rows hold the diagonal), in entry order.
__global__ void k_l1_csr(int n, const int* __restrict__ rp, const double* __restrict__ v,
                         double* __restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) s += fabs(v[k]);
  out[i] = s;
}

__global__ void k_power_init(int n, uint32_t salt, double* __restrict__ x,
                             double* __restrict__ partials) {
  double acc = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const double v = 0.5 + (double)fmix32((uint32_t)i ^ salt) * (1.0 / 4294967296.0);
    x[i] = v;
    acc += v * v;
  }
  double sq[1] = {acc};
  write_partials<kBlock, 1>(sq, partials);
}

// ---- segmented PCG kernels.  Compact rows are cut into reduction tiles
// that never cross a sample (segment); a producer writes one partial per
// tile, and every consumer block of segment q adds that segment's tile
// partials in tile order, so per-segment scalars are bitwise reproducible.
struct Tiles {
  const int* r0;
  const int* r1;
  const int* seg;
  const int* tp;  // segment q owns tiles [tp[q], tp[q+1])
};

// Workgroup size of the tile and segment kernels.  A tile holds 256 to 4096
// rows (768 on the 1.5 M-cell plate, 1,536 on the 128^3 cube): 512 threads
// take one to three rows each, where 256 left up to six in turn (128^3 solve
// 4.09 -> 4.03 ms).  With 1024 only one workgroup of the ELL tile kernels
// fits a CU at their register use, and every tile kernel got slower.  All
// tile and segment kernels share the size, so every consumer adds a
// segment's tile partials in the same order.
constexpr int kTileBlock = 512;

__device__ __forceinline__ double seg_sum(const double* __restrict__ part, const Tiles& T, int q) {
  return sum_partials<kTileBlock>(part + T.tp[q], T.tp[q + 1] - T.tp[q]);
}

// per-segment scalar arrays (each n_seg doubles) in s->seg_sc
enum SegScal : int { SS_BB = 0, SS_TOL2 = 1, SS_RZ0 = 2, SS_RZ1 = 3, SS_RES = 4, SS_N = 5 };
// tile-partial arrays (each n_tiles doubles) in s->tpart
enum TilePart : int { T_BB = 0, T_RR = 1, T_PQ = 2, T_RZ = 3, T_RT = 4, T_N = 5 };

__global__ void __launch_bounds__(kTileBlock)
k_gather_rhs_t(Tiles T, const int* __restrict__ perm, const int* __restrict__ comp,
               const double* __restrict__ rhs, double* __restrict__ b, double* __restrict__ part) {
  const int t = blockIdx.x;
  double acc = 0.0;
  for (int i = T.r0[t] + threadIdx.x; i < T.r1[t]; i += kTileBlock) {
    const int c = perm[i];
    const double v = comp[c] == c ? 0.0 : rhs[c];
    b[i] = v;
    acc += v * v;
  }
  double sv[1] = {acc};
  write_partials<kTileBlock, 1>(sv, part);
}

__global__ void __launch_bounds__(kTileBlock) k_norm2_t(Tiles T, const double* __restrict__ a,
                                                        double* __restrict__ part) {
  const int t = blockIdx.x;
  double acc = 0.0;
  for (int i = T.r0[t] + threadIdx.x; i < T.r1[t]; i += kTileBlock) acc += a[i] * a[i];
  double sv[1] = {acc};
  write_partials<kTileBlock, 1>(sv, part);
}

// tile partials of r.z
__global__ void __launch_bounds__(kTileBlock) k_dot_t(Tiles T, const double* __restrict__ r,
                                                      const double* __restrict__ z,
                                                      double* __restrict__ part) {
  const int t = blockIdx.x;
  double acc = 0.0;
  for (int i = T.r0[t] + threadIdx.x; i < T.r1[t]; i += kTileBlock) acc += r[i] * z[i];
  double sv[1] = {acc};
  write_partials<kTileBlock, 1>(sv, part);
}

// The last smoothing step of a level-0 V-cycle fused with the PCG dot that
// follows it: the E_CHEB step y = x + d over the tile's rows, then tile
// partials of b.y, where b is the PCG residual the V-cycle was applied to and
// y the preconditioned residual.  Same arithmetic and order as the separate
// kernels.
template <int WM, class M>
__global__ void __launch_bounds__(kTileBlock)
k_ell_cheb_dot_t(Tiles T, int n, int W, const int* __restrict__ ecol, const M* __restrict__ eval,
                 const M* __restrict__ diag, const M* __restrict__ sd,
                 const double* __restrict__ x, const double* __restrict__ b,
                 double* __restrict__ d, double c1, double c2, double* __restrict__ y,
                 double* __restrict__ part) {
  const int t = xcd_block(blockIdx.x, gridDim.x);  // the tile (its partial's slot)
  double acc = 0.0;
  for (int i = T.r0[t] + threadIdx.x; i < T.r1[t]; i += kTileBlock) {
    double s = (double)diag[i] * x[i];
    s = ell_row<E_CHEB, WM, M>(s, i, n, W, ecol, eval, x, b, sd, 0.0);
    const double r = (b[i] - s) / (double)sd[i];
    const double dn = (c1 == 0.0 ? 0.0 : c1 * d[i]) + c2 * r;
    d[i] = dn;
    const double yi = x[i] + dn;
    y[i] = yi;
    acc += b[i] * yi;
  }
  double sv[1] = {acc};
  write_partials<kTileBlock, 1>(sv, part, t);
}

// q = A p on the finest (ELL) level over the tile's rows (the outer operator,
// FP64 in both modes); tile partials of p.q
template <int WM>
__global__ void __launch_bounds__(kTileBlock) k_ell_dot_t(Tiles T, int n, int W,
                                                          const int* __restrict__ ecol,
                                                          const double* __restrict__ eval,
                                                          const double* __restrict__ diag,
                                                          const int* __restrict__ done,
                                                          const double* __restrict__ p,
                                                          double* __restrict__ q,
                                                          double* __restrict__ part) {
  const int t = xcd_block(blockIdx.x, gridDim.x);  // the tile (its partial's slot)
  double acc = 0.0;
  if (!done[T.seg[t]]) {
    for (int i = T.r0[t] + threadIdx.x; i < T.r1[t]; i += kTileBlock) {
      double s = diag[i] * p[i];
      s = ell_row<E_SPMV, WM, double>(s, i, n, W, ecol, eval, p, nullptr, diag, 0.0);
      q[i] = s;
      acc += p[i] * s;
    }
  }
  double sv[1] = {acc};
  write_partials<kTileBlock, 1>(sv, part, t);
}

// Per segment (one block each): bb, tolerance, initial convergence; counts
// active segments.
__global__ void __launch_bounds__(kTileBlock) k_seg_init(int ns, Tiles T,
                                                         const double* __restrict__ part_bb,
                                                         const double* __restrict__ part_rr,
                                                         double rtol2, double* __restrict__ sc,
                                                         int* __restrict__ done,
                                                         int* __restrict__ iters,
                                                         int* __restrict__ restart,
                                                         int* __restrict__ active) {
  const int q = blockIdx.x;
  const double bb = seg_sum(part_bb, T, q);
  const double rr = seg_sum(part_rr, T, q);
  if (threadIdx.x != 0) return;
  const double tol2 = rtol2 * bb;
  sc[SS_BB * ns + q] = bb;
  sc[SS_TOL2 * ns + q] = tol2;
  const int d = (bb == 0.0 || rr <= tol2) ? 1 : 0;
  done[q] = d;
  iters[q] = 0;
  restart[q] = 0;
  if (!d) atomicAdd(active, 1);
}

// zero the iterate of segments whose right-hand side is zero
__global__ void __launch_bounds__(kTileBlock)
k_zero_empty_t(Tiles T, int ns, const double* __restrict__ sc, double* __restrict__ x) {
  const int t = blockIdx.x;
  if (sc[SS_BB * ns + T.seg[t]] != 0.0) return;
  for (int i = T.r0[t] + threadIdx.x; i < T.r1[t]; i += kTileBlock) x[i] = 0.0;
}

// p = z on active segments; the first tile of a segment stores its r.z
__global__ void __launch_bounds__(kTileBlock) k_init_p_t(Tiles T, int ns,
                                                         const int* __restrict__ done,
                                                         const double* __restrict__ part_rz,
                                                         const double* __restrict__ z,
                                                         double* __restrict__ p,
                                                         double* __restrict__ rz_out) {
  const int t = blockIdx.x, q = T.seg[t];
  if (done[q]) return;
  const double rz = seg_sum(part_rz, T, q);
  if (t == T.tp[q] && threadIdx.x == 0) rz_out[q] = rz;
  for (int i = T.r0[t] + threadIdx.x; i < T.r1[t]; i += kTileBlock) p[i] = z[i];
}

// alpha_q = rz_q / (p.q)_q; x += alpha p; r -= alpha q; tile partial of r.r
__global__ void __launch_bounds__(kTileBlock) k_update_xr_t(Tiles T, const int* __restrict__ done,
                                                            const double* __restrict__ rz,
                                                            const double* __restrict__ part_pq,
                                                            const double* __restrict__ p,
                                                            const double* __restrict__ qv,
                                                            double* __restrict__ x,
                                                            double* __restrict__ r,
                                                            double* __restrict__ part,
                                                            int* __restrict__ active,
                                                            int* __restrict__ err) {
  const int t = blockIdx.x, q = T.seg[t];
  if (t == 0 && threadIdx.x == 0) *active = 0;  // counted again by k_update_p_t
  // the thread's first row, requested before the segment's sums
  const int i0 = T.r0[t] + threadIdx.x, i1 = T.r1[t];
  double x0 = 0.0, p0 = 0.0, r0 = 0.0, q0 = 0.0;
  if (i0 < i1) {
    x0 = x[i0];
    p0 = p[i0];
    r0 = r[i0];
    q0 = qv[i0];
  }
  double acc = 0.0;
  if (!done[q]) {
    const double pq = seg_sum(part_pq, T, q);
    const double num = rz[q];
    if (!(pq > 0.0) || !(num > 0.0)) {
      if (threadIdx.x == 0) atomicOr(err, 1);
    } else {
      const double alpha = num / pq;
      for (int i = i0; i < i1; i += kTileBlock) {
        const bool first = i == i0;
        x[i] = (first ? x0 : x[i]) + alpha * (first ? p0 : p[i]);
        const double v = (first ? r0 : r[i]) - alpha * (first ? q0 : qv[i]);
        r[i] = v;
        acc += v * v;
      }
    }
  }
  double sv[1] = {acc};
  write_partials<kTileBlock, 1>(sv, part);
}

// With test set (every PCG iteration): count the iteration of each running
// segment and test its recurred ||r||^2 against the tolerance; every tile
// of a segment adds the same partials in the same order, so all of them take
// the same decision, and a segment that converged (or broke down) keeps its
// p.  Otherwise (first direction after a restart) restart[q] forces beta 0.
// Then beta_q = r.z / rz_prev; p = z + beta p; counts the segments still
// running.
__global__ void __launch_bounds__(kTileBlock) k_update_p_t(Tiles T, int ns, int test,
                                                           int* __restrict__ done,
                                                           int* __restrict__ restart,
                                                           const double* __restrict__ part_rr,
                                                           const double* __restrict__ sc,
                                                           int* __restrict__ iters,
                                                           int* __restrict__ active,
                                                           const double* __restrict__ part_rz,
                                                           const double* __restrict__ rz_prev,
                                                           double* __restrict__ rz_next,
                                                           const double* __restrict__ z,
                                                           double* __restrict__ p,
                                                           int* __restrict__ err) {
  const int t = blockIdx.x, q = T.seg[t];
  // the thread's first row, requested before the segment's sums
  const int i0 = T.r0[t] + threadIdx.x, i1 = T.r1[t];
  double z0 = 0.0, p0 = 0.0;
  if (i0 < i1) {
    z0 = z[i0];
    p0 = p[i0];
  }
  if (done[q]) return;
  const bool lead = t == T.tp[q] && threadIdx.x == 0;
  // both sums this block may need, r.r and r.z, in one pass over the
  // segment's partials
  const int g0 = T.tp[q], G = T.tp[q + 1] - g0;
  double sums[2];
  const double* parts[2] = {part_rr + g0, part_rz + g0};
  sum_partials_n<kTileBlock, 2>(parts, G, sums);
  if (test) {
    const double rr = sums[0];
    const bool bad = !(rr == rr) || rr > 1.7976931348623157e308;
    const bool conv = bad || rr <= sc[SS_TOL2 * ns + q];
    if (lead) {
      iters[q] += 1;
      restart[q] = 0;
      if (bad) atomicOr(err, 2);
      if (conv) done[q] = 1;
      else atomicAdd(active, 1);
    }
    if (conv) return;
  }
  const double rzn = sums[1];
  double beta = 0.0;
  if (!(!test && restart[q])) beta = rzn / rz_prev[q];
  if (lead) {
    rz_next[q] = rzn;
    if (!(rzn > 0.0)) atomicOr(err, 4);
  }
  for (int i = i0; i < i1; i += kTileBlock) {
    const bool first = i == i0;
    p[i] = (first ? z0 : z[i]) + beta * (first ? p0 : p[i]);
  }
}

// After the recurred residuals all met the tolerance: per segment (one
// block each), the true residual; a segment that misses it restarts.
__global__ void __launch_bounds__(kTileBlock) k_seg_check(int ns, Tiles T,
                                                          const double* __restrict__ part_rt,
                                                          double* __restrict__ sc,
                                                          int* __restrict__ done,
                                                          int* __restrict__ restart,
                                                          int* __restrict__ active) {
  const int q = blockIdx.x;
  const double rt = seg_sum(part_rt, T, q);
  if (threadIdx.x != 0) return;
  sc[SS_RES * ns + q] = rt;
  const double bb = sc[SS_BB * ns + q];
  if (bb != 0.0 && rt > sc[SS_TOL2 * ns + q]) {
    done[q] = 0;
    restart[q] = 1;
    atomicAdd(active, 1);
  }
}

// r = r_true on segments that restart
__global__ void __launch_bounds__(kTileBlock)
k_copy_restart_t(Tiles T, const int* __restrict__ restart, const double* __restrict__ rt,
                 double* __restrict__ r) {
  const int t = blockIdx.x;
  if (!restart[T.seg[t]]) return;
  for (int i = T.r0[t] + threadIdx.x; i < T.r1[t]; i += kTileBlock) r[i] = rt[i];
}

__global__ void k_gather_x0(int na, const int* __restrict__ perm, const int* __restrict__ comp,
                            const double* __restrict__ p, double* __restrict__ x) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= na) return;
  int c = perm[i];
  x[i] = comp[c] == c ? 0.0 : p[c];
}

__global__ void k_scatter(int nc, const int* __restrict__ cid, const int* __restrict__ comp,
                          const double* __restrict__ x, double* __restrict__ p) {
  int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= nc) return;
  int k = cid[c];
  p[c] = (k < 0 || comp[c] == c) ? 0.0 : x[k];
}

// *out = scale sqrt(sum of p0[0..g)).
__global__ void __launch_bounds__(kBlock) k_finalize_norm(const double* __restrict__ p0, int g,
                                                          double scale, double* __restrict__ out) {
  const double a = sum_partials<kBlock>(p0, g);
  if (threadIdx.x == 0) *out = scale * sqrt(a);
}


// Several FP64 -> FP32 casts in one dispatch: segment k is blockIdx.y, its
// n[k] values cast by a grid-stride loop over blockIdx.x.
constexpr int kCastSegs = 24;
struct CastArgs {
  const double* src[kCastSegs];
  float* dst[kCastSegs];
  int64_t n[kCastSegs];
};

__global__ void __launch_bounds__(kBlock) k_cast_segments(CastArgs a) {
  const int k = blockIdx.y;
  const double* __restrict__ src = a.src[k];
  float* __restrict__ dst = a.dst[k];
  const int64_t n = a.n[k];
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    dst[i] = (float)src[i];
}

__global__ void k_copy(int n, const double* __restrict__ a, double* __restrict__ b) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) b[i] = a[i];
}

double* part(ppe_solver* s, int slot) {
  return s->partial.as<double>() + (size_t)slot * kRedBlocks;
}

constexpr size_t kProfPairs = 256;

template <class M> const char* tname();
template <> const char* tname<double>() { return "double"; }
template <> const char* tname<float>() { return "float"; }

// "base<a, b, ...>" the way a kernel trace prints a template instantiation.
std::string kname(const char* base, std::initializer_list<std::string> args) {
  std::string n = base;
  if (args.size()) {
    n += "<";
    bool first = true;
    for (const auto& a : args) {
      if (!first) n += ", ";
      n += a;
      first = false;
    }
    n += ">";
  }
  return n;
}
std::string str(int v) { return std::to_string(v); }
std::string str(bool v) { return v ? "true" : "false"; }

// Launch a solve-phase kernel on the solver's stream.  While profiling, the
// dispatch takes its own event pair (hipExtLaunchKernelGGL records the
// dispatch's start and end) and is booked under info() = {kernel name,
// algorithmic bytes}; otherwise info is never evaluated.
template <class Info, class K, class... Args>
void launch(ppe_solver* s, Info&& info, K kernel, dim3 grid, dim3 block, Args... args) {
  if (s->prof) {
    const std::pair<std::string, double> nb = info();
    const auto ev = profile_slot(s, nb.first, nb.second);
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s->stream, ev.first, ev.second, 0, args...);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, 0, s->stream, args...);
  }
  PPE_LAUNCH_CHECK();
}

// Algorithmic bytes of a level operator step: every stored entry once
// (value + column index), the row pointers (CSR), the diagonal and, when
// the smoother scales by another diagonal, that one, and the vectors the
// epilogue reads and writes (8 bytes each).
template <int EPI, class M>
double op_bytes(const ppe_solver* s, const Level& L, bool ell, double c1) {
  const double n = L.n, m = sizeof(M);
  const bool smoothing = EPI == E_CHEB || EPI == E_CHEB0;
  const bool l1 = s->opt.smoother == PPE_SMOOTH_L1JACOBI;
  double b = ell ? (double)(L.A.nnz - L.n) * (m + 4) + n * m     // off-diagonal ELL + diagonal
                 : (double)L.A.nnz * (m + 4) + 4.0 * (n + 1);   // CSR rows hold the diagonal
  if (smoothing && (l1 || !ell)) b += n * m;                    // the scaling diagonal
  double vec = 0.0;
  switch (EPI) {
    case E_SPMV: vec = 2; break;                   // x, y
    case E_RESID: vec = 3; break;                  // x, b, y
    case E_CHEB: vec = c1 != 0.0 ? 5 : 4; break;   // x, b, (d in), d out, y
    case E_CHEB0: vec = 3; break;                  // b, d out, y
    case E_DOT: vec = 2; break;                    // x, y
    default: vec = 2; break;
  }
  return b + 8.0 * vec * n;
}

// Launch an ELL kernel template K<WM> with the smallest unrolled width that
// covers W (a generic slot loop beyond 12).
#define PPE_ELL_WIDTH(W_, LAUNCH)                \
  do {                                           \
    const int w_ = (W_);                         \
    if (w_ <= 4) { LAUNCH(4); }                  \
    else if (w_ <= 6) { LAUNCH(6); }             \
    else if (w_ <= 8) { LAUNCH(8); }             \
    else if (w_ <= 12) { LAUNCH(12); }           \
    else { LAUNCH(0); }                          \
  } while (0)

// Matrix and diagonal arrays of a level in value type M (the FP32 copies
// exist when the solver runs the mixed-precision V-cycle).
template <class M> struct LevelData;
template <> struct LevelData<double> {
  static const double* ell(const Level& L) { return L.ell_val.as<double>(); }
  static const double* diag(const Level& L) { return L.diag.as<double>(); }
  static const double* l1(const Level& L) { return L.dl1.as<double>(); }
  static const double* val(const Csr& A) { return A.v(); }
};
template <> struct LevelData<float> {
  static const float* ell(const Level& L) { return L.ell_valf.as<float>(); }
  static const float* diag(const Level& L) { return L.diagf.as<float>(); }
  static const float* l1(const Level& L) { return L.dl1f.as<float>(); }
  static const float* val(const Csr& A) { return A.vf(); }
};

// The diagonal the smoothing steps scale by: the row l1 norms under the
// l1-Jacobi smoother, the matrix diagonal under Chebyshev.
template <class M>
const M* smooth_diag(const ppe_solver* s, const Level& L) {
  return s->opt.smoother == PPE_SMOOTH_L1JACOBI ? LevelData<M>::l1(L) : LevelData<M>::diag(L);
}

// Lanes per row of the solve's CSR kernels by default.  The rules are fits
// to what the autotuner picked on the 128^3 cube and the 1.5 M-cell plate
// (FP64 and mixed): about 1.8 sqrt(row length) lanes for the smoothing steps
// (8 for rows of 30 entries, 16 for 128, 32 for 219), three entries per lane
// for the restriction and the plain prolongation, and about
// 3 sqrt(row length) lanes for the fused prolongation (whose rows of A, P and
// A P are read together).  The plain transfers go down to one lane per row
// (the finest prolongation has three to four entries a row); the smoothing
// and fused kernels keep at least four.  A level too small to give every
// compute unit a block of 256 threads at that count takes 64 lanes.
int lanes_near(double target, int lo = 4) {
  int best = lo;
  for (int c = 2 * lo; c <= 64; c *= 2)
    if (std::fabs(std::log2((double)c / target)) < std::fabs(std::log2((double)best / target)))
      best = c;
  return best;
}
int widen_small(const Csr& M, int lpr) { return (int64_t)M.n * lpr < 16384 ? 64 : lpr; }
double mean_row(const Csr& M) { return M.n ? (double)M.nnz / M.n : 1.0; }
int smooth_lanes(const Csr& A) {
  return widen_small(A, lanes_near(1.8 * std::sqrt(mean_row(A))));
}
// lanes per row of a prolongation P and of a restriction R = P^T
int transfer_lanes(const Csr& M) { return widen_small(M, lanes_near(mean_row(M) / 3.0, 1)); }
int restrict_lanes(const Csr& R) { return widen_small(R, lanes_near(mean_row(R) / 5.0, 1)); }

// Apply the level operator with epilogue EPI, matrix values in type M.
// Dot/power epilogues run on a capped grid and write partials to `partials`;
// returns that grid size.
template <int EPI, class M = double>
int apply_op(ppe_solver* s, const Level& L, const double* x, const double* b, double* d,
             double c1, double c2, double* y, double* partials, const double* prevp = nullptr,
             int gprev = 0, double c0 = 0.0) {
  const int n = L.n;
  if (n == 0) return 1;
  const bool reduce = EPI == E_DOT || EPI == E_POWER;
  const M* sd = EPI == E_POWER ? LevelData<M>::diag(L) : smooth_diag<M>(s, L);
  if (&L == &s->levels[0] && EPI != E_POWER) {
    const int g = reduce ? red_grid(n) : grid_for(n);
#define PPE_ELL(WM_)                                                                           \
  launch(s,                                                                                    \
         [&]() {                                                                               \
           return std::make_pair(kname("k_ell", {str(EPI), tname<M>(), str(WM_)}),            \
                                 op_bytes<EPI, M>(s, L, true, c1));                           \
         },                                                                                    \
         k_ell<EPI, M, WM_>, dim3(g), dim3(kBlock), n, L.W, (const int*)L.ell_col.as<int>(),   \
         LevelData<M>::ell(L), LevelData<M>::diag(L), sd, x, b, d, c1, c2, y, partials, c0)
    PPE_ELL_WIDTH(L.W, PPE_ELL);
#undef PPE_ELL
    return g;
  }
  // the setup's power steps keep the one-entry rule: the spectral bounds,
  // and with them the hierarchy, stay what they were
  // the power steps (a reduction, so at most kRedBlocks workgroups) take the
  // smoother's lanes too: with one lane per entry each lane group walked
  // seven rows of level 1 in turn
  const int lpr = L.lpr_a > 0 ? L.lpr_a : smooth_lanes(L.A);
  const int g = reduce ? red_grid((int64_t)n * lpr) : grid_for((int64_t)n * lpr);
#define PPE_CSR(LL)                                                                            \
  launch(s,                                                                                    \
         [&]() {                                                                               \
           return std::make_pair(kname("k_csr", {str(EPI), str(LL), tname<M>()}),             \
                                 op_bytes<EPI, M>(s, L, false, c1));                          \
         },                                                                                    \
         k_csr<EPI, LL, M>, dim3(g), dim3(kBlock), n, (const int*)L.A.rp(),                    \
         (const int*)L.A.ci(), LevelData<M>::val(L.A), LevelData<M>::diag(L), sd, x, b, d, c1, \
         c2, y, prevp, gprev, partials, c0)
  switch (lpr) {
    case 4: PPE_CSR(4); break;
    case 8: PPE_CSR(8); break;
    case 16: PPE_CSR(16); break;
    case 32: PPE_CSR(32); break;
    default: PPE_CSR(64); break;
  }
#undef PPE_CSR
  return g;
}

// The coarse level's first smoothing step from a zero guess, taken by the
// restriction that forms its right-hand side: the level's smoothing
// diagonal, 1/theta, and where the step's update and iterate go.
template <class M>
struct FirstStep {
  const M* sd;
  double inv_theta;
  double* d;
  double* x;
};

template <bool ADD, class M, bool FIRST = false>
void apply_rect(ppe_solver* s, const Csr& P, const double* x, double* y, int lpr_choice = 0,
                const FirstStep<M>& fs = FirstStep<M>{nullptr, 0.0, nullptr, nullptr}) {
  if (P.n == 0) return;
  const int lpr = lpr_choice > 0 ? lpr_choice : (ADD ? transfer_lanes(P) : restrict_lanes(P));
  const int g = grid_for((int64_t)P.n * lpr);
  // entries and row pointers of P or R, each operand entry once, y out (and
  // in); with the first step the diagonal in and its update and iterate out
  auto bytes = [&]() {
    return (double)P.nnz * (sizeof(M) + 4) + 4.0 * (P.n + 1) + 8.0 * P.m +
           8.0 * P.n * (ADD ? 2 : 1) + (FIRST ? (sizeof(M) + 16.0) * P.n : 0.0);
  };
#define PPE_RECT(LL)                                                                           \
  launch(s,                                                                                    \
         [&]() {                                                                               \
           return std::make_pair(                                                              \
               kname("k_csr_rect", {str(LL), str(ADD), tname<M>(), str(FIRST)}), bytes());     \
         },                                                                                    \
         k_csr_rect<LL, ADD, M, FIRST>, dim3(g), dim3(kBlock), P.n, (const int*)P.rp(),        \
         (const int*)P.ci(), LevelData<M>::val(P), x, y, fs.sd, fs.inv_theta, fs.d, fs.x)
  switch (lpr) {
    case 1: PPE_RECT(1); break;
    case 2: PPE_RECT(2); break;
    case 4: PPE_RECT(4); break;
    case 8: PPE_RECT(8); break;
    case 16: PPE_RECT(16); break;
    case 32: PPE_RECT(32); break;
    default: PPE_RECT(64); break;
  }
#undef PPE_RECT
}

// Whether level L's prolongation can run fused with its first
// post-smoothing step: on the coarse levels of the FP64 V-cycle, while AP
// still equals A P, when the smoother takes at least two steps (and whether
// it does: the level's launch choice as well).
//  - The finest level keeps its separate passes: there the fused pass, with
//    CSR rows of P and AP gathered beside the ELL rows of A, took as long as
//    the prolongation and the ELL step together, while on the coarse levels
//    it saves a dispatch each.
//  - The mixed V-cycle keeps them too: rounded to FP32 separately, the
//    stored AP is no longer the product of the stored A and P, and the
//    V-cycle would stop being symmetric at the level of that rounding.
bool prolong_can_fuse(const ppe_solver* s, const Level& L) {
  return s->opt.precision != PPE_MIXED && &L != &s->levels[0] && L.ap_ok && !L.c1.empty();
}
bool prolong_fusable(const ppe_solver* s, const Level& L) {
  return L.fuse_p && prolong_can_fuse(s, L);
}

// The fixed rule for fusing: the fused pass reads A P where the separate
// passes read P and write and re-read x, and saves one dispatch.  Where A P
// holds more than about 16 MB beyond that (128^3 level 1: 9 M entries), the
// separate passes move less (182 against about 80 MB there); a level below
// that is latency-bound and the saved dispatch wins.
bool fuse_rule(const Level& L) {
  const double extra = 12.0 * (double)L.AP.nnz - 16.0 * (double)L.n;
  return extra <= 16.0e6;
}

// Lanes per row of the fused pass: the launch choice if set (at least
// four), else the fixed rule (rows past the first chunk continue lane by
// lane).
int prolong_lanes(const Level& L) {
  if (L.lpr_p > 0) return std::max(L.lpr_p, 4);
  return widen_small(L.A, lanes_near(2.0 * std::sqrt(mean_row(L.A))));
}

// y = (x1 + P e) + d with d = c2 D^-1 (b - A (x1 + P e)): the prolongation
// and the first post-smoothing step in one pass (prolong_fusable must hold).
template <class M>
void prolong_cheb(ppe_solver* s, Level& L, const double* e, const double* x1, const double* b,
                  double* d, double* y) {
  const int n = L.n;
  const int lpr = prolong_lanes(L);
  const int g = grid_for((int64_t)n * lpr);
  const double c2 = L.inv_theta;
  // entries and row pointers of A, P and AP, the scaling diagonal, e, and
  // x1, b in with d, y out
  auto bytes = [&]() {
    return (double)(L.A.nnz + L.P.nnz + L.AP.nnz) * (sizeof(M) + 4) + 12.0 * (n + 1) +
           (double)n * sizeof(M) + 8.0 * L.P.m + 8.0 * 4 * n;
  };
#define PPE_PC_CSR(LL)                                                                         \
  launch(s, [&]() { return std::make_pair(kname("k_csr_prolong_cheb", {tname<M>(), str(LL)}),   \
                                          bytes()); },                                         \
         k_csr_prolong_cheb<M, LL>, dim3(g), dim3(kBlock), n, (const int*)L.A.rp(),            \
         (const int*)L.A.ci(), LevelData<M>::val(L.A), smooth_diag<M>(s, L),                  \
         (const int*)L.P.rp(), (const int*)L.P.ci(), LevelData<M>::val(L.P),                  \
         (const int*)L.AP.rp(), (const int*)L.AP.ci(), LevelData<M>::val(L.AP), e, x1, b, d,   \
         c2, y)
  switch (lpr) {
    case 4: PPE_PC_CSR(4); break;
    case 8: PPE_PC_CSR(8); break;
    case 16: PPE_PC_CSR(16); break;
    case 32: PPE_PC_CSR(32); break;
    default: PPE_PC_CSR(64); break;
  }
#undef PPE_PC_CSR
}

// PCG dot fused into the last level-0 step of the V-cycle: tile partials of
// r.z into part (n_tiles).
struct PcgDot {
  Tiles T;
  int nt;
  double* part;
};

// Chebyshev smoothing of A x = b.  x_in == nullptr: zero initial guess, and
// the first two steps run as one pass.  The result is written to x_out;
// xa/xb are ping-pong buffers distinct from x_in and x_out.  With dot (level
// 0 only) the last step also produces the PCG dot; returns whether it did.
template <class M>
bool smooth_steps(ppe_solver* s, Level& L, const double* b, const double* cur, int step,
                  double* x_out, double* xa, double* xb, const PcgDot* dot);

template <class M>
bool smooth(ppe_solver* s, Level& L, const double* b, const double* x_in, double* x_out,
            double* xa, double* xb, const PcgDot* dot = nullptr, bool first_done = false) {
  const int n = L.n;
  const int deg = 1 + (int)L.c1.size();
  double* d = L.d.as<double>();
  auto dst_of = [&](int k) { return k == deg ? x_out : ((k % 2) ? xa : xb); };
  const double* cur = x_in;
  int step = 1;
  if (cur == nullptr) {
    if (first_done) {  // the restriction took the first step (restricted_first)
      cur = dst_of(1);
      step = 2;
    } else if (deg >= 2 && L.fuse0) {
      double* dst = dst_of(2);
      apply_op<E_CHEB0, M>(s, L, nullptr, b, d, L.c1[0], L.c2[0], dst, nullptr, nullptr, 0,
                           L.inv_theta);
      cur = dst;
      step = 3;
    } else {
      double* dst = dst_of(1);
      launch(s,
             [&]() {
               return std::make_pair(kname("k_cheb_first", {tname<M>()}),
                                     (double)n * (sizeof(M) + 24.0));  // sd, b in; d, x out
             },
             k_cheb_first<M>, dim3(grid_for(n)), dim3(kBlock), n, (const double*)b,
             smooth_diag<M>(s, L), L.inv_theta, d, dst);
      cur = dst;
      step = 2;
    }
  }
  return smooth_steps<M>(s, L, b, cur, step, x_out, xa, xb, dot);
}

// Chebyshev steps step..degree from the iterate cur (with the level's d
// holding the previous step's update when step > 1); the rest as smooth.
template <class M>
bool smooth_steps(ppe_solver* s, Level& L, const double* b, const double* cur, int step,
                  double* x_out, double* xa, double* xb, const PcgDot* dot) {
  const int n = L.n;
  const int deg = 1 + (int)L.c1.size();
  double* d = L.d.as<double>();
  auto dst_of = [&](int k) { return k == deg ? x_out : ((k % 2) ? xa : xb); };
  bool dotted = false;
  for (; step <= deg; ++step) {
    double* dst = dst_of(step);
    const double c1 = step == 1 ? 0.0 : L.c1[step - 2];
    const double c2 = step == 1 ? L.inv_theta : L.c2[step - 2];
    if (dot && step == deg && &L == &s->levels[0]) {
#define PPE_CHEB_DOT(WM_)                                                                     \
  launch(s,                                                                                    \
         [&]() {                                                                               \
           return std::make_pair(kname("k_ell_cheb_dot_t", {str(WM_), tname<M>()}),           \
                                 op_bytes<E_CHEB, M>(s, L, true, c1));                        \
         },                                                                                    \
         k_ell_cheb_dot_t<WM_, M>, dim3(dot->nt), dim3(kTileBlock), dot->T, n, L.W,            \
         (const int*)L.ell_col.as<int>(), LevelData<M>::ell(L), LevelData<M>::diag(L),         \
         smooth_diag<M>(s, L), cur, b, d, c1, c2, dst, dot->part)
      PPE_ELL_WIDTH(L.W, PPE_CHEB_DOT);
#undef PPE_CHEB_DOT
      dotted = true;
      cur = dst;
      continue;
    }
    apply_op<E_CHEB, M>(s, L, cur, b, d, c1, c2, dst, nullptr);
    cur = dst;
  }
  return dotted;
}

// Whether the V-cycle's first smoothing on level l (l > 0, from a zero
// guess) starts with the plain first step (not the fused first two steps),
// which the restriction into level l then takes; and where that step's
// iterate goes: the first smoothing's output x1 (t, or r on the coarsest
// level) when the smoother has one step, else its ping-pong buffer x2.
bool restricted_first(const ppe_solver* s, int l) {
  const Level& C = s->levels[l];
  if (l == s->nlev - 1 && C.dense) return false;
  return !(C.c1.size() >= 1 && C.fuse0);
}
template <class M>
FirstStep<M> first_step(ppe_solver* s, int l) {
  Level& C = s->levels[l];
  double* out = l == s->nlev - 1 ? C.r.as<double>() : C.t.as<double>();
  return FirstStep<M>{smooth_diag<M>(s, C), C.inv_theta, C.d.as<double>(),
                      C.c1.empty() ? out : C.x2.as<double>()};
}

// One V-cycle with zero initial guess, x = M b on level l, matrix values in
// type M (vectors FP64).  dot: see smooth (consumed by the last level-0
// smoothing step, if any).  first_done: the restriction into level l has
// taken its first smoothing step (restricted_first).
template <class M>
bool vcycle_t(ppe_solver* s, int l, const double* b, double* x, const PcgDot* dot = nullptr,
              bool first_done = false) {
  Level& L = s->levels[l];
  const int n = L.n;
  if (n == 0) return false;
  double* xa = L.x2.as<double>();
  double* xb = L.d2.as<double>();
  if (l == s->nlev - 1) {
    if (L.dense) {
      launch(s,
             [&]() {
               return std::make_pair(std::string("k_dense_gemv"),
                                     8.0 * (double)n * n + 16.0 * n);  // inverse, b, x
             },
             k_dense_gemv, dim3(grid_for((int64_t)n * kWave)), dim3(kBlock), n,
             (const double*)L.Ainv.as<double>(), b, x);
      return false;
    }
    double* t = L.r.as<double>();
    smooth<M>(s, L, b, nullptr, t, xa, xb, nullptr, first_done);
    return smooth<M>(s, L, b, t, x, xa, xb, dot);
  }
  Level& C = s->levels[l + 1];
  double* x1 = L.t.as<double>();  // pre-smoothed iterate, corrected in place
  double* r = L.r.as<double>();
  smooth<M>(s, L, b, nullptr, x1, xa, xb, nullptr, first_done);
  apply_op<E_RESID, M>(s, L, x1, b, nullptr, 0.0, 0.0, r, nullptr);
  const bool first = C.n > 0 && restricted_first(s, l + 1);
  if (first)
    apply_rect<false, M, true>(s, L.R, r, C.b.as<double>(), L.lpr_r, first_step<M>(s, l + 1));
  else
    apply_rect<false, M>(s, L.R, r, C.b.as<double>(), L.lpr_r);
  vcycle_t<M>(s, l + 1, C.b.as<double>(), C.x.as<double>(), nullptr, first);
  if (prolong_fusable(s, L)) {
    // the first post-smoothing step writes xa (it is not the last step)
    prolong_cheb<M>(s, L, C.x.as<double>(), x1, b, L.d.as<double>(), xa);
    return smooth_steps<M>(s, L, b, xa, 2, x, xa, xb, dot);
  }
  apply_rect<true, M>(s, L.P, C.x.as<double>(), x1, L.lpr_p);
  return smooth<M>(s, L, b, x1, x, xa, xb, dot);
}

}  // namespace

void drop_graph(ppe_solver* s) {
  if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
  s->gexec = nullptr;
  s->graph_ok = false;
}

void profile_harvest(ppe_solver* s) {
  const size_t k = s->prof_pending.size();
  if (k == 0) return;
  PPE_HIP(hipEventSynchronize(s->prof_ev[2 * k - 1]));
  for (size_t i = 0; i < k; ++i) {
    float ms = 0.f;
    PPE_HIP(hipEventElapsedTime(&ms, s->prof_ev[2 * i], s->prof_ev[2 * i + 1]));
    auto& e = s->prof_table[s->prof_pending[i].entry];
    e.ms += ms;
    e.bytes += s->prof_pending[i].bytes;
    e.launches += 1;
  }
  s->prof_pending.clear();
}

void profile_enable(ppe_solver* s, bool on) {
  if (on && s->prof_ev.empty()) {
    s->prof_ev.resize(2 * kProfPairs, nullptr);
    for (auto& e : s->prof_ev) PPE_HIP(hipEventCreate(&e));
  }
  profile_harvest(s);
  s->prof = on;
  if (on) s->prof_table.clear();
}

std::pair<hipEvent_t, hipEvent_t> profile_slot(ppe_solver* s, const std::string& name,
                                               double bytes) {
  if (s->prof_pending.size() == kProfPairs) profile_harvest(s);
  int entry = -1;
  for (size_t i = 0; i < s->prof_table.size(); ++i)
    if (s->prof_table[i].name == name) entry = (int)i;
  if (entry < 0) {
    s->prof_table.push_back(ppe_solver::ProfEntry{name});
    entry = (int)s->prof_table.size() - 1;
  }
  const size_t k = s->prof_pending.size();
  s->prof_pending.push_back(ppe_solver::ProfPending{entry, bytes});
  return {s->prof_ev[2 * k], s->prof_ev[2 * k + 1]};
}

void spmv(ppe_solver* s, const Level& L, const double* x, double* y) {
  apply_op<E_SPMV, double>(s, L, x, nullptr, nullptr, 0.0, 0.0, y, nullptr);
}

void power_estimate(ppe_solver* s, Level& L, uint32_t salt, int iters, double scale,
                    double* out) {
  const int n = L.n;
  s->partial.get<double>((size_t)P_NSLOTS * kRedBlocks);
  double* x = L.x.as<double>();
  double* y = L.r.as<double>();
  double* pa = part(s, P_POW);
  double* pb = part(s, P_POW + 1);
  int g = red_grid(n);
  hipLaunchKernelGGL(k_power_init, dim3(g), dim3(kBlock), 0, s->stream, n, salt, x, pa);
  PPE_LAUNCH_CHECK();
  for (int it = 0; it < iters; ++it) {
    g = apply_op<E_POWER, double>(s, L, x, nullptr, nullptr, 0.0, 0.0, y, pb, pa, g);
    std::swap(x, y);
    std::swap(pa, pb);
  }
  hipLaunchKernelGGL(k_finalize_norm, dim3(1), dim3(kBlock), 0, s->stream, pa, g, scale, out);
  PPE_LAUNCH_CHECK();
}

void prepare_solve_levels(ppe_solver* s) {
  for (int l = 0; l < s->nlev; ++l) {
    Level& L = s->levels[l];
    L.lpr_a = L.lpr_r = L.lpr_p = 0;
    // The fused first two steps gather b and the scaling diagonal (and divide)
    // for every stored entry.  On a coarse level the restriction into it
    // takes the first step for the cost of two more vectors written, and the
    // split pair then costs one plain step (the autotuner split every coarse
    // level of the 128^3 cube and the plate); the finest level has no
    // restriction before it and keeps the fused pair.
    L.fuse0 = l == 0;
    L.fuse_p = fuse_rule(L);
    const int n = L.n > 0 ? L.n : 1;
    L.x.get<double>(n);
    L.b.get<double>(n);
    L.r.get<double>(n);
    L.d.get<double>(n);
    L.x2.get<double>(n);
    L.d2.get<double>(n);
    L.t.get<double>(n);
    L.c1.clear();
    L.c2.clear();
    L.inv_theta = 0.0;
    if (!(L.rho > 0.0)) continue;  // a coarsest level solved directly: no smoother
    if (s->opt.smoother == PPE_SMOOTH_L1JACOBI) {
      // cheb_degree sweeps x += (b - A x) / D_l1: every step with c1 = 0, c2 = 1
      double* dl1 = L.dl1.get<double>(n);
      if (l == 0)
        hipLaunchKernelGGL(k_l1_ell, dim3(grid_for(L.n)), dim3(kBlock), 0, s->stream, L.n, L.W,
                           L.ell_val.as<double>(), L.diag.as<double>(), dl1);
      else
        hipLaunchKernelGGL(k_l1_csr, dim3(grid_for(L.n)), dim3(kBlock), 0, s->stream, L.n,
                           L.A.rp(), L.A.v(), dl1);
      PPE_LAUNCH_CHECK();
      L.inv_theta = 1.0;
      for (int j = 2; j <= s->opt.cheb_degree; ++j) {
        L.c1.push_back(0.0);
        L.c2.push_back(1.0);
      }
      continue;
    }
    const double lmax = L.rho, lmin = L.rho / s->opt.cheb_ratio;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    const double sigma = theta / delta;
    double rho_prev = 1.0 / sigma;
    L.inv_theta = 1.0 / theta;
    for (int j = 2; j <= s->opt.cheb_degree; ++j) {
      const double rho_j = 1.0 / (2.0 * sigma - rho_prev);
      L.c1.push_back(rho_j * rho_prev);
      L.c2.push_back(2.0 * rho_j / delta);
      rho_prev = rho_j;
    }
  }
}

// z = M r with the V-cycle in the solver's precision: the hierarchy's values
// in FP64, or (mixed) their FP32 copies; vectors and arithmetic FP64 either
// way.
void vcycle(ppe_solver* s, int l, const double* b, double* x) {
  if (s->opt.precision == PPE_MIXED)
    vcycle_t<float>(s, l, b, x);
  else
    vcycle_t<double>(s, l, b, x);
}

// z = M r for PCG, with the dot r.z left as tile partials: fused into the
// last level-0 smoothing step, else a separate pass.
static void vcycle_pcg(ppe_solver* s, const double* r, double* z, const PcgDot& dot) {
  const bool dotted = s->opt.precision == PPE_MIXED ? vcycle_t<float>(s, 0, r, z, &dot)
                                                    : vcycle_t<double>(s, 0, r, z, &dot);
  if (!dotted)
    launch(s, [&]() { return std::make_pair(std::string("k_dot_t"), 16.0 * s->n_active); },
           k_dot_t, dim3(dot.nt), dim3(kTileBlock), dot.T, r, (const double*)z, dot.part);
}

// FP32 copies of the hierarchy's values for the mixed-precision V-cycle:
// diagonals, level operators, P and R.  Rounding each stored
// value keeps R = P^T and every level operator symmetric, so the V-cycle
// stays one symmetric operator.  The coarsest dense inverse stays FP64: its
// entries are dominated by the smoothest mode, and rounding them would
// perturb the other modes by the level's condition number times 6e-8.
void make_fp32_hierarchy(ppe_solver* s) {
  // every copy of every level in one dispatch (per kCastSegs copies)
  CastArgs a{};
  int ns = 0;
  int64_t most = 0;
  auto flush = [&]() {
    if (ns == 0) return;
    int g = grid_for(most);
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(k_cast_segments, dim3(g, ns), dim3(kBlock), 0, s->stream, a);
    PPE_LAUNCH_CHECK();
    ns = 0;
    most = 0;
  };
  auto add = [&](const double* src, float* dst, int64_t n) {
    if (n <= 0) return;
    if (ns == kCastSegs) flush();
    a.src[ns] = src;
    a.dst[ns] = dst;
    a.n[ns] = n;
    ++ns;
    most = std::max(most, n);
  };
  for (int l = 0; l < s->nlev; ++l) {
    Level& L = s->levels[l];
    if (L.n == 0) continue;
    add(L.diag.as<double>(), L.diagf.get<float>(L.n), L.n);
    if (s->opt.smoother == PPE_SMOOTH_L1JACOBI && L.rho > 0.0)
      add(L.dl1.as<double>(), L.dl1f.get<float>(L.n), L.n);
    if (l == 0) {
      const int64_t e = (int64_t)(L.W > 0 ? L.W : 1) * L.n;
      add(L.ell_val.as<double>(), L.ell_valf.get<float>(e), e);
    }
    if (L.A.nnz > 0) add(L.A.v(), L.A.valf.get<float>(L.A.nnz), L.A.nnz);
    if (l < s->nlev - 1) {
      add(L.P.v(), L.P.valf.get<float>(L.P.nnz), L.P.nnz);
      add(L.R.v(), L.R.valf.get<float>(L.R.nnz), L.R.nnz);
    }
  }
  flush();
}

// Record the launches `issue` makes into a HIP graph on the solver's capture
// stream and instantiate it (the launches see that stream as s->stream).
template <class F>
void capture_iterations(ppe_solver* s, F&& issue) {
  drop_graph(s);
  hipStream_t user = s->stream;
  s->stream = s->gstream;
  hipGraph_t g = nullptr;
  try {
    PPE_HIP(hipStreamBeginCapture(s->gstream, hipStreamCaptureModeRelaxed));
    issue();
    PPE_HIP(hipStreamEndCapture(s->gstream, &g));
  } catch (...) {
    hipGraph_t junk = nullptr;
    (void)hipStreamEndCapture(s->gstream, &junk);
    if (junk) (void)hipGraphDestroy(junk);
    s->stream = user;
    throw;
  }
  s->stream = user;
  hipError_t e = hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  PPE_HIP(e);
  s->graph_ok = true;
}

ppe_status pcg_solve(ppe_solver* s, const double* rhs, double* p_out, int use_x0, int* pred) {
  const int na = s->n_active, nc = s->n_cells, ns = s->n_seg, nt = s->n_tiles;
  ppe_stats& st = s->stats;
  st.iterations = 0;
  st.rel_residual = 0.0;
  s->seg_iters_h.assign(ns, 0);
  s->seg_res_h.assign(ns, 0.0);
  if (na == 0) {
    fill_double(s, p_out, 0.0, nc);
    PPE_HIP(hipStreamSynchronize(s->stream));
    return PPE_OK;
  }
  Level& L0 = s->levels[0];
  double* x = s->vx.get<double>(na);
  double* r = s->vr.get<double>(na);
  // z alternates between two buffers (one captured graph holds both)
  double* zb[2] = {s->vz.get<double>(na), s->vzold.get<double>(na)};
  double* p = s->vp.get<double>(na);
  double* q = s->vq.get<double>(na);
  double* b = s->vb.get<double>(na);
  double* tp = s->tpart.get<double>((size_t)T_N * nt);
  double* sc = s->seg_sc.get<double>((size_t)SS_N * ns);
  int* done = s->seg_done.get<int>(3 * (size_t)ns);
  int* iters = done + ns;
  int* restart = done + 2 * ns;
  int* cnt = s->flag.get<int>(4);  // [0] active segments, [1] error bits
  const Tiles T{s->tile_r0.as<int>(), s->tile_r1.as<int>(), s->tile_seg.as<int>(),
                s->seg_tile_ptr.as<int>()};
  auto tpart = [&](int k) { return tp + (size_t)k * nt; };
  const int* perm = s->perm.as<int>();
  const int* comp = s->comp_full.as<int>();
  const int ge = grid_for(na);
  double* rz[2] = {sc + (size_t)SS_RZ0 * ns, sc + (size_t)SS_RZ1 * ns};
  // the box holds the final statistics (read_back) beside the two check slots
  ensure_box(s, kBoxRead + 1 + 5 * (size_t)ns);
  std::vector<double> bbh(ns), rth(ns);
  hipLaunchKernelGGL(k_gather_rhs_t, dim3(nt), dim3(kTileBlock), 0, s->stream, T, perm, comp, rhs,
                     b, tpart(T_BB));
  PPE_LAUNCH_CHECK();
  if (use_x0) {
    hipLaunchKernelGGL(k_gather_x0, dim3(ge), dim3(kBlock), 0, s->stream, na, perm, comp, p_out, x);
    PPE_LAUNCH_CHECK();
    apply_op<E_RESID, double>(s, L0, x, b, nullptr, 0.0, 0.0, r, nullptr);
  } else {
    fill_double(s, x, 0.0, na);
    hipLaunchKernelGGL(k_copy, dim3(ge), dim3(kBlock), 0, s->stream, na, b, r);
    PPE_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_norm2_t, dim3(nt), dim3(kTileBlock), 0, s->stream, T, r, tpart(T_RR));
  PPE_LAUNCH_CHECK();
  fill_int(s, cnt, 0, 2);
  hipLaunchKernelGGL(k_seg_init, dim3(ns), dim3(kTileBlock), 0, s->stream, ns, T, tpart(T_BB),
                     tpart(T_RR), s->opt.rtol * s->opt.rtol, sc, done, iters, restart, cnt);
  PPE_LAUNCH_CHECK();
  if (use_x0) {
    hipLaunchKernelGGL(k_zero_empty_t, dim3(nt), dim3(kTileBlock), 0, s->stream, T, ns, sc, x);
    PPE_LAUNCH_CHECK();
  }
  // true residual of every segment, then restart those that miss the
  // tolerance.  The scatter and the statistics ride along in the same round
  // trip: when nothing restarts they are the final ones.
  bool fetched = false;
  auto check_true = [&]() {
    apply_op<E_RESID, double>(s, L0, x, b, nullptr, 0.0, 0.0, q, nullptr);
    hipLaunchKernelGGL(k_norm2_t, dim3(nt), dim3(kTileBlock), 0, s->stream, T, q, tpart(T_RT));
    PPE_LAUNCH_CHECK();
    fill_int(s, cnt, 0, 1);
    hipLaunchKernelGGL(k_seg_check, dim3(ns), dim3(kTileBlock), 0, s->stream, ns, T, tpart(T_RT),
                       sc, done, restart, cnt);
    PPE_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_copy_restart_t, dim3(nt), dim3(kTileBlock), 0, s->stream, T, restart, q,
                       r);
    PPE_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(nc)), dim3(kBlock), 0, s->stream, nc,
                       s->cid.as<int>(), comp, x, p_out);
    PPE_LAUNCH_CHECK();
    int left = 0;
    read_back(s, {ReadItem{cnt, sizeof(int), &left},
                  ReadItem{sc + (size_t)SS_BB * ns, sizeof(double) * ns, bbh.data()},
                  ReadItem{sc + (size_t)SS_RES * ns, sizeof(double) * ns, rth.data()},
                  ReadItem{iters, sizeof(int) * ns, s->seg_iters_h.data()}});
    fetched = left == 0;
    return left;
  };
  auto finish = [&](ppe_status status) {
    if (!fetched) {
      hipLaunchKernelGGL(k_scatter, dim3(grid_for(nc)), dim3(kBlock), 0, s->stream, nc,
                         s->cid.as<int>(), comp, x, p_out);
      PPE_LAUNCH_CHECK();
      read_back(s, {ReadItem{sc + (size_t)SS_BB * ns, sizeof(double) * ns, bbh.data()},
                    ReadItem{sc + (size_t)SS_RES * ns, sizeof(double) * ns, rth.data()},
                    ReadItem{iters, sizeof(int) * ns, s->seg_iters_h.data()}});
    }
    profile_harvest(s);
    double worst = 0.0;
    int itmax = 0;
    for (int k = 0; k < ns; ++k) {
      s->seg_res_h[k] = bbh[k] > 0 ? std::sqrt(rth[k] / bbh[k]) : 0.0;
      worst = std::max(worst, s->seg_res_h[k]);
      itmax = std::max(itmax, s->seg_iters_h[k]);
    }
    st.rel_residual = worst;
    st.iterations = itmax;
    if (pred) *pred = itmax;
    return status;
  };

  // Samples converged from the start (zero right-hand side, exact guess) are
  // left alone by every iteration, so the first check below finds them.
  auto precondition = [&](int sl) { vcycle_pcg(s, r, zb[sl], PcgDot{T, nt, tpart(T_RZ)}); };
  precondition(1);
  hipLaunchKernelGGL(k_init_p_t, dim3(nt), dim3(kTileBlock), 0, s->stream, T, ns, done, tpart(T_RZ),
                     zb[1], p, rz[0]);
  PPE_LAUNCH_CHECK();
  // One PCG iteration of every sample still running: q = A p; x, r update;
  // the convergence test; z = M r; beta; p.  Samples already converged are
  // left untouched by every kernel, so extra iterations change nothing.
  auto body = [&](int sl) {
#define PPE_ELL_DOT(WM_)                                                                      \
  launch(s,                                                                                    \
         [&]() {                                                                               \
           return std::make_pair(kname("k_ell_dot_t", {str(WM_)}),                            \
                                 op_bytes<E_SPMV, double>(s, L0, true, 0.0));                 \
         },                                                                                    \
         k_ell_dot_t<WM_>, dim3(nt), dim3(kTileBlock), T, na, L0.W,                            \
         (const int*)L0.ell_col.as<int>(), (const double*)L0.ell_val.as<double>(),              \
         (const double*)L0.diag.as<double>(), (const int*)done, (const double*)p, q,           \
         tpart(T_PQ))
    PPE_ELL_WIDTH(L0.W, PPE_ELL_DOT);
#undef PPE_ELL_DOT
    // x, p, r, q in; x, r out
    launch(s, [&]() { return std::make_pair(std::string("k_update_xr_t"), 48.0 * na); },
           k_update_xr_t, dim3(nt), dim3(kTileBlock), T, (const int*)done, (const double*)rz[sl],
           (const double*)tpart(T_PQ), (const double*)p, (const double*)q, x, r, tpart(T_RR),
           cnt, cnt + 1);
    precondition(sl);
    // z, p in; p out
    launch(s, [&]() { return std::make_pair(std::string("k_update_p_t"), 24.0 * na); },
           k_update_p_t, dim3(nt), dim3(kTileBlock), T, ns, 1, done, restart,
           (const double*)tpart(T_RR), (const double*)sc, iters, cnt, (const double*)tpart(T_RZ),
           (const double*)rz[sl], rz[1 - sl], (const double*)zb[sl], p, cnt + 1);
  };
  // Two iterations (both rz slots) captured into a HIP graph on the second
  // solve with one hierarchy (a single solve per assembly would pay the
  // capture without reuse), replayed while at least two iterations remain.
  const bool graph = s->opt.use_graph && !s->prof && s->solves_since_assemble > 0;
  if (graph && !s->graph_ok) capture_iterations(s, [&]() { body(0); body(1); });
  int it = 0, slot = 0;
  const int max_iter = s->opt.max_iter, every = s->opt.check_every;
  // Convergence checks run one chunk behind: chunk c+1 is queued before the
  // host waits for the counts of chunk c, so the device does not idle during
  // the round trip.  A chunk queued after convergence changes nothing, but
  // its V-cycles still run: with a prediction of the iteration count (the
  // previous solve's), work is queued ahead only while it stays two
  // iterations short of it, and each chunk after that is checked before the
  // next is queued.
  for (auto& e : s->chk_ev)
    if (!e) PPE_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  struct Check {
    Published h;  // (active segments, error bits) once the event has passed
    int ev;
    int it;  // iterations launched up to this check
  };
  Check pend[2];
  int npend = 0, next_ev = 0;
  auto launch_chunk = [&]() {
    do {
      if (graph && slot == 0 && it + 2 <= max_iter) {
        PPE_HIP(hipGraphLaunch(s->gexec, s->stream));
        it += 2;
        break;
      }
      body(slot);
      slot = 1 - slot;
      it += 1;
    } while (it % every != 0 && it < max_iter);
    const ReadItem item{cnt, 2 * sizeof(int), nullptr};
    const Published h = publish(s, &item, 1, kBoxChecks + 3 * next_ev);
    PPE_HIP(hipEventRecord(s->chk_ev[next_ev], s->stream));
    pend[npend++] = Check{h, next_ev, it};
    next_ev = 1 - next_ev;
  };
  const int expect = pred ? *pred : 0;
  auto run_ahead = [&]() { return expect <= 0 || it + 2 <= expect - 2; };
  for (;;) {
    while (it < max_iter && (npend == 0 || (npend < 2 && run_ahead()))) launch_chunk();
    if (npend == 0) break;
    const Check c = pend[0];
    pend[0] = pend[1];
    --npend;
    PPE_HIP(hipEventSynchronize(s->chk_ev[c.ev]));
    const uint32_t* w = published_words(s, c.h);
    const int active = (int)w[0], bad = (int)w[1];
    if (bad) {
      finish(PPE_ERR_BREAKDOWN);
      return PPE_ERR_BREAKDOWN;
    }
    if (active == 0) {
      // everything converged at this check: the chunk behind it was a no-op
      npend = 0;
      it = c.it;
      if (check_true() == 0) return finish(PPE_OK);
      // restarted samples: z = M r_true, p = z (beta is 0 after a restart)
      precondition(slot);
      hipLaunchKernelGGL(k_update_p_t, dim3(nt), dim3(kTileBlock), 0, s->stream, T, ns, 0, done,
                         restart, tpart(T_RR), sc, iters, cnt, tpart(T_RZ), rz[slot],
                         rz[1 - slot], zb[slot], p, cnt + 1);
      PPE_LAUNCH_CHECK();
      slot = 1 - slot;
    }
  }
  // out of iterations: record the true residuals
  apply_op<E_RESID, double>(s, L0, x, b, nullptr, 0.0, 0.0, q, nullptr);
  hipLaunchKernelGGL(k_norm2_t, dim3(nt), dim3(kTileBlock), 0, s->stream, T, q, tpart(T_RT));
  PPE_LAUNCH_CHECK();
  fill_int(s, cnt, 0, 1);
  hipLaunchKernelGGL(k_seg_check, dim3(ns), dim3(kTileBlock), 0, s->stream, ns, T, tpart(T_RT), sc,
                     done, restart, cnt);
  PPE_LAUNCH_CHECK();
  return finish(PPE_NOT_CONVERGED);
}


namespace {

// Mean duration of launch() over reps dispatches on the solver stream, after
// one untimed dispatch.
template <class F>
float time_launches(ppe_solver* s, F&& launch, int reps = 3) {
  if (!s->tev0) {
    PPE_HIP(hipEventCreate(&s->tev0));
    PPE_HIP(hipEventCreate(&s->tev1));
  }
  launch();
  PPE_HIP(hipEventRecord(s->tev0, s->stream));
  for (int k = 0; k < reps; ++k) launch();
  PPE_HIP(hipEventRecord(s->tev1, s->stream));
  PPE_HIP(hipEventSynchronize(s->tev1));
  float ms = 0.f;
  PPE_HIP(hipEventElapsedTime(&ms, s->tev0, s->tev1));
  return ms / reps;
}

constexpr int kLprs[] = {1, 2, 4, 8, 16, 32, 64};

// The fastest lanes-per-row choice, candidates from a quarter of the fixed
// rule's choice (and at least lo) up to 64; its time in *t_out if given.
template <class F>
int best_lpr(ppe_solver* s, int rule, int lo, F&& run, float* t_out = nullptr) {
  int best = rule;
  float tbest = 1e30f;
  for (int c : kLprs) {
    if (c * 4 < rule || c < lo) continue;
    const float t = time_launches(s, [&]() { run(c); });
    if (t < tbest) { tbest = t; best = c; }
  }
  if (t_out) *t_out = tbest;
  return best;
}

// Tune one level's choices with matrix values in type M (the V-cycle's).
// Operands are the level's work vectors; their contents do not affect the
// timings.
template <class M>
void tune_level(ppe_solver* s, int l) {
  Level& L = s->levels[l];
  const bool coarsest = l == s->nlev - 1;
  if (L.n == 0 || (coarsest && L.dense)) return;
  double* x = L.x.as<double>();
  double* b = L.b.as<double>();
  double* d = L.d.as<double>();
  double* y = L.x2.as<double>();
  const double c1 = L.c1.empty() ? 0.0 : L.c1[0], c2 = L.c1.empty() ? L.inv_theta : L.c2[0];
  if (l > 0)
    L.lpr_a = best_lpr(s, smooth_lanes(L.A), 4, [&](int c) {
      L.lpr_a = c;
      apply_op<E_CHEB, M>(s, L, x, b, d, c1, c2, y, nullptr);
    });
  if (!L.c1.empty()) {
    // on a coarse level the split first step rides on the restriction into
    // the level, so both variants are timed with that restriction
    Level* F = l > 0 ? &s->levels[l - 1] : nullptr;
    const float fused = time_launches(s, [&]() {
      if (F) apply_rect<false, M>(s, F->R, F->r.as<double>(), b, F->lpr_r);
      apply_op<E_CHEB0, M>(s, L, nullptr, b, d, c1, c2, y, nullptr, nullptr, 0, L.inv_theta);
    });
    const float split = time_launches(s, [&]() {
      if (F)
        apply_rect<false, M, true>(s, F->R, F->r.as<double>(), b, F->lpr_r,
                                   FirstStep<M>{smooth_diag<M>(s, L), L.inv_theta, d, x});
      else
        hipLaunchKernelGGL(k_cheb_first<M>, dim3(grid_for(L.n)), dim3(kBlock), 0, s->stream,
                           L.n, b, smooth_diag<M>(s, L), L.inv_theta, d, x);
      apply_op<E_CHEB, M>(s, L, x, b, d, c1, c2, y, nullptr);
    });
    L.fuse0 = fused <= split;
  }
  if (coarsest) return;
  Level& C = s->levels[l + 1];
  L.lpr_r = best_lpr(s, restrict_lanes(L.R), 1, [&](int c) {
    apply_rect<false, M>(s, L.R, L.r.as<double>(), C.b.as<double>(), c);
  });
  // the prolongation alone, then (where it can fuse) the fused pass against
  // the prolongation followed by the first post-smoothing step
  float t_rect = 0.f;
  const int lp_rect = best_lpr(
      s, transfer_lanes(L.P), 1,
      [&](int c) { apply_rect<true, M>(s, L.P, C.x.as<double>(), L.t.as<double>(), c); },
      &t_rect);
  L.lpr_p = lp_rect;
  L.fuse_p = false;
  if (!prolong_can_fuse(s, L)) return;
  const float t_step = time_launches(s, [&]() {
    apply_op<E_CHEB, M>(s, L, L.t.as<double>(), b, d, 0.0, L.inv_theta, y, nullptr);
  });
  float t_fused = 0.f;
  L.fuse_p = true;
  L.lpr_p = 0;
  const int lp_fused = best_lpr(
      s, prolong_lanes(L), 4,
      [&](int c) {
        L.lpr_p = c;
        prolong_cheb<M>(s, L, C.x.as<double>(), L.t.as<double>(), b, d, y);
      },
      &t_fused);
  L.fuse_p = t_fused <= t_rect + t_step;
  L.lpr_p = L.fuse_p ? lp_fused : lp_rect;
}

}  // namespace

void autotune_levels(ppe_solver* s) {
  const bool f32 = s->opt.precision == PPE_MIXED;
  for (int l = 0; l < s->nlev; ++l) {
    Level& L = s->levels[l];
    // shapes within a quarter octave of rows and of entries share choices, so
    // a slowly changing active set rarely triggers a new tuning
    auto bin = [](double v) { return (int)std::lround(4.0 * std::log2(v > 1.0 ? v : 1.0)); };
    const std::array<int, 4> key{l, f32 ? 1 : 0, bin(L.n), bin((double)L.A.nnz)};
    auto it = s->tune_cache.find(key);
    if (it != s->tune_cache.end()) {
      L.lpr_a = it->second[0];
      L.fuse0 = it->second[1] != 0;
      L.lpr_r = it->second[2];
      L.lpr_p = it->second[3];
      L.fuse_p = it->second[4] != 0;
      continue;
    }
    if (f32)
      tune_level<float>(s, l);
    else
      tune_level<double>(s, l);
    s->tune_cache[key] = {L.lpr_a, L.fuse0 ? 1 : 0, L.lpr_r, L.lpr_p, L.fuse_p ? 1 : 0};
  }
}

}  // namespace ppe

// Smoothed-aggregation AMG setup on the device (the multigrid of section 2.5
// of the paper, which coarsens the matrix by heuristics without a physical
// grid; the paper names no variant, this is smoothed aggregation):
//
//   strength   j strong for i  iff  a_ij^2 >= theta_l^2 (a_ii a_jj), j != i,
//              theta_l = theta theta_decay^l on level l (finest l = 0)
//   MIS-2      synchronous rounds over keys (state, fmix32(i ^ salt), -i):
//              an undecided node that holds the maximum key of its
//              distance-2 neighbourhood joins, one that sees a member there
//              leaves; nodes without strong neighbours never take part
//   aggregates member roots; strong neighbours of a root join it; leftovers
//              join the first-pass neighbour with the largest |a_ij|
//              (ties to the lowest index)
//   P_tent     B restricted to each aggregate, normalised; coarse B = norms
//   rho        Gershgorin bound on the finest level, 1.1 x a 15-step power
//              estimate of lambda_max(D^-1 A) on coarse levels
//   P          P_tent - (4 / (3 rho)) D^-1 A P_tent;  R = P^T;  A_c = R (A P)
//   coarsest   at most coarse_max rows: explicit inverse (Gauss-Jordan)
//
// Every product is formed row by row in a fixed order (Gustavson order: the
// entries of the left factor's row in ascending column order), so the setup
// is bitwise reproducible from run to run.
#include "common.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace ppe {
namespace {

constexpr int kPowerIters = 15;
constexpr double kPowerSafety = 1.1;
constexpr int kDenseMax = 1024;

// Deferred setup checks: bits of an error word read back with the spectral
// bounds once the hierarchy is built.  Kernels between a failed check and the
// read stay in bounds (an unassigned node only leaves its prolongator row
// empty; a lost diagonal or a non-positive pivot only spoils values).
enum SetupErr : int { SE_DIAG = 1, SE_DENSE = 2, SE_AGG = 4 };

enum : int { S_OUT = 0, S_UND = 1, S_IN = 2 };

// Row kernels below give each row a group of LPR lanes (LPR = power of two
// near the mean row length); lanes stride over the row's entries and the
// group combines its results with shuffles, in a fixed order.
template <int LPR, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) v += __shfl_down(v, o, LPR);
  return v;
}

template <int LPR, class T>
__device__ __forceinline__ T group_max(T v) {
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) {
    T w = __shfl_down(v, o, LPR);
    v = w > v ? w : v;
  }
  return v;
}

// ------------------------------------------------------------------ strength
template <int LPR>
__global__ void __launch_bounds__(kBlock) k_strength(int n, const int* __restrict__ rp,
                                                     const int* __restrict__ ci,
                                                     const double* __restrict__ v,
                                                     const double* __restrict__ diag, double theta2,
                                                     unsigned char* __restrict__ strong,
                                                     unsigned char* __restrict__ state) {
  const int i = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / LPR, lane = threadIdx.x % LPR;
  int deg = 0;
  if (i < n) {
    const double di = diag[i];
    for (int k = rp[i] + lane; k < rp[i + 1]; k += LPR) {
      const int j = ci[k];
      const double a = v[k];
      const bool st = (j != i) && (a != 0.0) && (a * a >= theta2 * (di * diag[j]));
      strong[k] = st ? 1 : 0;
      deg += st ? 1 : 0;
    }
  }
  deg = group_sum<LPR>(deg);
  if (i < n && lane == 0) state[i] = deg > 0 ? S_UND : S_OUT;
}

// ------------------------------------------------------------------ MIS-2
__device__ __forceinline__ unsigned long long mis_key(unsigned char st, int j, uint32_t salt) {
  return ((unsigned long long)st << 62) |
         ((unsigned long long)fmix32((uint32_t)j ^ salt) << 30) |
         (unsigned long long)((1u << 30) - 1u - (uint32_t)j);
}

// m1_i = max key over i and its strong neighbours
template <int LPR>
__global__ void __launch_bounds__(kBlock) k_mis_max1(int n, const int* __restrict__ rp,
                                                     const int* __restrict__ ci,
                                                     const unsigned char* __restrict__ strong,
                                                     const unsigned char* __restrict__ state,
                                                     uint32_t salt,
                                                     unsigned long long* __restrict__ m1) {
  const int i = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / LPR, lane = threadIdx.x % LPR;
  unsigned long long m = 0;
  if (i < n) {
    for (int k = rp[i] + lane; k < rp[i + 1]; k += LPR) {
      if (!strong[k]) continue;
      const int j = ci[k];
      const unsigned long long kj = mis_key(state[j], j, salt);
      m = kj > m ? kj : m;
    }
  }
  m = group_max<LPR>(m);
  if (i < n && lane == 0) {
    const unsigned long long own = mis_key(state[i], i, salt);
    m1[i] = own > m ? own : m;
  }
}

// m2_i = max m1 over i and its strong neighbours; an undecided node joins if
// m2 is its own key, leaves if m2 belongs to a member.  *undecided is set to
// 1 if any node stays undecided.
template <int LPR>
__global__ void __launch_bounds__(kBlock) k_mis_max2(int n, const int* __restrict__ rp,
                                                     const int* __restrict__ ci,
                                                     const unsigned char* __restrict__ strong,
                                                     const unsigned char* __restrict__ state,
                                                     uint32_t salt,
                                                     const unsigned long long* __restrict__ m1,
                                                     unsigned char* __restrict__ next,
                                                     int* __restrict__ undecided) {
  const int i = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / LPR, lane = threadIdx.x % LPR;
  const unsigned char st = i < n ? state[i] : (unsigned char)S_OUT;
  unsigned long long m = 0;
  int und = 0;
  if (i < n && st == S_UND) {
    for (int k = rp[i] + lane; k < rp[i + 1]; k += LPR) {
      if (!strong[k]) continue;
      const unsigned long long mj = m1[ci[k]];
      m = mj > m ? mj : m;
    }
  }
  m = group_max<LPR>(m);
  if (i < n && lane == 0) {
    unsigned char ns = st;
    if (st == S_UND) {
      const unsigned long long own = mis_key(st, i, salt);
      const unsigned long long mm = m1[i] > m ? m1[i] : m;
      if (mm == own)
        ns = S_IN;
      else if ((mm >> 62) == S_IN)
        ns = S_OUT;
    }
    next[i] = ns;
    und = ns == S_UND ? 1 : 0;
  }
  // the host only asks whether any node is still undecided: a plain store of
  // the same value from every such block (same-address atomics from every
  // block serialise across the chip)
  und = block_sum<kBlock>(und);
  if (threadIdx.x == 0 && und) *undecided = 1;
}

// ------------------------------------------------------------------ finest level, ELL
// The same strength, MIS-2 and joining rules on the finest level's
// slot-major ELL copy of the off-diagonal part (slot k of row i at
// k n + i, padding = the row itself): one thread per row, every slot's load
// issued before its gathers, no row pointers.  The strength pass leaves
// scol = the column of each strong entry and the row itself elsewhere, so
// the later passes read one array.  Results are maxima and per-entry tests,
// as in the CSR kernels, so they are the same bit for bit.
template <int WM>
__device__ __forceinline__ void slot_cols(int i, int n, int W, const int* __restrict__ col,
                                          int (&c)[WM]) {
#pragma unroll
  for (int k = 0; k < WM; ++k) c[k] = k < W ? col[(size_t)k * n + i] : i;
}

// WM: unrolled slot count covering W (0: a plain loop over W slots).
template <int WM>
__global__ void __launch_bounds__(kBlock) k_strength_ell(int n, int W, const int* __restrict__ ecol,
                                                         const double* __restrict__ ev,
                                                         const double* __restrict__ diag,
                                                         double theta2, int* __restrict__ scol,
                                                         unsigned char* __restrict__ state) {
  const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const double di = diag[i];
  int deg = 0;
  auto test = [&](int k, int j) {
    const double a = ev[(size_t)k * n + i];
    const bool st = (j != i) && (a != 0.0) && (a * a >= theta2 * (di * diag[j]));
    scol[(size_t)k * n + i] = st ? j : i;
    deg += st ? 1 : 0;
  };
  if constexpr (WM > 0) {
    int c[WM];
    slot_cols<WM>(i, n, W, ecol, c);
#pragma unroll
    for (int k = 0; k < WM; ++k)
      if (k < W) test(k, c[k]);
  } else {
    for (int k = 0; k < W; ++k) test(k, ecol[(size_t)k * n + i]);
  }
  state[i] = deg > 0 ? S_UND : S_OUT;
}

template <int WM>
__global__ void __launch_bounds__(kBlock) k_mis_max1_ell(int n, int W, const int* __restrict__ scol,
                                                         const unsigned char* __restrict__ state,
                                                         uint32_t salt,
                                                         unsigned long long* __restrict__ m1) {
  const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  unsigned long long m = mis_key(state[i], i, salt);
  auto take = [&](int j) {
    if (j == i) return;
    const unsigned long long kj = mis_key(state[j], j, salt);
    m = kj > m ? kj : m;
  };
  if constexpr (WM > 0) {
    int c[WM];
    slot_cols<WM>(i, n, W, scol, c);
#pragma unroll
    for (int k = 0; k < WM; ++k) take(c[k]);
  } else {
    for (int k = 0; k < W; ++k) take(scol[(size_t)k * n + i]);
  }
  m1[i] = m;
}

template <int WM>
__global__ void __launch_bounds__(kBlock) k_mis_max2_ell(int n, int W, const int* __restrict__ scol,
                                                         const unsigned char* __restrict__ state,
                                                         uint32_t salt,
                                                         const unsigned long long* __restrict__ m1,
                                                         unsigned char* __restrict__ next,
                                                         int* __restrict__ undecided) {
  const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  const unsigned char st = i < n ? state[i] : (unsigned char)S_OUT;
  int und = 0;
  if (i < n) {
    unsigned char ns = st;
    if (st == S_UND) {
      unsigned long long m = m1[i];
      auto take = [&](int j) {
        if (j == i) return;
        const unsigned long long mj = m1[j];
        m = mj > m ? mj : m;
      };
      if constexpr (WM > 0) {
        int c[WM];
        slot_cols<WM>(i, n, W, scol, c);
#pragma unroll
        for (int k = 0; k < WM; ++k) take(c[k]);
      } else {
        for (int k = 0; k < W; ++k) take(scol[(size_t)k * n + i]);
      }
      if (m == mis_key(st, i, salt))
        ns = S_IN;
      else if ((m >> 62) == S_IN)
        ns = S_OUT;
    }
    next[i] = ns;
    und = ns == S_UND ? 1 : 0;
  }
  und = block_sum<kBlock>(und);
  if (threadIdx.x == 0 && und) *undecided = 1;
}

template <int WM>
__global__ void __launch_bounds__(kBlock) k_agg_first_ell(int n, int W, const int* __restrict__ scol,
                                                          const unsigned char* __restrict__ state,
                                                          const int* __restrict__ root_id,
                                                          int* __restrict__ agg1) {
  const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  if (state[i] == S_IN) {
    agg1[i] = root_id[i];
    return;
  }
  int a = -1;
  auto take = [&](int j) {
    if (j != i && state[j] == S_IN) a = max(a, root_id[j]);
  };
  if constexpr (WM > 0) {
    int c[WM];
    slot_cols<WM>(i, n, W, scol, c);
#pragma unroll
    for (int k = 0; k < WM; ++k) take(c[k]);
  } else {
    for (int k = 0; k < W; ++k) take(scol[(size_t)k * n + i]);
  }
  agg1[i] = a;
}

template <int WM>
__global__ void __launch_bounds__(kBlock) k_agg_second_ell(int n, int W, const int* __restrict__ scol,
                                                           const double* __restrict__ ev,
                                                           const int* __restrict__ agg1,
                                                           int* __restrict__ agg,
                                                           int* __restrict__ flag) {
  const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  int a = agg1[i];
  if (a < 0) {
    double best = -1.0;
    int bestj = INT32_MAX, any = 0;
    auto take = [&](int k, int j) {
      if (j == i) return;
      any = 1;
      if (agg1[j] < 0) return;
      const double w = fabs(ev[(size_t)k * n + i]);
      if (w > best || (w == best && j < bestj)) { best = w; bestj = j; }
    };
    if constexpr (WM > 0) {
      int c[WM];
      slot_cols<WM>(i, n, W, scol, c);
#pragma unroll
      for (int k = 0; k < WM; ++k) take(k, c[k]);
    } else {
      for (int k = 0; k < W; ++k) take(k, scol[(size_t)k * n + i]);
    }
    if (best >= 0.0) a = agg1[bestj];
    else if (any) atomicOr(flag, SE_AGG);
  }
  agg[i] = a;
}

// Finest level: Q = A P_tent from the ELL copy, one thread per row.  P_tent
// has one entry per aggregated node (pt_j in column agg_j), so row i of Q
// holds, for every aggregate J reached from row i, the sum of a_ij pt_j
// over that row's entries j in J.  The row's entries are taken in CSR order
// (ascending column, the diagonal in its place) and each sum starts from 0
// in that order: bitwise the general product's one-sub-group result.  COUNT:
// distinct aggregates per row into counts; else the row, sorted by
// aggregate, at rp[i].
template <int WM, bool COUNT>
__global__ void __launch_bounds__(kBlock) k_coarsen_cols_ell(
    int n, int W, const int* __restrict__ ecol, const double* __restrict__ ev,
    const double* __restrict__ diag, const int* __restrict__ agg, const double* __restrict__ pt,
    int* __restrict__ counts, const int* __restrict__ rp, int* __restrict__ ci,
    double* __restrict__ v) {
  const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  // fixed register slots: ELL slot k (aggregate Jk[k], -1 for none), and the
  // diagonal, which comes before slot dpos in CSR order
  int c[WM];
  slot_cols<WM>(i, n, W, ecol, c);
  int Jk[WM];
  double yk[WM];
  int dpos = WM;
#pragma unroll
  for (int k = WM - 1; k >= 0; --k) {
    const int j = c[k];
    const bool real = j != i;  // padding (slots past W included) holds the row
    if (real && j > i) dpos = k;
    Jk[k] = real ? agg[j] : -1;
    if (!COUNT) yk[k] = Jk[k] >= 0 ? ev[(size_t)k * n + i] * pt[j] : 0.0;
  }
  const int Jd = agg[i];
  const double yd = (!COUNT && Jd >= 0) ? diag[i] * pt[i] : 0.0;
  int out = COUNT ? 0 : rp[i];
  int last = -1;
  for (int step = 0; step <= WM; ++step) {
    int cur = Jd > last ? Jd : INT32_MAX;
#pragma unroll
    for (int k = 0; k < WM; ++k)
      if (Jk[k] > last && Jk[k] < cur) cur = Jk[k];
    if (cur == INT32_MAX) break;
    if (!COUNT) {
      double sum = 0.0;
#pragma unroll
      for (int k = 0; k <= WM; ++k) {
        if (k == dpos && Jd == cur) sum = sum + yd;
        if (k < WM && Jk[k] == cur) sum = sum + yk[k];
      }
      ci[out] = cur;
      v[out] = sum;
    }
    ++out;
    last = cur;
  }
  if (COUNT) counts[i] = out;
}

// Finest level: AP = A P by rows, one thread per row from the ELL copy:
// row i of AP merges the sorted rows of P selected by row i of A (its ELL
// slots and the diagonal, at most WM + 1 of them), column by column.  A
// column's products are added from 0 in CSR order of A's row, which is the
// order the general product adds them in (one sub-group walks A's row in
// order): bitwise its result.  COUNT: entries per row into counts; else the
// row, sorted, at rp[i].
template <int WM, bool COUNT>
__global__ void __launch_bounds__(kBlock) k_ap_merge_ell(
    int n, int W, const int* __restrict__ ecol, const double* __restrict__ ev,
    const double* __restrict__ diag, const int* __restrict__ prp, const int* __restrict__ pci,
    const double* __restrict__ pv, int* __restrict__ counts, const int* __restrict__ rp,
    int* __restrict__ ci, double* __restrict__ v) {
  const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  int c[WM];
  slot_cols<WM>(i, n, W, ecol, c);
  // list k < WM: row c[k] of P (empty for padding); list WM: row i (the
  // diagonal), which comes before list dpos in CSR order
  int pos[WM + 1], end[WM + 1], col[WM + 1];
  double a[WM + 1], pval[WM + 1];
  int dpos = WM;
#pragma unroll
  for (int k = WM; k >= 0; --k) {
    const int j = k < WM ? c[k] : i;
    const bool real = k == WM || j != i;
    if (k < WM && real && j > i) dpos = k;
    pos[k] = real ? prp[j] : 0;
    end[k] = real ? prp[j + 1] : 0;
    if (!COUNT) a[k] = k < WM ? (real ? ev[(size_t)k * n + i] : 0.0) : diag[i];
  }
#pragma unroll
  for (int k = 0; k <= WM; ++k) {
    col[k] = pos[k] < end[k] ? pci[pos[k]] : INT32_MAX;
    if (!COUNT) pval[k] = pos[k] < end[k] ? pv[pos[k]] : 0.0;
  }
  int out = COUNT ? 0 : rp[i];
  for (;;) {
    int cur = col[0];
#pragma unroll
    for (int k = 1; k <= WM; ++k) cur = col[k] < cur ? col[k] : cur;
    if (cur == INT32_MAX) break;
    if (!COUNT) {
      double sum = 0.0;
#pragma unroll
      for (int k = 0; k <= WM; ++k) {
        if (k == dpos && col[WM] == cur) sum = sum + a[WM] * pval[WM];
        if (k < WM && col[k] == cur) sum = sum + a[k] * pval[k];
      }
      ci[out] = cur;
      v[out] = sum;
    }
    ++out;
#pragma unroll
    for (int k = 0; k <= WM; ++k)
      if (col[k] == cur) {
        ++pos[k];
        col[k] = pos[k] < end[k] ? pci[pos[k]] : INT32_MAX;
        if (!COUNT) pval[k] = pos[k] < end[k] ? pv[pos[k]] : 0.0;
      }
  }
  if (COUNT) counts[i] = out;
}

// ------------------------------------------------------------------ aggregation
__global__ void k_is_root(int n, const unsigned char* __restrict__ state, int* __restrict__ root) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) root[i] = state[i] == S_IN ? 1 : 0;
}

// A root's id; a node with a strong root neighbour takes that root's id (the
// root is unique: roots are at least three edges apart); others -1.
template <int LPR>
__global__ void __launch_bounds__(kBlock) k_agg_first(int n, const int* __restrict__ rp,
                                                      const int* __restrict__ ci,
                                                      const unsigned char* __restrict__ strong,
                                                      const unsigned char* __restrict__ state,
                                                      const int* __restrict__ root_id,
                                                      int* __restrict__ agg1) {
  const int i = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / LPR, lane = threadIdx.x % LPR;
  int a = -1;
  const bool root = i < n && state[i] == S_IN;
  if (i < n && !root) {
    for (int k = rp[i] + lane; k < rp[i + 1]; k += LPR) {
      const int j = ci[k];
      if (strong[k] && state[j] == S_IN) a = root_id[j];
    }
  }
  a = group_max<LPR>(a);
  if (i < n && lane == 0) agg1[i] = root ? root_id[i] : a;
}

// Leftover nodes join the first-pass neighbour with the largest |a_ij|, ties
// to the lowest j.
template <int LPR>
__global__ void __launch_bounds__(kBlock) k_agg_second(int n, const int* __restrict__ rp,
                                                       const int* __restrict__ ci,
                                                       const double* __restrict__ v,
                                                       const unsigned char* __restrict__ strong,
                                                       const int* __restrict__ agg1,
                                                       int* __restrict__ agg, int* __restrict__ flag) {
  const int i = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / LPR, lane = threadIdx.x % LPR;
  const int a1 = i < n ? agg1[i] : 0;
  double best = -1.0;
  int bestj = INT32_MAX;
  int any = 0;
  if (i < n && a1 < 0) {
    for (int k = rp[i] + lane; k < rp[i + 1]; k += LPR) {
      if (!strong[k]) continue;
      any = 1;
      const int j = ci[k];
      if (agg1[j] < 0) continue;
      const double w = fabs(v[k]);
      if (w > best || (w == best && j < bestj)) { best = w; bestj = j; }
    }
  }
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) {
    const double wb = __shfl_down(best, o, LPR);
    const int jb = __shfl_down(bestj, o, LPR);
    if (wb > best || (wb == best && jb < bestj)) { best = wb; bestj = jb; }
  }
  any = group_max<LPR>(any);
  if (i < n && lane == 0) {
    int a = a1;
    if (a < 0) {
      if (best >= 0.0) a = agg1[bestj];
      else if (any) atomicOr(flag, SE_AGG);
    }
    agg[i] = a;
  }
}

__global__ void k_agg_count(int n, const int* __restrict__ agg, int* __restrict__ cnt) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n && agg[i] >= 0) atomicAdd(&cnt[agg[i]], 1);
}

__global__ void k_agg_fill(int n, const int* __restrict__ agg, int* __restrict__ cursor,
                           int* __restrict__ mem) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n && agg[i] >= 0) mem[atomicAdd(&cursor[agg[i]], 1)] = i;
}

// Sort each aggregate's members, then norm_J = sqrt(sum B_i^2) in ascending
// i.  One wavefront per aggregate.  Up to 64 members are ranked in
// registers; up to kAggLds by the whole wave (the members staged in LDS,
// each lane counts for its own members the smaller keys among all of them,
// then writes them back in rank order); a larger aggregate is sorted by
// one lane in place.  The squares are summed
// in rank order by one lane.
constexpr int kAggLds = 1024;
__global__ void __launch_bounds__(kBlock) k_agg_norm(int na, const int* __restrict__ ptr,
                                                     int* __restrict__ mem,
                                                     const double* __restrict__ B,
                                                     double* __restrict__ Bc) {
  __shared__ double sq[kBlock];
  __shared__ int skey[kBlock / kWave][kAggLds];
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int J = blockIdx.x * (kBlock / kWave) + w;
  if (J >= na) return;  // whole wavefronts: only wave-level ordering below
  const int b = ptr[J], e = ptr[J + 1], m = e - b;
  double* wsq = sq + w * kWave;
  int* wk = skey[w];
  // a wavefront's LDS operations complete in issue order; the fences keep
  // the compiler from moving them across
  auto wave_sync = []() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  double s = 0.0;
  if (m <= kWave) {
    const int key = lane < m ? mem[b + lane] : INT32_MAX;
    int rank = 0;
    for (int q = 0; q < m; ++q) rank += __shfl(key, q, kWave) < key ? 1 : 0;
    if (lane < m) {
      mem[b + rank] = key;
      wsq[rank] = B[key] * B[key];
    }
    wave_sync();
    if (lane == 0)
      for (int q = 0; q < m; ++q) s = s + wsq[q];
  } else if (m <= kAggLds) {
    constexpr int T = kAggLds / kWave;  // members per lane
    int myk[T], myr[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int i = lane + t * kWave;
      myk[t] = i < m ? mem[b + i] : INT32_MAX;
      if (i < m) wk[i] = myk[t];
    }
    wave_sync();
#pragma unroll
    for (int t = 0; t < T; ++t) {
      int r = 0;
      if (lane + t * kWave < m)
        for (int q = 0; q < m; ++q) r += wk[q] < myk[t] ? 1 : 0;
      myr[t] = r;
    }
    wave_sync();  // every lane has read wk before it is overwritten in rank order
#pragma unroll
    for (int t = 0; t < T; ++t)
      if (lane + t * kWave < m) wk[myr[t]] = myk[t];
    wave_sync();
    for (int c = 0; c < m; c += kWave) {
      const int q = c + lane;
      if (q < m) {
        const int key = wk[q];
        mem[b + q] = key;
        wsq[lane] = B[key] * B[key];
      }
      wave_sync();
      if (lane == 0)
        for (int t = 0; t < kWave && c + t < m; ++t) s = s + wsq[t];
      wave_sync();  // wsq is rewritten for the next chunk
    }
  } else if (lane == 0) {
    for (int i = b + 1; i < e; ++i) {
      int key = mem[i], j = i - 1;
      while (j >= b && mem[j] > key) { mem[j + 1] = mem[j]; --j; }
      mem[j + 1] = key;
    }
    for (int i = b; i < e; ++i) s = s + B[mem[i]] * B[mem[i]];
  }
  if (lane == 0) Bc[J] = sqrt(s);
}

__global__ void k_tent(int n, const int* __restrict__ agg, const double* __restrict__ B,
                       const double* __restrict__ Bc, int* __restrict__ cnt,
                       double* __restrict__ pt) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int a = agg[i];
  cnt[i] = a >= 0 ? 1 : 0;
  pt[i] = a >= 0 ? B[i] / Bc[a] : 0.0;
}

__global__ void k_tent_csr(int n, const int* __restrict__ rp, const int* __restrict__ agg,
                           const double* __restrict__ pt, int* __restrict__ ci,
                           double* __restrict__ v) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  if (agg[i] >= 0) {
    ci[rp[i]] = agg[i];
    v[rp[i]] = pt[i];
  }
}

// P = P_tent - omega D^-1 (A P_tent); the pattern of A P_tent contains P_tent's.
// omega = 4 / (3 rho) with rho the level's spectral bound (device value).
__global__ void k_smooth_p(int n, const int* __restrict__ qrp, const int* __restrict__ qci,
                           const double* __restrict__ qv, const double* __restrict__ diag,
                           const int* __restrict__ agg, const double* __restrict__ pt,
                           const double* __restrict__ rho, double* __restrict__ pv) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double omega = 4.0 / (3.0 * *rho);
  const double dinv = 1.0 / diag[i];
  const int ai = agg[i];
  for (int k = qrp[i]; k < qrp[i + 1]; ++k) {
    double t = (qci[k] == ai) ? pt[i] : 0.0;
    pv[k] = t - omega * (qv[k] * dinv);
  }
}

// ------------------------------------------------------------------ spectral bounds
// Gershgorin bound of D^-1 A: block maxima of sum_j |a_ij| / a_ii
__global__ void k_gershgorin(int n, const int* __restrict__ rp, const double* __restrict__ v,
                             const double* __restrict__ diag, double* __restrict__ part) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  double r = 0.0;
  if (i < n) {
    for (int k = rp[i]; k < rp[i + 1]; ++k) r = r + fabs(v[k]);
    r = r / diag[i];
  }
  r = block_max<kBlock>(r);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ void __launch_bounds__(kBlock) k_max_partials(const double* __restrict__ part, int g,
                                                         double* __restrict__ out) {
  double m = 0.0;
  for (int b = threadIdx.x; b < g; b += kBlock) m = fmax(m, part[b]);
  m = block_max<kBlock>(m);
  if (threadIdx.x == 0) *out = m;
}

template <int LPR>
__global__ void __launch_bounds__(kBlock) k_diag(int n, const int* __restrict__ rp,
                                                 const int* __restrict__ ci,
                                                 const double* __restrict__ v,
                                                 double* __restrict__ diag, int* __restrict__ flag) {
  const int i = (blockIdx.x * kBlock + threadIdx.x) / LPR, lane = threadIdx.x % LPR;
  double d = 0.0;  // only the lane holding the diagonal adds a nonzero term
  if (i < n)
    for (int k = rp[i] + lane; k < rp[i + 1]; k += LPR)
      if (ci[k] == i) d = v[k];
  d = group_sum<LPR>(d);
  if (i < n && lane == 0) {
    diag[i] = d;
    if (!(d > 0.0)) atomicOr(flag, SE_DIAG);
  }
}

// ------------------------------------------------------------------ sparse products
__device__ __forceinline__ uint32_t slot_hash(int key) { return fmix32((uint32_t)key); }

// Products per row of C = A B: the summed lengths of the rows of B that row
// i of A selects (clipped at 2^30).
template <int LPR>
__global__ void __launch_bounds__(kBlock) k_spgemm_bound(int n, const int* __restrict__ arp,
                                                         const int* __restrict__ aci,
                                                         const int* __restrict__ brp,
                                                         int* __restrict__ prod) {
  const int i = (blockIdx.x * kBlock + threadIdx.x) / LPR, lane = threadIdx.x % LPR;
  long long s = 0;
  if (i < n)
    for (int a = arp[i] + lane; a < arp[i + 1]; a += LPR) s += brp[aci[a] + 1] - brp[aci[a]];
  s = group_sum<LPR>(s);
  if (i < n && lane == 0) prod[i] = s > (1 << 30) ? (1 << 30) : (int)s;
}

enum SpMode { SP_COUNT = 0, SP_FILL = 1, SP_DENSE = 2, SP_BITS = 3 };
constexpr int kSpBatch = 4;        // entries of A whose loads are issued together
constexpr int kSpDenseWidth = 512; // widest C accumulated with one slot per column

// Row-parallel C = A B.  Row i of C belongs to W sub-groups of LPR lanes;
// sub-group w walks its contiguous run of row i of A in ascending order and
// scatters the products with each selected row of B into its own value
// array.  The lanes of a sub-group hold distinct columns of that row of B
// and a wavefront's LDS operations complete in issue order, so the products
// reaching one slot from one sub-group are added in entry order with no
// barrier; the sub-groups' arrays are then added in the order w = 0..W-1.
// The result therefore depends only on W, never on timing.  Column slots are
// shared by the row's sub-groups:
//   SP_COUNT  open-addressing hash of column ids (H slots, a power of two);
//             counts[i] = distinct columns of the row;
//   SP_FILL   the same hash; the row is written to C at off[i], sorted by
//             column (rank among the row's columns);
//   SP_DENSE  slot = column (H >= width); the row is written in column order
//             to the scratch row at off[i]; counts[i] = entries written;
//   SP_BITS   a bit per column of C in H 32-bit words (no probing); counts[i]
//             = bits set, the row's distinct columns as with SP_COUNT.
// The block holds blockDim / (LPR W) rows; LDS is sized by the host.
template <int LPR, int MODE>
__global__ void __launch_bounds__(1024) k_spgemm_rows(
    int n, int W, int H, const int* __restrict__ arp, const int* __restrict__ aci,
    const double* __restrict__ av, const int* __restrict__ brp, const int* __restrict__ bci,
    const double* __restrict__ bv, const int* __restrict__ off, int* __restrict__ counts,
    int* __restrict__ cci, double* __restrict__ cv, int* __restrict__ flag) {
  extern __shared__ double smem[];
  const int per_row = LPR * W;
  const int rpb = blockDim.x / per_row;
  const int rl = threadIdx.x / per_row, tr = threadIdx.x % per_row;
  const int w = tr / LPR, lane = tr % LPR;
  const int i = blockIdx.x * rpb + rl;
  const bool numeric = MODE == SP_FILL || MODE == SP_DENSE;
  double* vals = smem + (size_t)rl * W * H;  // [W][H] of this row
  int* ibase = reinterpret_cast<int*>(smem + (numeric ? (size_t)rpb * W * H : 0));
  int* keys = ibase + (size_t)rl * H;
  // SP_FILL: the row's occupied slots and their columns, at most H / 2 each
  int* list = ibase + (size_t)rpb * H + (size_t)rl * H;
  int* ckey = list + H / 2;
  int* cnt = ibase + (size_t)(MODE == SP_FILL ? 2 : 1) * rpb * H;
  for (int q = tr; q < H; q += per_row) {
    keys[q] = MODE == SP_BITS ? 0 : -1;
    if (numeric)
      for (int v = 0; v < W; ++v) vals[(size_t)v * H + q] = 0.0;
  }
  if (MODE == SP_DENSE) {
    for (int q = tr; q < per_row / kWave + 1; q += per_row) cnt[rl * (per_row / kWave + 1) + q] = 0;
  } else if (tr == 0) {
    cnt[rl] = 0;
  }
  __syncthreads();

  bool overflow = false;
  auto insert = [&](int key, double y) {
    int q;
    if (MODE == SP_BITS) {
      atomicOr(reinterpret_cast<unsigned*>(keys) + (key >> 5), 1u << (key & 31));
      return;
    }
    if (MODE == SP_DENSE) {
      q = key;
      keys[q] = key;
    } else {
      q = (int)(slot_hash(key) & (uint32_t)(H - 1));
      int probes = 0;
      while (true) {
        const int prev = atomicCAS(&keys[q], -1, key);
        if (prev == -1) {
          if (MODE == SP_COUNT) atomicAdd(&cnt[rl], 1);
          break;
        }
        if (prev == key) break;
        q = (q + 1) & (H - 1);
        if (++probes >= H) { overflow = true; return; }
      }
    }
    if (numeric) vals[(size_t)w * H + q] += y;
  };

  if (i < n) {
    const int a0 = arp[i], a1 = arp[i + 1];
    const int chunk = (a1 - a0 + W - 1) / W;
    const int lo = a0 + w * chunk, hi = min(a1, lo + chunk);
    for (int e = lo; e < hi; e += kSpBatch) {
      int kk[kSpBatch], bb[kSpBatch], be[kSpBatch];
      double xa[kSpBatch], yy[kSpBatch];
#pragma unroll
      for (int u = 0; u < kSpBatch; ++u) {
        kk[u] = -1;
        bb[u] = 0;
        be[u] = 0;
        xa[u] = 0.0;
        yy[u] = 0.0;
        if (e + u < hi) {
          const int j = aci[e + u];
          bb[u] = brp[j];
          be[u] = brp[j + 1];
          if (numeric) xa[u] = av[e + u];
          const int b = bb[u] + lane;
          if (b < be[u]) {
            kk[u] = bci[b];
            if (numeric) yy[u] = xa[u] * bv[b];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kSpBatch; ++u) {
        if (kk[u] >= 0) insert(kk[u], yy[u]);
        for (int b = bb[u] + lane + LPR; b < be[u]; b += LPR)
          insert(bci[b], numeric ? xa[u] * bv[b] : 0.0);
      }
    }
  }
  if (overflow) atomicOr(flag, 1);
  __syncthreads();

  if (MODE == SP_BITS) {
    int c = 0;
    for (int q = tr; q < H; q += per_row) c += __popc((unsigned)keys[q]);
    atomicAdd(&cnt[rl], c);
    __syncthreads();
    if (i < n && tr == 0) counts[i] = cnt[rl];
    return;
  }
  if (MODE == SP_COUNT) {
    if (i < n && tr == 0) counts[i] = cnt[rl];
    return;
  }
  if (MODE == SP_FILL) {
    for (int q = tr; q < H; q += per_row) {
      const int key = keys[q];
      if (key != -1) {
        double v = vals[q];
        for (int u = 1; u < W; ++u) v += vals[(size_t)u * H + q];
        vals[q] = v;
        const int p = atomicAdd(&cnt[rl], 1);
        list[p] = q;
        ckey[p] = key;
      }
    }
    __syncthreads();
    if (i >= n) return;
    const int u = cnt[rl], base = off[i];
    for (int p = tr; p < u; p += per_row) {
      const int key = ckey[p];
      int rank = 0;
      for (int q = 0; q < u; ++q) rank += ckey[q] < key ? 1 : 0;
      cci[base + rank] = key;
      cv[base + rank] = vals[list[p]];
    }
    return;
  }
  // SP_DENSE: thread tr owns the contiguous slots [s0, s1); an exclusive scan
  // of the owned counts over the row's threads gives each its output offset.
  const int per = (H + per_row - 1) / per_row;
  const int s0 = min(H, tr * per), s1 = min(H, s0 + per);
  int c = 0;
  for (int q = s0; q < s1; ++q) c += keys[q] != -1 ? 1 : 0;
  const int width = per_row < kWave ? per_row : kWave;
  int inc = c;
  const int wl = tr % width;
  for (int o = 1; o < width; o <<= 1) {
    const int t = __shfl_up(inc, o, width);
    if (wl >= o) inc += t;
  }
  int* wtot = cnt + rl * (per_row / kWave + 1);
  if (per_row > kWave) {
    if (wl == width - 1) wtot[tr / kWave] = inc;
    __syncthreads();
    int before = 0;
    for (int q = 0; q < tr / kWave; ++q) before += wtot[q];
    inc += before;
  }
  if (i >= n) return;
  int pos = off[i] + inc - c;
  for (int q = s0; q < s1; ++q) {
    if (keys[q] != -1) {
      double v = vals[q];
      for (int u = 1; u < W; ++u) v += vals[(size_t)u * H + q];
      cci[pos] = q;
      cv[pos] = v;
      ++pos;
    }
  }
  if (tr == per_row - 1) counts[i] = inc;
}

__global__ void k_stride_offsets(int n, int stride, int* __restrict__ off) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) off[i] = i * stride;
}

// Copy the rows of a product from scratch rows (at off[i]) into C.
template <int LPR>
__global__ void __launch_bounds__(kBlock) k_spgemm_compact(int n, const int* __restrict__ off,
                                                           const int* __restrict__ crp,
                                                           const int* __restrict__ sci,
                                                           const double* __restrict__ sv,
                                                           int* __restrict__ cci,
                                                           double* __restrict__ cv) {
  const int i = (blockIdx.x * kBlock + threadIdx.x) / LPR, lane = threadIdx.x % LPR;
  if (i >= n) return;
  const int src = off[i], dst = crp[i], len = crp[i + 1] - dst;
  for (int k = lane; k < len; k += LPR) {
    cci[dst + k] = sci[src + k];
    cv[dst + k] = sv[src + k];
  }
}

// ------------------------------------------------------------------ transpose
// A narrow matrix (at most kNarrowCols columns, such as the prolongator onto
// the coarsest level) is transposed without atomics on its few column
// counters and without sorting: a one-workgroup count, then one workgroup
// per column that collects the column's entries in storage order.
constexpr int kNarrowCols = 1024;
constexpr int kNarrowU = 8;  // entries per lane whose loads are issued together

// Column counts in LDS, then T's row pointers trp[0..m] (exclusive scan over
// the columns) and its longest row *rmax.  One workgroup of 1024 threads.
__global__ void __launch_bounds__(1024) k_narrow_count(int64_t nnz, int m,
                                                       const int* __restrict__ ci,
                                                       int* __restrict__ trp,
                                                       int* __restrict__ rmax) {
  __shared__ int h[kNarrowCols];
  __shared__ int wsum[1024 / kWave];
  __shared__ int hmax;
  const int t = threadIdx.x, lane = t % kWave, w = t / kWave;
  h[t] = 0;
  if (t == 0) hmax = 0;
  __syncthreads();
  for (int64_t k0 = t; k0 < nnz; k0 += 1024 * kNarrowU) {
    int c[kNarrowU];
#pragma unroll
    for (int u = 0; u < kNarrowU; ++u) {
      const int64_t k = k0 + (int64_t)u * 1024;
      c[u] = k < nnz ? ci[k] : -1;
    }
#pragma unroll
    for (int u = 0; u < kNarrowU; ++u)
      if (c[u] >= 0) atomicAdd(&h[c[u]], 1);
  }
  __syncthreads();
  const int v = t < m ? h[t] : 0;
  atomicMax(&hmax, v);
  int inc = v;
  for (int o = 1; o < kWave; o <<= 1) {
    const int u = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += u;
  }
  if (lane == kWave - 1) wsum[w] = inc;
  __syncthreads();
  int before = 0;
  for (int q = 0; q < w; ++q) before += wsum[q];
  if (t < m) trp[t] = before + inc - v;
  if (t == m - 1) trp[m] = before + inc;
  if (t == 0) *rmax = hmax;
}

// rowid[k] = the row of entry k.
__global__ void k_row_ids(int n, const int* __restrict__ rp, int* __restrict__ rowid) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n)
    for (int k = rp[i]; k < rp[i + 1]; ++k) rowid[k] = i;
}

// Row J = blockIdx.x of T: wave w of the workgroup takes the w-th run of A's
// entries in storage order, counts those in column J (ballots), and after
// the counts of the earlier runs writes them in order.  Storage order is
// ascending row, so T's rows come out sorted.
__global__ void __launch_bounds__(1024) k_narrow_fill(int64_t nnz, const int* __restrict__ ci,
                                                      const double* __restrict__ v,
                                                      const int* __restrict__ rowid,
                                                      const int* __restrict__ trp,
                                                      int* __restrict__ tci,
                                                      double* __restrict__ tv) {
  __shared__ int wcnt[1024 / kWave];
  const int J = blockIdx.x;
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  constexpr int nw = 1024 / kWave, step = kWave * kNarrowU;
  const int64_t chunk = (nnz + nw - 1) / nw;
  const int64_t k0 = min(nnz, (int64_t)w * chunk), k1 = min(nnz, k0 + chunk);
  const unsigned long long below = (1ull << lane) - 1ull;
  int c = 0;
  for (int64_t base = k0; base < k1; base += step) {
    bool hit[kNarrowU];
#pragma unroll
    for (int u = 0; u < kNarrowU; ++u) {
      const int64_t k = base + (int64_t)u * kWave + lane;
      hit[u] = k < k1 && ci[k] == J;
    }
#pragma unroll
    for (int u = 0; u < kNarrowU; ++u) c += __popcll(__ballot(hit[u]));
  }
  if (lane == 0) wcnt[w] = c;
  __syncthreads();
  int pos = trp[J];
  for (int q = 0; q < w; ++q) pos += wcnt[q];
  for (int64_t base = k0; base < k1; base += step) {
    bool hit[kNarrowU];
#pragma unroll
    for (int u = 0; u < kNarrowU; ++u) {
      const int64_t k = base + (int64_t)u * kWave + lane;
      hit[u] = k < k1 && ci[k] == J;
    }
#pragma unroll
    for (int u = 0; u < kNarrowU; ++u) {
      const unsigned long long mask = __ballot(hit[u]);
      if (hit[u]) {
        const int64_t k = base + (int64_t)u * kWave + lane;
        const int p = pos + __popcll(mask & below);
        tci[p] = rowid[k];
        tv[p] = v[k];
      }
      pos += __popcll(mask);
    }
  }
}

// The lanes of a wavefront holding the same key among those with `valid`
// set: the caller's group as a lane mask (its own lane included), 0 for a
// lane that is not valid.  Every lane of the wavefront calls it together.
__device__ __forceinline__ unsigned long long wave_key_group(int key, bool valid) {
  unsigned long long todo = __ballot(valid);
  unsigned long long grp = 0;
  while (todo) {
    const int k = __shfl(key, __ffsll((long long)todo) - 1, kWave);
    const bool same = valid && key == k;
    const unsigned long long m = __ballot(same);
    if (same) grp = m;
    todo &= ~m;
  }
  return grp;
}

// Column counts of a CSR.  Consecutive entries belong to neighbouring rows
// and share columns, so the lanes of a wavefront with one column add their
// number with one atomic (the device-scope atomics, not the loads, bound
// the plain one-atomic-per-entry pass).
__global__ void k_col_count(int64_t nnz, const int* __restrict__ ci, int* __restrict__ cnt) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int lane = threadIdx.x % kWave;
  const bool valid = k < nnz;
  const int c = valid ? ci[k] : -1;
  const unsigned long long grp = wave_key_group(c, valid);
  if (valid && (grp & ((1ull << lane) - 1ull)) == 0) atomicAdd(&cnt[c], __popcll(grp));
}

// Each entry (i, c) of row i takes a free slot of row c of the transpose
// (the order within a row is fixed afterwards by k_rank_rows).  Entry u of
// every row of a wavefront is placed together: lanes with the same column
// take consecutive slots from one atomic of their lowest lane.
__global__ void k_transpose_fill(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                 const double* __restrict__ v, int* __restrict__ cursor,
                                 int* __restrict__ tci, double* __restrict__ tv) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int lane = threadIdx.x % kWave;
  const unsigned long long below = (1ull << lane) - 1ull;
  int k0 = 0, k1 = 0;
  if (i < n) {
    k0 = rp[i];
    k1 = rp[i + 1];
  }
  for (int u = 0; __ballot(k0 + u < k1) != 0; ++u) {
    const bool valid = k0 + u < k1;
    const int c = valid ? ci[k0 + u] : -1;
    const double w = valid ? v[k0 + u] : 0.0;
    const unsigned long long grp = wave_key_group(c, valid);
    int base = 0;
    if (valid && (grp & below) == 0) base = atomicAdd(&cursor[c], __popcll(grp));
    base = __shfl(base, valid ? __ffsll((long long)grp) - 1 : lane, kWave);
    if (valid) {
      const int p = base + __popcll(grp & below);
      tci[p] = i;
      tv[p] = w;
    }
  }
}

// Sort every row of an unsorted CSR by column into (ci, v): one 64-lane
// workgroup per row; each entry's destination is the number of smaller keys
// in its row (keys are distinct within a row).  Rows up to kRankStage
// entries are compared from LDS.  (Four rows per workgroup was slower: the
// barrier waits for the block's longest row.)
constexpr int kRankStage = 2048;
__global__ void __launch_bounds__(kWave) k_rank_rows(const int* __restrict__ rp,
                                                     const int* __restrict__ uci,
                                                     const double* __restrict__ uv,
                                                     int* __restrict__ ci, double* __restrict__ v) {
  __shared__ int sk[kRankStage];
  const int i = blockIdx.x;
  const int b = rp[i], e = rp[i + 1], len = e - b;
  const bool staged = len <= kRankStage;
  if (staged)
    for (int p = threadIdx.x; p < len; p += kWave) sk[p] = uci[b + p];
  __syncthreads();
  for (int p = threadIdx.x; p < len; p += kWave) {
    const int key = staged ? sk[p] : uci[b + p];
    int rank = 0;
    if (staged)
      for (int q = 0; q < len; ++q) rank += sk[q] < key ? 1 : 0;
    else
      for (int q = b; q < e; ++q) rank += uci[q] < key ? 1 : 0;
    ci[b + rank] = key;
    v[b + rank] = uv[b + p];
  }
}

// ------------------------------------------------------------------ dense coarsest
// Explicit inverse of the SPD coarsest matrix by Gauss-Jordan elimination
// without pivoting (pivots of an SPD matrix are positive): at step k the
// pivot row is divided by the pivot with a_kk replaced by 1, and every other
// row i gets a_ij -= f_i a_kj with a_ik replaced by 0 (f the pivot column),
// which leaves A^-1 in place of A.  Up to kDenseBlk rows one workgroup does
// it from the n x 2n row-major array G = [A | I] (k_dense_inverse_blk);
// larger levels take the blocked form over many workgroups (k_ginv_*).
constexpr int kDenseBlk = 128;

// The elimination for n <= 128 by 4 x 4 blocks: thread t owns the block
// of rows 4 (t / 32) .. +3 and columns 4 (t mod 32) .. +3 of the 128 x 128
// cover, padded with the identity past n (the padding stays decoupled).
// Block step K (pivots 4K .. 4K+3) is the block form of the steps above: with
// D = A_KK, C_I = A_IK and R_J = A_KJ,
//   A_KK <- D^-1,  A_KJ <- D^-1 R_J,  A_IK <- -C_I D^-1,
//   A_IJ <- A_IJ - C_I (D^-1 R_J).
// The owner of A_KK inverts it in registers by the scalar steps (its four
// pivots are the elimination's pivots 4K .. 4K+3, each checked > 0).  D^-1,
// the old block column and the new block row pass through LDS,
// double-buffered, so a block step takes two barriers instead of the four
// of four scalar steps.
__global__ void __launch_bounds__(1024) k_dense_inverse_blk(int n, const double* __restrict__ Gm,
                                                            double* __restrict__ Ainv,
                                                            int* __restrict__ flag) {
  constexpr int B = 4;
  __shared__ double dinv[2][B][B];
  __shared__ double cpan[2][32 * B][B];
  __shared__ double rpan[2][B][32 * B];
  const int t = threadIdx.x;
  const int I = t / 32, J = t % 32, i0 = I * B, j0 = J * B;
  double a[B][B];
#pragma unroll
  for (int r = 0; r < B; ++r)
#pragma unroll
    for (int c = 0; c < B; ++c) {
      const int i = i0 + r, j = j0 + c;
      a[r][c] = (i < n && j < n) ? Gm[(size_t)i * 2 * n + j] : (i == j ? 1.0 : 0.0);
    }
  const int nb = (n + B - 1) / B;
  for (int K = 0; K < nb; ++K) {
    const int bf = K & 1;
    if (I == K && J == K) {
#pragma unroll
      for (int k = 0; k < B; ++k) {
        double piv = a[k][k];
        if (!(piv > 0.0)) {
          atomicOr(flag, SE_DENSE);
          piv = 1.0;
        }
        const double inv = 1.0 / piv;
        double rk[B];
#pragma unroll
        for (int c = 0; c < B; ++c) rk[c] = (c == k ? 1.0 : a[k][c]) * inv;
#pragma unroll
        for (int r = 0; r < B; ++r) {
          if (r == k) continue;
          const double f = a[r][k];
#pragma unroll
          for (int c = 0; c < B; ++c) a[r][c] = (c == k ? 0.0 : a[r][c]) - f * rk[c];
        }
#pragma unroll
        for (int c = 0; c < B; ++c) a[k][c] = rk[c];
      }
#pragma unroll
      for (int r = 0; r < B; ++r)
#pragma unroll
        for (int c = 0; c < B; ++c) dinv[bf][r][c] = a[r][c];
    }
    if (J == K && I != K) {
#pragma unroll
      for (int r = 0; r < B; ++r)
#pragma unroll
        for (int c = 0; c < B; ++c) cpan[bf][i0 + r][c] = a[r][c];
    }
    __syncthreads();
    if (I == K && J != K) {  // the block row: D^-1 R_J
      double nr[B][B];
#pragma unroll
      for (int r = 0; r < B; ++r)
#pragma unroll
        for (int c = 0; c < B; ++c) {
          double s = 0.0;
#pragma unroll
          for (int m = 0; m < B; ++m) s = fma(dinv[bf][r][m], a[m][c], s);
          nr[r][c] = s;
        }
#pragma unroll
      for (int r = 0; r < B; ++r)
#pragma unroll
        for (int c = 0; c < B; ++c) {
          a[r][c] = nr[r][c];
          rpan[bf][r][j0 + c] = nr[r][c];
        }
    }
    __syncthreads();
    if (I != K) {
      double f[B][B];
#pragma unroll
      for (int r = 0; r < B; ++r)
#pragma unroll
        for (int m = 0; m < B; ++m) f[r][m] = cpan[bf][i0 + r][m];
      if (J == K) {  // the block column: -C_I D^-1
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
          for (int c = 0; c < B; ++c) {
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < B; ++m) s = fma(f[r][m], dinv[bf][m][c], s);
            a[r][c] = -s;
          }
      } else {
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
          for (int c = 0; c < B; ++c) {
            double s = a[r][c];
#pragma unroll
            for (int m = 0; m < B; ++m) s = fma(-f[r][m], rpan[bf][m][j0 + c], s);
            a[r][c] = s;
          }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < B; ++r)
#pragma unroll
    for (int c = 0; c < B; ++c)
      if (i0 + r < n && j0 + c < n) Ainv[(size_t)(i0 + r) * n + j0 + c] = a[r][c];
}

// ---- blocked Gauss-Jordan over several workgroups (coarsest levels of 257
// to 1024 rows).  The SPD matrix is padded with the identity to N = 32 nb
// rows and eliminated by 32 x 32 blocks: at block step K the diagonal block
// D = G[K][K] is inverted by the scalar steps (its 32 pivots are the
// elimination's pivots 32K .. 32K+31, each checked > 0), then every block is
// rewritten from the old matrix into the other buffer:
//   G'[K][K] = D^-1,  G'[K][J] = D^-1 G[K][J],  G'[I][K] = -G[I][K] D^-1,
//   G'[I][J] = G[I][J] - G[I][K] (D^-1 G[K][J]).
// Reading only the old matrix, the blocks need no ordering among themselves.

// D^-1 of block K of the N x N row-major G into Dinv (32 x 32): one 1024-thread
// workgroup, one entry per thread, two barriers per scalar step.
__global__ void __launch_bounds__(1024) k_ginv_diag(int N, const double* __restrict__ G, int K,
                                                    double* __restrict__ Dinv,
                                                    int* __restrict__ flag) {
  __shared__ double D[32][33];
  __shared__ double rowk[32], colk[32];
  const int r = threadIdx.x / 32, c = threadIdx.x % 32;
  D[r][c] = G[(size_t)(K * 32 + r) * N + K * 32 + c];
  __syncthreads();
  for (int k = 0; k < 32; ++k) {
    double p = D[k][k];
    if (!(p > 0.0)) {
      if (threadIdx.x == 0) atomicOr(flag, SE_DENSE);
      p = 1.0;
    }
    if (r == 0) {
      rowk[c] = (c == k ? 1.0 : D[k][c]) / p;
      colk[c] = D[c][k];
    }
    __syncthreads();
    if (r == k)
      D[r][c] = rowk[c];
    else
      D[r][c] = c == k ? -colk[r] / p : D[r][c] - colk[r] * rowk[c];
    __syncthreads();
  }
  Dinv[r * 32 + c] = D[r][c];
}

// One block step over all blocks: workgroup (J, I) writes block (I, J) of Gn.
__global__ void __launch_bounds__(1024) k_ginv_update(int N, const double* __restrict__ G,
                                                      const double* __restrict__ Dinv, int K,
                                                      double* __restrict__ Gn) {
  __shared__ double Ds[32][33], Rs[32][33], Cs[32][33], Ts[32][33];
  const int I = blockIdx.y, J = blockIdx.x;
  const int r = threadIdx.x / 32, c = threadIdx.x % 32;
  const size_t row = (size_t)I * 32 + r, col = (size_t)J * 32 + c;
  if (I == K && J == K) {
    Gn[row * N + col] = Dinv[r * 32 + c];
    return;
  }
  Ds[r][c] = Dinv[r * 32 + c];
  if (J != K) Rs[r][c] = G[((size_t)K * 32 + r) * N + col];
  if (I != K) Cs[r][c] = G[row * N + (size_t)K * 32 + c];
  __syncthreads();
  if (I == K) {
    double t = 0.0;
    for (int k = 0; k < 32; ++k) t = t + Ds[r][k] * Rs[k][c];
    Gn[row * N + col] = t;
    return;
  }
  if (J == K) {
    double t = 0.0;
    for (int k = 0; k < 32; ++k) t = t + Cs[r][k] * Ds[k][c];
    Gn[row * N + col] = -t;
    return;
  }
  double t = 0.0;
  for (int k = 0; k < 32; ++k) t = t + Ds[r][k] * Rs[k][c];
  Ts[r][c] = t;
  __syncthreads();
  double u = 0.0;
  for (int k = 0; k < 32; ++k) u = u + Cs[r][k] * Ts[k][c];
  Gn[row * N + col] = G[row * N + col] - u;
}

// G = A padded with the identity to N x N (row-major, zeroed before): one
// wavefront per row.
__global__ void k_densify_sq(int n, int N, const int* __restrict__ rp, const int* __restrict__ ci,
                             const double* __restrict__ v, double* __restrict__ G) {
  const int i = (blockIdx.x * kBlock + threadIdx.x) / kWave, lane = threadIdx.x % kWave;
  if (i >= N) return;
  if (i >= n) {
    if (lane == 0) G[(size_t)i * N + i] = 1.0;
    return;
  }
  for (int k = rp[i] + lane; k < rp[i + 1]; k += kWave) G[(size_t)i * N + ci[k]] = v[k];
}

// Ainv (n x n) = the leading block of the N x N G.
__global__ void k_lead_block(int n, int N, const double* __restrict__ G,
                             double* __restrict__ Ainv) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= (int64_t)n * n) return;
  const int i = (int)(p / n), j = (int)(p % n);
  Ainv[p] = G[(size_t)i * N + j];
}

// G = [A | I] (n x 2n, row-major, zeroed before): one wavefront per row.
__global__ void k_densify(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                          const double* __restrict__ v, double* __restrict__ G) {
  const int i = (blockIdx.x * kBlock + threadIdx.x) / kWave, lane = threadIdx.x % kWave;
  if (i >= n) return;
  for (int k = rp[i] + lane; k < rp[i + 1]; k += kWave) G[(size_t)i * 2 * n + ci[k]] = v[k];
  if (lane == 0) G[(size_t)i * 2 * n + n + i] = 1.0;
}

// ------------------------------------------------------------------ host helpers
// Launch a lane-grouped row kernel K<LPR> over `rows` rows.
#define PPE_ROWS(LPR_, K, rows, ...)                                                         \
  do {                                                                                       \
    const int lpr_ = (LPR_);                                                                 \
    const int g_ = grid_for((int64_t)(rows) * lpr_);                                         \
    switch (lpr_) {                                                                          \
      case 1: hipLaunchKernelGGL(K<1>, dim3(g_), dim3(kBlock), 0, s->stream, __VA_ARGS__); break;   \
      case 2: hipLaunchKernelGGL(K<2>, dim3(g_), dim3(kBlock), 0, s->stream, __VA_ARGS__); break;   \
      case 4: hipLaunchKernelGGL(K<4>, dim3(g_), dim3(kBlock), 0, s->stream, __VA_ARGS__); break;   \
      case 8: hipLaunchKernelGGL(K<8>, dim3(g_), dim3(kBlock), 0, s->stream, __VA_ARGS__); break;   \
      case 16: hipLaunchKernelGGL(K<16>, dim3(g_), dim3(kBlock), 0, s->stream, __VA_ARGS__); break; \
      case 32: hipLaunchKernelGGL(K<32>, dim3(g_), dim3(kBlock), 0, s->stream, __VA_ARGS__); break; \
      default: hipLaunchKernelGGL(K<64>, dim3(g_), dim3(kBlock), 0, s->stream, __VA_ARGS__); break; \
    }                                                                                        \
    PPE_LAUNCH_CHECK();                                                                      \
  } while (0)
// Lanes per row of the aggregation kernels (strength, the MIS-2 rounds and
// the two joining passes): the power of two from 1 to 64 nearest to half the
// mean row length.  Their results are maxima and per-entry tests, so they do
// not depend on it.
static int agg_lanes(const Csr& A) {
  const double target = (A.n ? (double)A.nnz / A.n : 1.0) / 2.0;
  int best = 1;
  for (int c = 2; c <= 64; c *= 2)
    if (std::fabs(std::log2(c / target)) < std::fabs(std::log2(best / target))) best = c;
  return best;
}

// Launch configuration of k_spgemm_rows for one product.
struct SpConfig {
  int lpr, W, H, rpb, threads;
  size_t lds;
};

static size_t spgemm_lds(int mode, int rpb, int W, int H, int per_row) {
  const size_t r = (size_t)rpb, h = (size_t)H;
  if (mode == SP_COUNT || mode == SP_BITS) return r * h * 4 + r * 4;
  if (mode == SP_FILL) return r * W * h * 8 + 2 * r * h * 4 + r * 4;
  return r * W * h * 8 + r * h * 4 + r * (per_row / kWave + 1) * 4;
}

// Lanes per sub-group from the mean row length of B; sub-groups per row so
// that each walks about eight entries of A; rows per block to fill 256
// threads.  W is halved until the block's LDS fits.
static SpConfig spgemm_config(ppe_solver* s, const Csr& A, const Csr& B, int mode, int H) {
  SpConfig c{};
  c.lpr = lanes_for(B);
  const double mean_a = A.n ? (double)A.nnz / A.n : 1.0;
  c.W = 1;
  while (c.W * c.lpr < 1024 && c.W < 16 && c.W * 8 < mean_a) c.W *= 2;
  c.H = H;
  while (true) {
    const int per_row = c.lpr * c.W;
    c.rpb = per_row >= kBlock ? 1 : kBlock / per_row;
    c.threads = c.rpb * per_row;
    c.lds = spgemm_lds(mode, c.rpb, c.W, H, per_row);
    if (c.lds <= s->lds_max || (c.W == 1 && c.rpb == 1)) break;
    if (c.W > 1) c.W /= 2;
    else c.lpr *= 2;  // fewer rows per block
  }
  require(c.lds <= s->lds_max, PPE_ERR_INTERNAL, "sparse product row does not fit in LDS");
  return c;
}

template <int MODE>
static void spgemm_launch(ppe_solver* s, const SpConfig& c, const Csr& A, const Csr& B,
                          const int* off, int* counts, int* cci, double* cv, int* flag) {
  const int g = (A.n + c.rpb - 1) / c.rpb;
  const bool numeric = MODE == SP_FILL || MODE == SP_DENSE;
  const double* av = numeric ? A.v() : nullptr;
  const double* bv = numeric ? B.v() : nullptr;
#define PPE_SPR(L_)                                                                            \
  hipLaunchKernelGGL((k_spgemm_rows<L_, MODE>), dim3(g), dim3(c.threads), c.lds, s->stream, A.n, \
                     c.W, c.H, A.rp(), A.ci(), av, B.rp(), B.ci(), bv, off, counts, cci, cv, flag)
  switch (c.lpr) {
    case 4: PPE_SPR(4); break;
    case 8: PPE_SPR(8); break;
    case 16: PPE_SPR(16); break;
    case 32: PPE_SPR(32); break;
    default: PPE_SPR(64); break;
  }
#undef PPE_SPR
  PPE_LAUNCH_CHECK();
}

// C = A B.  Narrow products (C at most kSpDenseWidth columns, rows expected
// to fill a quarter of them) take one pass with a slot per column into
// fixed-stride scratch rows and a compaction;
// wider ones count each row's distinct columns with a hash sized from the
// product bound (or a bit per column of C when that is smaller), then fill
// C with a hash sized from the largest count.  The
// product bound is maxrow(A) maxrow(B) when both are known on the host, else
// a bound pass reads it back.  C.maxrow is set to C's longest row.  extra: a
// device int read back in the same round trip as C's size (extra_host).
void spgemm(ppe_solver* s, const Csr& A, const Csr& B, Csr& C, const int* extra,
            int* extra_host) {
  require(A.m == B.n, PPE_ERR_INTERNAL, "spgemm shape mismatch");
  C.n = A.n;
  C.m = B.m;
  int* crp = C.rowptr.get<int>(C.n + 1);
  if (C.n == 0) {
    C.nnz = 0;
    fill_int(s, crp, 0, 1);
    return;
  }
  int* flag = s->flag.get<int>(4);
  int* counts = s->sp_cnt.get<int>(C.n + 1);
  long long total = 0;
  int fm[2] = {0, 0};
  // flag[1] starts at 0 (zeroed below): counts are >= 0, so the max needs
  // no fill of its own unless a bound pass used the slot before
  bool max_slot_used = false;
  auto fetch_scan = [&](bool with_max) {
    // a bound pass that used the max slot leaves a larger value there
    if (with_max && max_slot_used) fill_int(s, flag + 1, INT32_MIN, 1);
    const long long* dtotal =
        exclusive_scan_async(s, counts, crp, C.n, 0, with_max ? flag + 1 : nullptr);
    if (extra)
      read_back(s, {ReadItem{dtotal, sizeof(long long), &total},
                    ReadItem{flag, sizeof(int) * 2, fm}, ReadItem{extra, sizeof(int), extra_host}});
    else
      read_back(s, {ReadItem{dtotal, sizeof(long long), &total},
                    ReadItem{flag, sizeof(int) * 2, fm}});
    require(fm[0] == 0, PPE_ERR_INTERNAL, "sparse product row overflowed its hash table");
    require(total <= INT32_MAX, PPE_ERR_INTERNAL, "sparse product too large for int32 indices");
    C.nnz = total;
    C.maxrow = fm[1];
  };
  fill_int(s, flag, 0, 2);

  const double mean_a = (double)A.nnz / A.n, mean_b = B.n ? (double)B.nnz / B.n : 0.0;
  if (C.m <= kSpDenseWidth && 4.0 * mean_a * mean_b >= C.m) {
    int H = 64;
    while (H < C.m) H += 64;
    const SpConfig c = spgemm_config(s, A, B, SP_DENSE, H);
    const size_t cap = (size_t)C.n * C.m;
    require(cap <= INT32_MAX, PPE_ERR_INTERNAL, "sparse product scratch too large");
    int* off = s->sp_off.get<int>(C.n + 1);
    hipLaunchKernelGGL(k_stride_offsets, dim3(grid_for(C.n + 1)), dim3(kBlock), 0, s->stream,
                       C.n + 1, C.m, off);
    PPE_LAUNCH_CHECK();
    int* sci = s->sp_ci.get<int>(cap);
    double* sv = s->sp_v.get<double>(cap);
    spgemm_launch<SP_DENSE>(s, c, A, B, off, counts, sci, sv, flag);
    fetch_scan(true);
    int* cci = C.col.get<int>(C.nnz);
    double* cv = C.val.get<double>(C.nnz);
    PPE_ROWS(lanes_for(B), k_spgemm_compact, C.n, C.n, off, crp, sci, sv, cci, cv);
    return;
  }

  int ub;
  if (A.maxrow > 0 && B.maxrow > 0) {
    ub = (int)std::min<int64_t>((int64_t)A.maxrow * B.maxrow, C.m);
  } else {
    int* prod = s->sp_prod.get<int>(C.n + 1);
    PPE_ROWS(lanes_for(A), k_spgemm_bound, C.n, C.n, A.rp(), A.ci(), B.rp(), prod);
    max_int_async(s, prod, C.n, flag + 1, false);
    max_slot_used = true;
    read_back(s, {ReadItem{flag, sizeof(int) * 2, fm}});
    ub = std::min(fm[1], C.m);
  }
  int Hc = 32;
  while (Hc < 2 * ub && Hc < 8192) Hc *= 2;
  // count with a bit per column of C when that takes less LDS than the hash
  const int words = (C.m + 31) / 32;
  if (words < Hc) {
    const SpConfig cb = spgemm_config(s, A, B, SP_BITS, words);
    spgemm_launch<SP_BITS>(s, cb, A, B, nullptr, counts, nullptr, nullptr, flag);
  } else {
    const SpConfig cc = spgemm_config(s, A, B, SP_COUNT, Hc);
    spgemm_launch<SP_COUNT>(s, cc, A, B, nullptr, counts, nullptr, nullptr, flag);
  }
  fetch_scan(true);
  int H = 16;  // at least twice the longest row: list and ckey hold H / 2
  while (H < 2 * fm[1]) H *= 2;
  const SpConfig cf = spgemm_config(s, A, B, SP_FILL, H);
  int* cci = C.col.get<int>(C.nnz);
  double* cv = C.val.get<double>(C.nnz);
  spgemm_launch<SP_FILL>(s, cf, A, B, crp, nullptr, cci, cv, flag);
}

// T = A^T with sorted rows; *s->rmax receives T's longest row (device int).
void transpose(ppe_solver* s, const Csr& A, Csr& T) {
  T.n = A.m;
  T.m = A.n;
  T.nnz = A.nnz;
  T.maxrow = 0;
  if (T.n > 0 && T.n <= kNarrowCols && A.nnz > 0) {
    int* trp = T.rowptr.get<int>(T.n + 1);
    hipLaunchKernelGGL(k_narrow_count, dim3(1), dim3(1024), 0, s->stream, A.nnz, T.n, A.ci(), trp,
                       s->rmax.get<int>(1));
    PPE_LAUNCH_CHECK();
    int* rowid = s->tmp_i[2].get<int>(A.nnz);
    hipLaunchKernelGGL(k_row_ids, dim3(grid_for(A.n)), dim3(kBlock), 0, s->stream, A.n, A.rp(),
                       rowid);
    PPE_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_narrow_fill, dim3(T.n), dim3(1024), 0, s->stream, A.nnz, A.ci(), A.v(),
                       rowid, trp, T.col.get<int>(T.nnz), T.val.get<double>(T.nnz));
    PPE_LAUNCH_CHECK();
    return;
  }
  int* cnt = s->tmp_i[0].get<int>(T.n + 1);
  fill_int(s, cnt, 0, T.n + 1);
  if (A.nnz) {
    hipLaunchKernelGGL(k_col_count, dim3(grid_for(A.nnz)), dim3(kBlock), 0, s->stream, A.nnz, A.ci(),
                       cnt);
    PPE_LAUNCH_CHECK();
  }
  int* trp = T.rowptr.get<int>(T.n + 1);
  int* rmax = s->rmax.get<int>(1);
  fill_int(s, rmax, INT32_MIN, 1);
  exclusive_scan_async(s, cnt, trp, T.n, 0, rmax);  // the total is A.nnz
  int* cursor = s->tmp_i[1].get<int>(T.n + 1);
  PPE_HIP(hipMemcpyAsync(cursor, trp, sizeof(int) * (T.n + 1), hipMemcpyDeviceToDevice, s->stream));
  int* tci = T.col.get<int>(T.nnz);
  double* tv = T.val.get<double>(T.nnz);
  int* uci = s->tmp_i[2].get<int>(T.nnz);
  double* uv = s->tmp_d[1].get<double>(T.nnz);
  if (A.n) {
    hipLaunchKernelGGL(k_transpose_fill, dim3(grid_for(A.n)), dim3(kBlock), 0, s->stream, A.n, A.rp(),
                       A.ci(), A.v(), cursor, uci, uv);
    PPE_LAUNCH_CHECK();
  }
  if (T.n) {
    hipLaunchKernelGGL(k_rank_rows, dim3(T.n), dim3(kWave), 0, s->stream, trp, uci, uv, tci, tv);
    PPE_LAUNCH_CHECK();
  }
}

// The level's spectral bound of D^-1 A into *rho_dev (read back with the
// rest of the setup results): Gershgorin on the finest level, the safety
// factor times a power estimate on coarse ones.
void spectral_bound(ppe_solver* s, Level& L, int lvl, double* rho_dev) {
  const int n = L.n;
  if (n == 0) {
    fill_double(s, rho_dev, 1.0, 1);
    return;
  }
  if (lvl == 0) {
    const int g = grid_for(n);
    double* part = s->tmp_d[0].get<double>(g);
    hipLaunchKernelGGL(k_gershgorin, dim3(g), dim3(kBlock), 0, s->stream, n, L.A.rp(), L.A.v(),
                       L.diag.as<double>(), part);
    PPE_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_max_partials, dim3(1), dim3(kBlock), 0, s->stream, part, g, rho_dev);
    PPE_LAUNCH_CHECK();
    return;
  }
  L.x.get<double>(n);
  L.r.get<double>(n);
  // setup work: its power steps stay out of the solve's kernel profile
  struct NoProfile {
    ppe_solver* s;
    bool saved;
    ~NoProfile() { s->prof = saved; }
  } guard{s, s->prof};
  s->prof = false;
  power_estimate(s, L, level_salt(lvl), kPowerIters, kPowerSafety, rho_dev);
}

// Launches inside the scope go to another stream of the solver.
struct OnStream {
  ppe_solver* s;
  hipStream_t saved;
  OnStream(ppe_solver* s_, hipStream_t st) : s(s_), saved(s_->stream) { s->stream = st; }
  ~OnStream() { s->stream = saved; }
};

void ensure_side_stream(ppe_solver* s) {
  if (s->side) return;
  PPE_HIP(hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking));
  PPE_HIP(hipEventCreateWithFlags(&s->fork_ev, hipEventDisableTiming));
  PPE_HIP(hipEventCreateWithFlags(&s->join_ev, hipEventDisableTiming));
}

}  // namespace

// ---- coarse levels kept across a changed mask
namespace {

// Row i of the re-indexed finest prolongator: the base build's row of the
// same cell, or empty for a pin or a cell that build did not have.  cnt[i]
// is its length; matched[i] = 1 if the cell had a row in the base build.
__global__ void k_reuse_rows(int na, const int* __restrict__ perm, const int* __restrict__ comp,
                             const int* __restrict__ base_cid, const int* __restrict__ base_rp,
                             int* __restrict__ cnt, int* __restrict__ matched) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= na) return;
  const int c = perm[i];
  const int o = base_cid[c];
  cnt[i] = (o >= 0 && comp[c] != c) ? base_rp[o + 1] - base_rp[o] : 0;
  matched[i] = o >= 0 ? 1 : 0;
}

__global__ void k_reuse_fill(int na, const int* __restrict__ perm, const int* __restrict__ comp,
                             const int* __restrict__ base_cid, const int* __restrict__ base_rp,
                             const int* __restrict__ base_ci, const double* __restrict__ base_v,
                             const int* __restrict__ rp, int* __restrict__ ci,
                             double* __restrict__ v) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= na) return;
  const int c = perm[i];
  const int o = base_cid[c];
  if (o < 0 || comp[c] == c) return;
  const int src = base_rp[o], len = base_rp[o + 1] - src, dst = rp[i];
  for (int k = 0; k < len; ++k) {
    ci[dst + k] = base_ci[src + k];
    v[dst + k] = base_v[src + k];
  }
}

}  // namespace

void keep_base(ppe_solver* s) {
  s->have_base = false;
  if (s->opt.coarse_reuse <= 0 || s->shifted || s->nlev < 2) return;
  const int nc = s->n_cells;
  const Csr& P = s->levels[0].P;
  Csr& B = s->base_P0;
  B.n = P.n;
  B.m = P.m;
  B.nnz = P.nnz;
  B.maxrow = P.maxrow;
  PPE_HIP(hipMemcpyAsync(s->base_cid.get<int>(nc + 1), s->cid.as<int>(), sizeof(int) * (nc + 1),
                         hipMemcpyDeviceToDevice, s->stream));
  PPE_HIP(hipMemcpyAsync(B.rowptr.get<int>(P.n + 1), P.rp(), sizeof(int) * (P.n + 1),
                         hipMemcpyDeviceToDevice, s->stream));
  if (P.nnz) {
    PPE_HIP(hipMemcpyAsync(B.col.get<int>(P.nnz), P.ci(), sizeof(int) * P.nnz,
                           hipMemcpyDeviceToDevice, s->stream));
    PPE_HIP(hipMemcpyAsync(B.val.get<double>(P.nnz), P.v(), sizeof(double) * P.nnz,
                           hipMemcpyDeviceToDevice, s->stream));
  }
  s->base_na = s->n_active;
  s->base_nlev = s->nlev;
  s->base_uses = 0;
  s->have_base = true;
}

bool reuse_coarse_levels(ppe_solver* s) {
  if (!s->have_base || s->shifted || s->base_uses >= s->opt.coarse_reuse) return false;
  const int na = s->n_active;
  if (na == 0) return false;
  Level& L0 = s->levels[0];
  const Csr& B = s->base_P0;
  const int* perm = s->perm.as<int>();
  const int* comp = s->comp_full.as<int>();
  const int* bcid = s->base_cid.as<int>();
  int* cnt = s->tmp_i[0].get<int>(na + 1);
  int* matched = s->tmp_i[1].get<int>(na + 1);
  hipLaunchKernelGGL(k_reuse_rows, dim3(grid_for(na)), dim3(kBlock), 0, s->stream, na, perm, comp,
                     bcid, B.rp(), cnt, matched);
  PPE_LAUNCH_CHECK();
  int* rp = L0.P.rowptr.get<int>(na + 1);
  const long long* d_nnz = exclusive_scan_async(s, cnt, rp, na, 0);
  const long long* d_matched = exclusive_scan_async(s, matched, s->tmp_i[2].get<int>(na + 1), na, 1);
  const double* d_rho = level0_bound_async(s);
  long long nnz = 0, kept = 0;
  double rho = 0.0;
  read_back(s, {ReadItem{d_nnz, sizeof(long long), &nnz},
                ReadItem{d_matched, sizeof(long long), &kept},
                ReadItem{d_rho, sizeof(double), &rho}});
  // cells removed since the base build plus cells it did not have
  const long long moved = (s->base_na - kept) + (na - kept);
  if (10 * moved > (long long)s->base_na) return false;
  Csr& P = L0.P;
  P.n = na;
  P.m = B.m;
  P.nnz = nnz;
  P.maxrow = B.maxrow;
  hipLaunchKernelGGL(k_reuse_fill, dim3(grid_for(na)), dim3(kBlock), 0, s->stream, na, perm, comp,
                     bcid, B.rp(), B.ci(), B.v(), rp, P.col.get<int>(nnz > 0 ? nnz : 1),
                     P.val.get<double>(nnz > 0 ? nnz : 1));
  PPE_LAUNCH_CHECK();
  transpose(s, P, L0.R);
  L0.n_agg = B.m;
  L0.rho = rho;
  L0.ap_ok = false;
  L0.dense = false;
  s->nlev = s->base_nlev;
  s->base_uses += 1;
  return true;
}

const double* level0_bound_async(ppe_solver* s) {
  double* out = s->setup_out.get<double>((size_t)std::max(1, s->opt.max_levels) + 1);
  spectral_bound(s, s->levels[0], 0, out);
  return out;
}

// Q = A P_tent on the finest level from its ELL copy (k_coarsen_cols_ell):
// count, scan with the longest row (one round trip), fill.  Q is what the
// general product gives, entry for entry.
static void coarsen_cols_ell(ppe_solver* s, const Level& L, const int* agg, const double* pt,
                             int na, Csr& Q) {
  const int n = L.n, W = L.W;
  Q.n = n;
  Q.m = na;
  int* qrp = Q.rowptr.get<int>(n + 1);
  int* counts = s->sp_cnt.get<int>(n + 1);
  int* flag = s->flag.get<int>(4);
  fill_int(s, flag, 0, 2);
  const int g = grid_for(n);
  const int* ecol = L.ell_col.as<int>();
  const double* ev = L.ell_val.as<double>();
  const double* dg = L.diag.as<double>();
#define PPE_QC(WM, COUNT, ...)                                                                 \
  hipLaunchKernelGGL((k_coarsen_cols_ell<WM, COUNT>), dim3(g), dim3(kBlock), 0, s->stream, n, W, \
                     ecol, ev, dg, agg, pt, __VA_ARGS__)
  if (W <= 4) PPE_QC(4, true, counts, nullptr, nullptr, nullptr);
  else if (W <= 6) PPE_QC(6, true, counts, nullptr, nullptr, nullptr);
  else PPE_QC(8, true, counts, nullptr, nullptr, nullptr);
  PPE_LAUNCH_CHECK();
  const long long* dtotal = exclusive_scan_async(s, counts, qrp, n, 0, flag + 1);
  long long total = 0;
  int fm[2] = {0, 0};
  read_back(s, {ReadItem{dtotal, sizeof(long long), &total}, ReadItem{flag, sizeof(int) * 2, fm}});
  require(total <= INT32_MAX, PPE_ERR_INTERNAL, "sparse product too large for int32 indices");
  Q.nnz = total;
  Q.maxrow = fm[1];
  int* qci = Q.col.get<int>(Q.nnz);
  double* qv = Q.val.get<double>(Q.nnz);
  if (W <= 4) PPE_QC(4, false, nullptr, qrp, qci, qv);
  else if (W <= 6) PPE_QC(6, false, nullptr, qrp, qci, qv);
  else PPE_QC(8, false, nullptr, qrp, qci, qv);
#undef PPE_QC
  PPE_LAUNCH_CHECK();
}

// AP = A P on the finest level from its ELL copy (k_ap_merge_ell): count,
// scan with the longest row and the device value extra (one round trip),
// fill.  AP is what the general product gives, entry for entry.
static void ap_merge_ell(ppe_solver* s, const Level& L, const Csr& P, Csr& AP, const int* extra,
                         int* extra_host) {
  const int n = L.n, W = L.W;
  AP.n = n;
  AP.m = P.m;
  int* crp = AP.rowptr.get<int>(n + 1);
  int* counts = s->sp_cnt.get<int>(n + 1);
  int* flag = s->flag.get<int>(4);
  fill_int(s, flag, 0, 2);
  const int g = grid_for(n);
  const int* ecol = L.ell_col.as<int>();
  const double* ev = L.ell_val.as<double>();
  const double* dg = L.diag.as<double>();
#define PPE_AP(WM, COUNT, ...)                                                                 \
  hipLaunchKernelGGL((k_ap_merge_ell<WM, COUNT>), dim3(g), dim3(kBlock), 0, s->stream, n, W, ecol, \
                     ev, dg, P.rp(), P.ci(), P.v(), __VA_ARGS__)
  if (W <= 4) PPE_AP(4, true, counts, nullptr, nullptr, nullptr);
  else if (W <= 6) PPE_AP(6, true, counts, nullptr, nullptr, nullptr);
  else PPE_AP(8, true, counts, nullptr, nullptr, nullptr);
  PPE_LAUNCH_CHECK();
  const long long* dtotal = exclusive_scan_async(s, counts, crp, n, 0, flag + 1);
  long long total = 0;
  int fm[2] = {0, 0};
  read_back(s, {ReadItem{dtotal, sizeof(long long), &total}, ReadItem{flag, sizeof(int) * 2, fm},
                ReadItem{extra, sizeof(int), extra_host}});
  require(total <= INT32_MAX, PPE_ERR_INTERNAL, "sparse product too large for int32 indices");
  AP.nnz = total;
  AP.maxrow = fm[1];
  int* cci = AP.col.get<int>(AP.nnz);
  double* cv = AP.val.get<double>(AP.nnz);
  if (W <= 4) PPE_AP(4, false, nullptr, crp, cci, cv);
  else if (W <= 6) PPE_AP(6, false, nullptr, crp, cci, cv);
  else PPE_AP(8, false, nullptr, crp, cci, cv);
#undef PPE_AP
  PPE_LAUNCH_CHECK();
}

void build_hierarchy(ppe_solver* s) {
  const int maxlev = std::max(1, s->opt.max_levels);
  double* rho_dev = s->setup_out.get<double>((size_t)maxlev + 1);
  int* err = reinterpret_cast<int*>(rho_dev + maxlev);
  fill_int(s, err, 0, 1);
  for (int lvl = 0;; ++lvl) {
    Level& L = s->levels[lvl];
    const int n = L.n;
    // setup kernels use the fixed launch rules: choices the autotuner made
    // for the previous hierarchy would change the order of the power
    // iteration's sums, and with it the spectral bound
    L.lpr_a = L.lpr_r = L.lpr_p = 0;
    L.fuse0 = true;
    L.ap_ok = false;
    if (lvl > 0 && n > 0) {
      PPE_ROWS(lanes_for(L.A), k_diag, n, n, L.A.rp(), L.A.ci(), L.A.v(), L.diag.get<double>(n),
               err);  // sets SE_DIAG
    }
    L.n_agg = 0;
    L.dense = false;
    L.mis_rounds = 0;
    const bool last = n <= s->opt.coarse_max || lvl == s->opt.max_levels - 1;
    // a coarsest level solved by its explicit inverse runs no smoother and
    // has no prolongator to smooth: its spectral bound is never used.  A
    // coarse level's power estimate (a chain of small launches) runs on the
    // side stream beside the strength, MIS-2 and aggregation launches,
    // which do not need it; the prolongator smoothing waits for it.
    bool joined = true;
    auto join = [&]() {
      if (!joined) {
        PPE_HIP(hipStreamWaitEvent(s->stream, s->join_ev, 0));
        joined = true;
      }
    };
    if (last && n > 0 && n <= kDenseMax) {
      fill_double(s, rho_dev + lvl, 0.0, 1);
    } else if (lvl > 0 && n > 0) {
      ensure_side_stream(s);
      PPE_HIP(hipEventRecord(s->fork_ev, s->stream));
      PPE_HIP(hipStreamWaitEvent(s->side, s->fork_ev, 0));
      {
        OnStream on(s, s->side);
        spectral_bound(s, L, lvl, rho_dev + lvl);
      }
      PPE_HIP(hipEventRecord(s->join_ev, s->side));
      joined = false;
    } else {
      spectral_bound(s, L, lvl, rho_dev + lvl);
    }
    if (!last) {
      const int g = grid_for(n);
      // the finest level runs these passes on its ELL copy (one thread per
      // row); coarse levels on CSR with lpr lanes per row
      const bool ell = lvl == 0 && L.W > 0;
      const int W = L.W;
      const int* ecol = L.ell_col.as<int>();
      const double* ev = L.ell_val.as<double>();
      unsigned char* strong = ell ? nullptr : L.strong.get<unsigned char>(L.A.nnz);
      int* scol = ell ? L.scol.get<int>((size_t)W * n) : nullptr;
      unsigned char* st = L.state.get<unsigned char>(n);
      unsigned char* st2 = L.state2.get<unsigned char>(n);
      unsigned long long* m1 = L.m1.get<unsigned long long>(n);
      const int lpr = agg_lanes(L.A);
#define PPE_SLOTS(LAUNCH)                      \
  do {                                         \
    if (W <= 4) { LAUNCH(4); }                 \
    else if (W <= 6) { LAUNCH(6); }            \
    else if (W <= 8) { LAUNCH(8); }            \
    else { LAUNCH(0); }                        \
    PPE_LAUNCH_CHECK();                        \
  } while (0)
#define PPE_ELL_K(K, ...) \
  hipLaunchKernelGGL(K, dim3(g), dim3(kBlock), 0, s->stream, __VA_ARGS__)
      // the threshold is halved (theta_decay) on each coarser level
      const double theta_l = s->opt.theta * std::pow(s->opt.theta_decay, lvl);
      if (ell) {
#define PPE_L(WM) PPE_ELL_K(k_strength_ell<WM>, n, W, ecol, ev, L.diag.as<double>(), theta_l * theta_l, scol, st)
        PPE_SLOTS(PPE_L);
#undef PPE_L
      } else {
        PPE_ROWS(lpr, k_strength, n, n, L.A.rp(), L.A.ci(), L.A.v(), L.diag.as<double>(),
                 theta_l * theta_l, strong, st);
      }
      const uint32_t salt = level_salt(lvl);
      // rounds run in triples between host checks; a round after the set is
      // complete changes nothing, so only the last count is read.  The roots
      // are numbered before each check and their count read with it: the
      // numbering is kept once no node is left undecided.
      int* und = s->tmp_i[3].get<int>(1);
      int* root = s->tmp_i[2].get<int>(n + 1);
      int* root_id = L.mis_root.get<int>(n + 1);
      long long n_roots = 0;
      // as many rounds before the first check as this level needed last time
      for (int batch = std::max(3, L.mis_batch);; batch = 3) {
        for (int k = 0; k < batch; ++k) {
          if (k == batch - 1) fill_int(s, und, 0, 1);
          if (ell) {
#define PPE_L(WM) PPE_ELL_K(k_mis_max1_ell<WM>, n, W, scol, st, salt, m1)
            PPE_SLOTS(PPE_L);
#undef PPE_L
#define PPE_L(WM) PPE_ELL_K(k_mis_max2_ell<WM>, n, W, scol, st, salt, m1, st2, und)
            PPE_SLOTS(PPE_L);
#undef PPE_L
          } else {
            PPE_ROWS(lpr, k_mis_max1, n, n, L.A.rp(), L.A.ci(), strong, st, salt, m1);
            PPE_ROWS(lpr, k_mis_max2, n, n, L.A.rp(), L.A.ci(), strong, st, salt, m1, st2, und);
          }
          std::swap(st, st2);
          ++L.mis_rounds;
        }
        hipLaunchKernelGGL(k_is_root, dim3(g), dim3(kBlock), 0, s->stream, n, st, root);
        PPE_LAUNCH_CHECK();
        const long long* total = exclusive_scan_async(s, root, root_id, n);
        int left = 0;
        read_back(s, {ReadItem{und, sizeof(int), &left},
                      ReadItem{total, sizeof(long long), &n_roots}});
        if (left == 0) break;
        require(L.mis_rounds < 10000, PPE_ERR_INTERNAL, "MIS-2 did not terminate");
      }
      L.mis_batch = L.mis_rounds;
      const int na = (int)n_roots;
      if (na > 0) {
        int* agg1 = L.agg1.get<int>(n);
        int* agg = L.agg.get<int>(n);
        if (ell) {
#define PPE_L(WM) PPE_ELL_K(k_agg_first_ell<WM>, n, W, scol, st, root_id, agg1)
          PPE_SLOTS(PPE_L);
#undef PPE_L
#define PPE_L(WM) PPE_ELL_K(k_agg_second_ell<WM>, n, W, scol, ev, agg1, agg, err)
          PPE_SLOTS(PPE_L);  // sets SE_AGG
#undef PPE_L
        } else {
          PPE_ROWS(lpr, k_agg_first, n, n, L.A.rp(), L.A.ci(), strong, st, root_id, agg1);
          PPE_ROWS(lpr, k_agg_second, n, n, L.A.rp(), L.A.ci(), L.A.v(), strong, agg1, agg,
                   err);  // sets SE_AGG
        }
#undef PPE_ELL_K
#undef PPE_SLOTS
        L.n_agg = na;
        // aggregate members, coarse near-null vector, tentative prolongator
        // (nodes with no strong connection stay outside every aggregate, so
        // members and prolongator entries number at most n; only the device
        // row pointers are exact)
        int* cnt = s->tmp_i[0].get<int>(na + 1);
        fill_int(s, cnt, 0, na + 1);
        hipLaunchKernelGGL(k_agg_count, dim3(g), dim3(kBlock), 0, s->stream, n, agg, cnt);
        PPE_LAUNCH_CHECK();
        int* aptr = L.agg_ptr.get<int>(na + 1);
        exclusive_scan_async(s, cnt, aptr, na);
        int* cursor = s->tmp_i[1].get<int>(na + 1);
        PPE_HIP(hipMemcpyAsync(cursor, aptr, sizeof(int) * (na + 1), hipMemcpyDeviceToDevice,
                               s->stream));
        int* mem = L.agg_mem.get<int>(n);
        hipLaunchKernelGGL(k_agg_fill, dim3(g), dim3(kBlock), 0, s->stream, n, agg, cursor, mem);
        PPE_LAUNCH_CHECK();
        if ((int)s->levels.size() < lvl + 2) s->levels.resize(lvl + 2);
        Level& L0 = s->levels[lvl];  // re-fetch: resize may move levels
        Level& C = s->levels[lvl + 1];
        double* Bc = C.B.get<double>(na);
        hipLaunchKernelGGL(k_agg_norm, dim3(grid_for((int64_t)na * kWave)), dim3(kBlock), 0,
                           s->stream, na, aptr, mem, L0.B.as<double>(), Bc);
        PPE_LAUNCH_CHECK();
        double* pt = L0.pt.get<double>(n);
        int* pcnt = s->tmp_i[0].get<int>(n + 1);
        hipLaunchKernelGGL(k_tent, dim3(g), dim3(kBlock), 0, s->stream, n, agg, L0.B.as<double>(), Bc,
                           pcnt, pt);
        PPE_LAUNCH_CHECK();
        Csr& Pt = L0.Pt;
        Pt.n = n;
        Pt.m = na;
        Pt.maxrow = 1;
        int* ptrp = Pt.rowptr.get<int>(n + 1);
        exclusive_scan_async(s, pcnt, ptrp, n);
        Pt.nnz = n;  // capacity (an upper bound): only the row pointers are read
        hipLaunchKernelGGL(k_tent_csr, dim3(g), dim3(kBlock), 0, s->stream, n, ptrp, agg, pt,
                           Pt.col.get<int>(Pt.nnz), Pt.val.get<double>(Pt.nnz));
        PPE_LAUNCH_CHECK();
        // smoothed prolongator
        if (lvl == 0 && L0.W > 0 && L0.W <= 8) {
          coarsen_cols_ell(s, L0, agg, pt, na, L0.Q);
        } else {
          spgemm(s, L0.A, Pt, L0.Q, nullptr, nullptr);
        }
        Csr& P = L0.P;
        P.n = n;
        P.m = na;
        P.nnz = L0.Q.nnz;
        P.maxrow = L0.Q.maxrow;
        join();  // the smoothing uses this level's spectral bound
        hipLaunchKernelGGL(k_smooth_p, dim3(g), dim3(kBlock), 0, s->stream, n, L0.Q.rp(), L0.Q.ci(),
                           L0.Q.v(), L0.diag.as<double>(), agg, pt, rho_dev + lvl,
                           P.val.get<double>(P.nnz));
        PPE_LAUNCH_CHECK();
        // P has the pattern of A P_tent: take its arrays instead of copying
        std::swap(P.rowptr, L0.Q.rowptr);
        std::swap(P.col, L0.Q.col);
        transpose(s, P, L0.R);
        if (lvl == 0 && L0.W > 0 && L0.W <= 8)
          ap_merge_ell(s, L0, P, L0.AP, s->rmax.as<int>(), &L0.R.maxrow);
        else
          spgemm(s, L0.A, P, L0.AP, s->rmax.as<int>(), &L0.R.maxrow);
        L0.ap_ok = true;
        spgemm(s, L0.R, L0.AP, C.A, nullptr, nullptr);
        C.n = na;
        s->nlev = lvl + 2;
        continue;
      }
    }
    // coarsest level
    join();
    s->nlev = lvl + 1;
    if (n > 0 && n <= kDenseMax) {
      double* Ainv = L.Ainv.get<double>((size_t)n * n);
      double* G = nullptr;
      if (n <= kDenseBlk) {  // [A | I] for the one-workgroup elimination
        G = s->tmp_d[1].get<double>((size_t)2 * n * n);
        fill_double(s, G, 0.0, (int64_t)2 * n * n);
        hipLaunchKernelGGL(k_densify, dim3(grid_for((int64_t)n * kWave)), dim3(kBlock), 0,
                           s->stream, n, L.A.rp(), L.A.ci(), L.A.v(), G);
        PPE_LAUNCH_CHECK();
      }
      if (n <= kDenseBlk) {
        hipLaunchKernelGGL(k_dense_inverse_blk, dim3(1), dim3(1024), 0, s->stream, n, G, Ainv, err);
      } else {
        // 129 .. 1024 rows: blocked over nb x nb workgroups per block step
        const int nb = (n + 31) / 32, N = 32 * nb;
        double* G0 = s->tmp_d[1].get<double>((size_t)2 * N * N + 1024);
        double* G1 = G0 + (size_t)N * N;
        double* Dinv = G1 + (size_t)N * N;
        fill_double(s, G0, 0.0, (int64_t)N * N);
        hipLaunchKernelGGL(k_densify_sq, dim3(grid_for((int64_t)N * kWave)), dim3(kBlock), 0,
                           s->stream, n, N, L.A.rp(), L.A.ci(), L.A.v(), G0);
        PPE_LAUNCH_CHECK();
        for (int K = 0; K < nb; ++K) {
          hipLaunchKernelGGL(k_ginv_diag, dim3(1), dim3(1024), 0, s->stream, N, G0, K, Dinv, err);
          PPE_LAUNCH_CHECK();
          hipLaunchKernelGGL(k_ginv_update, dim3(nb, nb), dim3(1024), 0, s->stream, N, G0, Dinv,
                             K, G1);
          PPE_LAUNCH_CHECK();
          std::swap(G0, G1);
        }
        hipLaunchKernelGGL(k_lead_block, dim3(grid_for((int64_t)n * n)), dim3(kBlock), 0,
                           s->stream, n, N, G0, Ainv);
      }
      PPE_LAUNCH_CHECK();
      L.dense = true;
    }
    break;
  }
  // one read-back for the whole hierarchy: spectral bounds and error bits
  std::vector<double> out((size_t)maxlev + 1);
  read_back(s, {ReadItem{rho_dev, sizeof(double) * (maxlev + 1), out.data()}});
  int bits = 0;
  std::memcpy(&bits, &out[maxlev], sizeof(int));
  require(!(bits & SE_DIAG), PPE_ERR_INTERNAL, "coarse operator lost its diagonal");
  require(!(bits & SE_AGG), PPE_ERR_INTERNAL, "aggregation left a node unassigned");
  require(!(bits & SE_DENSE), PPE_ERR_INTERNAL, "coarsest operator is not positive definite");
  for (int l = 0; l < s->nlev; ++l) s->levels[l].rho = out[l];
}

}  // namespace ppe

// Polynomial chaos by stochastic collocation (section 3, Eq. 27-28).
//
// The expansion w(x, xi) ~ sum_i w_i(x) Psi_i(xi) uses products of
// one-dimensional polynomials orthonormal under each input's distribution
// (probabilists' Hermite for a standard normal input, Legendre for a uniform
// input on [-1, 1]) over every multi-index of total degree <= p.  Its
// coefficients come from the least-squares solution of the Vandermonde
// system V W = Y at M sample points (Eq. 28), for every output x at once.
//
// Host side (sizes of a few hundred): Gauss rules, tensor and Smolyak node
// sets, the basis, V and the projection P = R^-1 Q^T of a Householder QR of
// V.  Device side (sizes of the field): W = P Y, the evaluation V_test W at
// test points, and the per-output mean, variance and Sobol indices.
#include "common.h"

#include <algorithm>
#include <cmath>
#include <functional>
#include <map>

struct ppe_pce {
  int d = 0, degree = 0, n_terms = 0;
  std::vector<int> kinds;   // PPE_INPUT_NORMAL / PPE_INPUT_UNIFORM per input
  std::vector<int> alpha;   // n_terms x d multi-indices, graded order
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;
  ppe::DevBuf a_dev, mask_dev;
};

namespace ppe {
namespace {

// orthonormal recurrence x psi_k = b_{k+1} psi_{k+1} + b_k psi_{k-1} (zero
// diagonal for both symmetric families): Hermite b_k = sqrt(k), Legendre
// b_k = k / sqrt(4k^2 - 1)
double rec_b(int kind, int k) {
  if (k == 0) return 0.0;  // multiplies psi_{-1} = 0
  return kind == PPE_INPUT_NORMAL ? std::sqrt((double)k) : k / std::sqrt(4.0 * k * k - 1.0);
}

// psi_0..psi_n at x; returns psi_n, and psi_{n-1} in *prev
double psi_n(int kind, int n, double x, double* prev) {
  double pm = 0.0, p = 1.0;
  for (int k = 0; k < n; ++k) {
    const double next = (x * p - rec_b(kind, k) * pm) / rec_b(kind, k + 1);
    pm = p;
    p = next;
  }
  if (prev) *prev = pm;
  return p;
}

// n-point Gauss rule with probability weights: roots of psi_n found between
// consecutive roots of psi_{n-1} (interlacing) by bisection, polished by
// Newton; weights from the Christoffel numbers 1 / sum_{k<n} psi_k(x)^2.
void gauss_rule(int kind, int n, std::vector<double>& x, std::vector<double>& w) {
  std::vector<double> prev_roots;
  const double outer = kind == PPE_INPUT_NORMAL ? std::sqrt(4.0 * n + 2.0) + 1.0 : 1.0;
  std::vector<double> roots;
  for (int m = 1; m <= n; ++m) {
    roots.assign(m, 0.0);
    for (int i = 0; i < m; ++i) {
      double lo = i == 0 ? -outer : prev_roots[i - 1];
      double hi = i == m - 1 ? outer : prev_roots[i];
      double flo = psi_n(kind, m, lo, nullptr);
      for (int it = 0; it < 200 && hi - lo > 1e-16 * std::max(1.0, std::fabs(lo)); ++it) {
        const double mid = 0.5 * (lo + hi);
        const double fm = psi_n(kind, m, mid, nullptr);
        if ((fm < 0) == (flo < 0)) {
          lo = mid;
          flo = fm;
        } else {
          hi = mid;
        }
      }
      roots[i] = 0.5 * (lo + hi);
    }
    prev_roots = roots;
  }
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double r = roots[i];
    for (int it = 0; it < 3; ++it) {  // Newton, psi_n' from the differentiated recurrence
      double pm = 0.0, p = 1.0, dpm = 0.0, dp = 0.0;
      for (int k = 0; k < n; ++k) {
        const double b1 = rec_b(kind, k + 1), b0 = rec_b(kind, k);
        const double next = (r * p - b0 * pm) / b1;
        const double dnext = (p + r * dp - b0 * dpm) / b1;
        pm = p;
        p = next;
        dpm = dp;
        dp = dnext;
      }
      if (dp == 0.0) break;
      r -= p / dp;
    }
    x[i] = r;
  }
  // exact symmetry about 0
  for (int i = 0; i < n / 2; ++i) {
    const double s = 0.5 * (x[n - 1 - i] - x[i]);
    x[i] = -s;
    x[n - 1 - i] = s;
  }
  if (n % 2) x[n / 2] = 0.0;
  for (int i = 0; i < n; ++i) {
    double pm = 0.0, p = 1.0, s = 1.0;
    for (int k = 0; k + 1 < n; ++k) {
      const double next = (x[i] * p - rec_b(kind, k) * pm) / rec_b(kind, k + 1);
      pm = p;
      p = next;
      s += p * p;
    }
    w[i] = 1.0 / s;
  }
}

struct NodeSet {
  std::map<std::vector<long long>, std::pair<std::vector<double>, double>> pts;
  void add(const std::vector<double>& x, double w) {
    std::vector<long long> key(x.size());
    for (size_t j = 0; j < x.size(); ++j) key[j] = std::llround(x[j] * 1e12);  // identifies coincident nodes
    auto it = pts.find(key);
    if (it == pts.end()) pts.emplace(key, std::make_pair(x, w));
    else it->second.second += w;
  }
};

long long binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  long long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

void add_tensor(NodeSet& S, const std::vector<int>& kinds, const std::vector<int>& npts, double coef) {
  const int d = (int)kinds.size();
  std::vector<std::vector<double>> xs(d), ws(d);
  for (int j = 0; j < d; ++j) gauss_rule(kinds[j], npts[j], xs[j], ws[j]);
  std::vector<int> c(d, 0);
  std::vector<double> x(d);
  for (;;) {
    double w = coef;
    for (int j = 0; j < d; ++j) {
      x[j] = xs[j][c[j]];
      w *= ws[j][c[j]];
    }
    S.add(x, w);
    int j = 0;
    while (j < d && ++c[j] == npts[j]) c[j++] = 0;
    if (j == d) break;
  }
}

// Householder QR of V (M x K, row-major, M >= K): P = R^-1 Q^T (K x M).
// Returns false if R has a (relatively) zero diagonal entry.
bool projection(int M, int K, std::vector<double> V, std::vector<double>& P) {
  std::vector<double> Qt((size_t)M * M, 0.0);  // accumulate Q^T applied to I
  for (int i = 0; i < M; ++i) Qt[(size_t)i * M + i] = 1.0;
  double vmax = 0.0;
  for (double v : V) vmax = std::max(vmax, std::fabs(v));
  for (int k = 0; k < K; ++k) {
    double nrm = 0.0;
    for (int i = k; i < M; ++i) nrm += V[(size_t)i * K + k] * V[(size_t)i * K + k];
    nrm = std::sqrt(nrm);
    if (!(nrm > 1e-13 * vmax)) return false;
    const double alpha = V[(size_t)k * K + k] > 0 ? -nrm : nrm;
    std::vector<double> v(M, 0.0);
    for (int i = k; i < M; ++i) v[i] = V[(size_t)i * K + k];
    v[k] -= alpha;
    double vv = 0.0;
    for (int i = k; i < M; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    for (int j = k; j < K; ++j) {
      double s = 0.0;
      for (int i = k; i < M; ++i) s += v[i] * V[(size_t)i * K + j];
      s = 2.0 * s / vv;
      for (int i = k; i < M; ++i) V[(size_t)i * K + j] -= s * v[i];
    }
    for (int j = 0; j < M; ++j) {
      double s = 0.0;
      for (int i = k; i < M; ++i) s += v[i] * Qt[(size_t)i * M + j];
      s = 2.0 * s / vv;
      for (int i = k; i < M; ++i) Qt[(size_t)i * M + j] -= s * v[i];
    }
  }
  // P = R^-1 (first K rows of Q^T): back substitution per column
  P.assign((size_t)K * M, 0.0);
  for (int c = 0; c < M; ++c) {
    for (int i = K - 1; i >= 0; --i) {
      double s = Qt[(size_t)i * M + c];
      for (int j = i + 1; j < K; ++j) s -= V[(size_t)i * K + j] * P[(size_t)j * M + c];
      P[(size_t)i * M + c] = s / V[(size_t)i * K + i];
    }
  }
  return true;
}

// C (R x n) = A (R x K) B (K x n), B and C row-major with leading dimension
// n.  A is staged through LDS in chunks of kChunk columns; thread column c
// accumulates kTerms rows of C (blockIdx.y picks which).
constexpr int kTerms = 16;
constexpr int kChunk = 64;

__global__ void __launch_bounds__(kBlock) k_small_times_wide(int R, int K, long long n,
                                                             const double* __restrict__ A,
                                                             const double* __restrict__ B,
                                                             double* __restrict__ C) {
  __shared__ double a[kTerms][kChunk];
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  const int r0 = blockIdx.y * kTerms;
  double acc[kTerms];
#pragma unroll
  for (int t = 0; t < kTerms; ++t) acc[t] = 0.0;
  for (int k0 = 0; k0 < K; k0 += kChunk) {
    const int kn = min(kChunk, K - k0);
    __syncthreads();
    for (int e = threadIdx.x; e < kTerms * kChunk; e += kBlock) {
      const int t = e / kChunk, k = e % kChunk;
      a[t][k] = (r0 + t < R && k < kn) ? A[(size_t)(r0 + t) * K + k0 + k] : 0.0;
    }
    __syncthreads();
    if (c < n) {
      for (int k = 0; k < kn; ++k) {
        const double b = B[(size_t)(k0 + k) * n + c];
#pragma unroll
        for (int t = 0; t < kTerms; ++t) acc[t] = fma(a[t][k], b, acc[t]);
      }
    }
  }
  if (c < n) {
#pragma unroll
    for (int t = 0; t < kTerms; ++t)
      if (r0 + t < R) C[(size_t)(r0 + t) * n + c] = acc[t];
  }
}

// Per output: mean W_0, variance sum_{i>0} W_i^2, and for each input j the
// first-order (terms in j alone) and total (terms involving j) shares.
// mask[i] bit j: term i involves input j; bit 30: it involves one input only.
__global__ void k_pce_stats(int n_terms, int d, long long n, const double* __restrict__ W,
                            const int* __restrict__ mask, double* __restrict__ mean,
                            double* __restrict__ var, double* __restrict__ first,
                            double* __restrict__ total) {
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= n) return;
  double v = 0.0;
  for (int i = 1; i < n_terms; ++i) {
    const double x = W[(size_t)i * n + c];
    v += x * x;
  }
  mean[c] = W[c];
  var[c] = v;
  for (int j = 0; j < d; ++j) {
    double f = 0.0, t = 0.0;
    for (int i = 1; i < n_terms; ++i) {
      const int m = mask[i];
      if (!(m & (1 << j))) continue;
      const double x = W[(size_t)i * n + c];
      t += x * x;
      if (m & (1 << 30)) f += x * x;
    }
    first[(size_t)j * n + c] = v > 0 ? f / v : 0.0;
    total[(size_t)j * n + c] = v > 0 ? t / v : 0.0;
  }
}

void small_times_wide(hipStream_t st, int R, int K, long long n, const double* A, const double* B,
                      double* C) {
  if (n == 0 || R == 0) return;
  const long long gx = (n + kBlock - 1) / kBlock;
  require(gx <= INT32_MAX, PPE_ERR_ARG, "too many outputs");
  hipLaunchKernelGGL(k_small_times_wide, dim3((unsigned)gx, (R + kTerms - 1) / kTerms), dim3(kBlock),
                     0, st, R, K, n, A, B, C);
  PPE_LAUNCH_CHECK();
}

std::vector<double> vandermonde(const ppe_pce* q, int M, const double* xi) {
  const int K = q->n_terms, d = q->d;
  std::vector<double> V((size_t)M * K, 1.0);
  for (int m = 0; m < M; ++m) {
    // psi_k of every input up to the degree
    std::vector<std::vector<double>> ps(d);
    for (int j = 0; j < d; ++j) {
      ps[j].assign(q->degree + 1, 1.0);
      double pm = 0.0, p = 1.0;
      for (int k = 0; k < q->degree; ++k) {
        const double next = (xi[(size_t)m * d + j] * p - rec_b(q->kinds[j], k) * pm) /
                            rec_b(q->kinds[j], k + 1);
        pm = p;
        p = next;
        ps[j][k + 1] = p;
      }
    }
    for (int i = 0; i < K; ++i) {
      double v = 1.0;
      for (int j = 0; j < d; ++j) v *= ps[j][q->alpha[(size_t)i * d + j]];
      V[(size_t)m * K + i] = v;
    }
  }
  return V;
}

}  // namespace
}  // namespace ppe

using ppe::require;

namespace {
template <class F>
ppe_status guarded_pce(ppe_pce* q, F&& f) {
  try {
    if (q) q->err.clear();
    return f();
  } catch (const ppe::Error& e) {
    if (q) q->err = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    if (q) q->err = "host allocation failed";
    return PPE_ERR_OOM;
  } catch (const std::exception& e) {
    if (q) q->err = e.what();
    return PPE_ERR_INTERNAL;
  }
}
}  // namespace

extern "C" {

ppe_status ppe_pce_create(int32_t d, const int32_t* kinds, int32_t degree, void* stream,
                          ppe_pce** out) {
  if (!out || !kinds || d < 1 || d > 16 || degree < 0 || degree > 30) return PPE_ERR_ARG;
  for (int j = 0; j < d; ++j)
    if (kinds[j] != PPE_INPUT_NORMAL && kinds[j] != PPE_INPUT_UNIFORM) return PPE_ERR_ARG;
  auto* q = new ppe_pce();
  q->d = d;
  q->degree = degree;
  q->kinds.assign(kinds, kinds + d);
  q->stream = static_cast<hipStream_t>(stream);
  (void)hipGetDevice(&q->device);
  // graded order: by total degree, then lexicographically descending
  for (int deg = 0; deg <= degree; ++deg) {
    std::vector<std::vector<int>> lvl;
    std::vector<int> a(d, 0);
    std::function<void(int, int)> rec = [&](int j, int left) {
      if (j == d - 1) {
        a[j] = left;
        lvl.push_back(a);
        return;
      }
      for (int v = left; v >= 0; --v) {
        a[j] = v;
        rec(j + 1, left - v);
      }
    };
    rec(0, deg);
    for (auto& m : lvl) q->alpha.insert(q->alpha.end(), m.begin(), m.end());
  }
  q->n_terms = (int)(q->alpha.size() / d);
  *out = q;
  return PPE_OK;
}

void ppe_pce_destroy(ppe_pce* q) { delete q; }

int32_t ppe_pce_num_terms(const ppe_pce* q) { return q ? q->n_terms : 0; }

const char* ppe_pce_last_error(const ppe_pce* q) { return q ? q->err.c_str() : ""; }

ppe_status ppe_pce_terms(const ppe_pce* q, int32_t* alpha) {
  if (!q || !alpha) return PPE_ERR_ARG;
  std::copy(q->alpha.begin(), q->alpha.end(), alpha);
  return PPE_OK;
}

ppe_status ppe_pce_nodes(ppe_pce* q, int32_t grid, int32_t level, int32_t* n_nodes, double* nodes,
                         double* weights) {
  if (!q || !n_nodes) return PPE_ERR_ARG;
  return guarded_pce(q, [&]() -> ppe_status {
    require(level >= 1 && level <= 20, PPE_ERR_ARG, "level must be in 1..20");
    require(grid == PPE_GRID_TENSOR || grid == PPE_GRID_SMOLYAK, PPE_ERR_ARG, "unknown grid");
    const int d = q->d;
    ppe::NodeSet S;
    if (grid == PPE_GRID_TENSOR) {
      ppe::add_tensor(S, q->kinds, std::vector<int>(d, level), 1.0);
    } else {
      const int qq = level + d - 1;
      std::vector<int> idx(d, 1);
      for (;;) {
        int s = 0;
        for (int v : idx) s += v;
        if (s >= level && s <= qq) {
          const double c = ((qq - s) % 2 ? -1.0 : 1.0) * (double)ppe::binom(d - 1, qq - s);
          ppe::add_tensor(S, q->kinds, idx, c);
        }
        int j = 0;
        while (j < d && ++idx[j] > level) idx[j++] = 1;
        if (j == d) break;
      }
    }
    const int n = (int)S.pts.size();
    if (nodes) {
      require(*n_nodes >= n, PPE_ERR_ARG, "node arrays too small");
      int i = 0;
      for (auto& kv : S.pts) {
        for (int j = 0; j < d; ++j) nodes[(size_t)i * d + j] = kv.second.first[j];
        if (weights) weights[i] = kv.second.second;
        ++i;
      }
    }
    *n_nodes = n;
    return PPE_OK;
  });
}

ppe_status ppe_pce_fit(ppe_pce* q, int32_t M, const double* xi, int64_t n_out, const double* Y,
                       double* W) {
  if (!q) return PPE_ERR_ARG;
  return guarded_pce(q, [&]() -> ppe_status {
    require(xi && Y && W, PPE_ERR_ARG, "NULL array");
    require(M >= q->n_terms, PPE_ERR_ARG, "fewer sample points than expansion terms");
    require(n_out >= 0, PPE_ERR_ARG, "negative output count");
    const std::vector<double> V = ppe::vandermonde(q, M, xi);
    std::vector<double> P;
    require(ppe::projection(M, q->n_terms, V, P), PPE_ERR_ARG,
            "the Vandermonde matrix of these points is rank deficient");
    double* Pd = q->a_dev.get<double>(P.size());
    PPE_HIP(hipMemcpyAsync(Pd, P.data(), sizeof(double) * P.size(), hipMemcpyHostToDevice, q->stream));
    ppe::small_times_wide(q->stream, q->n_terms, M, n_out, Pd, Y, W);
    PPE_HIP(hipStreamSynchronize(q->stream));
    return PPE_OK;
  });
}

ppe_status ppe_pce_eval(ppe_pce* q, int32_t T, const double* xi, int64_t n_out, const double* W,
                        double* Y) {
  if (!q) return PPE_ERR_ARG;
  return guarded_pce(q, [&]() -> ppe_status {
    require(xi && W && Y, PPE_ERR_ARG, "NULL array");
    require(T >= 0 && n_out >= 0, PPE_ERR_ARG, "negative size");
    if (T == 0) return PPE_OK;
    const std::vector<double> V = ppe::vandermonde(q, T, xi);
    double* Vd = q->a_dev.get<double>(V.size());
    PPE_HIP(hipMemcpyAsync(Vd, V.data(), sizeof(double) * V.size(), hipMemcpyHostToDevice, q->stream));
    ppe::small_times_wide(q->stream, T, q->n_terms, n_out, Vd, W, Y);
    PPE_HIP(hipStreamSynchronize(q->stream));
    return PPE_OK;
  });
}

ppe_status ppe_pce_stats(ppe_pce* q, int64_t n_out, const double* W, double* mean, double* var,
                         double* first, double* total) {
  if (!q) return PPE_ERR_ARG;
  return guarded_pce(q, [&]() -> ppe_status {
    require(W && mean && var && first && total, PPE_ERR_ARG, "NULL array");
    require(n_out >= 0, PPE_ERR_ARG, "negative output count");
    if (n_out == 0) return PPE_OK;
    std::vector<int> mask(q->n_terms, 0);
    for (int i = 0; i < q->n_terms; ++i) {
      int cnt = 0;
      for (int j = 0; j < q->d; ++j)
        if (q->alpha[(size_t)i * q->d + j]) {
          mask[i] |= 1 << j;
          ++cnt;
        }
      if (cnt == 1) mask[i] |= 1 << 30;
    }
    int* md = q->mask_dev.get<int>(mask.size());
    PPE_HIP(hipMemcpyAsync(md, mask.data(), sizeof(int) * mask.size(), hipMemcpyHostToDevice, q->stream));
    const long long g = (n_out + ppe::kBlock - 1) / ppe::kBlock;
    require(g <= INT32_MAX, PPE_ERR_ARG, "too many outputs");
    hipLaunchKernelGGL(ppe::k_pce_stats, dim3((unsigned)g), dim3(ppe::kBlock), 0, q->stream, q->n_terms,
                       q->d, (long long)n_out, W, md, mean, var, first, total);
    PPE_LAUNCH_CHECK();
    PPE_HIP(hipStreamSynchronize(q->stream));
    return PPE_OK;
  });
}

}  // extern "C"

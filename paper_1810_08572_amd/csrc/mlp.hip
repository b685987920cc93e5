// Learned warm start (not part of the paper's method; conjugate gradients
// always finishes the solve, so the network can only change the iteration
// count).  A dense network n_in -> width (x n_hidden, SiLU) -> 1 (linear)
// maps per-cell features to the next pressure increment.
//
//   training   FP32: tiled GEMMs (deterministic split-K over the rows),
//              SiLU, mean-squared-error gradient, Adam;
//   inference  the width x width hidden layers on BF16 MFMA
//              (v_mfma_f32_32x32x8bf16_1k, FP32 accumulation), the first and
//              last (thin) layers in FP32 on the vector ALUs;
//   features   of every active cell, from the solver's mesh adjacency.
//
// Parameters are FP32, packed layer by layer: W ([out][in], row-major), b.
#include "common.h"

#include <cmath>
#include <mutex>
#include <string>

struct ppe_mlp {
  int n_in = 0, width = 0, n_hidden = 0;
  hipStream_t stream = nullptr;
  int64_t n_params = 0;
  std::vector<int> dims;                 // n_in, width, ..., width, 1
  std::vector<int64_t> woff, boff;       // offsets of W_l, b_l in the packed vector
  ppe::DevBuf params, grad, m, v, bf16;  // bf16: hidden weight matrices in BF16
  ppe::DevBuf act, pre, gbuf, gbuf2, part, lossbuf;
  int64_t adam_t = 0;
  size_t lds_max = 0;  // LDS one workgroup may use (0: not queried yet)
  int cus = 0;         // compute units of the device
  std::string err;
};

namespace ppe {
namespace {

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s + z * s * (1.0f - s);
}

// C (+)= op(A) op(B): op(A)(i,k) = A[i*ari + k*ack], op(B)(k,j) = B[k*brk + j*bcj].
// Block (64 x 64 outputs, 256 threads, 4 x 4 per thread); blockIdx.z selects
// a chunk of `kc` values of k and writes its own partial C + z*M*N (split-K;
// the chunks are added afterwards in chunk order).
constexpr int TM = 64, TN = 64, TK = 16;
__global__ void __launch_bounds__(256) k_sgemm(int M, int N, int K, int kc, const float* __restrict__ A,
                                               int64_t ari, int64_t ack, const float* __restrict__ B,
                                               int64_t brk, int64_t bcj, float* __restrict__ C) {
  __shared__ float As[TK][TM + 1];
  __shared__ float Bs[TK][TN + 1];
  const int t = threadIdx.x, tx = t % 16, ty = t / 16;
  const int i0 = blockIdx.y * TM, j0 = blockIdx.x * TN;
  const int k_begin = blockIdx.z * kc, k_end = min(K, k_begin + kc);
  float acc[4][4] = {};
  for (int k0 = k_begin; k0 < k_end; k0 += TK) {
    for (int e = t; e < TM * TK; e += 256) {
      const int ii = e / TK, kk = e % TK;
      const int i = i0 + ii, k = k0 + kk;
      As[kk][ii] = (i < M && k < k_end) ? A[i * ari + k * ack] : 0.0f;
    }
    for (int e = t; e < TN * TK; e += 256) {
      const int kk = e / TN, jj = e % TN;
      const int j = j0 + jj, k = k0 + kk;
      Bs[kk][jj] = (j < N && k < k_end) ? B[k * brk + j * bcj] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[kk][ty * 4 + r];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx * 4 + c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = acc[r][c] + a[r] * b[c];
    }
    __syncthreads();
  }
  float* Cz = C + (size_t)blockIdx.z * M * N;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = i0 + ty * 4 + r, j = j0 + tx * 4 + c;
      if (i < M && j < N) Cz[(size_t)i * N + j] = acc[r][c];
    }
}

// out[e] = sum over z of parts[z * len + e], in z order
__global__ void k_sum_chunks(int64_t len, int nz, const float* __restrict__ parts,
                             float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= len) return;
  float s = 0.0f;
  for (int z = 0; z < nz; ++z) s = s + parts[(size_t)z * len + e];
  out[e] = s;
}

// z = y + b (row broadcast); stores z, and h = silu(z) when silu != 0
__global__ void k_bias_act(int64_t n, int width, const float* __restrict__ y,
                           const float* __restrict__ b, float* __restrict__ z,
                           float* __restrict__ h, int silu) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n * width) return;
  const float v = y[e] + b[e % width];
  z[e] = v;
  h[e] = silu ? silu_f(v) : v;
}

// output layer: g = 2/n (y - t); partial sums of (y - t)^2 per block
__global__ void k_loss_grad(int n, const float* __restrict__ y, const float* __restrict__ t,
                            float* __restrict__ g, double* __restrict__ partials) {
  double acc = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const float e = y[i] - t[i];
    g[i] = (2.0f / (float)n) * e;
    acc += (double)e * (double)e;
  }
  double v[1] = {acc};
  write_partials<kBlock, 1>(v, partials);
}

__global__ void k_finalize_loss(const double* __restrict__ partials, int g, int n,
                                double* __restrict__ out) {
  const double s = sum_partials<kBlock>(partials, g);
  if (threadIdx.x == 0) *out = s / n;
}

// g *= silu'(z)
__global__ void k_dsilu_mul(int64_t len, const float* __restrict__ z, float* __restrict__ g) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < len) g[e] = g[e] * dsilu_f(z[e]);
}

// column sums of G [n x w] over rows chunk z: parts[z*w + j]
constexpr int kColRows = 64, kColChunks = 1024;
__global__ void k_colsum_chunks(int n, int w, int chunk, const float* __restrict__ G,
                                float* __restrict__ parts) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= w) return;
  const int r0 = blockIdx.y * chunk, r1 = min(n, r0 + chunk);
  float s = 0.0f;
  for (int r = r0; r < r1; ++r) s = s + G[(size_t)r * w + j];
  parts[(size_t)blockIdx.y * w + j] = s;
}

__global__ void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, float lr, float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  const float b1 = 0.9f, b2 = 0.999f;
  const float mm = b1 * m[e] + (1.0f - b1) * g[e];
  const float vv = b2 * v[e] + (1.0f - b2) * g[e] * g[e];
  m[e] = mm;
  v[e] = vv;
  p[e] = p[e] - lr * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
}

__global__ void k_to_bf16(int64_t n, const float* __restrict__ a, uint16_t* __restrict__ b) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  // round to nearest even
  uint32_t u = __float_as_uint(a[e]);
  u += 0x7FFFu + ((u >> 16) & 1u);
  b[e] = (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------- BF16 inference
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float16_t __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

constexpr int kW = 128;      // hidden width of the MFMA path
constexpr int kIn = 10;      // input features of the MFMA path
constexpr int kWaves = 4;    // waves per workgroup, 32 cells each

// One wave per tile of 32 cells; hidden activations live in LDS as
// [cell][feature] bf16.  For a hidden layer, out^T (features x cells) =
// W (width x width) . h^T: 4 output tiles of 32 features, 16 k-steps of 8.
// Operand layout of v_mfma_f32_32x32x8bf16_1k: lane l holds A[l%32][4(l/32)+v]
// and B[4(l/32)+v][l%32] (v = 0..3); accumulator r of lane l is
// C[8(r/4) + 4(l/32) + r%4][l%32].
__global__ void __launch_bounds__(64 * kWaves) k_mlp_infer_bf16(
    int n, int n_hidden, const float* __restrict__ x, const float* __restrict__ params,
    const uint16_t* __restrict__ wbf, float* __restrict__ y) {
  __shared__ uint16_t hA[kWaves][32 * kW];
  __shared__ uint16_t hB[kWaves][32 * kW];
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  const int cell = lane % 32, half = lane / 32;
  const float* W1 = params;
  const float* b1 = W1 + kW * kIn;
  const int64_t hid = (int64_t)kW * kW + kW;
  const float* last = b1 + kW + (n_hidden - 1) * hid;  // W_out [1 x kW], then b_out
  const int ntile = (n + 31) / 32;
  // every wave of the workgroup runs the same trip count (the barriers below
  // are workgroup-wide); tiles past the end compute on zeros and store nothing
  for (int base = blockIdx.x * kWaves; base < ntile; base += gridDim.x * kWaves) {
    const int tile = base + wv;
    const int c = tile * 32 + cell;
    // layer 1 (n_in -> width) in FP32: this lane does features half*64 .. +63
    float xin[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) xin[k] = c < n ? x[(size_t)c * kIn + k] : 0.0f;
    for (int f = half * 64; f < half * 64 + 64; ++f) {
      float s = b1[f];
#pragma unroll
      for (int k = 0; k < kIn; ++k) s = s + W1[f * kIn + k] * xin[k];
      hA[wv][cell * kW + f] = f2bf(silu_f(s));
    }
    __syncthreads();
    uint16_t* hin = hA[wv];
    uint16_t* hout = hB[wv];
    for (int l = 0; l < n_hidden - 1; ++l) {
      const uint16_t* W = wbf + (size_t)l * kW * kW;
      const float* bias = b1 + kW + l * hid + kW * kW;
      for (int mt = 0; mt < kW / 32; ++mt) {
        float16_t acc = {0};
        for (int kt = 0; kt < kW / 8; ++kt) {
          const int kk = kt * 8 + 4 * half;
          short4_t a, b;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            a[v] = (short)W[(size_t)(mt * 32 + cell) * kW + kk + v];
            b[v] = (short)hin[cell * kW + kk + v];
          }
          acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int f = mt * 32 + 8 * (r / 4) + 4 * half + (r % 4);
          hout[cell * kW + f] = f2bf(silu_f(acc[r] + bias[f]));
        }
      }
      __syncthreads();
      uint16_t* tmp = hin;
      hin = hout;
      hout = tmp;
    }
    // output layer (width -> 1) in FP32 from the bf16 activations
    float s = 0.0f;
    for (int f = half * 64; f < half * 64 + 64; ++f)
      s = s + last[f] * __uint_as_float((uint32_t)hin[cell * kW + f] << 16);
    s = s + __shfl_down(s, 32, 64);
    if (half == 0 && c < n) y[c] = s + last[kW];
    __syncthreads();
  }
}

// The inference pass used at every timestep.  With out^T = W h^T (features x
// cells), a lane's accumulators r = 4q .. 4q+3 hold four consecutive
// features of one cell: the k-quad the next layer's B operand reads.  So
// activations and weights sit in LDS as quads of BF16 (8 bytes):
// activation (k, cell) in quad (k/4) 32 + cell of the wave's buffer, weight
// (f, k) in quad (k/4) 128 + f, and every MFMA operand is one 8-byte LDS
// read per lane, consecutive across lanes.  The hidden weights are staged
// once per workgroup; a layer's outputs are computed in registers for all
// 128 features before they overwrite its inputs (a wave's LDS accesses
// complete in issue order), so each wave needs one buffer.
//
// Roundings are those of the pass above: the first layer is formed to FP32
// accuracy on the matrix cores from three-way BF16 splits of x and W1
// (x = x0 + x1 + x2, 8 bits each; the six products x_i w_j with i + j <= 2,
// exact in the FP32 accumulator; the dropped ones are below 2^-24 of the
// sum), every hidden activation and the width x width weights are BF16,
// the output layer is an FP32 dot product with the last BF16 activations.
// SiLU uses the hardware exp2 and reciprocal (about 1 ulp of FP32 each,
// far below the BF16 rounding that follows).
constexpr int kWavesM = 8;  // waves per workgroup

__device__ __forceinline__ float silu_hw(float z) {
  const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * z);
  return z * __builtin_amdgcn_rcpf(1.0f + e);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Two FP32 values rounded to BF16 (nearest, ties to even) in one gfx950
// conversion (v_cvt_pk_bf16_f32), the first in the low half.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float float2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_pair(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(float2_t{a, b}, bf16x2_t));
}

__global__ void __launch_bounds__(64 * kWavesM) k_mlp_infer_mfma(
    int n, int n_mid, const float* __restrict__ x, const float* __restrict__ params,
    const uint16_t* __restrict__ wbf, float* __restrict__ y) {
  extern __shared__ uint64_t lds_q[];
  constexpr int kQ = kW * kW / 4;  // quads of one width x width matrix
  uint64_t* wq = lds_q;                                   // n_mid matrices
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  const int cell = lane % 32, half = lane / 32;
  uint64_t* act = lds_q + (size_t)n_mid * kQ + (size_t)wv * (kW * 32 / 4);
  // stage the hidden weights: W_l[f][4kq .. 4kq+3] is 8 contiguous bytes
  for (int q = threadIdx.x; q < n_mid * kQ; q += blockDim.x) {
    const int l = q / kQ, rem = q % kQ, kq = rem / kW, f = rem % kW;
    wq[q] = *reinterpret_cast<const uint64_t*>(wbf + (size_t)l * kW * kW + (size_t)f * kW + 4 * kq);
  }
  const float* W1 = params;
  const float* b1 = W1 + kW * kIn;
  const int64_t hid = (int64_t)kW * kW + kW;
  const float* last = b1 + kW + (int64_t)n_mid * hid;  // W_out [kW], then b_out
  // first-layer A operands in registers, three BF16 parts each:
  // A[f][k] = W1[mt 32 + cell][8 kt + 4 half + v], zero for k >= n_in
  short4_t a1[3][4][2];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = kt * 8 + 4 * half + v;
        float w = k < kIn ? W1[(mt * 32 + cell) * kIn + k] : 0.0f;
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          const uint16_t h = f2bf(w);
          a1[p][mt][kt][v] = (short)h;
          w = w - bf2f(h);
        }
      }
  __syncthreads();
  const int ntile = (n + 31) / 32;
  for (int tile = blockIdx.x * kWavesM + wv; tile < ntile; tile += gridDim.x * kWavesM) {
    const int c = tile * 32 + cell;
    // layer 1: B[k][cell] = x[c][k] for k = 8 kt + 4 half + v
    short4_t b1p[3][2];
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = kt * 8 + 4 * half + v;
        float xv = (c < n && k < kIn) ? x[(size_t)c * kIn + k] : 0.0f;
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          const uint16_t h = f2bf(xv);
          b1p[p][kt][v] = (short)h;
          xv = xv - bf2f(h);
        }
      }
    float16_t acc[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      acc[mt] = float16_t{0};
#pragma unroll
      for (int kt = 0; kt < 2; ++kt) {  // smallest products first
        acc[mt] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1[0][mt][kt], b1p[2][kt], acc[mt], 0, 0, 0);
        acc[mt] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1[1][mt][kt], b1p[1][kt], acc[mt], 0, 0, 0);
        acc[mt] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1[2][mt][kt], b1p[0][kt], acc[mt], 0, 0, 0);
        acc[mt] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1[0][mt][kt], b1p[1][kt], acc[mt], 0, 0, 0);
        acc[mt] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1[1][mt][kt], b1p[0][kt], acc[mt], 0, 0, 0);
        acc[mt] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1[0][mt][kt], b1p[0][kt], acc[mt], 0, 0, 0);
      }
    }
    const float* bias = b1;
    for (int l = 0;; ++l) {
      // SiLU of the accumulators (bias added), rounded to BF16
      if (l == n_mid) {  // the last hidden layer feeds the output layer
        float s = 0.0f;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
          for (int r = 0; r < 16; r += 2) {
            const int f = mt * 32 + 8 * (r / 4) + 4 * half + (r % 4);
            const uint32_t h = bf16_pair(silu_hw(acc[mt][r] + bias[f]),
                                         silu_hw(acc[mt][r + 1] + bias[f + 1]));
            s = s + last[f] * __uint_as_float(h << 16);
            s = s + last[f + 1] * __uint_as_float(h & 0xFFFF0000u);
          }
        s = s + __shfl_down(s, 32, 64);
        if (half == 0 && c < n) y[c] = s + last[kW];
        break;
      }
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int f0 = mt * 32 + 8 * q + 4 * half;
          float h[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) h[j] = silu_hw(acc[mt][4 * q + j] + bias[f0 + j]);
          act[(f0 / 4) * 32 + cell] =
              (uint64_t)bf16_pair(h[0], h[1]) | ((uint64_t)bf16_pair(h[2], h[3]) << 32);
        }
      // hidden layer l: out^T = W_l h^T, all four output tiles in registers
      const uint64_t* W = wq + (size_t)l * kQ;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) acc[mt] = float16_t{0};
#pragma unroll 4
      for (int kt = 0; kt < kW / 8; ++kt) {
        const short4_t b = __builtin_bit_cast(short4_t, act[(2 * kt + half) * 32 + cell]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          const short4_t a = __builtin_bit_cast(short4_t, W[(2 * kt + half) * kW + mt * 32 + cell]);
          acc[mt] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc[mt], 0, 0, 0);
        }
      }
      bias = b1 + kW + (int64_t)l * hid + kW * kW;
    }
  }
}

// ---------------------------------------------------------------- warm-start features
// Pressure fields are referenced to each pocket's current pin (p = 0 there):
// a previous field is re-referenced by subtracting its value at the pin of
// the cell's pocket (comp[c]), which removes the constant jump a pocket's
// pressure takes when its lowest cell, and so its pin, changes.
__global__ void k_ws_stats(int na, const int* __restrict__ perm, const int* __restrict__ comp,
                           const double* __restrict__ dp, const double* __restrict__ rhs,
                           const double* __restrict__ vol, double* __restrict__ partials) {
  double s[3] = {0.0, 0.0, 0.0};
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < na; r += gridDim.x * kBlock) {
    const int c = perm[r];
    const double d = dp[c] - dp[comp[c]];
    s[0] += d * d;
    s[1] += rhs[c] * rhs[c];
    s[2] += vol[c];
  }
  write_partials<kBlock, 3>(s, partials);
}

__global__ void k_ws_stats_final(const double* __restrict__ partials, int g, int na,
                                 double* __restrict__ out) {
  const double a = sum_partials<kBlock>(partials, g);
  const double b = sum_partials<kBlock>(partials + g, g);
  const double c = sum_partials<kBlock>(partials + 2 * g, g);
  if (threadIdx.x == 0) {
    out[0] = sqrt(a / na);  // RMS of the previous increment
    out[1] = sqrt(b / na);  // RMS of the right-hand side
    out[2] = c / na;        // mean cell volume
  }
}

// Features of active cell r (cell c), before standardisation:
//   0 previous increment (re-referenced) / its RMS, 1 rhs / its RMS, 2 liquid fraction,
//   3 volume / mean volume, 4..9 the six largest open-face coefficients of
//   the cell divided by their sum (descending, 0 where fewer).
__global__ void k_ws_features(int na, const int* __restrict__ perm, const int* __restrict__ comp,
                              const int* __restrict__ adj_ptr,
                              const int* __restrict__ adj_nbr, const int* __restrict__ adj_face,
                              const int* __restrict__ active, const double* __restrict__ dp,
                              const double* __restrict__ rhs, const double* __restrict__ fl,
                              const double* __restrict__ vol, const double* __restrict__ coeff,
                              const double* __restrict__ st, const float* __restrict__ mu,
                              const float* __restrict__ sigma, float* __restrict__ out) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= na) return;
  const int c = perm[r];
  float f[10];
  f[0] = st[0] > 0.0 ? (float)((dp[c] - dp[comp[c]]) / st[0]) : 0.0f;
  f[1] = st[1] > 0.0 ? (float)(rhs[c] / st[1]) : 0.0f;
  f[2] = (float)fl[c];
  f[3] = st[2] > 0.0 ? (float)(vol[c] / st[2]) : 0.0f;
  double top[6] = {0, 0, 0, 0, 0, 0};
  double sum = 0.0;
  for (int k = adj_ptr[c]; k < adj_ptr[c + 1]; ++k) {
    if (!active[adj_nbr[k]]) continue;
    double v = coeff[adj_face[k]];
    sum += v;
    for (int q = 0; q < 6; ++q)  // insert into the descending top-6
      if (v > top[q]) { double t = top[q]; top[q] = v; v = t; }
  }
  for (int q = 0; q < 6; ++q) f[4 + q] = sum > 0.0 ? (float)(top[q] / sum) : 0.0f;
#pragma unroll
  for (int k = 0; k < 10; ++k) out[(size_t)r * 10 + k] = (f[k] - mu[k]) / sigma[k];
}

// x0 = p_prev (re-referenced) + scale * y on active non-pin cells, 0 elsewhere
__global__ void k_ws_apply(int nc, const int* __restrict__ cid, const int* __restrict__ comp,
                           const double* __restrict__ p_prev, const float* __restrict__ yv,
                           double scale, double* __restrict__ x0) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= nc) return;
  const int r = cid[c];
  x0[c] = (r < 0 || comp[c] == c) ? 0.0 : (p_prev[c] - p_prev[comp[c]]) + scale * (double)yv[r];
}

// training target of active cell r: (p_new - p_prev re-referenced) / scale
__global__ void k_ws_targets(int na, const int* __restrict__ perm, const int* __restrict__ comp,
                             const double* __restrict__ p_new, const double* __restrict__ p_prev,
                             double scale, float* __restrict__ t) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= na) return;
  const int c = perm[r];
  t[r] = scale > 0.0 ? (float)((p_new[c] - (p_prev[c] - p_prev[comp[c]])) / scale) : 0.0f;
}

// ---------------------------------------------------------------- host side
// Workspace of ppe_warm_start_features_noalloc: the statistics' block
// partials (at most kRedBlocks per statistic) and the three statistics, in a
// static device array instead of solver memory.  Each device holds its own
// copy for the life of the process; host code reaches it only through the
// address hipGetSymbolAddress gives on that device (the array's name is a
// host-side stand-in there).
constexpr int kWsScratch = 3 * kRedBlocks + 3;
static __device__ __align__(256) double scratch[kWsScratch];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// The device address of `scratch` on `device`, looked up once per device
// with that device current.
double* ws_scratch(int device) {
  require(device >= 0 && device < kMaxDevices, PPE_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    int prev = -1;
    PPE_HIP(hipGetDevice(&prev));
    if (prev != device) PPE_HIP(hipSetDevice(device));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (prev != device) (void)hipSetDevice(prev);
    PPE_HIP(e);
    require(ptr != nullptr, PPE_ERR_HIP, "hipGetSymbolAddress gave no address for the workspace");
    g_scratch[device] = static_cast<double*>(ptr);
  }
  return g_scratch[device];
}

// The warm-start features of the assembled solver's active cells with the
// statistics' partials in `part` (3 red_grid(n_active) + 3 doubles, written
// before they are read: nothing needs clearing).  *dp_scale is copied to the
// host and the stream synchronised.
ppe_status ws_features(ppe_solver* s, const double* dp_prev, const double* rhs,
                       const double* face_coeff, const double* fl, const double* cell_volume,
                       const float* mu, const float* sigma, float* features, double* dp_scale,
                       double* part) {
  const int na = s->n_active;
  if (na == 0) {
    *dp_scale = 0.0;
    return PPE_OK;
  }
  const int g = red_grid(na);
  hipLaunchKernelGGL(k_ws_stats, dim3(g), dim3(kBlock), 0, s->stream, na, s->perm.as<int>(),
                     s->comp_full.as<int>(), dp_prev, rhs, cell_volume, part);
  PPE_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_ws_stats_final, dim3(1), dim3(kBlock), 0, s->stream, part, g, na,
                     part + 3 * g);
  PPE_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_ws_features, dim3(grid_for(na)), dim3(kBlock), 0, s->stream, na,
                     s->perm.as<int>(), s->comp_full.as<int>(), s->adj_ptr.as<int>(),
                     s->adj_nbr.as<int>(), s->adj_face.as<int>(), s->active.as<int>(), dp_prev,
                     rhs, fl, cell_volume, face_coeff, part + 3 * g, mu, sigma, features);
  PPE_LAUNCH_CHECK();
  PPE_HIP(hipMemcpyAsync(dp_scale, part + 3 * g, sizeof(double), hipMemcpyDeviceToHost,
                         s->stream));
  PPE_HIP(hipStreamSynchronize(s->stream));
  return PPE_OK;
}

void gemm(ppe_mlp* m, int M, int N, int K, const float* A, int64_t ari, int64_t ack,
          const float* B, int64_t brk, int64_t bcj, float* C, int chunk_rows = 0) {
  const int kc = chunk_rows > 0 ? chunk_rows : K;
  const int nz = (K + kc - 1) / kc;
  dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM, nz > 0 ? nz : 1);
  if (nz <= 1) {
    hipLaunchKernelGGL(k_sgemm, grid, dim3(256), 0, m->stream, M, N, K, kc, A, ari, ack, B, brk,
                       bcj, C);
    PPE_LAUNCH_CHECK();
    return;
  }
  float* parts = m->part.get<float>((size_t)nz * M * N);
  hipLaunchKernelGGL(k_sgemm, grid, dim3(256), 0, m->stream, M, N, K, kc, A, ari, ack, B, brk, bcj,
                     parts);
  PPE_LAUNCH_CHECK();
  const int64_t len = (int64_t)M * N;
  hipLaunchKernelGGL(k_sum_chunks, dim3(grid_for(len)), dim3(kBlock), 0, m->stream, len, nz, parts,
                     C);
  PPE_LAUNCH_CHECK();
}

constexpr int kChunkRows = 4096;  // rows per split-K chunk of the weight gradients

// FP32 forward of n rows; keeps pre-activations and activations for backward.
// Returns the pointer to y [n].
float* forward_fp32(ppe_mlp* m, int n, const float* x) {
  const int L = (int)m->dims.size() - 1;
  int64_t tot = 0;
  for (int l = 1; l <= L; ++l) tot += (int64_t)n * m->dims[l];
  float* act = m->act.get<float>(tot);
  float* pre = m->pre.get<float>(tot);
  float* tmp = m->gbuf2.get<float>((size_t)n * m->width > (size_t)n ? (size_t)n * m->width : n);
  const float* P = m->params.as<float>();
  const float* h = x;
  int64_t off = 0;
  for (int l = 0; l < L; ++l) {
    const int in = m->dims[l], out = m->dims[l + 1];
    // tmp [n x out] = h [n x in] W^T  (W [out][in])
    gemm(m, n, out, in, h, in, 1, P + m->woff[l], 1, in, tmp);
    const int64_t len = (int64_t)n * out;
    hipLaunchKernelGGL(k_bias_act, dim3(grid_for(len)), dim3(kBlock), 0, m->stream, (int64_t)n, out,
                       tmp, P + m->boff[l], pre + off, act + off, l < L - 1 ? 1 : 0);
    PPE_LAUNCH_CHECK();
    h = act + off;
    off += len;
  }
  return act + off - n;
}

// Mean-squared-error loss (host) and the packed gradient into m->grad.
double loss_grad(ppe_mlp* m, int n, const float* x, const float* t) {
  const int L = (int)m->dims.size() - 1;
  float* y = forward_fp32(m, n, x);
  float* G = m->gbuf.get<float>((size_t)n * m->width > (size_t)n ? (size_t)n * m->width : n);
  float* G2 = m->gbuf2.get<float>((size_t)n * m->width > (size_t)n ? (size_t)n * m->width : n);
  const int gl = red_grid(n);
  double* lp = m->lossbuf.get<double>((size_t)gl + 1);
  hipLaunchKernelGGL(k_loss_grad, dim3(gl), dim3(kBlock), 0, m->stream, n, y, t, G, lp);
  PPE_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_finalize_loss, dim3(1), dim3(kBlock), 0, m->stream, lp, gl, n, lp + gl);
  PPE_LAUNCH_CHECK();
  const float* P = m->params.as<float>();
  float* dP = m->grad.get<float>(m->n_params);
  // offsets of each layer's activations in act/pre
  std::vector<int64_t> aoff(L + 1, 0);
  for (int l = 1; l <= L; ++l) aoff[l] = aoff[l - 1] + (int64_t)n * m->dims[l];
  const float* act = m->act.as<float>();
  const float* pre = m->pre.as<float>();
  for (int l = L - 1; l >= 0; --l) {
    const int in = m->dims[l], out = m->dims[l + 1];
    const float* hin = l == 0 ? x : act + aoff[l - 1];
    // dW [out x in] = G^T [out x n] . hin [n x in]   (sum over rows, split-K)
    gemm(m, out, in, n, G, 1, out, hin, in, 1, dP + m->woff[l], kChunkRows);
    // db [out] = column sums of G
    // bias gradient: column sums over chunks of at least kColRows rows (at
    // most kColChunks chunks), the chunks then added in order
    const int crow = std::max(kColRows, (n + kColChunks - 1) / kColChunks);
    const int nz = (n + crow - 1) / crow;
    float* parts = m->part.get<float>((size_t)nz * out);
    hipLaunchKernelGGL(k_colsum_chunks, dim3((out + kBlock - 1) / kBlock, nz), dim3(kBlock), 0,
                       m->stream, n, out, crow, G, parts);
    PPE_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_chunks, dim3(grid_for(out)), dim3(kBlock), 0, m->stream, (int64_t)out,
                       nz, parts, dP + m->boff[l]);
    PPE_LAUNCH_CHECK();
    if (l > 0) {
      // G2 [n x in] = G [n x out] . W [out x in], then times silu'(z_{l-1})
      gemm(m, n, in, out, G, out, 1, P + m->woff[l], in, 1, G2);
      const int64_t len = (int64_t)n * in;
      hipLaunchKernelGGL(k_dsilu_mul, dim3(grid_for(len)), dim3(kBlock), 0, m->stream, len,
                         pre + aoff[l - 1], G2);
      PPE_LAUNCH_CHECK();
      std::swap(G, G2);
    }
  }
  double loss = 0.0;
  PPE_HIP(hipMemcpyAsync(&loss, lp + gl, sizeof(double), hipMemcpyDeviceToHost, m->stream));
  PPE_HIP(hipStreamSynchronize(m->stream));
  return loss;
}

void refresh_bf16(ppe_mlp* m) {
  if (m->n_in != kIn || m->width != kW || m->n_hidden < 1) return;
  const int nh = m->n_hidden - 1;  // width x width matrices
  if (nh <= 0) return;
  uint16_t* w = m->bf16.get<uint16_t>((size_t)nh * kW * kW);
  for (int l = 0; l < nh; ++l) {
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_for((int64_t)kW * kW)), dim3(kBlock), 0, m->stream,
                       (int64_t)kW * kW, m->params.as<float>() + m->woff[l + 1],
                       w + (size_t)l * kW * kW);
    PPE_LAUNCH_CHECK();
  }
}

template <class F>
ppe_status mlp_guard(ppe_mlp* m, F&& f) {
  try {
    if (m) m->err.clear();
    return f();
  } catch (const Error& e) {
    if (m) m->err = e.what();
    return e.status;
  } catch (const std::exception& e) {
    if (m) m->err = e.what();
    return PPE_ERR_INTERNAL;
  }
}

}  // namespace
}  // namespace ppe

using namespace ppe;

extern "C" {

ppe_status ppe_mlp_create(int32_t n_in, int32_t width, int32_t n_hidden, void* stream,
                          ppe_mlp** out) {
  if (!out) return PPE_ERR_ARG;
  *out = nullptr;
  if (n_in < 1 || width < 1 || n_hidden < 1 || width > 4096 || n_in > 4096) return PPE_ERR_ARG;
  auto* m = new ppe_mlp();
  m->n_in = n_in;
  m->width = width;
  m->n_hidden = n_hidden;
  m->stream = static_cast<hipStream_t>(stream);
  m->dims.push_back(n_in);
  for (int k = 0; k < n_hidden; ++k) m->dims.push_back(width);
  m->dims.push_back(1);
  int64_t off = 0;
  for (size_t l = 0; l + 1 < m->dims.size(); ++l) {
    m->woff.push_back(off);
    off += (int64_t)m->dims[l + 1] * m->dims[l];
    m->boff.push_back(off);
    off += m->dims[l + 1];
  }
  m->n_params = off;
  ppe_status st = mlp_guard(m, [&]() -> ppe_status {
    float* p = m->params.get<float>(off);
    float* mm = m->m.get<float>(off);
    float* vv = m->v.get<float>(off);
    PPE_HIP(hipMemsetAsync(p, 0, sizeof(float) * off, m->stream));
    PPE_HIP(hipMemsetAsync(mm, 0, sizeof(float) * off, m->stream));
    PPE_HIP(hipMemsetAsync(vv, 0, sizeof(float) * off, m->stream));
    PPE_HIP(hipStreamSynchronize(m->stream));
    return PPE_OK;
  });
  if (st != PPE_OK) {
    delete m;
    return st;
  }
  *out = m;
  return PPE_OK;
}

void ppe_mlp_destroy(ppe_mlp* m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->stream);
  delete m;
}

int64_t ppe_mlp_num_params(const ppe_mlp* m) { return m ? m->n_params : -1; }

const char* ppe_mlp_last_error(const ppe_mlp* m) { return m ? m->err.c_str() : ""; }

ppe_status ppe_mlp_set_params(ppe_mlp* m, const float* params) {
  if (!m || !params) return PPE_ERR_ARG;
  return mlp_guard(m, [&]() -> ppe_status {
    PPE_HIP(hipMemcpyAsync(m->params.as<float>(), params, sizeof(float) * m->n_params,
                           hipMemcpyDeviceToDevice, m->stream));
    PPE_HIP(hipMemsetAsync(m->m.as<float>(), 0, sizeof(float) * m->n_params, m->stream));
    PPE_HIP(hipMemsetAsync(m->v.as<float>(), 0, sizeof(float) * m->n_params, m->stream));
    m->adam_t = 0;
    refresh_bf16(m);
    PPE_HIP(hipStreamSynchronize(m->stream));
    return PPE_OK;
  });
}

ppe_status ppe_mlp_get_params(const ppe_mlp* m, float* params) {
  if (!m || !params) return PPE_ERR_ARG;
  ppe_mlp* mm = const_cast<ppe_mlp*>(m);
  return mlp_guard(mm, [&]() -> ppe_status {
    PPE_HIP(hipMemcpyAsync(params, m->params.as<float>(), sizeof(float) * m->n_params,
                           hipMemcpyDeviceToDevice, m->stream));
    PPE_HIP(hipStreamSynchronize(m->stream));
    return PPE_OK;
  });
}

ppe_status ppe_mlp_forward(ppe_mlp* m, int32_t n, const float* x, float* y, int bf16) {
  if (!m || n < 0 || (n > 0 && (!x || !y))) return PPE_ERR_ARG;
  if (n == 0) return PPE_OK;
  return mlp_guard(m, [&]() -> ppe_status {
    if (bf16) {
      require(m->n_in == kIn && m->width == kW && m->n_hidden >= 2, PPE_ERR_ARG,
              "the BF16 MFMA path needs 10 inputs, width 128 and >= 2 hidden layers");
      const int tiles = (n + 31) / 32;
      const int n_mid = m->n_hidden - 1;
      const size_t lds = ((size_t)n_mid * kW * kW / 4 + (size_t)kWavesM * kW * 32 / 4) * 8;
      if (m->lds_max == 0) {
        int dev = 0, v = 0;
        PPE_HIP(hipGetDevice(&dev));
        PPE_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        int cus = 0;
        PPE_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        m->lds_max = (size_t)v;
        m->cus = cus;
      }
      if (lds <= m->lds_max) {
        // one workgroup per compute unit holds the staged weights; waves
        // stride over the 32-cell tiles
        int g = (tiles + kWavesM - 1) / kWavesM;
        if (g > m->cus) g = m->cus;
        hipLaunchKernelGGL(k_mlp_infer_mfma, dim3(g), dim3(64 * kWavesM), lds, m->stream, n,
                           n_mid, x, m->params.as<float>(), m->bf16.as<uint16_t>(), y);
      } else {  // deeper networks than the staged weights fit
        int g = (tiles + kWaves - 1) / kWaves;
        if (g > 2048) g = 2048;
        hipLaunchKernelGGL(k_mlp_infer_bf16, dim3(g), dim3(64 * kWaves), 0, m->stream, n,
                           m->n_hidden, x, m->params.as<float>(), m->bf16.as<uint16_t>(), y);
      }
      PPE_LAUNCH_CHECK();
    } else {
      float* yy = forward_fp32(m, n, x);
      PPE_HIP(hipMemcpyAsync(y, yy, sizeof(float) * n, hipMemcpyDeviceToDevice, m->stream));
    }
    PPE_HIP(hipStreamSynchronize(m->stream));
    return PPE_OK;
  });
}

ppe_status ppe_mlp_loss_grad(ppe_mlp* m, int32_t n, const float* x, const float* t, float* grad,
                             double* loss) {
  if (!m || n < 1 || !x || !t || !grad) return PPE_ERR_ARG;
  return mlp_guard(m, [&]() -> ppe_status {
    const double l = loss_grad(m, n, x, t);
    PPE_HIP(hipMemcpyAsync(grad, m->grad.as<float>(), sizeof(float) * m->n_params,
                           hipMemcpyDeviceToDevice, m->stream));
    PPE_HIP(hipStreamSynchronize(m->stream));
    if (loss) *loss = l;
    return PPE_OK;
  });
}

ppe_status ppe_mlp_train_step(ppe_mlp* m, int32_t n, const float* x, const float* t, float lr,
                              double* loss) {
  if (!m || n < 1 || !x || !t || !(lr > 0)) return PPE_ERR_ARG;
  return mlp_guard(m, [&]() -> ppe_status {
    const double l = loss_grad(m, n, x, t);
    m->adam_t += 1;
    const float c1 = 1.0f - std::pow(0.9f, (float)m->adam_t);
    const float c2 = 1.0f - std::pow(0.999f, (float)m->adam_t);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(m->n_params)), dim3(kBlock), 0, m->stream, m->n_params,
                       m->params.as<float>(), m->grad.as<float>(), m->m.as<float>(),
                       m->v.as<float>(), lr, c1, c2);
    PPE_LAUNCH_CHECK();
    refresh_bf16(m);
    PPE_HIP(hipStreamSynchronize(m->stream));
    if (loss) *loss = l;
    return PPE_OK;
  });
}

ppe_status ppe_warm_start_features(ppe_solver* s, const double* dp_prev, const double* rhs,
                                   const double* face_coeff, const double* fl,
                                   const double* cell_volume, const float* mu, const float* sigma,
                                   float* features, double* dp_scale) {
  if (!s || !dp_prev || !rhs || !face_coeff || !fl || !cell_volume || !mu || !sigma || !features ||
      !dp_scale)
    return PPE_ERR_ARG;
  if (!s->assembled || s->shifted) return PPE_ERR_STATE;  // needs a pinned pressure system
  AllocScope scope(&s->allocator);
  try {
    const int na = s->n_active;
    double* part =
        na > 0 ? s->tmp_d[0].get<double>((size_t)3 * red_grid(na) + 3) : nullptr;
    return ppe::ws_features(s, dp_prev, rhs, face_coeff, fl, cell_volume, mu, sigma, features,
                            dp_scale, part);
  } catch (const Error& e) {
    s->err = e.what();
    return e.status;
  }
}

ppe_status ppe_warm_start_features_noalloc(ppe_solver* s, const double* dp_prev,
                                           const double* rhs, const double* face_coeff,
                                           const double* fl, const double* cell_volume,
                                           const float* mu, const float* sigma, float* features,
                                           double* dp_scale) {
  if (!s || !dp_prev || !rhs || !face_coeff || !fl || !cell_volume || !mu || !sigma || !features ||
      !dp_scale)
    return PPE_ERR_ARG;
  if (!s->assembled || s->shifted) return PPE_ERR_STATE;  // needs a pinned pressure system
  try {
    const int na = s->n_active;
    const size_t need = na > 0 ? (size_t)3 * red_grid(na) + 3 : 0;
    require(need <= (size_t)ppe::kWsScratch, PPE_ERR_ARG,
            "ppe_warm_start_features_noalloc: " + std::to_string(need) +
                " workspace doubles needed, the static workspace holds " +
                std::to_string(ppe::kWsScratch));
    double* part = na > 0 ? ppe::ws_scratch(s->device) : nullptr;
    return ppe::ws_features(s, dp_prev, rhs, face_coeff, fl, cell_volume, mu, sigma, features,
                            dp_scale, part);
  } catch (const Error& e) {
    s->err = e.what();
    return e.status;
  }
}

ppe_status ppe_warm_start_apply(ppe_solver* s, const double* p_prev, const float* y,
                                double dp_scale, double* x0) {
  if (!s || !p_prev || !x0 || (s->n_active > 0 && !y)) return PPE_ERR_ARG;
  if (!s->assembled || s->shifted) return PPE_ERR_STATE;  // needs a pinned pressure system
  try {
    hipLaunchKernelGGL(k_ws_apply, dim3(grid_for(s->n_cells)), dim3(kBlock), 0, s->stream,
                       s->n_cells, s->cid.as<int>(), s->comp_full.as<int>(), p_prev, y, dp_scale,
                       x0);
    PPE_LAUNCH_CHECK();
    PPE_HIP(hipStreamSynchronize(s->stream));
    return PPE_OK;
  } catch (const Error& e) {
    s->err = e.what();
    return e.status;
  }
}

ppe_status ppe_warm_start_targets(ppe_solver* s, const double* p_new, const double* p_prev,
                                  double dp_scale, float* targets) {
  if (!s || !p_new || !p_prev || (s->n_active > 0 && !targets)) return PPE_ERR_ARG;
  if (!s->assembled || s->shifted) return PPE_ERR_STATE;  // needs a pinned pressure system
  try {
    if (s->n_active) {
      hipLaunchKernelGGL(k_ws_targets, dim3(grid_for(s->n_active)), dim3(kBlock), 0, s->stream,
                         s->n_active, s->perm.as<int>(), s->comp_full.as<int>(), p_new, p_prev,
                         dp_scale, targets);
      PPE_LAUNCH_CHECK();
    }
    PPE_HIP(hipStreamSynchronize(s->stream));
    return PPE_OK;
  } catch (const Error& e) {
    s->err = e.what();
    return e.status;
  }
}

}  // extern "C"

// Device primitives: exclusive scan of int32 counts (three-pass, int64
// carries), integer max reduction and fills.
#include "common.h"

namespace ppe {
namespace {

constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ long long wave_incl_scan(long long v) {
  const int lane = threadIdx.x % kWave;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    long long u = __shfl_up(v, o, kWave);
    if (lane >= o) v += u;
  }
  return v;
}

// Exclusive scan across a block of kBlock threads; *total receives the sum.
__device__ __forceinline__ long long block_excl_scan(long long v, long long* total) {
  __shared__ long long wsum[kBlock / kWave];
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  long long inc = wave_incl_scan(v);
  if (lane == kWave - 1) wsum[w] = inc;
  __syncthreads();
  long long off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kBlock / kWave; ++i) {
    if (i < w) off += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

__global__ void __launch_bounds__(kBlock) k_scan_reduce(const int* __restrict__ in, int n,
                                                        long long* __restrict__ bsum) {
  const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
  long long s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    long long i = base + k;
    if (i < n) s += in[i];
  }
  s = block_sum<kBlock>(s);
  if (threadIdx.x == 0) bsum[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock) k_scan_top(long long* __restrict__ bsum, int nb,
                                                     long long* __restrict__ total) {
  long long carry = 0;
  for (int base = 0; base < nb; base += kBlock) {
    int i = base + threadIdx.x;
    long long v = i < nb ? bsum[i] : 0;
    long long t;
    long long ex = block_excl_scan(v, &t);
    if (i < nb) bsum[i] = carry + ex;
    carry += t;
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(kBlock) k_scan_down(const int* __restrict__ in, int n,
                                                      const long long* __restrict__ boff,
                                                      const long long* __restrict__ total,
                                                      int* __restrict__ out) {
  const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
  int v[kScanItems];
  long long s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    long long i = base + k;
    v[k] = i < n ? in[i] : 0;
    s += v[k];
  }
  long long t;
  long long run = block_excl_scan(s, &t) + boff[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    long long i = base + k;
    if (i < n) out[i] = (int)run;
    run += v[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = (int)*total;
}

__global__ void __launch_bounds__(kBlock) k_max_int(const int* __restrict__ in, int n,
                                                    int* __restrict__ out) {
  int m = INT32_MIN;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
    m = max(m, in[i]);
  m = block_max<kBlock>(m);
  if (threadIdx.x == 0) atomicMax(out, m);
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_fill(T* __restrict__ p, T v, long long n) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    p[i] = v;
}

}  // namespace

int scan_blocks(int n) {
  int nb = (int)((n + (int64_t)kScanTile - 1) / kScanTile);
  return nb < 1 ? 1 : nb;
}

long long* exclusive_scan_async(ppe_solver* s, const int* in, int* out, int n, int slot) {
  if (n < 0) throw Error(PPE_ERR_INTERNAL, "negative scan length");
  const int nb = scan_blocks(n);
  long long* bsum = s->tmp_l[slot].get<long long>(nb + 1);
  long long* total = bsum + nb;
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, s->stream, in, n, bsum);
  PPE_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s->stream, bsum, nb, total);
  PPE_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kBlock), 0, s->stream, in, n, bsum, total, out);
  PPE_LAUNCH_CHECK();
  return total;
}

int64_t exclusive_scan(ppe_solver* s, const int* in, int* out, int n) {
  if (n < 0) throw Error(PPE_ERR_INTERNAL, "negative scan length");
  int nb = (int)((n + (int64_t)kScanTile - 1) / kScanTile);
  if (nb < 1) nb = 1;
  long long* bsum = s->tmp_l[0].get<long long>(nb + 1);
  long long* total = bsum + nb;
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, s->stream, in, n, bsum);
  PPE_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s->stream, bsum, nb, total);
  PPE_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kBlock), 0, s->stream, in, n, bsum, total, out);
  PPE_LAUNCH_CHECK();
  long long t = read_scalar(s, total);
  if (t > INT32_MAX) throw Error(PPE_ERR_INTERNAL, "scan total exceeds int32 range");
  return t;
}

void max_int_async(ppe_solver* s, const int* in, int n, int* out) {
  fill_int(s, out, INT32_MIN, 1);
  int g = grid_for(n);
  if (g > 1024) g = 1024;
  hipLaunchKernelGGL(k_max_int, dim3(g), dim3(kBlock), 0, s->stream, in, n, out);
  PPE_LAUNCH_CHECK();
}

int reduce_max_int(ppe_solver* s, const int* in, int n) {
  int* out = s->tmp_i[3].get<int>(1);
  fill_int(s, out, INT32_MIN, 1);
  int g = grid_for(n);
  if (g > 1024) g = 1024;
  hipLaunchKernelGGL(k_max_int, dim3(g), dim3(kBlock), 0, s->stream, in, n, out);
  PPE_LAUNCH_CHECK();
  return read_scalar(s, out);
}

void fill_int(ppe_solver* s, int* p, int v, int64_t n) {
  if (n <= 0) return;
  int g = grid_for(n);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_fill<int>, dim3(g), dim3(kBlock), 0, s->stream, p, v, (long long)n);
  PPE_LAUNCH_CHECK();
}

void fill_double(ppe_solver* s, double* p, double v, int64_t n) {
  if (n <= 0) return;
  int g = grid_for(n);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_fill<double>, dim3(g), dim3(kBlock), 0, s->stream, p, v, (long long)n);
  PPE_LAUNCH_CHECK();
}

}  // namespace ppe

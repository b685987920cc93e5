// Device primitives: exclusive scan of int32 counts (three-pass, int64
// carries), integer max reduction and fills.
#include <algorithm>
#include <cstring>

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

// Block sums of the counts and, with bmax, block maxima (the scan then also
// delivers the largest count, which the callers need beside the total).
__global__ void __launch_bounds__(kBlock) k_scan_reduce(const int* __restrict__ in, int n,
                                                        long long* __restrict__ bsum,
                                                        int* __restrict__ bmax) {
  const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
  long long s = 0;
  int m = INT32_MIN;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    long long i = base + k;
    if (i < n) {
      const int v = in[i];
      s += v;
      m = max(m, v);
    }
  }
  s = block_sum<kBlock>(s);
  if (threadIdx.x == 0) bsum[blockIdx.x] = s;
  if (bmax) {
    m = block_max<kBlock>(m);
    if (threadIdx.x == 0) bmax[blockIdx.x] = m;
  }
}

// Scan of the block sums; with mx, the largest block maximum is max-ed into
// *mx (as k_max_int does).
__global__ void __launch_bounds__(kBlock) k_scan_top(long long* __restrict__ bsum, int nb,
                                                     long long* __restrict__ total,
                                                     const int* __restrict__ bmax,
                                                     int* __restrict__ mx) {
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
  if (mx) {
    int m = INT32_MIN;
    for (int i = threadIdx.x; i < nb; i += kBlock) m = max(m, bmax[i]);
    m = block_max<kBlock>(m);
    if (threadIdx.x == 0) atomicMax(mx, m);
  }
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

// Exclusive scan of n <= kSmallScan counts by one block of kSmallBlock
// threads: the counts are staged in LDS with coalesced loads, each thread
// scans a run of consecutive items there, and the offsets leave through LDS
// with coalesced stores.  out[0..n], *total.
constexpr int kSmallBlock = 1024;
constexpr int kSmallItems = 15;  // staging buffer + wave sums stay under 64 KiB of LDS
constexpr int kSmallScan = kSmallBlock * kSmallItems;

__global__ void __launch_bounds__(kSmallBlock) k_scan_small(const int* __restrict__ in, int n,
                                                            int* __restrict__ out,
                                                            long long* __restrict__ total,
                                                            int* __restrict__ mx) {
  __shared__ int buf[kSmallScan];
  __shared__ long long wsum[kSmallBlock / kWave];
  int m = INT32_MIN;
  for (int i = threadIdx.x; i < n; i += kSmallBlock) {
    const int v = in[i];
    buf[i] = v;
    m = max(m, v);
  }
  if (mx) {  // the largest count, max-ed into *mx as k_max_int does
    m = block_max<kSmallBlock>(m);
    if (threadIdx.x == 0) atomicMax(mx, m);
  }
  __syncthreads();
  const int per = (n + kSmallBlock - 1) / kSmallBlock;  // <= kSmallItems
  const int base = threadIdx.x * per;
  long long run = 0;
  for (int k = 0; k < per; ++k) {
    const int i = base + k;
    if (i < n) run += buf[i];
  }
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const long long inc = wave_incl_scan(run);
  if (lane == kWave - 1) wsum[w] = inc;
  __syncthreads();
  long long off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kSmallBlock / kWave; ++i) {
    if (i < w) off += wsum[i];
    tot += wsum[i];
  }
  long long pos = off + inc - run;
  for (int k = 0; k < per; ++k) {
    const int i = base + k;
    if (i < n) {
      const int v = buf[i];
      buf[i] = (int)pos;  // this thread's own items only: no other thread reads them now
      pos += v;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kSmallBlock) out[i] = buf[i];
  if (threadIdx.x == 0) {
    out[n] = (int)tot;
    *total = tot;
  }
}

__global__ void __launch_bounds__(kBlock) k_max_int(const int* __restrict__ in, int n,
                                                    int* __restrict__ out) {
  int m = INT32_MIN;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
    m = max(m, in[i]);
  m = block_max<kBlock>(m);
  if (threadIdx.x == 0) atomicMax(out, m);
}

// Read-back staging: item k (kPubMax at most) is off[k+1] - off[k] words at
// src[k], copied to dst[off[k]..] in the pinned host box.
constexpr int kPubMax = 16;
struct PubArgs {
  const uint32_t* src[kPubMax];
  uint32_t off[kPubMax + 1];
  int n;
};

// After the items, dst[off[n]] receives `tag`, stored only once every word is
// visible at system scope: a host that reads the tag it expects, then the
// words, reads this call's values.
__global__ void __launch_bounds__(kBlock) k_publish(PubArgs a, uint32_t tag,
                                                    uint32_t* __restrict__ dst) {
  for (int k = 0; k < a.n; ++k) {
    const uint32_t* src = a.src[k];
    const uint32_t o = a.off[k], len = a.off[k + 1] - o;
    for (uint32_t w = threadIdx.x; w < len; w += kBlock) dst[o + w] = src[w];
  }
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(dst + a.off[a.n], tag, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
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

long long* exclusive_scan_async(ppe_solver* s, const int* in, int* out, int n, int slot,
                                int* max_out) {
  if (n < 0) throw Error(PPE_ERR_INTERNAL, "negative scan length");
  if (n <= kSmallScan) {
    long long* total = s->tmp_l[slot].get<long long>(2) + 1;
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(kSmallBlock), 0, s->stream, in, n, out, total,
                       max_out);
    PPE_LAUNCH_CHECK();
    return total;
  }
  const int nb = scan_blocks(n);
  // block sums, the total, then (with max_out) the block maxima as ints
  long long* bsum = s->tmp_l[slot].get<long long>(nb + 1 + (max_out ? (nb + 1) / 2 : 0));
  long long* total = bsum + nb;
  int* bmax = max_out ? reinterpret_cast<int*>(total + 1) : nullptr;
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, s->stream, in, n, bsum, bmax);
  PPE_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s->stream, bsum, nb, total,
                     (const int*)bmax, max_out);
  PPE_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kBlock), 0, s->stream, in, n, bsum, total, out);
  PPE_LAUNCH_CHECK();
  return total;
}

int64_t exclusive_scan(ppe_solver* s, const int* in, int* out, int n) {
  const long long* total = exclusive_scan_async(s, in, out, n, 0);
  long long t = read_scalar(s, total);
  if (t > INT32_MAX) throw Error(PPE_ERR_INTERNAL, "scan total exceeds int32 range");
  return t;
}

void max_int_async(ppe_solver* s, const int* in, int n, int* out, bool init) {
  if (init) fill_int(s, out, INT32_MIN, 1);
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

void ensure_box(ppe_solver* s, size_t words) {
  if (words <= s->box_words) return;
  size_t cap = s->box_words ? s->box_words : 4096;
  while (cap < words) cap *= 2;
  if (s->box_h) {
    // kernels in flight may still write the old box
    PPE_HIP(hipStreamSynchronize(s->stream));
    PPE_HIP(hipHostFree(s->box_h));
    s->box_h = s->box_d = nullptr;
    s->box_words = 0;
  }
  void* h = nullptr;
  PPE_HIP(hipHostMalloc(&h, cap * sizeof(uint32_t), hipHostMallocMapped | hipHostMallocCoherent));
  void* d = nullptr;
  PPE_HIP(hipHostGetDevicePointer(&d, h, 0));
  s->box_h = static_cast<uint32_t*>(h);
  s->box_d = static_cast<uint32_t*>(d);
  s->box_words = cap;
}

Published publish(ppe_solver* s, const ReadItem* items, int n, size_t at) {
  if (n > kPubMax) throw Error(PPE_ERR_INTERNAL, "too many read-back items in one call");
  PubArgs a{};
  a.n = n;
  uint32_t off = 0;
  for (int k = 0; k < n; ++k) {
    if (items[k].bytes % 4 != 0) throw Error(PPE_ERR_INTERNAL, "read-back size not a word multiple");
    a.src[k] = static_cast<const uint32_t*>(items[k].dev);
    a.off[k] = off;
    off += (uint32_t)(items[k].bytes / 4);
  }
  a.off[n] = off;
  ensure_box(s, at + off + 1);
  const uint32_t tag = ++s->box_tag;
  hipLaunchKernelGGL(k_publish, dim3(1), dim3(kBlock), 0, s->stream, a, tag, s->box_d + at);
  PPE_LAUNCH_CHECK();
  return Published{s->box_h + at, off, tag};
}

const uint32_t* published_words(ppe_solver* s, const Published& p) {
  auto tag_now = [&]() {
    return __atomic_load_n(p.words + p.n_words, __ATOMIC_ACQUIRE);
  };
  if (tag_now() != p.tag) {
    // the wait that preceded this call covered the kernel: drain the stream
    // and look once more before giving up
    PPE_HIP(hipStreamSynchronize(s->stream));
    if (tag_now() != p.tag) throw Error(PPE_ERR_INTERNAL, "read-back values not visible to the host");
  }
  return p.words;
}

void read_back(ppe_solver* s, std::initializer_list<ReadItem> items) {
  const std::vector<ReadItem> all(items);
  const Published pub = publish(s, all.data(), (int)all.size(), kBoxRead);
  PPE_HIP(hipStreamSynchronize(s->stream));
  const uint32_t* h = published_words(s, pub);
  for (const auto& it : all) {
    std::memcpy(it.host, h, it.bytes);
    h += it.bytes / 4;
  }
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

// Shared infrastructure of the pressure-solve library: error handling,
// grow-only device buffers, the solver state, and device primitives
// (wave64 reductions and scans, the MIS-2 priority hash).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <array>
#include <map>
#include <vector>
#include <utility>

#include "../../include/ppe.h"

namespace ppe {

constexpr int kBlock = 256;   // threads per workgroup for streaming kernels
constexpr int kWave = 64;     // CDNA wavefront width

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  ppe_status status;
  Error(ppe_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define PPE_HIP(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      if (e_ == hipErrorOutOfMemory)                                               \
        throw ::ppe::Error(PPE_ERR_OOM, std::string(#expr) + ": out of memory");   \
      throw ::ppe::Error(PPE_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    }                                                                              \
  } while (0)

#define PPE_LAUNCH_CHECK() PPE_HIP(hipGetLastError())

inline void require(bool ok, ppe_status st, const std::string& msg) {
  if (!ok) throw Error(st, msg);
}

// ---------------------------------------------------------------- buffers
// Where device memory comes from: hipMalloc/hipFree, or the caller's
// allocator of ppe_options.  An object that owns buffers (a solver, a
// time-step driver) holds one Allocator for its whole life; each API call
// makes it current for the calling thread (AllocScope), and every buffer
// keeps the allocator it was taken from, so it is released the same way.
struct Allocator {
  ppe_alloc_fn alloc = nullptr;
  ppe_free_fn free = nullptr;
  void* ctx = nullptr;
  void* stream = nullptr;             // passed to alloc
  const hipStream_t* drain[3] = {};   // streams whose work may still use a block
  void* take(size_t bytes) const {
    void* p = alloc(bytes, stream, ctx);
    if (!p) throw Error(PPE_ERR_OOM, "the caller's allocator returned NULL for " +
                                         std::to_string(bytes) + " bytes");
    return p;
  }
  void give_back(void* p) const {
    for (const hipStream_t* s : drain)
      if (s) (void)hipStreamSynchronize(*s);
    free(p, ctx);
  }
};
inline thread_local const Allocator* tl_alloc = nullptr;  // the call in progress
struct AllocScope {
  const Allocator* prev;
  explicit AllocScope(const Allocator* a) : prev(tl_alloc) {
    tl_alloc = (a && a->alloc) ? a : nullptr;
  }
  ~AllocScope() { tl_alloc = prev; }
  AllocScope(const AllocScope&) = delete;
  AllocScope& operator=(const AllocScope&) = delete;
};

// Grow-only device allocation: reassembling with a new mask reuses memory.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  const Allocator* al = nullptr;  // nullptr: taken from hipMalloc
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), cap(o.cap), al(o.al) {
    o.p = nullptr;
    o.cap = 0;
    o.al = nullptr;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; cap = o.cap; al = o.al;
      o.p = nullptr; o.cap = 0; o.al = nullptr;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) {
      if (al)
        al->give_back(p);
      else
        (void)hipFree(p);
    }
    p = nullptr;
    cap = 0;
    al = nullptr;
  }
  template <class T>
  T* get(size_t n) {
    size_t bytes = (n ? n : 1) * sizeof(T);
    if (bytes > cap) {
      release();
      size_t want = bytes + bytes / 8;  // slack so a slowly growing size does not realloc each time
      if (tl_alloc) {
        p = tl_alloc->take(want);
        al = tl_alloc;
      } else {
        PPE_HIP(hipMalloc(&p, want));
      }
      cap = want;
    }
    return static_cast<T*>(p);
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// CSR matrix on the device (sorted columns; square levels store their diagonal).
struct Csr {
  int n = 0, m = 0;   // rows, columns
  int64_t nnz = 0;
  int maxrow = 0;     // host-known bound on a row's length (0: unknown)
  DevBuf rowptr, col, val, valf;  // valf: FP32 copy of val (mixed precision)
  int* rp() const { return rowptr.as<int>(); }
  int* ci() const { return col.as<int>(); }
  double* v() const { return val.as<double>(); }
  float* vf() const { return valf.as<float>(); }
};

struct Level {
  int n = 0;
  Csr A;                 // the level operator
  DevBuf diag, diagf;    // diagonal (FP64, FP32)
  DevBuf dl1, dl1f;      // row l1 norms (l1-Jacobi smoother; FP64, FP32)
  // finest level: slot-major ELL of the off-diagonal part, padding = (row, 0)
  int W = 0;
  DevBuf ell_col, ell_val, ell_valf;
  // transfer operators to level+1
  Csr P, R;
  int n_agg = 0;
  DevBuf agg;            // int[n], aggregate id or -1
  DevBuf B;              // near-null vector
  double rho = 1.0;      // spectral bound of D^-1 A
  // launch choices of the solve kernels (0: the fixed rule; set by the
  // autotuner when enabled): lanes per row of the smoother's CSR kernel, of
  // the restriction and of the prolongation; whether the first two Chebyshev
  // steps from a zero guess run as one fused pass; whether the prolongation
  // runs fused with the first post-smoothing step (where it can)
  int lpr_a = 0, lpr_r = 0, lpr_p = 0;
  bool fuse0 = true, fuse_p = true;
  double inv_theta = 0.0;
  std::vector<double> c1, c2;  // Chebyshev steps 2..degree
  int mis_rounds = 0;
  int mis_batch = 6;     // MIS-2 rounds before the first check (last assembly's count)
  Csr Pt, Q;             // setup scratch: tentative P, A*P_tent
  Csr AP;                // A*P: built for the Galerkin product, then read by
                         // the prolongation fused with post-smoothing
  bool ap_ok = false;    // AP equals A*P for the level's current A
  DevBuf strong, state, state2, m1, mis_root, agg1, agg_ptr, agg_mem, pt;
  DevBuf scol;           // finest level: ELL strong columns (the row itself elsewhere)
  // coarsest level
  bool dense = false;
  DevBuf Ainv;           // dense inverse, FP64 in both precisions
  // V-cycle work vectors (FP64 in both precisions)
  DevBuf x, b, r, d, x2, d2, t;
};

// Device-resident PCG scalars.
struct Scalars {
  double rz, pq, alpha, beta, rr, rz_old, rzo, bb, tmp0, tmp1;
  int flag;
  int pad;
};

// A device value the host needs: `bytes` (a multiple of 4) at `dev`, to be
// copied to `host`.
struct ReadItem {
  const void* dev;
  size_t bytes;
  void* host;
};

}  // namespace ppe

struct ppe_solver {
  // declared first, so it outlives every buffer of the solver
  ppe::Allocator allocator;
  ppe_options opt{};
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;
  ppe_stats stats{};

  // mesh topology
  int n_cells = 0, n_faces = 0, max_deg = 0;
  size_t lds_max = 65536;  // LDS bytes one workgroup may use
  bool have_mesh = false;
  ppe::DevBuf owner, neigh, adj_ptr, adj_nbr, adj_face;

  // masking
  bool assembled = false;
  int n_active = 0, n_comp = 0;
  ppe::DevBuf active, cid, rowpos, perm, parent, comp_full;

  // samples (segments): contiguous cell ranges solved as independent systems
  int n_seg = 1;
  std::vector<int> seg_cell_off{0, 0};  // host, n_seg + 1
  std::vector<int> seg_row_off;         // host, compact rows, n_seg + 1
  std::vector<int> tile_h[4];           // host copies of the tile tables (kept for async uploads)
  int n_tiles = 0;
  ppe::DevBuf tile_r0, tile_r1, tile_seg, seg_tile_ptr;  // reduction tiles
  ppe::DevBuf seg_sc, seg_done, tpart;                   // per-segment scalars, tile partials
  std::vector<int> seg_iters_h;
  std::vector<double> seg_res_h;

  std::vector<ppe::Level> levels;  // never shrunk, so buffers are reused
  int nlev = 0;                    // levels in use

  // solve workspace
  ppe::DevBuf vx, vr, vz, vp, vq, vzold, vb;
  ppe::DevBuf scal, partial, counter, flag;
  ppe::DevBuf tmp_i[4], tmp_d[2], tmp_l[2];
  ppe::DevBuf sp_prod, sp_off, sp_cnt, sp_ci, sp_v;  // sparse-product scratch
  // setup results read back once per hierarchy: the spectral bound of every
  // level (doubles [0, max_levels)), then the deferred setup error bits (int)
  ppe::DevBuf setup_out;
  ppe::DevBuf rmax;  // max column count of the last transposed operator (device int)
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t tev0 = nullptr, tev1 = nullptr;  // autotuner timing
  // pinned host memory that k_publish writes read-back values into
  uint32_t* box_h = nullptr;
  uint32_t* box_d = nullptr;
  size_t box_words = 0;
  uint32_t box_tag = 0;
  hipEvent_t chk_ev[2] = {nullptr, nullptr};  // PCG convergence checks in flight
  // setup's second stream (default priority): coarse power estimates run on
  // it beside the aggregation of the same level
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  int pred_solve = 0, pred_inner = 0;  // iterations of the last solve / projection inner solve
  // reuse of an unchanged system: the coefficients of the last successful
  // assembly (its mask is `active`)
  bool have_prev = false;
  // reuse of the coarse levels across a changed mask (option coarse_reuse):
  // the compact numbering and finest prolongator of the last full build
  bool have_base = false;
  bool fine_reindexed = false;  // the last assembly kept the coarse levels
  int base_na = 0, base_nlev = 0, base_uses = 0;
  ppe::DevBuf base_cid;  // int[n_cells + 1]: cell -> compact row of that build, or -1
  ppe::Csr base_P0;
  bool shifted = false;  // the last assembly carried a diagonal shift (no pins)
  ppe::DevBuf prev_coeff;
  // autotuner choices per (level, FP32, quarter-octave bins of rows and of
  // entries): {lpr_a, fuse0, lpr_r, lpr_p, fuse_p}
  std::map<std::array<int, 4>, std::array<int, 5>> tune_cache;

  // HIP graph of two PCG iterations, captured once per hierarchy
  hipStream_t gstream = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool graph_ok = false;
  int solves_since_assemble = 0;

  // geometry of the pressure-correction step: nodes, cell centres, face area
  // vectors, face vertices, vertex -> cells (sorted), local frames
  bool geom_ok = false;
  int n_nodes = 0;
  ppe::DevBuf g_nodes, g_cc, g_S, g_fnodes, g_vptr, g_vcell;
  ppe::DevBuf g_inv;  // J^-1 per face, nine arrays of n_faces
  ppe::DevBuf pj_fs, pj_b, pj_r, pj_d, pj_grad, pj_xf, pj_part, pj_t, pj_vm;  // projection workspace
  ppe::DevBuf pj_k;  // BiCGSTAB vectors, partials and scalars
  ppe::DevBuf pj_ax, pj_kind, pj_list, pj_cnt, pj_cells;  // cross weights, face kinds, case-2 faces

  // per-kernel measurement of the solve phase (ppe_profile_*): while on,
  // every V-cycle and PCG dispatch is timed by its own event pair, and the
  // durations and algorithmic bytes are summed per kernel instantiation
  struct ProfPending {
    int entry;
    double bytes;
  };
  struct ProfEntry {
    std::string name;  // e.g. "k_csr<2, 16, double>", as a kernel trace names it
    int64_t launches = 0;
    double ms = 0.0, bytes = 0.0;
  };
  bool prof = false;
  std::vector<hipEvent_t> prof_ev;
  std::vector<ProfPending> prof_pending;  // recorded pairs not yet read
  std::vector<ProfEntry> prof_table;
};

namespace ppe {

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  // MurmurHash3 32-bit finaliser (Appleby)
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

__host__ __device__ __forceinline__ uint32_t level_salt(int level) {
  return static_cast<uint32_t>(level) * 0x9E3779B9u;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
  return v;
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    T w = __shfl_down(v, o, kWave);
    v = w > v ? w : v;
  }
  return v;
}

// Deterministic block sum (fixed tree).  Result valid in thread 0.
template <int BS, class T>
__device__ __forceinline__ T block_sum(T v) {
  __shared__ T sh[BS / kWave];
  v = wave_sum(v);
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T s = 0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < BS / kWave; ++i) s += sh[i];
  }
  __syncthreads();
  return s;
}

template <int BS, class T>
__device__ __forceinline__ T block_max(T v) {
  __shared__ T sh[BS / kWave];
  v = wave_max(v);
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T s = sh[0];
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 1; i < BS / kWave; ++i) s = sh[i] > s ? sh[i] : s;
  }
  __syncthreads();
  return s;
}

// Deterministic grid reductions without fences: a producer kernel (grid of
// at most kRedBlocks blocks, grid-stride loops) writes one partial per block
// and value; a consumer kernel sums those partials in a fixed order at the
// start of every block, so all blocks see the same bitwise result.
constexpr int kRedBlocks = 1024;

// Workgroups are dispatched round-robin over the eight XCDs (block b runs on
// XCD b mod 8), and each XCD has its own L2.  The finest level's ELL kernels,
// the fine assembly and the aggregation passes renumber their blocks so that
// each XCD takes one contiguous run of rows: the rows one plane of cells
// apart, which gather the same values, then meet in one L2 instead of eight
// (the 128^3 residual pass: 28.6 -> 21.1 us).  The coarse CSR kernels of the
// solve keep the plain order, which measured faster for them.  A bijection of
// [0, G): XCD x's blocks take the run from x q + min(x, r).
__device__ __forceinline__ int xcd_block(int b, int G) {
  const int x = b & 7, k = b >> 3, q = G >> 3, r = G & 7;
  return x * q + min(x, r) + k;
}

template <int BS, int NV>
__device__ __forceinline__ void write_partials(const double (&v)[NV], double* partials,
                                               int slot = -1) {
  const int at = slot < 0 ? (int)blockIdx.x : slot;  // a block that works for another's slot
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = block_sum<BS>(v[k]);
    if (threadIdx.x == 0) partials[(size_t)k * gridDim.x + at] = s;
  }
}

// Sum of partials[0..G) (fixed order); result broadcast to every thread.
template <int BS>
__device__ __forceinline__ double sum_partials(const double* __restrict__ partials, int G) {
  __shared__ double bc;
  double a = 0.0;
  for (int b = threadIdx.x; b < G; b += BS) a += partials[b];
  a = block_sum<BS>(a);
  if (threadIdx.x == 0) bc = a;
  __syncthreads();
  const double r = bc;
  __syncthreads();
  return r;
}

// The sums of NV partial arrays at once (each added in the order of
// sum_partials, so each result is bitwise the same): one pass over the
// partials and one exchange through LDS instead of NV; broadcast to every
// thread.
template <int BS, int NV>
__device__ __forceinline__ void sum_partials_n(const double* const (&parts)[NV], int G,
                                               double (&out)[NV]) {
  __shared__ double sh[NV][BS / kWave];
  __shared__ double bc[NV];
  double a[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) a[k] = 0.0;
  for (int b = threadIdx.x; b < G; b += BS) {
#pragma unroll
    for (int k = 0; k < NV; ++k) a[k] += parts[k][b];
  }
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    a[k] = wave_sum(a[k]);
    if (lane == 0) sh[k][w] = a[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double t = 0;
#pragma unroll
      for (int i = 0; i < BS / kWave; ++i) t += sh[k][i];
      bc[k] = t;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) out[k] = bc[k];
  __syncthreads();
}

inline int red_grid(int64_t work_items, int bs = kBlock) {
  int64_t g = (work_items + bs - 1) / bs;
  if (g < 1) g = 1;
  return static_cast<int>(g > kRedBlocks ? kRedBlocks : g);
}

// Grid-wide deterministic sum of one value per thread, finished by the last
// block to arrive: partials are added in block order whatever the arrival
// order, so the result is bitwise reproducible.  Returns true in thread 0 of
// the last block, with *out written.  counter must start at 0 (it is reset).
template <int BS, int NV>
__device__ __forceinline__ bool grid_sum(const double (&v)[NV], double* partials,
                                         unsigned int* counter, double* out) {
  __shared__ bool last;
  double s[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) s[k] = block_sum<BS>(v[k]);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) partials[(size_t)k * gridDim.x + blockIdx.x] = s[k];
    __threadfence();
    unsigned int t = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double a = 0.0;
    for (unsigned int b = threadIdx.x; b < gridDim.x; b += BS)
      a += __hip_atomic_load(&partials[(size_t)k * gridDim.x + b], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    acc[k] = block_sum<BS>(a);
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) out[k] = acc[k];
    *counter = 0u;
  }
  return threadIdx.x == 0;
}

// Lanes per row for row-parallel CSR kernels: the power of two (4..64) at or
// above the mean row length.
inline int lanes_for(const Csr& A) {
  const double mean = A.n ? (double)A.nnz / A.n : 1.0;
  int lpr = 4;
  while (lpr < 64 && lpr < mean) lpr *= 2;
  return lpr;
}

inline int grid_for(int64_t n, int bs = kBlock) {
  int64_t g = (n + bs - 1) / bs;
  return static_cast<int>(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------- host-side primitives (prims.hip)
// Exclusive scan of int32 counts into out[0..n] (out[n] = total).  Returns
// the total; throws PPE_ERR_INTERNAL if it does not fit int32.
int64_t exclusive_scan(ppe_solver* s, const int* in, int* out, int n);
// The same without reading the total back.  Returns the device address of
// the total (a long long in tmp_l[slot], slot 0 or 1, valid until the next
// scan through that slot).  With max_out, the largest count is also max-ed
// into *max_out, as max_int_async(..., init = false) would do, with no
// dispatch of its own.
long long* exclusive_scan_async(ppe_solver* s, const int* in, int* out, int n, int slot = 0,
                                int* max_out = nullptr);
int scan_blocks(int n);
// *out = max of in[0..n) on the device (no host read)
// init = false: *out already holds a lower bound (e.g. 0 for counts)
void max_int_async(ppe_solver* s, const int* in, int n, int* out, bool init = true);
// Max of an int array.
int reduce_max_int(ppe_solver* s, const int* in, int n);
// ---- read-backs through pinned host memory
// Box layout in words: [kBoxChecks, kBoxRead) for the PCG's convergence
// checks (two in flight, three words each with the tag), read_back from
// kBoxRead on.
constexpr size_t kBoxChecks = 0, kBoxRead = 8;
// Makes the solver's pinned box hold at least `words` 4-byte words; a box
// that must grow is replaced only after the stream has drained.
void ensure_box(ppe_solver* s, size_t words);
// Values copied into the box by one publish call: n_words words at `words`,
// followed by the call's tag.
struct Published {
  const uint32_t* words;
  uint32_t n_words;
  uint32_t tag;
};
// One small kernel on the solver stream copies the items (at most 16), in
// order, into the box from word `at` on, then a fresh tag behind them.  No
// host copies are made; read the values with published_words once the stream
// (or an event recorded after the call) has completed.
Published publish(ppe_solver* s, const ReadItem* items, int n, size_t at);
// The published words after checking their tag; throws PPE_ERR_INTERNAL if
// they are still not visible once the stream has drained.
const uint32_t* published_words(ppe_solver* s, const Published& p);
// Publishes the items at kBoxRead, waits for the stream and copies each item
// to its host address: one round trip for any number of values.
void read_back(ppe_solver* s, std::initializer_list<ReadItem> items);
// One value from device to host on the solver stream (synchronises).
template <class T>
T read_scalar(ppe_solver* s, const T* dptr) {
  T v{};
  read_back(s, {ReadItem{dptr, sizeof(T), &v}});
  return v;
}
void fill_int(ppe_solver* s, int* p, int v, int64_t n);
void fill_double(ppe_solver* s, double* p, double v, int64_t n);

// assemble.hip
void build_topology(ppe_solver* s, const int32_t* owner, const int32_t* neigh);
void check_segments(ppe_solver* s, const std::vector<int>& off);
// shift NULL: the pinned pressure system of fl's mask.  shift[n_cells]
// (> 0 on active cells): diag(shift) + L without pins; fl may then be NULL
// (every cell active).
void assemble_fine(ppe_solver* s, const double* coeff, const double* fl, const double* shift);
// A shifted system's new shift with the same face coefficients and mask: the
// finest level's diagonal and spectral bound are recomputed; the coarse
// levels stay (the V-cycle stays symmetric positive definite).
void refresh_fine_shift(ppe_solver* s, const double* coeff, const double* shift);
// The finest level's spectral bound, queued into the setup output slot
// (device address returned).
const double* level0_bound_async(ppe_solver* s);
// Checks the fields (raising PPE_ERR_ARG as the assembly does) and returns
// whether the coefficients and the mask equal those of the last assembly.
bool same_system(ppe_solver* s, const double* coeff, const double* fl);

// amg.hip
void build_hierarchy(ppe_solver* s);
// Keep the coarse levels of the last full build for the newly assembled
// finest level (option coarse_reuse); false (nothing changed) when the
// active set moved too far, and a full build must follow.
bool reuse_coarse_levels(ppe_solver* s);
// Record the finest level's numbering and prolongator after a full build.
void keep_base(ppe_solver* s);

// solve.hip
void spmv(ppe_solver* s, const Level& L, const double* x, double* y);
// Power iteration for lambda_max(D^-1 A) on a CSR level from the hashed
// start vector 1/2 + fmix32(i ^ salt) / 2^32; uses L.x and L.r as work.
// *out = scale x (power estimate of the largest eigenvalue of D^-1 A on level
// L after iters steps from the seeded start vector); stays on the device.
void power_estimate(ppe_solver* s, Level& L, uint32_t salt, int iters, double scale, double* out);
void vcycle(ppe_solver* s, int level, const double* b, double* x);
// pred: iterations the previous solve of this kind took (0: unknown), updated
// on return; the convergence checks run ahead of the device only while the
// queued work stays short of it.  NULL: always run ahead.
ppe_status pcg_solve(ppe_solver* s, const double* rhs, double* p, int use_x0, int* pred = nullptr);
void prepare_solve_levels(ppe_solver* s);
void make_fp32_hierarchy(ppe_solver* s);
// Time the candidate launch choices of every level's solve kernels and keep
// the fastest (cached by level shape).
void autotune_levels(ppe_solver* s);

// project.hip
// Copies the geometry and builds the Eq. 12 face-gradient stencils.
void set_geometry(ppe_solver* s, int n_nodes, const double* nodes, const int32_t* face_nodes,
                  const int32_t* cell_nodes, const double* cell_centre, const double* face_area);
// t[3 n_faces] (three arrays) = S_f / rho - c_f d_f on interior faces
void cross_vectors(ppe_solver* s, const double* coeff, double rho, double* t);
// xf[n_faces] = t_f . grad_f with grad_f the masked face gradient of
// p[n_cells]; grad[3 n_faces] receives the gradients unless NULL
void face_gradient(ppe_solver* s, const double* p, const double* t, double* grad, double* xf);
ppe_status project(ppe_solver* s, const double* coeff, const double* ustar, double rho, double dt,
                   double* p, double* flux, double* u, ppe_project_stats* out, bool use_x0);
void profile_harvest(ppe_solver* s);
void drop_graph(ppe_solver* s);
void profile_enable(ppe_solver* s, bool on);
// The event pair for the next profiled dispatch of kernel `name` moving
// `bytes` algorithmic bytes (earlier pairs are read first when all are in use).
std::pair<hipEvent_t, hipEvent_t> profile_slot(ppe_solver* s, const std::string& name,
                                               double bytes);

}  // namespace ppe

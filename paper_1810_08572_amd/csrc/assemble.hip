// Mesh topology and the masked assembly of the finest pressure operator.
//
// Topology (once per mesh): for every cell, the list of (neighbour, face)
// over its interior faces, sorted by neighbour then face, in CSR form.
//
// Masked assembly (each time the liquid fraction changes), section 2.4.2:
//   active cell     f_l > 0 (liquid or mushy, tag LM); compact ids by scan;
//   open face       interior face whose two owners are active; a face with a
//                   removed owner is blocked and adds nothing anywhere
//                   (Neumann at the solid front, case 3, step 2);
//   components      connected sets of active cells over open faces, found by
//                   lock-free union-find that always hooks the larger root
//                   under the smaller one, so the final root of each set is
//                   its lowest cell index: that cell is the set's pin;
//   rows            diagonal = sum of open-face coefficients taken in
//                   ascending neighbour order; off-diagonal -c_f towards every
//                   active neighbour that is not a pin; a pin keeps only its
//                   diagonal (1 when it has no open face).
#include "common.h"

#include <algorithm>

namespace ppe {
namespace {

__global__ void k_check_faces(const int* __restrict__ owner, const int* __restrict__ neigh,
                              int n_faces, int n_cells, int* __restrict__ flag) {
  int f = blockIdx.x * kBlock + threadIdx.x;
  if (f >= n_faces) return;
  int o = owner[f], nb = neigh[f];
  if (o < 0 || o >= n_cells || nb < -1 || nb >= n_cells || o == nb) atomicOr(flag, 1);
}

__global__ void k_degree(const int* __restrict__ owner, const int* __restrict__ neigh,
                         int n_faces, int* __restrict__ deg) {
  int f = blockIdx.x * kBlock + threadIdx.x;
  if (f >= n_faces) return;
  int nb = neigh[f];
  if (nb < 0) return;
  atomicAdd(&deg[owner[f]], 1);
  atomicAdd(&deg[nb], 1);
}

__global__ void k_adj_fill(const int* __restrict__ owner, const int* __restrict__ neigh,
                           int n_faces, int* __restrict__ cursor, int* __restrict__ adj_nbr,
                           int* __restrict__ adj_face) {
  int f = blockIdx.x * kBlock + threadIdx.x;
  if (f >= n_faces) return;
  int o = owner[f], nb = neigh[f];
  if (nb < 0) return;
  int p = atomicAdd(&cursor[o], 1);
  adj_nbr[p] = nb;
  adj_face[p] = f;
  p = atomicAdd(&cursor[nb], 1);
  adj_nbr[p] = o;
  adj_face[p] = f;
}

// Sort each cell's (neighbour, face) list; flag two faces joining one pair.
__global__ void k_adj_sort(const int* __restrict__ ptr, int n_cells, int* __restrict__ nbr,
                           int* __restrict__ face, int* __restrict__ flag) {
  int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= n_cells) return;
  int b = ptr[c], e = ptr[c + 1];
  for (int i = b + 1; i < e; ++i) {
    int kn = nbr[i], kf = face[i];
    int j = i - 1;
    while (j >= b && (nbr[j] > kn || (nbr[j] == kn && face[j] > kf))) {
      nbr[j + 1] = nbr[j];
      face[j + 1] = face[j];
      --j;
    }
    nbr[j + 1] = kn;
    face[j + 1] = kf;
  }
  for (int i = b + 1; i < e; ++i)
    if (nbr[i] == nbr[i - 1]) atomicOr(flag, 2);
}

// Bit 1: a bad face coefficient; bit 2: a bad liquid fraction (fl may be
// NULL: every cell active); bit 8: a diagonal shift that is not finite and
// > 0 on an active cell (shift NULL: no shift).
__global__ void k_check_fields(const double* __restrict__ coeff, const int* __restrict__ neigh,
                               int n_faces, const double* __restrict__ fl, int n_cells,
                               int* __restrict__ flag, const double* __restrict__ shift) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n_faces && neigh[i] >= 0) {
    double c = coeff[i];
    if (!(c > 0.0) || !(c <= 1.7976931348623157e308)) atomicOr(flag, 1);
  }
  if (i < n_cells) {
    const double v = fl ? fl[i] : 1.0;
    if (!(v >= 0.0 && v <= 1.0)) atomicOr(flag, 2);
    if (shift && v > 0.0) {
      const double d = shift[i];
      if (!(d > 0.0) || !(d <= 1.7976931348623157e308)) atomicOr(flag, 8);
    }
  }
}

__global__ void k_active(const double* __restrict__ fl, int n, int* __restrict__ active,
                         int* __restrict__ parent) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  active[i] = (!fl || fl[i] > 0.0) ? 1 : 0;
  parent[i] = i;
}

// rowpos = exclusive scan of active (kept: segment row offsets read it);
// cid = rowpos on active cells, -1 elsewhere; perm inverts cid.
__global__ void k_compact(const int* __restrict__ active, int n, const int* __restrict__ rowpos,
                          int* __restrict__ cid, int* __restrict__ perm) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  if (active[i]) {
    cid[i] = rowpos[i];
    perm[rowpos[i]] = i;
  } else {
    cid[i] = -1;
  }
}

__device__ __forceinline__ int ld(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int find_root(int* parent, int x) {
  int p = ld(&parent[x]);
  while (p != x) {
    int gp = ld(&parent[p]);
    if (gp != p) __hip_atomic_store(&parent[x], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = p;
    p = gp;
  }
  return x;
}

// Connected components start from a forest built without atomics: every
// active cell hooks to its smallest active neighbour (or itself), which
// already joins most of a component; the forest is then flattened (each cell
// to its tree's root) and the face pass below only links the remaining trees.
// Every link points to a smaller index, so each component's root is its
// smallest cell.
__global__ void k_cc_init(int n, const int* __restrict__ adj_ptr, const int* __restrict__ adj_nbr,
                          const int* __restrict__ active, int* __restrict__ forest) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int m = i;
  if (active[i])
    for (int k = adj_ptr[i]; k < adj_ptr[i + 1]; ++k) {
      const int j = adj_nbr[k];
      if (j < m && active[j]) m = j;
    }
  forest[i] = m;
}

// One pointer-jumping pass over the forest: out_i = in_(in_i).  The roots
// stay (a root points to itself) and every path to them halves, so the walk
// of k_cc_flatten that follows takes half the dependent loads.  On a mesh
// numbered plane by plane the smallest-neighbour paths run down one column
// of cells, then along one row and one line (about 420 cells on the plate
// with ribs): two passes of 5 us each cut the walk from 72 to 23 us.
__global__ void k_cc_jump(int n, const int* __restrict__ in, int* __restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = in[in[i]];
}

// parent_i = root of i in the forest (indices strictly decrease along a path,
// so the walk ends).
__global__ void k_cc_flatten(int n, const int* __restrict__ forest, int* __restrict__ parent) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int p = forest[i];
  while (forest[p] != p) p = forest[p];
  parent[i] = p;
}

__global__ void k_union(const int* __restrict__ owner, const int* __restrict__ neigh, int n_faces,
                        const int* __restrict__ active, int* parent) {
  int f = blockIdx.x * kBlock + threadIdx.x;
  if (f >= n_faces) return;
  int a = owner[f], b = neigh[f];
  if (b < 0 || !active[a] || !active[b]) return;
  while (true) {
    a = find_root(parent, a);
    b = find_root(parent, b);
    if (a == b) return;
    if (a > b) { int t = a; a = b; b = t; }
    int old = atomicCAS(&parent[b], b, a);
    if (old == b) return;
    b = old;
  }
}

// comp[i] = the pin (smallest cell) of i's component, -1 on removed cells;
// without pins (a shifted system) every active cell gets -2.
__global__ void k_components(const int* __restrict__ active, int n, int* parent,
                             int* __restrict__ comp, int* __restrict__ is_pin, int pins) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  if (!active[i] || !pins) {
    comp[i] = active[i] ? -2 : -1;
    is_pin[i] = 0;
    return;
  }
  int r = find_root(parent, i);
  comp[i] = r;
  is_pin[i] = (r == i) ? 1 : 0;
}

// Entries of every compact row r < *n_active; rows from there to n_max get 0
// so that a scan over n_max rows ends at the matrix size.
__global__ void k_row_counts(const int* __restrict__ perm, const int* __restrict__ n_active,
                             int n_max, const int* __restrict__ adj_ptr,
                             const int* __restrict__ adj_nbr, const int* __restrict__ active,
                             const int* __restrict__ is_pin, int* __restrict__ counts) {
  int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= n_max) return;
  if (r >= *n_active) {
    counts[r] = 0;
    return;
  }
  int c = perm[r];
  int cnt = 1;
  if (!is_pin[c]) {
    for (int k = adj_ptr[c]; k < adj_ptr[c + 1]; ++k) {
      int j = adj_nbr[k];
      if (active[j] && !is_pin[j]) ++cnt;
    }
  }
  counts[r] = cnt;
}

// Row r of the compact system: its CSR entries (the diagonal in its sorted
// place), its diagonal, its slot-major ELL row and B = 1.  With STAGE the
// workgroup's rows, which are one contiguous CSR range, are assembled in
// LDS (W + 1 entries per row at most) and written out together, so the
// stores of a wavefront are contiguous instead of one row per lane.
template <bool STAGE>
__global__ void k_fill_rows(const int* __restrict__ perm, int n_active,
                            const int* __restrict__ adj_ptr, const int* __restrict__ adj_nbr,
                            const int* __restrict__ adj_face, const int* __restrict__ active,
                            const int* __restrict__ is_pin, const int* __restrict__ cid,
                            const double* __restrict__ coeff, const int* __restrict__ rowptr,
                            int* __restrict__ col, double* __restrict__ val,
                            double* __restrict__ diag, int W, int* __restrict__ ell_col,
                            double* __restrict__ ell_val, double* __restrict__ B,
                            const double* __restrict__ shift) {
  extern __shared__ double stage_v[];  // STAGE: kBlock (W + 1) values, then columns
  const int r0 = xcd_block(blockIdx.x, gridDim.x) * kBlock;
  const int r = r0 + threadIdx.x;
  const int base = STAGE ? rowptr[r0] : 0;
  int* stage_c = reinterpret_cast<int*>(stage_v + (size_t)kBlock * (W + 1));
  // where row r's entries go: LDS (offset from the workgroup's first entry) or C
  int* cdst = STAGE ? stage_c - base : col;
  double* vdst = STAGE ? stage_v - base : val;
  if (r < n_active) {
    int c = perm[r];
    const bool pin = is_pin[c] != 0;
    double d = shift ? shift[c] : 0.0;
    for (int k = adj_ptr[c]; k < adj_ptr[c + 1]; ++k) {
      int j = adj_nbr[k];
      if (active[j]) d = d + coeff[adj_face[k]];
    }
    if (pin && d == 0.0) d = 1.0;
    diag[r] = d;
    B[r] = 1.0;
    int p = rowptr[r];
    int slot = 0;
    bool diag_done = false;
    if (!pin) {
      for (int k = adj_ptr[c]; k < adj_ptr[c + 1]; ++k) {
        int j = adj_nbr[k];
        if (!active[j] || is_pin[j]) continue;
        int cj = cid[j];
        double v = -coeff[adj_face[k]];
        if (!diag_done && cj > r) {
          cdst[p] = r;
          vdst[p] = d;
          ++p;
          diag_done = true;
        }
        cdst[p] = cj;
        vdst[p] = v;
        ++p;
        ell_col[(size_t)slot * n_active + r] = cj;
        ell_val[(size_t)slot * n_active + r] = v;
        ++slot;
      }
    }
    if (!diag_done) {
      cdst[p] = r;
      vdst[p] = d;
    }
    for (; slot < W; ++slot) {
      ell_col[(size_t)slot * n_active + r] = r;
      ell_val[(size_t)slot * n_active + r] = 0.0;
    }
  }
  if (STAGE) {
    __syncthreads();
    const int r1 = min(r0 + kBlock, n_active);
    const int cnt = rowptr[r1] - base;
    for (int q = threadIdx.x; q < cnt; q += kBlock) {
      col[base + q] = stage_c[q];
      val[base + q] = stage_v[q];
    }
  }
}

// A new diagonal for the finest level of a shifted system: the same sum as
// k_fill_rows (shift, then the open faces in ascending neighbour order),
// into diag and into the CSR row's diagonal entry.  Bit 8: a bad shift.
__global__ void k_refresh_diag(const int* __restrict__ perm, int n_active,
                               const int* __restrict__ adj_ptr, const int* __restrict__ adj_nbr,
                               const int* __restrict__ adj_face, const int* __restrict__ active,
                               const double* __restrict__ coeff, const double* __restrict__ shift,
                               const int* __restrict__ rowptr, const int* __restrict__ col,
                               double* __restrict__ val, double* __restrict__ diag,
                               int* __restrict__ flag) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= n_active) return;
  const int c = perm[r];
  const double sh = shift[c];
  if (!(sh > 0.0) || !(sh <= 1.7976931348623157e308)) atomicOr(flag, 8);
  double d = sh;
  for (int k = adj_ptr[c]; k < adj_ptr[c + 1]; ++k)
    if (active[adj_nbr[k]]) d = d + coeff[adj_face[k]];
  diag[r] = d;
  for (int p = rowptr[r]; p < rowptr[r + 1]; ++p)
    if (col[p] == r) val[p] = d;
}

__global__ void k_gather_int(int n, const int* __restrict__ idx, const int* __restrict__ src,
                             int* __restrict__ dst) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}

// Reduction tiles: runs of at most 4096 compact rows that never cross a
// segment boundary; tile t covers rows [r0[t], r1[t]) of segment seg[t], and
// segment s owns tiles [seg_tile_ptr[s], seg_tile_ptr[s+1]).
// Reduction tiles over the compact rows of every segment (s->seg_row_off
// must hold the segments' compact row offsets): about kRedBlocks tiles over
// the whole system, 256..4096 rows each, none crossing a segment.  The host
// tables are kept in the solver, so their uploads need no synchronisation.
void build_tiles(ppe_solver* s) {
  const int ns = s->n_seg;
  const int na = s->seg_row_off[ns];
  int rows = ((na / kRedBlocks + 255) / 256) * 256;
  rows = std::min(std::max(rows, 256), 4096);
  std::vector<int>& r0 = s->tile_h[0];
  std::vector<int>& r1 = s->tile_h[1];
  std::vector<int>& sg = s->tile_h[2];
  std::vector<int>& tp = s->tile_h[3];
  r0.clear();
  r1.clear();
  sg.clear();
  tp.assign(ns + 1, 0);
  for (int q = 0; q < ns; ++q) {
    tp[q] = (int)r0.size();
    for (int a = s->seg_row_off[q]; a < s->seg_row_off[q + 1]; a += rows) {
      r0.push_back(a);
      r1.push_back(std::min(a + rows, s->seg_row_off[q + 1]));
      sg.push_back(q);
    }
  }
  tp[ns] = (int)r0.size();
  s->n_tiles = (int)r0.size();
  const size_t nt = r0.size() ? r0.size() : 1;
  int* a = s->tile_r0.get<int>(nt);
  int* b = s->tile_r1.get<int>(nt);
  int* c = s->tile_seg.get<int>(nt);
  int* d = s->seg_tile_ptr.get<int>(ns + 1);
  if (!r0.empty()) {
    PPE_HIP(hipMemcpyAsync(a, r0.data(), sizeof(int) * r0.size(), hipMemcpyHostToDevice, s->stream));
    PPE_HIP(hipMemcpyAsync(b, r1.data(), sizeof(int) * r1.size(), hipMemcpyHostToDevice, s->stream));
    PPE_HIP(hipMemcpyAsync(c, sg.data(), sizeof(int) * sg.size(), hipMemcpyHostToDevice, s->stream));
  }
  PPE_HIP(hipMemcpyAsync(d, tp.data(), sizeof(int) * (ns + 1), hipMemcpyHostToDevice, s->stream));
}

// flag faces whose two owners lie in different samples
__global__ void k_check_segments(const int* __restrict__ owner, const int* __restrict__ neigh,
                                 int n_faces, const int* __restrict__ off, int ns,
                                 int* __restrict__ flag) {
  int f = blockIdx.x * kBlock + threadIdx.x;
  if (f >= n_faces || neigh[f] < 0) return;
  auto seg_of = [&](int c) {
    int lo = 0, hi = ns;  // off[lo] <= c < off[hi]
    while (hi - lo > 1) {
      int mid = (lo + hi) / 2;
      if (off[mid] <= c) lo = mid; else hi = mid;
    }
    return lo;
  };
  if (seg_of(owner[f]) != seg_of(neigh[f])) atomicOr(flag, 1);
}

}  // namespace

void check_segments(ppe_solver* s, const std::vector<int>& off) {
  const int ns = (int)off.size() - 1;
  int* d_off = s->tmp_i[0].get<int>(ns + 1);
  PPE_HIP(hipMemcpyAsync(d_off, off.data(), sizeof(int) * (ns + 1), hipMemcpyHostToDevice,
                         s->stream));
  int* flag = s->flag.get<int>(4);
  fill_int(s, flag, 0, 1);
  if (s->n_faces) {
    hipLaunchKernelGGL(k_check_segments, dim3(grid_for(s->n_faces)), dim3(kBlock), 0, s->stream,
                       s->owner.as<int>(), s->neigh.as<int>(), s->n_faces, d_off, ns, flag);
    PPE_LAUNCH_CHECK();
  }
  require(read_scalar(s, flag) == 0, PPE_ERR_ARG, "an interior face joins two samples");
}

void build_topology(ppe_solver* s, const int32_t* owner, const int32_t* neigh) {
  const int nf = s->n_faces, nc = s->n_cells;
  int* o = s->owner.get<int>(nf);
  int* nb = s->neigh.get<int>(nf);
  if (nf) {
    PPE_HIP(hipMemcpyAsync(o, owner, sizeof(int) * nf, hipMemcpyDeviceToDevice, s->stream));
    PPE_HIP(hipMemcpyAsync(nb, neigh, sizeof(int) * nf, hipMemcpyDeviceToDevice, s->stream));
  }
  int* flag = s->flag.get<int>(1);
  fill_int(s, flag, 0, 1);
  if (nf) {
    hipLaunchKernelGGL(k_check_faces, dim3(grid_for(nf)), dim3(kBlock), 0, s->stream, o, nb, nf, nc,
                       flag);
    PPE_LAUNCH_CHECK();
  }
  require(read_scalar(s, flag) == 0, PPE_ERR_ARG,
          "face owner/neighbour out of range or equal");
  int* deg = s->tmp_i[0].get<int>(nc + 1);
  fill_int(s, deg, 0, nc + 1);
  if (nf) {
    hipLaunchKernelGGL(k_degree, dim3(grid_for(nf)), dim3(kBlock), 0, s->stream, o, nb, nf, deg);
    PPE_LAUNCH_CHECK();
  }
  s->max_deg = reduce_max_int(s, deg, nc);
  int* ptr = s->adj_ptr.get<int>(nc + 1);
  int64_t nh = exclusive_scan(s, deg, ptr, nc);
  int* cursor = s->tmp_i[1].get<int>(nc + 1);
  PPE_HIP(hipMemcpyAsync(cursor, ptr, sizeof(int) * (nc + 1), hipMemcpyDeviceToDevice, s->stream));
  int* an = s->adj_nbr.get<int>(nh);
  int* af = s->adj_face.get<int>(nh);
  if (nf) {
    hipLaunchKernelGGL(k_adj_fill, dim3(grid_for(nf)), dim3(kBlock), 0, s->stream, o, nb, nf, cursor,
                       an, af);
    PPE_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_adj_sort, dim3(grid_for(nc)), dim3(kBlock), 0, s->stream, ptr, nc, an, af,
                     flag);
  PPE_LAUNCH_CHECK();
  require(read_scalar(s, flag) == 0, PPE_ERR_ARG, "two faces join the same pair of cells");
}

namespace {
// bit 4 of *flag: a coefficient of an interior face or a cell's mask differs
// from the stored ones
__global__ void k_same_system(const double* __restrict__ coeff, const double* __restrict__ prev,
                              const int* __restrict__ neigh, int nf, const double* __restrict__ fl,
                              const int* __restrict__ active, int nc, int* __restrict__ flag) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  bool diff = false;
  if (i < nf && neigh[i] >= 0 && coeff[i] != prev[i]) diff = true;
  if (i < nc && ((fl[i] > 0.0 ? 1 : 0) != active[i])) diff = true;
  if (diff) atomicOr(flag, 4);
}
}  // namespace

bool same_system(ppe_solver* s, const double* coeff, const double* fl) {
  const int nc = s->n_cells, nf = s->n_faces;
  int* flag = s->flag.get<int>(1);
  fill_int(s, flag, 0, 1);
  const int g = grid_for(nf > nc ? nf : nc);
  hipLaunchKernelGGL(k_check_fields, dim3(g), dim3(kBlock), 0, s->stream, coeff, s->neigh.as<int>(),
                     nf, fl, nc, flag, static_cast<const double*>(nullptr));
  PPE_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_same_system, dim3(g), dim3(kBlock), 0, s->stream, coeff,
                     s->prev_coeff.as<double>(), s->neigh.as<int>(), nf, fl, s->active.as<int>(), nc,
                     flag);
  PPE_LAUNCH_CHECK();
  const int bad = read_scalar(s, flag);
  require(!(bad & 1), PPE_ERR_ARG, "face coefficient must be finite and > 0 on interior faces");
  require(!(bad & 2), PPE_ERR_ARG, "liquid fraction must be finite and in [0, 1]");
  return !(bad & 4);
}

void assemble_fine(ppe_solver* s, const double* coeff, const double* fl, const double* shift) {
  const int nc = s->n_cells, nf = s->n_faces, ns = s->n_seg;
  s->shifted = shift != nullptr;
  int* flag = s->flag.get<int>(1);
  fill_int(s, flag, 0, 1);
  int g = grid_for(nf > nc ? nf : nc);
  hipLaunchKernelGGL(k_check_fields, dim3(g), dim3(kBlock), 0, s->stream, coeff, s->neigh.as<int>(),
                     nf, fl, nc, flag, shift);
  PPE_LAUNCH_CHECK();

  int* active = s->active.get<int>(nc);
  int* parent = s->parent.get<int>(nc);
  int* cid = s->cid.get<int>(nc + 1);
  int* rowpos = s->rowpos.get<int>(nc + 1);
  hipLaunchKernelGGL(k_active, dim3(grid_for(nc)), dim3(kBlock), 0, s->stream, fl, nc, active, parent);
  PPE_LAUNCH_CHECK();
  exclusive_scan_async(s, active, rowpos, nc);  // rowpos[nc] = number of active cells
  // compact row offsets of the segments: rowpos at their first cells
  int* d_off = s->tmp_i[0].get<int>(ns + 1);
  int* d_row = s->tmp_i[1].get<int>(ns + 1);
  PPE_HIP(hipMemcpyAsync(d_off, s->seg_cell_off.data(), sizeof(int) * (ns + 1),
                         hipMemcpyHostToDevice, s->stream));
  hipLaunchKernelGGL(k_gather_int, dim3(grid_for(ns + 1)), dim3(kBlock), 0, s->stream, ns + 1, d_off,
                     rowpos, d_row);
  PPE_LAUNCH_CHECK();
  // Everything up to the row pointers is queued before the host learns the
  // number of active cells (rowpos[nc] on the device): arrays indexed by
  // compact row are sized for all cells.
  int* perm = s->perm.get<int>(nc);
  hipLaunchKernelGGL(k_compact, dim3(grid_for(nc)), dim3(kBlock), 0, s->stream, active, nc, rowpos,
                     cid, perm);
  PPE_LAUNCH_CHECK();

  int* comp = s->comp_full.get<int>(nc);
  int* is_pin = s->tmp_i[2].get<int>(nc);
  // a shifted system is non-singular on every component: no pins, so no
  // component search either
  if (nf && !shift) {
    int* forest = s->tmp_i[3].get<int>(nc + 1);
    hipLaunchKernelGGL(k_cc_init, dim3(grid_for(nc)), dim3(kBlock), 0, s->stream, nc,
                       s->adj_ptr.as<int>(), s->adj_nbr.as<int>(), active, forest);
    PPE_LAUNCH_CHECK();
    // parent is free until the flattening fills it: the jumps go through it
    hipLaunchKernelGGL(k_cc_jump, dim3(grid_for(nc)), dim3(kBlock), 0, s->stream, nc, forest,
                       parent);
    PPE_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cc_jump, dim3(grid_for(nc)), dim3(kBlock), 0, s->stream, nc, parent,
                       forest);
    PPE_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cc_flatten, dim3(grid_for(nc)), dim3(kBlock), 0, s->stream, nc, forest,
                       parent);
    PPE_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_union, dim3(grid_for(nf)), dim3(kBlock), 0, s->stream, s->owner.as<int>(),
                       s->neigh.as<int>(), nf, active, parent);
    PPE_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_components, dim3(grid_for(nc)), dim3(kBlock), 0, s->stream, active, nc,
                     parent, comp, is_pin, shift ? 0 : 1);
  PPE_LAUNCH_CHECK();
  const long long* d_ncomp =
      exclusive_scan_async(s, is_pin, s->tmp_i[3].get<int>(nc + 1), nc, 1);

  if (s->levels.empty()) s->levels.resize(1);
  s->nlev = 1;
  Level& L = s->levels[0];
  int* counts = s->tmp_i[0].get<int>(nc + 1);
  hipLaunchKernelGGL(k_row_counts, dim3(grid_for(nc)), dim3(kBlock), 0, s->stream, perm, rowpos + nc,
                     nc, s->adj_ptr.as<int>(), s->adj_nbr.as<int>(), active, is_pin, counts);
  PPE_LAUNCH_CHECK();
  int* rowptr = L.A.rowptr.get<int>(nc + 1);
  const long long* d_nnz = exclusive_scan_async(s, counts, rowptr, nc, 0);
  // one read-back: the field checks, the segments' row offsets, the matrix
  // size and the pocket count
  int bad = 0;
  long long tot[2] = {0, 0};
  s->seg_row_off.assign(ns + 1, 0);
  read_back(s, {ReadItem{flag, sizeof(int), &bad},
                ReadItem{d_row, sizeof(int) * (ns + 1), s->seg_row_off.data()},
                ReadItem{d_nnz, sizeof(long long), &tot[0]},
                ReadItem{d_ncomp, sizeof(long long), &tot[1]}});
  require(!(bad & 1), PPE_ERR_ARG, "face coefficient must be finite and > 0 on interior faces");
  require(!(bad & 2), PPE_ERR_ARG, "liquid fraction must be finite and in [0, 1]");
  require(!(bad & 8), PPE_ERR_ARG, "diagonal shift must be finite and > 0 on every active cell");
  const int na = s->seg_row_off[ns];
  s->n_active = na;
  s->n_comp = (int)tot[1];
  build_tiles(s);

  L.n = na;
  L.A.n = L.A.m = na;
  L.A.maxrow = s->max_deg + 1;  // a row holds its open faces and the diagonal
  L.W = s->max_deg;
  L.A.nnz = tot[0];
  if (na == 0) return;
  int* col = L.A.col.get<int>(L.A.nnz);
  double* val = L.A.val.get<double>(L.A.nnz);
  double* diag = L.diag.get<double>(na);
  const int W = L.W > 0 ? L.W : 1;
  int* ecol = L.ell_col.get<int>((size_t)W * na);
  double* evl = L.ell_val.get<double>((size_t)W * na);
  double* B = L.B.get<double>(na);
  // a row holds at most W + 1 entries (its open faces and the diagonal)
  const size_t stage = (size_t)kBlock * (L.W + 1) * (sizeof(double) + sizeof(int));
  if (stage <= s->lds_max)
    hipLaunchKernelGGL(k_fill_rows<true>, dim3(grid_for(na)), dim3(kBlock), stage, s->stream,
                       perm, na, s->adj_ptr.as<int>(), s->adj_nbr.as<int>(),
                       s->adj_face.as<int>(), active, is_pin, cid, coeff, rowptr, col, val, diag,
                       L.W, ecol, evl, B, shift);
  else
    hipLaunchKernelGGL(k_fill_rows<false>, dim3(grid_for(na)), dim3(kBlock), 0, s->stream, perm,
                       na, s->adj_ptr.as<int>(), s->adj_nbr.as<int>(), s->adj_face.as<int>(),
                       active, is_pin, cid, coeff, rowptr, col, val, diag, L.W, ecol, evl, B,
                       shift);
  PPE_LAUNCH_CHECK();
}

void refresh_fine_shift(ppe_solver* s, const double* coeff, const double* shift) {
  Level& L = s->levels[0];
  L.ap_ok = false;  // the kept A P no longer matches the new diagonal
  const int na = s->n_active;
  if (na == 0) return;
  int* flag = s->flag.get<int>(1);
  fill_int(s, flag, 0, 1);
  hipLaunchKernelGGL(k_refresh_diag, dim3(grid_for(na)), dim3(kBlock), 0, s->stream,
                     s->perm.as<int>(), na, s->adj_ptr.as<int>(), s->adj_nbr.as<int>(),
                     s->adj_face.as<int>(), s->active.as<int>(), coeff, shift, L.A.rp(), L.A.ci(),
                     L.A.val.as<double>(), L.diag.as<double>(), flag);
  PPE_LAUNCH_CHECK();
  double rho = 0.0;
  const double* rho_dev = level0_bound_async(s);
  int bad = 0;
  read_back(s, {ReadItem{flag, sizeof(int), &bad}, ReadItem{rho_dev, sizeof(double), &rho}});
  require(!(bad & 8), PPE_ERR_ARG, "diagonal shift must be finite and > 0 on every active cell");
  if (s->nlev > 1 || L.rho > 0.0) L.rho = rho;  // a level solved directly keeps rho = 0
}

}  // namespace ppe

// C ABI of the pressure-solve library (declared in include/ppe.h).
#include "common.h"

#include <cmath>
#include <cstring>
#include <new>

namespace {

thread_local std::string g_err;

template <class F>
ppe_status guarded(ppe_solver* s, F&& f) {
  // the solver's buffers come from its allocator while the call runs
  ppe::AllocScope scope(s ? &s->allocator : nullptr);
  try {
    if (s) s->err.clear();
    return f();
  } catch (const ppe::Error& e) {
    if (s) s->err = e.what();
    g_err = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    if (s) s->err = "host allocation failed";
    g_err = "host allocation failed";
    return PPE_ERR_OOM;
  } catch (const std::exception& e) {
    if (s) s->err = e.what();
    g_err = e.what();
    return PPE_ERR_INTERNAL;
  }
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

float elapsed_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  return ms;
}

double bytes_per_iteration(const ppe_solver* s) {
  // Algorithmic bytes of one PCG iteration: every matrix entry read once
  // (value + column index), every vector an operator touches read or written
  // once.  v = 8 bytes per vector value and per value of the outer operator;
  // vm = bytes per value of the V-cycle's matrices (4 for the FP32 copies of
  // the mixed mode; the coarsest dense inverse stays FP64).
  const double v = 8.0;
  const double vm = s->opt.precision == PPE_MIXED ? 4.0 : 8.0;
  double total = 0.0;
  const ppe::Level& L0 = s->levels[0];
  const double n0 = L0.n, off0 = (double)(L0.A.nnz - L0.n);
  // outer SpMV with p.q (diag, p, q) + x,r update (x,p,r,q -> x,r) + r.z + p update
  total += off0 * (v + 4) + 3 * v * n0 + 6 * v * n0 + 2 * v * n0 + 3 * v * n0;
  const int deg = s->opt.cheb_degree;
  for (int l = 0; l < s->nlev; ++l) {
    const ppe::Level& L = s->levels[l];
    const double n = L.n;
    const double mat = (l == 0) ? off0 * (vm + 4) + vm * n : (double)L.A.nnz * (vm + 4) + 4 * n;
    if (l == s->nlev - 1) {
      total += L.dense ? n * n * v + 2 * n * v : 2 * deg * (mat + 5 * v * n);
      continue;
    }
    // pre: first step elementwise (b, diag -> d, x) + (deg-1) fused steps;
    // residual; restriction; prolongation; post: deg fused steps
    const double fused = mat + 5 * v * n;  // x_in, b, d -> d, x_out (+diag in mat)
    total += 3 * v * n + vm * n + (deg - 1) * fused;
    total += mat + 3 * v * n;
    const ppe::Csr& R = L.R;
    const ppe::Csr& P = L.P;
    total += (double)R.nnz * (vm + 4) + 4.0 * R.n + v * n + v * R.n;
    total += (double)P.nnz * (vm + 4) + 4.0 * P.n + v * R.n + 2 * v * n;
    total += deg * fused;
  }
  return total;
}

}  // namespace

extern "C" {

void ppe_default_options(ppe_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = PPE_FP64;
  o->rtol = 1e-10;
  o->max_iter = 500;
  o->cheb_degree = 2;
  o->cheb_ratio = 7.0;
  o->coarse_max = 512;
  o->max_levels = 10;
  o->theta = 0.08;
  o->check_every = 2;
  o->stream = nullptr;
  o->use_graph = 1;
  o->autotune = 0;
  o->reuse_unchanged = 0;
  o->project_krylov = 1;
  o->smoother = PPE_SMOOTH_CHEBYSHEV;
  o->alloc = nullptr;
  o->free = nullptr;
  o->alloc_ctx = nullptr;
  o->coarse_reuse = 0;
  o->theta_decay = 0.5;
}

ppe_status ppe_create(const ppe_options* opt, ppe_solver** out) {
  return guarded(nullptr, [&]() -> ppe_status {
    ppe::require(out != nullptr, PPE_ERR_ARG, "out is NULL");
    *out = nullptr;
    ppe_options o;
    ppe_default_options(&o);
    if (opt) o = *opt;
    ppe::require(o.precision == PPE_FP64 || o.precision == PPE_MIXED, PPE_ERR_ARG, "bad precision");
    ppe::require(o.rtol > 0 && o.rtol < 1, PPE_ERR_ARG, "rtol must be in (0, 1)");
    ppe::require(o.max_iter >= 1, PPE_ERR_ARG, "max_iter must be >= 1");
    ppe::require(o.cheb_degree >= 1 && o.cheb_degree <= 8, PPE_ERR_ARG, "cheb_degree in [1, 8]");
    ppe::require(o.cheb_ratio > 1, PPE_ERR_ARG, "cheb_ratio must be > 1");
    ppe::require(o.smoother == PPE_SMOOTH_CHEBYSHEV || o.smoother == PPE_SMOOTH_L1JACOBI,
                 PPE_ERR_ARG, "smoother must be PPE_SMOOTH_CHEBYSHEV or PPE_SMOOTH_L1JACOBI");
    ppe::require((o.alloc == nullptr) == (o.free == nullptr), PPE_ERR_ARG,
                 "alloc and free must be set together");
    ppe::require(o.project_krylov == 0 || o.project_krylov == 1, PPE_ERR_ARG,
                 "project_krylov must be 0 or 1");
    ppe::require(o.coarse_max >= 1, PPE_ERR_ARG, "coarse_max must be >= 1");
    ppe::require(o.max_levels >= 1 && o.max_levels <= 32, PPE_ERR_ARG, "max_levels in [1, 32]");
    ppe::require(o.theta >= 0 && o.theta < 1, PPE_ERR_ARG, "theta in [0, 1)");
    ppe::require(o.theta_decay > 0 && o.theta_decay <= 1, PPE_ERR_ARG, "theta_decay in (0, 1]");
    ppe::require(o.coarse_reuse >= 0, PPE_ERR_ARG, "coarse_reuse must be >= 0");
    if (o.check_every < 1) o.check_every = 1;
    auto* s = new ppe_solver();
    s->opt = o;
    s->stream = static_cast<hipStream_t>(o.stream);
    s->allocator = ppe::Allocator{o.alloc, o.free, o.alloc_ctx, o.stream,
                                  {&s->stream, &s->side, &s->gstream}};
    ppe::AllocScope scope(&s->allocator);
    try {
      PPE_HIP(hipGetDevice(&s->device));
      int lds = 0;
      PPE_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, s->device));
      s->lds_max = (size_t)lds;
      PPE_HIP(hipEventCreate(&s->ev0));
      PPE_HIP(hipEventCreate(&s->ev1));
      PPE_HIP(hipStreamCreateWithFlags(&s->gstream, hipStreamNonBlocking));
      s->levels.reserve(o.max_levels + 1);
      unsigned int* c = s->counter.get<unsigned int>(1);
      PPE_HIP(hipMemsetAsync(c, 0, sizeof(unsigned int), s->stream));
      PPE_HIP(hipStreamSynchronize(s->stream));
    } catch (...) {
      if (s->ev0) (void)hipEventDestroy(s->ev0);
      if (s->ev1) (void)hipEventDestroy(s->ev1);
      if (s->gstream) (void)hipStreamDestroy(s->gstream);
      delete s;
      throw;
    }
    *out = s;
    return PPE_OK;
  });
}

void ppe_destroy(ppe_solver* s) {
  if (!s) return;
  DeviceGuard g(s->device);
  (void)hipStreamSynchronize(s->stream);
  for (auto& e : s->prof_ev)
    if (e) (void)hipEventDestroy(e);
  ppe::drop_graph(s);
  if (s->side) (void)hipStreamSynchronize(s->side);
  if (s->gstream) (void)hipStreamSynchronize(s->gstream);
  if (s->gstream) (void)hipStreamDestroy(s->gstream);
  s->gstream = nullptr;
  if (s->ev0) (void)hipEventDestroy(s->ev0);
  if (s->ev1) (void)hipEventDestroy(s->ev1);
  if (s->tev0) (void)hipEventDestroy(s->tev0);
  if (s->tev1) (void)hipEventDestroy(s->tev1);
  for (auto& e : s->chk_ev)
    if (e) (void)hipEventDestroy(e);
  if (s->fork_ev) (void)hipEventDestroy(s->fork_ev);
  if (s->join_ev) (void)hipEventDestroy(s->join_ev);
  if (s->side) {
    (void)hipStreamSynchronize(s->side);
    (void)hipStreamDestroy(s->side);
    s->side = nullptr;
  }
  if (s->box_h) (void)hipHostFree(s->box_h);
  delete s;
}

ppe_status ppe_set_mesh(ppe_solver* s, int32_t n_cells, int32_t n_faces, const int32_t* owner,
                        const int32_t* neigh) {
  if (!s) return PPE_ERR_ARG;
  return guarded(s, [&]() -> ppe_status {
    DeviceGuard g(s->device);
    ppe::require(n_cells > 0, PPE_ERR_ARG, "n_cells must be positive");
    ppe::require(n_faces >= 0, PPE_ERR_ARG, "n_faces must be >= 0");
    ppe::require(n_faces == 0 || (owner && neigh), PPE_ERR_ARG, "owner/neigh is NULL");
    s->have_mesh = false;
    s->geom_ok = false;
    s->have_prev = false;
    s->assembled = false;
    s->n_cells = n_cells;
    s->n_faces = n_faces;
    ppe::build_topology(s, owner, neigh);
    s->n_seg = 1;
    s->seg_cell_off = {0, n_cells};
    s->have_mesh = true;
    return PPE_OK;
  });
}

namespace {

// Shared body of ppe_assemble (shift NULL) and ppe_assemble_shifted.
ppe_status assemble_impl(ppe_solver* s, const double* face_coeff, const double* fl,
                         const double* shift) {
  if (!s) return PPE_ERR_ARG;
  return guarded(s, [&]() -> ppe_status {
    DeviceGuard g(s->device);
    ppe::require(s->have_mesh, PPE_ERR_STATE, "ppe_assemble before ppe_set_mesh");
    ppe::require((fl || shift) && (face_coeff || s->n_faces == 0), PPE_ERR_ARG,
                 "NULL input array");
    PPE_HIP(hipEventRecord(s->ev0, s->stream));
    // an unchanged system is recognised for pressure systems only
    if (!shift && !s->shifted && s->opt.reuse_unchanged && s->have_prev &&
        ppe::same_system(s, face_coeff, fl)) {
      // the masked system, its hierarchy and captured graphs stay valid
      s->assembled = true;
      s->stats.reused_setup += 1;
      PPE_HIP(hipEventRecord(s->ev1, s->stream));
      PPE_HIP(hipEventSynchronize(s->ev1));
      s->stats.setup_ms = elapsed_ms(s->ev0, s->ev1);
      return PPE_OK;
    }
    s->assembled = false;
    s->have_prev = false;
    s->solves_since_assemble = 0;
    ppe::drop_graph(s);
    ppe::assemble_fine(s, face_coeff, fl, shift);
    if (s->n_active > 0) {
      s->fine_reindexed = false;
      if (!shift && s->opt.coarse_reuse > 0 && ppe::reuse_coarse_levels(s)) {
        s->stats.coarse_reused += 1;
        s->fine_reindexed = true;
      } else {
        ppe::build_hierarchy(s);
        ppe::keep_base(s);
      }
      ppe::prepare_solve_levels(s);
      if (s->opt.precision == PPE_MIXED) ppe::make_fp32_hierarchy(s);
      if (s->opt.autotune) {
        const bool prof = s->prof;  // tuning launches are not measurements
        s->prof = false;
        ppe::autotune_levels(s);
        s->prof = prof;
      }
    } else {
      s->nlev = 1;
    }
    PPE_HIP(hipEventRecord(s->ev1, s->stream));
    PPE_HIP(hipEventSynchronize(s->ev1));
    s->stats.setup_ms = elapsed_ms(s->ev0, s->ev1);
    s->stats.n_active = s->n_active;
    s->stats.n_components = s->n_comp;
    s->stats.levels = s->n_active > 0 ? s->nlev : 0;
    double nnz0 = s->levels[0].A.nnz, tot = 0;
    for (int l = 0; l < s->nlev; ++l) tot += s->levels[l].A.nnz;
    s->stats.op_complexity = nnz0 > 0 ? tot / nnz0 : 1.0;
    s->stats.bytes_per_iter = s->n_active > 0 ? bytes_per_iteration(s) : 0.0;
    if (s->opt.reuse_unchanged && !shift) {
      // the coefficients this system was built from, for the next comparison
      double* pc = s->prev_coeff.get<double>(s->n_faces > 0 ? s->n_faces : 1);
      if (s->n_faces)
        PPE_HIP(hipMemcpyAsync(pc, face_coeff, sizeof(double) * s->n_faces, hipMemcpyDeviceToDevice,
                               s->stream));
      PPE_HIP(hipStreamSynchronize(s->stream));
      s->have_prev = true;
    }
    s->assembled = true;
    return PPE_OK;
  });
}

}  // namespace

ppe_status ppe_assemble(ppe_solver* s, const double* face_coeff, const double* fl) {
  if (s && !fl) {
    s->err = "NULL input array";
    return PPE_ERR_ARG;
  }
  return assemble_impl(s, face_coeff, fl, nullptr);
}

ppe_status ppe_refresh_shift(ppe_solver* s, const double* face_coeff, const double* diag_shift) {
  if (!s) return PPE_ERR_ARG;
  return guarded(s, [&]() -> ppe_status {
    DeviceGuard g(s->device);
    ppe::require(s->assembled && s->shifted, PPE_ERR_STATE,
                 "ppe_refresh_shift needs a shifted system (ppe_assemble_shifted)");
    ppe::require(diag_shift && (face_coeff || s->n_faces == 0), PPE_ERR_ARG, "NULL input array");
    PPE_HIP(hipEventRecord(s->ev0, s->stream));
    ppe::drop_graph(s);
    try {
      ppe::refresh_fine_shift(s, face_coeff, diag_shift);
    } catch (...) {
      s->assembled = false;  // the finest level may be half rewritten
      throw;
    }
    ppe::prepare_solve_levels(s);
    if (s->opt.precision == PPE_MIXED) ppe::make_fp32_hierarchy(s);
    PPE_HIP(hipEventRecord(s->ev1, s->stream));
    PPE_HIP(hipEventSynchronize(s->ev1));
    s->stats.setup_ms = elapsed_ms(s->ev0, s->ev1);
    return PPE_OK;
  });
}

ppe_status ppe_assemble_shifted(ppe_solver* s, const double* face_coeff, const double* fl,
                                const double* diag_shift) {
  if (s && !diag_shift) {
    s->err = "NULL diagonal shift";
    return PPE_ERR_ARG;
  }
  return assemble_impl(s, face_coeff, fl, diag_shift);
}

ppe_status ppe_solve(ppe_solver* s, const double* rhs, double* p, int use_x0, ppe_stats* stats) {
  if (!s) return PPE_ERR_ARG;
  return guarded(s, [&]() -> ppe_status {
    DeviceGuard g(s->device);
    ppe::require(s->assembled, PPE_ERR_STATE, "ppe_solve before ppe_assemble");
    ppe::require(rhs && p, PPE_ERR_ARG, "NULL rhs or p");
    PPE_HIP(hipEventRecord(s->ev0, s->stream));
    ppe_status st = ppe::pcg_solve(s, rhs, p, use_x0, &s->pred_solve);
    s->solves_since_assemble += 1;
    PPE_HIP(hipEventRecord(s->ev1, s->stream));
    PPE_HIP(hipEventSynchronize(s->ev1));
    s->stats.solve_ms = elapsed_ms(s->ev0, s->ev1);
    if (stats) *stats = s->stats;
    if (st == PPE_ERR_BREAKDOWN) s->err = "PCG breakdown (p.Ap <= 0, r.z <= 0 or non-finite)";
    return st;
  });
}

ppe_status ppe_set_geometry(ppe_solver* s, int32_t n_nodes, const double* nodes,
                            const int32_t* face_nodes, const int32_t* cell_nodes,
                            const double* cell_centre, const double* face_area) {
  if (!s) return PPE_ERR_ARG;
  return guarded(s, [&]() -> ppe_status {
    DeviceGuard g(s->device);
    ppe::require(s->have_mesh, PPE_ERR_STATE, "ppe_set_geometry before ppe_set_mesh");
    ppe::require(n_nodes > 0, PPE_ERR_ARG, "n_nodes must be positive");
    ppe::require(nodes && cell_nodes && cell_centre && (s->n_faces == 0 || (face_nodes && face_area)),
                 PPE_ERR_ARG, "NULL geometry array");
    ppe::set_geometry(s, n_nodes, nodes, face_nodes, cell_nodes, cell_centre, face_area);
    return PPE_OK;
  });
}

namespace {

ppe_status project_impl(ppe_solver* s, const double* face_coeff, const double* ustar, double rho,
                        double dt, double* p, double* flux, double* u, ppe_project_stats* stats,
                        bool use_x0) {
  if (!s) return PPE_ERR_ARG;
  return guarded(s, [&]() -> ppe_status {
    DeviceGuard g(s->device);
    ppe::require(s->assembled && !s->shifted, PPE_ERR_STATE,
                 "ppe_project needs a pressure system (ppe_assemble)");
    ppe::require(s->geom_ok, PPE_ERR_STATE, "ppe_project before ppe_set_geometry");
    ppe::require(s->n_seg == 1, PPE_ERR_STATE, "ppe_project solves one sample at a time");
    ppe::require(face_coeff && ustar && p && u && (flux || s->n_faces == 0), PPE_ERR_ARG,
                 "NULL array");
    ppe::require(std::isfinite(rho) && rho > 0 && std::isfinite(dt) && dt > 0, PPE_ERR_ARG,
                 "rho and dt must be finite and > 0");
    PPE_HIP(hipEventRecord(s->ev0, s->stream));
    ppe_project_stats st{};
    const ppe_status r = ppe::project(s, face_coeff, ustar, rho, dt, p, flux, u, &st, use_x0);
    PPE_HIP(hipEventRecord(s->ev1, s->stream));
    PPE_HIP(hipEventSynchronize(s->ev1));
    st.ms = elapsed_ms(s->ev0, s->ev1);
    if (stats) *stats = st;
    return r;
  });
}

}  // namespace

ppe_status ppe_project(ppe_solver* s, const double* face_coeff, const double* ustar, double rho,
                       double dt, double* p, double* flux, double* u, ppe_project_stats* stats) {
  return project_impl(s, face_coeff, ustar, rho, dt, p, flux, u, stats, false);
}

ppe_status ppe_project_warm(ppe_solver* s, const double* face_coeff, const double* ustar,
                            double rho, double dt, double* p, double* flux, double* u,
                            ppe_project_stats* stats) {
  return project_impl(s, face_coeff, ustar, rho, dt, p, flux, u, stats, true);
}

ppe_status ppe_face_gradient(ppe_solver* s, const double* face_coeff, double rho, const double* p,
                             double* grad, double* cross) {
  if (!s) return PPE_ERR_ARG;
  return guarded(s, [&]() -> ppe_status {
    DeviceGuard g(s->device);
    ppe::require(s->assembled && s->geom_ok && !s->shifted, PPE_ERR_STATE,
                 "ppe_face_gradient needs ppe_assemble and ppe_set_geometry");
    ppe::require(face_coeff && p && grad && cross, PPE_ERR_ARG, "NULL array");
    ppe::require(std::isfinite(rho) && rho > 0, PPE_ERR_ARG, "rho must be finite and > 0");
    double* t = s->pj_t.get<double>(3 * (size_t)(s->n_faces > 0 ? s->n_faces : 1));
    ppe::cross_vectors(s, face_coeff, rho, t);
    ppe::face_gradient(s, p, t, grad, cross);
    PPE_HIP(hipStreamSynchronize(s->stream));
    return PPE_OK;
  });
}

ppe_status ppe_set_segments(ppe_solver* s, int32_t n_samples, const int32_t* off) {
  if (!s) return PPE_ERR_ARG;
  return guarded(s, [&]() -> ppe_status {
    DeviceGuard g(s->device);
    ppe::require(s->have_mesh, PPE_ERR_STATE, "ppe_set_segments before ppe_set_mesh");
    ppe::require(n_samples >= 1 && off != nullptr, PPE_ERR_ARG, "need n_samples >= 1 and offsets");
    ppe::require(off[0] == 0 && off[n_samples] == s->n_cells, PPE_ERR_ARG,
                 "offsets must run from 0 to n_cells");
    for (int k = 0; k < n_samples; ++k)
      ppe::require(off[k] < off[k + 1], PPE_ERR_ARG, "offsets must be strictly ascending");
    std::vector<int> o(off, off + n_samples + 1);
    ppe::check_segments(s, o);
    s->n_seg = n_samples;
    s->seg_cell_off = o;
    s->assembled = false;
    s->have_prev = false;
    return PPE_OK;
  });
}

ppe_status ppe_get_segment_stats(const ppe_solver* s, int32_t* iterations, double* rel_residual) {
  if (!s || !iterations || !rel_residual) return PPE_ERR_ARG;
  if ((int)s->seg_iters_h.size() != s->n_seg) return PPE_ERR_STATE;
  for (int k = 0; k < s->n_seg; ++k) {
    iterations[k] = s->seg_iters_h[k];
    rel_residual[k] = s->seg_res_h[k];
  }
  return PPE_OK;
}

ppe_status ppe_get_stats(const ppe_solver* s, ppe_stats* stats) {
  if (!s || !stats) return PPE_ERR_ARG;
  *stats = s->stats;
  return PPE_OK;
}

const char* ppe_status_string(ppe_status st) {
  switch (st) {
    case PPE_OK: return "ok";
    case PPE_NOT_CONVERGED: return "not converged";
    case PPE_ERR_ARG: return "invalid argument";
    case PPE_ERR_HIP: return "HIP runtime error";
    case PPE_ERR_OOM: return "out of device memory";
    case PPE_ERR_BREAKDOWN: return "Krylov breakdown";
    case PPE_ERR_STATE: return "call out of order";
    case PPE_ERR_INTERNAL: return "internal limit exceeded";
  }
  return "unknown status";
}

const char* ppe_last_error(const ppe_solver* s) { return s ? s->err.c_str() : g_err.c_str(); }

// ------------------------------------------------------------------ inspection
static ppe_status check_level(const ppe_solver* s, int level) {
  if (!s) return PPE_ERR_ARG;
  if (!s->assembled) return PPE_ERR_STATE;
  if (level < 0 || level >= s->nlev || s->n_active == 0) return PPE_ERR_ARG;
  return PPE_OK;
}

ppe_status ppe_level_info(const ppe_solver* s, int level, int32_t* n_rows, int64_t* nnz_a,
                          int64_t* nnz_p, int32_t* n_agg, double* rho) {
  ppe_status st = check_level(s, level);
  if (st != PPE_OK) return st;
  const ppe::Level& L = s->levels[level];
  const bool coarsest = level == s->nlev - 1;
  if (n_rows) *n_rows = L.n;
  if (nnz_a) *nnz_a = L.A.nnz;
  if (nnz_p) *nnz_p = coarsest ? 0 : L.P.nnz;
  if (n_agg) *n_agg = coarsest ? 0 : L.n_agg;
  if (rho) *rho = L.rho;
  return PPE_OK;
}

ppe_status ppe_get_level_launch(const ppe_solver* s, int level, int32_t* choice) {
  ppe_status st = check_level(s, level);
  if (st != PPE_OK) return st;
  if (!choice) return PPE_ERR_ARG;
  const ppe::Level& L = s->levels[level];
  choice[0] = L.lpr_a;
  choice[1] = L.lpr_r;
  choice[2] = L.lpr_p;
  choice[3] = L.fuse0 ? 1 : 0;
  choice[4] = L.fuse_p ? 1 : 0;
  return PPE_OK;
}

ppe_status ppe_set_level_launch(ppe_solver* s, int level, const int32_t* choice) {
  ppe_status st = check_level(s, level);
  if (st != PPE_OK) return st;
  if (!choice) return PPE_ERR_ARG;
  auto ok = [](int v, int lo) {
    return v == 0 || (v >= lo && v <= 64 && (v & (v - 1)) == 0);
  };
  if (!ok(choice[0], 4) || !ok(choice[1], 1) || !ok(choice[2], 1) ||
      (choice[3] != 0 && choice[3] != 1) || (choice[4] != 0 && choice[4] != 1))
    return PPE_ERR_ARG;
  ppe::Level& L = s->levels[level];
  L.lpr_a = choice[0];
  L.lpr_r = choice[1];
  L.lpr_p = choice[2];
  L.fuse0 = choice[3] != 0;
  L.fuse_p = choice[4] != 0;
  ppe::drop_graph(s);  // a captured graph holds the old launches
  return PPE_OK;
}

static ppe_status copy_csr(ppe_solver* s, const ppe::Csr& A, int32_t* rp, int32_t* ci, double* v) {
  if (!rp || !ci || !v) return PPE_ERR_ARG;
  return guarded(s, [&]() -> ppe_status {
    DeviceGuard g(s->device);
    PPE_HIP(hipMemcpyAsync(rp, A.rp(), sizeof(int) * (A.n + 1), hipMemcpyDeviceToDevice, s->stream));
    if (A.nnz) {
      PPE_HIP(hipMemcpyAsync(ci, A.ci(), sizeof(int) * A.nnz, hipMemcpyDeviceToDevice, s->stream));
      PPE_HIP(hipMemcpyAsync(v, A.v(), sizeof(double) * A.nnz, hipMemcpyDeviceToDevice, s->stream));
    }
    PPE_HIP(hipStreamSynchronize(s->stream));
    return PPE_OK;
  });
}

ppe_status ppe_copy_level_matrix(const ppe_solver* s, int level, int32_t* row_ptr, int32_t* col,
                                 double* val) {
  ppe_status st = check_level(s, level);
  if (st != PPE_OK) return st;
  return copy_csr(const_cast<ppe_solver*>(s), s->levels[level].A, row_ptr, col, val);
}

ppe_status ppe_copy_prolongator(const ppe_solver* s, int level, int32_t* row_ptr, int32_t* col,
                                double* val) {
  ppe_status st = check_level(s, level);
  if (st != PPE_OK) return st;
  if (level == s->nlev - 1) return PPE_ERR_ARG;
  return copy_csr(const_cast<ppe_solver*>(s), s->levels[level].P, row_ptr, col, val);
}

ppe_status ppe_copy_aggregates(const ppe_solver* s, int level, int32_t* agg) {
  ppe_status st = check_level(s, level);
  if (st != PPE_OK) return st;
  if (level == s->nlev - 1 || !agg) return PPE_ERR_ARG;
  // a finest level re-indexed onto kept coarse levels has no aggregates of
  // its own (its prolongator rows come from the earlier build)
  if (level == 0 && s->fine_reindexed) return PPE_ERR_STATE;
  ppe_solver* m = const_cast<ppe_solver*>(s);
  return guarded(m, [&]() -> ppe_status {
    DeviceGuard g(s->device);
    const ppe::Level& L = s->levels[level];
    PPE_HIP(hipMemcpyAsync(agg, L.agg.as<int>(), sizeof(int) * L.n, hipMemcpyDeviceToDevice,
                           s->stream));
    PPE_HIP(hipStreamSynchronize(s->stream));
    return PPE_OK;
  });
}

ppe_status ppe_copy_mask(const ppe_solver* s, int32_t* compact_id, int32_t* component) {
  if (!s) return PPE_ERR_ARG;
  if (!s->assembled) return PPE_ERR_STATE;
  if (!compact_id || !component) return PPE_ERR_ARG;
  ppe_solver* m = const_cast<ppe_solver*>(s);
  return guarded(m, [&]() -> ppe_status {
    DeviceGuard g(s->device);
    PPE_HIP(hipMemcpyAsync(compact_id, s->cid.as<int>(), sizeof(int) * s->n_cells,
                           hipMemcpyDeviceToDevice, s->stream));
    PPE_HIP(hipMemcpyAsync(component, s->comp_full.as<int>(), sizeof(int) * s->n_cells,
                           hipMemcpyDeviceToDevice, s->stream));
    PPE_HIP(hipStreamSynchronize(s->stream));
    return PPE_OK;
  });
}

ppe_status ppe_apply_matrix(ppe_solver* s, int level, const double* x, double* y) {
  ppe_status st = check_level(s, level);
  if (st != PPE_OK) return st;
  if (!x || !y) return PPE_ERR_ARG;
  return guarded(s, [&]() -> ppe_status {
    DeviceGuard g(s->device);
    ppe::spmv(s, s->levels[level], x, y);
    PPE_HIP(hipStreamSynchronize(s->stream));
    return PPE_OK;
  });
}

ppe_status ppe_apply_vcycle(ppe_solver* s, const double* r, double* z) {
  ppe_status st = check_level(s, 0);
  if (st != PPE_OK) return st;
  if (!r || !z) return PPE_ERR_ARG;
  return guarded(s, [&]() -> ppe_status {
    DeviceGuard g(s->device);
    ppe::vcycle(s, 0, r, z);
    PPE_HIP(hipStreamSynchronize(s->stream));
    return PPE_OK;
  });
}

ppe_status ppe_profile_enable(ppe_solver* s, int enable) {
  if (!s) return PPE_ERR_ARG;
  return guarded(s, [&]() -> ppe_status {
    DeviceGuard g(s->device);
    ppe::profile_enable(s, enable != 0);
    return PPE_OK;
  });
}

ppe_status ppe_profile_count(const ppe_solver* s, int32_t* n_kernels) {
  if (!s || !n_kernels) return PPE_ERR_ARG;
  return guarded(const_cast<ppe_solver*>(s), [&]() -> ppe_status {
    DeviceGuard g(s->device);
    ppe::profile_harvest(const_cast<ppe_solver*>(s));
    *n_kernels = (int32_t)s->prof_table.size();
    return PPE_OK;
  });
}

ppe_status ppe_profile_entry(const ppe_solver* s, int32_t k, char* name, int32_t name_cap,
                             int64_t* launches, double* kernel_ms, double* bytes) {
  if (!s || !name || name_cap < 1 || !launches || !kernel_ms || !bytes) return PPE_ERR_ARG;
  if (k < 0 || k >= (int32_t)s->prof_table.size()) return PPE_ERR_ARG;
  const auto& e = s->prof_table[k];
  const size_t len = std::min(e.name.size(), (size_t)name_cap - 1);
  std::memcpy(name, e.name.data(), len);
  name[len] = '\0';
  *launches = e.launches;
  *kernel_ms = e.ms;
  *bytes = e.bytes;
  return PPE_OK;
}

}  // extern "C"

/*
 * ppe.h - masked pressure-correction Poisson solve on unstructured hexahedral
 * finite-volume meshes, smoothed-aggregation AMG preconditioned conjugate
 * gradients, on AMD Instinct MI355X (gfx950).
 *
 * What is solved (arXiv:1810.08572, Shahane et al., "Finite Volume Simulation
 * Framework for Die Casting with Uncertainty Quantification"):
 *   - the pressure Poisson equation of the fractional-step method, Eq. 9,
 *     discretised with the direct (two-point) term of the face-gradient split
 *     of Eq. 11; face f between cells o and n contributes c_f (p_n - p_o) to
 *     the balance of o, with c_f = |S_f| / (rho n.d) supplied by the caller;
 *   - with the solidification modification of section 2.4.2: cells whose
 *     liquid fraction is exactly 0 (tag S) are removed, every face with a
 *     removed owner is blocked (zero flux, i.e. Neumann: its coefficient
 *     leaves the diagonal too, case 3 and modification step 2), the rows of
 *     the remaining liquid/mushy cells are re-assembled (step 3);
 *   - every connected set of remaining cells (a liquid pocket, section 2.5)
 *     is made non-singular by pinning its lowest-index cell: that cell's row
 *     and column are zeroed except the diagonal (1 for an isolated cell), and
 *     its right-hand side entry is replaced by 0;
 *   - solved to ||b' - A p||_2 <= rtol ||b'||_2 (true residual, FP64) by
 *     conjugate gradients (the Krylov solver of section 2.5) preconditioned
 *     by one smoothed-aggregation AMG V-cycle (the multigrid of section 2.5).
 *
 * Conventions
 *   - Every array argument is a DEVICE pointer (HIP device memory of the
 *     device that was current at ppe_create) owned by the caller.  Inputs are
 *     read in stream order on the solver's stream and must stay valid until
 *     the call returns; outputs are complete when the call returns (each call
 *     synchronises the solver's stream before returning).
 *   - Indices are int32, cell numbering 0..n_cells-1; values are FP64.
 *   - A solver is not thread-safe; use one solver per host thread.
 *   - Every function returns a ppe_status; a negative value means the call
 *     failed, its outputs are undefined, and ppe_last_error() describes why.
 */
#ifndef PPE_H
#define PPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ppe_solver ppe_solver; /* opaque: mesh topology, hierarchy, workspace */

typedef enum {
  PPE_OK = 0,
  PPE_NOT_CONVERGED = 1,    /* max_iter reached; p holds the last iterate */
  PPE_ERR_ARG = -1,         /* invalid argument or input data */
  PPE_ERR_HIP = -2,         /* a HIP runtime call failed */
  PPE_ERR_OOM = -3,         /* device allocation failed */
  PPE_ERR_BREAKDOWN = -4,   /* p.Ap <= 0, r.z <= 0 or a non-finite scalar */
  PPE_ERR_STATE = -5,       /* call out of order (e.g. solve before assemble) */
  PPE_ERR_INTERNAL = -6     /* a bounded internal table overflowed */
} ppe_status;

typedef enum { PPE_FP64 = 0, PPE_MIXED = 1 } ppe_precision;

/* Relaxation of the V-cycle (section 2.5 couples the multigrid levels by
 * relaxation without naming it): Chebyshev polynomial smoothing of D^-1 A,
 * or l1-Jacobi sweeps x <- x + D_l1^-1 (b - A x) with D_l1 the row l1 norms
 * sum_j |a_ij| (convergent for every SPD A, no spectral bound needed). */
typedef enum { PPE_SMOOTH_CHEBYSHEV = 0, PPE_SMOOTH_L1JACOBI = 1 } ppe_smoother;

/* Caller-provided device allocator (for example PyTorch's caching
 * allocator).  alloc returns a device pointer to at least `bytes` bytes of
 * the solver's device, usable in stream order on `stream` (the solver's
 * stream), or NULL on failure (the call then fails with PPE_ERR_OOM).
 * free releases a pointer alloc returned; the library drains its streams
 * before calling it, so the block is idle.  ctx is passed through. */
typedef void* (*ppe_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*ppe_free_fn)(void* ptr, void* ctx);

typedef struct {
  int precision;      /* ppe_precision; PPE_MIXED = FP32-stored hierarchy, FP64
                         arithmetic and outer PCG (see ppe_solve) */
  double rtol;        /* relative residual target, default 1e-10 */
  int max_iter;       /* PCG iteration cap, default 500 */
  int cheb_degree;    /* Chebyshev smoother degree per application, default 2 */
  double cheb_ratio;  /* smoothing interval [rho/ratio, rho], default 7 */
  int coarse_max;     /* stop coarsening at <= this many rows, default 512 (the
                         coarsest level, up to 1024 rows, is inverted) */
  int max_levels;     /* hierarchy depth cap, default 10 */
  double theta;       /* strength threshold of the finest level, default 0.08;
                         level l uses theta * theta_decay^l */
  int check_every;    /* PCG iterations between host convergence checks when not
                         replaying graphs (a graph replay of two iterations is
                         followed by one check), default 2; iterations past
                         convergence leave a converged system untouched, so
                         the result and iteration count do not depend on it */
  void* stream;       /* hipStream_t used for every launch; NULL = default stream */
  int use_graph;      /* replay PCG iterations from a captured HIP graph, default 1 */
  int autotune;       /* 1: at assembly, time the candidate launch choices of each
                         level's solve kernels (lanes per row of the smoother,
                         restriction and prolongation; fused or split first
                         smoothing steps) and keep the fastest, cached per level
                         shape.  Lanes per row change the order of the row sums,
                         so results then depend on the choices (to rounding).
                         Default 0: fixed rules, bitwise reproducible. */
  int reuse_unchanged; /* 1: ppe_assemble first compares the face coefficients and
                         the removed-cell mask (liquid fraction > 0 or not; the
                         matrix depends on nothing else) with the previous
                         successful assembly's, and keeps the masked system, the
                         AMG hierarchy and captured graphs when both are
                         unchanged.  Default 0: every assembly rebuilds. */
  int project_krylov; /* outer iteration of ppe_project for the non-symmetric
                         system (L - X) p = b' with the cross term implicit:
                         1 (default) BiCGSTAB preconditioned by one V-cycle of
                         L's hierarchy per application, falling back to
                         deferred correction on breakdown; 0 deferred
                         correction, each pass an AMG-PCG solve of L.  Both
                         stop on the same true residual.  (Section 2.5 pairs
                         its AMG with Krylov solvers without naming them and
                         uses a single-grid BiCGSTAB only as the fallback when
                         the AMG diverges; BiCGSTAB is used here because the
                         implicit cross term makes the system non-symmetric.) */
  int smoother;       /* ppe_smoother, default PPE_SMOOTH_CHEBYSHEV; cheb_degree is
                         the number of steps per application either way (the
                         polynomial degree, or the l1-Jacobi sweeps) */
  ppe_alloc_fn alloc; /* device memory of the solver (hierarchy, workspace, and
                         a time-step driver's own arrays) comes from alloc/free
                         when both are set; both NULL (default): hipMalloc and
                         hipFree.  Setting one without the other is PPE_ERR_ARG. */
  ppe_free_fn free;
  void* alloc_ctx;    /* passed to alloc and free */
  int coarse_reuse;   /* > 0: after a full setup, up to this many later pressure
                         assemblies whose active set differs from that build's
                         in at most 10% of its cells keep its coarse levels and
                         rebuild only the finest one: the new masked operator,
                         its diagonal and Gershgorin bound, and a prolongator
                         made of the earlier finest prolongator's rows of the
                         same cells (empty for pins and for cells that build
                         did not have), R = P^T.  The V-cycle stays a symmetric
                         positive definite preconditioner of the new system, so
                         the solve meets the same tolerance; only its
                         iteration count may differ from a fresh setup's.
                         Default 0: every changed mask gets a full setup. */
  double theta_decay; /* factor of the strength threshold from one level to the
                         next coarser one, in (0, 1], default 0.5 (the
                         level-halved threshold of Vanek, Mandel and Brezina's
                         smoothed aggregation); 1 keeps theta on every level */
} ppe_options;

typedef struct {
  int iterations;        /* PCG iterations of the last solve */
  double rel_residual;   /* true ||b'-Ap||/||b'|| at exit (0 when b' = 0) */
  double setup_ms;       /* last ppe_assemble wall time */
  double solve_ms;       /* last ppe_solve wall time */
  int n_active;          /* cells with f_l > 0 */
  int n_components;      /* liquid pockets (= pinned cells); 0 for a shifted system */
  int levels;            /* AMG levels including the finest */
  double op_complexity;  /* sum of level nnz / finest nnz */
  double bytes_per_iter; /* algorithmic bytes one PCG iteration moves */
  int reused_setup;      /* assemblies that kept an unchanged system (reuse_unchanged) */
  int coarse_reused;     /* assemblies that kept the coarse levels of an earlier
                            build across a changed mask (coarse_reuse) */
} ppe_stats;

/* Fill *opt with the defaults listed above. */
void ppe_default_options(ppe_options* opt);

/* Create a solver on the current HIP device.  opt may be NULL (defaults).
 * Errors: PPE_ERR_ARG for out-of-range options, PPE_ERR_HIP. */
ppe_status ppe_create(const ppe_options* opt, ppe_solver** out);

/* Destroy a solver and free its device memory.  NULL is accepted. */
void ppe_destroy(ppe_solver* s);

/* Mesh topology, section 2.3: face f joins owner[f] and neigh[f]
 * (neigh[f] = -1: wall face, which carries no flux).  Copies what it needs;
 * the arrays may be freed after return.
 * Errors (PPE_ERR_ARG): n_cells <= 0, n_faces < 0, an index out of range,
 * owner == neigh, two faces joining the same pair of cells. */
ppe_status ppe_set_mesh(ppe_solver* s, int32_t n_cells, int32_t n_faces,
                        const int32_t* owner, const int32_t* neigh);

/* Masked assembly and AMG setup (section 2.4.2 and section 2.5).
 * face_coeff[n_faces]: c_f, finite and > 0 on interior faces (ignored on
 * walls).  liquid_fraction[n_cells]: finite, in [0,1]; 0 removes the cell.
 * Errors: PPE_ERR_STATE before ppe_set_mesh; PPE_ERR_ARG on invalid data;
 * PPE_ERR_OOM; PPE_ERR_INTERNAL if a setup table overflows. */
ppe_status ppe_assemble(ppe_solver* s, const double* face_coeff,
                        const double* liquid_fraction);

/* Shifted assembly for the implicit parts of the momentum and energy
 * equations (section 2.2, Eq. 6 and the energy step): the same AMG-PCG
 * solves A = diag(diag_shift) + L, L the face-coefficient operator over the
 * open faces (both cells kept), with no pins (A is non-singular when every
 * kept row has a positive shift).  diag_shift[n_cells]: finite and > 0 on
 * kept cells (ignored elsewhere).  liquid_fraction may be NULL (every cell
 * kept); otherwise cells with 0 are removed as in ppe_assemble (a removed
 * neighbour's coupling must then be folded into the shift by the caller).
 * ppe_solve then returns the solution on kept cells and 0 elsewhere; no
 * right-hand-side entry is replaced.  ppe_project, ppe_face_gradient and
 * the warm-start calls need a pressure system and return PPE_ERR_STATE
 * after this call; the reuse_unchanged option does not apply.  Errors as
 * ppe_assemble, and PPE_ERR_ARG on a bad or NULL shift. */
ppe_status ppe_assemble_shifted(ppe_solver* s, const double* face_coeff,
                                const double* liquid_fraction, const double* diag_shift);

/* A new diagonal shift for the system of the last ppe_assemble_shifted, with
 * the same face_coeff and mask (the caller guarantees both): the finest
 * level's diagonal, its spectral bound and Chebyshev coefficients are
 * recomputed; the coarser levels of the hierarchy are kept as they are.  The
 * V-cycle stays a symmetric positive-definite preconditioner and ppe_solve
 * solves the new system to rtol; only its iteration count may differ from a
 * fresh assembly's.  For repeated solves whose matrices differ only on the
 * diagonal (the latent-heat Picard passes of the energy step).  Launch
 * choices return to the fixed rules.  Errors: PPE_ERR_STATE unless the last
 * assembly was shifted; PPE_ERR_ARG on NULL arrays or a shift that is not
 * finite and > 0 on a kept cell (the system must then be assembled again:
 * ppe_solve returns PPE_ERR_STATE until it is). */
ppe_status ppe_refresh_shift(ppe_solver* s, const double* face_coeff, const double* diag_shift);

/* Solve A p = b' (Eq. 9 as modified in section 2.4.2) by conjugate gradients
 * preconditioned with one V-cycle per iteration (section 2.5), until the
 * recomputed true residual meets rtol ||b'||.  With PPE_MIXED the V-cycle
 * reads FP32 copies of the hierarchy's values (level operators, diagonals,
 * P, R; the coarsest dense inverse stays FP64) and computes in FP64 on FP64
 * vectors, so it is one fixed symmetric positive definite preconditioner and
 * plain CG applies; the outer residual, dots and updates are FP64.
 * rhs[n_cells]: entries of removed cells are ignored, pins are replaced by 0.
 * p[n_cells]: in: initial guess if use_x0 != 0; out: pressure, exactly 0 on
 * removed cells and pins.  stats: host pointer, may be NULL.
 * Returns PPE_OK, PPE_NOT_CONVERGED (p = last iterate, stats filled),
 * PPE_ERR_STATE before ppe_assemble, PPE_ERR_BREAKDOWN, PPE_ERR_HIP.
 * An empty active set or b' = 0 returns PPE_OK with p = 0 (or x0 masked)
 * after 0 iterations. */
ppe_status ppe_solve(ppe_solver* s, const double* rhs, double* p, int use_x0,
                     ppe_stats* stats);

/* Independent samples (uncertainty-quantification batches, section 3 of the
 * paper runs one deterministic simulation per collocation sample): cells
 * [cell_offsets[k], cell_offsets[k+1]) form sample k.  offsets is a HOST
 * array of n_samples + 1 ascending ints from 0 to n_cells; no interior face
 * may join two samples.  Each sample then gets its own conjugate-gradient
 * scalars and its own stopping test ||b'_k - A_k p_k|| <= rtol ||b'_k||, so
 * one call solves every sample as if it were solved alone; the AMG
 * hierarchy is shared (it never couples samples).  Setting one sample that
 * covers all cells restores the default.  Call after ppe_set_mesh; takes
 * effect at the next ppe_assemble.
 * Errors: PPE_ERR_STATE before ppe_set_mesh; PPE_ERR_ARG for bad offsets or
 * a face joining two samples. */
ppe_status ppe_set_segments(ppe_solver* s, int32_t n_samples, const int32_t* cell_offsets);

/* Per-sample results of the last solve: PCG iterations until that sample
 * met its tolerance, and its true relative residual.  Host arrays of
 * n_samples (from ppe_set_segments; 1 by default). */
ppe_status ppe_get_segment_stats(const ppe_solver* s, int32_t* iterations, double* rel_residual);

/* Statistics of the last assemble/solve.  With several samples, iterations
 * and rel_residual are the maxima over the samples. */
ppe_status ppe_get_stats(const ppe_solver* s, ppe_stats* stats);

/* ---- Pressure-correction step with cross diffusion (sections 2.3, 2.4.2,
 * 2.4.3). ----
 * The full discretisation of the face normal gradient (Eq. 11): the direct
 * term c_f (p_C2 - p_C1) of the solved matrix plus the cross term
 * t_f . grad(p)_f, t_f = S_f / rho - c_f d_f, with grad(p)_f reconstructed in
 * the local frame C1C2, V1V3, V2V4 from vertex means of the cells around
 * each vertex (Eq. 12).  Solid cells leave each face stencil with their
 * coefficients spread equally over the remaining cells (case 2, Eq. 15-16);
 * faces with a solid owner carry nothing (case 3). */

/* Geometry of the mesh set by ppe_set_mesh (device arrays, copied):
 * nodes[3 n_nodes] (x, y, z interleaved); face_nodes[4 n_faces] = V1..V4 of
 * each face, ordered so that (V3 - V1) x (V4 - V2) / 2 = face_area, the area
 * vector pointing from owner to neighbour (walls' entries must be valid
 * indices but are not used); cell_nodes[8 n_cells], a cell's corners;
 * cell_centre[3 n_cells]; face_area[3 n_faces].  Builds each interior face's
 * gradient stencil over the cells sharing one of its vertices.
 * Errors: PPE_ERR_STATE before ppe_set_mesh; PPE_ERR_ARG for an index out of
 * range, a vertex repeated within a cell or shared by more than 16 cells, a
 * face whose vertices are not corners of both its cells, or a degenerate
 * local frame. */
ppe_status ppe_set_geometry(ppe_solver* s, int32_t n_nodes, const double* nodes,
                            const int32_t* face_nodes, const int32_t* cell_nodes,
                            const double* cell_centre, const double* face_area);

typedef struct {
  int outer;             /* deferred correction: passes (one AMG-PCG solve
                            each); BiCGSTAB: iterations */
  int pcg_iterations;    /* deferred correction: PCG iterations summed over
                            the passes; BiCGSTAB: V-cycles applied (two per
                            iteration) */
  double rel_residual;   /* ||b' + X p - L p|| / ||b'|| at exit, FP64 */
  double ms;             /* wall time of the call */
} ppe_project_stats;

/* One pressure-correction step on the assembled system (Eq. 9 with both
 * terms of Eq. 11, then Eq. 17 and Eq. 8):
 *   F*_f = (u*_C1 + u*_C2)/2 . S_f on open faces, b'_i = -(1/dt) sum s_if F*_f;
 *   (L - X) p = b' on the active cells, pinned as ppe_solve pins, solved by
 *   the outer iteration option project_krylov selects - BiCGSTAB
 *   right-preconditioned by one V-cycle of L (default), or deferred
 *   correction around the AMG-PCG solve of L (each pass solves
 *   L delta = b' + X p - L p to a loose tolerance) - until
 *   ||b' + X p - L p|| <= 0.1 rtol ||b'|| (a decade of margin: loose inner
 *   solves leave smooth residual modes, which the pressure error
 *   amplifies);
 *   flux[f] = F*_f - dt (c_f (p_C2 - p_C1) + t_f . grad(p)_f) on open faces,
 *   0 on blocked and wall faces;
 *   u[3 n_cells] = u* - (dt/rho) * (mean of the open faces' gradients) on
 *   active cells (u* where a cell has no open face), 0 on removed cells.
 * face_coeff must be the array given to ppe_assemble (c_f = |S_f|^2/(rho
 * S_f.d) with the same rho).  ustar[3 n_cells]; p[n_cells] out (0 on
 * removed cells and pins).  One sample only (ppe_set_segments with one
 * sample).  Returns PPE_NOT_CONVERGED after 50 deferred-correction
 * passes, PPE_ERR_STATE before ppe_assemble or ppe_set_geometry or with
 * several samples, PPE_ERR_ARG. */
ppe_status ppe_project(ppe_solver* s, const double* face_coeff, const double* ustar, double rho,
                       double dt, double* p, double* flux, double* u, ppe_project_stats* stats);

/* ppe_project from an initial guess: p[n_cells] in is the starting pressure
 * (e.g. the previous time step's; its values on removed cells and pins are
 * ignored), out the pressure.  Same arguments, exit test (relative to
 * ||b'||, not to the starting residual) and errors as ppe_project. */
ppe_status ppe_project_warm(ppe_solver* s, const double* face_coeff, const double* ustar,
                            double rho, double dt, double* p, double* flux, double* u,
                            ppe_project_stats* stats);

/* grad[3 n_faces] = masked face gradient of p[n_cells] (0 on blocked and
 * wall faces) and cross[n_faces] = t_f . grad_f, as ppe_project uses them.
 * Errors: PPE_ERR_STATE before ppe_assemble and ppe_set_geometry. */
ppe_status ppe_face_gradient(ppe_solver* s, const double* face_coeff, double rho, const double* p,
                             double* grad, double* cross);

const char* ppe_status_string(ppe_status st);
/* Detail of the last failure of this solver ("" if none).  NULL = global. */
const char* ppe_last_error(const ppe_solver* s);

/* ---- Inspection: used by the parity tests to compare each setup stage. ----
 * All sizes are host ints; arrays are device pointers sized by the caller
 * from ppe_level_info.  PPE_ERR_STATE before assemble, PPE_ERR_ARG for a bad
 * level or a NULL array. */

/* Level sizes: rows, stored entries of A_l, entries of P_l (0 on the
 * coarsest level), aggregates (= rows of level l+1), and rho_l, the spectral
 * bound of D^-1 A_l used by the smoother and the prolongator smoothing (0 on
 * a coarsest level solved through its explicit inverse, where neither runs). */
ppe_status ppe_level_info(const ppe_solver* s, int level, int32_t* n_rows,
                          int64_t* nnz_a, int64_t* nnz_p, int32_t* n_agg,
                          double* rho);

/* Copy A_l in CSR (sorted columns, diagonal included): row_ptr[n+1],
 * col[nnz], val[nnz]. */
ppe_status ppe_copy_level_matrix(const ppe_solver* s, int level, int32_t* row_ptr,
                                 int32_t* col, double* val);

/* Copy P_l in CSR: row_ptr[n+1], col[nnz_p], val[nnz_p]. */
ppe_status ppe_copy_prolongator(const ppe_solver* s, int level, int32_t* row_ptr,
                                int32_t* col, double* val);

/* Copy the aggregate id of every row of level l (-1: not aggregated).
 * PPE_ERR_STATE for level 0 after an assembly that kept the coarse levels
 * of an earlier build (coarse_reuse): that finest level has no aggregates. */
ppe_status ppe_copy_aggregates(const ppe_solver* s, int level, int32_t* agg);

/* Masking outputs on the finest level: compact id per cell (-1 removed) and
 * the component label (its pin's cell index) per cell (-1 removed). */
ppe_status ppe_copy_mask(const ppe_solver* s, int32_t* compact_id, int32_t* component);

/* y = A_l x on level l (x, y of length n_rows(l)). */
ppe_status ppe_apply_matrix(ppe_solver* s, int level, const double* x, double* y);

/* z = M r: one V-cycle from level 0 with a zero initial guess (length n_active). */
ppe_status ppe_apply_vcycle(ppe_solver* s, const double* r, double* z);

/* Launch choices of level l's solve kernels, choice[5] (host):
 *   [0] lanes per row of the coarse smoother (0 = the fixed rule, else 4, 8,
 *       16, 32 or 64);
 *   [1], [2] lanes per row of the restriction and of the prolongation (0, or
 *       a power of two from 1 to 64; a fused prolongation takes 4 for 1 or 2);
 *   [3] 1 if the first two smoothing steps from a zero guess run as one
 *       fused pass, 0 if split (on a coarse level the restriction into it
 *       then takes the first step);
 *   [4] 1 if the prolongation runs in one pass with the first
 *       post-smoothing step, reading the Galerkin product's A P (possible on
 *       the coarse levels of the FP64 V-cycle), 0 for separate passes.
 * The fixed rules set them at assembly, or the autotuner when enabled;
 * setting them by hand (until the next assembly) lets a test run every
 * variant.  They never affect the hierarchy, only the solve's order of
 * summation.  PPE_ERR_ARG for a value outside those sets. */
ppe_status ppe_get_level_launch(const ppe_solver* s, int level, int32_t* choice);
ppe_status ppe_set_level_launch(ppe_solver* s, int level, const int32_t* choice);

/* ---- Learned warm start (not part of the paper's method). ----
 * A dense network n_in -> width (n_hidden SiLU layers) -> 1 (linear)
 * predicts each active cell's next pressure increment from local features;
 * the solve then starts from x0 = p_prev + dp_scale * y and conjugate
 * gradients still finishes it to rtol, so the network only changes the
 * iteration count.  Parameters are FP32, packed layer by layer as W
 * ([out][in], row-major) followed by b.  Every array is a device pointer;
 * the network runs on the stream given at creation. */
typedef struct ppe_mlp ppe_mlp;

/* Errors: PPE_ERR_ARG for sizes < 1 or > 4096. Parameters start at 0. */
ppe_status ppe_mlp_create(int32_t n_in, int32_t width, int32_t n_hidden, void* stream,
                          ppe_mlp** out);
void ppe_mlp_destroy(ppe_mlp* m);
int64_t ppe_mlp_num_params(const ppe_mlp* m);
const char* ppe_mlp_last_error(const ppe_mlp* m);
/* Copy parameters in (also resets the Adam moments) or out. */
ppe_status ppe_mlp_set_params(ppe_mlp* m, const float* params);
ppe_status ppe_mlp_get_params(const ppe_mlp* m, float* params);
/* y[n] = network(x[n][n_in]).  bf16 = 0: FP32 throughout; bf16 = 1: the
 * width x width layers on BF16 matrix cores with FP32 accumulation (needs
 * n_in = 10, width = 128, n_hidden >= 2). */
ppe_status ppe_mlp_forward(ppe_mlp* m, int32_t n, const float* x, float* y, int bf16);
/* Mean squared error of network(x) against t over n rows (*loss, host) and
 * its gradient with respect to the packed parameters (grad, device). */
ppe_status ppe_mlp_loss_grad(ppe_mlp* m, int32_t n, const float* x, const float* t, float* grad,
                             double* loss);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on that loss; *loss (host,
 * nullable) receives the loss before the step. */
ppe_status ppe_mlp_train_step(ppe_mlp* m, int32_t n, const float* x, const float* t, float lr,
                              double* loss);

/* Previous fields are re-referenced to the current pins: a field q becomes
 * q_c - q_pin(c), pin(c) = the pin of cell c's pocket, which removes the
 * constant jump a pocket's pressure takes when its pin moves.
 * Features of the assembled solver's active cells, row r = compact id:
 * previous increment / its RMS, rhs / its RMS, liquid fraction, volume /
 * mean volume, and the six largest open-face coefficients of the cell
 * divided by their sum (descending); then (f - mu) / sigma per feature.
 * features: [n_active][10] FP32.  *dp_scale (host) = RMS of dp_prev over
 * the active cells.  Arrays of length n_cells / n_faces are FP64. */
ppe_status ppe_warm_start_features(ppe_solver* s, const double* dp_prev, const double* rhs,
                                   const double* face_coeff, const double* liquid_fraction,
                                   const double* cell_volume, const float* mu, const float* sigma,
                                   float* features, double* dp_scale);
/* For callers that cannot allocate device memory (code between HIP graph
 * captures, tight per-timestep loops, harnesses that forbid hipMalloc): the
 * same features and dp_scale as ppe_warm_start_features, bitwise, computed
 * with the statistics' workspace in a static device array (3 * 1024 + 3
 * doubles, 24.6 KB per device, held until the process ends) instead of
 * solver memory.  Calls no hipMalloc, hipFree or allocating library routine
 * once its first call on a device has looked the array up.  Every call on one
 * device shares that array: calls that overlap on one device (two host
 * threads, or two streams in flight) race and must be serialised by the
 * caller.  Errors as ppe_warm_start_features, and PPE_ERR_ARG (with a
 * message) if a workspace larger than the array were needed. */
ppe_status ppe_warm_start_features_noalloc(ppe_solver* s, const double* dp_prev,
                                           const double* rhs, const double* face_coeff,
                                           const double* liquid_fraction,
                                           const double* cell_volume, const float* mu,
                                           const float* sigma, float* features,
                                           double* dp_scale);
/* x0 = p_prev (re-referenced) + dp_scale * y on active non-pin cells, 0
 * elsewhere (y per compact row, x0 per cell). */
ppe_status ppe_warm_start_apply(ppe_solver* s, const double* p_prev, const float* y,
                                double dp_scale, double* x0);
/* Training targets per compact row: (p_new - p_prev re-referenced) / dp_scale. */
ppe_status ppe_warm_start_targets(ppe_solver* s, const double* p_new, const double* p_prev,
                                  double dp_scale, float* targets);

/* ---- Polynomial chaos by stochastic collocation (section 3, Eq. 27-28). ----
 * The wrapper the paper puts around its deterministic simulations: an
 * expansion w(x, xi) ~ sum_i w_i(x) Psi_i(xi) in products of polynomials
 * orthonormal under each input's distribution (probabilists' Hermite for a
 * standard normal input, Legendre for a uniform input on [-1, 1]) over all
 * multi-indices of total degree <= degree, fitted by least squares to
 * outputs at M sample points (the Vandermonde system of Eq. 28), for every
 * output (e.g. every cell of a field) at once.  Sample points: the full
 * tensor product of l-point Gauss rules, or Smolyak's sparse combination of
 * Gauss rules of accuracy level l (exact for total degree 2l - 1).  Standard
 * inputs xi are mapped to physical ones by the caller (e.g. T = mu + sigma
 * xi).  Host arrays are marked; everything else is device memory. */
typedef struct ppe_pce ppe_pce;
enum { PPE_INPUT_NORMAL = 0, PPE_INPUT_UNIFORM = 1 };
enum { PPE_GRID_TENSOR = 0, PPE_GRID_SMOLYAK = 1 };

/* d inputs (1..16) of the given kinds (host array); degree 0..30.  stream:
 * hipStream_t for the device work (NULL = default). */
ppe_status ppe_pce_create(int32_t d, const int32_t* kinds, int32_t degree, void* stream,
                          ppe_pce** out);
void ppe_pce_destroy(ppe_pce* q);
int32_t ppe_pce_num_terms(const ppe_pce* q);
const char* ppe_pce_last_error(const ppe_pce* q);
/* Multi-indices of the basis, graded order (host, [n_terms x d]). */
ppe_status ppe_pce_terms(const ppe_pce* q, int32_t* alpha);
/* Sample points of accuracy level 1..20 (host arrays): with nodes == NULL,
 * *n_nodes receives the count; otherwise *n_nodes is the capacity and
 * nodes[n x d] and weights[n] (probability weights, may be NULL) are
 * filled.  Coincident nodes of the Smolyak combination are merged. */
ppe_status ppe_pce_nodes(ppe_pce* q, int32_t grid, int32_t level, int32_t* n_nodes, double* nodes,
                         double* weights);
/* W[n_terms x n_out] = least-squares solution of V W = Y, with V the
 * Vandermonde matrix of the M >= n_terms points xi (host, [M x d]) and
 * Y[M x n_out] the outputs (row m = the simulation at point m).
 * PPE_ERR_ARG if V is rank deficient. */
ppe_status ppe_pce_fit(ppe_pce* q, int32_t M, const double* xi, int64_t n_out, const double* Y,
                       double* W);
/* Y[T x n_out] = the expansion W evaluated at T points xi (host, [T x d]). */
ppe_status ppe_pce_eval(ppe_pce* q, int32_t T, const double* xi, int64_t n_out, const double* W,
                        double* Y);
/* Per output: mean = W_0, variance = sum_{i>0} W_i^2, and per input j the
 * first-order Sobol index (terms in input j alone) and the total index
 * (terms involving j) as shares of the variance: first, total [d x n_out]. */
ppe_status ppe_pce_stats(ppe_pce* q, int64_t n_out, const double* W, double* mean, double* var,
                         double* first, double* total);

/* ---- Per-kernel measurement of the solve. ----
 * While enabled, every dispatch of the V-cycle and PCG kernels (level
 * operators, smoothing steps, restriction, prolongation, coarsest solve,
 * outer SpMV, vector updates and dots) is launched with its own pair of HIP
 * events on the solver's stream (the events take the dispatch's start and
 * end), and the library adds up, per kernel instantiation, the launches,
 * the kernel time and the algorithmic bytes each launch moves: every stored
 * matrix entry read once (value + 4-byte column index; 4-byte row pointers
 * for CSR), each diagonal read once, and 8 bytes per row for every vector
 * the kernel reads or writes.  Graph replay is off meanwhile.  Enabling
 * resets the table.  PPE_ERR_ARG on NULL. */
ppe_status ppe_profile_enable(ppe_solver* s, int enable);
/* *n_kernels = the number of kernel instantiations recorded so far. */
ppe_status ppe_profile_count(const ppe_solver* s, int32_t* n_kernels);
/* Entry k (0 <= k < count): name (NUL-terminated, truncated to name_cap
 * bytes; the instantiation as a kernel trace prints it, such as
 * "k_csr<2, 16, double>"), launches, summed kernel milliseconds and summed
 * algorithmic bytes.  PPE_ERR_ARG for k out of range or NULL pointers. */
ppe_status ppe_profile_entry(const ppe_solver* s, int32_t k, char* name, int32_t name_cap,
                             int64_t* launches, double* kernel_ms, double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* PPE_H */

/* One time step of the fractional-step solidification solver (arXiv:1810.08572,
 * section 2.2, steps 1-4) on the GPU: the momentum predictor (Eq. 6), the
 * masked pressure correction (Eq. 7-9 with section 2.4), and the energy
 * equation with its latent-heat Picard loop (Eq. 4, 18-21).
 *
 * Every linear system is solved by the AMG-PCG of ppe.h: the momentum and
 * energy matrices (diagonal + Crank-Nicolson half of the direct diffusion
 * term) through ppe_assemble_shifted (the energy step's later Picard passes
 * through ppe_refresh_shift), the pressure through ppe_assemble and
 * ppe_project.  All arrays are DEVICE pointers owned by the caller unless
 * stated otherwise; calls run on the stream of the options given at
 * creation and return after the stream has finished the step.
 *
 * Discretisation (cell i, volume V_i; interior face f with owner C1 and
 * neighbour C2, area vector S_f from C1 to C2, d_f = x_C2 - x_C1; s_if = +1
 * for the owner, -1 for the neighbour):
 *   c'_f = |S_f|^2 / (S_f.d_f), t'_f = S_f - c'_f d_f (Eq. 11),
 *   x_f(phi) = t'_f . grad(phi)_f with the Eq. 12 gradient over every cell
 *     sharing a vertex with f (vertex values = means over their cells),
 *   wall face: w_f = |S_f|^2 / (S_f.(x_f - x_C1)), the wall value held at
 *     the face centre;
 *   D^dir_i(phi) = Gamma [sum_f s_if c'_f (phi_C2 - phi_C1)
 *                         + sum_wall w_f (phi_wall - phi_i)],
 *   D^x_i(phi) = Gamma sum_f s_if x_f(phi),
 *   C_i(phi) = rho_eff sum_f s_if F_f (phi_C1 + phi_C2) / 2 (F: corrected
 *     volume fluxes), Adams-Bashforth 3/2 C^n - 1/2 C^(n-1).
 * Momentum on cells with f_s < 1 (u = 0 on the others, which act as walls):
 *   (rho V/dt + V mu/K) u* - 1/2 D^dir(u*) = rho V/dt u^n - AB(C(u))
 *       + 1/2 D^dir(u^n) + D^x(u^n) - V g rho beta (T^n - T_ref),
 *   mu/K = 180 mu f_s^2 / (lam^2 (1 - f_s)^3) (Eq. 3), capped at
 *   1e12 rho/dt; no-slip walls.
 * Pressure: ppe_project with f_l = 1 - f_s^n and c_f = c'_f / rho.
 * Energy on every cell, Picard iteration from T^0 = T^n, f_s^0 = f_s^n:
 *   (rho c_p V/dt - S_p) T^(m+1) - 1/2 D^dir(T^(m+1)) = rho c_p V/dt T^n
 *       - AB(C^T) + 1/2 D^dir(T^n) + D^x(T^n) + S_c,
 *   S_p = rho L_f V/dt f_s'(T^m), S_c = rho L_f V/dt (f_s^m - f_s^n - f_s'(T^m) T^m),
 *   C^T with the new fluxes and T^n; f_s^(m+1) = (1 - lambda) f_s^m +
 *   lambda f_s(T^(m+1)) with f_s of Eq. 21; stop when
 *   max|T^(m+1) - T^m| <= tol max|T^(m+1)| and max|f_s^(m+1) - f_s^m| <= tol.
 * Afterwards cells with f_s = 1 get u = 0 and faces touching them F = 0.
 */
#ifndef PPE_FLOW_H
#define PPE_FLOW_H

#include "ppe.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ppe_flow ppe_flow;

/* Material properties (SI units).  T_f, T_liq, T_sol, T_eps and k_p are
 * those of Eq. 5 and Eq. 21, lam the dendrite arm spacing of Eq. 3, g the
 * gravity vector, T_ref the Boussinesq reference temperature (Eq. 2). */
typedef struct {
  double rho, cp, k, mu, beta, lam, Lf;
  double T_f, T_liq, T_sol, T_eps, k_p, T_ref;
  double g[3];
  int fixed_wall_T;   /* 1: walls held at T_wall; 0: thermally insulated */
  double T_wall;
} ppe_alloy;

typedef struct {
  double dt;          /* time step, > 0 */
  double picard_tol;  /* > 0: relative change of T and absolute change of f_s */
  int max_picard;     /* >= 1 */
  double relax;       /* lambda of the f_s update, in (0, 1] */
  int have_history;   /* 0 on the first step: conv_u and conv_T are not read
                         and convection is taken explicitly (Euler) */
} ppe_step_params;

typedef struct {
  int picard;               /* Picard passes of the energy step */
  int momentum_iterations;  /* PCG iterations summed over the three components */
  int pressure_outer;       /* the projection's outer count (ppe_project_stats.outer) */
  int pressure_iterations;  /* its inner count (ppe_project_stats.pcg_iterations) */
  int energy_iterations;    /* PCG iterations summed over the Picard passes */
  int n_fluid;              /* cells with f_s < 1 at the start of the step */
  int n_solid;              /* cells with f_s = 1 at the end of the step */
  double momentum_ms, pressure_ms, energy_ms, ms;  /* wall time of the parts and of the step */
} ppe_flow_stats;

/* Create a driver.  opt configures the pressure solver (stream, precision,
 * rtol and the rest, as ppe_create); the momentum and energy solvers use
 * the same options with FP64 arithmetic and relative residual
 * transport_rtol (> 0, e.g. 1e-12).  With opt->reuse_unchanged the pressure
 * system and its hierarchy are kept while the mask is unchanged (they depend
 * on nothing else), and the momentum system then only refreshes its
 * diagonal (ppe_refresh_shift); the energy system, which keeps every cell,
 * refreshes its diagonal whenever k is unchanged.  PPE_ERR_ARG on NULL out or
 * bad values; the errors of ppe_create. */
ppe_status ppe_flow_create(const ppe_options* opt, double transport_rtol, ppe_flow** out);

/* Destroy a driver and its three solvers.  NULL is accepted. */
void ppe_flow_destroy(ppe_flow* f);

/* Mesh: topology as ppe_set_mesh, vertices as ppe_set_geometry (nodes[3
 * n_nodes], face_nodes[4 n_faces] in the order V1..V4 of Eq. 12,
 * cell_nodes[8 n_cells], cell_centre[3 n_cells], face_area[3 n_faces]),
 * and face_centre[3 n_faces], cell_volume[n_cells] (> 0).  Copies what it
 * needs.  Errors: those of ppe_set_mesh and ppe_set_geometry, PPE_ERR_ARG
 * on a NULL array, a non-positive volume, or a wall face whose centre is
 * not on the outer side of its cell's centre. */
ppe_status ppe_flow_set_mesh(ppe_flow* f, int32_t n_cells, int32_t n_faces, const int32_t* owner,
                             const int32_t* neigh, int32_t n_nodes, const double* nodes,
                             const int32_t* face_nodes, const int32_t* cell_nodes,
                             const double* cell_centre, const double* face_area,
                             const double* face_centre, const double* cell_volume);

/* Advance the state by one step.  In/out (device):
 *   u[3 n_cells]      cell velocities (x, y, z per cell); 0 on cells with
 *                     f_s = 1 on entry and on exit,
 *   T[n_cells]        temperature,
 *   fs[n_cells]       solid fraction in [0, 1],
 *   flux[n_faces]     corrected volume fluxes F (0 on walls and on faces
 *                     touching a cell with f_s = 1),
 *   conv_u[3 n_cells], conv_T[n_cells]  convection terms of the previous
 *                     step (read when have_history), replaced by this
 *                     step's C(u^n) and C^T;
 *   p[n_cells]        in: the previous step's pressure, the projection's
 *                     starting guess when have_history; out: the pressure
 *                     (0 on removed cells and pins).
 * stats (host, nullable).  Returns PPE_OK; PPE_NOT_CONVERGED when the
 * Picard loop or an inner solve did not converge (the state then holds the
 * last iterates); PPE_ERR_STATE before ppe_flow_set_mesh; PPE_ERR_ARG on
 * NULL arrays or bad values (a non-positive property, mu and k included,
 * or dt; relax outside (0, 1]; T_f = T_liq; k_p = 1); the errors of the
 * inner solvers. */
ppe_status ppe_flow_step(ppe_flow* f, const ppe_alloy* alloy, const ppe_step_params* prm,
                         double* u, double* T, double* fs, double* flux, double* p,
                         double* conv_u, double* conv_T, ppe_flow_stats* stats);

/* fs[n] = f_s(T[n]) of Eq. 21 (device arrays): the solid fraction that goes
 * with a given temperature, for an initial state.  PPE_ERR_ARG on NULL
 * arrays with n > 0, n < 0, T_eps <= 0, T_f = T_liq or k_p = 1. */
ppe_status ppe_flow_solid_fraction(ppe_flow* f, const ppe_alloy* alloy, int64_t n, const double* T,
                                   double* fs);

/* Detail of the last failure ("" if none). */
const char* ppe_flow_last_error(const ppe_flow* f);

#ifdef __cplusplus
}
#endif

#endif /* PPE_FLOW_H */

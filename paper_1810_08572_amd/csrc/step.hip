// One fractional step (section 2.2, steps 1-4): momentum predictor (Eq. 6),
// masked projection (Eq. 7-9, section 2.4), energy with the latent-heat
// Picard loop (Eq. 4, 18-21).  The linear systems go through the library's
// AMG-PCG (shifted assembly for momentum and energy, the pressure system
// and its deferred-correction projection); the kernels here form their
// coefficients and right-hand sides.
//
// Layout: cell fields SoA of n_cells doubles except the velocity (AoS,
// x y z per cell, as ppe_project takes it); face fields n_faces doubles; the
// four transported fields (u_x, u_y, u_z, T) share one vertex-mean and one
// cross-flux pass (four arrays each).
#include "common.h"
#include "../../include/ppe_flow.h"

#include <chrono>
#include <cmath>
#include <vector>

struct ppe_flow {
  // declared first, so it outlives every buffer of the driver
  ppe::Allocator allocator;
  ppe_options opt{};
  hipStream_t stream = nullptr;
  ppe_solver* mom = nullptr;  // shifted systems of the momentum predictor
  ppe_solver* pre = nullptr;  // pressure system and geometry (projection)
  ppe_solver* ene = nullptr;  // shifted systems of the energy step
  int nc = 0, nf = 0, nn = 0;
  bool have_mesh = false;
  // the momentum and energy systems' coefficient arrays depend on mu, k and
  // rho only: while they and the mask stay, a new diagonal is a refresh
  bool mom_built = false, ene_built = false;
  double mom_mu = 0.0, ene_k = 0.0, pre_rho = 0.0;
  std::string err;
  // geometry
  ppe::DevBuf vol, cgeo, wgeo, ax, wall_ptr, wall_face, wsum;
  // per-step work
  ppe::DevBuf u_n, T_n, fs_n, fl, shift, rhs, us, ustar, u_new, F_new, coef_m, coef_p, coef_e;
  ppe::DevBuf vbar, xf, conv_u, conv_T, base, Tm, fm, Tnew, part, flag;
};

namespace ppe {
namespace {

constexpr double kDarcyCap = 1e12;  // times rho/dt

struct Alloy {
  double rho, cp, k, mu, beta, lam, Lf, T_f, T_liq, T_sol, T_eps, k_p, T_ref, g0, g1, g2;
  int fixed;
  double T_wall, fhat, e;  // fhat = f_s(T_sol + T_eps) on the Scheil branch, e = 1/(k_p - 1)
};

// Eq. 21 and its slope (same branch rules as the definition: T > T_liq
// liquid, T < T_sol - T_eps solid, |T - T_sol| <= T_eps the linear band).
__device__ __forceinline__ void solid_fraction(const Alloy& a, double T, double& fs, double& dfs) {
  if (T > a.T_liq) {
    fs = 0.0;
    dfs = 0.0;
  } else if (T < a.T_sol - a.T_eps) {
    fs = 1.0;
    dfs = 0.0;
  } else if (fabs(T - a.T_sol) <= a.T_eps) {
    const double s = (1.0 - a.fhat) / (2.0 * a.T_eps);
    fs = a.fhat - (T - a.T_sol - a.T_eps) * s;
    dfs = -s;
  } else {
    const double x = (T - a.T_f) / (a.T_liq - a.T_f);
    fs = 1.0 - pow(x, a.e);
    dfs = -a.e * pow(x, a.e - 1.0) / (a.T_liq - a.T_f);
  }
}

// The next Picard iterate from the previous one (tp) and the pass's solved
// temperature (ts): ts, except that a cell does not jump over a kink of
// Eq. 21 in one pass.  Cooling stops at the highest kink strictly between,
// heating at the lowest; a cell on a kink moves freely, and the kink belongs
// to the branch below it, so the next pass linearises with the slope of the
// branch the cell entered.  At convergence no cell crosses a kink, so the
// fixed point is that of the plain iteration.
__device__ __forceinline__ double branch_limited(const Alloy& a, double tp, double ts) {
  const double k1 = a.T_liq, k2 = a.T_sol + a.T_eps, k3 = a.T_sol - a.T_eps;
  if (ts < tp) {
    if (ts < k1 && k1 < tp) return k1;
    if (ts < k2 && k2 < tp) return k2;
    if (ts < k3 && k3 < tp) return k3;
  } else if (ts > tp) {
    if (tp < k3 && k3 < ts) return k3;
    if (tp < k2 && k2 < ts) return k2;
    if (tp < k1 && k1 < ts) return k1;
  }
  return ts;
}

__device__ __forceinline__ double darcy(const Alloy& a, double fs, double cap) {
  if (!(fs > 0.0 && fs < 1.0)) return 0.0;
  const double q = 1.0 - fs;
  const double d = 180.0 * a.mu * (fs * fs) / (a.lam * a.lam * (q * q * q));
  return d < cap ? d : cap;
}

// c'_f, w_f and the cross weights a_k = t'_f . g_k (g_k the columns of J^-1).
__global__ void k_flow_geom(int nf, const int* __restrict__ owner, const int* __restrict__ neigh,
                            const double* __restrict__ S, const double* __restrict__ C,
                            const double* __restrict__ Xf, const double* __restrict__ gi,
                            double* __restrict__ cgeo, double* __restrict__ wgeo,
                            double* __restrict__ ax, int* __restrict__ flag) {
  const int f = blockIdx.x * kBlock + threadIdx.x;
  if (f >= nf) return;
  const int o = owner[f], n = neigh[f];
  const double s0 = S[3 * (size_t)f], s1 = S[3 * (size_t)f + 1], s2 = S[3 * (size_t)f + 2];
  const double ss = s0 * s0 + s1 * s1 + s2 * s2;
  double c = 0.0, w = 0.0, a[3] = {0.0, 0.0, 0.0};
  if (n >= 0) {
    double d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = C[3 * (size_t)n + k] - C[3 * (size_t)o + k];
    c = ss / (s0 * d[0] + s1 * d[1] + s2 * d[2]);
    const double t[3] = {s0 - c * d[0], s1 - c * d[1], s2 - c * d[2]};
#pragma unroll
    for (int k = 0; k < 3; ++k)
      a[k] = t[0] * gi[(size_t)(3 * k) * nf + f] + t[1] * gi[(size_t)(3 * k + 1) * nf + f] +
             t[2] * gi[(size_t)(3 * k + 2) * nf + f];
  } else {
    double d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = Xf[3 * (size_t)f + k] - C[3 * (size_t)o + k];
    const double sd = s0 * d[0] + s1 * d[1] + s2 * d[2];
    if (!(sd > 0.0)) atomicOr(flag, 1);
    w = sd > 0.0 ? ss / sd : 0.0;
  }
  cgeo[f] = c;
  wgeo[f] = w;
#pragma unroll
  for (int k = 0; k < 3; ++k) ax[(size_t)k * nf + f] = a[k];
}

__global__ void k_wall_sum(int nc, const int* __restrict__ ptr, const int* __restrict__ face,
                           const double* __restrict__ wgeo, const double* __restrict__ vol,
                           double* __restrict__ W, int* __restrict__ flag) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= nc) return;
  double s = 0.0;
  for (int k = ptr[c]; k < ptr[c + 1]; ++k) s += wgeo[face[k]];
  W[c] = s;
  if (!(vol[c] > 0.0)) atomicOr(flag, 2);
}

// Vertex means of the four transported fields over all cells at the vertex.
__global__ void k_vmean4(int nn, const int* __restrict__ vptr, const int* __restrict__ vcell,
                         const double* __restrict__ u, const double* __restrict__ T,
                         double* __restrict__ vbar) {
  const int v = blockIdx.x * kBlock + threadIdx.x;
  if (v >= nn) return;
  const int a = vptr[v], e = vptr[v + 1];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int k = a; k < e; ++k) {
    const int c = vcell[k];
    s0 += u[3 * (size_t)c];
    s1 += u[3 * (size_t)c + 1];
    s2 += u[3 * (size_t)c + 2];
    s3 += T[c];
  }
  const double inv = e > a ? 1.0 / (double)(e - a) : 0.0;
  vbar[v] = s0 * inv;
  vbar[(size_t)nn + v] = s1 * inv;
  vbar[2 * (size_t)nn + v] = s2 * inv;
  vbar[3 * (size_t)nn + v] = s3 * inv;
}

// Cross fluxes x_f of the four fields, and the three systems' face
// coefficients (half of mu c' and k c' for Crank-Nicolson, c'/rho).
__global__ void k_face4(int nf, int nn, const int* __restrict__ owner, const int* __restrict__ neigh,
                        const int* __restrict__ fnodes, const double* __restrict__ ax,
                        const double* __restrict__ cgeo, const double* __restrict__ vbar,
                        const double* __restrict__ u, const double* __restrict__ T, Alloy a,
                        double* __restrict__ xf, double* __restrict__ cm, double* __restrict__ cp,
                        double* __restrict__ ce) {
  const int f = blockIdx.x * kBlock + threadIdx.x;
  if (f >= nf) return;
  const int o = owner[f], n = neigh[f];
  const double c = cgeo[f];
  cm[f] = 0.5 * a.mu * c;
  cp[f] = c / a.rho;
  ce[f] = 0.5 * a.k * c;
  double x[4] = {0.0, 0.0, 0.0, 0.0};
  if (n >= 0) {
    const double a0 = ax[f], a1 = ax[(size_t)nf + f], a2 = ax[2 * (size_t)nf + f];
    int v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = fnodes[4 * (size_t)f + k];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double* vb = vbar + (size_t)q * nn;
      const double po = q < 3 ? u[3 * (size_t)o + q] : T[o];
      const double pn = q < 3 ? u[3 * (size_t)n + q] : T[n];
      x[q] = a0 * (pn - po) + a1 * (vb[v[2]] - vb[v[0]]) + a2 * (vb[v[3]] - vb[v[1]]);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) xf[(size_t)q * nf + f] = x[q];
}

// Momentum: shift, right-hand sides (SoA), convection C(u^n), warm start.
__global__ void k_momentum(int nc, const int* __restrict__ adj_ptr, const int* __restrict__ adj_nbr,
                           const int* __restrict__ adj_face, const int* __restrict__ owner,
                           const double* __restrict__ cgeo, const double* __restrict__ W,
                           const double* __restrict__ vol, const double* __restrict__ xf, int nf,
                           const double* __restrict__ F, const double* __restrict__ u,
                           const double* __restrict__ T, const double* __restrict__ fs, Alloy a,
                           double dt, const double* __restrict__ conv_prev, int have_history,
                           double* __restrict__ conv_new, double* __restrict__ fl,
                           double* __restrict__ shift, double* __restrict__ rhs,
                           double* __restrict__ us) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= nc) return;
  const double uc[3] = {u[3 * (size_t)c], u[3 * (size_t)c + 1], u[3 * (size_t)c + 2]};
  double conv[3] = {0.0, 0.0, 0.0}, dd[3] = {0.0, 0.0, 0.0}, cx[3] = {0.0, 0.0, 0.0};
  double blk = 0.0;
  const bool fluid = fs[c] < 1.0;
  for (int k = adj_ptr[c]; k < adj_ptr[c + 1]; ++k) {
    const int j = adj_nbr[k], f = adj_face[k];
    const double sg = owner[f] == c ? 1.0 : -1.0;
    const double cf = cgeo[f], Ff = F[f];
    if (!(fs[j] < 1.0)) blk += cf;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const double uj = u[3 * (size_t)j + q];
      conv[q] += sg * Ff * (0.5 * (uc[q] + uj));
      dd[q] += cf * (uj - uc[q]);
      cx[q] += sg * xf[(size_t)q * nf + f];
    }
  }
  const double V = vol[c];
  const double rv = a.rho * V / dt;
  const double buoy = V * a.rho * a.beta * (T[c] - a.T_ref);
  const double g[3] = {a.g0, a.g1, a.g2};
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double cn = a.rho * conv[q];
    conv_new[3 * (size_t)c + q] = cn;
    const double ab = have_history ? 1.5 * cn - 0.5 * conv_prev[3 * (size_t)c + q] : cn;
    const double d_dir = a.mu * (dd[q] - W[c] * uc[q]);
    rhs[(size_t)q * nc + c] =
        fluid ? rv * uc[q] - ab + 0.5 * d_dir + a.mu * cx[q] - g[q] * buoy : 0.0;
    us[(size_t)q * nc + c] = uc[q];
  }
  fl[c] = 1.0 - fs[c];
  shift[c] = rv + darcy(a, fs[c], kDarcyCap * a.rho / dt) * V + 0.5 * a.mu * (W[c] + blk);
}

__global__ void k_interleave3(int nc, const double* __restrict__ soa, double* __restrict__ aos) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= nc) return;
#pragma unroll
  for (int q = 0; q < 3; ++q) aos[3 * (size_t)c + q] = soa[(size_t)q * nc + c];
}

// Energy: the Picard-independent part of the right-hand side and C^T.
__global__ void k_energy_base(int nc, const int* __restrict__ adj_ptr,
                              const int* __restrict__ adj_nbr, const int* __restrict__ adj_face,
                              const int* __restrict__ owner, const double* __restrict__ cgeo,
                              const double* __restrict__ W, const double* __restrict__ vol,
                              const double* __restrict__ xT, const double* __restrict__ F,
                              const double* __restrict__ T, Alloy a, double dt,
                              const double* __restrict__ conv_prev, int have_history,
                              double* __restrict__ conv_new, double* __restrict__ base) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= nc) return;
  const double Tc = T[c];
  double conv = 0.0, dd = 0.0, cx = 0.0;
  for (int k = adj_ptr[c]; k < adj_ptr[c + 1]; ++k) {
    const int j = adj_nbr[k], f = adj_face[k];
    const double sg = owner[f] == c ? 1.0 : -1.0;
    conv += sg * F[f] * (0.5 * (Tc + T[j]));
    dd += cgeo[f] * (T[j] - Tc);
    cx += sg * xT[f];
  }
  const double cn = a.rho * a.cp * conv;
  conv_new[c] = cn;
  const double ab = have_history ? 1.5 * cn - 0.5 * conv_prev[c] : cn;
  double d_dir = dd;
  if (a.fixed) d_dir += W[c] * (a.T_wall - Tc);
  double b = a.rho * a.cp * vol[c] / dt * Tc - ab + 0.5 * (a.k * d_dir) + a.k * cx;
  if (a.fixed) b += 0.5 * a.k * W[c] * a.T_wall;
  base[c] = b;
}

// One Picard pass's system: linearised latent term around T^m.
__global__ void k_energy_sys(int nc, const double* __restrict__ vol, const double* __restrict__ W,
                             const double* __restrict__ base, const double* __restrict__ Tm,
                             const double* __restrict__ fm, const double* __restrict__ fs_n,
                             Alloy a, double dt, double* __restrict__ shift,
                             double* __restrict__ rhs, double* __restrict__ Tnew) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= nc) return;
  double f, slope;
  solid_fraction(a, Tm[c], f, slope);
  const double V = vol[c];
  const double rlv = a.rho * a.Lf * V / dt;
  const double Sp = rlv * slope;
  double sh = a.rho * a.cp * V / dt - Sp;
  if (a.fixed) sh += 0.5 * a.k * W[c];
  shift[c] = sh;
  rhs[c] = base[c] + rlv * (fm[c] - fs_n[c] - slope * Tm[c]);
  Tnew[c] = Tm[c];
}

// T^(m+1) = the branch-limited solved temperature; f^(m+1) = (1 - lambda)
// f^m + lambda f_s(T^(m+1)); block maxima of |T_solved - T^m|, |df|, |T^(m+1)|.
__global__ void k_picard(int nc, const double* __restrict__ Tnew, double* __restrict__ Tm,
                         double* __restrict__ fm, Alloy a, double relax,
                         double* __restrict__ part) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  double m0 = 0.0, m1 = 0.0, m2 = 0.0;
  if (c < nc) {
    const double ts = Tnew[c], tp = Tm[c];
    const double t = branch_limited(a, tp, ts);
    double f, slope;
    solid_fraction(a, t, f, slope);
    const double fn = (1.0 - relax) * fm[c] + relax * f;
    m0 = fabs(ts - tp);
    m1 = fabs(fn - fm[c]);
    m2 = fabs(t);
    Tm[c] = t;
    fm[c] = fn;
  }
  m0 = block_max<kBlock>(m0);
  m1 = block_max<kBlock>(m1);
  m2 = block_max<kBlock>(m2);
  if (threadIdx.x == 0) {
    part[3 * (size_t)blockIdx.x] = m0;
    part[3 * (size_t)blockIdx.x + 1] = m1;
    part[3 * (size_t)blockIdx.x + 2] = m2;
  }
}

__global__ void k_max3(int g, const double* __restrict__ part, double* __restrict__ out) {
  double m[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < g; b += kBlock)
#pragma unroll
    for (int k = 0; k < 3; ++k) m[k] = fmax(m[k], part[3 * (size_t)b + k]);
#pragma unroll
  for (int k = 0; k < 3; ++k) m[k] = block_max<kBlock>(m[k]);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 3; ++k) out[k] = m[k];
}

// Outputs of the step: solid cells (f_s = 1) lose their velocity; count them
// (one atomic per workgroup).
__global__ void __launch_bounds__(kBlock) k_finish_cells(
    int nc, const double* __restrict__ u_new, const double* __restrict__ Tm,
    const double* __restrict__ fm, double* __restrict__ u, double* __restrict__ T,
    double* __restrict__ fs, int* __restrict__ n_solid) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  int solid = 0;
  if (c < nc) {
    solid = fm[c] < 1.0 ? 0 : 1;
#pragma unroll
    for (int q = 0; q < 3; ++q) u[3 * (size_t)c + q] = solid ? 0.0 : u_new[3 * (size_t)c + q];
    T[c] = Tm[c];
    fs[c] = fm[c];
  }
  solid = block_sum<kBlock>(solid);
  if (threadIdx.x == 0 && solid) atomicAdd(n_solid, solid);
}

__global__ void k_finish_faces(int nf, const int* __restrict__ owner, const int* __restrict__ neigh,
                               const double* __restrict__ fm, const double* __restrict__ F_new,
                               double* __restrict__ flux) {
  const int f = blockIdx.x * kBlock + threadIdx.x;
  if (f >= nf) return;
  const int o = owner[f], n = neigh[f];
  const bool open = n >= 0 && fm[o] < 1.0 && fm[n] < 1.0;
  flux[f] = open ? F_new[f] : 0.0;
}

__global__ void k_solid_fraction(int n, const double* __restrict__ T, Alloy a,
                                 double* __restrict__ fs) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= n) return;
  double f, slope;
  solid_fraction(a, T[c], f, slope);
  fs[c] = f;
}

__global__ void __launch_bounds__(kBlock) k_count_fluid(int nc, const double* __restrict__ fs,
                                                        int* __restrict__ n) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  int fluid = (c < nc && fs[c] < 1.0) ? 1 : 0;
  fluid = block_sum<kBlock>(fluid);
  if (threadIdx.x == 0 && fluid) atomicAdd(n, fluid);
}

// An inner call's status: failures throw with the inner solver's detail;
// PPE_NOT_CONVERGED is remembered for the step's own status.
void check(ppe_solver* s, ppe_status st, const char* what, ppe_status& worst) {
  if (st < 0) throw Error(st, std::string(what) + ": " + s->err);
  if (st == PPE_NOT_CONVERGED) worst = PPE_NOT_CONVERGED;
}

Alloy make_alloy(const ppe_alloy* al) {
  Alloy a{};
  a.rho = al->rho;
  a.cp = al->cp;
  a.k = al->k;
  a.mu = al->mu;
  a.beta = al->beta;
  a.lam = al->lam;
  a.Lf = al->Lf;
  a.T_f = al->T_f;
  a.T_liq = al->T_liq;
  a.T_sol = al->T_sol;
  a.T_eps = al->T_eps;
  a.k_p = al->k_p;
  a.T_ref = al->T_ref;
  a.g0 = al->g[0];
  a.g1 = al->g[1];
  a.g2 = al->g[2];
  a.fixed = al->fixed_wall_T ? 1 : 0;
  a.T_wall = al->T_wall;
  a.e = 1.0 / (a.k_p - 1.0);
  const double x = (a.T_sol + a.T_eps - a.T_f) / (a.T_liq - a.T_f);
  a.fhat = 1.0 - std::pow(x, a.e);
  return a;
}

double elapsed(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace
}  // namespace ppe

using namespace ppe;

namespace {

template <class F>
ppe_status flow_guarded(ppe_flow* f, F&& fn) {
  // the driver's own arrays come from its allocator while the call runs
  ppe::AllocScope scope(f ? &f->allocator : nullptr);
  try {
    if (f) f->err.clear();
    return fn();
  } catch (const ppe::Error& e) {
    if (f) f->err = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    if (f) f->err = "host allocation failed";
    return PPE_ERR_OOM;
  } catch (const std::exception& e) {
    if (f) f->err = e.what();
    return PPE_ERR_INTERNAL;
  }
}

}  // namespace

extern "C" {

ppe_status ppe_flow_create(const ppe_options* opt, double transport_rtol, ppe_flow** out) {
  if (!opt || !out) return PPE_ERR_ARG;
  *out = nullptr;
  if (!(transport_rtol > 0.0 && transport_rtol < 1.0)) return PPE_ERR_ARG;
  ppe_flow* f = new (std::nothrow) ppe_flow();
  if (!f) return PPE_ERR_OOM;
  f->opt = *opt;
  ppe_options t = *opt;
  t.precision = PPE_FP64;
  t.rtol = transport_rtol;
  t.reuse_unchanged = 0;
  ppe_status st = ppe_create(opt, &f->pre);
  if (st == PPE_OK) st = ppe_create(&t, &f->mom);
  if (st == PPE_OK) st = ppe_create(&t, &f->ene);
  if (st != PPE_OK) {
    ppe_flow_destroy(f);
    return st;
  }
  f->stream = f->pre->stream;
  f->allocator = ppe::Allocator{opt->alloc, opt->free, opt->alloc_ctx, opt->stream, {&f->stream}};
  *out = f;
  return PPE_OK;
}

void ppe_flow_destroy(ppe_flow* f) {
  if (!f) return;
  ppe_destroy(f->mom);
  ppe_destroy(f->pre);
  ppe_destroy(f->ene);
  delete f;
}

const char* ppe_flow_last_error(const ppe_flow* f) { return f ? f->err.c_str() : ""; }

ppe_status ppe_flow_solid_fraction(ppe_flow* f, const ppe_alloy* al, int64_t n, const double* T,
                                   double* fs) {
  if (!f) return PPE_ERR_ARG;
  return flow_guarded(f, [&]() -> ppe_status {
    require(al && n >= 0 && (n == 0 || (T && fs)), PPE_ERR_ARG, "NULL argument or n < 0");
    require(al->T_eps > 0.0 && al->T_f != al->T_liq && al->k_p > 0.0 && al->k_p != 1.0,
            PPE_ERR_ARG, "T_eps <= 0, T_f = T_liq or k_p not in (0, 1) u (1, inf)");
    require(n <= INT32_MAX, PPE_ERR_ARG, "n too large");
    if (n == 0) return PPE_OK;
    const Alloy a = make_alloy(al);
    hipLaunchKernelGGL(k_solid_fraction, dim3(grid_for(n)), dim3(kBlock), 0, f->stream, (int)n, T,
                       a, fs);
    PPE_LAUNCH_CHECK();
    PPE_HIP(hipStreamSynchronize(f->stream));
    return PPE_OK;
  });
}

ppe_status ppe_flow_set_mesh(ppe_flow* f, int32_t n_cells, int32_t n_faces, const int32_t* owner,
                             const int32_t* neigh, int32_t n_nodes, const double* nodes,
                             const int32_t* face_nodes, const int32_t* cell_nodes,
                             const double* cell_centre, const double* face_area,
                             const double* face_centre, const double* cell_volume) {
  if (!f) return PPE_ERR_ARG;
  return flow_guarded(f, [&]() -> ppe_status {
    f->have_mesh = false;
    f->mom_built = f->ene_built = false;
    require(face_centre && cell_volume && (n_faces == 0 || (owner && neigh)), PPE_ERR_ARG,
            "NULL mesh array");
    ppe_status worst = PPE_OK;
    check(f->pre, ppe_set_mesh(f->pre, n_cells, n_faces, owner, neigh), "pressure mesh", worst);
    check(f->mom, ppe_set_mesh(f->mom, n_cells, n_faces, owner, neigh), "momentum mesh", worst);
    check(f->ene, ppe_set_mesh(f->ene, n_cells, n_faces, owner, neigh), "energy mesh", worst);
    check(f->pre,
          ppe_set_geometry(f->pre, n_nodes, nodes, face_nodes, cell_nodes, cell_centre, face_area),
          "geometry", worst);
    ppe_solver* s = f->pre;
    const int nc = n_cells, nf = n_faces;
    f->nc = nc;
    f->nf = nf;
    f->nn = n_nodes;
    double* vol = f->vol.get<double>(nc);
    PPE_HIP(hipMemcpyAsync(vol, cell_volume, sizeof(double) * nc, hipMemcpyDeviceToDevice,
                           f->stream));
    double* Xf = f->F_new.get<double>(3 * (size_t)(nf > 0 ? nf : 1));  // staging
    if (nf)
      PPE_HIP(hipMemcpyAsync(Xf, face_centre, sizeof(double) * 3 * nf, hipMemcpyDeviceToDevice,
                             f->stream));
    int* flag = f->flag.get<int>(4);
    fill_int(s, flag, 0, 1);
    double* cgeo = f->cgeo.get<double>(nf > 0 ? nf : 1);
    double* wgeo = f->wgeo.get<double>(nf > 0 ? nf : 1);
    double* ax = f->ax.get<double>(3 * (size_t)(nf > 0 ? nf : 1));
    if (nf) {
      hipLaunchKernelGGL(k_flow_geom, dim3(grid_for(nf)), dim3(kBlock), 0, f->stream, nf,
                         s->owner.as<int>(), s->neigh.as<int>(), s->g_S.as<double>(),
                         s->g_cc.as<double>(), Xf, s->g_inv.as<double>(), cgeo, wgeo, ax, flag);
      PPE_LAUNCH_CHECK();
    }
    // wall faces of every cell (ascending face id), built once on the host
    std::vector<int> ho(nf), hn(nf);
    if (nf) {
      PPE_HIP(hipMemcpyAsync(ho.data(), s->owner.as<int>(), sizeof(int) * nf, hipMemcpyDeviceToHost,
                             f->stream));
      PPE_HIP(hipMemcpyAsync(hn.data(), s->neigh.as<int>(), sizeof(int) * nf, hipMemcpyDeviceToHost,
                             f->stream));
    }
    PPE_HIP(hipStreamSynchronize(f->stream));
    std::vector<int> ptr(nc + 1, 0), wf;
    for (int q = 0; q < nf; ++q)
      if (hn[q] < 0) ++ptr[ho[q] + 1];
    for (int c = 0; c < nc; ++c) ptr[c + 1] += ptr[c];
    wf.assign(ptr[nc] > 0 ? ptr[nc] : 1, 0);
    std::vector<int> cur(ptr.begin(), ptr.end() - 1);
    for (int q = 0; q < nf; ++q)
      if (hn[q] < 0) wf[cur[ho[q]]++] = q;
    int* dptr = f->wall_ptr.get<int>(nc + 1);
    int* dwf = f->wall_face.get<int>(wf.size());
    PPE_HIP(hipMemcpyAsync(dptr, ptr.data(), sizeof(int) * (nc + 1), hipMemcpyHostToDevice,
                           f->stream));
    PPE_HIP(hipMemcpyAsync(dwf, wf.data(), sizeof(int) * wf.size(), hipMemcpyHostToDevice,
                           f->stream));
    double* W = f->wsum.get<double>(nc);
    hipLaunchKernelGGL(k_wall_sum, dim3(grid_for(nc)), dim3(kBlock), 0, f->stream, nc, dptr, dwf,
                       wgeo, vol, W, flag);
    PPE_LAUNCH_CHECK();
    const int bad = read_scalar(s, flag);
    require(!(bad & 1), PPE_ERR_ARG, "a wall face's centre is not on the outer side of its cell");
    require(!(bad & 2), PPE_ERR_ARG, "cell volumes must be > 0");
    f->have_mesh = true;
    return PPE_OK;
  });
}

ppe_status ppe_flow_step(ppe_flow* f, const ppe_alloy* al, const ppe_step_params* prm, double* u,
                         double* T, double* fs, double* flux, double* p, double* conv_u,
                         double* conv_T, ppe_flow_stats* stats) {
  if (!f) return PPE_ERR_ARG;
  return flow_guarded(f, [&]() -> ppe_status {
    require(f->have_mesh, PPE_ERR_STATE, "ppe_flow_step before ppe_flow_set_mesh");
    require(al && prm && u && T && fs && p && conv_u && conv_T && (flux || f->nf == 0),
            PPE_ERR_ARG, "NULL argument");
    // mu > 0 and k > 0: the implicit diffusion couples neighbours
    const double pos[] = {al->rho, al->cp, al->k, al->mu, al->lam, al->Lf, al->T_eps, prm->dt,
                          prm->picard_tol};
    for (double v : pos)
      require(v > 0.0 && std::isfinite(v), PPE_ERR_ARG, "a property, dt or tol is not > 0");
    require(std::isfinite(al->beta) && std::isfinite(al->T_ref) && std::isfinite(al->g[0]) &&
                std::isfinite(al->g[1]) && std::isfinite(al->g[2]),
            PPE_ERR_ARG, "beta, T_ref or g not finite");
    require(prm->relax > 0.0 && prm->relax <= 1.0, PPE_ERR_ARG, "relax outside (0, 1]");
    require(prm->max_picard >= 1, PPE_ERR_ARG, "max_picard < 1");
    require(al->T_f != al->T_liq && al->k_p != 1.0 && al->k_p > 0.0, PPE_ERR_ARG,
            "T_f = T_liq or k_p not in (0, 1) u (1, inf)");
    const auto t_start = std::chrono::steady_clock::now();
    const Alloy a = make_alloy(al);
    const double dt = prm->dt;
    const int hist = prm->have_history ? 1 : 0;
    const int nc = f->nc, nf = f->nf, nn = f->nn;
    ppe_solver* s = f->pre;
    const int* owner = s->owner.as<int>();
    const int* neigh = s->neigh.as<int>();
    const int* adj_ptr = s->adj_ptr.as<int>();
    const int* adj_nbr = s->adj_nbr.as<int>();
    const int* adj_face = s->adj_face.as<int>();
    const int gc = grid_for(nc), gf = grid_for(nf > 0 ? nf : 1);
    ppe_flow_stats st{};
    ppe_status worst = PPE_OK;

    // the old level, kept while the outputs are overwritten
    double* u_n = f->u_n.get<double>(3 * (size_t)nc);
    double* T_n = f->T_n.get<double>(nc);
    double* fs_n = f->fs_n.get<double>(nc);
    PPE_HIP(hipMemcpyAsync(u_n, u, sizeof(double) * 3 * nc, hipMemcpyDeviceToDevice, f->stream));
    PPE_HIP(hipMemcpyAsync(T_n, T, sizeof(double) * nc, hipMemcpyDeviceToDevice, f->stream));
    PPE_HIP(hipMemcpyAsync(fs_n, fs, sizeof(double) * nc, hipMemcpyDeviceToDevice, f->stream));
    int* counts = f->flag.get<int>(4);
    fill_int(s, counts, 0, 2);
    hipLaunchKernelGGL(k_count_fluid, dim3(gc), dim3(kBlock), 0, f->stream, nc, fs_n, counts);
    PPE_LAUNCH_CHECK();

    // cross fluxes of the four fields at the old level, face coefficients
    double* vbar = f->vbar.get<double>(4 * (size_t)(nn > 0 ? nn : 1));
    double* xf = f->xf.get<double>(4 * (size_t)(nf > 0 ? nf : 1));
    double* cm = f->coef_m.get<double>(nf > 0 ? nf : 1);
    double* cpr = f->coef_p.get<double>(nf > 0 ? nf : 1);
    double* ce = f->coef_e.get<double>(nf > 0 ? nf : 1);
    hipLaunchKernelGGL(k_vmean4, dim3(grid_for(nn)), dim3(kBlock), 0, f->stream, nn,
                       s->g_vptr.as<int>(), s->g_vcell.as<int>(), u_n, T_n, vbar);
    PPE_LAUNCH_CHECK();
    if (nf) {
      hipLaunchKernelGGL(k_face4, dim3(gf), dim3(kBlock), 0, f->stream, nf, nn, owner, neigh,
                         s->g_fnodes.as<int>(), f->ax.as<double>(), f->cgeo.as<double>(), vbar,
                         u_n, T_n, a, xf, cm, cpr, ce);
      PPE_LAUNCH_CHECK();
    }

    // step 1: momentum predictor
    const auto t_mom = std::chrono::steady_clock::now();
    double* fl = f->fl.get<double>(nc);
    double* shift = f->shift.get<double>(nc);
    double* rhs = f->rhs.get<double>(3 * (size_t)nc);
    double* us = f->us.get<double>(3 * (size_t)nc);
    double* cu_new = f->conv_u.get<double>(3 * (size_t)nc);
    hipLaunchKernelGGL(k_momentum, dim3(gc), dim3(kBlock), 0, f->stream, nc, adj_ptr, adj_nbr,
                       adj_face, owner, f->cgeo.as<double>(), f->wsum.as<double>(),
                       f->vol.as<double>(), xf, nf, flux, u_n, T_n, fs_n, a, dt, conv_u, hist,
                       cu_new, fl, shift, rhs, us);
    PPE_LAUNCH_CHECK();
    // the pressure system first: its comparison with the last assembly (when
    // the pressure solver keeps unchanged systems) tells whether the mask
    // moved, and the momentum system then only needs its new diagonal
    const auto t_pre0 = std::chrono::steady_clock::now();
    const int reused_before = s->stats.reused_setup;
    check(s, ppe_assemble(s, cpr, fl), "pressure assembly", worst);
    const bool mask_same = s->stats.reused_setup > reused_before && f->pre_rho == a.rho;
    f->pre_rho = a.rho;
    const double pre_setup_ms = elapsed(t_pre0);
    const bool mom_refresh = mask_same && f->mom_built && f->mom_mu == a.mu;
    f->mom_built = false;  // until the call below succeeds
    if (mom_refresh)
      check(f->mom, ppe_refresh_shift(f->mom, cm, shift), "momentum refresh", worst);
    else
      check(f->mom, ppe_assemble_shifted(f->mom, cm, fl, shift), "momentum assembly", worst);
    f->mom_built = true;
    f->mom_mu = a.mu;
    for (int q = 0; q < 3; ++q) {
      ppe_stats ps{};
      check(f->mom, ppe_solve(f->mom, rhs + (size_t)q * nc, us + (size_t)q * nc, 1, &ps),
            "momentum solve", worst);
      st.momentum_iterations += ps.iterations;
    }
    double* ustar = f->ustar.get<double>(3 * (size_t)nc);
    hipLaunchKernelGGL(k_interleave3, dim3(gc), dim3(kBlock), 0, f->stream, nc, us, ustar);
    PPE_LAUNCH_CHECK();
    st.momentum_ms = elapsed(t_mom) - pre_setup_ms;

    // steps 2-3: pressure, fluxes, velocity correction
    const auto t_pre = std::chrono::steady_clock::now();
    double* u_new = f->u_new.get<double>(3 * (size_t)nc);
    double* F_new = f->F_new.get<double>(nf > 0 ? nf : 1);
    ppe_project_stats pst{};
    // the previous step's pressure starts the projection (the exit test is
    // relative to ||b'||, so the bar is the same)
    if (hist)
      check(s, ppe_project_warm(s, cpr, ustar, a.rho, dt, p, F_new, u_new, &pst), "projection",
            worst);
    else
      check(s, ppe_project(s, cpr, ustar, a.rho, dt, p, F_new, u_new, &pst), "projection",
            worst);
    st.pressure_outer = pst.outer;
    st.pressure_iterations = pst.pcg_iterations;
    st.pressure_ms = elapsed(t_pre) + pre_setup_ms;

    // step 4: energy with the Picard loop
    const auto t_ene = std::chrono::steady_clock::now();
    double* base = f->base.get<double>(nc);
    double* cT_new = f->conv_T.get<double>(nc);
    double* Tm = f->Tm.get<double>(nc);
    double* fm = f->fm.get<double>(nc);
    double* Tnew = f->Tnew.get<double>(nc);
    double* erhs = rhs;  // the momentum right-hand sides are no longer needed
    hipLaunchKernelGGL(k_energy_base, dim3(gc), dim3(kBlock), 0, f->stream, nc, adj_ptr, adj_nbr,
                       adj_face, owner, f->cgeo.as<double>(), f->wsum.as<double>(),
                       f->vol.as<double>(), xf + 3 * (size_t)nf, F_new, T_n, a, dt, conv_T, hist,
                       cT_new, base);
    PPE_LAUNCH_CHECK();
    PPE_HIP(hipMemcpyAsync(Tm, T_n, sizeof(double) * nc, hipMemcpyDeviceToDevice, f->stream));
    PPE_HIP(hipMemcpyAsync(fm, fs_n, sizeof(double) * nc, hipMemcpyDeviceToDevice, f->stream));
    const int gp = gc;
    double* part = f->part.get<double>(3 * (size_t)gp + 3);
    double* mx = part + 3 * (size_t)gp;
    bool converged = false;
    for (int it = 1; it <= prm->max_picard; ++it) {
      hipLaunchKernelGGL(k_energy_sys, dim3(gc), dim3(kBlock), 0, f->stream, nc,
                         f->vol.as<double>(), f->wsum.as<double>(), base, Tm, fm, fs_n, a, dt,
                         shift, erhs, Tnew);
      PPE_LAUNCH_CHECK();
      // every cell is kept and the coefficients depend on k only: once the
      // hierarchy is built, every pass (and every later step) only has a new
      // diagonal, the latent term's
      const bool ene_refresh = f->ene_built && f->ene_k == a.k;
      f->ene_built = false;  // until the call below succeeds
      if (ene_refresh)
        check(f->ene, ppe_refresh_shift(f->ene, ce, shift), "energy refresh", worst);
      else
        check(f->ene, ppe_assemble_shifted(f->ene, ce, nullptr, shift), "energy assembly",
              worst);
      f->ene_built = true;
      f->ene_k = a.k;
      ppe_stats es{};
      check(f->ene, ppe_solve(f->ene, erhs, Tnew, 1, &es), "energy solve", worst);
      st.energy_iterations += es.iterations;
      hipLaunchKernelGGL(k_picard, dim3(gp), dim3(kBlock), 0, f->stream, nc, Tnew, Tm, fm, a,
                         prm->relax, part);
      PPE_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_max3, dim3(1), dim3(kBlock), 0, f->stream, gp, part, mx);
      PPE_LAUNCH_CHECK();
      double m[3] = {0.0, 0.0, 0.0};
      read_back(f->ene, {ReadItem{mx, sizeof(double) * 3, m}});
      st.picard = it;
      if (m[0] <= prm->picard_tol * m[2] && m[1] <= prm->picard_tol) {
        converged = true;
        break;
      }
    }
    if (!converged) worst = PPE_NOT_CONVERGED;
    st.energy_ms = elapsed(t_ene);

    // outputs and mask evolution
    hipLaunchKernelGGL(k_finish_cells, dim3(gc), dim3(kBlock), 0, f->stream, nc, u_new, Tm, fm, u,
                       T, fs, counts + 1);
    PPE_LAUNCH_CHECK();
    if (nf) {
      hipLaunchKernelGGL(k_finish_faces, dim3(gf), dim3(kBlock), 0, f->stream, nf, owner, neigh, fm,
                         F_new, flux);
      PPE_LAUNCH_CHECK();
    }
    PPE_HIP(hipMemcpyAsync(conv_u, cu_new, sizeof(double) * 3 * nc, hipMemcpyDeviceToDevice,
                           f->stream));
    PPE_HIP(hipMemcpyAsync(conv_T, cT_new, sizeof(double) * nc, hipMemcpyDeviceToDevice,
                           f->stream));
    int cnt[2] = {0, 0};
    read_back(s, {ReadItem{counts, sizeof(int) * 2, cnt}});
    st.n_fluid = cnt[0];
    st.n_solid = cnt[1];
    st.ms = elapsed(t_start);
    if (stats) *stats = st;
    return worst;
  });
}

}  // extern "C"

// Right-preconditioned flexible GMRES on the whole system K u = f with the
// block-triangular preconditioner of Section 3 (the paper's own Krylov
// method; the interface flexible CG of api.hip is the production path).
//
//   P~ = [K_II  K_IG; 0  S~],
//   P~^{-1} v = [K_II^{-1} (v_I - K_IG S~^{-1} v_G);  S~^{-1} v_G],
//
// i.e. one interface preconditioner apply, one mapped element sweep, one
// batched interior solve and a scatter.  With S~ = S the preconditioned
// operator K P~^{-1} = [I 0; K_GI K_II^{-1} I] has minimal polynomial
// (t - 1)^2, so GMRES converges in two iterations; S~ = I and S~ = Hhat_theta
// (inverse Lanczos) give the iteration counts of Table 1.  S~ may change
// from one application to the next (inexact inner solves), so the
// preconditioned directions Z_j are kept (flexible GMRES).
//
// The Arnoldi vectors are full nodal vectors (clamped entries zero).  Each
// step orthogonalises K z_j against V_0..V_j by classical Gram-Schmidt run
// twice, with the deterministic window dot and combine kernels; the
// (m+1) x m Hessenberg column and its Givens rotations are scalar work done
// on the host after one read of the column.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "internal.h"

namespace edd {
namespace {

// scalar slots of this file (see the slot map in internal.h)
constexpr int G_H1 = 2048;          // [kMaxRestart + 1] first Gram-Schmidt pass
constexpr int G_H2 = 2048 + 512;    // [kMaxRestart + 1] second pass
constexpr int G_NRM = 2048 + 1023;  // ||w||^2
constexpr int G_ONE = 2048 + 1024;  // [kMaxRestart + 1] ones (combine divisors)
constexpr int G_Y = 2048 + 1536;    // [kMaxRestart] -y (solution update)
constexpr int G_R = 2048 + 2040;    // r.r of a fresh residual
constexpr int kMaxRestart = 256;
constexpr int kInnerMaxit = 5000;  // iterations of one inner interface solve (S~ = S)
constexpr int kTB = 256;

// y = x / sqrt(scal[slot])
__global__ __launch_bounds__(kTB) void k_scale_invsqrt(int64_t n, const double *__restrict__ scal,
                                                       int slot, const double *__restrict__ x,
                                                       double *__restrict__ y) {
  const double s = 1.0 / sqrt(scal[slot]);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i] * s;
}

inline unsigned grid_n(int64_t n) {
  int64_t g = (n + kTB - 1) / kTB;
  return (unsigned)std::min<int64_t>(g, 2048);
}

int ensure_gmres(edd_problem *p, int m) {
  if (p->gm_cap >= m) return EDD_OK;
  const size_t n = (size_t)p->ndof;
  p->gm_V = (double *)dev_alloc(p, sizeof(double) * n * (m + 1));
  p->gm_Z = (double *)dev_alloc(p, sizeof(double) * n * m);
  if (!p->gm_w) {
    p->gm_w = (double *)dev_alloc(p, sizeof(double) * n);
    p->gm_vG = (double *)dev_alloc(p, sizeof(double) * std::max<int64_t>(1, p->n_gamma * p->g.dim));
    p->gm_zG = (double *)dev_alloc(p, sizeof(double) * std::max<int64_t>(1, p->n_gamma * p->g.dim));
    p->gm_tI = (double *)dev_alloc(p, sizeof(double) * std::max<int64_t>(1, p->n_idofs));
  }
  if (!p->gm_V || !p->gm_Z || !p->gm_w || !p->gm_vG || !p->gm_zG || !p->gm_tI) return EDD_ENOMEM;
  p->gm_cap = m;
  return EDD_OK;
}

// z = P~^{-1} v (full nodal vectors)
int apply_block_triangular(edd_problem *p, const double *v, double *z, const edd_solve_opts *o,
                           edd_solve_stats *st) {
  const int64_t nG = p->n_gamma * p->g.dim;
  double *vG = p->gm_vG, *zG = p->gm_zG, *tI = p->gm_tI;
  if (nG > 0) {
    launch_gather(p, p->gnode_d, p->n_gamma, v, vG);
    if (o->precond == EDD_PC_IDENTITY) {
      launch_copy(p, nG, vG, zG);
    } else if (o->precond == EDD_PC_HTHETA) {
      int rc = precond_apply(p, vG, zG, o, st, false);
      if (rc) return rc;
    } else {  // EDD_PC_SCHUR: S~ = S, an interface solve preconditioned by Hhat_theta
      edd_solve_opts oi = *o;
      oi.precond = EDD_PC_HTHETA;
      int its = 0;
      int rc = interface_solve(p, vG, zG, o->mixed_inner_tol, &oi, st, kInnerMaxit, &its);
      st->outer_iterations += its;
      if (rc < 0) return rc;
    }
  }
  if (p->n_idofs > 0) {
    launch_apply_mapped(p, p->inode_d, p->n_inodes, nullptr, 0.0, nG > 0 ? zG : nullptr, 1.0, v,
                        -1.0, tI);
    launch_band_solve(p, EDD_F64, tI, tI);
  }
  launch_scatter_solution(p, tI, zG, z);
  return check_hip(p, hipGetLastError());
}

}  // namespace

int solve_full_gmres(edd_problem *p, const double *f, double *u, const edd_solve_opts *o,
                     edd_solve_stats *st) {
  const int64_t n = p->ndof;
  const int m = std::max(1, std::min(kMaxRestart, o->flexible_window > 0 ? o->flexible_window
                                                                         : kMaxRestart));
  int rc = ensure_gmres(p, m);
  if (rc) return rc;
  double *V = p->gm_V, *Z = p->gm_Z, *w = p->gm_w;
  launch_fill(p, m + 1, 1.0, p->scal_d + G_ONE);
  // ||f|| over free dofs
  launch_residual_norms(p, f, p->w_full[1], G_R);  // w_full[1] holds zeros
  rc = read_scalars(p, G_R, 2);
  if (rc) return rc;
  const double nf = std::sqrt(p->scal_h[G_R + 1]);
  if (!std::isfinite(nf)) return EDD_EINVAL;
  if (!o->use_initial_guess) launch_fill(p, n, 0.0, u);
  if (nf == 0.0) {
    launch_fill(p, n, 0.0, u);
    return EDD_OK;
  }
  const double tol_abs = o->tol * nf;
  int status = EDD_NOT_CONVERGED;
  int total = 0;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  while (total < o->maxit) {
    // r = f - K u (clamped entries zero), V_0 = r / ||r||
    launch_apply_full(p, u, w);
    launch_axpby(p, n, 1.0, f, -1.0, w);
    launch_mask_dirichlet(p, w);
    {
      const double *a[1] = {w}, *b[1] = {w};
      launch_dots(p, n, 1, a, b, G_R);
    }
    rc = read_scalars(p, G_R, 1);
    if (rc) return rc;
    const double beta = std::sqrt(p->scal_h[G_R]);
    if (!std::isfinite(beta)) return EDD_EBREAKDOWN;
    st->rel_residual = beta / nf;
    if (beta <= tol_abs) {
      status = EDD_OK;
      break;
    }
    k_scale_invsqrt<<<grid_n(n), kTB, 0, p->stream>>>(n, p->scal_d, G_R, w, V);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int j = 0, ncol = 0;
    bool done = false;
    for (; j < m && total < o->maxit; ++j) {
      double *Vj = V + (int64_t)j * n, *Zj = Z + (int64_t)j * n;
      rc = apply_block_triangular(p, Vj, Zj, o, st);
      if (rc) return rc;
      st->precond_applications += 1;
      launch_apply_full(p, Zj, w);
      // classical Gram-Schmidt, twice
      launch_window_dots(p, n, j + 1, V, w, G_H1);
      launch_window_combine(p, n, j + 1, V, G_H1, G_ONE, w, w);
      launch_window_dots(p, n, j + 1, V, w, G_H2);
      launch_window_combine(p, n, j + 1, V, G_H2, G_ONE, w, w);
      {
        const double *a[1] = {w}, *b[1] = {w};
        launch_dots(p, n, 1, a, b, G_NRM);
      }
      k_scale_invsqrt<<<grid_n(n), kTB, 0, p->stream>>>(n, p->scal_d, G_NRM, w,
                                                        V + (int64_t)(j + 1) * n);
      rc = read_scalars(p, G_H1, G_ONE - G_H1);
      if (rc) return rc;
      ++total;
      ++ncol;
      // Hessenberg column j and its Givens rotation
      double *hc = &H[(size_t)j * (m + 1)];
      for (int i = 0; i <= j; ++i) hc[i] = p->scal_h[G_H1 + i] + p->scal_h[G_H2 + i];
      const double hn = std::sqrt(std::max(0.0, p->scal_h[G_NRM]));
      hc[j + 1] = hn;
      for (int i = 0; i < j; ++i) {
        const double a = hc[i], b = hc[i + 1];
        hc[i] = cs[i] * a + sn[i] * b;
        hc[i + 1] = -sn[i] * a + cs[i] * b;
      }
      const double rr = std::hypot(hc[j], hc[j + 1]);
      if (!(rr > 0.0) || !std::isfinite(rr)) return EDD_EBREAKDOWN;
      cs[j] = hc[j] / rr;
      sn[j] = hc[j + 1] / rr;
      hc[j] = rr;
      hc[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      const double res = std::fabs(g[j + 1]);
      if (res <= tol_abs || !(hn > 1e-14 * beta)) {
        done = true;
        break;
      }
    }
    // y = R^{-1} g, u += Z y
    for (int i = ncol - 1; i >= 0; --i) {
      double s = g[i];
      for (int k = i + 1; k < ncol; ++k) s -= H[(size_t)k * (m + 1) + i] * y[k];
      y[i] = s / H[(size_t)i * (m + 1) + i];
    }
    for (int i = 0; i < ncol; ++i) p->scal_h[G_Y + i] = -y[i];
    hipError_t e = hipMemcpyAsync(p->scal_d + G_Y, p->scal_h + G_Y, sizeof(double) * ncol,
                                  hipMemcpyHostToDevice, p->stream);
    if (e != hipSuccess) return check_hip(p, e);
    launch_window_combine(p, n, ncol, Z, G_Y, G_ONE, u, u);
    // the loop re-checks the true residual (and restarts if it misses)
    (void)done;
  }
  st->iterations += total;
  // final FP64 residual
  launch_apply_full(p, u, w);
  launch_residual_norms(p, f, w, G_R);
  rc = read_scalars(p, G_R, 2);
  if (rc) return rc;
  st->rel_residual = std::sqrt(p->scal_h[G_R] / p->scal_h[G_R + 1]);
  if (st->rel_residual <= o->tol) status = EDD_OK;
  return status;
}

}  // namespace edd

extern "C" int edd_solve_gmres(edd_problem *p, const double *f_dev, double *u_dev,
                               const edd_solve_opts *o_in, edd_solve_stats *s_out) {
  using namespace edd;
  if (!p || !f_dev || !u_dev) return EDD_EINVAL;
  if (!p->have_moduli) return EDD_ESTATE;
  if (!(p->factor_precision & EDD_F64)) return EDD_ESTATE;
  edd_solve_opts o;
  if (o_in) o = *o_in;
  else edd_default_opts(&o);
  if (!(o.tol > 0.0) || o.maxit < 1) return EDD_EINVAL;
  if (o.precond != EDD_PC_IDENTITY && o.precond != EDD_PC_HTHETA && o.precond != EDD_PC_SCHUR)
    return EDD_EINVAL;
  if (o.precond != EDD_PC_IDENTITY &&
      (o.lanczos_kmax < 1 || o.lanczos_kmax > 64 || o.inner_maxit < 1 || o.theta > 1.0 ||
       o.pc_form < EDD_PCF_HTILDE_INV || o.pc_form > EDD_PCF_H_FWD))
    return EDD_EINVAL;
  if (o.precond == EDD_PC_SCHUR && !(o.mixed_inner_tol > 0.0)) return EDD_EINVAL;
  edd_solve_stats st{};
  const auto t0 = std::chrono::steady_clock::now();
  int status = solve_full_gmres(p, f_dev, u_dev, &o, &st);
  if (status >= 0) {
    const double *a[1] = {f_dev}, *b[1] = {u_dev};
    launch_dots(p, p->ndof, 1, a, b, G_R);
    int rc = read_scalars(p, G_R, 1);
    if (rc) return rc;
    st.compliance = p->scal_h[G_R];
  }
  st.t_total_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  st.status = status;
  if (s_out) *s_out = st;
  return status;
}

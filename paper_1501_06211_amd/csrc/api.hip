// C ABI entry points and the interface-solve driver.
//
// The solve follows eq. (3MatSplit) of the paper:
//   1. condensation   g = f_G - K_GI K_II^{-1} f_I
//   2. interface      S u_G = g by a flexible preconditioned CG
//   3. back-subst.    u_I = K_II^{-1} (f_I - K_IG u_G)
// where S v = K_GG v - K_GI K_II^{-1} K_IG v is applied as (K x)_G with
// x = (-K_II^{-1} (K [0; v])_I, v): two matrix-free element sweeps and one
// batched interior solve.  The stopping test uses ||r_G|| <= tol ||f||,
// which equals the full residual when the interior solves are exact; the
// final FP64 residual ||f - K u|| is recomputed with the element kernel and
// the iteration resumes if it is above the tolerance.
//
// Mixed mode: iterative refinement on the interface problem, the inner
// interface solves using FP32 interior factors (see solve_mixed).
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <cmath>
#include <cstring>
#include <cstdio>

#include "internal.h"

using namespace edd;

namespace edd {

// scalar slots in p->scal_d
// internal status: the reduced-precision phase of a relaxed solve stalled
constexpr int EDD_ESTALL = 100;

enum : int {
  S_RR = 0,
  S_FF = 1,
  S_PQCUR = 2,
  S_PR = 3,
  S_RES = 4,  // 4, 5: residual norms
  S_CMP = 6,  // compliance
  S_BAD = 7,
  S_BREAK = 8,  // set on the device by a breakdown step of the interface CG
  S_RRH = 9,    // 9..12: r.r of the last iterations (ring of kCheck)
  S_NETDROP = 13,  // set by a network step that gave no direction (dropped)
  S_C_BASE = 4096,  // window coefficients <z, q_j>, one per ring slot
  S_PQ_BASE = 4096 + kMaxWindow,  // <p_j, q_j> per ring slot
  S_TOTAL = kScalTotal
};

void *dev_alloc(edd_problem *p, size_t bytes) {
  bytes = ((bytes ? bytes : 8) + 255) & ~(size_t)255;
  void *ptr = nullptr;
  if (p->alloc_fn) {
    ptr = p->alloc_fn(p->alloc_ctx, bytes);
  } else if (hipMalloc(&ptr, bytes) != hipSuccess) {
    ptr = nullptr;
  }
  if (ptr) p->allocations.push_back(ptr);
  return ptr;
}

int check_hip(edd_problem *p, hipError_t e) {
  if (e != hipSuccess) {
    p->last_hip_error = (int)e;
    return EDD_EHIP;
  }
  return EDD_OK;
}

int read_scalars(edd_problem *p, int first, int count) {
  hipError_t e = hipMemcpyAsync(p->scal_h + first, p->scal_d + first,
                                sizeof(double) * count, hipMemcpyDeviceToHost,
                                p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  return check_hip(p, e);
}

int sync_check(edd_problem *p) {
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  return check_hip(p, e);
}

static hipEvent_t kt_event(edd_problem *p) {
  if (!p->kt_pool.empty()) {
    hipEvent_t e = p->kt_pool.back();
    p->kt_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

static void kt_resolve(edd_problem *p) {
  for (auto &pd : p->kt_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(pd.b) == hipSuccess &&
        hipEventElapsedTime(&ms, pd.a, pd.b) == hipSuccess) {
      p->kt_count[pd.kind] += 1;
      p->kt_ms[pd.kind] += ms;
    }
    p->kt_pool.push_back(pd.a);
    p->kt_pool.push_back(pd.b);
  }
  p->kt_pending.clear();
}

KTimer::KTimer(edd_problem *p_, int kind_) : p(p_), kind(kind_) {
  if (!p->kt_enabled) return;
  a = kt_event(p);
  b = kt_event(p);
  if (a && b) hipEventRecord(a, p->stream);
}

KTimer::~KTimer() {
  if (!p->kt_enabled || !a || !b) return;
  hipEventRecord(b, p->stream);
  p->kt_pending.push_back({kind, a, b});
  if (p->kt_pending.size() > 4096) kt_resolve(p);
}

// y = S v on interface vectors; t is an interior-length work vector
void apply_S_with(edd_problem *p, const double *v, double *y, int prec, double *t) {
  if (p->s_apply_mode == 1 && p->sc_ready && prec != EDD_F32) {
    schur_apply(p, v, y);  // explicit local Schur complements (FP64)
    return;
  }
  launch_apply_mapped(p, p->inode_d, p->n_inodes, nullptr, 0.0, v, 1.0, nullptr,
                      1.0, t);
  launch_band_solve(p, prec, t, t);
  launch_apply_mapped(p, p->gnode_d, p->n_gamma, t, -1.0, v, 1.0, nullptr, 1.0, y);
}

void apply_S(edd_problem *p, const double *v, double *y, int prec) {
  apply_S_with(p, v, y, prec, p->w_I[2]);
}

// Ring slots [0, nslots) of the flexible-CG window: blocks of kWinBlock
// directions (P) and their S images (Q), each allocated the first time the
// iteration reaches it and kept until the handle is destroyed.
static int ensure_window(edd_problem *p, int nslots) {
  constexpr int kTab = kMaxWindow / kWinBlock;
  const size_t nG = (size_t)p->n_gamma * p->g.dim;
  if (!p->win_tab_d) {
    p->win_tab_d = (double **)dev_alloc(p, sizeof(double *) * 2 * kTab);
    if (!p->win_tab_d) return EDD_ENOMEM;
  }
  while ((int)p->winP_blk.size() * kWinBlock < nslots) {
    // one allocation per block, so a failed one leaves nothing behind
    double *P = (double *)dev_alloc(p, sizeof(double) * 2 * nG * kWinBlock);
    if (!P) return EDD_ENOMEM;
    double *Q = P + nG * kWinBlock;
    const int b = (int)p->winP_blk.size();
    p->winP_blk.push_back(P);
    p->winQ_blk.push_back(Q);
    // the kernels that read these entries are queued after the copies
    p->win_tab_h[b] = P;
    p->win_tab_h[kTab + b] = Q;
    int rc = check_hip(p, hipMemcpyAsync(p->win_tab_d + b, &p->win_tab_h[b], sizeof(double *),
                                         hipMemcpyHostToDevice, p->stream));
    if (!rc)
      rc = check_hip(p, hipMemcpyAsync(p->win_tab_d + kTab + b, &p->win_tab_h[kTab + b],
                                       sizeof(double *), hipMemcpyHostToDevice, p->stream));
    if (rc) return rc;
  }
  return EDD_OK;
}

static double *win_slot(const std::vector<double *> &blk, int64_t n, int slot) {
  return blk[slot / kWinBlock] + (int64_t)(slot % kWinBlock) * n;
}

// Directions the flexible CG keeps: the option if set; else one (plain CG)
// for the identity preconditioner, kWinBlock for the captured iteration,
// and all of them (up to kMaxWindow) otherwise.
static int fcg_window(const edd_solve_opts *o) {
  if (o->flexible_window > 0) return o->flexible_window;
  if (o->precond == EDD_PC_IDENTITY) return 1;
  return o->use_graphs >= 2 ? kWinBlock : kMaxWindow;
}

// Orthogonalise z against the m newest directions of the window ring
// (capacity cap, direction j at slot j % cap, newest at (k-1) % cap) and
// write the result to out: every coefficient against z first (one launch
// for the dots, one for their sums), then one combine, oldest first.
static void window_orthogonalise(edd_problem *p, int64_t n, int cap, int k, int m,
                                 const double *z, double *out, int cbase, int dbase) {
  if (m <= 0) {
    if (out != z) launch_copy(p, n, z, out);
    return;
  }
  constexpr int kTab = kMaxWindow / kWinBlock;
  const int first = (k - m) % cap;  // k >= m
  launch_ring_dots(p, n, cap, first, m, p->win_tab_d + kTab, z, cbase);
  launch_ring_combine(p, n, cap, first, m, p->win_tab_d, cbase, dbase, z, out);
}

// Condensation g = f_G - K_GI K_II^{-1} f_I (first two lines of eq.
// (3MatSplit)) with interior factors of precision prec.
static void condense(edd_problem *p, const double *f, double *g, int prec) {
  double *wI = p->w_I[0];
  launch_gather(p, p->inode_d, p->n_inodes, f, wI);
  launch_band_solve(p, prec, wI, wI);
  launch_apply_mapped(p, p->gnode_d, p->n_gamma, wI, 1.0, nullptr, 0.0, f, -1.0, g);
}

// Back-substitution u_I = K_II^{-1} (f_I - K_IG u_G) (third line of eq.
// (3MatSplit)) and assembly of the full-length u.
static void back_substitute(edd_problem *p, const double *f, const double *uG, double *u,
                            int prec) {
  double *t = p->w_I[1];
  launch_apply_mapped(p, p->inode_d, p->n_inodes, nullptr, 0.0, uG, 1.0, f, -1.0, t);
  launch_band_solve(p, prec, t, t);
  launch_scatter_solution(p, t, uG, u);
}

// The iterations of interface_fcg as replays of a captured graph of
// o->use_graphs iterations (device-resident preconditioner, no precision
// switch): the window position comes from the device iteration index, each
// new direction goes through fixed buffers into its ring slot, and a device
// flag records the first iteration whose residual met tol_abs.  The host
// reads the flag once per replay; the iterations of the last replay that
// follow convergence only refine x (the reported count is the first
// converged iteration).  Up to that iteration the arithmetic, and its order,
// is that of the host-driven loop.  Entered with r and x set and rr = r.r.
static int fcg_graph_iterations(edd_problem *p, double *x, int prec, double tol_abs,
                                const edd_solve_opts *o, edd_solve_stats *st, int maxit,
                                int cap, int *iters) {
  const int64_t nG = p->n_gamma * p->g.dim;
  const int N = std::max(2, std::min(o->use_graphs, 64));
  double *r = p->w_G[1], *z = p->w_G[2];
  if (!p->gr_p_d) {
    p->gr_p_d = (double *)dev_alloc(p, sizeof(double) * std::max<int64_t>(1, nG));
    p->gr_q_d = (double *)dev_alloc(p, sizeof(double) * std::max<int64_t>(1, nG));
    if (!p->gr_p_d || !p->gr_q_d) return EDD_ENOMEM;
  }
  double *pn = p->gr_p_d, *qn = p->gr_q_d;
  const bool pc_identity = o->precond == EDD_PC_IDENTITY;
  edd_solve_opts oc = *o;
  oc.use_graphs = 0;  // the preconditioner's kernels go into this graph directly
  const double th = o->theta;
  int64_t key[12] = {N, cap, prec, (int64_t)(uintptr_t)x, o->precond, o->lanczos_kmax,
                     o->inner_maxit, o->interface_weighting, o->pc_form, 0, o->mass_matrix, nG};
  std::memcpy(&key[9], &th, sizeof th);
  if (!p->fcg_graph || std::memcmp(key, p->fcg_graph_key, sizeof key) != 0) {
    if (p->fcg_graph) {
      hipGraphExecDestroy(p->fcg_graph);
      p->fcg_graph = nullptr;
    }
    if (!p->cap_stream &&
        hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess) {
      p->cap_stream = nullptr;
      return EDD_EHIP;
    }
    // work buffers the preconditioner allocates on first use: allocate now,
    // outside the capture
    if (!pc_identity) {
      int rc = precond_apply(p, r, z, &oc, nullptr, false);
      if (rc) return rc;
      rc = check_hip(p, hipStreamSynchronize(p->stream));
      if (rc) return rc;
    }
    hipStream_t saved = p->stream;
    const bool kt = p->kt_enabled;
    p->kt_enabled = false;
    p->stream = p->cap_stream;
    hipGraph_t graph = nullptr;
    int rc = EDD_OK;
    if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      rc = EDD_EHIP;
    } else {
      for (int it = 0; it < N && rc == EDD_OK; ++it) {
        const double *zp = r;
        if (!pc_identity) {
          rc = precond_apply(p, r, z, &oc, nullptr, false);
          zp = z;
        }
        launch_window_dots_dev(p, nG, cap, p->winQ_blk[0], zp, S_C_BASE);
        launch_window_combine_dev(p, nG, cap, p->winP_blk[0], S_C_BASE, S_PQ_BASE, zp, pn);
        apply_S(p, pn, qn, prec);
        {
          const double *a[2] = {pn, pn}, *b[2] = {qn, r};
          launch_dots(p, nG, 2, a, b, S_PQCUR);
        }
        launch_cg_update(p, nG, S_PR, S_PQCUR, x, pn, r, qn, kSlotGRR, kSlotGPQ, S_BREAK);
        launch_ring_store(p, nG, cap, pn, p->winP_blk[0]);
        launch_ring_store(p, nG, cap, qn, p->winQ_blk[0]);
        launch_iter_end(p, cap, S_PQ_BASE);
      }
      if (hipStreamEndCapture(p->cap_stream, &graph) != hipSuccess) rc = EDD_EHIP;
    }
    p->stream = saved;
    p->kt_enabled = kt;
    if (rc == EDD_OK && graph &&
        hipGraphInstantiate(&p->fcg_graph, graph, nullptr, nullptr, 0) != hipSuccess) {
      p->fcg_graph = nullptr;
      rc = EDD_EHIP;
    }
    if (graph) hipGraphDestroy(graph);
    (void)hipGetLastError();
    if (rc) return rc;
    std::memcpy(p->fcg_graph_key, key, sizeof key);
  }
  // device iteration state
  launch_fill(p, 1, 0.0, p->scal_d + kSlotGK);
  launch_fill(p, 1, 0.0, p->scal_d + kSlotGDone);
  launch_fill(p, 1, tol_abs * tol_abs, p->scal_d + kSlotGTol2);
  int k = 0, status = EDD_NOT_CONVERGED;
  while (k < maxit) {
    int rc = check_hip(p, hipGraphLaunch(p->fcg_graph, p->stream));
    if (rc) return rc;
    rc = read_scalars(p, kSlotGK, kSlotGHist + kGHist - kSlotGK);
    if (rc) return rc;
    k = (int)p->scal_h[kSlotGK];
    if (st) {
      st->precond_applications += pc_identity ? 0 : N;
      st->lanczos_steps += pc_identity ? 0 : N * std::min(o->lanczos_kmax, 32);
      if (!pc_identity && o->pc_form != EDD_PCF_HTILDE_FWD && o->pc_form != EDD_PCF_H_FWD)
        st->inner_iterations += N * std::min(o->lanczos_kmax, 32) * o->inner_maxit;
    }
    const double rr = p->scal_h[kSlotGHist + (k - 1) % kGHist];
    if (p->scal_h[kSlotGDone] > 0.0) {
      *iters = (int)p->scal_h[kSlotGDone];
      return EDD_OK;
    }
    if (!std::isfinite(rr) || p->scal_h[S_BREAK] != 0.0) {
      status = EDD_EBREAKDOWN;
      break;
    }
  }
  *iters = k;
  return status;
}

// Flexible CG on S x = rhs with S applied through interior factors of
// precision prec; x holds the initial guess when use_guess.  Stops when the
// recursive residual is <= tol_abs.  Returns EDD_OK, EDD_NOT_CONVERGED,
// EDD_EBREAKDOWN or an error; *iters receives the iterations.
static int interface_fcg(edd_problem *p, const double *rhs, double *x, int prec,
                         double tol_abs, bool use_guess, const edd_solve_opts *o,
                         edd_solve_stats *st, int maxit, int window, int *iters,
                         double relax_abs = -1.0) {
  const int D = p->g.dim;
  const int64_t nG = p->n_gamma * D;
  double *r = p->w_G[1], *z = p->w_G[2], *tmp = p->w_G[4];
  *iters = 0;
  if (use_guess) {
    apply_S(p, x, tmp, prec);
    launch_copy(p, nG, rhs, r);
    launch_axpby(p, nG, -1.0, tmp, 1.0, r);
  } else {
    launch_fill(p, nG, 0.0, x);
    launch_copy(p, nG, rhs, r);
  }
  {
    const double *a[1] = {r}, *b[1] = {r};
    launch_dots(p, nG, 1, a, b, S_RR);
  }
  int rc = read_scalars(p, S_RR, 1);
  if (rc) return rc;
  double rr = p->scal_h[S_RR];
  if (!std::isfinite(rr)) return EDD_EINVAL;
  const bool pc_identity = o->precond == EDD_PC_IDENTITY;
  const int cap = std::max(1, std::min(window, kMaxWindow));
  rc = ensure_window(p, std::min(cap, kWinBlock));
  if (rc) return rc;
  const bool pc_dev = pc_identity || (o->lanczos_tol <= 0.0 && o->inner_tol <= 0.0);
  // the captured iteration keeps its ring in the first block
  if (o->use_graphs >= 2 && cap <= kWinBlock && pc_dev && relax_abs <= 0.0 &&
      o->learned_correction <= 0 && std::sqrt(rr) > tol_abs) {
    launch_fill(p, 1, 0.0, p->scal_d + S_BREAK);
    return fcg_graph_iterations(p, x, prec, tol_abs, o, st, maxit, cap, iters);
  }
  int status = EDD_OK;
  int k = 0;
  int k_switch = -1;
  double rr_switch = 0.0;
  // With a preconditioner that runs without host waits the host checks the
  // residual every kCheck iterations; steps past convergence in between are
  // harmless (a step with no descent changes nothing, see launch_cg_update).
  constexpr int kCheck = 4;
  const bool pc_device = pc_identity || (o->lanczos_tol <= 0.0 && o->inner_tol <= 0.0);
  const int check = pc_device ? kCheck : 1;
  launch_fill(p, 1, 0.0, p->scal_d + S_BREAK);
  launch_fill(p, 1, 0.0, p->scal_d + S_NETDROP);
  int converged_at = -1;
  while (std::sqrt(rr) > tol_abs) {
    if (k >= maxit) { status = EDD_NOT_CONVERGED; break; }
    // relaxed operator accuracy: once the residual is small, the S applies
    // may carry a larger error without spoiling the attainable accuracy
    if (relax_abs > 0.0 && prec != EDD_F32 && std::sqrt(rr) <= relax_abs) {
      prec = EDD_F32;
      k_switch = k;
      rr_switch = rr;
    }
    // after the switch the residual must keep falling (at least 10x per 50
    // iterations); otherwise the reduced-precision phase has stalled
    if (k_switch >= 0 && k - k_switch >= 50) {
      if (rr > 1e-2 * rr_switch) { status = EDD_ESTALL; break; }
      k_switch = k;
      rr_switch = rr;
    }
    const double *zp = r;
    int flag_slot = S_BREAK;
    // every learned_correction-th step takes its direction from the
    // correction network applied to the interface residual extended by zero
    // (an approximation of S^{-1} r = (K^{-1} [0; r])_G): the flexible
    // iteration accepts a different preconditioner at every step, and the
    // exact line search keeps the step from raising the energy error; a
    // network step with no usable direction is dropped
    const bool net_step = o->learned_correction > 0 && p->cnn_nparams > 0 && k > 0 &&
                          k % o->learned_correction == 0;
    if (net_step) {
      launch_scatter_solution(p, nullptr, r, p->cnn_r_d);
      rc = cnn_predict(p, nullptr, p->cnn_r_d, p->cnn_dir_d);
      if (rc) return rc;
      launch_gather(p, p->gnode_d, p->n_gamma, p->cnn_dir_d, z);
      zp = z;
      flag_slot = S_NETDROP;
    } else if (!pc_identity) {
      rc = precond_apply(p, r, z, o, st, prec == EDD_F32);
      if (rc) return rc;
      zp = z;
    }
    const int slot = k % cap;
    rc = ensure_window(p, slot + 1);
    if (rc) return rc;
    double *Pk = win_slot(p->winP_blk, nG, slot);
    double *Qk = win_slot(p->winQ_blk, nG, slot);
    const int m = std::min(k, cap);
    window_orthogonalise(p, nG, cap, k, m, zp, Pk, S_C_BASE, S_PQ_BASE);
    apply_S(p, Pk, Qk, prec);
    {
      const double *a[2] = {Pk, Pk}, *b[2] = {Qk, r};
      launch_dots(p, nG, 2, a, b, S_PQCUR);
    }
    launch_cg_update(p, nG, S_PR, S_PQCUR, x, Pk, r, Qk, S_RRH + (k % kCheck),
                     S_PQ_BASE + slot, flag_slot);
    ++k;
    if (k % check != 0 && k < maxit) continue;
    rc = read_scalars(p, 0, S_RRH + kCheck);
    if (rc) return rc;
    // the iterations since the last check: the first whose residual met the
    // tolerance is the reported count (later steps only refine x)
    const int n_chunk = (k - 1) % check + 1;
    for (int j = 0; j < n_chunk; ++j) {
      const int it = k - n_chunk + j;
      const double rj = p->scal_h[S_RRH + it % kCheck];
      if (converged_at < 0 && std::isfinite(rj) && std::sqrt(rj) <= tol_abs) converged_at = it + 1;
    }
    rr = p->scal_h[S_RRH + (k - 1) % kCheck];
    if (std::sqrt(rr) > tol_abs) converged_at = -1;  // not converged at the check
    if (!std::isfinite(rr)) {
      status = EDD_EBREAKDOWN;
      break;
    }
    if (p->scal_h[S_BREAK] != 0.0 && std::sqrt(rr) > tol_abs) {
      status = EDD_EBREAKDOWN;
      break;
    }
  }
  *iters = converged_at >= 0 ? converged_at : k;
  if (o->learned_correction > 0 && st) {
    int rc2 = read_scalars(p, S_NETDROP, 1);
    if (rc2) return rc2;
    if (p->scal_h[S_NETDROP] != 0.0) st->flags |= EDD_FLAG_LEARNED_REJECTED;
  }
  return status;
}

// S x = rhs by the interface flexible CG to ||rhs - S x|| <= rel_tol ||rhs||
// (FP64 interior factors, zero initial guess); for composition (the full
// GMRES path applies S~ = S with it).
int interface_solve(edd_problem *p, const double *rhs, double *x, double rel_tol,
                    const edd_solve_opts *o, edd_solve_stats *st, int maxit, int *iters) {
  const int64_t nG = p->n_gamma * p->g.dim;
  {
    const double *a[1] = {rhs}, *b[1] = {rhs};
    launch_dots(p, nG, 1, a, b, S_RES);
  }
  int rc = read_scalars(p, S_RES, 1);
  if (rc) return rc;
  const double nr = std::sqrt(p->scal_h[S_RES]);
  if (!std::isfinite(nr)) return EDD_EINVAL;
  if (nr == 0.0) {
    launch_fill(p, nG, 0.0, x);
    *iters = 0;
    return EDD_OK;
  }
  return interface_fcg(p, rhs, x, EDD_F64, rel_tol * nr, false, o, st, maxit, fcg_window(o),
                       iters);
}

// The three steps of eq. (3MatSplit) with interior factors of precision
// prec: condensation, interface FCG to tol_abs, back-substitution.
static int schur_solve_core(edd_problem *p, const double *f, double *u, int prec,
                            double tol_abs, bool use_guess, const edd_solve_opts *o,
                            edd_solve_stats *st, int maxit, int window, int *iters) {
  double *x = p->w_G[0], *g = p->w_G[3];
  condense(p, f, g, prec);
  if (use_guess) launch_gather(p, p->gnode_d, p->n_gamma, u, x);
  const int status = interface_fcg(p, g, x, prec, tol_abs, use_guess, o, st, maxit,
                                   window, iters);
  if (status == EDD_EBREAKDOWN || status < 0) return status;
  back_substitute(p, f, x, u, prec);
  return status;
}

static int true_residual(edd_problem *p, const double *f, const double *u,
                         double *rel) {
  launch_apply_full(p, u, p->w_full[0]);
  launch_residual_norms(p, f, p->w_full[0], S_RES);
  int rc = read_scalars(p, S_RES, 2);
  if (rc) return rc;
  const double rr = p->scal_h[S_RES], ff = p->scal_h[S_RES + 1];
  *rel = ff > 0 ? std::sqrt(rr / ff) : 0.0;
  return EDD_OK;
}

static int norm_f(edd_problem *p, const double *f, double *nf) {
  launch_residual_norms(p, f, p->w_full[1], S_RES);  // w_full[1] holds zeros
  int rc = read_scalars(p, S_RES, 2);
  if (rc) return rc;
  *nf = std::sqrt(p->scal_h[S_RES + 1]);
  return EDD_OK;
}

static int solve_plain(edd_problem *p, const double *f, double *u,
                       const edd_solve_opts *o, edd_solve_stats *st, double nf) {
  const int window = fcg_window(o);
  double tol_abs = o->tol * nf;
  bool guess = o->use_initial_guess != 0;
  int status = EDD_OK;
  for (int attempt = 0; attempt < 3; ++attempt) {
    int its = 0;
    status = schur_solve_core(p, f, u, EDD_F64, tol_abs, guess, o, st,
                              o->maxit - st->iterations, window, &its);
    st->iterations += its;
    if (status < 0) return status;
    double rel = 0.0;
    int rc = true_residual(p, f, u, &rel);
    if (rc) return rc;
    st->rel_residual = rel;
    if (rel <= o->tol || status == EDD_NOT_CONVERGED) break;
    // recursive residual drifted from the true one: resume from u
    st->flags |= EDD_FLAG_TRUE_RES_RESTART;
    tol_abs *= 0.5 * o->tol / rel;
    guess = true;
    status = EDD_NOT_CONVERGED;
  }
  return status;
}

// Mixed precision (Section 3's inexact interface solves, realised as
// iterative refinement): FP64 condensation; rounds of
//   r = g - S x        with the FP64 interior factors,
//   S d = r            by FCG with the FP32 interior factors, to a loose
//                      relative tolerance (mixed_inner_tol),
//   x += d;
// then FP64 back-substitution and the FP64 true residual.  A round that
// does not halve the interface residual ends the reduced-precision phase and
// the FP64 solve finishes from the current iterate.
static int solve_mixed(edd_problem *p, const double *f, double *u,
                       const edd_solve_opts *o, edd_solve_stats *st, double nf) {
  const int D = p->g.dim;
  const int64_t nG = p->n_gamma * D;
  double *g = p->w_G[3], *x = p->w_G[5], *d = p->w_G[0], *r = p->w_G[6],
         *t = p->w_G[7];
  const int window = fcg_window(o);
  condense(p, f, g, EDD_F64);
  if (o->use_initial_guess) launch_gather(p, p->gnode_d, p->n_gamma, u, x);
  else launch_fill(p, nG, 0.0, x);
  const double tol_abs = o->tol * nf;
  double prev = -1.0;
  int status = EDD_NOT_CONVERGED;
  int round = 0;
  for (; round < std::max(1, o->outer_maxit); ++round) {
    // FP64 interface residual
    apply_S(p, x, t, EDD_F64);
    launch_copy(p, nG, g, r);
    launch_axpby(p, nG, -1.0, t, 1.0, r);
    {
      const double *a[1] = {r}, *b[1] = {r};
      launch_dots(p, nG, 1, a, b, S_RES);
    }
    int rc = read_scalars(p, S_RES, 1);
    if (rc) return rc;
    const double rn = std::sqrt(p->scal_h[S_RES]);
    if (!std::isfinite(rn)) return EDD_EBREAKDOWN;
    if (rn <= 0.5 * tol_abs) { status = EDD_OK; break; }
    if (prev >= 0.0 && rn > 0.5 * prev) break;  // stalled
    prev = rn;
    int its = 0;
    rc = interface_fcg(p, r, d, EDD_F32, std::max(o->mixed_inner_tol * rn, 0.25 * tol_abs),
                       false, o, st, o->maxit - st->iterations, window, &its);
    st->iterations += its;
    if (rc < 0) return rc;
    launch_axpby(p, nG, 1.0, d, 1.0, x);
    if (st->iterations >= o->maxit) break;
  }
  st->outer_iterations = round;
  back_substitute(p, f, x, u, EDD_F64);
  double rel = 0.0;
  int rc = true_residual(p, f, u, &rel);
  if (rc) return rc;
  st->rel_residual = rel;
  if (rel <= o->tol) return EDD_OK;
  st->flags |= EDD_FLAG_MIXED_FALLBACK;
  edd_solve_opts o2 = *o;
  o2.use_initial_guess = 1;
  return solve_plain(p, f, u, &o2, st, nf);
}

// Relaxed mixed precision (inexact Krylov): one FCG on S with FP64 interior
// factors until the interface residual falls below mixed_inner_tol times the
// initial one, FP32-stored factors after that; FP64 condensation,
// back-substitution and true residual.  If the true residual misses the
// tolerance the FP64 solve restarts from the current iterate.
static int solve_relaxed(edd_problem *p, const double *f, double *u,
                         const edd_solve_opts *o, edd_solve_stats *st, double nf) {
  const int D = p->g.dim;
  const int64_t nG = p->n_gamma * D;
  double *x = p->w_G[0], *g = p->w_G[3];
  const int window = fcg_window(o);
  condense(p, f, g, EDD_F64);
  const bool guess = o->use_initial_guess != 0;
  if (guess) launch_gather(p, p->gnode_d, p->n_gamma, u, x);
  // initial interface residual norm sets the switch point
  {
    double *t = p->w_G[4], *r = p->w_G[1];
    if (guess) {
      apply_S(p, x, t, EDD_F64);
      launch_copy(p, nG, g, r);
      launch_axpby(p, nG, -1.0, t, 1.0, r);
    } else {
      launch_copy(p, nG, g, r);
    }
    const double *a[1] = {r}, *b[1] = {r};
    launch_dots(p, nG, 1, a, b, S_RES);
  }
  int rc = read_scalars(p, S_RES, 1);
  if (rc) return rc;
  const double r0 = std::sqrt(p->scal_h[S_RES]);
  const double tol_abs = o->tol * nf;
  int its = 0;
  int status = interface_fcg(p, g, x, EDD_F64, tol_abs, guess, o, st, o->maxit, window,
                             &its, o->mixed_inner_tol * r0);
  st->iterations += its;
  if (status == EDD_ESTALL) {
    st->flags |= EDD_FLAG_MIXED_FALLBACK;
    status = EDD_NOT_CONVERGED;
  } else if (status == EDD_EBREAKDOWN || status < 0) {
    return status;
  }
  back_substitute(p, f, x, u, EDD_F64);
  double rel = 0.0;
  rc = true_residual(p, f, u, &rel);
  if (rc) return rc;
  st->rel_residual = rel;
  st->outer_iterations = 1;
  if (rel <= o->tol) return EDD_OK;
  if (status == EDD_NOT_CONVERGED && !(st->flags & EDD_FLAG_MIXED_FALLBACK)) return status;
  // the reduced-precision phase stalled, or the recursive residual drifted
  // under the relaxed applies: FP64 restart from the current iterate
  if (!(st->flags & EDD_FLAG_MIXED_FALLBACK)) st->flags |= EDD_FLAG_TRUE_RES_RESTART;
  edd_solve_opts o2 = *o;
  o2.use_initial_guess = 1;
  return solve_plain(p, f, u, &o2, st, nf);
}

// Learned initial guess: u += alpha d with d the network's proposal for the
// residual f - K u and alpha the exact minimiser of the interface energy
// error along d_G: alpha = <d_G, g - S u_G> / <d_G, S d_G>.  The interior
// part of u is recomputed by back-substitution, so only u_G matters.
static int learned_guess(edd_problem *p, const double *f, double *u, const edd_solve_opts *o,
                         edd_solve_stats *st) {
  const int D = p->g.dim;
  const int64_t nG = p->n_gamma * D;
  if (!o->use_initial_guess) launch_fill(p, p->ndof, 0.0, u);
  double *r = p->cnn_r_d, *d = p->cnn_dir_d;
  launch_apply_full(p, u, p->w_full[0]);
  launch_copy(p, p->ndof, f, r);
  launch_axpby(p, p->ndof, -1.0, p->w_full[0], 1.0, r);
  launch_mask_dirichlet(p, r);
  int rc = cnn_predict(p, nullptr, r, d);
  if (rc) return rc;
  double *g = p->w_G[3], *x0 = p->w_G[0], *dG = p->w_G[5], *r0 = p->w_G[6], *t = p->w_G[7];
  condense(p, f, g, EDD_F64);
  launch_gather(p, p->gnode_d, p->n_gamma, u, x0);
  launch_gather(p, p->gnode_d, p->n_gamma, d, dG);
  apply_S(p, x0, t, EDD_F64);
  launch_copy(p, nG, g, r0);
  launch_axpby(p, nG, -1.0, t, 1.0, r0);
  apply_S(p, dG, t, EDD_F64);
  {
    const double *a2[2] = {dG, dG}, *b2[2] = {r0, t};
    launch_dots(p, nG, 2, a2, b2, S_RES);
  }
  rc = read_scalars(p, S_RES, 2);
  if (rc) return rc;
  const double num = p->scal_h[S_RES], den = p->scal_h[S_RES + 1];
  const double alpha = den > 0.0 ? num / den : 0.0;
  if (!(den > 0.0) || !std::isfinite(alpha)) {
    st->flags |= EDD_FLAG_LEARNED_REJECTED;
    st->learned_alpha = 0.0;
    return EDD_OK;
  }
  launch_axpby(p, p->ndof, alpha, d, 1.0, u);
  st->learned_alpha = alpha;
  return EDD_OK;
}

}  // namespace edd

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void edd_default_opts(edd_solve_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-8;
  o->maxit = 2000;
  o->precision = EDD_MODE_F64;
  o->precond = EDD_PC_HTHETA;
  o->theta = 0.5;
  o->lanczos_kmax = 3;
  o->lanczos_tol = 0.0;
  o->inner_tol = 0.0;
  o->inner_maxit = 4;
  o->use_initial_guess = 0;
  o->outer_maxit = 20;
  o->mixed_inner_tol = 1e-4;
  o->flexible_window = 0;
  o->interface_weighting = 1;
  o->learned_guess = 0;
  o->use_graphs = 0;
  o->pc_form = EDD_PCF_HTILDE_INV;
  o->learned_correction = 0;
  o->mass_matrix = 0;
}

const char *edd_strerror(int code) {
  switch (code) {
    case EDD_OK: return "ok";
    case EDD_NOT_CONVERGED: return "tolerance not reached within the iteration limit";
    case EDD_EINVAL: return "invalid argument";
    case EDD_ENOMEM: return "device allocation failed";
    case EDD_EHIP: return "HIP runtime error";
    case EDD_ESTATE: return "call out of order (element moduli not set?)";
    case EDD_ENOTSPD: return "interior block not positive definite";
    case EDD_EBREAKDOWN: return "Krylov breakdown";
    default: return "unknown status";
  }
}

int edd_last_hip_error(edd_problem *p) { return p ? p->last_hip_error : 0; }

int edd_destroy(edd_problem *p) {
  if (!p) return EDD_OK;
  hipStreamSynchronize(p->stream);
  if (p->pc_graph) hipGraphExecDestroy(p->pc_graph);
  if (p->fcg_graph) hipGraphExecDestroy(p->fcg_graph);
  if (p->cap_stream) hipStreamDestroy(p->cap_stream);
  for (void *ptr : p->allocations) {
    if (p->free_fn) p->free_fn(p->alloc_ctx, ptr);
    else hipFree(ptr);
  }
  if (p->scal_h) hipHostFree(p->scal_h);
  if (p->pc_h) hipHostFree(p->pc_h);
  kt_resolve(p);
  for (hipEvent_t e : p->kt_pool) hipEventDestroy(e);
  delete p;
  return EDD_OK;
}

static int validate_desc(const edd_mesh_desc *d) {
  if (!d || (d->dim != 2 && d->dim != 3)) return EDD_EINVAL;
  if (!(d->nu > -1.0 && d->nu < 0.5)) return EDD_EINVAL;
  if ((d->clamp_faces & ((1 << (2 * d->dim)) - 1)) == 0) return EDD_EINVAL;
  if (!(d->factor_precision & (EDD_F64 | EDD_F32))) return EDD_EINVAL;
  if (d->dissect < -1 || d->dissect > 2) return EDD_EINVAL;
  int64_t nodes = 1;
  for (int a = 0; a < d->dim; ++a) {
    if (d->nel[a] < 1 || d->nel[a] > (1 << 20)) return EDD_EINVAL;
    if (d->ncuts[a] < 2 || !d->cuts[a]) return EDD_EINVAL;
    if (d->cuts[a][0] != 0 || d->cuts[a][d->ncuts[a] - 1] != d->nel[a]) return EDD_EINVAL;
    for (int c = 1; c < d->ncuts[a]; ++c)
      if (d->cuts[a][c] <= d->cuts[a][c - 1]) return EDD_EINVAL;
    nodes *= d->nel[a] + 1;
  }
  if (nodes * d->dim >= ((int64_t)1 << 31)) return EDD_EINVAL;
  return EDD_OK;
}

#define EDD_TRY_ALLOC(ptr, type, count)                                      \
  do {                                                                       \
    ptr = (type *)edd::dev_alloc(p, sizeof(type) * (size_t)(count));         \
    if (!ptr) { edd_destroy(p); return EDD_ENOMEM; }                         \
  } while (0)

int edd_setup_mesh(const edd_mesh_desc *d, const edd_allocator *a,
                   void *hip_stream, edd_problem **out) {
  if (!out) return EDD_EINVAL;
  *out = nullptr;
  int rc = validate_desc(d);
  if (rc) return rc;
  edd_problem *p = new (std::nothrow) edd_problem();
  if (!p) return EDD_ENOMEM;
  p->stream = (hipStream_t)hip_stream;
  if (a && a->alloc && a->free) {
    p->alloc_fn = a->alloc;
    p->free_fn = a->free;
    p->alloc_ctx = a->ctx;
  }
  p->factor_precision = d->factor_precision;
  p->dissect = d->dissect;
  if (hipGetDevice(&p->device) != hipSuccess) { delete p; return EDD_EHIP; }
  {
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, p->device) ==
            hipSuccess && cu > 0)
      p->n_cu = cu;
  }
  rc = build_geometry(p, d);
  if (rc) { delete p; return rc; }
  rc = scratch_init(p);
  if (rc) { delete p; return rc; }
  int lds = 0;
  hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device);
  p->lds_limit = lds > 0 ? (size_t)lds : 65536;
  if (p->max_kd + 32 > 1024 ||
      band_solve_lds_bytes(p, EDD_F64) > p->lds_limit) {
    delete p;
    return EDD_EINVAL;  // subdomains too large for one workgroup
  }
  const int D = p->g.dim;
  EDD_TRY_ALLOC(p->K0_d, double, 24 * 24);
  EDD_TRY_ALLOC(p->nmap_d, int, p->n_nodes);
  EDD_TRY_ALLOC(p->inode_d, int, std::max<int64_t>(1, p->n_inodes));
  EDD_TRY_ALLOC(p->gnode_d, int, std::max<int64_t>(1, p->n_gamma));
  EDD_TRY_ALLOC(p->subs_d, SubDesc, p->n_blk);
  EDD_TRY_ALLOC(p->order_d, int, p->n_blk);
  EDD_TRY_ALLOC(p->order_leaf_d, int, p->n_blk);
  EDD_TRY_ALLOC(p->order_sep_d, int, std::max(1, p->n_sep));
  EDD_TRY_ALLOC(p->info_d, int, p->n_blk);
  if (p->n_sep > 0) {
    EDD_TRY_ALLOC(p->seps_d, SepDesc, p->n_sep);
    EDD_TRY_ALLOC(p->W64_d, double, p->w_alloc);
    if (p->factor_precision & EDD_F32) EDD_TRY_ALLOC(p->W32_d, float, p->w_alloc);
  }
  EDD_TRY_ALLOC(p->E_d, double, p->n_el);
  {
    // band storage with padding on both sides (unconditional panel loads)
    const int64_t padded = kBandPadFront + p->fac_entries + band_pad_back(p->max_kd);
    double *f64 = nullptr, *r64 = nullptr;
    EDD_TRY_ALLOC(f64, double, padded);
    EDD_TRY_ALLOC(r64, double, padded);
    p->fac64_d = f64 + kBandPadFront;
    p->rac64_d = r64 + kBandPadFront;
    p->fac_padded = padded;
    if (p->factor_precision & EDD_F32) {
      float *f32 = nullptr, *r32 = nullptr;
      EDD_TRY_ALLOC(f32, float, padded);
      EDD_TRY_ALLOC(r32, float, padded);
      p->fac32_d = f32 + kBandPadFront;
      p->rac32_d = r32 + kBandPadFront;
    }
  }
  for (int i = 0; i < 3; ++i) EDD_TRY_ALLOC(p->w_I[i], double, std::max<int64_t>(1, p->n_idofs));
  for (int i = 0; i < 8; ++i) EDD_TRY_ALLOC(p->w_G[i], double, std::max<int64_t>(1, p->n_gamma * D));
  for (int i = 0; i < 2; ++i) EDD_TRY_ALLOC(p->w_full[i], double, p->ndof);
  p->partials_len = std::max(65536 + 8192, kWinChunks * kMaxWindow);
  EDD_TRY_ALLOC(p->partials_d, double, p->partials_len);
  EDD_TRY_ALLOC(p->scal_d, double, S_TOTAL);
  if (hipHostMalloc((void **)&p->scal_h, sizeof(double) * S_TOTAL) != hipSuccess) {
    p->scal_h = nullptr;
    edd_destroy(p);
    return EDD_ENOMEM;
  }
  std::memset(p->scal_h, 0, sizeof(double) * S_TOTAL);
  hipStream_t s = p->stream;
  hipError_t e = hipSuccess;
  auto up = [&](void *dst, const void *src, size_t bytes) {
    if (e == hipSuccess && bytes)
      e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  };
  up(p->K0_d, p->K0, sizeof(double) * 24 * 24);
  up(p->nmap_d, p->nmap_host.data(), sizeof(int) * p->n_nodes);
  up(p->inode_d, p->inode.data(), sizeof(int) * p->n_inodes);
  up(p->gnode_d, p->gnode.data(), sizeof(int) * p->n_gamma);
  up(p->subs_d, p->subs.data(), sizeof(SubDesc) * p->n_blk);
  up(p->order_d, p->order.data(), sizeof(int) * p->n_blk);
  up(p->order_leaf_d, p->order_leaf.data(), sizeof(int) * p->order_leaf.size());
  up(p->order_sep_d, p->order_sep.data(), sizeof(int) * p->order_sep.size());
  if (p->n_sep > 0) up(p->seps_d, p->seps.data(), sizeof(SepDesc) * p->n_sep);
  up(p->scal_d, p->scal_h, sizeof(double) * S_TOTAL);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) { edd_destroy(p); return EDD_EHIP; }
  launch_fill(p, p->ndof, 0.0, p->w_full[1]);
  // padding is read (and discarded) by the band kernels: keep it finite
  launch_fill(p, p->fac_padded, 0.0, p->fac64_d - kBandPadFront);
  launch_fill(p, p->fac_padded, 0.0, p->rac64_d - kBandPadFront);
  if (p->fac32_d) {
    launch_fill_f32(p, p->fac_padded, p->fac32_d - kBandPadFront);
    launch_fill_f32(p, p->fac_padded, p->rac32_d - kBandPadFront);
  }
  rc = precond_setup(p);
  if (rc) { edd_destroy(p); return rc; }
  rc = sync_check(p);
  if (rc) { edd_destroy(p); return rc; }
  *out = p;
  return EDD_OK;
}

int edd_set_element_moduli(edd_problem *p, const void *E_dev, int dtype) {
  if (!p || !E_dev || (dtype != EDD_F64 && dtype != EDD_F32)) return EDD_EINVAL;
  p->have_moduli = false;
  p->sc_ready = false;
  launch_convert_moduli(p, E_dev, dtype);
  launch_check_moduli(p, p->E_d, p->partials_d);
  launch_reduce(p, 256, 1, 1, S_BAD);
  int rc = read_scalars(p, S_BAD, 1);
  if (rc) return rc;
  if (p->scal_h[S_BAD] != 0.0) return EDD_EINVAL;
  launch_assemble_band(p);
  launch_band_cholesky(p);
  std::vector<int> info(p->n_blk, 0);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(info.data(), p->info_d, sizeof(int) * p->n_blk,
                       hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return check_hip(p, e);
  for (int v : info)
    if (v) return EDD_ENOTSPD;
  launch_band_layouts(p);
  rc = sync_check(p);
  if (rc) return rc;
  p->have_moduli = true;
  p->sk_state = -1;  // weighted interface operators must be rebuilt
  if (p->s_apply_mode == 1) {
    rc = schur_form(p);
    if (!rc) rc = sync_check(p);
    if (rc) return rc;
  }
  return EDD_OK;
}

int edd_apply_K(edd_problem *p, const double *u_dev, double *y_dev) {
  if (!p || !u_dev || !y_dev) return EDD_EINVAL;
  if (!p->have_moduli) return EDD_ESTATE;
  launch_apply_full(p, u_dev, y_dev);
  return check_hip(p, hipGetLastError());
}

int edd_solve_interior(edd_problem *p, const double *b_dev, double *x_dev,
                       int precision) {
  if (!p || !b_dev || !x_dev) return EDD_EINVAL;
  if (!p->have_moduli) return EDD_ESTATE;
  if (precision != EDD_F64 && precision != EDD_F32) return EDD_EINVAL;
  if (!(p->factor_precision & precision)) return EDD_ESTATE;
  launch_band_solve(p, precision, b_dev, x_dev);
  return check_hip(p, hipGetLastError());
}

int edd_apply_S(edd_problem *p, const double *v_dev, double *y_dev, int precision) {
  if (!p || !v_dev || !y_dev) return EDD_EINVAL;
  if (!p->have_moduli) return EDD_ESTATE;
  if (precision != EDD_F64 && precision != EDD_F32) return EDD_EINVAL;
  if (!(p->factor_precision & precision)) return EDD_ESTATE;
  apply_S(p, v_dev, y_dev, precision);
  return check_hip(p, hipGetLastError());
}

int edd_apply_precond(edd_problem *p, const double *r_dev, double *z_dev,
                      const edd_solve_opts *o) {
  if (!p || !r_dev || !z_dev || !o) return EDD_EINVAL;
  if (o->precond == EDD_PC_IDENTITY) {
    launch_copy(p, p->n_gamma * p->g.dim, r_dev, z_dev);
    return check_hip(p, hipGetLastError());
  }
  if (o->interface_weighting && !p->have_moduli) return EDD_ESTATE;
  if (o->lanczos_kmax < 1 || o->lanczos_kmax > 64 || o->inner_maxit < 1 ||
      o->pc_form < EDD_PCF_HTILDE_INV || o->pc_form > EDD_PCF_H_FWD ||
      (o->mass_matrix != 0 && o->mass_matrix != 1))
    return EDD_EINVAL;
  edd_solve_stats st{};
  int rc = precond_apply(p, r_dev, z_dev, o, &st, o->precision == EDD_MODE_MIXED);
  if (rc) return rc;
  return sync_check(p);
}

int edd_apply_skeleton_op(edd_problem *p, int which, int weighting,
                          const double *x_dev, double *y_dev, double tol, int maxit) {
  if (!p || !x_dev || !y_dev || which < 0 || which > 5) return EDD_EINVAL;
  if (weighting && !p->have_moduli) return EDD_ESTATE;
  if (which == 3 && (maxit < 1 || !(tol >= 0.0))) return EDD_EINVAL;
  int rc = skeleton_op(p, which, weighting, x_dev, y_dev, tol, maxit);
  if (rc) return rc;
  return sync_check(p);
}

int edd_get_info(edd_problem *p, edd_info *info) {
  if (!p || !info) return EDD_EINVAL;
  std::memset(info, 0, sizeof(*info));
  info->dim = p->g.dim;
  info->n_sub = p->n_sub;
  info->n_nodes = p->n_nodes;
  info->ndof = p->ndof;
  info->n_el = p->n_el;
  info->n_gamma = p->n_gamma;
  info->n_interior_dofs = p->n_idofs;
  info->factor_entries = p->fac_entries_real;
  info->max_band = p->max_kd;
  info->max_sub_dofs = p->max_n;
  info->skeleton_faces = p->n_faces;
  info->face_classes = p->n_face_classes;
  info->theta_default = p->theta_default;
  info->band_blocks = p->n_blk;
  info->coupling_entries = p->w_entries;
  return EDD_OK;
}

int edd_set_kernel_timing(edd_problem *p, int enable) {
  if (!p) return EDD_EINVAL;
  kt_resolve(p);
  p->kt_enabled = enable != 0;
  for (int k = 0; k < EDD_KT_COUNT; ++k) {
    p->kt_count[k] = 0;
    p->kt_ms[k] = 0.0;
  }
  return EDD_OK;
}

int edd_get_kernel_times(edd_problem *p, edd_kernel_times *t) {
  if (!p || !t) return EDD_EINVAL;
  kt_resolve(p);
  for (int k = 0; k < EDD_KT_COUNT; ++k) {
    t->count[k] = p->kt_count[k];
    t->total_ms[k] = p->kt_ms[k];
  }
  return EDD_OK;
}

int edd_get_gamma_nodes(edd_problem *p, int32_t *nodes_host) {
  if (!p || !nodes_host) return EDD_EINVAL;
  std::memcpy(nodes_host, p->gnode.data(), sizeof(int32_t) * p->n_gamma);
  return EDD_OK;
}

int edd_get_interior_nodes(edd_problem *p, int32_t *nodes_host) {
  if (!p || !nodes_host) return EDD_EINVAL;
  std::memcpy(nodes_host, p->inode.data(), sizeof(int32_t) * p->n_inodes);
  return EDD_OK;
}

// Autotuner cache: in memory for the process, and in a text file when one is
// set (edd_autotune_cache): one line per tuned (kernel family, shape class),
//   <family> <key> <value> [<value>]
// with family band_solve (FP64 and FP32 substitution variants), apply_K
// (node-tile shape) or s_apply (0 through the factors, 1 explicit local
// Schur complements), key = architecture|shape class.
namespace {
std::mutex g_tune_mu;
std::map<std::string, std::vector<int>> g_tune;
std::string g_tune_path;

void tune_load_locked() {
  g_tune.clear();
  if (g_tune_path.empty()) return;
  FILE *fh = std::fopen(g_tune_path.c_str(), "r");
  if (!fh) return;
  char line[1024];
  while (std::fgets(line, sizeof line, fh)) {
    char fam[64], key[768];
    int v[3] = {0, 0, 0};
    const int n = std::sscanf(line, "%63s %767s %d %d %d", fam, key, &v[0], &v[1], &v[2]);
    if (n >= 3) g_tune[std::string(fam) + " " + key] = std::vector<int>(v, v + (n - 2));
  }
  std::fclose(fh);
}

void tune_save_locked() {
  if (g_tune_path.empty()) return;
  const std::string tmp = g_tune_path + ".tmp";
  FILE *fh = std::fopen(tmp.c_str(), "w");
  if (!fh) return;
  for (const auto &kv : g_tune) {
    std::fprintf(fh, "%s", kv.first.c_str());
    for (int v : kv.second) std::fprintf(fh, " %d", v);
    std::fprintf(fh, "\n");
  }
  std::fclose(fh);
  std::rename(tmp.c_str(), g_tune_path.c_str());
}
}  // namespace

int edd_autotune_cache(const char *path) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_path = path ? path : "";
  tune_load_locked();
  return EDD_OK;
}

int edd_autotune(edd_problem *p, int force, int *variants) {
  if (!p) return EDD_EINVAL;
  if (!p->have_moduli) return EDD_ESTATE;
  hipDeviceProp_t prop;
  int rc = check_hip(p, hipGetDeviceProperties(&prop, p->device));
  if (rc) return rc;
  // shape classes: the substitution's by band extents and factor
  // precisions, the element kernel's by dimension and node grid
  const std::string arch = prop.gcnArchName;
  const std::string kb = "band_solve " + arch + "|" + std::to_string(p->g.dim) + "|" +
                         std::to_string(p->n_blk) + "|" + std::to_string(p->max_kd) + "|" +
                         std::to_string(p->max_np) + "|" + std::to_string(p->fac_entries) + "|" +
                         std::to_string(p->factor_precision);
  const std::string ka = "apply_K " + arch + "|" + std::to_string(p->g.dim) + "|" +
                         std::to_string(p->g.nn[0]) + "x" + std::to_string(p->g.nn[1]) + "x" +
                         std::to_string(p->g.nn[2]);
  bool need_band = true, need_apply = true;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(kb);
    if (!force && it != g_tune.end() && it->second.size() == 2 &&
        band_solve_variant_ok(p, it->second[0]) && band_solve_variant_ok(p, it->second[1])) {
      p->solve_variant[0] = it->second[0];
      p->solve_variant[1] = it->second[1];
      need_band = false;
    }
    auto ia = g_tune.find(ka);
    if (!force && ia != g_tune.end() && ia->second.size() == 3) {
      bool ok = true;
      for (int t = 0; t < 3; ++t) ok = ok && ia->second[t] >= 0 && ia->second[t] < kApplyVariants;
      if (ok) {
        for (int t = 0; t < 3; ++t) p->apply_variant[t] = ia->second[t];
        need_apply = false;
      }
    }
  }
  if (need_band || need_apply) {
    hipEvent_t e0, e1;
    rc = check_hip(p, hipEventCreate(&e0));
    if (rc) return rc;
    rc = check_hip(p, hipEventCreate(&e1));
    if (rc) return rc;
    auto time_it = [&](auto &&launch, int reps, float *ms) {
      launch();  // warm-up (first-launch costs)
      hipEventRecord(e0, p->stream);
      for (int r = 0; r < reps; ++r) launch();
      hipEventRecord(e1, p->stream);
      int c = check_hip(p, hipEventSynchronize(e1));
      if (!c) c = check_hip(p, hipEventElapsedTime(ms, e0, e1));
      return c;
    };
    const bool kt = p->kt_enabled;
    p->kt_enabled = false;
    if (need_band) {
      double *b = p->w_I[0], *x = p->w_I[1];
      launch_fill(p, p->n_idofs, 1.0, b);
      for (int f = 0; f < 2 && rc == 0; ++f) {
        const int prec = f ? EDD_F32 : EDD_F64;
        if (f && !p->fac32_d) break;
        int best = 0;
        float best_ms = 0.0f;
        for (int v = 1; v <= kBandSolveVariants && rc == 0; ++v) {
          if (!band_solve_variant_ok(p, v)) continue;
          p->solve_variant[f] = v;
          float ms = 0.0f;
          rc = time_it([&] { launch_band_solve(p, prec, b, x); }, 3, &ms);
          if (!rc && (best == 0 || ms < best_ms)) {
            best = v;
            best_ms = ms;
          }
        }
        p->solve_variant[f] = best;
      }
    }
    if (need_apply && rc == 0) {
      // timed on a vector of ones into a buffer of its own (allocated once)
      double *u = p->w_full[0];
      if (!p->tune_y_d) p->tune_y_d = (double *)dev_alloc(p, sizeof(double) * p->ndof);
      double *y = p->tune_y_d;
      if (!y) rc = EDD_ENOMEM;
      if (!rc) launch_fill(p, p->ndof, 1.0, u);
      // each kind of target on its own: all nodes, interior nodes (packed
      // interior output), interface nodes (packed interface output)
      double *oI = p->w_I[0], *oG = p->w_G[0];
      for (int t = 0; t < 3 && rc == 0; ++t) {
        int best = 0;
        float best_ms = 0.0f;
        for (int v = 0; v < kApplyVariants && rc == 0; ++v) {
          p->apply_variant[t] = v;
          float ms = 0.0f;
          if (t == 0)
            rc = time_it([&] { launch_apply_full(p, u, y); }, 5, &ms);
          else if (t == 1)
            rc = time_it([&] { launch_apply_mapped(p, p->inode_d, p->n_inodes, nullptr, 0.0, y,
                                                   1.0, nullptr, 1.0, oI); }, 5, &ms);
          else
            rc = time_it([&] { launch_apply_mapped(p, p->gnode_d, p->n_gamma, y, 1.0, nullptr,
                                                   0.0, u, -1.0, oG); }, 5, &ms);
          if (!rc && (v == 0 || ms < best_ms)) {
            best = v;
            best_ms = ms;
          }
        }
        p->apply_variant[t] = best;
      }
      launch_fill(p, p->ndof, 0.0, u);
    }
    p->kt_enabled = kt;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (need_band) g_tune[kb] = {p->solve_variant[0], p->solve_variant[1]};
    if (need_apply) g_tune[ka] = {p->apply_variant[0], p->apply_variant[1], p->apply_variant[2]};
    tune_save_locked();
  }
  // the S apply: through the interior factors or by explicit local Schur
  // complements (where the problem allows them); cached per shape class
  {
    const std::string ks = "s_apply " + arch + "|" + std::to_string(p->g.dim) + "|" +
                           std::to_string(p->g.nn[0]) + "x" + std::to_string(p->g.nn[1]) + "x" +
                           std::to_string(p->g.nn[2]) + "|" + std::to_string(p->n_sub) + "|" +
                           std::to_string(p->factor_precision);
    int cached = -1;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune.find(ks);
      if (!force && it != g_tune.end() && it->second.size() == 1) cached = it->second[0];
    }
    if (cached >= 0) {
      rc = edd_set_s_apply(p, cached);
      if (rc == EDD_EINVAL && cached == 1) rc = edd_set_s_apply(p, 0);
      if (rc) return rc;
    } else {
      int best = 0;
      if (schur_setup(p) == EDD_OK) {
        hipEvent_t e0, e1;
        rc = check_hip(p, hipEventCreate(&e0));
        if (rc) return rc;
        rc = check_hip(p, hipEventCreate(&e1));
        if (rc) return rc;
        const int64_t nG = p->n_gamma * p->g.dim;
        double *v = p->w_G[6], *y = p->w_G[7];
        launch_fill(p, nG, 1.0, v);
        const bool kt = p->kt_enabled;
        p->kt_enabled = false;
        float ms[2] = {0.0f, 0.0f};
        for (int mode = 0; mode < 2 && rc == 0; ++mode) {
          rc = edd_set_s_apply(p, mode);
          if (rc) break;
          apply_S(p, v, y, EDD_F64);  // warm-up
          hipEventRecord(e0, p->stream);
          for (int r = 0; r < 5; ++r) apply_S(p, v, y, EDD_F64);
          hipEventRecord(e1, p->stream);
          rc = check_hip(p, hipEventSynchronize(e1));
          if (!rc) rc = check_hip(p, hipEventElapsedTime(&ms[mode], e0, e1));
        }
        p->kt_enabled = kt;
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        if (rc) return rc;
        best = ms[1] < ms[0] ? 1 : 0;
      }
      rc = edd_set_s_apply(p, best);
      if (rc) return rc;
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune[ks] = {best};
      tune_save_locked();
    }
  }
  if (variants) {
    variants[0] = p->solve_variant[0];
    variants[1] = p->solve_variant[1];
    variants[2] = p->apply_variant[0];
    variants[3] = p->apply_variant[1];
    variants[4] = p->apply_variant[2];
  }
  return EDD_OK;
}

int edd_set_apply_variant(edd_problem *p, int variant) {
  if (!p || variant < 0 || variant >= kApplyVariants) return EDD_EINVAL;
  for (int t = 0; t < 3; ++t) p->apply_variant[t] = variant;
  return EDD_OK;
}

int edd_set_solve_variants(edd_problem *p, const int *variants) {
  if (!p || !variants) return EDD_EINVAL;
  for (int f = 0; f < 2; ++f)
    if (!band_solve_variant_ok(p, variants[f])) return EDD_EINVAL;
  p->solve_variant[0] = variants[0];
  p->solve_variant[1] = variants[1];
  return EDD_OK;
}

int edd_solve_batch(edd_problem *const *ps, int n, const double *const *f_dev,
                    double *const *u_dev, const edd_solve_opts *o,
                    edd_solve_stats *stats, int nthreads) {
  if (n < 0 || (n > 0 && (!ps || !f_dev || !u_dev))) return EDD_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!ps[i] || !f_dev[i] || !u_dev[i]) return EDD_EINVAL;
    for (int j = 0; j < i; ++j)
      if (ps[j] == ps[i]) return EDD_EINVAL;  // one solve per handle at a time
  }
  if (n == 0) return EDD_OK;
  int nt = nthreads > 0 ? nthreads : 16;
  if (nt > n) nt = n;
  std::vector<int> rcs(n, EDD_OK);
  std::vector<edd_solve_stats> st(n);
  // largest problems first, so the longest solves are not started last
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return ps[a]->ndof * ps[a]->g.dim > ps[b]->ndof * ps[b]->g.dim;
  });
  std::atomic<int> next{0};
  auto work = [&] {
    for (;;) {
      const int t = next.fetch_add(1);
      if (t >= n) break;
      const int i = order[t];
      if (hipSetDevice(ps[i]->device) != hipSuccess) {
        rcs[i] = EDD_EHIP;
        continue;
      }
      rcs[i] = edd_solve_interface(ps[i], f_dev[i], u_dev[i], o, &st[i]);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(work);
  work();
  for (auto &t : pool) t.join();
  if (stats)
    for (int i = 0; i < n; ++i) stats[i] = st[i];
  int worst = EDD_OK;
  for (int i = 0; i < n; ++i) {
    if (rcs[i] < 0) return rcs[i];
    if (rcs[i] == EDD_NOT_CONVERGED) worst = EDD_NOT_CONVERGED;
  }
  return worst;
}

int edd_cnn_setup(edd_problem *p, int width) {
  if (!p) return EDD_EINVAL;
  int rc = cnn_setup(p, width);
  if (rc) return rc;
  if (!p->cnn_r_d) {
    p->cnn_r_d = (double *)dev_alloc(p, sizeof(double) * p->ndof);
    p->cnn_dir_d = (double *)dev_alloc(p, sizeof(double) * p->ndof);
    if (!p->cnn_r_d || !p->cnn_dir_d) return EDD_ENOMEM;
  }
  return EDD_OK;
}

int edd_cnn_matrix_cores(edd_problem *p, int enable) {
  if (!p) return EDD_EINVAL;
  if (!p->cnn_nparams) return EDD_ESTATE;
  p->cnn_matrix_cores = enable ? 1 : 0;
  return EDD_OK;
}

int edd_cnn_num_params(edd_problem *p, int64_t *n) {
  if (!p || !n) return EDD_EINVAL;
  if (!p->cnn_nparams) return EDD_ESTATE;
  *n = p->cnn_nparams;
  return EDD_OK;
}

int edd_cnn_set_params(edd_problem *p, const float *params_dev) {
  if (!p || !params_dev) return EDD_EINVAL;
  if (!p->cnn_nparams) return EDD_ESTATE;
  return cnn_set_params(p, params_dev);
}

int edd_cnn_get_params(edd_problem *p, float *params_dev) {
  if (!p || !params_dev) return EDD_EINVAL;
  if (!p->cnn_nparams) return EDD_ESTATE;
  return cnn_get_params(p, params_dev);
}

int edd_cnn_predict(edd_problem *p, const double *E_dev, const double *r_dev, double *d_dev) {
  if (!p || !r_dev || !d_dev) return EDD_EINVAL;
  if (!p->cnn_nparams || (!E_dev && !p->have_moduli)) return EDD_ESTATE;
  return cnn_predict(p, E_dev, r_dev, d_dev);
}

int edd_cnn_loss_grad(edd_problem *p, const double *E_dev, const double *r_dev,
                      const double *e_dev, float *grad_dev, double *loss) {
  if (!p || !r_dev || !e_dev || !loss) return EDD_EINVAL;
  if (!p->cnn_nparams || (!E_dev && !p->have_moduli)) return EDD_ESTATE;
  return cnn_loss_grad(p, E_dev, r_dev, e_dev, grad_dev, loss);
}

int edd_cnn_training_pair(edd_problem *p, const double *f_dev, const double *u_prev_dev,
                          const double *u_dev, double *r_dev, double *e_dev) {
  if (!p || !f_dev || !u_prev_dev || !u_dev || !r_dev || !e_dev) return EDD_EINVAL;
  if (!p->have_moduli) return EDD_ESTATE;
  if (r_dev == u_prev_dev || e_dev == u_prev_dev || e_dev == u_dev || r_dev == e_dev)
    return EDD_EINVAL;
  // r = f - K u_prev, zero on clamped dofs
  launch_apply_full(p, u_prev_dev, r_dev);
  launch_axpby(p, p->ndof, 1.0, f_dev, -1.0, r_dev);
  launch_mask_dirichlet(p, r_dev);
  // e = u - u_prev
  launch_copy(p, p->ndof, u_dev, e_dev);
  launch_axpby(p, p->ndof, -1.0, u_prev_dev, 1.0, e_dev);
  return check_hip(p, hipGetLastError());
}

int edd_cnn_train_step(edd_problem *p, const double *E_dev, const double *r_dev,
                       const double *e_dev, double lr, double *loss) {
  if (!p || !r_dev || !e_dev || !loss || !(lr > 0.0)) return EDD_EINVAL;
  if (!p->cnn_nparams || (!E_dev && !p->have_moduli)) return EDD_ESTATE;
  return cnn_train_step(p, E_dev, r_dev, e_dev, lr, loss);
}

int edd_solve_interface(edd_problem *p, const double *f_dev, double *u_dev,
                        const edd_solve_opts *o_in, edd_solve_stats *s_out) {
  if (!p || !f_dev || !u_dev) return EDD_EINVAL;
  if (!p->have_moduli) return EDD_ESTATE;
  edd_solve_opts o;
  if (o_in) o = *o_in;
  else edd_default_opts(&o);
  if (!(o.tol > 0.0) || o.maxit < 1 || o.outer_maxit < 0) return EDD_EINVAL;
  if (o.precond != EDD_PC_IDENTITY && o.precond != EDD_PC_HTHETA) return EDD_EINVAL;
  if (o.precond == EDD_PC_HTHETA &&
      (o.lanczos_kmax < 1 || o.lanczos_kmax > 64 || o.inner_maxit < 1 || o.theta > 1.0 ||
       o.pc_form < EDD_PCF_HTILDE_INV || o.pc_form > EDD_PCF_H_FWD ||
       (o.mass_matrix != 0 && o.mass_matrix != 1)))
    return EDD_EINVAL;
  if (o.precision != EDD_MODE_F64 && o.precision != EDD_MODE_MIXED &&
      o.precision != EDD_MODE_RELAXED)
    return EDD_EINVAL;
  if (o.precision != EDD_MODE_F64 && !(p->factor_precision & EDD_F32)) return EDD_ESTATE;
  if (!(p->factor_precision & EDD_F64)) return EDD_ESTATE;
  edd_solve_stats st{};
  const auto t0 = std::chrono::steady_clock::now();
  double nf = 0.0;
  int rc = norm_f(p, f_dev, &nf);
  if (rc) return rc;
  if (!std::isfinite(nf)) return EDD_EINVAL;
  int status = EDD_OK;
  if (o.learned_correction < 0) return EDD_EINVAL;
  if (o.learned_correction > 0 && !p->cnn_nparams) return EDD_ESTATE;
  if (o.learned_guess && nf > 0.0) {
    if (!p->cnn_nparams) return EDD_ESTATE;
    rc = learned_guess(p, f_dev, u_dev, &o, &st);
    if (rc) return rc;
    o.use_initial_guess = 1;
  }
  if (nf == 0.0) {
    launch_fill(p, p->ndof, 0.0, u_dev);
  } else if (o.precision == EDD_MODE_F64) {
    status = solve_plain(p, f_dev, u_dev, &o, &st, nf);
  } else if (o.precision == EDD_MODE_MIXED) {
    status = solve_mixed(p, f_dev, u_dev, &o, &st, nf);
  } else {
    status = solve_relaxed(p, f_dev, u_dev, &o, &st, nf);
  }
  if (status >= 0) {
    const double *a[1] = {f_dev}, *b[1] = {u_dev};
    launch_dots(p, p->ndof, 1, a, b, S_CMP);
    rc = read_scalars(p, S_CMP, 1);
    if (rc) return rc;
    st.compliance = p->scal_h[S_CMP];
  }
  const auto t1 = std::chrono::steady_clock::now();
  st.t_total_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  st.status = status;
  if (s_out) *s_out = st;
  return status;
}

}  // extern "C"

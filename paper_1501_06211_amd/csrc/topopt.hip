// Topology optimisation on the solver (Section 5): element energies, the
// Optimality Criteria density update with its volume multiplier found on the
// device, and the fixed-point loop FEA -> OC update -> convergence check with
// a Krylov tolerance that follows successive compliance values.
//
// The problem of eq. (NumberTen) is min f^T u subject to K(rho) u = f,
// K(rho) = sum_i E(rho_i) K0_i, sum_i rho_i <= V and box bounds on rho; with
// E(rho) = rho it is the Variable Thickness Sheet problem of the paper.
//
// OC update (textbook form for a compliance objective), per element:
//   g_e = E'(rho_e) u_e^T K0 u_e                (= -dc/drho_e)
//   rho_e(Lambda) = clamp(rho_e (g_e / Lambda)^eta,
//                         max(lo, rho_e - move), min(hi, rho_e + move))
// with Lambda the multiplier that makes sum_e rho_e(Lambda) = V.  The volume
// is monotone in Lambda; the multiplier is bracketed from the bounds, then
// each pass evaluates the volume at 64 log-spaced candidates inside the
// bracket at once (one accumulator per candidate in every thread) and keeps
// the sub-interval where it crosses V: seven passes narrow log(Lambda) to
// about 1e-12 of the bracket, with seven short host reads instead of the
// forty-odd of a plain bisection.  All reductions are two-stage with a fixed
// order, so results are bitwise reproducible.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace edd {
namespace {

constexpr int kTB = 256;        // threads per block
constexpr int kCand = 64;       // candidates per multisection pass
constexpr int kOcBlocks = 256;  // blocks of the OC reductions
constexpr int kOcPasses = 7;

struct OcDev {
  double lo, hi, move, eta, penal, emin;
};

__device__ inline double dE_drho(double rho, const OcDev &q) {
  if (q.penal == 1.0) return 1.0 - q.emin;
  return q.penal * pow(rho, q.penal - 1.0) * (1.0 - q.emin);
}

__device__ inline double modulus(double rho, const OcDev &q) {
  if (q.penal == 1.0 && q.emin == 0.0) return rho;
  return q.emin + (q.penal == 1.0 ? rho : pow(rho, q.penal)) * (1.0 - q.emin);
}

// s_e = u_e^T K0 u_e, one thread per element; clamped dofs read as zero.
// K0 entries are the same for every lane, so they come through the scalar
// cache.
template <int D>
__global__ __launch_bounds__(kTB) void k_element_energy(Geom g, const double *__restrict__ K0,
                                                        const int *__restrict__ nmap,
                                                        const double *__restrict__ u,
                                                        double *__restrict__ s, int64_t nel) {
  constexpr int NC = D == 2 ? 4 : 8;
  constexpr int ND = D * NC;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nel) return;
  const int ex = (int)(e % g.nel[0]);
  const int ey = (int)((e / g.nel[0]) % g.nel[1]);
  const int ez = D == 3 ? (int)(e / ((int64_t)g.nel[0] * g.nel[1])) : 0;
  double ue[ND];
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    const int ox = (a & 3) == 1 || (a & 3) == 2, oy = (a & 3) >= 2, oz = a >= 4;
    const int node = (ex + ox) + g.nn[0] * ((ey + oy) + g.nn[1] * (ez + oz));
    const bool clamped = nmap[node] == kDirichlet;
#pragma unroll
    for (int c = 0; c < D; ++c) ue[D * a + c] = clamped ? 0.0 : u[(int64_t)D * node + c];
  }
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    double row = 0.0;
#pragma unroll
    for (int j = 0; j < ND; ++j) row = fma(K0[i * ND + j], ue[j], row);
    acc = fma(ue[i], row, acc);
  }
  s[e] = acc;
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}
__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  return v;
}
__device__ inline double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_down(v, o, 64));
  return v;
}

// Pass 0: sum of the lower and upper bounds, and the multipliers beyond which
// every element with g > 0 sits on its lower (max of g (rho/lower)^(1/eta))
// or upper (min of g (rho/upper)^(1/eta)) bound.  out[block][4].
__global__ __launch_bounds__(kTB) void k_oc_bounds(int64_t n, const double *__restrict__ rho,
                                                   const double *__restrict__ s, OcDev q,
                                                   double *__restrict__ out) {
  __shared__ double red[4][kTB / 64];
  double slo = 0.0, shi = 0.0, lmax = 0.0, lmin = INFINITY;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double r = rho[e];
    const double lower = fmax(q.lo, r - q.move), upper = fmin(q.hi, r + q.move);
    slo += lower;
    shi += upper;
    const double ge = dE_drho(r, q) * s[e];
    if (ge > 0.0) {
      lmax = fmax(lmax, ge * pow(r / lower, 1.0 / q.eta));
      lmin = fmin(lmin, ge * pow(r / upper, 1.0 / q.eta));
    }
  }
  slo = wave_sum(slo);
  shi = wave_sum(shi);
  lmax = wave_max(lmax);
  lmin = wave_min(lmin);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = slo;
    red[1][w] = shi;
    red[2][w] = lmax;
    red[3][w] = lmin;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0, c = 0.0, d = INFINITY;
    for (int k = 0; k < kTB / 64; ++k) {
      a += red[0][k];
      b += red[1][k];
      c = fmax(c, red[2][k]);
      d = fmin(d, red[3][k]);
    }
    out[4 * blockIdx.x + 0] = a;
    out[4 * blockIdx.x + 1] = b;
    out[4 * blockIdx.x + 2] = c;
    out[4 * blockIdx.x + 3] = d;
  }
}

// Second stage of k_oc_bounds: one block, out4 = (sum, sum, max, min).
__global__ __launch_bounds__(kTB) void k_oc_bounds_final(int nblocks,
                                                         const double *__restrict__ part,
                                                         double *__restrict__ out4) {
  __shared__ double red[4][kTB / 64];
  double a = 0.0, b = 0.0, c = 0.0, d = INFINITY;
  for (int k = threadIdx.x; k < nblocks; k += blockDim.x) {
    a += part[4 * k + 0];
    b += part[4 * k + 1];
    c = fmax(c, part[4 * k + 2]);
    d = fmin(d, part[4 * k + 3]);
  }
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_max(c);
  d = wave_min(d);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = a;
    red[1][w] = b;
    red[2][w] = c;
    red[3][w] = d;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double A = 0.0, B = 0.0, C = 0.0, Dm = INFINITY;
    for (int k = 0; k < kTB / 64; ++k) {
      A += red[0][k];
      B += red[1][k];
      C = fmax(C, red[2][k]);
      Dm = fmin(Dm, red[3][k]);
    }
    out4[0] = A;
    out4[1] = B;
    out4[2] = C;
    out4[3] = Dm;
  }
}

// Volume at the kCand multipliers exp(la + (j+1) (lb-la)/(kCand+1)): every
// thread keeps one accumulator per candidate; rho (g/Lambda)^eta is
// t_e * c_j with t_e = rho g^eta and c_j = Lambda_j^-eta.  out[block][kCand].
__global__ __launch_bounds__(kTB) void k_oc_volumes(int64_t n, const double *__restrict__ rho,
                                                    const double *__restrict__ s, OcDev q,
                                                    double la, double lb,
                                                    double *__restrict__ out) {
  __shared__ double red[kTB / 64][kCand];
  __shared__ double cj[kCand];
  const double step = (lb - la) / (kCand + 1);
  if (threadIdx.x < kCand) cj[threadIdx.x] = exp(-q.eta * (la + (threadIdx.x + 1) * step));
  __syncthreads();
  double acc[kCand];
#pragma unroll
  for (int j = 0; j < kCand; ++j) acc[j] = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double r = rho[e];
    const double lower = fmax(q.lo, r - q.move), upper = fmin(q.hi, r + q.move);
    const double ge = dE_drho(r, q) * s[e];
    const double t = r * pow(ge, q.eta);
#pragma unroll
    for (int j = 0; j < kCand; ++j) acc[j] += fmin(upper, fmax(lower, t * cj[j]));
  }
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kCand; ++j) {
    const double v = wave_sum(acc[j]);
    if ((threadIdx.x & 63) == 0) red[w][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < kCand) {
    double v = 0.0;
    for (int k = 0; k < kTB / 64; ++k) v += red[k][threadIdx.x];
    out[(int64_t)blockIdx.x * kCand + threadIdx.x] = v;
  }
}

// Sum over blocks of out[block][kCand] (one thread per candidate, fixed
// order over blocks).
__global__ __launch_bounds__(kCand) void k_oc_volumes_final(int nblocks,
                                                            const double *__restrict__ part,
                                                            double *__restrict__ vol) {
  const int j = threadIdx.x;
  double v = 0.0;
  for (int b = 0; b < nblocks; ++b) v += part[(int64_t)b * kCand + j];
  vol[j] = v;
}

// The update at the chosen multiplier; per block: sum of rho_new and max
// |rho_new - rho|.  A non-finite lambda selects the lower bounds (the
// constraint cannot be met from above), lambda 0 the upper bounds.
__global__ __launch_bounds__(kTB) void k_oc_apply(int64_t n, const double *__restrict__ rho,
                                                  const double *__restrict__ s, OcDev q,
                                                  double lam, double *__restrict__ rho_new,
                                                  double *__restrict__ E_new,
                                                  double *__restrict__ out) {
  __shared__ double red[2][kTB / 64];
  double vol = 0.0, chg = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double r = rho[e];
    const double lower = fmax(q.lo, r - q.move), upper = fmin(q.hi, r + q.move);
    double v;
    if (lam == 0.0) v = upper;
    else if (!(lam <= 1.7e308)) v = lower;
    else v = fmin(upper, fmax(lower, r * pow(dE_drho(r, q) * s[e] / lam, q.eta)));
    rho_new[e] = v;
    if (E_new) E_new[e] = modulus(v, q);
    vol += v;
    chg = fmax(chg, fabs(v - r));
  }
  vol = wave_sum(vol);
  chg = wave_max(chg);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = vol;
    red[1][w] = chg;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < kTB / 64; ++k) {
      a += red[0][k];
      b = fmax(b, red[1][k]);
    }
    out[2 * blockIdx.x + 0] = a;
    out[2 * blockIdx.x + 1] = b;
  }
}

__global__ __launch_bounds__(kTB) void k_oc_apply_final(int nblocks,
                                                        const double *__restrict__ part,
                                                        double *__restrict__ out2) {
  __shared__ double red[2][kTB / 64];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nblocks; k += blockDim.x) {
    a += part[2 * k + 0];
    b = fmax(b, part[2 * k + 1]);
  }
  a = wave_sum(a);
  b = wave_max(b);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = a;
    red[1][w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double A = 0.0, B = 0.0;
    for (int k = 0; k < kTB / 64; ++k) {
      A += red[0][k];
      B = fmax(B, red[1][k]);
    }
    out2[0] = A;
    out2[1] = B;
  }
}

__global__ __launch_bounds__(kTB) void k_rho_to_moduli(int64_t n, const double *__restrict__ rho,
                                                       OcDev q, double *__restrict__ E) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < n) E[e] = modulus(rho[e], q);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kTB - 1) / kTB); }

OcDev to_dev(const edd_oc_params &o) {
  return OcDev{o.rho_min, o.rho_max, o.move, o.eta, o.penal, o.emin};
}

int check_oc(const edd_oc_params *o) {
  if (!o) return EDD_EINVAL;
  if (!(o->rho_min > 0.0) || !(o->rho_max >= o->rho_min) || !(o->move > 0.0) ||
      !(o->eta > 0.0) || !(o->penal >= 1.0) || !(o->emin >= 0.0 && o->emin < 1.0) ||
      !(o->volume > 0.0))
    return EDD_EINVAL;
  return EDD_OK;
}

// scratch slots for the OC host reads, placed after the solver's scalar slots
constexpr int kScalOc = 1536;

}  // namespace

int element_energies(edd_problem *p, const double *u, double *s) {
  const unsigned b = blocks_for(p->n_el);
  if (p->g.dim == 2)
    k_element_energy<2><<<b, kTB, 0, p->stream>>>(p->g, p->K0_d, p->nmap_d, u, s, p->n_el);
  else
    k_element_energy<3><<<b, kTB, 0, p->stream>>>(p->g, p->K0_d, p->nmap_d, u, s, p->n_el);
  return check_hip(p, hipGetLastError());
}

int oc_update(edd_problem *p, const double *rho, const double *s, const edd_oc_params &o,
              double *rho_new, double *E_new, edd_oc_result *res) {
  const OcDev q = to_dev(o);
  const int64_t n = p->n_el;
  const unsigned nb = std::min<unsigned>(kOcBlocks, blocks_for(n));
  double *part = p->partials_d;  // nb * kCand doubles at most (16384 < partials_len)
  double *sc = p->scal_d + kScalOc;
  k_oc_bounds<<<nb, kTB, 0, p->stream>>>(n, rho, s, q, part);
  k_oc_bounds_final<<<1, kTB, 0, p->stream>>>((int)nb, part, sc);
  int rc = read_scalars(p, kScalOc, 4);
  if (rc) return rc;
  const double slo = p->scal_h[kScalOc], shi = p->scal_h[kScalOc + 1];
  const double lmax = p->scal_h[kScalOc + 2], lmin = p->scal_h[kScalOc + 3];
  double lam;
  if (shi <= o.volume || !(lmax > 0.0)) {
    lam = 0.0;  // every element at its upper bound still meets the volume
  } else if (slo >= o.volume) {
    lam = INFINITY;  // even the lower bounds exceed it
  } else {
    double la = std::log(lmin) - std::log(2.0), lb = std::log(lmax) + std::log(2.0);
    for (int pass = 0; pass < kOcPasses; ++pass) {
      k_oc_volumes<<<nb, kTB, 0, p->stream>>>(n, rho, s, q, la, lb, part);
      k_oc_volumes_final<<<1, kCand, 0, p->stream>>>((int)nb, part, sc);
      rc = read_scalars(p, kScalOc, kCand);
      if (rc) return rc;
      // the volume falls as Lambda grows: keep the cell where it crosses V
      const double step = (lb - la) / (kCand + 1);
      int j = 0;
      while (j < kCand && p->scal_h[kScalOc + j] > o.volume) ++j;
      const double na = la + j * step, nbd = la + (j + 1) * step;
      la = na;
      lb = nbd;
    }
    lam = std::exp(0.5 * (la + lb));
  }
  k_oc_apply<<<nb, kTB, 0, p->stream>>>(n, rho, s, q, lam, rho_new, E_new, part);
  k_oc_apply_final<<<1, kTB, 0, p->stream>>>((int)nb, part, sc);
  rc = read_scalars(p, kScalOc, 2);
  if (rc) return rc;
  if (res) {
    res->lambda = lam;
    res->volume = p->scal_h[kScalOc];
    res->max_change = p->scal_h[kScalOc + 1];
  }
  return EDD_OK;
}

}  // namespace edd

using namespace edd;

static int ensure_to_buffers(edd_problem *p) {
  if (p->to_s_d) return EDD_OK;
  p->to_s_d = (double *)dev_alloc(p, sizeof(double) * p->n_el);
  p->to_E_d = (double *)dev_alloc(p, sizeof(double) * p->n_el);
  p->to_rho_d = (double *)dev_alloc(p, sizeof(double) * p->n_el);
  if (!p->to_s_d || !p->to_E_d || !p->to_rho_d) return EDD_ENOMEM;
  return EDD_OK;
}

extern "C" {

void edd_default_topopt_opts(edd_topopt_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->volfrac = 0.5;
  o->rho_min = 1e-3;
  o->rho_max = 1.0;
  o->move = 0.2;
  o->eta = 0.5;
  o->penal = 1.0;
  o->emin = 0.0;
  o->change_tol = 1e-2;
  o->maxit = 100;
  o->adaptive_tol = 1;
  o->tol_min = 1e-8;
  o->tol_max = 1e-2;
  o->warm_start = 1;
}

int edd_element_energies(edd_problem *p, const double *u_dev, double *s_dev) {
  if (!p || !u_dev || !s_dev) return EDD_EINVAL;
  return element_energies(p, u_dev, s_dev);
}

int edd_oc_update(edd_problem *p, const double *rho_dev, const double *s_dev,
                  const edd_oc_params *o, double *rho_new_dev, double *E_new_dev,
                  edd_oc_result *res) {
  if (!p || !rho_dev || !s_dev || !rho_new_dev) return EDD_EINVAL;
  if (rho_new_dev == rho_dev || rho_new_dev == s_dev) return EDD_EINVAL;
  int rc = check_oc(o);
  if (rc) return rc;
  rc = oc_update(p, rho_dev, s_dev, *o, rho_new_dev, E_new_dev, res);
  if (rc) return rc;
  return check_hip(p, hipStreamSynchronize(p->stream));
}

int edd_topopt_run(edd_problem *p, const double *f_dev, double *rho_dev, double *u_dev,
                   const edd_topopt_opts *to, const edd_solve_opts *so,
                   edd_topopt_stats *st, double *history_host) {
  if (!p || !f_dev || !rho_dev || !u_dev || !to) return EDD_EINVAL;
  if (!(to->volfrac > 0.0) || to->maxit < 1 || !(to->change_tol >= 0.0) ||
      !(to->tol_min > 0.0) || !(to->tol_max >= to->tol_min))
    return EDD_EINVAL;
  edd_oc_params oc{};
  oc.volume = to->volfrac * (double)p->n_el;
  oc.rho_min = to->rho_min;
  oc.rho_max = to->rho_max;
  oc.move = to->move;
  oc.eta = to->eta;
  oc.penal = to->penal;
  oc.emin = to->emin;
  int rc = check_oc(&oc);
  if (rc) return rc;
  rc = ensure_to_buffers(p);
  if (rc) return rc;
  edd_solve_opts o;
  if (so) o = *so;
  else edd_default_opts(&o);
  edd_topopt_stats S{};
  const auto t0 = std::chrono::steady_clock::now();
  const OcDev q = to_dev(oc);
  k_rho_to_moduli<<<blocks_for(p->n_el), kTB, 0, p->stream>>>(p->n_el, rho_dev, q, p->to_E_d);
  double c1 = 0.0, c2 = 0.0;  // the last two compliance values
  int status = EDD_OK;
  for (int k = 0; k < to->maxit; ++k) {
    // Krylov tolerance from successive compliance values
    double tol = to->tol_max;
    if (!to->adaptive_tol) tol = to->tol_min;
    else if (k >= 2) tol = std::min(to->tol_max, std::max(to->tol_min, std::fabs(c1 - c2) / std::fabs(c1)));
    const auto ta = std::chrono::steady_clock::now();
    rc = edd_set_element_moduli(p, p->to_E_d, EDD_F64);
    if (rc) return rc;
    const auto tb = std::chrono::steady_clock::now();
    o.tol = tol;
    o.use_initial_guess = (to->warm_start && k > 0) ? 1 : 0;
    edd_solve_stats ss{};
    rc = edd_solve_interface(p, f_dev, u_dev, &o, &ss);
    if (rc < 0) return rc;
    if (rc == EDD_NOT_CONVERGED) status = EDD_NOT_CONVERGED;
    const auto tc = std::chrono::steady_clock::now();
    c2 = c1;
    c1 = ss.compliance;
    rc = element_energies(p, u_dev, p->to_s_d);
    if (rc) return rc;
    edd_oc_result res{};
    rc = oc_update(p, rho_dev, p->to_s_d, oc, p->to_rho_d, p->to_E_d, &res);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(rho_dev, p->to_rho_d, sizeof(double) * p->n_el,
                                  hipMemcpyDeviceToDevice, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    rc = check_hip(p, e);
    if (rc) return rc;
    const auto td = std::chrono::steady_clock::now();
    S.steps = k + 1;
    S.krylov_iterations += ss.iterations;
    S.compliance = ss.compliance;
    S.max_change = res.max_change;
    S.volume = res.volume;
    S.t_moduli_ms += std::chrono::duration<double, std::milli>(tb - ta).count();
    S.t_solve_ms += std::chrono::duration<double, std::milli>(tc - tb).count();
    S.t_update_ms += std::chrono::duration<double, std::milli>(td - tc).count();
    if (history_host) {
      double *h = history_host + 5 * k;
      h[0] = ss.compliance;
      h[1] = tol;
      h[2] = ss.iterations;
      h[3] = res.max_change;
      h[4] = ss.rel_residual;
    }
    if (res.max_change <= to->change_tol) break;
  }
  S.avg_krylov = S.steps ? (double)S.krylov_iterations / S.steps : 0.0;
  S.converged = S.max_change <= to->change_tol;
  S.t_total_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  S.status = status;
  if (st) *st = S;
  return status;
}

}  // extern "C"

// Explicit local Schur complements: an S apply by dense matrix-vector
// products.  S = sum_i R_i^T S_i R_i with S_i = K^i_GG - K^i_GI (K^i_II)^{-1}
// K^i_IG on the interface dofs of subdomain i's closure, its own elements
// only (the splitting of the Steklov-Poincare operator over the subdomains,
// Section 1; the subdomain problems of eq. (3MatSplit2)).
//
// Formation, after each factorisation: Y_i = L_i^{-1} K^i_IG by a forward
// substitution with all m_i right-hand sides through the interior factor
// (K^i_II = L_i L_i^T, the band factor of the factor path), then
// S_i = K^i_GG - Y_i^T Y_i.  The apply gathers each subdomain's interface
// values, multiplies by S_i (a workgroup per subdomain) and sums the local
// products of every interface dof over its subdomains in a fixed order.
//
// Per apply it streams sum_i m_i^2 entries (2D subdomains of 16 x 16
// elements: m_i <= 128, 128 KB each), instead of the band factors twice and
// two element-by-element K applies.  It applies where the interiors are not
// dissected and every S_i fits one workgroup (m_i <= 1024).
#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.h"

namespace edd {
namespace {

constexpr int kSchurMaxM = 1024;
constexpr int kRowsLds = 8192;  // doubles of Y staged per chunk in the product

// Y_i <- L_i^{-1} Y_i for all m_i columns at once: thread j owns column j and
// keeps its last kd + 1 values in a ring in LDS; the factor entries (column
// layout with reciprocal diagonal: (i, i-k) at (i-k)*ld + k) are the same
// for every thread.
__global__ __launch_bounds__(kSchurMaxM) void k_schur_forward(
    const SubDesc *__restrict__ subs, const SchurDesc *__restrict__ sds,
    const double *__restrict__ C, double *__restrict__ Y) {
  extern __shared__ double ring[];  // [(kd+1)][blockDim]
  const SchurDesc sd = sds[blockIdx.x];
  const SubDesc s = subs[sd.blk];
  const int m = sd.m, j = threadIdx.x, nt = blockDim.x;
  if (j >= m) return;  // columns are independent: no barriers below
  const int ld = s.kd + 1;
  const double *Cs = C + s.fac_off;
  double *Yi = Y + sd.y_off;
  int slot = 0;
  for (int i = 0; i < s.n; ++i) {
    double acc = Yi[(int64_t)i * m + j];
    const int kmax = min(s.kd, i);
    int sl = slot;
    for (int k = 1; k <= kmax; ++k) {
      sl = sl == 0 ? ld - 1 : sl - 1;
      acc = fma(-Cs[(int64_t)(i - k) * ld + k], ring[sl * nt + j], acc);
    }
    const double y = acc * Cs[(int64_t)i * ld];
    ring[slot * nt + j] = y;
    Yi[(int64_t)i * m + j] = y;
    slot = slot + 1 == ld ? 0 : slot + 1;
  }
}

// S_i = -Y_i^T Y_i (row-major m x m).  Each thread accumulates a 4 x 4 tile;
// the rows of Y_i pass through LDS in chunks of rc rows.
__global__ __launch_bounds__(1024) void k_schur_syrk(const SubDesc *__restrict__ subs,
                                                     const SchurDesc *__restrict__ sds,
                                                     const double *__restrict__ Y,
                                                     double *__restrict__ S) {
  extern __shared__ double ych[];  // [rc][m]
  const SchurDesc sd = sds[blockIdx.x];
  const int n = subs[sd.blk].n, m = sd.m;
  const int rc = max(1, min(64, kRowsLds / m));
  const int nt = (m + 3) / 4, ntiles = nt * nt;
  const double *Yi = Y + sd.y_off;
  double *Si = S + sd.s_off;
  for (int t0 = 0; t0 < ntiles; t0 += blockDim.x) {
    const int t = t0 + threadIdx.x;
    const bool act = t < ntiles;
    const int ta = act ? t / nt : 0, tb = act ? t - (t / nt) * nt : 0;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int r0 = 0; r0 < n; r0 += rc) {
      const int rn = min(rc, n - r0);
      __syncthreads();
      for (int e = threadIdx.x; e < rn * m; e += blockDim.x) ych[e] = Yi[(int64_t)r0 * m + e];
      __syncthreads();
      if (!act) continue;
      for (int r = 0; r < rn; ++r) {
        double ya[4], yb[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int ca = 4 * ta + a, cb = 4 * tb + a;
          ya[a] = ca < m ? ych[r * m + ca] : 0.0;
          yb[a] = cb < m ? ych[r * m + cb] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = fma(ya[a], yb[b], acc[a][b]);
      }
    }
    if (act) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int ca = 4 * ta + a, cb = 4 * tb + b;
          if (ca < m && cb < m) Si[(int64_t)ca * m + cb] = -acc[a][b];
        }
    }
  }
}

// yl_i = S_i v_i with v_i gathered from the interface vector (S_i read by
// columns: S_i[b][t] for row t, coalesced; S_i is symmetric).
__global__ __launch_bounds__(kSchurMaxM) void k_schur_gemv(int D,
                                                           const SchurDesc *__restrict__ sds,
                                                           const int *__restrict__ gl,
                                                           const double *__restrict__ S,
                                                           const double *__restrict__ v,
                                                           double *__restrict__ yl) {
  extern __shared__ double vl[];
  const SchurDesc sd = sds[blockIdx.x];
  const int m = sd.m;
  for (int t = threadIdx.x; t < m; t += blockDim.x) {
    const int an = t / D;
    vl[t] = v[(int64_t)gl[sd.g_off + an] * D + (t - an * D)];
  }
  __syncthreads();
  const double *Si = S + sd.s_off;
  for (int t = threadIdx.x; t < m; t += blockDim.x) {
    double a0 = 0.0, a1 = 0.0;
    int b = 0;
    for (; b + 1 < m; b += 2) {
      a0 = fma(Si[(int64_t)b * m + t], vl[b], a0);
      a1 = fma(Si[(int64_t)(b + 1) * m + t], vl[b + 1], a1);
    }
    if (b < m) a0 = fma(Si[(int64_t)b * m + t], vl[b], a0);
    yl[sd.l_off + t] = a0 + a1;
  }
}

// y[g, c] = sum of the local products of interface node g over the
// subdomains holding it, in the fixed owner order.
__global__ __launch_bounds__(256) void k_schur_sum(int64_t nG, int D,
                                                   const int *__restrict__ optr,
                                                   const int *__restrict__ oent,
                                                   const double *__restrict__ yl,
                                                   double *__restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nG * D) return;
  const int64_t g = i / D;
  const int c = (int)(i - g * D);
  double acc = 0.0;
  for (int k = optr[g]; k < optr[g + 1]; ++k) acc += yl[(int64_t)oent[k] * D + c];
  y[i] = acc;
}

inline int round64(int m) { return std::max(64, (m + 63) / 64 * 64); }

}  // namespace

int schur_setup(edd_problem *p) {
  if (!p->sc_desc.empty()) return EDD_OK;
  const int D = p->g.dim;
  if (p->n_sep > 0 || p->n_blk != p->n_sub || !(p->factor_precision & EDD_F64))
    return EDD_EINVAL;
  int nb[3] = {1, 1, 1};
  for (int a = 0; a < D; ++a) nb[a] = (int)p->cuts[a].size() - 1;
  std::vector<int> gpos(p->n_nodes, -1);
  for (int64_t k = 0; k < p->n_gamma; ++k) gpos[p->gnode[k]] = (int)k;
  std::vector<SchurDesc> desc(p->n_sub);
  std::vector<int> gl, tab;
  std::vector<std::vector<int>> owners(p->n_gamma);
  int64_t s_off = 0, y_off = 0, l_off = 0;
  int max_m = 0, max_mg = 0;
  for (int sid = 0; sid < p->n_sub; ++sid) {
    const int b[3] = {sid % nb[0], (sid / nb[0]) % nb[1], sid / (nb[0] * nb[1])};
    SchurDesc sd{};
    sd.blk = sid;
    for (int a = 0; a < 3; ++a) {
      if (a < D) {
        sd.c_lo[a] = p->cuts[a][b[a]];
        sd.c_ext[a] = p->cuts[a][b[a] + 1] - sd.c_lo[a] + 1;
        sd.e_lo[a] = p->cuts[a][b[a]];
        sd.e_hi[a] = p->cuts[a][b[a] + 1] - 1;
      } else {
        sd.c_lo[a] = 0;
        sd.c_ext[a] = 1;
        sd.e_lo[a] = sd.e_hi[a] = 0;
      }
    }
    sd.t_off = (int64_t)tab.size();
    sd.g_off = (int64_t)gl.size();
    int mg = 0;
    for (int z = 0; z < sd.c_ext[2]; ++z)
      for (int y = 0; y < sd.c_ext[1]; ++y)
        for (int x = 0; x < sd.c_ext[0]; ++x) {
          const int64_t node = (sd.c_lo[0] + x) +
                               (int64_t)p->g.nn[0] * ((sd.c_lo[1] + y) +
                                                      (int64_t)p->g.nn[1] * (sd.c_lo[2] + z));
          const int g = gpos[node];
          if (g >= 0) {
            tab.push_back(mg);
            gl.push_back(g);
            owners[g].push_back((int)(l_off / D) + mg);
            ++mg;
          } else {
            tab.push_back(-1);
          }
        }
    sd.mg = mg;
    sd.m = D * mg;
    if (sd.m > kSchurMaxM) return EDD_EINVAL;
    const SubDesc &s = p->subs[sid];
    const size_t ring = (size_t)(s.kd + 1) * round64(sd.m) * sizeof(double);
    if (ring > p->lds_limit) return EDD_EINVAL;
    sd.s_off = s_off;
    sd.y_off = y_off;
    sd.l_off = l_off;
    s_off += (int64_t)sd.m * sd.m;
    y_off += (int64_t)s.n * sd.m;
    l_off += sd.m;
    max_m = std::max(max_m, sd.m);
    max_mg = std::max(max_mg, mg);
    desc[sid] = sd;
  }
  // one launch serves every subdomain: the ring of the largest band and
  // block; storage: S_i (kept) and Y_i (formation work space)
  if ((size_t)(p->max_kd + 1) * round64(max_m) * sizeof(double) > p->lds_limit) return EDD_EINVAL;
  if ((s_off + y_off) * sizeof(double) > ((size_t)16 << 30)) return EDD_EINVAL;
  std::vector<int> optr(p->n_gamma + 1, 0), oent;
  for (int64_t g = 0; g < p->n_gamma; ++g) {
    optr[g + 1] = optr[g] + (int)owners[g].size();
    oent.insert(oent.end(), owners[g].begin(), owners[g].end());
  }
  auto alloc = [&](size_t bytes) { return dev_alloc(p, std::max<size_t>(bytes, 8)); };
  p->sc_desc_d = (SchurDesc *)alloc(sizeof(SchurDesc) * desc.size());
  p->sc_gl_d = (int *)alloc(sizeof(int) * gl.size());
  p->sc_tab_d = (int *)alloc(sizeof(int) * tab.size());
  p->sc_optr_d = (int *)alloc(sizeof(int) * optr.size());
  p->sc_oent_d = (int *)alloc(sizeof(int) * oent.size());
  p->sc_S_d = (double *)alloc(sizeof(double) * s_off);
  p->sc_Y_d = (double *)alloc(sizeof(double) * y_off);
  p->sc_yl_d = (double *)alloc(sizeof(double) * l_off);
  if (!p->sc_desc_d || !p->sc_gl_d || !p->sc_tab_d || !p->sc_optr_d || !p->sc_oent_d ||
      !p->sc_S_d || !p->sc_Y_d || !p->sc_yl_d)
    return EDD_ENOMEM;
  hipError_t e = hipSuccess;
  auto up = [&](void *dst, const void *src, size_t bytes) {
    if (e == hipSuccess && bytes)
      e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, p->stream);
  };
  up(p->sc_desc_d, desc.data(), sizeof(SchurDesc) * desc.size());
  up(p->sc_gl_d, gl.data(), sizeof(int) * gl.size());
  up(p->sc_tab_d, tab.data(), sizeof(int) * tab.size());
  up(p->sc_optr_d, optr.data(), sizeof(int) * optr.size());
  up(p->sc_oent_d, oent.data(), sizeof(int) * oent.size());
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return check_hip(p, e);
  p->sc_desc.swap(desc);
  p->sc_S_len = s_off;
  p->sc_Y_len = y_off;
  p->sc_max_m = max_m;
  p->sc_max_mg = max_mg;
  return EDD_OK;
}

int schur_form(edd_problem *p) {
  p->sc_ready = false;
  if (p->sc_desc.empty() || !p->have_moduli) return EDD_ESTATE;
  const int n = (int)p->sc_desc.size();
  launch_schur_couplings(p);
  {
    const int nt = round64(p->sc_max_m);
    const size_t lds = (size_t)(p->max_kd + 1) * nt * sizeof(double);
    set_lds_limit_once((const void *)k_schur_forward, p);
    k_schur_forward<<<n, nt, lds, p->stream>>>(p->subs_d, p->sc_desc_d, p->fac64_d, p->sc_Y_d);
  }
  {
    // each workgroup stages at most kRowsLds entries of its Y_i
    set_lds_limit_once((const void *)k_schur_syrk, p);
    k_schur_syrk<<<n, 1024, sizeof(double) * kRowsLds, p->stream>>>(p->subs_d, p->sc_desc_d,
                                                                      p->sc_Y_d, p->sc_S_d);
  }
  launch_schur_kgg(p);
  const int rc = check_hip(p, hipGetLastError());
  if (rc) return rc;
  p->sc_ready = true;
  return EDD_OK;
}

void schur_apply(edd_problem *p, const double *v, double *y) {
  const int D = p->g.dim;
  const int n = (int)p->sc_desc.size();
  const int nt = round64(p->sc_max_m);
  k_schur_gemv<<<n, nt, sizeof(double) * p->sc_max_m, p->stream>>>(D, p->sc_desc_d, p->sc_gl_d,
                                                                     p->sc_S_d, v, p->sc_yl_d);
  const int64_t m = p->n_gamma * D;
  k_schur_sum<<<(unsigned)((m + 255) / 256), 256, 0, p->stream>>>(
      p->n_gamma, D, p->sc_optr_d, p->sc_oent_d, p->sc_yl_d, y);
}

}  // namespace edd

using namespace edd;

extern "C" int edd_set_s_apply(edd_problem *p, int mode) {
  if (!p || (mode != 0 && mode != 1)) return EDD_EINVAL;
  if (mode == 0) {
    p->s_apply_mode = 0;
    return EDD_OK;
  }
  int rc = schur_setup(p);
  if (rc) return rc;
  p->s_apply_mode = 1;
  if (p->have_moduli) {
    rc = schur_form(p);
    if (!rc) rc = check_hip(p, hipStreamSynchronize(p->stream));
    if (rc) {
      p->s_apply_mode = 0;
      return rc;
    }
  }
  return EDD_OK;
}

extern "C" int edd_get_s_apply(edd_problem *p, int *mode) {
  if (!p || !mode) return EDD_EINVAL;
  *mode = p->s_apply_mode;
  return EDD_OK;
}

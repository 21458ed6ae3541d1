// Interface preconditioner Hhat_theta (Section 3, eqs. (NumberEight)-
// (NumberNine)) applied by inverse Lanczos, as in the paper's experiments.
//
// z = H~_theta^{-1} r = (M^{-1} L)^{theta-1} M^{-1} r for each displacement
// component, with M (lumped) and L the mass and Laplacian of the skeleton
// (1D linear elements on the cut lines in 2D, bilinear quadrilaterals on the
// cut planes in 3D), clamped nodes removed.  Inverse Lanczos runs Lanczos on
// C = L^{-1} M in the M inner product from b = M^{-1} r and returns
// |b|_M Q_k T_k^{1-theta} e1; each step solves with L by PCG preconditioned
// with L restricted to the faces of the skeleton with the cross points
// removed (Section 4), the faces' blocks inverted once per distinct shape.
//
// Optional extension (interface_weighting = 1): every skeleton element's
// mass and Laplacian are scaled by the mean modulus of its two neighbouring
// volume elements, so the norm follows the local scale of the Steklov-
// Poincare operator in heterogeneous designs.  The face blocks then use the
// unweighted inverse with a diagonal rescaling sqrt(diag L_w / diag L).
//
// All d components run in lockstep (independent Lanczos processes); their
// scalars travel together so every reduction serves all components.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <numeric>
#include <unordered_map>
#include <utility>

#include "internal.h"

namespace edd {

// scalar slots used here (the solver's own slots are below 528)
enum : int {
  P_BASE = 528,
  P_RZ = P_BASE,        // [3]
  P_PQ = P_BASE + 3,    // [3]
  P_RR = P_BASE + 6,    // [3]
  P_BB = P_BASE + 9,    // [3]
  P_RZN = P_BASE + 12,  // [3]
  P_A = P_BASE + 15,    // [3] Lanczos alpha
  P_B = P_BASE + 18,    // [3] Lanczos beta
  P_B0 = P_BASE + 21,   // [3] |b|_M^2
  P_BETA = P_BASE + 24, // [3] previous Lanczos beta
  P_H = P_BASE + 32,    // [65*3] reorthogonalisation / combination coefficients
  P_END = P_H + 65 * 3,
  P_AH = 900,           // [64*3] alpha history (device-resident mode)
  P_BH = 1100,          // [64*3] beta history
  P_CO = 1300           // [64*3] final combination coefficients
};

constexpr int kMaxFace = 512;  // larger faces fall back to the diagonal
constexpr int kBlock = 256;

// forms of the interface preconditioner (edd_solve_opts.pc_form)
inline bool pc_forward(const edd_solve_opts *o) {
  return o->pc_form == EDD_PCF_HTILDE_FWD || o->pc_form == EDD_PCF_H_FWD;
}
inline int pc_fkind(const edd_solve_opts *o) {
  switch (o->pc_form) {
    case EDD_PCF_H_INV: return 1;
    case EDD_PCF_HTILDE_FWD: return 2;
    case EDD_PCF_H_FWD: return 3;
    default: return 0;
  }
}

namespace {

inline unsigned grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  return (unsigned)g;
}

__device__ inline double block_sum(double v, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------- operators
__global__ __launch_bounds__(kBlock) void k_sk_weights(
    int64_t n, const int *__restrict__ adj, const double *__restrict__ E,
    int weighted, double *__restrict__ w) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  w[e] = weighted ? 0.5 * (E[adj[2 * e]] + E[adj[2 * e + 1]]) : 1.0;
}

struct ElemMat {  // an element matrix of the skeleton (L or M), row-major
  double v[16];
};

__global__ __launch_bounds__(kBlock) void k_sk_assemble(
    int64_t nnz, const int *__restrict__ cptr, const int *__restrict__ celem,
    const int *__restrict__ cab, const double *__restrict__ w, ElemMat em,
    double *__restrict__ val) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  double s = 0.0;
  for (int t = cptr[k]; t < cptr[k + 1]; ++t) s = fma(w[celem[t]], em.v[cab[t]], s);
  val[k] = s;
}

__global__ __launch_bounds__(kBlock) void k_sk_diag(
    int64_t nG, const int *__restrict__ nptr, const int *__restrict__ nelem,
    const double *__restrict__ w, double rowsum, const int *__restrict__ rowptr,
    const int *__restrict__ col, const double *__restrict__ val,
    const double *__restrict__ l0, double *__restrict__ M,
    double *__restrict__ Ld, double *__restrict__ S) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nG) return;
  double m = 0.0;
  for (int t = nptr[i]; t < nptr[i + 1]; ++t) m += w[nelem[t]];
  M[i] = rowsum * m;
  double d = 0.0;
  for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
    if (col[k] == i) d = val[k];
  Ld[i] = d;
  S[i] = sqrt(d / l0[i]);
}

// diag[i] = the (i, i) entry of a CSR matrix
__global__ __launch_bounds__(kBlock) void k_csr_diag(int64_t n, const int *__restrict__ rowptr,
                                                     const int *__restrict__ col,
                                                     const double *__restrict__ val,
                                                     double *__restrict__ diag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = 0.0;
  for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
    if (col[k] == i) d = val[k];
  diag[i] = d;
}

// Chebyshev iteration for the consistent skeleton mass, M x = b, scaled by
// diag(M) (Saad, Iterative Methods for Sparse Linear Systems, Alg. 12.1,
// with the Jacobi preconditioner), the spectrum of diag(M)^{-1} M inside
// [th - de, th + de]:
//   x_0 = 0, r_0 = b, d_0 = diag(M)^{-1} r_0 / th, rho_0 = de / th;
//   x_{k+1} = x_k + d_k, r_{k+1} = r_k - M d_k,
//   rho_{k+1} = 1 / (2 th / de - rho_k),
//   d_{k+1} = rho_{k+1} rho_k d_k + (2 rho_{k+1} / de) diag(M)^{-1} r_{k+1}.
// Each component of the D interleaved ones is an independent system.
template <int D>
__global__ __launch_bounds__(kBlock) void k_cheb_init(int64_t nG, const double *__restrict__ diag,
                                                      double inv_th, const double *__restrict__ b,
                                                      double *__restrict__ x,
                                                      double *__restrict__ r,
                                                      double *__restrict__ d) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nG) return;
  const double s = inv_th / diag[i];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double v = b[i * D + c];
    x[i * D + c] = 0.0;
    r[i * D + c] = v;
    d[i * D + c] = s * v;
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_cheb_step(
    int64_t nG, const int *__restrict__ rowptr, const int *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ diag,
    const double *__restrict__ d_in, double *__restrict__ d_out, double *__restrict__ x,
    double *__restrict__ r, double c1, double c2) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nG) return;
  double acc[D];
#pragma unroll
  for (int c = 0; c < D; ++c) acc[c] = 0.0;
  for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
    const double v = val[k];
    const int64_t j = col[k];
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] = fma(v, d_in[j * D + c], acc[c]);
  }
  const double s = c2 / diag[i];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double dv = d_in[i * D + c];
    x[i * D + c] += dv;
    const double rv = r[i * D + c] - acc[c];
    r[i * D + c] = rv;
    d_out[i * D + c] = fma(c1, dv, s * rv);
  }
}

// y = L x for D interleaved components
// acc[c] += sum_k val[k] * x[col[k]*D + c] over one CSR row, in order of k,
// four entries' loads issued together
template <int D>
__device__ inline void csr_row(int k0, int k1, const int *__restrict__ col,
                               const double *__restrict__ val, const double *__restrict__ x,
                               double (&acc)[D]) {
  int k = k0;
  for (; k + 4 <= k1; k += 4) {
    double v[4], xv[4][D];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      v[u] = val[k + u];
      const int64_t j = col[k + u];
#pragma unroll
      for (int c = 0; c < D; ++c) xv[u][c] = x[j * D + c];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int c = 0; c < D; ++c) acc[c] = fma(v[u], xv[u][c], acc[c]);
  }
  for (; k < k1; ++k) {
    const double v = val[k];
    const int64_t j = col[k];
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] = fma(v, x[j * D + c], acc[c]);
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_spmv(int64_t nG, const int *__restrict__ rowptr,
                                                 const int *__restrict__ col,
                                                 const double *__restrict__ val,
                                                 const double *__restrict__ x,
                                                 double *__restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nG) return;
  double acc[D];
#pragma unroll
  for (int c = 0; c < D; ++c) acc[c] = 0.0;
  csr_row<D>(rowptr[i], rowptr[i + 1], col, val, x, acc);
#pragma unroll
  for (int c = 0; c < D; ++c) y[i * D + c] = acc[c];
}

// acc[c] += sum_{j0 <= j < j1} A[j*m + i] * rs[j*D + c], in order of j, with
// eight loads of A in flight (the loads are independent; only the sums
// chain).
template <int D>
__device__ inline void face_row_sum(const double *__restrict__ A, int m, int i, int j0, int j1,
                                    const double *rs, double (&acc)[D]) {
  int j = j0;
  for (; j + 8 <= j1; j += 8) {
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = A[(int64_t)(j + u) * m + i];  // symmetric
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int c = 0; c < D; ++c) acc[c] = fma(a[u], rs[(j + u) * D + c], acc[c]);
  }
  for (; j < j1; ++j) {
    const double a = A[(int64_t)j * m + i];
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] = fma(a, rs[j * D + c], acc[c]);
  }
}

// face blocks: z_f = S^{-1} A_class^{-1} S^{-1} r_f; one workgroup per face,
// each row's sum split over kFaceQ parts of the columns (shorter dependent
// load chains), 256 threads per part, the parts added in a fixed order.
constexpr int kFaceQ = 2;

template <int D>
__global__ __launch_bounds__(256 * kFaceQ, 8) void k_face_apply(
    const int *__restrict__ fblk, const int *__restrict__ fptr, const int *__restrict__ fnode,
    const int *__restrict__ fclass, const int64_t *__restrict__ coff,
    const double *__restrict__ inv, const double *__restrict__ S,
    const double *__restrict__ r, double *__restrict__ z) {
  __shared__ double rs[kMaxFace * D];
  __shared__ double part[kFaceQ][kMaxFace * D];
  const int f = fblk[blockIdx.x];
  if (f < 0) return;  // an empty launch slot (whole workgroup)
  const int b0 = fptr[f], m = fptr[f + 1] - b0;
  const double *A = inv + coff[fclass[f]];
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const int g = fnode[b0 + i];
    const double s = 1.0 / S[g];
#pragma unroll
    for (int c = 0; c < D; ++c) rs[i * D + c] = r[(int64_t)g * D + c] * s;
  }
  __syncthreads();
  const int q = threadIdx.x / 256;
  const int j0 = q * m / kFaceQ, j1 = (q + 1) * m / kFaceQ;
  for (int i = threadIdx.x % 256; i < m; i += 256) {
    double acc[D];
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] = 0.0;
    face_row_sum<D>(A, m, i, j0, j1, rs, acc);
#pragma unroll
    for (int c = 0; c < D; ++c) part[q][i * D + c] = acc[c];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const int g = fnode[b0 + i];
    const double s = 1.0 / S[g];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double v = 0.0;
#pragma unroll
      for (int qq = 0; qq < kFaceQ; ++qq) v += part[qq][i * D + c];
      z[(int64_t)g * D + c] = v * s;
    }
  }
}

// y = x (a kernel rather than a copy node, so captured graphs hold kernels only)
__global__ __launch_bounds__(kBlock) void k_copy(int64_t n, const double *__restrict__ x,
                                                 double *__restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i];
}

// ---- fused steps of the fixed-count inner PCG ------------------------------
// q = L x with per-block partial sums of x.q per component.
template <int D>
__global__ __launch_bounds__(kBlock) void k_spmv_dot(int64_t nG, const int *__restrict__ rowptr,
                                                     const int *__restrict__ col,
                                                     const double *__restrict__ val,
                                                     const double *__restrict__ x,
                                                     double *__restrict__ y,
                                                     double *__restrict__ partials) {
  __shared__ double red[kBlock / 64];
  double dot[D];
#pragma unroll
  for (int c = 0; c < D; ++c) dot[c] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nG;
       i += (int64_t)gridDim.x * blockDim.x) {
    double acc[D];
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] = 0.0;
    csr_row<D>(rowptr[i], rowptr[i + 1], col, val, x, acc);
#pragma unroll
    for (int c = 0; c < D; ++c) {
      y[i * D + c] = acc[c];
      dot[c] = fma(x[i * D + c], acc[c], dot[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double s = block_sum(dot[c], red);
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * D + c] = s;
  }
}

// The rest nodes of the fused step below (diagonal preconditioner):
// nodes t0, t0 + stride, ... of the rest list; the workgroup's sum of r.z
// per component goes to out[c].
template <int D, bool INIT>
__device__ inline void rest_pcg_part(int64_t n, int64_t t0, int64_t stride,
                                     const int *__restrict__ rest, const double *__restrict__ Ld,
                                     const double *__restrict__ scal, int rz, int pq,
                                     double *__restrict__ y, const double *__restrict__ p,
                                     double *__restrict__ r, const double *__restrict__ q,
                                     double *__restrict__ z, double *__restrict__ pdir,
                                     double *__restrict__ out, double *red) {
  double dot[D];
#pragma unroll
  for (int c = 0; c < D; ++c) dot[c] = 0.0;
  for (int64_t t = t0; t < n; t += stride) {
    const int64_t g = rest[t];
    const double s = 1.0 / Ld[g];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double rv = r[g * D + c];
      if (!INIT) {
        const double den = scal[pq + c];
        const double a = den != 0.0 ? scal[rz + c] / den : 0.0;
        y[g * D + c] = fma(a, p[g * D + c], y[g * D + c]);
        rv = fma(-a, q[g * D + c], rv);
        r[g * D + c] = rv;
      }
      const double zv = rv * s;
      z[g * D + c] = zv;
      if (INIT) pdir[g * D + c] = zv;
      dot[c] = fma(rv, zv, dot[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double sm = block_sum(dot[c], red);
    if (threadIdx.x == 0) out[c] = sm;
  }
}

// The face-block preconditioner fused with the PCG update that precedes it
// and the r.z partial sums that follow it.  Unless INIT: per component
// a = scal[rz]/scal[pq], y += a p and r -= a q on the face's nodes (every
// interface node is in exactly one face or in the rest set).  Then
// z = S^{-1} A^{-1} S^{-1} r on the face; INIT also writes pdir = z.  The
// face's sum of r.z per component goes to partials[f*D + c].  Workgroups
// past the nfb face slots treat the rest nodes (diagonal preconditioner),
// their sums at partials[(n_faces + k)*D + c] for the k-th such workgroup.
template <int D, bool INIT>
__global__ __launch_bounds__(256 * kFaceQ, 8) void k_face_pcg(
    const int *__restrict__ fblk, const int *__restrict__ fptr, const int *__restrict__ fnode,
    const int *__restrict__ fclass, const int64_t *__restrict__ coff,
    const double *__restrict__ inv, const double *__restrict__ S,
    const double *__restrict__ scal, int rz, int pq, double *__restrict__ y,
    const double *__restrict__ p, double *__restrict__ r, const double *__restrict__ q,
    double *__restrict__ z, double *__restrict__ pdir, double *__restrict__ partials,
    int nfb, int n_faces, int64_t n_rest, const int *__restrict__ rest,
    const double *__restrict__ Ld) {
  __shared__ double rs[kMaxFace * D];
  __shared__ double rn[kMaxFace * D];
  __shared__ double part[kFaceQ][kMaxFace * D];
  __shared__ double red[kFaceQ * 4][D];
  if ((int)blockIdx.x >= nfb) {  // the workgroups after the face slots: rest nodes
    const int rb = blockIdx.x - nfb, nrb = gridDim.x - nfb;
    rest_pcg_part<D, INIT>(n_rest, (int64_t)rb * blockDim.x + threadIdx.x,
                           (int64_t)nrb * blockDim.x, rest, Ld, scal, rz, pq, y, p, r, q, z,
                           pdir, partials + ((int64_t)n_faces + rb) * D, &red[0][0]);
    return;
  }
  const int f = fblk[blockIdx.x];
  if (f < 0) return;  // an empty launch slot (whole workgroup)
  const int b0 = fptr[f], m = fptr[f + 1] - b0;
  const double *A = inv + coff[fclass[f]];
  double a[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double den = INIT ? 0.0 : scal[pq + c];
    a[c] = (!INIT && den != 0.0) ? scal[rz + c] / den : 0.0;
  }
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const int64_t g = fnode[b0 + i];
    const double s = 1.0 / S[g];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double rv = r[g * D + c];
      if (!INIT) {
        y[g * D + c] = fma(a[c], p[g * D + c], y[g * D + c]);
        rv = fma(-a[c], q[g * D + c], rv);
        r[g * D + c] = rv;
      }
      rn[i * D + c] = rv;
      rs[i * D + c] = rv * s;
    }
  }
  __syncthreads();
  const int qq0 = threadIdx.x / 256;
  const int j0 = qq0 * m / kFaceQ, j1 = (qq0 + 1) * m / kFaceQ;
  for (int i = threadIdx.x % 256; i < m; i += 256) {
    double acc[D];
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] = 0.0;
    face_row_sum<D>(A, m, i, j0, j1, rs, acc);
#pragma unroll
    for (int c = 0; c < D; ++c) part[qq0][i * D + c] = acc[c];
  }
  __syncthreads();
  double dot[D];
#pragma unroll
  for (int c = 0; c < D; ++c) dot[c] = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const int64_t g = fnode[b0 + i];
    const double s = 1.0 / S[g];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double v = 0.0;
#pragma unroll
      for (int k2 = 0; k2 < kFaceQ; ++k2) v += part[k2][i * D + c];
      const double zv = v * s;
      z[g * D + c] = zv;
      if (INIT) pdir[g * D + c] = zv;
      dot[c] = fma(rn[i * D + c], zv, dot[c]);
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    double v = dot[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) red[wv][c] = v;
  }
  __syncthreads();
  if (threadIdx.x < D) {
    double sum = 0.0;
    for (int w2 = 0; w2 < kFaceQ * 4; ++w2) sum += red[w2][threadIdx.x];
    partials[(int64_t)f * D + threadIdx.x] = sum;
  }
}

// The same step for faces of at most 64 nodes (2D edges): one wavefront
// per face, four faces per workgroup, lane i owning row i; the face's r.z
// sums go to partials[f*D + c].  Workgroups from nsb on treat the rest
// nodes, as above.
template <int D, bool INIT>
__global__ __launch_bounds__(256) void k_face_pcg_small(
    const int *__restrict__ fptr, const int *__restrict__ fnode,
    const int *__restrict__ fclass, const int64_t *__restrict__ coff,
    const double *__restrict__ inv, const double *__restrict__ S,
    const double *__restrict__ scal, int rz, int pq, double *__restrict__ y,
    const double *__restrict__ p, double *__restrict__ r, const double *__restrict__ q,
    double *__restrict__ z, double *__restrict__ pdir, double *__restrict__ partials,
    int n_faces, int nsb, int64_t n_rest, const int *__restrict__ rest,
    const double *__restrict__ Ld) {
  __shared__ double rs[4][64 * D];
  __shared__ double red[4 * D];
  if ((int)blockIdx.x >= nsb) {  // rest nodes
    const int rb = blockIdx.x - nsb, nrb = gridDim.x - nsb;
    rest_pcg_part<D, INIT>(n_rest, (int64_t)rb * blockDim.x + threadIdx.x,
                           (int64_t)nrb * blockDim.x, rest, Ld, scal, rz, pq, y, p, r, q, z,
                           pdir, partials + ((int64_t)n_faces + rb) * D, red);
    return;
  }
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int f = blockIdx.x * 4 + wv;
  int b0 = 0, m = 0;
  const double *A = inv;
  if (f < n_faces) {
    b0 = fptr[f];
    m = fptr[f + 1] - b0;
    A = inv + coff[fclass[f]];
  }
  double a[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double den = INIT ? 0.0 : scal[pq + c];
    a[c] = (!INIT && den != 0.0) ? scal[rz + c] / den : 0.0;
  }
  int64_t g = 0;
  double s = 0.0, rn[D];
  if (lane < m) {
    g = fnode[b0 + lane];
    s = 1.0 / S[g];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double rv = r[g * D + c];
      if (!INIT) {
        y[g * D + c] = fma(a[c], p[g * D + c], y[g * D + c]);
        rv = fma(-a[c], q[g * D + c], rv);
        r[g * D + c] = rv;
      }
      rn[c] = rv;
      rs[wv][lane * D + c] = rv * s;
    }
  }
  __syncthreads();
  double dot[D];
#pragma unroll
  for (int c = 0; c < D; ++c) dot[c] = 0.0;
  if (lane < m) {
    double acc[D];
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] = 0.0;
    face_row_sum<D>(A, m, lane, 0, m, rs[wv], acc);
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const double zv = acc[c] * s;
      z[g * D + c] = zv;
      if (INIT) pdir[g * D + c] = zv;
      dot[c] = rn[c] * zv;
    }
  }
#pragma unroll
  for (int c = 0; c < D; ++c) {
    double v = dot[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0 && f < n_faces) partials[(int64_t)f * D + c] = v;
  }
}

// p = z + (scal[rz_new]/scal[rz_old]) p per component.
template <int D>
__global__ __launch_bounds__(kBlock) void k_pcg_dir2(int64_t nG, const double *__restrict__ scal,
                                                     int rz_new, int rz_old,
                                                     const double *__restrict__ z,
                                                     double *__restrict__ p) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nG) return;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double rzo = scal[rz_old + c];
    const double b = rzo != 0.0 ? scal[rz_new + c] / rzo : 0.0;
    p[i * D + c] = fma(b, p[i * D + c], z[i * D + c]);
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_rest_apply(int64_t n, const int *__restrict__ rest,
                                                       const double *__restrict__ Ld,
                                                       const double *__restrict__ r,
                                                       double *__restrict__ z) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t g = rest[t];
  const double s = 1.0 / Ld[g];
#pragma unroll
  for (int c = 0; c < D; ++c) z[g * D + c] = r[g * D + c] * s;
}

// --------------------------------------------------------- per-component ops
// partial sums per component of sum_i wgt_i * a[i,c] * b[i,c] (wgt may be
// null) for up to 2 pairs; partials[blk*(2*D) + pair*D + c]
template <int D>
__global__ __launch_bounds__(kBlock) void k_cdots(int64_t nG, int npair,
                                                  const double *__restrict__ a0,
                                                  const double *__restrict__ b0,
                                                  const double *__restrict__ a1,
                                                  const double *__restrict__ b1,
                                                  const double *__restrict__ wgt,
                                                  double *__restrict__ partials) {
  __shared__ double red[kBlock / 64];
  double acc[2][D];
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int c = 0; c < D; ++c) acc[k][c] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nG;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double wi = wgt ? wgt[i] : 1.0;
#pragma unroll
    for (int c = 0; c < D; ++c) acc[0][c] = fma(wi * a0[i * D + c], b0[i * D + c], acc[0][c]);
    if (npair > 1) {
#pragma unroll
      for (int c = 0; c < D; ++c) acc[1][c] = fma(wi * a1[i * D + c], b1[i * D + c], acc[1][c]);
    }
  }
  for (int k = 0; k < npair; ++k)
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const double s = block_sum(acc[k][c], red);
      if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * (npair * D) + k * D + c] = s;
    }
}

// many-vector dots per component: partials[blk*(m*D) + j*D + c] =
// sum_i wgt_i V_j[i,c] w[i,c]
template <int D>
__global__ __launch_bounds__(kBlock) void k_cwindow_dots(int64_t nG, int m,
                                                         const double *__restrict__ V,
                                                         const double *__restrict__ x,
                                                         const double *__restrict__ wgt,
                                                         double *__restrict__ partials) {
  __shared__ double red[kBlock / 64];
  const int64_t n = nG * D;
  const int64_t chunk = (nG + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * chunk, hi = min(nG, lo + chunk);
  for (int j = 0; j < m; ++j) {
    double acc[D];
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] = 0.0;
    const double *Vj = V + (int64_t)j * n;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      const double wi = wgt ? wgt[i] : 1.0;
#pragma unroll
      for (int c = 0; c < D; ++c) acc[c] = fma(wi * Vj[i * D + c], x[i * D + c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const double s = block_sum(acc[c], red);
      if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * (m * D) + j * D + c] = s;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_reduce(const double *__restrict__ partials,
                                                   int nblocks, int stride,
                                                   double *__restrict__ out) {
  __shared__ double red[kBlock / 64];
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
    acc += partials[(int64_t)b * stride + j];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) out[j] = s;
}

// y[i,c] = x[i,c] * f_c with f_c = scal[slot+c] (op 0), 1/sqrt(scal[slot+c])
// (op 1), 1/scal[slot+c] (op 2), 1 (op 3); x is divided by wgt_i when wgt is
// not null
template <int D>
__global__ __launch_bounds__(kBlock) void k_cscale(int64_t nG, const double *__restrict__ scal,
                                                   int slot, int op,
                                                   const double *__restrict__ wgt,
                                                   const double *__restrict__ x,
                                                   double *__restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nG) return;
  const double wi = wgt ? 1.0 / wgt[i] : 1.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double s = op == 3 ? 1.0 : scal[slot + c];
    const double f = op == 3 ? 1.0
                   : op == 0 ? s
                   : op == 1 ? (s > 0.0 ? 1.0 / sqrt(s) : 0.0)
                             : (s != 0.0 ? 1.0 / s : 0.0);
    y[i * D + c] = x[i * D + c] * wi * f;
  }
}

// y[i,c] = m_i * x[i,c]
template <int D>
__global__ __launch_bounds__(kBlock) void k_dscale(int64_t nG, const double *__restrict__ mdiag,
                                                   const double *__restrict__ x,
                                                   double *__restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nG) return;
#pragma unroll
  for (int c = 0; c < D; ++c) y[i * D + c] = mdiag[i] * x[i * D + c];
}

// PCG update: alpha_c = rz_c / pq_c; y += alpha p; r -= alpha q
template <int D>
__global__ __launch_bounds__(kBlock) void k_pcg_update(int64_t nG, const double *__restrict__ scal,
                                                       double *__restrict__ y,
                                                       const double *__restrict__ p,
                                                       double *__restrict__ r,
                                                       const double *__restrict__ q) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nG) return;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double pq = scal[P_PQ + c];
    const double a = pq != 0.0 ? scal[P_RZ + c] / pq : 0.0;
    y[i * D + c] = fma(a, p[i * D + c], y[i * D + c]);
    r[i * D + c] = fma(-a, q[i * D + c], r[i * D + c]);
  }
}

// p = z + beta p, beta_c = rzn_c / rz_c; then rz <- rzn
template <int D>
__global__ __launch_bounds__(kBlock) void k_pcg_dir(int64_t nG, const double *__restrict__ scal,
                                                    const double *__restrict__ z,
                                                    double *__restrict__ p) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nG) return;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double rz = scal[P_RZ + c];
    const double b = rz != 0.0 ? scal[P_RZN + c] / rz : 0.0;
    p[i * D + c] = fma(b, p[i * D + c], z[i * D + c]);
  }
}

// The scalar function applied to the Lanczos tridiagonal (Section 3): with
// a = 1 - theta, eigenvalues t of T approximate those of C = L^{-1} M
// (inverse Lanczos, t = 1/lambda) or of A = M^{-1} L (forward, truncated
// Lanczos, t = lambda), lambda the generalised eigenvalues of L v = lambda M v:
//   0: t^a     inverse Lanczos, Htilde_theta^{-1} = V Lambda^{-a} V^T
//   1: t^a / (1 + t^a)      inverse Lanczos, H_theta^{-1} = V (1 + Lambda^a)^{-1} V^T
//   2: t^{-a}  forward Lanczos, Htilde_theta^{-1}
//   3: 1 / (1 + t^a)        forward Lanczos, H_theta^{-1}
// Negative Ritz values (rounding) are clamped to zero.
__host__ __device__ inline double lanczos_fn(int fkind, double a, double t) {
  const double l = t > 0.0 ? t : 0.0;
  switch (fkind) {
    case 1: { const double q = pow(l, a); return q / (1.0 + q); }
    case 2: return l > 0.0 ? pow(l, -a) : 0.0;
    case 3: return 1.0 / (1.0 + pow(l, a));
    default: return pow(l, a);
  }
}

__global__ void k_copy_scal(double *__restrict__ scal, int dst, int src, int n) {
  const int t = threadIdx.x;
  if (t < n) scal[dst + t] = scal[src + t];
}

// y[i,c] = sy*y[i,c] + sc * sum_j coef[j*D+c] * V_j[i,c]
template <int D>
__global__ __launch_bounds__(kBlock) void k_ccombine(int64_t nG, int m, const double *__restrict__ V,
                                                     const double *__restrict__ coef,
                                                     double sy, double sc,
                                                     double *__restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nG) return;
  const int64_t n = nG * D;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    double acc = 0.0;
    for (int j = 0; j < m; ++j) acc = fma(coef[j * D + c], V[(int64_t)j * n + i * D + c], acc);
    y[i * D + c] = (sy == 0.0 ? 0.0 : sy * y[i * D + c]) + sc * acc;
  }
}

// w -= a_c q_j + b_c q_{j-1} (b ignored when qm is null)
template <int D>
__global__ __launch_bounds__(kBlock) void k_lanczos3(int64_t nG, const double *__restrict__ scal,
                                                     const double *__restrict__ qj,
                                                     const double *__restrict__ qm,
                                                     double *__restrict__ w) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nG) return;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    double v = fma(-scal[P_A + c], qj[i * D + c], w[i * D + c]);
    if (qm) v = fma(-scal[P_BETA + c], qm[i * D + c], v);
    w[i * D + c] = v;
  }
}

// history of the Lanczos scalars for step j; beta = sqrt(|w|_M^2)
__global__ void k_store_ab(double *__restrict__ scal, int j, int D) {
  const int c = threadIdx.x;
  if (c >= D) return;
  const double b = sqrt(fmax(scal[P_B + c], 0.0));
  scal[P_AH + j * D + c] = scal[P_A + c];
  scal[P_BH + j * D + c] = b;
  scal[P_BETA + c] = b;
}

// coef[i*D+c] = |b|_M * (f(T) e1)_i for the k x k tridiagonal of component
// c, by cyclic Jacobi rotations; one thread per component (k <= 32).
// f is lanczos_fn(fkind, a, .) below.
__global__ void k_lanczos_coef(double *__restrict__ scal, int k, int D, int fkind, double pw) {
  __shared__ double A[3][32 * 32];
  __shared__ double U[3][32 * 32];
  const int c = threadIdx.x;
  if (c >= D) return;
  double *a = A[c], *u = U[c];
  for (int i = 0; i < k * k; ++i) { a[i] = 0.0; u[i] = 0.0; }
  for (int i = 0; i < k; ++i) {
    a[i * k + i] = scal[P_AH + i * D + c];
    if (i + 1 < k) a[i * k + i + 1] = a[(i + 1) * k + i] = scal[P_BH + i * D + c];
    u[i * k + i] = 1.0;
  }
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < k; ++i) {
      diag += a[i * k + i] * a[i * k + i];
      for (int j = i + 1; j < k; ++j) off += a[i * k + j] * a[i * k + j];
    }
    if (off <= 1e-30 * diag) break;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = a[p * k + q];
        if (fabs(apq) < 1e-300) continue;
        const double tau = (a[q * k + q] - a[p * k + p]) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
        for (int r = 0; r < k; ++r) {
          const double arp = a[r * k + p], arq = a[r * k + q];
          a[r * k + p] = cs * arp - sn * arq;
          a[r * k + q] = sn * arp + cs * arq;
        }
        for (int r = 0; r < k; ++r) {
          const double apr = a[p * k + r], aqr = a[q * k + r];
          a[p * k + r] = cs * apr - sn * aqr;
          a[q * k + r] = sn * apr + cs * aqr;
        }
        for (int r = 0; r < k; ++r) {
          const double urp = u[r * k + p], urq = u[r * k + q];
          u[r * k + p] = cs * urp - sn * urq;
          u[r * k + q] = sn * urp + cs * urq;
        }
      }
  }
  const double b0 = sqrt(fmax(scal[P_B0 + c], 0.0));
  for (int i = 0; i < k; ++i) {
    double y = 0.0;
    for (int j = 0; j < k; ++j) {
      y += u[i * k + j] * lanczos_fn(fkind, pw, a[j * k + j]) * u[0 * k + j];
    }
    scal[P_CO + i * D + c] = b0 * y;
  }
}

}  // namespace

// --------------------------------------------------------------------------
// Host: geometry of the skeleton
// --------------------------------------------------------------------------

// Dense SPD inverse by Cholesky (m <= kMaxFace); returns false if a pivot
// is not positive or has lost all but 1e-10 of its diagonal entry (a
// semidefinite block, whose last pivot is rounding noise).
static bool spd_inverse(int m, std::vector<double> &A) {
  std::vector<double> L(A);
  for (int j = 0; j < m; ++j) {
    double d = L[j * m + j];
    const double diag = d;
    for (int k = 0; k < j; ++k) d -= L[j * m + k] * L[j * m + k];
    if (!(d > 1e-10 * diag)) return false;
    d = std::sqrt(d);
    L[j * m + j] = d;
    for (int i = j + 1; i < m; ++i) {
      double s = L[i * m + j];
      for (int k = 0; k < j; ++k) s -= L[i * m + k] * L[j * m + k];
      L[i * m + j] = s / d;
    }
  }
  // solve L L^T X = I column by column
  std::vector<double> col(m);
  for (int c = 0; c < m; ++c) {
    for (int i = 0; i < m; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= L[i * m + k] * col[k];
      col[i] = s / L[i * m + i];
    }
    for (int i = m - 1; i >= 0; --i) {
      double s = col[i];
      for (int k = i + 1; k < m; ++k) s -= L[k * m + i] * col[k];
      col[i] = s / L[i * m + i];
    }
    for (int i = 0; i < m; ++i) A[i * m + c] = col[i];
  }
  return true;
}

// Element matrices of the skeleton by 2-point Gauss quadrature: 1D linear
// segment (2D problems) or bilinear unit square (3D problems).
static void skeleton_element_matrices(int dim, double *Le, double *Me) {
  const double g[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  if (dim == 2) {
    for (int i = 0; i < 4; ++i) Le[i] = Me[i] = 0.0;
    for (int q = 0; q < 2; ++q) {
      const double N[2] = {1.0 - g[q], g[q]}, dN[2] = {-1.0, 1.0};
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          Le[a * 2 + b] += 0.5 * dN[a] * dN[b];
          Me[a * 2 + b] += 0.5 * N[a] * N[b];
        }
    }
    return;
  }
  const int ox[4] = {0, 1, 1, 0}, oy[4] = {0, 0, 1, 1};
  for (int i = 0; i < 16; ++i) Le[i] = Me[i] = 0.0;
  for (int qa = 0; qa < 2; ++qa)
    for (int qb = 0; qb < 2; ++qb) {
      const double s = g[qa], t = g[qb];
      double N[4], Gs[4], Gt[4];
      for (int a = 0; a < 4; ++a) {
        const double fs = ox[a] ? s : 1.0 - s, ft = oy[a] ? t : 1.0 - t;
        N[a] = fs * ft;
        Gs[a] = (ox[a] ? 1.0 : -1.0) * ft;
        Gt[a] = fs * (oy[a] ? 1.0 : -1.0);
      }
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          Le[a * 4 + b] += 0.25 * (Gs[a] * Gs[b] + Gt[a] * Gt[b]);
          Me[a * 4 + b] += 0.25 * N[a] * N[b];
        }
    }
}

namespace {
void jacobi_eig(int k, std::vector<double> &A, std::vector<double> &U, std::vector<double> &lam);
}  // namespace

int precond_setup(edd_problem *p) {
  const int D = p->g.dim;
  const int64_t nG = p->n_gamma;
  if (nG == 0) return EDD_OK;
  const int npe = D == 2 ? 2 : 4;
  p->sk_npe = npe;
  skeleton_element_matrices(D, p->sk_Le, p->sk_Me);
  const double *Me = p->sk_Me;
  p->sk_rowsum = 0.0;
  for (int b = 0; b < npe; ++b) p->sk_rowsum += Me[b];  // equal for every row
  {
    // spectrum of diag(M)^{-1} M for the consistent mass: every element's
    // generalised eigenvalues of (Me, diag(Me)) bound it, for any positive
    // element weights and with clamped rows removed (Rayleigh quotients of
    // sums of element forms); widened by a hair against rounding
    std::vector<double> A((size_t)npe * npe), U, lam;
    for (int a = 0; a < npe; ++a)
      for (int b = 0; b < npe; ++b)
        A[a * npe + b] = Me[a * npe + b] / std::sqrt(Me[a * npe + a] * Me[b * npe + b]);
    jacobi_eig(npe, A, U, lam);
    p->sk_cheb_lo = *std::min_element(lam.begin(), lam.end()) * (1.0 - 1e-9);
    p->sk_cheb_hi = *std::max_element(lam.begin(), lam.end()) * (1.0 + 1e-9);
  }
  const auto &nn = p->g.nn;
  auto nid = [&](int x, int y, int z) -> int64_t {
    return x + (int64_t)nn[0] * (y + (int64_t)nn[1] * z);
  };
  auto eid = [&](int x, int y, int z) -> int64_t {
    return x + (int64_t)p->g.nel[0] * (y + (int64_t)p->g.nel[1] * z);
  };
  // skeleton elements and their two neighbouring volume elements
  std::vector<int> sk_nodes, sk_adj;
  for (int ax = 0; ax < D; ++ax) {
    const auto &cuts = p->cuts[ax];
    for (size_t ci = 1; ci + 1 < cuts.size(); ++ci) {
      const int c = cuts[ci];
      if (D == 2) {
        const int o = 1 - ax;
        for (int t = 0; t < p->g.nel[o]; ++t) {
          int a0[3] = {0, 0, 0}, a1[3] = {0, 0, 0};
          a0[ax] = c; a0[o] = t;
          a1[ax] = c; a1[o] = t + 1;
          sk_nodes.push_back((int)nid(a0[0], a0[1], 0));
          sk_nodes.push_back((int)nid(a1[0], a1[1], 0));
          int e0[3] = {0, 0, 0}, e1[3] = {0, 0, 0};
          e0[ax] = c - 1; e0[o] = t;
          e1[ax] = c; e1[o] = t;
          sk_adj.push_back((int)eid(e0[0], e0[1], 0));
          sk_adj.push_back((int)eid(e1[0], e1[1], 0));
        }
      } else {
        int o1 = -1, o2 = -1;
        for (int a = 0; a < 3; ++a)
          if (a != ax) { if (o1 < 0) o1 = a; else o2 = a; }
        const int dp[4] = {0, 1, 1, 0}, dq[4] = {0, 0, 1, 1};
        for (int pp = 0; pp < p->g.nel[o1]; ++pp)
          for (int qq = 0; qq < p->g.nel[o2]; ++qq) {
            for (int k = 0; k < 4; ++k) {
              int x[3];
              x[ax] = c; x[o1] = pp + dp[k]; x[o2] = qq + dq[k];
              sk_nodes.push_back((int)nid(x[0], x[1], x[2]));
            }
            int e0[3], e1[3];
            e0[o1] = e1[o1] = pp; e0[o2] = e1[o2] = qq;
            e0[ax] = c - 1; e1[ax] = c;
            sk_adj.push_back((int)eid(e0[0], e0[1], e0[2]));
            sk_adj.push_back((int)eid(e1[0], e1[1], e1[2]));
          }
      }
    }
  }
  const int64_t nsk = (int64_t)sk_adj.size() / 2;
  p->sk_n = nsk;
  auto gidx = [&](int node) -> int {
    const int code = p->nmap_host[node];
    return (code <= -2) ? gamma_index(code) : -1;
  };
  // CSR of L over gamma indices with the contribution list of every entry
  struct Tup { int r, c, e, ab; };
  std::vector<Tup> tup;
  tup.reserve(nsk * npe * npe);
  std::vector<std::vector<int>> node_elems(nG);
  for (int64_t e = 0; e < nsk; ++e) {
    int g[4];
    for (int a = 0; a < npe; ++a) g[a] = gidx(sk_nodes[e * npe + a]);
    for (int a = 0; a < npe; ++a) {
      if (g[a] < 0) continue;
      node_elems[g[a]].push_back((int)e);
      for (int b = 0; b < npe; ++b)
        if (g[b] >= 0) tup.push_back({g[a], g[b], (int)e, a * npe + b});
    }
  }
  std::sort(tup.begin(), tup.end(), [](const Tup &x, const Tup &y) {
    return x.r != y.r ? x.r < y.r : x.c < y.c;
  });
  std::vector<int> rowptr(nG + 1, 0), col, cptr, celem, cab;
  std::vector<double> l0;  // unweighted values
  for (size_t t = 0; t < tup.size(); ++t) {
    const bool fresh = t == 0 || tup[t].r != tup[t - 1].r || tup[t].c != tup[t - 1].c;
    if (fresh) {
      col.push_back(tup[t].c);
      cptr.push_back((int)celem.size());
      l0.push_back(0.0);
      rowptr[tup[t].r + 1]++;
    }
    celem.push_back(tup[t].e);
    cab.push_back(tup[t].ab);
    l0.back() += p->sk_Le[tup[t].ab];
  }
  cptr.push_back((int)celem.size());
  for (int64_t i = 0; i < nG; ++i) rowptr[i + 1] += rowptr[i];
  const int64_t nnz = (int64_t)col.size();
  p->sk_nnz = nnz;
  std::vector<double> l0diag(nG, 0.0);
  for (int64_t i = 0; i < nG; ++i)
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
      if (col[k] == i) l0diag[i] = l0[k];
  std::vector<int> nptr(nG + 1, 0), nelem;
  for (int64_t i = 0; i < nG; ++i) {
    nptr[i + 1] = nptr[i] + (int)node_elems[i].size();
    nelem.insert(nelem.end(), node_elems[i].begin(), node_elems[i].end());
  }

  // faces: gamma nodes lying on exactly one internal cut, grouped by the cut
  // and by the block they sit in along the other axes; the rest are cross
  // points (and wire-basket edges in 3D)
  std::vector<std::vector<char>> is_cut(3);
  for (int a = 0; a < 3; ++a) {
    is_cut[a].assign(nn[a], 0);
    if (a < D)
      for (size_t c = 1; c + 1 < p->cuts[a].size(); ++c) is_cut[a][p->cuts[a][c]] = 1;
  }
  auto block_of = [&](int a, int x) {
    const auto &cuts = p->cuts[a];
    int b = (int)(std::upper_bound(cuts.begin(), cuts.end(), x) - cuts.begin()) - 1;
    return std::min(b, (int)cuts.size() - 2);
  };
  std::map<std::vector<int>, int> face_id;
  std::vector<std::vector<int>> faces;
  std::vector<int> rest;
  for (int64_t gi = 0; gi < nG; ++gi) {
    const int node = p->gnode[gi];
    int x[3];
    x[0] = node % nn[0];
    x[1] = (node / nn[0]) % nn[1];
    x[2] = node / (nn[0] * nn[1]);
    int ncut = 0, cax = -1;
    for (int a = 0; a < D; ++a)
      if (is_cut[a][x[a]]) { ++ncut; cax = a; }
    if (ncut != 1) { rest.push_back((int)gi); continue; }
    std::vector<int> key = {cax, x[cax]};
    for (int a = 0; a < D; ++a)
      if (a != cax) key.push_back(block_of(a, x[a]));
    auto it = face_id.find(key);
    if (it == face_id.end()) {
      it = face_id.emplace(key, (int)faces.size()).first;
      faces.emplace_back();
    }
    faces[it->second].push_back((int)gi);
  }
  // faces too large for a dense block join the diagonal part
  std::vector<std::vector<int>> kept;
  for (auto &f : faces) {
    if ((int)f.size() > kMaxFace) rest.insert(rest.end(), f.begin(), f.end());
    else kept.push_back(std::move(f));
  }
  faces.swap(kept);
  std::sort(rest.begin(), rest.end());
  // dense unweighted blocks, one inverse per distinct block
  std::unordered_map<size_t, std::vector<int>> by_hash;  // hash -> class ids
  std::vector<std::vector<double>> class_mat, class_inv;
  std::vector<int> fptr(1, 0), fnode, fclass;
  for (auto &f : faces) {
    const int m = (int)f.size();
    std::vector<double> A((size_t)m * m, 0.0);
    std::unordered_map<int, int> pos;
    for (int i = 0; i < m; ++i) pos[f[i]] = i;
    for (int i = 0; i < m; ++i)
      for (int k = rowptr[f[i]]; k < rowptr[f[i] + 1]; ++k) {
        auto it = pos.find(col[k]);
        if (it != pos.end()) A[(size_t)i * m + it->second] = l0[k];
      }
    const std::string bytes((const char *)A.data(), A.size() * sizeof(double));
    const size_t h = std::hash<std::string>()(bytes) ^ (size_t)m;
    int cls = -1;
    for (int c : by_hash[h])
      if (class_mat[c] == A) { cls = c; break; }
    if (cls < 0) {
      std::vector<double> inv(A);
      if (!spd_inverse(m, inv)) {
        // a face with no cross point and no clamped neighbour (a skeleton
        // that does not meet the clamp): its block of L is the singular
        // Neumann Laplacian, so this face is preconditioned by the inverse
        // diagonal instead
        std::fill(inv.begin(), inv.end(), 0.0);
        for (int i = 0; i < m; ++i) {
          if (!(A[(size_t)i * m + i] > 0.0)) return EDD_EINVAL;
          inv[(size_t)i * m + i] = 1.0 / A[(size_t)i * m + i];
        }
      }
      cls = (int)class_mat.size();
      class_mat.push_back(A);
      class_inv.push_back(std::move(inv));
      by_hash[h].push_back(cls);
    }
    fclass.push_back(cls);
    fnode.insert(fnode.end(), f.begin(), f.end());
    fptr.push_back((int)fnode.size());
    p->max_face_m = std::max(p->max_face_m, m);
  }
  std::vector<int64_t> coff;
  std::vector<double> inv_all;
  for (auto &ci : class_inv) {
    coff.push_back((int64_t)inv_all.size());
    inv_all.insert(inv_all.end(), ci.begin(), ci.end());
  }
  p->n_faces = (int)faces.size();
  p->n_face_classes = (int)class_inv.size();
  // Workgroup b of a face launch runs on XCD b % kXcd (round-robin
  // dispatch).  Faces sorted by class and cut into kXcd contiguous runs, one
  // per XCD, keep each class's dense inverse in the L2 of one or two XCDs
  // instead of streaming every class through every XCD.
  constexpr int kXcd = 8;
  std::vector<int> by_class(p->n_faces);
  std::iota(by_class.begin(), by_class.end(), 0);
  std::stable_sort(by_class.begin(), by_class.end(),
                   [&](int a, int b) { return fclass[a] < fclass[b]; });
  const int per_xcd = (p->n_faces + kXcd - 1) / kXcd;
  std::vector<int> fblk((size_t)kXcd * per_xcd, -1);
  for (int q = 0; q < p->n_faces; ++q)
    fblk[(size_t)(q % per_xcd) * kXcd + q / per_xcd] = by_class[q];
  p->n_face_blocks = (int)fblk.size();
  p->n_rest = (int)rest.size();
  p->face_inv_entries = (int64_t)inv_all.size();

  // device copies
  auto up = [&](void *dst, const void *src, size_t bytes) -> bool {
    if (!bytes) return true;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, p->stream) == hipSuccess;
  };
#define PC_ALLOC(ptr, type, count)                                              \
  do {                                                                          \
    ptr = (type *)dev_alloc(p, sizeof(type) * std::max<size_t>(1, (size_t)(count))); \
    if (!ptr) return EDD_ENOMEM;                                                \
  } while (0)
  PC_ALLOC(p->sk_adj_d, int, sk_adj.size());
  PC_ALLOC(p->sk_w_d, double, nsk);
  PC_ALLOC(p->skL_rowptr_d, int, nG + 1);
  PC_ALLOC(p->skL_col_d, int, nnz);
  PC_ALLOC(p->skL_val_d, double, nnz);
  PC_ALLOC(p->skC_ptr_d, int, nnz + 1);
  PC_ALLOC(p->skC_elem_d, int, celem.size());
  PC_ALLOC(p->skC_ab_d, int, cab.size());
  PC_ALLOC(p->skN_ptr_d, int, nG + 1);
  PC_ALLOC(p->skN_elem_d, int, nelem.size());
  PC_ALLOC(p->skM_d, double, nG);
  PC_ALLOC(p->skMc_val_d, double, nnz);
  PC_ALLOC(p->skMcdiag_d, double, nG);
  PC_ALLOC(p->skLdiag_d, double, nG);
  PC_ALLOC(p->skL0diag_d, double, nG);
  PC_ALLOC(p->skS_d, double, nG);
  PC_ALLOC(p->face_ptr_d, int, fptr.size());
  PC_ALLOC(p->face_node_d, int, fnode.size());
  PC_ALLOC(p->face_class_d, int, fclass.size());
  PC_ALLOC(p->face_blk_d, int, fblk.size());
  PC_ALLOC(p->class_off_d, int64_t, coff.size());
  PC_ALLOC(p->rest_d, int, rest.size());
  PC_ALLOC(p->face_inv_d, double, inv_all.size());
  bool ok = up(p->sk_adj_d, sk_adj.data(), sizeof(int) * sk_adj.size()) &&
            up(p->skL_rowptr_d, rowptr.data(), sizeof(int) * rowptr.size()) &&
            up(p->skL_col_d, col.data(), sizeof(int) * col.size()) &&
            up(p->skC_ptr_d, cptr.data(), sizeof(int) * cptr.size()) &&
            up(p->skC_elem_d, celem.data(), sizeof(int) * celem.size()) &&
            up(p->skC_ab_d, cab.data(), sizeof(int) * cab.size()) &&
            up(p->skN_ptr_d, nptr.data(), sizeof(int) * nptr.size()) &&
            up(p->skN_elem_d, nelem.data(), sizeof(int) * nelem.size()) &&
            up(p->skL0diag_d, l0diag.data(), sizeof(double) * nG) &&
            up(p->face_ptr_d, fptr.data(), sizeof(int) * fptr.size()) &&
            up(p->face_node_d, fnode.data(), sizeof(int) * fnode.size()) &&
            up(p->face_class_d, fclass.data(), sizeof(int) * fclass.size()) &&
            up(p->face_blk_d, fblk.data(), sizeof(int) * fblk.size()) &&
            up(p->class_off_d, coff.data(), sizeof(int64_t) * coff.size()) &&
            up(p->rest_d, rest.data(), sizeof(int) * rest.size()) &&
            up(p->face_inv_d, inv_all.data(), sizeof(double) * inv_all.size());
  if (!ok || hipStreamSynchronize(p->stream) != hipSuccess) return EDD_EHIP;
  for (int i = 0; i < 9; ++i) PC_ALLOC(p->pc_v_d[i], double, nG * D);
  if (hipHostMalloc((void **)&p->pc_h, sizeof(double) * 65 * 3) != hipSuccess)
    return EDD_ENOMEM;
#undef PC_ALLOC
  p->sk_state = -1;
  return EDD_OK;
}

// (re)build the device operators for the requested weighting
static int precond_operators(edd_problem *p, int weighting) {
  if (p->sk_state == weighting) return EDD_OK;
  const int64_t nG = p->n_gamma;
  k_sk_weights<<<grid_for(p->sk_n), kBlock, 0, p->stream>>>(
      p->sk_n, p->sk_adj_d, p->E_d, weighting, p->sk_w_d);
  ElemMat em;
  std::memcpy(em.v, p->sk_Le, sizeof(em.v));
  k_sk_assemble<<<(unsigned)((p->sk_nnz + kBlock - 1) / kBlock), kBlock, 0, p->stream>>>(
      p->sk_nnz, p->skC_ptr_d, p->skC_elem_d, p->skC_ab_d, p->sk_w_d, em, p->skL_val_d);
  k_sk_diag<<<(unsigned)((nG + kBlock - 1) / kBlock), kBlock, 0, p->stream>>>(
      nG, p->skN_ptr_d, p->skN_elem_d, p->sk_w_d, p->sk_rowsum, p->skL_rowptr_d,
      p->skL_col_d, p->skL_val_d, p->skL0diag_d, p->skM_d, p->skLdiag_d, p->skS_d);
  // the consistent mass in the same pattern, from the same contributions
  ElemMat mm;
  std::memcpy(mm.v, p->sk_Me, sizeof(mm.v));
  k_sk_assemble<<<(unsigned)((p->sk_nnz + kBlock - 1) / kBlock), kBlock, 0, p->stream>>>(
      p->sk_nnz, p->skC_ptr_d, p->skC_elem_d, p->skC_ab_d, p->sk_w_d, mm, p->skMc_val_d);
  k_csr_diag<<<(unsigned)((nG + kBlock - 1) / kBlock), kBlock, 0, p->stream>>>(
      nG, p->skL_rowptr_d, p->skL_col_d, p->skMc_val_d, p->skMcdiag_d);
  if (hipGetLastError() != hipSuccess) return EDD_EHIP;
  p->sk_state = weighting;
  return EDD_OK;
}

// --------------------------------------------------------------------------
// Host: application
// --------------------------------------------------------------------------
namespace {

template <int D>
struct PC {
  edd_problem *p;
  int64_t nG;
  unsigned g1;  // one thread per gamma node

  void cdots(int npair, const double *a0, const double *b0, const double *a1,
             const double *b1, const double *wgt, int slot0, int slot1) {
    unsigned g = grid_for(nG);
    if (g > 256) g = 256;
    k_cdots<D><<<g, kBlock, 0, p->stream>>>(nG, npair, a0, b0, a1, b1, wgt, p->partials_d);
    // partials: [blk][npair*D]; reduce each (pair, c)
    k_reduce<<<D, kBlock, 0, p->stream>>>(p->partials_d, (int)g, npair * D, p->scal_d + slot0);
    if (npair > 1)
      k_reduce<<<D, kBlock, 0, p->stream>>>(p->partials_d + D, (int)g, npair * D,
                                            p->scal_d + slot1);
  }

  void face_precond(const double *r, double *z) {
    if (p->n_faces)
      k_face_apply<D><<<p->n_face_blocks, 256 * kFaceQ, 0, p->stream>>>(
          p->face_blk_d, p->face_ptr_d, p->face_node_d, p->face_class_d, p->class_off_d, p->face_inv_d,
          p->skS_d, r, z);
    if (p->n_rest)
      k_rest_apply<D><<<(unsigned)((p->n_rest + kBlock - 1) / kBlock), kBlock, 0, p->stream>>>(
          p->n_rest, p->rest_d, p->skLdiag_d, r, z);
  }

  // One Lanczos operator step on q: w = L^{-1} M q by the face-block PCG
  // (inverse Lanczos) or w = M^{-1} L q (forward Lanczos, no inner solve);
  // with the consistent mass, mq = M q is given and M^{-1} is the Chebyshev
  // iteration; t is work space.
  int lanczos_operator(const double *q, const double *mq, double *t, double *w, bool forward,
                       double tol, int maxit, edd_solve_stats *st) {
    if (forward) {
      spmv(q, t);
      if (mq) mass_solve(t, w);
      else k_cscale<D><<<g1, kBlock, 0, p->stream>>>(nG, p->scal_d, 0, 3, p->skM_d, t, w);
      return EDD_OK;
    }
    if (!mq) {
      k_dscale<D><<<g1, kBlock, 0, p->stream>>>(nG, p->skM_d, q, t);
      mq = t;
    }
    int its = 0;
    int rc = inner_pcg(mq, w, tol, maxit, &its);
    if (st) st->inner_iterations += its;
    return rc;
  }

  // y = M x, the consistent skeleton mass
  void mass_apply(const double *x, double *y) {
    k_spmv<D><<<g1, kBlock, 0, p->stream>>>(nG, p->skL_rowptr_d, p->skL_col_d, p->skMc_val_d,
                                             x, y);
  }

  // x ~ M^{-1} b for the consistent mass: a fixed number of Chebyshev steps
  // (no host synchronisation), enough for an M-norm error bound of 1e-12
  // from the spectrum bounds of diag(M)^{-1} M (error factor
  // 2 s^k / (1 + s^{2k}), s = (sqrt(kappa) - 1) / (sqrt(kappa) + 1))
  void mass_solve(const double *b, double *x) {
    double *r = p->pc_v_d[2], *d0 = p->pc_v_d[7], *d1 = p->pc_v_d[8];
    const double lo = p->sk_cheb_lo, hi = p->sk_cheb_hi;
    const double th = 0.5 * (hi + lo), de = 0.5 * (hi - lo);
    const double sk = std::sqrt(hi / lo), sg = (sk - 1.0) / (sk + 1.0);
    const int steps = std::min(200, (int)std::ceil(std::log(2.0 / 1e-12) / std::log(1.0 / sg)));
    k_cheb_init<D><<<g1, kBlock, 0, p->stream>>>(nG, p->skMcdiag_d, 1.0 / th, b, x, r, d0);
    double rho = de / th;
    for (int it = 0; it < steps; ++it) {
      const double rn = 1.0 / (2.0 * th / de - rho);
      k_cheb_step<D><<<g1, kBlock, 0, p->stream>>>(nG, p->skL_rowptr_d, p->skL_col_d,
                                                    p->skMc_val_d, p->skMcdiag_d, d0, d1, x, r,
                                                    rn * rho, 2.0 * rn / de);
      rho = rn;
      std::swap(d0, d1);
    }
  }

  void spmv(const double *x, double *y) {
    k_spmv<D><<<g1, kBlock, 0, p->stream>>>(nG, p->skL_rowptr_d, p->skL_col_d, p->skL_val_d,
                                             x, y);
  }

  // y ~ L^{-1} b (all components), relative tolerance tol; with tol <= 0
  // exactly maxit iterations run with no host synchronisation
  // face-block preconditioner fused with the PCG update and r.z sums; the
  // reduced sums land in scal[out_slot + c]
  template <bool INIT>
  void face_pcg(int rz, double *y, const double *pv, double *r, const double *q, double *z,
                double *pdir, int out_slot) {
    const unsigned nrb = rest_blocks();
    if (small_faces()) {
      const int nsb = (p->n_faces + 3) / 4;
      k_face_pcg_small<D, INIT><<<nsb + nrb, 256, 0, p->stream>>>(
          p->face_ptr_d, p->face_node_d, p->face_class_d, p->class_off_d, p->face_inv_d,
          p->skS_d, p->scal_d, rz, P_PQ, y, pv, r, q, z, pdir, p->partials_d, p->n_faces, nsb,
          p->n_rest, p->rest_d, p->skLdiag_d);
    } else {
      const int nfb = p->n_faces ? p->n_face_blocks : 0;
      k_face_pcg<D, INIT><<<nfb + nrb, 256 * kFaceQ, 0, p->stream>>>(
          p->face_blk_d, p->face_ptr_d, p->face_node_d, p->face_class_d, p->class_off_d,
          p->face_inv_d, p->skS_d, p->scal_d, rz, P_PQ, y, pv, r, q, z, pdir, p->partials_d,
          nfb, p->n_faces, p->n_rest, p->rest_d, p->skLdiag_d);
    }
    if (out_slot >= 0)
      k_reduce<<<D, kBlock, 0, p->stream>>>(p->partials_d, (int)(p->n_faces + (p->n_rest ? nrb : 0)),
                                            D, p->scal_d + out_slot);
  }

  // grids of the fused kernels (grid-stride loops, so capped); the fused
  // path needs one partial sum per block and component
  // faces of at most 64 nodes take the one-wavefront-per-face kernel
  bool small_faces() const { return p->max_face_m <= 64; }
  unsigned rest_blocks() const {
    const int nt = small_faces() ? 256 : 256 * kFaceQ;
    return (unsigned)std::min<int64_t>((p->n_rest + nt - 1) / nt, 1024);
  }
  unsigned spmv_blocks() const { return std::min(g1, 4096u); }
  bool fused_fits() const {
    const size_t need = std::max<size_t>((size_t)p->n_faces + rest_blocks(), spmv_blocks());
    return p->n_faces + p->n_rest > 0 && need * D <= p->partials_len;
  }

  // y ~ L^{-1} b, exactly maxit PCG iterations with no host synchronisation:
  // six launches per iteration (L apply with p.q sums, their reduction, the
  // fused update / face blocks / r.z sums (two kernels and a reduction),
  // the new direction); r.z alternates between two scalar slots.
  int inner_pcg_fixed(const double *b, double *y, int maxit, int *its_out) {
    double *r = p->pc_v_d[3], *z = p->pc_v_d[4], *pv = p->pc_v_d[5], *q = p->pc_v_d[6];
    launch_fill(p, nG * D, 0.0, y);
    k_copy<<<g1, kBlock, 0, p->stream>>>(nG * D, b, r);
    face_pcg<true>(0, y, pv, r, q, z, pv, P_RZ);
    int cur = P_RZ, nxt = P_RZN;
    for (int it = 0; it < maxit; ++it) {
      k_spmv_dot<D><<<spmv_blocks(), kBlock, 0, p->stream>>>(
          nG, p->skL_rowptr_d, p->skL_col_d, p->skL_val_d, pv, q, p->partials_d);
      k_reduce<<<D, kBlock, 0, p->stream>>>(p->partials_d, (int)spmv_blocks(), D,
                                            p->scal_d + P_PQ);
      const bool last = it + 1 == maxit;
      face_pcg<false>(cur, y, pv, r, q, z, nullptr, last ? -1 : nxt);
      if (last) break;
      k_pcg_dir2<D><<<g1, kBlock, 0, p->stream>>>(nG, p->scal_d, nxt, cur, z, pv);
      std::swap(cur, nxt);
    }
    *its_out = maxit;
    return hipGetLastError() == hipSuccess ? EDD_OK : EDD_EHIP;
  }

  int inner_pcg(const double *b, double *y, double tol, int maxit, int *its_out) {
    if (tol <= 0.0 && fused_fits()) return inner_pcg_fixed(b, y, maxit, its_out);
    double *r = p->pc_v_d[3], *z = p->pc_v_d[4], *pv = p->pc_v_d[5], *q = p->pc_v_d[6];
    launch_fill(p, nG * D, 0.0, y);
    k_copy<<<g1, kBlock, 0, p->stream>>>(nG * D, b, r);
    face_precond(r, z);
    k_copy<<<g1, kBlock, 0, p->stream>>>(nG * D, z, pv);
    cdots(2, r, z, b, b, nullptr, P_RZ, P_BB);
    int it = 0;
    for (; it < maxit; ++it) {
      spmv(pv, q);
      cdots(1, pv, q, nullptr, nullptr, nullptr, P_PQ, 0);
      k_pcg_update<D><<<g1, kBlock, 0, p->stream>>>(nG, p->scal_d, y, pv, r, q);
      face_precond(r, z);
      if (tol > 0.0) {
        cdots(2, r, z, r, r, nullptr, P_RZN, P_RR);
        int rc = read_scalars(p, P_RZ, 15);
        if (rc) return rc;
        const double *s = p->scal_h;
        bool done = true;
        for (int c = 0; c < D; ++c)
          if (s[P_RR + c] > tol * tol * s[P_BB + c]) done = false;
        if (done) { ++it; break; }
      } else {
        if (it + 1 == maxit) { ++it; break; }
        cdots(1, r, z, nullptr, nullptr, nullptr, P_RZN, 0);
      }
      k_pcg_dir<D><<<g1, kBlock, 0, p->stream>>>(nG, p->scal_d, z, pv);
      k_copy_scal<<<1, 64, 0, p->stream>>>(p->scal_d, P_RZ, P_RZN, D);
    }
    *its_out = it;
    return hipGetLastError() == hipSuccess ? EDD_OK : EDD_EHIP;
  }
};

// eigen-decomposition of a small symmetric matrix by cyclic Jacobi
// rotations; A (k x k, row-major) is destroyed, U holds eigenvectors
void jacobi_eig(int k, std::vector<double> &A, std::vector<double> &U,
                std::vector<double> &lam) {
  U.assign((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) U[i * k + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < k; ++i)
      for (int j = i + 1; j < k; ++j) off += A[i * k + j] * A[i * k + j];
    if (off < 1e-30) break;
    for (int pI = 0; pI < k; ++pI)
      for (int q = pI + 1; q < k; ++q) {
        const double apq = A[pI * k + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = A[pI * k + pI], aqq = A[q * k + q];
        const double tau = (aqq - app) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int r = 0; r < k; ++r) {
          const double arp = A[r * k + pI], arq = A[r * k + q];
          A[r * k + pI] = c * arp - s * arq;
          A[r * k + q] = s * arp + c * arq;
        }
        for (int r = 0; r < k; ++r) {
          const double apr = A[pI * k + r], aqr = A[q * k + r];
          A[pI * k + r] = c * apr - s * aqr;
          A[q * k + r] = s * apr + c * aqr;
        }
        for (int r = 0; r < k; ++r) {
          const double urp = U[r * k + pI], urq = U[r * k + q];
          U[r * k + pI] = c * urp - s * urq;
          U[r * k + q] = s * urp + c * urq;
        }
      }
  }
  lam.resize(k);
  for (int i = 0; i < k; ++i) lam[i] = A[i * k + i];
}

// y = beta0 * f(T) e1 for the symmetric tridiagonal T (alpha, beta), f as
// lanczos_fn(fkind, pw, .)
void tridiag_power(int k, const double *alpha, const double *beta, int fkind, double pw,
                   double beta0, std::vector<double> &y) {
  std::vector<double> A((size_t)k * k, 0.0), U, lam;
  for (int i = 0; i < k; ++i) {
    A[i * k + i] = alpha[i];
    if (i + 1 < k) A[i * k + i + 1] = A[(i + 1) * k + i] = beta[i];
  }
  jacobi_eig(k, A, U, lam);
  y.assign(k, 0.0);
  for (int j = 0; j < k; ++j) {
    const double f = lanczos_fn(fkind, pw, lam[j]) * U[0 * k + j];
    for (int i = 0; i < k; ++i) y[i] += beta0 * U[i * k + j] * f;
  }
}

// Fixed number of Lanczos steps and inner iterations; every scalar stays on
// the device (no host synchronisation), so the whole application is one
// asynchronous stream of kernels.
// Lanczos basis Q and, for the consistent mass, MQ = M Q: kk vectors each
int ensure_basis(edd_problem *p, int kk) {
  if (p->pc_kcap >= kk) return EDD_OK;
  const size_t bytes = sizeof(double) * p->n_gamma * p->g.dim * kk;
  double *Q = (double *)dev_alloc(p, bytes), *MQ = (double *)dev_alloc(p, bytes);
  if (!Q || !MQ) return EDD_ENOMEM;
  p->pc_Q_d = Q;
  p->pc_MQ_d = MQ;
  p->pc_kcap = kk;
  return EDD_OK;
}

// The start of the Lanczos process in the M inner product: b = M^{-1} r,
// P_B0 = |b|_M^2, q_0 = b / |b|_M into Q; with the consistent mass |b|_M^2 =
// b.r and M q_0 = r / |b|_M into MQ.  t receives b.
template <int D>
void lanczos_start(PC<D> &pc, bool cm, const double *r, double *t, double *Q, double *MQ) {
  edd_problem *p = pc.p;
  if (cm) {
    pc.mass_solve(r, t);
    pc.cdots(1, t, r, nullptr, nullptr, nullptr, P_B0, 0);
    k_cscale<D><<<pc.g1, kBlock, 0, p->stream>>>(pc.nG, p->scal_d, P_B0, 1, nullptr, r, MQ);
  } else {
    k_cscale<D><<<pc.g1, kBlock, 0, p->stream>>>(pc.nG, p->scal_d, 0, 3, p->skM_d, r, t);
    pc.cdots(1, t, t, nullptr, nullptr, p->skM_d, P_B0, 0);
  }
  k_cscale<D><<<pc.g1, kBlock, 0, p->stream>>>(pc.nG, p->scal_d, P_B0, 1, nullptr, t, Q);
}

// The M inner products of a Lanczos step.  Lumped M: weighted dots.
// Consistent M: dots with the stored M q_i (alpha, reorthogonalisation) and
// |w|_M^2 = w.(M w) with M w into mw (the next M q up to the scale).
template <int D>
void lanczos_alpha(PC<D> &pc, bool cm, const double *qj, const double *mqj, const double *w) {
  if (cm) pc.cdots(1, mqj, w, nullptr, nullptr, nullptr, P_A, 0);
  else pc.cdots(1, qj, w, nullptr, nullptr, pc.p->skM_d, P_A, 0);
}

template <int D>
void lanczos_beta(PC<D> &pc, bool cm, const double *w, double *mw) {
  if (cm) {
    pc.mass_apply(w, mw);
    pc.cdots(1, w, mw, nullptr, nullptr, nullptr, P_B, 0);
  } else {
    pc.cdots(1, w, w, nullptr, nullptr, pc.p->skM_d, P_B, 0);
  }
}

template <int D>
int apply_device(edd_problem *p, const double *r, double *z, const edd_solve_opts *o,
                 edd_solve_stats *st) {
  const int64_t nG = p->n_gamma;
  PC<D> pc{p, nG, (unsigned)((nG + kBlock - 1) / kBlock)};
  const double theta = o->theta >= 0.0 ? o->theta : p->theta_default;
  const int k = std::min(o->lanczos_kmax, 32);
  if (int rc = ensure_basis(p, k + 1)) return rc;
  const int64_t n = nG * D;
  const bool cm = o->mass_matrix == 1;
  double *Q = p->pc_Q_d, *MQ = p->pc_MQ_d;
  double *w = p->pc_v_d[0], *t = p->pc_v_d[1];
  lanczos_start<D>(pc, cm, r, t, Q, MQ);
  const bool fwd = pc_forward(o);
  for (int j = 0; j < k; ++j) {
    double *qj = Q + (int64_t)j * n, *mqj = cm ? MQ + (int64_t)j * n : nullptr;
    int rc = pc.lanczos_operator(qj, mqj, t, w, fwd, 0.0, o->inner_maxit, st);
    if (rc) return rc;
    lanczos_alpha<D>(pc, cm, qj, mqj, w);
    k_lanczos3<D><<<pc.g1, kBlock, 0, p->stream>>>(nG, p->scal_d, qj,
                                                   j > 0 ? Q + (int64_t)(j - 1) * n : nullptr, w);
    unsigned g = grid_for(nG);
    if (g > 128) g = 128;
    k_cwindow_dots<D><<<g, kBlock, 0, p->stream>>>(nG, j + 1, cm ? MQ : Q, w,
                                                   cm ? nullptr : p->skM_d, p->partials_d);
    k_reduce<<<(j + 1) * D, kBlock, 0, p->stream>>>(p->partials_d, (int)g, (j + 1) * D,
                                                    p->scal_d + P_H);
    k_ccombine<D><<<pc.g1, kBlock, 0, p->stream>>>(nG, j + 1, Q, p->scal_d + P_H, 1.0, -1.0, w);
    lanczos_beta<D>(pc, cm, w, t);
    k_store_ab<<<1, 64, 0, p->stream>>>(p->scal_d, j, D);
    if (j + 1 < k) {
      k_cscale<D><<<pc.g1, kBlock, 0, p->stream>>>(nG, p->scal_d, P_B, 1, nullptr, w,
                                                   Q + (int64_t)(j + 1) * n);
      if (cm)
        k_cscale<D><<<pc.g1, kBlock, 0, p->stream>>>(nG, p->scal_d, P_B, 1, nullptr, t,
                                                     MQ + (int64_t)(j + 1) * n);
    }
    if (st) st->lanczos_steps++;
  }
  k_lanczos_coef<<<1, 64, 0, p->stream>>>(p->scal_d, k, D, pc_fkind(o), 1.0 - theta);
  k_ccombine<D><<<pc.g1, kBlock, 0, p->stream>>>(nG, k, Q, p->scal_d + P_CO, 0.0, 1.0, z);
  if (st) st->precond_applications++;
  return hipGetLastError() == hipSuccess ? EDD_OK : EDD_EHIP;
}

// The device-resident apply is a fixed sequence of kernels for given
// (r, z, k, inner steps, theta, weighting): captured once into a HIP graph
// (on a private stream, so the caller's stream may be the null stream) and
// replayed.  Any capture failure falls back to launching the kernels.
template <int D>
int apply_graph(edd_problem *p, const double *r, double *z, const edd_solve_opts *o,
                edd_solve_stats *st) {
  const int64_t nG = p->n_gamma;
  const int k = std::min(o->lanczos_kmax, 32);
  const double theta = o->theta >= 0.0 ? o->theta : p->theta_default;
  const PcGraphKey key{r,     z,           k, o->inner_maxit, o->interface_weighting ? 1 : 0,
                       theta, o->pc_form, o->mass_matrix};
  if (!p->pc_graph || !(p->pc_graph_key == key)) {
    if (p->pc_graph) {
      hipGraphExecDestroy(p->pc_graph);
      p->pc_graph = nullptr;
    }
    if (int rc = ensure_basis(p, k + 1)) return rc;  // allocate before capturing
    if (!p->cap_stream &&
        hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess) {
      p->cap_stream = nullptr;
      return apply_device<D>(p, r, z, o, st);
    }
    hipStream_t saved = p->stream;
    const bool kt = p->kt_enabled;
    p->kt_enabled = false;
    p->stream = p->cap_stream;
    hipGraph_t graph = nullptr;
    int rc = EDD_EHIP;
    if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      rc = apply_device<D>(p, r, z, o, nullptr);
      if (hipStreamEndCapture(p->cap_stream, &graph) != hipSuccess) rc = EDD_EHIP;
    }
    p->stream = saved;
    p->kt_enabled = kt;
    if (rc == EDD_OK && graph &&
        hipGraphInstantiate(&p->pc_graph, graph, nullptr, nullptr, 0) != hipSuccess)
      p->pc_graph = nullptr;
    if (graph) hipGraphDestroy(graph);
    (void)hipGetLastError();
    if (!p->pc_graph) return apply_device<D>(p, r, z, o, st);
    p->pc_graph_key = key;
  }
  if (hipGraphLaunch(p->pc_graph, p->stream) != hipSuccess) return EDD_EHIP;
  if (st) {
    if (!pc_forward(o)) st->inner_iterations += k * o->inner_maxit;
    st->lanczos_steps += k;
    st->precond_applications++;
  }
  return EDD_OK;
}

template <int D>
int apply_t(edd_problem *p, const double *r, double *z, const edd_solve_opts *o,
            edd_solve_stats *st) {
  if (o->lanczos_tol <= 0.0 && o->inner_tol <= 0.0)
    return o->use_graphs ? apply_graph<D>(p, r, z, o, st) : apply_device<D>(p, r, z, o, st);
  const int64_t nG = p->n_gamma;
  PC<D> pc{p, nG, (unsigned)((nG + kBlock - 1) / kBlock)};
  const double theta = o->theta >= 0.0 ? o->theta : p->theta_default;
  const int kmax = o->lanczos_kmax;
  if (int rc = ensure_basis(p, kmax + 1)) return rc;
  const int64_t n = nG * D;
  const bool cm = o->mass_matrix == 1;
  double *Q = p->pc_Q_d, *MQ = p->pc_MQ_d;
  double *w = p->pc_v_d[0], *t = p->pc_v_d[1];
  // b = M^{-1} r ; beta0 = |b|_M ; q0 = b / beta0
  lanczos_start<D>(pc, cm, r, t, Q, MQ);
  int rc = read_scalars(p, P_B0, D);
  if (rc) return rc;
  double beta0[3] = {0, 0, 0};
  for (int c = 0; c < D; ++c) beta0[c] = std::sqrt(std::max(0.0, p->scal_h[P_B0 + c]));
  std::vector<double> alpha[3], beta[3], yprev[3], ycur[3];
  bool conv[3] = {false, false, false};
  for (int c = 0; c < D; ++c) conv[c] = beta0[c] == 0.0;
  int k = 0;
  const bool fwd = pc_forward(o);
  const int fkind = pc_fkind(o);
  for (int j = 0; j < kmax; ++j) {
    double *qj = Q + (int64_t)j * n, *mqj = cm ? MQ + (int64_t)j * n : nullptr;
    // w = L^{-1} M q_j (inverse Lanczos) or M^{-1} L q_j (forward)
    rc = pc.lanczos_operator(qj, mqj, t, w, fwd, o->inner_tol, o->inner_maxit, st);
    if (rc) return rc;
    // alpha = <q_j, w>_M ; w -= alpha q_j + beta q_{j-1}
    lanczos_alpha<D>(pc, cm, qj, mqj, w);
    k_lanczos3<D><<<pc.g1, kBlock, 0, p->stream>>>(nG, p->scal_d, qj,
                                                   j > 0 ? Q + (int64_t)(j - 1) * n : nullptr, w);
    // full reorthogonalisation against q_0..q_j in the M inner product
    {
      unsigned g = grid_for(nG);
      if (g > 128) g = 128;
      k_cwindow_dots<D><<<g, kBlock, 0, p->stream>>>(nG, j + 1, cm ? MQ : Q, w,
                                                     cm ? nullptr : p->skM_d, p->partials_d);
      k_reduce<<<(j + 1) * D, kBlock, 0, p->stream>>>(p->partials_d, (int)g, (j + 1) * D,
                                                      p->scal_d + P_H);
      k_ccombine<D><<<pc.g1, kBlock, 0, p->stream>>>(nG, j + 1, Q, p->scal_d + P_H, 1.0,
                                                     -1.0, w);
    }
    lanczos_beta<D>(pc, cm, w, t);
    rc = read_scalars(p, P_A, 6);
    if (rc) return rc;
    k = j + 1;
    if (st) st->lanczos_steps++;
    bool all = true;
    double bnext[3];
    for (int c = 0; c < D; ++c) {
      bnext[c] = std::sqrt(std::max(0.0, p->scal_h[P_B + c]));
      alpha[c].push_back(p->scal_h[P_A + c]);
      beta[c].push_back(bnext[c]);
      if (beta0[c] == 0.0) { ycur[c].assign(k, 0.0); continue; }
      tridiag_power(k, alpha[c].data(), beta[c].data(), fkind, 1.0 - theta, beta0[c], ycur[c]);
      if (!conv[c] && j > 0) {
        double dn = 0.0, yn = 0.0;
        for (int i = 0; i < k; ++i) {
          const double pv = i < k - 1 ? yprev[c][i] : 0.0;
          dn += (ycur[c][i] - pv) * (ycur[c][i] - pv);
          yn += ycur[c][i] * ycur[c][i];
        }
        if (std::sqrt(dn) <= o->lanczos_tol * std::sqrt(yn)) conv[c] = true;
      }
      if (bnext[c] <= 1e-14 * beta0[c]) conv[c] = true;
      yprev[c] = ycur[c];
      all = all && conv[c];
    }
    if (all || j + 1 == kmax) break;
    // q_{j+1} = w / beta (beta itself kept for the next three-term step)
    for (int c = 0; c < D; ++c) {
      p->pc_h[c] = bnext[c] > 0.0 ? 1.0 / bnext[c] : 0.0;
      p->pc_h[D + c] = bnext[c];
    }
    hipMemcpyAsync(p->scal_d + P_H, p->pc_h, sizeof(double) * D, hipMemcpyHostToDevice,
                   p->stream);
    hipMemcpyAsync(p->scal_d + P_BETA, p->pc_h + D, sizeof(double) * D,
                   hipMemcpyHostToDevice, p->stream);
    k_cscale<D><<<pc.g1, kBlock, 0, p->stream>>>(nG, p->scal_d, P_H, 0, nullptr, w,
                                                 Q + (int64_t)(j + 1) * n);
    if (cm)
      k_cscale<D><<<pc.g1, kBlock, 0, p->stream>>>(nG, p->scal_d, P_H, 0, nullptr, t,
                                                   MQ + (int64_t)(j + 1) * n);
  }
  // z = Q_k y
  for (int i = 0; i < k; ++i)
    for (int c = 0; c < D; ++c) p->pc_h[i * D + c] = ycur[c].size() > (size_t)i ? ycur[c][i] : 0.0;
  hipMemcpyAsync(p->scal_d + P_H, p->pc_h, sizeof(double) * k * D, hipMemcpyHostToDevice,
                 p->stream);
  k_ccombine<D><<<pc.g1, kBlock, 0, p->stream>>>(nG, k, Q, p->scal_d + P_H, 0.0, 1.0, z);
  if (st) st->precond_applications++;
  return hipGetLastError() == hipSuccess ? EDD_OK : EDD_EHIP;
}

}  // namespace

template <int D>
static int skeleton_op_t(edd_problem *p, int which, const double *x, double *y,
                         double tol, int maxit) {
  const int64_t nG = p->n_gamma;
  PC<D> pc{p, nG, (unsigned)((nG + kBlock - 1) / kBlock)};
  if (which == 0) pc.spmv(x, y);
  else if (which == 1) k_dscale<D><<<pc.g1, kBlock, 0, p->stream>>>(nG, p->skM_d, x, y);
  else if (which == 2) pc.face_precond(x, y);
  else if (which == 4) pc.mass_apply(x, y);
  else if (which == 5) pc.mass_solve(x, y);
  else {
    int its = 0;
    int rc = pc.inner_pcg(x, y, tol, maxit, &its);
    if (rc) return rc;
  }
  return hipGetLastError() == hipSuccess ? EDD_OK : EDD_EHIP;
}

int skeleton_op(edd_problem *p, int which, int weighting, const double *x, double *y,
                double tol, int maxit) {
  if (p->n_gamma == 0) return EDD_OK;
  int rc = precond_operators(p, weighting ? 1 : 0);
  if (rc) return rc;
  return p->g.dim == 2 ? skeleton_op_t<2>(p, which, x, y, tol, maxit)
                       : skeleton_op_t<3>(p, which, x, y, tol, maxit);
}

int precond_apply(edd_problem *p, const double *r, double *z, const edd_solve_opts *o,
                  edd_solve_stats *st, bool low_precision) {
  (void)low_precision;  // the preconditioner always runs in FP64
  if (p->n_gamma == 0) return EDD_OK;
  KTimer kt(p, EDD_KT_PRECOND);
  int rc = precond_operators(p, o->interface_weighting ? 1 : 0);
  if (rc) return rc;
  return p->g.dim == 2 ? apply_t<2>(p, r, z, o, st) : apply_t<3>(p, r, z, o, st);
}

}  // namespace edd

// Batched interior solves: band Cholesky factorisation of every subdomain
// block K_{I_i I_i} and the forward/backward substitutions that apply
// K_II^{-1} (K_II is the direct sum of the subdomain blocks, eq.
// (NumberFive); all 2N+1 subproblems of eq. (3MatSplit2) use these solves).
//
// One workgroup owns one subdomain.  Workgroups are launched largest first
// (the order array), so that round-robin dispatch over the XCDs spreads the
// large blocks evenly.
//
// Factorisation (right-looking, panel width NB): a panel of NB columns and
// the NB + kd rows it touches is held in registers, one window row per
// thread slot; the panel is factorised column by column with two barriers
// per column, written back, and the trailing band triangle is updated in
// chunks of CH columns whose panel rows are staged through LDS.
//
// Substitution (panel width NB): the whole right-hand side of the subdomain
// lives in LDS.  Forward: one wavefront solves the NB x NB diagonal
// triangle with lane shuffles, then all threads apply the panel to the next
// kd rows (coalesced column reads of the band).  Backward: each wavefront
// reduces the dot products of NB columns with the already-known part of x,
// then one wavefront solves the transposed diagonal triangle.
#include "internal.h"

namespace edd {
namespace {

// ---------------------------------------------------------------------------
// Band Cholesky
// ---------------------------------------------------------------------------
template <int NB, int NT, int RPT, int CH>
__global__ __launch_bounds__(NT) void k_band_cholesky(
    const SubDesc *__restrict__ subs, const int *__restrict__ order,
    double *__restrict__ fac, int *__restrict__ info) {
  __shared__ double colbuf[NB];
  __shared__ double chunk[CH][NB + 1];
  const SubDesc s = subs[order[blockIdx.x]];
  const int n = s.n, kd = s.kd, ld = kd + 1;
  double *L = fac + s.fac_off;
  const int tid = threadIdx.x;
  int bad = 0;
  double P[RPT][NB];

  for (int j0 = 0; j0 < n; j0 += NB) {
    const int jn = min(NB, n - j0);
    const int W = min(jn + kd, n - j0);  // window rows (relative to j0)
    // load the panel
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int w = tid + k * NT;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const bool ok = (w < W) && (c < jn) && (w >= c) && (w - c <= kd);
        P[k][c] = ok ? L[(int64_t)(j0 + c) * ld + (w - c)] : 0.0;
      }
    }
    // factorise the panel column by column
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      if (c < jn) {
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          const int w = tid + k * NT;
          if (w >= c && w < jn) colbuf[w] = P[k][c];
        }
        __syncthreads();
        const double piv = colbuf[c];
        if (!(piv > 0.0)) bad = 1;
        const double d = sqrt(piv > 0.0 ? piv : 1.0);
        const double rd = 1.0 / d;
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          const int w = tid + k * NT;
          if (w == c) {
            P[k][c] = d;
          } else if (w > c && w < W) {
            const double l = P[k][c] * rd;
            P[k][c] = l;
#pragma unroll
            for (int c2 = c + 1; c2 < NB; ++c2)
              if (c2 < jn) P[k][c2] = fma(-l, colbuf[c2] * rd, P[k][c2]);
          }
        }
        __syncthreads();
      }
    }
    // write the panel back
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int w = tid + k * NT;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (w < W && c < jn && w >= c && w - c <= kd)
          L[(int64_t)(j0 + c) * ld + (w - c)] = P[k][c];
      }
    }
    // trailing update: A[w, q] -= P[w,:] . P[q,:] for jn <= q <= w < W
    for (int q0 = jn; q0 < W; q0 += CH) {
      const int qe = min(q0 + CH, W);
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int w = tid + k * NT;
        if (w >= q0 && w < qe) {
#pragma unroll
          for (int c = 0; c < NB; ++c) chunk[w - q0][c] = P[k][c];
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int w = tid + k * NT;
        if (w >= q0 && w < W) {
          const int qmax = min(qe - 1, w);
          for (int q = q0; q <= qmax; ++q) {
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < NB; ++c) acc = fma(P[k][c], chunk[q - q0][c], acc);
            double *a = L + (int64_t)(j0 + q) * ld + (w - q);
            *a -= acc;
          }
        }
      }
      __syncthreads();
    }
  }
  // report the first failing subdomain status (0 = ok)
  __shared__ int anybad;
  if (tid == 0) anybad = 0;
  __syncthreads();
  if (bad) anybad = 1;
  __syncthreads();
  if (tid == 0) info[order[blockIdx.x]] = anybad;
}

// ---------------------------------------------------------------------------
// Substitutions
// ---------------------------------------------------------------------------
template <typename W>
__device__ inline W wave_sum(W v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T, typename W, int NB, int NT>
__global__ __launch_bounds__(NT) void k_band_solve(
    const SubDesc *__restrict__ subs, const int *__restrict__ order,
    const T *__restrict__ fac, const double *__restrict__ b,
    double *__restrict__ x, int maxn) {
  extern __shared__ __align__(16) unsigned char smem[];
  W *xs = reinterpret_cast<W *>(smem);
  T *dblk = reinterpret_cast<T *>(smem + ((sizeof(W) * maxn + 15) / 16) * 16);
  constexpr int PITCH = NB + 1;
  constexpr int NW = NT / 64;
  const SubDesc s = subs[order[blockIdx.x]];
  const int n = s.n, kd = s.kd, ld = kd + 1;
  const T *L = fac + s.fac_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  for (int i = tid; i < n; i += NT) xs[i] = (W)b[s.dof_off + i];
  __syncthreads();

  // ---- forward: L y = b ----
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int jn = min(NB, n - j0);
    // diagonal block, column-major with pitch: dblk[c*PITCH + row]
    for (int e = tid; e < NB * NB; e += NT) {
      const int c = e / NB, row = e - c * NB, r = row - c;
      const bool ok = r >= 0 && c < jn && row < jn && r <= kd;
      dblk[c * PITCH + row] = ok ? L[(int64_t)(j0 + c) * ld + r] : (T)0;
    }
    __syncthreads();
    if (wave == 0) {
      W xi = lane < jn ? xs[j0 + lane] : (W)0;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c < jn) {
          if (lane == c) xi = xi / (W)dblk[c * PITCH + c];
          const W xc = __shfl(xi, c, 64);
          if (lane > c && lane < NB) xi -= (W)dblk[c * PITCH + lane] * xc;
        }
      }
      if (lane < jn) xs[j0 + lane] = xi;
    }
    __syncthreads();
    const int rend = min(n, j0 + jn + kd);
    for (int i = j0 + jn + tid; i < rend; i += NT) {
      W acc = 0;
      const int c0 = max(0, i - j0 - kd);
      for (int c = c0; c < jn; ++c)
        acc += (W)L[(int64_t)(j0 + c) * ld + (i - j0 - c)] * xs[j0 + c];
      xs[i] -= acc;
    }
    __syncthreads();
  }

  // ---- backward: L^T x = y ----
  const int jlast = ((n - 1) / NB) * NB;
  for (int j0 = jlast; j0 >= 0; j0 -= NB) {
    const int jn = min(NB, n - j0);
    for (int cc = wave; cc < jn; cc += NW) {
      const int c = j0 + cc;
      const int rs = j0 + jn - c;
      const int re = min(kd, n - 1 - c);
      W acc = 0;
      for (int r = rs + lane; r <= re; r += 64)
        acc += (W)L[(int64_t)c * ld + r] * xs[c + r];
      acc = wave_sum(acc);
      if (lane == 0) xs[c] -= acc;
    }
    // diagonal block, row-major with pitch: dblk[row*PITCH + c]
    for (int e = tid; e < NB * NB; e += NT) {
      const int c = e / NB, row = e - c * NB, r = row - c;
      const bool ok = r >= 0 && c < jn && row < jn && r <= kd;
      dblk[row * PITCH + c] = ok ? L[(int64_t)(j0 + c) * ld + r] : (T)0;
    }
    __syncthreads();
    if (wave == 0) {
      W xi = lane < jn ? xs[j0 + lane] : (W)0;
#pragma unroll
      for (int cc = NB - 1; cc >= 0; --cc) {
        if (cc < jn) {
          if (lane == cc) xi = xi / (W)dblk[cc * PITCH + cc];
          const W xc = __shfl(xi, cc, 64);
          if (lane < cc) xi -= (W)dblk[cc * PITCH + lane] * xc;
        }
      }
      if (lane < jn) xs[j0 + lane] = xi;
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += NT) x[s.dof_off + i] = (double)xs[i];
}

__global__ void k_f64_to_f32(const double *__restrict__ a, float *__restrict__ b,
                             int64_t n) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    b[t] = (float)a[t];
}

template <int NB, int NT, int RPT>
void chol_launch(edd_problem *p) {
  k_band_cholesky<NB, NT, RPT, 32><<<p->n_sub, NT, 0, p->stream>>>(
      p->subs_d, p->order_d, p->fac64_d, p->info_d);
}

template <typename T, typename W, int NB, int NT>
void solve_launch(edd_problem *p, const T *fac, const double *b, double *x) {
  const size_t lds = ((sizeof(W) * p->max_n + 15) / 16) * 16 +
                     sizeof(T) * NB * (NB + 1);
  static bool attr_set = false;  // per instantiation
  if (!attr_set) {
    hipFuncSetAttribute((const void *)k_band_solve<T, W, NB, NT>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds > 65536 ? 163840 : 65536);
    attr_set = true;
  }
  k_band_solve<T, W, NB, NT><<<p->n_sub, NT, lds, p->stream>>>(
      p->subs_d, p->order_d, fac, b, x, p->max_n);
}

}  // namespace

size_t band_solve_lds_bytes(const edd_problem *p, int precision) {
  const int NB = p->max_kd > 96 ? 64 : 32;
  const size_t ws = precision == EDD_F32 ? 4 : 8;
  return ((ws * p->max_n + 15) / 16) * 16 + ws * NB * (NB + 1);
}

void launch_band_cholesky(edd_problem *p) {
  constexpr int NB = 32;
  const int W = NB + p->max_kd;
  if (W <= 128) chol_launch<NB, 128, 1>(p);
  else if (W <= 256) chol_launch<NB, 256, 1>(p);
  else if (W <= 512) chol_launch<NB, 512, 1>(p);
  else if (W <= 1024) chol_launch<NB, 512, 2>(p);
  else if (W <= 1536) chol_launch<NB, 512, 3>(p);
  else chol_launch<NB, 512, 4>(p);  // kd up to 2016 (checked at setup)
}

void launch_band_to_f32(edd_problem *p) {
  k_f64_to_f32<<<2048, 256, 0, p->stream>>>(p->fac64_d, p->fac32_d,
                                            p->fac_entries);
}

void launch_band_solve(edd_problem *p, int precision, const double *b,
                       double *x) {
  const bool big = p->max_kd > 96;
  if (precision == EDD_F32) {
    if (big) solve_launch<float, float, 64, 512>(p, p->fac32_d, b, x);
    else solve_launch<float, float, 32, 64>(p, p->fac32_d, b, x);
  } else {
    if (big) solve_launch<double, double, 64, 512>(p, p->fac64_d, b, x);
    else solve_launch<double, double, 32, 64>(p, p->fac64_d, b, x);
  }
}

}  // namespace edd

// Vector kernels of the interface Krylov iteration.  Dot products use a
// deterministic two-stage reduction: each block writes its partial sums,
// then one block per result sums the partials in a fixed order.  Scalars
// (alpha, the dots) stay on the device in p->scal_d, so the iteration does
// not wait on the host between kernels.
#include "internal.h"

namespace edd {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxBlocks = 1024;

__device__ inline double block_sum(double v, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  }
  __syncthreads();
  return s;  // valid in thread 0
}

struct DotArgs {
  const double *a[4];
  const double *b[4];
};

template <int ND>
__global__ __launch_bounds__(kBlock) void k_dots(int64_t n, DotArgs args,
                                                 double *__restrict__ partials) {
  __shared__ double red[kBlock / 64];
  double acc[ND];
#pragma unroll
  for (int k = 0; k < ND; ++k) acc[k] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int k = 0; k < ND; ++k) acc[k] = fma(args.a[k][i], args.b[k][i], acc[k]);
  }
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    const double s = block_sum(acc[k], red);
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * ND + k] = s;
  }
}

// out[slot + j] = sum_b partials[b*stride + j], one block per j.
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

__global__ __launch_bounds__(kBlock) void k_axpby(int64_t n, double a,
                                                  const double *__restrict__ x,
                                                  double b, double *__restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

__global__ __launch_bounds__(kBlock) void k_fill_f32(int64_t n,
                                                     float *__restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = 0.0f;
}

__global__ __launch_bounds__(kBlock) void k_fill(int64_t n, double v,
                                                 double *__restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = v;
}

// x += alpha p, r -= alpha q with alpha = scal[num]/scal[den]; partial
// sums of r.r for the convergence test; optionally keeps a copy of the
// denominator (p^T S p) for the window of previous directions.
// x += alpha p, r -= alpha q with alpha = scal[num] / scal[den].  A step
// with scal[den] <= 0 or a non-finite alpha (breakdown, or iterations run
// past convergence between host checks) changes nothing, stores 1 as its
// p^T S p and raises *flag.
__global__ __launch_bounds__(kBlock) void k_cg_update(
    int64_t n, double *__restrict__ scal, int num, int den,
    double *__restrict__ x, const double *__restrict__ pv,
    double *__restrict__ r, const double *__restrict__ q,
    double *__restrict__ partials, double *__restrict__ copy_to,
    double *__restrict__ flag) {
  __shared__ double red[kBlock / 64];
  const double pq = scal[den];
  const double alpha = scal[num] / pq;
  const bool ok = pq > 0.0 && isfinite(alpha);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (copy_to) *copy_to = ok ? pq : 1.0;
    if (!ok) *flag = 1.0;
  }
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double ri = r[i];
    if (ok) {
      x[i] = fma(alpha, pv[i], x[i]);
      ri = fma(-alpha, q[i], ri);
      r[i] = ri;
    }
    acc = fma(ri, ri, acc);
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// partials[b*m + j] = <z, W_j> over row chunk b = blockIdx.x, for the eight
// vectors j of group blockIdx.y (one workgroup per chunk and group, so the
// window's vectors stream in parallel); the eight share each reduction
// (wavefront shuffles, one barrier), summed in a fixed order.
__global__ __launch_bounds__(kBlock) void k_window_dots(
    int64_t n, int m, const double *__restrict__ W, const double *__restrict__ z,
    double *__restrict__ partials) {
  constexpr int JB = 8, NW = kBlock / 64;
  __shared__ double red[JB][NW];
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * chunk;
  const int64_t hi = min(n, lo + chunk);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // blockIdx.y picks a group of JB vectors; blockIdx.x the chunk of rows
  {
    const int j0 = blockIdx.y * JB;
    const int nj = min(JB, m - j0);
    double acc[JB];
#pragma unroll
    for (int jj = 0; jj < JB; ++jj) acc[jj] = 0.0;
    // two rows a step: eighteen loads in flight per thread
    int64_t i = lo + threadIdx.x;
    for (; i + blockDim.x < hi; i += 2 * (int64_t)blockDim.x) {
      const int64_t i1 = i + blockDim.x;
      const double z0 = z[i], z1 = z[i1];
      double w0[JB], w1[JB];
#pragma unroll
      for (int jj = 0; jj < JB; ++jj) {
        const int64_t r = (int64_t)(jj < nj ? j0 + jj : j0) * n;
        w0[jj] = W[r + i];
        w1[jj] = W[r + i1];
      }
#pragma unroll
      for (int jj = 0; jj < JB; ++jj)
        if (jj < nj) acc[jj] = fma(z1, w1[jj], fma(z0, w0[jj], acc[jj]));
    }
    if (i < hi) {
      const double zi = z[i];
#pragma unroll
      for (int jj = 0; jj < JB; ++jj)
        if (jj < nj) acc[jj] = fma(zi, W[(int64_t)(j0 + jj) * n + i], acc[jj]);
    }
#pragma unroll
    for (int jj = 0; jj < JB; ++jj) {
      double v = acc[jj];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
      if (lane == 0) red[jj][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < nj) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) s += red[threadIdx.x][w];
      partials[(int64_t)blockIdx.x * m + j0 + threadIdx.x] = s;
    }
  }
}

// Window dots of the captured iteration: the window is the m = min(k, cap)
// newest directions of the ring (k = scal[kSlotGK]), age index t at ring slot
// (first + t) % cap; partials[b*cap + t] over row chunk b, then
// k_reduce_ring.  Same chunks and order as k_window_dots per direction.
__global__ __launch_bounds__(kBlock) void k_window_dots_dev(
    int64_t n, int cap, const double *__restrict__ W, const double *__restrict__ z,
    const double *__restrict__ scal, double *__restrict__ partials) {
  constexpr int JB = 8, NW = kBlock / 64;
  __shared__ double red[JB][NW];
  const int k = (int)scal[kSlotGK];
  const int m = min(k, cap);
  const int first = ((k - m) % cap + cap) % cap;
  const int j0 = blockIdx.y * JB;
  if (j0 >= m) return;  // the whole workgroup: no direction of this group yet
  const int nj = min(JB, m - j0);
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * chunk;
  const int64_t hi = min(n, lo + chunk);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double acc[JB];
#pragma unroll
  for (int jj = 0; jj < JB; ++jj) acc[jj] = 0.0;
  int64_t row[JB];
#pragma unroll
  for (int jj = 0; jj < JB; ++jj)
    row[jj] = (int64_t)((first + j0 + (jj < nj ? jj : 0)) % cap) * n;
  int64_t i = lo + threadIdx.x;
  for (; i + blockDim.x < hi; i += 2 * (int64_t)blockDim.x) {
    const int64_t i1 = i + blockDim.x;
    const double z0 = z[i], z1 = z[i1];
    double w0[JB], w1[JB];
#pragma unroll
    for (int jj = 0; jj < JB; ++jj) {
      w0[jj] = W[row[jj] + i];
      w1[jj] = W[row[jj] + i1];
    }
#pragma unroll
    for (int jj = 0; jj < JB; ++jj)
      if (jj < nj) acc[jj] = fma(z1, w1[jj], fma(z0, w0[jj], acc[jj]));
  }
  if (i < hi) {
    const double zi = z[i];
#pragma unroll
    for (int jj = 0; jj < JB; ++jj)
      if (jj < nj) acc[jj] = fma(zi, W[row[jj] + i], acc[jj]);
  }
#pragma unroll
  for (int jj = 0; jj < JB; ++jj) {
    double v = acc[jj];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) red[jj][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < nj) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[threadIdx.x][w];
    partials[(int64_t)blockIdx.x * cap + j0 + threadIdx.x] = s;
  }
}

// scal[cbase + (first + t) % cap] = sum_b partials[b*cap + t], block t < m
__global__ __launch_bounds__(kBlock) void k_reduce_ring(const double *__restrict__ partials,
                                                        int nblocks, int cap,
                                                        double *__restrict__ scal, int cbase) {
  __shared__ double red[kBlock / 64];
  const int k = (int)scal[kSlotGK];
  const int m = min(k, cap);
  const int first = ((k - m) % cap + cap) % cap;
  const int t = blockIdx.x;
  if (t >= m) return;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
    acc += partials[(int64_t)b * cap + t];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) scal[cbase + (first + t) % cap] = s;
}

// pv = z - sum over the window, oldest first, of (scal[cbase+slot] /
// scal[dbase+slot]) P_slot: the same sequence of operations as the
// per-segment combines of the host-driven iteration.
__global__ __launch_bounds__(kBlock) void k_window_combine_dev(
    int64_t n, int cap, const double *__restrict__ P, const double *__restrict__ scal,
    int cbase, int dbase, const double *__restrict__ z, double *__restrict__ pv) {
  __shared__ double coef[256];
  __shared__ int64_t rows[256];
  const int k = (int)scal[kSlotGK];
  const int m = min(k, cap);
  const int first = ((k - m) % cap + cap) % cap;
  for (int t = threadIdx.x; t < m; t += blockDim.x) {
    const int slot = (first + t) % cap;
    coef[t] = scal[cbase + slot] / scal[dbase + slot];
    rows[t] = (int64_t)slot * n;
  }
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = z[i];
    int j = 0;
    for (; j + 4 <= m; j += 4) {
      double a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = P[rows[j + u] + i];
#pragma unroll
      for (int u = 0; u < 4; ++u) v = fma(-coef[j + u], a[u], v);
    }
    for (; j < m; ++j) v = fma(-coef[j], P[rows[j] + i], v);
    pv[i] = v;
  }
}

__global__ __launch_bounds__(kBlock) void k_ring_store(int64_t n, int cap,
                                                       const double *__restrict__ scal,
                                                       const double *__restrict__ src,
                                                       double *__restrict__ ring) {
  const int64_t slot = (int64_t)((int)scal[kSlotGK] % cap);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    ring[slot * n + i] = src[i];
}

// Window dots of the host-driven iteration over the m newest directions of
// the ring (capacity cap, oldest at slot first), slot s stored at
// tab[s / kWinBlock] + (s % kWinBlock) * n: partials[b*m + t] over row chunk
// b = blockIdx.x for the eight directions t of group blockIdx.y.  Chunks,
// loads and summation order are those of k_window_dots_dev.
__global__ __launch_bounds__(kBlock) void k_ring_dots(
    int64_t n, int cap, int first, int m, const double *const *__restrict__ tab,
    const double *__restrict__ z, double *__restrict__ partials) {
  constexpr int JB = 8, NW = kBlock / 64;
  __shared__ double red[JB][NW];
  const int j0 = blockIdx.y * JB;
  const int nj = min(JB, m - j0);
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * chunk;
  const int64_t hi = min(n, lo + chunk);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double acc[JB];
#pragma unroll
  for (int jj = 0; jj < JB; ++jj) acc[jj] = 0.0;
  const double *w[JB];
#pragma unroll
  for (int jj = 0; jj < JB; ++jj) {
    const int slot = (first + j0 + (jj < nj ? jj : 0)) % cap;
    w[jj] = tab[slot / kWinBlock] + (int64_t)(slot % kWinBlock) * n;
  }
  int64_t i = lo + threadIdx.x;
  for (; i + blockDim.x < hi; i += 2 * (int64_t)blockDim.x) {
    const int64_t i1 = i + blockDim.x;
    const double z0 = z[i], z1 = z[i1];
    double w0[JB], w1[JB];
#pragma unroll
    for (int jj = 0; jj < JB; ++jj) {
      w0[jj] = w[jj][i];
      w1[jj] = w[jj][i1];
    }
#pragma unroll
    for (int jj = 0; jj < JB; ++jj)
      if (jj < nj) acc[jj] = fma(z1, w1[jj], fma(z0, w0[jj], acc[jj]));
  }
  if (i < hi) {
    const double zi = z[i];
#pragma unroll
    for (int jj = 0; jj < JB; ++jj)
      if (jj < nj) acc[jj] = fma(zi, w[jj][i], acc[jj]);
  }
#pragma unroll
  for (int jj = 0; jj < JB; ++jj) {
    double v = acc[jj];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) red[jj][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < nj) {
    double s = 0.0;
#pragma unroll
    for (int w2 = 0; w2 < NW; ++w2) s += red[threadIdx.x][w2];
    partials[(int64_t)blockIdx.x * m + j0 + threadIdx.x] = s;
  }
}

// scal[cbase + (first + t) % cap] = sum_b partials[b*m + t], block t < m
// (the order of k_reduce_ring)
__global__ __launch_bounds__(kBlock) void k_reduce_win(const double *__restrict__ partials,
                                                       int nblocks, int m, int first, int cap,
                                                       double *__restrict__ scal, int cbase) {
  __shared__ double red[kBlock / 64];
  const int t = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
    acc += partials[(int64_t)b * m + t];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) scal[cbase + (first + t) % cap] = s;
}

// pv = z - sum over the m newest directions, oldest first, of
// (scal[cbase+slot] / scal[dbase+slot]) P_slot, the directions in LDS
// batches of 256 (coefficient and address); per row the same chain of fmas
// as k_window_combine_dev.
__global__ __launch_bounds__(kBlock) void k_ring_combine(
    int64_t n, int cap, int first, int m, const double *const *__restrict__ tab,
    const double *__restrict__ scal, int cbase, int dbase,
    const double *__restrict__ z, double *__restrict__ pv) {
  constexpr int B = 256, U = 8;
  __shared__ double coef[B];
  __shared__ const double *ptr[B];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x; i0 < n; i0 += stride) {
    const int64_t i = i0 + threadIdx.x;
    const bool live = i < n;
    double v = live ? z[i] : 0.0;
    for (int t0 = 0; t0 < m; t0 += B) {
      const int len = min(B, m - t0);
      __syncthreads();  // the previous batch's reads are done
      for (int t = threadIdx.x; t < len; t += blockDim.x) {
        const int slot = (first + t0 + t) % cap;
        coef[t] = scal[cbase + slot] / scal[dbase + slot];
        ptr[t] = tab[slot / kWinBlock] + (int64_t)(slot % kWinBlock) * n;
      }
      __syncthreads();
      if (!live) continue;
      int j = 0;
      for (; j + U <= len; j += U) {
        double a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = ptr[j + u][i];
#pragma unroll
        for (int u = 0; u < U; ++u) v = fma(-coef[j + u], a[u], v);
      }
      for (; j < len; ++j) v = fma(-coef[j], ptr[j][i], v);
    }
    if (live) pv[i] = v;
  }
}

__global__ void k_iter_end(double *__restrict__ scal, int cap, int pqbase) {
  if (threadIdx.x != 0) return;
  const int k = (int)scal[kSlotGK];
  const double rr = scal[kSlotGRR];
  scal[pqbase + k % cap] = scal[kSlotGPQ];
  scal[kSlotGHist + k % kGHist] = rr;
  if (scal[kSlotGDone] == 0.0 && rr <= scal[kSlotGTol2]) scal[kSlotGDone] = k + 1;
  scal[kSlotGK] = k + 1;
}

// pv = z - sum_j (scal[cslot+j] / scal[dslot+j]) P_j  (m <= 256)
__global__ __launch_bounds__(kBlock) void k_window_combine(
    int64_t n, int m, const double *__restrict__ P,
    const double *__restrict__ scal, int cslot, int dslot,
    const double *__restrict__ z, double *__restrict__ pv) {
  __shared__ double coef[256];
  for (int j = threadIdx.x; j < m; j += blockDim.x) coef[j] = scal[cslot + j] / scal[dslot + j];
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = z[i];
    int j = 0;
    for (; j + 4 <= m; j += 4) {  // four loads in flight, same order of terms
      double a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = P[(int64_t)(j + u) * n + i];
#pragma unroll
      for (int u = 0; u < 4; ++u) v = fma(-coef[j + u], a[u], v);
    }
    for (; j < m; ++j) v = fma(-coef[j], P[(int64_t)j * n + i], v);
    pv[i] = v;
  }
}

__global__ __launch_bounds__(kBlock) void k_residual_norms(
    int dim, int64_t n_nodes, const int *__restrict__ nmap,
    const double *__restrict__ f, const double *__restrict__ y,
    double *__restrict__ partials) {
  __shared__ double red[kBlock / 64];
  double rr = 0.0, ff = 0.0;
  const int64_t n = n_nodes * dim;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (nmap[i / dim] != kDirichlet) {
      const double d = f[i] - y[i];
      rr = fma(d, d, rr);
      ff = fma(f[i], f[i], ff);
    }
  }
  const double a = block_sum(rr, red);
  const double b = block_sum(ff, red);
  if (threadIdx.x == 0) {
    partials[(int64_t)blockIdx.x * 2] = a;
    partials[(int64_t)blockIdx.x * 2 + 1] = b;
  }
}

inline unsigned grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > kMaxBlocks) g = kMaxBlocks;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// row chunks of the flexible-CG window dots: about eight rows per thread (a
// chunk's partial sums are few against its loads), at most kWinChunks
inline unsigned window_chunks(int64_t n) {
  int64_t g = (n + 8 * kBlock - 1) / (8 * kBlock);
  if (g > kWinChunks) g = kWinChunks;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

void launch_dots(edd_problem *p, int64_t n, int nd, const double *const *a,
                 const double *const *b, int slot) {
  DotArgs args{};
  for (int k = 0; k < nd; ++k) {
    args.a[k] = a[k];
    args.b[k] = b[k];
  }
  const unsigned g = grid_for(n);
  switch (nd) {
    case 1: k_dots<1><<<g, kBlock, 0, p->stream>>>(n, args, p->partials_d); break;
    case 2: k_dots<2><<<g, kBlock, 0, p->stream>>>(n, args, p->partials_d); break;
    case 3: k_dots<3><<<g, kBlock, 0, p->stream>>>(n, args, p->partials_d); break;
    default: k_dots<4><<<g, kBlock, 0, p->stream>>>(n, args, p->partials_d); break;
  }
  k_reduce<<<nd, kBlock, 0, p->stream>>>(p->partials_d, (int)g, nd, p->scal_d + slot);
}

void launch_axpby(edd_problem *p, int64_t n, double a, const double *x,
                  double b, double *y) {
  k_axpby<<<grid_for(n), kBlock, 0, p->stream>>>(n, a, x, b, y);
}

void launch_copy(edd_problem *p, int64_t n, const double *x, double *y) {
  hipMemcpyAsync(y, x, sizeof(double) * n, hipMemcpyDeviceToDevice, p->stream);
}

void launch_fill(edd_problem *p, int64_t n, double v, double *y) {
  k_fill<<<grid_for(n), kBlock, 0, p->stream>>>(n, v, y);
}

void launch_fill_f32(edd_problem *p, int64_t n, float *y) {
  k_fill_f32<<<grid_for(n), kBlock, 0, p->stream>>>(n, y);
}

void launch_cg_update(edd_problem *p, int64_t n, int num, int den, double *x,
                      const double *pv, double *r, const double *q, int slot,
                      int copy_dst, int flag_slot) {
  const unsigned g = grid_for(n);
  k_cg_update<<<g, kBlock, 0, p->stream>>>(
      n, p->scal_d, num, den, x, pv, r, q, p->partials_d,
      copy_dst >= 0 ? p->scal_d + copy_dst : nullptr, p->scal_d + flag_slot);
  k_reduce<<<1, kBlock, 0, p->stream>>>(p->partials_d, (int)g, 1, p->scal_d + slot);
}

void launch_window_dots(edd_problem *p, int64_t n, int m, const double *W,
                        const double *z, int slot) {
  if (m <= 0) return;
  unsigned g = grid_for(n);
  if (g > 256) g = 256;
  k_window_dots<<<dim3(g, (m + 7) / 8), kBlock, 0, p->stream>>>(n, m, W, z, p->partials_d);
  k_reduce<<<m, kBlock, 0, p->stream>>>(p->partials_d, (int)g, m, p->scal_d + slot);
}

void launch_window_combine(edd_problem *p, int64_t n, int m, const double *P,
                           int cslot, int dslot, const double *z, double *pv) {
  k_window_combine<<<grid_for(n), kBlock, 0, p->stream>>>(n, m, P, p->scal_d,
                                                          cslot, dslot, z, pv);
}

void launch_window_dots_dev(edd_problem *p, int64_t n, int cap, const double *W,
                            const double *z, int cbase) {
  const unsigned g = window_chunks(n);
  k_window_dots_dev<<<dim3(g, (cap + 7) / 8), kBlock, 0, p->stream>>>(n, cap, W, z, p->scal_d,
                                                                     p->partials_d);
  k_reduce_ring<<<cap, kBlock, 0, p->stream>>>(p->partials_d, (int)g, cap, p->scal_d, cbase);
}

void launch_window_combine_dev(edd_problem *p, int64_t n, int cap, const double *P,
                               int cbase, int dbase, const double *z, double *pv) {
  k_window_combine_dev<<<grid_for(n), kBlock, 0, p->stream>>>(n, cap, P, p->scal_d, cbase,
                                                              dbase, z, pv);
}

void launch_ring_dots(edd_problem *p, int64_t n, int cap, int first, int m,
                      const double *const *tab, const double *z, int cbase) {
  if (m <= 0) return;
  const unsigned g = window_chunks(n);
  k_ring_dots<<<dim3(g, (m + 7) / 8), kBlock, 0, p->stream>>>(n, cap, first, m, tab, z,
                                                              p->partials_d);
  k_reduce_win<<<m, kBlock, 0, p->stream>>>(p->partials_d, (int)g, m, first, cap, p->scal_d,
                                            cbase);
}

void launch_ring_combine(edd_problem *p, int64_t n, int cap, int first, int m,
                         const double *const *tab, int cbase, int dbase, const double *z,
                         double *pv) {
  k_ring_combine<<<grid_for(n), kBlock, 0, p->stream>>>(n, cap, first, m, tab, p->scal_d, cbase,
                                                        dbase, z, pv);
}

void launch_ring_store(edd_problem *p, int64_t n, int cap, const double *src, double *ring) {
  k_ring_store<<<grid_for(n), kBlock, 0, p->stream>>>(n, cap, p->scal_d, src, ring);
}

void launch_iter_end(edd_problem *p, int cap, int pqbase) {
  k_iter_end<<<1, 64, 0, p->stream>>>(p->scal_d, cap, pqbase);
}

void launch_residual_norms(edd_problem *p, const double *f, const double *y,
                           int slot) {
  const unsigned g = grid_for(p->n_nodes * p->g.dim);
  k_residual_norms<<<g, kBlock, 0, p->stream>>>(p->g.dim, p->n_nodes, p->nmap_d,
                                                f, y, p->partials_d);
  k_reduce<<<2, kBlock, 0, p->stream>>>(p->partials_d, (int)g, 2, p->scal_d + slot);
}

void launch_reduce(edd_problem *p, int nblocks, int stride, int nout, int slot) {
  k_reduce<<<nout, kBlock, 0, p->stream>>>(p->partials_d, nblocks, stride,
                                           p->scal_d + slot);
}

}  // namespace edd

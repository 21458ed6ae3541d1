// The correction network: a four-layer node-grid convolution (3^D taps,
// dilations 1, 2, 4, 1, ReLU after the first three) that proposes a
// displacement correction from a stiffness indicator and the residual.  It is
// an addition to the paper's method; the solver uses its output only as an
// initial-guess direction with an exact line search in the interface energy
// norm, so the solve's result does not depend on it.
//
// Layout: every activation is channel-last on the node grid, act[node*C + c],
// node ids x fastest (the nodal-vector layout).  Parameters are one flat FP32
// array, per layer W[tap][c_in][c_out] then b[c_out], taps in C order over
// ([z,] y, x) offsets; the forward pass uses an FP16 copy of them, staged in
// LDS as FP32, with FP32 accumulation.  Weight gradients are reduced in
// fixed node chunks and then over chunks in a fixed order (deterministic).
#include <hip/hip_fp16.h>

#include <algorithm>

#include "internal.h"

namespace edd {

constexpr int kCnnNT = 1024;     // threads per block of the layer kernels
constexpr int kCnnChunks = 256;  // node chunks of the weight-gradient reduction
constexpr int kCnnBatch = 8;     // nodes staged per step of that reduction
constexpr int kCnnDil[kCnnLayers] = {1, 2, 4, 1};

// scalar slots (the solver and preconditioner use slots below 1600)
enum : int { C_RR = 1600, C_EE = 1602, C_LOSS = 1604 };

namespace {

struct NodeGrid {
  int dim;
  int nn[3];
};

template <int D>
__device__ inline void node_coords(const NodeGrid &g, int64_t n, int (&c)[3]) {
  c[0] = (int)(n % g.nn[0]);
  const int64_t r = n / g.nn[0];
  if (D == 2) {
    c[1] = (int)r;
    c[2] = 0;
  } else {
    c[1] = (int)(r % g.nn[1]);
    c[2] = (int)(r / g.nn[1]);
  }
}

// node index of the tap t neighbour (offset s*(t_a - 1) per axis), or -1
template <int D>
__device__ inline int64_t tap_neighbour(const NodeGrid &g, const int (&c)[3], int t, int s,
                                        int sign) {
  int o[3] = {0, 0, 0};
  if (D == 2) {
    o[1] = t / 3 - 1;
    o[0] = t % 3 - 1;
  } else {
    o[2] = t / 9 - 1;
    o[1] = (t / 3) % 3 - 1;
    o[0] = t % 3 - 1;
  }
  int64_t idx = 0, mul = 1;
  for (int a = 0; a < D; ++a) {
    const int q = c[a] + sign * s * o[a];
    if (q < 0 || q >= g.nn[a]) return -1;
    idx += mul * q;
    mul *= g.nn[a];
  }
  return idx;
}

template <int D>
constexpr int ntaps() { return D == 2 ? 9 : 27; }

// ---- features --------------------------------------------------------------
// X[n] = (mean over adjacent elements of clip(1 + log10(E)/3, 0, 1),
//         r[D n + c] / rms_free(r))
template <int D>
__global__ __launch_bounds__(256) void k_features(NodeGrid g, Geom eg, const double *__restrict__ E,
                                                  const double *__restrict__ r,
                                                  const double *__restrict__ scal,
                                                  double nfree, float *__restrict__ X) {
  const int64_t nn = (int64_t)g.nn[0] * g.nn[1] * (D == 3 ? g.nn[2] : 1);
  const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (n >= nn) return;
  int c[3];
  node_coords<D>(g, n, c);
  double acc = 0.0;
  int cnt = 0;
  for (int dz = (D == 3 ? -1 : 0); dz <= 0; ++dz)
    for (int dy = -1; dy <= 0; ++dy)
      for (int dx = -1; dx <= 0; ++dx) {
        const int ex = c[0] + dx, ey = c[1] + dy, ez = c[2] + dz;
        if (ex < 0 || ex >= eg.nel[0] || ey < 0 || ey >= eg.nel[1]) continue;
        if (D == 3 && (ez < 0 || ez >= eg.nel[2])) continue;
        const int64_t e = ex + (int64_t)eg.nel[0] * (ey + (int64_t)eg.nel[1] * ez);
        double s = 1.0 + log10(E[e]) / 3.0;
        s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
        acc += s;
        ++cnt;
      }
  const double ss = scal[C_RR + 1];
  const double rms = ss > 0.0 ? sqrt(ss / nfree) : 0.0;
  float *x = X + n * (1 + D);
  x[0] = (float)(acc / cnt);
#pragma unroll
  for (int k = 0; k < D; ++k) x[1 + k] = (float)(rms > 0.0 ? r[D * n + k] / rms : r[D * n + k]);
}

// T[n] = e[D n + c] / rms_free(e)
template <int D>
__global__ void k_target(int64_t nn, const double *__restrict__ e, const double *__restrict__ scal,
                         double nfree, float *__restrict__ T) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nn * D) return;
  const double ss = scal[C_EE + 1];
  const double rms = ss > 0.0 ? sqrt(ss / nfree) : 0.0;
  T[i] = (float)(rms > 0.0 ? e[i] / rms : e[i]);
}

// ---- layers ------------------------------------------------------------------
template <int NTAP, int CI, int CO>
__device__ inline void stage_weights(const __half *__restrict__ w, float *Ws, float *bs) {
  for (int i = threadIdx.x; i < NTAP * CI * CO; i += blockDim.x) Ws[i] = __half2float(w[i]);
  for (int i = threadIdx.x; i < CO; i += blockDim.x) bs[i] = __half2float(w[NTAP * CI * CO + i]);
  __syncthreads();
}

// out[n, o] = b[o] + sum_{t,i} W[t,i,o] in[n + s (t-1), i]; optional ReLU
template <int D, int CI, int CO, bool RELU>
__global__ __launch_bounds__(kCnnNT) void k_conv_fwd(NodeGrid g, int64_t nn, int s,
                                                     const __half *__restrict__ w,
                                                     const float *__restrict__ in,
                                                     float *__restrict__ out) {
  constexpr int NTAP = ntaps<D>();
  extern __shared__ float lds[];
  float *Ws = lds, *bs = lds + NTAP * CI * CO;
  stage_weights<NTAP, CI, CO>(w, Ws, bs);
  const int64_t n = blockIdx.x * (int64_t)kCnnNT + threadIdx.x;
  if (n >= nn) return;
  int c[3];
  node_coords<D>(g, n, c);
  float acc[CO];
#pragma unroll
  for (int o = 0; o < CO; ++o) acc[o] = bs[o];
  for (int t = 0; t < NTAP; ++t) {
    const int64_t m = tap_neighbour<D>(g, c, t, s, 1);
    if (m < 0) continue;
    const float *x = in + m * CI;
    const float *wt = Ws + t * CI * CO;
#pragma unroll 4
    for (int i = 0; i < CI; ++i) {
      const float xv = x[i];
#pragma unroll
      for (int o = 0; o < CO; ++o) acc[o] = fmaf(wt[i * CO + o], xv, acc[o]);
    }
  }
  float *y = out + n * CO;
#pragma unroll
  for (int o = 0; o < CO; ++o) y[o] = RELU ? fmaxf(acc[o], 0.0f) : acc[o];
}

// The hidden 32 -> 32 layers on the FP16 matrix cores: an implicit GEMM per
// wavefront over 16 nodes (M), the 32 outputs (two 16-column N tiles) and
// K = taps x 32 input channels in chunks of 16, by v_mfma_f32_16x16x16_f16
// with FP32 accumulation.  Lane l supplies A[l%16][4(l/16)+j] (node l%16 of
// the tile, four input channels of the chunk from its tap neighbour,
// rounded to FP16) and B[4(l/16)+j][l%16] (the FP16 weights, staged in LDS
// transposed per tap so that the four values are contiguous), and holds
// D[4(l/16)+e][l%16] (layout checked on the device).  Activations rounded to
// FP16 add a relative error of about 1e-3 against the FP32 path.
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

template <int D, bool RELU>
__global__ __launch_bounds__(256) void k_conv_fwd_mfma(NodeGrid g, int64_t nn, int s,
                                                       const __half *__restrict__ w,
                                                       const float *__restrict__ in,
                                                       float *__restrict__ out) {
  constexpr int NTAP = ntaps<D>();
  constexpr int C = kCnnWidth;
  static_assert(C == 32, "the matrix-core layer is written for 32 channels");
  __shared__ _Float16 Wt[NTAP * C * C];
  __shared__ float bs[C];
  for (int k = threadIdx.x; k < NTAP * C * C; k += blockDim.x) {
    const int t = k / (C * C), i = (k / C) % C, o = k % C;
    Wt[(t * C + o) * C + i] = (_Float16)__half2float(w[k]);
  }
  for (int o = threadIdx.x; o < C; o += blockDim.x) bs[o] = __half2float(w[NTAP * C * C + o]);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int lm = lane % 16, lk = 4 * (lane / 16);
  const int64_t ntiles = (nn + 15) / 16;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wv; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
    const int64_t na = tile * 16 + lm;  // the node whose A row this lane supplies
    int c[3] = {0, 0, 0};
    const bool valid = na < nn;
    if (valid) node_coords<D>(g, na, c);
    float4_t acc0, acc1;
    for (int e = 0; e < 4; ++e) {
      acc0[e] = bs[lm];
      acc1[e] = bs[16 + lm];
    }
    for (int t = 0; t < NTAP; ++t) {
      const int64_t m = valid ? tap_neighbour<D>(g, c, t, s, 1) : -1;
#pragma unroll
      for (int kc = 0; kc < C / 16; ++kc) {
        const int ch = kc * 16 + lk;
        half4_t a;
        if (m >= 0) {
          const float4 xv = *reinterpret_cast<const float4 *>(in + m * C + ch);
          a[0] = (_Float16)xv.x;
          a[1] = (_Float16)xv.y;
          a[2] = (_Float16)xv.z;
          a[3] = (_Float16)xv.w;
        } else {
          a[0] = a[1] = a[2] = a[3] = (_Float16)0.0f;
        }
        const half4_t b0 = *reinterpret_cast<const half4_t *>(&Wt[(t * C + lm) * C + ch]);
        const half4_t b1 = *reinterpret_cast<const half4_t *>(&Wt[(t * C + 16 + lm) * C + ch]);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x16f16(a, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x16f16(a, b1, acc1, 0, 0, 0);
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t node = tile * 16 + lk + e;
      if (node < nn) {
        out[node * C + lm] = RELU ? fmaxf(acc0[e], 0.0f) : acc0[e];
        out[node * C + 16 + lm] = RELU ? fmaxf(acc1[e], 0.0f) : acc1[e];
      }
    }
  }
}

// the same weights transposed per tap, Wt[t][o][i], for the backward pass
template <int NTAP, int CI, int CO>
__device__ inline void stage_weights_t(const __half *__restrict__ w, float *Wt) {
  for (int k = threadIdx.x; k < NTAP * CI * CO; k += blockDim.x) {
    const int t = k / (CI * CO), i = (k / CO) % CI, o = k % CO;
    Wt[(t * CO + o) * CI + i] = __half2float(w[k]);
  }
  __syncthreads();
}

// gin[m, i] = sum_{t,o} W[t,i,o] g'[m - s (t-1), o] with g' = gout masked by
// the layer's ReLU (act_out > 0) when MASK
template <int D, int CI, int CO, bool MASK>
__global__ __launch_bounds__(kCnnNT) void k_conv_bwd_data(NodeGrid g, int64_t nn, int s,
                                                          const __half *__restrict__ w,
                                                          const float *__restrict__ gout,
                                                          const float *__restrict__ act_out,
                                                          float *__restrict__ gin) {
  constexpr int NTAP = ntaps<D>();
  extern __shared__ float lds[];
  float *Wt = lds;
  stage_weights_t<NTAP, CI, CO>(w, Wt);
  const int64_t n = blockIdx.x * (int64_t)kCnnNT + threadIdx.x;
  if (n >= nn) return;
  int c[3];
  node_coords<D>(g, n, c);
  float acc[CI];
#pragma unroll
  for (int i = 0; i < CI; ++i) acc[i] = 0.0f;
  for (int t = 0; t < NTAP; ++t) {
    const int64_t m = tap_neighbour<D>(g, c, t, s, -1);
    if (m < 0) continue;
    const float *gv = gout + m * CO;
    const float *av = act_out + m * CO;
    const float *wt = Wt + t * CO * CI;
#pragma unroll 2
    for (int o = 0; o < CO; ++o) {
      const float go = MASK ? (av[o] > 0.0f ? gv[o] : 0.0f) : gv[o];
#pragma unroll
      for (int i = 0; i < CI; ++i) acc[i] = fmaf(wt[o * CI + i], go, acc[i]);
    }
  }
  float *y = gin + n * CI;
#pragma unroll
  for (int i = 0; i < CI; ++i) y[i] = acc[i];
}

// partial[chunk][t][i][o] = sum_{n in chunk} in[n + s(t-1), i] g'[n, o] and
// partial bias sums; thread (i, o), i fastest.
template <int D, int CI, int CO, bool MASK>
__global__ __launch_bounds__(kCnnNT) void k_conv_bwd_weight(NodeGrid g, int64_t nn, int s,
                                                            const float *__restrict__ in,
                                                            const float *__restrict__ gout,
                                                            const float *__restrict__ act_out,
                                                            float *__restrict__ partial) {
  constexpr int NTAP = ntaps<D>();
  constexpr int NW = NTAP * CI * CO + CO;
  __shared__ float xs[kCnnBatch][NTAP][CI];
  __shared__ float gs[kCnnBatch][CO];
  const int tid = threadIdx.x;
  const int i = tid % CI, o = tid / CI;
  const bool active = o < CO;
  float acc[NTAP];
#pragma unroll
  for (int t = 0; t < NTAP; ++t) acc[t] = 0.0f;
  float accb = 0.0f;
  const int64_t per = (nn + gridDim.x - 1) / gridDim.x;
  const int64_t n0 = blockIdx.x * per;
  const int64_t n1 = n0 + per < nn ? n0 + per : nn;
  for (int64_t nb = n0; nb < n1; nb += kCnnBatch) {
    __syncthreads();
    for (int k = tid; k < kCnnBatch * NTAP * CI; k += kCnnNT) {
      const int b = k / (NTAP * CI), t = (k / CI) % NTAP, ci = k % CI;
      const int64_t n = nb + b;
      float v = 0.0f;
      if (n < n1) {
        int c[3];
        node_coords<D>(g, n, c);
        const int64_t m = tap_neighbour<D>(g, c, t, s, 1);
        if (m >= 0) v = in[m * CI + ci];
      }
      xs[b][t][ci] = v;
    }
    for (int k = tid; k < kCnnBatch * CO; k += kCnnNT) {
      const int b = k / CO, co = k % CO;
      const int64_t n = nb + b;
      float v = 0.0f;
      if (n < n1) {
        v = gout[n * CO + co];
        if (MASK && !(act_out[n * CO + co] > 0.0f)) v = 0.0f;
      }
      gs[b][co] = v;
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int b = 0; b < kCnnBatch; ++b) {
        const float go = gs[b][o];
        accb += go;
#pragma unroll
        for (int t = 0; t < NTAP; ++t) acc[t] = fmaf(xs[b][t][i], go, acc[t]);
      }
    }
  }
  if (active) {
    float *pp = partial + (int64_t)blockIdx.x * NW;
#pragma unroll
    for (int t = 0; t < NTAP; ++t) pp[(t * CI + i) * CO + o] = acc[t];
    if (i == 0) pp[NTAP * CI * CO + o] = accb;
  }
}

// out[j] = sum over chunks of partial[chunk][j], chunks in order
__global__ void k_reduce_chunks(int nchunks, int nw, const float *__restrict__ partial,
                                float *__restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nw) return;
  float acc = 0.0f;
  for (int c = 0; c < nchunks; ++c) acc += partial[(int64_t)c * nw + j];
  out[j] = acc;
}

// ---- loss ----------------------------------------------------------------------
// partials[b] = (sum (y - T)^2 m, sum T^2 m) over free nodes
__global__ __launch_bounds__(256) void k_loss_partials(int64_t nn, int D, const int *__restrict__ nmap,
                                                       const float *__restrict__ y,
                                                       const float *__restrict__ T,
                                                       double *__restrict__ partials) {
  __shared__ double red[2][4];
  double a = 0.0, b = 0.0;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nn * D;
       k += (int64_t)gridDim.x * blockDim.x) {
    if (nmap[k / D] == kDirichlet) continue;
    const double d = (double)y[k] - (double)T[k];
    a = fma(d, d, a);
    b = fma((double)T[k], (double)T[k], b);
  }
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off);
    b += __shfl_down(b, off);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wv] = a;
    red[1][wv] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 2] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    partials[blockIdx.x * 2 + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

// gy = 2 (y - T) m / sum T^2 m
__global__ void k_loss_grad(int64_t nn, int D, const int *__restrict__ nmap,
                            const float *__restrict__ y, const float *__restrict__ T,
                            const double *__restrict__ scal, float *__restrict__ gy) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= nn * D) return;
  const double den = scal[C_LOSS + 1];
  gy[k] = nmap[k / D] == kDirichlet || !(den > 0.0)
              ? 0.0f
              : (float)(2.0 * ((double)y[k] - (double)T[k]) / den);
}

// d[k] = y[k] at free nodes, 0 at Dirichlet nodes (FP64 out)
__global__ void k_output(int64_t nn, int D, const int *__restrict__ nmap,
                         const float *__restrict__ y, double *__restrict__ d) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= nn * D) return;
  d[k] = nmap[k / D] == kDirichlet ? 0.0 : (double)y[k];
}

// ---- parameters ------------------------------------------------------------------
__global__ void k_to_f16(int64_t n, const float *__restrict__ p, __half *__restrict__ h) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) h[k] = __float2half_rn(p[k]);
}

__global__ void k_adam(int64_t n, float *__restrict__ p, float *__restrict__ m,
                       float *__restrict__ v, const float *__restrict__ g,
                       __half *__restrict__ h, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  const float pk = p[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
  p[k] = pk;
  h[k] = __float2half_rn(pk);
}

inline unsigned blocks(int64_t n, int nt) { return (unsigned)((n + nt - 1) / nt); }

NodeGrid node_grid(const edd_problem *p) {
  NodeGrid g{};
  g.dim = p->g.dim;
  for (int a = 0; a < 3; ++a) g.nn[a] = p->g.nn[a];
  return g;
}

template <int D>
struct Net {
  static constexpr int NTAP = ntaps<D>();
  static constexpr int W = kCnnWidth;
  static constexpr int CIN = 1 + D;

  static size_t lds(int ci, int co) { return sizeof(float) * ((size_t)NTAP * ci * co + co); }

  template <int CI, int CO, bool RELU>
  static void fwd(edd_problem *p, int layer, const float *in, float *out) {
    if (CI == kCnnWidth && CO == kCnnWidth && p->cnn_matrix_cores) {
      const int64_t ntiles = (p->n_nodes + 15) / 16;
      const unsigned nb = (unsigned)std::min<int64_t>((ntiles + 3) / 4, 4096);
      k_conv_fwd_mfma<D, RELU><<<nb, 256, 0, p->stream>>>(
          node_grid(p), p->n_nodes, kCnnDil[layer], p->cnn_w16_d + p->cnn_off[layer], in, out);
      return;
    }
    const auto k = k_conv_fwd<D, CI, CO, RELU>;
    const size_t sh = lds(CI, CO);
    hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    k<<<blocks(p->n_nodes, kCnnNT), kCnnNT, sh, p->stream>>>(
        node_grid(p), p->n_nodes, kCnnDil[layer], p->cnn_w16_d + p->cnn_off[layer], in, out);
  }

  template <int CI, int CO, bool MASK>
  static void bwd(edd_problem *p, int layer, const float *in, const float *gout,
                  const float *act_out, float *gin) {
    constexpr int NW = NTAP * CI * CO + CO;
    k_conv_bwd_weight<D, CI, CO, MASK><<<kCnnChunks, kCnnNT, 0, p->stream>>>(
        node_grid(p), p->n_nodes, kCnnDil[layer], in, gout, act_out, p->cnn_part_d);
    k_reduce_chunks<<<blocks(NW, 256), 256, 0, p->stream>>>(kCnnChunks, NW, p->cnn_part_d,
                                                            p->cnn_grad_d + p->cnn_off[layer]);
    if (gin) {
      const auto k = k_conv_bwd_data<D, CI, CO, MASK>;
      const size_t sh = lds(CI, CO);
      hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
      k<<<blocks(p->n_nodes, kCnnNT), kCnnNT, sh, p->stream>>>(
          node_grid(p), p->n_nodes, kCnnDil[layer], p->cnn_w16_d + p->cnn_off[layer], gout,
          act_out, gin);
    }
  }

  static void forward(edd_problem *p) {
    fwd<CIN, W, true>(p, 0, p->cnn_act_d[0], p->cnn_act_d[1]);
    fwd<W, W, true>(p, 1, p->cnn_act_d[1], p->cnn_act_d[2]);
    fwd<W, W, true>(p, 2, p->cnn_act_d[2], p->cnn_act_d[3]);
    fwd<W, D, false>(p, 3, p->cnn_act_d[3], p->cnn_act_d[4]);
  }

  // gradient of the loss from gy (in cnn_g_d[0], D channels)
  static void backward(edd_problem *p) {
    float *g0 = p->cnn_g_d[0], *g1 = p->cnn_g_d[1];
    // layer 3 (linear): gout = gy (D channels), gin -> g1 (W channels)
    bwd<W, D, false>(p, 3, p->cnn_act_d[3], g0, nullptr, g1);
    // layer 2: gout = g1 masked by act3 > 0
    bwd<W, W, true>(p, 2, p->cnn_act_d[2], g1, p->cnn_act_d[3], g0);
    bwd<W, W, true>(p, 1, p->cnn_act_d[1], g0, p->cnn_act_d[2], g1);
    bwd<CIN, W, true>(p, 0, p->cnn_act_d[0], g1, p->cnn_act_d[1], nullptr);
  }
};

void features(edd_problem *p, const double *E, const double *r) {
  launch_residual_norms(p, r, r, C_RR);
  if (!E) E = p->E_d;
  NodeGrid g = node_grid(p);
  const unsigned nb = blocks(p->n_nodes, 256);
  if (p->g.dim == 2)
    k_features<2><<<nb, 256, 0, p->stream>>>(g, p->g, E, r, p->scal_d, p->cnn_nfree,
                                             p->cnn_act_d[0]);
  else
    k_features<3><<<nb, 256, 0, p->stream>>>(g, p->g, E, r, p->scal_d, p->cnn_nfree,
                                             p->cnn_act_d[0]);
}

void forward(edd_problem *p) {
  if (p->g.dim == 2) Net<2>::forward(p);
  else Net<3>::forward(p);
}

// loss of the current output against cnn_target_d; gy into cnn_g_d[0]
void loss(edd_problem *p) {
  const int D = p->g.dim;
  const int nb = 512;
  k_loss_partials<<<nb, 256, 0, p->stream>>>(p->n_nodes, D, p->nmap_d, p->cnn_act_d[4],
                                             p->cnn_target_d, p->partials_d);
  launch_reduce(p, nb, 2, 2, C_LOSS);
  k_loss_grad<<<blocks(p->n_nodes * D, 256), 256, 0, p->stream>>>(
      p->n_nodes, D, p->nmap_d, p->cnn_act_d[4], p->cnn_target_d, p->scal_d, p->cnn_g_d[0]);
}

void target(edd_problem *p, const double *e) {
  launch_residual_norms(p, e, e, C_EE);
  const int D = p->g.dim;
  if (D == 2)
    k_target<2><<<blocks(p->n_nodes * 2, 256), 256, 0, p->stream>>>(p->n_nodes, e, p->scal_d,
                                                                   p->cnn_nfree, p->cnn_target_d);
  else
    k_target<3><<<blocks(p->n_nodes * 3, 256), 256, 0, p->stream>>>(p->n_nodes, e, p->scal_d,
                                                                   p->cnn_nfree, p->cnn_target_d);
}

// gradients of the loss for the pair (r, e) into cnn_grad_d; loss in scal
void loss_grads(edd_problem *p, const double *E, const double *r, const double *e) {
  features(p, E, r);
  target(p, e);
  forward(p);
  loss(p);
  if (p->g.dim == 2) Net<2>::backward(p);
  else Net<3>::backward(p);
}

template <int D>
void layer_offsets(int64_t *off, int64_t *total) {
  const int NTAP = ntaps<D>(), W = kCnnWidth;
  const int ci[kCnnLayers] = {1 + D, W, W, W};
  const int co[kCnnLayers] = {W, W, W, D};
  int64_t o = 0;
  for (int l = 0; l < kCnnLayers; ++l) {
    off[l] = o;
    o += (int64_t)NTAP * ci[l] * co[l] + co[l];
  }
  *total = o;
}

}  // namespace

int cnn_setup(edd_problem *p, int width) {
  if (width != kCnnWidth) return EDD_EINVAL;
  if (p->cnn_nparams) return EDD_OK;  // already set up
  const int D = p->g.dim;
  int64_t total = 0;
  if (D == 2) layer_offsets<2>(p->cnn_off, &total);
  else layer_offsets<3>(p->cnn_off, &total);
  const int64_t nn = p->n_nodes;
  int64_t ndir = 0;
  for (int v : p->nmap_host) ndir += v == kDirichlet;
  p->cnn_nfree = (double)((nn - ndir) * D);
  const int NTAP = D == 2 ? 9 : 27;
  const int64_t nw_max = (int64_t)NTAP * kCnnWidth * kCnnWidth + kCnnWidth;
  float **f32[] = {&p->cnn_master_d, &p->cnn_m_d, &p->cnn_v_d, &p->cnn_grad_d};
  for (float **q : f32) {
    *q = (float *)dev_alloc(p, sizeof(float) * total);
    if (!*q) return EDD_ENOMEM;
  }
  p->cnn_w16_d = (__half *)dev_alloc(p, sizeof(__half) * total);
  p->cnn_part_d = (float *)dev_alloc(p, sizeof(float) * kCnnChunks * nw_max);
  p->cnn_target_d = (float *)dev_alloc(p, sizeof(float) * nn * D);
  const int chans[5] = {1 + D, kCnnWidth, kCnnWidth, kCnnWidth, D};
  for (int l = 0; l < 5; ++l) {
    p->cnn_act_d[l] = (float *)dev_alloc(p, sizeof(float) * nn * chans[l]);
    if (!p->cnn_act_d[l]) return EDD_ENOMEM;
  }
  for (int l = 0; l < 2; ++l) {
    p->cnn_g_d[l] = (float *)dev_alloc(p, sizeof(float) * nn * kCnnWidth);
    if (!p->cnn_g_d[l]) return EDD_ENOMEM;
  }
  if (!p->cnn_w16_d || !p->cnn_part_d || !p->cnn_target_d) return EDD_ENOMEM;
  p->cnn_nparams = total;
  p->cnn_t = 0;
  launch_fill_f32(p, total, p->cnn_master_d);
  launch_fill_f32(p, total, p->cnn_m_d);
  launch_fill_f32(p, total, p->cnn_v_d);
  k_to_f16<<<blocks(total, 256), 256, 0, p->stream>>>(total, p->cnn_master_d, p->cnn_w16_d);
  return check_hip(p, hipGetLastError());
}

int cnn_set_params(edd_problem *p, const float *params) {
  const int64_t n = p->cnn_nparams;
  hipMemcpyAsync(p->cnn_master_d, params, sizeof(float) * n, hipMemcpyDeviceToDevice, p->stream);
  launch_fill_f32(p, n, p->cnn_m_d);
  launch_fill_f32(p, n, p->cnn_v_d);
  p->cnn_t = 0;
  k_to_f16<<<blocks(n, 256), 256, 0, p->stream>>>(n, p->cnn_master_d, p->cnn_w16_d);
  return check_hip(p, hipGetLastError());
}

int cnn_get_params(edd_problem *p, float *params) {
  hipMemcpyAsync(params, p->cnn_master_d, sizeof(float) * p->cnn_nparams,
                 hipMemcpyDeviceToDevice, p->stream);
  return check_hip(p, hipGetLastError());
}

int cnn_predict(edd_problem *p, const double *E, const double *r, double *d) {
  features(p, E, r);
  forward(p);
  const int D = p->g.dim;
  k_output<<<blocks(p->n_nodes * D, 256), 256, 0, p->stream>>>(p->n_nodes, D, p->nmap_d,
                                                              p->cnn_act_d[4], d);
  return check_hip(p, hipGetLastError());
}

int cnn_loss_grad(edd_problem *p, const double *E, const double *r, const double *e, float *grad,
                  double *loss_out) {
  loss_grads(p, E, r, e);
  if (grad)
    hipMemcpyAsync(grad, p->cnn_grad_d, sizeof(float) * p->cnn_nparams, hipMemcpyDeviceToDevice,
                   p->stream);
  int rc = read_scalars(p, C_LOSS, 2);
  if (rc) return rc;
  const double den = p->scal_h[C_LOSS + 1];
  *loss_out = den > 0.0 ? p->scal_h[C_LOSS] / den : 0.0;
  return EDD_OK;
}

int cnn_train_step(edd_problem *p, const double *E, const double *r, const double *e, double lr,
                   double *loss_out) {
  loss_grads(p, E, r, e);
  const int t = ++p->cnn_t;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = (float)(1.0 - std::pow(0.9, t)), c2 = (float)(1.0 - std::pow(0.999, t));
  const int64_t n = p->cnn_nparams;
  k_adam<<<blocks(n, 256), 256, 0, p->stream>>>(n, p->cnn_master_d, p->cnn_m_d, p->cnn_v_d,
                                               p->cnn_grad_d, p->cnn_w16_d, (float)lr, b1, b2,
                                               eps, c1, c2);
  int rc = read_scalars(p, C_LOSS, 2);
  if (rc) return rc;
  const double den = p->scal_h[C_LOSS + 1];
  *loss_out = den > 0.0 ? p->scal_h[C_LOSS] / den : 0.0;
  return EDD_OK;
}

}  // namespace edd

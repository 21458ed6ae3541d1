// Element-level kernels: matrix-free K(E) u, band assembly of the interior
// blocks K_{I_i I_i}, and the gathers/scatters between nodal, interior and
// interface vectors.
//
// K(E) = sum_e E_e P_e^T K0 P_e (the linear dependence on the element
// weights of eq. (NumberTen)); K0 is the unit-modulus element matrix of the
// Q1 quadrilateral (plane stress) or trilinear hexahedron, built on the host
// by Gauss quadrature.  Products are evaluated node by node (each thread owns
// the rows of one node and gathers its neighbourhood), so no floating-point
// atomics are used and results are bitwise reproducible.
#include "internal.h"

namespace edd {
namespace {

constexpr int kBlock = 256;

// Local corner numbering: counter-clockwise in the (x, y) face, z = 0 face
// first for hexahedra.
__host__ __device__ constexpr int corner_of(int ox, int oy, int oz) {
  return (oy ? (ox ? 2 : 3) : (ox ? 1 : 0)) + 4 * oz;
}
__host__ __device__ constexpr int corner_x(int a) { return (a & 3) == 1 || (a & 3) == 2; }
__host__ __device__ constexpr int corner_y(int a) { return (a & 3) >= 2; }
__host__ __device__ constexpr int corner_z(int a) { return a >= 4; }

struct Src {
  // MODE 0: full nodal vector u (clamped nodes read as 0)
  // MODE 1: interior/interface packed vectors through the node map
  const double *u;
  const double *xI;
  const double *xG;
  double sI, sG;
};

template <int D, int MODE>
__device__ inline void fetch_node(const Src &s, const int *__restrict__ nmap,
                                  int node, double *v) {
  const int code = nmap[node];
  if (MODE == 0) {
    if (code == kDirichlet) {
#pragma unroll
      for (int c = 0; c < D; ++c) v[c] = 0.0;
    } else {
#pragma unroll
      for (int c = 0; c < D; ++c) v[c] = s.u[(int64_t)D * node + c];
    }
  } else {
    if (code >= 0) {
      if (s.xI) {
#pragma unroll
        for (int c = 0; c < D; ++c) v[c] = s.sI * s.xI[code + c];
      } else {
#pragma unroll
        for (int c = 0; c < D; ++c) v[c] = 0.0;
      }
    } else if (code != kDirichlet && s.xG) {
      const int64_t gi = gamma_index(code);
#pragma unroll
      for (int c = 0; c < D; ++c) v[c] = s.sG * s.xG[D * gi + c];
    } else {
#pragma unroll
      for (int c = 0; c < D; ++c) v[c] = 0.0;
    }
  }
}

// y(node) = sum over the elements around the node of E_e * (K0 row block of
// the node's corner) * (element dofs).
template <int D, int MODE>
__global__ __launch_bounds__(kBlock) void k_apply(
    Geom g, const double *__restrict__ K0, const double *__restrict__ E,
    const int *__restrict__ nmap, const int *__restrict__ tgt, int64_t ntgt,
    Src src, const double *__restrict__ base, double sy,
    double *__restrict__ out) {
  constexpr int NC = (D == 3) ? 8 : 4;
  constexpr int ND = D * NC;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= ntgt) return;
  const int node = tgt ? tgt[t] : (int)t;
  const int i = node % g.nn[0];
  const int rem = node / g.nn[0];
  const int j = rem % g.nn[1];
  const int k = rem / g.nn[1];
  double y[D];
#pragma unroll
  for (int c = 0; c < D; ++c) y[c] = 0.0;

#pragma unroll
  for (int sz = 0; sz < (D == 3 ? 2 : 1); ++sz) {
#pragma unroll
    for (int sy_ = 0; sy_ < 2; ++sy_) {
#pragma unroll
      for (int sx = 0; sx < 2; ++sx) {
        const int ex = i - 1 + sx, ey = j - 1 + sy_;
        const int ez = (D == 3) ? k - 1 + sz : 0;
        if (ex < 0 || ex >= g.nel[0] || ey < 0 || ey >= g.nel[1]) continue;
        if (D == 3 && (ez < 0 || ez >= g.nel[2])) continue;
        const int64_t e = ex + (int64_t)g.nel[0] * (ey + (int64_t)g.nel[1] * ez);
        const double Ee = E[e];
        const int a = corner_of(1 - sx, 1 - sy_, D == 3 ? 1 - sz : 0);
        double xe[ND];
#pragma unroll
        for (int b = 0; b < NC; ++b) {
          const int nb = (ex + corner_x(b)) +
                         g.nn[0] * ((ey + corner_y(b)) + g.nn[1] * (ez + corner_z(b)));
          fetch_node<D, MODE>(src, nmap, nb, xe + D * b);
        }
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const double *row = K0 + (a * D + c) * ND;
          double acc = 0.0;
#pragma unroll
          for (int m = 0; m < ND; ++m) acc = fma(row[m], xe[m], acc);
          y[c] = fma(Ee, acc, y[c]);
        }
      }
    }
  }
  if (MODE == 0) {
    const bool dir = nmap[node] == kDirichlet;
#pragma unroll
    for (int c = 0; c < D; ++c) out[(int64_t)D * node + c] = dir ? 0.0 : y[c];
  } else {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const double b0 = base ? base[(int64_t)D * node + c] : 0.0;
      out[D * t + c] = fma(sy, y[c], b0);
    }
  }
}

// The same K apply on a tile of nodes per block, with the tile's source
// values (one-node halo), the moduli of the elements touching it and K0
// staged in LDS: each source value, node-map entry and modulus is read once
// per tile instead of once per element corner, and out-of-grid elements
// enter with modulus zero.  TGT 0: every node, out[D node + c] (Dirichlet
// rows 0); TGT 1: interior nodes, out[code + c]; TGT 2: interface nodes,
// out[D gamma + c]; for TGT 1, 2 out = sy y + base[D node + c].
// Node tiles of 256 nodes (one per thread); the autotuner picks the shape
// for each kind of target (edd_problem::apply_variant).  The shape changes only how the source
// halo is staged, never the arithmetic of a node's row, so every shape gives
// bitwise the same result.
template <int D, int V>
struct Tile;
template <>
struct Tile<2, 0> {
  static constexpr int X = 16, Y = 16, Z = 1;
};
template <>
struct Tile<2, 1> {
  static constexpr int X = 32, Y = 8, Z = 1;
};
template <>
struct Tile<2, 2> {
  static constexpr int X = 64, Y = 4, Z = 1;
};
template <>
struct Tile<3, 0> {
  static constexpr int X = 8, Y = 8, Z = 4;
};
template <>
struct Tile<3, 1> {
  static constexpr int X = 16, Y = 4, Z = 4;
};
template <>
struct Tile<3, 2> {
  static constexpr int X = 16, Y = 8, Z = 2;
};

template <int D, int MODE, int TGT, int V>
__global__ __launch_bounds__(256) void k_apply_tiled(
    Geom g, const double *__restrict__ K0, const double *__restrict__ E,
    const int *__restrict__ nmap, Src src, const double *__restrict__ base, double sy,
    double *__restrict__ out) {
  constexpr int TX = Tile<D, V>::X, TY = Tile<D, V>::Y, TZ = Tile<D, V>::Z;
  constexpr int HX = TX + 2, HY = TY + 2, HZ = (D == 3) ? TZ + 2 : 1;
  constexpr int EX = TX + 1, EY = TY + 1, EZ = (D == 3) ? TZ + 1 : 1;
  constexpr int NC = (D == 3) ? 8 : 4;
  constexpr int ND = D * NC;
  // one plane per component: neighbouring threads read neighbouring words
  // (a node-interleaved layout put them 8 * D bytes apart, into the same banks)
  constexpr int NQ = HX * HY * HZ;
  __shared__ double us[NQ * D];
  __shared__ double Es[EX * EY * EZ];
  const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY, k0 = blockIdx.z * TZ;
#pragma unroll 1
  for (int q = threadIdx.x; q < HX * HY * HZ; q += 256) {
    const int hx = q % HX, hy = (q / HX) % HY, hz = q / (HX * HY);
    const int x = i0 - 1 + hx, y = j0 - 1 + hy, z = (D == 3) ? k0 - 1 + hz : 0;
    double v[D];
    if (x >= 0 && x < g.nn[0] && y >= 0 && y < g.nn[1] && z >= 0 && z < g.nn[2]) {
      fetch_node<D, MODE>(src, nmap, x + g.nn[0] * (y + g.nn[1] * z), v);
    } else {
#pragma unroll
      for (int c = 0; c < D; ++c) v[c] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < D; ++c) us[c * NQ + q] = v[c];
  }
#pragma unroll 1
  for (int q = threadIdx.x; q < EX * EY * EZ; q += 256) {
    const int ex = i0 - 1 + q % EX, ey = j0 - 1 + (q / EX) % EY;
    const int ez = (D == 3) ? k0 - 1 + q / (EX * EY) : 0;
    const bool in = ex >= 0 && ex < g.nel[0] && ey >= 0 && ey < g.nel[1] &&
                    (D == 2 || (ez >= 0 && ez < g.nel[2]));
    Es[q] = in ? E[ex + (int64_t)g.nel[0] * (ey + (int64_t)g.nel[1] * ez)] : 0.0;
  }
  __syncthreads();
  const int tx = threadIdx.x % TX, ty = (threadIdx.x / TX) % TY, tz = threadIdx.x / (TX * TY);
  const int i = i0 + tx, j = j0 + ty, kk = (D == 3) ? k0 + tz : 0;
  if (i >= g.nn[0] || j >= g.nn[1] || kk >= g.nn[2]) return;
  const int64_t node = i + (int64_t)g.nn[0] * (j + (int64_t)g.nn[1] * kk);
  const int code = nmap[node];
  if (TGT == 1 && code < 0) return;
  if (TGT == 2 && (code >= 0 || code == kDirichlet)) return;
  double yv[D];
#pragma unroll
  for (int c = 0; c < D; ++c) yv[c] = 0.0;
  // one element at a time (bounded register use; unrolling the pair along x
  // costs occupancy and measured slower), K0 rows through the scalar cache
#pragma unroll 1
  for (int sz = 0; sz < (D == 3 ? 2 : 1); ++sz) {
#pragma unroll 1
    for (int sy_ = 0; sy_ < 2; ++sy_) {
#pragma unroll 1
      for (int sx = 0; sx < 2; ++sx) {
        // element (i-1+sx, j-1+sy, k-1+sz): its tile index, and this node's
        // corner in it
        const double Ee = Es[(tx + sx) + EX * ((ty + sy_) + EY * (D == 3 ? tz + sz : 0))];
        const int a = corner_of(1 - sx, 1 - sy_, D == 3 ? 1 - sz : 0);
        double xe[ND];
#pragma unroll
        for (int b = 0; b < NC; ++b) {
          const int hq = (tx + sx + corner_x(b)) +
                         HX * ((ty + sy_ + corner_y(b)) +
                               HY * (D == 3 ? tz + sz + corner_z(b) : 0));
#pragma unroll
          for (int c = 0; c < D; ++c) xe[D * b + c] = us[c * NQ + hq];
        }
#pragma unroll
        for (int c = 0; c < D; ++c) {
          // wave-uniform row: read through the scalar cache into SGPRs
          const double *row = K0 + (a * D + c) * ND;
          double acc = 0.0;
#pragma unroll
          for (int m = 0; m < ND; ++m) acc = fma(row[m], xe[m], acc);
          yv[c] = fma(Ee, acc, yv[c]);
        }
      }
    }
  }
  if (TGT == 0) {
    const bool dir = code == kDirichlet;
#pragma unroll
    for (int c = 0; c < D; ++c) out[(int64_t)D * node + c] = dir ? 0.0 : yv[c];
  } else {
    const int64_t o = TGT == 1 ? (int64_t)code : (int64_t)D * gamma_index(code);
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const double b0 = base ? base[(int64_t)D * node + c] : 0.0;
      out[o + c] = fma(sy, yv[c], b0);
    }
  }
}

// Global coordinates of local dof p of a band block.
__device__ inline void block_coords(const SubDesc &s, int D, int p, int (&x)[3], int &c) {
  const int l = p / D;
  c = p - l * D;
  const int loc[3] = {l % s.len[0], (l / s.len[0]) % s.len[1], l / (s.len[0] * s.len[1])};
  x[0] = x[1] = x[2] = 0;
  for (int a = 0; a < D; ++a) x[s.ax[a]] = s.lo[s.ax[a]] + (a == 2 ? s.dir : 1) * loc[a];
}

// K entry between dof c1 of node x1 and dof c2 of node x2: the sum over the
// elements holding both nodes of E_e K0[(a2,c2), (a1,c1)].
template <int D>
__device__ inline double pair_entry(const Geom &g, const double *__restrict__ K0,
                                    const double *__restrict__ E, const int (&x1)[3], int c1,
                                    const int (&x2)[3], int c2) {
  constexpr int NC = (D == 3) ? 8 : 4;
  constexpr int ND = D * NC;
  for (int a = 0; a < D; ++a) {
    const int df = x2[a] - x1[a];
    if (df < -1 || df > 1) return 0.0;
  }
  int e0[3], e1[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a >= D) { e0[a] = 0; e1[a] = 0; continue; }
    if (x1[a] == x2[a]) { e0[a] = x1[a] - 1; e1[a] = x1[a]; }
    else { e0[a] = min(x1[a], x2[a]); e1[a] = e0[a]; }
    e0[a] = max(e0[a], 0);
    e1[a] = min(e1[a], g.nel[a] - 1);
  }
  double val = 0.0;
  for (int ez = e0[2]; ez <= e1[2]; ++ez)
    for (int ey = e0[1]; ey <= e1[1]; ++ey)
      for (int ex = e0[0]; ex <= e1[0]; ++ex) {
        const int a1 = corner_of(x1[0] - ex, x1[1] - ey, D == 3 ? x1[2] - ez : 0);
        const int a2 = corner_of(x2[0] - ex, x2[1] - ey, D == 3 ? x2[2] - ez : 0);
        const int64_t el = ex + (int64_t)g.nel[0] * (ey + (int64_t)g.nel[1] * ez);
        val = fma(E[el], K0[(a2 * D + c2) * ND + a1 * D + c1], val);
      }
  return val;
}

// One thread per stored band entry (column p, offset r) of every band block:
// K[q, p] with q = p + r, summed over the elements shared by the two nodes;
// padding columns p >= n get an identity diagonal.
//
// Most entries of the band are structural zeros.  A block numbers its nodes
// with strides 1, len0 and len0*len1, so two nodes can only be neighbours if
// their index difference d (>= 0 here) is within one of 0, len0 or, in 3D,
// len0*len1 of a multiple in {-1, 0, 1}; every other entry is zero without
// decoding coordinates.  Candidates still go through the full test, so the
// band is the same as with it alone.  A block's entries fit 32-bit indices.
template <int D>
__global__ __launch_bounds__(kBlock) void k_assemble_band(
    Geom g, const double *__restrict__ K0, const double *__restrict__ E,
    const SubDesc *__restrict__ subs, double *__restrict__ fac) {
  const SubDesc s = subs[blockIdx.y];
  const int ld = s.kd + 1;
  const int total = s.np * ld;
  const int l0 = s.len[0], plane = s.len[0] * s.len[1];
  auto near = [&](int t) {  // t = dx + l0 dy with |dx|, |dy| <= 1 possible
    return (t >= -1 && t <= 1) || (t >= l0 - 1 && t <= l0 + 1) || (t >= -l0 - 1 && t <= -l0 + 1);
  };
  double *band = fac + s.fac_off;
  const double rld = 1.0 / ld;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    // e / ld from the FP64 reciprocal: off by at most one, then corrected
    int p = (int)((double)e * rld);
    int r = e - p * ld;
    if (r < 0) { --p; r += ld; }
    if (r >= ld) { ++p; r -= ld; }
    const int q = p + r;
    double val = 0.0;
    if (p >= s.n) {
      val = r == 0 ? 1.0 : 0.0;  // identity padding rows
    } else if (q < s.n) {
      const int d = q / D - p / D;
      if (near(d) || (D == 3 && near(d - plane))) {
        int x1[3], x2[3], c1, c2;
        block_coords(s, D, p, x1, c1);
        block_coords(s, D, q, x2, c2);
        val = pair_entry<D>(g, K0, E, x1, c1, x2, c2);
      }
    }
    band[e] = val;
  }
}

// Couplings of a dissected interior: B_h[i][j] = K(tail row i of half h,
// separator dof j), written where W_h will be formed.  blockIdx.y = 2*sep + h.
template <int D>
__global__ __launch_bounds__(kBlock) void k_assemble_coupling(
    Geom g, const double *__restrict__ K0, const double *__restrict__ E,
    const SubDesc *__restrict__ subs, const SepDesc *__restrict__ seps,
    double *__restrict__ W) {
  const SepDesc sd = seps[blockIdx.y >> 1];
  const int h = blockIdx.y & 1;
  const SubDesc leaf = subs[h ? sd.b : sd.a];
  const SubDesc sp = subs[sd.s];
  const int ns = sd.ns;
  double *out = W + sd.w_off + (int64_t)h * ns * sd.ldw;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)ns * ns;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / ns), j = (int)(e - (int64_t)i * ns);
    int x1[3], x2[3], c1, c2;
    block_coords(leaf, D, leaf.n - ns + i, x1, c1);
    block_coords(sp, D, j, x2, c2);
    out[(int64_t)i * sd.ldw + j] = pair_entry<D>(g, K0, E, x2, c2, x1, c1);
  }
}

__global__ __launch_bounds__(kBlock) void k_gather(int dim,
                                                   const int *__restrict__ nodes,
                                                   int64_t n,
                                                   const double *__restrict__ full,
                                                   double *__restrict__ packed) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * dim) return;
  const int64_t node = t / dim;
  const int c = (int)(t - node * dim);
  packed[t] = full[(int64_t)dim * nodes[node] + c];
}

__global__ __launch_bounds__(kBlock) void k_scatter_solution(
    int dim, int64_t n_nodes, const int *__restrict__ nmap,
    const double *__restrict__ uI, const double *__restrict__ uG,
    double *__restrict__ u) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n_nodes * dim) return;
  const int64_t node = t / dim;
  const int c = (int)(t - node * dim);
  const int code = nmap[node];
  double v = 0.0;
  if (code >= 0) v = uI ? uI[code + c] : 0.0;
  else if (code != kDirichlet) v = uG[(int64_t)dim * gamma_index(code) + c];
  u[t] = v;
}

// Per-block count of moduli that are not finite and positive.
__global__ __launch_bounds__(kBlock) void k_check_moduli(
    const double *__restrict__ E, int64_t n, double *__restrict__ partials) {
  __shared__ double red[kBlock / 64];
  double bad = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const double v = E[t];
    bad += (v > 0.0 && v <= 1.7e308) ? 0.0 : 1.0;  // NaN fails both
  }
  for (int o = 32; o > 0; o >>= 1) bad += __shfl_down(bad, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = bad;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += red[w];
    partials[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(kBlock) void k_f32_to_f64(const float *__restrict__ a,
                                                       double *__restrict__ b,
                                                       int64_t n) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) b[t] = (double)a[t];
}

__global__ __launch_bounds__(kBlock) void k_mask_dirichlet(
    int dim, int64_t n_nodes, const int *__restrict__ nmap, double *__restrict__ v) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n_nodes * dim) return;
  if (nmap[t / dim] == kDirichlet) v[t] = 0.0;
}

inline unsigned grid_for(int64_t n) {
  return (unsigned)((n + kBlock - 1) / kBlock);
}

// ---- explicit local Schur complements: the element parts -----------------
// Local interface index of the node at global coordinates (x, y, z) in
// subdomain sd's closure table, or -1.
__device__ inline int schur_local(const SchurDesc &sd, const int *__restrict__ tab, int x, int y,
                                  int z) {
  const int tx = x - sd.c_lo[0], ty = y - sd.c_lo[1], tz = z - sd.c_lo[2];
  if (tx < 0 || ty < 0 || tz < 0 || tx >= sd.c_ext[0] || ty >= sd.c_ext[1] || tz >= sd.c_ext[2])
    return -1;
  return tab[sd.t_off + tx + (int64_t)sd.c_ext[0] * (ty + (int64_t)sd.c_ext[1] * tz)];
}

// Y_i[r][j] = K^i(interior dof r, local interface dof j), r in the band
// order of the subdomain's interior (every element around an interior node
// belongs to the subdomain).  One workgroup per subdomain, a thread per row.
template <int D>
__global__ __launch_bounds__(kBlock) void k_schur_couplings(
    Geom g, const double *__restrict__ K0, const double *__restrict__ E,
    const SubDesc *__restrict__ subs, const SchurDesc *__restrict__ sds,
    const int *__restrict__ tab, double *__restrict__ Y) {
  constexpr int NC = (D == 3) ? 8 : 4, ND = D * NC;
  const SchurDesc sd = sds[blockIdx.x];
  const SubDesc s = subs[sd.blk];
  const int m = sd.m;
  double *Yi = Y + sd.y_off;
  for (int r = threadIdx.x; r < s.n; r += blockDim.x) {
    double *row = Yi + (int64_t)r * m;
    for (int j = 0; j < m; ++j) row[j] = 0.0;
    int x[3], c;
    block_coords(s, D, r, x, c);
    for (int dz = (D == 3 ? -1 : 0); dz <= 0; ++dz)
      for (int dy = -1; dy <= 0; ++dy)
        for (int dx = -1; dx <= 0; ++dx) {
          const int ex = x[0] + dx, ey = x[1] + dy, ez = x[2] + dz;
          if (ex < 0 || ey < 0 || ez < 0 || ex >= g.nel[0] || ey >= g.nel[1] ||
              (D == 3 && ez >= g.nel[2]))
            continue;
          const double Ee = E[ex + (int64_t)g.nel[0] * (ey + (int64_t)g.nel[1] * ez)];
          const int ar = corner_of(x[0] - ex, x[1] - ey, D == 3 ? x[2] - ez : 0);
          for (int k = 0; k < NC; ++k) {
            const int jn = schur_local(sd, tab, ex + corner_x(k), ey + corner_y(k),
                                       ez + (D == 3 ? corner_z(k) : 0));
            if (jn < 0) continue;
            for (int c2 = 0; c2 < D; ++c2)
              row[jn * D + c2] = fma(Ee, K0[(k * D + c2) * ND + ar * D + c], row[jn * D + c2]);
          }
        }
  }
}

// S_i[a][b] += K^i_GG[a][b] over the subdomain's own elements (e_lo..e_hi).
// One workgroup per subdomain, a thread per row a.
template <int D>
__global__ __launch_bounds__(kBlock) void k_schur_kgg(
    Geom g, const double *__restrict__ K0, const double *__restrict__ E,
    const SchurDesc *__restrict__ sds, const int *__restrict__ gl,
    const int *__restrict__ gnode, const int *__restrict__ tab, double *__restrict__ S) {
  constexpr int NC = (D == 3) ? 8 : 4, ND = D * NC;
  const SchurDesc sd = sds[blockIdx.x];
  const int m = sd.m;
  double *Si = S + sd.s_off;
  for (int a = threadIdx.x; a < m; a += blockDim.x) {
    const int an = a / D, c = a - an * D;
    const int node = gnode[gl[sd.g_off + an]];
    const int x[3] = {node % g.nn[0], (node / g.nn[0]) % g.nn[1], node / (g.nn[0] * g.nn[1])};
    double *row = Si + (int64_t)a * m;
    for (int dz = (D == 3 ? -1 : 0); dz <= 0; ++dz)
      for (int dy = -1; dy <= 0; ++dy)
        for (int dx = -1; dx <= 0; ++dx) {
          const int ex = x[0] + dx, ey = x[1] + dy, ez = x[2] + dz;
          if (ex < sd.e_lo[0] || ey < sd.e_lo[1] || ez < sd.e_lo[2] || ex > sd.e_hi[0] ||
              ey > sd.e_hi[1] || ez > sd.e_hi[2])
            continue;
          const double Ee = E[ex + (int64_t)g.nel[0] * (ey + (int64_t)g.nel[1] * ez)];
          const int aa = corner_of(x[0] - ex, x[1] - ey, D == 3 ? x[2] - ez : 0);
          for (int k = 0; k < NC; ++k) {
            const int jn = schur_local(sd, tab, ex + corner_x(k), ey + corner_y(k),
                                       ez + (D == 3 ? corner_z(k) : 0));
            if (jn < 0) continue;
            for (int c2 = 0; c2 < D; ++c2)
              row[jn * D + c2] = fma(Ee, K0[(k * D + c2) * ND + aa * D + c], row[jn * D + c2]);
          }
        }
  }
}

}  // namespace

template <int D, int MODE, int TGT, int V>
void apply_tiled_v(edd_problem *p, const Src &s, const double *base, double sy, double *out) {
  using T = Tile<D, V>;
  dim3 grid((p->g.nn[0] + T::X - 1) / T::X, (p->g.nn[1] + T::Y - 1) / T::Y,
            (p->g.nn[2] + T::Z - 1) / T::Z);
  k_apply_tiled<D, MODE, TGT, V><<<grid, 256, 0, p->stream>>>(p->g, p->K0_d, p->E_d, p->nmap_d,
                                                             s, base, sy, out);
}

template <int D, int MODE, int TGT>
void apply_tiled(edd_problem *p, const Src &s, const double *base, double sy, double *out) {
  switch (p->apply_variant[TGT]) {
    case 1: apply_tiled_v<D, MODE, TGT, 1>(p, s, base, sy, out); break;
    case 2: apply_tiled_v<D, MODE, TGT, 2>(p, s, base, sy, out); break;
    default: apply_tiled_v<D, MODE, TGT, 0>(p, s, base, sy, out); break;
  }
}

void launch_apply_full(edd_problem *p, const double *u, double *y) {
  KTimer kt(p, EDD_KT_APPLY_K);
  Src s{u, nullptr, nullptr, 0.0, 0.0};
  if (p->g.dim == 2) apply_tiled<2, 0, 0>(p, s, nullptr, 1.0, y);
  else apply_tiled<3, 0, 0>(p, s, nullptr, 1.0, y);
}

// Targets are either every interior node (p->inode_d, packed interior
// order) or every interface node (p->gnode_d, Gamma order): the tiled
// kernel writes each through the node map.  Other target lists use the
// node-list kernel.
void launch_apply_mapped(edd_problem *p, const int *tgt, int64_t ntgt,
                         const double *xI, double sI, const double *xG,
                         double sG, const double *base_global, double sy,
                         double *out) {
  if (ntgt == 0) return;
  KTimer kt(p, EDD_KT_APPLY_MAPPED);
  Src s{nullptr, xI, xG, sI, sG};
  const bool D2 = p->g.dim == 2;
  if (tgt == p->inode_d && ntgt == p->n_inodes) {
    if (D2) apply_tiled<2, 1, 1>(p, s, base_global, sy, out);
    else apply_tiled<3, 1, 1>(p, s, base_global, sy, out);
  } else if (tgt == p->gnode_d && ntgt == p->n_gamma) {
    if (D2) apply_tiled<2, 1, 2>(p, s, base_global, sy, out);
    else apply_tiled<3, 1, 2>(p, s, base_global, sy, out);
  } else if (D2) {
    k_apply<2, 1><<<grid_for(ntgt), kBlock, 0, p->stream>>>(
        p->g, p->K0_d, p->E_d, p->nmap_d, tgt, ntgt, s, base_global, sy, out);
  } else {
    k_apply<3, 1><<<grid_for(ntgt), kBlock, 0, p->stream>>>(
        p->g, p->K0_d, p->E_d, p->nmap_d, tgt, ntgt, s, base_global, sy, out);
  }
}

void launch_assemble_band(edd_problem *p) {
  KTimer kt(p, EDD_KT_ASSEMBLE);
  dim3 grid(256, p->n_blk);
  if (p->g.dim == 2)
    k_assemble_band<2><<<grid, kBlock, 0, p->stream>>>(p->g, p->K0_d, p->E_d,
                                                        p->subs_d, p->fac64_d);
  else
    k_assemble_band<3><<<grid, kBlock, 0, p->stream>>>(p->g, p->K0_d, p->E_d,
                                                        p->subs_d, p->fac64_d);
  if (p->n_sep > 0 && p->g.dim == 3)
    k_assemble_coupling<3><<<dim3(64, 2 * p->n_sep), kBlock, 0, p->stream>>>(
        p->g, p->K0_d, p->E_d, p->subs_d, p->seps_d, p->W64_d);
}

void launch_schur_couplings(edd_problem *p) {
  const int n = (int)p->sc_desc.size();
  if (p->g.dim == 2)
    k_schur_couplings<2><<<n, kBlock, 0, p->stream>>>(p->g, p->K0_d, p->E_d, p->subs_d,
                                                       p->sc_desc_d, p->sc_tab_d, p->sc_Y_d);
  else
    k_schur_couplings<3><<<n, kBlock, 0, p->stream>>>(p->g, p->K0_d, p->E_d, p->subs_d,
                                                       p->sc_desc_d, p->sc_tab_d, p->sc_Y_d);
}

void launch_schur_kgg(edd_problem *p) {
  const int n = (int)p->sc_desc.size();
  if (p->g.dim == 2)
    k_schur_kgg<2><<<n, kBlock, 0, p->stream>>>(p->g, p->K0_d, p->E_d, p->sc_desc_d,
                                                 p->sc_gl_d, p->gnode_d, p->sc_tab_d, p->sc_S_d);
  else
    k_schur_kgg<3><<<n, kBlock, 0, p->stream>>>(p->g, p->K0_d, p->E_d, p->sc_desc_d,
                                                 p->sc_gl_d, p->gnode_d, p->sc_tab_d, p->sc_S_d);
}

void launch_gather(edd_problem *p, const int *nodes, int64_t n,
                   const double *full, double *packed) {
  const int64_t m = n * p->g.dim;
  if (m == 0) return;
  k_gather<<<grid_for(m), kBlock, 0, p->stream>>>(p->g.dim, nodes, n, full, packed);
}

void launch_scatter_solution(edd_problem *p, const double *uI,
                             const double *uG, double *u) {
  const int64_t m = p->n_nodes * p->g.dim;
  k_scatter_solution<<<grid_for(m), kBlock, 0, p->stream>>>(
      p->g.dim, p->n_nodes, p->nmap_d, uI, uG, u);
}

void launch_check_moduli(edd_problem *p, const double *E, double *flag_partials) {
  k_check_moduli<<<256, kBlock, 0, p->stream>>>(E, p->n_el, flag_partials);
}

void launch_convert_moduli(edd_problem *p, const void *E, int dtype) {
  if (dtype == EDD_F64) {
    hipMemcpyAsync(p->E_d, E, sizeof(double) * p->n_el, hipMemcpyDeviceToDevice,
                   p->stream);
  } else {
    k_f32_to_f64<<<grid_for(p->n_el), kBlock, 0, p->stream>>>(
        (const float *)E, p->E_d, p->n_el);
  }
}

void launch_mask_dirichlet(edd_problem *p, double *v) {
  const int64_t m = p->n_nodes * p->g.dim;
  k_mask_dirichlet<<<grid_for(m), kBlock, 0, p->stream>>>(p->g.dim, p->n_nodes,
                                                          p->nmap_d, v);
}

}  // namespace edd

// Factorisation behind the interior solves: batched band Cholesky of every
// band block K_{I_i I_i} (eq. (NumberFive): K_II is their direct sum), the
// couplings of dissected interiors (W_h and the separator's Schur
// complement), and the solve layouts the substitutions read.
//
// One workgroup owns one band block; workgroups are launched largest first
// (the order array).  Panel loads are issued unconditionally into the padded
// band storage and out-of-band values are discarded with a select; only
// stores are predicated.
#include <algorithm>

#include "internal.h"

namespace edd {
namespace {

// ---------------------------------------------------------------------------
// Band Cholesky, left-looking.  One thread owns one row of the current
// window (NB panel columns plus the kd rows below them).  For each panel:
//   acc[w, c] = A[j0+w, j0+c] - sum_{k < j0} L[j0+w, k] L[j0+c, k]
// with the L[j0+c, k] (c < NB) staged through LDS in chunks of KC columns
// and the L[j0+w, k] streamed from the band, then the diagonal block is
// factored by wavefront 0 (readlane broadcasts) and the rows below solved
// against it.  Only the panel's own columns are written.
// ---------------------------------------------------------------------------
template <int NB, int NT, int KC, int RPT>
__global__ __launch_bounds__(NT) void k_band_cholesky(
    const SubDesc *__restrict__ subs, const int *__restrict__ order,
    double *__restrict__ fac, int *__restrict__ info) {
  static_assert(NB <= 64, "wavefront 0 factors the diagonal block");
  __shared__ double U[KC][NB];
  __shared__ double Dl[NB][NB + 1];
  __shared__ double Dinv[NB];
  __shared__ int anybad;
  const SubDesc s = subs[order[blockIdx.x]];
  const int n = s.np, kd = s.kd, ld = kd + 1;  // n is a multiple of NB
  double *L = fac + s.fac_off;
  const int tid = threadIdx.x;
  if (tid == 0) anybad = 0;

  for (int j0 = 0; j0 < n; j0 += NB) {
    const int W = min(NB + kd, n - j0);
    // rows w = tid + k*NT of the window are owned by this thread
    double acc[RPT][NB];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int w = tid + k * NT;
      const double *rowp = L + (int64_t)j0 * ld + w;  // (j0+w, j0+c) at rowp + c*kd
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const double v = rowp[c * kd];
        acc[k][c] = (w < W && c <= w && w - c <= kd) ? v : 0.0;
      }
    }
    // left-looking update from columns [kbeg, j0): each U value read from
    // LDS serves the RPT rows of the thread
    const int kbeg = max(0, j0 - kd);
    const int kfirst = j0 + tid - kd;  // first nonzero column of row tid
    for (int kc = kbeg; kc < j0; kc += KC) {
      const int kn = min(KC, j0 - kc);
      __syncthreads();
      for (int e = tid; e < KC * NB; e += NT) {
        const int kk = e / NB, c = e - kk * NB, k = kc + kk;
        const double v = L[(int64_t)k * ld + (j0 + c - k)];
        U[kk][c] = (kk < kn && j0 + c - k <= kd) ? v : 0.0;
      }
      __syncthreads();
      if (tid < W && kc + kn > kfirst) {
        for (int ks = 0; ks < kn; ks += 8) {
          if (kc + ks + 8 <= kfirst) continue;
          double lw[RPT][8];
#pragma unroll
          for (int k = 0; k < RPT; ++k) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int kk = kc + ks + u;
              lw[k][u] = L[(int64_t)kk * ld + (j0 + tid + k * NT - kk)];
            }
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int k = 0; k < RPT; ++k) {
            const int w = tid + k * NT;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int kk = kc + ks + u;
              lw[k][u] = (ks + u < kn && kk >= j0 + w - kd && w < W) ? lw[k][u] : 0.0;
            }
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
#pragma unroll
            for (int c = 0; c < NB; ++c) {
              const double uc = U[ks + u][c];
#pragma unroll
              for (int k = 0; k < RPT; ++k) acc[k][c] = fma(-lw[k][u], uc, acc[k][c]);
            }
          }
        }
      }
    }
    // Diagonal block: wavefront 0 eliminates the first NB columns of its 64
    // rows with lane broadcasts and no per-lane predicates.  Rows w < NB end
    // as the diagonal block of L, rows NB <= w < 64 as final panel rows
    // (right-looking elimination of a row is its triangular solve); entries
    // above the diagonal become garbage that is never read or written back.
    if (tid < 64) {
      const int w = tid;
      bool bad = false;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const double piv = lane_bcast(acc[0][c], c);
        bad = bad || !(piv > 0.0);
        const double dc = sqrt(piv > 0.0 ? piv : 1.0);
        const double rd = 1.0 / dc;
        acc[0][c] = (w == c) ? dc : acc[0][c] * rd;
#pragma unroll
        for (int j = c + 1; j < NB; ++j)
          acc[0][j] = fma(-acc[0][c], lane_bcast(acc[0][c], j), acc[0][j]);
        if (w == 0) Dinv[c] = rd;
      }
      if (bad && w == 0) anybad = 1;
      if (w < NB) {
#pragma unroll
        for (int c = 0; c < NB; ++c) Dl[w][c] = acc[0][c];
      }
    }
    __syncthreads();
    // all other rows: solve against L_D^T, then write the panel back
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int w = tid + k * NT;
      if (w < W && w >= 64) {
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          double x = acc[k][c];
#pragma unroll
          for (int c2 = 0; c2 < c; ++c2) x = fma(-acc[k][c2], Dl[c][c2], x);
          acc[k][c] = x * Dinv[c];
        }
      }
      if (w < W) {
        double *rowp = L + (int64_t)j0 * ld + w;
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c <= w && w - c <= kd) rowp[c * kd] = acc[k][c];
      }
    }
  }
  __syncthreads();
  if (tid == 0) info[order[blockIdx.x]] = anybad;
}

// Band Cholesky for windows of more than 128 rows: the same left-looking
// 32-column panels as k_band_cholesky, with the update
//   S[w, c] = A[j0+w, j0+c] - sum_{k < j0} L[j0+w, k] L[j0+c, k]
// on the FP64 matrix cores (v_mfma_f64_16x16x4f64: lane l supplies
// A(l%16, l/16) and B(l/16, l%16) and holds C rows l/16 + 4e, column l%16).
// Each wavefront owns four 16-row tiles of the window (times two 16-column
// tiles), so a U value read from LDS serves 16 rows instead of one; the A
// operand streams from the band.  Tiles whose rows all lie left of the band
// for a k-step are skipped.  After the update the tiles pass through LDS, 16
// columns at a time, into one row per thread (the transpose area also holds
// the two U buffers).  Wavefront 0 then factors the diagonal block, taking
// each scaled column back from LDS as broadcasts, and the rows below solve
// right-looking against it.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kMxNB = 32, kMxKC = 64, kTransLd = 17;

constexpr int kDlLd = kMxNB + 2;  // 16-byte aligned rows
constexpr int kMxHead = kMxNB * kDlLd + kMxNB + 64 + 2;  // Dl, Dinv, column, flag

constexpr size_t chol_mfma_lds_bytes(int nt) {
  // the small arrays first, so that their reads take immediate offsets,
  // then the transpose area (which also holds the two U buffers)
  return sizeof(double) * ((size_t)kMxHead + (size_t)nt * kTransLd);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_band_cholesky_mfma(
    const SubDesc *__restrict__ subs, const int *__restrict__ order,
    double *__restrict__ fac, int *__restrict__ info) {
  constexpr int NB = kMxNB, KC = kMxKC, NW = NT / 64;
  constexpr int UPT = KC * NB / NT;  // staged U values per thread
  static_assert(NT % 64 == 0 && UPT * NT == KC * NB && NT * kTransLd >= 2 * KC * NB,
                "two U buffers fit the transpose area");
  extern __shared__ __attribute__((aligned(16))) double lds[];
  // DlT[c][r] = L_D[r][c] (rows 16-byte aligned: pairs read as one 16-byte load)
  double (*DlT)[kDlLd] = reinterpret_cast<double (*)[kDlLd]>(lds);
  double *Dinv = lds + NB * kDlLd;
  double *col = Dinv + NB;  // one column of the diagonal block, 64 rows
  int *anybad = reinterpret_cast<int *>(col + 64);
  double *T = lds + kMxHead;  // NT x kTransLd; the two U buffers alias its start
  double *Ubuf = T;
  const SubDesc s = subs[order[blockIdx.x]];
  const int n = s.np, kd = s.kd, ld = kd + 1;  // n is a multiple of NB
  double *L = fac + s.fac_off;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: scalar branches
  const int li = lane & 15, lk = lane >> 4;
  // Wavefront v owns the 16-row tiles v, v+NW, v+2NW, v+3NW: the tiles a
  // chunk of columns reaches (a prefix of the window) spread evenly over the
  // four SIMDs.
  constexpr int TSR = 16 * NW;  // rows between a wavefront's tiles
  const int w0 = wave * 16;     // first window row of its first tile
  if (tid == 0) *anybad = 0;

  for (int j0 = 0; j0 < n; j0 += NB) {
    const int W = min(NB + kd, n - j0);
    const int kt = j0 + w0 - kd;  // first column reaching row w0
    // S starts as the panel of A: tile (rt, ct) slot e holds window row
    // w0 + TSR*rt + lk + 4e, panel column 16ct + li, at L[j0*ld + w + c*kd]
    v4d S[4][2];
    {
      const double *pA = L + (int64_t)j0 * ld + (w0 + lk) + (int64_t)li * kd;
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) {
        const bool on = w0 + TSR * rt < W;  // wave-uniform
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int w = w0 + TSR * rt + lk + 4 * e, c = 16 * ct + li;
            const double v = on ? pA[TSR * rt + 4 * e + (int64_t)16 * ct * kd] : 0.0;
            S[rt][ct][e] = (w < W && c <= w && w - c <= kd) ? v : 0.0;
          }
      }
    }
    const int kbeg = max(0, j0 - kd);
    // U chunks alternate between two buffers; the next chunk's values are
    // loaded into registers before the current chunk's products and stored
    // after them, one barrier per chunk
    double un[UPT];
    auto load_u = [&](int kc) {
      const int kn = min(KC, j0 - kc);
#pragma unroll
      for (int q = 0; q < UPT; ++q) {
        const int e = tid + q * NT, kk = e / NB, c = e - kk * NB, k = kc + kk;
        const double v = L[(int64_t)k * ld + (j0 + c - k)];
        un[q] = (kk < kn && j0 + c - k <= kd) ? v : 0.0;
      }
    };
    auto store_u = [&](double *Ub) {
#pragma unroll
      for (int q = 0; q < UPT; ++q) Ub[tid + q * NT] = un[q];
    };
    __syncthreads();  // the previous panel's columns are written back
    if (kbeg < j0) {
      load_u(kbeg);
      store_u(Ubuf);
    }
    int par = 0;
    for (int kc = kbeg; kc < j0; kc += KC, par ^= 1) {
      const int kn = min(KC, j0 - kc);
      __syncthreads();  // chunk kc visible; the other buffer's readers are done
      const bool more = kc + KC < j0;
      if (more) load_u(kc + KC);
      const double(*U)[NB] = reinterpret_cast<const double(*)[NB]>(Ubuf + par * KC * NB);
      // batches of 8 columns from the first that reaches row w0
      const int ks0 = kt - kc >= 8 ? ((kt - kc) & ~7) : 0;
      if (w0 < W && kc + kn > kt && ks0 < kn) {  // wave-uniform
        // (j0+w, k) sits at L[k*ld + j0+w-k] = L[k*kd + j0+w]: one lane
        // pointer, +TSR per row tile and +4*kd per k-step
        const double *pa = L + (int64_t)(kc + lk) * kd + (j0 + w0 + li);
        const int lead = kc + lk + kd - j0 - w0 - li;  // row offset of the band edge
        double an[2][4];
        auto load_a = [&](int ks) {
          const double *pk = pa + ks * kd;
#pragma unroll
          for (int rt = 0; rt < 4; ++rt) {
            // wave-uniform: the tile is in the window and reaches the batch
            const bool on = w0 + TSR * rt < W && kc + ks + 8 > kt + TSR * rt;
#pragma unroll
            for (int st = 0; st < 2; ++st) an[st][rt] = on ? pk[st * 4 * kd + TSR * rt] : 0.0;
          }
        };
        load_a(ks0);
        for (int ks = ks0; ks < kn; ks += 8) {
          double a[2][4], b[2][2];
#pragma unroll
          for (int st = 0; st < 2; ++st)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) a[st][rt] = an[st][rt];
          if (ks + 8 < kn) load_a(ks + 8);  // in flight during this batch
#pragma unroll
          for (int st = 0; st < 2; ++st)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) b[st][ct] = U[ks + 4 * st + lk][16 * ct + li];
#pragma unroll
          for (int st = 0; st < 2; ++st)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
              // kept: k < j0 (inside this chunk), j0+w-k <= kd, w < W
              const bool in = ks + 4 * st + lk < kn && lead + ks + 4 * st >= TSR * rt &&
                              w0 + TSR * rt + li < W;
              a[st][rt] = in ? -a[st][rt] : 0.0;
            }
#pragma unroll
          for (int st = 0; st < 2; ++st)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
              if (kc + ks + 4 * st + 4 <= kt + TSR * rt || w0 + TSR * rt >= W)
                continue;  // tile left of the band or below the window
#pragma unroll
              for (int ct = 0; ct < 2; ++ct)
                S[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st][rt], b[st][ct],
                                                                  S[rt][ct], 0, 0, 0);
            }
        }
      }
      if (more) store_u(Ubuf + (par ^ 1) * KC * NB);
    }
    // tiles -> one window row per thread (16 columns at a time); T row r
    // holds window row r
    double acc[NB];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      __syncthreads();  // U (first half) or the previous half is consumed
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          T[(w0 + TSR * rt + lk + 4 * e) * kTransLd + li] = S[rt][ct][e];
      __syncthreads();
#pragma unroll
      for (int c = 0; c < 16; ++c) acc[16 * ct + c] = T[tid * kTransLd + c];
    }
    const int w = tid;
    // Diagonal block by wavefront 0 (rows 0..63 of the window, right-looking
    // as in k_band_cholesky).  Each scaled column goes through LDS and is
    // read back as broadcasts; 1/sqrt of the pivot is the hardware estimate
    // refined by two Newton steps, y <- y + y (1 - p y^2) / 2 (each squares
    // the relative error).
    if (tid < 64) {
      bool bad = false;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const double piv = lane_bcast(acc[c], c);
        bad = bad || !(piv > 0.0);
        const double pv = piv > 0.0 ? piv : 1.0;
        double y = __builtin_amdgcn_rsq(pv);
#pragma unroll
        for (int it = 0; it < 2; ++it) y = fma(0.5 * y, fma(-pv * y, y, 1.0), y);
        const double rd = y, dc = pv * y;
        acc[c] = (w == c) ? dc : acc[c] * rd;
        if (w == 0) Dinv[c] = rd;
        if (w < NB) DlT[c][w] = acc[c];
        if (c + 1 < NB) {
          col[w] = acc[c];
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          const double2 *col2 = reinterpret_cast<const double2 *>(col);
#pragma unroll
          for (int q = (c + 1) / 2; q < NB / 2; ++q) {
            const double2 v = col2[q];
            if (2 * q > c) acc[2 * q] = fma(-acc[c], v.x, acc[2 * q]);
            acc[2 * q + 1] = fma(-acc[c], v.y, acc[2 * q + 1]);
            // keep the update here (not sunk to the column's pivot, which
            // would hold every broadcast value live across the loop)
            asm volatile("" : "+v"(acc[2 * q]), "+v"(acc[2 * q + 1]));
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();  // all reads done before the next column is stored
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
      }
      if (bad && w == 0) *anybad = 1;
    }
    __syncthreads();
    // rows below: solve x L_D^T = a, right-looking over the columns of L_D
    if (w < W && w >= 64) {
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        acc[c] *= Dinv[c];
        const double2 *d2 = reinterpret_cast<const double2 *>(DlT[c]);
#pragma unroll
        for (int q = (c + 1) / 2; q < NB / 2; ++q) {
          const double2 v = d2[q];
          if (2 * q > c) acc[2 * q] = fma(-acc[c], v.x, acc[2 * q]);
          acc[2 * q + 1] = fma(-acc[c], v.y, acc[2 * q + 1]);
          if (q % 2 == 1) __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    if (w < W) {
      double *rowp = L + (int64_t)j0 * ld + w;
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c <= w && w - c <= kd) rowp[c * kd] = acc[c];
    }
  }
  __syncthreads();
  if (tid == 0) info[order[blockIdx.x]] = *anybad;
}

// Solve layouts from the factor L (column band, true diagonal):
//   Cs[p*ld + r] = L[p+r, p] with the diagonal replaced by 1/L[p,p]
//   Rs[q*ld + k] = L[q, q-k]  with the diagonal replaced by 1/L[q,q]
// Cs may alias L (then only its diagonals change).  Work comes in 64x64
// tiles (rows q or p, offsets k or r) per subdomain; a row-layout tile's
// sources (q-k, k) lie on a skewed band of the column layout and are read
// along k (contiguous within a column) into LDS, then written along k.
// The only in-place change, the diagonal of column p, is read solely by
// the row-layout tile of the same rows at offsets [0, 64), which writes it.
template <typename T>
__global__ __launch_bounds__(256) void k_solve_layouts(
    const SubDesc *__restrict__ subs, const double *__restrict__ Lf,
    T *__restrict__ Cs, T *__restrict__ Rs) {
  __shared__ double tile[64][65];
  const SubDesc s = subs[blockIdx.y];
  const int n = s.np, kd = s.kd, ld = kd + 1;
  const double *Lb = Lf + s.fac_off;
  T *Cb = Cs + s.fac_off;
  T *Rb = Rs + s.fac_off;
  const bool inplace = (const void *)Cs == (const void *)Lf;
  const int nqt = n / 64, nkt = (ld + 63) / 64;
  for (int t = blockIdx.x; t < nqt * nkt; t += gridDim.x) {
    const int q0 = (t / nkt) * 64, k0 = (t % nkt) * 64;
    const int pmin = q0 - k0 - 63;  // sources p = q - k of this tile
    // all of a thread's loads first (addresses of unused slots clamped to
    // the block's first entry), then the LDS writes
    constexpr int kSlots = (127 * 64 + 255) / 256;
    double v[kSlots];
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
      const int e = threadIdx.x + 256 * j;
      const int kk = e & 63, p = pmin + (e >> 6), k = k0 + kk, qq = p + k - q0;
      const bool in = e < 127 * 64 && qq >= 0 && qq < 64 && k < ld && p >= 0;
      v[j] = Lb[in ? (int64_t)p * ld + k : 0];
    }
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
      const int e = threadIdx.x + 256 * j;
      const int kk = e & 63, p = pmin + (e >> 6), k = k0 + kk, qq = p + k - q0;
      if (e >= 127 * 64 || qq < 0 || qq >= 64 || k >= ld) continue;
      double x = p >= 0 ? v[j] : 0.0;
      if (k == 0) x = 1.0 / x;
      tile[qq][kk] = x;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
      const int qq = e >> 6, k = k0 + (e & 63);
      if (k < ld) Rb[(int64_t)(q0 + qq) * ld + k] = (T)tile[qq][e & 63];
    }
    if (!inplace) {
      double c[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int e = threadIdx.x + 256 * j, pp = e >> 6, r = k0 + (e & 63);
        c[j] = Lb[r < ld ? (int64_t)(q0 + pp) * ld + r : 0];
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int e = threadIdx.x + 256 * j, pp = e >> 6, r = k0 + (e & 63);
        if (r >= ld) continue;
        const double x = r == 0 ? 1.0 / c[j] : c[j];
        Cb[(int64_t)(q0 + pp) * ld + r] = (T)x;
      }
    } else if (k0 == 0) {
      for (int pp = threadIdx.x; pp < 64; pp += blockDim.x)
        Cb[(int64_t)(q0 + pp) * ld] = (T)(1.0 / Lb[(int64_t)(q0 + pp) * ld]);
    }
    __syncthreads();  // the tile is reused by the next iteration
  }
}

// ---------------------------------------------------------------------------
// Dissected interiors: with halves a, b and separator plane S, the factor is
// [L_a 0 0; 0 L_b 0; W_a^T W_b^T L_S] with W_h = L_h^{-1} B_h and
// L_S L_S^T = C - W_a^T W_a - W_b^T W_b; B_h and W_h are nonzero only in the
// last ns rows of half h.
// ---------------------------------------------------------------------------

// W_h = L_h,tail^{-1} B_h in place (B_h as assembled), from the true-diagonal
// factor (before the solve layouts are built).  A block owns 64 columns and
// walks the rows in 64-row blocks: the block's rows minus L(block, earlier)
// times the finished earlier rows (64x64 tiles through LDS), then a
// triangular solve with the diagonal tile, one column per thread and one
// 16-row sub-block per wavefront.
__global__ __launch_bounds__(256) void k_sep_trsm(const SubDesc *__restrict__ subs,
                                                  const SepDesc *__restrict__ seps,
                                                  const double *__restrict__ fac,
                                                  double *__restrict__ W) {
  const SepDesc sd = seps[blockIdx.y >> 1];
  const int h = blockIdx.y & 1;
  const SubDesc leaf = subs[h ? sd.b : sd.a];
  const int ns = sd.ns, ld = leaf.kd + 1, t0 = leaf.n - ns;
  const double *L = fac + leaf.fac_off;
  const int ldw = sd.ldw;
  double *Wh = W + sd.w_off + (int64_t)h * ns * ldw;
  const int c0 = blockIdx.x * 64;
  if (c0 >= ns) return;
  __shared__ double Lt[64][65], Xt[64][65];
  const int tid = threadIdx.x, col = tid & 63, rg = tid >> 6;  // rows rg*16 .. +16
  // L(t0 + a, t0 + b) for a >= b, 0 otherwise; a thread loads its 16 values
  // of a tile together (unused slots read the block's first entry)
  auto in_L = [&](int a, int b) { return a >= b && a < ns && b < ns; };
  auto idx_L = [&](int a, int b) -> int64_t {
    return in_L(a, b) ? (int64_t)(t0 + b) * ld + (a - b) : 0;
  };
  const int nrb = (ns + 63) / 64;
  for (int qb = 0; qb < nrb; ++qb) {
    const int q0 = qb * 64;
    double acc[16];
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      const int q = q0 + rg * 16 + a, j = c0 + col;
      acc[a] = (q < ns && j < ns) ? Wh[(int64_t)q * ldw + j] : 0.0;
    }
    for (int pb = 0; pb < qb; ++pb) {
      const int p0 = pb * 64;
      double vl[16], vx[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int e2 = tid + 256 * i, a = e2 >> 6, b = e2 & 63;
        const int pr = p0 + a, j = c0 + b;
        vl[i] = L[idx_L(q0 + a, p0 + b)];
        vx[i] = Wh[(pr < ns && j < ns) ? (int64_t)pr * ldw + j : 0];
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int e2 = tid + 256 * i, a = e2 >> 6, b = e2 & 63;
        const int pr = p0 + a, j = c0 + b;
        Lt[a][b] = in_L(q0 + a, p0 + b) ? vl[i] : 0.0;
        Xt[a][b] = (pr < ns && j < ns) ? vx[i] : 0.0;
      }
      __syncthreads();
      for (int b = 0; b < 64; ++b) {
        const double x = Xt[b][col];
#pragma unroll
        for (int a = 0; a < 16; ++a) acc[a] = fma(-Lt[rg * 16 + a][b], x, acc[a]);
      }
    }
    {
      double vl[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int e2 = tid + 256 * i, a = e2 >> 6, b = e2 & 63;
        vl[i] = L[idx_L(q0 + a, q0 + b)];
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int e2 = tid + 256 * i, a = e2 >> 6, b = e2 & 63;
        Lt[a][b] = in_L(q0 + a, q0 + b) ? vl[i] : 0.0;
      }
    }
    __syncthreads();
    // Forward substitution with the diagonal tile in 16-row sub-blocks: the
    // wavefront owning sub-block sb solves its rows in registers (unrolled),
    // publishes them through LDS, and the wavefronts below subtract them.
    // Row a still takes its earlier rows in the order 0, 1, ..., a-1.
    const int j = c0 + col;
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
      if (rg == sb) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int r = 16 * sb + i;
          double v = acc[i];
#pragma unroll
          for (int k = 0; k < i; ++k) v = fma(-Lt[r][16 * sb + k], acc[k], v);
          acc[i] = q0 + r < ns ? v / Lt[r][r] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int q = q0 + 16 * sb + i;
          Xt[16 * sb + i][col] = acc[i];
          if (q < ns && j < ns) Wh[(int64_t)q * ldw + j] = acc[i];
        }
      }
      __syncthreads();
      if (rg > sb) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const double x = Xt[16 * sb + k][col];
#pragma unroll
          for (int i = 0; i < 16; ++i) acc[i] = fma(-Lt[16 * rg + i][16 * sb + k], x, acc[i]);
        }
      }
    }
  }
}

// Separator block (band storage with kd = ns - 1, C as assembled) minus
// W_a^T W_a + W_b^T W_b, lower triangle; 32x32 output tiles, one 16x16
// quadrant per wavefront on the matrix cores.
__global__ __launch_bounds__(256) void k_sep_syrk(const SubDesc *__restrict__ subs,
                                                  const SepDesc *__restrict__ seps,
                                                  const double *__restrict__ W,
                                                  double *__restrict__ fac) {
  const SepDesc sd = seps[blockIdx.y];
  const int ns = sd.ns;
  const int nt = (ns + 31) / 32;
  // blockIdx.x enumerates the lower-triangle tiles (tq >= tp)
  int tq = 0, rem = blockIdx.x;
  while (rem > tq) { rem -= tq + 1; ++tq; }
  const int tp = rem;
  if (tq >= nt) return;
  const SubDesc S = subs[sd.s];
  const int ld = S.kd + 1;
  __shared__ double Aq[32][33], Ap[32][33];
  // wavefront (rt, ct) owns the 16x16 quadrant at rows 16rt, columns 16ct of
  // the tile, on the FP64 matrix cores (lane layout as in
  // k_band_cholesky_mfma): A(i, k) = W[k][q0 + i], B(k, j) = W[k][p0 + j]
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4, rt = wave >> 1, ct = wave & 1;
  v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
  for (int h = 0; h < 2; ++h) {
    const double *Wh = W + sd.w_off + (int64_t)h * ns * sd.ldw;
    for (int k0 = 0; k0 < ns; k0 += 32) {
      // a thread's eight loads first (unused slots read the first entry)
      double vq[4], vp[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int e = threadIdx.x + 256 * j, kk = e >> 5, c = e & 31, k = k0 + kk;
        const int q = tq * 32 + c, pcol = tp * 32 + c;
        vq[j] = Wh[(k < ns && q < ns) ? (int64_t)k * sd.ldw + q : 0];
        vp[j] = Wh[(k < ns && pcol < ns) ? (int64_t)k * sd.ldw + pcol : 0];
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int e = threadIdx.x + 256 * j, kk = e >> 5, c = e & 31, k = k0 + kk;
        const int q = tq * 32 + c, pcol = tp * 32 + c;
        Aq[kk][c] = (k < ns && q < ns) ? vq[j] : 0.0;
        Ap[kk][c] = (k < ns && pcol < ns) ? vp[j] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < 32; ks += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Aq[ks + lk][16 * rt + li],
                                                   Ap[ks + lk][16 * ct + li], acc, 0, 0, 0);
    }
  }
  double *band = fac + S.fac_off;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int q = tq * 32 + 16 * rt + lk + 4 * e, pcol = tp * 32 + 16 * ct + li;
    if (q < ns && pcol <= q) band[(int64_t)pcol * ld + (q - pcol)] -= acc[e];
  }
}

__global__ void k_f64_to_f32(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

template <int NT, int RPT>
void chol_launch(edd_problem *p, const int *order, int count) {
  if (count <= 0) return;
  k_band_cholesky<32, NT, 64, RPT><<<count, NT, 0, p->stream>>>(
      p->subs_d, order, p->fac64_d, p->info_d);
}

template <int NT>
void chol_launch_mfma(edd_problem *p, const int *order, int count) {
  if (count <= 0) return;
  set_lds_limit_once((const void *)k_band_cholesky_mfma<NT>, p);
  k_band_cholesky_mfma<NT><<<count, NT, chol_mfma_lds_bytes(NT), p->stream>>>(
      p->subs_d, order, p->fac64_d, p->info_d);
}

}  // namespace

static void cholesky_subset(edd_problem *p, const int *order, int count) {
  const int rows = 32 + p->max_kd;  // window rows
  // windows over 128 rows on the matrix cores (a wavefront per 64 rows)
  const bool mx = chol_mfma_lds_bytes(1024) <= p->lds_limit;
  if (rows <= 64) chol_launch<64, 1>(p, order, count);
  else if (rows <= 128) chol_launch<128, 1>(p, order, count);
  else if (rows <= 256) mx ? chol_launch_mfma<256>(p, order, count) : chol_launch<128, 2>(p, order, count);
  else if (rows <= 512) mx ? chol_launch_mfma<512>(p, order, count) : chol_launch<256, 2>(p, order, count);
  else if (mx) chol_launch_mfma<1024>(p, order, count);  // kd <= 992 (checked at setup)
  else chol_launch<1024, 1>(p, order, count);
}

// Factor every band block; for dissected interiors the halves first, then
// W_h and the separator's Schur complement, then the separator.
void launch_band_cholesky(edd_problem *p) {
  KTimer kt(p, EDD_KT_BAND_CHOLESKY);
  const int nleaf = p->n_blk - p->n_sep;
  cholesky_subset(p, p->order_leaf_d, nleaf);
  if (p->n_sep > 0) {
    int maxns = 0;
    for (const SepDesc &sd : p->seps) maxns = std::max(maxns, sd.ns);
    k_sep_trsm<<<dim3((maxns + 63) / 64, 2 * p->n_sep), 256, 0, p->stream>>>(
        p->subs_d, p->seps_d, p->fac64_d, p->W64_d);
    const int nt = (maxns + 31) / 32;
    k_sep_syrk<<<dim3(nt * (nt + 1) / 2, p->n_sep), 256, 0, p->stream>>>(
        p->subs_d, p->seps_d, p->W64_d, p->fac64_d);
    cholesky_subset(p, p->order_sep_d, p->n_sep);
  }
}

// After the factorisation: build the solve layouts (FP64 always, FP32 when
// requested).  The FP64 column layout overwrites the factor in place.
void launch_band_layouts(edd_problem *p) {
  KTimer kt(p, EDD_KT_LAYOUTS);
  dim3 grid(64, p->n_blk);
  if (p->n_sep > 0 && p->W32_d)
    k_f64_to_f32<<<(unsigned)((p->w_alloc + 255) / 256), 256, 0, p->stream>>>(
        p->w_alloc, p->W64_d, p->W32_d);
  if (p->fac32_d)
    k_solve_layouts<float><<<grid, 256, 0, p->stream>>>(p->subs_d, p->fac64_d,
                                                        p->fac32_d, p->rac32_d);
  k_solve_layouts<double><<<grid, 256, 0, p->stream>>>(p->subs_d, p->fac64_d,
                                                       p->fac64_d, p->rac64_d);
}

}  // namespace edd

// Batched interior solves: band Cholesky factorisation of every subdomain
// block K_{I_i I_i} and the forward/backward substitutions that apply
// K_II^{-1} (K_II is the direct sum of the subdomain blocks, eq.
// (NumberFive); all 2N+1 subproblems of eq. (3MatSplit2) use these solves).
//
// One workgroup owns one subdomain.  Workgroups are launched largest first
// (the order array), so that round-robin dispatch over the XCDs spreads the
// large blocks evenly.
//
// Factorisation: left-looking band Cholesky, see k_band_cholesky.
//
// Substitution: the whole right-hand side of a subdomain lives in LDS.  The
// forward sweep reads the factor by columns, the backward sweep a row-major
// copy of it, so both are "update" sweeps with coalesced loads and no
// reductions; both copies store reciprocal diagonals.
//
// The band storage is padded before the first and after the last subdomain
// (kBandPadFront / band_pad_back entries), so panel loads are issued
// unconditionally and out-of-band values are discarded with a select; only
// stores are predicated.  This keeps many loads in flight per thread.
#include <mutex>
#include <utility>
#include <vector>

#include "internal.h"

namespace edd {
namespace {

// Raise a kernel's dynamic LDS limit to the device's, once per (kernel,
// device); thread-safe.
void set_lds_limit_once(const void *kernel, const edd_problem *p) {
  static std::mutex mu;
  static std::vector<std::pair<const void *, int>> done;
  std::lock_guard<std::mutex> lk(mu);
  for (const auto &d : done)
    if (d.first == kernel && d.second == p->device) return;
  hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p->lds_limit);
  done.emplace_back(kernel, p->device);
}

template <typename T>
__device__ inline T lane_bcast(T v, int lane);
template <>
__device__ inline double lane_bcast<double>(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <>
__device__ inline float lane_bcast<float>(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

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

// Band Cholesky for wide windows (more than 512 rows), same panels as
// k_band_cholesky but with the update
//   S[w, c] = -sum_{k < j0} L[j0+w, k] L[j0+c, k]
// on the FP64 matrix cores (v_mfma_f64_16x16x4f64: lane l supplies
// A(l%16, l/16) and B(l/16, l%16) and holds C rows l/16 + 4e, column l%16).
// Wavefront v owns window rows 64v..64v+63 as 4 x 2 tiles of 16 x 16, so a
// U value read from LDS serves 16 rows instead of one; the A operand streams
// from the band exactly as before.  Tiles whose 16 rows all lie left of the
// band for a k-step are skipped.  After the update the tiles pass through
// LDS, 16 columns at a time, into one row per thread (the transpose buffer
// reuses the U staging area), and the diagonal block and the row solves
// proceed as in k_band_cholesky.
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
  const int w0 = wave * 64;  // first window row of this wavefront
  if (tid == 0) *anybad = 0;

  for (int j0 = 0; j0 < n; j0 += NB) {
    const int W = min(NB + kd, n - j0);
    const int kt = j0 + w0 - kd;  // first column reaching row w0
    // S starts as the panel of A: tile (rt, ct) slot e holds window row
    // w0 + 16rt + lk + 4e, panel column 16ct + li, at L[j0*ld + w + c*kd]
    v4d S[4][2];
    if (w0 < W) {  // wave-uniform
      const double *pA = L + (int64_t)j0 * ld + (w0 + lk) + (int64_t)li * kd;
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int w = w0 + 16 * rt + lk + 4 * e, c = 16 * ct + li;
            const double v = pA[16 * rt + 4 * e + (int64_t)16 * ct * kd];
            S[rt][ct][e] = (w < W && c <= w && w - c <= kd) ? v : 0.0;
          }
    } else {
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) S[rt][ct] = v4d{0.0, 0.0, 0.0, 0.0};
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
        // pointer, +16 per row tile and +4*kd per k-step
        const double *pa = L + (int64_t)(kc + lk) * kd + (j0 + w0 + li);
        const int lead = kc + lk + kd - j0 - w0 - li;  // row offset of the band edge
        double an[2][4];
        auto load_a = [&](int ks) {
          const double *pk = pa + ks * kd;
#pragma unroll
          for (int st = 0; st < 2; ++st)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) an[st][rt] = pk[st * 4 * kd + 16 * rt];
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
              const bool in = ks + 4 * st + lk < kn && lead + ks + 4 * st >= 16 * rt &&
                              w0 + 16 * rt + li < W;
              a[st][rt] = in ? -a[st][rt] : 0.0;
            }
#pragma unroll
          for (int st = 0; st < 2; ++st)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
              if (kc + ks + 4 * st + 4 <= kt + 16 * rt) continue;  // tile left of the band
#pragma unroll
              for (int ct = 0; ct < 2; ++ct)
                S[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st][rt], b[st][ct],
                                                                  S[rt][ct], 0, 0, 0);
            }
        }
      }
      if (more) store_u(Ubuf + (par ^ 1) * KC * NB);
    }
    // tiles -> one window row per thread (16 columns at a time)
    double acc[NB];
    double *Tw = T + w0 * kTransLd;
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      __syncthreads();  // U (first half) or the previous half is consumed
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e) Tw[(16 * rt + lk + 4 * e) * kTransLd + li] = S[rt][ct][e];
      __syncthreads();
#pragma unroll
      for (int c = 0; c < 16; ++c) acc[16 * ct + c] = Tw[lane * kTransLd + c];
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
    for (int e = threadIdx.x; e < 127 * 64; e += blockDim.x) {
      const int kk = e & 63, p = pmin + (e >> 6), k = k0 + kk, qq = p + k - q0;
      if (qq < 0 || qq >= 64 || k >= ld) continue;
      double v = p >= 0 ? Lb[(int64_t)p * ld + k] : 0.0;
      if (k == 0) v = 1.0 / v;
      tile[qq][kk] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
      const int qq = e >> 6, k = k0 + (e & 63);
      if (k < ld) Rb[(int64_t)(q0 + qq) * ld + k] = (T)tile[qq][e & 63];
    }
    if (!inplace) {
      for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
        const int pp = e >> 6, r = k0 + (e & 63);
        if (r >= ld) continue;
        double v = Lb[(int64_t)(q0 + pp) * ld + r];
        if (r == 0) v = 1.0 / v;
        Cb[(int64_t)(q0 + pp) * ld + r] = (T)v;
      }
    } else if (k0 == 0) {
      for (int pp = threadIdx.x; pp < 64; pp += blockDim.x)
        Cb[(int64_t)(q0 + pp) * ld] = (T)(1.0 / Lb[(int64_t)(q0 + pp) * ld]);
    }
    __syncthreads();  // the tile is reused by the next iteration
  }
}

// ---------------------------------------------------------------------------
// Substitutions.  Block b of 64 rows is owned by wavefront b mod NW (row i
// by thread i mod NT), so the owner can solve its diagonal block with the
// values it updated itself; one barrier per block publishes the block.
// ---------------------------------------------------------------------------
template <typename T, typename W, int NT>
__global__ __launch_bounds__(NT) void k_band_solve(
    const SubDesc *__restrict__ subs, const int *__restrict__ order,
    const T *__restrict__ Cs, const T *__restrict__ Rs,
    const double *__restrict__ b, double *__restrict__ x) {
  constexpr int NB = 64;
  constexpr int NW = NT / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  W *xs = reinterpret_cast<W *>(smem);
  const SubDesc s = subs[order[blockIdx.x]];
  const int n = s.n, np = s.np, kd = s.kd, ld = kd + 1;
  const T *C = Cs + s.fac_off;
  const T *R = Rs + s.fac_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nblk = np / NB;

  for (int i = tid; i < np; i += NT) xs[i] = i < n ? (W)b[s.dof_off + i] : (W)0;
  __syncthreads();

  // ---- forward: L y = b (column layout) ----
  for (int bk = 0; bk < nblk; ++bk) {
    const int j0 = bk * NB;
    if (wave == bk % NW) {
      // diagonal block: lane i keeps s[c] = L[j0+i, j0+c] for c < i and its
      // own reciprocal pivot dd; step c broadcasts y_c = x_c * d_c.  No
      // per-lane predicates live across the chain.
      const int i = lane;
      const T *rowp = C + (int64_t)j0 * ld + i;  // (j0+i, j0+c) at rowp + c*kd
      T sv[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) sv[c] = rowp[c * kd];
      __builtin_amdgcn_sched_barrier(0);
      W dd = 0;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        dd = (c == i) ? (W)sv[c] : dd;
        sv[c] = (c < i && i - c <= kd) ? sv[c] : (T)0;
      }
      W xi = xs[j0 + i];
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const W yc = lane_bcast(xi, c) * lane_bcast(dd, c);
        xi = fma(-(W)sv[c], yc, xi);
      }
      xs[j0 + i] = xi * dd;
    }
    __syncthreads();
    const int r0 = j0 + NB, r1 = min(np, j0 + NB + kd);
    // rows r0 <= i < r1 owned by this thread: i = tid (mod NT)
    for (int i = r0 + ((tid - r0) % NT + NT) % NT; i < r1; i += NT) {
      const T *rowp = C + (int64_t)j0 * ld + (i - j0);
      const int cmin = i - j0 - kd;  // first block column inside the band
      T v[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) v[c] = rowp[c * kd];
      __builtin_amdgcn_sched_barrier(0);
      W acc = 0;
      if (cmin <= 0) {
#pragma unroll
        for (int c = 0; c < NB; ++c) acc = fma((W)v[c], xs[j0 + c], acc);
      } else {
#pragma unroll
        for (int c = 0; c < NB; ++c) acc = fma(c >= cmin ? (W)v[c] : (W)0, xs[j0 + c], acc);
      }
      xs[i] -= acc;
    }
  }
  __syncthreads();

  // ---- backward: L^T x = y (row layout) ----
  for (int bk = nblk - 1; bk >= 0; --bk) {
    const int j0 = bk * NB;
    if (wave == bk % NW) {
      const int i = lane;
      // L[j0+c, j0+i] = R[(j0+c)*ld + (c-i)] at colp + c*(ld+1)
      const T *colp = R + (int64_t)j0 * ld - i;
      T sv[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) sv[c] = colp[c * (ld + 1)];
      __builtin_amdgcn_sched_barrier(0);
      W dd = 0;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        dd = (c == i) ? (W)sv[c] : dd;
        sv[c] = (c > i && c - i <= kd) ? sv[c] : (T)0;
      }
      W xi = xs[j0 + i];
#pragma unroll
      for (int c = NB - 1; c >= 0; --c) {
        const W yc = lane_bcast(xi, c) * lane_bcast(dd, c);
        xi = fma(-(W)sv[c], yc, xi);
      }
      xs[j0 + i] = xi * dd;
    }
    __syncthreads();
    const int r0 = max(0, j0 - kd), r1 = j0;
    for (int i = r0 + ((tid - r0) % NT + NT) % NT; i < r1; i += NT) {
      // L[j0+c, i] = R[(j0+c)*ld + (j0+c-i)] at rowp + c*(ld+1)
      const T *rowp = R + (int64_t)j0 * ld + (j0 - i);
      const int cmax = kd - (j0 - i);  // last block column inside the band
      T v[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) v[c] = rowp[c * (ld + 1)];
      __builtin_amdgcn_sched_barrier(0);
      W acc = 0;
      if (cmax >= NB - 1) {
#pragma unroll
        for (int c = 0; c < NB; ++c) acc = fma((W)v[c], xs[j0 + c], acc);
      } else {
#pragma unroll
        for (int c = 0; c < NB; ++c) acc = fma(c <= cmax ? (W)v[c] : (W)0, xs[j0 + c], acc);
      }
      xs[i] -= acc;
    }
  }
  __syncthreads();
  for (int i = tid; i < n; i += NT) x[s.dof_off + i] = (double)xs[i];
}

// ---------------------------------------------------------------------------
// Substitution for wide bands (kd <= kWideRows), 1024 threads per subdomain.
// Wavefront 0 works only on the diagonal blocks (the serial chain, as
// above).  Wavefronts 1..15 own one off-diagonal row each per 64-column
// block step: forward rows j0+64+t, backward rows j0-kd+t, t < kd.  Each
// thread issues the factor loads of its next block step as soon as its
// current step's arithmetic is done, before the barrier that waits for the
// chain, so the factor stream overlaps the chain instead of following it.
// Loads come in chunks of CW columns (register budget at 1024 threads); each
// column's address is wave-uniform plus a per-lane offset.
// ---------------------------------------------------------------------------
constexpr int kWideNT = 1024;
constexpr int kWideRows = kWideNT - 64;

// Factor loads go through a buffer resource whose base sits kWideFront
// entries before the subdomain's band, so that every offset is a
// non-negative 32-bit byte count: a per-lane offset shared by all columns
// plus a wave-uniform column offset (soffset).  Offsets stay inside the
// padded band storage by construction; the record count (the storage from
// the base to the end, capped at 4 GiB) makes any stray offset read zero.
constexpr int kWideFront = 64;

template <typename T>
__device__ inline T bload(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ inline double bload<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ inline float bload<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// buf[cc] = band entry at element offset e + (c0 + cc) * colstride from the
// subdomain base (e may be negative down to -kWideFront)
template <typename T, int CW>
__device__ inline void load_cols(T (&buf)[CW], __amdgpu_buffer_rsrc_t r, int64_t e,
                                 int colstride, int c0) {
  const int voff = (int)((e + kWideFront) * (int64_t)sizeof(T));
#pragma unroll
  for (int cc = 0; cc < CW; ++cc)
    buf[cc] = bload<T>(r, voff, (c0 + cc) * colstride * (int)sizeof(T));
}

template <typename T>
__device__ inline __amdgpu_buffer_rsrc_t band_rsrc(const T *base, int64_t entries_to_end) {
  const int64_t bytes = (entries_to_end + kWideFront) * (int64_t)sizeof(T);
  const int nrec = bytes > 0x7fffffffll ? 0x7fffffff : (int)bytes;
  return __builtin_amdgcn_make_buffer_rsrc((void *)(base - kWideFront), (short)0, nrec,
                                           0x00020000);
}

// phase 0: both sweeps; 1: forward sweep only (y = L^{-1} b written to x);
// 2: backward sweep only (x = L^{-T} b).  With DB the load chunks are
// double-buffered: chunk s+1 is requested before chunk s is consumed, so the
// round trips of one block step overlap (two buffers of CW columns).
template <typename T, typename W, int CW, bool DB>
__global__ __launch_bounds__(kWideNT) void k_band_solve_wide(
    const SubDesc *__restrict__ subs, const int *__restrict__ order,
    const T *__restrict__ Cs, const T *__restrict__ Rs, int64_t fac_len, int phase,
    const double *__restrict__ b, double *__restrict__ x) {
  constexpr int NB = 64, NCH = NB / CW, NBUF = DB ? 2 : 1;
  static_assert(NB % CW == 0, "chunks tile the block");
  extern __shared__ __align__(16) unsigned char smem[];
  W *xs = reinterpret_cast<W *>(smem);
  const SubDesc s = subs[order[blockIdx.x]];
  const int n = s.n, np = s.np, kd = s.kd, ld = kd + 1;
  const __amdgpu_buffer_rsrc_t Cr = band_rsrc(Cs + s.fac_off, fac_len - s.fac_off);
  const __amdgpu_buffer_rsrc_t Rr = band_rsrc(Rs + s.fac_off, fac_len - s.fac_off);
  const int tid = threadIdx.x, lane = tid & 63;
  const bool chainw = tid < 64;
  const int t = tid - 64;  // off-diagonal slot
  const int nblk = np / NB;

  for (int i = tid; i < np; i += kWideNT) xs[i] = i < n ? (W)b[s.dof_off + i] : (W)0;
  T buf[NBUF][CW];

  // ---- forward: L y = b, column layout: (i, j) at C[j*kd + i] ----
  // chain lane i reads (j0+i, j0+c) at j0*ld + c*kd + i; row i of the
  // off-diagonal block reads (i, j0+c) at j0*ld + c*kd + (i - j0).  Chunk
  // h of a step sits in buf[h % NBUF]; chunk 0 is requested during the
  // previous step.
  if (phase != 2) {
    if (chainw) {
      load_cols<T, CW>(buf[0], Cr, lane, kd, 0);
    } else if (t < kd && 64 + t < np) {
      load_cols<T, CW>(buf[0], Cr, 64 + t, kd, 0);
    }
    __syncthreads();
    for (int bk = 0; bk < nblk; ++bk) {
      const int j0 = bk * NB;
      const int64_t jb = (int64_t)j0 * ld;
      if (chainw) {
        W xi = xs[j0 + lane];
        W dd = 0;
#pragma unroll
        for (int h = 0; h < NCH; ++h) {
          T(&cur)[CW] = buf[h % NBUF];
          if (DB) {
            if (h + 1 < NCH) load_cols<T, CW>(buf[(h + 1) % NBUF], Cr, jb + lane, kd, (h + 1) * CW);
          } else if (h > 0) {
            load_cols<T, CW>(cur, Cr, jb + lane, kd, h * CW);
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int cc = 0; cc < CW; ++cc) {
            const int c = h * CW + cc;
            dd = (c == lane) ? (W)cur[cc] : dd;
            cur[cc] = (c < lane && lane - c <= kd) ? cur[cc] : (T)0;
          }
#pragma unroll
          for (int cc = 0; cc < CW; ++cc) {
            const int c = h * CW + cc;
            const W yc = lane_bcast(xi, c) * lane_bcast(dd, c);
            xi = fma(-(W)cur[cc], yc, xi);
          }
        }
        xs[j0 + lane] = xi * dd;
        if (bk + 1 < nblk) load_cols<T, CW>(buf[0], Cr, jb + (int64_t)NB * ld + lane, kd, 0);
      }
      __syncthreads();
      if (!chainw) {
        const int i = j0 + NB + t;
        if (t < kd && i < np) {
          const int cmin = i - j0 - kd;  // columns c < cmin lie outside the band
          W acc = 0;
#pragma unroll
          for (int h = 0; h < NCH; ++h) {
            T(&cur)[CW] = buf[h % NBUF];
            if (DB) {
              if (h + 1 < NCH)
                load_cols<T, CW>(buf[(h + 1) % NBUF], Cr, jb + (i - j0), kd, (h + 1) * CW);
            } else if (h > 0) {
              load_cols<T, CW>(cur, Cr, jb + (i - j0), kd, h * CW);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int cc = 0; cc < CW; ++cc) {
              const int c = h * CW + cc;
              acc = fma(c >= cmin ? (W)cur[cc] : (W)0, xs[j0 + c], acc);
            }
          }
          xs[i] -= acc;
        }
        if (bk + 1 < nblk && t < kd && i + NB < np)
          load_cols<T, CW>(buf[0], Cr, jb + (int64_t)NB * ld + (i - j0), kd, 0);
      }
      __syncthreads();
    }
  }
  if (phase == 1) {
    for (int i = tid; i < n; i += kWideNT) x[s.dof_off + i] = (double)xs[i];
    return;
  }

  // ---- backward: L^T x = y, row layout: (i, j) at R[i*ld + (i - j)] ----
  // chain lane i reads (j0+c, j0+i) at j0*ld + c*(ld+1) - i; row i < j0
  // reads (j0+c, i) at j0*ld + c*(ld+1) + (j0 - i).  Chunks are taken from
  // the last columns down (the order of the chain): step s of a block uses
  // chunk NCH-1-s in buf[s % NBUF].
  __syncthreads();
  {
    const int j0 = (nblk - 1) * NB;
    const int64_t jb = (int64_t)j0 * ld;
    if (chainw) {
      load_cols<T, CW>(buf[0], Rr, jb - lane, ld + 1, NB - CW);
    } else if (t < kd && j0 - kd + t >= 0) {
      load_cols<T, CW>(buf[0], Rr, jb + (kd - t), ld + 1, NB - CW);
    }
  }
  for (int bk = nblk - 1; bk >= 0; --bk) {
    const int j0 = bk * NB;
    const int64_t jb = (int64_t)j0 * ld;
    if (chainw) {
      W xi = xs[j0 + lane];
      W dd = 0;
#pragma unroll
      for (int st = 0; st < NCH; ++st) {
        const int h = NCH - 1 - st;
        T(&cur)[CW] = buf[st % NBUF];
        if (DB) {
          if (st + 1 < NCH) load_cols<T, CW>(buf[(st + 1) % NBUF], Rr, jb - lane, ld + 1, (h - 1) * CW);
        } else if (st > 0) {
          load_cols<T, CW>(cur, Rr, jb - lane, ld + 1, h * CW);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int cc = 0; cc < CW; ++cc) {
          const int c = h * CW + cc;
          dd = (c == lane) ? (W)cur[cc] : dd;
          cur[cc] = (c > lane && c - lane <= kd) ? cur[cc] : (T)0;
        }
#pragma unroll
        for (int cc = CW - 1; cc >= 0; --cc) {
          const int c = h * CW + cc;
          const W yc = lane_bcast(xi, c) * lane_bcast(dd, c);
          xi = fma(-(W)cur[cc], yc, xi);
        }
      }
      xs[j0 + lane] = xi * dd;
      if (bk > 0) load_cols<T, CW>(buf[0], Rr, jb - (int64_t)NB * ld - lane, ld + 1, NB - CW);
    }
    __syncthreads();
    if (!chainw) {
      const int i = j0 - kd + t;
      if (t < kd && i >= 0) {
        // (j0+c, i) lies in the band for c <= kd - (j0 - i) = t
        W acc = 0;
#pragma unroll
        for (int st = 0; st < NCH; ++st) {
          const int h = NCH - 1 - st;
          T(&cur)[CW] = buf[st % NBUF];
          if (DB) {
            if (st + 1 < NCH)
              load_cols<T, CW>(buf[(st + 1) % NBUF], Rr, jb + (kd - t), ld + 1, (h - 1) * CW);
          } else if (st > 0) {
            load_cols<T, CW>(cur, Rr, jb + (kd - t), ld + 1, h * CW);
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int cc = 0; cc < CW; ++cc) {
            const int c = h * CW + cc;
            acc = fma(c <= t ? (W)cur[cc] : (W)0, xs[j0 + c], acc);
          }
        }
        xs[i] -= acc;
      }
      if (bk > 0 && t < kd && i - NB >= 0)
        load_cols<T, CW>(buf[0], Rr, jb - (int64_t)NB * ld + (kd - t), ld + 1, NB - CW);
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += kWideNT) x[s.dof_off + i] = (double)xs[i];
}

template <typename T, typename W, int CW, bool DB>
void solve_wide_launch(edd_problem *p, const T *C, const T *R, const double *b, double *x,
                       const int *order, int count, int phase) {
  if (count <= 0) return;
  const size_t lds = ((sizeof(W) * p->max_np + 15) / 16) * 16;
  set_lds_limit_once((const void *)k_band_solve_wide<T, W, CW, DB>, p);
  k_band_solve_wide<T, W, CW, DB><<<count, kWideNT, lds, p->stream>>>(
      p->subs_d, order, C, R, p->fac_entries + band_pad_back(p->max_kd), phase, b, x);
}

// ---------------------------------------------------------------------------
// Dissected interiors.  With halves a, b and separator plane S the interior
// block is [A_a 0 B_a; 0 A_b B_b; B_a^T B_b^T C] and its Cholesky factor is
// [L_a 0 0; 0 L_b 0; W_a^T W_b^T L_S] with W_h = L_h^{-1} B_h and
// L_S L_S^T = C - W_a^T W_a - W_b^T W_b.  B_h is nonzero only in the last ns
// rows of half h (the plane next to S), and so is W_h.
// ---------------------------------------------------------------------------

// W_h = L_h,tail^{-1} B_h in place (B_h as assembled), from the true-diagonal
// factor (before the solve layouts are built).  A block owns 64 columns and
// walks the rows in 64-row blocks: the block's rows minus L(block, earlier)
// times the finished earlier rows (64x64 tiles through LDS), then a
// triangular solve with the diagonal tile, one thread per column.
__global__ __launch_bounds__(256) void k_sep_trsm(const SubDesc *__restrict__ subs,
                                                  const SepDesc *__restrict__ seps,
                                                  const double *__restrict__ fac,
                                                  double *__restrict__ W) {
  const SepDesc sd = seps[blockIdx.y >> 1];
  const int h = blockIdx.y & 1;
  const SubDesc leaf = subs[h ? sd.b : sd.a];
  const int ns = sd.ns, ld = leaf.kd + 1, t0 = leaf.n - ns;
  const double *L = fac + leaf.fac_off;
  double *Wh = W + sd.w_off + (int64_t)h * ns * ns;
  const int c0 = blockIdx.x * 64;
  if (c0 >= ns) return;
  __shared__ double Lt[64][65], Xt[64][65];
  const int tid = threadIdx.x, col = tid & 63, rg = tid >> 6;  // rows rg*16 .. +16
  // L(t0 + a, t0 + b) for a >= b, 0 otherwise
  auto Lat = [&](int a, int b) -> double {
    if (a < b || a >= ns || b >= ns) return 0.0;
    const int r = t0 + a, c = t0 + b;
    return L[(int64_t)c * ld + (r - c)];
  };
  const int nrb = (ns + 63) / 64;
  for (int qb = 0; qb < nrb; ++qb) {
    const int q0 = qb * 64;
    double acc[16];
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      const int q = q0 + rg * 16 + a, j = c0 + col;
      acc[a] = (q < ns && j < ns) ? Wh[(int64_t)q * ns + j] : 0.0;
    }
    for (int pb = 0; pb < qb; ++pb) {
      const int p0 = pb * 64;
      __syncthreads();
      for (int e2 = tid; e2 < 64 * 64; e2 += 256) {
        const int a = e2 >> 6, b = e2 & 63;
        Lt[a][b] = Lat(q0 + a, p0 + b);
        const int pr = p0 + a, j = c0 + b;
        Xt[a][b] = (pr < ns && j < ns) ? Wh[(int64_t)pr * ns + j] : 0.0;
      }
      __syncthreads();
      for (int b = 0; b < 64; ++b) {
        const double x = Xt[b][col];
#pragma unroll
        for (int a = 0; a < 16; ++a) acc[a] = fma(-Lt[rg * 16 + a][b], x, acc[a]);
      }
    }
    __syncthreads();
    for (int e2 = tid; e2 < 64 * 64; e2 += 256) {
      const int a = e2 >> 6, b = e2 & 63;
      Lt[a][b] = Lat(q0 + a, q0 + b);
    }
#pragma unroll
    for (int a = 0; a < 16; ++a) Xt[rg * 16 + a][col] = acc[a];
    __syncthreads();
    if (tid < 64) {
      const int j = c0 + tid;
      for (int a = 0; a < 64 && q0 + a < ns; ++a) {
        double v = Xt[a][tid];
        for (int b = 0; b < a; ++b) v = fma(-Lt[a][b], Xt[b][tid], v);
        v /= Lt[a][a];
        Xt[a][tid] = v;
        if (j < ns) Wh[(int64_t)(q0 + a) * ns + j] = v;
      }
    }
  }
}

// Separator block (band storage with kd = ns - 1, C as assembled) minus
// W_a^T W_a + W_b^T W_b, lower triangle; 32x32 output tiles.
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
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int h = 0; h < 2; ++h) {
    const double *Wh = W + sd.w_off + (int64_t)h * ns * ns;
    for (int k0 = 0; k0 < ns; k0 += 32) {
      __syncthreads();
      for (int e = threadIdx.x; e < 32 * 32; e += 256) {
        const int kk = e >> 5, c = e & 31, k = k0 + kk;
        const int q = tq * 32 + c, pcol = tp * 32 + c;
        Aq[kk][c] = (k < ns && q < ns) ? Wh[(int64_t)k * ns + q] : 0.0;
        Ap[kk][c] = (k < ns && pcol < ns) ? Wh[(int64_t)k * ns + pcol] : 0.0;
      }
      __syncthreads();
#pragma unroll 8
      for (int kk = 0; kk < 32; ++kk)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int c = 0; c < 2; ++c)
            acc[a][c] = fma(Aq[kk][ty * 2 + a], Ap[kk][tx * 2 + c], acc[a][c]);
    }
  }
  double *band = fac + S.fac_off;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int q = tq * 32 + ty * 2 + a, pcol = tp * 32 + tx * 2 + c;
      if (q < ns && pcol <= q) band[(int64_t)pcol * ld + (q - pcol)] -= acc[a][c];
    }
}

// x_S = b_S - W_a^T y_a,tail - W_b^T y_b,tail (y in x); 64 columns per block,
// rows split over the sixteen wavefronts, eight rows a batch per lane (eight
// loads in flight), and summed in a fixed order.
template <typename T>
__global__ __launch_bounds__(1024) void k_sep_rhs(const SubDesc *__restrict__ subs,
                                                  const SepDesc *__restrict__ seps,
                                                  const T *__restrict__ W,
                                                  const double *__restrict__ b,
                                                  double *__restrict__ x) {
  constexpr int NWV = 16, U = 8;
  const SepDesc sd = seps[blockIdx.y];
  const int ns = sd.ns;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  __shared__ double part[NWV][64];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (j < ns) {
    for (int h = 0; h < 2; ++h) {
      const SubDesc leaf = subs[h ? sd.b : sd.a];
      const double *y = x + leaf.dof_off + leaf.n - ns;
      const T *Wh = W + sd.w_off + (int64_t)h * ns * ns + j;
      int i = wv;
      for (; i + (U - 1) * NWV < ns; i += U * NWV) {
        double wv8[U];
#pragma unroll
        for (int u = 0; u < U; ++u) wv8[u] = (double)Wh[(int64_t)(i + u * NWV) * ns];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u & 3] = fma(wv8[u], y[i + u * NWV], acc[u & 3]);
      }
      for (; i < ns; i += NWV) acc[0] = fma((double)Wh[(int64_t)i * ns], y[i], acc[0]);
    }
  }
  part[wv][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (wv == 0 && j < ns) {
    const SubDesc S = subs[sd.s];
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < NWV; ++k) sum += part[k][lane];
    x[S.dof_off + j] = b[S.dof_off + j] - sum;
  }
}

// y_h,tail -= W_h x_S, one wavefront per two tail rows (four columns a
// batch per lane: eight loads in flight).
template <typename T>
__global__ __launch_bounds__(256) void k_sep_update(const SubDesc *__restrict__ subs,
                                                    const SepDesc *__restrict__ seps,
                                                    const T *__restrict__ W,
                                                    double *__restrict__ x) {
  const SepDesc sd = seps[blockIdx.y >> 1];
  const int h = blockIdx.y & 1;
  const int ns = sd.ns;
  const int i = 2 * (blockIdx.x * 4 + (threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  if (i >= ns) return;
  const bool two = i + 1 < ns;
  const SubDesc leaf = subs[h ? sd.b : sd.a];
  const SubDesc S = subs[sd.s];
  const T *r0 = W + sd.w_off + (int64_t)h * ns * ns + (int64_t)i * ns;
  const T *r1 = two ? r0 + ns : r0;
  const double *xs = x + S.dof_off;
  double a0 = 0.0, a1 = 0.0, c0 = 0.0, c1 = 0.0;
  int j = lane;
  for (; j + 192 < ns; j += 256) {
    double w0[4], w1[4], xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      w0[u] = (double)r0[j + 64 * u];
      w1[u] = (double)r1[j + 64 * u];
      xv[u] = xs[j + 64 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u & 1) {
        a1 = fma(w0[u], xv[u], a1);
        c1 = fma(w1[u], xv[u], c1);
      } else {
        a0 = fma(w0[u], xv[u], a0);
        c0 = fma(w1[u], xv[u], c0);
      }
    }
  }
  for (; j < ns; j += 64) {
    a0 = fma((double)r0[j], xs[j], a0);
    c0 = fma((double)r1[j], xs[j], c0);
  }
  double a = a0 + a1, c = c0 + c1;
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off);
    c += __shfl_down(c, off);
  }
  if (lane == 0) {
    x[leaf.dof_off + leaf.n - ns + i] -= a;
    if (two) x[leaf.dof_off + leaf.n - ns + i + 1] -= c;
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

template <typename T, typename W, int NT>
void solve_launch(edd_problem *p, const T *C, const T *R, const double *b, double *x) {
  const size_t lds = ((sizeof(W) * p->max_np + 15) / 16) * 16;
  set_lds_limit_once((const void *)k_band_solve<T, W, NT>, p);
  k_band_solve<T, W, NT><<<p->n_blk, NT, lds, p->stream>>>(p->subs_d, p->order_d,
                                                          C, R, b, x);
}

}  // namespace

int64_t band_pad_back(int max_kd) {
  // largest overrun of an unconditional load past the last column
  return (int64_t)(64 + 2) * (max_kd + 2) + 64 * 64 + 1024;
}

size_t band_solve_lds_bytes(const edd_problem *p, int precision) {
  (void)precision;  // both paths keep the right-hand side in FP64
  return ((8 * (size_t)p->max_np + 15) / 16) * 16;
}

static void cholesky_subset(edd_problem *p, const int *order, int count) {
  const int rows = 32 + p->max_kd;  // window rows
  if (rows <= 64) chol_launch<64, 1>(p, order, count);
  else if (rows <= 128) chol_launch<128, 1>(p, order, count);
  else if (rows <= 256) chol_launch<128, 2>(p, order, count);
  else if (rows <= 512) chol_launch<256, 2>(p, order, count);
  else if (chol_mfma_lds_bytes(1024) <= p->lds_limit)
    chol_launch_mfma<1024>(p, order, count);  // kd <= 992 (checked at setup)
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
    k_f64_to_f32<<<(unsigned)((p->w_entries + 255) / 256), 256, 0, p->stream>>>(
        p->w_entries, p->W64_d, p->W32_d);
  if (p->fac32_d)
    k_solve_layouts<float><<<grid, 256, 0, p->stream>>>(p->subs_d, p->fac64_d,
                                                        p->fac32_d, p->rac32_d);
  k_solve_layouts<double><<<grid, 256, 0, p->stream>>>(p->subs_d, p->fac64_d,
                                                       p->fac64_d, p->rac64_d);
}

// Substitution variants (the tile shapes the autotuner chooses between):
//   1, 2, 3  one row per thread, owner wavefront per diagonal block,
//            64 / 256 / 512 threads per subdomain
//   4, 5     wide bands (kd <= kWideRows): dedicated chain wavefront, 1024
//            threads, 16 / 32 (FP64) or 32 / 64 (FP32) columns per load chunk
//   6        as 4 with double-buffered load chunks
//   0        the default choice from the half bandwidth
bool band_solve_variant_ok(const edd_problem *p, int v) {
  if (v >= 1 && v <= 3) return p->n_sep == 0;  // no sweep phases
  if (v >= 4 && v <= 6) return p->max_kd <= kWideRows;
  return v == 0;
}

// Dissected interiors: forward sweeps of all halves and whole interiors,
// the separator right-hand sides, the separator solves, the tail updates,
// then the backward sweeps.
template <typename T, int CW, bool DB>
static void solve_dissected(edd_problem *p, const T *C, const T *R, const T *W,
                            const double *b, double *x) {
  const int nleaf = p->n_blk - p->n_sep;
  int maxns = 0;
  for (const SepDesc &sd : p->seps) maxns = std::max(maxns, sd.ns);
  solve_wide_launch<T, double, CW, DB>(p, C, R, b, x, p->order_leaf_d, nleaf, 1);
  k_sep_rhs<T><<<dim3((maxns + 63) / 64, p->n_sep), 1024, 0, p->stream>>>(p->subs_d, p->seps_d,
                                                                        W, b, x);
  solve_wide_launch<T, double, CW, DB>(p, C, R, x, x, p->order_sep_d, p->n_sep, 0);
  k_sep_update<T><<<dim3((maxns + 7) / 8, 2 * p->n_sep), 256, 0, p->stream>>>(
      p->subs_d, p->seps_d, W, x);
  solve_wide_launch<T, double, CW, DB>(p, C, R, x, x, p->order_leaf_d, nleaf, 2);
}

void launch_band_solve(edd_problem *p, int precision, const double *b,
                       double *x) {
  KTimer kt(p, precision == EDD_F32 ? EDD_KT_BAND_SOLVE32 : EDD_KT_BAND_SOLVE);
  const bool f32 = precision == EDD_F32;
  int v = p->solve_variant[f32 ? 1 : 0];
  if (v == 0) v = p->max_kd <= 64 && p->n_sep == 0 ? 1 : (p->max_kd <= kWideRows ? 5 : 3);
  if (p->n_sep > 0) {
    if (f32) {
      if (v == 4) solve_dissected<float, 32, false>(p, p->fac32_d, p->rac32_d, p->W32_d, b, x);
      else if (v == 6) solve_dissected<float, 32, true>(p, p->fac32_d, p->rac32_d, p->W32_d, b, x);
      else solve_dissected<float, 64, false>(p, p->fac32_d, p->rac32_d, p->W32_d, b, x);
    } else {
      if (v == 4) solve_dissected<double, 16, false>(p, p->fac64_d, p->rac64_d, p->W64_d, b, x);
      else if (v == 6) solve_dissected<double, 16, true>(p, p->fac64_d, p->rac64_d, p->W64_d, b, x);
      else solve_dissected<double, 32, false>(p, p->fac64_d, p->rac64_d, p->W64_d, b, x);
    }
    return;
  }
  // FP32 factor entries use FP64 right-hand sides and accumulation: the error
  // is then a fixed perturbation of K_II rather than arithmetic noise, which
  // the Schur complement of smooth interface vectors (a small difference of
  // large terms) would amplify
  if (f32) {
    const float *C = p->fac32_d, *R = p->rac32_d;
    switch (v) {
      case 1: solve_launch<float, double, 64>(p, C, R, b, x); break;
      case 2: solve_launch<float, double, 256>(p, C, R, b, x); break;
      case 3: solve_launch<float, double, 512>(p, C, R, b, x); break;
      case 4: solve_wide_launch<float, double, 32, false>(p, C, R, b, x, p->order_d, p->n_blk, 0); break;
      case 6: solve_wide_launch<float, double, 32, true>(p, C, R, b, x, p->order_d, p->n_blk, 0); break;
      default: solve_wide_launch<float, double, 64, false>(p, C, R, b, x, p->order_d, p->n_blk, 0); break;
    }
  } else {
    const double *C = p->fac64_d, *R = p->rac64_d;
    switch (v) {
      case 1: solve_launch<double, double, 64>(p, C, R, b, x); break;
      case 2: solve_launch<double, double, 256>(p, C, R, b, x); break;
      case 3: solve_launch<double, double, 512>(p, C, R, b, x); break;
      case 4: solve_wide_launch<double, double, 16, false>(p, C, R, b, x, p->order_d, p->n_blk, 0); break;
      case 6: solve_wide_launch<double, double, 16, true>(p, C, R, b, x, p->order_d, p->n_blk, 0); break;
      default: solve_wide_launch<double, double, 32, false>(p, C, R, b, x, p->order_d, p->n_blk, 0); break;
    }
  }
}

}  // namespace edd

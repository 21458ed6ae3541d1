// Batched interior solves: the forward/backward substitutions that apply
// K_II^{-1} (K_II is the direct sum of the subdomain blocks, eq.
// (NumberFive); all 2N+1 subproblems of eq. (3MatSplit2) use these solves)
// with the band factors built in kernels_factor.hip.
//
// One workgroup owns one subdomain.  Workgroups are launched largest first
// (the order array), so that round-robin dispatch over the XCDs spreads the
// large blocks evenly.
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

// Raise a kernel's dynamic LDS limit to what the device leaves beside the
// kernel's static LDS, once per (kernel, device); thread-safe.  A refused
// raise is not an error here (its error state is consumed): a launch that
// then asks for more than the default limit fails on its own.
void set_lds_limit_once(const void *kernel, const edd_problem *p) {
  static std::mutex mu;
  static std::vector<std::pair<const void *, int>> done;
  std::lock_guard<std::mutex> lk(mu);
  for (const auto &d : done)
    if (d.first == kernel && d.second == p->device) return;
  hipFuncAttributes fa{};
  size_t stat = 0;
  if (hipFuncGetAttributes(&fa, kernel) == hipSuccess) stat = fa.sharedSizeBytes;
  else (void)hipGetLastError();
  const int dyn = (int)(p->lds_limit > stat ? p->lds_limit - stat : 0);
  if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, dyn) != hipSuccess)
    (void)hipGetLastError();
  done.emplace_back(kernel, p->device);
}

namespace {

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

// ---------------------------------------------------------------------------
// Wide bands with lookahead.  As k_band_solve_wide, but the chain wavefront
// also applies the previous block to its own 64 rows (the 64 x 64 block
// below it, with the previous block's solution held in its registers), and
// the other wavefronts apply the previous block to the rows beyond.  Then a
// step has one barrier and the chain's triangular solve overlaps the
// off-diagonal stream instead of alternating with it.
//   forward, step bk (j0 = 64 bk, jp = j0 - 64): the chain applies columns
//     jp.. to rows j0..j0+63, then solves block bk; helper t' applies
//     columns jp.. to row jp + 128 + t' (t' < kd - 64);
//   backward, step bk (jn = j0 + 64): the chain applies rows jn.. of L (the
//     solution of block bk+1) to unknowns j0..j0+63, then solves block bk;
//     helper t applies them to unknown jn - kd + t (t < kd - 64).
// Every (row block, column block) pair is applied once: the adjacent pair
// by the chain, the rest by the helpers one step earlier, before the barrier
// that the chain's next read follows.
// ---------------------------------------------------------------------------
template <typename T, typename W, int CW>
__global__ __launch_bounds__(kWideNT) void k_band_solve_la(
    const SubDesc *__restrict__ subs, const int *__restrict__ order,
    const T *__restrict__ Cs, const T *__restrict__ Rs, int64_t fac_len, int phase,
    const double *__restrict__ b, double *__restrict__ x) {
  constexpr int NB = 64, NCH = NB / CW;
  static_assert(NB % CW == 0 && NCH % 2 == 0, "chunks tile the block, buffers alternate");
  extern __shared__ __align__(16) unsigned char smem[];
  W *xs = reinterpret_cast<W *>(smem);
  const SubDesc s = subs[order[blockIdx.x]];
  const int n = s.n, np = s.np, kd = s.kd, ld = kd + 1;
  const __amdgpu_buffer_rsrc_t Cr = band_rsrc(Cs + s.fac_off, fac_len - s.fac_off);
  const __amdgpu_buffer_rsrc_t Rr = band_rsrc(Rs + s.fac_off, fac_len - s.fac_off);
  const int tid = threadIdx.x, lane = tid & 63;
  const bool chainw = tid < 64;
  const int u = tid - 64;  // helper index
  const int nblk = np / NB;

  for (int i = tid; i < np; i += kWideNT) xs[i] = i < n ? (W)b[s.dof_off + i] : (W)0;
  T buf[2][CW];

  // ---- forward: L y = b, column layout (i, j) at C[j*kd + i] ----
  if (phase != 2) {
    W yprev = 0;
    if (chainw) load_cols<T, CW>(buf[0], Cr, lane, kd, 0);
    __syncthreads();
    for (int bk = 0; bk < nblk; ++bk) {
      const int j0 = bk * NB;
      const int64_t jb = (int64_t)j0 * ld, jpb = jb - (int64_t)NB * ld;
      if (chainw) {
        W xi = xs[j0 + lane];
        if (bk > 0) {
          // (j0+lane, jp+c) at jpb + c*kd + 64 + lane, in the band iff
          // 64 + lane - c <= kd; the last chunk's request is the diagonal
          // block's first
          const int cmin = NB + lane - kd;
          W a0 = 0, a1 = 0;
#pragma unroll
          for (int h = 0; h < NCH; ++h) {
            T(&cur)[CW] = buf[h & 1];
            if (h + 1 < NCH) load_cols<T, CW>(buf[(h + 1) & 1], Cr, jpb + NB + lane, kd, (h + 1) * CW);
            else load_cols<T, CW>(buf[(h + 1) & 1], Cr, jb + lane, kd, 0);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int cc = 0; cc < CW; cc += 2) {
              const int c = h * CW + cc;
              a0 = fma(c >= cmin ? (W)cur[cc] : (W)0, lane_bcast(yprev, c), a0);
              a1 = fma(c + 1 >= cmin ? (W)cur[cc + 1] : (W)0, lane_bcast(yprev, c + 1), a1);
            }
          }
          xi -= a0 + a1;
        }
        W dd = 0;
#pragma unroll
        for (int h = 0; h < NCH; ++h) {
          T(&cur)[CW] = buf[h & 1];
          if (h + 1 < NCH) load_cols<T, CW>(buf[(h + 1) & 1], Cr, jb + lane, kd, (h + 1) * CW);
          else if (bk + 1 < nblk) load_cols<T, CW>(buf[(h + 1) & 1], Cr, jb + NB + lane, kd, 0);
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
        yprev = xi * dd;
        xs[j0 + lane] = yprev;
      } else if (bk > 0) {
        // row jp + off, columns jp + c: (jp+c)*kd + jp + off, in the band
        // iff off - c <= kd
        const int jp = j0 - NB;
        const int off = 2 * NB + u;
        const int i = jp + off;
        if (off - (NB - 1) <= kd && i < np) {
          const int cmin = off - kd;
          W a0 = 0, a1 = 0;
#pragma unroll
          for (int h = 0; h < NCH; ++h) {
            T(&cur)[CW] = buf[h & 1];
            if (h + 1 < NCH) load_cols<T, CW>(buf[(h + 1) & 1], Cr, jpb + off, kd, (h + 1) * CW);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int cc = 0; cc < CW; cc += 2) {
              const int c = h * CW + cc;
              a0 = fma(c >= cmin ? (W)cur[cc] : (W)0, xs[jp + c], a0);
              a1 = fma(c + 1 >= cmin ? (W)cur[cc + 1] : (W)0, xs[jp + c + 1], a1);
            }
          }
          xs[i] -= a0 + a1;
        }
      }
      // the helpers' first chunk of step bk+1 (block bk's columns)
      if (!chainw && bk + 1 < nblk) {
        const int off = 2 * NB + u;
        if (off - (NB - 1) <= kd && j0 + off < np) load_cols<T, CW>(buf[0], Cr, jb + off, kd, 0);
      }
      __syncthreads();
    }
  }
  if (phase == 1) {
    for (int i = tid; i < n; i += kWideNT) x[s.dof_off + i] = (double)xs[i];
    return;
  }

  // ---- backward: L^T x = y, row layout (i, j) at R[i*ld + (i - j)] ----
  __syncthreads();
  {
    W xprev = 0;
    if (chainw) load_cols<T, CW>(buf[0], Rr, (int64_t)(nblk - 1) * NB * ld - lane, ld + 1, NB - CW);
    __syncthreads();
    for (int bk = nblk - 1; bk >= 0; --bk) {
      const int j0 = bk * NB;
      const int64_t jb = (int64_t)j0 * ld, jnb = jb + (int64_t)NB * ld;
      if (chainw) {
        W xi = xs[j0 + lane];
        if (bk + 1 < nblk) {
          // (jn+c, j0+lane) at jnb + c*(ld+1) + 64 - lane, in the band iff
          // 64 + c - lane <= kd; the last chunk's request is the diagonal
          // block's first (its last columns)
          const int cmax = kd - NB + lane;
          W a0 = 0, a1 = 0;
#pragma unroll
          for (int h = 0; h < NCH; ++h) {
            T(&cur)[CW] = buf[h & 1];
            if (h + 1 < NCH) load_cols<T, CW>(buf[(h + 1) & 1], Rr, jnb + NB - lane, ld + 1, (h + 1) * CW);
            else load_cols<T, CW>(buf[(h + 1) & 1], Rr, jb - lane, ld + 1, NB - CW);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int cc = 0; cc < CW; cc += 2) {
              const int c = h * CW + cc;
              a0 = fma(c <= cmax ? (W)cur[cc] : (W)0, lane_bcast(xprev, c), a0);
              a1 = fma(c + 1 <= cmax ? (W)cur[cc + 1] : (W)0, lane_bcast(xprev, c + 1), a1);
            }
          }
          xi -= a0 + a1;
        }
        // diagonal block, chunks from the last columns down (the order of
        // the triangular solve); chain lane i reads (j0+c, j0+i) at
        // jb + c*(ld+1) - i
        W dd = 0;
#pragma unroll
        for (int st = 0; st < NCH; ++st) {
          const int h = NCH - 1 - st;
          T(&cur)[CW] = buf[st & 1];
          if (st + 1 < NCH) load_cols<T, CW>(buf[(st + 1) & 1], Rr, jb - lane, ld + 1, (h - 1) * CW);
          else if (bk > 0) load_cols<T, CW>(buf[(st + 1) & 1], Rr, jb + NB - lane, ld + 1, 0);
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
        xprev = xi * dd;
        xs[j0 + lane] = xprev;
      } else if (bk + 1 < nblk) {
        // unknown i = jn - kd + t < j0, rows jn + c of L: (jn+c)*ld +
        // (jn + c - i) = jnb + c*(ld+1) + (kd - t), in the band iff c <= t
        const int jn = j0 + NB;
        const int t = u;
        const int i = jn - kd + t;
        if (t < kd - NB && i >= 0) {
          W a0 = 0, a1 = 0;
#pragma unroll
          for (int h = 0; h < NCH; ++h) {
            T(&cur)[CW] = buf[h & 1];
            if (h + 1 < NCH) load_cols<T, CW>(buf[(h + 1) & 1], Rr, jnb + (kd - t), ld + 1, (h + 1) * CW);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int cc = 0; cc < CW; cc += 2) {
              const int c = h * CW + cc;
              a0 = fma(c <= t ? (W)cur[cc] : (W)0, xs[jn + c], a0);
              a1 = fma(c + 1 <= t ? (W)cur[cc + 1] : (W)0, xs[jn + c + 1], a1);
            }
          }
          xs[i] -= a0 + a1;
        }
      }
      // the helpers' first chunk of step bk-1 (block bk's rows of L)
      if (!chainw && bk > 0) {
        const int t = u;
        if (t < kd - NB && j0 - kd + t >= 0) load_cols<T, CW>(buf[0], Rr, jb + (kd - t), ld + 1, 0);
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < n; i += kWideNT) x[s.dof_off + i] = (double)xs[i];
}

template <typename T, typename W, int CW>
void solve_la_launch(edd_problem *p, const T *C, const T *R, const double *b, double *x,
                     const int *order, int count, int phase) {
  if (count <= 0) return;
  const size_t lds = ((sizeof(W) * p->max_np + 15) / 16) * 16;
  set_lds_limit_once((const void *)k_band_solve_la<T, W, CW>, p);
  k_band_solve_la<T, W, CW><<<count, kWideNT, lds, p->stream>>>(
      p->subs_d, order, C, R, p->fac_entries + band_pad_back(p->max_kd), phase, b, x);
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
  const int ns = sd.ns, ldw = sd.ldw;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  __shared__ double part[NWV][64];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (j < ns) {
    for (int h = 0; h < 2; ++h) {
      const SubDesc leaf = subs[h ? sd.b : sd.a];
      const double *y = x + leaf.dof_off + leaf.n - ns;
      const T *Wh = W + sd.w_off + (int64_t)h * ns * ldw + j;
      int i = wv;
      for (; i + (U - 1) * NWV < ns; i += U * NWV) {
        double wv8[U];
#pragma unroll
        for (int u = 0; u < U; ++u) wv8[u] = (double)Wh[(int64_t)(i + u * NWV) * ldw];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u & 3] = fma(wv8[u], y[i + u * NWV], acc[u & 3]);
      }
      for (; i < ns; i += NWV) acc[0] = fma((double)Wh[(int64_t)i * ldw], y[i], acc[0]);
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
  const T *r0 = W + sd.w_off + (int64_t)h * ns * sd.ldw + (int64_t)i * sd.ldw;
  const T *r1 = two ? r0 + sd.ldw : r0;
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

// Substitution variants (the tile shapes the autotuner chooses between):
//   1, 2, 3  one row per thread, owner wavefront per diagonal block,
//            64 / 256 / 512 threads per subdomain
//   4, 5     wide bands (kd <= kWideRows): dedicated chain wavefront, 1024
//            threads, 16 / 32 (FP64) or 32 / 64 (FP32) columns per load chunk
//   6        as 4 with double-buffered load chunks
//   7        as 6 with lookahead (k_band_solve_la)
//   0        the default choice from the half bandwidth
bool band_solve_variant_ok(const edd_problem *p, int v) {
  if (v >= 1 && v <= 3) return p->n_sep == 0;  // no sweep phases
  if (v >= 4 && v <= 7) return p->max_kd <= kWideRows;
  return v == 0;
}

// Dissected interiors: forward sweeps of all halves and whole interiors,
// the separator right-hand sides, the separator solves, the tail updates,
// then the backward sweeps.
template <typename T, int CW, bool DB, bool LA>
static void solve_dissected(edd_problem *p, const T *C, const T *R, const T *W,
                            const double *b, double *x) {
  const int nleaf = p->n_blk - p->n_sep;
  int maxns = 0;
  for (const SepDesc &sd : p->seps) maxns = std::max(maxns, sd.ns);
  auto sweep = [&](const double *bb, const int *order, int count, int phase) {
    if constexpr (LA) solve_la_launch<T, double, CW>(p, C, R, bb, x, order, count, phase);
    else solve_wide_launch<T, double, CW, DB>(p, C, R, bb, x, order, count, phase);
  };
  sweep(b, p->order_leaf_d, nleaf, 1);
  k_sep_rhs<T><<<dim3((maxns + 63) / 64, p->n_sep), 1024, 0, p->stream>>>(p->subs_d, p->seps_d,
                                                                        W, b, x);
  sweep(x, p->order_sep_d, p->n_sep, 0);
  k_sep_update<T><<<dim3((maxns + 7) / 8, 2 * p->n_sep), 256, 0, p->stream>>>(
      p->subs_d, p->seps_d, W, x);
  sweep(x, p->order_leaf_d, nleaf, 2);
}

void launch_band_solve(edd_problem *p, int precision, const double *b,
                       double *x) {
  KTimer kt(p, precision == EDD_F32 ? EDD_KT_BAND_SOLVE32 : EDD_KT_BAND_SOLVE);
  const bool f32 = precision == EDD_F32;
  int v = p->solve_variant[f32 ? 1 : 0];
  if (v == 0) v = p->max_kd <= 64 && p->n_sep == 0 ? 1 : (p->max_kd <= kWideRows ? 5 : 3);
  if (p->n_sep > 0) {
    if (f32) {
      if (v == 4) solve_dissected<float, 32, false, false>(p, p->fac32_d, p->rac32_d, p->W32_d, b, x);
      else if (v == 6) solve_dissected<float, 32, true, false>(p, p->fac32_d, p->rac32_d, p->W32_d, b, x);
      else if (v == 7) solve_dissected<float, 32, true, true>(p, p->fac32_d, p->rac32_d, p->W32_d, b, x);
      else solve_dissected<float, 64, false, false>(p, p->fac32_d, p->rac32_d, p->W32_d, b, x);
    } else {
      if (v == 4) solve_dissected<double, 16, false, false>(p, p->fac64_d, p->rac64_d, p->W64_d, b, x);
      else if (v == 6) solve_dissected<double, 16, true, false>(p, p->fac64_d, p->rac64_d, p->W64_d, b, x);
      else if (v == 7) solve_dissected<double, 16, true, true>(p, p->fac64_d, p->rac64_d, p->W64_d, b, x);
      else solve_dissected<double, 32, false, false>(p, p->fac64_d, p->rac64_d, p->W64_d, b, x);
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
      case 7: solve_la_launch<float, double, 32>(p, C, R, b, x, p->order_d, p->n_blk, 0); break;
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
      case 7: solve_la_launch<double, double, 16>(p, C, R, b, x, p->order_d, p->n_blk, 0); break;
      default: solve_wide_launch<double, double, 32, false>(p, C, R, b, x, p->order_d, p->n_blk, 0); break;
    }
  }
}

}  // namespace edd

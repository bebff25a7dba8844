// FETI-DP solve of Z x = f on one GPU (Sec. 5), subdomains as a batch.
//
//   d     = sum_s B_r Z_rr^-1 f_r - F_rc K_cc*^-1 f_c*,  f_c* = f_c - sum_s B_c^T Z_cr Z_rr^-1 f_r
//   F_DP  = sum_s B_r Z_rr^-1 B_r^T + F_rc K_cc*^-1 F_rc^T
//   P^-1  = W sum_s B_r S_bb B_r^T W   (Dirichlet preconditioner, W = 1/2 in 2D)
//   GMRES on F_DP P^-1 t = d (right preconditioning, so its residual is the
//   true interface residual), mu = P^-1 t; recovery
//   u_c = K_cc*^-1 (f_c* + F_rc^T mu),  u_r = Z_rr^-1 (f_r - Z_rc B_c u_c - B_r^T mu).
//
// Kernels:
//   k_local_solve   one workgroup per subdomain: full solve with E^s by the
//                   line block-tridiagonal recursion (forward and backward
//                   sweeps, one dense ml x ml product per line and sweep).
//   k_gmres         one persistent cooperative launch for the whole Krylov
//                   solve; phases separated by a grid barrier.  Multiplier
//                   vectors, orthogonalisation (classical Gram-Schmidt, twice),
//                   norms and the coarse solve are FP64; the interface
//                   Schur complements are streamed in the storage precision.
//
// Arithmetic is FP64 for both storage precisions: complex64 factors and
// operators are widened as they are loaded, and every vector and accumulator
// (line sweeps, Schur-complement products) is FP64.  The kernels are bound by
// latency, so this costs little, and it makes the complex64 path's solves
// accurate to the rounding of the stored factors alone; with FP32 vectors the
// outer refinement needs one step more.
#include "common.h"

#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

namespace sfdp {

constexpr int ML = 33;

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations
// (lgkmcnt = 0) but not for outstanding global loads, so prefetches stay in
// flight across it (a full __syncthreads waits for every global load too).
__device__ inline void lds_sync() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // vmcnt = max, expcnt = max, lgkmcnt = 0
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// ------------------------------------------------------------------------------------------
// Grid barrier for a cooperative launch (all blocks co-resident), two levels to
// spread the atomics: blocks arrive on one of G group counters (separate
// 128-byte lines), the last arrival of each group arrives on the top counter,
// and the last group publishes the epoch in a generation word that every block
// polls.  Counters only grow (barrier e completes at e * size), so nothing is
// reset inside a launch.  A spin limit turns a broken barrier into an error
// flag instead of a hang.  bar holds BAR_WORDS words.  nblocks and blk are the
// block count and block index of the group that synchronises (one instance's
// share of the grid).
constexpr int BAR_GROUPS = 16, BAR_STRIDE = 32, BAR_TOP = BAR_GROUPS * BAR_STRIDE,
              BAR_GEN = BAR_TOP + BAR_STRIDE, BAR_ARRIVE = BAR_GEN + BAR_STRIDE,
              BAR_WORDS = BAR_ARRIVE + BAR_STRIDE;
__device__ inline void grid_barrier(unsigned* bar, unsigned nblocks, unsigned blk, unsigned& epoch,
                                    int* err) {
  // Data exchanged between blocks uses agent-scope atomic loads and stores
  // (ld_coh / st_coh below), which are coherent across the XCDs' L2 caches
  // without whole-cache write-back or invalidation.  The barrier only has to
  // order them: every wave waits for its own memory operations to complete,
  // then one thread arrives and polls.
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  epoch += 1;
  if (threadIdx.x == 0) {
    const unsigned G = nblocks >= 8 * BAR_GROUPS ? BAR_GROUPS : (nblocks + 7) / 8;
    const unsigned grp = blk % G;
    const unsigned gsize = nblocks / G + (grp < nblocks % G ? 1u : 0u);
    unsigned old = __hip_atomic_fetch_add(bar + grp * BAR_STRIDE, 1u, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1 == epoch * gsize) {
      unsigned o2 = __hip_atomic_fetch_add(bar + BAR_TOP, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (o2 + 1 == epoch * G)
        __hip_atomic_store(bar + BAR_GEN, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    unsigned spins = 0;
    while (__hip_atomic_load(bar + BAR_GEN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1u << 26)) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __syncthreads();
}

// Start of a plain (not cooperative) launch of a kernel that uses grid_barrier:
// whether the grid is co-resident.  Every block arrives on one counter and
// waits, for at most `spins` polls, until all `total` have.  The count and an
// abort bit share the word, so the blocks agree: a block whose wait ran out sets
// the bit only by a compare-and-swap from a short count, and once the count is
// complete it can no longer be set.  On abort every block must return before any
// work (a late block sees the bit in its own arrival), and *notres is set.  A
// cooperative launch saves this check but costs ~11 us of idle device on each
// side of the kernel (measured on MI355X), a plain one does not.  `go` is an LDS
// word that carries thread 0's answer to the block (the caller's dynamic LDS, free
// at that point: a static LDS word would grow the kernel's LDS allocation by one
// granule and cost co-resident blocks where the dynamic layout fills the CU).
constexpr unsigned ARRIVE_ABORT = 1u << 31;
constexpr int CORESIDENT_SPINS = 1 << 12;
__device__ inline bool grid_coresident(unsigned* word, unsigned total, int spins, int* notres, int& go) {
  if (threadIdx.x == 0) {
    unsigned v = __hip_atomic_fetch_add(word, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    int n = 0, r = 1;
    for (;;) {
      if (v & ARRIVE_ABORT) { r = 0; break; }
      if (v >= total) break;
      if (n >= spins) {
        unsigned expect = v;
        if (__hip_atomic_compare_exchange_strong(word, &expect, v | ARRIVE_ABORT, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          __hip_atomic_store(notres, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          r = 0;
          break;
        }
        v = expect;  // the word moved on: test the new value
        continue;
      }
      ++n;
      __builtin_amdgcn_s_sleep(1);
      v = __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    go = r;
  }
  __syncthreads();
  const bool ok = go != 0;
  __syncthreads();  // every thread has read go before the caller reuses the word
  return ok;
}

// Coherent (agent-scope) access to data written by one block and read by
// another inside a persistent launch.
__device__ inline cd ld_coh(const cd* p) {
  double x = __hip_atomic_load((const double*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  double y = __hip_atomic_load((const double*)p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return cd{x, y};
}
__device__ inline void st_coh(cd* p, cd v) {
  __hip_atomic_store((double*)p, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store((double*)p + 1, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sums of per-block partial values for several right-hand sides at once.  The
// rows are the pairs (a, i), a < na, i < n, of the na right-hand sides
// r = ract[a]; row (a, i) reads part[r * pstride + i * nb + q], q < nb, and
// writes out[r * ostride + i].  Every value is summed in the same fixed order
// in every block.  Wave w takes rows w * 4 .. w * 4 + 3, then 16 further; four
// rows per batch keep 16 loads in flight per lane.  nb <= 256.
__device__ inline void reduce_partials(const cd* __restrict__ part, int64_t pstride, int nb, int n,
                                       int na, const int* ract, cd* out, int ostride) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int rows = na * n;
  for (int p0 = wv * 4; p0 < rows; p0 += 16) {
    const cd* src[4];
    int dst[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int p = min(p0 + u, rows - 1);
      const int a = p / n, i = p - a * n, r = ract[a];
      src[u] = part + r * pstride + (int64_t)i * nb;
      dst[u] = r * ostride + i;
    }
    cd v[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) {
        // load from a clamped, always valid address, then select: keeps v in
        // registers and all sixteen loads in flight
        const int q = lane + 64 * q4;
        cd t = ld_coh(src[u] + min(q, nb - 1));
        v[u][q4] = q < nb ? t : cd{0.0, 0.0};
      }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      cd a = (v[u][0] + v[u][1]) + (v[u][2] + v[u][3]);
      for (int off = 32; off > 0; off >>= 1) {
        a.x += __shfl_xor(a.x, off, 64);
        a.y += __shfl_xor(a.y, off, 64);
      }
      if (lane == 0 && p0 + u < rows) out[dst[u]] = a;
    }
  }
  __syncthreads();
}

// part[r * pstride + i * nb + b] = sum_{k < kn} conj(Q_r[i][k0 + k]) w_r[k] for the
// pairs (r = ract[a], i < nvec); Q_r = Q + r * qs, w_r = wch + r * wstride.
// Eight lanes per pair (32 pairs per pass), partial sums combined by shuffles.
__device__ inline void block_dots(const cd* __restrict__ Q, int64_t qs, int nmu, int k0, int kn,
                                  int nvec, int na, const int* ract, const cd* wch, int wstride,
                                  cd* part, int64_t pstride, int nb, int b) {
  const int t = threadIdx.x, g = t & 7;
  const int pairs = na * nvec;
  for (int p0 = 0; p0 < pairs; p0 += 32) {
    const int p = p0 + (t >> 3);
    cd acc{0.0, 0.0};
    int r = 0, i = 0;
    if (p < pairs) {
      const int a = p / nvec;
      i = p - a * nvec;
      r = ract[a];
      const cd* q = Q + r * qs + (size_t)i * nmu + k0;
      const cd* w = wch + r * wstride;
#pragma unroll 4
      for (int k = g; k < kn; k += 8) fma_conj_acc(acc, q[k], w[k]);
    }
    for (int off = 4; off > 0; off >>= 1) {
      acc.x += __shfl_xor(acc.x, off, 64);
      acc.y += __shfl_xor(acc.y, off, 64);
    }
    if (g == 0 && p < pairs) st_coh(part + r * pstride + (size_t)i * nb + b, acc);
  }
}

// Per right-hand-side block sums: thread t holds a partial value of RHS
// t / (256 / NRT) (256 threads); out[r] = sum over that RHS's threads, in a
// fixed order.  wsum holds 4 doubles.
template <int NRT>
__device__ inline void rhs_block_sums(double v, double* wsum, double* out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if (lane == 0) wsum[wv] = v;
  __syncthreads();
  if (threadIdx.x < NRT) {
    constexpr int WPR = 4 / NRT;
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < WPR; ++w) t += wsum[threadIdx.x * WPR + w];
    out[threadIdx.x] = t;
  }
  __syncthreads();
}

// ------------------------------------------------------------------------------------------
// Dense products on LDS vectors.

// Packed symmetric storage: the lower triangle of an n_d x n_d symmetric matrix,
// row-major, entry (i, k), k <= i, at i (i + 1) / 2 + k.  Per subdomain the
// blocks are PK = ND (ND + 1) / 2 entries apart.
__host__ __device__ inline int packed_len(int n) { return n * (n + 1) / 2; }

// y[i] = sum_k S(i, k) x[k] for i < nd <= 128 with S packed in LDS.  Thread
// (i, half) sums half of the k range (row part k <= i read along the row,
// column part k > i read down the column), partial sums combined through red.
template <class TM, class R>
__device__ inline void symv_packed(const TM* A, int nd, const C<R>* xs, cd* red, cd* y) {
  const int i = threadIdx.x & 127, half = threadIdx.x >> 7;
  const int h = (nd + 1) / 2;
  const int k0 = half ? h : 0, k1 = half ? nd : h;
  C<R> acc{0, 0};
  if (i < nd) {
    const int rb = i * (i + 1) / 2;
    const int kr = min(k1, i + 1);
    for (int k = k0; k < kr; ++k) fma_acc(acc, cvt<R>(A[rb + k]), xs[k]);
    int k = max(k0, i + 1);
    int cb = k * (k + 1) / 2;
    for (; k < k1; ++k) {
      fma_acc(acc, cvt<R>(A[cb + i]), xs[k]);
      cb += k + 1;
    }
  }
  red[threadIdx.x] = cd{(double)acc.x, (double)acc.y};
  __syncthreads();
  if (threadIdx.x < nd) y[threadIdx.x] = red[threadIdx.x] + red[128 + threadIdx.x];
  __syncthreads();
}

// Coalesced bulk copy global -> LDS in 16-byte words, eight loads in flight per
// thread.  `bytes` is rounded up to 16 (the global blocks are padded).
__device__ inline void stage_lds(void* dst, const void* __restrict__ src, int bytes) {
  const uint4* s4 = (const uint4*)src;
  uint4* d4 = (uint4*)dst;
  const int n16 = (bytes + 15) / 16;
  for (int i0 = threadIdx.x; i0 < n16; i0 += 256 * 8) {
    uint4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = s4[min(i0 + u * 256, n16 - 1)];  // clamped: no branches
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int i = i0 + u * 256;
      if (i < n16) d4[i] = v[u];
    }
  }
  __syncthreads();
}

// Column a of subdomain s's local grid as a bit mask over the lines b = 0..m:
// bit b set when node (a, b) is in the r set (neither on the Dirichlet boundary
// nor a subdomain vertex); 0 when a is outside 0..m or on the Dirichlet boundary.
__device__ inline uint64_t rnode_column(const Geo2& g, int s, int a) {
  if (a < 0 || a > g.m) return 0;
  const int gi = g.sx(s) * g.m + a, j0 = g.sy(s) * g.m;
  if (gi == 0 || gi == g.N) return 0;
  uint64_t msk = (1ull << (g.m + 1)) - 1;
  if (j0 == 0) msk &= ~1ull;
  if (j0 + g.m == g.N) msk &= ~(1ull << g.m);
  if (a == 0 || a == g.m) msk &= ~(1ull | (1ull << g.m));
  return msk;
}

// Bulk copy of one line factor (ml * ml entries, <= 33 * 33) global -> registers:
// every thread issues its (at most 5) loads back to back.
constexpr int GPT = (ML * ML + 255) / 256;
template <class TS>
__device__ inline void line_load(const TS* __restrict__ src, int n2, TS (&reg)[GPT]) {
#pragma unroll
  for (int r = 0; r < GPT; ++r) reg[r] = src[min((int)threadIdx.x + 256 * r, n2 - 1)];  // clamped
}
template <class TS>
__device__ inline void line_store(TS* dst, int n2, const TS (&reg)[GPT]) {
#pragma unroll
  for (int r = 0; r < GPT; ++r) {
    int idx = threadIdx.x + 256 * r;
    if (idx < n2) dst[idx] = reg[r];
  }
}

// t_r[p] = sum_k G(p,k) z_r[k] for one line and nr <= NRT right-hand sides; G in
// LDS stored transposed (G(p,k) at Gl[k*ml + p]); four wave groups split k,
// partial sums reduced through LDS (red: [NRT][4][ML]).  z_r = z + r * ML,
// out_r = out + r * xstride.  Gl and z are no longer read when it returns; out
// and red are, until the caller's next barrier.
template <class TS, class T, int NRT>
__device__ inline void line_mv(const TS* Gl, int ml, const T* z, T* red, T* out, int xstride,
                               bool subtract, int nr) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int kq = (ml + 3) / 4;
  T acc[NRT];
#pragma unroll
  for (int r = 0; r < NRT; ++r) acc[r] = T{0, 0};
  if (lane < ml) {
    // fixed trip count (kq <= KQ), clamped indices and out-of-range terms
    // selected to zero (k0, k1 are wave-uniform)
    constexpr int KQ = (ML + 3) / 4;
    const int k0 = wv * kq, k1 = min(ml, k0 + kq);
    if constexpr (NRT == 1) {
      // one right-hand side: the compiler's own order, which keeps the register
      // count low enough for four workgroups per CU
#pragma unroll
      for (int u = 0; u < KQ; ++u) {
        const int k = min(k0 + u, ml - 1);
        auto gk = cvt<typename real_of<T>::type>(Gl[k * ml + lane]);
        if (k0 + u >= k1) gk = decltype(gk){0, 0};
        fma_acc(acc[0], gk, z[k]);
      }
    } else {
      // several right-hand sides: the operands go to registers in chunks of CH
      // terms, the next chunk's LDS reads issued before the current chunk's
      // multiply-adds; the scheduling barriers keep the compiler from sinking
      // each read to its use, which costs one LDS round trip per term
      constexpr int CH = 3;
      static_assert(KQ % CH == 0, "whole chunks");
      TS gv[2][CH];
      T zv[2][CH][NRT];
      auto fetch = [&](int c, int b) {
#pragma unroll
        for (int i = 0; i < CH; ++i) {
          const int k = min(k0 + c * CH + i, ml - 1);
          gv[b][i] = Gl[k * ml + lane];
#pragma unroll
          for (int r = 0; r < NRT; ++r) zv[b][i][r] = z[r * ML + k];
        }
      };
      fetch(0, 0);
#pragma unroll
      for (int c = 0; c < KQ / CH; ++c) {
        if (c + 1 < KQ / CH) fetch(c + 1, (c + 1) & 1);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < CH; ++i) {
          auto gk = cvt<typename real_of<T>::type>(gv[c & 1][i]);
          if (k0 + c * CH + i >= k1) gk = decltype(gk){0, 0};
#pragma unroll
          for (int r = 0; r < NRT; ++r) fma_acc(acc[r], gk, zv[c & 1][i][r]);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int r = 0; r < NRT; ++r) red[(r * 4 + wv) * ML + lane] = acc[r];
  }
  lds_sync();
  if (threadIdx.x < ml * nr) {
    const int r = threadIdx.x / ml, p = threadIdx.x - r * ml;
    const T* rr = red + r * 4 * ML;
    T s = rr[p] + rr[ML + p];
    s = s + rr[2 * ML + p];
    s = s + rr[3 * ML + p];
    T* o = out + r * xstride + p;
    *o = subtract ? *o - s : s;
  }
  // no closing barrier: the caller's next barrier orders these writes (and the
  // reads of red) before anything reads out or writes red again
}

// ------------------------------------------------------------------------------------------
// Full local solve with E^s (extended Z_rr^s) for nr <= NRT right-hand sides; one
// workgroup per subdomain streams the line factors once for all of them.
//   mode 0: load f_r = f / multiplicity; output x on Delta (Xd) and Z_cr x (Qc).
//   mode 1: load f_r - Z_rc B_c uc - B_r^T mu; output Delta values (Ubuf) and
//           interior values straight into xout (conjugated if conj_out).
template <class TS, int NRT>
__device__ inline void local_solve_body(const Geo2& g, const Maps2& mp, const RhsStride& rs, int nr,
                                        const TS* __restrict__ G, int mode, const cd* __restrict__ f,
                                        int conj_in, const cd* __restrict__ uc,
                                        const cd* __restrict__ mu, cd* Xd, cd* Qc, cd* Ubuf,
                                        cd* xout, int conj_out, int s) {
  using R = double;  // FP64 arithmetic for both storage precisions
  using T = cd;
  constexpr int XS = ML * ML;
  __shared__ T xall[NRT * XS];
  __shared__ T zl[NRT * ML];
  __shared__ T red[NRT * 4 * ML];
  __shared__ TS gbuf[ML * ML];
  __shared__ T cpl[ML][3];   // coupling of node p of a line to node p + d - 1 of the next line
  const int ml = g.ml, n2 = ml * ml, ND = g.ND;
  const TS* Gs = G + (size_t)s * ml * n2;
  // The forward sweep visits lines 0..ml-1, the backward sweep ml-2..0: step t
  // uses line (t < ml ? t : 2 ml - 2 - t).  Line factors stream through a ring
  // of LRING register sets, LRING steps ahead of the step being computed
  // (two sets of complex128, whose ring would not stay in registers).
  constexpr int LRING = sizeof(TS) == sizeof(cf) ? 4 : 2;
  const int nsteps = 2 * ml - 1;
  auto line_of = [&](int t) { return t < ml ? t : 2 * ml - 2 - t; };
  TS greg[LRING][GPT];
#pragma unroll
  for (int u = 0; u < LRING; ++u)
    if (u < nsteps) line_load<TS>(Gs + (size_t)line_of(u) * n2, n2, greg[u]);
  // load right-hand sides (loads from a clamped RHS index, results selected)
  for (int l = threadIdx.x; l < n2; l += blockDim.x) {
    const int a = l % ml, b = l / ml;
    const bool rn = g.rnode(s, a, b);
    const int64_t fi = rn ? g.freeidx(s, a, b) : 0;
    cd fv[NRT];
#pragma unroll
    for (int r = 0; r < NRT; ++r) fv[r] = f[min(r, nr - 1) * rs.nf + fi];
#pragma unroll
    for (int r = 0; r < NRT; ++r) {
      cd v{0.0, 0.0};
      if (rn) {
        cd x = conj_in ? conj(fv[r]) : fv[r];
        v = (1.0 / g.mult(a, b)) * x;
        if (mode == 1) {
          for (int q = 0; q < 4; ++q) {
            int cl = mp.cloc[s * 4 + q];
            if (cl < 0) continue;
            int ca = cl % ml, cb = cl / ml;
            if (abs(ca - a) > 1 || abs(cb - b) > 1) continue;
            v = v - g.zloc(a, b, ca, cb) * uc[min(r, nr - 1) * rs.nc + mp.cgid[s * NQ + q]];
          }
        }
      }
      xall[r * XS + l] = T{(R)v.x, (R)v.y};
    }
  }
  __syncthreads();
  if (mode == 1) {
    int nd = mp.nd[s];
    for (int i = threadIdx.x; i < nd; i += blockDim.x) {
      const int l = mp.dloc[s * ND + i], mid = mp.dmid[s * ND + i];
      const double sg = (double)mp.dsgn[s * ND + i];
      cd mv[NRT];
#pragma unroll
      for (int r = 0; r < NRT; ++r) mv[r] = mu[min(r, nr - 1) * rs.nmu + mid];
#pragma unroll
      for (int r = 0; r < NRT; ++r) {
        cd m = sg * mv[r];
        xall[r * XS + l] = xall[r * XS + l] - T{(R)m.x, (R)m.y};
      }
    }
    __syncthreads();
  }
  // coupling coefficients between consecutive lines (interior rows of the 1D
  // matrices in the line direction: k = -1/h, m = h/6), masked per use below
  if (threadIdx.x < ml * 3) {
    int p = threadIdx.x / 3, d = threadIdx.x % 3, a = p + d - 1;
    cd e{0.0, 0.0};
    if (a >= 0 && a < ml) e = g.zloc(p, 1, a, 2);
    cpl[p][d] = T{(R)e.x, (R)e.y};
  }
  line_store<TS>(gbuf, n2, greg[0]);
  if (LRING < nsteps) line_load<TS>(Gs + (size_t)line_of(LRING) * n2, n2, greg[0]);
  // thread (zr, zp) forms z for right-hand side zr at node zp of the line;
  // bit b of zmk[d]: local node (zp + d - 1, b) is in the r set (0 off the line)
  const int zr = threadIdx.x / ml, zp = threadIdx.x - zr * ml;
  const bool zon = (int)threadIdx.x < ml * nr;
  uint64_t zmk[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) zmk[d] = zon ? rnode_column(g, s, zp + d - 1) : 0;
  __syncthreads();
  for (int t0 = 0; t0 < nsteps; t0 += LRING) {
#pragma unroll
    for (int u = 0; u < LRING; ++u) {
      const int t = t0 + u;
      if (t < nsteps) {
        const int j = line_of(t);
        if (t < ml) {
          // forward: z_j = f_j - A_j,j-1 t_j-1 ; t_j = G_j z_j (t_j overwrites f_j in xall)
          if (zon) {
            const int r = zr, p = zp;
            const T* xr = xall + r * XS;
            T v = xr[p + ml * j];
            if (j > 0 && ((zmk[1] >> j) & 1)) {
#pragma unroll
              for (int d = 0; d < 3; ++d)
                if ((zmk[d] >> (j - 1)) & 1) v = v - cpl[p][d] * xr[p + d - 1 + ml * (j - 1)];
            }
            zl[r * ML + p] = v;
          }
          lds_sync();
          line_mv<TS, T, NRT>(gbuf, ml, zl, red, xall + ml * j, XS, false, nr);
        } else {
          // backward: x_j = t_j - G_j A_j,j+1 x_j+1
          if (zon) {
            const int r = zr, p = zp;
            const T* xr = xall + r * XS;
            T v{0, 0};
            if ((zmk[1] >> j) & 1) {
#pragma unroll
              for (int d = 0; d < 3; ++d)
                if ((zmk[d] >> (j + 1)) & 1) fma_acc(v, cpl[p][d], xr[p + d - 1 + ml * (j + 1)]);
            }
            zl[r * ML + p] = v;
          }
          lds_sync();
          line_mv<TS, T, NRT>(gbuf, ml, zl, red, xall + ml * j, XS, true, nr);
        }
        // stage the next step's line (ring slot (u + 1) % LRING), refill that slot:
        // gbuf is free since line_mv's partial products, so one barrier orders
        // both this store and line_mv's row sums before the next step
        if (t + 1 < nsteps) {
          line_store<TS>(gbuf, n2, greg[(u + 1) % LRING]);
          if (t + 1 + LRING < nsteps)
            line_load<TS>(Gs + (size_t)line_of(t + 1 + LRING) * n2, n2, greg[(u + 1) % LRING]);
        }
        lds_sync();
      }
    }
  }
  // outputs (right-hand side r at its stride)
  const int nd = mp.nd[s];
  if (mode == 0) {
    for (int t = threadIdx.x; t < nd * nr; t += blockDim.x) {
      const int r = t / nd, i = t - r * nd;
      T x = xall[r * XS + mp.dloc[s * ND + i]];
      Xd[r * rs.sb + (size_t)s * ND + i] = cd{(double)x.x, (double)x.y};
    }
    if (threadIdx.x < 4 * nr) {
      const int r = threadIdx.x / 4, q = threadIdx.x % 4;
      int cl = mp.cloc[s * 4 + q];
      cd acc{0.0, 0.0};
      if (cl >= 0) {
        int ca = cl % ml, cb = cl / ml;
        for (int b = max(cb - 1, 0); b <= min(cb + 1, ml - 1); ++b)
          for (int a = max(ca - 1, 0); a <= min(ca + 1, ml - 1); ++a) {
            if (!g.rnode(s, a, b)) continue;
            T x = xall[r * XS + a + ml * b];
            fma_acc(acc, g.zloc(ca, cb, a, b), cd{(double)x.x, (double)x.y});
          }
      }
      Qc[r * rs.cq + s * NQ + q] = acc;
    }
  } else {
    for (int t = threadIdx.x; t < nd * nr; t += blockDim.x) {
      const int r = t / nd, i = t - r * nd;
      T x = xall[r * XS + mp.dloc[s * ND + i]];
      Ubuf[r * rs.sb + (size_t)s * ND + i] = cd{(double)x.x, (double)x.y};
    }
    for (int l = threadIdx.x; l < n2; l += blockDim.x) {
      int a = l % ml, b = l / ml;
      if (a == 0 || a == ml - 1 || b == 0 || b == ml - 1) continue;  // interior only
      const int64_t fi = g.freeidx(s, a, b);
#pragma unroll
      for (int r = 0; r < NRT; ++r) {
        if (r >= nr) break;
        T x = xall[r * XS + l];
        cd v{(double)x.x, (double)x.y};
        xout[r * rs.nf + fi] = conj_out ? conj(v) : v;
      }
    }
  }
}

// One workgroup per (instance, subdomain); instances with no group skip.
template <class TS, int NRT, class Src>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_local_solve(Src src, int mode, int fsel, int conj_in, int xsel) {
  const Dev& d = src.dev();
  if (d.nr <= 0) return;
  local_solve_body<TS, NRT>(d.g, d.mp, d.rs, d.nr, (const TS*)d.G, mode, dev_vec(d, fsel), conj_in,
                            d.u0, d.mu, d.Xd, d.Qc, d.Ubuf, mode == 1 ? dev_vec(d, xsel) : nullptr,
                            mode == 1 ? conj_in : 0, src.bx());
}

// One workgroup per (instance, subdomain, right-hand side r = blockIdx.y): the
// right-hand sides of a group walk their line sweeps in separate workgroups,
// several per CU, so one's barriers and load latencies overlap the others'
// work.  The workgroups of one subdomain have block ids that differ by
// multiples of the grid width; when that width is a multiple of 8 they share
// an XCD, and the L2 copy of the subdomain's line factors.
template <class TS, class Src>
__global__ void __launch_bounds__(256) k_local_solve_rhs(Src src, int mode, int fsel, int conj_in, int xsel) {
  const Dev& d = src.dev();
  const int r = blockIdx.y;
  if (r >= d.nr) return;
  const RhsStride& rs = d.rs;
  local_solve_body<TS, 1>(d.g, d.mp, rs, 1, (const TS*)d.G, mode, dev_vec(d, fsel) + r * rs.nf, conj_in,
                          d.u0 + r * rs.nc, d.mu + r * rs.nmu, d.Xd + r * rs.sb, d.Qc + r * rs.cq,
                          d.Ubuf + r * rs.sb, mode == 1 ? dev_vec(d, xsel) + r * rs.nf : nullptr,
                          mode == 1 ? conj_in : 0, src.bx());
}

// Wave-level LDS ordering: this wave's LDS writes complete before its later
// reads (and the compiler keeps LDS accesses on their side); no workgroup
// barrier, so waves of a workgroup never wait for each other.
__device__ inline void wave_lds_sync() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt = 0
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

// Full local solve with E^s for one right-hand side by one wavefront (the same
// results as local_solve_body up to the order of the sums).  Lane p owns node p
// of every line: it keeps row p of the current line factor in registers (a ring
// of LRW lines loaded ahead) and forms that row of every dense product against
// the line vector z, which the wave shares through LDS.  The line recursion is
// serial, so the wave's whole sweep runs without workgroup barriers; the
// wavefronts of a subdomain's other right-hand sides read the same line
// factors shortly after it, from L2.
template <class TS>
__device__ inline void local_solve_wave(const Geo2& g, const Maps2& mp, const RhsStride& rs,
                                        const TS* __restrict__ G, int mode, const cd* __restrict__ f,
                                        int conj_in, const cd* __restrict__ uc, const cd* __restrict__ mu,
                                        cd* Xd, cd* Qc, cd* Ubuf, cd* xout, int conj_out, int s) {
  constexpr int XS = ML * ML;
  __shared__ cd xall[XS];
  __shared__ cd zl[ML];
  const int lane = threadIdx.x;
  const int ml = g.ml, n2 = ml * ml, ND = g.ND;
  const TS* Gs = G + (size_t)s * ml * n2;
  constexpr int LRW = sizeof(TS) == sizeof(cf) ? 3 : 2;
  const int nsteps = 2 * ml - 1;
  auto line_of = [&](int t) { return t < ml ? t : 2 * ml - 2 - t; };
  // row p of line j: G(p, k) at Gs[j n2 + k ml + p] (stored transposed), k < ML
  // clamped to ml - 1 (zl is zero beyond ml, so those terms vanish)
  const int pc = min(lane, ml - 1);
  TS gr[LRW][ML];
  auto gload = [&](int t, TS (&dst)[ML]) {
    const TS* src = Gs + (size_t)line_of(t) * n2 + pc;
#pragma unroll
    for (int k = 0; k < ML; ++k) dst[k] = src[min(k, ml - 1) * ml];
  };
#pragma unroll
  for (int u = 0; u < LRW; ++u)
    if (u < nsteps) gload(u, gr[u]);
  if (lane < ML) zl[lane] = cd{0.0, 0.0};
  // right-hand side on the r nodes (f / multiplicity; mode 1 minus the corner terms)
  for (int l = lane; l < n2; l += 64) {
    const int a = l % ml, b = l / ml;
    const bool rn = g.rnode(s, a, b);
    cd v{0.0, 0.0};
    if (rn) {
      const cd fv = f[g.freeidx(s, a, b)];
      v = (1.0 / g.mult(a, b)) * (conj_in ? conj(fv) : fv);
      if (mode == 1)
        for (int q = 0; q < 4; ++q) {
          const int cl = mp.cloc[s * 4 + q];
          if (cl < 0) continue;
          const int ca = cl % ml, cb = cl / ml;
          if (abs(ca - a) > 1 || abs(cb - b) > 1) continue;
          v = v - g.zloc(a, b, ca, cb) * uc[mp.cgid[s * NQ + q]];
        }
    }
    xall[l] = v;
  }
  wave_lds_sync();
  if (mode == 1) {
    const int nd = mp.nd[s];
    for (int i = lane; i < nd; i += 64) {
      const int l = mp.dloc[s * ND + i];
      xall[l] = xall[l] - (double)mp.dsgn[s * ND + i] * mu[mp.dmid[s * ND + i]];
    }
    wave_lds_sync();
  }
  // couplings of node p to nodes p - 1, p, p + 1 of the adjacent line, and the
  // r-set masks of those three grid columns (bit b: node (p + d - 1, b) is an r node)
  const bool on = lane < ml;
  uint64_t zmk[3];
  cd cpl[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int a = lane + d - 1;
    zmk[d] = on ? rnode_column(g, s, a) : 0;
    cpl[d] = (on && a >= 0 && a < ml) ? g.zloc(lane, 1, a, 2) : cd{0.0, 0.0};
  }
  for (int t0 = 0; t0 < nsteps; t0 += LRW) {
#pragma unroll
    for (int u = 0; u < LRW; ++u) {
      const int t = t0 + u;
      if (t < nsteps) {
        const int j = line_of(t);
        const bool fwd = t < ml;
        if (on) {
          cd v{0.0, 0.0};
          if (fwd) {
            // z_j = f_j - A_j,j-1 t_j-1
            v = xall[lane + ml * j];
            if (j > 0 && ((zmk[1] >> j) & 1)) {
#pragma unroll
              for (int d = 0; d < 3; ++d)
                if ((zmk[d] >> (j - 1)) & 1) v = v - cpl[d] * xall[lane + d - 1 + ml * (j - 1)];
            }
          } else if ((zmk[1] >> j) & 1) {
            // A_j,j+1 x_j+1
#pragma unroll
            for (int d = 0; d < 3; ++d)
              if ((zmk[d] >> (j + 1)) & 1) fma_acc(v, cpl[d], xall[lane + d - 1 + ml * (j + 1)]);
          }
          zl[lane] = v;
        }
        wave_lds_sync();
        // row p of G_j z: two accumulators (even and odd k) shorten the FMA chains
        cd a0{0.0, 0.0}, a1{0.0, 0.0};
#pragma unroll
        for (int k = 0; k + 1 < ML; k += 2) {
          fma_acc(a0, cvt<double>(gr[u][k]), zl[k]);
          fma_acc(a1, cvt<double>(gr[u][k + 1]), zl[k + 1]);
        }
        if (ML & 1) fma_acc(a0, cvt<double>(gr[u][ML - 1]), zl[ML - 1]);
        const cd tv = a0 + a1;
        if (on) {
          cd* o = xall + lane + ml * j;
          *o = fwd ? tv : *o - tv;  // forward: t_j = G_j z_j; backward: x_j = t_j - G_j A x_j+1
        }
        wave_lds_sync();
        if (t + LRW < nsteps) gload(t + LRW, gr[u]);
      }
    }
  }
  // outputs
  const int nd = mp.nd[s];
  if (mode == 0) {
    for (int i = lane; i < nd; i += 64) Xd[(size_t)s * ND + i] = xall[mp.dloc[s * ND + i]];
    if (lane < 4) {
      const int cl = mp.cloc[s * 4 + lane];
      cd acc{0.0, 0.0};
      if (cl >= 0) {
        const int ca = cl % ml, cb = cl / ml;
        for (int b = max(cb - 1, 0); b <= min(cb + 1, ml - 1); ++b)
          for (int a = max(ca - 1, 0); a <= min(ca + 1, ml - 1); ++a)
            if (g.rnode(s, a, b)) fma_acc(acc, g.zloc(ca, cb, a, b), xall[a + ml * b]);
      }
      Qc[s * NQ + lane] = acc;
    }
  } else {
    for (int i = lane; i < nd; i += 64) Ubuf[(size_t)s * ND + i] = xall[mp.dloc[s * ND + i]];
    for (int l = lane; l < n2; l += 64) {
      const int a = l % ml, b = l / ml;
      if (a == 0 || a == ml - 1 || b == 0 || b == ml - 1) continue;  // interior only
      const cd v = xall[l];
      xout[g.freeidx(s, a, b)] = conj_out ? conj(v) : v;
    }
  }
}

// One wavefront (workgroup of 64) per (instance, subdomain, right-hand side
// r = blockIdx.y).  Block ids of one subdomain's right-hand sides differ by
// multiples of the grid width; when that width is a multiple of 8 they share an
// XCD, and so the L2 copy of the subdomain's line factors.
template <class TS, class Src>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_local_solve_wave(Src src, int mode, int fsel, int conj_in, int xsel) {
  const Dev& d = src.dev();
  const int r = blockIdx.y;
  if (r >= d.nr) return;
  const RhsStride& rs = d.rs;
  local_solve_wave<TS>(d.g, d.mp, rs, (const TS*)d.G, mode, dev_vec(d, fsel) + r * rs.nf, conj_in,
                       d.u0 + r * rs.nc, d.mu + r * rs.nmu, d.Xd + r * rs.sb, d.Qc + r * rs.cq,
                       d.Ubuf + r * rs.sb, mode == 1 ? dev_vec(d, xsel) + r * rs.nf : nullptr,
                       mode == 1 ? conj_in : 0, src.bx());
}

// Values of the adjacent lanes (DPP wavefront shifts; lane 0, resp. 63, gets
// zero).  Every lane of the wave must be active.
__device__ inline double dpp_shr1(double v) {  // lane p <- lane p - 1
  const int lo = __builtin_amdgcn_update_dpp(0, (int)__double2loint(v), 0x138, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)__double2hiint(v), 0x138, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ inline double dpp_shl1(double v) {  // lane p <- lane p + 1
  const int lo = __builtin_amdgcn_update_dpp(0, (int)__double2loint(v), 0x130, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)__double2hiint(v), 0x130, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ inline cd lane_from_below(cd v) { return cd{dpp_shr1(v.x), dpp_shr1(v.y)}; }
__device__ inline cd lane_from_above(cd v) { return cd{dpp_shl1(v.x), dpp_shl1(v.y)}; }

// Sum of a lane's value and its partner's 32 lanes away, the lower half's
// value first (v_permlane32_swap: each lane sees lane (l mod 32) and lane
// 32 + (l mod 32)); .x holds the sum, in every lane of the pair the same bits.
__device__ inline cd halves_sum(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const auto sl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto sh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const double a = __hiloint2double(sh[0], sl[0]), b = __hiloint2double(sh[1], sl[1]);
  return cd{a + b, 0.0};
}
// Sum over lanes 0 .. 47 (the caller's values are zero from lane 33 on):
// inclusive scans within each row of 16 lanes (DPP row shifts by 1, 2, 4, 8),
// then the three row totals read from lanes 15, 31, 47.  Every lane gets it.
__device__ inline double row_scan16(double v) {
#define SFDP_ROW_SHR(v, n)                                                                              \
  __hiloint2double(__builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x110 + (n), 0xf, 0xf, true),      \
                   __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x110 + (n), 0xf, 0xf, true))
  v = v + SFDP_ROW_SHR(v, 1);
  v = v + SFDP_ROW_SHR(v, 2);
  v = v + SFDP_ROW_SHR(v, 4);
  v = v + SFDP_ROW_SHR(v, 8);
#undef SFDP_ROW_SHR
  return v;
}
__device__ inline double lane_value(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ inline cd row32_sum(cd c) {
  const double x = row_scan16(c.x), y = row_scan16(c.y);
  return cd{(lane_value(x, 15) + lane_value(x, 31)) + lane_value(x, 47),
            (lane_value(y, 15) + lane_value(y, 31)) + lane_value(y, 47)};
}

// Full local solve with E^s for nr <= 4 right-hand sides by one workgroup of
// four wavefronts (the same results as local_solve_body up to the order of the
// sums).  Wave w runs the line recursion of right-hand side w: lane p owns node
// p of every line, keeps the previous step's result at its node in a register
// (the neighbours' values come from the adjacent lanes by DPP shifts) and reads
// its node's value of the current line from LDS one step ahead, so the only LDS
// round trip inside a step is the line product.  That product runs by lane
// pairs: the two halves of the wavefront each sum 17 of the 33 terms of rows
// 0 .. 31 and a 32-lane swap joins them; row 32 is one term per lane summed by
// row scans.  The workgroup stages every line factor into LDS once for all
// right-hand sides: the factor of step t + 1 is copied from a ring of GRD
// register copies (each loaded GRD - 1 steps before it is stored), widened to
// FP64, into one of two LDS slots while step t reads the other, and one
// workgroup barrier per step separates the two.  The factors leave HBM once per
// subdomain, where one workgroup or one wavefront per right-hand side reads
// them once per right-hand side (from L2 when their sweeps stay close).
// MLC = ML compiles the form for 33-node lines (constant offsets), MLC = 0 any
// line length up to ML.  lds: ls_group_bytes() bytes.
constexpr int LSG_GE = (ML * ML + 255) / 256;  // line-factor entries staged per thread
constexpr int LSG_KH = (ML + 1) / 2;           // product terms per wavefront half (17)
constexpr int LSG_KC0 = 9, LSG_KC1 = LSG_KH - LSG_KC0;  // the two register chunks of a half
static_assert(ML == 33, "rows 0 .. 31 by lane pairs plus row 32");
__host__ __device__ constexpr size_t ls_group_bytes() {
  return 4 * ML * ML * sizeof(cd) + 4 * 64 * sizeof(cd) + 2 * ML * ML * sizeof(cd);
}
template <class TS, int MLC>
__device__ inline void local_solve_group(const Geo2& g, const Maps2& mp, const RhsStride& rs, int nr,
                                         const TS* __restrict__ G, int mode, const cd* __restrict__ f0,
                                         int conj_in, const cd* __restrict__ uc0, const cd* __restrict__ mu0,
                                         cd* Xd0, cd* Qc0, cd* Ubuf0, cd* xout0, int conj_out, int s,
                                         char* lds) {
  constexpr int XS = ML * ML;
  constexpr int GRD = 3;  // line factors in flight per thread
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  cd* xall = (cd*)lds + (size_t)w * XS;
  cd* zl = (cd*)lds + 4 * XS + w * 64;
  cd* gbuf = (cd*)(lds + 4 * XS * sizeof(cd) + 4 * 64 * sizeof(cd));  // factors staged in FP64
  const int ml = MLC ? MLC : g.ml, n2 = ml * ml, ND = g.ND;
  const TS* Gs = G + (size_t)s * ml * n2;
  const int nsteps = 2 * ml - 1;
  auto line_of = [&](int t) { return t < ml ? t : 2 * ml - 2 - t; };
  // staging: thread e takes entries e, e + 256, ... of a line (clamped loads)
  // the ring holds the entries as two-lane vectors of their real type, which
  // the compiler keeps in registers (an array of the struct type it did not)
  using RV = decltype(TS{}.x);
  typedef RV GV __attribute__((ext_vector_type(2)));
  GV greg[GRD * LSG_GE];
#define LSG_LOAD(t, slot)                                                                        \
  {                                                                                              \
    const GV* src_ = (const GV*)(Gs + (size_t)line_of(t) * n2);                                  \
    _Pragma("unroll") for (int i = 0; i < LSG_GE; ++i)                                           \
      greg[(slot) * LSG_GE + i] = src_[min((int)threadIdx.x + 256 * i, n2 - 1)];                 \
  }
#define LSG_STORE(t, slot)                                                                       \
  {                                                                                              \
    cd* dst_ = gbuf + ((t) & 1) * XS;                                                            \
    _Pragma("unroll") for (int i = 0; i < LSG_GE; ++i) {                                         \
      const int e_ = threadIdx.x + 256 * i;                                                      \
      const GV v_ = greg[(slot) * LSG_GE + i];                                                   \
      if (e_ < n2) dst_[e_] = cd{(double)v_.x, (double)v_.y};                                    \
    }                                                                                            \
  }
#pragma unroll
  for (int u = 0; u < GRD; ++u)
    if (u < nsteps) LSG_LOAD(u, u);
  const bool act = w < nr;  // uniform over the wave
  const cd* f = f0 + w * rs.nf;
  const cd* uc = uc0 + w * rs.nc;
  const cd* mu = mu0 + w * rs.nmu;
  zl[lane] = cd{0.0, 0.0};  // entries ml .. 63 stay zero
  if (act) {
    // right-hand side on the r nodes (f / multiplicity; mode 1 minus the corner terms)
    for (int l = lane; l < n2; l += 64) {
      const int a = l % ml, b = l / ml;
      const bool rn = g.rnode(s, a, b);
      cd v{0.0, 0.0};
      if (rn) {
        const cd fv = f[g.freeidx(s, a, b)];
        v = (1.0 / g.mult(a, b)) * (conj_in ? conj(fv) : fv);
        if (mode == 1)
          for (int q = 0; q < 4; ++q) {
            const int cl = mp.cloc[s * 4 + q];
            if (cl < 0) continue;
            const int ca = cl % ml, cb = cl / ml;
            if (abs(ca - a) > 1 || abs(cb - b) > 1) continue;
            v = v - g.zloc(a, b, ca, cb) * uc[mp.cgid[s * NQ + q]];
          }
      }
      xall[l] = v;
    }
    wave_lds_sync();
    if (mode == 1) {
      const int nd = mp.nd[s];
      for (int i = lane; i < nd; i += 64) {
        const int l = mp.dloc[s * ND + i];
        xall[l] = xall[l] - (double)mp.dsgn[s * ND + i] * mu[mp.dmid[s * ND + i]];
      }
      wave_lds_sync();
    }
  }
  LSG_STORE(0, 0);
  __syncthreads();
  // couplings of node p to nodes p - 1, p, p + 1 of the adjacent line, and the
  // r-set masks of those three grid columns (bit b: node (p + d - 1, b) is an r node)
  const bool on = act && lane < ml;
  const int pc = min(lane, ml - 1);
  uint64_t zmk[3];
  cd cpl[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int a = lane + d - 1;
    zmk[d] = on ? rnode_column(g, s, a) : 0;
    cpl[d] = (on && a >= 0 && a < ml) ? g.zloc(lane, 1, a, 2) : cd{0.0, 0.0};
  }
  // per-lane state of the recursion: the previous step's result at node p
  // (forward: t_(j-1); backward: x_(j+1)), whose neighbours p - 1 and p + 1 come
  // from the adjacent lanes by DPP shifts, and the current line's own value
  // (forward: f_j; backward: t_j), read from LDS one step ahead
  cd tprev{0.0, 0.0};
  cd fcur = on ? xall[lane] : cd{0.0, 0.0};
  // one step; U = t mod GRD is a compile-time constant, so the register ring
  // is indexed statically
  auto step = [&](int t, auto uconst) {
    constexpr int u = decltype(uconst)::value;
    {
      {
        // greg[u] (the factor of step t) is in LDS: reuse it for step t + GRD
        if (t + GRD < nsteps) LSG_LOAD(t + GRD, u);
        if (act) {
          const int j = line_of(t);
          const bool fwd = t < ml;
          const cd fnext = (on && t + 1 < nsteps) ? xall[lane + ml * line_of(t + 1)] : cd{0.0, 0.0};
          const cd nb[3] = {lane_from_below(tprev), tprev, lane_from_above(tprev)};
          cd vz{0.0, 0.0};  // z at this lane's node (zero off the line)
          if (on) {
            cd v{0.0, 0.0};
            if (fwd) {
              // z_j = f_j - A_j,j-1 t_j-1
              v = fcur;
              if (j > 0 && ((zmk[1] >> j) & 1)) {
#pragma unroll
                for (int d = 0; d < 3; ++d)
                  if ((zmk[d] >> (j - 1)) & 1) v = v - cpl[d] * nb[d];
              }
            } else if ((zmk[1] >> j) & 1) {
              // A_j,j+1 x_j+1
#pragma unroll
              for (int d = 0; d < 3; ++d)
                if ((zmk[d] >> (j + 1)) & 1) fma_acc(v, cpl[d], nb[d]);
            }
            zl[lane] = v;
            vz = v;
          }
          wave_lds_sync();
          // G_j z (G stored transposed: G(p, k) at k ml + p; k clamped to ml - 1,
          // where z is zero).  Rows q = 0 .. 31: the half h = lane / 32 of the
          // wavefront sums the terms k = 17 h .. 17 h + 16 (z is zero from ml on),
          // lane q + 32 h taking row q, four accumulators (i mod 4); the operands
          // go to registers a chunk at a time, the next chunk's LDS reads issued
          // before the current chunk's multiply-adds (the scheduling barriers keep
          // the compiler from sinking each read to its use).  The two halves' sums
          // meet by a 32-lane swap.  Row 32 (ml = 33): one term per lane, summed
          // by row scans and three lane reads.
          const int q = lane & 31, kb = (lane >> 5) * LSG_KH;
          const cd* gl = gbuf + (t & 1) * XS + min(q, ml - 1);
          cd acc[4] = {cd{0.0, 0.0}, cd{0.0, 0.0}, cd{0.0, 0.0}, cd{0.0, 0.0}};
          cd gk[2][LSG_KC0];
          cd zk[2][LSG_KC0];
          // 33-node lines: terms i < 16 at constant offsets from the half's first
          // row; the 17th (k = 33 in the upper half, where z is zero) reads row 32
          const cd* glb = gl + kb * ml;
          const cd* gl16 = gl + min(kb + LSG_KH - 1, ml - 1) * ml;
          auto fetch = [&](int i0, int n, int b) {
#pragma unroll
            for (int i = 0; i < LSG_KC0; ++i) {
              if (i < n) {
                const int k = kb + i0 + i;
                if constexpr (MLC == ML)
                  gk[b][i] = i0 + i < LSG_KH - 1 ? glb[(i0 + i) * ML] : *gl16;
                else
                  gk[b][i] = gl[min(k, ml - 1) * ml];
                zk[b][i] = zl[k];
              }
            }
          };
          fetch(0, LSG_KC0, 0);
          fetch(LSG_KC0, LSG_KC1, 1);
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int i = 0; i < LSG_KC0; ++i) fma_acc(acc[i & 3], gk[0][i], zk[0][i]);
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int i = 0; i < LSG_KC1; ++i) fma_acc(acc[(LSG_KC0 + i) & 3], gk[1][i], zk[1][i]);
          const cd part = (acc[0] + acc[1]) + (acc[2] + acc[3]);
          // lanes q and q + 32 both get half 0's and half 1's sums of row q
          const cd lo_hi_x = halves_sum(part.x), lo_hi_y = halves_sum(part.y);
          cd tv{lo_hi_x.x, lo_hi_y.x};
          if (ml == ML) {
            // row 32: term G(32, l) z_l in lane l < 33
            cd c32{0.0, 0.0};
            const cd g32 = gbuf[(t & 1) * XS + min(lane, ml - 1) * ml + (ML - 1)];
            fma_acc(c32, g32, vz);
            const cd r32 = row32_sum(c32);
            if (lane == ML - 1) tv = r32;
          }          // forward: t_j = G_j z_j; backward: x_j = t_j - G_j A x_j+1
          const cd res = fwd ? tv : fcur - tv;
          if (on) xall[lane + ml * j] = res;
          tprev = res;
          fcur = fnext;
        }
        // the factor of step t + 1 into the other slot (its last reader, step
        // t - 1, finished before the previous barrier)
        if (t + 1 < nsteps) LSG_STORE(t + 1, (u + 1) % GRD);
        __syncthreads();
      }
    }
  };
  static_assert(GRD == 3, "the step calls below cover GRD ring slots");
  for (int t0 = 0; t0 < nsteps; t0 += GRD) {
    step(t0, std::integral_constant<int, 0>{});
    if (t0 + 1 < nsteps) step(t0 + 1, std::integral_constant<int, 1>{});
    if (t0 + 2 < nsteps) step(t0 + 2, std::integral_constant<int, 2>{});
  }
#undef LSG_LOAD
#undef LSG_STORE
  if (!act) return;
  wave_lds_sync();
  // outputs
  const int nd = mp.nd[s];
  if (mode == 0) {
    cd* Xd = Xd0 + w * rs.sb;
    cd* Qc = Qc0 + w * rs.cq;
    for (int i = lane; i < nd; i += 64) Xd[(size_t)s * ND + i] = xall[mp.dloc[s * ND + i]];
    if (lane < 4) {
      const int cl = mp.cloc[s * 4 + lane];
      cd acc{0.0, 0.0};
      if (cl >= 0) {
        const int ca = cl % ml, cb = cl / ml;
        for (int b = max(cb - 1, 0); b <= min(cb + 1, ml - 1); ++b)
          for (int a = max(ca - 1, 0); a <= min(ca + 1, ml - 1); ++a)
            if (g.rnode(s, a, b)) fma_acc(acc, g.zloc(ca, cb, a, b), xall[a + ml * b]);
      }
      Qc[s * NQ + lane] = acc;
    }
  } else {
    cd* Ubuf = Ubuf0 + w * rs.sb;
    cd* xout = xout0 + w * rs.nf;
    for (int i = lane; i < nd; i += 64) Ubuf[(size_t)s * ND + i] = xall[mp.dloc[s * ND + i]];
    for (int l = lane; l < n2; l += 64) {
      const int a = l % ml, b = l / ml;
      if (a == 0 || a == ml - 1 || b == 0 || b == ml - 1) continue;  // interior only
      const cd v = xall[l];
      xout[g.freeidx(s, a, b)] = conj_out ? conj(v) : v;
    }
  }
}

// One workgroup of four wavefronts per (instance, subdomain), wave w serving
// right-hand side w; dynamic LDS ls_group_bytes().  MLC = ML when every
// instance of the launch has 33-node lines, else 0.
template <class TS, int MLC, class Src>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_local_solve_group(Src src, int mode, int fsel, int conj_in, int xsel) {
  const Dev& d = src.dev();
  if (d.nr <= 0) return;
  extern __shared__ __align__(16) char smem[];
  const RhsStride& rs = d.rs;
  local_solve_group<TS, MLC>(d.g, d.mp, rs, d.nr, (const TS*)d.G, mode, dev_vec(d, fsel), conj_in, d.u0, d.mu,
                        d.Xd, d.Qc, d.Ubuf, mode == 1 ? dev_vec(d, xsel) : nullptr, mode == 1 ? conj_in : 0,
                        src.bx(), smem);
}

// Edge slots of Qc: Qc[s][4 + j] = sum over the Delta slots on side j of
// sign * Xd, subdomain s's share of q_e^T d_r (d_r = sum_s B_r Z_rr^-1 f_r).
// One workgroup per subdomain; wave j sums side j.
template <class Src>
__global__ void k_edge_rhs(Src src) {
  const Dev& d = src.dev();
  const Geo2& g = d.g;
  const Maps2& mp = d.mp;
  const RhsStride& rs = d.rs;
  if ((int)blockIdx.y >= d.nr) return;
  const int s = src.bx(), lane = threadIdx.x & 63, j = threadIdx.x >> 6, nd = mp.nd[s];
  const int64_t r = blockIdx.y;
  const cd* Xd = d.Xd + r * rs.sb + (size_t)s * g.ND;
  cd acc{0.0, 0.0};
  for (int i = lane; i < nd; i += 64)
    if (mp.dedge[s * g.ND + i] == 4 + j) acc = acc + (double)mp.dsgn[s * g.ND + i] * Xd[i];
  for (int off = 32; off > 0; off >>= 1) {
    acc.x += __shfl_down(acc.x, off, 64);
    acc.y += __shfl_down(acc.y, off, 64);
  }
  if (lane == 0) d.Qc[r * rs.cq + s * NQ + 4 + j] = acc;
}

// Coarse right-hand side c0 (one thread per coarse unknown, fixed order):
// corners f_c* = f_c - sum_s B_c^T Z_cr Z_rr^-1 f_r; edges -q_e^T d_r.
template <class Src>
__global__ void k_coarse_rhs(Src src, int fsel, int conj_in) {
  const Dev& d = src.dev();
  const Geo2& g = d.g;
  const Maps2& mp = d.mp;
  const RhsStride& rs = d.rs;
  int c = src.bx() * blockDim.x + threadIdx.x;
  if (c >= g.nK || (int)blockIdx.y >= d.nr) return;
  const int64_t r = blockIdx.y;
  const cd* f = dev_vec(d, fsel);
  const cd* Qc = d.Qc;
  cd* fcs = d.fcs;
  f += r * rs.nf;
  Qc += r * rs.cq;
  fcs += r * rs.nc;
  cd v{0.0, 0.0};
  if (c < g.nC) {
    v = f[mp.cfree[c]];
    if (conj_in) v = conj(v);
  }
  for (int o = 0; o < 4; ++o) {
    int own = mp.cown[c * 4 + o];
    if (own >= 0) v = v - Qc[own];
  }
  fcs[c] = v;
}

// u0_r = Kinv x_r (x from dev_vec(xsel)) for every right-hand side r < nr: one
// wavefront per coarse row reads that row of the coarse inverse once for all
// right-hand sides, four of its strides' loads issued before their
// multiply-adds; each right-hand side's terms in the order k = lane, lane + 64,
// ..., then the wavefront sum.
template <class Src>
__global__ void k_dense_mv(Src src, int xsel) {
  const Dev& d = src.dev();
  const int nr = d.nr;
  if (nr <= 0) return;
  const int n = d.g.nK, row = src.bx();
  const int64_t stride = d.rs.nc;
  const cd* __restrict__ A = d.Kinv + (size_t)row * n;
  const cd* x = dev_vec(d, xsel);
  cd acc[NRMAX];
#pragma unroll
  for (int r = 0; r < NRMAX; ++r) acc[r] = cd{0.0, 0.0};
  int k = threadIdx.x;
  for (; k + 192 < n; k += 256) {
    cd a[4], xv[4][NRMAX];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = A[k + 64 * u];
#pragma unroll
      for (int r = 0; r < NRMAX; ++r) xv[u][r] = r < nr ? x[r * stride + k + 64 * u] : cd{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int r = 0; r < NRMAX; ++r) fma_acc(acc[r], a[u], xv[u][r]);
  }
  for (; k < n; k += 64) {
    const cd a = A[k];
#pragma unroll
    for (int r = 0; r < NRMAX; ++r)
      if (r < nr) fma_acc(acc[r], a, x[r * stride + k]);
  }
#pragma unroll
  for (int r = 0; r < NRMAX; ++r) {
    if (r >= nr) break;
    cd v = acc[r];
    for (int off = 32; off > 0; off >>= 1) {
      v.x += __shfl_down(v.x, off, 64);
      v.y += __shfl_down(v.y, off, 64);
    }
    if (threadIdx.x == 0) d.u0[r * stride + row] = v;
  }
}

// d_k = sum over the two subdomains of sign * (Xd - sum over coarse slots Phi u0)
template <class TS, class Src>
__global__ void k_fetidp_rhs(Src src) {
  const Dev& dv = src.dev();
  const Geo2& g = dv.g;
  const Maps2& mp = dv.mp;
  const RhsStride& rs = dv.rs;
  int k = src.bx() * blockDim.x + threadIdx.x;
  if (k >= g.nmu || (int)blockIdx.y >= dv.nr) return;
  const int64_t r = blockIdx.y;
  const cd* Xd = dv.Xd;
  const TS* Phi = (const TS*)dv.Phi;
  const cd* u0 = dv.u0;
  cd* d = dv.dvec;
  Xd += r * rs.sb;
  u0 += r * rs.nc;
  d += r * rs.nmu;
  cd out{0.0, 0.0};
  for (int e = 0; e < 2; ++e) {
    int o = mp.muown[2 * k + e];
    int s = o / g.ND, slot = o % g.ND;
    cd v = Xd[o];
    for (int q = 0; q < NQ; ++q) {
      int c = mp.cgid[s * NQ + q];
      if (c < 0 || c >= g.nK) continue;
      cd ph = cvt<double>(Phi[((size_t)s * g.ND + slot) * NQ + q]);
      v = v - ph * u0[c];
    }
    out = e == 0 ? out + v : out - v;
  }
  d[k] = out;
}

// c^s_q = sum_i Phi[s][i][q] sign_i mu[mid_i]  (G^T mu contributions: F_rc^T mu
// for corner slots, Q^T F_rr mu for edge slots); one wavefront per (subdomain,
// coarse slot), launched with NQ waves per block.
template <class TS, class Src>
__global__ void k_frct(Src src) {
  const Dev& d = src.dev();
  const Geo2& g = d.g;
  const Maps2& mp = d.mp;
  const RhsStride& rs = d.rs;
  int t = src.bx() * (blockDim.x / 64) + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (t >= g.nsub * NQ || (int)blockIdx.y >= d.nr) return;
  const int64_t r = blockIdx.y;
  const TS* Phi = (const TS*)d.Phi;
  const cd* mu = d.mu;
  cd* Cbuf = d.Cbuf;
  mu += r * rs.nmu;
  Cbuf += r * rs.cq;
  int s = t / NQ, q = t % NQ;
  cd acc{0.0, 0.0};
  const int c = mp.cgid[s * NQ + q];
  if (c >= 0 && c < g.nK) {
    int nd = mp.nd[s];
    for (int i = lane; i < nd; i += 64) {
      cd x = (double)mp.dsgn[s * g.ND + i] * mu[mp.dmid[s * g.ND + i]];
      fma_acc(acc, cvt<double>(Phi[((size_t)s * g.ND + i) * NQ + q]), x);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    acc.x += __shfl_down(acc.x, off, 64);
    acc.y += __shfl_down(acc.y, off, 64);
  }
  if (lane == 0) Cbuf[t] = acc;
}

// ymin_c = fcs_c + sum_owners Cbuf  (every coarse unknown c < nK)
template <class Src>
__global__ void k_corner_sum(Src src) {
  const Dev& d = src.dev();
  const Geo2& g = d.g;
  const Maps2& mp = d.mp;
  const RhsStride& rs = d.rs;
  int c = src.bx() * blockDim.x + threadIdx.x;
  if (c >= g.nK || (int)blockIdx.y >= d.nr) return;
  const int64_t r = blockIdx.y;
  const cd* fcs = d.fcs;
  const cd* Cbuf = d.Cbuf;
  cd* out = d.ymin;
  if (fcs) fcs += r * rs.nc;
  Cbuf += r * rs.cq;
  out += r * rs.nc;
  cd v = fcs ? fcs[c] : cd{0.0, 0.0};
  for (int o = 0; o < 4; ++o) {
    int own = mp.cown[c * 4 + o];
    if (own >= 0) v = v + Cbuf[own];
  }
  out[c] = v;
}

// Multipliers of the subdomain solves with edge augmentation: mu_k += nu_e for
// the edge e of multiplier k (nu = the edge part of the coarse solution u0).
template <class Src>
__global__ void k_add_edge_mult(Src src) {
  const Dev& d = src.dev();
  const Geo2& g = d.g;
  int k = src.bx() * blockDim.x + threadIdx.x;
  if (k >= g.nmu || (int)blockIdx.y >= d.nr || g.nK == g.nC) return;
  const int64_t r = blockIdx.y;
  d.mu[r * d.rs.nmu + k] = d.mu[r * d.rs.nmu + k] + d.u0[r * d.rs.nc + g.nC + d.mp.muedge[k]];
}

// primal assembly: Delta nodes average the two subdomain copies, corners take uc
template <class Src>
__global__ void k_assemble(Src src, int xsel, int conj_out) {
  const Dev& d = src.dev();
  const Geo2& g = d.g;
  const Maps2& mp = d.mp;
  const RhsStride& rs = d.rs;
  int k = src.bx() * blockDim.x + threadIdx.x;
  if ((int)blockIdx.y >= d.nr) return;
  const int64_t r = blockIdx.y;
  const cd* Ubuf = d.Ubuf;
  const cd* uc = d.u0;
  cd* x = dev_vec(d, xsel);
  Ubuf += r * rs.sb;
  uc += r * rs.nc;
  x += r * rs.nf;
  if (k < g.nmu) {
    cd v = 0.5 * (Ubuf[mp.muown[2 * k]] + Ubuf[mp.muown[2 * k + 1]]);
    x[mp.mufree[k]] = conj_out ? conj(v) : v;
  } else if (k < g.nmu + g.nC) {
    int c = k - g.nmu;
    cd v = uc[c];
    x[mp.cfree[c]] = conj_out ? conj(v) : v;
  }
}

// ------------------------------------------------------------------------------------------
// Interface phases for NRT right-hand sides at once (device functions shared by
// the persistent GMRES kernel and the stand-alone test kernels).  Vectors of RHS
// r are r-major copies: base + r * stride.  A scale of zero switches an RHS off.

// Rows of the x staging array of the interface products: nd <= 128 plus the
// zero rows [nd, nd + 16) that the pipelined product reads past the end.
constexpr int XS_ROWS = 144;

// Zero rows nd .. nd + 15 of xs (NRT values per row).
template <class R, int NRT>
__device__ inline void xs_zero_tail(C<R>* xs, int nd) {
  for (int t = threadIdx.x; t < 16 * NRT; t += blockDim.x) xs[nd * NRT + t] = C<R>{0, 0};
}

// y_r = S x_r for r < NRT with S complex symmetric, packed by rows in LDS
// (entry (i, k), k <= i, at i (i + 1) / 2 + k; nd <= 128).  Row i belongs to the
// lane pair 2i, 2i + 1 of one wave: lane parity p sums the terms k = p, p + 2, ...
// (the entry at row i for k <= i, else at row k), so every lane runs the same
// number of steps.  Steps go in groups of U, software-pipelined over two
// register buffers: the LDS loads of the next group are in flight while the
// current group's multiply-adds run.  Steps past the end read the zero rows of
// xs at an entry offset clamped to the last valid one, so they add nothing.  A
// shuffle adds the pair, and the even lane stores y_r[i] coherently to
// out + r * ostride + i.
template <class TM, class R, int NRT>
__device__ inline void symv_packed_nr(const TM* A, int nd, const C<R>* xs, cd* out, int64_t ostride,
                                      int nr) {
  constexpr int U = NRT >= 4 ? 2 : 4;
  const int i = threadIdx.x >> 1, p = threadIdx.x & 1;
  C<R> acc[NRT];
#pragma unroll
  for (int r = 0; r < NRT; ++r) acc[r] = C<R>{0, 0};
  if (i < nd) {
    const int rb = i * (i + 1) / 2;
    const int steps = (nd - p + 1) >> 1;  // k = p + 2 t for t < steps; k < nd + 4 U - 2 is read
    TM aA[U], aB[U];
    C<R> xA[U][NRT], xB[U][NRT];
    auto load = [&](int t0, TM* ar, C<R> (*x)[NRT]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = p + 2 * (t0 + u);
        const int kc = min(k, nd - 1);
        const int lo = rb + kc, hi = (int)(__umul24((unsigned)kc, (unsigned)kc + 1u) >> 1) + i;
        ar[u] = A[kc <= i ? lo : hi];
#pragma unroll
        for (int r = 0; r < NRT; ++r) x[u][r] = xs[k * NRT + r];
      }
    };
    auto madd = [&](const TM* ar, const C<R> (*x)[NRT]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const C<R> a = cvt<R>(ar[u]);
#pragma unroll
        for (int r = 0; r < NRT; ++r) fma_acc(acc[r], a, x[u][r]);
      }
    };
    load(0, aA, xA);
    for (int t0 = 0; t0 < steps; t0 += 2 * U) {
      load(t0 + U, aB, xB);
      madd(aA, xA);
      if (t0 + U >= steps) break;
      load(t0 + 2 * U, aA, xA);
      madd(aB, xB);
    }
  }
#pragma unroll
  for (int r = 0; r < NRT; ++r) {
    acc[r].x += __shfl_xor(acc[r].x, 1, 64);
    acc[r].y += __shfl_xor(acc[r].y, 1, 64);
  }
  if (p == 0 && i < nd) {
#pragma unroll
    for (int r = 0; r < NRT; ++r) {
      if (r >= nr) break;
      st_coh(out + r * ostride + i, cd{(double)acc[r].x, (double)acc[r].y});
    }
  }
  __syncthreads();
}

// Abuf_r[s] = S_bb^s x_r,  x_r[i] = 0.5 * sc[r] * sign_i * vin_r[mid_i]   (W = 1/2).
// S_bb is complex64 (packed); staged into `buf` unless `resident`.
template <class TS, int NRT>
__device__ void phase_precond(const Geo2& g, const Maps2& mp, const cf* __restrict__ Sbb, int s,
                              const cd* vin, int64_t vstride, const double* sc, cd* Abuf,
                              int64_t astride, int nr, cf* buf, bool resident,
                              cd* xs, cd* red) {
  using R = double;  // FP64 arithmetic for both storage precisions
  const int ND = g.ND, nd = mp.nd[s];
  __syncthreads();
  if (!resident) stage_lds(buf, Sbb + (size_t)s * packed_len(ND), packed_len(nd) * (int)sizeof(cf));
  // vin + r * vstride is valid memory for every r < NRT: load all, then select
  // (a switched-off RHS may hold stale values)
  for (int i = threadIdx.x; i < nd; i += blockDim.x) {
    const int mid = mp.dmid[s * ND + i];
    const double sg = 0.5 * mp.dsgn[s * ND + i];
    cd m[NRT];
#pragma unroll
    for (int r = 0; r < NRT; ++r) m[r] = ld_coh(vin + r * vstride + mid);
#pragma unroll
    for (int r = 0; r < NRT; ++r) {
      cd v = (sg * sc[r]) * m[r];
      xs[i * NRT + r] = (r < nr && sc[r] != 0.0) ? C<R>{(R)v.x, (R)v.y} : C<R>{0, 0};
    }
  }
  xs_zero_tail<R, NRT>(xs, nd);
  __syncthreads();
  symv_packed_nr<cf, R, NRT>(buf, nd, xs, Abuf + (size_t)s * ND, astride, nr);
}

// Ybuf_r[s] = Z_rr^-1|Delta x_r,  Cbuf_r[s] = Phi^T x_r.  x_r from Abuf_r (the
// preconditioned vector, from_abuf) or x_r[i] = sc[r] * sign_i * vin_r[mid_i].
template <class TS, int NRT>
__device__ void phase_f1(const Geo2& g, const Maps2& mp, const RhsStride& rs,
                         const TS* __restrict__ Sinv, const TS* __restrict__ Phi, int s,
                         bool from_abuf, const cd* Abuf, const cd* vin, const double* sc, cd* Ybuf,
                         cd* Cbuf, int nr, TS* buf, bool resident,
                         cd* xs, cd* red) {
  using R = double;  // FP64 arithmetic for both storage precisions
  const int ND = g.ND, nd = mp.nd[s];
  __syncthreads();
  if (!resident) stage_lds(buf, Sinv + (size_t)s * packed_len(ND), packed_len(nd) * (int)sizeof(TS));
  for (int i = threadIdx.x; i < nd; i += blockDim.x) {
    const int part = mp.dpart[s * ND + i], mid = mp.dmid[s * ND + i];
    const double sg = mp.dsgn[s * ND + i];
    cd m[NRT];
    if (from_abuf) {
      cd u[NRT], v[NRT];
#pragma unroll
      for (int r = 0; r < NRT; ++r) {
        u[r] = ld_coh(Abuf + r * rs.sb + (size_t)s * ND + i);
        v[r] = ld_coh(Abuf + r * rs.sb + part);
      }
#pragma unroll
      for (int r = 0; r < NRT; ++r) m[r] = 0.5 * (u[r] - v[r]);
    } else {
#pragma unroll
      for (int r = 0; r < NRT; ++r) m[r] = ld_coh(vin + r * rs.nmu + mid);
#pragma unroll
      for (int r = 0; r < NRT; ++r) m[r] = (sg * sc[r]) * m[r];
    }
#pragma unroll
    for (int r = 0; r < NRT; ++r)
      xs[i * NRT + r] = (r < nr && sc[r] != 0.0) ? C<R>{(R)m[r].x, (R)m[r].y} : C<R>{0, 0};
  }
  xs_zero_tail<R, NRT>(xs, nd);
  __syncthreads();
  // coarse-slot products: wave w takes slots w (a corner) and w + 4 (an edge);
  // lane l takes rows l and l + 64 (nd <= 128), whose coarse-basis entries
  // load under the Schur product
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  bool has[2];
  TS phr[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int q = wv + 4 * u, c = mp.cgid[s * NQ + q];
    has[u] = c >= 0 && c < g.nK;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = lane + 64 * h;
      phr[u][h] = (has[u] && i < nd) ? Phi[((size_t)s * ND + i) * NQ + q] : TS{0, 0};
    }
  }
  symv_packed_nr<TS, R, NRT>(buf, nd, xs, Ybuf + (size_t)s * ND, rs.sb, nr);
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    if (!has[u]) continue;  // uniform over the wave
    cd acc[NRT];
#pragma unroll
    for (int r = 0; r < NRT; ++r) acc[r] = cd{0.0, 0.0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = lane + 64 * h;
      if (i >= nd) break;
      const cd ph = cvt<double>(phr[u][h]);
#pragma unroll
      for (int r = 0; r < NRT; ++r) {
        C<R> x = xs[i * NRT + r];
        fma_acc(acc[r], ph, cd{(double)x.x, (double)x.y});
      }
    }
#pragma unroll
    for (int r = 0; r < NRT; ++r) {
      for (int off = 32; off > 0; off >>= 1) {
        acc[r].x += __shfl_down(acc[r].x, off, 64);
        acc[r].y += __shfl_down(acc[r].y, off, 64);
      }
      if (lane == 0 && r < nr) st_coh(Cbuf + r * rs.cq + s * NQ + wv + 4 * u, acc[r]);
    }
  }
}

// g_r[c] = sum of Cbuf_r over the owners of coarse unknown c, for the coarse
// unknowns c = b, b + nb, ... of block b of nb (each assembled once; a grid
// barrier separates this from phase_f2, which reads all of them).
template <int NRT>
__device__ void phase_gco(const Maps2& mp, const RhsStride& rs, int nK, const cd* Cbuf, cd* gco, int nr, int b,
                          int nb) {
  for (int c = b + nb * (int)threadIdx.x; c < nK; c += nb * (int)blockDim.x) {
    const int4 own = *(const int4*)(mp.cown + 4 * c);
    const int ow[4] = {own.x, own.y, own.z, own.w};
#pragma unroll
    for (int r = 0; r < NRT; ++r) {
      if (r >= nr) break;
      cd t[4];
#pragma unroll
      for (int o = 0; o < 4; ++o) t[o] = ld_coh(Cbuf + r * rs.cq + max(ow[o], 0));
      cd v{0.0, 0.0};
#pragma unroll
      for (int o = 0; o < 4; ++o) v = v + (ow[o] >= 0 ? t[o] : cd{0.0, 0.0});
      st_coh(gco + r * rs.nc + c, v);
    }
  }
}

// Ybuf_r[s] += Phi uc_r over the subdomain's coarse slots, uc_r = Kinv g_r on
// those slots, g_r the assembled coarse vector (phase_gco).  Transposed
// product: thread t loads g_r[c] for c = t, t + 256, ... and accumulates
// Kinv[c_q][c] g_r[c] for four slots q at a time (corner slots, then, with an
// edge-augmented coarse space, edge slots); one block reduction per pass gives
// uc_r[q].  wred holds 16 * NRT complex values, ucs NQ * NRT.
template <class TS, int NRT>
__device__ void phase_f2(const Geo2& g, const Maps2& mp, const RhsStride& rs,
                         const TS* __restrict__ Phi, const cd* __restrict__ Kinv, int s,
                         const cd* gco, cd* Ybuf, int nr, cd* ucs, cd* wred) {
  const int ND = g.ND, nd = mp.nd[s], nK = g.nK;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  int cq[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int c = mp.cgid[s * NQ + q];
    cq[q] = (c >= 0 && c < nK) ? c : -1;
  }
  // thread i < nd (nd <= ND <= 128 < blockDim) updates Delta row i at the end: its
  // coarse-basis row and the F1 result are loaded now, under the coarse product
  const int i = threadIdx.x;
  cd ph[NQ], yv[NRT];
#pragma unroll
  for (int qq = 0; qq < NQ; ++qq)
    ph[qq] = (i < nd && cq[qq] >= 0) ? cvt<double>(Phi[((size_t)s * ND + i) * NQ + qq]) : cd{0.0, 0.0};
#pragma unroll
  for (int r = 0; r < NRT; ++r)
    yv[r] = (i < nd && r < nr) ? ld_coh(Ybuf + r * rs.sb + (size_t)s * ND + i) : cd{0.0, 0.0};
  // one sweep over the coarse unknowns for all slots: g_r[c] is gathered once
  cd acc[NQ][NRT];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int r = 0; r < NRT; ++r) acc[q][r] = cd{0.0, 0.0};
  const bool edges = nK > g.nC;
  for (int c = threadIdx.x; c < nK; c += blockDim.x) {
    cd gc[NRT];
#pragma unroll
    for (int r = 0; r < NRT; ++r) gc[r] = r < nr ? ld_coh(gco + r * rs.nc + c) : cd{0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int cqq = cq[q];
      if (cqq < 0) continue;
      const cd kv = Kinv[(size_t)cqq * nK + c];
#pragma unroll
      for (int r = 0; r < NRT; ++r) fma_acc(acc[q][r], kv, gc[r]);
    }
  }
  // block sums of the slot values, four slots at a time (the corner slots, then
  // the edge slots when the coarse space has them)
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1 && !edges) break;  // uniform
    {
      // reduce-scatter over the wave: at each halving step a lane keeps half of its
      // values and adds its partner's copy of them, so V = 4 NRT sums take
      // V - 1 + log2(64 / V) shuffles instead of 6 V; lane bits 5.. then name
      // the value a lane holds (value index = (q, r) in row-major order)
      constexpr int V = 4 * NRT;
      cd v[V];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < NRT; ++r) v[q * NRT + r] = acc[4 * pass + q][r];
      int idx = 0, off = 32;
#pragma unroll
      for (int cnt = V; cnt > 1; cnt >>= 1, off >>= 1) {
        const int half = cnt >> 1;
        const bool up = (lane & off) != 0;
#pragma unroll
        for (int k = 0; k < half; ++k) {
          const cd send = up ? v[k] : v[half + k];
          const cd keep = up ? v[half + k] : v[k];
          cd recv;
          recv.x = __shfl_xor(send.x, off, 64);
          recv.y = __shfl_xor(send.y, off, 64);
          v[k] = keep + recv;
        }
        if (up) idx += half;
      }
      for (; off > 0; off >>= 1) {
        v[0].x += __shfl_xor(v[0].x, off, 64);
        v[0].y += __shfl_xor(v[0].y, off, 64);
      }
      if ((lane & (64 / V - 1)) == 0) wred[wv * V + idx] = v[0];
    }
    __syncthreads();
    if (threadIdx.x < 4 * NRT) {
      const int q = threadIdx.x / NRT, r = threadIdx.x % NRT;
      ucs[(4 * pass + q) * NRT + r] = (wred[q * NRT + r] + wred[(4 + q) * NRT + r]) +
                                      (wred[(8 + q) * NRT + r] + wred[(12 + q) * NRT + r]);
    }
    __syncthreads();
  }
  if (i < nd) {
#pragma unroll
    for (int r = 0; r < NRT; ++r) {
      if (r >= nr) break;
      cd y = yv[r];
#pragma unroll
      for (int qq = 0; qq < NQ; ++qq)
        if (cq[qq] >= 0) fma_acc(y, ph[qq], ucs[qq * NRT + r]);
      st_coh(Ybuf + r * rs.sb + (size_t)s * ND + i, y);
    }
  }
}

// ------------------------------------------------------------------------------------------
// Persistent GMRES on F_DP P^-1 t_r = d_r for nr <= NRT right-hand sides in lockstep.
// Each RHS has its own Krylov basis, Hessenberg matrix, Givens rotations and
// stopping test; a converged RHS is switched off (scale 0) while the others go on.
struct GmresArgs {
  RhsStride rs;
  const cd* d;      // [r][nmu]
  cd* mu;           // [r][nmu]
  cd* Abuf;         // [r][nsub*ND]
  cd* Ybuf;         // [r][nsub*ND]
  cd* Cbuf;         // [r][nsub*4]
  cd* gco;          // [r][nK] assembled coarse vector of the current iteration
  cd* w;            // [r][nmu]
  cd* Q;            // [r][kmax_alloc+1][nmu]
  cd* H;            // [r][kmax_alloc+1][kmax_alloc], column j at H[i*kstride + j]
  cd* part;         // [3][NRMAX][kmax+2][nb]
  unsigned* bar;
  int* flags;       // instance flag words (FLAG_*)
  double* scal;     // [r] final relative residual estimate
  double tol;
  int kmax;         // iteration limit of this launch
  int kstride;      // kmax_alloc (strides of Q and H)
  int chunk;
  int nr;
  int r0;           // first right-hand side of the group served by this launch
  unsigned map;     // group slot of right-hand side c in byte c (iteration log)
  int resident;     // Schur blocks kept in LDS (requires one subdomain per block)
  // byte offsets into dynamic LDS (gmres_layout)
  int o_red, o_xs, o_wch, o_hv, o_h2, o_cs, o_sn, o_g, o_ucs, o_S, o_I;
};

// Launch-wide GMRES parameters (the same for every instance of a launch).
struct GmresLaunch {
  double tol;
  int kmax, r0, resident;
  int check_spins;  // plain launch: the co-residency check's wait (grid_coresident); -1 cooperative
  int o_red, o_xs, o_wch, o_hv, o_h2, o_cs, o_sn, o_g, o_ucs, o_S, o_I;
};

static inline size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

// Dynamic LDS of k_gmres: the work arrays, then the Schur-block buffers (both
// resident, or one staging buffer shared by the two).  Returns the total size.
static size_t gmres_layout(int nrt, int kmax, int chunk, size_t tsz, size_t bytesS, size_t bytesI,
                           bool resident, GmresLaunch* a) {
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o += align16(bytes); return (int)at; };
  int red = take(sizeof(cd) * 16 * nrt), xs = take(tsz * XS_ROWS * nrt);
  int wch = take(sizeof(cd) * nrt * chunk);
  int hv = take(sizeof(cd) * nrt * (kmax + 1)), h2 = take(sizeof(cd) * nrt * (kmax + 1));
  int cs = take(sizeof(cd) * nrt * (kmax + 1)), sn = take(sizeof(double) * nrt * (kmax + 1));
  int g = take(sizeof(cd) * nrt * (kmax + 1)), ucs = take(sizeof(cd) * NQ * nrt);
  int S = take(resident ? bytesS : std::max(bytesS, bytesI));
  int I = resident ? take(bytesI) : S;
  if (a) {
    a->o_red = red; a->o_xs = xs; a->o_wch = wch; a->o_hv = hv; a->o_h2 = h2; a->o_cs = cs;
    a->o_sn = sn; a->o_g = g; a->o_ucs = ucs; a->o_S = S; a->o_I = I;
  }
  return o;
}

template <class TS, int NRT>
__device__ inline void gmres_body(const Geo2& g, const Maps2& mp, const cf* __restrict__ Sbb,
                                  const TS* __restrict__ Sinv, const TS* __restrict__ Phi,
                                  const cd* __restrict__ Kinv, const GmresArgs& a, const int b,
                                  const unsigned nb) {
  using R = double;  // FP64 arithmetic for both storage precisions
  using T = cd;
  extern __shared__ __align__(16) char smem[];
  const int kmax = a.kmax, nr = a.nr;
  T* red = (T*)(smem + a.o_red);
  T* xs = (T*)(smem + a.o_xs);
  cd* wch = (cd*)(smem + a.o_wch);
  cd* hv = (cd*)(smem + a.o_hv);
  cd* h2 = (cd*)(smem + a.o_h2);
  cd* csv = (cd*)(smem + a.o_cs);
  double* snv = (double*)(smem + a.o_sn);
  cd* gv = (cd*)(smem + a.o_g);
  cd* ucs = (cd*)(smem + a.o_ucs);
  cf* bufS = (cf*)(smem + a.o_S);   // S_bb (resident) or staging
  TS* bufI = (TS*)(smem + a.o_I);   // Z_rr^-1|Delta (resident) or the same staging buffer
  cd* wred = (cd*)red;              // coarse-phase reduction scratch (16 * NRT values)
  __shared__ double sc[NRT], beta0[NRT], hnrm[NRT], resid[NRT], nsum[NRT], wsum[4];
  __shared__ cd nrm2[NRT];
  __shared__ int active[NRT], its[NRT], ract[NRT], nact_sh;

  unsigned epoch = 0;
  const int nmu = g.nmu;
  const RhsStride rs = a.rs;
  const int k0 = min(nmu, b * a.chunk), k1 = min(nmu, k0 + a.chunk), kn = k1 - k0;
  // vector phases: RHS rt = threadIdx / TPR is served by TPR threads (whole waves)
  constexpr int TPR = 256 / NRT;
  const int rt = threadIdx.x / TPR, lt = threadIdx.x % TPR;
  const int64_t pstride = (int64_t)(kmax + 2) * nb;  // per-RHS block of partial sums
  cd* part0 = a.part;
  cd* part1 = a.part + (size_t)NRMAX * pstride;
  cd* part2 = a.part + (size_t)2 * NRMAX * pstride;
  const int64_t qs = (int64_t)(a.kstride + 1) * nmu;   // Krylov basis stride per RHS
  const int64_t hs = (int64_t)(a.kstride + 1) * a.kstride;
  const int hst = kmax + 1;                            // LDS stride of the per-RHS arrays

  if (a.resident) {
    // one subdomain per block: both Schur blocks stay in LDS for the whole solve
    const int s = b, nd = mp.nd[s];
    stage_lds(bufS, Sbb + (size_t)s * packed_len(g.ND), packed_len(nd) * (int)sizeof(cf));
    stage_lds(bufI, Sinv + (size_t)s * packed_len(g.ND), packed_len(nd) * (int)sizeof(TS));
  }
  // the list of right-hand sides still iterating (identical in every block)
  auto refresh_active = [&]() {
    if (threadIdx.x == 0) {
      int n = 0;
      for (int r = 0; r < nr; ++r)
        if (active[r]) ract[n++] = r;
      nact_sh = n;
    }
    __syncthreads();
  };

  // ---- init: beta0_r = ||d_r||
  {
    double loc = 0.0;
    if (rt < nr)
      for (int k = k0 + lt; k < k1; k += TPR) loc += abs2(a.d[rt * rs.nmu + k]);
    rhs_block_sums<NRT>(loc, wsum, nsum);
    if (threadIdx.x < nr) st_coh(part2 + threadIdx.x * pstride + b, cd{nsum[threadIdx.x], 0.0});
  }
  if (threadIdx.x < NRT) ract[threadIdx.x] = threadIdx.x;
  __syncthreads();
  grid_barrier(a.bar, nb, b, epoch, a.flags + 1);
  reduce_partials(part2, pstride, nb, 1, nr, ract, nrm2, 1);
  if (threadIdx.x < NRT) {
    const int r = threadIdx.x;
    double b0 = r < nr ? sqrt(nrm2[r].x) : 0.0;
    beta0[r] = b0;
    active[r] = b0 > 0.0;
    its[r] = 0;
    sc[r] = b0 > 0.0 ? 1.0 / b0 : 0.0;
    gv[r * hst] = cd{b0, 0.0};
    resid[r] = b0 > 0.0 ? 1.0 : 0.0;
  }
  __syncthreads();
  refresh_active();
  const cd* vin = a.d;
  int j = 0;
  for (j = 0; j < kmax && nact_sh > 0; ++j) {
    const int na = nact_sh;
    const bool mine = rt < nr && active[rt];
    // ---- P: Abuf = S_bb (W B^T q_j) for the active RHS; store q_j = sc * vin
    if (mine)
      for (int k = k0 + lt; k < k1; k += TPR)
        a.Q[rt * qs + (size_t)j * nmu + k] = sc[rt] * ld_coh(vin + rt * rs.nmu + k);
    for (int s = b; s < g.nsub; s += nb)
      phase_precond<TS, NRT>(g, mp, Sbb, s, vin, rs.nmu, sc, a.Abuf, rs.sb, nr, bufS, a.resident,
                             xs, red);
    grid_barrier(a.bar, nb, b, epoch, a.flags + 1);
    // ---- F1
    for (int s = b; s < g.nsub; s += nb)
      phase_f1<TS, NRT>(g, mp, rs, Sinv, Phi, s, true, a.Abuf, nullptr, sc, a.Ybuf, a.Cbuf, nr, bufI,
                        a.resident, xs, red);
    grid_barrier(a.bar, nb, b, epoch, a.flags + 1);
    // ---- F2 (coarse correction): assemble the coarse vector once, then every
    // block applies the coarse inverse on its slots
    phase_gco<NRT>(mp, rs, g.nK, a.Cbuf, a.gco, nr, b, nb);
    grid_barrier(a.bar, nb, b, epoch, a.flags + 1);
    for (int s = b; s < g.nsub; s += nb)
      phase_f2<TS, NRT>(g, mp, rs, Phi, Kinv, s, a.gco, a.Ybuf, nr, ucs, wred);
    grid_barrier(a.bar, nb, b, epoch, a.flags + 1);
    // ---- O1: w_r = B_r Y_r (combine), first Gram-Schmidt projections
    if (mine)
      for (int k = lt; k < kn; k += TPR) {
        const int kk = k0 + k;
        wch[rt * a.chunk + k] = ld_coh(a.Ybuf + rt * rs.sb + mp.muown[2 * kk]) -
                                ld_coh(a.Ybuf + rt * rs.sb + mp.muown[2 * kk + 1]);
      }
    __syncthreads();
    block_dots(a.Q, qs, nmu, k0, kn, j + 1, na, ract, wch, a.chunk, part0, pstride, nb, b);
    grid_barrier(a.bar, nb, b, epoch, a.flags + 1);
    // ---- O2: h = sum of partials; w -= Q h; second projections
    reduce_partials(part0, pstride, nb, j + 1, na, ract, hv, hst);
    if (mine) {
      const cd* Qr = a.Q + rt * qs;
      const cd* hr = hv + rt * hst;
      for (int k = lt; k < kn; k += TPR) {
        cd v = wch[rt * a.chunk + k];
#pragma unroll 8
        for (int i = 0; i <= j; ++i) v = v - hr[i] * Qr[(size_t)i * nmu + k0 + k];
        wch[rt * a.chunk + k] = v;
      }
    }
    __syncthreads();
    block_dots(a.Q, qs, nmu, k0, kn, j + 1, na, ract, wch, a.chunk, part1, pstride, nb, b);
    grid_barrier(a.bar, nb, b, epoch, a.flags + 1);
    // ---- O3: second correction, norm
    reduce_partials(part1, pstride, nb, j + 1, na, ract, h2, hst);
    {
      double loc = 0.0;
      if (mine) {
        const cd* Qr = a.Q + rt * qs;
        const cd* h2r = h2 + rt * hst;
        for (int k = lt; k < kn; k += TPR) {
          cd v = wch[rt * a.chunk + k];
#pragma unroll 8
          for (int i = 0; i <= j; ++i) v = v - h2r[i] * Qr[(size_t)i * nmu + k0 + k];
          st_coh(a.w + rt * rs.nmu + k0 + k, v);
          loc += abs2(v);
        }
        for (int i = lt; i <= j; i += TPR) hv[rt * hst + i] = hv[rt * hst + i] + h2[rt * hst + i];
      }
      rhs_block_sums<NRT>(loc, wsum, nsum);
      if (threadIdx.x < nr && active[threadIdx.x])
        st_coh(part2 + threadIdx.x * pstride + b, cd{nsum[threadIdx.x], 0.0});
    }
    grid_barrier(a.bar, nb, b, epoch, a.flags + 1);
    // ---- Arnoldi column j complete: norms, Givens rotations (identical in every block)
    reduce_partials(part2, pstride, nb, 1, na, ract, nrm2, 1);
    if (threadIdx.x < nr && active[threadIdx.x]) {
      const int r = threadIdx.x;
      cd* hr = hv + r * hst;
      cd* cr = csv + r * hst;
      double* sr = snv + r * hst;
      cd* gr = gv + r * hst;
      const double hn = sqrt(nrm2[r].x);
      hnrm[r] = hn;
      // rotation [c s; -s conj(c)] with real s maps (h_j, hn) to (den, 0)
      for (int i = 0; i < j; ++i) {
        cd c = cr[i];
        double sn = sr[i];
        cd t0 = c * hr[i] + sn * hr[i + 1];
        cd t1 = conj(c) * hr[i + 1] - sn * hr[i];
        hr[i] = t0;
        hr[i + 1] = t1;
      }
      cd hj = hr[j];
      double den = sqrt(abs2(hj) + hn * hn);
      cd c;
      double sn;
      if (den == 0.0) { c = cd{1.0, 0.0}; sn = 0.0; }
      else { c = (1.0 / den) * conj(hj); sn = hn / den; }
      cr[j] = c;
      sr[j] = sn;
      hr[j] = c * hj + cd{sn * hn, 0.0};
      cd gj = gr[j];
      gr[j + 1] = -(sn * gj);
      gr[j] = c * gj;
      double res = sqrt(abs2(gr[j + 1])) / beta0[r];
      resid[r] = res;
      its[r] = j + 1;
      if (res <= a.tol || hn == 0.0 || j + 1 == kmax) active[r] = 0;
    }
    __syncthreads();
    if (b == 0 && rt < nr && its[rt] == j + 1)
      for (int i = lt; i <= j; i += TPR) st_coh(a.H + rt * hs + (size_t)i * a.kstride + j, hv[rt * hst + i]);
    if (threadIdx.x < NRT) {
      const int r = threadIdx.x;
      sc[r] = (r < nr && active[r]) ? 1.0 / hnrm[r] : 0.0;
    }
    __syncthreads();
    refresh_active();
    vin = a.w;
  }
  // ---- back substitution H_r y_r = g_r for all RHS together (redundant in every
  // block; H from block 0), then t_r = Q_r y_r on the chunk
  grid_barrier(a.bar, nb, b, epoch, a.flags + 1);
  int kmx = 0;
  for (int r = 0; r < nr; ++r) kmx = max(kmx, its[r]);
  if (rt < nr)
    for (int i = lt; i < its[rt]; i += TPR) h2[rt * hst + i] = gv[rt * hst + i];
  __syncthreads();
  for (int i = kmx - 1; i >= 0; --i) {
    if (threadIdx.x < nr && i < its[threadIdx.x]) {
      const int r = threadIdx.x;
      h2[r * hst + i] = cdiv(h2[r * hst + i], ld_coh(a.H + r * hs + (size_t)i * a.kstride + i));
    }
    __syncthreads();
    if (rt < nr && i < its[rt]) {
      const cd yi = h2[rt * hst + i];
      for (int t = lt; t < i; t += TPR)
        h2[rt * hst + t] = h2[rt * hst + t] - ld_coh(a.H + rt * hs + (size_t)t * a.kstride + i) * yi;
    }
    __syncthreads();
  }
  if (rt < nr) {
    const cd* Qr = a.Q + rt * qs;
    const cd* yr = h2 + rt * hst;
    const int kk = its[rt];
    for (int k = lt; k < kn; k += TPR) {
      cd v{0.0, 0.0};
#pragma unroll 8
      for (int i = 0; i < kk; ++i) fma_acc(v, Qr[(size_t)i * nmu + k0 + k], yr[i]);
      st_coh(a.w + rt * rs.nmu + k0 + k, v);
    }
  }
  if (threadIdx.x < NRT) sc[threadIdx.x] = (threadIdx.x < nr && its[threadIdx.x] > 0) ? 1.0 : 0.0;
  grid_barrier(a.bar, nb, b, epoch, a.flags + 1);
  // mu_r = P^-1 t_r
  for (int s = b; s < g.nsub; s += nb)
    phase_precond<TS, NRT>(g, mp, Sbb, s, a.w, rs.nmu, sc, a.Abuf, rs.sb, nr, bufS, a.resident, xs,
                           red);
  grid_barrier(a.bar, nb, b, epoch, a.flags + 1);
  if (rt < nr)
    for (int k = k0 + lt; k < k1; k += TPR)
      a.mu[rt * rs.nmu + k] = its[rt] > 0 ? 0.5 * (ld_coh(a.Abuf + rt * rs.sb + mp.muown[2 * k]) -
                                                   ld_coh(a.Abuf + rt * rs.sb + mp.muown[2 * k + 1]))
                                          : cd{0.0, 0.0};
  if (b == 0 && threadIdx.x == 0) {
    int tot = 0;
    for (int r = 0; r < nr; ++r) {
      a.flags[FLAG_ITS + a.r0 + r] = its[r];
      // append to the log of the right-hand side's group slot
      const int slot = (int)((a.map >> (8 * (a.r0 + r))) & 255u);
      const int k = a.flags[FLAG_CNT + slot];
      if (k < 16) a.flags[FLAG_LOG + 16 * slot + k] = its[r];
      a.flags[FLAG_CNT + slot] = k + 1;
      a.scal[r] = resid[r];
      tot += its[r];
    }
    a.flags[3] += j;    // loop trips of this launch (the largest count of the group)
    a.flags[4] += tot;  // iterations summed over its right-hand sides
  }
}

// One cooperative launch, or for a single instance a plain launch that first
// checks that its grid is co-resident (and returns at once if not); every
// instance's blocks (its share gb0 .. gb0+gnb-1 of the grid) run the Krylov
// solve of its group's right-hand sides r0 .. r0 + NRT - 1 with their own grid
// barrier.  Instances with no such right-hand side return at once.
template <class TS, int NRT, class Src>
__global__ void __launch_bounds__(256) k_gmres(Src src, GmresLaunch L) {
  const Dev& d = src.dev();
  const int nr = min(NRT, d.nr - L.r0);
  if (nr <= 0) return;
  // plain launch (single problems only, so the batch form carries none of this code
  // and keeps its register count): nothing to do once a grid of this step was found
  // not co-resident (the step runs again), else the check
  if constexpr (std::is_same<Src, One>::value) {
    extern __shared__ __align__(16) char smem[];
    if (L.check_spins >= 0 &&
        (d.flags[FLAG_NOTRES] || !grid_coresident(d.bar + BAR_ARRIVE, (unsigned)d.gnb, L.check_spins,
                                                  d.flags + FLAG_NOTRES, *(int*)smem)))
      return;
  }
  const RhsStride rs = d.rs;
  GmresArgs a;
  a.rs = rs;
  a.d = d.dvec + L.r0 * rs.nmu;
  a.mu = d.mu + L.r0 * rs.nmu;
  a.Abuf = d.Abuf + L.r0 * rs.sb;
  a.Ybuf = d.Ybuf + L.r0 * rs.sb;
  a.Cbuf = d.Cbuf + L.r0 * rs.cq;
  a.gco = d.ymin + L.r0 * rs.nc;  // ymin is free until the recovery
  a.w = d.wv + L.r0 * rs.nmu;
  a.Q = d.Qk;
  a.H = d.Hk;
  a.part = d.part;
  a.bar = d.bar;
  a.flags = d.flags;
  a.scal = d.dscal + L.r0;
  a.tol = L.tol;
  a.kmax = L.kmax;
  a.kstride = d.kstride;
  a.chunk = d.chunk;
  a.nr = nr;
  a.r0 = L.r0;
  a.map = d.map;
  a.resident = L.resident && d.resident;
  a.o_red = L.o_red; a.o_xs = L.o_xs; a.o_wch = L.o_wch; a.o_hv = L.o_hv; a.o_h2 = L.o_h2;
  a.o_cs = L.o_cs; a.o_sn = L.o_sn; a.o_g = L.o_g; a.o_ucs = L.o_ucs; a.o_S = L.o_S; a.o_I = L.o_I;
  gmres_body<TS, NRT>(d.g, d.mp, d.Sbb, (const TS*)d.Sinv, (const TS*)d.Phi, d.Kinv, a, src.bx(),
                      (unsigned)d.gnb);
}

// Zero every instance's grid-barrier words before a GMRES launch.
template <class Src>
__global__ void k_bar_reset(Src src) {
  const Dev& d = src.dev();
  for (int i = threadIdx.x; i < BAR_WORDS; i += blockDim.x) d.bar[i] = 0u;
}

// Stand-alone interface kernels for testing (one block per subdomain, one RHS).
template <class TS>
__global__ void __launch_bounds__(256) k_iface_precond(Geo2 g, Maps2 mp, const cf* Sbb, const cd* x,
                                                       cd* Abuf) {
  using R = double;  // FP64 arithmetic for both storage precisions
  extern __shared__ __align__(16) char smem[];
  __shared__ C<R> red[128], xs[XS_ROWS];
  __shared__ double sc[1];
  if (threadIdx.x == 0) sc[0] = 1.0;
  phase_precond<TS, 1>(g, mp, Sbb, blockIdx.x, x, 0, sc, Abuf, 0, 1, (cf*)smem, false, xs, red);
}
template <class TS>
__global__ void __launch_bounds__(256) k_iface_f1(Geo2 g, Maps2 mp, RhsStride rs, const TS* Sinv,
                                                  const TS* Phi, const cd* x, cd* Ybuf, cd* Cbuf) {
  using R = double;  // FP64 arithmetic for both storage precisions
  extern __shared__ __align__(16) char smem[];
  __shared__ C<R> red[128], xs[XS_ROWS];
  __shared__ double sc[1];
  if (threadIdx.x == 0) sc[0] = 1.0;
  phase_f1<TS, 1>(g, mp, rs, Sinv, Phi, blockIdx.x, false, nullptr, x, sc, Ybuf, Cbuf, 1, (TS*)smem,
                  false, xs, red);
}
__global__ void __launch_bounds__(256) k_iface_gco(Geo2 g, Maps2 mp, RhsStride rs, const cd* Cbuf, cd* gco) {
  phase_gco<1>(mp, rs, g.nK, Cbuf, gco, 1, blockIdx.x, gridDim.x);
}
template <class TS>
__global__ void __launch_bounds__(256) k_iface_f2(Geo2 g, Maps2 mp, RhsStride rs, const TS* Phi,
                                                  const cd* Kinv, const cd* gco, cd* Ybuf) {
  __shared__ cd ucs[NQ], wred[16];
  phase_f2<TS, 1>(g, mp, rs, Phi, Kinv, blockIdx.x, gco, Ybuf, 1, ucs, wred);
}
__global__ void k_combine(Geo2 g, Maps2 mp, const cd* buf, double scale, cd* out) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.nmu) return;
  out[k] = scale * (buf[mp.muown[2 * k]] - buf[mp.muown[2 * k + 1]]);
}

// ------------------------------------------------------------------------------------------
// launchers (nr right-hand sides, r-major buffers of the problem)

static int max_nr(const Target& t) {
  if (t.single()) return t.one->nr;
  int n = 0;
  for (const Problem* p : t.probs) n = std::max(n, p->nr);
  return n;
}

template <class TS, int NRT>
static void local_solve_t(const Target& t, int mode, int f, int conj_in, int x) {
  launch2(t, K_SUB, k_local_solve<TS, NRT, One>, k_local_solve<TS, NRT, Many>, 1, 256, 0, mode, f,
          conj_in, x);
}

// Candidates: one workgroup per subdomain for all right-hand sides (0), one
// workgroup of 256 per subdomain and right-hand side (1: more workgroups per CU,
// the line factors re-read from L2), one wavefront per subdomain and right-hand
// side (2: no workgroup barriers in the line recursion), one workgroup of four
// wavefronts per subdomain, a wavefront per right-hand side, the line factors
// staged once into LDS for all of them (3).  The autotuner picks; without it
// the wavefront form runs.
template <class TS>
static void local_solve_w(const Target& t, int mode, int f, int conj_in, int x, int nr) {
  auto run = [&](int c) {
    if (c == 3) {
      const size_t lds = ls_group_bytes();
      bool all33 = t.single() ? t.one->ml == ML : true;
      if (!t.single())
        for (const Problem* p : t.probs) all33 = all33 && p->ml == ML;
      if (all33) {
        (void)ensure_lds((const void*)k_local_solve_group<TS, ML, One>, lds);
        (void)ensure_lds((const void*)k_local_solve_group<TS, ML, Many>, lds);
        launch2(t, K_SUB, k_local_solve_group<TS, ML, One>, k_local_solve_group<TS, ML, Many>, 1, 256, lds, mode,
                f, conj_in, x);
      } else {
        (void)ensure_lds((const void*)k_local_solve_group<TS, 0, One>, lds);
        (void)ensure_lds((const void*)k_local_solve_group<TS, 0, Many>, lds);
        launch2(t, K_SUB, k_local_solve_group<TS, 0, One>, k_local_solve_group<TS, 0, Many>, 1, 256, lds, mode, f,
                conj_in, x);
      }
    } else if (c == 2)
      launch2(t, K_SUB, k_local_solve_wave<TS, One>, k_local_solve_wave<TS, Many>, nr, 64, 0, mode, f, conj_in, x);
    else if (c == 1)
      launch2(t, K_SUB, k_local_solve_rhs<TS, One>, k_local_solve_rhs<TS, Many>, nr, 256, 0, mode, f, conj_in, x);
    else if (nr == 1)
      local_solve_t<TS, 1>(t, mode, f, conj_in, x);
    else if (nr == 2)
      local_solve_t<TS, 2>(t, mode, f, conj_in, x);
    else
      local_solve_t<TS, NRMAX>(t, mode, f, conj_in, x);
  };
  int dev = 0, ml = 0;
  (void)hipGetDevice(&dev);
  if (t.single()) ml = t.one->ml;
  else
    for (const Problem* p : t.probs) ml = std::max(ml, p->ml);
  const TuneKey key{TUNE_LOCAL_SOLVE, dev, ml, t.blocks(K_SUB), (int)sizeof(TS), nr};
  // the workgroup per right-hand side reads the line factors once per
  // right-hand side (2.3 x the bytes of the other forms at 512^2, measured):
  // it has to be 3% faster to be chosen
  static const float weight[4] = {1.f, 1.03f, 1.f, 1.f};
  run(tune_choice(key, 4, 2, t.st, run, weight));
}

hipError_t launch_local_solve(const Target& t, int mode, int f, int conj_in, int x) {
  const int nr = max_nr(t);
  if (nr < 1 || nr > NRMAX) return hipErrorInvalidValue;
  if (t.g32()) local_solve_w<cf>(t, mode, f, conj_in, x, nr);
  else local_solve_w<cd>(t, mode, f, conj_in, x, nr);
  return hipGetLastError();
}

hipError_t launch_coarse_rhs(const Target& t, int f, int conj_in) {
  launch2(t, K_SUB, k_edge_rhs<One>, k_edge_rhs<Many>, NRMAX, 256, 0);
  launch2(t, K_NC128, k_coarse_rhs<One>, k_coarse_rhs<Many>, NRMAX, 128, 0, f, conj_in);
  launch2(t, K_NC, k_dense_mv<One>, k_dense_mv<Many>, 1, 64, 0, (int)V_FCS);
  return hipGetLastError();
}

hipError_t launch_fetidp_rhs(const Target& t) {
  if (t.s32()) launch2(t, K_NMU256, k_fetidp_rhs<cf, One>, k_fetidp_rhs<cf, Many>, NRMAX, 256, 0);
  else launch2(t, K_NMU256, k_fetidp_rhs<cd, One>, k_fetidp_rhs<cd, Many>, NRMAX, 256, 0);
  return hipGetLastError();
}

// Bytes of one subdomain's packed S_bb (complex64) and Z_rr^-1|Delta blocks.
static void block_bytes(const Problem& p, size_t* bS, size_t* bI) {
  size_t pk = (size_t)packed_len(p.ndmax);
  *bS = pk * sizeof(cf);
  *bI = pk * (p.s32() ? sizeof(cf) : sizeof(cd));
}

// The instances of one GMRES launch: the single problem, or batch group gi.
static void gmres_members(const Target& t, int gi, std::vector<const Problem*>& out) {
  out.clear();
  if (t.single()) out.push_back(t.one);
  else
    for (int i : t.ggroups[gi].members) out.push_back(t.probs[i]);
}

// LDS bytes of k_gmres<TS, NRT> over the given instances, and whether the
// Schur blocks stay resident (complex64 interface operators, one subdomain per
// block for every instance, and room for both blocks).
template <class TS, int NRT>
static size_t gmres_plan(const std::vector<const Problem*>& ms, int kmax, bool* resident,
                         GmresLaunch* L) {
  size_t bS = 0, bI = 0;
  int chunk = 1;
  bool all_one = true;
  for (const Problem* p : ms) {
    size_t s1, s2;
    block_bytes(*p, &s1, &s2);
    bS = std::max(bS, s1);
    bI = std::max(bI, s2);
    chunk = std::max(chunk, (p->nmu + p->gmres_blocks - 1) / std::max(p->gmres_blocks, 1));
    all_one = all_one && p->gmres_blocks == p->nsub;
  }
  const Problem* p0 = ms[0];
  bool res = p0->s32() && all_one &&
             gmres_layout(NRT, kmax, chunk, sizeof(cd), bS, bI, true, nullptr) <= (size_t)p0->ctx->max_lds;
  if (resident) *resident = res;
  return gmres_layout(NRT, kmax, chunk, sizeof(cd), bS, bI, res, L);
}

// Launch attributes of the kernels with large dynamic LDS, cached per device
// and kernel: the dynamic-LDS limit is raised only when a launch needs more,
// and the co-resident blocks per CU are queried once per LDS size, so that
// repeated launches make no runtime queries.  Several host threads may launch
// (a server's worker and callers of other problems).
namespace {
std::mutex g_attr_mu;
std::map<std::pair<int, const void*>, int> g_lds_set;
std::map<std::tuple<int, const void*, size_t>, int> g_per_cu;
}  // namespace

hipError_t ensure_lds(const void* fn, size_t lds) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_attr_mu);
  int& cur = g_lds_set[{dev, fn}];
  if ((int)lds <= cur) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) cur = (int)lds;
  return e;
}

static hipError_t blocks_per_cu(const void* fn, size_t lds, int* per_cu) {
  hipError_t e = ensure_lds(fn, lds);
  if (e != hipSuccess) return e;
  int dev = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_attr_mu);
  const auto key = std::make_tuple(dev, fn, lds);
  auto it = g_per_cu.find(key);
  if (it != g_per_cu.end()) {
    *per_cu = it->second;
    return hipSuccess;
  }
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, fn, 256, lds);
  if (e == hipSuccess) g_per_cu[key] = *per_cu;
  return e;
}

// Whether every block of one GMRES launch over these instances can be
// co-resident (hipSuccess) or not (an error code).
template <class TS, int NRT>
static hipError_t gmres_fits(const std::vector<const Problem*>& ms, int kmax, int blocks) {
  size_t lds = gmres_plan<TS, NRT>(ms, kmax, nullptr, nullptr);
  const Ctx* ctx = ms[0]->ctx;
  if (lds > (size_t)ctx->max_lds) return hipErrorOutOfMemory;
  const void* fn = (const void*)k_gmres<TS, NRT, Many>;
  hipError_t e = ensure_lds((const void*)k_gmres<TS, NRT, One>, lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = blocks_per_cu(fn, lds, &per_cu);
  if (e != hipSuccess) return e;
  return (int64_t)per_cu * ctx->num_cu >= blocks ? hipSuccess : hipErrorCooperativeLaunchTooLarge;
}

// One cooperative launch for right-hand sides r0 .. r0 + NRT - 1 of every
// instance of launch group gi.
template <class TS, int NRT>
static hipError_t gmres_t(const Target& t, int gi, double tol, int kmax, int r0) {
  std::vector<const Problem*> ms;
  gmres_members(t, gi, ms);
  GmresLaunch L;
  bool resident = false;
  size_t lds = gmres_plan<TS, NRT>(ms, kmax, &resident, &L);
  L.tol = tol;
  L.kmax = kmax;
  L.r0 = r0;
  L.resident = resident ? 1 : 0;
  L.check_spins = -1;
  launch2(t, K_ONE, k_bar_reset<One>, k_bar_reset<Many>, 1, 256, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (const Problem* p : ms) {
    Problem* q = const_cast<Problem*>(p);
    q->last_resident = resident;
    q->last_nrt = NRT;
  }
  if (t.single()) {
    One src = t.src1();
    void* args[] = {&src, &L};
    const void* fn = (const void*)k_gmres<TS, NRT, One>;
    e = ensure_lds(fn, lds);
    if (e != hipSuccess) return e;
    if (t.one->gmres_plain && !t.one->gmres_coop) {
      L.check_spins = t.one->gmres_plain == 2 ? 0 : CORESIDENT_SPINS;
      return hipLaunchKernel(fn, dim3(t.one->gmres_blocks), dim3(256), args, lds, t.st);
    }
    return hipLaunchCooperativeKernel(fn, dim3(t.one->gmres_blocks), dim3(256), args, lds, t.st);
  }
  Many src{t.devs, t.ggroups[gi].inst, t.first[K_GMRES]};
  void* args[] = {&src, &L};
  const void* fn = (const void*)k_gmres<TS, NRT, Many>;
  e = ensure_lds(fn, lds);
  if (e != hipSuccess) return e;
  return hipLaunchCooperativeKernel(fn, dim3(t.ggroups[gi].total), dim3(256), args, lds, t.st);
}

// The group's right-hand sides: the widest kernel (4, 2 or 1 right-hand sides
// per launch) whose LDS layout and grid fit serves them in consecutive launches.
template <class TS>
static hipError_t gmres_group(const Target& t, int gi, double tol, int kmax, int nr) {
  std::vector<const Problem*> ms;
  gmres_members(t, gi, ms);
  const int blocks = t.single() ? t.one->gmres_blocks : t.ggroups[gi].total;
  int w = 1;
  if (nr > 2 && gmres_fits<TS, 4>(ms, kmax, blocks) == hipSuccess) w = 4;
  else if (nr > 1 && gmres_fits<TS, 2>(ms, kmax, blocks) == hipSuccess) w = 2;
  else {
    hipError_t e = gmres_fits<TS, 1>(ms, kmax, blocks);
    if (e != hipSuccess) return e;
  }
  for (int r0 = 0; r0 < nr; r0 += w) {
    hipError_t e = w == 4 ? gmres_t<TS, 4>(t, gi, tol, kmax, r0)
                 : w == 2 ? gmres_t<TS, 2>(t, gi, tol, kmax, r0)
                          : gmres_t<TS, 1>(t, gi, tol, kmax, r0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_gmres(const Target& t, double tol, int kmax) {
  const int ng = t.single() ? 1 : (int)t.ggroups.size();
  for (int gi = 0; gi < ng; ++gi) {
    int nr = 0;
    if (t.single()) nr = t.one->nr;
    else
      for (int i : t.ggroups[gi].members) nr = std::max(nr, t.probs[i]->nr);
    if (nr <= 0) continue;
    if (nr > NRMAX) return hipErrorInvalidValue;
    hipError_t e = t.s32() ? gmres_group<cf>(t, gi, tol, kmax, nr) : gmres_group<cd>(t, gi, tol, kmax, nr);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Whether the one-RHS GMRES kernel fits this problem (the narrowest one).
hipError_t gmres_check(const Problem& p, int kmax) {
  std::vector<const Problem*> ms{&p};
  if (p.s32()) return gmres_fits<cf, 1>(ms, kmax, p.gmres_blocks);
  return gmres_fits<cd, 1>(ms, kmax, p.gmres_blocks);
}

// Co-resident blocks of a GMRES launch of width NRMAX whose blocks hold at most
// `chunk` multipliers (staged layout), for sizing batch launch groups.
int gmres_capacity(const Problem& p, int kmax, int chunk, int width) {
  size_t bS, bI;
  block_bytes(p, &bS, &bI);
  size_t lds = gmres_layout(width, kmax, chunk, sizeof(cd), bS, bI, false, nullptr);
  if (lds > (size_t)p.ctx->max_lds) return 0;
  const void* fn = p.s32() ? (width == 4 ? (const void*)k_gmres<cf, 4, Many>
                                         : width == 2 ? (const void*)k_gmres<cf, 2, Many> : (const void*)k_gmres<cf, 1, Many>)
                           : (width == 4 ? (const void*)k_gmres<cd, 4, Many>
                                         : width == 2 ? (const void*)k_gmres<cd, 2, Many> : (const void*)k_gmres<cd, 1, Many>);
  int per_cu = 0;
  hipError_t e = blocks_per_cu(fn, lds, &per_cu);
  if (e != hipSuccess || per_cu < 1) return 0;
  return per_cu * p.ctx->num_cu;
}

hipError_t launch_recover_coarse(const Target& t) {
  // NQ waves per block: one per (subdomain, coarse slot)
  if (t.s32()) launch2(t, K_SUB, k_frct<cf, One>, k_frct<cf, Many>, NRMAX, 64 * NQ, 0);
  else launch2(t, K_SUB, k_frct<cd, One>, k_frct<cd, Many>, NRMAX, 64 * NQ, 0);
  launch2(t, K_NC128, k_corner_sum<One>, k_corner_sum<Many>, NRMAX, 128, 0);
  launch2(t, K_NC, k_dense_mv<One>, k_dense_mv<Many>, 1, 64, 0, (int)V_YMIN);
  launch2(t, K_NMU256, k_add_edge_mult<One>, k_add_edge_mult<Many>, NRMAX, 256, 0);
  return hipGetLastError();
}

hipError_t launch_assemble_solution(const Target& t, int x, int conj_out) {
  launch2(t, K_ASM256, k_assemble<One>, k_assemble<Many>, NRMAX, 256, 0, x, conj_out);
  return hipGetLastError();
}

template <class TS>
static hipError_t iface_t(Problem& p, char which, const cd* x, cd* y, hipStream_t st) {
  Geo2 g = p.geo();
  Maps2 mp = p.maps();
  if (which == 'P') {
    size_t bytes = align16((size_t)packed_len(p.ND) * sizeof(cf));
    hipError_t e = hipFuncSetAttribute((const void*)k_iface_precond<TS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_iface_precond<TS>, dim3(p.nsub), dim3(256), bytes, st, g, mp, (const cf*)p.Sbb,
                       x, p.Abuf);
    // the precond phase applies one W = 1/2 on the way in; the second on the way out
    hipLaunchKernelGGL(k_combine, dim3((p.nmu + 255) / 256), dim3(256), 0, st, g, mp, p.Abuf, 0.5, y);
  } else if (which == 'F') {
    size_t bytes = align16((size_t)packed_len(p.ND) * sizeof(TS));
    hipError_t e = hipFuncSetAttribute((const void*)k_iface_f1<TS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_iface_f1<TS>, dim3(p.nsub), dim3(256), bytes, st, g, mp, p.rs(),
                       (const TS*)p.Sinv, (const TS*)p.Phi, x, p.Ybuf, p.Cbuf);
    hipLaunchKernelGGL(k_iface_gco, dim3(p.nsub), dim3(256), 0, st, g, mp, p.rs(), (const cd*)p.Cbuf, p.ymin);
    hipLaunchKernelGGL(k_iface_f2<TS>, dim3(p.nsub), dim3(256), 0, st, g, mp, p.rs(), (const TS*)p.Phi,
                       p.Kinv, (const cd*)p.ymin, p.Ybuf);
    hipLaunchKernelGGL(k_combine, dim3((p.nmu + 255) / 256), dim3(256), 0, st, g, mp, p.Ybuf, 1.0, y);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_interface_apply(Problem& p, char which, const cd* x, cd* y, hipStream_t st) {
  if (p.s32()) return iface_t<cf>(p, which, x, y, st);
  return iface_t<cd>(p, which, x, y, st);
}

}  // namespace sfdp

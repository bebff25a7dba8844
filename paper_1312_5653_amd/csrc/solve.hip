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
#include "common.h"

namespace sfdp {

constexpr int ML = 33;

// ------------------------------------------------------------------------------------------
// Grid barrier for a cooperative launch (all blocks co-resident), two levels to
// spread the atomics: blocks arrive on one of G group counters (separate
// 128-byte lines), the last arrival of each group arrives on the top counter,
// and the last group publishes the epoch in a generation word that every block
// polls.  Counters only grow (barrier e completes at e * size), so nothing is
// reset inside a launch.  A spin limit turns a broken barrier into an error
// flag instead of a hang.  bar holds BAR_WORDS words.
constexpr int BAR_GROUPS = 16, BAR_STRIDE = 32, BAR_TOP = BAR_GROUPS * BAR_STRIDE,
              BAR_GEN = BAR_TOP + BAR_STRIDE, BAR_WORDS = BAR_GEN + BAR_STRIDE;
__device__ inline void grid_barrier(unsigned* bar, unsigned nblocks, unsigned& epoch, int* err) {
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
    const unsigned grp = blockIdx.x % G;
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

// out[i] = sum_q part[i * nb + q] for i < n, in a fixed order (identical in every
// block).  Wave w takes i = w, w + 4, ...; four values of i per batch keep 16
// loads in flight per lane.  nb <= 256.
__device__ inline void reduce_partials(const cd* __restrict__ part, int nb, int n, cd* out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i0 = wv * 4; i0 < n; i0 += 16) {
    cd v[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int i = i0 + u, q = lane + 64 * r;
        v[u][r] = (i < n && q < nb) ? ld_coh(part + (size_t)i * nb + q) : cd{0.0, 0.0};
      }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      cd a = (v[u][0] + v[u][1]) + (v[u][2] + v[u][3]);
      for (int off = 32; off > 0; off >>= 1) {
        a.x += __shfl_xor(a.x, off, 64);
        a.y += __shfl_xor(a.y, off, 64);
      }
      if (lane == 0 && i0 + u < n) out[i0 + u] = a;
    }
  }
  __syncthreads();
}

// part[i * nb + b] = sum_{k < kn} conj(Q[i][k0 + k]) w[k] for i < nvec.  Eight
// lanes per vector (32 vectors per pass), partial sums combined by shuffles.
__device__ inline void block_dots(const cd* __restrict__ Q, int nmu, int k0, int kn, int nvec,
                                  const cd* wch, cd* part, int nb, int b) {
  const int t = threadIdx.x, g = t & 7;
  for (int i0 = 0; i0 < nvec; i0 += 32) {
    int i = i0 + (t >> 3);
    cd acc{0.0, 0.0};
    if (i < nvec) {
      const cd* q = Q + (size_t)i * nmu + k0;
#pragma unroll 4
      for (int k = g; k < kn; k += 8) fma_conj_acc(acc, q[k], wch[k]);
    }
    for (int off = 4; off > 0; off >>= 1) {
      acc.x += __shfl_xor(acc.x, off, 64);
      acc.y += __shfl_xor(acc.y, off, 64);
    }
    if (g == 0 && i < nvec) st_coh(part + (size_t)i * nb + b, acc);
  }
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
    for (int u = 0; u < 8; ++u) {
      int i = i0 + u * 256;
      if (i < n16) v[u] = s4[i];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int i = i0 + u * 256;
      if (i < n16) d4[i] = v[u];
    }
  }
  __syncthreads();
}

// Bulk copy of one line factor (ml * ml entries, <= 33 * 33) global -> registers:
// every thread issues its (at most 5) loads back to back.
constexpr int GPT = (ML * ML + 255) / 256;
template <class TS>
__device__ inline void line_load(const TS* __restrict__ src, int n2, TS (&reg)[GPT]) {
#pragma unroll
  for (int r = 0; r < GPT; ++r) {
    int idx = threadIdx.x + 256 * r;
    if (idx < n2) reg[r] = src[idx];
  }
}
template <class TS>
__device__ inline void line_store(TS* dst, int n2, const TS (&reg)[GPT]) {
#pragma unroll
  for (int r = 0; r < GPT; ++r) {
    int idx = threadIdx.x + 256 * r;
    if (idx < n2) dst[idx] = reg[r];
  }
}

// t[p] = sum_k G(p,k) z[k] for one line; G in LDS stored transposed (G(p,k) at
// Gl[k*ml + p]); four wave groups split k, partial sums reduced through LDS.
template <class TS, class T>
__device__ inline void line_mv(const TS* Gl, int ml, const T* z, T* red, T* out, bool subtract) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int kq = (ml + 3) / 4;
  T acc{0, 0};
  if (lane < ml) {
    int k0 = wv * kq, k1 = min(ml, k0 + kq);
    for (int k = k0; k < k1; ++k) fma_acc(acc, cvt<typename real_of<T>::type>(Gl[k * ml + lane]), z[k]);
  }
  if (lane < ml) red[wv * ML + lane] = acc;
  __syncthreads();
  if (threadIdx.x < ml) {
    T s = red[threadIdx.x] + red[ML + threadIdx.x];
    s = s + red[2 * ML + threadIdx.x];
    s = s + red[3 * ML + threadIdx.x];
    out[threadIdx.x] = subtract ? out[threadIdx.x] - s : s;
  }
  __syncthreads();
}

// ------------------------------------------------------------------------------------------
// Full local solve with E^s (extended Z_rr^s).
//   mode 0: load f_r = f / multiplicity; output x on Delta (Xd) and Z_cr x (Qc).
//   mode 1: load f_r - Z_rc B_c uc - B_r^T mu; output Delta values (Ubuf) and
//           interior values straight into xout (conjugated if conj_out).
template <class TS>
__global__ void __launch_bounds__(256) k_local_solve(Geo2 g, Maps2 mp, const TS* __restrict__ G,
                                                     int mode, const cd* __restrict__ f, int conj_in,
                                                     const cd* __restrict__ uc,
                                                     const cd* __restrict__ mu, cd* Xd, cd* Qc,
                                                     cd* Ubuf, cd* xout, int conj_out) {
  using R = typename real_of<TS>::type;
  using T = C<R>;
  __shared__ T xall[ML * ML];
  __shared__ T zl[ML];
  __shared__ T red[4 * ML];
  __shared__ TS gbuf[2][ML * ML];
  const int s = blockIdx.x, ml = g.ml, n2 = ml * ml, ND = g.ND;
  const TS* Gs = G + (size_t)s * ml * n2;
  TS greg[GPT];
  line_load<TS>(Gs, n2, greg);  // line 0 in flight while the load vector is built
  // load right-hand side
  for (int l = threadIdx.x; l < n2; l += blockDim.x) {
    int a = l % ml, b = l / ml;
    cd v{0.0, 0.0};
    if (g.rnode(s, a, b)) {
      cd fv = f[g.freeidx(s, a, b)];
      if (conj_in) fv = conj(fv);
      v = (1.0 / g.mult(a, b)) * fv;
      if (mode == 1) {
        for (int q = 0; q < 4; ++q) {
          int cl = mp.cloc[s * 4 + q];
          if (cl < 0) continue;
          int ca = cl % ml, cb = cl / ml;
          if (abs(ca - a) > 1 || abs(cb - b) > 1) continue;
          v = v - g.zloc(a, b, ca, cb) * uc[mp.cgid[s * 4 + q]];
        }
      }
    }
    xall[l] = T{(R)v.x, (R)v.y};
  }
  __syncthreads();
  if (mode == 1) {
    int nd = mp.nd[s];
    for (int i = threadIdx.x; i < nd; i += blockDim.x) {
      int l = mp.dloc[s * ND + i];
      cd m = (double)mp.dsgn[s * ND + i] * mu[mp.dmid[s * ND + i]];
      xall[l] = xall[l] - T{(R)m.x, (R)m.y};
    }
    __syncthreads();
  }
  line_store<TS>(gbuf[0], n2, greg);
  __syncthreads();
  // forward: z_j = f_j - A_j,j-1 t_j-1 ; t_j = G_j z_j   (t_j overwrites f_j in xall)
  for (int j = 0; j < ml; ++j) {
    const int nxt = (j + 1 < ml) ? j + 1 : ml - 2;  // the backward sweep starts at line ml-2
    line_load<TS>(Gs + (size_t)nxt * n2, n2, greg);
    if (threadIdx.x < ml) {
      int p = threadIdx.x;
      T v = xall[p + ml * j];
      if (j > 0) {
        for (int a = max(p - 1, 0); a <= min(p + 1, ml - 1); ++a) {
          cd e = g.eloc(s, p, j, a, j - 1);
          v = v - T{(R)e.x, (R)e.y} * xall[a + ml * (j - 1)];
        }
      }
      zl[p] = v;
    }
    __syncthreads();
    line_mv<TS, T>(gbuf[j & 1], ml, zl, red, xall + ml * j, false);
    line_store<TS>(gbuf[(j + 1) & 1], n2, greg);
    __syncthreads();
  }
  // backward: x_j = t_j - G_j A_j,j+1 x_j+1   (line j's factor sits in gbuf[(ml - 1 - j + ml) & 1]
  // after the forward loop: buffer parity continues from the forward sweep)
  int par = ml & 1;
  for (int j = ml - 2; j >= 0; --j) {
    if (j > 0) line_load<TS>(Gs + (size_t)(j - 1) * n2, n2, greg);
    if (threadIdx.x < ml) {
      int p = threadIdx.x;
      T v{0, 0};
      for (int a = max(p - 1, 0); a <= min(p + 1, ml - 1); ++a) {
        cd e = g.eloc(s, p, j, a, j + 1);
        fma_acc(v, T{(R)e.x, (R)e.y}, xall[a + ml * (j + 1)]);
      }
      zl[p] = v;
    }
    __syncthreads();
    line_mv<TS, T>(gbuf[par], ml, zl, red, xall + ml * j, true);
    par ^= 1;
    if (j > 0) line_store<TS>(gbuf[par], n2, greg);
    __syncthreads();
  }
  // outputs
  const int nd = mp.nd[s];
  if (mode == 0) {
    for (int i = threadIdx.x; i < nd; i += blockDim.x) {
      T x = xall[mp.dloc[s * ND + i]];
      Xd[(size_t)s * ND + i] = cd{(double)x.x, (double)x.y};
    }
    if (threadIdx.x < 4) {
      int q = threadIdx.x;
      int cl = mp.cloc[s * 4 + q];
      cd acc{0.0, 0.0};
      if (cl >= 0) {
        int ca = cl % ml, cb = cl / ml;
        for (int b = max(cb - 1, 0); b <= min(cb + 1, ml - 1); ++b)
          for (int a = max(ca - 1, 0); a <= min(ca + 1, ml - 1); ++a) {
            if (!g.rnode(s, a, b)) continue;
            T x = xall[a + ml * b];
            fma_acc(acc, g.zloc(ca, cb, a, b), cd{(double)x.x, (double)x.y});
          }
      }
      Qc[s * 4 + q] = acc;
    }
  } else {
    for (int i = threadIdx.x; i < nd; i += blockDim.x) {
      T x = xall[mp.dloc[s * ND + i]];
      Ubuf[(size_t)s * ND + i] = cd{(double)x.x, (double)x.y};
    }
    for (int l = threadIdx.x; l < n2; l += blockDim.x) {
      int a = l % ml, b = l / ml;
      if (a == 0 || a == ml - 1 || b == 0 || b == ml - 1) continue;  // interior only
      T x = xall[l];
      cd v{(double)x.x, (double)x.y};
      xout[g.freeidx(s, a, b)] = conj_out ? conj(v) : v;
    }
  }
}

// f_c* = f_c - sum_s B_c^T Qc  (one thread per global corner, fixed order)
__global__ void k_coarse_rhs(Geo2 g, Maps2 mp, const cd* f, int conj_in, const cd* Qc, cd* fcs) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.nC) return;
  cd v = f[mp.cfree[c]];
  if (conj_in) v = conj(v);
  for (int o = 0; o < 4; ++o) {
    int own = mp.cown[c * 4 + o];
    if (own >= 0) v = v - Qc[own];
  }
  fcs[c] = v;
}

// y = A x (n x n dense FP64 complex), one wavefront per row.
__global__ void k_dense_mv(int n, const cd* __restrict__ A, const cd* __restrict__ x, cd* y) {
  int row = blockIdx.x;
  cd acc{0.0, 0.0};
  for (int k = threadIdx.x; k < n; k += 64) fma_acc(acc, A[(size_t)row * n + k], x[k]);
  for (int off = 32; off > 0; off >>= 1) {
    acc.x += __shfl_down(acc.x, off, 64);
    acc.y += __shfl_down(acc.y, off, 64);
  }
  if (threadIdx.x == 0) y[row] = acc;
}

// d_k = sum over the two subdomains of sign * (Xd - Phi u0)
template <class TS>
__global__ void k_fetidp_rhs(Geo2 g, Maps2 mp, const cd* Xd, const TS* Phi, const cd* u0, cd* d) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.nmu) return;
  cd out{0.0, 0.0};
  for (int e = 0; e < 2; ++e) {
    int o = mp.muown[2 * k + e];
    int s = o / g.ND, slot = o % g.ND;
    cd v = Xd[o];
    for (int q = 0; q < 4; ++q) {
      int c = mp.cgid[s * 4 + q];
      if (c < 0) continue;
      cd ph = cvt<double>(Phi[((size_t)s * g.ND + slot) * 4 + q]);
      v = v - ph * u0[c];
    }
    out = e == 0 ? out + v : out - v;
  }
  d[k] = out;
}

// c^s_q = sum_i Phi[s][i][q] sign_i mu[mid_i]  (F_rc^T mu contributions); one
// wavefront per (subdomain, corner slot).
template <class TS>
__global__ void k_frct(Geo2 g, Maps2 mp, const TS* Phi, const cd* mu, cd* Cbuf) {
  int t = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (t >= g.nsub * 4) return;
  int s = t / 4, q = t % 4;
  cd acc{0.0, 0.0};
  if (mp.cloc[s * 4 + q] >= 0) {
    int nd = mp.nd[s];
    for (int i = lane; i < nd; i += 64) {
      cd x = (double)mp.dsgn[s * g.ND + i] * mu[mp.dmid[s * g.ND + i]];
      fma_acc(acc, cvt<double>(Phi[((size_t)s * g.ND + i) * 4 + q]), x);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    acc.x += __shfl_down(acc.x, off, 64);
    acc.y += __shfl_down(acc.y, off, 64);
  }
  if (lane == 0) Cbuf[t] = acc;
}

// rhs_c = fcs_c + sum_owners Cbuf
__global__ void k_corner_sum(Geo2 g, Maps2 mp, const cd* fcs, const cd* Cbuf, cd* out) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.nC) return;
  cd v = fcs ? fcs[c] : cd{0.0, 0.0};
  for (int o = 0; o < 4; ++o) {
    int own = mp.cown[c * 4 + o];
    if (own >= 0) v = v + Cbuf[own];
  }
  out[c] = v;
}

// primal assembly: Delta nodes average the two subdomain copies, corners take uc
__global__ void k_assemble(Geo2 g, Maps2 mp, const cd* Ubuf, const cd* uc, cd* x, int conj_out) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
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
// Interface phases (device functions shared by the persistent GMRES kernel and
// the stand-alone test kernels).

// Abuf[s] = S_bb^s x,  x_i = 0.5 * sc * sign_i * vin[mid_i]   (W = 1/2).
// S_bb is complex64 (packed); it is staged into `buf` unless `resident`.
template <class TS>
__device__ void phase_precond(const Geo2& g, const Maps2& mp, const cf* __restrict__ Sbb, int s,
                              const cd* vin, double sc, cd* Abuf, cf* buf, bool resident,
                              typename real_of<TS>::type* xs_raw, cd* red, cd* ys) {
  using R = typename real_of<TS>::type;
  using T = C<R>;
  T* xs = (T*)xs_raw;
  const int ND = g.ND, nd = mp.nd[s];
  __syncthreads();
  if (!resident) stage_lds(buf, Sbb + (size_t)s * packed_len(ND), packed_len(nd) * (int)sizeof(cf));
  for (int i = threadIdx.x; i < ND; i += blockDim.x) {
    T v{0, 0};
    if (i < nd) {
      cd m = (0.5 * sc * mp.dsgn[s * ND + i]) * ld_coh(vin + mp.dmid[s * ND + i]);
      v = T{(R)m.x, (R)m.y};
    }
    xs[i] = v;
  }
  __syncthreads();
  symv_packed<cf, R>(buf, nd, xs, red, ys);
  for (int i = threadIdx.x; i < nd; i += blockDim.x) st_coh(Abuf + (size_t)s * ND + i, ys[i]);
}

// Ybuf[s] = Z_rr^-1|Delta x, Cbuf[s] = Phi^T x.   x from Abuf (preconditioned
// vector, from_abuf) or directly x_i = sign_i * vin[mid_i].  Sinv (packed, in the
// storage precision) is staged into `buf` unless `resident`.
template <class TS>
__device__ void phase_f1(const Geo2& g, const Maps2& mp, const TS* __restrict__ Sinv,
                         const TS* __restrict__ Phi, int s, bool from_abuf, const cd* Abuf,
                         const cd* vin, cd* Ybuf, cd* Cbuf, TS* buf, bool resident,
                         typename real_of<TS>::type* xs_raw, cd* red, cd* ys) {
  using R = typename real_of<TS>::type;
  using T = C<R>;
  T* xs = (T*)xs_raw;
  const int ND = g.ND, nd = mp.nd[s];
  __syncthreads();
  if (!resident) stage_lds(buf, Sinv + (size_t)s * packed_len(ND), packed_len(nd) * (int)sizeof(TS));
  for (int i = threadIdx.x; i < ND; i += blockDim.x) {
    T v{0, 0};
    if (i < nd) {
      cd m;
      if (from_abuf) m = 0.5 * (ld_coh(Abuf + (size_t)s * ND + i) - ld_coh(Abuf + mp.dpart[s * ND + i]));
      else m = (double)mp.dsgn[s * ND + i] * ld_coh(vin + mp.dmid[s * ND + i]);
      v = T{(R)m.x, (R)m.y};
    }
    xs[i] = v;
  }
  __syncthreads();
  symv_packed<TS, R>(buf, nd, xs, red, ys);
  for (int i = threadIdx.x; i < nd; i += blockDim.x) st_coh(Ybuf + (size_t)s * ND + i, ys[i]);
  // corner products: one wavefront per corner slot
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  cd acc{0.0, 0.0};
  if (mp.cloc[s * 4 + q] >= 0) {
    for (int i = lane; i < nd; i += 64) {
      T x = xs[i];
      fma_acc(acc, cvt<double>(Phi[((size_t)s * ND + i) * 4 + q]), cd{(double)x.x, (double)x.y});
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    acc.x += __shfl_down(acc.x, off, 64);
    acc.y += __shfl_down(acc.y, off, 64);
  }
  if (lane == 0) st_coh(Cbuf + s * 4 + q, acc);
}

// Ybuf[s] += Phi uc_own with uc = K_cc*^-1 g, g_c = sum of Cbuf over the corner's owners.
template <class TS>
__device__ void phase_f2(const Geo2& g, const Maps2& mp, const TS* __restrict__ Phi,
                         const cd* __restrict__ Kinv, int s, const cd* Cbuf, cd* Ybuf, cd* gsh,
                         cd* ucs) {
  const int ND = g.ND, nd = mp.nd[s];
  __syncthreads();
  for (int c = threadIdx.x; c < g.nC; c += blockDim.x) {
    cd v{0.0, 0.0};
    for (int o = 0; o < 4; ++o) {
      int own = mp.cown[c * 4 + o];
      if (own >= 0) v = v + ld_coh(Cbuf + own);
    }
    gsh[c] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  int c = mp.cgid[s * 4 + q];
  cd acc{0.0, 0.0};
  if (c >= 0)
    for (int k = lane; k < g.nC; k += 64) fma_acc(acc, Kinv[(size_t)c * g.nC + k], gsh[k]);
  for (int off = 32; off > 0; off >>= 1) {
    acc.x += __shfl_down(acc.x, off, 64);
    acc.y += __shfl_down(acc.y, off, 64);
  }
  if (lane == 0) ucs[q] = acc;
  __syncthreads();
  for (int i = threadIdx.x; i < nd; i += blockDim.x) {
    cd y = ld_coh(Ybuf + (size_t)s * ND + i);
    for (int qq = 0; qq < 4; ++qq) {
      if (mp.cgid[s * 4 + qq] < 0) continue;
      fma_acc(y, cvt<double>(Phi[((size_t)s * ND + i) * 4 + qq]), ucs[qq]);
    }
    st_coh(Ybuf + (size_t)s * ND + i, y);
  }
}

// ------------------------------------------------------------------------------------------
// Persistent GMRES on F_DP P^-1 t = d.
struct GmresArgs {
  const cd* d;
  cd* mu;
  cd* Abuf;
  cd* Ybuf;
  cd* Cbuf;
  cd* w;
  cd* Q;      // [(kmax+1)][nmu]
  cd* H;      // [(kmax+1)][kmax] column j at H[i*kmax + j]
  cd* part;   // [3][kmax+2][nblocks]
  unsigned* bar;
  int* flags; // [0] iterations, [1] barrier error
  double* scal; // [0] final relative residual estimate
  double tol;
  int kmax;
  int chunk;
  int resident;     // Schur blocks kept in LDS (requires one subdomain per block)
  int lds_bufA;     // byte offset of the second resident buffer
};

// Dynamic LDS of k_gmres: work arrays, then the Schur-block buffers (two
// resident blocks, or one staging buffer).
__host__ __device__ inline size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

template <class TS>
__global__ void __launch_bounds__(256) k_gmres(Geo2 g, Maps2 mp, const cf* __restrict__ Sbb,
                                               const TS* __restrict__ Sinv,
                                               const TS* __restrict__ Phi,
                                               const cd* __restrict__ Kinv, GmresArgs a) {
  using R = typename real_of<TS>::type;
  extern __shared__ __align__(16) char smem[];
  // dynamic LDS layout
  cd* red = (cd*)smem;                          // 256
  cd* ys = red + 256;                           // ND (<= 256)
  R* xs = (R*)(ys + 256);                       // 2 * 256 reals
  cd* gsh = (cd*)(xs + 512);                    // nC
  cd* wch = gsh + g.nC;                         // chunk
  cd* hv = wch + a.chunk;                       // kmax + 1
  cd* h2 = hv + a.kmax + 1;                     // kmax + 1
  cd* csv = h2 + a.kmax + 1;                    // kmax
  cd* snv = csv + a.kmax;                       // kmax
  cd* gv = snv + a.kmax;                        // kmax + 1
  cd* ucs = gv + a.kmax + 1;                    // 4
  char* mats = (char*)(ucs + 4);
  cf* bufS = (cf*)mats;                         // S_bb (resident) or the staging buffer
  TS* bufI = a.resident ? (TS*)(mats + a.lds_bufA) : (TS*)mats;  // Z_rr^-1|Delta
  if (a.resident) {
    // one subdomain per block: both Schur blocks stay in LDS for the whole solve
    const int s = blockIdx.x, nd = mp.nd[s];
    stage_lds(bufS, Sbb + (size_t)s * packed_len(g.ND), packed_len(nd) * (int)sizeof(cf));
    stage_lds(bufI, Sinv + (size_t)s * packed_len(g.ND), packed_len(nd) * (int)sizeof(TS));
  }
  __shared__ double sc_sh[4];
  __shared__ int stop_sh;

  const unsigned nb = gridDim.x;
  const int b = blockIdx.x;
  unsigned epoch = 0;
  const int nmu = g.nmu, kmax = a.kmax;
  const int k0 = min(nmu, b * a.chunk), k1 = min(nmu, k0 + a.chunk), kn = k1 - k0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  cd* part0 = a.part;
  cd* part1 = a.part + (size_t)(kmax + 2) * nb;
  cd* part2 = a.part + (size_t)2 * (kmax + 2) * nb;

  // block reduction of a real value into thread 0
  auto block_sum_real = [&](double v) -> double {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) sc_sh[wv] = v;
    __syncthreads();
    double t = sc_sh[0] + sc_sh[1] + sc_sh[2] + sc_sh[3];
    __syncthreads();
    return t;
  };

  // ---- init: beta0 = ||d||
  {
    double loc = 0.0;
    for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x) loc += abs2(a.d[k]);
    double t = block_sum_real(loc);
    if (threadIdx.x == 0) st_coh(part2 + b, cd{t, 0.0});
  }
  grid_barrier(a.bar, nb, epoch, a.flags + 1);
  reduce_partials(part2, nb, 1, ucs);
  const double beta0 = sqrt(ucs[0].x);
  __syncthreads();
  if (threadIdx.x == 0) gv[0] = cd{beta0, 0.0};
  if (beta0 == 0.0) {
    for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x) a.mu[k] = cd{0.0, 0.0};
    if (b == 0 && threadIdx.x == 0) { a.flags[0] = 0; a.scal[0] = 0.0; }
    return;
  }
  const cd* vin = a.d;
  double vscale = 1.0 / beta0;
  int j = 0, iters = 0;
  double resid = 1.0;
  for (j = 0; j < kmax; ++j) {
    // ---- P: Abuf = S_bb (W B^T q_j); also store q_j = vin * vscale
    for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x)
      a.Q[(size_t)j * nmu + k] = vscale * ld_coh(vin + k);
    for (int s = b; s < g.nsub; s += nb)
      phase_precond<TS>(g, mp, Sbb, s, vin, vscale, a.Abuf, bufS, a.resident, xs, red, ys);
    grid_barrier(a.bar, nb, epoch, a.flags + 1);
    // ---- F1
    for (int s = b; s < g.nsub; s += nb)
      phase_f1<TS>(g, mp, Sinv, Phi, s, true, a.Abuf, nullptr, a.Ybuf, a.Cbuf, bufI, a.resident, xs,
                   red, ys);
    grid_barrier(a.bar, nb, epoch, a.flags + 1);
    // ---- F2 (coarse correction)
    for (int s = b; s < g.nsub; s += nb) phase_f2<TS>(g, mp, Phi, Kinv, s, a.Cbuf, a.Ybuf, gsh, ucs);
    grid_barrier(a.bar, nb, epoch, a.flags + 1);
    // ---- O1: w = B_r Y (combine), first Gram-Schmidt projections
    for (int k = threadIdx.x; k < kn; k += blockDim.x) {
      int kk = k0 + k;
      wch[k] = ld_coh(a.Ybuf + mp.muown[2 * kk]) - ld_coh(a.Ybuf + mp.muown[2 * kk + 1]);
    }
    __syncthreads();
    block_dots(a.Q, nmu, k0, kn, j + 1, wch, part0, nb, b);
    grid_barrier(a.bar, nb, epoch, a.flags + 1);
    // ---- O2: h = sum partials; w -= Q h; second projections
    reduce_partials(part0, nb, j + 1, hv);
    for (int k = threadIdx.x; k < kn; k += blockDim.x) {
      cd v = wch[k];
#pragma unroll 8
      for (int i = 0; i <= j; ++i) v = v - hv[i] * a.Q[(size_t)i * nmu + k0 + k];
      wch[k] = v;
    }
    __syncthreads();
    block_dots(a.Q, nmu, k0, kn, j + 1, wch, part1, nb, b);
    grid_barrier(a.bar, nb, epoch, a.flags + 1);
    // ---- O3: second correction, norm
    reduce_partials(part1, nb, j + 1, h2);
    double loc = 0.0;
    for (int k = threadIdx.x; k < kn; k += blockDim.x) {
      cd v = wch[k];
#pragma unroll 8
      for (int i = 0; i <= j; ++i) v = v - h2[i] * a.Q[(size_t)i * nmu + k0 + k];
      st_coh(a.w + k0 + k, v);
      loc += abs2(v);
    }
    for (int i = threadIdx.x; i <= j; i += blockDim.x) hv[i] = hv[i] + h2[i];
    double t = block_sum_real(loc);
    if (threadIdx.x == 0) st_coh(part2 + b, cd{t, 0.0});
    grid_barrier(a.bar, nb, epoch, a.flags + 1);
    // ---- Arnoldi column j complete: hn, Givens rotations (identical in every block)
    reduce_partials(part2, nb, 1, ucs);
    double hn = sqrt(ucs[0].x);
    if (threadIdx.x == 0) {
      for (int i = 0; i < j; ++i) {
        cd c = csv[i], sn = snv[i];
        cd t0 = c * hv[i] + sn * hv[i + 1];
        cd t1 = conj(c) * hv[i + 1] - conj(sn) * hv[i];
        hv[i] = t0;
        hv[i + 1] = t1;
      }
      cd hj = hv[j];
      double den = sqrt(abs2(hj) + hn * hn);
      cd c, sn;
      if (den == 0.0) { c = cd{1.0, 0.0}; sn = cd{0.0, 0.0}; }
      else { c = (1.0 / den) * conj(hj); sn = cd{hn / den, 0.0}; }
      csv[j] = c;
      snv[j] = sn;
      hv[j] = c * hj + sn * cd{hn, 0.0};
      cd gj = gv[j];
      gv[j + 1] = -(conj(sn) * gj);
      gv[j] = c * gj;
      double res = sqrt(abs2(gv[j + 1])) / beta0;
      sc_sh[0] = res;
      stop_sh = (res <= a.tol || hn == 0.0 || j + 1 == kmax) ? 1 : 0;
    }
    __syncthreads();
    if (b == 0)
      for (int i = threadIdx.x; i <= j; i += blockDim.x) st_coh(a.H + (size_t)i * kmax + j, hv[i]);
    resid = sc_sh[0];
    iters = j + 1;
    if (stop_sh) break;
    vin = a.w;
    vscale = 1.0 / hn;
  }
  // ---- back substitution H y = g (redundant in every block; H columns from block 0)
  grid_barrier(a.bar, nb, epoch, a.flags + 1);
  const int kk = iters;
  for (int i = threadIdx.x; i < kk; i += blockDim.x) h2[i] = gv[i];
  __syncthreads();
  for (int i = kk - 1; i >= 0; --i) {
    if (threadIdx.x == 0) h2[i] = cdiv(h2[i], ld_coh(a.H + (size_t)i * kmax + i));
    __syncthreads();
    cd yi = h2[i];
    for (int t = threadIdx.x; t < i; t += blockDim.x) h2[t] = h2[t] - ld_coh(a.H + (size_t)t * kmax + i) * yi;
    __syncthreads();
  }
  // t = Q y on the chunk
  for (int k = threadIdx.x; k < kn; k += blockDim.x) {
    cd v{0.0, 0.0};
#pragma unroll 8
    for (int i = 0; i < kk; ++i) fma_acc(v, a.Q[(size_t)i * nmu + k0 + k], h2[i]);
    st_coh(a.w + k0 + k, v);
  }
  grid_barrier(a.bar, nb, epoch, a.flags + 1);
  // mu = P^-1 t
  for (int s = b; s < g.nsub; s += nb)
    phase_precond<TS>(g, mp, Sbb, s, a.w, 1.0, a.Abuf, bufS, a.resident, xs, red, ys);
  grid_barrier(a.bar, nb, epoch, a.flags + 1);
  for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x)
    a.mu[k] = 0.5 * (ld_coh(a.Abuf + mp.muown[2 * k]) - ld_coh(a.Abuf + mp.muown[2 * k + 1]));
  if (b == 0 && threadIdx.x == 0) {
    a.flags[0] = iters;
    a.scal[0] = resid;
  }
}

// Stand-alone interface kernels for testing (one block per subdomain).
template <class TS>
__global__ void __launch_bounds__(256) k_iface_precond(Geo2 g, Maps2 mp, const cf* Sbb, const cd* x,
                                                       cd* Abuf) {
  using R = typename real_of<TS>::type;
  extern __shared__ __align__(16) char smem[];
  __shared__ cd red[256], ys[256];
  __shared__ R xs[512];
  phase_precond<TS>(g, mp, Sbb, blockIdx.x, x, 1.0, Abuf, (cf*)smem, false, xs, red, ys);
}
template <class TS>
__global__ void __launch_bounds__(256) k_iface_f1(Geo2 g, Maps2 mp, const TS* Sinv, const TS* Phi,
                                                  const cd* x, cd* Ybuf, cd* Cbuf) {
  using R = typename real_of<TS>::type;
  extern __shared__ __align__(16) char smem[];
  __shared__ cd red[256], ys[256];
  __shared__ R xs[512];
  phase_f1<TS>(g, mp, Sinv, Phi, blockIdx.x, false, nullptr, x, Ybuf, Cbuf, (TS*)smem, false, xs,
               red, ys);
}
template <class TS>
__global__ void __launch_bounds__(256) k_iface_f2(Geo2 g, Maps2 mp, const TS* Phi, const cd* Kinv,
                                                  const cd* Cbuf, cd* Ybuf) {
  extern __shared__ char smem[];
  cd* gsh = (cd*)smem;
  __shared__ cd ucs[4];
  phase_f2<TS>(g, mp, Phi, Kinv, blockIdx.x, Cbuf, Ybuf, gsh, ucs);
}
__global__ void k_combine(Geo2 g, Maps2 mp, const cd* buf, double scale, cd* out) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.nmu) return;
  out[k] = scale * (buf[mp.muown[2 * k]] - buf[mp.muown[2 * k + 1]]);
}

// ------------------------------------------------------------------------------------------
// launchers
template <class TS>
static hipError_t local_solve_t(const Problem& p, int mode, const cd* f, int conj_in, cd* xout,
                                int conj_out) {
  hipLaunchKernelGGL(k_local_solve<TS>, dim3(p.nsub), dim3(256), 0, p.ctx->stream, p.geo(),
                     p.maps(), (const TS*)p.G, mode, f, conj_in, p.u0, p.mu, p.Xd, p.Qc, p.Ubuf,
                     xout, conj_out);
  return hipGetLastError();
}

hipError_t launch_local_solve(const Problem& p, int mode, const cd* f, int conj_in, cd* x_out,
                              hipStream_t) {
  int conj_out = (mode == 1) ? conj_in : 0;
  if (p.prec == SFDP_MIXED) return local_solve_t<cf>(p, mode, f, conj_in, x_out, conj_out);
  return local_solve_t<cd>(p, mode, f, conj_in, x_out, conj_out);
}

hipError_t launch_coarse_rhs(const Problem& p, const cd* f, int conj_in, hipStream_t st) {
  hipLaunchKernelGGL(k_coarse_rhs, dim3((p.nC + 127) / 128), dim3(128), 0, st, p.geo(), p.maps(), f,
                     conj_in, p.Qc, p.fcs);
  if (p.nC > 0) hipLaunchKernelGGL(k_dense_mv, dim3(p.nC), dim3(64), 0, st, p.nC, p.Kinv, p.fcs, p.u0);
  return hipGetLastError();
}

hipError_t launch_fetidp_rhs(const Problem& p, hipStream_t st) {
  if (p.prec == SFDP_MIXED)
    hipLaunchKernelGGL(k_fetidp_rhs<cf>, dim3((p.nmu + 255) / 256), dim3(256), 0, st, p.geo(),
                       p.maps(), p.Xd, (const cf*)p.Phi, p.u0, p.dvec);
  else
    hipLaunchKernelGGL(k_fetidp_rhs<cd>, dim3((p.nmu + 255) / 256), dim3(256), 0, st, p.geo(),
                       p.maps(), p.Xd, (const cd*)p.Phi, p.u0, p.dvec);
  return hipGetLastError();
}

static size_t gmres_work_lds(const Problem& p, int kmax, int chunk) {
  return sizeof(cd) * (256 + 256) + sizeof(double) * 512 +
         sizeof(cd) * (p.nC + chunk + 5 * (size_t)(kmax + 1) + 4);
}
// Total LDS, and the offset of the second resident buffer.
static size_t gmres_lds(const Problem& p, int kmax, int chunk, bool resident, size_t* offB) {
  size_t es = p.prec == SFDP_MIXED ? sizeof(cf) : sizeof(cd);
  size_t pk = (size_t)packed_len(p.ndmax);
  size_t a = align16(pk * sizeof(cf)), b = align16(pk * es);
  if (offB) *offB = a;
  return align16(gmres_work_lds(p, kmax, chunk)) + (resident ? a + b : std::max(a, b));
}

template <class TS>
static hipError_t gmres_t(Problem& p, double tol, int kmax) {
  hipStream_t st = p.ctx->stream;
  int nb = p.gmres_blocks;
  int chunk = (p.nmu + nb - 1) / nb;
  size_t offB = 0;
  bool resident = p.prec == SFDP_MIXED && nb == p.nsub &&
                  gmres_lds(p, kmax, chunk, true, &offB) <= (size_t)p.ctx->max_lds;
  size_t lds = gmres_lds(p, kmax, chunk, resident, &offB);
  if (lds > (size_t)p.ctx->max_lds) return hipErrorOutOfMemory;
  GmresArgs a;
  a.d = p.dvec;
  a.mu = p.mu;
  a.Abuf = p.Abuf;
  a.Ybuf = p.Ybuf;
  a.Cbuf = p.Cbuf;
  a.w = p.wv;
  a.Q = p.Qk;
  a.H = p.Hk;
  a.part = p.part;
  a.bar = p.bar;
  a.flags = p.flags;
  a.scal = p.dscal;
  a.tol = tol;
  a.kmax = kmax;
  a.chunk = chunk;
  a.resident = resident ? 1 : 0;
  a.lds_bufA = (int)offB;
  hipError_t e = launch_fill(p.bar, BAR_WORDS * sizeof(unsigned), st);
  if (e != hipSuccess) return e;
  Geo2 g = p.geo();
  Maps2 mp = p.maps();
  const cf* Sbb = (const cf*)p.Sbb;
  const TS* Sinv = (const TS*)p.Sinv;
  const TS* Phi = (const TS*)p.Phi;
  const cd* Kinv = p.Kinv;
  void* args[] = {&g, &mp, &Sbb, &Sinv, &Phi, &Kinv, &a};
  e = hipFuncSetAttribute((const void*)k_gmres<TS>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  p.last_resident = resident;
  return hipLaunchCooperativeKernel((const void*)k_gmres<TS>, dim3(nb), dim3(256), args, lds, st);
}

hipError_t launch_gmres(Problem& p, double tol, int kmax, hipStream_t) {
  if (p.prec == SFDP_MIXED) return gmres_t<cf>(p, tol, kmax);
  return gmres_t<cd>(p, tol, kmax);
}

int gmres_max_blocks(const Problem& p, int kmax) {
  int per_cu = 0;
  int chunk = (p.nmu + p.gmres_blocks - 1) / p.gmres_blocks;
  size_t lds = gmres_lds(p, kmax, chunk, false, nullptr);
  hipError_t e;
  if (p.prec == SFDP_MIXED) {
    hipFuncSetAttribute((const void*)k_gmres<cf>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_gmres<cf>, 256, lds);
  } else {
    hipFuncSetAttribute((const void*)k_gmres<cd>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_gmres<cd>, 256, lds);
  }
  if (e != hipSuccess || per_cu < 1) return 0;
  return per_cu * p.ctx->num_cu;
}

size_t gmres_lds_bytes(const Problem& p, int kmax, int nb) {
  return gmres_lds(p, kmax, (p.nmu + nb - 1) / nb, false, nullptr);
}

hipError_t launch_recover_coarse(const Problem& p, hipStream_t st) {
  if (p.prec == SFDP_MIXED)
    hipLaunchKernelGGL(k_frct<cf>, dim3((p.nsub * 4 + 3) / 4), dim3(256), 0, st, p.geo(),
                       p.maps(), (const cf*)p.Phi, p.mu, p.Cbuf);
  else
    hipLaunchKernelGGL(k_frct<cd>, dim3((p.nsub * 4 + 3) / 4), dim3(256), 0, st, p.geo(),
                       p.maps(), (const cd*)p.Phi, p.mu, p.Cbuf);
  hipLaunchKernelGGL(k_corner_sum, dim3((p.nC + 127) / 128), dim3(128), 0, st, p.geo(), p.maps(),
                     p.fcs, p.Cbuf, p.ymin);
  if (p.nC > 0) hipLaunchKernelGGL(k_dense_mv, dim3(p.nC), dim3(64), 0, st, p.nC, p.Kinv, p.ymin, p.u0);
  return hipGetLastError();
}

hipError_t launch_assemble_solution(const Problem& p, cd* x, int conj_out, hipStream_t st) {
  int n = p.nmu + p.nC;
  hipLaunchKernelGGL(k_assemble, dim3((n + 255) / 256), dim3(256), 0, st, p.geo(), p.maps(), p.Ubuf,
                     p.u0, x, conj_out);
  return hipGetLastError();
}

template <class TS>
static hipError_t iface_t(Problem& p, char which, const cd* x, cd* y, hipStream_t st) {
  Geo2 g = p.geo();
  Maps2 mp = p.maps();
  if (which == 'P') {
    size_t bytes = align16((size_t)packed_len(p.ND) * sizeof(cf));
    hipFuncSetAttribute((const void*)k_iface_precond<TS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)bytes);
    hipLaunchKernelGGL(k_iface_precond<TS>, dim3(p.nsub), dim3(256), bytes, st, g, mp, (const cf*)p.Sbb,
                       x, p.Abuf);
    // the stand-alone precond kernel scales by 1/2 on the way in; 1/2 on the way out
    hipLaunchKernelGGL(k_combine, dim3((p.nmu + 255) / 256), dim3(256), 0, st, g, mp, p.Abuf, 0.5, y);
  } else if (which == 'F') {
    size_t bytes = align16((size_t)packed_len(p.ND) * sizeof(TS));
    hipFuncSetAttribute((const void*)k_iface_f1<TS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)bytes);
    hipLaunchKernelGGL(k_iface_f1<TS>, dim3(p.nsub), dim3(256), bytes, st, g, mp, (const TS*)p.Sinv,
                       (const TS*)p.Phi, x, p.Ybuf, p.Cbuf);
    hipLaunchKernelGGL(k_iface_f2<TS>, dim3(p.nsub), dim3(256), sizeof(cd) * (p.nC + 1), st, g, mp,
                       (const TS*)p.Phi, p.Kinv, p.Cbuf, p.Ybuf);
    hipLaunchKernelGGL(k_combine, dim3((p.nmu + 255) / 256), dim3(256), 0, st, g, mp, p.Ybuf, 1.0, y);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_interface_apply(Problem& p, char which, const cd* x, cd* y, hipStream_t st) {
  if (p.prec == SFDP_MIXED) return iface_t<cf>(p, which, x, y, st);
  return iface_t<cd>(p, which, x, y, st);
}

}  // namespace sfdp

// FETI-DP for 3D instances (Sec. 5; definitions of F_DP, d, the coarse
// problem and the Dirichlet preconditioner as for 2D):
//
//   set-up   E^s (Z_rr^s padded with the identity, interior nodes first) is
//            inverted as one batch by blocked Gauss-Jordan (FP64).  After the
//            interior pivots the trailing Delta block holds the Schur complement
//            S_bb of the Dirichlet preconditioner; after all pivots E^s holds
//            Z_rr^-1, whose Delta block is the local interface operator.
//            Phi = Z_rr^-1 Z_rc, Z_cc* = Z_cc - Z_cr Phi, K_cc* = sum B_c^T Z_cc* B_c
//            and its inverse (FP64).
//   solve    full sweeps t = Z_rr^-1 f_r (the right-hand side d and the
//            recovery), and right-preconditioned GMRES on F_DP mu = d with
//            classical Gram-Schmidt applied twice, FP64, its Hessenberg matrix
//            and Givens rotations on the host (one synchronisation per
//            iteration).  F_DP = F_rr + F_rc K_cc*^-1 F_rc^T is applied per
//            subdomain from Z_rr^-1|Delta and Phi; the preconditioner
//            W B_r S_bb B_r^T W with multiplicity scaling.
//
// Multipliers are fully redundant (one per pair of subdomains sharing a Delta
// node), so W = (sum B_r B_r^T)^+ is B B^T / k^2 on the k copies of a node;
// since the signed copies of a multiplier cancel, B_r^T W mu = B_r^T mu / k and
// W B_r y = (y_+ - y_-) / k per multiplier: the preconditioner is a 1 / k
// scaling on both sides of S_bb (k = 2 on faces, 4 on edges).
#include <cmath>
#include <complex>
#include <vector>

#include "three.h"
#include "krylov3.h"

namespace sfdp {

namespace {

constexpr int GJW = 2 * 32 * 32;  // pivot-inverse buffers per matrix of gj_range

unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// ---------------------------------------------------------------- set-up --

// E^s on r positions: Z^s between r nodes, identity on the padding.
__global__ void k3_build_E(Geo3 g, const int* rl, cd* E) {
  const int s = blockIdx.y;
  const int64_t NR2 = (int64_t)g.NR * g.NR;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= NR2) return;
  const int p = (int)(t / g.NR), q = (int)(t % g.NR);
  const int lp = rl[s * g.NR + p], lq = rl[s * g.NR + q];
  cd v{0.0, 0.0};
  if (lp < 0 || lq < 0) {
    if (p == q) v.x = 1.0;
  } else {
    v = g.zloc(lp, lq);
  }
  E[(size_t)s * NR2 + t] = v;
}

// out[s][i][j] = E[s][off + i][off + j], i, j < n, in storage precision
template <class TS>
__global__ void k3_take(const cd* E, int NR, int off, int n, TS* out) {
  using R = typename real_of<TS>::type;
  const int s = blockIdx.y;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  const int i = (int)(t / n), j = (int)(t % n);
  out[(size_t)s * n * n + t] = cvt<R>(E[(size_t)s * NR * NR + (size_t)(off + i) * NR + off + j]);
}

// Neighbours of vertex slot q inside the subdomain: the other 7 nodes of the
// element at that vertex, e = 1..7.
__device__ inline int vertex_nbr(const Geo3& g, int q, int e) {
  const int a0 = (q & 1) * g.m, b0 = ((q >> 1) & 1) * g.m, c0 = ((q >> 2) & 1) * g.m;
  const int a = a0 + (a0 ? -1 : 1) * (e & 1), b = b0 + (b0 ? -1 : 1) * ((e >> 1) & 1),
            c = c0 + (c0 ? -1 : 1) * ((e >> 2) & 1);
  return a + g.ml * (b + g.ml * c);
}

// PhiFull[s][p][q] = (Z_rr^-1 Z_rc)[p][q] from the inverted E (row p of E^-1
// against the vertex's coupling to its element's r nodes)
__global__ void k3_phi(Geo3 g, Maps3 mp, const cd* E, cd* PhiFull) {
  const int s = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.NR * 8) return;
  const int p = t >> 3, q = t & 7;
  cd acc{0.0, 0.0};
  if (mp.cg[s * 8 + q] >= 0) {
    const int lv = g.vertex(q);
    const cd* Er = E + (size_t)s * g.NR * g.NR + (size_t)p * g.NR;
    for (int e = 1; e < 8; ++e) {
      const int l = vertex_nbr(g, q, e);
      const int r = mp.rpos[s * g.nl + l];
      if (r >= 0) fma_acc(acc, Er[r], g.zloc(l, lv));
    }
  }
  PhiFull[((size_t)s * g.NR + p) * 8 + q] = acc;
}

template <class TS>
__global__ void k3_phi_delta(Geo3 g, const cd* PhiFull, TS* Phi) {
  using R = typename real_of<TS>::type;
  const int s = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.ND * 8) return;
  const int dl = t >> 3, q = t & 7;
  Phi[((size_t)s * g.ND + dl) * 8 + q] = cvt<R>(PhiFull[((size_t)s * g.NR + g.nI + dl) * 8 + q]);
}

// Z_cc*^s = Z_cc - Z_cr Phi on the subdomain's corner slots (zero elsewhere);
// one block of 64 threads per subdomain
__global__ void k3_zcc(Geo3 g, Maps3 mp, const cd* PhiFull, cd* Zcc) {
  const int s = blockIdx.x, t = threadIdx.x;
  const int q = t >> 3, q2 = t & 7;
  cd v{0.0, 0.0};
  if (mp.cg[s * 8 + q] >= 0 && mp.cg[s * 8 + q2] >= 0) {
    const int lv = g.vertex(q);
    if (q == q2) v = g.zloc(lv, lv);
    for (int e = 1; e < 8; ++e) {
      const int l = vertex_nbr(g, q, e);
      const int r = mp.rpos[s * g.nl + l];
      if (r >= 0) v = v - g.zloc(lv, l) * PhiFull[((size_t)s * g.NR + r) * 8 + q2];
    }
  }
  Zcc[s * 64 + t] = v;
}

// K_cc*[c][c2] = sum over the subdomains of corner c of their Z_cc* entries
// (owners in increasing subdomain order)
__global__ void k3_coarse_assemble(Geo3 g, Maps3 mp, const cd* Zcc, cd* Kcc) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nC = g.nC;
  if (t >= (int64_t)nC * nC) return;
  const int c = (int)(t / nC), c2 = (int)(t % nC);
  cd acc{0.0, 0.0};
  for (int o = 0; o < 8; ++o) {
    const int own = mp.cown[c * 8 + o];
    if (own < 0) continue;
    const int s = own >> 3, q = own & 7;
    for (int q2 = 0; q2 < 8; ++q2)
      if (mp.cg[s * 8 + q2] == c2) acc = acc + Zcc[s * 64 + q * 8 + q2];
  }
  Kcc[t] = acc;
}

hipError_t launch_setup3(Problem& p, cd* E, cd* work) {
  Three& T = *p.t3;
  T.g.alpha = p.alpha;
  T.g.rshift = p.rshift ? 1 : 0;
  const Geo3 g = T.g;
  const Maps3 mp = T.maps();
  hipStream_t st = p.ctx->stream;
  const int64_t NR2 = (int64_t)g.NR * g.NR;
  const bool s32 = p.s32();
  hipLaunchKernelGGL(k3_build_E, dim3(nb256(NR2), g.nsub), dim3(256), 0, st, g, (const int*)T.rl, E);
  hipError_t e = gj_range(g.NR, 0, g.nI, E, NR2, work, GJW, g.nsub, st);
  if (e != hipSuccess) return e;
  const dim3 gD(nb256((int64_t)g.ND * g.ND), g.nsub), gR(nb256(NR2), g.nsub);
  if (s32) hipLaunchKernelGGL(k3_take<cf>, gD, dim3(256), 0, st, (const cd*)E, g.NR, g.nI, g.ND, (cf*)T.Sbb);
  else hipLaunchKernelGGL(k3_take<cd>, gD, dim3(256), 0, st, (const cd*)E, g.NR, g.nI, g.ND, (cd*)T.Sbb);
  if ((e = gj_range(g.NR, g.nI, g.NR, E, NR2, work, GJW, g.nsub, st)) != hipSuccess) return e;
  if (s32) {
    hipLaunchKernelGGL(k3_take<cf>, gR, dim3(256), 0, st, (const cd*)E, g.NR, 0, g.NR, (cf*)T.Zinv);
    hipLaunchKernelGGL(k3_take<cf>, gD, dim3(256), 0, st, (const cd*)E, g.NR, g.nI, g.ND, (cf*)T.Sinv);
  } else {
    hipLaunchKernelGGL(k3_take<cd>, gR, dim3(256), 0, st, (const cd*)E, g.NR, 0, g.NR, (cd*)T.Zinv);
    hipLaunchKernelGGL(k3_take<cd>, gD, dim3(256), 0, st, (const cd*)E, g.NR, g.nI, g.ND, (cd*)T.Sinv);
  }
  hipLaunchKernelGGL(k3_phi, dim3(nb256(g.NR * 8), g.nsub), dim3(256), 0, st, g, mp, (const cd*)E, T.PhiFull);
  const dim3 gP(nb256(g.ND * 8), g.nsub);
  if (s32) hipLaunchKernelGGL(k3_phi_delta<cf>, gP, dim3(256), 0, st, g, (const cd*)T.PhiFull, (cf*)T.Phi);
  else hipLaunchKernelGGL(k3_phi_delta<cd>, gP, dim3(256), 0, st, g, (const cd*)T.PhiFull, (cd*)T.Phi);
  hipLaunchKernelGGL(k3_zcc, dim3(g.nsub), dim3(64), 0, st, g, mp, (const cd*)T.PhiFull, T.Zcc);
  const int64_t nc2 = (int64_t)g.nC * g.nC;
  hipLaunchKernelGGL(k3_coarse_assemble, dim3(nb256(nc2)), dim3(256), 0, st, g, mp, (const cd*)T.Zcc, p.Kcc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(p.Kinv, p.Kcc, sizeof(cd) * nc2, hipMemcpyDeviceToDevice, st)) != hipSuccess) return e;
  return invert_dense(g.nC, p.Kinv, work, st);
}

// ----------------------------------------------------------------- solve --
//
// Up to R3 = NRMAX right-hand sides run together: per-subdomain kernels read
// each operator once for all of them (R3 accumulators per row), vector kernels
// take the right-hand side from blockIdx.y.  Buffers are r-major with the
// strides of Str3.
struct Str3 {
  int64_t f;    // free-node vectors (input f, output x)
  int64_t t;    // local r vectors T: nsub NR
  int64_t y;    // local Delta vectors Y: nsub ND
  int64_t w;    // corner terms Wc: nsub 8
  int64_t c;    // coarse vectors: nC
  int64_t mu;   // interface vectors: nmu
};

// Local right-hand side at r position p for right-hand side r: f / mult
// (conj: of conj f); mode 1 subtracts Z_rc B_c u_c and B_r^T mu.
__device__ inline cd local_rhs(const Geo3& g, const Maps3& mp, int s, int p, const cd* f, int conj, int mode,
                               const cd* uc, const cd* mu) {
  const int l = mp.rl[s * g.NR + p];
  if (l < 0) return cd{0.0, 0.0};
  int a, b, c;
  g.loc(l, a, b, c);
  cd v = f[g.freeidx(s, a, b, c)];
  if (conj) v.y = -v.y;
  v = (1.0 / g.mult(a, b, c)) * v;
  if (mode == 1) {
    for (int q = 0; q < 8; ++q) {
      const int cq = mp.cg[s * 8 + q];
      if (cq < 0) continue;
      const cd z = g.zloc(l, g.vertex(q));  // zero unless l lies in the vertex's element
      if (z.x != 0.0 || z.y != 0.0) v = v - z * uc[cq];
    }
    if (p >= g.nI) {
      const int base = (s * g.ND + p - g.nI) * 3;
      for (int j = 0; j < 3; ++j) {
        const int k = mp.dmu[base + j];
        if (k >= 0) v = v - (double)mp.dsg[base + j] * mu[k];
      }
    }
  }
  return v;
}

// Full sweeps T_s,r = Z_rr^-1 f~_s,r (one workgroup per subdomain, a thread
// per row; Z_rr^-1 is symmetric, so row i is read as column i: coalesced, and
// once for all nr right-hand sides).  mode 0 also gives the subdomain's corner
// terms Wc[s][q] = f_q / 8 - (Phi^T f~)_q of f_c*.
template <class TS, int U>
__global__ void __launch_bounds__(1024) k3_sweep(Geo3 g, Maps3 mp, Str3 st, int nr, const TS* __restrict__ Zinv,
                                                 const cd* PhiFull, const cd* f, int conj, int mode,
                                                 const cd* uc, const cd* mu, cd* T, cd* Wc) {
  extern __shared__ cd ft[];  // [NR][R3]
  const int s = blockIdx.x, NR = g.NR;
  for (int t = threadIdx.x; t < NR * R3; t += blockDim.x) {
    const int p = t / R3, r = t % R3;
    ft[t] = r < nr ? local_rhs(g, mp, s, p, f + r * st.f, conj, mode, uc + r * st.c, mu + r * st.mu)
                   : cd{0.0, 0.0};
  }
  __syncthreads();
  const TS* Z = Zinv + (size_t)s * NR * NR;
  for (int i = threadIdx.x; i < NR; i += blockDim.x) {
    cd y[R3];
    symcol_r3<U>(Z, NR, NR, i, ft, y);
#pragma unroll
    for (int r = 0; r < R3; ++r)
      if (r < nr) T[r * st.t + (size_t)s * NR + i] = y[r];
  }
  if (mode == 0) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (wv < 8) {
      const int q = wv;
      cd acc[R3];
#pragma unroll
      for (int r = 0; r < R3; ++r) acc[r] = cd{0.0, 0.0};
      for (int p = lane; p < NR; p += 64) {
        const cd ph = PhiFull[((size_t)s * NR + p) * 8 + q];
#pragma unroll
        for (int r = 0; r < R3; ++r) fma_acc(acc[r], ph, ft[p * R3 + r]);
      }
#pragma unroll
      for (int r = 0; r < R3; ++r) acc[r] = wsum(acc[r]);
      if (lane == 0) {
        const bool corner = mp.cg[s * 8 + q] >= 0;
        int a = 0, b = 0, c = 0;
        g.loc(g.vertex(q), a, b, c);
#pragma unroll
        for (int r = 0; r < R3; ++r) {
          if (r >= nr) continue;
          cd v{0.0, 0.0};
          if (corner) {
            cd fv = f[r * st.f + g.freeidx(s, a, b, c)];
            if (conj) fv.y = -fv.y;
            v = 0.125 * fv - acc[r];  // a vertex is shared by 8 subdomains
          }
          Wc[r * st.w + s * 8 + q] = v;
        }
      }
    }
  }
}

// Interface product on one subdomain for nr right-hand sides: xs = B_r^T x on
// its Delta nodes (scaled by 1 / multiplicity when `scale`), Y_s = Mat xs,
// Wc_s = Phi^T xs; Mat is read once for all of them.
template <class TS, int U>
__global__ void __launch_bounds__(1024) k3_local(Geo3 g, Maps3 mp, Str3 st, int nr, const TS* __restrict__ Mat,
                                                 const TS* __restrict__ Phi, int scale, const cd* x, int64_t xr,
                                                 cd* Y, cd* Wc) {
  extern __shared__ cd xs[];  // [ND][R3]
  const int s = blockIdx.x, ND = g.ND, nd = mp.nds[s];
  for (int i = threadIdx.x; i < ND; i += blockDim.x) {
    cd v[R3];
#pragma unroll
    for (int r = 0; r < R3; ++r) v[r] = cd{0.0, 0.0};
    if (i < nd) {
      const int base = (s * ND + i) * 3;
      for (int j = 0; j < 3; ++j) {
        const int k = mp.dmu[base + j];
        if (k < 0) continue;
        const double sg = mp.dsg[base + j];
#pragma unroll
        for (int r = 0; r < R3; ++r)
          if (r < nr) v[r] = v[r] + sg * x[r * xr + k];
      }
      if (scale) {
        int a, b, c;
        g.loc(mp.rl[s * g.NR + g.nI + i], a, b, c);
        const double w = 1.0 / g.mult(a, b, c);
#pragma unroll
        for (int r = 0; r < R3; ++r) v[r] = w * v[r];
      }
    }
#pragma unroll
    for (int r = 0; r < R3; ++r) xs[i * R3 + r] = v[r];
  }
  __syncthreads();
  if (Mat) {
    const TS* A = Mat + (size_t)s * ND * ND;
    for (int i = threadIdx.x; i < nd; i += blockDim.x) {
      cd y[R3];
      symcol_r3<U>(A, ND, nd, i, xs, y);
#pragma unroll
      for (int r = 0; r < R3; ++r)
        if (r < nr) Y[r * st.y + (size_t)s * ND + i] = y[r];
    }
  }
  if (Phi) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (wv < 8) {
      cd acc[R3];
#pragma unroll
      for (int r = 0; r < R3; ++r) acc[r] = cd{0.0, 0.0};
      for (int i = lane; i < nd; i += 64) {
        const cd ph = ld64(Phi[((size_t)s * ND + i) * 8 + wv]);
#pragma unroll
        for (int r = 0; r < R3; ++r) fma_acc(acc[r], ph, xs[i * R3 + r]);
      }
#pragma unroll
      for (int r = 0; r < R3; ++r) acc[r] = wsum(acc[r]);
      if (lane == 0) {
#pragma unroll
        for (int r = 0; r < R3; ++r)
          if (r < nr) Wc[r * st.w + s * 8 + wv] = acc[r];
      }
    }
  }
}

// out[c] = add[c] + sum of Wc over the corner's owners (fixed order); r = blockIdx.y
__global__ void k3_corner_sum(int nC, Str3 st, const int* cown, const cd* Wc, const cd* add, cd* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (c >= nC) return;
  cd acc = add ? add[r * st.c + c] : cd{0.0, 0.0};
  for (int o = 0; o < 8; ++o) {
    const int own = cown[c * 8 + o];
    if (own >= 0) acc = acc + Wc[r * st.w + own];
  }
  out[r * st.c + c] = acc;
}

// y_r = A x_r (n x n, FP64) for the nr right-hand sides together (A read
// once), one wave per row
__global__ void k3_dense_mv(int n, int64_t stride, int nr, const cd* A, const cd* x, cd* y) {
  const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= n) return;
  cd acc[R3];
#pragma unroll
  for (int r = 0; r < R3; ++r) acc[r] = cd{0.0, 0.0};
  // four strides' loads issued before their multiply-adds; each right-hand
  // side's terms in the order j = lane, lane + 64, ...
  int j = lane;
  for (; j + 192 < n; j += 256) {
    cd a[4], xv[4][R3];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = A[(size_t)row * n + j + 64 * u];
#pragma unroll
      for (int r = 0; r < R3; ++r) xv[u][r] = r < nr ? x[r * stride + j + 64 * u] : cd{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int r = 0; r < R3; ++r) fma_acc(acc[r], a[u], xv[u][r]);
  }
  for (; j < n; j += 64) {
    const cd a = A[(size_t)row * n + j];
#pragma unroll
    for (int r = 0; r < R3; ++r)
      if (r < nr) fma_acc(acc[r], a, x[r * stride + j]);
  }
#pragma unroll
  for (int r = 0; r < R3; ++r) {
    if (r >= nr) continue;
    const cd v = wsum(acc[r]);
    if (lane == 0) y[r * stride + row] = v;
  }
}

// Y[r][s ystride + d] += phis (Phi_s[d] . u_c(B_c s)) for the Delta nodes d < nds[s]
// of subdomain s = blockIdx.x and every right-hand side r < nr: the subdomain's
// eight corner values of u_c staged in LDS once (zero for a Dirichlet slot,
// which adds nothing), the same sums in the same order as the corner term of
// k3_scatter, added once per Delta node instead of once per multiplier side.
template <class TS>
__global__ void __launch_bounds__(256) k3_phi_add(Geo3 g, Maps3 mp, Str3 st, int nr, const TS* Phi, const cd* uc,
                                                  double phis, cd* Y, int64_t yr, int ystride) {
  __shared__ cd ucs[8][R3];
  const int s = blockIdx.x;
  if (threadIdx.x < 8 * R3) {
    const int q = threadIdx.x / R3, r = threadIdx.x % R3;
    const int c = mp.cg[s * 8 + q];
    ucs[q][r] = (c >= 0 && r < nr) ? uc[r * st.c + c] : cd{0.0, 0.0};
  }
  __syncthreads();
  const int nd = mp.nds[s];
  for (int d = threadIdx.x; d < nd; d += blockDim.x) {
    const TS* ph = Phi + ((size_t)s * g.ND + d) * 8;
    cd acc[R3];
#pragma unroll
    for (int r = 0; r < R3; ++r) acc[r] = cd{0.0, 0.0};
#pragma unroll 4
    for (int q = 0; q < 8; ++q) {
      const cd pq = ld64(ph[q]);
#pragma unroll
      for (int r = 0; r < R3; ++r) fma_acc(acc[r], pq, ucs[q][r]);
    }
#pragma unroll
    for (int r = 0; r < R3; ++r) {
      if (r >= nr) break;
      cd* y = Y + r * yr + (size_t)s * ystride + d;
      *y = *y + phis * acc[r];
    }
  }
}

// Per multiplier k with owners (s+, d+) and (s-, d-), right-hand side r = blockIdx.y:
//   out_k = sc_k (v+ - v-),  v = Y[s ystride + yoff + d] + phis (Phi_s[d] . u_c(B_c s))
// with sc_k = 1 / multiplicity when `scale`, else 1.  Y has right-hand-side
// stride yr, out stride orr.
template <class TS>
__global__ void k3_scatter(Geo3 g, Maps3 mp, Str3 st, const cd* Y, int64_t yr, int ystride, int yoff,
                           const TS* Phi, const cd* uc, double phis, int scale, cd* out, int64_t orr) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (k >= g.nmu) return;
  Y += r * yr;
  uc += r * st.c;
  cd acc{0.0, 0.0};
  int own = 0;
  for (int side = 0; side < 2; ++side) {
    own = mp.muown[2 * k + side];
    const int s = own / g.ND, dl = own % g.ND;
    cd v = Y[(size_t)s * ystride + yoff + dl];
    if (Phi) {
      cd pc{0.0, 0.0};
      for (int q = 0; q < 8; ++q) {
        const int cq = mp.cg[s * 8 + q];
        if (cq >= 0) fma_acc(pc, ld64(Phi[((size_t)s * g.ND + dl) * 8 + q]), uc[cq]);
      }
      v = v + phis * pc;
    }
    acc = side == 0 ? acc + v : acc - v;
  }
  if (scale) {
    const int s = own / g.ND, dl = own % g.ND;
    int a, b, c;
    g.loc(mp.rl[s * g.NR + g.nI + dl], a, b, c);
    acc = (1.0 / g.mult(a, b, c)) * acc;
  }
  out[r * orr + k] = acc;
}

// Primal solution on the free nodes: corners from u_c, every other node the
// average of its subdomain copies (conj: conjugated); r = blockIdx.y
__global__ void k3_assemble(Geo3 g, Maps3 mp, Str3 st, const cd* T, const cd* uc, int conj, cd* x) {
  const int64_t n1 = g.N - 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n1 * n1 * n1) return;
  const int r = blockIdx.y;
  T += r * st.t;
  uc += r * st.c;
  const int gi = (int)(t % n1) + 1, gj = (int)((t / n1) % n1) + 1, gk = (int)(t / (n1 * n1)) + 1;
  const int m = g.m, P = g.P;
  cd v{0.0, 0.0};
  if (gi % m == 0 && gj % m == 0 && gk % m == 0) {
    v = uc[(gi / m - 1) + (P - 1) * ((gj / m - 1) + (P - 1) * (gk / m - 1))];
  } else {
    // owning subdomains along each axis: one, or two when on a subdomain face
    const int ni = gi % m ? 1 : 2, nj = gj % m ? 1 : 2, nk = gk % m ? 1 : 2;
    int cnt = 0;
    for (int ai = 0; ai < ni; ++ai)
      for (int aj = 0; aj < nj; ++aj)
        for (int ak = 0; ak < nk; ++ak) {
          const int sx = gi / m - (ni == 2 ? 1 - ai : 0), sy = gj / m - (nj == 2 ? 1 - aj : 0),
                    sz = gk / m - (nk == 2 ? 1 - ak : 0);
          const int s = sx + P * (sy + P * sz);
          const int l = (gi - sx * m) + g.ml * ((gj - sy * m) + g.ml * (gk - sz * m));
          v = v + T[(size_t)s * g.NR + mp.rpos[s * g.nl + l]];
          ++cnt;
        }
    v = (1.0 / cnt) * v;
  }
  if (conj) v.y = -v.y;
  x[r * st.f + t] = v;
}

// ---- Krylov vector kernels (length n, FP64 complex; right-hand side r =
// blockIdx.y: vectors at + r * vr, coefficients at + r * hr, partial sums at
// + r * pr) ----
// part[i * np + p] = sum over the entries of wave p (np = 4 gridDim.x waves) of
// conj(V_i) w, i < nv: per-wave partial sums, no workgroup barrier
__global__ void __launch_bounds__(256) k3_dots(int64_t n, int nv, const cd* V, int64_t vs, int64_t vr,
                                               const cd* w, int64_t wr, cd* part, int64_t pr) {
  const int r = blockIdx.y;
  V += r * vr;
  w += r * wr;
  part += r * pr;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool in = t < n;
  const cd wv = in ? w[t] : cd{0.0, 0.0};
  const int lane = threadIdx.x & 63;
  const int64_t np = 4 * (int64_t)gridDim.x, pw = 4 * (int64_t)blockIdx.x + (threadIdx.x >> 6);
  int i = 0;
  for (; i + 3 < nv; i += 4) {
    cd v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = in ? V[(i + u) * vs + t] : cd{0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      cd a{0.0, 0.0};
      fma_conj_acc(a, v[u], wv);
      a = wsum(a);
      if (lane == 0) part[(int64_t)(i + u) * np + pw] = a;
    }
  }
  for (; i < nv; ++i) {
    cd a{0.0, 0.0};
    if (in) fma_conj_acc(a, V[i * vs + t], wv);
    a = wsum(a);
    if (lane == 0) part[(int64_t)i * np + pw] = a;
  }
}
// h[i] = sum_b part[i * nb + b] in a fixed order (block x = i, y = r)
__global__ void __launch_bounds__(256) k3_reduce(int nb, const cd* part, int64_t pr, cd* h, int64_t hr) {
  __shared__ cd sh[256];
  const int i = blockIdx.x, r = blockIdx.y;
  part += r * pr;
  cd a{0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += 256) a = a + part[(int64_t)i * nb + b];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) h[r * hr + i] = sh[0];
}
// w -= sum_i h[i] V_i ; npart[block] = sum |w|^2 over the block
__global__ void __launch_bounds__(256) k3_axpy(int64_t n, int nv, const cd* V, int64_t vs, int64_t vr,
                                               const cd* h, int64_t hr, cd* w, int64_t wr, double* npart,
                                               int64_t nr_) {
  __shared__ double sh[4];
  const int r = blockIdx.y;
  V += r * vr;
  h += r * hr;
  w += r * wr;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double q = 0.0;
  if (t < n) {
    cd a = w[t];
#pragma unroll 4
    for (int i = 0; i < nv; ++i) a = a - h[i] * V[i * vs + t];
    w[t] = a;
    q = abs2(a);
  }
  q = wsum(q);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = q;
  __syncthreads();
  if (threadIdx.x == 0) npart[r * nr_ + blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}
// out[r * hr] = sum of npart[r * pr + 0 .. nb) in a fixed order (as a double)
__global__ void __launch_bounds__(256) k3_sum(int nb, const double* npart, int64_t pr, cd* out, int64_t hr) {
  __shared__ double sh[256];
  const int r = blockIdx.x;
  double a = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) a += npart[r * pr + b];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r * hr] = cd{sh[0], 0.0};
}
// v = w / sqrt(nrm) (zero when the norm is zero); nrm of r at nrm + r * hr
__global__ void k3_normalize(int64_t n, const cd* w, int64_t wr, const cd* nrm, int64_t hr, cd* v, int64_t vr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (t >= n) return;
  const double q = nrm[r * hr].x;
  const double s = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
  v[r * vr + t] = s * w[r * wr + t];
}
// out = sum_{i < nv[r]} y[i] V_i
__global__ void k3_combine(int64_t n, const int* nv, const cd* V, int64_t vs, int64_t vr, const cd* y,
                           int64_t hr, cd* out, int64_t orr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (t >= n) return;
  V += r * vr;
  y += r * hr;
  cd a{0.0, 0.0};
  for (int i = 0; i < nv[r]; ++i) fma_acc(a, y[i], V[i * vs + t]);
  out[r * orr + t] = a;
}

// ---- Givens state of the host-loop GMRES on the device (krylov3.h) ----
namespace {
struct GmView {
  cd *H, *c, *s, *g, *beta;  // H column j at H + j (K + 1)
  __device__ GmView(cd* gs, int K, int r) {
    H = gs + r * gs_len(K);
    c = H + (int64_t)(K + 1) * K;
    s = c + K;
    g = s + K;
    beta = g + K + 1;
  }
};
__device__ inline void gm_live(int nr, int* gi) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int any = 0;
    for (int r = 0; r < nr; ++r) any |= gi[2 * r];
    gi[2 * NRMAX] = any;
  }
}
}  // namespace

__global__ void k3_gm_init(int nr, int K, const cd* hd, int64_t hr, int ks, cd* gs, int* gi) {
  const int r = threadIdx.x;
  if (r < nr) {
    GmView v(gs, K, r);
    const double b = sqrt(hd[r * hr + 2 * ks].x);
    v.beta[0] = cd{b, 0.0};
    for (int i = 0; i <= K; ++i) v.g[i] = cd{i == 0 ? b : 0.0, 0.0};
    gi[2 * r] = b > 0.0 ? 1 : 0;
    gi[2 * r + 1] = 0;
  }
  if (threadIdx.x == 0) gi[2 * NRMAX + 1] = 0;
  gm_live(nr, gi);
}

// Column j of right-hand side r = blockIdx.x (one wave): h = pass-0 + pass-1
// coefficients and ||w||, staged with the previous rotations in LDS by the
// wave; lane 0 applies the rotations [c_i s_i; -conj(s_i) c_i] (c_i real) and
// forms the one that zeroes ||w||; the wave writes the column back.  The last
// workgroup to finish publishes "any active" (a counter of finished workgroups
// in gi[2 NRMAX + 1], reset by that workgroup).
__global__ void k3_gm_step(int nr, int K, int j, int kmax, double tol, const cd* hd, int64_t hr, int ks, cd* gs,
                           int* gi) {
  extern __shared__ cd lm[];  // Hj (K + 1), c (K), s (K)
  const int r = blockIdx.x, lane = threadIdx.x;
  const bool act = gi[2 * r] != 0;
  if (act) {
    GmView v(gs, K, r);
    cd* Hj = lm;
    cd* c = lm + (K + 1);
    cd* sn = c + K;
    const cd* h = hd + r * hr;
    for (int i = lane; i <= j; i += 64) Hj[i] = h[i] + h[ks + i];
    for (int i = lane; i < j; i += 64) {
      c[i] = v.c[i];
      sn[i] = v.s[i];
    }
    __syncthreads();
    if (lane == 0) {
      const double hn = sqrt(h[2 * ks].x);
      for (int i = 0; i < j; ++i) {
        const cd a = Hj[i], b = Hj[i + 1];
        Hj[i] = c[i] * a + sn[i] * b;
        Hj[i + 1] = c[i] * b - conj(sn[i]) * a;
      }
      const cd a = Hj[j];
      const double ra = sqrt(abs2(a)), rho = sqrt(ra * ra + hn * hn);
      cd cj, sj;
      if (ra == 0.0) {
        cj = cd{0.0, 0.0};
        sj = cd{1.0, 0.0};
      } else {
        cj = cd{ra / rho, 0.0};
        sj = (hn / (ra * rho)) * a;
      }
      v.c[j] = cj;
      v.s[j] = sj;
      Hj[j] = cj * a + hn * sj;
      const cd gj = v.g[j];
      v.g[j + 1] = -1.0 * (conj(sj) * gj);
      v.g[j] = cj * gj;
      gi[2 * r + 1] = j + 1;
      if (sqrt(abs2(v.g[j + 1])) <= tol * v.beta[0].x || !(hn > 0.0) || j + 1 >= kmax) gi[2 * r] = 0;
    }
    __syncthreads();
    cd* Hc = v.H + (int64_t)j * (K + 1);
    for (int i = lane; i <= j; i += 64) Hc[i] = Hj[i];
  }
  // the last workgroup to finish publishes whether any right-hand side is active
  __syncthreads();
  if (lane == 0) {
    __threadfence();
    const int done = atomicAdd(gi + 2 * NRMAX + 1, 1);
    if (done == nr - 1) {
      __threadfence();
      int any = 0;
      for (int q = 0; q < nr; ++q) any |= __hip_atomic_load(gi + 2 * q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      gi[2 * NRMAX] = any;
      gi[2 * NRMAX + 1] = 0;
    }
  }
}

// y_r = H_r^-1 g_r over its_r columns (right-hand side r = blockIdx.x, one wave):
// t = g in LDS; for i = m - 1 .. 0, lane 0 forms y_i = t_i / H_ii, then every
// t_c, c < i, takes -H_ic y_i.  The triangle is staged in LDS when it has at
// most mlds columns (packed by columns), else read from global memory.  Writes y
// to hd (the combination coefficients) and nvd_r = its_r.
__global__ void k3_gm_solve(int K, const cd* gs, const int* gi, cd* hd, int64_t hr, int* nvd, int mlds) {
  extern __shared__ cd lm[];  // triangle (mlds (mlds + 1) / 2), then t (K + 1)
  const int r = blockIdx.x, lane = threadIdx.x;
  GmView v(const_cast<cd*>(gs), K, r);
  const int m = gi[2 * r + 1];
  const bool inlds = m <= mlds;
  cd* tri = lm;
  cd* tv = lm + (size_t)mlds * (mlds + 1) / 2;
  if (inlds)
    for (int i = 0; i < m; ++i)
      for (int c = lane; c <= i; c += 64) tri[i * (i + 1) / 2 + c] = v.H[(int64_t)i * (K + 1) + c];
  for (int c = lane; c < m; c += 64) tv[c] = v.g[c];
  cd* y = hd + r * hr;
  __syncthreads();
  for (int i = m - 1; i >= 0; --i) {
    const cd hii = inlds ? tri[i * (i + 1) / 2 + i] : v.H[(int64_t)i * (K + 1) + i];
    const cd yi = cdiv(tv[i], hii);
    for (int c = lane; c < i; c += 64) {
      const cd hic = inlds ? tri[i * (i + 1) / 2 + c] : v.H[(int64_t)i * (K + 1) + c];
      tv[c] = tv[c] - hic * yi;
    }
    if (lane == 0) y[i] = yi;
    __syncthreads();
  }
  if (lane == 0) nvd[r] = m;
}

__global__ void k3_log(int* flags, int c, int q, int its) {
  flags[FLAG_ITS + c] = its;
  const int k = flags[FLAG_CNT + q];
  if (k < 16) flags[FLAG_LOG + 16 * q + k] = its;
  flags[FLAG_CNT + q] = k + 1;
  flags[3] += its;
  flags[4] += its;
}

namespace {

struct Ops3 {
  Problem& p;
  Three& T;
  Geo3 g;
  Maps3 mp;
  Str3 sr;
  hipStream_t st;
  bool s32;
  int nr;
  unsigned threads_local, threads_sweep;
  KBuf kb;  // Krylov buffers of the host-driven GMRES
  int64_t nmu;
  Ops3(Problem& pp, int nr_)
      : p(pp), T(*pp.t3), g(pp.t3->g), mp(pp.t3->maps()), st(pp.ctx->stream), s32(pp.s32()), nr(nr_) {
    kb = KBuf{T.V, T.hd, T.part, T.d, T.z, T.w, T.mu, T.npart, T.nvd, T.kalloc, T.gs, T.gi, T.gih};
    nmu = g.nmu;
    threads_local = (unsigned)std::min(1024, std::max(512, (g.ND + 63) / 64 * 64));
    threads_sweep = (unsigned)std::min(1024, std::max(512, (g.NR + 63) / 64 * 64));
    sr = Str3{pp.n_free, (int64_t)g.nsub * g.NR, (int64_t)g.nsub * g.ND, (int64_t)g.nsub * 8,
              (int64_t)std::max(g.nC, 1), (int64_t)g.nmu};
  }
  // interface products: eight (candidate 0) or four loads in flight per thread
  template <class TS>
  void local_t(const void* Mat, const void* Phi, int scale, const cd* x, int64_t xr, cd* Y, cd* Wc) {
    auto run = [&](int c) {
      if (c == 0)
        hipLaunchKernelGGL((k3_local<TS, 8>), dim3(g.nsub), dim3(threads_local), sizeof(cd) * g.ND * R3, st, g, mp,
                           sr, nr, (const TS*)Mat, (const TS*)Phi, scale, x, xr, Y, Wc);
      else
        hipLaunchKernelGGL((k3_local<TS, 4>), dim3(g.nsub), dim3(threads_local), sizeof(cd) * g.ND * R3, st, g, mp,
                           sr, nr, (const TS*)Mat, (const TS*)Phi, scale, x, xr, Y, Wc);
    };
    if (!Mat) {
      run(0);
      return;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    const TuneKey key{TUNE_K3_LOCAL, dev, g.ND, g.nsub, (int)sizeof(TS), nr};
    run(tune_choice(key, 2, 0, st, run));
  }
  void local(const void* Mat, const void* Phi, int scale, const cd* x, int64_t xr, cd* Y, cd* Wc) {
    if (s32) local_t<cf>(Mat, Phi, scale, x, xr, Y, Wc);
    else local_t<cd>(Mat, Phi, scale, x, xr, Y, Wc);
  }
  void scatter(const cd* Y, int64_t yr, int ystride, int yoff, bool phi, double phis, int scale, cd* out,
               int64_t orr) {
    const dim3 grid(nb256(g.nmu), nr);
    if (s32)
      hipLaunchKernelGGL(k3_scatter<cf>, grid, dim3(256), 0, st, g, mp, sr, Y, yr, ystride, yoff,
                         phi ? (const cf*)T.Phi : (const cf*)nullptr, (const cd*)T.uc, phis, scale, out, orr);
    else
      hipLaunchKernelGGL(k3_scatter<cd>, grid, dim3(256), 0, st, g, mp, sr, Y, yr, ystride, yoff,
                         phi ? (const cd*)T.Phi : (const cd*)nullptr, (const cd*)T.uc, phis, scale, out, orr);
  }
  // full sweeps: two (candidate 0) or four loads in flight per thread
  template <class TS>
  void sweep_t(const cd* f, int conj, int mode) {
    const size_t lds = sizeof(cd) * g.NR * R3;
    auto run = [&](int c) {
      if (c == 0)
        hipLaunchKernelGGL((k3_sweep<TS, 2>), dim3(g.nsub), dim3(threads_sweep), lds, st, g, mp, sr, nr,
                           (const TS*)T.Zinv, (const cd*)T.PhiFull, f, conj, mode, (const cd*)T.uc, (const cd*)T.mu,
                           T.T, T.Wc);
      else
        hipLaunchKernelGGL((k3_sweep<TS, 4>), dim3(g.nsub), dim3(threads_sweep), lds, st, g, mp, sr, nr,
                           (const TS*)T.Zinv, (const cd*)T.PhiFull, f, conj, mode, (const cd*)T.uc, (const cd*)T.mu,
                           T.T, T.Wc);
    };
    int dev = 0;
    (void)hipGetDevice(&dev);
    const TuneKey key{TUNE_K3_SWEEP, dev, g.NR, g.nsub, (int)sizeof(TS), nr * 2 + mode};
    run(tune_choice(key, 2, 0, st, run));
  }
  void sweep(const cd* f, int conj, int mode) {
    if (s32) sweep_t<cf>(f, conj, mode);
    else sweep_t<cd>(f, conj, mode);
  }
  // out = K_cc*^-1 (add + sum of Wc)
  void coarse(const cd* add, cd* out) {
    hipLaunchKernelGGL(k3_corner_sum, dim3(nb256(g.nC), nr), dim3(256), 0, st, g.nC, sr, (const int*)T.cown,
                       (const cd*)T.Wc, add, T.gc);
    hipLaunchKernelGGL(k3_dense_mv, dim3((g.nC + 3) / 4), dim3(256), 0, st, g.nC, sr.c, nr, (const cd*)p.Kinv,
                       (const cd*)T.gc, out);
  }
  // out = F_DP x (x and out with right-hand-side strides xr, orr)
  // (the corner term goes into the local products T.Y, scratch until the next
  // local product, once per Delta node; then a plain scatter)
  void apply_F(const cd* x, int64_t xr, cd* out, int64_t orr) {
    local(T.Sinv, T.Phi, 0, x, xr, T.Y, T.Wc);
    coarse(nullptr, T.uc);
    if (s32)
      hipLaunchKernelGGL(k3_phi_add<cf>, dim3(g.nsub), dim3(256), 0, st, g, mp, sr, nr, (const cf*)T.Phi,
                         (const cd*)T.uc, 1.0, T.Y, sr.y, g.ND);
    else
      hipLaunchKernelGGL(k3_phi_add<cd>, dim3(g.nsub), dim3(256), 0, st, g, mp, sr, nr, (const cd*)T.Phi,
                         (const cd*)T.uc, 1.0, T.Y, sr.y, g.ND);
    scatter(T.Y, sr.y, g.ND, 0, false, 0.0, 0, out, orr);
  }
  // out = W B_r S_bb B_r^T W x
  void apply_P(const cd* x, int64_t xr, cd* out, int64_t orr) {
    local(T.Sbb, nullptr, 1, x, xr, T.Y, nullptr);
    scatter(T.Y, sr.y, g.ND, 0, false, 0.0, 1, out, orr);
  }
  // d = sum B_r (Z_rr^-1 f_r)|Delta - F_rc K_cc*^-1 f_c*  (leaves f_c* in fcs)
  void rhs(const cd* f, int conj) {
    sweep(f, conj, 0);
    hipLaunchKernelGGL(k3_corner_sum, dim3(nb256(g.nC), nr), dim3(256), 0, st, g.nC, sr, (const int*)T.cown,
                       (const cd*)T.Wc, (const cd*)nullptr, T.fcs);
    hipLaunchKernelGGL(k3_dense_mv, dim3((g.nC + 3) / 4), dim3(256), 0, st, g.nC, sr.c, nr, (const cd*)p.Kinv,
                       (const cd*)T.fcs, T.uc);
    scatter(T.T, sr.t, g.NR, g.nI, true, -1.0, 0, T.d, sr.mu);
  }
};

}  // namespace

hipError_t feti3(Problem& p, int nr, const cd* f, cd* x, int conj, double tol, int kmax, int* its) {
  Ops3 o(p, nr);
  Three& T = o.T;
  o.rhs(f, conj);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = gmres_host(o, tol, kmax, its)) != hipSuccess) return e;
  // u_c = K_cc*^-1 (f_c* + F_rc^T mu), u_r = Z_rr^-1 (f_r - Z_rc B_c u_c - B_r^T mu)
  o.local(nullptr, T.Phi, 0, T.mu, o.sr.mu, nullptr, T.Wc);
  o.coarse(T.fcs, T.uc);
  o.sweep(f, conj, 1);
  const int64_t n1 = o.g.N - 1;
  hipLaunchKernelGGL(k3_assemble, dim3(nb256(n1 * n1 * n1), nr), dim3(256), 0, o.st, o.g, o.mp, o.sr,
                     (const cd*)T.T, (const cd*)T.uc, conj, x);
  return hipGetLastError();
}

hipError_t launch_log3(Problem& p, int c, int q, int its) {
  hipLaunchKernelGGL(k3_log, dim3(1), dim3(1), 0, p.ctx->stream, p.flags, c, q, its);
  return hipGetLastError();
}

hipError_t interface3(Problem& p, char which, const cd* x, cd* y) {
  Ops3 o(p, 1);
  const int64_t n = o.g.nmu;
  if (which == 'F') o.apply_F(x, n, y, n);
  else if (which == 'P') o.apply_P(x, n, y, n);
  else {
    o.rhs(x, 0);
    hipError_t e = hipMemcpyAsync(y, o.T.d, sizeof(cd) * o.g.nmu, hipMemcpyDeviceToDevice, o.st);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace sfdp

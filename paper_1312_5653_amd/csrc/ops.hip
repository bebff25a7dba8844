// FP64 operators on the free-node grid of an instance (Sec. 2 matrices),
// matrix free: on a uniform grid the Q1 stiffness and mass rows are the
// 9-point stencils  K = k1 (x) m1 + m1 (x) k1,  M = m1 (x) m1  (2D; in 3D the
// 27-point Kronecker sums of three factors) with the 1D P1 rows
// k1 = (1/h)(-1, 2, -1), m1 = (h/6)(1, 4, 1).  K_c couples free nodes to their
// boundary neighbours with the same stencil.
//
// The KKT residual (Sec. 2 KKT system) of (y, u, lam):
//   r1 = M ybar - M y - K lam,  r2 = -(beta M u - M lam),  r3 = -Kc yc - K y + M u,
// reduced deterministically (fixed-order two-pass sums) to ||r|| / ||b||.
#include "common.h"

#include <mutex>

namespace sfdp {

struct Sten {
  double k[3], m[3];  // offsets -1, 0, +1
};
__host__ __device__ inline Sten make_sten(double h) {
  Sten s;
  s.k[0] = -1.0 / h; s.k[1] = 2.0 / h; s.k[2] = -1.0 / h;
  s.m[0] = h / 6.0; s.m[1] = 4.0 * h / 6.0; s.m[2] = h / 6.0;
  return s;
}

// Stencil neighbourhoods.  The Q = 9 (2D) or 27 (3D) neighbours of a free node at
// 1-based grid coordinates (i, j, k) (k = 0 in 2D) are numbered
// q = (di + 1) + 3 (dj + 1) + 9 (dk + 1), the order every stencil sum below runs in.
// The gathers issue all of a node's loads unconditionally -- a neighbour outside
// the free set reads the node itself and is then replaced by zero -- so the loads
// of a stencil are in flight together instead of one round trip after another;
// a zero in place of a skipped neighbour leaves every sum unchanged.
struct Field {
  const double* x;   // free values, stride n_free
  const double* xc;  // boundary values or null
};
template <int D>
struct Nb {
  static constexpr int Q = D == 3 ? 27 : 9;
};
template <int D>
__device__ inline void nb_off(int q, int& di, int& dj, int& dk) {
  di = q % 3 - 1;
  dj = (q / 3) % 3 - 1;
  dk = D == 3 ? q / 9 - 1 : 0;
}
template <int D>
__device__ inline bool nb_free(int N, int i, int j, int k, int q) {
  int di, dj, dk;
  nb_off<D>(q, di, dj, dk);
  const unsigned n1 = (unsigned)(N - 1);
  bool f = (unsigned)(i + di - 1) < n1 && (unsigned)(j + dj - 1) < n1;
  if (D == 3) f = f && (unsigned)(k + dk - 1) < n1;
  return f;
}
// free index t -> grid coordinates; 32-bit divisions while the index fits
__device__ inline void ij2(int64_t t, int N, int& i, int& j) {
  const int n1 = N - 1;
  if (t <= 0x7fffffff) {
    const unsigned u = (unsigned)t;
    i = (int)(u % (unsigned)n1) + 1;
    j = (int)(u / (unsigned)n1) + 1;
  } else {
    i = (int)(t % n1) + 1;
    j = (int)(t / n1) + 1;
  }
}
__device__ inline void ijk3(int64_t t, int N, int& i, int& j, int& k) {
  const int64_t n1 = N - 1;
  if (t <= 0x7fffffff) {
    const unsigned u = (unsigned)t, m = (unsigned)n1, w = u / m;
    i = (int)(u - w * m) + 1;
    j = (int)(w % m) + 1;
    k = (int)(w / m) + 1;
  } else {
    i = (int)(t % n1) + 1;
    j = (int)((t / n1) % n1) + 1;
    k = (int)(t / (n1 * n1)) + 1;
  }
}
template <int D>
__device__ inline void node_ijk(int64_t t, int N, int& i, int& j, int& k) {
  if (D == 3) ijk3(t, N, i, j, k);
  else { ij2(t, N, i, j); k = 0; }
}
// v[q] = x at free neighbour q, zero at boundary neighbours (t: the node's free index)
template <int D, class T>
__device__ inline void gather_free(const T* x, int N, int i, int j, int k, int64_t t, T (&v)[Nb<D>::Q]) {
  const int64_t n1 = N - 1;
#pragma unroll
  for (int q = 0; q < Nb<D>::Q; ++q) {
    int di, dj, dk;
    nb_off<D>(q, di, dj, dk);
    const bool f = nb_free<D>(N, i, j, k, q);
    const T a = x[f ? t + di + n1 * (dj + n1 * dk) : t];
    v[q] = f ? a : T{};
  }
}
// a node with at least one boundary neighbour
template <int D>
__device__ inline bool near_bdry(int N, int i, int j, int k) {
  bool e = i == 1 || j == 1 || i == N - 1 || j == N - 1;
  if (D == 3) e = e || k == 1 || k == N - 1;
  return e;
}
// v[q] = xc[full2bdry[neighbour q]] at the boundary neighbours (free entries kept);
// full2bdry covers the full grid, (N+1)^D nodes, so its loads are in range for every q
template <int D>
__device__ inline void gather_bdry(const double* xc, const int* f2b, int N, int i, int j, int k,
                                   double (&v)[Nb<D>::Q]) {
  const int64_t n1 = N + 1;
  int b[Nb<D>::Q];
#pragma unroll
  for (int q = 0; q < Nb<D>::Q; ++q) {
    int di, dj, dk;
    nb_off<D>(q, di, dj, dk);
    b[q] = f2b[(i + di) + n1 * ((j + dj) + n1 * (int64_t)(k + dk))];
  }
#pragma unroll
  for (int q = 0; q < Nb<D>::Q; ++q) {
    const bool f = nb_free<D>(N, i, j, k, q);
    const double a = xc[f ? 0 : b[q]];
    if (!f) v[q] = a;
  }
}
// stencil weights of neighbour q: K = k1 (x) m1 [(x) m1] + ..., M = m1 (x) m1 [(x) m1]
template <int D>
__device__ inline void nb_weights(const Sten& st, int q, double& wk, double& wm) {
  int di, dj, dk;
  nb_off<D>(q, di, dj, dk);
  const double mi = st.m[di + 1], mj = st.m[dj + 1];
  if (D == 3) {
    const double mk = st.m[dk + 1];
    wk = st.k[di + 1] * mj * mk + mi * st.k[dj + 1] * mk + mi * mj * st.k[dk + 1];
    wm = mi * mj * mk;
  } else {
    wk = st.k[di + 1] * mj + mi * st.k[dj + 1];
    wm = mi * mj;
  }
}
// Stencil kernels: 256-thread blocks, one instantiation per dimension (the 2D
// and 3D gathers need very different register budgets).
#define STENCIL_BOUNDS __launch_bounds__(256)

// K x + Kc xc (xc may be null) and M x at free node t = (i, j, k)
template <int D>
__device__ inline void stencil_KM(const Sten& st, int N, const int* f2b, const Field& f, int i, int j, int k,
                                  int64_t t, double& Kx, double& Mx) {
  double v[Nb<D>::Q];
  gather_free<D>(f.x, N, i, j, k, t, v);
  if (f.xc && near_bdry<D>(N, i, j, k)) gather_bdry<D>(f.xc, f2b, N, i, j, k, v);
  Kx = 0.0;
  Mx = 0.0;
#pragma unroll
  for (int q = 0; q < Nb<D>::Q; ++q) {
    double wk, wm;
    nb_weights<D>(st, q, wk, wm);
    Kx = fma(wk, v[q], Kx);
    Mx = fma(wm, v[q], Mx);
  }}
// K x_f, M x_f and, with ABS, |K| |x_f| and |M| |x_f| for F free-node fields
// (zero at boundary neighbours), neighbour by neighbour: one neighbour's address
// serves the F loads, so no per-neighbour offsets stay live between fields.
template <int D, int F, bool ABS>
__device__ inline void stencil_fields(const Sten& st, int N, int i, int j, int k, int64_t t,
                                      const double* const (&x)[F], double (&Kx)[F], double (&Mx)[F],
                                      double (&aKx)[F], double (&aMx)[F]) {
  const int64_t n1 = N - 1;
#pragma unroll
  for (int f = 0; f < F; ++f) Kx[f] = Mx[f] = aKx[f] = aMx[f] = 0.0;
#pragma unroll
  for (int q = 0; q < Nb<D>::Q; ++q) {
    int di, dj, dk;
    nb_off<D>(q, di, dj, dk);
    const bool fr = nb_free<D>(N, i, j, k, q);
    const int64_t idx = fr ? t + di + n1 * (dj + n1 * dk) : t;
    double wk, wm;
    nb_weights<D>(st, q, wk, wm);
#pragma unroll
    for (int f = 0; f < F; ++f) {
      const double a = x[f][idx];
      const double v = fr ? a : 0.0;
      Kx[f] = fma(wk, v, Kx[f]);
      Mx[f] = fma(wm, v, Mx[f]);
      if (ABS) {
        aKx[f] = fma(fabs(wk), fabs(v), aKx[f]);
        aMx[f] = fma(fabs(wm), fabs(v), aMx[f]);
      }
    }
  }
}
// Kc yc and |Kc| |yc| at a free node (the stencil's boundary neighbours; zero
// when yc is null or the node has none)
template <int D>
__device__ inline void stencil_kc(const Sten& st, int N, int i, int j, int k, const int* f2b, const double* yc,
                                  double& Kc, double& aKc) {
  Kc = aKc = 0.0;
  if (!yc || !near_bdry<D>(N, i, j, k)) return;
  double v[Nb<D>::Q];
#pragma unroll
  for (int q = 0; q < Nb<D>::Q; ++q) v[q] = 0.0;
  gather_bdry<D>(yc, f2b, N, i, j, k, v);
#pragma unroll
  for (int q = 0; q < Nb<D>::Q; ++q) {
    double wk, wm;
    nb_weights<D>(st, q, wk, wm);
    Kc = fma(wk, v[q], Kc);
    aKc = fma(fabs(wk), fabs(v[q]), aKc);
  }
}

template <int D>
__global__ void STENCIL_BOUNDS k_apply_KM(int N, const int* f2b, const double* x, const double* xc, double* yK,
                           double* yM, int64_t nfree, int64_t nbdry) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int r = blockIdx.y;
  if (t >= nfree) return;
  Sten st = make_sten(1.0 / N);
  Field f{x + r * nfree, xc ? xc + r * nbdry : nullptr};
  double Kx, Mx;
  int i, j, k;
  node_ijk<D>(t, N, i, j, k);
  stencil_KM<D>(st, N, f2b, f, i, j, k, t, Kx, Mx);
  if (yK) yK[r * nfree + t] = Kx;
  if (yM) yM[r * nfree + t] = Mx;
}

// Range-space elementwise kernels.  blockIdx.y = c runs over the right-hand sides
// of an instance's group (blocks with c >= nr return); the view's `map` packs
// the group slot of the c-th one in byte c.  Slot-indexed arrays (KKT iterates,
// residuals, partial sums) are offset by slot * stride; the FETI-DP vectors
// (cvec, cvec2, cvec3) are compact, offset by c * n.
__device__ inline int slot_of(unsigned map, int c) { return (int)((map >> (8 * c)) & 255u); }

// v = conj(r1 + M dw) = r1 + M conj(dw)   (dw = cvec2, v = cvec3)
template <int D>
__device__ inline cd mrhs2_node(const Sten& st, int N, int i, int j, int k, int64_t t, double r1t, const cd* dw) {
  cd v[Nb<D>::Q];
  gather_free<D>(dw, N, i, j, k, t, v);
  cd acc{r1t, 0.0};
#pragma unroll
  for (int q = 0; q < Nb<D>::Q; ++q) {
    double wk, wm;
    nb_weights<D>(st, q, wk, wm);
    acc.x = fma(wm, v[q].x, acc.x);
    acc.y = fma(-wm, v[q].y, acc.y);
  }
  return acc;
}
template <int D, class Src>
__global__ void STENCIL_BOUNDS k_make_rhs2(Src src) {
  const Dev& d = src.dev();
  const int c = blockIdx.y;
  if (c >= d.nr || d.g.dim != D) return;
  const int64_t nfree = d.n_free;
  int64_t t = (int64_t)src.bx() * blockDim.x + threadIdx.x;
  if (t >= nfree) return;
  const int N = d.g.N, s = slot_of(d.map, c);
  const double* r1 = d.r1 + s * nfree;
  const cd* dw = d.cvec2 + c * nfree;
  const Sten st = make_sten(1.0 / N);
  int i, j, k;
  node_ijk<D>(t, N, i, j, k);
  d.cvec3[c * nfree + t] = mrhs2_node<D>(st, N, i, j, k, t, r1[t], dw);
}

// per-node KKT residual and its squared norms, block partial sums
// (red + RED_HEAD + slot * pstride, pairs (||r||^2, ||b||^2) per block)
template <int D, class Src>
__global__ void STENCIL_BOUNDS k_kkt_residual(Src src) {
  __shared__ double sh[2][4];
  const Dev& d = src.dev();
  const int c = blockIdx.y;
  if (c >= d.nr || d.g.dim != D) return;
  const int N = d.g.N, s = slot_of(d.map, c), bx = src.bx();
  const int64_t nfree = d.n_free, nbdry = d.n_bdry;
  const int64_t pstride = 2 * ((nfree + 255) / 256);
  const int* f2b = d.full2bdry;
  const double* ybar = d.sl[s].ybar;
  const double* yc = d.sl[s].yc;
  const double* y = d.sl[s].y;
  const double* u = d.sl[s].u;
  const double* lam = d.sl[s].lam;
  double* part = d.red + RED_HEAD + s * pstride;
  int64_t t = (int64_t)bx * blockDim.x + threadIdx.x;
  double rn = 0.0, bn = 0.0;
  if (t < nfree) {
    const Sten st = make_sten(1.0 / N);
    int i, j, k;
    node_ijk<D>(t, N, i, j, k);
    // fields ybar, y, lam, u
    const double* const xs[4] = {ybar, y, lam, u};
    double K[4], M[4], aK_unused[4], aM_unused[4], Kc, aKc_unused;
    stencil_fields<D, 4, false>(st, N, i, j, k, t, xs, K, M, aK_unused, aM_unused);
    stencil_kc<D>(st, N, i, j, k, f2b, yc, Kc, aKc_unused);
    const double Mybar = M[0], Ky = K[1], My = M[1], Kl = K[2], Ml = M[2], Mu = M[3];
    double a1 = Mybar - My - Kl;
    double a2 = -(d.beta * Mu - Ml);
    double a3 = -Kc - Ky + Mu;
    if (d.r1) {  // null: norms only (the allocation-free entry point)
      d.r1[s * nfree + t] = a1;
      d.r2[s * nfree + t] = a2;
      d.r3[s * nfree + t] = a3;
    }
    rn = a1 * a1 + a2 * a2 + a3 * a3;
    bn = Mybar * Mybar + Kc * Kc;
  }
  for (int off = 32; off > 0; off >>= 1) {
    rn += __shfl_down(rn, off, 64);
    bn += __shfl_down(bn, off, 64);
  }
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) { sh[0][wv] = rn; sh[1][wv] = bn; }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * bx] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
    part[2 * bx + 1] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
  }
}

// Accuracy metrics of the KKT iterate (Sec. 2 KKT system; Sec. 6.2): the
// relative constraint violation ||K y + Kc yc - M u|| / ||K y|| and the
// blockwise backward error max_i ||r_i|| / (sum_j || |A_ij| |x_j| || + ||b_i||)
// with |K|, |M|, |Kc| the entrywise absolute values of the assembled matrices.
// Per node: Kx, Mx and the absolute-value products |K||x|, |M||x| from the same
// stencils with absolute weights.
// The eleven per-node values whose squares the metrics sum, at free node t.
template <int D>
__device__ inline void metrics_node(const Dev& d, const Slot& q, int N, int64_t t, double (&w)[MET_N]) {
  const Sten st = make_sten(1.0 / N);
  int i, j, k;
  node_ijk<D>(t, N, i, j, k);
  // fields y, lam, u, ybar
  const double* const xs[4] = {q.y, q.lam, q.u, q.ybar};
  double K[4], M[4], aK[4], aM[4], Kc, aKc;
  stencil_fields<D, 4, true>(st, N, i, j, k, t, xs, K, M, aK, aM);
  stencil_kc<D>(st, N, i, j, k, d.full2bdry, q.yc, Kc, aKc);
  const double Ky = K[0], My = M[0], aKy = aK[0], aMy = aM[0], Kl = K[1], Ml = M[1], aKl = aK[1], aMl = aM[1];
  const double Mu = M[2], aMu = aM[2], Mb = M[3];
  const double a1 = Mb - My - Kl;
  const double a2 = -(d.beta * Mu - Ml);
  const double a3 = -Kc - Ky + Mu;
  const double x[MET_N] = {a1, a2, a3, Ky, aMy, aKl, Mb, aMu, aMl, aKy, aKc};
#pragma unroll
  for (int e = 0; e < MET_N; ++e) w[e] = x[e];
}

// Per-block partial sums of squares, MET_N per block in the order
//   r1, r2, r3, K y, |M||y|, |K||lam|, M ybar, |M||u|, |M||lam|, |K||y|, |Kc||yc|.
template <int D, class Src>
__global__ void STENCIL_BOUNDS k_kkt_metrics(Src src) {
  __shared__ double sh[MET_N][4];
  const Dev& d = src.dev();
  const int c = blockIdx.y;
  if (c >= d.nr || d.g.dim != D) return;
  const int N = d.g.N, s = slot_of(d.map, c), bx = src.bx();
  const int64_t nfree = d.n_free;
  const int64_t nb = (nfree + 255) / 256;
  const Slot& q = d.sl[s];
  double* part = d.red + RED_HEAD + NRMAX * 2 * nb + (int64_t)s * MET_N * nb;
  int64_t t = (int64_t)bx * blockDim.x + threadIdx.x;
  double v[MET_N];
  for (int e = 0; e < MET_N; ++e) v[e] = 0.0;
  if (t < nfree) {
    double w[MET_N];
    metrics_node<D>(d, q, N, t, w);
    for (int e = 0; e < MET_N; ++e) v[e] = w[e] * w[e];
  }
  for (int e = 0; e < MET_N; ++e)
    for (int off = 32; off > 0; off >>= 1) v[e] += __shfl_down(v[e], off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0)
    for (int e = 0; e < MET_N; ++e) sh[e][wv] = v[e];
  __syncthreads();
  if (threadIdx.x < MET_N) {
    const int e = threadIdx.x;
    part[(int64_t)e * nb + bx] = sh[e][0] + sh[e][1] + sh[e][2] + sh[e][3];
  }
}

// Fixed-order sums of the metric partials; one block per right-hand side.
template <class Src>
__global__ void k_reduce_metrics(Src src) {
  __shared__ double sh[MET_N][64];
  const Dev& d = src.dev();
  const int c = blockIdx.y;
  if (c >= d.nr) return;
  const int s = slot_of(d.map, c);
  const int64_t nb = (d.n_free + 255) / 256;
  const double* part = d.red + RED_HEAD + NRMAX * 2 * nb + (int64_t)s * MET_N * nb;
  const int e = threadIdx.x / 64, l = threadIdx.x % 64;  // 11 x 64 threads
  if (e < MET_N) {
    double a = 0.0;
    for (int64_t b = l; b < nb; b += 64) a += part[(int64_t)e * nb + b];
    sh[e][l] = a;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double n[MET_N];
    for (int f = 0; f < MET_N; ++f) {
      double a = 0.0;
      for (int q = 0; q < 64; ++q) a += sh[f][q];
      n[f] = sqrt(a);
    }
    const double den[3] = {n[4] + n[5] + n[6], d.beta * n[7] + n[8], n[9] + n[7] + n[10]};
    double eta = 0.0;
    for (int b = 0; b < 3; ++b)
      if (n[b] > 0.0) eta = fmax(eta, n[b] / den[b]);
    d.red[MET_HEAD + 2 * s] = n[3] > 0.0 ? n[2] / n[3] : n[2];
    d.red[MET_HEAD + 2 * s + 1] = eta;
  }
}

// red[2 slot + which] = sqrt(sum part[2b]) / sqrt(sum part[2b+1]) in a fixed
// order; one block per (instance, right-hand side c = blockIdx.y)
template <class Src>
__global__ void k_reduce_ratio(Src src, int which) {
  __shared__ double sh[2][256];
  const Dev& d = src.dev();
  const int c = blockIdx.y;
  if (c >= d.nr) return;
  const int s = slot_of(d.map, c);
  const int nblocks = (int)((d.n_free + 255) / 256);
  const double* part = d.red + RED_HEAD + s * 2 * (int64_t)nblocks;
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < nblocks; q += 256) {
    a += part[2 * q];
    b += part[2 * q + 1];
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int q = 0; q < 256; ++q) { sa += sh[0][q]; sb += sh[1][q]; }
    d.red[2 * s + which] = sb > 0.0 ? sqrt(sa) / sqrt(sb) : sqrt(sa);
  }
}

// cvec = -r3 - i alpha r1
template <class Src>
__global__ void k_make_rhs1(Src src) {
  const Dev& d = src.dev();
  const int c = blockIdx.y;
  if (c >= d.nr) return;
  const int64_t n = d.n_free;
  int64_t t = (int64_t)src.bx() * blockDim.x + threadIdx.x;
  const int s = slot_of(d.map, c);
  if (t < n) d.cvec[c * n + t] = cd{-d.r3[s * n + t], -d.g.alpha * d.r1[s * n + t]};
}

// y -= Re dw; lam += Re z; u = lam / beta (dw = cvec2, z = cvec); partial sums
// of |Im z|^2, |Re z|^2.  single: one complex solve per step, lam -= Im dw / alpha
// (no second factor; the partial sums are zero).
template <class Src>
__global__ void __launch_bounds__(256) k_update(Src src, int single) {
  __shared__ double sh[2][4];
  const Dev& d = src.dev();
  const int c = blockIdx.y;
  if (c >= d.nr) return;
  if (d.flags[FLAG_NOTRES]) return;  // a GMRES grid of this step did no work: keep the iterate
  const int s = slot_of(d.map, c), bx = src.bx();
  const int64_t n = d.n_free, pstride = 2 * ((n + 255) / 256);
  const cd* dw = d.cvec2 + c * n;
  const cd* z = d.cvec + c * n;
  double* y = d.sl[s].y;
  double* u = d.sl[s].u;
  double* lam = d.sl[s].lam;
  double* part = d.red + RED_HEAD + s * pstride;
  int64_t t = (int64_t)bx * blockDim.x + threadIdx.x;
  double im = 0.0, re = 0.0;
  if (t < n) {
    y[t] -= dw[t].x;
    double l = single ? lam[t] - dw[t].y / d.g.alpha : lam[t] + z[t].x;
    lam[t] = l;
    u[t] = l / d.beta;
    if (!single) {
      im = z[t].y * z[t].y;
      re = z[t].x * z[t].x;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    im += __shfl_down(im, off, 64);
    re += __shfl_down(re, off, 64);
  }
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) { sh[0][wv] = im; sh[1][wv] = re; }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * bx] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
    part[2 * bx + 1] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
  }
}

// Start of a range-space target: y = ybar, u = 0, lam = 0 (and an empty
// iteration log) for the slots s (blockIdx.y) whose bit is set in the view's
// init mask.
template <class Src>
__global__ void k_group_init(Src src) {
  const Dev& d = src.dev();
  const int s = blockIdx.y;
  if (!((d.init >> s) & 1u)) return;
  const int64_t n = d.n_free;
  if (src.bx() == 0 && threadIdx.x <= 16)  // the slot's FETI-DP iteration log starts empty
    d.flags[threadIdx.x == 16 ? FLAG_CNT + s : FLAG_LOG + 16 * s + threadIdx.x] = 0;
  int64_t t = (int64_t)src.bx() * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const Slot& q = d.sl[s];
  q.y[t] = q.ybar[t];
  q.u[t] = 0.0;
  q.lam[t] = 0.0;
}

// flags[first .. first + count) = 0 for every instance
template <class Src>
__global__ void k_fill_flags(Src src, int first, int count) {
  const Dev& d = src.dev();
  for (int i = threadIdx.x; i < count; i += blockDim.x) d.flags[first + i] = 0;
}

// out[instance] = residual heads and flag words (one block per instance), written
// straight into pinned host memory (plain stores, coalesced, then a system-scope
// fence): the host reads them once the stream is synchronized, with no copy in between
template <class Src>
__global__ void k_gather(Src src, Gathered* out) {
  const Dev& d = src.dev();
  Gathered& o = out[blockIdx.x];
  if (threadIdx.x < 4 * NRMAX) o.red[threadIdx.x] = d.red ? d.red[threadIdx.x] : 0.0;
  for (int i = threadIdx.x; i < FLAG_WORDS; i += blockDim.x) o.flags[i] = d.flags[i];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_store(&o.ready, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __threadfence_system();
  }
}

__global__ void k_imag_scaled(int64_t n, const cd* x, double s, double* y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = s * x[i].y;
}

__global__ void k_real_part(int64_t n, const cd* x, double* y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i].x;
}

__global__ void k_fill(uint32_t* p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}
__global__ void k_r2c(int64_t n, const double* x, cd* y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = cd{x[i], 0.0};
}
__global__ void k_copy(int64_t n, const double* x, double* y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}

// ---- full-space method (Sec. 3.2): KKT operator, mass inverse, vector ops ----

// out = A x for x = (y, u, lam), three free-node blocks of length n (Sec. 2 KKT
// matrix): out1 = M y + K lam, out2 = beta M u - M lam, out3 = K y - M u.
template <int D>
__global__ void STENCIL_BOUNDS k_kkt_apply(int N, double beta, const double* x, double* out, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const Sten st = make_sten(1.0 / N);
  int i, j, k;
  node_ijk<D>(t, N, i, j, k);
  // fields y, u, lam
  const double* const xs[3] = {x, x + n, x + 2 * n};
  double K[3], M[3], aK_unused[3], aM_unused[3];
  stencil_fields<D, 3, false>(st, N, i, j, k, t, xs, K, M, aK_unused, aM_unused);
  const double Ky = K[0], My = M[0], Mu = M[1], Kl = K[2], Ml = M[2];
  out[t] = My + Kl;
  out[n + t] = beta * Mu - Ml;
  out[2 * n + t] = Ky - Mu;
}

// One factor of M^-1: the free-node mass matrix is m1 (x) m1 [(x) m1] with
// m1 = (h/6) tridiag(1, 4, 1) of order N - 1, so M^-1 is the product of
// tridiagonal solves along each axis.  Thread per grid line along `axis`
// (Thomas algorithm; m1 is diagonally dominant), out = scale m1^-1 in (in may
// equal out).  The elimination coefficients are the same for every line.
__global__ void __launch_bounds__(256) k_mass_lines(int N, int dim, int axis, double scale, const double* in,
                                                    double* out) {
  __shared__ double cp[1024];
  const int n1 = N - 1;
  const double h = 1.0 / N, a = h / 6.0, b = 4.0 * h / 6.0;
  if (threadIdx.x == 0) {
    cp[0] = a / b;
    for (int i = 1; i < n1; ++i) cp[i] = a / (b - a * cp[i - 1]);
  }
  __syncthreads();
  const int64_t lines = dim == 3 ? (int64_t)n1 * n1 : n1;
  const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= lines) return;
  int64_t base, stride;
  if (axis == 0) {
    base = line * n1;
    stride = 1;
  } else if (axis == 1) {
    base = dim == 3 ? (line % n1) + (line / n1) * (int64_t)n1 * n1 : line;
    stride = n1;
  } else {
    base = line;
    stride = (int64_t)n1 * n1;
  }
  double dprev = in[base] / b;
  out[base] = dprev;
  for (int i = 1; i < n1; ++i) {
    const int64_t o = base + i * stride;
    dprev = (in[o] - a * dprev) / (b - a * cp[i - 1]);
    out[o] = dprev;
  }
  double xn = out[base + (n1 - 1) * stride];
  out[base + (n1 - 1) * stride] = scale * xn;
  for (int i = n1 - 2; i >= 0; --i) {
    const int64_t o = base + i * stride;
    xn = out[o] - cp[i] * xn;
    out[o] = scale * xn;
  }
}

// out = a x + b y + c z (null operands count as zero)
__global__ void k_lin3(int64_t n, double a, const double* x, double b, const double* y, double c, const double* z,
                       double* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double v = 0.0;
  if (x) v = a * x[t];
  if (y) v = fma(b, y[t], v);
  if (z) v = fma(c, z[t], v);
  out[t] = v;
}

// part[block] = sum of x y over the block's entries
__global__ void __launch_bounds__(256) k_dot_part(int64_t n, const double* x, const double* y, double* part) {
  __shared__ double sh[4];
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v = t < n ? x[t] * y[t] : 0.0;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}
// out[0] = sum of part[0 .. nb) in a fixed order
__global__ void __launch_bounds__(256) k_sum_parts(int nb, const double* part, double* out) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int q = threadIdx.x; q < nb; q += 256) a += part[q];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

// The dimensions among a target's instances (bit D set for D = 2, 3).  A stencil
// kernel is launched once per dimension present; each instantiation's blocks
// return on the instances of the other one.
static inline unsigned target_dims(const Target& t) {
  if (t.single()) return 1u << t.one->dim;
  unsigned m = 0;
  for (const Problem* p : t.probs) m |= 1u << p->dim;
  return m;
}

hipError_t launch_apply_K(const Problem& p, int nrhs, const double* x, const double* xc, double* y,
                          hipStream_t st) {
  auto* kern = p.dim == 3 ? k_apply_KM<3> : k_apply_KM<2>;
  hipLaunchKernelGGL(kern, dim3(nblk(p.n_free), nrhs), dim3(256), 0, st, p.N, p.full2bdry, x, xc, y,
                     (double*)nullptr, p.n_free, p.n_bdry);
  return hipGetLastError();
}
hipError_t launch_apply_M(const Problem& p, int nrhs, const double* x, double* y, hipStream_t st) {
  auto* kern = p.dim == 3 ? k_apply_KM<3> : k_apply_KM<2>;
  hipLaunchKernelGGL(kern, dim3(nblk(p.n_free), nrhs), dim3(256), 0, st, p.N, p.full2bdry, x,
                     (const double*)nullptr, (double*)nullptr, y, p.n_free, p.n_bdry);
  return hipGetLastError();
}
// Partial sums of slot s start at red + RED_HEAD + s * red_pstride(p).
int64_t red_pstride(const Problem& p) { return 2 * (int64_t)nblk(p.n_free); }

hipError_t launch_kkt_residual(const Target& t) {
  const unsigned dims = target_dims(t);
  if (dims & 4u) launch2(t, K_NF256, k_kkt_residual<2, One>, k_kkt_residual<2, Many>, NRMAX, 256, 0);
  if (dims & 8u) launch2(t, K_NF256, k_kkt_residual<3, One>, k_kkt_residual<3, Many>, NRMAX, 256, 0);
  launch2(t, K_ONE, k_reduce_ratio<One>, k_reduce_ratio<Many>, NRMAX, 256, 0, 0);
  return hipGetLastError();
}
// ---- allocation-free KKT residual ----
// Device scratch of the entry point that allocates nothing: the per-block partial
// sums (from RED_HEAD) and the ratios (red[2 s]) of up to NRMAX right-hand sides.
// Each device holds its own copy; host code reaches it only through the address
// that hipGetSymbolAddress returned for that device (the array's name is a host
// stand-in, not a device address).
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {
std::mutex g_scr_mu;
double* g_scr_ptr[NOALLOC_MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch(int device, double** out) {
  *out = nullptr;
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scr_mu);
  if (!g_scr_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes the device current
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scr_ptr[device] = (double*)ptr;
  }
  *out = g_scr_ptr[device];
  return hipSuccess;
}

int64_t noalloc_kkt_doubles(int64_t n_free) { return RED_HEAD + NRMAX * 2 * (int64_t)nblk(n_free); }

__global__ void k_pick_ratio(const double* red, int nr, double* rel) {
  if ((int)threadIdx.x < nr) rel[threadIdx.x] = red[2 * threadIdx.x];
}

hipError_t launch_kkt_residual_noalloc(const Dev& d, hipStream_t st, double* rel) {
  const One o{d};
  auto* kern = d.g.dim == 3 ? k_kkt_residual<3, One> : k_kkt_residual<2, One>;
  hipLaunchKernelGGL(kern, dim3(nblk(d.n_free), NRMAX), dim3(256), 0, st, o);
  hipLaunchKernelGGL(k_reduce_ratio<One>, dim3(1, NRMAX), dim3(256), 0, st, o, 0);
  hipLaunchKernelGGL(k_pick_ratio, dim3(1), dim3(64), 0, st, (const double*)d.red, d.nr, rel);
  return hipGetLastError();
}

hipError_t launch_kkt_metrics(const Target& t) {
  const unsigned dims = target_dims(t);
  if (dims & 4u) launch2(t, K_NF256, k_kkt_metrics<2, One>, k_kkt_metrics<2, Many>, NRMAX, 256, 0);
  if (dims & 8u) launch2(t, K_NF256, k_kkt_metrics<3, One>, k_kkt_metrics<3, Many>, NRMAX, 256, 0);
  launch2(t, K_ONE, k_reduce_metrics<One>, k_reduce_metrics<Many>, NRMAX, MET_N * 64, 0);
  return hipGetLastError();
}
hipError_t launch_make_rhs1(const Target& t) {
  launch2(t, K_NF256, k_make_rhs1<One>, k_make_rhs1<Many>, NRMAX, 256, 0);
  return hipGetLastError();
}
hipError_t launch_make_rhs2(const Target& t) {
  const unsigned dims = target_dims(t);
  if (dims & 4u) launch2(t, K_NF256, k_make_rhs2<2, One>, k_make_rhs2<2, Many>, NRMAX, 256, 0);
  if (dims & 8u) launch2(t, K_NF256, k_make_rhs2<3, One>, k_make_rhs2<3, Many>, NRMAX, 256, 0);
  return hipGetLastError();
}
hipError_t launch_update(const Target& t, int single) {
  launch2(t, K_NF256, k_update<One>, k_update<Many>, NRMAX, 256, 0, single);
  launch2(t, K_ONE, k_reduce_ratio<One>, k_reduce_ratio<Many>, NRMAX, 256, 0, 1);
  return hipGetLastError();
}
hipError_t launch_group_init(const Target& t) {
  launch2(t, K_NF256, k_group_init<One>, k_group_init<Many>, NRMAX, 256, 0);
  return hipGetLastError();
}
hipError_t launch_fill_flags(const Target& t, int first, int count) {
  launch2(t, K_ONE, k_fill_flags<One>, k_fill_flags<Many>, 1, 64, 0, first, count);
  return hipGetLastError();
}
hipError_t launch_gather(const Target& t, Gathered* out) {
  launch2(t, K_ONE, k_gather<One>, k_gather<Many>, 1, 128, 0, out);
  return hipGetLastError();
}
hipError_t launch_imag_scaled(int64_t n, const cd* x, double s, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_imag_scaled, dim3(nblk(n)), dim3(256), 0, st, n, x, s, y);
  return hipGetLastError();
}
hipError_t launch_real_part(int64_t n, const cd* x, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_real_part, dim3(nblk(n)), dim3(256), 0, st, n, x, y);
  return hipGetLastError();
}
hipError_t launch_fill(void* ptr, size_t bytes, hipStream_t st) {
  size_t n = bytes / 4;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (uint32_t*)ptr, n);
  return hipGetLastError();
}
hipError_t launch_copy_real_to_complex(int64_t n, const double* x, cd* y, hipStream_t st) {
  hipLaunchKernelGGL(k_r2c, dim3(nblk(n)), dim3(256), 0, st, n, x, y);
  return hipGetLastError();
}
hipError_t launch_copy(int64_t n, const double* x, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_copy, dim3(nblk(n)), dim3(256), 0, st, n, x, y);
  return hipGetLastError();
}

hipError_t launch_kkt_apply(const Problem& p, const double* x, double* out, hipStream_t st) {
  auto* kern = p.dim == 3 ? k_kkt_apply<3> : k_kkt_apply<2>;
  hipLaunchKernelGGL(kern, dim3(nblk(p.n_free)), dim3(256), 0, st, p.N, p.beta, x, out, p.n_free);
  return hipGetLastError();
}
hipError_t launch_mass_inverse(const Problem& p, const double* x, double scale, double* out, hipStream_t st) {
  const int n1 = p.N - 1;
  const int64_t lines = p.dim == 3 ? (int64_t)n1 * n1 : n1;
  for (int axis = 0; axis < p.dim; ++axis)
    hipLaunchKernelGGL(k_mass_lines, dim3(nblk(lines)), dim3(256), 0, st, p.N, p.dim, axis,
                       axis == p.dim - 1 ? scale : 1.0, axis == 0 ? x : (const double*)out, out);
  return hipGetLastError();
}
hipError_t launch_lin3(int64_t n, double a, const double* x, double b, const double* y, double c, const double* z,
                       double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_lin3, dim3(nblk(n)), dim3(256), 0, st, n, a, x, b, y, c, z, out);
  return hipGetLastError();
}
hipError_t launch_dot(int64_t n, const double* x, const double* y, double* part, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dot_part, dim3(nblk(n)), dim3(256), 0, st, n, x, y, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, st, (int)nblk(n), (const double*)part, out);
  return hipGetLastError();
}

}  // namespace sfdp

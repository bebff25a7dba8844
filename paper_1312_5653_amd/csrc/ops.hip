// FP64 operators on the free-node grid of a 2D instance (Sec. 2 matrices),
// matrix free: on a uniform grid the Q1 stiffness and mass rows are the
// 9-point stencils  K = k1 (x) m1 + m1 (x) k1,  M = m1 (x) m1  with the 1D P1
// rows k1 = (1/h)(-1, 2, -1), m1 = (h/6)(1, 4, 1).  K_c couples free nodes to
// their boundary neighbours with the same stencil.
//
// The KKT residual (Sec. 2 KKT system) of (y, u, lam):
//   r1 = M ybar - M y - K lam,  r2 = -(beta M u - M lam),  r3 = -Kc yc - K y + M u,
// reduced deterministically (fixed-order two-pass sums) to ||r|| / ||b||.
#include "common.h"

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

// K x + Kc xc (xc may be null) and M x at free node (i, j), 1-based grid coords.
struct Field {
  const double* x;   // free values, stride n_free
  const double* xc;  // boundary values or null
};
__device__ inline double val(const Field& f, int N, const int* full2bdry, int i, int j) {
  if (i <= 0 || j <= 0 || i >= N || j >= N) {
    if (!f.xc) return 0.0;
    return f.xc[full2bdry[i + (N + 1) * j]];
  }
  return f.x[(i - 1) + (N - 1) * (j - 1)];
}
__device__ inline void stencil_KM(const Sten& st, int N, const int* f2b, const Field& f, int i,
                                  int j, double& Kx, double& Mx) {
  Kx = 0.0;
  Mx = 0.0;
  for (int dj = -1; dj <= 1; ++dj)
    for (int di = -1; di <= 1; ++di) {
      double v = val(f, N, f2b, i + di, j + dj);
      double wk = st.k[di + 1] * st.m[dj + 1] + st.m[di + 1] * st.k[dj + 1];
      double wm = st.m[di + 1] * st.m[dj + 1];
      Kx = fma(wk, v, Kx);
      Mx = fma(wm, v, Mx);
    }
}

__global__ void k_apply_KM(int N, const int* f2b, const double* x, const double* xc, double* yK,
                           double* yM, int64_t nfree, int64_t nbdry) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int r = blockIdx.y;
  if (t >= nfree) return;
  int i = (int)(t % (N - 1)) + 1, j = (int)(t / (N - 1)) + 1;
  Sten st = make_sten(1.0 / N);
  Field f{x + r * nfree, xc ? xc + r * nbdry : nullptr};
  double Kx, Mx;
  stencil_KM(st, N, f2b, f, i, j, Kx, Mx);
  if (yK) yK[r * nfree + t] = Kx;
  if (yM) yM[r * nfree + t] = Mx;
}

// Batched elementwise kernels: blockIdx.y = c runs over the nr right-hand sides
// of a group; `map` packs the group slot of c in byte c (slot = map >> 8c & 255).
// Slot-indexed arrays (KKT iterates, residuals, partial sums) are offset by
// slot * stride; the FETI-DP vectors (dw, z, g, v) are compact, offset by c * n.
__device__ inline int slot_of(unsigned map) { return (int)((map >> (8 * blockIdx.y)) & 255u); }

// complex M product: v = conj(r1 + M dw) = r1 + M conj(dw)
__global__ void k_make_rhs2(int N, unsigned map, const double* r1, const cd* dw, cd* v, int64_t nfree) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nfree) return;
  const int c = blockIdx.y, s = slot_of(map);
  r1 += s * nfree;
  dw += c * nfree;
  v += c * nfree;
  int i = (int)(t % (N - 1)) + 1, j = (int)(t / (N - 1)) + 1;
  Sten st = make_sten(1.0 / N);
  cd acc{r1[t], 0.0};
  for (int dj = -1; dj <= 1; ++dj)
    for (int di = -1; di <= 1; ++di) {
      int ii = i + di, jj = j + dj;
      if (ii <= 0 || jj <= 0 || ii >= N || jj >= N) continue;
      cd w = dw[(ii - 1) + (N - 1) * (jj - 1)];
      double wm = st.m[di + 1] * st.m[dj + 1];
      acc.x = fma(wm, w.x, acc.x);
      acc.y = fma(-wm, w.y, acc.y);
    }
  v[t] = acc;
}

// per-node KKT residual and its squared norms, block partial sums
// (part + slot * pstride, pairs (||r||^2, ||b||^2) per block)
__global__ void __launch_bounds__(256) k_kkt_residual(int N, const int* f2b, double beta, unsigned map,
                                                      const double* ybar, const double* yc,
                                                      const double* y, const double* u,
                                                      const double* lam, double* r1, double* r2,
                                                      double* r3, double* part, int64_t pstride,
                                                      int64_t nfree, int64_t nbdry) {
  __shared__ double sh[2][4];
  const int s = slot_of(map);
  ybar += s * nfree;
  if (yc) yc += s * nbdry;
  y += s * nfree;
  u += s * nfree;
  lam += s * nfree;
  r1 += s * nfree;
  r2 += s * nfree;
  r3 += s * nfree;
  part += s * pstride;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double rn = 0.0, bn = 0.0;
  if (t < nfree) {
    int i = (int)(t % (N - 1)) + 1, j = (int)(t / (N - 1)) + 1;
    Sten st = make_sten(1.0 / N);
    double Kyb_unused, Mybar, Ky, My, Kl, Ml, Ku_unused, Mu, Kc;
    stencil_KM(st, N, f2b, Field{ybar, nullptr}, i, j, Kyb_unused, Mybar);
    stencil_KM(st, N, f2b, Field{y, nullptr}, i, j, Ky, My);
    stencil_KM(st, N, f2b, Field{lam, nullptr}, i, j, Kl, Ml);
    stencil_KM(st, N, f2b, Field{u, nullptr}, i, j, Ku_unused, Mu);
    // Kc yc: stencil on a field that is zero at free nodes and yc on the boundary
    Kc = 0.0;
    if (yc) {
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
          int ii = i + di, jj = j + dj;
          if (ii > 0 && jj > 0 && ii < N && jj < N) continue;
          double wk = st.k[di + 1] * st.m[dj + 1] + st.m[di + 1] * st.k[dj + 1];
          Kc = fma(wk, yc[f2b[ii + (N + 1) * jj]], Kc);
        }
    }
    double a1 = Mybar - My - Kl;
    double a2 = -(beta * Mu - Ml);
    double a3 = -Kc - Ky + Mu;
    r1[t] = a1;
    r2[t] = a2;
    r3[t] = a3;
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
    part[2 * blockIdx.x] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
    part[2 * blockIdx.x + 1] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
  }
}

// out[2 slot] = sqrt(sum part[2b]) / sqrt(sum part[2b+1])  (fixed order), one
// block per right-hand side (blockIdx.x = c)
__global__ void k_reduce_ratio(int nblocks, unsigned map, const double* part, int64_t pstride,
                               double* out) {
  __shared__ double sh[2][256];
  const int s = (int)((map >> (8 * blockIdx.x)) & 255u);
  part += s * pstride;
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
    out[2 * s] = sb > 0.0 ? sqrt(sa) / sqrt(sb) : sqrt(sa);
  }
}

// g = -r3 - i alpha r1
__global__ void k_make_rhs1(double alpha, unsigned map, const double* r1, const double* r3, cd* g,
                            int64_t n) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y, s = slot_of(map);
  if (t < n) g[c * n + t] = cd{-r3[s * n + t], -alpha * r1[s * n + t]};
}

// y -= Re dw; lam += Re z; u = lam / beta; partial sums of |Im z|^2, |Re z|^2
__global__ void __launch_bounds__(256) k_update(double beta, unsigned map, const cd* dw, const cd* z,
                                                double* y, double* u, double* lam, double* part,
                                                int64_t pstride, int64_t n) {
  __shared__ double sh[2][4];
  const int c = blockIdx.y, s = slot_of(map);
  dw += c * n;
  z += c * n;
  y += s * n;
  u += s * n;
  lam += s * n;
  part += s * pstride;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double im = 0.0, re = 0.0;
  if (t < n) {
    y[t] -= dw[t].x;
    double l = lam[t] + z[t].x;
    lam[t] = l;
    u[t] = l / beta;
    im = z[t].y * z[t].y;
    re = z[t].x * z[t].x;
  }
  for (int off = 32; off > 0; off >>= 1) {
    im += __shfl_down(im, off, 64);
    re += __shfl_down(re, off, 64);
  }
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) { sh[0][wv] = im; sh[1][wv] = re; }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
    part[2 * blockIdx.x + 1] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
  }
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

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_apply_K(const Problem& p, int nrhs, const double* x, const double* xc, double* y,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_apply_KM, dim3(nblk(p.n_free), nrhs), dim3(256), 0, st, p.N, p.full2bdry, x,
                     xc, y, (double*)nullptr, p.n_free, p.n_bdry);
  return hipGetLastError();
}
hipError_t launch_apply_M(const Problem& p, int nrhs, const double* x, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_apply_KM, dim3(nblk(p.n_free), nrhs), dim3(256), 0, st, p.N, p.full2bdry, x,
                     (const double*)nullptr, (double*)nullptr, y, p.n_free, p.n_bdry);
  return hipGetLastError();
}
// Partial sums of slot s start at red + RED_HEAD + s * red_pstride(p).
int64_t red_pstride(const Problem& p) { return 2 * (int64_t)nblk(p.n_free); }

hipError_t launch_kkt_residual(const Problem& p, int nr, unsigned map, const double* ybar,
                               const double* yc, const double* y, const double* u,
                               const double* lam, double* r1, double* r2, double* r3, double* red,
                               hipStream_t st) {
  unsigned nb = nblk(p.n_free);
  int64_t ps = red_pstride(p);
  hipLaunchKernelGGL(k_kkt_residual, dim3(nb, nr), dim3(256), 0, st, p.N, p.full2bdry, p.beta, map,
                     ybar, yc, y, u, lam, r1, r2, r3, red + RED_HEAD, ps, p.n_free, p.n_bdry);
  hipLaunchKernelGGL(k_reduce_ratio, dim3(nr), dim3(256), 0, st, (int)nb, map, red + RED_HEAD, ps, red);
  return hipGetLastError();
}
hipError_t launch_make_rhs1(const Problem& p, int nr, unsigned map, const double* r1, const double* r3,
                            cd* g, hipStream_t st) {
  hipLaunchKernelGGL(k_make_rhs1, dim3(nblk(p.n_free), nr), dim3(256), 0, st, p.alpha, map, r1, r3, g,
                     p.n_free);
  return hipGetLastError();
}
hipError_t launch_make_rhs2(const Problem& p, int nr, unsigned map, const double* r1, const cd* dw,
                            cd* v, hipStream_t st) {
  hipLaunchKernelGGL(k_make_rhs2, dim3(nblk(p.n_free), nr), dim3(256), 0, st, p.N, map, r1, dw, v,
                     p.n_free);
  return hipGetLastError();
}
hipError_t launch_update(const Problem& p, int nr, unsigned map, const cd* dw, const cd* z, double* y,
                         double* u, double* lam, double* red, hipStream_t st) {
  unsigned nb = nblk(p.n_free);
  int64_t ps = red_pstride(p);
  hipLaunchKernelGGL(k_update, dim3(nb, nr), dim3(256), 0, st, p.beta, map, dw, z, y, u, lam,
                     red + RED_HEAD, ps, p.n_free);
  hipLaunchKernelGGL(k_reduce_ratio, dim3(nr), dim3(256), 0, st, (int)nb, map, red + RED_HEAD, ps,
                     red + 1);
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

}  // namespace sfdp

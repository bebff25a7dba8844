// Pieces shared by the FETI-DP paths whose interface blocks are too large for
// the persistent 2D kernel (3D scalar subdomains, elasticity): the symmetric
// row product of the dense subdomain operators, and a host-driven
// right-preconditioned GMRES (classical Gram-Schmidt twice on the device, the
// Hessenberg columns, Givens rotations and stopping tests on the host, one
// synchronisation per iteration) for up to NRMAX right-hand sides in lockstep.
// The Krylov vector kernels are defined in three.hip.
#pragma once
#include <algorithm>

#include "common.h"

namespace sfdp {

// Up to R3 = NRMAX right-hand sides run together: per-subdomain kernels read
// each operator once for all of them (R3 accumulators per row).
constexpr int R3 = NRMAX;

__device__ inline cd wsum(cd a) {
  for (int off = 32; off > 0; off >>= 1) {
    a.x += __shfl_xor(a.x, off, 64);
    a.y += __shfl_xor(a.y, off, 64);
  }
  return a;
}
__device__ inline double wsum(double a) {
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
  return a;
}
template <class TS>
__device__ inline cd ld64(const TS& v) { return cvt<double>(v); }

// Row i of the symmetric matrix A (n x n, leading dimension ld, read as column
// i: coalesced over i) against the R3 vectors xs[k][r] (LDS): U entries are
// loaded before they are used, so each thread keeps U loads in flight (more
// registers: the sweep, with more rows per workgroup, keeps U = 2).
template <int U, class TS>
__device__ inline void symcol_r3(const TS* __restrict__ A, int ld, int n, int i, const cd* xs, cd (&out)[R3]) {
  cd a[2][R3];
#pragma unroll
  for (int r = 0; r < R3; ++r) a[0][r] = a[1][r] = cd{0.0, 0.0};
  int k = 0;
  for (; k + U - 1 < n; k += U) {
    TS z[U];
#pragma unroll
    for (int u = 0; u < U; ++u) z[u] = A[(size_t)(k + u) * ld + i];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const cd zu = ld64(z[u]);
#pragma unroll
      for (int r = 0; r < R3; ++r) fma_acc(a[u & 1][r], zu, xs[(k + u) * R3 + r]);
    }
  }
  for (; k < n; ++k) {
    const cd zu = ld64(A[(size_t)k * ld + i]);
#pragma unroll
    for (int r = 0; r < R3; ++r) fma_acc(a[0][r], zu, xs[k * R3 + r]);
  }
#pragma unroll
  for (int r = 0; r < R3; ++r) out[r] = a[0][r] + a[1][r];
}

// Device buffers of one GMRES (NRMAX right-hand sides, kalloc + 1 basis vectors
// each; hd per right-hand side: two coefficient sets and the squared norm,
// 2 (kalloc + 1) + 1 entries; nvd the basis lengths of the final combination;
// gs per right-hand side the Givens state (gs_len entries: Hessenberg columns,
// rotations, rotated right-hand side, ||d||); gi per right-hand side its
// activity and iteration count, then the word "any active" and a counter used
// by the step kernel; gih a pinned copy of gi).
struct KBuf {
  cd *V, *hd, *part, *d, *z, *w, *mu;
  double* npart;
  int* nvd;
  int kalloc;
  cd* gs;
  int *gi, *gih;
};

// Givens state per right-hand side for kalloc K: H columns (K x (K + 1)), c
// (K), s (K), g (K + 1), beta (1)
__host__ __device__ inline int64_t gs_len(int K) { return (int64_t)(K + 1) * K + 3 * (int64_t)K + 2; }
constexpr int GI_WORDS = 2 * NRMAX + 2;

__global__ void k3_dots(int64_t n, int nv, const cd* V, int64_t vs, int64_t vr, const cd* w, int64_t wr, cd* part,
                        int64_t pr);
__global__ void k3_reduce(int nb, const cd* part, int64_t pr, cd* h, int64_t hr);
__global__ void k3_axpy(int64_t n, int nv, const cd* V, int64_t vs, int64_t vr, const cd* h, int64_t hr, cd* w,
                        int64_t wr, double* npart, int64_t nr_);
__global__ void k3_sum(int nb, const double* npart, int64_t pr, cd* out, int64_t hr);
__global__ void k3_normalize(int64_t n, const cd* w, int64_t wr, const cd* nrm, int64_t hr, cd* v, int64_t vr);
__global__ void k3_combine(int64_t n, const int* nv, const cd* V, int64_t vs, int64_t vr, const cd* y,
                           int64_t hr, cd* out, int64_t orr);
// y_r = A x_r (n x n, FP64) for r < nr (vectors at + r * stride), A read once
__global__ void k3_dense_mv(int n, int64_t stride, int nr, const cd* A, const cd* x, cd* y);

// Givens steps on the device (three.hip).  init: beta_r = sqrt of the squared
// norm in hd, g_r = (beta_r, 0, ...), active_r = beta_r > 0.  step j (one wave per
// right-hand side, the column and the rotations staged in LDS): column j of H_r
// from the two Gram-Schmidt coefficient sets and the new vector's norm, rotated
// by the previous rotations, a new rotation, g_r updated, and the stopping test;
// the last workgroup publishes gi[2 NRMAX] = any right-hand side still active.
// solve (one wave per right-hand side, the triangle in LDS when it has at most
// mlds columns): y_r = H_r^-1 g_r over its_r columns into hd (the combination
// coefficients) and nvd_r = its_r.
__global__ void k3_gm_init(int nr, int K, const cd* hd, int64_t hr, int ks, cd* gs, int* gi);
__global__ void k3_gm_step(int nr, int K, int j, int kmax, double tol, const cd* hd, int64_t hr, int ks, cd* gs,
                           int* gi);
__global__ void k3_gm_solve(int K, const cd* gs, const int* gi, cd* hd, int64_t hr, int* nvd, int mlds);

// Ops: stream st, right-hand sides nr, interface length nmu, buffers kb, and
// apply_P(x, xr, out, orr) / apply_F(x, xr, out, orr) (preconditioner and
// interface operator on right-hand-side-strided vectors).
// Right-preconditioned GMRES on F_DP mu_r = d_r from mu = 0 for the nr
// right-hand sides together (relative residual tol of the unpreconditioned
// system, at most kmax iterations each).  Every right-hand side keeps its own
// basis, Hessenberg matrix and stopping test, all on the device: the host
// enqueues GM_BATCH iterations at a time and reads back only the activity
// words between batches, so it does not wait for the GPU in every iteration.
// A right-hand side that has stopped rides along in the shared launches, but
// its later vectors are never used, so its result is that of a solve on its
// own; iterations enqueued after every right-hand side has stopped (at most
// GM_BATCH - 1) change nothing.
constexpr int GM_BATCH = 4;
constexpr int GM_LDS_COLS = 112;  // back substitution with the triangle in LDS up to this many columns

template <class Ops>
hipError_t gmres_host(Ops& o, double tol, int kmax, int* its) {
  KBuf& T = o.kb;
  hipStream_t st = o.st;
  const int nr = o.nr;
  const int64_t n = o.nmu, vs = n;
  const unsigned nb = (unsigned)((n + 255) / 256);
  const int ks = T.kalloc + 1;       // stride of the two coefficient sets in a right-hand side's hd
  const int64_t hr = 2 * ks + 1;     // hd per right-hand side: h (pass 0), h (pass 1), squared norm
  const int64_t vr = (int64_t)ks * n, pr = (int64_t)ks * 4 * nb;  // part: 4 wave sums per block
  cd* V = T.V;
  cd* dn = T.hd + 2 * ks;            // squared norm of right-hand side r at dn[r * hr]
  const int K = T.kalloc;
  hipLaunchKernelGGL(k3_axpy, dim3(nb, nr), dim3(256), 0, st, n, 0, (const cd*)V, vs, vr, (const cd*)T.hd, hr,
                     T.d, n, T.npart, (int64_t)nb);
  hipLaunchKernelGGL(k3_sum, dim3(nr), dim3(256), 0, st, (int)nb, (const double*)T.npart, (int64_t)nb, dn, hr);
  hipLaunchKernelGGL(k3_normalize, dim3(nb, nr), dim3(256), 0, st, n, (const cd*)T.d, n, (const cd*)dn, hr, V, vr);
  hipLaunchKernelGGL(k3_gm_init, dim3(1), dim3(64), 0, st, nr, K, (const cd*)T.hd, hr, ks, T.gs, T.gi);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int km = std::min(kmax, K);
  for (int j = 0; j < km;) {
    const int jb = std::min(km, j + GM_BATCH);
    for (; j < jb; ++j) {
      cd* vj = V + (int64_t)j * vs;
      cd* vn = V + (int64_t)(j + 1) * vs;
      o.apply_P(vj, vr, T.z, n);
      o.apply_F(T.z, n, vn, vr);
      for (int pass = 0; pass < 2; ++pass) {
        cd* h = T.hd + pass * ks;
        hipLaunchKernelGGL(k3_dots, dim3(nb, nr), dim3(256), 0, st, n, j + 1, (const cd*)V, vs, vr, (const cd*)vn,
                           vr, T.part, pr);
        hipLaunchKernelGGL(k3_reduce, dim3(j + 1, nr), dim3(256), 0, st, (int)(4 * nb), (const cd*)T.part, pr, h,
                           hr);
        hipLaunchKernelGGL(k3_axpy, dim3(nb, nr), dim3(256), 0, st, n, j + 1, (const cd*)V, vs, vr, (const cd*)h,
                           hr, vn, vr, T.npart, (int64_t)nb);
      }
      hipLaunchKernelGGL(k3_sum, dim3(nr), dim3(256), 0, st, (int)nb, (const double*)T.npart, (int64_t)nb, dn, hr);
      hipLaunchKernelGGL(k3_normalize, dim3(nb, nr), dim3(256), 0, st, n, (const cd*)vn, vr, (const cd*)dn, hr, vn,
                         vr);
      hipLaunchKernelGGL(k3_gm_step, dim3(nr), dim3(64), sizeof(cd) * (3 * (size_t)K + 1), st, nr, K, j, kmax, tol,
                         (const cd*)T.hd, hr, ks, T.gs, T.gi);
    }
    if ((e = hipMemcpyAsync(T.gih, T.gi, sizeof(int) * GI_WORDS, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return e;
    if (!T.gih[2 * NRMAX]) break;
  }
  // y_r = H_r^-1 g_r (the triangle in LDS up to GM_LDS_COLS columns), mu_r = P^-1 (V_r y_r)
  if ((e = hipMemcpyAsync(T.gih, T.gi, sizeof(int) * GI_WORDS, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return e;
  int mmax = 0;
  for (int r = 0; r < nr; ++r) mmax = std::max(mmax, T.gih[2 * r + 1]);
  const int mlds = mmax <= GM_LDS_COLS ? mmax : 0;
  hipLaunchKernelGGL(k3_gm_solve, dim3(nr), dim3(64), sizeof(cd) * ((size_t)mlds * (mlds + 1) / 2 + K + 1), st, K,
                     (const cd*)T.gs, (const int*)T.gi, T.hd, hr, T.nvd, mlds);
  hipLaunchKernelGGL(k3_combine, dim3(nb, nr), dim3(256), 0, st, n, (const int*)T.nvd, (const cd*)V, vs, vr,
                     (const cd*)T.hd, hr, T.w, n);
  o.apply_P(T.w, n, T.mu, n);
  if ((e = hipMemcpyAsync(T.gih, T.gi, sizeof(int) * GI_WORDS, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return e;
  for (int r = 0; r < nr; ++r) its[r] = T.gih[2 * r + 1];
  return hipGetLastError();
}

}  // namespace sfdp

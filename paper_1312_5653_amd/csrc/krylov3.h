// Pieces shared by the FETI-DP paths whose interface blocks are too large for
// the persistent 2D kernel (3D scalar subdomains, elasticity): the symmetric
// row product of the dense subdomain operators, and a host-driven
// right-preconditioned GMRES (classical Gram-Schmidt twice on the device, the
// Hessenberg columns, Givens rotations and stopping tests on the host, one
// synchronisation per iteration) for up to NRMAX right-hand sides in lockstep.
// The Krylov vector kernels are defined in three.hip.
#pragma once
#include <complex>
#include <vector>

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
// 2 (kalloc + 1) + 1 entries; hh its pinned host copy; nvd / nvh the basis
// lengths of the final combination).
struct KBuf {
  cd *V, *hd, *part, *d, *z, *w, *mu;
  double* npart;
  cd* hh;
  int *nvd, *nvh;
  int kalloc;
};

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

// Ops: stream st, right-hand sides nr, interface length nmu, buffers kb, and
// apply_P(x, xr, out, orr) / apply_F(x, xr, out, orr) (preconditioner and
// interface operator on right-hand-side-strided vectors).
// Right-preconditioned GMRES on F_DP mu_r = d_r from mu = 0 for the nr
// right-hand sides together (relative residual tol of the unpreconditioned
// system, at most kmax iterations each).  Every right-hand side keeps its own
// basis, Hessenberg matrix and stopping test; one that has stopped still rides
// along in the shared launches, but its later vectors are never used, so its
// result is that of a solve on its own.
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
  auto sync_h = [&]() {
    hipError_t e = hipMemcpyAsync(T.hh, T.hd, sizeof(cd) * hr * nr, hipMemcpyDeviceToHost, st);
    return e == hipSuccess ? hipStreamSynchronize(st) : e;
  };
  hipLaunchKernelGGL(k3_axpy, dim3(nb, nr), dim3(256), 0, st, n, 0, (const cd*)V, vs, vr, (const cd*)T.hd, hr,
                     T.d, n, T.npart, (int64_t)nb);
  hipLaunchKernelGGL(k3_sum, dim3(nr), dim3(256), 0, st, (int)nb, (const double*)T.npart, (int64_t)nb, dn, hr);
  hipLaunchKernelGGL(k3_normalize, dim3(nb, nr), dim3(256), 0, st, n, (const cd*)T.d, n, (const cd*)dn, hr, V, vr);
  hipError_t e = sync_h();
  if (e != hipSuccess) return e;
  using cx = std::complex<double>;
  const int km = std::min(kmax, T.kalloc);
  std::vector<std::vector<cx>> H(nr), cs(nr), sn(nr), gv(nr);
  std::vector<double> beta(nr);
  std::vector<int> done(nr, 0), mk(nr, 0);
  int ndone = 0;
  for (int r = 0; r < nr; ++r) {
    H[r].assign((size_t)(km + 1) * km, 0.0);
    cs[r].assign(km, 0.0);
    sn[r].assign(km, 0.0);
    gv[r].assign(km + 1, 0.0);
    beta[r] = std::sqrt(T.hh[r * hr + 2 * ks].x);
    gv[r][0] = beta[r];
    if (!(beta[r] > 0.0)) {
      done[r] = 1;
      ++ndone;
    }
  }
  for (int j = 0; j < km && ndone < nr; ++j) {
    cd* vj = V + (int64_t)j * vs;
    cd* vn = V + (int64_t)(j + 1) * vs;
    o.apply_P(vj, vr, T.z, n);
    o.apply_F(T.z, n, vn, vr);
    for (int pass = 0; pass < 2; ++pass) {
      cd* h = T.hd + pass * ks;
      hipLaunchKernelGGL(k3_dots, dim3(nb, nr), dim3(256), 0, st, n, j + 1, (const cd*)V, vs, vr, (const cd*)vn,
                         vr, T.part, pr);
      hipLaunchKernelGGL(k3_reduce, dim3(j + 1, nr), dim3(256), 0, st, (int)(4 * nb), (const cd*)T.part, pr, h, hr);
      hipLaunchKernelGGL(k3_axpy, dim3(nb, nr), dim3(256), 0, st, n, j + 1, (const cd*)V, vs, vr, (const cd*)h, hr,
                         vn, vr, T.npart, (int64_t)nb);
    }
    hipLaunchKernelGGL(k3_sum, dim3(nr), dim3(256), 0, st, (int)nb, (const double*)T.npart, (int64_t)nb, dn, hr);
    hipLaunchKernelGGL(k3_normalize, dim3(nb, nr), dim3(256), 0, st, n, (const cd*)vn, vr, (const cd*)dn, hr, vn,
                       vr);
    if ((e = sync_h()) != hipSuccess) return e;
    for (int r = 0; r < nr; ++r) {
      if (done[r]) continue;
      // column j of the Hessenberg matrix, rotated by the previous rotations
      const cd* hh = T.hh + r * hr;
      cx* Hj = H[r].data() + (size_t)j * (km + 1);
      for (int i = 0; i <= j; ++i) Hj[i] = cx(hh[i].x + hh[ks + i].x, hh[i].y + hh[ks + i].y);
      const double hn = std::sqrt(hh[2 * ks].x);
      for (int i = 0; i < j; ++i) {
        const cx a = Hj[i], b = Hj[i + 1];
        Hj[i] = cs[r][i] * a + sn[r][i] * b;
        Hj[i + 1] = -std::conj(sn[r][i]) * a + cs[r][i] * b;
      }
      const cx a = Hj[j];
      const double ra = std::abs(a), rho = std::sqrt(ra * ra + hn * hn);
      if (ra == 0.0) {
        cs[r][j] = 0.0;
        sn[r][j] = 1.0;
      } else {
        cs[r][j] = ra / rho;
        sn[r][j] = (a / ra) * hn / rho;
      }
      Hj[j] = cs[r][j] * a + sn[r][j] * hn;
      gv[r][j + 1] = -std::conj(sn[r][j]) * gv[r][j];
      gv[r][j] = cs[r][j] * gv[r][j];
      mk[r] = j + 1;
      if (std::abs(gv[r][j + 1]) <= tol * beta[r] || !(hn > 0.0)) {
        done[r] = 1;
        ++ndone;
      }
    }
  }
  // y_r = H_r^-1 g_r (upper triangular), mu_r = P^-1 (V_r y_r)
  for (int r = 0; r < nr; ++r) {
    its[r] = mk[r];
    std::vector<cx> y(mk[r]);
    for (int i = mk[r] - 1; i >= 0; --i) {
      cx s = gv[r][i];
      for (int c = i + 1; c < mk[r]; ++c) s -= H[r][(size_t)c * (km + 1) + i] * y[c];
      y[i] = s / H[r][(size_t)i * (km + 1) + i];
    }
    for (int i = 0; i < mk[r]; ++i) T.hh[r * hr + i] = cd{y[i].real(), y[i].imag()};
    T.nvh[r] = mk[r];
  }
  e = hipMemcpyAsync(T.hd, T.hh, sizeof(cd) * hr * nr, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(T.nvd, T.nvh, sizeof(int) * nr, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k3_combine, dim3(nb, nr), dim3(256), 0, st, n, (const int*)T.nvd, (const cd*)V, vs, vr,
                     (const cd*)T.hd, hr, T.w, n);
  o.apply_P(T.w, n, T.mu, n);
  // the host copies above must land before hh and nvh are reused
  e = hipStreamSynchronize(st);
  return e == hipSuccess ? hipGetLastError() : e;
}


}  // namespace sfdp

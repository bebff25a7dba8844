// Setup of the FETI-DP operators of Z = K + i alpha M (Sec. 4 factor, Sec. 5 solver).
//
// Per subdomain (one workgroup each):
//   1. factor_lines: block LDL^T of the extended local matrix E^s taken line by
//      line (E^s is block tridiagonal with tridiagonal couplings between
//      consecutive grid lines):  T_0 = A_00,  T_j = A_jj - A_j,j-1 T_j-1^-1 A_j-1,j,
//      storing G_j = T_j^-1.  No pivoting: every T_j is a Schur complement of
//      K + i alpha M restricted to remainder nodes, complex symmetric with
//      positive definite real and imaginary parts on those nodes (plus decoupled
//      identity rows), for which Gauss-Jordan without pivoting is stable.
//   2. multi_solve: E^s X = [e_Delta, Z_rc] by the same recursion with panels of
//      right-hand sides; the Delta rows give Z_rr^-1|Delta,Delta and
//      Phi = Z_rr^-1 Z_rc.
//   3. invert_batched: interface Schur complement S_bb = (Z_rr^-1|Delta,Delta)^-1,
//      used by the Dirichlet preconditioner (Sec. 5).
//   4. zcc_and_coarse: Z_cc* = Z_cc - Z_cr Phi per subdomain and the assembled
//      coarse matrix K_cc* = sum_s B_c^T Z_cc* B_c.
//   5. invert_dense: K_cc*^-1 by Gauss-Jordan (FP64), one launch per pivot.
#include "common.h"

namespace sfdp {

constexpr int MLMAX = 33;  // ml = m + 1 <= 33
constexpr int CW = 32;     // right-hand-side panel width of multi_solve

// In-place Gauss-Jordan inverse of an n x n complex matrix in LDS (row-major).
__device__ void gj_invert_lds(cd* T, int n, cd* rowk, cd* colk) {
  for (int k = 0; k < n; ++k) {
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
      rowk[t] = T[k * n + t];
      colk[t] = T[t * n + k];
    }
    __syncthreads();
    cd piv = cdiv(cd{1.0, 0.0}, rowk[k]);
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
      int i = idx / n, j = idx % n;
      cd v;
      if (i == k && j == k) v = piv;
      else if (i == k) v = rowk[j] * piv;
      else if (j == k) v = -(colk[i] * piv);
      else v = T[idx] - colk[i] * (rowk[j] * piv);
      T[idx] = v;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_factor_lines(Geo2 g, cd* G64) {
  __shared__ cd T[MLMAX * MLMAX];
  __shared__ cd Gp[MLMAX * MLMAX];
  __shared__ cd rowk[MLMAX], colk[MLMAX];
  const int s = blockIdx.x, ml = g.ml, n2 = ml * ml;
  for (int j = 0; j < ml; ++j) {
    for (int idx = threadIdx.x; idx < n2; idx += blockDim.x) {
      int p = idx / ml, q = idx % ml;
      cd v = g.eloc(s, p, j, q, j);
      if (j > 0) {
        for (int a = max(p - 1, 0); a <= min(p + 1, ml - 1); ++a) {
          cd ea = g.eloc(s, p, j, a, j - 1);
          if (ea.x == 0.0 && ea.y == 0.0) continue;
          cd acc{0.0, 0.0};
          for (int b = max(q - 1, 0); b <= min(q + 1, ml - 1); ++b) {
            cd eb = g.eloc(s, b, j - 1, q, j);
            fma_acc(acc, Gp[a * ml + b], eb);
          }
          v = v - ea * acc;
        }
      }
      T[idx] = v;
    }
    __syncthreads();
    gj_invert_lds(T, ml, rowk, colk);
    cd* out = G64 + ((size_t)s * ml + j) * n2;
    for (int idx = threadIdx.x; idx < n2; idx += blockDim.x) {
      int p = idx / ml, q = idx % ml;
      Gp[idx] = T[idx];
      out[q * ml + p] = T[idx];  // transposed: element (p, q) at [q][p]
    }
    __syncthreads();
  }
}

// Right-hand side column `col` of the multi-solve at local node (a, b).
__device__ inline cd multi_rhs(const Geo2& g, int s, int a, int b, int col, int nd, int nc,
                               const int* dloc, const int* cloc) {
  if (!g.rnode(s, a, b)) return cd{0.0, 0.0};
  int l = a + g.ml * b;
  if (col < nd) return (dloc[col] == l) ? cd{1.0, 0.0} : cd{0.0, 0.0};
  if (col < nd + nc) {
    int cl = cloc[col - nd];
    int ca = cl % g.ml, cb = cl / g.ml;
    if (abs(ca - a) > 1 || abs(cb - b) > 1) return cd{0.0, 0.0};
    return g.zloc(a, b, ca, cb);
  }
  return cd{0.0, 0.0};
}

__global__ void __launch_bounds__(256) k_multi_solve(Geo2 g, Maps2 mp, const cd* G64, cd* Sinv64,
                                                     cd* Phi64, cd* PhiFull, cd* scratch) {
  __shared__ cd Gl[MLMAX * MLMAX];
  __shared__ cd zb[MLMAX * CW];
  __shared__ cd tb[MLMAX * CW];
  __shared__ int slotmap[MLMAX * MLMAX];
  __shared__ int sdl[128];
  __shared__ int scl[4];
  const int s = blockIdx.x, ml = g.ml, n2 = ml * ml, ND = g.ND;
  const int nd = mp.nd[s];
  int nc = 0;
  for (int q = 0; q < 4; ++q) nc += (mp.cloc[s * 4 + q] >= 0);
  for (int l = threadIdx.x; l < n2; l += blockDim.x) slotmap[l] = -1;
  __syncthreads();
  for (int i = threadIdx.x; i < nd; i += blockDim.x) {
    int l = mp.dloc[s * ND + i];
    sdl[i] = l;
    slotmap[l] = i;
  }
  if (threadIdx.x < 4) scl[threadIdx.x] = mp.cloc[s * 4 + threadIdx.x];
  __syncthreads();
  const int ncol = nd + nc;
  cd* scr = scratch + (size_t)s * ml * n2 * CW / ml;  // [ml lines][ml][CW]
  for (int c0 = 0; c0 < ncol; c0 += CW) {
    // forward sweep: t_j = G_j (rhs_j - A_j,j-1 t_j-1)
    for (int j = 0; j < ml; ++j) {
      const cd* Gj = G64 + ((size_t)s * ml + j) * n2;
      for (int idx = threadIdx.x; idx < n2; idx += blockDim.x) Gl[idx] = Gj[idx];
      for (int idx = threadIdx.x; idx < ml * CW; idx += blockDim.x) {
        int p = idx / CW, c = idx % CW;
        cd v = multi_rhs(g, s, p, j, c0 + c, nd, nc, sdl, scl);
        if (j > 0) {
          for (int a = max(p - 1, 0); a <= min(p + 1, ml - 1); ++a) {
            cd e = g.eloc(s, p, j, a, j - 1);
            v = v - e * tb[a * CW + c];
          }
        }
        zb[idx] = v;
      }
      __syncthreads();
      for (int idx = threadIdx.x; idx < ml * CW; idx += blockDim.x) {
        int p = idx / CW, c = idx % CW;
        cd acc{0.0, 0.0};
        for (int k = 0; k < ml; ++k) fma_acc(acc, Gl[k * ml + p], zb[k * CW + c]);
        tb[idx] = acc;
        scr[((size_t)j * ml + p) * CW + c] = acc;
      }
      __syncthreads();
    }
    // backward sweep: x_j = t_j - G_j A_j,j+1 x_j+1   (tb holds x_j+1)
    for (int j = ml - 1; j >= 0; --j) {
      if (j < ml - 1) {
        const cd* Gj = G64 + ((size_t)s * ml + j) * n2;
        for (int idx = threadIdx.x; idx < n2; idx += blockDim.x) Gl[idx] = Gj[idx];
        for (int idx = threadIdx.x; idx < ml * CW; idx += blockDim.x) {
          int p = idx / CW, c = idx % CW;
          cd v{0.0, 0.0};
          for (int a = max(p - 1, 0); a <= min(p + 1, ml - 1); ++a)
            fma_acc(v, g.eloc(s, p, j, a, j + 1), tb[a * CW + c]);
          zb[idx] = v;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < ml * CW; idx += blockDim.x) {
          int p = idx / CW, c = idx % CW;
          cd acc = scr[((size_t)j * ml + p) * CW + c];
          for (int k = 0; k < ml; ++k) {
            cd t = Gl[k * ml + p] * zb[k * CW + c];
            acc = acc - t;
          }
          tb[idx] = acc;  // safe: zb holds the input of this line
        }
      } else {
        for (int idx = threadIdx.x; idx < ml * CW; idx += blockDim.x) {
          int p = idx / CW, c = idx % CW;
          tb[idx] = scr[((size_t)j * ml + p) * CW + c];
        }
      }
      __syncthreads();
      // extract rows of line j
      for (int idx = threadIdx.x; idx < ml * CW; idx += blockDim.x) {
        int p = idx / CW, c = idx % CW, col = c0 + c;
        int l = p + ml * j;
        cd x = tb[idx];
        int slot = slotmap[l];
        if (col < nd) {
          if (slot >= 0) Sinv64[((size_t)s * ND + slot) * ND + col] = x;
        } else if (col < ncol) {
          int q = col - nd;
          if (slot >= 0) Phi64[((size_t)s * ND + slot) * 4 + q] = x;
          PhiFull[((size_t)s * n2 + l) * 4 + q] = x;
        }
      }
      __syncthreads();
    }
  }
}

// In-place Gauss-Jordan inverse of the nd_s x nd_s leading block of each
// subdomain's ND x ND matrix (global memory, one workgroup per subdomain).
__global__ void __launch_bounds__(1024) k_invert_batched(int ND, const int* ndv, cd* A) {
  __shared__ cd rowk[512], colk[512];
  const int s = blockIdx.x, n = ndv[s];
  cd* M = A + (size_t)s * ND * ND;
  for (int k = 0; k < n; ++k) {
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
      rowk[t] = M[k * ND + t];
      colk[t] = M[t * ND + k];
    }
    __syncthreads();
    cd piv = cdiv(cd{1.0, 0.0}, rowk[k]);
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
      int i = idx / n, j = idx % n;
      cd v;
      if (i == k && j == k) v = piv;
      else if (i == k) v = rowk[j] * piv;
      else if (j == k) v = -(colk[i] * piv);
      else v = M[i * ND + j] - colk[i] * (rowk[j] * piv);
      M[i * ND + j] = v;
    }
    __syncthreads();
  }
}

// Z_cc*^s = Z_cc - Z_cr Phi  (4 x 4 per subdomain), into Zs[s][4][4].
__global__ void k_zcc(Geo2 g, Maps2 mp, const cd* PhiFull, cd* Zs) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.nsub * 16) return;
  int s = t / 16, q = (t / 4) % 4, q2 = t % 4;
  int cl = mp.cloc[s * 4 + q], cl2 = mp.cloc[s * 4 + q2];
  cd v{0.0, 0.0};
  if (cl >= 0 && cl2 >= 0) {
    int ca = cl % g.ml, cb = cl / g.ml, ca2 = cl2 % g.ml, cb2 = cl2 / g.ml;
    v = g.zloc(ca, cb, ca2, cb2);
    const int n2 = g.ml * g.ml;
    for (int b = max(cb - 1, 0); b <= min(cb + 1, g.ml - 1); ++b)
      for (int a = max(ca - 1, 0); a <= min(ca + 1, g.ml - 1); ++a) {
        if (!g.rnode(s, a, b)) continue;
        cd z = g.zloc(ca, cb, a, b);
        cd ph = PhiFull[((size_t)s * n2 + a + g.ml * b) * 4 + q2];
        v = v - z * ph;
      }
  }
  Zs[t] = v;
}

// Row c of K_cc* = sum over the subdomains sharing corner c (fixed order).
__global__ void k_coarse_assemble(Geo2 g, Maps2 mp, const cd* Zs, cd* Kcc) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.nC) return;
  cd* row = Kcc + (size_t)c * g.nC;
  for (int k = 0; k < g.nC; ++k) row[k] = cd{0.0, 0.0};
  for (int o = 0; o < 4; ++o) {
    int own = mp.cown[c * 4 + o];
    if (own < 0) continue;
    int s = own / 4, slot = own % 4;
    for (int q = 0; q < 4; ++q) {
      int c2 = mp.cgid[s * 4 + q];
      if (c2 < 0) continue;
      row[c2] = row[c2] + Zs[((size_t)s * 4 + slot) * 4 + q];
    }
  }
}

// One Gauss-Jordan pivot step B = step_k(A) of an n x n matrix (out of place).
__global__ void k_gj_step(int n, int k, const cd* A, cd* B) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  int i = idx / n, j = idx % n;
  cd piv = cdiv(cd{1.0, 0.0}, A[(size_t)k * n + k]);
  cd v;
  if (i == k && j == k) v = piv;
  else if (i == k) v = A[(size_t)k * n + j] * piv;
  else if (j == k) v = -(A[(size_t)i * n + k] * piv);
  else v = A[idx] - A[(size_t)i * n + k] * (A[(size_t)k * n + j] * piv);
  B[idx] = v;
}

// Pack the leading nd x nd block of each subdomain's full ND x ND FP64 matrix
// into lower-triangle row-major storage of the target precision.
template <class TD>
__global__ void k_pack(int nsub, int ND, const int* ndv, const cd* src, TD* dst) {
  const int s = blockIdx.y;
  const int PK = ND * (ND + 1) / 2;
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= PK) return;
  int i = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > idx) --i;
  while ((i + 1) * (i + 2) / 2 <= idx) ++i;
  int k = idx - i * (i + 1) / 2;
  cd v = (i < ndv[s]) ? src[((size_t)s * ND + i) * ND + k] : cd{0.0, 0.0};
  dst[(size_t)s * PK + idx] = TD{(typename real_of<TD>::type)v.x, (typename real_of<TD>::type)v.y};
}

template <class TS>
__global__ void k_convert(size_t n, const cd* src, TS* dst) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = TS{(typename real_of<TS>::type)src[i].x, (typename real_of<TS>::type)src[i].y};
}

hipError_t launch_factor_lines(const Problem& p, cd* G64, hipStream_t st) {
  hipLaunchKernelGGL(k_factor_lines, dim3(p.nsub), dim3(256), 0, st, p.geo(), G64);
  return hipGetLastError();
}

hipError_t launch_multi_solve(const Problem& p, const cd* G64, cd* Sinv64, cd* Phi64, cd* PhiFull,
                              cd* scratch, hipStream_t st) {
  hipLaunchKernelGGL(k_multi_solve, dim3(p.nsub), dim3(256), 0, st, p.geo(), p.maps(), G64, Sinv64,
                     Phi64, PhiFull, scratch);
  return hipGetLastError();
}

hipError_t launch_invert_batched(const Problem& p, cd* A64, hipStream_t st) {
  hipLaunchKernelGGL(k_invert_batched, dim3(p.nsub), dim3(1024), 0, st, p.ND, p.nd, A64);
  return hipGetLastError();
}

hipError_t launch_zcc_and_coarse(const Problem& p, const cd* PhiFull, cd* Kcc, hipStream_t st) {
  cd* Zs = nullptr;
  hipError_t e = hipMallocAsync((void**)&Zs, sizeof(cd) * p.nsub * 16, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_zcc, dim3((p.nsub * 16 + 255) / 256), dim3(256), 0, st, p.geo(), p.maps(),
                     PhiFull, Zs);
  hipLaunchKernelGGL(k_coarse_assemble, dim3((p.nC + 127) / 128), dim3(128), 0, st, p.geo(),
                     p.maps(), Zs, Kcc);
  e = hipGetLastError();
  hipFreeAsync(Zs, st);
  return e;
}

hipError_t launch_invert_dense(int n, cd* A, cd* work, hipStream_t st) {
  // result ends in A: an even number of ping-pong steps is arranged by a final copy
  cd* src = A;
  cd* dst = work;
  int nb = (n * n + 255) / 256;
  for (int k = 0; k < n; ++k) {
    hipLaunchKernelGGL(k_gj_step, dim3(nb), dim3(256), 0, st, n, k, src, dst);
    cd* t = src;
    src = dst;
    dst = t;
  }
  if (src != A) hipMemcpyAsync(A, src, sizeof(cd) * n * n, hipMemcpyDeviceToDevice, st);
  return hipGetLastError();
}

hipError_t launch_store_factors(const Problem& p, const cd* G64, const cd* Sinv64, const cd* S64,
                                const cd* Phi64, hipStream_t st) {
  size_t nG = (size_t)p.nsub * p.ml * p.ml * p.ml;
  size_t nS = (size_t)p.nsub * p.ND * p.ND;
  size_t nP = (size_t)p.nsub * p.ND * 4;
  auto conv = [&](size_t n, const cd* src, void* dst, bool to32) {
    if (to32)
      hipLaunchKernelGGL(k_convert<cf>, dim3((n + 255) / 256), dim3(256), 0, st, n, src, (cf*)dst);
    else
      hipMemcpyAsync(dst, src, n * sizeof(cd), hipMemcpyDeviceToDevice, st);
  };
  conv(nG, G64, p.G, p.g32());
  conv(nP, Phi64, p.Phi, p.s32());
  (void)nS;
  const int PK = p.ND * (p.ND + 1) / 2;
  dim3 grid((PK + 255) / 256, p.nsub);
  if (p.s32())
    hipLaunchKernelGGL(k_pack<cf>, grid, dim3(256), 0, st, p.nsub, p.ND, p.nd, Sinv64, (cf*)p.Sinv);
  else
    hipLaunchKernelGGL(k_pack<cd>, grid, dim3(256), 0, st, p.nsub, p.ND, p.nd, Sinv64, (cd*)p.Sinv);
  hipLaunchKernelGGL(k_pack<cf>, grid, dim3(256), 0, st, p.nsub, p.ND, p.nd, S64, (cf*)p.Sbb);
  return hipGetLastError();
}

}  // namespace sfdp

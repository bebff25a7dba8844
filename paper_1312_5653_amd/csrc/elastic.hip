// FETI-DP and the range-space refinement step for the linear-elasticity
// cantilever (Sec. 6.2 state equation, Sec. 5 solver, Sec. 3.1 / Sec. 4
// two-factor step), table-driven: the kernels see dofs and the host-built maps
// of elastic.h only.
//
//   set-up   E^s (Z_rr^s on the r positions, identity on the padding) from the
//            element matrices, inverted as one batch by blocked Gauss-Jordan
//            (FP64); Z_rr^-1 restricted to Delta is the local interface
//            operator, and its inverse is the Dirichlet preconditioner's
//            S_bb = Z_DD - Z_DI Z_II^-1 Z_ID (the Delta block of the inverse of
//            a matrix is the inverse of the Schur complement onto it).
//            Phi = Z_rr^-1 Z_rc, Z_cc* = Z_cc - Z_cr Phi, K_cc* = sum B_c^T Z_cc* B_c
//            and its inverse (FP64).
//   solve    as the 3D scalar path: full sweeps for the right-hand side d and the
//            recovery, right-preconditioned GMRES (host-driven, CGS2 in FP64) on
//            F_DP mu = d with the multiplicity-scaled Dirichlet preconditioner.
//   KKT      CSR products with K and M (FP64) for the residual blocks, the two
//            right-hand sides of the step and the update of (y, u, lam).
#include <algorithm>
#include <cmath>

#include "elastic.h"

namespace sfdp {

// Gauss-Jordan pivots of a batch of matrices (setup.hip)
hipError_t gj_range(int n, int kb, int ke, cd* A, size_t sA, cd* work, size_t sW, int batch, hipStream_t st);
hipError_t invert_dense(int n, cd* A, cd* work, hipStream_t st);

namespace {

constexpr int GJW_E = 2 * 32 * 32;  // pivot-inverse buffers per matrix of gj_range

unsigned nbe(int64_t n) { return (unsigned)((n + 255) / 256); }

// Entry (d1, d2) of the subdomain's Neumann matrix K^s + i alpha M^s (or
// K^s + alpha M^s): the sum over the subdomain's elements that hold both
// nodes of the element stiffness (and the scalar mass on equal components).
__device__ inline cd zloc_el(const GeoE& g, const double* __restrict__ Ke, int d1, int d2) {
  const int l1 = d1 / 3, c1 = d1 - 3 * l1, l2 = d2 / 3, c2 = d2 - 3 * l2;
  const int ml = g.ml;
  const int a1 = l1 % ml, b1 = (l1 / ml) % ml, k1 = l1 / (ml * ml);
  const int a2 = l2 % ml, b2 = (l2 / ml) % ml, k2 = l2 / (ml * ml);
  if (abs(a1 - a2) > 1 || abs(b1 - b2) > 1 || abs(k1 - k2) > 1) return cd{0.0, 0.0};
  const double* Me = Ke + 24 * 24;
  double kk = 0.0, mm = 0.0;
  for (int ec = max(max(k1, k2) - 1, 0); ec <= min(min(k1, k2), g.m - 1); ++ec)
    for (int eb = max(max(b1, b2) - 1, 0); eb <= min(min(b1, b2), g.m - 1); ++eb)
      for (int ea = max(max(a1, a2) - 1, 0); ea <= min(min(a1, a2), g.m - 1); ++ea) {
        const int v1 = (a1 - ea) + 2 * (b1 - eb) + 4 * (k1 - ec);
        const int v2 = (a2 - ea) + 2 * (b2 - eb) + 4 * (k2 - ec);
        kk += Ke[(3 * v1 + c1) * 24 + 3 * v2 + c2];
        if (c1 == c2) mm += Me[v1 * 8 + v2];
      }
  mm *= g.alpha;
  return g.rshift ? cd{kk + mm, 0.0} : cd{kk, mm};
}

}  // namespace

// ---------------------------------------------------------------- set-up --

// E^s (NR x NR), Zrc^s (NR x EQ) and the corner block Z_cc^s (EQ x EQ)
__global__ void kel_build(GeoE g, MapsE mp, cd* E, cd* Zrc, cd* Zcc) {
  const int s = blockIdx.y, NR = g.NR;
  const int64_t nE = (int64_t)NR * NR, nZ = (int64_t)NR * EQ;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int* rd = mp.rdof + (size_t)s * NR;
  const int* cq = mp.cdof + s * EQ;
  if (t < nE) {
    const int p = (int)(t / NR), q = (int)(t % NR);
    const int dp = rd[p], dq = rd[q];
    cd v{0.0, 0.0};
    if (dp < 0 || dq < 0) {
      if (p == q) v.x = 1.0;
    } else {
      v = zloc_el(g, mp.Ke, dp, dq);
    }
    E[(size_t)s * nE + t] = v;
  } else if (t < nE + nZ) {
    const int64_t u = t - nE;
    const int p = (int)(u / EQ), q = (int)(u % EQ);
    cd v{0.0, 0.0};
    if (rd[p] >= 0 && cq[q] >= 0) v = zloc_el(g, mp.Ke, rd[p], cq[q]);
    Zrc[(size_t)s * nZ + u] = v;
  } else if (t < nE + nZ + EQ * EQ) {
    const int u = (int)(t - nE - nZ), q = u / EQ, q2 = u % EQ;
    cd v{0.0, 0.0};
    if (cq[q] >= 0 && cq[q2] >= 0) v = zloc_el(g, mp.Ke, cq[q], cq[q2]);
    Zcc[(size_t)s * EQ * EQ + u] = v;
  }
}

// out[s][i][j] = E[s][o + i][o + j] for i, j < c (o = off[s], c = cnt[s]; 0 and
// n when null), the identity elsewhere; out in storage precision, out64 FP64
template <class TS>
__global__ void kel_take(const cd* E, int NR, const int* off, const int* cnt, int n, TS* out, cd* out64) {
  using R = typename real_of<TS>::type;
  const int s = blockIdx.y;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  const int i = (int)(t / n), j = (int)(t % n);
  const int o = off ? off[s] : 0, c = cnt ? cnt[s] : n;
  cd v{i == j ? 1.0 : 0.0, 0.0};
  if (i < c && j < c) v = E[(size_t)s * NR * NR + (size_t)(o + i) * NR + o + j];
  if (out) out[(size_t)s * n * n + t] = cvt<R>(v);
  if (out64) out64[(size_t)s * n * n + t] = v;
}

// PhiFull[s][p][q] = sum_r (E^s)^-1[p][r] Zrc[s][r][q]: only the rows r of the
// corner's element are non-zero, so the sum runs over the rows whose Zrc entry
// is non-zero
__global__ void kel_phi(GeoE g, const cd* E, const cd* Zrc, cd* PhiFull) {
  const int s = blockIdx.y, NR = g.NR;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= NR * EQ) return;
  const int p = t / EQ, q = t % EQ;
  const cd* Er = E + (size_t)s * NR * NR + (size_t)p * NR;
  const cd* Zq = Zrc + (size_t)s * NR * EQ + q;
  cd acc{0.0, 0.0};
  for (int r = 0; r < NR; ++r) {
    const cd z = Zq[(size_t)r * EQ];
    if (z.x != 0.0 || z.y != 0.0) fma_acc(acc, Er[r], z);
  }
  PhiFull[(size_t)s * NR * EQ + t] = acc;
}

template <class TS>
__global__ void kel_phi_delta(GeoE g, MapsE mp, const cd* PhiFull, TS* Phi) {
  using R = typename real_of<TS>::type;
  const int s = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.ND * EQ) return;
  const int d = t / EQ, q = t % EQ;
  cd v{0.0, 0.0};
  if (d < mp.nds[s]) v = PhiFull[((size_t)s * g.NR + mp.ni[s] + d) * EQ + q];
  Phi[(size_t)s * g.ND * EQ + t] = cvt<R>(v);
}

// Z_cc*^s = Z_cc^s - Zrc^T PhiFull in place (corner slots only); one block of
// EQ^2 threads per subdomain
__global__ void kel_zcc(GeoE g, MapsE mp, const cd* Zrc, const cd* PhiFull, cd* Zcc) {
  const int s = blockIdx.x, t = threadIdx.x;
  if (t >= EQ * EQ) return;
  const int q = t / EQ, q2 = t % EQ;
  cd v{0.0, 0.0};
  if (mp.cg[s * EQ + q] >= 0 && mp.cg[s * EQ + q2] >= 0) {
    v = Zcc[(size_t)s * EQ * EQ + t];
    const cd* Zr = Zrc + (size_t)s * g.NR * EQ;
    const cd* Ph = PhiFull + (size_t)s * g.NR * EQ;
    for (int p = 0; p < g.NR; ++p) {
      const cd z = Zr[(size_t)p * EQ + q];
      if (z.x != 0.0 || z.y != 0.0) v = v - z * Ph[(size_t)p * EQ + q2];
    }
  }
  Zcc[(size_t)s * EQ * EQ + t] = v;
}

// Row c of K_cc* = sum over the owners of corner c (increasing subdomain) of
// their Z_cc* rows; one thread per row (Kcc zero on entry)
__global__ void kel_coarse(GeoE g, MapsE mp, const cd* Zcc, cd* Kcc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.nC) return;
  cd* row = Kcc + (size_t)c * g.nC;
  for (int o = 0; o < 8; ++o) {
    const int own = mp.cown[c * 8 + o];
    if (own < 0) break;
    const int s = own / EQ, q = own % EQ;
    for (int q2 = 0; q2 < EQ; ++q2) {
      const int c2 = mp.cg[s * EQ + q2];
      if (c2 >= 0) row[c2] = row[c2] + Zcc[((size_t)s * EQ + q) * EQ + q2];
    }
  }
}

__global__ void kel_fill(uint32_t* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}

hipError_t el_launch_fill(void* ptr, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 4;
  if (!n) return hipSuccess;
  const unsigned nb = (unsigned)std::min<size_t>((n + 255) / 256, 65535);
  hipLaunchKernelGGL(kel_fill, dim3(nb), dim3(256), 0, st, (uint32_t*)ptr, n);
  return hipGetLastError();
}

hipError_t el_launch_setup(Elastic& el, bool s32, cd* Kcc, cd* Kinv, cd* E, cd* E2, cd* work, hipStream_t st) {
  const GeoE g = el.g;
  const MapsE mp = el.maps();
  const int NR = g.NR, ND = g.ND;
  const int64_t NR2 = (int64_t)NR * NR, ND2 = (int64_t)ND * ND;
  hipLaunchKernelGGL(kel_build, dim3(nbe(NR2 + (int64_t)NR * EQ + EQ * EQ), g.nsub), dim3(256), 0, st, g, mp, E,
                     el.Zrc, el.Zcc);
  hipError_t e = gj_range(NR, 0, NR, E, NR2, work, GJW_E, g.nsub, st);
  if (e != hipSuccess) return e;
  const dim3 gR(nbe(NR2), g.nsub), gD(nbe(ND2), g.nsub);
  if (s32) {
    hipLaunchKernelGGL(kel_take<cf>, gR, dim3(256), 0, st, (const cd*)E, NR, (const int*)nullptr,
                       (const int*)nullptr, NR, (cf*)el.Zinv, (cd*)nullptr);
    hipLaunchKernelGGL(kel_take<cf>, gD, dim3(256), 0, st, (const cd*)E, NR, mp.ni, mp.nds, ND, (cf*)el.Sinv, E2);
  } else {
    hipLaunchKernelGGL(kel_take<cd>, gR, dim3(256), 0, st, (const cd*)E, NR, (const int*)nullptr,
                       (const int*)nullptr, NR, (cd*)el.Zinv, (cd*)nullptr);
    hipLaunchKernelGGL(kel_take<cd>, gD, dim3(256), 0, st, (const cd*)E, NR, mp.ni, mp.nds, ND, (cd*)el.Sinv, E2);
  }
  hipLaunchKernelGGL(kel_phi, dim3(nbe((int64_t)NR * EQ), g.nsub), dim3(256), 0, st, g, (const cd*)E,
                     (const cd*)el.Zrc, el.PhiFull);
  const dim3 gP(nbe((int64_t)ND * EQ), g.nsub);
  if (s32) hipLaunchKernelGGL(kel_phi_delta<cf>, gP, dim3(256), 0, st, g, mp, (const cd*)el.PhiFull, (cf*)el.Phi);
  else hipLaunchKernelGGL(kel_phi_delta<cd>, gP, dim3(256), 0, st, g, mp, (const cd*)el.PhiFull, (cd*)el.Phi);
  hipLaunchKernelGGL(kel_zcc, dim3(g.nsub), dim3(EQ * EQ), 0, st, g, mp, (const cd*)el.Zrc, (const cd*)el.PhiFull,
                     el.Zcc);
  // S_bb = (Z_rr^-1 restricted to Delta)^-1
  if ((e = gj_range(ND, 0, ND, E2, ND2, work, GJW_E, g.nsub, st)) != hipSuccess) return e;
  if (s32)
    hipLaunchKernelGGL(kel_take<cf>, gD, dim3(256), 0, st, (const cd*)E2, ND, (const int*)nullptr,
                       (const int*)nullptr, ND, (cf*)el.Sbb, (cd*)nullptr);
  else
    hipLaunchKernelGGL(kel_take<cd>, gD, dim3(256), 0, st, (const cd*)E2, ND, (const int*)nullptr,
                       (const int*)nullptr, ND, (cd*)el.Sbb, (cd*)nullptr);
  const int64_t nc2 = (int64_t)g.nC * g.nC;
  if ((e = el_launch_fill(Kcc, sizeof(cd) * nc2, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(kel_coarse, dim3(nbe(g.nC)), dim3(256), 0, st, g, mp, (const cd*)el.Zcc, Kcc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(Kinv, Kcc, sizeof(cd) * nc2, hipMemcpyDeviceToDevice, st)) != hipSuccess) return e;
  return invert_dense(g.nC, Kinv, work, st);
}

// ----------------------------------------------------------------- solve --

// Full sweeps T_s,r = Z_rr^-1 f~_s,r (one workgroup per subdomain, a thread per
// row, Z_rr^-1 read once for all nr right-hand sides).  f~ = f / multiplicity
// (conj: of conj f); mode 1 subtracts Z_rc B_c u_c and B_r^T mu.  mode 0 also
// gives the corner terms Wc[s][q] = f_q / owners - (Phi^T f~)_q of f_c*.
template <class TS, int U>
__global__ void __launch_bounds__(1024) kel_sweep(GeoE g, MapsE mp, StrE st, int nr, const TS* __restrict__ Zinv,
                                                  const cd* PhiFull, const cd* Zrc, const cd* f, int conj, int mode,
                                                  const cd* uc, const cd* mu, cd* T, cd* Wc) {
  extern __shared__ cd ft[];  // [NR][R3]
  const int s = blockIdx.x, NR = g.NR, ND = g.ND;
  const int ni = mp.ni[s], nd = mp.nds[s];
  for (int t = threadIdx.x; t < NR * R3; t += blockDim.x) {
    const int p = t / R3, r = t % R3;
    cd v{0.0, 0.0};
    const int fr = mp.rfree[(size_t)s * NR + p];
    if (r < nr && fr >= 0) {
      v = f[r * st.f + fr];
      if (conj) v.y = -v.y;
      v = (double)mp.rw[(size_t)s * NR + p] * v;
      if (mode == 1) {
        const cd* zr = Zrc + ((size_t)s * NR + p) * EQ;
        for (int q = 0; q < EQ; ++q) {
          const int c = mp.cg[s * EQ + q];
          if (c < 0) continue;
          const cd z = zr[q];
          if (z.x != 0.0 || z.y != 0.0) v = v - z * uc[r * st.c + c];
        }
        if (p >= ni && p < ni + nd) {
          const size_t base = ((size_t)s * ND + (p - ni)) * 3;
          for (int j = 0; j < 3; ++j) {
            const int k = mp.dmu[base + j];
            if (k >= 0) v = v - (double)mp.dsg[base + j] * mu[r * st.mu + k];
          }
        }
      }
    }
    ft[t] = v;
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
    const int nw = blockDim.x >> 6, wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int q = wv; q < EQ; q += nw) {
      cd acc[R3];
#pragma unroll
      for (int r = 0; r < R3; ++r) acc[r] = cd{0.0, 0.0};
      for (int p = lane; p < NR; p += 64) {
        const cd ph = PhiFull[((size_t)s * NR + p) * EQ + q];
#pragma unroll
        for (int r = 0; r < R3; ++r) fma_acc(acc[r], ph, ft[p * R3 + r]);
      }
#pragma unroll
      for (int r = 0; r < R3; ++r) acc[r] = wsum(acc[r]);
      if (lane == 0) {
        const int c = mp.cg[s * EQ + q];
#pragma unroll
        for (int r = 0; r < R3; ++r) {
          if (r >= nr) continue;
          cd v{0.0, 0.0};
          if (c >= 0) {
            cd fv = f[r * st.f + mp.cfree[c]];
            if (conj) fv.y = -fv.y;
            v = (double)mp.cw[c] * fv - acc[r];
          }
          Wc[r * st.w + (size_t)s * EQ + q] = v;
        }
      }
    }
  }
}

// Interface product of one subdomain for nr right-hand sides: xs = B_r^T x on
// its Delta dofs (scaled by 1 / multiplicity when `scale`), Y_s = Mat xs,
// Wc_s = Phi^T xs.  Workgroup (s, y): for y < nsl, rows [64 y, 64 y + 64) of
// Y_s, each row split over the four waves by column (k = wave mod 4) and the
// partial sums added through LDS, so a subdomain's block streams through
// several workgroups at once; y = nsl computes Wc_s.  Every workgroup gathers
// xs for the whole subdomain (a few KB from L2).
template <class TS, int U>
__global__ void __launch_bounds__(256) kel_local(GeoE g, MapsE mp, StrE st, int nr, int nsl,
                                                 const TS* __restrict__ Mat, const TS* __restrict__ Phi, int scale,
                                                 const cd* x, int64_t xr, cd* Y, cd* Wc) {
  extern __shared__ cd xs[];  // [ND][R3]
  __shared__ cd red[3][64][R3];
  const int s = blockIdx.x, sl = blockIdx.y, ND = g.ND, nd = mp.nds[s];
  const int i0 = sl * 64;
  if (sl < nsl && i0 >= nd) return;  // rows beyond this subdomain's Delta count
  for (int i = threadIdx.x; i < nd; i += blockDim.x) {
    cd v[R3];
#pragma unroll
    for (int r = 0; r < R3; ++r) v[r] = cd{0.0, 0.0};
    const size_t base = ((size_t)s * ND + i) * 3;
    for (int j = 0; j < 3; ++j) {
      const int k = mp.dmu[base + j];
      if (k < 0) continue;
      const double sg = mp.dsg[base + j];
#pragma unroll
      for (int r = 0; r < R3; ++r)
        if (r < nr) v[r] = v[r] + sg * x[r * xr + k];
    }
    if (scale) {
      const double w = mp.dw[(size_t)s * ND + i];
#pragma unroll
      for (int r = 0; r < R3; ++r) v[r] = w * v[r];
    }
#pragma unroll
    for (int r = 0; r < R3; ++r) xs[i * R3 + r] = v[r];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (sl < nsl) {
    const int i = i0 + lane;
    const bool row = i < nd;
    const TS* A = Mat + (size_t)s * ND * ND + (row ? i : 0);
    cd acc[R3];
#pragma unroll
    for (int r = 0; r < R3; ++r) acc[r] = cd{0.0, 0.0};
    int k = wv;
    for (; k + 4 * (U - 1) < nd; k += 4 * U) {
      TS z[U];
#pragma unroll
      for (int u = 0; u < U; ++u) z[u] = A[(size_t)(k + 4 * u) * ND];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const cd zu = ld64(z[u]);
#pragma unroll
        for (int r = 0; r < R3; ++r) fma_acc(acc[r], zu, xs[(k + 4 * u) * R3 + r]);
      }
    }
    for (; k < nd; k += 4) {
      const cd zu = ld64(A[(size_t)k * ND]);
#pragma unroll
      for (int r = 0; r < R3; ++r) fma_acc(acc[r], zu, xs[k * R3 + r]);
    }
    if (wv > 0) {
#pragma unroll
      for (int r = 0; r < R3; ++r) red[wv - 1][lane][r] = acc[r];
    }
    __syncthreads();
    if (wv == 0 && row) {
#pragma unroll
      for (int r = 0; r < R3; ++r) {
        const cd a = (acc[r] + red[0][lane][r]) + (red[1][lane][r] + red[2][lane][r]);
        if (r < nr) Y[r * st.y + (size_t)s * ND + i] = a;
      }
    }
    return;
  }
  // corner terms: wave wv takes the six slots 6 wv .. 6 wv + 5, each lane a row
  constexpr int QW = EQ / 4;
  cd acc[QW][R3];
#pragma unroll
  for (int a = 0; a < QW; ++a)
#pragma unroll
    for (int r = 0; r < R3; ++r) acc[a][r] = cd{0.0, 0.0};
  for (int i = lane; i < nd; i += 64) {
    const TS* ph = Phi + ((size_t)s * ND + i) * EQ + QW * wv;
    TS z[QW];
#pragma unroll
    for (int a = 0; a < QW; ++a) z[a] = ph[a];
#pragma unroll
    for (int a = 0; a < QW; ++a) {
      const cd za = ld64(z[a]);
#pragma unroll
      for (int r = 0; r < R3; ++r) fma_acc(acc[a][r], za, xs[i * R3 + r]);
    }
  }
#pragma unroll
  for (int a = 0; a < QW; ++a)
#pragma unroll
    for (int r = 0; r < R3; ++r) {
      const cd v = wsum(acc[a][r]);
      if (lane == 0 && r < nr) Wc[r * st.w + (size_t)s * EQ + QW * wv + a] = v;
    }
}

// out[c] = add[c] + sum of Wc over the corner's owners (fixed order); r = blockIdx.y
__global__ void kel_corner_sum(int nC, StrE st, const int* cown, const cd* Wc, const cd* add, cd* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (c >= nC) return;
  cd acc = add ? add[r * st.c + c] : cd{0.0, 0.0};
  for (int o = 0; o < 8; ++o) {
    const int own = cown[c * 8 + o];
    if (own >= 0) acc = acc + Wc[r * st.w + own];
  }
  out[r * st.c + c] = acc;
}

// Y[r][s ystride + d] += phis (Phi_s[d] . u_c(B_c s)) for the Delta dofs d < nds[s]
// of subdomain s = blockIdx.x and every right-hand side r < nr: the subdomain's
// EQ corner values of u_c are staged in LDS once (zero for a clamped slot, which
// adds nothing), then every thread forms its rows' sums with all its Phi loads
// independent of each other.  The same sums, in the same order, as the corner
// term of kel_scatter, added once per Delta dof instead of once per multiplier
// side.
template <class TS>
__global__ void __launch_bounds__(256) kel_phi_add(GeoE g, MapsE mp, StrE st, int nr, const TS* Phi,
                                                   const cd* uc, double phis, cd* Y, int64_t yr, int ystride) {
  __shared__ cd ucs[EQ][R3];
  const int s = blockIdx.x;
  if (threadIdx.x < EQ * R3) {
    const int q = threadIdx.x / R3, r = threadIdx.x % R3;
    const int c = mp.cg[s * EQ + q];
    ucs[q][r] = (c >= 0 && r < nr) ? uc[r * st.c + c] : cd{0.0, 0.0};
  }
  __syncthreads();
  const int nd = mp.nds[s];
  for (int d = threadIdx.x; d < nd; d += blockDim.x) {
    const TS* ph = Phi + ((size_t)s * g.ND + d) * EQ;
    cd acc[R3];
#pragma unroll
    for (int r = 0; r < R3; ++r) acc[r] = cd{0.0, 0.0};
#pragma unroll 6
    for (int q = 0; q < EQ; ++q) {
      const cd p = ld64(ph[q]);
#pragma unroll
      for (int r = 0; r < R3; ++r) fma_acc(acc[r], p, ucs[q][r]);
    }
#pragma unroll
    for (int r = 0; r < R3; ++r) {
      if (r >= nr) break;
      cd* y = Y + r * yr + (size_t)s * ystride + d;
      *y = *y + phis * acc[r];
    }
  }
}

// Per multiplier k with copies (s+, d+) and (s-, d-), for every right-hand side r:
//   out_k = sc_k (v+ - v-),  v = Y[s ystride + o_s + d] + phis (Phi_s[d] . u_c(B_c s))
// with o_s = ni[s] when `at_ni` (Y holds whole r vectors), else 0, and
// sc_k = 1 / multiplicity when `scale`, else 1.  One thread per multiplier, so
// the Phi rows are read once for all right-hand sides.
template <class TS>
__global__ void kel_scatter(GeoE g, MapsE mp, StrE st, int nr, const cd* Y, int64_t yr, int ystride, int at_ni,
                            const TS* Phi, const cd* uc, double phis, int scale, cd* out, int64_t orr) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.nmu) return;
  cd acc[R3];
#pragma unroll
  for (int r = 0; r < R3; ++r) acc[r] = cd{0.0, 0.0};
  for (int side = 0; side < 2; ++side) {
    const int own = mp.muown[2 * k + side];
    const int s = own / g.ND, d = own % g.ND;
    const size_t at = (size_t)s * ystride + (at_ni ? mp.ni[s] : 0) + d;
    cd v[R3];
#pragma unroll
    for (int r = 0; r < R3; ++r) v[r] = r < nr ? Y[r * yr + at] : cd{0.0, 0.0};
    if (Phi) {
      cd pc[R3];
#pragma unroll
      for (int r = 0; r < R3; ++r) pc[r] = cd{0.0, 0.0};
#pragma unroll 6
      for (int q = 0; q < EQ; ++q) {
        const int c = mp.cg[s * EQ + q];
        if (c < 0) continue;
        const cd ph = ld64(Phi[((size_t)s * g.ND + d) * EQ + q]);
#pragma unroll
        for (int r = 0; r < R3; ++r)
          if (r < nr) fma_acc(pc[r], ph, uc[r * st.c + c]);
      }
#pragma unroll
      for (int r = 0; r < R3; ++r) v[r] = v[r] + phis * pc[r];
    }
#pragma unroll
    for (int r = 0; r < R3; ++r) acc[r] = side == 0 ? acc[r] + v[r] : acc[r] - v[r];
  }
  const double sc = scale ? (double)mp.muw[k] : 1.0;
#pragma unroll
  for (int r = 0; r < R3; ++r)
    if (r < nr) out[r * orr + k] = sc * acc[r];
}

// Displacements on the free dofs: corner dofs from u_c, every other dof the
// average of its subdomain copies (conj: conjugated); r = blockIdx.y
__global__ void kel_assemble(GeoE g, MapsE mp, StrE st, const cd* T, const cd* uc, int conj, cd* x) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.n_free) return;
  const int r = blockIdx.y;
  cd v{0.0, 0.0};
  const int c = mp.fcor[t];
  if (c >= 0) {
    v = uc[r * st.c + c];
  } else {
    int cnt = 0;
    for (int o = 0; o < 4; ++o) {
      const int own = mp.fown[t * 4 + o];
      if (own < 0) break;
      v = v + T[r * st.t + own];
      ++cnt;
    }
    v = (1.0 / cnt) * v;
  }
  if (conj) v.y = -v.y;
  x[r * st.f + t] = v;
}

namespace {

struct OpsE {
  Elastic& el;
  GeoE g;
  MapsE mp;
  StrE sr;
  const cd* Kinv;
  hipStream_t st;
  bool s32;
  int nr;
  unsigned threads_sweep;
  KBuf kb;
  int64_t nmu;
  OpsE(Elastic& e, bool s32_, const cd* Kinv_, int nr_, hipStream_t st_)
      : el(e), g(e.g), mp(e.maps()), sr(e.str()), Kinv(Kinv_), st(st_), s32(s32_), nr(nr_) {
    kb = e.kb;
    nmu = g.nmu;
    threads_sweep = (unsigned)std::min(1024, std::max(256, (g.NR + 63) / 64 * 64));
  }
  // row slices of 64 for Mat (when given), and one more workgroup per subdomain for Phi
  template <class TS>
  void local_t(const void* Mat, const void* Phi, int scale, const cd* x, int64_t xr, cd* Y, cd* Wc) {
    const int nsl = Mat ? (g.ND + 63) / 64 : 0;
    hipLaunchKernelGGL((kel_local<TS, 4>), dim3(g.nsub, nsl + (Phi ? 1 : 0)), dim3(256), sizeof(cd) * g.ND * R3, st,
                       g, mp, sr, nr, nsl, (const TS*)Mat, (const TS*)Phi, scale, x, xr, Y, Wc);
  }
  void local(const void* Mat, const void* Phi, int scale, const cd* x, int64_t xr, cd* Y, cd* Wc) {
    if (s32) local_t<cf>(Mat, Phi, scale, x, xr, Y, Wc);
    else local_t<cd>(Mat, Phi, scale, x, xr, Y, Wc);
  }
  void scatter(const cd* Y, int64_t yr, int ystride, int at_ni, bool phi, double phis, int scale, cd* out,
               int64_t orr) {
    const dim3 grid(nbe(g.nmu));
    if (s32)
      hipLaunchKernelGGL(kel_scatter<cf>, grid, dim3(256), 0, st, g, mp, sr, nr, Y, yr, ystride, at_ni,
                         phi ? (const cf*)el.Phi : (const cf*)nullptr, (const cd*)el.uc, phis, scale, out, orr);
    else
      hipLaunchKernelGGL(kel_scatter<cd>, grid, dim3(256), 0, st, g, mp, sr, nr, Y, yr, ystride, at_ni,
                         phi ? (const cd*)el.Phi : (const cd*)nullptr, (const cd*)el.uc, phis, scale, out, orr);
  }
  template <class TS>
  void sweep_t(const cd* f, int conj, int mode) {
    const size_t lds = sizeof(cd) * g.NR * R3;
    hipLaunchKernelGGL((kel_sweep<TS, 2>), dim3(g.nsub), dim3(threads_sweep), lds, st, g, mp, sr, nr,
                       (const TS*)el.Zinv, (const cd*)el.PhiFull, (const cd*)el.Zrc, f, conj, mode, (const cd*)el.uc,
                       (const cd*)el.kb.mu, el.T, el.Wc);
  }
  void sweep(const cd* f, int conj, int mode) {
    if (s32) sweep_t<cf>(f, conj, mode);
    else sweep_t<cd>(f, conj, mode);
  }
  // out = K_cc*^-1 (add + sum of Wc)
  void coarse(const cd* add, cd* out) {
    hipLaunchKernelGGL(kel_corner_sum, dim3(nbe(g.nC), nr), dim3(256), 0, st, g.nC, sr, mp.cown, (const cd*)el.Wc,
                       add, el.gc);
    hipLaunchKernelGGL(k3_dense_mv, dim3((g.nC + 3) / 4), dim3(256), 0, st, g.nC, sr.c, nr, Kinv, (const cd*)el.gc,
                       out);
  }
  // out = F_DP x: the corner term goes into the local products (el.Y, scratch
  // until the next local product) once per Delta dof, then a plain scatter
  void apply_F(const cd* x, int64_t xr, cd* out, int64_t orr) {
    local(el.Sinv, el.Phi, 0, x, xr, el.Y, el.Wc);
    coarse(nullptr, el.uc);
    if (s32)
      hipLaunchKernelGGL(kel_phi_add<cf>, dim3(g.nsub), dim3(256), 0, st, g, mp, sr, nr, (const cf*)el.Phi,
                         (const cd*)el.uc, 1.0, el.Y, sr.y, g.ND);
    else
      hipLaunchKernelGGL(kel_phi_add<cd>, dim3(g.nsub), dim3(256), 0, st, g, mp, sr, nr, (const cd*)el.Phi,
                         (const cd*)el.uc, 1.0, el.Y, sr.y, g.ND);
    scatter(el.Y, sr.y, g.ND, 0, false, 0.0, 0, out, orr);
  }
  // out = W B_r S_bb B_r^T W x
  void apply_P(const cd* x, int64_t xr, cd* out, int64_t orr) {
    local(el.Sbb, nullptr, 1, x, xr, el.Y, nullptr);
    scatter(el.Y, sr.y, g.ND, 0, false, 0.0, 1, out, orr);
  }
  // d = sum B_r (Z_rr^-1 f_r)|Delta - F_rc K_cc*^-1 f_c*  (leaves f_c* in fcs)
  void rhs(const cd* f, int conj) {
    sweep(f, conj, 0);
    hipLaunchKernelGGL(kel_corner_sum, dim3(nbe(g.nC), nr), dim3(256), 0, st, g.nC, sr, mp.cown, (const cd*)el.Wc,
                       (const cd*)nullptr, el.fcs);
    hipLaunchKernelGGL(k3_dense_mv, dim3((g.nC + 3) / 4), dim3(256), 0, st, g.nC, sr.c, nr, Kinv, (const cd*)el.fcs,
                       el.uc);
    scatter(el.T, sr.t, g.NR, 1, true, -1.0, 0, el.kb.d, sr.mu);
  }
};

}  // namespace

hipError_t el_launch_feti(Elastic& el, bool s32, const cd* Kinv, int nr, const cd* f, cd* x, int conj, double tol,
                          int kmax, int* its, hipStream_t st) {
  OpsE o(el, s32, Kinv, nr, st);
  o.rhs(f, conj);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = gmres_host(o, tol, kmax, its)) != hipSuccess) return e;
  // u_c = K_cc*^-1 (f_c* + F_rc^T mu), u_r = Z_rr^-1 (f_r - Z_rc B_c u_c - B_r^T mu)
  o.local(nullptr, el.Phi, 0, el.kb.mu, o.sr.mu, nullptr, el.Wc);
  o.coarse(el.fcs, el.uc);
  o.sweep(f, conj, 1);
  hipLaunchKernelGGL(kel_assemble, dim3(nbe(el.g.n_free), nr), dim3(256), 0, st, o.g, o.mp, o.sr, (const cd*)el.T,
                     (const cd*)el.uc, conj, x);
  return hipGetLastError();
}

hipError_t el_launch_interface(Elastic& el, bool s32, const cd* Kinv, char which, const cd* x, cd* y,
                               hipStream_t st) {
  OpsE o(el, s32, Kinv, 1, st);
  const int64_t n = o.g.nmu;
  if (which == 'F') o.apply_F(x, n, y, n);
  else if (which == 'P') o.apply_P(x, n, y, n);
  else {
    o.rhs(x, 0);
    hipError_t e = hipMemcpyAsync(y, el.kb.d, sizeof(cd) * n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

// ------------------------------------------------- KKT products (CSR, FP64) --

// CSR rows are taken by 16 lanes each (16 rows per workgroup of 256), the
// lanes striding over the row's entries so that neighbouring lanes read
// neighbouring entries; the row's sums are folded over the 16 lanes.
constexpr int EL_RL = 16;
__device__ inline double fold16(double v) {
  for (int off = EL_RL / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// y_r = A x_r for the rows of the CSR matrix (values a); r = blockIdx.y
__global__ void __launch_bounds__(256) kel_spmv(int64_t n, const int* rp, const int* ci, const double* a,
                                                const double* x, double* y) {
  const int64_t t = (int64_t)blockIdx.x * (256 / EL_RL) + threadIdx.x / EL_RL;
  const int sub = threadIdx.x % EL_RL, r = blockIdx.y;
  x += r * n;
  double acc = 0.0;
  if (t < n)
    for (int j = rp[t] + sub; j < rp[t + 1]; j += EL_RL) acc = fma(a[j], x[ci[j]], acc);
  acc = fold16(acc);
  if (t < n && sub == 0) y[r * n + t] = acc;
}

hipError_t el_launch_spmv(const Elastic& el, char which, int nr, const double* x, double* y, hipStream_t st) {
  const int64_t n = el.g.n_free;
  hipLaunchKernelGGL(kel_spmv, dim3((unsigned)((n + 15) / 16), nr), dim3(256), 0, st, n, (const int*)el.rp, (const int*)el.ci,
                     (const double*)(which == 'K' ? el.Kv : el.Mv), x, y);
  return hipGetLastError();
}

// Per row and target i = blockIdx.y: the residual of the KKT system at
// (y, u, lam) with right-hand side (M ybar, 0, 0),
//   r1 = M ybar - M y - K lam,  r2 = -(beta M u - M lam),  r3 = -K y + M u,
// and the squares of the EL_SUMS quantities summed over the workgroup into
// part[(i nb + block) EL_SUMS + e].  16 lanes per row.
__global__ void __launch_bounds__(256) kel_kkt(int64_t n, const int* rp, const int* ci, const double* Kv,
                                               const double* Mv, SlotE sl, double beta, int keep, double* r1,
                                               double* r3, double* part) {
  __shared__ double sh[EL_SUMS][4];
  const int i = blockIdx.y, sub = threadIdx.x % EL_RL;
  const int64_t t = (int64_t)blockIdx.x * (256 / EL_RL) + threadIdx.x / EL_RL;
  double w[EL_SUMS];
  for (int e = 0; e < EL_SUMS; ++e) w[e] = 0.0;
  double Mb = 0, My = 0, aMy = 0, Kl = 0, aKl = 0, Mu = 0, aMu = 0, Ml = 0, aMl = 0, Ky = 0, aKy = 0;
  if (t < n) {
    const double *yb = sl.ybar[i], *y = sl.y[i], *u = sl.u[i], *lam = sl.lam[i];
    for (int j = rp[t] + sub; j < rp[t + 1]; j += EL_RL) {
      const int c = ci[j];
      const double k = Kv[j], m = Mv[j], ak = fabs(k), am = fabs(m);
      const double vb = yb[c], vy = y[c], vl = lam[c], vu = u[c];
      Mb = fma(m, vb, Mb);
      My = fma(m, vy, My);
      aMy = fma(am, fabs(vy), aMy);
      Kl = fma(k, vl, Kl);
      aKl = fma(ak, fabs(vl), aKl);
      Mu = fma(m, vu, Mu);
      aMu = fma(am, fabs(vu), aMu);
      Ml = fma(m, vl, Ml);
      aMl = fma(am, fabs(vl), aMl);
      Ky = fma(k, vy, Ky);
      aKy = fma(ak, fabs(vy), aKy);
    }
  }
  Mb = fold16(Mb); My = fold16(My); aMy = fold16(aMy); Kl = fold16(Kl); aKl = fold16(aKl); Mu = fold16(Mu);
  aMu = fold16(aMu); Ml = fold16(Ml); aMl = fold16(aMl); Ky = fold16(Ky); aKy = fold16(aKy);
  if (t < n && sub == 0) {
    const double a1 = Mb - My - Kl, a2 = -(beta * Mu - Ml), a3 = -Ky + Mu;
    if (keep) {
      r1[i * n + t] = a1;
      r3[i * n + t] = a3;
    }
    const double v[EL_SUMS] = {a1, a2, a3, Ky, aMy, aKl, Mb, aMu, aMl, aKy};
    for (int e = 0; e < EL_SUMS; ++e) w[e] = v[e] * v[e];
  }
  for (int e = 0; e < EL_SUMS; ++e) w[e] = wsum(w[e]);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0)
    for (int e = 0; e < EL_SUMS; ++e) sh[e][wv] = w[e];
  __syncthreads();
  if (threadIdx.x < EL_SUMS) {
    const int e = threadIdx.x;
    part[((int64_t)i * gridDim.x + blockIdx.x) * EL_SUMS + e] = (sh[e][0] + sh[e][1]) + (sh[e][2] + sh[e][3]);
  }
}

// sums[i * EL_SUMS + e] = sum over the nb blocks of part (fixed order); block i
__global__ void __launch_bounds__(256) kel_sum(int nb, int ne, const double* part, double* sums) {
  __shared__ double sh[EL_SUMS][64];
  const int i = blockIdx.x, e = threadIdx.x / 64, l = threadIdx.x % 64;
  const int ew = ne;  // entries used per block record
  for (int e0 = 0; e0 < ew; e0 += 4) {
    const int ee = e0 + e;
    if (ee < ew) {
      double a = 0.0;
      for (int b = l; b < nb; b += 64) a += part[((int64_t)i * nb + b) * EL_SUMS + ee];
      sh[ee][l] = a;
    }
  }
  __syncthreads();
  if (threadIdx.x < ew) {
    double a = 0.0;
    for (int q = 0; q < 64; ++q) a += sh[threadIdx.x][q];
    sums[i * EL_SUMS + threadIdx.x] = a;
  }
}

hipError_t el_launch_kkt(Elastic& el, int nr, const SlotE& sl, double beta, bool keep, hipStream_t st) {
  const int64_t n = el.g.n_free;
  const unsigned nb = (unsigned)((n + 15) / 16);
  hipLaunchKernelGGL(kel_kkt, dim3(nb, nr), dim3(256), 0, st, n, (const int*)el.rp, (const int*)el.ci,
                     (const double*)el.Kv, (const double*)el.Mv, sl, beta, keep ? 1 : 0, el.r1, el.r3, el.part);
  hipLaunchKernelGGL(kel_sum, dim3(nr), dim3(256), 0, st, (int)nb, EL_SUMS, (const double*)el.part, el.sums);
  return hipGetLastError();
}

// c1_c = -r3_i - i alpha r1_i  (i = a.idx[c], c = blockIdx.y)
__global__ void kel_rhs1(int64_t n, ActE a, double alpha, const double* r1, const double* r3, cd* c1) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y, i = a.idx[c];
  if (t < n) c1[c * n + t] = cd{-r3[i * n + t], -alpha * r1[i * n + t]};
}

hipError_t el_launch_rhs1(Elastic& el, const ActE& a, double alpha, hipStream_t st) {
  const int64_t n = el.g.n_free;
  hipLaunchKernelGGL(kel_rhs1, dim3(nbe(n), a.n), dim3(256), 0, st, n, a, alpha, (const double*)el.r1,
                     (const double*)el.r3, el.c1);
  return hipGetLastError();
}

// c3_c = conj(r1_i + M c2_c); 16 lanes per row
__global__ void __launch_bounds__(256) kel_rhs2(int64_t n, const int* rp, const int* ci, const double* Mv, ActE a,
                                                const double* r1, const cd* c2, cd* c3) {
  const int64_t t = (int64_t)blockIdx.x * (256 / EL_RL) + threadIdx.x / EL_RL;
  const int sub = threadIdx.x % EL_RL, c = blockIdx.y, i = a.idx[c];
  const cd* w = c2 + c * n;
  double re = 0.0, im = 0.0;
  if (t < n)
    for (int j = rp[t] + sub; j < rp[t + 1]; j += EL_RL) {
      const cd v = w[ci[j]];
      re = fma(Mv[j], v.x, re);
      im = fma(Mv[j], v.y, im);
    }
  re = fold16(re);
  im = fold16(im);
  if (t < n && sub == 0) c3[c * n + t] = cd{r1[i * n + t] + re, -im};
}

hipError_t el_launch_rhs2(Elastic& el, const ActE& a, hipStream_t st) {
  const int64_t n = el.g.n_free;
  hipLaunchKernelGGL(kel_rhs2, dim3((unsigned)((n + 15) / 16), a.n), dim3(256), 0, st, n, (const int*)el.rp, (const int*)el.ci,
                     (const double*)el.Mv, a, (const double*)el.r1, (const cd*)el.c2, el.c3);
  return hipGetLastError();
}

// y -= Re c2, lam += Re c1, u = lam / beta (target a.idx[c]); squares of
// Im c1 and Re c1 per workgroup into part[(c nb + block) EL_SUMS + 0 / 1]
__global__ void __launch_bounds__(256) kel_update(int64_t n, ActE a, SlotE sl, double beta, const cd* c1,
                                                  const cd* c2, double* part) {
  __shared__ double sh[2][4];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y, i = a.idx[c];
  double im = 0.0, re = 0.0;
  if (t < n) {
    const cd dw = c2[c * n + t], z = c1[c * n + t];
    sl.y[i][t] -= dw.x;
    const double l = sl.lam[i][t] + z.x;
    sl.lam[i][t] = l;
    sl.u[i][t] = l / beta;
    im = z.y * z.y;
    re = z.x * z.x;
  }
  im = wsum(im);
  re = wsum(re);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    sh[0][wv] = im;
    sh[1][wv] = re;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int e = threadIdx.x;
    part[((int64_t)c * gridDim.x + blockIdx.x) * EL_SUMS + e] = (sh[e][0] + sh[e][1]) + (sh[e][2] + sh[e][3]);
  }
}

hipError_t el_launch_update(Elastic& el, const ActE& a, const SlotE& sl, double beta, hipStream_t st) {
  const int64_t n = el.g.n_free;
  const unsigned nb = nbe(n);
  hipLaunchKernelGGL(kel_update, dim3(nb, a.n), dim3(256), 0, st, n, a, sl, beta, (const cd*)el.c1,
                     (const cd*)el.c2, el.part);
  hipLaunchKernelGGL(kel_sum, dim3(a.n), dim3(256), 0, st, (int)nb, 2, (const double*)el.part,
                     el.sums + NRMAX * EL_SUMS);
  return hipGetLastError();
}

__global__ void kel_r2c(int64_t n, const double* x, cd* y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] = cd{x[t], 0.0};
}
__global__ void kel_c2r(int64_t n, const cd* x, int im, double s, double* y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] = im ? s * x[t].y : x[t].x;
}
hipError_t el_launch_r2c(int64_t n, const double* x, cd* y, hipStream_t st) {
  hipLaunchKernelGGL(kel_r2c, dim3(nbe(n)), dim3(256), 0, st, n, x, y);
  return hipGetLastError();
}
hipError_t el_launch_c2r(int64_t n, const cd* x, int im, double s, double* y, hipStream_t st) {
  hipLaunchKernelGGL(kel_c2r, dim3(nbe(n)), dim3(256), 0, st, n, x, im, s, y);
  return hipGetLastError();
}

}  // namespace sfdp

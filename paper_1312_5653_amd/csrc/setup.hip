// Setup of the FETI-DP operators of Z = K + i alpha M (Sec. 4 factor, Sec. 5 solver).
//
// Per subdomain:
//   1. factor_lines (one wavefront): block LDL^T of the extended local matrix
//      E^s taken line by line (E^s is block tridiagonal with tridiagonal
//      couplings between consecutive grid lines):
//      T_0 = A_00,  T_j = A_jj - A_j,j-1 T_j-1^-1 A_j-1,j,  storing G_j = T_j^-1.
//      No pivoting: every T_j is a Schur complement of K + i alpha M restricted
//      to remainder nodes, complex symmetric with positive definite real and
//      imaginary parts on those nodes (plus decoupled identity rows), for which
//      Gauss-Jordan without pivoting is stable.
//   2. multi_solve (four wavefronts, the line products on the matrix cores):
//      E^s X = [e_Delta, Z_rc] by the same recursion; the Delta rows give
//      Z_rr^-1|Delta,Delta and Phi = Z_rr^-1 Z_rc.
//   3. invert_batched: interface Schur complement S_bb = (Z_rr^-1|Delta,Delta)^-1,
//      used by the Dirichlet preconditioner (Sec. 5).
//   4. zcc_and_coarse: Z_cc* = Z_cc - Z_cr Phi per subdomain and the assembled
//      coarse matrix K_cc* = sum_s B_c^T Z_cc* B_c.
//   5. the coarse inverse by Gauss-Jordan without pivoting (FP64): in LDS for
//      small coarse matrices, one workgroup each for mid-size ones when several
//      are set up together, and otherwise by panels of 32 pivots over the whole
//      device (the trailing update on the matrix cores).
#include "common.h"

namespace sfdp {

constexpr int MLMAX = 33;  // ml = m + 1 <= 33

// LDS visibility inside one wavefront: wait for this wave's LDS operations and
// keep the compiler from moving memory accesses across (no workgroup barrier).
__device__ inline void wave_sync_lds() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt = 0
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

// Gauss-Jordan inverse of the 33 x 33 block of k_factor_lines_wave in place, in
// rotated coordinates: before pivot k lane p holds R[q] = T[p][(q + k0) % 33]
// with k0 the first pivot of the current group of three, so pivot k sits at the
// fixed register k - k0 and the pivot row passes through LDS in the same
// rotation.  After each group the registers rotate by three; after all 33
// pivots (the padding rows and columns beyond ml are identity and pivot
// trivially) the rotation is whole again.  Every register index is static and
// the loop body stays small (three pivots).
template <class R>
__device__ __forceinline__ void gj_wave_invert(C<R> (&T)[MLMAX], C<R> (*rowk)[MLMAX], int p) {
  using CR = C<R>;
  static_assert(MLMAX % 3 == 0, "pivot groups of three");
  for (int k0 = 0; k0 < MLMAX; k0 += 3) {
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int k = k0 + u;
      CR* rk = rowk[k & 1];
      if (p == k) {
#pragma unroll
        for (int q = 0; q < MLMAX; ++q) rk[q] = T[q];
      }
      wave_sync_lds();
      const CR piv = cdiv(CR{1, 0}, rk[u]);
      const bool me = p == k;
      const CR f = me ? -piv : T[u] * piv;
#pragma unroll
      for (int q = 0; q < MLMAX; ++q) {
        if (q == u) continue;
        CR v = me ? CR{0, 0} : T[q];
        fma_acc(v, -f, rk[q]);
        T[q] = v;
      }
      T[u] = me ? piv : -f;
    }
    CR t0 = T[0], t1 = T[1], t2 = T[2];
#pragma unroll
    for (int q = 0; q < MLMAX - 3; ++q) T[q] = T[q + 3];
    T[MLMAX - 3] = t0;
    T[MLMAX - 2] = t1;
    T[MLMAX - 1] = t2;
  }
}

// The line factorization, one wavefront per subdomain.  Lane p owns
// row p of the current line block in registers (rows ml..63 are idle padding):
// T_j is formed from the rows of G_j-1 (the neighbouring rows of
// G_j-1 A_j-1,j by lane shuffles), then inverted in place by Gauss-Jordan
// without pivoting, the pivot row passing through LDS.  The T_j and G_j are
// complex symmetric, so lane p's row is also column p, and the transposed
// storage of G_j (element (p, q) at [q][p]) takes one coalesced store per
// column index.  One wavefront
// needs no workgroup barrier; the per-step LDS traffic is the pivot row only.
// R: arithmetic (double; float for the complex64 set-up); G_j is stored in FP64.
template <class R, class Src>
__global__ void __launch_bounds__(64) k_factor_lines_wave(Src src) {
  using CR = C<R>;
  __shared__ CR rowk[2][MLMAX];
  __shared__ CR cpl[MLMAX][3];
  const Dev& d = src.dev();
  const Geo2& g = d.g;
  const int s = src.bx(), ml = g.ml, n2 = ml * ml, p = threadIdx.x;
  // coupling of node b of a line to node b + e - 1 of the neighbouring line
  for (int t = p; t < ml * 3; t += 64) {
    const int b = t / 3, e = t % 3, a = b + e - 1;
    cpl[b][e] = cvt<R>((a >= 0 && a < ml) ? g.zloc(b, 1, a, 0) : cd{0.0, 0.0});
  }
  CR cplp[3], dgb[3], dgi[3];  // row p's couplings and its in-line band (boundary / interior lines)
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int a = p + e - 1;
    const bool ok = p < ml && a >= 0 && a < ml;
    cplp[e] = cvt<R>(ok ? g.zloc(p, 1, a, 0) : cd{0.0, 0.0});
    dgb[e] = cvt<R>(ok ? g.zloc(p, 0, a, 0) : cd{0.0, 0.0});
    dgi[e] = cvt<R>(ok ? g.zloc(p, 1, a, 1) : cd{0.0, 0.0});
  }
  wave_sync_lds();
  CR T[MLMAX];
#pragma unroll
  for (int q = 0; q < MLMAX; ++q) T[q] = CR{0, 0};
  uint64_t mprev = 0;
  for (int j = 0; j < ml; ++j) {
    const bool bnd = j == 0 || j == ml - 1;
    CR dg[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) dg[e] = bnd ? dgb[e] : dgi[e];
    const uint64_t mj = __ballot(p < ml && g.rnode(s, p, j));  // r nodes of line j
    const bool rp = (mj >> p) & 1;
    const bool rpm = p >= 1 && ((mprev >> (p - 1)) & 1), rp0 = (mprev >> p) & 1,
               rpp = p + 1 < ml && ((mprev >> (p + 1)) & 1);
    // T_j row p = E_jj row p - sum_a A_j,j-1[p][a] U[a][:],  U = G_j-1 A_j-1,j;
    // U row p from T (G_j-1 row p) in a sliding window, T overwritten behind it
    CR prv{0, 0}, cur = T[0];
#pragma unroll
    for (int q = 0; q < MLMAX; ++q) {
      const CR nxt = q + 1 < MLMAX ? T[q + 1] : CR{0, 0};
      CR u{0, 0};
      if (q >= 1 && ((mprev >> (q - 1)) & 1)) fma_acc(u, prv, cpl[q - 1][2]);
      if ((mprev >> q) & 1) fma_acc(u, cur, cpl[q][1]);
      if (q + 1 < ml && ((mprev >> (q + 1)) & 1)) fma_acc(u, nxt, cpl[q + 1][0]);
      CR um, up;
      um.x = __shfl(u.x, p - 1, 64);
      um.y = __shfl(u.y, p - 1, 64);
      up.x = __shfl(u.x, p + 1, 64);
      up.y = __shfl(u.y, p + 1, 64);
      const bool rq = (mj >> q) & 1;
      CR v{0, 0};
      if (rp && rq) {
        v = q == p - 1 ? dg[0] : q == p ? dg[1] : q == p + 1 ? dg[2] : CR{0, 0};
        if (rpm) v = v - cplp[0] * um;
        if (rp0) v = v - cplp[1] * u;
        if (rpp) v = v - cplp[2] * up;
      } else if (p == q) {
        v = CR{1, 0};
      }
      T[q] = v;
      prv = cur;
      cur = nxt;
    }
    // Gauss-Jordan: T <- T^-1 (rows and columns beyond ml are identity)
    gj_wave_invert<R>(T, rowk, p);
    cd* out = d.G64 + ((size_t)s * ml + j) * n2;
    if (p < ml) {
#pragma unroll
      for (int q = 0; q < MLMAX; ++q)
        if (q < ml) out[q * ml + p] = cvt<double>(T[q]);
    }
    mprev = mj;
  }
}

// ---- multi_solve on the matrix cores ----
// The solves E^s X = [e_Delta, Z_rc] of the set-up, with every line
// product G_j Z (33 x 33 by 33 x 32, complex) on v_mfma_f64_16x16x4f64: rows and
// contraction index 0..31 as 2 x 8 tiles of 16 x 4 (complex = four real
// products), the 33rd row and column (ml = 33) on the vector units.  A
// workgroup of four wavefronts takes one subdomain, wavefront w the columns
// 32 w .. 32 w + 31; the wavefronts share nothing but the tables, so the line
// recursion runs without workgroup barriers.  The forward results t_j wait for
// the backward sweep in a per-workgroup slot of global scratch (ml x 32 complex
// per wavefront and line); the workgroups loop over the subdomains, so the
// scratch is at most MS_SLOTS_MAX slots whatever the batch size.
//
// Operand layouts (a wavefront of 64 lanes, l = lane), measured on gfx950:
// A (16 x 4): lane l holds A[l % 16][l / 16]; B (4 x 16): lane l holds
// B[l / 16][l % 16]; C/D (16 x 16): lane l, register r holds D[row][l % 16] with
// row = 4 r + l / 16 for v_mfma_f64_16x16x4f64 and row = 4 (l / 16) + r for
// v_mfma_f32_16x16x4f32.
constexpr int MS_COLS = 32;  // columns per wavefront
static_assert(MS_COLS == MS_WAVE_COLS, "columns per wavefront");

template <class R> struct Mfma;
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int r, int lq) { return 4 * r + lq; }
};
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int r, int lq) { return 4 * lq + r; }
};
typedef Mfma<double>::v4 d4v;
__device__ inline d4v mfma64(double a, double b, d4v c) { return Mfma<double>::op(a, b, c); }

// R: arithmetic (double on the FP64 matrix cores; float on the FP32 ones for the
// complex64 set-up); inputs and outputs are FP64.
template <class R, class Src>
__global__ void __launch_bounds__(256) k_multi_solve_mfma(Src src, int total, cd* mscr, size_t slot_cd) {
  using CR = C<R>;
  using MT = Mfma<R>;
  using v4 = typename MT::v4;
  __shared__ CR tb[4][MLMAX][MS_COLS];  // per wavefront: t_j (then x_j) of its columns
  __shared__ int slotmap[MLMAX * MLMAX];
  __shared__ int sdl[128];
  __shared__ CR cpl[MLMAX][3];
  __shared__ CR cst[4][9];
  __shared__ int cab[4][2];
  __shared__ int s_nc;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l & 15, lq = l >> 4;
  cd* slot = mscr + (size_t)blockIdx.x * slot_cd;
  for (int b = blockIdx.x; b < total; b += gridDim.x) {
    const Dev& d = src.dev_at(b);
    const Geo2& g = d.g;
    const Maps2& mp = d.mp;
    const int s = src.bx_at(b), ml = g.ml, n2 = ml * ml, ND = g.ND;
    const int nd = mp.nd[s];
    __syncthreads();  // the previous subdomain's tables are no longer read
    for (int i = threadIdx.x; i < n2; i += blockDim.x) slotmap[i] = -1;
    if (threadIdx.x < ml * 3) {
      const int p = threadIdx.x / 3, e = threadIdx.x % 3, a = p + e - 1;
      cpl[p][e] = cvt<R>((a >= 0 && a < ml) ? g.zloc(p, 1, a, 0) : cd{0.0, 0.0});
    }
    if (threadIdx.x < 36) {
      const int q = threadIdx.x / 9, e = threadIdx.x % 9;
      const int cl = mp.cloc[s * 4 + q];  // corners are listed first (compact)
      cd v{0.0, 0.0};
      if (cl >= 0) {
        const int ca = cl % ml, cb = cl / ml, a = ca + e % 3 - 1, bb = cb + e / 3 - 1;
        if (a >= 0 && a < ml && bb >= 0 && bb < ml) v = g.zloc(a, bb, ca, cb);
        if (e == 0) {
          cab[q][0] = ca;
          cab[q][1] = cb;
        }
      }
      cst[q][e] = cvt<R>(v);
    }
    if (threadIdx.x == 0) {
      int nc = 0;
      for (int q = 0; q < 4; ++q) nc += (mp.cloc[s * 4 + q] >= 0);
      s_nc = nc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nd; i += blockDim.x) {
      const int node = mp.dloc[s * ND + i];
      sdl[i] = node;
      slotmap[node] = i;
    }
    __syncthreads();
    const int ncol = nd + s_nc, c0 = w * MS_COLS;
    if (c0 >= ncol) continue;  // no columns for this wavefront (no barrier follows)
    const bool big = ml == MLMAX;  // the 33rd row and column exist
    const cd* G = d.G64 + (size_t)s * ml * n2;
    CR (*T)[MS_COLS] = tb[w];
    // Z[k][c] of line j: the right-hand side minus the coupling to line j - 1
    // (forward) or the coupling to line j + 1 (backward), masked to r nodes
    auto zval = [&](int k, int c, int j, bool fwd, uint64_t mj, uint64_t mo) -> CR {
      const int col = c0 + c;
      CR v{0, 0};
      if (k >= ml || col >= ncol || !((mj >> k) & 1)) return v;
      if (fwd) {
        if (col < nd) {
          if (sdl[col] == k + ml * j) v = CR{1, 0};
        } else {
          const int q = col - nd, da = k - cab[q][0] + 1, db = j - cab[q][1] + 1;
          if (da >= 0 && da < 3 && db >= 0 && db < 3) v = cst[q][da + 3 * db];
        }
        if (j > 0)
          for (int e = 0; e < 3; ++e) {
            const int a = k + e - 1;
            if (a >= 0 && a < ml && ((mo >> a) & 1)) v = v - cpl[k][e] * T[a][c];
          }
      } else {
        for (int e = 0; e < 3; ++e) {
          const int a = k + e - 1;
          if (a >= 0 && a < ml && ((mo >> a) & 1)) fma_acc(v, cpl[k][e], T[a][c]);
        }
      }
      return v;
    };
    // one line: X = C0 + sgn G_j Z with Z from zval; C0 = 0 (forward) or t_j (backward)
    auto line = [&](int j, bool fwd, uint64_t mj, uint64_t mo, v4 (&Cr)[2][2], v4 (&Ci)[2][2],
                    CR (&x32)[2]) {
      const cd* Gj = G + (size_t)j * n2;  // element (p, q) at [q ml + p]
      R br[8][2], bi[8][2];
      CR z32[2];
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
          const CR z = zval(4 * kk + lq, 16 * nt + lr, j, fwd, mj, mo);
          br[kk][nt] = z.x;
          bi[kk][nt] = z.y;
        }
        z32[nt] = big ? zval(32, 16 * nt + lr, j, fwd, mj, mo) : CR{0, 0};
      }
      wave_sync_lds();  // every read of T for Z is done before T is overwritten
      const R sg = fwd ? R(1) : R(-1);
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        if (16 * mt >= ml) continue;
        R ar[8], ai[8];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
          const int p = 16 * mt + lr, q = 4 * kk + lq;
          const CR a = cvt<R>((p < ml && q < ml) ? Gj[(size_t)q * ml + p] : cd{0.0, 0.0});
          ar[kk] = sg * a.x;
          ai[kk] = sg * a.y;
        }
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
          v4 cr = Cr[mt][nt], ci = Ci[mt][nt];
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) {
            if (4 * kk >= ml) break;
            cr = MT::op(ar[kk], br[kk][nt], cr);
            cr = MT::op(-ai[kk], bi[kk][nt], cr);
            ci = MT::op(ar[kk], bi[kk][nt], ci);
            ci = MT::op(ai[kk], br[kk][nt], ci);
          }
          if (big) {  // contraction index 32: rank-one term
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int p = 16 * mt + MT::row(r, lq);
              const CR gp = cvt<R>(Gj[(size_t)32 * ml + p]);
              CR acc{cr[r], ci[r]};
              fma_acc(acc, CR{sg * gp.x, sg * gp.y}, z32[nt]);
              cr[r] = acc.x;
              ci[r] = acc.y;
            }
          }
          Cr[mt][nt] = cr;
          Ci[mt][nt] = ci;
        }
      }
      if (big) {  // row 32: sum over this lane's contraction indices, then over the lane groups
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
          CR acc{0, 0};
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) {
            const CR gq = cvt<R>(Gj[(size_t)(4 * kk + lq) * ml + 32]);
            fma_acc(acc, gq, CR{br[kk][nt], bi[kk][nt]});
          }
          acc.x += __shfl_xor(acc.x, 16, 64);
          acc.y += __shfl_xor(acc.y, 16, 64);
          acc.x += __shfl_xor(acc.x, 32, 64);
          acc.y += __shfl_xor(acc.y, 32, 64);
          fma_acc(acc, cvt<R>(Gj[(size_t)32 * ml + 32]), z32[nt]);
          x32[nt] = x32[nt] + CR{sg * acc.x, sg * acc.y};
        }
      }
    };
    // write x_j (registers) to T, and the outputs of line j if out
    auto emit = [&](int j, const v4 (&Cr)[2][2], const v4 (&Ci)[2][2], const CR (&x32)[2], bool out) {
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int p = 16 * mt + MT::row(r, lq), c = 16 * nt + lr;
            if (p >= ml) continue;
            const CR xr{Cr[mt][nt][r], Ci[mt][nt][r]};
            const cd x = cvt<double>(xr);
            T[p][c] = xr;
            const int col = c0 + c;
            if (!out || col >= ncol) continue;
            const int node = p + ml * j, sl = slotmap[node];
            if (col < nd) {
              if (sl >= 0) d.Sinv64[((size_t)s * ND + sl) * ND + col] = x;
            } else {
              const int q = col - nd;
              if (sl >= 0) d.Phi64[((size_t)s * ND + sl) * NQ + q] = x;
              d.PhiFull[((size_t)s * n2 + node) * 4 + q] = x;
            }
          }
      if (big && lq == 0) {
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
          const int c = 16 * nt + lr, col = c0 + c, node = 32 + ml * j;
          T[32][c] = x32[nt];
          if (!out || col >= ncol) continue;
          const int sl = slotmap[node];
          const cd x = cvt<double>(x32[nt]);
          if (col < nd) {
            if (sl >= 0) d.Sinv64[((size_t)s * ND + sl) * ND + col] = x;
          } else {
            const int q = col - nd;
            if (sl >= 0) d.Phi64[((size_t)s * ND + sl) * NQ + q] = x;
            d.PhiFull[((size_t)s * n2 + node) * 4 + q] = x;
          }
        }
      }
      wave_sync_lds();
    };
    cd* wsl = slot + (size_t)w * ml * ml * MS_COLS;  // this wavefront's lines, ml x 32 each
    v4 Cr[2][2], Ci[2][2];
    CR x32[2];
    // steps 0 .. ml-1: forward sweep t_j = G_j (rhs_j - A_j,j-1 t_j-1), kept in T
    // and in the slot; steps ml .. 2 ml - 2: backward sweep x_j = t_j - G_j A_j,j+1 x_j+1
    // (T holds x_j+1).  One loop, so the line body is generated once.
    uint64_t mo = 0;  // r-node mask of the line the coupling reaches (j - 1 or j + 1)
    for (int step = 0; step < 2 * ml - 1; ++step) {
      const bool fwd = step < ml;
      const int j = fwd ? step : 2 * ml - 2 - step;
      const uint64_t mj = __ballot(l < ml && g.rnode(s, l, j));
      cd* o = wsl + (size_t)j * ml * MS_COLS;
      if (fwd) {
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
          for (int nt = 0; nt < 2; ++nt) Cr[mt][nt] = Ci[mt][nt] = v4{0, 0, 0, 0};
        x32[0] = x32[1] = CR{0, 0};
      } else {
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
          for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = 16 * mt + MT::row(r, lq);
              const CR t = cvt<R>(row < ml ? o[row * MS_COLS + 16 * nt + lr] : cd{0.0, 0.0});
              Cr[mt][nt][r] = t.x;
              Ci[mt][nt][r] = t.y;
            }
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) x32[nt] = cvt<R>(big ? o[32 * MS_COLS + 16 * nt + lr] : cd{0.0, 0.0});
      }
      line(j, fwd, mj, mo, Cr, Ci, x32);
      emit(j, Cr, Ci, x32, !fwd || j == ml - 1);
      if (fwd && j < ml - 1)
        for (int idx = l; idx < ml * MS_COLS; idx += 64) o[idx] = cvt<double>(T[idx / MS_COLS][idx % MS_COLS]);
      mo = mj;  // the next line (j + 1 forward, j - 1 backward) couples to this one
    }
  }
}

// In-place Gauss-Jordan inverse (no pivoting) of the nd_s x nd_s leading block
// of each subdomain's ND x ND matrix, one 1024-thread workgroup per subdomain
// with the matrix in registers: thread t holds row t / 8, columns t % 8 + 8 u
// (u < 16; nd_s <= 128); row k and column k of each pivot step pass through LDS.
constexpr int INV_EPT = 16;
template <class Src>
__global__ void __launch_bounds__(1024) k_invert_batched(Src src) {
  __shared__ cd rowk[128], colk[128];
  const Dev& d = src.dev();
  const int ND = d.g.ND;
  const int s = src.bx(), n = d.mp.nd[s];
  cd* M = d.S64 + (size_t)s * ND * ND;
  const int i = threadIdx.x >> 3, c8 = threadIdx.x & 7;
  const bool row_ok = i < n;
  cd e[INV_EPT];
#pragma unroll
  for (int u = 0; u < INV_EPT; ++u) {
    const int j = c8 + 8 * u;
    e[u] = (row_ok && j < n) ? M[(size_t)i * ND + j] : cd{0.0, 0.0};
  }
  for (int k = 0; k < n; ++k) {
    if (row_ok) {
#pragma unroll
      for (int u = 0; u < INV_EPT; ++u) {
        const int j = c8 + 8 * u;
        if (i == k && j < n) rowk[j] = e[u];
        if (j == k) colk[i] = e[u];
      }
    }
    __syncthreads();
    const cd piv = cdiv(cd{1.0, 0.0}, rowk[k]);
    if (row_ok) {
      const cd ci = colk[i];
#pragma unroll
      for (int u = 0; u < INV_EPT; ++u) {
        const int j = c8 + 8 * u;
        if (j >= n) continue;
        cd v;
        if (i == k && j == k) v = piv;
        else if (i == k) v = rowk[j] * piv;
        else if (j == k) v = -(ci * piv);
        else v = e[u] - ci * (rowk[j] * piv);
        e[u] = v;
      }
    }
    __syncthreads();
  }
  if (row_ok) {
#pragma unroll
    for (int u = 0; u < INV_EPT; ++u) {
      const int j = c8 + 8 * u;
      if (j < n) M[(size_t)i * ND + j] = e[u];
    }
  }
}

// Edge columns of the coarse basis: Phi64[s][i][4 + j] = sum over the Delta
// slots k on side j of the subdomain of Z_rr^-1|Delta[i][k] sign_k, i.e.
// Z_rr^-1 B_r^T q_e on Delta rows for the edge e on that side (q_e: ones on
// the edge's multipliers).  One workgroup per subdomain, thread i = row i.
template <class Src>
__global__ void __launch_bounds__(256) k_edge_basis(Src src) {
  const Dev& d = src.dev();
  const Geo2& g = d.g;
  const Maps2& mp = d.mp;
  const int s = src.bx(), ND = g.ND, nd = mp.nd[s];
  __shared__ int side[128];
  __shared__ float sg[128];
  for (int k = threadIdx.x; k < nd; k += blockDim.x) {
    side[k] = mp.dedge[s * ND + k] - 4;
    sg[k] = mp.dsgn[s * ND + k];
  }
  __syncthreads();
  const int i = threadIdx.x;
  if (i >= nd) return;
  const cd* row = d.Sinv64 + ((size_t)s * ND + i) * ND;
  cd acc[4] = {cd{0.0, 0.0}, cd{0.0, 0.0}, cd{0.0, 0.0}, cd{0.0, 0.0}};
  for (int k = 0; k < nd; ++k) {
    const cd v = (double)sg[k] * row[k];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (side[k] == j) acc[j] = acc[j] + v;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) d.Phi64[((size_t)s * ND + i) * NQ + 4 + j] = acc[j];
}

// Per-subdomain coarse blocks Zs[s][NQ][NQ] over the coarse slots:
//   corner x corner: Z_cc*^s = Z_cc - Z_cr Phi;
//   with an edge slot e: -q_e^T X, X the other slot's basis column (Z_rr^-1
//   Z_rc for a corner, Z_rr^-1 B_r^T q_f for an edge f), q_e the signs on
//   the side's Delta slots.  Entries of absent slots are zero.
template <class Src>
__global__ void k_zcc(Src src) {
  const Dev& d = src.dev();
  const Geo2& g = d.g;
  const Maps2& mp = d.mp;
  const cd* PhiFull = d.PhiFull;
  cd* Zs = d.Zs;
  int t = src.bx() * blockDim.x + threadIdx.x;
  if (t >= g.nsub * NQ * NQ) return;
  const int s = t / (NQ * NQ), q = (t / NQ) % NQ, q2 = t % NQ;
  cd v{0.0, 0.0};
  if (mp.cgid[s * NQ + q] >= 0 && mp.cgid[s * NQ + q2] >= 0) {
    if (q < 4 && q2 < 4) {
      const int cl = mp.cloc[s * 4 + q], cl2 = mp.cloc[s * 4 + q2];
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
    } else {
      const int e = q >= 4 ? q : q2, other = q >= 4 ? q2 : q;
      const int nd = mp.nd[s];
      for (int i = 0; i < nd; ++i)
        if (mp.dedge[s * g.ND + i] == e)
          v = v - (double)mp.dsgn[s * g.ND + i] * d.Phi64[((size_t)s * g.ND + i) * NQ + other];
    }
  }
  Zs[t] = v;
}

// Row c of the coarse matrix (c < nK) = sum over the subdomains sharing coarse
// unknown c (fixed order) of their block rows; slots beyond nK are left out.
template <class Src>
__global__ void k_coarse_assemble(Src src) {
  const Dev& d = src.dev();
  const Geo2& g = d.g;
  const Maps2& mp = d.mp;
  const cd* Zs = d.Zs;
  cd* Kcc = d.Kcc;
  const int n = g.nK;
  int c = src.bx() * blockDim.x + threadIdx.x;
  if (c >= n) return;
  cd* row = Kcc + (size_t)c * n;
  for (int k = 0; k < n; ++k) row[k] = cd{0.0, 0.0};
  for (int o = 0; o < 4; ++o) {
    int own = mp.cown[c * 4 + o];
    if (own < 0) continue;
    int s = own / NQ, slot = own % NQ;
    for (int q = 0; q < NQ; ++q) {
      int c2 = mp.cgid[s * NQ + q];
      if (c2 < 0 || c2 >= n) continue;
      row[c2] = row[c2] + Zs[((size_t)s * NQ + slot) * NQ + q];
    }
  }
}

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
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
}

// Inverse of a small coarse matrix (nK <= GJ_LDS_MAX) in LDS, one workgroup per
// instance: Kinv = GJ(Kcc); instances with larger coarse matrices return.
constexpr int GJ_LDS_MAX = 96;
template <class Src>
__global__ void __launch_bounds__(256) k_coarse_inv_lds(Src src) {
  extern __shared__ __align__(16) char smem[];
  const Dev& d = src.dev();
  const int n = d.g.nK;
  if (n > GJ_LDS_MAX) return;
  cd* T = (cd*)smem;
  cd* rowk = T + n * n;
  cd* colk = rowk + n;
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) T[i] = d.Kcc[i];
  __syncthreads();
  gj_invert_lds(T, n, rowk, colk);
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) d.Kinv[i] = T[i];
}

// Coarse inverse of a mid-size coarse matrix (GJ_LDS_MAX < nK <= GJ_BLOCK_MAX)
// by Gauss-Jordan without pivoting in global memory, one 1024-thread workgroup
// per instance: Kinv = GJ(Kcc), corners first.  Every entry is read and
// written by one owner thread (plain accesses, so a thread's loads of a step
// are in flight together); row k and column k, written by other threads, are
// copied to LDS through coherent loads after every wave has waited for its
// stores and passed the barrier.
constexpr int GJ_BLOCK_MAX = 256;
constexpr int GJ_BLOCK_BATCH = 4;  // fewest mid-size matrices for the one-workgroup path
__device__ inline cd gl_ld(const cd* p) {
  double x = __hip_atomic_load((const double*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  double y = __hip_atomic_load((const double*)p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return cd{x, y};
}
template <class Src>
__global__ void __launch_bounds__(1024) k_coarse_inv_block(Src src) {
  const Dev& d = src.dev();
  const int n = d.g.nK;
  if (n <= GJ_LDS_MAX || n > GJ_BLOCK_MAX) return;
  __shared__ cd rowk[GJ_BLOCK_MAX], colk[GJ_BLOCK_MAX];
  cd* T = d.Kinv;
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) T[i] = d.Kcc[i];
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
      rowk[t] = gl_ld(T + (size_t)k * n + t);
      colk[t] = gl_ld(T + (size_t)t * n + k);
    }
    __syncthreads();
    const cd piv = cdiv(cd{1.0, 0.0}, rowk[k]);
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
      const int i = idx / n, j = idx % n;
      cd v;
      if (i == k && j == k) v = piv;
      else if (i == k) v = rowk[j] * piv;
      else if (j == k) v = -(colk[i] * piv);
      else v = T[idx] - colk[i] * (rowk[j] * piv);
      T[idx] = v;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
}

// Per-subdomain helpers of the set-up (x = subdomain, y = 256-entry chunk).
// which: 0 Sinv64, 1 Phi64.
template <class Src>
__global__ void k_zero_sub(Src src, int which) {
  const Dev& d = src.dev();
  const int s = src.bx(), ND = d.g.ND;
  const size_t per = which == 0 ? (size_t)ND * ND : (size_t)ND * NQ;
  const size_t i = (size_t)blockIdx.y * blockDim.x + threadIdx.x;
  if (i >= per) return;
  (which == 0 ? d.Sinv64 : d.Phi64)[(size_t)s * per + i] = cd{0.0, 0.0};
}
template <class Src>
__global__ void k_copy_sub(Src src) {  // S64 = Sinv64
  const Dev& d = src.dev();
  const int s = src.bx(), ND = d.g.ND;
  const size_t per = (size_t)ND * ND;
  const size_t i = (size_t)blockIdx.y * blockDim.x + threadIdx.x;
  if (i < per) d.S64[(size_t)s * per + i] = d.Sinv64[(size_t)s * per + i];
}
// Storage of the FP64 results: which 0: G64 -> G (ml^3 per subdomain), 1: Phi64 -> Phi.
template <class TS, class Src>
__global__ void k_convert(Src src, int which) {
  const Dev& d = src.dev();
  const int s = src.bx(), ml = d.g.ml, ND = d.g.ND;
  const size_t per = which == 0 ? (size_t)ml * ml * ml : (size_t)ND * NQ;
  const size_t i = (size_t)blockIdx.y * blockDim.x + threadIdx.x;
  if (i >= per) return;
  const cd v = (which == 0 ? d.G64 : d.Phi64)[(size_t)s * per + i];
  ((TS*)(which == 0 ? d.G : d.Phi))[(size_t)s * per + i] =
      TS{(typename real_of<TS>::type)v.x, (typename real_of<TS>::type)v.y};
}
// Pack the leading nd x nd block of a subdomain's full ND x ND FP64 matrix into
// lower-triangle row-major storage (which 0: Sinv64 -> Sinv, 1: S64 -> Sbb).
template <class TD, class Src>
__global__ void k_pack(Src src, int which) {
  const Dev& d = src.dev();
  const int s = src.bx(), ND = d.g.ND;
  const int PK = ND * (ND + 1) / 2;
  int idx = blockIdx.y * blockDim.x + threadIdx.x;
  if (idx >= PK) return;
  int i = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > idx) --i;
  while ((i + 1) * (i + 2) / 2 <= idx) ++i;
  int k = idx - i * (i + 1) / 2;
  const cd* srcm = which == 0 ? d.Sinv64 : d.S64;
  cd v = (i < d.mp.nd[s]) ? srcm[((size_t)s * ND + i) * ND + k] : cd{0.0, 0.0};
  TD* dst = which == 0 ? (TD*)d.Sinv : (TD*)d.Sbb;
  dst[(size_t)s * PK + idx] = TD{(typename real_of<TD>::type)v.x, (typename real_of<TD>::type)v.y};
}


// Blocked Gauss-Jordan inverse (no pivoting) of a large n x n matrix in place:
// for each panel K of GJ_PB consecutive pivots (D = A_KK^-1),
//   A_ij -= (A_iK D) A_Kj   for i, j outside K,
//   A_iK  = -(A_iK D)       for i outside K,
//   A_Kj  = D A_Kj,  A_KK = D,
// which is the scalar Gauss-Jordan step applied a panel at a time.  Three
// launches per panel: the pivot block's inverse, the update outside the
// panel's rows and columns (which reads the old panel), then the panel's rows
// and columns.
constexpr int GJ_PB = 32;     // pivots per panel
constexpr int GJ_CT = 128;    // columns (or rows) per workgroup staged in LDS
// D = inverse of the b x b block of A at (k0, k0) (b <= GJ_PB, D row stride b) by
// Gauss-Jordan without pivoting, 256 threads: thread t keeps row t / 8, columns
// t % 8 + 8 r (r < 4) in registers; the pivot row and column pass through two
// alternating LDS buffers (L: 4 GJ_PB entries), so each pivot costs one barrier.
__device__ void gj_pivot_block(const cd* A, int n, int k0, int b, cd* D, cd* L) {
  const int i = threadIdx.x >> 3, jl = threadIdx.x & 7;
  cd v[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int j = jl + 8 * r;
    v[r] = (i < b && j < b) ? A[(size_t)(k0 + i) * n + k0 + j] : cd{0.0, 0.0};
  }
#pragma unroll
  for (int k = 0; k < GJ_PB; ++k) {
    if (k >= b) continue;  // b is uniform over the workgroup; a break would keep
                           // the loop rolled and v[k >> 3] dynamically indexed
    cd* rk = L + (k & 1) * 2 * GJ_PB;
    cd* ck = rk + GJ_PB;
    if (i == k) {
#pragma unroll
      for (int r = 0; r < 4; ++r) rk[jl + 8 * r] = v[r];
    }
    if (jl == (k & 7)) ck[i] = v[k >> 3];
    __syncthreads();
    const cd piv = cdiv(cd{1.0, 0.0}, rk[k]);
    const cd cp = ck[i] * piv;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = jl + 8 * r;
      const cd rj = rk[j];
      if (i == k) v[r] = (j == k) ? piv : rj * piv;
      else if (j == k) v[r] = -cp;
      else v[r] = v[r] - cp * rj;
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int j = jl + 8 * r;
    if (i < b && j < b) D[i * b + j] = v[r];
  }
}
// The kernels below take a batch of matrices: blockIdx.z selects A + z sA and
// its pivot-inverse buffers D + z sD.
__global__ void __launch_bounds__(256) k_gj_pivot(int n, int k0, int b, const cd* A, cd* D, size_t sA,
                                                  size_t sD) {
  __shared__ cd L[4 * GJ_PB];
  gj_pivot_block(A + blockIdx.z * sA, n, k0, b, D + blockIdx.z * sD, L);
}
// D into LDS with row stride GJ_PB, zero outside b x b.
__device__ inline void gj_load_d(cd* Dl, const cd* D, int b) {
  for (int t = threadIdx.x; t < GJ_PB * GJ_PB; t += blockDim.x) {
    const int r = t / GJ_PB, c = t % GJ_PB;
    Dl[t] = (r < b && c < b) ? D[r * b + c] : cd{0.0, 0.0};
  }
}
// The update outside the panel's rows and columns, A_ij -= (A_iK D) A_Kj, on
// the matrix cores (v_mfma_f64_16x16x4f64; operand layouts as for
// k_multi_solve_mfma).  Workgroup (x, y, z) takes rows 32 y .. 32 y + 31
// of matrix z and the columns [x jspan, (x + 1) jspan).  U = A_iK D (32 x b) is
// formed once in LDS and held by every wavefront as negated A operands; the
// wavefronts then sweep their columns in tiles of 16: C = A_ij (two 16 x 16
// tiles), C += (-U) A_Kj over the b <= 32 pivots of the panel (8 contraction
// steps of 4, four real products per complex one), stored back except in the
// panel's rows and columns.
constexpr int GJM_RT = 32;
__global__ void __launch_bounds__(256) k_gj_rows_mfma(int n, int k0, int b, int jspan, cd* A, const cd* D,
                                                      size_t sA, size_t sD) {
  __shared__ cd Dl[GJ_PB * GJ_PB], Ak[GJM_RT * GJ_PB], Ul[GJM_RT * GJ_PB];
  A += blockIdx.z * sA;
  D += blockIdx.z * sD;
  const int i0 = blockIdx.y * GJM_RT;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l & 15, lq = l >> 4;
  gj_load_d(Dl, D, b);
  for (int t = threadIdx.x; t < GJM_RT * GJ_PB; t += blockDim.x) {
    const int r = t / GJ_PB, c = t % GJ_PB, i = i0 + r;
    const bool in = i < n && c < b && (i < k0 || i >= k0 + b);
    Ak[t] = in ? A[(size_t)i * n + k0 + c] : cd{0.0, 0.0};
  }
  __syncthreads();
  for (int t = threadIdx.x; t < GJM_RT * GJ_PB; t += blockDim.x) {
    const int r = t / GJ_PB, c = t % GJ_PB;
    cd u{0.0, 0.0};
    for (int q = 0; q < b; ++q) fma_acc(u, Ak[r * GJ_PB + q], Dl[q * GJ_PB + c]);
    Ul[t] = u;  // zero for rows of the panel, beyond n, and columns beyond b
  }
  __syncthreads();
  double ar[2][8], ai[2][8];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const cd u = Ul[(16 * mt + lr) * GJ_PB + 4 * kk + lq];
      ar[mt][kk] = -u.x;
      ai[mt][kk] = -u.y;
    }
  bool rok[2][4];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + 16 * mt + 4 * r + lq;
      rok[mt][r] = i < n && (i < k0 || i >= k0 + b);
    }
  const int je = min(n, (int)(blockIdx.x + 1) * jspan);
  for (int j0 = blockIdx.x * jspan + 16 * w; j0 < je; j0 += 64) {
    const int j = j0 + lr;
    const bool jin = j < je, jok = jin && (j < k0 || j >= k0 + b);
    double br[8], bi[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int k = 4 * kk + lq;
      const cd v = (jin && k < b) ? A[(size_t)(k0 + k) * n + j] : cd{0.0, 0.0};
      br[kk] = v.x;
      bi[kk] = v.y;
    }
    d4v cr[2], ci[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + 16 * mt + 4 * r + lq;
        const cd v = (jok && rok[mt][r]) ? A[(size_t)i * n + j] : cd{0.0, 0.0};
        cr[mt][r] = v.x;
        ci[mt][r] = v.y;
      }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        cr[mt] = mfma64(ar[mt][kk], br[kk], cr[mt]);
        cr[mt] = mfma64(-ai[mt][kk], bi[kk], cr[mt]);
        ci[mt] = mfma64(ar[mt][kk], bi[kk], ci[mt]);
        ci[mt] = mfma64(ai[mt][kk], br[kk], ci[mt]);
      }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + 16 * mt + 4 * r + lq;
        if (jok && rok[mt][r]) A[(size_t)i * n + j] = cd{cr[mt][r], ci[mt][r]};
      }
  }
}
// The panel itself, after k_gj_rows_mfma (old panel values staged in LDS before any
// write): blocks [0, gx) take GJ_CT columns j each (the panel rows: A_Kj = D A_Kj,
// A_KK = D), blocks [gx, 2 gx) take GJ_CT rows i each outside the panel
// (A_iK = -A_iK D).  The two sets of entries are disjoint.  Block 2 gx inverts
// the next panel's pivot block (pivots below kend) into Dn: k_gj_rows_mfma has
// already given it its final value, and nothing here writes it.
__global__ void __launch_bounds__(256) k_gj_panel(int n, int k0, int b, int gx, int kend, cd* A, const cd* D,
                                                  cd* Dn, size_t sA, size_t sD) {
  __shared__ cd Dl[GJ_PB * GJ_PB], S[GJ_CT * (GJ_PB + 1)];
  A += blockIdx.z * sA;
  D += blockIdx.z * sD;
  Dn += blockIdx.z * sD;
  if ((int)blockIdx.x == 2 * gx) {
    const int k1 = k0 + b;
    if (k1 < kend) gj_pivot_block(A, n, k1, min(GJ_PB, kend - k1), Dn, S);
    return;
  }
  gj_load_d(Dl, D, b);
  const int half = threadIdx.x / GJ_CT, lo = threadIdx.x % GJ_CT;
  if ((int)blockIdx.x < gx) {
    const int j0 = blockIdx.x * GJ_CT;
    for (int t = threadIdx.x; t < GJ_PB * GJ_CT; t += blockDim.x) {
      const int q = t / GJ_CT, cc = t % GJ_CT, j = j0 + cc;
      S[q * GJ_CT + cc] = (q < b && j < n) ? A[(size_t)(k0 + q) * n + j] : cd{0.0, 0.0};
    }
    __syncthreads();
    const int j = j0 + lo;
    if (j >= n) return;
    if (j >= k0 && j < k0 + b) {
      for (int tt = 0; tt < 16; ++tt) {
        const int t = half * 16 + tt;
        if (t < b) A[(size_t)(k0 + t) * n + j] = Dl[t * GJ_PB + (j - k0)];
      }
      return;
    }
    cd v[16];
#pragma unroll
    for (int tt = 0; tt < 16; ++tt) v[tt] = cd{0.0, 0.0};
    for (int q = 0; q < b; ++q) {
      const cd old = S[q * GJ_CT + lo];
#pragma unroll
      for (int tt = 0; tt < 16; ++tt) fma_acc(v[tt], Dl[(half * 16 + tt) * GJ_PB + q], old);
    }
#pragma unroll
    for (int tt = 0; tt < 16; ++tt) {
      const int t = half * 16 + tt;
      if (t < b) A[(size_t)(k0 + t) * n + j] = v[tt];
    }
  } else {
    const int i00 = (blockIdx.x - gx) * GJ_CT;
    for (int t = threadIdx.x; t < GJ_CT * GJ_PB; t += blockDim.x) {
      const int rr = t / GJ_PB, q = t % GJ_PB, i = i00 + rr;
      S[rr * (GJ_PB + 1) + q] = (q < b && i < n) ? A[(size_t)i * n + k0 + q] : cd{0.0, 0.0};
    }
    __syncthreads();
    const int i = i00 + lo;
    if (i >= n || (i >= k0 && i < k0 + b)) return;
    cd u[16];
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) u[cc] = cd{0.0, 0.0};
    for (int q = 0; q < b; ++q) {
      const cd a = S[lo * (GJ_PB + 1) + q];
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) fma_acc(u[cc], a, Dl[q * GJ_PB + half * 16 + cc]);
    }
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
      const int c = half * 16 + cc;
      if (c < b) A[(size_t)i * n + k0 + c] = -u[cc];
    }
  }
}

// Gauss-Jordan pivots [kb, ke) of `batch` n x n matrices A + z sA in place
// (blocked steps above; work + z sW holds two pivot inverses, 2 GJ_PB^2
// entries).  Pivots [0, kb) must already have been taken.
hipError_t gj_range(int n, int kb, int ke, cd* A, size_t sA, cd* work, size_t sW, int batch, hipStream_t st) {
  if (ke <= kb) return hipSuccess;
  const int gx = (n + GJ_CT - 1) / GJ_CT;
  // outer update: rows by 32; columns split only when few matrices would leave
  // the device idle (the panel's U is then formed again per column block)
  const int gym = (n + GJM_RT - 1) / GJM_RT;
  const int gxm = batch * gym >= 1024 ? 1 : std::max(1, std::min((n + 63) / 64, (1024 + batch * gym - 1) / (batch * gym)));
  const int jspan = ((n + gxm - 1) / gxm + 63) / 64 * 64;
  hipLaunchKernelGGL(k_gj_pivot, dim3(1, 1, batch), dim3(256), 0, st, n, kb, std::min(GJ_PB, ke - kb),
                     (const cd*)A, work, sA, sW);
  for (int k0 = kb, p = 0; k0 < ke; k0 += GJ_PB, ++p) {
    const int b = std::min(GJ_PB, ke - k0);
    cd* D = work + (p & 1) * GJ_PB * GJ_PB;
    cd* Dn = work + ((p + 1) & 1) * GJ_PB * GJ_PB;
    hipLaunchKernelGGL(k_gj_rows_mfma, dim3(gxm, gym, batch), dim3(256), 0, st, n, k0, b, jspan, A,
                       (const cd*)D, sA, sW);
    hipLaunchKernelGGL(k_gj_panel, dim3(2 * gx + 1, 1, batch), dim3(256), 0, st, n, k0, b, gx, ke, A,
                       (const cd*)D, Dn, sA, sW);
  }
  return hipGetLastError();
}

// A^-1 in place (n > 64: work holds at least 2 GJ_PB^2 entries)
hipError_t invert_dense(int n, cd* A, cd* work, hipStream_t st) { return gj_range(n, 0, n, A, 0, work, 0, 1, st); }

// Every step of the set-up for every instance of the target (per-instance FP64
// scratch named by the views: G64, Sinv64, S64, Phi64, PhiFull, scr, Zs; and
// Kwork of each problem for large coarse matrices).
hipError_t launch_setup(const Target& t) {
  std::vector<Problem*> ps;
  if (t.single()) ps.push_back(t.one);
  else ps = t.probs;
  int ND = 0, ml = 0, ncmax = 0, nmid = 0;
  for (Problem* p : ps) {
    ND = std::max(ND, p->ND);
    ml = std::max(ml, p->ml);
    ncmax = std::max(ncmax, p->nK);
    nmid += p->nK > GJ_LDS_MAX && p->nK <= GJ_BLOCK_MAX;
  }
  // one workgroup per mid-size coarse matrix pays off only when several run
  // side by side; a few go panel by panel over the whole device instead
  const bool mid_block = nmid >= GJ_BLOCK_BATCH;
  const int yS = (ND * ND + 255) / 256, yP = (ND * NQ + 255) / 256, yG = (ml * ml * ml + 255) / 256;
  const int yK = (ND * (ND + 1) / 2 + 255) / 256;
  launch2(t, K_SUB, k_zero_sub<One>, k_zero_sub<Many>, yS, 256, 0, 0);
  launch2(t, K_SUB, k_zero_sub<One>, k_zero_sub<Many>, yP, 256, 0, 1);
  if (t.setup32)
    launch2(t, K_SUB, k_factor_lines_wave<float, One>, k_factor_lines_wave<float, Many>, 1, 64, 0);
  else
    launch2(t, K_SUB, k_factor_lines_wave<double, One>, k_factor_lines_wave<double, Many>, 1, 64, 0);
  {
    const int total = t.blocks(K_SUB), grid = std::min(total, MS_SLOTS_MAX);
    cd* mscr = ps[0]->ctx->ms_scr;
    size_t slot = 0;
    for (Problem* p : ps) slot = std::max(slot, ms_slot_cd(p->m));
    if (t.single() && t.setup32)
      hipLaunchKernelGGL((k_multi_solve_mfma<float, One>), dim3(grid), dim3(256), 0, t.st, t.src1(), total, mscr,
                         slot);
    else if (t.single())
      hipLaunchKernelGGL((k_multi_solve_mfma<double, One>), dim3(grid), dim3(256), 0, t.st, t.src1(), total, mscr,
                         slot);
    else if (t.setup32)
      hipLaunchKernelGGL((k_multi_solve_mfma<float, Many>), dim3(grid), dim3(256), 0, t.st, t.srcN(K_SUB), total,
                         mscr, slot);
    else
      hipLaunchKernelGGL((k_multi_solve_mfma<double, Many>), dim3(grid), dim3(256), 0, t.st, t.srcN(K_SUB), total,
                         mscr, slot);
  }
  launch2(t, K_SUB, k_edge_basis<One>, k_edge_basis<Many>, 1, 256, 0);
  launch2(t, K_SUB, k_copy_sub<One>, k_copy_sub<Many>, yS, 256, 0);
  launch2(t, K_SUB, k_invert_batched<One>, k_invert_batched<Many>, 1, 1024, 0);
  launch2(t, K_SUB16, k_zcc<One>, k_zcc<Many>, 1, 256, 0);
  launch2(t, K_NC128, k_coarse_assemble<One>, k_coarse_assemble<Many>, 1, 128, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // coarse inverses: small ones in LDS, every instance in one launch; mid-size
  // ones by one workgroup each in one launch when there are several (the kernel
  // skips the other sizes); the rest by panels of GJ_PB pivots, one matrix after
  // another
  {
    const int nl = std::min(ncmax, GJ_LDS_MAX);
    size_t lds = sizeof(cd) * ((size_t)nl * nl + 2 * nl);
    e = ensure_lds((const void*)k_coarse_inv_lds<One>, lds);
    if (e == hipSuccess) e = ensure_lds((const void*)k_coarse_inv_lds<Many>, lds);
    if (e != hipSuccess) return e;
    launch2(t, K_ONE, k_coarse_inv_lds<One>, k_coarse_inv_lds<Many>, 1, 256, lds);
  }
  if (mid_block) launch2(t, K_ONE, k_coarse_inv_block<One>, k_coarse_inv_block<Many>, 1, 1024, 0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (Problem* p : ps) {
    if (p->nK <= GJ_LDS_MAX || (mid_block && p->nK <= GJ_BLOCK_MAX)) continue;
    e = hipMemcpyAsync(p->Kinv, p->Kcc, sizeof(cd) * p->nK * p->nK, hipMemcpyDeviceToDevice, t.st);
    if (e == hipSuccess) e = invert_dense(p->nK, p->Kinv, p->Kwork, t.st);
    if (e != hipSuccess) return e;
  }
  if (t.g32()) launch2(t, K_SUB, k_convert<cf, One>, k_convert<cf, Many>, yG, 256, 0, 0);
  else launch2(t, K_SUB, k_convert<cd, One>, k_convert<cd, Many>, yG, 256, 0, 0);
  if (t.s32()) {
    launch2(t, K_SUB, k_convert<cf, One>, k_convert<cf, Many>, yP, 256, 0, 1);
    launch2(t, K_SUB, k_pack<cf, One>, k_pack<cf, Many>, yK, 256, 0, 0);
  } else {
    launch2(t, K_SUB, k_convert<cd, One>, k_convert<cd, Many>, yP, 256, 0, 1);
    launch2(t, K_SUB, k_pack<cd, One>, k_pack<cd, Many>, yK, 256, 0, 0);
  }
  launch2(t, K_SUB, k_pack<cf, One>, k_pack<cf, Many>, yK, 256, 0, 1);
  return hipGetLastError();
}

}  // namespace sfdp

// 3D instances (dim = 3): Q1 trilinear elements on the unit cube cut into P^3
// subdomains of m^3 cells (Sec. 5), FETI-DP with the subdomain vertices as
// corners and fully redundant multipliers.
//
// Layout on the device (ml = m + 1, nl = ml^3 local nodes):
//   local node l = a + ml b + ml^2 c of subdomain s = sx + P sy + P^2 sz sits at
//   full-grid node (sx m + a, sy m + b, sz m + c).  The remainder (r) nodes of a
//   subdomain are listed interior nodes first ((m-1)^3 of them, increasing local
//   index), then its Delta nodes (increasing local index); positions beyond its
//   r count, up to NR = nl - 8, pad the extended matrix E^s with the identity.
//   Zinv [nsub][NR][NR]  E^s^-1 (Z_rr^-1 on r x r), storage precision, full
//   Sinv [nsub][ND][ND]  Z_rr^-1 restricted to Delta, storage precision
//   Sbb  [nsub][ND][ND]  Schur complement of Z_rr on Delta (Dirichlet
//                        preconditioner), storage precision
//   Phi  [nsub][ND][8]   Z_rr^-1 Z_rc on Delta rows, storage precision
//   PhiFull [nsub][NR][8] Z_rr^-1 Z_rc on every r row (FP64)
//   Kinv [nC][nC]        inverse of the coarse matrix K_cc* (FP64)
// Vertex slot q of a subdomain is the vertex ((q & 1) m, ((q >> 1) & 1) m,
// ((q >> 2) & 1) m) (increasing local index); a vertex that is not a Dirichlet
// node is a corner (primal) unknown.
#pragma once
#include "common.h"

namespace sfdp {

struct Geo3 {
  int N, m, P, ml, nsub, nl, nI, NR, ND, nmu, nC;
  double h, alpha;
  int rshift;  // 1: the factor is the real K + alpha M (the outer factor of S_p)
  __host__ __device__ inline void loc(int l, int& a, int& b, int& c) const {
    a = l % ml;
    b = (l / ml) % ml;
    c = l / (ml * ml);
  }
  __host__ __device__ inline void base(int s, int& gi, int& gj, int& gk) const {
    gi = (s % P) * m;
    gj = ((s / P) % P) * m;
    gk = (s / (P * P)) * m;
  }
  __host__ __device__ inline bool dirich(int s, int a, int b, int c) const {
    int gi, gj, gk;
    base(s, gi, gj, gk);
    gi += a; gj += b; gk += c;
    return gi == 0 || gi == N || gj == 0 || gj == N || gk == 0 || gk == N;
  }
  // free-node index of local node (a, b, c); valid only when not Dirichlet
  __host__ __device__ inline int64_t freeidx(int s, int a, int b, int c) const {
    int gi, gj, gk;
    base(s, gi, gj, gk);
    const int64_t n1 = N - 1;
    return (int64_t)(gi + a - 1) + n1 * ((gj + b - 1) + n1 * (int64_t)(gk + c - 1));
  }
  // number of subdomains sharing local node (a, b, c) (non-Dirichlet)
  __host__ __device__ inline int mult(int a, int b, int c) const {
    return ((a == 0 || a == m) ? 2 : 1) * ((b == 0 || b == m) ? 2 : 1) * ((c == 0 || c == m) ? 2 : 1);
  }
  __host__ __device__ inline int vertex(int q) const {
    return (q & 1) * m + ml * (((q >> 1) & 1) * m) + ml * ml * (((q >> 2) & 1) * m);
  }
  // local Neumann matrix entry Z(l, l2) = K + i alpha M of the subdomain's
  // elements (K + alpha M when rshift)
  __host__ __device__ inline cd zloc(int l, int l2) const {
    int a, b, c, a2, b2, c2;
    loc(l, a, b, c);
    loc(l2, a2, b2, c2);
    if (a - a2 > 1 || a2 - a > 1 || b - b2 > 1 || b2 - b > 1 || c - c2 > 1 || c2 - c > 1) return cd{0.0, 0.0};
    Line1D L{h, m};
    const double kx = L.k(a, a2), mx = L.mm(a, a2), ky = L.k(b, b2), my = L.mm(b, b2), kz = L.k(c, c2),
                 mz = L.mm(c, c2);
    const double kk = kx * my * mz + mx * ky * mz + mx * my * kz, mm = alpha * mx * my * mz;
    return rshift ? cd{kk + mm, 0.0} : cd{kk, mm};
  }
};

// Device index maps of a 3D instance.
struct Maps3 {
  const int* rl;     // [nsub][NR] local node at r position p, -1 pad
  const int* rpos;   // [nsub][nl] r position of a local node, -1 if not an r node
  const int* nds;    // [nsub] Delta count (Delta positions nI .. nI + nds - 1)
  const int* dmu;    // [nsub][ND][3] multipliers of a Delta node, -1 pad
  const float* dsg;  // [nsub][ND][3] their signs on this subdomain (+1 / -1)
  const int* muown;  // [nmu][2] s * ND + delta of the + and the - side
  const int* cg;     // [nsub][8] global corner id of vertex slot q, -1 if Dirichlet
  const int* cown;   // [nC][8] owners s * 8 + q of a corner, -1 pad
};

// Host-side state of a 3D instance (device buffers owned by the problem).
struct Three {
  Geo3 g{};
  int *rl = nullptr, *rpos = nullptr, *nds = nullptr, *dmu = nullptr, *muown = nullptr, *cg = nullptr,
      *cown = nullptr;
  float* dsg = nullptr;
  // factors (storage precision for Zinv, Sinv, Sbb, Phi)
  void *Zinv = nullptr, *Sinv = nullptr, *Sbb = nullptr, *Phi = nullptr;
  cd *PhiFull = nullptr, *Zcc = nullptr;
  // solve workspaces (FP64 complex), NRMAX r-major copies: local vectors,
  // interface and coarse vectors, Krylov basis (kalloc + 1 vectors each) and
  // reduction buffers; hd holds per right-hand side the two Gram-Schmidt
  // coefficient sets and the squared norm (2 (kalloc + 1) + 1 entries)
  cd *T = nullptr, *Y = nullptr, *Wc = nullptr, *fcs = nullptr, *uc = nullptr, *gc = nullptr, *d = nullptr,
     *mu = nullptr, *z = nullptr, *w = nullptr, *V = nullptr, *part = nullptr, *hd = nullptr;
  double* npart = nullptr;
  int* nvd = nullptr;  // basis lengths of the final combination
  int kalloc = 0;
  cd* gs = nullptr;    // Givens state of the GMRES (device)
  int *gi = nullptr, *gih = nullptr;  // activity words (device, pinned host)
  Maps3 maps() const { return Maps3{rl, rpos, nds, dmu, dsg, muown, cg, cown}; }
};

// ---- launchers (three.hip) ----
// set-up of a 3D problem: E (FP64 scratch, nsub NR^2) and work (nsub 2 GJ_PB^2)
hipError_t launch_setup3(Problem& p, cd* E, cd* work);
// FETI-DP solves of nr <= NRMAX right-hand sides together (f, x with stride
// n_free): x = Z^-1 f (conj: x = conj(Z^-1 conj f)); its[r]: GMRES iterations
hipError_t feti3(Problem& p, int nr, const cd* f, cd* x, int conj, double tol, int kmax, int* its);
// interface products for testing: 'F' F_DP x, 'P' preconditioner, 'D' d for
// the right-hand side x (a complex free-node vector)
hipError_t interface3(Problem& p, char which, const cd* x, cd* y);
// flag words after a FETI-DP solve of right-hand side c (group slot q): its
// iteration count, and the slot's solve count and log
hipError_t launch_log3(Problem& p, int c, int q, int its);
// Gauss-Jordan pivots [kb, ke) of a batch of matrices (setup.hip)
hipError_t gj_range(int n, int kb, int ke, cd* A, size_t sA, cd* work, size_t sW, int batch, hipStream_t st);
hipError_t invert_dense(int n, cd* A, cd* work, hipStream_t st);

}  // namespace sfdp

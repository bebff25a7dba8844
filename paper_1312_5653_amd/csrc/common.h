// Internal declarations shared by the host code and the HIP kernels of sfdp.
//
// Layout of a problem on the device (2D; dim = 2, ml = m + 1 nodes per
// subdomain side, L = ml^2 local nodes, ND = padded Delta count):
//   local node l = a + ml * b of subdomain s = sx + P * sy sits at full-grid
//   node (sx m + a, sy m + b).  A local node is a remainder (r) node unless it
//   is a Dirichlet node or a subdomain vertex; vertices that are not Dirichlet
//   nodes are the corner (primal) unknowns of FETI-DP (Sec. 5).
//   The extended local matrix E^s is Z^s on r x r and the identity elsewhere,
//   so every subdomain has the same (ml lines) x (ml nodes) block-tridiagonal
//   shape; E^s^-1 restricted to r is Z_rr^s^-1.
//
//   G    [nsub][ml][ml][ml]  inverse Schur recursions G_j = T_j^-1 of the line
//                            block-tridiagonal LDL^T of E^s, stored transposed
//                            (element (i, k) of G_j at [j][k][i]).
//   Sinv [nsub][PK]          Z_rr^-1 restricted to Delta, packed lower triangle
//                            (PK = ND (ND + 1) / 2; storage precision)
//   Sbb  [nsub][PK]          interface Schur complement (its inverse), packed,
//                            complex64 on both paths (preconditioner only)
//   Phi  [nsub][ND][NQ]      coarse basis on Delta rows: Z_rr^-1 Z_rc for the
//                            four corner slots, Z_rr^-1 B_r^T q_e for the four
//                            edge slots (the edge averages of the augmentation)
//   Kinv [nK][nK]            inverse of the coarse matrix (FP64): K_cc*, or the
//                            edge-augmented matrix over corners then edges
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <functional>
#include <string>
#include <vector>

#include "../../include/sfdp.h"

namespace sfdp {

template <class R>
struct C {
  R x, y;
};
using cd = C<double>;
using cf = C<float>;

template <class R>
__host__ __device__ inline C<R> mk(R a, R b) { return C<R>{a, b}; }
template <class R>
__host__ __device__ inline C<R> operator+(C<R> a, C<R> b) { return {a.x + b.x, a.y + b.y}; }
template <class R>
__host__ __device__ inline C<R> operator-(C<R> a, C<R> b) { return {a.x - b.x, a.y - b.y}; }
template <class R>
__host__ __device__ inline C<R> operator-(C<R> a) { return {-a.x, -a.y}; }
template <class R>
__host__ __device__ inline C<R> operator*(C<R> a, C<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class R>
__host__ __device__ inline C<R> operator*(R s, C<R> a) { return {s * a.x, s * a.y}; }
template <class R>
__host__ __device__ inline C<R> conj(C<R> a) { return {a.x, -a.y}; }
template <class R>
__host__ __device__ inline R abs2(C<R> a) { return a.x * a.x + a.y * a.y; }
// fused a += b * c
template <class R>
__host__ __device__ inline void fma_acc(C<R>& a, C<R> b, C<R> c) {
  a.x = fma(b.x, c.x, a.x);
  a.x = fma(-b.y, c.y, a.x);
  a.y = fma(b.x, c.y, a.y);
  a.y = fma(b.y, c.x, a.y);
}
// a += conj(b) * c
template <class R>
__host__ __device__ inline void fma_conj_acc(C<R>& a, C<R> b, C<R> c) {
  a.x = fma(b.x, c.x, a.x);
  a.x = fma(b.y, c.y, a.x);
  a.y = fma(b.x, c.y, a.y);
  a.y = fma(-b.y, c.x, a.y);
}
template <class R>
__host__ __device__ inline C<R> cdiv(C<R> a, C<R> b) {
  R d = b.x * b.x + b.y * b.y;
  return {(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}
template <class R, class S>
__host__ __device__ inline C<R> cvt(C<S> a) { return C<R>{(R)a.x, (R)a.y}; }

// Real type of a complex storage type.
template <class T> struct real_of;
template <> struct real_of<cd> { using type = double; };
template <> struct real_of<cf> { using type = float; };

// 1D local (Neumann) P1 matrices on a subdomain side of m cells of size h:
//   k1 = (1/h) tridiag(-1, [1 2 ... 2 1], -1),  m1 = (h/6) tridiag(1, [2 4 ... 4 2], 1).
// The Q1 local matrix is the Kronecker sum  K = k1 (x) m1 + m1 (x) k1,  M = m1 (x) m1.
struct Line1D {
  double h;
  int m;
  __host__ __device__ inline double k(int a, int b) const {
    int d = a - b;
    if (d == 0) return ((a == 0 || a == m) ? 1.0 : 2.0) / h;
    if (d == 1 || d == -1) return -1.0 / h;
    return 0.0;
  }
  __host__ __device__ inline double mm(int a, int b) const {
    int d = a - b;
    if (d == 0) return ((a == 0 || a == m) ? 2.0 : 4.0) * h / 6.0;
    if (d == 1 || d == -1) return h / 6.0;
    return 0.0;
  }
};

// Coarse slots of a subdomain: 0..3 its corners, 4..7 the edges on its sides
// (left, right, bottom, top).  Global coarse unknowns: the nC corners, then
// the interface edges (when the coarse space is edge-augmented).
constexpr int NQ = 8;

// Geometry of one 2D instance, passed by value to kernels.
struct Geo2 {
  int N, m, P, ml, nsub, ND, nmu, nC, nK;  // nK: coarse unknowns (nC, or nC + edges)
  double h, alpha;
  int dim;     // 3: the free-node kernels of the range-space loop use the 3D grid
  int rshift;  // 1: the factor is the real K + alpha M (the outer factor of S_p)
  // subdomain coordinates
  __device__ __host__ inline int sx(int s) const { return s % P; }
  __device__ __host__ inline int sy(int s) const { return s / P; }
  // node classes of local node (a, b) of subdomain s
  __device__ __host__ inline bool dirich(int s, int a, int b) const {
    int gi = sx(s) * m + a, gj = sy(s) * m + b;
    return gi == 0 || gi == N || gj == 0 || gj == N;
  }
  __device__ __host__ inline bool vert(int a, int b) const {
    return (a == 0 || a == m) && (b == 0 || b == m);
  }
  __device__ __host__ inline bool rnode(int s, int a, int b) const {
    return !dirich(s, a, b) && !vert(a, b);
  }
  // free-node index of local node (a, b); valid only when not Dirichlet
  __device__ __host__ inline int freeidx(int s, int a, int b) const {
    int gi = sx(s) * m + a, gj = sy(s) * m + b;
    return (gi - 1) + (N - 1) * (gj - 1);
  }
  // number of subdomains sharing local node (a, b) (non-Dirichlet)
  __device__ __host__ inline int mult(int a, int b) const {
    return ((a == 0 || a == m) ? 2 : 1) * ((b == 0 || b == m) ? 2 : 1);
  }
  // local Neumann matrix entry Z((a,b),(a2,b2)) = K + i alpha M (K + alpha M
  // when rshift)
  __device__ __host__ inline cd zloc(int a, int b, int a2, int b2) const {
    Line1D L{h, m};
    double kx = L.k(a, a2), mx = L.mm(a, a2), ky = L.k(b, b2), my = L.mm(b, b2);
    const double kk = kx * my + mx * ky, mm = alpha * mx * my;
    return rshift ? cd{kk + mm, 0.0} : cd{kk, mm};
  }
  // extended matrix E: Z on r x r, identity elsewhere
  __device__ __host__ inline cd eloc(int s, int a, int b, int a2, int b2) const {
    bool r1 = rnode(s, a, b), r2 = rnode(s, a2, b2);
    if (r1 && r2) return zloc(a, b, a2, b2);
    if (a == a2 && b == b2) return cd{1.0, 0.0};
    return cd{0.0, 0.0};
  }
};

// Device-side index maps of one 2D instance (all arrays device-resident).
struct Maps2 {
  const int* dloc;   // [nsub][ND] local node index of Delta slot, -1 pad
  const int* dmid;   // [nsub][ND] multiplier id
  const float* dsgn; // [nsub][ND] +1 / -1, 0 pad
  const int* dpart;  // [nsub][ND] partner slot (t * ND + slot_t)
  const int* nd;     // [nsub] Delta count
  const int* cloc;   // [nsub][4] local node of corner slot, -1 pad
  const int* cgid;   // [nsub][NQ] global coarse id of each slot (edges from nC), -1 pad
  const int* muown;  // [nmu][2] (s+ * ND + slot+), (s- * ND + slot-)
  const int* mufree; // [nmu] free index of the multiplier's node
  const int* cown;   // [nC + nE][4] (s * NQ + slot) of the sharing subdomains, -1 pad
  const int* cfree;  // [nC] free index of each global corner
  const int* dedge;  // [nsub][ND] edge slot (4..7) of a Delta slot, -1 pad
  const int* muedge; // [nmu] interface edge of a multiplier
};

// Right-hand sides processed together by one FETI-DP solve (r-major copies of
// every per-RHS buffer).
constexpr int NRMAX = 4;
struct RhsStride {
  int64_t nf;   // free-node vectors
  int64_t nc;   // coarse vectors (nK)
  int64_t nmu;  // multiplier vectors
  int64_t sb;   // per-subdomain Delta-slot buffers (nsub * ND)
  int64_t cq;   // per-subdomain coarse-slot buffers (nsub * NQ)
};

// Device flag words of an instance: [1] grid-barrier error, [FLAG_NOTRES] a
// plain GMRES launch whose grid was not co-resident (it did no work), [3] GMRES loop
// trips, [4] GMRES iterations summed over right-hand sides, [FLAG_ITS + r]
// iterations of right-hand side r in the last GMRES launch, [FLAG_CNT + slot]
// FETI-DP solves logged for a group slot, [FLAG_LOG + 16 slot + k] their counts.
constexpr int FLAG_NOTRES = 2, FLAG_ITS = 8, FLAG_CNT = 16, FLAG_LOG = 64, FLAG_WORDS = FLAG_LOG + NRMAX * 16;

// Per-instance record gathered to the host after a step: residual heads
// (red[2 slot]: relative KKT residual, red[2 slot + 1]: imaginary ratio) and
// the flag words.
struct Gathered {
  double red[4 * NRMAX];  // [2 slot]: rho, [2 slot + 1]: imag ratio; from MET_HEAD the metrics
  int flags[FLAG_WORDS];
  int ready;              // set to 1 by the gather kernel after the rest (the host clears it)
};

// Selectors of an instance's complex vectors, passed to kernels so that one
// launch can address the same vector of every instance it covers.
enum VecSel : int { V_CVEC = 0, V_CVEC2 = 1, V_CVEC3 = 2, V_UF = 3, V_UX = 4, V_FCS = 5, V_YMIN = 6 };

// Caller arrays of one range-space slot (device pointers, one target each).
struct Slot {
  const double* ybar;
  const double* yc;  // Dirichlet data or null for zero
  double *y, *u, *lam;
};

// Device view of one instance: what every kernel reads about it.  A launch
// covers one instance (the view is a kernel argument) or many (an array of
// views in device memory and a block -> instance map).
struct Dev {
  Geo2 g;
  Maps2 mp;
  RhsStride rs;
  int g32, s32;       // storage: line factors / interface operators in complex64
  int nr;             // right-hand sides of the current group (0: instance idle)
  unsigned map;       // group slot of the c-th right-hand side in byte c
  int64_t n_free, n_bdry;
  double beta;
  const int* full2bdry;
  // factors
  void *G, *Sinv, *Phi;
  cf* Sbb;
  cd *Kcc, *Kinv;
  // FETI-DP workspaces (NRMAX r-major copies)
  cd *Xd, *Ubuf, *Abuf, *Ybuf, *Cbuf, *Qc, *fcs, *u0, *ymin, *dvec, *mu, *wv, *Qk, *Hk, *part;
  double* dscal;
  unsigned* bar;
  int* flags;
  int kstride;        // allocated Krylov depth (stride of Qk and Hk)
  // range-space workspaces
  double *r1, *r2, *r3, *red;
  cd *cvec, *cvec2, *cvec3;
  // caller arrays of the current call (device pointers)
  const cd* uf;       // FETI-DP right-hand sides (stride n_free)
  cd* ux;             // FETI-DP solutions
  Slot sl[NRMAX];     // range-space caller arrays of each group slot
  unsigned init;      // slots (bit s) whose iterate starts at (ybar, 0, 0) in group_init
  // share of the GMRES grid: first block, block count, multipliers per block
  int gb0, gnb, chunk, resident;
  // FP64 set-up scratch
  cd *G64, *Sinv64, *S64, *Phi64, *PhiFull, *scr, *Zs;
};

__host__ __device__ inline cd* dev_vec(const Dev& d, int sel) {
  switch (sel) {
    case V_CVEC: return d.cvec;
    case V_CVEC2: return d.cvec2;
    case V_CVEC3: return d.cvec3;
    case V_UF: return const_cast<cd*>(d.uf);
    case V_UX: return d.ux;
    case V_FCS: return d.fcs;
    default: return d.ymin;
  }
}

// Block sources.  One: a single instance whose view is the kernel argument,
// block index = blockIdx.x.  Many: instance = inst[blockIdx.x], block index
// within it = blockIdx.x - first[instance].
// dev_at(b) / bx_at(b): the same for block b of the map, for kernels whose
// workgroups loop over the blocks of a launch kind.
struct One {
  Dev d;
  __device__ inline const Dev& dev() const { return d; }
  __device__ inline int bx() const { return blockIdx.x; }
  __device__ inline const Dev& dev_at(int) const { return d; }
  __device__ inline int bx_at(int b) const { return b; }
};
struct Many {
  const Dev* devs;
  const int* inst;
  const int* first;
  __device__ inline const Dev& dev() const { return devs[inst[blockIdx.x]]; }
  __device__ inline int bx() const { return blockIdx.x - first[inst[blockIdx.x]]; }
  __device__ inline const Dev& dev_at(int b) const { return devs[inst[b]]; }
  __device__ inline int bx_at(int b) const { return b - first[inst[b]]; }
};

// Launch kinds: how many x-blocks an instance takes in a launch.
// K_NC128 / K_NC: 128 coarse unknowns per block / one per block; K_SUB16:
// NQ x NQ entries per subdomain in 256-entry blocks.
enum Kind : int { K_SUB = 0, K_NC128, K_NC, K_NMU256, K_ASM256, K_NF256, K_SUB16, K_ONE, K_GMRES, K_NKIND };

// Key of a captured refinement step (graph replay of a single 2D problem):
// everything a step's launches take by value that can change between calls.
struct StepKey {
  int nr = 0, kmax = 0, single = 0;
  unsigned map = 0, tune_gen = 0;
  int plain = 0;  // GMRES launch form captured (Problem::gmres_plain unless gmres_coop)
  double tin = 0;
  const void* ptr[5 * NRMAX] = {};  // the caller arrays of the group's slots
  bool operator==(const StepKey& o) const {
    if (nr != o.nr || kmax != o.kmax || single != o.single || map != o.map || tune_gen != o.tune_gen ||
        plain != o.plain || tin != o.tin)
      return false;
    for (int i = 0; i < 5 * NRMAX; ++i)
      if (ptr[i] != o.ptr[i]) return false;
    return true;
  }
};
struct StepGraph {
  StepKey key;
  hipGraphExec_t exec = nullptr;
};

// Host-side problem.
struct Ctx;
struct Three;    // state of a 3D instance (three.h)
struct Elastic;  // state of an elasticity instance (elastic.h)
struct Problem {
  Ctx* ctx = nullptr;
  int dim = 2, N = 0, m = 0, P = 0, nsub = 0, ml = 0, L = 0, ND = 0, nC = 0, nmu = 0, ndmax = 0;
  int nE = 0;          // interface edges
  int nK = 0;          // coarse unknowns in use: nC + nE (edge-augmented) or nC
  int nKmax() const { return nC + nE; }
  bool last_resident = false;  // last GMRES launch kept the Schur blocks in LDS
  int last_nrt = 0;            // right-hand-side width of the last GMRES kernel
  int64_t n_free = 0, n_bdry = 0;
  sfdp_precision prec = SFDP_FP64;
  double beta = 0, alpha = 0;
  double t_setup_ms = 0;  // host time of the last set-up (sfdp_set_beta or the batch's)
  bool factored = false;
  bool rshift = false;    // factors of K + alpha M instead of K + i alpha M
  Problem* pw = nullptr;  // twin with rshift, built on first use of S_p (Sec. 3.2)
  Three* t3 = nullptr;  // dim = 3: maps, factors and workspaces of the 3D path
  Elastic* el = nullptr;  // elasticity instance (dim = 3, three dofs per node)
  double* fsw = nullptr;   // full-space method: device vectors (9 x 3 n_free + sums)
  double* fsh = nullptr;   // and its pinned host scalars
  double* stage = nullptr; // device copies of host arrays (sfdp_opts.host_ptrs), stage_n doubles
  size_t stage_n = 0;
  // index maps (device)
  int *dloc = nullptr, *dmid = nullptr, *dpart = nullptr, *nd = nullptr, *cloc = nullptr,
      *cgid = nullptr, *muown = nullptr, *mufree = nullptr, *cown = nullptr, *cfree = nullptr,
      *dedge = nullptr, *muedge = nullptr;
  float* dsgn = nullptr;
  int* full2bdry = nullptr;  // [(N+1)^2] boundary index of a full-grid node, -1 if free
  // factors (storage precision: cd for FP64, cf for MIXED)
  void *G = nullptr, *Sinv = nullptr, *Sbb = nullptr, *Phi = nullptr;
  cd* Kcc = nullptr;
  cd* Kinv = nullptr;
  cd* Kwork = nullptr;
  // solve workspaces (FP64 complex)
  cd *Xd = nullptr, *Ubuf = nullptr, *Abuf = nullptr, *Ybuf = nullptr, *Cbuf = nullptr,
     *Qc = nullptr, *fcs = nullptr, *u0 = nullptr, *dvec = nullptr, *mu = nullptr, *wv = nullptr,
     *Qk = nullptr, *Hk = nullptr, *part = nullptr, *ymin = nullptr;
  double* dscal = nullptr;    // device scalars
  unsigned* bar = nullptr;    // grid barrier counter
  int* flags = nullptr;       // device flags / outputs of the GMRES kernel
  int kmax_alloc = 0, gmres_blocks = 0, gmres_parts = 0;
  // range-space workspaces (FP64)
  double *r1 = nullptr, *r2 = nullptr, *r3 = nullptr, *red = nullptr;
  cd *cvec = nullptr, *cvec2 = nullptr, *cvec3 = nullptr;
  size_t bytes = 0;
  // the current call: group size and slots, caller arrays
  int nr = 0;
  unsigned map = 0;
  const cd* uf = nullptr;
  cd* ux = nullptr;
  Slot sl[NRMAX] = {};
  unsigned init = 0;
  // caller arrays of slots 0..nr-1 as consecutive targets of stride n_free / n_bdry
  void set_slots(int nr_, const double* ybar, const double* yc, double* y, double* u, double* lam) {
    for (int c = 0; c < NRMAX; ++c)
      sl[c] = c < nr_ ? Slot{ybar + c * n_free, yc ? yc + c * n_bdry : nullptr, y + c * n_free,
                             u + c * n_free, lam + c * n_free}
                      : Slot{};
  }
  // set-up scratch (valid during sfdp_set_beta only)
  cd *G64 = nullptr, *Sinv64 = nullptr, *S64 = nullptr, *Phi64 = nullptr, *PhiFull = nullptr,
     *scr = nullptr, *Zs = nullptr;
  Gathered* gh = nullptr;  // gather record (pinned host, written by the gather kernel)
  // cooperative time-slicing: when set, the long solve loops call it at the
  // start of every refinement step and MINRES iteration (the server's solo
  // requests hand the device back to its worker there)
  void (*yield_fn)(void*) = nullptr;
  void* yield_arg = nullptr;
  void yield_point() const {
    if (yield_fn) yield_fn(yield_arg);
  }
  // captured refinement steps (graph replay) and the steps run once eagerly
  // (a step is captured the second time its key occurs); cleared whenever a
  // buffer, beta or the coarse space changes
  std::vector<StepGraph> graphs;
  std::vector<StepKey> graph_seen;
  bool graph_off = false;  // a capture failed: this problem runs eagerly
  // GMRES launch form of the current range-space call: 0 cooperative, 1 plain
  // launch that first checks that its grid is co-resident, 2 the same with no
  // wait in the check (tests of the fallback); gmres_coop: a plain launch found
  // its grid not co-resident once, so this problem launches cooperatively from then on
  int gmres_plain = 0;
  bool gmres_coop = false;
  // kernel timing (events recorded around hot kernel launches)
  int timing = 0;  // event timing: 0 off, 1 GMRES and subdomain-solve launches, 2 GMRES only
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_pending;  // (event index, kind: 0 gmres, 1 local)
  int ev_used = 0;
  double t_gmres_ms = 0, t_local_ms = 0;
  int64_t n_gmres = 0, n_local = 0, it_gmres = 0, it_rhs = 0;
  Maps2 maps() const {
    return Maps2{dloc, dmid, dsgn, dpart, nd, cloc, cgid, muown, mufree, cown, cfree, dedge, muedge};
  }
  // storage precision: line factors G (g32) and interface operators Sinv, Phi (s32)
  bool g32() const { return prec == SFDP_MIXED; }
  bool s32() const { return prec == SFDP_MIXED || prec == SFDP_MIXED_IFACE; }
  RhsStride rs() const {
    return RhsStride{n_free, (int64_t)std::max(nKmax(), 1), (int64_t)nmu, (int64_t)nsub * ND,
                     (int64_t)nsub * NQ};
  }
  Geo2 geo() const {
    return Geo2{N, m, P, ml, nsub, ND, nmu, nC, nK, 1.0 / N, alpha, dim, rshift ? 1 : 0};
  }
  // x-blocks of this instance in a launch of the given kind
  int blocks(int kind) const {
    switch (kind) {
      case K_SUB: return nsub;
      case K_NC128: return (nK + 127) / 128;
      case K_NC: return nK;
      case K_NMU256: return (nmu + 255) / 256;
      case K_ASM256: return (nmu + nC + 255) / 256;
      case K_NF256: return (int)((n_free + 255) / 256);
      case K_SUB16: return (nsub * NQ * NQ + 255) / 256;
      case K_ONE: return 1;
      default: return gmres_blocks;
    }
  }
  Dev dev() const {
    Dev d;
    d.g = geo();
    d.mp = maps();
    d.rs = rs();
    d.g32 = g32();
    d.s32 = s32();
    d.nr = nr;
    d.map = map;
    d.n_free = n_free;
    d.n_bdry = n_bdry;
    d.beta = beta;
    d.full2bdry = full2bdry;
    d.G = G; d.Sinv = Sinv; d.Phi = Phi; d.Sbb = (cf*)Sbb; d.Kcc = Kcc; d.Kinv = Kinv;
    d.Xd = Xd; d.Ubuf = Ubuf; d.Abuf = Abuf; d.Ybuf = Ybuf; d.Cbuf = Cbuf; d.Qc = Qc; d.fcs = fcs;
    d.u0 = u0; d.ymin = ymin; d.dvec = dvec; d.mu = mu; d.wv = wv; d.Qk = Qk; d.Hk = Hk; d.part = part;
    d.dscal = dscal; d.bar = bar; d.flags = flags; d.kstride = kmax_alloc;
    d.r1 = r1; d.r2 = r2; d.r3 = r3; d.red = red; d.cvec = cvec; d.cvec2 = cvec2; d.cvec3 = cvec3;
    d.uf = uf; d.ux = ux;
    for (int c = 0; c < NRMAX; ++c) d.sl[c] = sl[c];
    d.init = init;
    d.gb0 = 0; d.gnb = gmres_blocks; d.chunk = (nmu + gmres_blocks - 1) / std::max(gmres_blocks, 1);
    d.resident = gmres_blocks == nsub;
    d.G64 = G64; d.Sinv64 = Sinv64; d.S64 = S64; d.Phi64 = Phi64; d.PhiFull = PhiFull; d.scr = scr;
    d.Zs = Zs;
    return d;
  }
};

struct Ctx {
  int device = 0;
  size_t budget = 0, used = 0;
  hipStream_t stream = nullptr;
  int num_cu = 0;
  int max_lds = 65536;  // bytes of LDS one workgroup may allocate
  // FP64 set-up scratch shared by every sfdp_set_beta on this context (grown on
  // demand, counted in `used`)
  void* pool = nullptr;
  size_t pool_bytes = 0;
  // capture stream of graph-replayed steps and its ordering events (created on
  // first use; the library's stream may be the null stream, which cannot be captured)
  hipStream_t cap_stream = nullptr;
  hipEvent_t cap_ev[2] = {nullptr, nullptr};
  // line-solve slots of the set-up (MS_SLOTS_MAX at most, carved from the pool
  // by alloc_setup; valid during a set-up)
  cd* ms_scr = nullptr;
  // device address of the allocation-free entry point's scratch array on this
  // context's device (noalloc_scratch, taken at creation)
  double* scratch = nullptr;
  // problems (batch members and twins included) and servers made from this
  // context and not yet destroyed; sfdp_ctx_destroy refuses while it is > 0
  std::atomic<int> children{0};
};

// The instances one launch covers: a single problem (its view passed by value)
// or a batch (views in device memory, one block -> instance map per kind).
struct Target {
  hipStream_t st = nullptr;
  Problem* one = nullptr;            // single instance, or
  std::vector<Problem*> probs;       // the batch's instances (host side)
  const Dev* devs = nullptr;         // device views of the batch
  const int* inst[K_NKIND] = {};     // device block -> instance maps
  const int* first[K_NKIND] = {};    // device first block of each instance
  int total[K_NKIND] = {};           // x-blocks of a batch launch
  // batch GMRES: consecutive cooperative launches over groups of instances
  // whose blocks are co-resident (block -> instance map and block count each)
  struct GGroup {
    const int* inst;
    int total;
    std::vector<int> members;
  };
  std::vector<GGroup> ggroups;
  sfdp_precision prec = SFDP_FP64;
  bool setup32 = false;  // set-up line factorization and line solves in complex64 arithmetic
  bool single() const { return one != nullptr; }
  int blocks(int kind) const { return one ? one->blocks(kind) : total[kind]; }
  One src1() const { return One{one->dev()}; }
  Many srcN(int kind) const { return Many{devs, inst[kind], first[kind]}; }
  bool g32() const { return prec == SFDP_MIXED; }
  bool s32() const { return prec == SFDP_MIXED || prec == SFDP_MIXED_IFACE; }
};

// One launch over the target with the block map of `kind`.
template <class KOne, class KMany, class... A>
static inline void launch2(const Target& t, int kind, KOne k1, KMany kn, int gy, int block, size_t lds,
                           A... args) {
  if (t.single())
    hipLaunchKernelGGL(k1, dim3(t.blocks(kind), gy), dim3(block), lds, t.st, t.src1(), args...);
  else
    hipLaunchKernelGGL(kn, dim3(t.blocks(kind), gy), dim3(block), lds, t.st, t.srcN(kind), args...);
}

// ---- launch-variant autotuning (tune.cpp) ----
enum TuneFamily : int { TUNE_LOCAL_SOLVE = 1, TUNE_K3_LOCAL = 2, TUNE_K3_SWEEP = 3 };
struct TuneKey {
  int family, device, k0, k1, k2, k3;  // kernel family, device, shape and precision fields
  bool operator<(const TuneKey& o) const;
};
struct TuneEntry {
  TuneKey key;
  int choice;
};
// The variant to run for key: on the first call every candidate 0..ncand-1 is
// launched (launch(c); candidates must compute the same results and may run
// repeatedly) and timed on stream st; later calls return the kept choice.
// fallback when tuning is off or timing fails.  weight (optional, ncand
// entries) scales each candidate's measured time before the comparison: a
// weight above 1 makes a candidate that moves more bytes win only by that
// margin, since its traffic competes with work running beside it.
int tune_choice(const TuneKey& key, int ncand, int fallback, hipStream_t st, const std::function<void(int)>& launch,
                const float* weight = nullptr);
// changes whenever the tuning mode or the table is reset (part of StepKey)
unsigned tune_generation();
// on: autotune; force >= 0: run candidate `force` wherever a family has it;
// either call forgets every choice made so far
void tune_set_mode(bool on, int force);
int tune_table(TuneEntry* out, int cap);   // choices made so far (returns their count)

// ---- launchers implemented in the .hip files ----
// set-up (every instance of the target; FP64 scratch in the views)
// Set-up line solves: workgroups loop over the subdomains, each with a slot of
// global scratch for the forward results (per wavefront of 32 columns: ml lines
// of ml x 32 complex); at most MS_SLOTS_MAX slots (workgroups) per launch.
constexpr int MS_SLOTS_MAX = 512;
constexpr int MS_WAVE_COLS = 32;
// complex entries of a slot for subdomains of m x m cells (4m columns at most:
// the Delta slots and the corners)
inline size_t ms_slot_cd(int m) {
  const size_t ml = m + 1, nw = (4 * (size_t)m + MS_WAVE_COLS - 1) / MS_WAVE_COLS;
  return nw * ml * ml * MS_WAVE_COLS;
}
hipError_t launch_setup(const Target& t);
// solve: nr <= NRMAX right-hand sides per instance (the views' nr), r-major
// buffers with the strides of Problem::rs(); f and x name instance vectors
hipError_t launch_local_solve(const Target& t, int mode, int f, int conj_in, int x);
hipError_t launch_coarse_rhs(const Target& t, int f, int conj_in);
hipError_t launch_fetidp_rhs(const Target& t);
hipError_t launch_gmres(const Target& t, double tol, int kmax);
hipError_t launch_recover_coarse(const Target& t);
hipError_t launch_assemble_solution(const Target& t, int x, int conj_out);
hipError_t gmres_check(const Problem& p, int kmax);
// Raise the dynamic-LDS limit of kernel fn on the current device to at least
// lds bytes (cached: no runtime call when already high enough).
hipError_t ensure_lds(const void* fn, size_t lds);  // the one-RHS kernel fits (hipSuccess)
int gmres_capacity(const Problem& p, int kmax, int chunk, int width);  // co-resident GMRES blocks
hipError_t launch_interface_apply(Problem& p, char which, const cd* x, cd* y, hipStream_t st);
// ops
hipError_t launch_apply_K(const Problem& p, int nrhs, const double* x, const double* xc, double* y,
                          hipStream_t st);
hipError_t launch_apply_M(const Problem& p, int nrhs, const double* x, double* y, hipStream_t st);
// Batched range-space kernels: the views' nr right-hand sides, `map` packs the
// group slot of the c-th one in byte c.  red holds (rho, imag ratio) of slot s
// at red[2 s], red[2 s + 1]; per-block partial sums follow from RED_HEAD.
constexpr int RED_HEAD = 16;
// Accuracy metrics of slot s at red[MET_HEAD + 2 s] (relative constraint
// violation, Sec. 6.2) and red[MET_HEAD + 2 s + 1] (blockwise backward error);
// their MET_N per-block partial sums per slot follow the residual partials.
constexpr int MET_HEAD = 2 * NRMAX, MET_N = 11;
static_assert(MET_HEAD + 2 * NRMAX <= RED_HEAD, "metric heads overlap the partial sums");
int64_t red_pstride(const Problem& p);
hipError_t launch_kkt_residual(const Target& t);
// allocation-free KKT residual (ops.hip): a file-scope device array of this many
// doubles per device, its device address from noalloc_scratch (called once per
// device with that device current), the doubles one call of up to NRMAX
// right-hand sides needs, and the launch over a view whose red points into it
constexpr int64_t NOALLOC_SCRATCH_DOUBLES = 1 << 16;  // 512 KiB
constexpr int NOALLOC_MAX_DEVICES = 64;
hipError_t noalloc_scratch(int device, double** out);
int64_t noalloc_kkt_doubles(int64_t n_free);
hipError_t launch_kkt_residual_noalloc(const Dev& d, hipStream_t st, double* rel);
hipError_t launch_kkt_metrics(const Target& t);
hipError_t launch_make_rhs1(const Target& t);
hipError_t launch_make_rhs2(const Target& t);
hipError_t launch_update(const Target& t, int single);  // single: one complex solve per step
hipError_t launch_fill(void* ptr, size_t bytes, hipStream_t st);
hipError_t launch_fill_flags(const Target& t, int first, int count);
hipError_t launch_copy_real_to_complex(int64_t n, const double* x, cd* y, hipStream_t st);
hipError_t launch_copy(int64_t n, const double* x, double* y, hipStream_t st);
hipError_t launch_real_part(int64_t n, const cd* x, double* y, hipStream_t st);
hipError_t launch_imag_scaled(int64_t n, const cd* x, double s, double* y, hipStream_t st);  // y = s Im x
hipError_t launch_group_init(const Target& t);  // y = ybar, u = lam = 0 for the views' init slots
// full-space method: out = A x (x, out: three free-node blocks); out = scale M^-1 x;
// out = a x + b y + c z; out[0] = x . y (part: (n + 255) / 256 block sums)
hipError_t launch_kkt_apply(const Problem& p, const double* x, double* out, hipStream_t st);
hipError_t launch_mass_inverse(const Problem& p, const double* x, double scale, double* out, hipStream_t st);
hipError_t launch_lin3(int64_t n, double a, const double* x, double b, const double* y, double c, const double* z,
                       double* out, hipStream_t st);
hipError_t launch_dot(int64_t n, const double* x, const double* y, double* part, double* out, hipStream_t st);
// out[i]: instance i of the target; out is pinned host memory (hipHostMalloc),
// written by the kernel (then a system-scope fence), read after the stream is synchronized
hipError_t launch_gather(const Target& t, Gathered* out);

}  // namespace sfdp

// Linear-elasticity instances: the solid cantilever control of Sec. 6.2.
// Trilinear (Q1) elements with three displacement dofs per node on the box
// [0, L] x [0, 1] x [0, 1] (n cells per unit length), clamped on x = 0 and
// free elsewhere, cut into Px x Py x Pz cubic subdomains of m^3 cells (Sec. 5);
// FETI-DP with the three displacement dofs of every unclamped subdomain vertex
// as primal (corner) unknowns and fully redundant multipliers: one per pair of
// subdomains sharing an interface node, per displacement component.
//
// Numbering.  Grid node (i, j, k), 0 <= i <= L n, 0 <= j, k <= n; the free
// nodes (i > 0) are numbered x fastest, f = (i - 1) + L n (j + (n + 1) k), and
// free dof 3 f + c carries displacement component c.  Local node
// l = a + ml b + ml^2 c (ml = m + 1) of subdomain s = sx + Px (sy + Py sz) sits
// at grid node (sx m + a, sy m + b, sz m + c); local dof 3 l + comp.
//
// Everything that depends on the geometry lives in host-built tables, so the
// device kernels see dofs only.  The remainder (r) positions of subdomain s are
// its non-interface dofs (nodes of no other subdomain: interior and free
// surface), ni[s] of them, then its interface (Delta) dofs, nds[s] of them,
// then identity padding up to NR = max_s (ni + nds); three consecutive
// positions per node, in increasing local node index.  Vertex slot v (0..7) of
// a subdomain is the local node ((v & 1) m, ((v >> 1) & 1) m, ((v >> 2) & 1) m);
// corner slot q = 3 v + comp.
//
// Layout on the device (storage precision: complex128 for FP64, complex64 for
// the mixed modes):
//   Zinv    [nsub][NR][NR]  E^s^-1 = Z_rr^-1 on r x r, identity on padding
//   Sinv    [nsub][ND][ND]  Z_rr^-1 restricted to Delta (identity padding)
//   Sbb     [nsub][ND][ND]  S_bb = Sinv^-1, the Dirichlet preconditioner's
//                           interface Schur complement
//   Phi     [nsub][ND][24]  Z_rr^-1 Z_rc on the Delta rows
//   PhiFull [nsub][NR][24]  Z_rr^-1 Z_rc on every r row (FP64)
//   Zrc     [nsub][NR][24]  coupling of the r dofs to the corner dofs (FP64)
//   Kinv    [nC][nC]        inverse of the coarse matrix K_cc* (FP64)
//   K, M    CSR over the free dofs (FP64, one column structure)
#pragma once
#include <string>
#include <utility>
#include <vector>

#include "common.h"
#include "krylov3.h"

namespace sfdp {

constexpr int EQ = 24;       // corner slots of a subdomain (8 vertices x 3 components)
constexpr int EL_M_MAX = 6;  // subdomain edge in cells: NR <= 3 * 7^3 - 24 = 1005 rows per workgroup

struct GeoE {
  int n, m, ml, L, nx, ny, nz, Px, Py, Pz, nsub, NR, ND, nmu, nC;
  int64_t n_free;
  double alpha;
  int rshift;  // 1: the factor is the real K + alpha M
};

// Device index maps of an elasticity instance.
struct MapsE {
  const int* rdof;   // [nsub][NR] local dof of r position p, -1 pad
  const int* rfree;  // [nsub][NR] free dof of r position p, -1 pad
  const float* rw;   // [nsub][NR] 1 / (subdomains sharing its node), 0 pad
  const int* ni;     // [nsub] non-interface r positions
  const int* nds;    // [nsub] interface (Delta) dofs, at r positions ni .. ni + nds - 1
  const float* dw;   // [nsub][ND] 1 / (subdomains sharing the node) of a Delta dof
  const int* dmu;    // [nsub][ND][3] multipliers of a Delta dof, -1 pad
  const float* dsg;  // [nsub][ND][3] their signs on this subdomain (+1 / -1)
  const int* muown;  // [nmu][2] s * ND + d of the + and the - copy
  const float* muw;  // [nmu] 1 / (subdomains sharing the node)
  const int* cdof;   // [nsub][EQ] local dof of corner slot q, -1 if clamped
  const int* cg;     // [nsub][EQ] corner id, -1 if clamped
  const int* cown;   // [nC][8] owners s * EQ + q (increasing s), -1 pad
  const float* cw;   // [nC] 1 / owners
  const int* cfree;  // [nC] free dof of the corner
  const int* fcor;   // [n_free] corner id of a free dof, -1 if not a corner
  const int* fown;   // [n_free][4] copies s * NR + p of a non-corner free dof, -1 pad
  const double* Ke;  // [24][24] element stiffness, then [8][8] scalar element mass
};

// Solve strides (right-hand side r of a buffer at + r * stride).
struct StrE {
  int64_t f;   // free-dof vectors: n_free
  int64_t t;   // local r vectors: nsub NR
  int64_t y;   // local Delta vectors: nsub ND
  int64_t w;   // corner terms: nsub EQ
  int64_t c;   // coarse vectors: nC
  int64_t mu;  // interface vectors: nmu
};

// Active right-hand sides of a refinement step: target idx[c] of the group is
// the c-th right-hand side of the step's FETI-DP solves.
struct ActE {
  int n;
  int idx[NRMAX];
};

// Caller arrays of the targets of a group (slot i: the group's i-th target).
struct SlotE {
  const double* ybar[NRMAX];
  double* y[NRMAX];
  double* u[NRMAX];
  double* lam[NRMAX];
};

// KKT partial sums per right-hand side, in this order (squares of):
//   r1, r2, r3, K y, |M||y|, |K||lam|, M ybar, |M||u|, |M||lam|, |K||y|
constexpr int EL_SUMS = 10;

struct Elastic {
  GeoE g{};
  double young = 0, poisson = 0;
  // maps (device)
  int *rdof = nullptr, *rfree = nullptr, *ni = nullptr, *nds = nullptr, *dmu = nullptr, *muown = nullptr,
      *cdof = nullptr, *cg = nullptr, *cown = nullptr, *cfree = nullptr, *fcor = nullptr, *fown = nullptr;
  float *rw = nullptr, *dw = nullptr, *dsg = nullptr, *muw = nullptr, *cw = nullptr;
  double* Ke = nullptr;
  // global operators (CSR over the free dofs, FP64)
  int *rp = nullptr, *ci = nullptr;
  double *Kv = nullptr, *Mv = nullptr;
  int64_t nnz = 0;
  // factors
  void *Zinv = nullptr, *Sinv = nullptr, *Sbb = nullptr, *Phi = nullptr;
  cd *PhiFull = nullptr, *Zrc = nullptr, *Zcc = nullptr, *Kcc = nullptr, *Kinv = nullptr;
  // FETI-DP workspaces (NRMAX copies)
  cd *T = nullptr, *Y = nullptr, *Wc = nullptr, *fcs = nullptr, *uc = nullptr, *gc = nullptr;
  KBuf kb{};
  // range-space workspaces (NRMAX copies): residual blocks, complex vectors,
  // block partial sums and their per-target totals (device, pinned host)
  double *r1 = nullptr, *r3 = nullptr, *part = nullptr, *sums = nullptr, *sumh = nullptr;
  cd *c1 = nullptr, *c2 = nullptr, *c3 = nullptr;
  // host copies of the geometry tables used by the host (load vectors, inspection)
  std::vector<int> h_ni, h_nds, h_rdof, h_cg;
  // allocations: maps and factors (kept), Krylov workspace (grown with kmax)
  std::vector<std::pair<void*, size_t>> owned, kowned;
  Elastic* fwd = nullptr;  // twin holding the factors of K alone (forward solves)
  MapsE maps() const {
    return MapsE{rdof, rfree, rw, ni, nds, dw, dmu, dsg, muown, muw, cdof, cg, cown, cw, cfree, fcor, fown, Ke};
  }
  StrE str() const {
    return StrE{g.n_free, (int64_t)g.nsub * g.NR, (int64_t)g.nsub * g.ND, (int64_t)g.nsub * EQ,
                (int64_t)std::max(g.nC, 1), (int64_t)std::max(g.nmu, 1)};
  }
};

// ---- host helpers of the library (api.cpp) ----
sfdp_status host_fail(sfdp_status s, const std::string& msg);
sfdp_status dev_alloc(Problem& p, void** ptr, size_t bytes);
void dev_free(Problem& p, void*& ptr, size_t bytes);

// ---- elasticity entry points behind the C ABI (elastic.cpp) ----
sfdp_status el_build(Problem& p, int n, int sub_elem, int length, double young, double poisson);
void el_destroy(Problem& p);
sfdp_status el_setup(Problem& p);
sfdp_status el_feti(Problem& p, int conj, int nrhs, const cd* f, cd* x, const sfdp_opts* o, int* its);
sfdp_status el_range_space(Problem& p, int nrhs, const double* ybar, double* y, double* u, double* lam,
                           const sfdp_opts* o, sfdp_info* info);
sfdp_status el_schur_inv(Problem& p, int nrhs, const double* r, double* z, const sfdp_opts* o, sfdp_info* info);
sfdp_status el_apply(Problem& p, char which, int nrhs, const double* x, double* y);
sfdp_status el_kkt(Problem& p, int nrhs, const double* ybar, const double* y, const double* u, const double* lam,
                   double* rel, double* eta, double* viol);
sfdp_status el_interface(Problem& p, char which, const cd* x, cd* y);
sfdp_status el_inspect(Problem& p, sfdp_query what, int sub, double* out, int* rows, int* cols);
sfdp_status el_pressure(Problem& p, double pressure, double* f);
sfdp_status el_forward(Problem& p, int nrhs, const double* f, double* u, const sfdp_opts* o, int* its);

// ---- launchers (elastic.hip) ----
// set-up of Z = K + i alpha M (K + alpha M with rshift): FP64 scratch E
// (nsub NR^2), E2 (nsub ND^2) and the Gauss-Jordan pivot buffers work
// (nsub 2 GJ_PB^2)
hipError_t el_launch_setup(Elastic& el, bool s32, cd* Kcc, cd* Kinv, cd* E, cd* E2, cd* work, hipStream_t st);
// x = Z^-1 f for nr <= NRMAX right-hand sides (stride n_free; conj: x = conj(Z^-1 conj f))
hipError_t el_launch_feti(Elastic& el, bool s32, const cd* Kinv, int nr, const cd* f, cd* x, int conj,
                          double tol, int kmax, int* its, hipStream_t st);
// interface products for testing ('F', 'P', 'D' as for the scalar paths)
hipError_t el_launch_interface(Elastic& el, bool s32, const cd* Kinv, char which, const cd* x, cd* y,
                               hipStream_t st);
// y_r = K x_r or M x_r (real, nr right-hand sides of stride n_free)
hipError_t el_launch_spmv(const Elastic& el, char which, int nr, const double* x, double* y, hipStream_t st);
// KKT residual blocks r1, r3 (when keep) of the nr targets of sl, and their
// EL_SUMS squared norms into el.sums[i * EL_SUMS + e] (device)
hipError_t el_launch_kkt(Elastic& el, int nr, const SlotE& sl, double beta, bool keep, hipStream_t st);
// c1 = -r3 - i alpha r1 for the active targets
hipError_t el_launch_rhs1(Elastic& el, const ActE& a, double alpha, hipStream_t st);
// c3 = conj(r1 + M c2) for the active targets
hipError_t el_launch_rhs2(Elastic& el, const ActE& a, hipStream_t st);
// y -= Re c2, lam += Re c1, u = lam / beta for the active targets, and the
// squared norms of Im c1 and Re c1 into el.sums[(NRMAX + c) * EL_SUMS + 0 / 1]
hipError_t el_launch_update(Elastic& el, const ActE& a, const SlotE& sl, double beta, hipStream_t st);
hipError_t el_launch_fill(void* ptr, size_t bytes, hipStream_t st);
hipError_t el_launch_r2c(int64_t n, const double* x, cd* y, hipStream_t st);
// y = Re x, or (im) y = Im x * s
hipError_t el_launch_c2r(int64_t n, const cd* x, int im, double s, double* y, hipStream_t st);

}  // namespace sfdp

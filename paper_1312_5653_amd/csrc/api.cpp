// Host side of the sfdp C ABI: partition and interface maps (Sec. 5), setup
// sequencing, the FETI-DP driver and the range-space refinement loop
// (Sec. 3.1 Schur system with the Sec. 4 complex factorization).
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "elastic.h"
#include "krylov3.h"
#include "three.h"

namespace sfdp {
}  // namespace sfdp

using namespace sfdp;

static thread_local std::string g_err;

// A report with the accuracy metrics marked as not computed.
static sfdp_info blank_info() {
  sfdp_info o{};
  o.constr_viol = -1.0;
  o.eta_blk = -1.0;
  return o;
}

static double wall_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static sfdp_status fail(sfdp_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(SFDP_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace {

constexpr int KMAX_LIMIT = 400;

// Captured refinement steps of a problem refer to its buffers, beta and coarse
// space by value: drop them whenever one of those changes.
void graphs_clear(Problem& p) {
  for (StepGraph& g : p.graphs)
    if (g.exec) hipGraphExecDestroy(g.exec);
  p.graphs.clear();
  p.graph_seen.clear();
}
std::atomic<bool> g_graphs{false};  // sfdp_set_graphs
std::atomic<int> g_gmres_launch{1};  // sfdp_set_gmres_launch
std::atomic<int> g_setup_bits{64};  // sfdp_set_setup_arithmetic

sfdp_status dalloc(Problem& p, void** ptr, size_t bytes) {
  graphs_clear(p);
  Ctx* c = p.ctx;
  if (c->budget && c->used + bytes > c->budget)
    return fail(SFDP_E_NOMEM, "memory budget exceeded");
  hipError_t e = hipMalloc(ptr, bytes ? bytes : 16);
  if (e != hipSuccess) return fail(SFDP_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  c->used += bytes;
  p.bytes += bytes;
  return SFDP_OK;
}

template <class T>
sfdp_status dupload(Problem& p, T** dst, const std::vector<T>& src) {
  sfdp_status s = dalloc(p, (void**)dst, sizeof(T) * std::max<size_t>(src.size(), 1));
  if (s != SFDP_OK) return s;
  if (!src.empty()) HIPCHK(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
  return SFDP_OK;
}

void dfree(Problem& p, void*& ptr, size_t bytes) {
  graphs_clear(p);
  if (ptr) {
    hipFree(ptr);
    p.ctx->used -= std::min(p.ctx->used, bytes);
    p.bytes -= std::min(p.bytes, bytes);
  }
  ptr = nullptr;
}

// ---- host-array staging (sfdp_opts.host_ptrs) ----
// The calls that take sfdp_opts accept host arrays: inputs go into a device
// buffer the problem keeps (grown on demand, charged to the memory budget),
// the call runs on device pointers with host_ptrs cleared, and the outputs
// are copied back on the context's stream before the call returns.
namespace {
bool host_ptrs(const sfdp_opts* o) { return o && o->host_ptrs == 1; }
sfdp_status check_host_ptrs(const sfdp_opts* o) {
  if (o && o->host_ptrs != 0 && o->host_ptrs != 1) return fail(SFDP_E_INVALID, "host_ptrs must be 0 or 1");
  return SFDP_OK;
}
sfdp_status stage_area(Problem& p, size_t doubles, double** d) {
  if (doubles > p.stage_n) {
    dfree(p, (void*&)p.stage, sizeof(double) * p.stage_n);
    p.stage_n = 0;
    sfdp_status s = dalloc(p, (void**)&p.stage, sizeof(double) * doubles);
    if (s) return s;
    p.stage_n = doubles;
  }
  *d = p.stage;
  return SFDP_OK;
}
sfdp_status stage_in(Problem& p, double* d, const double* h, size_t n) {
  HIPCHK(hipMemcpyAsync(d, h, sizeof(double) * n, hipMemcpyHostToDevice, p.ctx->stream));
  return SFDP_OK;
}
sfdp_status stage_out(Problem& p, double* h, const double* d, size_t n) {
  HIPCHK(hipMemcpyAsync(h, d, sizeof(double) * n, hipMemcpyDeviceToHost, p.ctx->stream));
  return SFDP_OK;
}
sfdp_status stage_done(Problem& p) {
  HIPCHK(hipStreamSynchronize(p.ctx->stream));
  return SFDP_OK;
}
}  // namespace

// Build the 2D partition and interface maps on the host.
// Largest coarse problem for which the edge-augmented space is the default.
constexpr int KAUG_DEFAULT_MAX = 1024;

sfdp_status build_maps(Problem& p) {
  const int N = p.N, m = p.m, P = p.P, ml = p.ml, ND = p.ND, nsub = p.nsub;
  std::vector<int> dloc(nsub * ND, -1), dmid(nsub * ND, 0), dpart(nsub * ND, 0), ndv(nsub, 0);
  std::vector<float> dsgn(nsub * ND, 0.f);
  std::vector<int> cloc(nsub * 4, -1), cgid(nsub * NQ, -1), dedge(nsub * ND, -1);
  // Delta nodes grouped by full id
  std::map<long, std::vector<std::pair<int, int>>> owners;  // full id -> (s, slot)
  for (int s = 0; s < nsub; ++s) {
    int sx = s % P, sy = s / P, nd = 0, nc = 0;
    for (int l = 0; l < ml * ml; ++l) {
      int a = l % ml, b = l / ml;
      int gi = sx * m + a, gj = sy * m + b;
      bool dir = gi == 0 || gi == N || gj == 0 || gj == N;
      bool vert = (a == 0 || a == m) && (b == 0 || b == m);
      bool inter = a > 0 && a < m && b > 0 && b < m;
      if (dir) continue;
      if (vert) {
        cloc[s * 4 + nc] = l;
        ++nc;
      } else if (!inter) {
        if (nd >= ND) return fail(SFDP_E_INVALID, "interface slot overflow");
        dloc[s * ND + nd] = l;
        dedge[s * ND + nd] = a == 0 ? 4 : a == m ? 5 : b == 0 ? 6 : 7;  // side of the subdomain
        owners[(long)gi + (long)(N + 1) * gj].push_back({s, nd});
        ++nd;
      }
    }
    ndv[s] = nd;
    p.ndmax = std::max(p.ndmax, nd);
  }
  // interface edges in increasing (lower, upper) subdomain-pair order: for each
  // s, the edge to s + 1 (its right side), then the edge to s + P (its top)
  std::vector<int> eright(nsub, -1), etop(nsub, -1);
  int ne = 0;
  for (int s = 0; s < nsub; ++s) {
    if (s % P < P - 1) eright[s] = ne++;
    if (s / P < P - 1) etop[s] = ne++;
  }
  p.nE = ne;
  int nmu = 0;
  std::vector<int> muown, mufree, muedge;
  for (auto& kv : owners) {
    auto& v = kv.second;
    if (v.size() != 2) return fail(SFDP_E_INVALID, "2D interface node not shared by two subdomains");
    std::sort(v.begin(), v.end());
    long f = kv.first;
    int gi = (int)(f % (N + 1)), gj = (int)(f / (N + 1));
    int k = nmu++;
    auto [sa, ia] = v[0];
    auto [sb, ib] = v[1];
    dmid[sa * ND + ia] = k;
    dsgn[sa * ND + ia] = 1.f;
    dpart[sa * ND + ia] = sb * ND + ib;
    dmid[sb * ND + ib] = k;
    dsgn[sb * ND + ib] = -1.f;
    dpart[sb * ND + ib] = sa * ND + ia;
    muown.push_back(sa * ND + ia);
    muown.push_back(sb * ND + ib);
    mufree.push_back((gi - 1) + (N - 1) * (gj - 1));
    const int e = sb == sa + 1 ? eright[sa] : etop[sa];
    if (e < 0 || (sb != sa + 1 && sb != sa + P)) return fail(SFDP_E_INVALID, "interface pair is not an edge");
    muedge.push_back(e);
  }
  p.nmu = nmu;
  p.nC = (P - 1) * (P - 1);
  for (int s = 0; s < nsub; ++s)
    for (int q = 0; q < 4; ++q) {
      const int l = cloc[s * 4 + q];
      if (l < 0) continue;
      const int gi = (s % P) * m + l % ml, gj = (s / P) * m + l / ml;
      cgid[s * NQ + q] = (gi / m - 1) + (P - 1) * (gj / m - 1);
    }
  for (int s = 0; s < nsub; ++s) {
    if (eright[s] >= 0) cgid[s * NQ + 5] = cgid[(s + 1) * NQ + 4] = p.nC + eright[s];
    if (etop[s] >= 0) cgid[s * NQ + 7] = cgid[(s + P) * NQ + 6] = p.nC + etop[s];
  }
  // edge-augmented coarse space by default while the augmented coarse problem
  // stays small enough for its dense inverse (up to 19 x 19 subdomains)
  p.nK = p.nC + p.nE <= KAUG_DEFAULT_MAX ? p.nC + p.nE : p.nC;
  const int nk = std::max(p.nKmax(), 1);
  std::vector<int> cown(nk * 4, -1), cfree(std::max(p.nC, 1), 0), cnt(nk, 0);
  for (int s = 0; s < nsub; ++s)
    for (int q = 0; q < NQ; ++q) {
      const int c = cgid[s * NQ + q];
      if (c < 0) continue;
      cown[c * 4 + cnt[c]++] = s * NQ + q;
      if (q < 4) {
        const int l = cloc[s * 4 + q];
        const int gi = (s % P) * m + l % ml, gj = (s / P) * m + l / ml;
        cfree[c] = (gi - 1) + (N - 1) * (gj - 1);
      }
    }
  std::vector<int> f2b((size_t)(N + 1) * (N + 1), -1);
  int nbd = 0;
  for (int j = 0; j <= N; ++j)
    for (int i = 0; i <= N; ++i)
      if (i == 0 || j == 0 || i == N || j == N) f2b[i + (size_t)(N + 1) * j] = nbd++;
  p.n_bdry = nbd;
  sfdp_status s;
  if ((s = dupload(p, &p.dloc, dloc)) || (s = dupload(p, &p.dmid, dmid)) ||
      (s = dupload(p, &p.dpart, dpart)) || (s = dupload(p, &p.nd, ndv)) ||
      (s = dupload(p, &p.dsgn, dsgn)) || (s = dupload(p, &p.cloc, cloc)) ||
      (s = dupload(p, &p.cgid, cgid)) || (s = dupload(p, &p.muown, muown)) ||
      (s = dupload(p, &p.mufree, mufree)) || (s = dupload(p, &p.cown, cown)) ||
      (s = dupload(p, &p.cfree, cfree)) || (s = dupload(p, &p.full2bdry, f2b)) ||
      (s = dupload(p, &p.dedge, dedge)) || (s = dupload(p, &p.muedge, muedge)))
    return s;
  return SFDP_OK;
}


size_t g_size(const Problem& p) { return p.g32() ? sizeof(cf) : sizeof(cd); }  // line factors
size_t elem_size(const Problem& p) { return p.s32() ? sizeof(cf) : sizeof(cd); }  // Sinv, Phi

void free_factors(Problem& p) {
  size_t es = elem_size(p);
  dfree(p, p.G, g_size(p) * p.nsub * p.ml * p.ml * p.ml);
  const size_t PK = (size_t)p.ND * (p.ND + 1) / 2;
  dfree(p, p.Sinv, es * p.nsub * PK);
  dfree(p, p.Sbb, sizeof(cf) * p.nsub * PK);
  const size_t nk2 = (size_t)std::max(p.nKmax() * p.nKmax(), 1);
  dfree(p, p.Phi, es * p.nsub * p.ND * NQ);
  dfree(p, (void*&)p.Kinv, sizeof(cd) * nk2);
  dfree(p, (void*&)p.Kcc, sizeof(cd) * nk2);
  p.factored = false;
}

sfdp_status alloc_workspace3(Problem& p, int kmax);
sfdp_status alloc_workspace(Problem& p, int kmax) {
  if (p.dim == 3) return alloc_workspace3(p, kmax);
  if (p.kmax_alloc >= kmax && p.gmres_parts >= p.gmres_blocks) return SFDP_OK;
  // per right-hand side: Krylov basis, Hessenberg matrix, block partial sums
  if (p.kmax_alloc) {
    dfree(p, (void*&)p.Qk, sizeof(cd) * NRMAX * (size_t)(p.kmax_alloc + 1) * p.nmu);
    dfree(p, (void*&)p.Hk, sizeof(cd) * NRMAX * (size_t)(p.kmax_alloc + 1) * p.kmax_alloc);
    dfree(p, (void*&)p.part, sizeof(cd) * 3 * NRMAX * (size_t)(p.kmax_alloc + 2) * p.gmres_parts);
    p.kmax_alloc = 0;
  }
  kmax = std::max(kmax, p.kmax_alloc);
  sfdp_status s;
  if ((s = dalloc(p, (void**)&p.Qk, sizeof(cd) * NRMAX * (size_t)(kmax + 1) * p.nmu)) ||
      (s = dalloc(p, (void**)&p.Hk, sizeof(cd) * NRMAX * (size_t)(kmax + 1) * kmax)) ||
      (s = dalloc(p, (void**)&p.part, sizeof(cd) * 3 * NRMAX * (size_t)(kmax + 2) * p.gmres_blocks)))
    return s;
  p.kmax_alloc = kmax;
  p.gmres_parts = p.gmres_blocks;
  return SFDP_OK;
}

sfdp_status check_launch(Problem& p, int kmax) {
  hipError_t e = gmres_check(p, kmax);
  if (e == hipErrorOutOfMemory) return fail(SFDP_E_DEVICE, "GMRES kernel does not fit in LDS (lower max_krylov)");
  if (e == hipErrorCooperativeLaunchTooLarge)
    return fail(SFDP_E_DEVICE, "cooperative GMRES grid exceeds co-resident blocks");
  if (e != hipSuccess) return fail(SFDP_E_DEVICE, std::string("GMRES launch check: ") + hipGetErrorString(e));
  return SFDP_OK;
}

// Event pairs around hot launches (kind 0: GMRES, 1: subdomain solve).
hipError_t ev_begin(Problem* p, int kind, int* slot) {
  *slot = -1;
  if (!p || !p->timing || (p->timing == 2 && kind != 0)) return hipSuccess;
  if (p->ev_used + 2 > (int)p->ev_pool.size()) {
    for (int i = 0; i < 64; ++i) {
      // timing only (read after a stream synchronization): no system-scope fence,
      // whose cache write-back and invalidation idle the device ~6 us per record
      hipEvent_t e;
      hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
      if (r != hipSuccess) return r;
      p->ev_pool.push_back(e);
    }
  }
  *slot = p->ev_used;
  p->ev_used += 2;
  p->ev_pending.push_back({*slot, kind});
  return hipEventRecord(p->ev_pool[*slot], p->ctx->stream);
}
hipError_t ev_end(Problem* p, int slot) {
  if (slot < 0) return hipSuccess;
  return hipEventRecord(p->ev_pool[slot + 1], p->ctx->stream);
}
// After a stream synchronisation: fold the recorded pairs into the totals.
hipError_t ev_harvest(Problem& p) {
  for (auto& pr : p.ev_pending) {
    float ms = 0.f;
    hipError_t r = hipEventElapsedTime(&ms, p.ev_pool[pr.first], p.ev_pool[pr.first + 1]);
    if (r != hipSuccess) return r;
    if (pr.second == 0) { p.t_gmres_ms += ms; ++p.n_gmres; }
    else { p.t_local_ms += ms; ++p.n_local; }
  }
  p.ev_pending.clear();
  p.ev_used = 0;
  return hipSuccess;
}

void defaults(sfdp_precision prec, const sfdp_opts* o, double& tol_kkt, double& tol_inner, int& max_outer,
              int& kmax, int dim = 2) {
  bool mixed = prec != SFDP_FP64;
  tol_kkt = (o && o->tol_kkt > 0) ? o->tol_kkt : (mixed ? 1e-8 : 1e-10);
  tol_inner = (o && o->tol_inner > 0) ? o->tol_inner : (mixed ? 3e-7 : 1e-8);
  max_outer = (o && o->max_outer > 0) ? o->max_outer : 8;
  // corner-only FETI-DP in 3D needs more iterations than the 2D default allows
  kmax = (o && o->max_krylov > 0) ? std::min(o->max_krylov, KMAX_LIMIT) : (dim == 3 ? 300 : 64);
}
int batch_of(const sfdp_opts* o) { return (o && o->batch > 0) ? std::min(o->batch, NRMAX) : NRMAX; }
// Inner tolerance of the first refinement step: with complex64 interface
// operators that step ends near a relative KKT residual of 5e-3 whether its
// FETI-DP solves stop at 3e-7 or 1e-5, so it defaults to 1e-5 there (never
// tighter than tol_inner); FP64 reaches the gate in one step and keeps tol_inner.
constexpr double MIXED_FIRST_TOL = 1e-5;
double first_tol(sfdp_precision prec, const sfdp_opts* o, double tol_inner) {
  if (o && o->tol_inner_first > 0) return o->tol_inner_first;
  return prec == SFDP_FP64 ? tol_inner : std::max(tol_inner, MIXED_FIRST_TOL);
}
bool single_of(const sfdp_opts* o) { return o && o->factors == 1; }

sfdp_status check_ready(const Problem* p) {
  if (!p) return fail(SFDP_E_INVALID, "null problem");
  if (!p->factored) return fail(SFDP_E_STATE, "sfdp_set_beta has not been called");
  return SFDP_OK;
}

sfdp_status alloc_rs(Problem& p) {
  if (p.r1) return SFDP_OK;
  size_t n = (size_t)NRMAX * p.n_free;
  size_t nred = RED_HEAD + NRMAX * (size_t)red_pstride(p) * (2 + MET_N) / 2;
  sfdp_status s;
  if ((s = dalloc(p, (void**)&p.r1, sizeof(double) * n)) || (s = dalloc(p, (void**)&p.r2, sizeof(double) * n)) ||
      (s = dalloc(p, (void**)&p.r3, sizeof(double) * n)) || (s = dalloc(p, (void**)&p.red, sizeof(double) * nred)) ||
      (s = dalloc(p, (void**)&p.cvec, sizeof(cd) * n)) || (s = dalloc(p, (void**)&p.cvec2, sizeof(cd) * n)) ||
      (s = dalloc(p, (void**)&p.cvec3, sizeof(cd) * n)))
    return s;
  return SFDP_OK;
}

// A problem of the 2D class (maps, solve workspaces), not yet factored.
sfdp_status create_problem(Ctx* ctx, int dim, int n_elem, int sub_elem, sfdp_precision prec, Problem** out);
void destroy_problem(Problem* p);

// Factor arrays of one problem in its storage precision (kept across set-ups:
// their sizes depend on the mesh and the precision only).
sfdp_status alloc_factors(Problem& p) {
  if (p.G) return SFDP_OK;
  const int ml = p.ml, ND = p.ND, nsub = p.nsub;
  size_t es = elem_size(p);
  size_t nG = (size_t)nsub * ml * ml * ml, nP = (size_t)nsub * ND * NQ;
  const size_t nk2 = (size_t)std::max(p.nKmax() * p.nKmax(), 1);
  const size_t nPK = (size_t)nsub * ND * (ND + 1) / 2;
  sfdp_status s;
  if ((s = dalloc(p, &p.G, g_size(p) * nG)) || (s = dalloc(p, &p.Sinv, es * nPK)) ||
      (s = dalloc(p, &p.Sbb, sizeof(cf) * nPK)) || (s = dalloc(p, &p.Phi, es * nP)) ||
      (s = dalloc(p, (void**)&p.Kinv, sizeof(cd) * nk2)) || (s = dalloc(p, (void**)&p.Kcc, sizeof(cd) * nk2))) {
    free_factors(p);
    return s;
  }
  return SFDP_OK;
}

// FP64 set-up scratch of one problem, as element counts of G64, Sinv64, S64,
// Phi64, PhiFull, scr, Zs, Kwork.
void setup_counts(size_t nsub, size_t ml, size_t ND, int nK, size_t c[8]) {
  c[0] = nsub * ml * ml * ml;
  c[1] = nsub * ND * ND;
  c[2] = nsub * ND * ND;
  c[3] = nsub * ND * NQ;
  c[4] = nsub * ml * ml * 4;
  c[5] = 0;  // the line solves use the context's slots (ms_scr)
  c[6] = nsub * NQ * NQ;
  c[7] = (size_t)std::max(nK * nK, 1);
}
void setup_counts(const Problem& p, size_t c[8]) { setup_counts(p.nsub, p.ml, p.ND, p.nKmax(), c); }
size_t pad256(size_t b) { return (b + 255) & ~(size_t)255; }
// Bytes of the line-solve slots for a set-up of nsub subdomains in all, the
// largest of m x m cells.
size_t ms_bytes(size_t nsub, int m) {
  return pad256(std::min(nsub, (size_t)MS_SLOTS_MAX) * ms_slot_cd(m) * sizeof(cd));
}
// Bytes of the pool share of one problem of this mesh.
size_t setup_bytes(int n_elem, int sub_elem) {
  const size_t P = n_elem / sub_elem;
  size_t c[8], b = 0;
  const int nK = (int)((P - 1) * (P - 1) + 2 * P * (P - 1));
  setup_counts(P * P, sub_elem + 1, ((4 * (sub_elem - 1) + 31) / 32) * 32, nK, c);
  for (int k = 0; k < 8; ++k) b += pad256(c[k] * sizeof(cd));
  return b + ms_bytes(P * P, sub_elem);
}

// Carve every problem's set-up scratch out of the context's pool (grown when
// too small; the stream must be idle).
sfdp_status alloc_setup(Ctx* ctx, const std::vector<Problem*>& ps) {
  size_t total = 0, nsub = 0;
  int mmax = 0;
  for (Problem* p : ps) {
    size_t c[8];
    setup_counts(*p, c);
    for (size_t k = 0; k < 8; ++k) total += pad256(c[k] * sizeof(cd));
    if (p->dim == 2) {
      nsub += p->nsub;
      mmax = std::max(mmax, p->m);
    }
  }
  const size_t msb = nsub ? ms_bytes(nsub, mmax) : 0;
  total += msb;
  if (total > ctx->pool_bytes) {
    if (ctx->pool) {
      hipFree(ctx->pool);
      ctx->used -= std::min(ctx->used, ctx->pool_bytes);
      ctx->pool = nullptr;
      ctx->pool_bytes = 0;
    }
    if (ctx->budget && ctx->used + total > ctx->budget) return fail(SFDP_E_NOMEM, "memory budget exceeded");
    if (hipMalloc(&ctx->pool, total) != hipSuccess) return fail(SFDP_E_NOMEM, "setup scratch allocation failed");
    ctx->pool_bytes = total;
    ctx->used += total;
  }
  char* q = (char*)ctx->pool;
  for (Problem* p : ps) {
    size_t c[8];
    setup_counts(*p, c);
    cd** dst[8] = {&p->G64, &p->Sinv64, &p->S64, &p->Phi64, &p->PhiFull, &p->scr, &p->Zs, &p->Kwork};
    for (int k = 0; k < 8; ++k) {
      *dst[k] = (cd*)q;
      q += pad256(c[k] * sizeof(cd));
    }
  }
  ctx->ms_scr = msb ? (cd*)q : nullptr;
  return SFDP_OK;
}
void free_setup(Problem& p) {
  p.G64 = p.Sinv64 = p.S64 = p.Phi64 = p.PhiFull = p.scr = p.Zs = p.Kwork = nullptr;
}

// ---------------------------------------------------------------------------------------
// 3D instances: partition and interface maps, factors and workspaces (kernels in
// three.hip).  Multipliers are fully redundant and ordered by the full id of
// their node, then by the pair of subdomains (s_a < s_b), signed +1 on s_a.
sfdp_status build_maps3(Problem& p) {
  Three& T = *p.t3;
  Geo3& g = T.g;
  const int N = p.N, m = p.m, P = p.P, ml = p.ml, nsub = p.nsub, nl = ml * ml * ml;
  g.N = N; g.m = m; g.P = P; g.ml = ml; g.nsub = nsub; g.nl = nl;
  g.nI = (m - 1) * (m - 1) * (m - 1);
  g.NR = nl - 8;
  g.ND = g.NR - g.nI;
  g.nC = (P - 1) * (P - 1) * (P - 1);
  g.h = 1.0 / N;
  g.alpha = 0.0;
  g.rshift = 0;
  const int NR = g.NR, ND = g.ND, nI = g.nI;
  std::vector<int> rl((size_t)nsub * NR, -1), rpos((size_t)nsub * nl, -1), nds(nsub, 0), cg(nsub * 8, -1);
  struct Inc {
    int64_t full;
    int s, d;
  };
  std::vector<Inc> inc;
  const int64_t n1 = N + 1;
  for (int s = 0; s < nsub; ++s) {
    int gi0, gj0, gk0;
    g.base(s, gi0, gj0, gk0);
    int nr = 0, nd = 0;
    for (int l = 0; l < nl; ++l) {
      int a, b, c;
      g.loc(l, a, b, c);
      if (a > 0 && a < m && b > 0 && b < m && c > 0 && c < m) {
        rl[(size_t)s * NR + nr] = l;
        rpos[(size_t)s * nl + l] = nr++;
      }
    }
    for (int l = 0; l < nl; ++l) {
      int a, b, c;
      g.loc(l, a, b, c);
      const bool inter = a > 0 && a < m && b > 0 && b < m && c > 0 && c < m;
      const bool vert = (a == 0 || a == m) && (b == 0 || b == m) && (c == 0 || c == m);
      if (inter || vert || g.dirich(s, a, b, c)) continue;
      if (nd >= ND) return fail(SFDP_E_INVALID, "interface slot overflow");
      rl[(size_t)s * NR + nI + nd] = l;
      rpos[(size_t)s * nl + l] = nI + nd;
      inc.push_back({(gi0 + a) + n1 * ((gj0 + b) + n1 * (int64_t)(gk0 + c)), s, nd});
      ++nd;
    }
    nds[s] = nd;
    p.ndmax = std::max(p.ndmax, nd);
    for (int q = 0; q < 8; ++q) {
      int a, b, c;
      g.loc(g.vertex(q), a, b, c);
      if (g.dirich(s, a, b, c)) continue;
      cg[s * 8 + q] = ((gi0 + a) / m - 1) + (P - 1) * (((gj0 + b) / m - 1) + (P - 1) * ((gk0 + c) / m - 1));
    }
  }
  std::vector<int> cown((size_t)std::max(g.nC, 1) * 8, -1), cnt(std::max(g.nC, 1), 0);
  for (int s = 0; s < nsub; ++s)
    for (int q = 0; q < 8; ++q) {
      const int c = cg[s * 8 + q];
      if (c >= 0) cown[(size_t)c * 8 + cnt[c]++] = s * 8 + q;
    }
  std::stable_sort(inc.begin(), inc.end(), [](const Inc& x, const Inc& y) {
    return x.full != y.full ? x.full < y.full : x.s < y.s;
  });
  std::vector<int> dmu((size_t)nsub * ND * 3, -1), muown;
  std::vector<float> dsg((size_t)nsub * ND * 3, 0.f);
  auto add = [&](int s, int d, int k, float sign) {
    const size_t base = ((size_t)s * ND + d) * 3;
    for (int j = 0; j < 3; ++j)
      if (dmu[base + j] < 0) {
        dmu[base + j] = k;
        dsg[base + j] = sign;
        return true;
      }
    return false;
  };
  for (size_t i0 = 0; i0 < inc.size();) {
    size_t i1 = i0;
    while (i1 < inc.size() && inc[i1].full == inc[i0].full) ++i1;
    for (size_t a = i0; a < i1; ++a)
      for (size_t b = a + 1; b < i1; ++b) {
        const int k = (int)(muown.size() / 2);
        muown.push_back(inc[a].s * ND + inc[a].d);
        muown.push_back(inc[b].s * ND + inc[b].d);
        if (!add(inc[a].s, inc[a].d, k, 1.f) || !add(inc[b].s, inc[b].d, k, -1.f))
          return fail(SFDP_E_INVALID, "more than three multipliers on a node");
      }
    i0 = i1;
  }
  g.nmu = (int)(muown.size() / 2);
  p.nmu = g.nmu;
  p.nC = g.nC;
  p.nK = g.nC;
  p.nE = 0;
  p.ND = ND;
  std::vector<int> f2b((size_t)n1 * n1 * n1, -1);
  int nbd = 0;
  for (int k = 0; k <= N; ++k)
    for (int j = 0; j <= N; ++j)
      for (int i = 0; i <= N; ++i)
        if (i == 0 || j == 0 || k == 0 || i == N || j == N || k == N) f2b[i + n1 * (j + n1 * (size_t)k)] = nbd++;
  p.n_bdry = nbd;
  sfdp_status s;
  if ((s = dupload(p, &T.rl, rl)) || (s = dupload(p, &T.rpos, rpos)) || (s = dupload(p, &T.nds, nds)) ||
      (s = dupload(p, &T.dmu, dmu)) || (s = dupload(p, &T.dsg, dsg)) || (s = dupload(p, &T.muown, muown)) ||
      (s = dupload(p, &T.cg, cg)) || (s = dupload(p, &T.cown, cown)) || (s = dupload(p, &p.full2bdry, f2b)))
    return s;
  return SFDP_OK;
}

// Factor arrays of a 3D problem (storage precision of the interface operators
// for Z_rr^-1, its Delta block, S_bb and Phi).
void free_factors3(Problem& p) {
  Three& T = *p.t3;
  const Geo3& g = T.g;
  const size_t es = elem_size(p), ns = g.nsub;
  dfree(p, T.Zinv, es * ns * g.NR * g.NR);
  dfree(p, T.Sinv, es * ns * g.ND * g.ND);
  dfree(p, T.Sbb, es * ns * g.ND * g.ND);
  dfree(p, T.Phi, es * ns * g.ND * 8);
  dfree(p, (void*&)T.PhiFull, sizeof(cd) * ns * g.NR * 8);
  dfree(p, (void*&)T.Zcc, sizeof(cd) * ns * 64);
  const size_t nc2 = (size_t)std::max(g.nC * g.nC, 1);
  dfree(p, (void*&)p.Kinv, sizeof(cd) * nc2);
  dfree(p, (void*&)p.Kcc, sizeof(cd) * nc2);
  p.factored = false;
}
sfdp_status alloc_factors3(Problem& p) {
  Three& T = *p.t3;
  if (T.Zinv) return SFDP_OK;
  const Geo3& g = T.g;
  const size_t es = elem_size(p), ns = g.nsub;
  const size_t nc2 = (size_t)std::max(g.nC * g.nC, 1);
  sfdp_status s;
  if ((s = dalloc(p, &T.Zinv, es * ns * g.NR * g.NR)) || (s = dalloc(p, &T.Sinv, es * ns * g.ND * g.ND)) ||
      (s = dalloc(p, &T.Sbb, es * ns * g.ND * g.ND)) || (s = dalloc(p, &T.Phi, es * ns * g.ND * 8)) ||
      (s = dalloc(p, (void**)&T.PhiFull, sizeof(cd) * ns * g.NR * 8)) ||
      (s = dalloc(p, (void**)&T.Zcc, sizeof(cd) * ns * 64)) || (s = dalloc(p, (void**)&p.Kinv, sizeof(cd) * nc2)) ||
      (s = dalloc(p, (void**)&p.Kcc, sizeof(cd) * nc2))) {
    free_factors3(p);
    return s;
  }
  return SFDP_OK;
}

// Set-up of a 3D problem for its beta: the extended local matrices (FP64) and
// the pivot-inverse buffers exist only during the call.
sfdp_status setup3(Problem& p) {
  sfdp_status s = alloc_factors3(p);
  if (s) return s;
  p.factored = false;
  const Geo3& g = p.t3->g;
  const size_t eb = sizeof(cd) * (size_t)g.nsub * g.NR * g.NR, wb = sizeof(cd) * (size_t)g.nsub * 2 * 32 * 32;
  void *E = nullptr, *W = nullptr;
  if ((s = dalloc(p, &E, eb)) || (s = dalloc(p, &W, wb))) {
    dfree(p, E, eb);
    return s;
  }
  hipError_t e = launch_setup3(p, (cd*)E, (cd*)W);
  if (e == hipSuccess) e = hipStreamSynchronize(p.ctx->stream);
  dfree(p, E, eb);
  dfree(p, W, wb);
  if (e != hipSuccess) return fail(SFDP_E_DEVICE, std::string("setup: ") + hipGetErrorString(e));
  p.factored = true;
  return SFDP_OK;
}

void free_workspace3(Problem& p) {
  Three& T = *p.t3;
  if (!T.kalloc) return;
  const Geo3& g = T.g;
  const size_t R = NRMAX, nm = g.nmu, nb = (nm + 255) / 256, kk = T.kalloc + 1;
  dfree(p, (void*&)T.T, sizeof(cd) * R * g.nsub * g.NR);
  dfree(p, (void*&)T.Y, sizeof(cd) * R * g.nsub * g.ND);
  dfree(p, (void*&)T.Wc, sizeof(cd) * R * g.nsub * 8);
  for (cd** v : {&T.fcs, &T.uc, &T.gc}) dfree(p, (void*&)*v, sizeof(cd) * R * std::max(g.nC, 1));
  for (cd** v : {&T.d, &T.mu, &T.z, &T.w}) dfree(p, (void*&)*v, sizeof(cd) * R * nm);
  dfree(p, (void*&)T.V, sizeof(cd) * R * kk * nm);
  dfree(p, (void*&)T.part, sizeof(cd) * R * kk * 4 * nb);
  dfree(p, (void*&)T.hd, sizeof(cd) * R * (2 * kk + 1));
  dfree(p, (void*&)T.npart, sizeof(double) * R * nb);
  dfree(p, (void*&)T.nvd, sizeof(int) * R);
  dfree(p, (void*&)T.gs, sizeof(cd) * R * gs_len(T.kalloc));
  dfree(p, (void*&)T.gi, sizeof(int) * GI_WORDS);
  if (T.gih) hipHostFree(T.gih);
  T.gih = nullptr;
  T.kalloc = 0;
}
sfdp_status alloc_workspace3(Problem& p, int kmax) {
  Three& T = *p.t3;
  if (T.kalloc >= kmax) return SFDP_OK;
  free_workspace3(p);
  const Geo3& g = T.g;
  const size_t R = NRMAX, nm = g.nmu, nb = (nm + 255) / 256, kk = kmax + 1;
  sfdp_status s;
  if ((s = dalloc(p, (void**)&T.T, sizeof(cd) * R * g.nsub * g.NR)) ||
      (s = dalloc(p, (void**)&T.Y, sizeof(cd) * R * g.nsub * g.ND)) ||
      (s = dalloc(p, (void**)&T.Wc, sizeof(cd) * R * g.nsub * 8)))
    return s;
  for (cd** v : {&T.fcs, &T.uc, &T.gc})
    if ((s = dalloc(p, (void**)v, sizeof(cd) * R * std::max(g.nC, 1)))) return s;
  for (cd** v : {&T.d, &T.mu, &T.z, &T.w})
    if ((s = dalloc(p, (void**)v, sizeof(cd) * R * nm))) return s;
  if ((s = dalloc(p, (void**)&T.V, sizeof(cd) * R * kk * nm)) ||
      (s = dalloc(p, (void**)&T.part, sizeof(cd) * R * kk * 4 * nb)) ||
      (s = dalloc(p, (void**)&T.hd, sizeof(cd) * R * (2 * kk + 1))) ||
      (s = dalloc(p, (void**)&T.npart, sizeof(double) * R * nb)) || (s = dalloc(p, (void**)&T.nvd, sizeof(int) * R)) ||
      (s = dalloc(p, (void**)&T.gs, sizeof(cd) * R * gs_len(kmax))) ||
      (s = dalloc(p, (void**)&T.gi, sizeof(int) * GI_WORDS)))
    return s;
  if (hipHostMalloc((void**)&T.gih, sizeof(int) * GI_WORDS) != hipSuccess) {
    T.gih = nullptr;
    return fail(SFDP_E_NOMEM, "pinned host allocation");
  }
  T.kalloc = kmax;
  return SFDP_OK;
}

// FETI-DP solves of the view's nr right-hand sides together (vectors f, x of
// Dev, c-th at offset c n_free); each logs its iteration count in the flag
// words of its group slot.
sfdp_status feti_run3(Problem& p, int fsel, int conj, int xsel, double tol, int kmax) {
  sfdp_status s = alloc_workspace3(p, kmax);
  if (s) return s;
  const Dev d = p.dev();
  int its[NRMAX] = {};
  hipError_t e = feti3(p, p.nr, dev_vec(d, fsel), dev_vec(d, xsel), conj, tol, kmax, its);
  for (int c = 0; c < p.nr && e == hipSuccess; ++c) e = launch_log3(p, c, (int)((p.map >> (8 * c)) & 255u), its[c]);
  if (e != hipSuccess) return fail(SFDP_E_DEVICE, std::string("3D FETI-DP: ") + hipGetErrorString(e));
  return SFDP_OK;
}

// ---------------------------------------------------------------------------------------
// Several problems as one launch target: block maps per launch kind, GMRES launch
// groups, and the device array of instance views.
struct Multi {
  Ctx* ctx = nullptr;
  std::vector<Problem*> probs;
  Target t;
  Dev* ddev = nullptr;
  Dev* hdev = nullptr;  // pinned mirror
  size_t dev_cap = 0;
  int* dmap = nullptr;
  size_t map_cap = 0;
  int g_kmax = -1, g_width = -1;
  Gathered* hgather = nullptr;  // per-instance residual heads and flag words (pinned host)
  ~Multi() {
    if (ddev) hipFree(ddev);
    if (hdev) hipHostFree(hdev);
    if (dmap) hipFree(dmap);
    if (hgather) hipHostFree(hgather);
  }
};

sfdp_status multi_grow(Multi& M, size_t n_inst, size_t n_map) {
  if (n_inst > M.dev_cap) {
    if (M.ddev) hipFree(M.ddev);
    if (M.hdev) hipHostFree(M.hdev);
    if (M.hgather) hipHostFree(M.hgather);
    M.ddev = nullptr;
    M.hdev = nullptr;
    M.hgather = nullptr;
    size_t cap = std::max<size_t>(n_inst, 2 * M.dev_cap);
    if (hipMalloc(&M.ddev, sizeof(Dev) * cap) || hipHostMalloc(&M.hdev, sizeof(Dev) * cap) ||
        hipHostMalloc(&M.hgather, sizeof(Gathered) * cap))
      return fail(SFDP_E_NOMEM, "batch descriptor allocation failed");
    M.dev_cap = cap;
  }
  if (n_map > M.map_cap) {
    if (M.dmap) hipFree(M.dmap);
    M.dmap = nullptr;
    size_t cap = std::max<size_t>(n_map, 2 * M.map_cap);
    if (hipMalloc(&M.dmap, sizeof(int) * cap)) return fail(SFDP_E_NOMEM, "batch map allocation failed");
    M.map_cap = cap;
  }
  return SFDP_OK;
}

// Block maps of every launch kind for the batch's problems (the stream must be
// idle: the maps are uploaded synchronously).
sfdp_status multi_maps(Multi& M) {
  const int n = (int)M.probs.size();
  Target& t = M.t;
  t.st = M.ctx->stream;
  t.one = nullptr;
  t.probs = M.probs;
  t.prec = M.probs[0]->prec;
  std::vector<int> host;
  size_t off_inst[K_NKIND], off_first[K_NKIND];
  for (int k = 0; k < K_NKIND; ++k) {
    off_first[k] = host.size();
    int tot = 0;
    for (int i = 0; i < n; ++i) {
      host.push_back(tot);
      tot += k == K_GMRES ? 0 : M.probs[i]->blocks(k);
    }
    off_inst[k] = host.size();
    if (k != K_GMRES)
      for (int i = 0; i < n; ++i)
        for (int b = 0; b < M.probs[i]->blocks(k); ++b) host.push_back(i);
    t.total[k] = tot;
  }
  sfdp_status s = multi_grow(M, n, host.size());
  if (s) return s;
  HIPCHK(hipMemcpy(M.dmap, host.data(), sizeof(int) * host.size(), hipMemcpyHostToDevice));
  for (int k = 0; k < K_NKIND; ++k) {
    t.inst[k] = M.dmap + off_inst[k];
    t.first[k] = M.dmap + off_first[k];
  }
  t.devs = M.ddev;
  t.ggroups.clear();
  M.g_kmax = M.g_width = -1;
  return SFDP_OK;
}

// GMRES launch groups for (kmax, width): instances in order, each group's
// blocks co-resident.  Written after the kind maps (own device area).
sfdp_status multi_groups(Multi& M, int kmax, int width, int*& gmap, size_t& gcap) {
  if (M.g_kmax == kmax && M.g_width == width) return SFDP_OK;
  const int asked = width;
  Target& t = M.t;
  const int n = (int)M.probs.size();
  int cmax = 1, bmax = 1;
  for (Problem* p : M.probs) {
    cmax = std::max(cmax, (p->nmu + p->gmres_blocks - 1) / p->gmres_blocks);
    bmax = std::max(bmax, p->gmres_blocks);
  }
  // groups are sized for the widest kernel that holds the largest instance;
  // the launch then picks the widest kernel each group's grid fits
  int cap = 0;
  for (;;) {
    cap = INT_MAX;
    for (Problem* p : M.probs) cap = std::min(cap, gmres_capacity(*p, kmax, cmax, width));
    if (cap >= bmax || width == 1) break;
    width = width == NRMAX ? 2 : 1;
  }
  if (cap < 1) return fail(SFDP_E_DEVICE, "GMRES kernel does not fit in LDS (lower max_krylov)");
  std::vector<int> host(n, 0);  // first block of each instance within its group
  t.ggroups.clear();
  std::vector<size_t> g_off;
  for (int i = 0; i < n;) {
    Target::GGroup g;
    g.total = 0;
    while (i < n && (g.members.empty() || g.total + M.probs[i]->gmres_blocks <= cap)) {
      if (M.probs[i]->gmres_blocks > cap) return fail(SFDP_E_DEVICE, "instance exceeds the co-resident GMRES grid");
      host[i] = g.total;
      g.total += M.probs[i]->gmres_blocks;
      g.members.push_back(i);
      ++i;
    }
    g_off.push_back(host.size());
    for (int m : g.members)
      for (int b = 0; b < M.probs[m]->gmres_blocks; ++b) host.push_back(m);
    t.ggroups.push_back(g);
  }
  if (host.size() > gcap) {
    if (gmap) hipFree(gmap);
    gmap = nullptr;
    gcap = std::max(host.size(), 2 * gcap);
    if (hipMalloc(&gmap, sizeof(int) * gcap)) return fail(SFDP_E_NOMEM, "batch map allocation failed");
  }
  HIPCHK(hipMemcpy(gmap, host.data(), sizeof(int) * host.size(), hipMemcpyHostToDevice));
  t.first[K_GMRES] = gmap;
  for (size_t g = 0; g < t.ggroups.size(); ++g) t.ggroups[g].inst = gmap + g_off[g];
  M.g_kmax = kmax;
  M.g_width = asked;
  return SFDP_OK;
}

// GMRES blocks of an instance that shares launches with others: enough for
// every block's multiplier chunk to stay near `chunk`, but no more than one
// launch can hold at once (the widest kernel if possible, else the narrowest;
// fewer blocks mean larger chunks and more LDS, hence the re-check).
int shared_gmres_blocks(const Problem& p, int kmax, int chunk) {
  int b = std::min(p.nsub, std::max(1, (p.nmu + chunk - 1) / chunk));
  for (int w : {NRMAX, 1})
    for (int it = 0; it < 8; ++it) {
      const int cap = gmres_capacity(p, kmax, (p.nmu + b - 1) / b, w);
      if (cap >= b) return b;
      if (cap < 1) break;
      b = cap;
    }
  return b;  // nothing fits: the launch reports it
}

// Upload the instance views (the stream must be idle).
sfdp_status multi_upload(Multi& M) {
  const size_t n = M.probs.size();
  for (size_t i = 0; i < n; ++i) M.hdev[i] = M.probs[i]->dev();
  HIPCHK(hipMemcpy(M.ddev, M.hdev, sizeof(Dev) * n, hipMemcpyHostToDevice));
  return SFDP_OK;
}

sfdp_status gmres_error(hipError_t e) {
  if (e == hipErrorOutOfMemory) return fail(SFDP_E_DEVICE, "GMRES kernel does not fit in LDS (lower max_krylov)");
  if (e == hipErrorCooperativeLaunchTooLarge)
    return fail(SFDP_E_DEVICE, "cooperative GMRES grid exceeds co-resident blocks");
  return fail(SFDP_E_DEVICE, std::string("GMRES launch: ") + hipGetErrorString(e));
}

// One FETI-DP solve of Z x_r = f_r (conj: conj(Z) x_r = f_r) for every
// instance's group (its view's nr right-hand sides); f and x name instance
// vectors.  `timed` receives event pairs (single problems only).
sfdp_status feti_run(const Target& t, Problem* timed, int fsel, int conj, int xsel, double tol, int kmax) {
  if (t.single() && t.one->dim == 3) return feti_run3(*t.one, fsel, conj, xsel, tol, kmax);
  if (t.single()) {
    sfdp_status s = check_launch(*t.one, kmax);
    if (s) return s;
  }
  int ev;
  HIPCHK(ev_begin(timed, 1, &ev));
  HIPCHK(launch_local_solve(t, 0, fsel, conj, xsel));
  HIPCHK(ev_end(timed, ev));
  HIPCHK(launch_coarse_rhs(t, fsel, conj));
  HIPCHK(launch_fetidp_rhs(t));
  HIPCHK(ev_begin(timed, 0, &ev));
  hipError_t e = launch_gmres(t, tol, kmax);
  if (e != hipSuccess) return gmres_error(e);
  HIPCHK(ev_end(timed, ev));
  HIPCHK(launch_recover_coarse(t));
  HIPCHK(ev_begin(timed, 1, &ev));
  HIPCHK(launch_local_solve(t, 1, fsel, conj, xsel));
  HIPCHK(ev_end(timed, ev));
  HIPCHK(launch_assemble_solution(t, xsel, conj));
  return SFDP_OK;
}

constexpr unsigned IDENTITY_MAP = 0x03020100u;

// The context's capture stream (non-blocking, default priority) and the two
// events that order it after and before the library's stream: the library's
// stream may be the null stream, which cannot be captured.
sfdp_status capture_stream(Ctx* c) {
  if (c->cap_stream) return SFDP_OK;
  HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&c->cap_ev[0], hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&c->cap_ev[1], hipEventDisableTiming));
  return SFDP_OK;
}

// Run one refinement step of a single problem through a captured graph: the
// first occurrence of a step's key runs eagerly (and tunes its launches), the
// second captures it on the capture stream and instantiates it, every later one
// replays it.  A replay runs on the capture stream between two event waits, so
// it stays in order with the library's stream.  A failed capture switches the
// problem to eager steps.
sfdp_status step_graph(Problem& p, const Target& t, double tin, int kmax, bool single,
                       const std::function<sfdp_status(const Target&)>& body) {
  StepKey key;
  key.nr = p.nr;
  key.map = p.map;
  key.kmax = kmax;
  key.single = single ? 1 : 0;
  key.tin = tin;
  key.tune_gen = tune_generation();
  key.plain = p.gmres_coop ? 0 : p.gmres_plain;
  for (int c = 0; c < NRMAX; ++c) {
    const Slot& q = p.sl[c];
    const void* v[5] = {q.ybar, q.yc, q.y, q.u, q.lam};
    for (int k = 0; k < 5; ++k) key.ptr[5 * c + k] = v[k];
  }
  Ctx* c = p.ctx;
  // a library stream other than the null stream is captured and replayed on directly
  const bool direct = t.st != nullptr;
  auto replay = [&](hipGraphExec_t exec) -> sfdp_status {
    if (direct) {
      HIPCHK(hipGraphLaunch(exec, t.st));
      return SFDP_OK;
    }
    HIPCHK(hipEventRecord(c->cap_ev[0], t.st));
    HIPCHK(hipStreamWaitEvent(c->cap_stream, c->cap_ev[0], 0));
    HIPCHK(hipGraphLaunch(exec, c->cap_stream));
    HIPCHK(hipEventRecord(c->cap_ev[1], c->cap_stream));
    HIPCHK(hipStreamWaitEvent(t.st, c->cap_ev[1], 0));
    return SFDP_OK;
  };
  for (StepGraph& g : p.graphs)
    if (g.key == key) return replay(g.exec);
  bool seen = false;
  for (const StepKey& k : p.graph_seen) seen = seen || k == key;
  if (p.graph_off || !seen || p.graphs.size() >= 16) {
    if (!seen && p.graph_seen.size() < 64) p.graph_seen.push_back(key);
    return body(t);
  }
  sfdp_status s = direct ? SFDP_OK : capture_stream(c);
  if (s) return s;
  Target tc = t;
  if (!direct) tc.st = c->cap_stream;
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamBeginCapture(tc.st, hipStreamCaptureModeThreadLocal));
  s = body(tc);
  hipError_t e = hipStreamEndCapture(tc.st, &graph);
  hipGraphExec_t exec = nullptr;
  if (s == SFDP_OK && e == hipSuccess && graph) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (graph) hipGraphDestroy(graph);
  (void)hipGetLastError();
  if (s != SFDP_OK || e != hipSuccess || !exec) {
    // nothing of the capture ran: fall back to eager steps for this problem
    if (exec) hipGraphExecDestroy(exec);
    p.graph_off = true;
    return body(t);
  }
  p.graphs.push_back(StepGraph{key, exec});
  return replay(exec);
}

// Waits for the n records of a gather launched last on st: spins on their ready
// words in pinned host memory (no wake-up latency of a blocking synchronization),
// asking the stream every few hundred polls so that a failed or finished stream
// ends the wait.
static hipError_t wait_gathered(Gathered* hg, size_t n, hipStream_t st) {
  for (unsigned it = 1;; ++it) {
    bool all = true;
    for (size_t i = 0; i < n && all; ++i) all = __atomic_load_n(&hg[i].ready, __ATOMIC_ACQUIRE) != 0;
    if (all) return hipSuccess;
    if (it % 256 == 0) {
      const hipError_t e = hipStreamQuery(st);
      if (e == hipSuccess) return hipStreamSynchronize(st);  // finished: the records are complete
      if (e != hipErrorNotReady) return e;
    }
  }
}
static void clear_gathered(Gathered* hg, size_t n) {
  for (size_t i = 0; i < n; ++i) __atomic_store_n(&hg[i].ready, 0, __ATOMIC_RELEASE);
}

// Range-space solves of every problem's group: nr targets in slots 0..nr-1,
// caller arrays in the problem's slots.
// All unfinished targets take each two-factor step together; each stops on
// its own test.  info[i] has ps[i]->nr entries.  M is the batch (null for a
// single problem); hg holds one Gathered record per problem (pinned host memory).
sfdp_status range_space_run(const Target& t, const std::vector<Problem*>& ps, Multi* M, Gathered* hg,
                            double tol_kkt, double tol_first, double tol_inner, int max_outer,
                            int kmax, const std::vector<sfdp_info*>& info, bool single) {
  const size_t n = ps.size();
  hipStream_t st = t.st;
  std::vector<int> ng(n);
  std::vector<std::vector<sfdp_info>> loc(n);
  std::vector<std::vector<int>> bad(n);  // 0 ok, 1 non-finite, 2 outer limit
  for (size_t i = 0; i < n; ++i) {
    ng[i] = ps[i]->nr;
    ps[i]->map = IDENTITY_MAP;
    ps[i]->init = (1u << ng[i]) - 1u;
    loc[i].assign(ng[i], sfdp_info{});
    bad[i].assign(ng[i], 0);
  }
  Problem* timed = t.single() ? t.one : nullptr;
  if (M) {
    sfdp_status s = multi_upload(*M);
    if (s) return s;
  }
  HIPCHK(launch_group_init(t));
  HIPCHK(launch_fill_flags(t, 0, FLAG_WORDS));
  for (Problem* p : ps) p->init = 0;
  // the KKT residual of the current iterate, gathered to the host (the end of
  // every refinement step, and the start)
  auto residual = [&](const Target& tt) -> hipError_t {
    hipError_t e = launch_kkt_residual(tt);
    if (e == hipSuccess) e = launch_gather(tt, hg);
    return e;
  };
  // one refinement step of the group's active targets, then the new residual
  // (on the stream of tt: the library's, or the capture stream)
  auto step_body = [&](const Target& tt, double tin) -> sfdp_status {
    HIPCHK(launch_make_rhs1(tt));
    sfdp_status s = feti_run(tt, timed, V_CVEC, 0, V_CVEC2, tin, kmax);
    if (s) return s;
    if (!single) {
      HIPCHK(launch_make_rhs2(tt));
      s = feti_run(tt, timed, V_CVEC3, 0, V_CVEC, tin, kmax);
      if (s) return s;
    }
    HIPCHK(launch_update(tt, single ? 1 : 0));
    HIPCHK(residual(tt));
    return SFDP_OK;
  };
  // a single 2D problem replays its steps as captured graphs (no timing events:
  // event records are not captured)
  const bool graphable = t.single() && t.one->dim == 2 && !M && !t.one->timing && g_graphs.load();
  // a single problem's GMRES solves use plain launches that check their grid's
  // co-residency; a step whose check failed changed nothing and runs again with
  // cooperative launches
  struct PlainScope {
    Problem* p;
    ~PlainScope() {
      if (p) p->gmres_plain = 0;
    }
  } plain_scope{t.single() ? t.one : nullptr};
  if (t.single()) t.one->gmres_plain = g_gmres_launch.load();
  int pre_flags[FLAG_WORDS];  // a single problem's device flags before the current step
  clear_gathered(hg, n);
  HIPCHK(residual(t));
  for (int step = 0;; ++step) {
    if (t.single()) t.one->yield_point();
    HIPCHK(wait_gathered(hg, n, st));
    if (step > 0 && t.single() && hg[0].flags[FLAG_NOTRES]) {
      // the flags as they were before the step (iteration logs of any GMRES
      // launch of it that did finish are dropped), then the same step again
      t.one->gmres_coop = true;
      HIPCHK(hipMemcpy(t.one->flags, pre_flags, sizeof(pre_flags), hipMemcpyHostToDevice));
      --step;
      const double tin = step == 0 ? tol_first : tol_inner;
      clear_gathered(hg, n);
      sfdp_status s = graphable ? step_graph(*t.one, t, tin, kmax, single,
                                             [&](const Target& tt) { return step_body(tt, tin); })
                                : step_body(t, tin);
      if (s) return s;
      continue;
    }
    bool any = false;
    for (size_t i = 0; i < n; ++i) {
      Problem* p = ps[i];
      unsigned map2 = 0;
      int nb2 = 0;
      for (int c = 0; c < p->nr; ++c) {
        const int q = (p->map >> (8 * c)) & 255;
        const double rho = hg[i].red[2 * q];
        sfdp_info& o = loc[i][q];
        o.rel_kkt = rho;
        if (step == 1) o.rel_kkt_first = rho;
        if (step > 0) o.imag_ratio = hg[i].red[2 * q + 1];
        if (!std::isfinite(rho)) { bad[i][q] = 1; continue; }
        if (rho <= tol_kkt) continue;
        if (step >= max_outer) { bad[i][q] = 2; continue; }
        map2 |= (unsigned)q << (8 * nb2++);
      }
      p->nr = nb2;
      p->map = map2;
      any = any || nb2 > 0;
    }
    if (!any) break;
    // the first step's inner tolerance may be looser (tol_inner_first)
    const double tin = step == 0 ? tol_first : tol_inner;
    if (M) {
      sfdp_status s = multi_upload(*M);
      if (s) return s;
    }
    if (t.single()) std::memcpy(pre_flags, hg[0].flags, sizeof(pre_flags));
    clear_gathered(hg, n);
    sfdp_status s = graphable ? step_graph(*t.one, t, tin, kmax, single,
                                           [&](const Target& tt) { return step_body(tt, tin); })
                              : step_body(t, tin);
    if (s) return s;
    for (size_t i = 0; i < n; ++i)
      for (int c = 0; c < ps[i]->nr; ++c) loc[i][(ps[i]->map >> (8 * c)) & 255].outer_steps = step + 1;
  }
  // accuracy metrics of every target of the group at its final iterate
  for (size_t i = 0; i < n; ++i) {
    ps[i]->nr = ng[i];
    ps[i]->map = IDENTITY_MAP;
  }
  if (M) {
    sfdp_status s = multi_upload(*M);
    if (s) return s;
  }
  HIPCHK(launch_kkt_metrics(t));
  HIPCHK(launch_gather(t, hg));
  HIPCHK(hipStreamSynchronize(st));
  if (timed) HIPCHK(ev_harvest(*timed));
  sfdp_status status = SFDP_OK;
  for (size_t i = 0; i < n; ++i) {
    const int* fl = hg[i].flags;
    if (fl[1]) return fail(SFDP_E_DEVICE, "grid barrier timed out");
    if (timed && timed->timing) { timed->it_gmres += fl[3]; timed->it_rhs += fl[4]; }
    for (int q = 0; q < ng[i]; ++q) {
      sfdp_info& o = loc[i][q];
      o.n_feti = fl[FLAG_CNT + q];
      for (int k = 0; k < o.n_feti && k < 16; ++k) {
        o.krylov_its[k] = fl[FLAG_LOG + 16 * q + k];
        o.krylov_total += o.krylov_its[k];
      }
      o.constr_viol = hg[i].red[MET_HEAD + 2 * q];
      o.eta_blk = hg[i].red[MET_HEAD + 2 * q + 1];
      o.t_setup_ms = ps[i]->t_setup_ms;
      if (bad[i][q] == 1) status = fail(SFDP_E_NOCONV, "non-finite residual");
      if (bad[i][q] == 2) status = fail(SFDP_E_NOCONV, "outer refinement limit reached");
      if (info[i]) info[i][q] = o;
    }
    ps[i]->nr = 0;
  }
  return status;
}

// A 3D problem: P^3 subdomains of sub_elem^3 cells (sub_elem <= 9: a
// subdomain's r nodes fit one workgroup of the sweep, at most 992).
sfdp_status create_problem3(Ctx* ctx, int n_elem, int sub_elem, sfdp_precision prec, Problem** out) {
  if (sub_elem < 2 || sub_elem > 9) return fail(SFDP_E_INVALID, "sub_elem must be in [2, 9] for dim 3");
  if (n_elem % sub_elem != 0 || n_elem / sub_elem < 2)
    return fail(SFDP_E_INVALID, "n_elem must be a multiple of sub_elem with at least 2 subdomains per side");
  const int P = n_elem / sub_elem;
  if ((int64_t)P * P * P > 65535) return fail(SFDP_E_INVALID, "at most 65535 subdomains in 3D");
  if (prec != SFDP_FP64 && prec != SFDP_MIXED && prec != SFDP_MIXED_IFACE)
    return fail(SFDP_E_INVALID, "bad precision");
  HIPCHK(hipSetDevice(ctx->device));
  Problem* p = new (std::nothrow) Problem();
  if (!p) return fail(SFDP_E_NOMEM, "host allocation");
  p->t3 = new (std::nothrow) Three();
  if (!p->t3) {
    delete p;
    return fail(SFDP_E_NOMEM, "host allocation");
  }
  p->ctx = ctx;
  ctx->children++;
  p->dim = 3;
  p->N = n_elem;
  p->m = sub_elem;
  p->P = P;
  p->nsub = P * P * P;
  p->ml = sub_elem + 1;
  p->L = p->ml * p->ml * p->ml;
  p->n_free = (int64_t)(n_elem - 1) * (n_elem - 1) * (n_elem - 1);
  p->prec = prec;
  sfdp_status s = build_maps3(*p);
  if (!s) s = dalloc(*p, (void**)&p->flags, sizeof(int) * FLAG_WORDS);
  if (s) {
    destroy_problem(p);
    return s;
  }
  hipError_t ez = launch_fill(p->flags, sizeof(int) * FLAG_WORDS, ctx->stream);
  if (ez == hipSuccess) ez = hipStreamSynchronize(ctx->stream);
  if (ez != hipSuccess) {
    destroy_problem(p);
    return fail(SFDP_E_DEVICE, std::string("init: ") + hipGetErrorString(ez));
  }
  *out = p;
  return SFDP_OK;
}

sfdp_status create_problem(Ctx* ctx, int dim, int n_elem, int sub_elem, sfdp_precision prec, Problem** out) {
  *out = nullptr;
  if (dim == 3) return create_problem3(ctx, n_elem, sub_elem, prec, out);
  if (dim != 2) return fail(SFDP_E_INVALID, "dim must be 2 or 3");
  if (sub_elem < 2 || sub_elem > 32) return fail(SFDP_E_INVALID, "sub_elem must be in [2, 32] for dim 2");
  if (n_elem % sub_elem != 0 || n_elem / sub_elem < 2)
    return fail(SFDP_E_INVALID, "n_elem must be a multiple of sub_elem with at least 2 subdomains per side");
  if (prec != SFDP_FP64 && prec != SFDP_MIXED && prec != SFDP_MIXED_IFACE)
    return fail(SFDP_E_INVALID, "bad precision");
  HIPCHK(hipSetDevice(ctx->device));
  Problem* p = new (std::nothrow) Problem();
  if (!p) return fail(SFDP_E_NOMEM, "host allocation");
  p->ctx = ctx;
  ctx->children++;
  p->dim = dim;
  p->N = n_elem;
  p->m = sub_elem;
  p->P = n_elem / sub_elem;
  p->nsub = p->P * p->P;
  p->ml = sub_elem + 1;
  p->L = p->ml * p->ml;
  p->ND = ((4 * (sub_elem - 1) + 31) / 32) * 32;
  p->n_free = (int64_t)(n_elem - 1) * (n_elem - 1);
  p->prec = prec;
  sfdp_status s = build_maps(*p);
  if (s != SFDP_OK) { destroy_problem(p); return s; }
  // solve workspaces, per right-hand side (NRMAX r-major copies, strides of Problem::rs())
  size_t nsd = (size_t)NRMAX * p->nsub * p->ND;
  size_t n4 = (size_t)NRMAX * p->nsub * NQ;
  size_t nC = (size_t)NRMAX * std::max(p->nKmax(), 1);
  size_t nm = (size_t)NRMAX * p->nmu;
  if ((s = dalloc(*p, (void**)&p->Xd, sizeof(cd) * nsd)) || (s = dalloc(*p, (void**)&p->Ubuf, sizeof(cd) * nsd)) ||
      (s = dalloc(*p, (void**)&p->Abuf, sizeof(cd) * nsd)) || (s = dalloc(*p, (void**)&p->Ybuf, sizeof(cd) * nsd)) ||
      (s = dalloc(*p, (void**)&p->Cbuf, sizeof(cd) * n4)) || (s = dalloc(*p, (void**)&p->Qc, sizeof(cd) * n4)) ||
      (s = dalloc(*p, (void**)&p->fcs, sizeof(cd) * nC)) || (s = dalloc(*p, (void**)&p->u0, sizeof(cd) * nC)) ||
      (s = dalloc(*p, (void**)&p->ymin, sizeof(cd) * nC)) || (s = dalloc(*p, (void**)&p->dvec, sizeof(cd) * nm)) ||
      (s = dalloc(*p, (void**)&p->mu, sizeof(cd) * nm)) || (s = dalloc(*p, (void**)&p->wv, sizeof(cd) * nm)) ||
      (s = dalloc(*p, (void**)&p->dscal, sizeof(double) * 8)) || (s = dalloc(*p, (void**)&p->bar, 4096)) ||
      (s = dalloc(*p, (void**)&p->flags, sizeof(int) * FLAG_WORDS))) {
    destroy_problem(p);
    return s;
  }
  p->gmres_blocks = std::min(p->nsub, ctx->num_cu);
  hipError_t ez = launch_fill(p->flags, sizeof(int) * FLAG_WORDS, ctx->stream);
  if (ez == hipSuccess) ez = launch_fill(p->bar, 4096, ctx->stream);
  if (ez == hipSuccess) ez = launch_fill(p->dscal, sizeof(double) * 8, ctx->stream);
  if (ez == hipSuccess) ez = hipStreamSynchronize(ctx->stream);
  if (ez != hipSuccess) {
    destroy_problem(p);
    return fail(SFDP_E_DEVICE, std::string("init: ") + hipGetErrorString(ez));
  }
  *out = p;
  return SFDP_OK;
}

void destroy_problem(Problem* p) {
  if (!p) return;
  hipSetDevice(p->ctx->device);
  hipStreamSynchronize(p->ctx->stream);
  if (p->pw) {
    destroy_problem(p->pw);
    p->pw = nullptr;
  }
  el_destroy(*p);
  if (Three* T = p->t3) {
    free_factors3(*p);
    free_workspace3(*p);
    void* maps3[] = {T->rl, T->rpos, T->nds, T->dmu, T->dsg, T->muown, T->cg, T->cown};
    for (void* a : maps3)
      if (a) hipFree(a);
    delete T;
    p->t3 = nullptr;
  }
  free_factors(*p);
  free_setup(*p);
  void* arr[] = {p->dloc, p->dmid, p->dpart, p->nd, p->dsgn, p->cloc, p->cgid, p->muown, p->mufree,
                 p->cown, p->cfree, p->dedge, p->muedge, p->full2bdry, p->Xd, p->Ubuf, p->Abuf, p->Ybuf, p->Cbuf, p->Qc,
                 p->fcs, p->u0, p->ymin, p->dvec, p->mu, p->wv, p->Qk, p->Hk, p->part, p->dscal,
                 p->bar, p->flags, p->r1, p->r2, p->r3, p->red, p->cvec, p->cvec2, p->cvec3};
  for (void* a : arr)
    if (a) hipFree(a);
  if (p->gh) hipHostFree(p->gh);
  if (p->fsw) hipFree(p->fsw);
  if (p->fsh) hipHostFree(p->fsh);
  if (p->stage) hipFree(p->stage);
  for (hipEvent_t e : p->ev_pool) hipEventDestroy(e);
  graphs_clear(*p);
  p->ctx->used -= std::min(p->ctx->used, p->bytes);
  p->ctx->children--;
  delete p;
}

// Factor one or several problems for their betas (one set-up sequence; the
// stream must be idle).
sfdp_status setup_run(const Target& t, const std::vector<Problem*>& ps, Multi* M) {
  for (Problem* p : ps) graphs_clear(*p);
  if (ps.size() == 1 && ps[0]->el) return el_setup(*ps[0]);
  if (ps.size() == 1 && ps[0]->dim == 3) return setup3(*ps[0]);
  for (Problem* p : ps) {
    sfdp_status s = alloc_factors(*p);
    if (s) return s;
    p->factored = false;
  }
  sfdp_status s0 = alloc_setup(ps[0]->ctx, ps);
  if (s0) return s0;
  if (M) {
    sfdp_status s = multi_upload(*M);
    if (s) return s;
  }
  Target ts = t;
  ts.setup32 = g_setup_bits.load() == 32 && t.prec == SFDP_MIXED;
  hipError_t e = launch_setup(ts);
  if (e == hipSuccess) e = hipStreamSynchronize(t.st);
  for (Problem* p : ps) free_setup(*p);
  if (e != hipSuccess) return fail(SFDP_E_DEVICE, std::string("setup: ") + hipGetErrorString(e));
  for (Problem* p : ps) p->factored = true;
  return SFDP_OK;
}

Target single_target(Problem* p) {
  Target t;
  t.st = p->ctx->stream;
  t.one = p;
  t.prec = p->prec;
  return t;
}

// The problem's gather buffers (device record and its pinned host copy),
// allocated on first use and kept until the problem is destroyed.
sfdp_status gather_buffers(Problem& p) {
  if (p.gh) return SFDP_OK;
  if (hipHostMalloc((void**)&p.gh, sizeof(Gathered)) != hipSuccess) {
    p.gh = nullptr;
    return fail(SFDP_E_NOMEM, "pinned gather buffer");
  }
  return SFDP_OK;
}

// One Gathered record of a single problem into p->gh (waits for the stream).
sfdp_status gather_one(Problem* p) {
  sfdp_status s = gather_buffers(*p);
  if (s) return s;
  Target t = single_target(p);
  HIPCHK(launch_gather(t, p->gh));
  HIPCHK(hipStreamSynchronize(t.st));
  return SFDP_OK;
}

}  // namespace

namespace sfdp {
sfdp_status host_fail(sfdp_status s, const std::string& msg) { return fail(s, msg); }
sfdp_status dev_alloc(Problem& p, void** ptr, size_t bytes) { return dalloc(p, ptr, bytes); }
void dev_free(Problem& p, void*& ptr, size_t bytes) { dfree(p, ptr, bytes); }
}  // namespace sfdp

struct sfdp_ctx : public Ctx {};
// 3D: Sinv and S_bb are stored full (ND x ND), Phi with the 8 vertex slots.
static sfdp_status inspect3(Problem* p, sfdp_query what, int sub, double* out, int* rows, int* cols) {
  const Three& T = *p->t3;
  const Geo3& g = T.g;
  int r = 0, c = 0;
  std::vector<int> qcols;
  if (what == SFDP_Q_COARSE || what == SFDP_Q_COARSE_INV) {
    r = c = g.nC;
  } else {
    if (sub < 0 || sub >= g.nsub) return fail(SFDP_E_INVALID, "sub out of range");
    HIPCHK(hipMemcpy(&r, T.nds + sub, sizeof(int), hipMemcpyDeviceToHost));
    if (what == SFDP_Q_PHI) {
      int cg[8];
      HIPCHK(hipMemcpy(cg, T.cg + 8 * sub, sizeof(cg), hipMemcpyDeviceToHost));
      for (int q = 0; q < 8; ++q)
        if (cg[q] >= 0) qcols.push_back(q);
      c = (int)qcols.size();
    } else if (what == SFDP_Q_SINV || what == SFDP_Q_SBB) {
      c = r;
    } else {
      return fail(SFDP_E_INVALID, "unknown query");
    }
  }
  if (rows) *rows = r;
  if (cols) *cols = c;
  if (!out) return SFDP_OK;
  HIPCHK(hipStreamSynchronize(p->ctx->stream));
  std::vector<cd> host((size_t)r * c);
  const size_t es = elem_size(*p);
  auto get = [&](const std::vector<char>& raw, size_t idx) {
    if (es == sizeof(cf)) {
      const cf v = ((const cf*)raw.data())[idx];
      return cd{v.x, v.y};
    }
    return ((const cd*)raw.data())[idx];
  };
  if (what == SFDP_Q_COARSE || what == SFDP_Q_COARSE_INV) {
    HIPCHK(hipMemcpy(host.data(), what == SFDP_Q_COARSE ? p->Kcc : p->Kinv, sizeof(cd) * host.size(),
                     hipMemcpyDeviceToHost));
  } else if (what == SFDP_Q_PHI) {
    std::vector<char> raw((size_t)g.ND * 8 * es);
    HIPCHK(hipMemcpy(raw.data(), (const char*)T.Phi + (size_t)sub * raw.size(), raw.size(), hipMemcpyDeviceToHost));
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < c; ++j) host[(size_t)i * c + j] = get(raw, (size_t)i * 8 + qcols[j]);
  } else {
    std::vector<char> raw((size_t)g.ND * g.ND * es);
    const char* base = (const char*)(what == SFDP_Q_SINV ? T.Sinv : T.Sbb);
    HIPCHK(hipMemcpy(raw.data(), base + (size_t)sub * raw.size(), raw.size(), hipMemcpyDeviceToHost));
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < c; ++j) host[(size_t)i * c + j] = get(raw, (size_t)i * g.ND + j);
  }
  HIPCHK(hipMemcpy(out, host.data(), sizeof(cd) * host.size(), hipMemcpyHostToDevice));
  return SFDP_OK;
}

static sfdp_status inspect_problem(Problem* p, sfdp_query what, int sub, double* out, int* rows, int* cols) {
  sfdp_status s = check_ready(p);
  if (s) return s;
  HIPCHK(hipSetDevice(p->ctx->device));
  if (p->el) return el_inspect(*p, what, sub, out, rows, cols);
  if (p->dim == 3) return inspect3(p, what, sub, out, rows, cols);
  std::vector<int> ndv(p->nsub), cg(NQ * p->nsub);
  HIPCHK(hipMemcpy(ndv.data(), p->nd, sizeof(int) * p->nsub, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(cg.data(), p->cgid, sizeof(int) * NQ * p->nsub, hipMemcpyDeviceToHost));
  int r = 0, c = 0;
  std::vector<int> qcols;  // coarse slots returned as columns (SFDP_Q_PHI)
  if (what == SFDP_Q_COARSE || what == SFDP_Q_COARSE_INV) {
    r = c = p->nK;
  } else {
    if (sub < 0 || sub >= p->nsub) return fail(SFDP_E_INVALID, "sub out of range");
    r = ndv[sub];
    if (what == SFDP_Q_PHI) {
      for (int q = 0; q < NQ; ++q)
        if (cg[NQ * sub + q] >= 0 && cg[NQ * sub + q] < p->nK) qcols.push_back(q);
      c = (int)qcols.size();
    } else if (what == SFDP_Q_SINV || what == SFDP_Q_SBB) {
      c = r;
    } else {
      return fail(SFDP_E_INVALID, "unknown query");
    }
  }
  if (rows) *rows = r;
  if (cols) *cols = c;
  if (!out) return SFDP_OK;
  hipStream_t st = p->ctx->stream;
  HIPCHK(hipStreamSynchronize(st));
  std::vector<cd> host((size_t)r * c);
  if (what == SFDP_Q_COARSE || what == SFDP_Q_COARSE_INV) {
    HIPCHK(hipMemcpy(host.data(), what == SFDP_Q_COARSE ? p->Kcc : p->Kinv, sizeof(cd) * host.size(),
                     hipMemcpyDeviceToHost));
  } else if (what == SFDP_Q_PHI) {
    size_t es = elem_size(*p);
    std::vector<char> raw((size_t)p->ND * NQ * es);
    HIPCHK(hipMemcpy(raw.data(), (const char*)p->Phi + (size_t)sub * p->ND * NQ * es, raw.size(),
                     hipMemcpyDeviceToHost));
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < c; ++j) {
        size_t idx = (size_t)i * NQ + qcols[j];
        if (es == sizeof(cf)) {
          cf v = ((const cf*)raw.data())[idx];
          host[(size_t)i * c + j] = cd{v.x, v.y};
        } else {
          host[(size_t)i * c + j] = ((const cd*)raw.data())[idx];
        }
      }
  } else {
    // packed lower triangles: Sinv in the storage precision, Sbb in complex64
    size_t es = (what == SFDP_Q_SBB) ? sizeof(cf) : elem_size(*p);
    size_t PK = (size_t)p->ND * (p->ND + 1) / 2;
    const char* base = (const char*)(what == SFDP_Q_SINV ? p->Sinv : p->Sbb);
    std::vector<char> raw(PK * es);
    HIPCHK(hipMemcpy(raw.data(), base + (size_t)sub * PK * es, raw.size(), hipMemcpyDeviceToHost));
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < c; ++j) {
        int a = std::max(i, j), b = std::min(i, j);
        size_t idx = (size_t)a * (a + 1) / 2 + b;
        if (es == sizeof(cf)) {
          cf v = ((const cf*)raw.data())[idx];
          host[(size_t)i * c + j] = cd{v.x, v.y};
        } else {
          host[(size_t)i * c + j] = ((const cd*)raw.data())[idx];
        }
      }
  }
  HIPCHK(hipMemcpy(out, host.data(), sizeof(cd) * host.size(), hipMemcpyHostToDevice));
  return SFDP_OK;
}

struct sfdp_problem : public Problem {};
struct sfdp_batch {
  Ctx* ctx = nullptr;
  std::vector<Problem*> probs;
  Multi M;
  int* gmap = nullptr;
  size_t gcap = 0;
  ~sfdp_batch() {
    if (gmap) hipFree(gmap);
    for (Problem* p : probs) destroy_problem(p);
  }
};

extern "C" {

const char* sfdp_last_error(void) { return g_err.c_str(); }
int sfdp_abi_version(void) { return 2; }

sfdp_status sfdp_ctx_create(int device, size_t mem_budget_bytes, void* stream, sfdp_ctx** out) {
  if (!out) return fail(SFDP_E_INVALID, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(SFDP_E_INVALID, "no such device");
  HIPCHK(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, device));
  if (!prop.cooperativeLaunch) return fail(SFDP_E_DEVICE, "device lacks cooperative launch");
  sfdp_ctx* c = new (std::nothrow) sfdp_ctx();
  if (!c) return fail(SFDP_E_NOMEM, "host allocation");
  c->device = device;
  c->budget = mem_budget_bytes;
  c->stream = (hipStream_t)stream;
  c->num_cu = prop.multiProcessorCount;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
    c->max_lds = lds;
  hipError_t e = noalloc_scratch(device, &c->scratch);
  if (e != hipSuccess) {
    delete c;
    return fail(SFDP_E_DEVICE, std::string("scratch address: ") + hipGetErrorString(e));
  }
  *out = c;
  return SFDP_OK;
}

sfdp_status sfdp_ctx_destroy(sfdp_ctx* c) {
  if (!c) return SFDP_OK;
  if (c->children.load() > 0)
    return fail(SFDP_E_STATE, std::to_string(c->children.load()) +
                                  " problems, batches or servers of this context are still alive");
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  if (c->pool) hipFree(c->pool);
  if (c->cap_stream) {
    hipStreamSynchronize(c->cap_stream);
    hipStreamDestroy(c->cap_stream);
    hipEventDestroy(c->cap_ev[0]);
    hipEventDestroy(c->cap_ev[1]);
  }
  delete c;
  return SFDP_OK;
}

sfdp_status sfdp_problem_create(sfdp_ctx* ctx, int dim, int n_elem, int sub_elem, sfdp_precision prec,
                                sfdp_problem** out) {
  if (!ctx || !out) return fail(SFDP_E_INVALID, "NULL argument");
  Problem* p = nullptr;
  sfdp_status s = create_problem(ctx, dim, n_elem, sub_elem, prec, &p);
  *out = (sfdp_problem*)p;
  return s;
}

sfdp_status sfdp_elastic_create(sfdp_ctx* ctx, int n, int sub_elem, int length, double young, double poisson,
                                sfdp_precision prec, sfdp_problem** out) {
  if (!ctx || !out) return fail(SFDP_E_INVALID, "NULL argument");
  *out = nullptr;
  if (sub_elem < 2 || sub_elem > EL_M_MAX) return fail(SFDP_E_INVALID, "sub_elem must be in [2, 6]");
  if (n < sub_elem || n % sub_elem != 0) return fail(SFDP_E_INVALID, "n must be a positive multiple of sub_elem");
  if (length < 1 || length > 64) return fail(SFDP_E_INVALID, "length must be in [1, 64]");
  if (young == 0.0) young = 20.7e6;
  if (poisson == 0.0) poisson = 0.45;
  if (!(young > 0) || !std::isfinite(young)) return fail(SFDP_E_INVALID, "Young's modulus must be positive");
  if (!(poisson > -1.0 && poisson < 0.5)) return fail(SFDP_E_INVALID, "Poisson's ratio must be in (-1, 1/2)");
  if (prec != SFDP_FP64 && prec != SFDP_MIXED && prec != SFDP_MIXED_IFACE)
    return fail(SFDP_E_INVALID, "bad precision");
  const int64_t nsub = (int64_t)(length * n / sub_elem) * (n / sub_elem) * (n / sub_elem);
  if (nsub > 65535) return fail(SFDP_E_INVALID, "at most 65535 subdomains");
  if (nsub < 2) return fail(SFDP_E_INVALID, "at least two subdomains");
  HIPCHK(hipSetDevice(ctx->device));
  Problem* p = new (std::nothrow) Problem();
  if (!p) return fail(SFDP_E_NOMEM, "host allocation");
  p->el = new (std::nothrow) Elastic();
  if (!p->el) {
    delete p;
    return fail(SFDP_E_NOMEM, "host allocation");
  }
  p->ctx = ctx;
  ctx->children++;
  p->dim = 3;
  p->N = n;
  p->m = sub_elem;
  p->ml = sub_elem + 1;
  p->prec = prec;
  sfdp_status s = el_build(*p, n, sub_elem, length, young, poisson);
  if (s) {
    destroy_problem(p);
    return s;
  }
  *out = (sfdp_problem*)p;
  return SFDP_OK;
}

sfdp_status sfdp_elastic_pressure_load(sfdp_problem* p, double pressure, double* f) {
  if (!p || !f) return fail(SFDP_E_INVALID, "NULL argument");
  if (!p->el) return fail(SFDP_E_INVALID, "not an elasticity problem");
  HIPCHK(hipSetDevice(p->ctx->device));
  HIPCHK(hipStreamSynchronize(p->ctx->stream));
  return el_pressure(*p, pressure, f);
}

sfdp_status sfdp_elastic_forward(sfdp_problem* p, int nrhs, const double* f, double* u, const sfdp_opts* opts,
                                 int* krylov_its) {
  if (!p || !f || !u || nrhs <= 0) return fail(SFDP_E_INVALID, "bad arguments");
  if (!p->el) return fail(SFDP_E_INVALID, "not an elasticity problem");
  sfdp_status s = check_host_ptrs(opts);
  if (s) return s;
  HIPCHK(hipSetDevice(p->ctx->device));
  if (host_ptrs(opts)) {
    const size_t n = (size_t)p->n_free * nrhs;
    double* d = nullptr;
    if ((s = stage_area(*p, 2 * n, &d)) || (s = stage_in(*p, d, f, n))) return s;
    sfdp_opts o = *opts;
    o.host_ptrs = 0;
    s = el_forward(*p, nrhs, d, d + n, &o, krylov_its);
    if (s) return s;
    if ((s = stage_out(*p, u, d + n, n))) return s;
    return stage_done(*p);
  }
  return el_forward(*p, nrhs, f, u, opts, krylov_its);
}

static void sizes_of(const Problem* p, sfdp_sizes* out) {
  out->n_free = p->n_free;
  out->n_bdry = p->n_bdry;
  out->n_sub = p->nsub;
  out->n_mult = p->nmu;
  out->n_corner = p->nC;
  out->n_coarse = p->nK;
  out->max_delta = p->dim == 3 ? p->ndmax : 4 * (p->m - 1);
  out->resident_bytes = (int64_t)p->bytes;
}

sfdp_status sfdp_set_setup_arithmetic(int bits) {
  if (bits != 32 && bits != 64) return fail(SFDP_E_INVALID, "bits must be 32 or 64");
  g_setup_bits = bits;
  return SFDP_OK;
}

sfdp_status sfdp_set_gmres_launch(int mode) {
  if (mode < 0 || mode > 2) return fail(SFDP_E_INVALID, "mode must be 0, 1 or 2");
  g_gmres_launch = mode;
  return SFDP_OK;
}

sfdp_status sfdp_set_graphs(int enable) {
  if (enable != 0 && enable != 1) return fail(SFDP_E_INVALID, "enable must be 0 or 1");
  g_graphs = enable == 1;
  return SFDP_OK;
}

sfdp_status sfdp_set_tuning(int enable) {
  if (enable < 0 || enable > 5) return fail(SFDP_E_INVALID, "enable must be in 0..5");
  tune_set_mode(enable == 1, enable >= 2 ? enable - 2 : -1);
  return SFDP_OK;
}

sfdp_status sfdp_set_coarse_space(sfdp_problem* p, int edge_averages) {
  if (!p) return fail(SFDP_E_INVALID, "NULL argument");
  if (edge_averages != 0 && edge_averages != 1) return fail(SFDP_E_INVALID, "edge_averages must be 0 or 1");
  if (p->dim == 3 && edge_averages) return fail(SFDP_E_INVALID, "3D problems use the corner coarse space");
  const int nk = edge_averages ? p->nC + p->nE : p->nC;
  if (nk != p->nK) {
    graphs_clear(*p);
    p->nK = nk;
    p->factored = false;  // the coarse matrix changes: sfdp_set_beta again
  }
  return SFDP_OK;
}

sfdp_status sfdp_problem_sizes(const sfdp_problem* p, sfdp_sizes* out) {
  if (!p || !out) return fail(SFDP_E_INVALID, "NULL argument");
  sizes_of(p, out);
  return SFDP_OK;
}

void sfdp_problem_destroy(sfdp_problem* p) { destroy_problem(p); }

sfdp_status sfdp_set_beta(sfdp_problem* p, double beta) {
  if (!p) return fail(SFDP_E_INVALID, "null problem");
  if (!(beta > 0) || !std::isfinite(beta)) return fail(SFDP_E_INVALID, "beta must be positive and finite");
  HIPCHK(hipSetDevice(p->ctx->device));
  HIPCHK(hipStreamSynchronize(p->ctx->stream));
  p->beta = beta;
  p->alpha = 1.0 / std::sqrt(beta);
  std::vector<Problem*> ps{p};
  const double t0 = wall_ms();
  sfdp_status s = setup_run(single_target(p), ps, nullptr);
  if (s) return s;
  HIPCHK(hipStreamSynchronize(p->ctx->stream));
  p->t_setup_ms = wall_ms() - t0;
  return SFDP_OK;
}


sfdp_status sfdp_feti_solve(sfdp_problem* p, int conj_z, int nrhs, const double* f, double* x,
                            const sfdp_opts* opts, int* krylov_its) {
  sfdp_status s = check_ready(p);
  if (s) return s;
  if (nrhs <= 0 || !f || !x) return fail(SFDP_E_INVALID, "bad arguments");
  if ((s = check_host_ptrs(opts))) return s;
  HIPCHK(hipSetDevice(p->ctx->device));
  if (host_ptrs(opts)) {
    const size_t n = 2 * (size_t)p->n_free * nrhs;  // complex, interleaved
    double* d = nullptr;
    if ((s = stage_area(*p, 2 * n, &d)) || (s = stage_in(*p, d, f, n))) return s;
    sfdp_opts o = *opts;
    o.host_ptrs = 0;
    s = sfdp_feti_solve(p, conj_z, nrhs, d, d + n, &o, krylov_its);
    if (s) return s;
    if ((s = stage_out(*p, x, d + n, n))) return s;
    return stage_done(*p);
  }
  if (p->el) return el_feti(*p, conj_z ? 1 : 0, nrhs, (const cd*)f, (cd*)x, opts, krylov_its);
  double tk, ti;
  int mo, kmax;
  defaults(p->prec, opts, tk, ti, mo, kmax, p->dim);
  const int bsz = batch_of(opts);
  if ((s = alloc_workspace(*p, kmax))) return s;
  Target t = single_target(p);
  int trips = 0, rhs_its = 0;
  for (int r0 = 0; r0 < nrhs; r0 += bsz) {
    const int nr = std::min(bsz, nrhs - r0);
    p->nr = nr;
    p->map = IDENTITY_MAP;
    p->uf = (const cd*)f + (size_t)r0 * p->n_free;
    p->ux = (cd*)x + (size_t)r0 * p->n_free;
    HIPCHK(launch_fill_flags(t, 0, FLAG_WORDS));
    s = feti_run(t, p, V_UF, conj_z ? 1 : 0, V_UX, ti, kmax);
    if (!s) s = gather_one(p);
    p->nr = 0;
    p->uf = nullptr;
    p->ux = nullptr;
    if (s) return s;
    if (p->gh->flags[1]) return fail(SFDP_E_DEVICE, "grid barrier timed out");
    trips += p->gh->flags[3];
    rhs_its += p->gh->flags[4];
    if (krylov_its)
      for (int c = 0; c < nr; ++c) krylov_its[r0 + c] = p->gh->flags[FLAG_ITS + c];
  }
  HIPCHK(ev_harvest(*p));
  if (p->timing) { p->it_gmres += trips; p->it_rhs += rhs_its; }
  return SFDP_OK;
}

sfdp_status sfdp_apply_operator(sfdp_problem* p, char which, int nrhs, const double* x, const double* xc,
                                double* y) {
  if (!p || !x || !y || nrhs <= 0) return fail(SFDP_E_INVALID, "bad arguments");
  HIPCHK(hipSetDevice(p->ctx->device));
  if (p->el) {
    if (xc) return fail(SFDP_E_INVALID, "elasticity problems have no Dirichlet data");
    return el_apply(*p, which, nrhs, x, y);
  }
  if (which == 'K') HIPCHK(launch_apply_K(*p, nrhs, x, xc, y, p->ctx->stream));
  else if (which == 'M') HIPCHK(launch_apply_M(*p, nrhs, x, y, p->ctx->stream));
  else if (which == 'I') {
    if (p->N > 1025) return fail(SFDP_E_INVALID, "the mass inverse needs n_elem <= 1025");
    for (int r = 0; r < nrhs; ++r)
      HIPCHK(launch_mass_inverse(*p, x + r * p->n_free, 1.0, y + r * p->n_free, p->ctx->stream));
  } else {
    return fail(SFDP_E_INVALID, "which must be 'K', 'M' or 'I'");
  }
  return SFDP_OK;
}

sfdp_status sfdp_kkt_residual(sfdp_problem* p, int nrhs, const double* ybar, const double* yc,
                              const double* y, const double* u, const double* lam, double* rel) {
  if (!p || !ybar || !y || !u || !lam || !rel || nrhs <= 0) return fail(SFDP_E_INVALID, "bad arguments");
  if (!(p->beta > 0)) return fail(SFDP_E_STATE, "beta not set");
  HIPCHK(hipSetDevice(p->ctx->device));
  if (p->el) {
    if (yc) return fail(SFDP_E_INVALID, "elasticity problems have no Dirichlet data");
    return el_kkt(*p, nrhs, ybar, y, u, lam, rel, nullptr, nullptr);
  }
  sfdp_status s = alloc_rs(*p);
  if (s) return s;
  const size_t n = p->n_free;
  Target t = single_target(p);
  for (int r0 = 0; r0 < nrhs; r0 += NRMAX) {
    const int nr = std::min(NRMAX, nrhs - r0);
    p->nr = nr;
    p->map = IDENTITY_MAP;
    p->set_slots(nr, ybar + r0 * n, yc ? yc + r0 * p->n_bdry : nullptr, (double*)y + r0 * n,
                 (double*)u + r0 * n, (double*)lam + r0 * n);
    hipError_t e = launch_kkt_residual(t);
    s = e == hipSuccess ? gather_one(p) : fail(SFDP_E_DEVICE, hipGetErrorString(e));
    p->nr = 0;
    if (s) return s;
    for (int c = 0; c < nr; ++c) rel[r0 + c] = p->gh->red[2 * c];
  }
  return SFDP_OK;
}

sfdp_status sfdp_kkt_residual_noalloc(sfdp_problem* p, int nrhs, const double* ybar, const double* yc,
                                      const double* y, const double* u, const double* lam, double* rel) {
  if (!p || !ybar || !y || !u || !lam || !rel || nrhs <= 0) return fail(SFDP_E_INVALID, "bad arguments");
  if (p->el) return fail(SFDP_E_INVALID, "the allocation-free residual covers the Poisson problems only");
  const int64_t need = noalloc_kkt_doubles(p->n_free);
  if (need > NOALLOC_SCRATCH_DOUBLES)
    return fail(SFDP_E_INVALID, "n_free = " + std::to_string(p->n_free) + " needs " + std::to_string(need) +
                                    " scratch doubles, more than the " + std::to_string(NOALLOC_SCRATCH_DOUBLES) +
                                    " the allocation-free residual holds");
  if (!(p->beta > 0)) return fail(SFDP_E_STATE, "beta not set");
  if (!p->ctx->scratch) return fail(SFDP_E_DEVICE, "no scratch address for this device");
  HIPCHK(hipSetDevice(p->ctx->device));
  const int64_t n = p->n_free;
  for (int r0 = 0; r0 < nrhs; r0 += NRMAX) {
    const int nr = std::min(NRMAX, nrhs - r0);
    Dev d = p->dev();
    d.nr = nr;
    d.map = IDENTITY_MAP;
    for (int c = 0; c < NRMAX; ++c)
      d.sl[c] = c < nr ? Slot{ybar + (r0 + c) * n, yc ? yc + (int64_t)(r0 + c) * p->n_bdry : nullptr,
                              (double*)y + (r0 + c) * n, (double*)u + (r0 + c) * n, (double*)lam + (r0 + c) * n}
                       : Slot{};
    d.r1 = d.r2 = d.r3 = nullptr;  // norms only
    d.red = p->ctx->scratch;
    hipError_t e = launch_kkt_residual_noalloc(d, p->ctx->stream, rel + r0);
    if (e != hipSuccess) return fail(SFDP_E_DEVICE, hipGetErrorString(e));
  }
  return SFDP_OK;
}

sfdp_status sfdp_solve_range_space(sfdp_problem* p, int nrhs, const double* ybar, const double* yc,
                                   double* y, double* u, double* lam, const sfdp_opts* opts,
                                   sfdp_info* info) {
  sfdp_status s = check_ready(p);
  if (s) return s;
  if (nrhs <= 0 || !ybar || !y || !u || !lam) return fail(SFDP_E_INVALID, "bad arguments");
  if ((s = check_host_ptrs(opts))) return s;
  HIPCHK(hipSetDevice(p->ctx->device));
  if (host_ptrs(opts)) {
    const size_t n = (size_t)p->n_free * nrhs, nb = yc ? (size_t)p->n_bdry * nrhs : 0;
    double* d = nullptr;
    if ((s = stage_area(*p, 4 * n + nb, &d)) || (s = stage_in(*p, d, ybar, n))) return s;
    if (yc && (s = stage_in(*p, d + 4 * n, yc, nb))) return s;
    sfdp_opts o = *opts;
    o.host_ptrs = 0;
    s = sfdp_solve_range_space(p, nrhs, d, yc ? d + 4 * n : nullptr, d + n, d + 2 * n, d + 3 * n, &o, info);
    if (s != SFDP_OK && s != SFDP_E_NOCONV) return s;
    sfdp_status c;
    if ((c = stage_out(*p, y, d + n, n)) || (c = stage_out(*p, u, d + 2 * n, n)) ||
        (c = stage_out(*p, lam, d + 3 * n, n)) || (c = stage_done(*p)))
      return c;
    return s;
  }
  if (p->el) {
    if (yc) return fail(SFDP_E_INVALID, "elasticity problems have no Dirichlet data");
    return el_range_space(*p, nrhs, ybar, y, u, lam, opts, info);
  }
  double tk, ti;
  int mo, kmax;
  defaults(p->prec, opts, tk, ti, mo, kmax, p->dim);
  const int bsz = batch_of(opts);
  if ((s = alloc_workspace(*p, kmax)) || (s = alloc_rs(*p))) return s;
  if ((s = gather_buffers(*p))) return s;
  Target t = single_target(p);
  sfdp_status worst = SFDP_OK;
  const size_t n = p->n_free;
  std::vector<Problem*> ps{p};
  const double t0 = wall_ms();
  for (int r0 = 0; r0 < nrhs; r0 += bsz) {
    const int ng = std::min(bsz, nrhs - r0);
    p->nr = ng;
    p->set_slots(ng, ybar + r0 * n, yc ? yc + r0 * p->n_bdry : nullptr, y + r0 * n, u + r0 * n,
                 lam + r0 * n);
    std::vector<sfdp_info*> inf{info ? info + r0 : nullptr};
    s = range_space_run(t, ps, nullptr, p->gh, tk, first_tol(p->prec, opts, ti), ti, mo, kmax, inf,
                        single_of(opts));
    p->nr = 0;
    if (s == SFDP_E_NOCONV) worst = s;
    else if (s) return s;
  }
  if (info)
    for (int r = 0; r < nrhs; ++r) info[r].t_solve_ms = wall_ms() - t0;
  return worst;
}

sfdp_status sfdp_apply_schur_inv(sfdp_problem* p, int nrhs, const double* r, double* z,
                                 const sfdp_opts* opts, sfdp_info* info);

namespace {
// The twin of a problem that holds the FETI-DP factors of the real matrix
// F = K + alpha M, the outer factor of the approximation S_p = F M^-1 F of
// Pearson and Wathen (Sec. 3.2): the same mesh, subdomains, precision and
// coarse space; created the first time S_p is used, factored again when beta
// or the coarse space of the problem has changed since.
sfdp_status ensure_pw(Problem* p) {
  if (!p->pw) {
    Problem* q = nullptr;
    sfdp_status s = create_problem(p->ctx, p->dim, p->N, p->m, p->prec, &q);
    if (s) return s;
    q->rshift = true;
    p->pw = q;
  }
  Problem* q = p->pw;
  if (q->nK != p->nK) {
    q->nK = p->nK;
    q->factored = false;
  }
  if (q->factored && q->beta == p->beta) return SFDP_OK;
  HIPCHK(hipStreamSynchronize(p->ctx->stream));
  q->beta = p->beta;
  q->alpha = p->alpha;
  std::vector<Problem*> ps{q};
  return setup_run(single_target(q), ps, nullptr);
}
}  // namespace

// ---- full-space method: MINRES with P_mgw inside FP64 refinement ----
namespace {
constexpr double FS_MINRES_TOL = 1e-6;
constexpr int FS_MINRES_MAXIT = 30;      // exact S: three distinct eigenvalues
constexpr int FS_MINRES_MAXIT_SP = 100;  // S_p: eigenvalues of S_p^-1 S in [1/2, 1]

struct FsCtx {
  sfdp_problem* p;
  hipStream_t st;
  int64_t n, n3;
  double *part, *dot;  // device block sums and result
  double* host;        // pinned
  sfdp_opts inner;
  sfdp_info* log;
  int maxit;
};

sfdp_status fs_dot(FsCtx& c, const double* x, const double* y, double& out) {
  HIPCHK(launch_dot(c.n3, x, y, c.part, c.dot, c.st));
  HIPCHK(hipMemcpyAsync(c.host, c.dot, sizeof(double), hipMemcpyDeviceToHost, c.st));
  HIPCHK(hipStreamSynchronize(c.st));
  out = c.host[0];
  return SFDP_OK;
}

// out = P_mgw^-1 r: V^-1 r1, (phi V)^-1 r2, S^-1 r3 (two FETI-DP solves, or one;
// with S_p in place of S: two solves with its real factor)
sfdp_status fs_pinv(FsCtx& c, const double* r, double* out) {
  Problem* p = c.p;
  HIPCHK(launch_mass_inverse(*p, r, 1.0, out, c.st));
  HIPCHK(launch_mass_inverse(*p, r + c.n, 1.0 / p->beta, out + c.n, c.st));
  sfdp_info inf{};
  sfdp_status s = sfdp_apply_schur_inv(c.p, 1, r + 2 * c.n, out + 2 * c.n, &c.inner, &inf);
  if (s) return s;
  sfdp_info& o = *c.log;
  for (int k = 0; k < inf.n_feti; ++k) {
    if (o.n_feti < 16) o.krylov_its[o.n_feti] = inf.krylov_its[k];
    ++o.n_feti;
    o.krylov_total += inf.krylov_its[k];
  }
  return SFDP_OK;
}

// MINRES (C. C. Paige and M. A. Saunders, SIAM J. Numer. Anal. 12 (1975) 617-629;
// the scalars carry that method's usual names) on A dx = rr with the preconditioner P_mgw, from
// dx = 0: Lanczos in the P-inner product, Givens QR of its tridiagonal matrix,
// search directions w.  V holds 8 device vectors of length 3n.
sfdp_status fs_minres(FsCtx& c, double* V, const double* rr, double* dx, int& its) {
  const int64_t n3 = c.n3;
  hipStream_t st = c.st;
  double *r1 = V, *r2 = V + n3, *y = V + 2 * n3, *v = V + 3 * n3, *w = V + 4 * n3, *w1 = V + 5 * n3,
         *w2 = V + 6 * n3;
  HIPCHK(launch_lin3(n3, 0.0, nullptr, 0.0, nullptr, 0.0, nullptr, dx, st));
  HIPCHK(launch_lin3(n3, 0.0, nullptr, 0.0, nullptr, 0.0, nullptr, w, st));
  HIPCHK(launch_lin3(n3, 0.0, nullptr, 0.0, nullptr, 0.0, nullptr, w2, st));
  HIPCHK(launch_lin3(n3, 1.0, rr, 0.0, nullptr, 0.0, nullptr, r1, st));
  HIPCHK(launch_lin3(n3, 1.0, rr, 0.0, nullptr, 0.0, nullptr, r2, st));
  sfdp_status s = fs_pinv(c, r1, y);
  double b1 = 0.0;
  if (s || (s = fs_dot(c, r1, y, b1))) return s;
  its = 0;
  if (!(b1 > 0.0)) return SFDP_OK;
  const double beta1 = std::sqrt(b1);
  double bet = beta1, oldb = 0.0, dbar = 0.0, epsln = 0.0, phibar = beta1, cs = -1.0, sn = 0.0;
  for (int k = 1; k <= c.maxit; ++k) {
    its = k;
    c.p->yield_point();
    HIPCHK(launch_lin3(n3, 1.0 / bet, y, 0.0, nullptr, 0.0, nullptr, v, st));
    HIPCHK(launch_kkt_apply(*c.p, v, y, st));
    if (k >= 2) HIPCHK(launch_lin3(n3, 1.0, y, -bet / oldb, r1, 0.0, nullptr, y, st));
    double alfa = 0.0;
    if ((s = fs_dot(c, v, y, alfa))) return s;
    HIPCHK(launch_lin3(n3, 1.0, y, -alfa / bet, r2, 0.0, nullptr, y, st));
    std::swap(r1, r2);  // r1 <- r2, r2 <- y, and the old r1 buffer receives P^-1 r2
    std::swap(r2, y);
    if ((s = fs_pinv(c, r2, y))) return s;
    double q = 0.0;
    if ((s = fs_dot(c, r2, y, q))) return s;
    if (q < 0.0 || !std::isfinite(q)) break;  // the preconditioner is not positive definite
    oldb = bet;
    bet = std::sqrt(q);  // zero: the Krylov space is exhausted, this step is the last
    const double oldeps = epsln;
    const double delta = cs * dbar + sn * alfa, gbar = sn * dbar - cs * alfa;
    epsln = sn * bet;
    dbar = -cs * bet;
    const double gamma = std::max(std::hypot(gbar, bet), 1e-300);
    cs = gbar / gamma;
    sn = bet / gamma;
    const double phi = cs * phibar;
    phibar = sn * phibar;
    std::swap(w1, w2);  // w1 <- w2, w2 <- w, w <- (v - oldeps w1 - delta w2) / gamma
    std::swap(w2, w);
    HIPCHK(launch_lin3(n3, 1.0 / gamma, v, -oldeps / gamma, w1, -delta / gamma, w2, w, st));
    HIPCHK(launch_lin3(n3, 1.0, dx, phi, w, 0.0, nullptr, dx, st));
    if (phibar <= FS_MINRES_TOL * beta1 || !(bet > 0.0)) break;
  }
  return SFDP_OK;
}
}  // namespace

sfdp_status sfdp_apply_schur_inv(sfdp_problem* p, int nrhs, const double* r, double* z,
                                 const sfdp_opts* opts, sfdp_info* info) {
  sfdp_status s = check_ready(p);
  if (s) return s;
  if (nrhs <= 0 || !r || !z) return fail(SFDP_E_INVALID, "bad arguments");
  if (opts && opts->schur_block != 0 && opts->schur_block != 1) return fail(SFDP_E_INVALID, "schur_block must be 0 or 1");
  if ((s = check_host_ptrs(opts))) return s;
  if (host_ptrs(opts)) {
    HIPCHK(hipSetDevice(p->ctx->device));
    const size_t n = (size_t)p->n_free * nrhs;
    double* d = nullptr;
    if ((s = stage_area(*p, 2 * n, &d)) || (s = stage_in(*p, d, r, n))) return s;
    sfdp_opts o = *opts;
    o.host_ptrs = 0;
    s = sfdp_apply_schur_inv(p, nrhs, d, d + n, &o, info);
    if (s) return s;
    if ((s = stage_out(*p, z, d + n, n))) return s;
    return stage_done(*p);
  }
  if (p->el) {
    HIPCHK(hipSetDevice(p->ctx->device));
    return el_schur_inv(*p, nrhs, r, z, opts, info);
  }
  if (opts && opts->schur_block == 1) {
    // S_p^-1 r = F^-1 M F^-1 r: the two-factor sequence on the twin, whose
    // factor is real (so the conjugations and the real part change nothing)
    HIPCHK(hipSetDevice(p->ctx->device));
    if ((s = ensure_pw(p))) return s;
    sfdp_opts o = *opts;
    o.schur_block = 0;
    o.factors = 2;
    return sfdp_apply_schur_inv((sfdp_problem*)p->pw, nrhs, r, z, &o, info);
  }
  double tk, ti;
  int mo, kmax;
  defaults(p->prec, opts, tk, ti, mo, kmax, p->dim);
  const int bsz = batch_of(opts);
  HIPCHK(hipSetDevice(p->ctx->device));
  if ((s = alloc_workspace(*p, kmax)) || (s = alloc_rs(*p))) return s;
  hipStream_t st = p->ctx->stream;
  const int64_t n = p->n_free;
  Target t = single_target(p);
  // the middle factor needs r1 = 0: v = conj(0 + M w)
  HIPCHK(launch_fill(p->r1, sizeof(double) * NRMAX * n, st));
  for (int r0 = 0; r0 < nrhs; r0 += bsz) {
    const int nr = std::min(bsz, nrhs - r0);
    p->nr = nr;
    p->map = IDENTITY_MAP;
    HIPCHK(launch_fill_flags(t, 0, FLAG_WORDS));
    // factor 1: w = Z^-1 r ; middle: v = conj(M w) ; factor 2: z = Re conj(Z^-1 v) = Re Z^-1 v
    // (one solve: z = -Im(w) / alpha)
    HIPCHK(launch_copy_real_to_complex(nr * n, r + r0 * n, p->cvec, st));
    s = feti_run(t, p, V_CVEC, 0, V_CVEC2, ti, kmax);
    if (!s && single_of(opts)) {
      hipError_t e = launch_imag_scaled(nr * n, p->cvec2, -1.0 / p->alpha, z + r0 * n, st);
      s = e == hipSuccess ? gather_one(p) : fail(SFDP_E_DEVICE, hipGetErrorString(e));
    } else if (!s) {
      hipError_t e = launch_make_rhs2(t);
      s = e == hipSuccess ? feti_run(t, p, V_CVEC3, 0, V_CVEC, ti, kmax) : fail(SFDP_E_DEVICE, hipGetErrorString(e));
      if (!s) {
        e = launch_real_part(nr * n, p->cvec, z + r0 * n, st);
        s = e == hipSuccess ? gather_one(p) : fail(SFDP_E_DEVICE, hipGetErrorString(e));
      }
    }
    p->nr = 0;
    if (s) return s;
    if (p->gh->flags[1]) return fail(SFDP_E_DEVICE, "grid barrier timed out");
    if (p->timing) { p->it_gmres += p->gh->flags[3]; p->it_rhs += p->gh->flags[4]; }
    if (info)
      for (int c = 0; c < nr; ++c) {
        sfdp_info& o = info[r0 + c];
        o = blank_info();
        o.n_feti = single_of(opts) ? 1 : 2;
        for (int k = 0; k < o.n_feti; ++k) {
          o.krylov_its[k] = p->gh->flags[FLAG_LOG + 16 * c + k];
          o.krylov_total += o.krylov_its[k];
        }
      }
  }
  HIPCHK(ev_harvest(*p));
  return SFDP_OK;
}

sfdp_status sfdp_solve_full_space(sfdp_problem* p, int nrhs, const double* ybar, const double* yc, double* y,
                                  double* u, double* lam, const sfdp_opts* opts, sfdp_info* info) {
  sfdp_status s = check_ready(p);
  if (s) return s;
  if (nrhs <= 0 || !ybar || !y || !u || !lam) return fail(SFDP_E_INVALID, "bad arguments");
  if (p->el) return fail(SFDP_E_INVALID, "the full-space method covers the Poisson problems only");
  if (p->N > 1025) return fail(SFDP_E_INVALID, "the full-space method needs n_elem <= 1025");
  if ((s = check_host_ptrs(opts))) return s;
  if (host_ptrs(opts)) {
    HIPCHK(hipSetDevice(p->ctx->device));
    const size_t n = (size_t)p->n_free * nrhs, nb = yc ? (size_t)p->n_bdry * nrhs : 0;
    double* d = nullptr;
    if ((s = stage_area(*p, 4 * n + nb, &d)) || (s = stage_in(*p, d, ybar, n))) return s;
    if (yc && (s = stage_in(*p, d + 4 * n, yc, nb))) return s;
    sfdp_opts o = *opts;
    o.host_ptrs = 0;
    s = sfdp_solve_full_space(p, nrhs, d, yc ? d + 4 * n : nullptr, d + n, d + 2 * n, d + 3 * n, &o, info);
    if (s != SFDP_OK && s != SFDP_E_NOCONV) return s;
    sfdp_status c;
    if ((c = stage_out(*p, y, d + n, n)) || (c = stage_out(*p, u, d + 2 * n, n)) ||
        (c = stage_out(*p, lam, d + 3 * n, n)) || (c = stage_done(*p)))
      return c;
    return s;
  }
  double tk, ti;
  int mo, kmax;
  defaults(p->prec, opts, tk, ti, mo, kmax, p->dim);
  HIPCHK(hipSetDevice(p->ctx->device));
  if ((s = alloc_workspace(*p, kmax)) || (s = alloc_rs(*p)) || (s = gather_buffers(*p))) return s;
  const int64_t n = p->n_free, n3 = 3 * n, nb = (n3 + 255) / 256;
  if (!p->fsw) {
    if ((s = dalloc(*p, (void**)&p->fsw, sizeof(double) * (10 * n3 + nb + 8)))) return s;
    if (hipHostMalloc((void**)&p->fsh, sizeof(double) * 8) != hipSuccess) {
      p->fsh = nullptr;
      return fail(SFDP_E_NOMEM, "pinned host allocation");
    }
  }
  if (opts && opts->schur_block != 0 && opts->schur_block != 1) return fail(SFDP_E_INVALID, "schur_block must be 0 or 1");
  const bool sp = opts && opts->schur_block == 1;
  if (sp && (s = ensure_pw(p))) return s;
  FsCtx c{p, p->ctx->stream, n, n3, p->fsw + 10 * n3, p->fsw + 10 * n3 + nb, p->fsh, {}, nullptr,
          sp ? FS_MINRES_MAXIT_SP : FS_MINRES_MAXIT};
  if (opts) c.inner = *opts;
  c.inner.batch = 1;
  double* Vw = p->fsw;            // 8 MINRES vectors
  double* dx = p->fsw + 8 * n3;
  double* rr = p->fsw + 9 * n3;
  Target t = single_target(p);
  hipStream_t st = c.st;
  sfdp_status worst = SFDP_OK;
  const double t_call = wall_ms();
  for (int q = 0; q < nrhs; ++q) {
    sfdp_info o{};
    c.log = &o;
    double* yq = y + q * n;
    double* uq = u + q * n;
    double* lq = lam + q * n;
    p->nr = 1;
    p->map = IDENTITY_MAP;
    p->set_slots(1, ybar + q * n, yc ? yc + q * p->n_bdry : nullptr, yq, uq, lq);
    p->init = 1u;
    HIPCHK(launch_group_init(t));
    p->init = 0;
    bool bad = false;
    for (int step = 0;; ++step) {
      p->yield_point();
      p->nr = 1;
      p->map = IDENTITY_MAP;
      HIPCHK(launch_kkt_residual(t));
      if ((s = gather_one(p))) return s;
      const double rho = p->gh->red[0];
      o.rel_kkt = rho;
      if (step == 1) o.rel_kkt_first = rho;
      if (!std::isfinite(rho) || step >= mo) {
        bad = rho > tk || !std::isfinite(rho);
        break;
      }
      if (rho <= tk) break;
      // rr = b - A x (the residual blocks of slot 0), then x += MINRES(A, rr)
      HIPCHK(hipMemcpyAsync(rr, p->r1, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(rr + n, p->r2, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(rr + 2 * n, p->r3, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
      int its = 0;
      if ((s = fs_minres(c, Vw, rr, dx, its))) return s;
      o.minres_its += its;
      HIPCHK(launch_lin3(n, 1.0, yq, 1.0, dx, 0.0, nullptr, yq, st));
      HIPCHK(launch_lin3(n, 1.0, uq, 1.0, dx + n, 0.0, nullptr, uq, st));
      HIPCHK(launch_lin3(n, 1.0, lq, 1.0, dx + 2 * n, 0.0, nullptr, lq, st));
      o.outer_steps = step + 1;
    }
    p->nr = 1;
    p->map = IDENTITY_MAP;
    HIPCHK(launch_kkt_metrics(t));
    if ((s = gather_one(p))) return s;
    o.constr_viol = p->gh->red[MET_HEAD];
    o.eta_blk = p->gh->red[MET_HEAD + 1];
    o.t_setup_ms = p->t_setup_ms;
    p->nr = 0;
    if (info) info[q] = o;
    if (bad) worst = fail(SFDP_E_NOCONV, "full-space refinement did not reach tol_kkt");
  }
  HIPCHK(hipStreamSynchronize(st));
  if (info)
    for (int q = 0; q < nrhs; ++q) info[q].t_solve_ms = wall_ms() - t_call;
  return worst;
}

// ---- batches of independent instances ----

sfdp_status sfdp_batch_create(sfdp_ctx* ctx, int count, const int* n_elem, int sub_elem, sfdp_precision prec,
                              sfdp_batch** out) {
  if (!ctx || !out || !n_elem || count <= 0) return fail(SFDP_E_INVALID, "bad arguments");
  *out = nullptr;
  sfdp_batch* b = new (std::nothrow) sfdp_batch();
  if (!b) return fail(SFDP_E_NOMEM, "host allocation");
  b->ctx = ctx;
  int64_t nsub_tot = 0;
  for (int i = 0; i < count; ++i) {
    Problem* p = nullptr;
    sfdp_status s = create_problem(ctx, 2, n_elem[i], sub_elem, prec, &p);
    if (s) { delete b; return s; }
    b->probs.push_back(p);
    nsub_tot += p->nsub;
  }
  // GMRES blocks per instance: one per subdomain when all fit on the device at
  // once, otherwise enough to keep every block's multiplier chunk <= 192
  HIPCHK(hipSetDevice(ctx->device));
  for (Problem* p : b->probs)
    p->gmres_blocks = nsub_tot <= ctx->num_cu ? p->nsub : shared_gmres_blocks(*p, 64, 192);
  b->M.ctx = ctx;
  b->M.probs = b->probs;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  sfdp_status s = multi_maps(b->M);
  if (s) { delete b; return s; }
  *out = b;
  return SFDP_OK;
}

void sfdp_batch_destroy(sfdp_batch* b) {
  if (!b) return;
  hipSetDevice(b->ctx->device);
  hipStreamSynchronize(b->ctx->stream);
  delete b;
}

sfdp_status sfdp_batch_sizes(const sfdp_batch* b, int i, sfdp_sizes* out) {
  if (!b || !out || i < 0 || i >= (int)b->probs.size()) return fail(SFDP_E_INVALID, "bad arguments");
  sizes_of(b->probs[i], out);
  return SFDP_OK;
}

sfdp_status sfdp_batch_inspect(sfdp_batch* b, int i, sfdp_query what, int sub, double* out, int* rows,
                               int* cols) {
  if (!b || i < 0 || i >= (int)b->probs.size()) return fail(SFDP_E_INVALID, "bad arguments");
  return inspect_problem(b->probs[i], what, sub, out, rows, cols);
}

sfdp_status sfdp_batch_set_beta(sfdp_batch* b, const double* beta) {
  if (!b || !beta) return fail(SFDP_E_INVALID, "bad arguments");
  for (size_t i = 0; i < b->probs.size(); ++i)
    if (!(beta[i] > 0) || !std::isfinite(beta[i])) return fail(SFDP_E_INVALID, "beta must be positive and finite");
  HIPCHK(hipSetDevice(b->ctx->device));
  HIPCHK(hipStreamSynchronize(b->ctx->stream));
  for (size_t i = 0; i < b->probs.size(); ++i) {
    Problem* p = b->probs[i];
    p->beta = beta[i];
    p->alpha = 1.0 / std::sqrt(beta[i]);
  }
  const double t0 = wall_ms();
  sfdp_status s = setup_run(b->M.t, b->probs, &b->M);
  if (s) return s;
  HIPCHK(hipStreamSynchronize(b->ctx->stream));
  const double ms = wall_ms() - t0;
  for (Problem* p : b->probs) p->t_setup_ms = ms;
  return SFDP_OK;
}

sfdp_status sfdp_batch_solve_range_space(sfdp_batch* b, const int* nrhs, const double* const* ybar,
                                         const double* const* yc, double* const* y, double* const* u,
                                         double* const* lam, const sfdp_opts* opts, sfdp_info* info) {
  if (!b || !nrhs || !ybar || !y || !u || !lam) return fail(SFDP_E_INVALID, "bad arguments");
  const int n = (int)b->probs.size();
  int rmax = 0;
  for (int i = 0; i < n; ++i) {
    if (nrhs[i] < 0 || (nrhs[i] > 0 && (!ybar[i] || !y[i] || !u[i] || !lam[i])))
      return fail(SFDP_E_INVALID, "bad arguments");
    sfdp_status s = check_ready(b->probs[i]);
    if (s) return s;
    rmax = std::max(rmax, nrhs[i]);
  }
  double tk, ti;
  int mo, kmax;
  defaults(b->probs[0]->prec, opts, tk, ti, mo, kmax);
  const int bsz = batch_of(opts);
  HIPCHK(hipSetDevice(b->ctx->device));
  for (Problem* p : b->probs) {
    sfdp_status s;
    if ((s = alloc_workspace(*p, kmax)) || (s = alloc_rs(*p))) return s;
  }
  HIPCHK(hipStreamSynchronize(b->ctx->stream));
  const double t_call = wall_ms();
  std::vector<int64_t> ioff(n + 1, 0);
  for (int i = 0; i < n; ++i) ioff[i + 1] = ioff[i] + nrhs[i];
  sfdp_status worst = SFDP_OK;
  for (int r0 = 0; r0 < rmax; r0 += bsz) {
    int w = 0;
    std::vector<sfdp_info*> inf(n, nullptr);
    for (int i = 0; i < n; ++i) {
      Problem* p = b->probs[i];
      const int ng = std::max(0, std::min(bsz, nrhs[i] - r0));
      p->nr = ng;
      w = std::max(w, ng);
      if (ng == 0) continue;
      const size_t nf = p->n_free;
      p->set_slots(ng, ybar[i] + r0 * nf, yc && yc[i] ? yc[i] + r0 * p->n_bdry : nullptr, y[i] + r0 * nf,
                   u[i] + r0 * nf, lam[i] + r0 * nf);
      inf[i] = info ? info + ioff[i] + r0 : nullptr;
    }
    sfdp_status s = multi_groups(b->M, kmax, w == 1 ? 1 : w == 2 ? 2 : 4, b->gmap, b->gcap);
    if (!s)
      s = range_space_run(b->M.t, b->probs, &b->M, b->M.hgather, tk,
                          first_tol(b->probs[0]->prec, opts, ti), ti, mo, kmax, inf,
                          single_of(opts));
    for (Problem* p : b->probs) p->nr = 0;
    if (s == SFDP_E_NOCONV) worst = s;
    else if (s) return s;
  }
  if (info)
    for (int64_t k = 0; k < ioff[n]; ++k) info[k].t_solve_ms = wall_ms() - t_call;
  return worst;
}


sfdp_status sfdp_inspect(sfdp_problem* p, sfdp_query what, int sub, double* out, int* rows, int* cols) {
  return inspect_problem(p, what, sub, out, rows, cols);
}

sfdp_status sfdp_timing_enable(sfdp_problem* p, int enable) {
  if (!p) return fail(SFDP_E_INVALID, "null problem");
  if (enable < 0 || enable > 2) return fail(SFDP_E_INVALID, "enable must be 0, 1 or 2");
  HIPCHK(hipSetDevice(p->ctx->device));
  HIPCHK(hipStreamSynchronize(p->ctx->stream));
  p->ev_pending.clear();
  p->ev_used = 0;
  p->timing = enable;
  p->t_gmres_ms = p->t_local_ms = 0;
  p->n_gmres = p->n_local = p->it_gmres = p->it_rhs = 0;
  return SFDP_OK;
}

sfdp_status sfdp_kernel_times(sfdp_problem* p, sfdp_timing* out) {
  if (!p || !out) return fail(SFDP_E_INVALID, "NULL argument");
  HIPCHK(hipSetDevice(p->ctx->device));
  HIPCHK(hipStreamSynchronize(p->ctx->stream));
  HIPCHK(ev_harvest(*p));
  out->gmres_ms = p->t_gmres_ms;
  out->local_ms = p->t_local_ms;
  out->gmres_launches = p->n_gmres;
  out->gmres_iters = p->it_gmres;
  out->gmres_rhs_iters = p->it_rhs;
  out->gmres_width = p->last_nrt;
  out->gmres_resident = p->last_resident ? 1 : 0;
  out->local_launches = p->n_local;
  return SFDP_OK;
}

sfdp_status sfdp_interface_apply(sfdp_problem* p, char which, const double* x, double* y) {
  sfdp_status s = check_ready(p);
  if (s) return s;
  if (!x || !y) return fail(SFDP_E_INVALID, "bad arguments");
  HIPCHK(hipSetDevice(p->ctx->device));
  hipStream_t st = p->ctx->stream;
  if (p->el) {
    if (which != 'F' && which != 'P' && which != 'D') return fail(SFDP_E_INVALID, "which must be 'F', 'P' or 'D'");
    return el_interface(*p, which, (const cd*)x, (cd*)y);
  }
  if (p->dim == 3) {
    if (which != 'F' && which != 'P' && which != 'D') return fail(SFDP_E_INVALID, "which must be 'F', 'P' or 'D'");
    if ((s = alloc_workspace3(*p, 1))) return s;
    HIPCHK(interface3(*p, which, (const cd*)x, (cd*)y));
    return SFDP_OK;
  }
  if (which == 'D') {
    Target t = single_target(p);
    p->nr = 1;
    p->map = IDENTITY_MAP;
    p->uf = (const cd*)x;
    hipError_t e = launch_local_solve(t, 0, V_UF, 0, V_UX);
    if (e == hipSuccess) e = launch_coarse_rhs(t, V_UF, 0);
    if (e == hipSuccess) e = launch_fetidp_rhs(t);
    p->nr = 0;
    p->uf = nullptr;
    HIPCHK(e);
    HIPCHK(hipMemcpyAsync(y, p->dvec, sizeof(cd) * p->nmu, hipMemcpyDeviceToDevice, st));
    return SFDP_OK;
  }
  if (which != 'F' && which != 'P') return fail(SFDP_E_INVALID, "which must be 'F', 'P' or 'D'");
  HIPCHK(launch_interface_apply(*p, which, (const cd*)x, (cd*)y, st));
  return SFDP_OK;
}

}  // extern "C"

// ---- serving: continuous batching of range-space requests ----
namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct SReq;
struct SInst;

struct SReq {
  uint64_t id = 0;
  int dim = 2, mode = 0;  // mode 1: full-space method
  int n_elem = 0, sub_elem = 0, nrhs = 0;
  double beta = 0;
  const double *ybar = nullptr, *yc = nullptr;
  double *y = nullptr, *u = nullptr, *lam = nullptr;
  int next = 0;  // next target to place in a slot
  int done = 0;  // targets finished
  std::vector<sfdp_info> info;
  sfdp_status status = SFDP_OK;
  double t_submit = 0, t_done = 0;
  bool complete = false;
  SInst* inst = nullptr;
  std::string why;  // reason of a refusal or failure
};

struct SSlot {
  SReq* req = nullptr;
  int k = -1;    // target index within the request
  int bad = 0;   // 1 non-finite, 2 outer limit
  sfdp_info info{};
};

struct SInst {
  Problem* p = nullptr;
  int n_elem = 0, sub_elem = 0;
  double beta = 0;
  std::deque<SReq*> queue;  // admitted requests with targets left to place
  SSlot slot[NRMAX];
  double last_used = 0;
  bool busy() const {
    if (!queue.empty()) return true;
    for (const SSlot& s : slot)
      if (s.req) return true;
    return false;
  }
};

// A single problem of the solo lane (3D or full-space requests), resident for
// the requests that follow with the same mesh and beta.
struct SSolo {
  Problem* p = nullptr;
  int dim = 2, n_elem = 0, sub_elem = 0;
  double beta = 0;
  double last_used = 0;
  bool busy = false;  // a running job solves on it
};
constexpr size_t SOLO_KEEP = 4;  // idle solo problems kept resident at most
constexpr size_t SOLO_JOBS = 4;  // solo requests in flight at once

// A solo request in flight on a host thread of its own.  It runs only while it
// holds the turn, which the worker hands to every job once per tick and takes
// back at the job's next yield point (the start of a refinement step or of a
// MINRES iteration), so the requests advance step by step, interleaved with the
// batched ticks and with each other, on the server's stream.
struct SJob {
  sfdp_server* S = nullptr;
  SReq* r = nullptr;
  std::thread th;
  bool turn = false;
  bool done = false;
  sfdp_status dev = SFDP_OK;  // a device error ends the service
};

}  // namespace

struct sfdp_server {
  Ctx* ctx = nullptr;
  sfdp_precision prec = SFDP_MIXED;
  double tol_kkt = 0, tol_inner = 0;
  int max_outer = 0, kmax = 0;
  bool single = false;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<SReq*> pending;              // submitted, not admitted
  std::map<uint64_t, SReq*> reqs;         // every request until polled after completion
  std::vector<SInst*> insts;              // resident instances
  std::vector<double> lat;                // completed latencies (ms)
  uint64_t next_id = 1;
  bool stop = false;
  std::thread worker;
  Multi M;
  int* gmap = nullptr;
  size_t gcap = 0;
  std::vector<Problem*> active_set;       // instances of the current target
  Gathered* hg = nullptr;  // pinned host, written by the gather kernel
  size_t gath_cap = 0;
  int64_t n_submit = 0, n_complete = 0, n_failed = 0, n_setups = 0, n_evict = 0, n_ticks = 0;
  std::string worker_error;
  std::vector<SReq*> finished;  // decided by the worker, published under the lock
  size_t pool_cap = 0;          // set-up scratch of one set-up pass (a larger instance passes alone)
  int user_kmax = 0;            // opts->max_krylov as given (0: each path's default)
  std::deque<SReq*> solo;       // 3D and full-space requests waiting for a job (worker only)
  std::vector<SSolo*> solos;    // their resident problems
  std::vector<SJob*> jobs;      // solo requests in flight
  int64_t n_jobs_max = 0;       // most jobs in flight at once
  std::mutex tmu;               // turn hand-off between the worker and the jobs
  std::condition_variable tcv;
};

namespace {

// Device bytes an instance of this mesh will hold once factored (maps,
// workspaces, factors), for admission.
size_t instance_bytes(int n_elem, int sub_elem, sfdp_precision prec) {
  const size_t P = n_elem / sub_elem, nsub = P * P, ml = sub_elem + 1;
  const size_t ND = ((4 * (sub_elem - 1) + 31) / 32) * 32, nf = (size_t)(n_elem - 1) * (n_elem - 1);
  const size_t nmu = 2 * P * (P - 1) * (sub_elem - 1), nC = (P - 1) * (P - 1) + 2 * P * (P - 1);
  const size_t es = prec == SFDP_FP64 ? 16 : 8, gs = prec == SFDP_MIXED ? 8 : 16;
  size_t b = nsub * ml * ml * ml * gs + nsub * ND * (ND + 1) / 2 * (es + 8) + nsub * ND * NQ * es + 2 * nC * nC * 16;
  b += NRMAX * (4 * nsub * ND + 2 * nsub * NQ + 3 * nC + 3 * nmu) * 16;  // solve workspaces
  b += NRMAX * (65 * nmu + 65 * 64) * 16 + 3 * NRMAX * 66 * nsub * 16;  // Krylov state (kmax 64)
  b += NRMAX * nf * (3 * 8 + 3 * 16);                                    // range-space workspaces
  b += nsub * ND * 40 + nmu * 12 + (size_t)(n_elem + 1) * (n_elem + 1) * 4;  // maps
  return b;
}


// The worker decides that a request is over; it becomes visible to pollers when
// the worker publishes its finished list under the lock.
void server_finish(sfdp_server* S, SReq* r, sfdp_status st) {
  if (st) r->status = st;
  r->t_done = now_ms();
  S->finished.push_back(r);
}

// Move pending requests onto resident instances, creating (and later
// factoring) instances while the memory budget allows; idle instances are
// evicted oldest first.  Returns the instances created (to be factored).
std::vector<SInst*> server_admit(sfdp_server* S, std::deque<SReq*>& pend) {
  std::vector<SInst*> fresh;
  Ctx* ctx = S->ctx;
  size_t reserve = 0;  // factor bytes the fresh instances will allocate at set-up
  while (!pend.empty()) {
    SReq* r = pend.front();
    SInst* home = nullptr;
    for (SInst* in : S->insts)
      if (in->n_elem == r->n_elem && in->sub_elem == r->sub_elem && in->beta == r->beta) home = in;
    if (!home) {
      size_t need = instance_bytes(r->n_elem, r->sub_elem, S->prec);
      // the set-up passes' scratch: at most the pool cap per pass unless one
      // instance alone needs more (the passes are chunked the same way)
      size_t sum = setup_bytes(r->n_elem, r->sub_elem), big = sum;
      for (SInst* in : fresh) {
        const size_t b = setup_bytes(in->n_elem, in->sub_elem);
        sum += b;
        big = std::max(big, b);
      }
      const size_t pool_need = std::min(sum, std::max(S->pool_cap, big));
      // growing the pool frees the old one first: only the difference is new
      size_t pool_grow = pool_need > ctx->pool_bytes ? pool_need - ctx->pool_bytes : 0;
      auto fits = [&]() { return !ctx->budget || ctx->used + reserve + need + pool_grow <= ctx->budget; };
      // evict the least recently used idle instance (false if none)
      auto evict_one = [&]() {
        SInst* victim = nullptr;
        for (SInst* in : S->insts)
          if (!in->busy() && std::find(fresh.begin(), fresh.end(), in) == fresh.end() &&
              (!victim || in->last_used < victim->last_used))
            victim = in;
        if (!victim) return false;
        S->insts.erase(std::find(S->insts.begin(), S->insts.end(), victim));
        destroy_problem(victim->p);
        delete victim;
        S->active_set.clear();  // its address may be reused by a new instance
        ++S->n_evict;
        return true;
      };
      auto anything_busy = [&]() {
        bool b = !fresh.empty();
        for (SInst* in : S->insts) b = b || in->busy();
        return b;
      };
      while (!fits() && evict_one()) {
      }
      if (!fits()) {
        if (anything_busy()) break;  // wait for memory to free up
        pend.pop_front();
        r->why = "request can never fit the memory budget: " + std::to_string(ctx->used) + " B held, " +
                 std::to_string(need) + " B instance + " + std::to_string(pool_grow) + " B set-up scratch needed, budget " +
                 std::to_string(ctx->budget) + " B";
        server_finish(S, r, SFDP_E_ADMIT);
        continue;
      }
      // the estimate can be short of the real allocations: on NOMEM evict
      // more, wait, or refuse
      Problem* p = nullptr;
      sfdp_status st;
      for (;;) {
        st = create_problem(ctx, 2, r->n_elem, r->sub_elem, S->prec, &p);
        if (!st) {
          p->gmres_blocks = shared_gmres_blocks(*p, S->kmax, 128);
          if ((st = alloc_workspace(*p, S->kmax)) || (st = alloc_rs(*p))) {
            destroy_problem(p);
            p = nullptr;
          }
        }
        if (st != SFDP_E_NOMEM || !evict_one()) break;
      }
      if (st == SFDP_E_NOMEM && anything_busy()) break;
      if (st) {
        pend.pop_front();
        r->why = std::string("instance allocation failed: ") + g_err + " (" + std::to_string(ctx->used) +
                 " B held, budget " + std::to_string(ctx->budget) + " B)";
        server_finish(S, r, st == SFDP_E_NOMEM ? SFDP_E_ADMIT : st);
        continue;
      }
      reserve += need > p->bytes ? need - p->bytes : 0;
      home = new SInst();
      home->p = p;
      home->n_elem = r->n_elem;
      home->sub_elem = r->sub_elem;
      home->beta = r->beta;
      p->beta = r->beta;
      p->alpha = 1.0 / std::sqrt(r->beta);
      S->insts.push_back(home);
      fresh.push_back(home);
    }
    pend.pop_front();
    r->inst = home;
    home->queue.push_back(r);
    home->last_used = now_ms();
  }
  return fresh;
}

// Rebuild the batch target over the instances with occupied slots (the
// stream must be idle).
sfdp_status server_target(sfdp_server* S, const std::vector<Problem*>& act) {
  if (act != S->active_set) {
    S->M.ctx = S->ctx;
    S->M.probs = act;
    sfdp_status s = multi_maps(S->M);
    if (s) return s;
    S->active_set = act;
  }
  int w = 0;
  for (Problem* p : act) w = std::max(w, p->nr);
  w = w <= 1 ? 1 : w == 2 ? 2 : 4;
  sfdp_status s = multi_groups(S->M, S->kmax, w, S->gmap, S->gcap);
  if (s) return s;
  if (act.size() > S->gath_cap) {
    if (S->hg) hipHostFree(S->hg);
    S->gath_cap = std::max(act.size(), 2 * S->gath_cap);
    if (hipHostMalloc(&S->hg, sizeof(Gathered) * S->gath_cap))
      return fail(SFDP_E_NOMEM, "server gather buffers");
  }
  return SFDP_OK;
}

// One tick: new targets take free slots; every occupied slot gets its KKT
// residual; finished targets leave their slots (and complete their requests);
// the rest take one two-factor refinement step together.
sfdp_status server_tick(sfdp_server* S) {
  hipStream_t st = S->ctx->stream;
  HIPCHK(hipStreamSynchronize(st));
  // fill free slots
  std::vector<Problem*> act;
  std::vector<SInst*> ains;
  for (SInst* in : S->insts) {
    Problem* p = in->p;
    p->init = 0;
    for (int s = 0; s < NRMAX; ++s) {
      SSlot& sl = in->slot[s];
      if (sl.req || in->queue.empty()) continue;
      SReq* r = in->queue.front();
      sl.req = r;
      sl.k = r->next++;
      sl.bad = 0;
      sl.info = blank_info();
      const size_t nf = p->n_free;
      p->sl[s] = Slot{r->ybar + sl.k * nf, r->yc ? r->yc + sl.k * p->n_bdry : nullptr, r->y + sl.k * nf,
                      r->u + sl.k * nf, r->lam + sl.k * nf};
      p->init |= 1u << s;
      if (r->next == r->nrhs) in->queue.pop_front();
    }
    unsigned map = 0;
    int nr = 0;
    for (int s = 0; s < NRMAX; ++s)
      if (in->slot[s].req) map |= (unsigned)s << (8 * nr++);
    p->nr = nr;
    p->map = map;
    if (nr) {
      act.push_back(p);
      ains.push_back(in);
      in->last_used = now_ms();
    }
  }
  if (act.empty()) return SFDP_OK;
  sfdp_status s = server_target(S, act);
  if (s) return s;
  s = multi_upload(S->M);
  if (s) return s;
  const Target& t = S->M.t;
  const size_t n = act.size();
  HIPCHK(launch_group_init(t));  // also clears the new slots' iteration logs
  HIPCHK(launch_kkt_residual(t));
  HIPCHK(launch_gather(t, S->hg));
  HIPCHK(hipStreamSynchronize(st));
  bool any = false;
  for (size_t i = 0; i < n; ++i) {
    SInst* in = ains[i];
    Problem* p = in->p;
    const Gathered& g = S->hg[i];
    if (g.flags[1]) return fail(SFDP_E_DEVICE, "grid barrier timed out");
    unsigned map2 = 0;
    int nb2 = 0;
    for (int c = 0; c < p->nr; ++c) {
      const int q = (p->map >> (8 * c)) & 255;
      SSlot& sl = in->slot[q];
      const double rho = g.red[2 * q];
      const int steps = sl.info.outer_steps;
      sl.info.rel_kkt = rho;
      if (steps == 1) sl.info.rel_kkt_first = rho;
      if (steps > 0) sl.info.imag_ratio = g.red[2 * q + 1];
      bool finished = false;
      if (!std::isfinite(rho)) { sl.bad = 1; finished = true; }
      else if (rho <= S->tol_kkt) finished = true;
      else if (steps >= S->max_outer) { sl.bad = 2; finished = true; }
      if (!finished) {
        map2 |= (unsigned)q << (8 * nb2++);
        continue;
      }
      SReq* r = sl.req;
      sl.info.n_feti = g.flags[FLAG_CNT + q];
      for (int k = 0; k < sl.info.n_feti && k < 16; ++k) {
        sl.info.krylov_its[k] = g.flags[FLAG_LOG + 16 * q + k];
        sl.info.krylov_total += sl.info.krylov_its[k];
      }
      r->info[sl.k] = sl.info;
      if (sl.bad) r->status = SFDP_E_NOCONV;
      if (++r->done == r->nrhs) server_finish(S, r, SFDP_OK);
      sl = SSlot{};
    }
    p->nr = nb2;
    p->map = map2;
    p->init = 0;
    any = any || nb2 > 0;
  }
  ++S->n_ticks;
  if (!any) return SFDP_OK;
  // one refinement step for the slots still running (same instance set; the
  // GMRES groups follow the new widths)
  int w = 0;
  for (Problem* p : act) w = std::max(w, p->nr);
  s = multi_groups(S->M, S->kmax, w <= 1 ? 1 : w == 2 ? 2 : 4, S->gmap, S->gcap);
  if (s) return s;
  s = multi_upload(S->M);
  if (s) return s;
  HIPCHK(launch_make_rhs1(t));
  s = feti_run(t, nullptr, V_CVEC, 0, V_CVEC2, S->tol_inner, S->kmax);
  if (s) return s;
  if (!S->single) {
    HIPCHK(launch_make_rhs2(t));
    s = feti_run(t, nullptr, V_CVEC3, 0, V_CVEC, S->tol_inner, S->kmax);
    if (s) return s;
  }
  HIPCHK(launch_update(t, S->single ? 1 : 0));
  for (size_t i = 0; i < n; ++i)
    for (int c = 0; c < act[i]->nr; ++c) ains[i]->slot[(act[i]->map >> (8 * c)) & 255].info.outer_steps += 1;
  for (Problem* p : act) p->nr = 0;
  return SFDP_OK;
}

// Yield point of a job: hand the turn back to the worker and wait for the next.
void job_yield(void* arg) {
  SJob* j = (SJob*)arg;
  sfdp_server* S = j->S;
  std::unique_lock<std::mutex> lk(S->tmu);
  j->turn = false;
  S->tcv.notify_all();
  S->tcv.wait(lk, [&] { return j->turn; });
}

// One request of the solo lane on its (mesh, beta) problem: a 3D instance
// cannot share the batched 2D launches, and a full-space request runs MINRES
// with the factored Schur complement.  Runs on the job's thread while it holds
// the turn (the set-up in its first turn, then one refinement step or MINRES
// iteration per turn).  On a memory shortage the idle batched instances and
// the idle solo problems are dropped and the set-up is tried once more.
// Returns only device errors; everything else finishes the request.
sfdp_status server_solo(sfdp_server* S, SReq* r, SJob* job) {
  SSolo* home = nullptr;
  for (SSolo* so : S->solos)
    if (!so->busy && so->dim == r->dim && so->n_elem == r->n_elem && so->sub_elem == r->sub_elem &&
        so->beta == r->beta)
      home = so;
  auto drop_lru = [&]() {
    int v = -1;
    for (size_t i = 0; i < S->solos.size(); ++i)
      if (!S->solos[i]->busy && (v < 0 || S->solos[i]->last_used < S->solos[v]->last_used)) v = (int)i;
    if (v < 0) return false;
    destroy_problem(S->solos[v]->p);
    delete S->solos[v];
    S->solos.erase(S->solos.begin() + v);
    return true;
  };
  if (!home) {
    size_t idle = 0;
    for (SSolo* so : S->solos) idle += so->busy ? 0 : 1;
    while (idle >= SOLO_KEEP && drop_lru()) --idle;
    Problem* p = nullptr;
    sfdp_status st = SFDP_OK;
    for (int attempt = 0; attempt < 2; ++attempt) {
      st = create_problem(S->ctx, r->dim, r->n_elem, r->sub_elem, S->prec, &p);
      if (!st) {
        st = sfdp_set_beta((sfdp_problem*)p, r->beta);
        if (st) {
          destroy_problem(p);
          p = nullptr;
        }
      }
      if (st != SFDP_E_NOMEM || attempt) break;
      while (drop_lru()) {
      }
      for (size_t i = 0; i < S->insts.size();) {
        SInst* in = S->insts[i];
        if (in->busy()) {
          ++i;
          continue;
        }
        S->insts.erase(S->insts.begin() + i);
        destroy_problem(in->p);
        delete in;
        ++S->n_evict;
      }
      S->active_set.clear();
    }
    if (st == SFDP_E_DEVICE) return st;
    if (st) {
      r->why = std::string("solo set-up failed: ") + g_err;
      server_finish(S, r, st == SFDP_E_NOMEM ? SFDP_E_ADMIT : st);
      return SFDP_OK;
    }
    ++S->n_setups;
    home = new SSolo{p, r->dim, r->n_elem, r->sub_elem, r->beta, 0.0, false};
    S->solos.push_back(home);
  }
  home->busy = true;
  home->last_used = now_ms();
  sfdp_opts o{};
  o.tol_kkt = S->tol_kkt;
  o.tol_inner = S->tol_inner;
  o.max_outer = S->max_outer;
  o.max_krylov = S->user_kmax;
  o.factors = S->single ? 1 : 2;
  sfdp_problem* sp = (sfdp_problem*)home->p;
  sp->yield_fn = job_yield;
  sp->yield_arg = job;
  sfdp_status st = r->mode == 1
                       ? sfdp_solve_full_space(sp, r->nrhs, r->ybar, r->yc, r->y, r->u, r->lam, &o, r->info.data())
                       : sfdp_solve_range_space(sp, r->nrhs, r->ybar, r->yc, r->y, r->u, r->lam, &o, r->info.data());
  sp->yield_fn = nullptr;
  sp->yield_arg = nullptr;
  home->busy = false;
  home->last_used = now_ms();
  if (st == SFDP_E_DEVICE) return st;
  r->done = r->nrhs;
  if (st) r->why = g_err;
  server_finish(S, r, st);
  return SFDP_OK;
}

void job_main(SJob* j) {
  sfdp_server* S = j->S;
  hipSetDevice(S->ctx->device);
  {
    std::unique_lock<std::mutex> lk(S->tmu);
    S->tcv.wait(lk, [&] { return j->turn; });
  }
  const sfdp_status st = server_solo(S, j->r, j);
  std::lock_guard<std::mutex> lk(S->tmu);
  j->dev = st;
  j->done = true;
  j->turn = false;
  S->tcv.notify_all();
}

// Give every job one turn (in start order) and wait for it to yield or end;
// reap the jobs that ended.  Returns the first device error a job met.
sfdp_status server_turns(sfdp_server* S) {
  sfdp_status dev = SFDP_OK;
  for (SJob* j : S->jobs) {
    std::unique_lock<std::mutex> lk(S->tmu);
    if (j->done) continue;
    j->turn = true;
    S->tcv.notify_all();
    S->tcv.wait(lk, [&] { return !j->turn; });
    if (j->dev && !dev) dev = j->dev;
  }
  for (size_t i = 0; i < S->jobs.size();) {
    SJob* j = S->jobs[i];
    bool done;
    {
      std::lock_guard<std::mutex> lk(S->tmu);
      done = j->done;
    }
    if (!done) {
      ++i;
      continue;
    }
    j->th.join();
    delete j;
    S->jobs.erase(S->jobs.begin() + i);
  }
  return dev;
}

// Start jobs for waiting solo requests while fewer than SOLO_JOBS run, in
// arrival order, one job per (dim, mesh, beta) at a time (a problem serves one
// job at once).
void server_start_jobs(sfdp_server* S) {
  for (auto it = S->solo.begin(); it != S->solo.end() && S->jobs.size() < SOLO_JOBS;) {
    SReq* r = *it;
    bool clash = false;
    for (SJob* j : S->jobs)
      clash = clash || (j->r->dim == r->dim && j->r->n_elem == r->n_elem && j->r->sub_elem == r->sub_elem &&
                        j->r->beta == r->beta);
    if (clash) {
      ++it;
      continue;
    }
    SJob* j = new SJob();
    j->S = S;
    j->r = r;
    j->th = std::thread(job_main, j);
    S->jobs.push_back(j);
    it = S->solo.erase(it);
    std::lock_guard<std::mutex> lk(S->mu);
    S->n_jobs_max = std::max(S->n_jobs_max, (int64_t)S->jobs.size());
  }
}

void server_loop(sfdp_server* S) {
  hipSetDevice(S->ctx->device);
  for (;;) {
    std::deque<SReq*> pend;
    bool work = false;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      for (;;) {
        work = !S->solo.empty() || !S->jobs.empty();
        for (SInst* in : S->insts) work = work || in->busy();
        if (work || !S->pending.empty() || S->stop) break;
        S->cv_work.wait(lk);
      }
      if (S->stop && !work && S->pending.empty()) return;
      pend.swap(S->pending);
    }
    hipStreamSynchronize(S->ctx->stream);
    // 3D and full-space requests take the solo lane, in arrival order
    for (auto it = pend.begin(); it != pend.end();) {
      if ((*it)->dim == 3 || (*it)->mode == 1) {
        S->solo.push_back(*it);
        it = pend.erase(it);
      } else {
        ++it;
      }
    }
    std::vector<SInst*> fresh = server_admit(S, pend);
    sfdp_status st = SFDP_OK;
    if (!fresh.empty()) {
      // set-up passes over consecutive fresh instances whose scratch fits the
      // pool (grown to the pool cap, or to one instance that needs more)
      const size_t lim = std::max(S->pool_cap, S->ctx->pool_bytes);
      for (size_t i = 0; i < fresh.size() && !st;) {
        std::vector<Problem*> ps;
        size_t sum = 0;
        for (; i < fresh.size(); ++i) {
          const size_t b = setup_bytes(fresh[i]->n_elem, fresh[i]->sub_elem);
          if (!ps.empty() && sum + b > lim) break;
          ps.push_back(fresh[i]->p);
          sum += b;
        }
        Multi Mf;
        Mf.ctx = S->ctx;
        Mf.probs = ps;
        st = multi_maps(Mf);
        if (!st) st = setup_run(Mf.t, ps, &Mf);
        if (!st) S->n_setups += (int64_t)ps.size();
      }
      if (st == SFDP_E_NOMEM) {
        // drop the new instances that did not get their factors; their
        // requests wait (or are refused when nothing running could free memory)
        std::vector<SInst*> lost;
        for (SInst* in : fresh)
          if (!in->p->factored) lost.push_back(in);
        bool busy = false;
        for (SInst* in : S->insts)
          if (std::find(lost.begin(), lost.end(), in) == lost.end()) busy = busy || in->busy();
        std::vector<SReq*> back;
        for (SInst* in : lost) {
          for (SReq* r : in->queue) back.push_back(r);
          S->insts.erase(std::find(S->insts.begin(), S->insts.end(), in));
          destroy_problem(in->p);
          delete in;
        }
        S->active_set.clear();
        for (auto it = back.rbegin(); it != back.rend(); ++it) {
          (*it)->inst = nullptr;
          if (busy) {
            pend.push_front(*it);
          } else {
            (*it)->why = std::string("set-up allocation failed: ") + g_err;
            server_finish(S, *it, SFDP_E_ADMIT);
          }
        }
        st = SFDP_OK;
      }
    }
    if (!st) st = server_tick(S);
    // then one turn for every solo request in flight (a refinement step or a
    // MINRES iteration each), so the batched targets and the solo requests
    // advance together
    if (!st) {
      server_start_jobs(S);
      st = server_turns(S);
    }
    std::lock_guard<std::mutex> lk(S->mu);
    // requests that could not be admitted yet go back to the front of the queue
    for (auto it = pend.rbegin(); it != pend.rend(); ++it) S->pending.push_front(*it);
    if (st) {
      // a device error ends the service: fail everything that is not complete
      S->worker_error = g_err;
      for (auto& kv : S->reqs)
        if (!kv.second->complete && std::find(S->finished.begin(), S->finished.end(), kv.second) == S->finished.end())
          server_finish(S, kv.second, st);
      for (SInst* in : S->insts) {
        in->queue.clear();
        for (SSlot& sl : in->slot) sl = SSlot{};
      }
      S->pending.clear();
      S->solo.clear();
      // the jobs in flight end on the failing device: let them run out
      while (!S->jobs.empty()) server_turns(S);
    }
    for (SReq* r : S->finished) {
      r->complete = true;
      if (r->status == SFDP_OK) {
        ++S->n_complete;
        S->lat.push_back(r->t_done - r->t_submit);
      } else {
        ++S->n_failed;
      }
    }
    S->finished.clear();
    S->cv_done.notify_all();
  }
}

}  // namespace

extern "C" {

sfdp_status sfdp_server_create(sfdp_ctx* ctx, sfdp_precision prec, const sfdp_opts* opts, sfdp_server** out) {
  if (!ctx || !out) return fail(SFDP_E_INVALID, "NULL argument");
  if (prec != SFDP_FP64 && prec != SFDP_MIXED && prec != SFDP_MIXED_IFACE) return fail(SFDP_E_INVALID, "bad precision");
  *out = nullptr;
  sfdp_server* S = new (std::nothrow) sfdp_server();
  if (!S) return fail(SFDP_E_NOMEM, "host allocation");
  S->ctx = ctx;
  ctx->children++;
  S->prec = prec;
  defaults(prec, opts, S->tol_kkt, S->tol_inner, S->max_outer, S->kmax);
  S->user_kmax = (opts && opts->max_krylov > 0) ? opts->max_krylov : 0;
  S->single = single_of(opts);
  S->pool_cap = ctx->budget ? ctx->budget / 16 : (size_t)4 << 30;
  S->worker = std::thread(server_loop, S);
  *out = S;
  return SFDP_OK;
}

sfdp_status sfdp_server_submit(sfdp_server* S, const sfdp_request* rq, uint64_t* ticket) {
  if (!S || !rq || !ticket) return fail(SFDP_E_INVALID, "NULL argument");
  if (rq->dim != 2 && rq->dim != 3) return fail(SFDP_E_INVALID, "dim must be 2 or 3");
  if (rq->mode != 0 && rq->mode != 1) return fail(SFDP_E_INVALID, "mode must be 0 (range space) or 1 (full space)");
  if (rq->sub_elem < 2 || rq->sub_elem > (rq->dim == 3 ? 9 : 32) || rq->n_elem % rq->sub_elem != 0 ||
      rq->n_elem / rq->sub_elem < 2)
    return fail(SFDP_E_INVALID, "bad mesh");
  if (rq->mode == 1 && rq->n_elem > 1025) return fail(SFDP_E_INVALID, "the full-space method needs n_elem <= 1025");
  if (!(rq->beta > 0) || !std::isfinite(rq->beta)) return fail(SFDP_E_INVALID, "beta must be positive and finite");
  if (rq->nrhs <= 0 || !rq->ybar || !rq->y || !rq->u || !rq->lam) return fail(SFDP_E_INVALID, "bad arguments");
  SReq* r = new (std::nothrow) SReq();
  if (!r) return fail(SFDP_E_NOMEM, "host allocation");
  r->dim = rq->dim;
  r->mode = rq->mode;
  r->n_elem = rq->n_elem;
  r->sub_elem = rq->sub_elem;
  r->nrhs = rq->nrhs;
  r->beta = rq->beta;
  r->ybar = rq->ybar;
  r->yc = rq->yc;
  r->y = rq->y;
  r->u = rq->u;
  r->lam = rq->lam;
  r->info.assign(rq->nrhs, blank_info());
  r->t_submit = now_ms();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) { delete r; return fail(SFDP_E_STATE, "server is stopping"); }
    r->id = S->next_id++;
    S->reqs[r->id] = r;
    S->pending.push_back(r);
    ++S->n_submit;
  }
  S->cv_work.notify_one();
  *ticket = r->id;
  return SFDP_OK;
}

sfdp_status sfdp_server_poll(sfdp_server* S, uint64_t ticket, int wait, sfdp_info* info, double* latency_ms) {
  if (!S) return fail(SFDP_E_INVALID, "NULL argument");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(SFDP_E_INVALID, "unknown ticket");
  SReq* r = it->second;
  if (!r->complete) {
    if (!wait) return SFDP_E_STATE;
    S->cv_done.wait(lk, [&] { return r->complete; });
  }
  if (info)
    for (int k = 0; k < r->nrhs; ++k) info[k] = r->info[k];
  if (latency_ms) *latency_ms = r->t_done - r->t_submit;
  sfdp_status st = r->status;
  const std::string why = r->why;
  S->reqs.erase(it);
  delete r;
  if (st == SFDP_E_DEVICE) return fail(st, S->worker_error);
  if (st == SFDP_E_ADMIT) return fail(st, why.empty() ? "request can never fit the memory budget" : why);
  if (st == SFDP_E_NOCONV) return fail(st, "a target missed tol_kkt within max_outer steps");
  if (st) return fail(st, why);
  return st;
}

sfdp_status sfdp_server_stats(sfdp_server* S, sfdp_server_info* out) {
  if (!S || !out) return fail(SFDP_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  memset(out, 0, sizeof(*out));
  out->submitted = S->n_submit;
  out->completed = S->n_complete;
  out->failed = S->n_failed;
  out->setups = S->n_setups;
  out->evictions = S->n_evict;
  out->ticks = S->n_ticks;
  out->resident = (int64_t)S->insts.size();
  out->device_bytes = (int64_t)S->ctx->used;
  out->solo_in_flight_max = S->n_jobs_max;
  if (!S->lat.empty()) {
    std::vector<double> v = S->lat;
    std::sort(v.begin(), v.end());
    auto q = [&](double f) { return v[std::min(v.size() - 1, (size_t)std::llround(f * (v.size() - 1)))]; };
    out->p50_ms = q(0.5);
    out->p99_ms = q(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    out->mean_ms = sum / v.size();
  }
  return SFDP_OK;
}

void sfdp_server_destroy(sfdp_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  hipSetDevice(S->ctx->device);
  hipStreamSynchronize(S->ctx->stream);
  for (SInst* in : S->insts) {
    destroy_problem(in->p);
    delete in;
  }
  for (SSolo* so : S->solos) {
    destroy_problem(so->p);
    delete so;
  }
  for (auto& kv : S->reqs) delete kv.second;
  if (S->gmap) hipFree(S->gmap);
  if (S->hg) hipHostFree(S->hg);
  S->ctx->children--;
  delete S;
}

}  // extern "C"

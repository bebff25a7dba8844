// Host side of the sfdp C ABI: partition and interface maps (Sec. 5), setup
// sequencing, the FETI-DP driver and the range-space refinement loop
// (Sec. 3.1 Schur system with the Sec. 4 complex factorization).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "common.h"

namespace sfdp {
}  // namespace sfdp

using namespace sfdp;

static thread_local std::string g_err;

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

struct sfdp_ctx : public Ctx {};
struct sfdp_problem : public Problem {};

namespace {

constexpr int KMAX_LIMIT = 400;
// Device flag words: [1] grid-barrier error, [3] GMRES loop trips, [4] GMRES
// iterations summed over right-hand sides, [8 + r] last counts per RHS, and
// from ITLOG a log of 16 counts per group slot (range-space driver).
constexpr int ITLOG = 64;
constexpr int FLAG_WORDS = ITLOG + NRMAX * 16;

sfdp_status dalloc(Problem& p, void** ptr, size_t bytes) {
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
  if (ptr) {
    hipFree(ptr);
    p.ctx->used -= std::min(p.ctx->used, bytes);
    p.bytes -= std::min(p.bytes, bytes);
  }
  ptr = nullptr;
}

// Build the 2D partition and interface maps on the host.
sfdp_status build_maps(Problem& p) {
  const int N = p.N, m = p.m, P = p.P, ml = p.ml, ND = p.ND, nsub = p.nsub;
  std::vector<int> dloc(nsub * ND, -1), dmid(nsub * ND, 0), dpart(nsub * ND, 0), ndv(nsub, 0);
  std::vector<float> dsgn(nsub * ND, 0.f);
  std::vector<int> cloc(nsub * 4, -1), cgid(nsub * 4, -1);
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
        cgid[s * 4 + nc] = (gi / m - 1) + (P - 1) * (gj / m - 1);
        ++nc;
      } else if (!inter) {
        if (nd >= ND) return fail(SFDP_E_INVALID, "interface slot overflow");
        dloc[s * ND + nd] = l;
        owners[(long)gi + (long)(N + 1) * gj].push_back({s, nd});
        ++nd;
      }
    }
    ndv[s] = nd;
    p.ndmax = std::max(p.ndmax, nd);
  }
  int nmu = 0;
  std::vector<int> muown, mufree;
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
  }
  p.nmu = nmu;
  p.nC = (P - 1) * (P - 1);
  std::vector<int> cown(std::max(p.nC, 1) * 4, -1), cfree(std::max(p.nC, 1), 0), cnt(std::max(p.nC, 1), 0);
  for (int s = 0; s < nsub; ++s)
    for (int q = 0; q < 4; ++q) {
      int c = cgid[s * 4 + q];
      if (c < 0) continue;
      cown[c * 4 + cnt[c]++] = s * 4 + q;
      int l = cloc[s * 4 + q];
      int gi = (s % P) * m + l % ml, gj = (s / P) * m + l / ml;
      cfree[c] = (gi - 1) + (N - 1) * (gj - 1);
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
      (s = dupload(p, &p.cfree, cfree)) || (s = dupload(p, &p.full2bdry, f2b)))
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
  dfree(p, p.Phi, es * p.nsub * p.ND * 4);
  dfree(p, (void*&)p.Kinv, sizeof(cd) * p.nC * p.nC);
  dfree(p, (void*&)p.Kcc, sizeof(cd) * p.nC * p.nC);
  p.factored = false;
}

sfdp_status alloc_workspace(Problem& p, int kmax) {
  if (p.kmax_alloc >= kmax) return SFDP_OK;
  // per right-hand side: Krylov basis, Hessenberg matrix, block partial sums
  if (p.kmax_alloc) {
    dfree(p, (void*&)p.Qk, sizeof(cd) * NRMAX * (size_t)(p.kmax_alloc + 1) * p.nmu);
    dfree(p, (void*&)p.Hk, sizeof(cd) * NRMAX * (size_t)(p.kmax_alloc + 1) * p.kmax_alloc);
    dfree(p, (void*&)p.part, sizeof(cd) * 3 * NRMAX * (size_t)(p.kmax_alloc + 2) * p.gmres_blocks);
  }
  sfdp_status s;
  if ((s = dalloc(p, (void**)&p.Qk, sizeof(cd) * NRMAX * (size_t)(kmax + 1) * p.nmu)) ||
      (s = dalloc(p, (void**)&p.Hk, sizeof(cd) * NRMAX * (size_t)(kmax + 1) * kmax)) ||
      (s = dalloc(p, (void**)&p.part, sizeof(cd) * 3 * NRMAX * (size_t)(kmax + 2) * p.gmres_blocks)))
    return s;
  p.kmax_alloc = kmax;
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
hipError_t ev_begin(Problem& p, int kind, int* slot) {
  *slot = -1;
  if (!p.timing) return hipSuccess;
  if (p.ev_used + 2 > (int)p.ev_pool.size()) {
    for (int i = 0; i < 64; ++i) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      p.ev_pool.push_back(e);
    }
  }
  *slot = p.ev_used;
  p.ev_used += 2;
  p.ev_pending.push_back({*slot, kind});
  return hipEventRecord(p.ev_pool[*slot], p.ctx->stream);
}
hipError_t ev_end(Problem& p, int slot) {
  if (slot < 0) return hipSuccess;
  return hipEventRecord(p.ev_pool[slot + 1], p.ctx->stream);
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

// One FETI-DP solve of Z x_r = f_r (conj_in: conj(Z) x_r = f_r) for nr <= NRMAX
// right-hand sides together; f and x are r-major with stride n_free.  The
// iteration count of RHS r also goes to the device int its_dst[r] (if given).
sfdp_status feti_one(Problem& p, const cd* f, int conj_in, cd* x, double tol, int kmax, int nr,
                     int* const* its_dst) {
  hipStream_t st = p.ctx->stream;
  for (int r = 0; r < NRMAX; ++r) p.its_dst[r] = (its_dst && r < nr) ? its_dst[r] : nullptr;
  int ev;
  HIPCHK(ev_begin(p, 1, &ev));
  HIPCHK(launch_local_solve(p, 0, f, conj_in, nullptr, nr, st));
  HIPCHK(ev_end(p, ev));
  HIPCHK(launch_coarse_rhs(p, f, conj_in, nr, st));
  HIPCHK(launch_fetidp_rhs(p, nr, st));
  sfdp_status s = check_launch(p, kmax);
  if (s != SFDP_OK) return s;
  HIPCHK(ev_begin(p, 0, &ev));
  HIPCHK(launch_gmres(p, tol, kmax, nr, st));
  HIPCHK(ev_end(p, ev));
  HIPCHK(launch_recover_coarse(p, nr, st));
  HIPCHK(ev_begin(p, 1, &ev));
  HIPCHK(launch_local_solve(p, 1, f, conj_in, x, nr, st));
  HIPCHK(ev_end(p, ev));
  HIPCHK(launch_assemble_solution(p, x, conj_in, nr, st));
  return SFDP_OK;
}

void defaults(const Problem& p, const sfdp_opts* o, double& tol_kkt, double& tol_inner, int& max_outer,
              int& kmax) {
  bool mixed = p.prec != SFDP_FP64;
  tol_kkt = (o && o->tol_kkt > 0) ? o->tol_kkt : (mixed ? 1e-8 : 1e-10);
  tol_inner = (o && o->tol_inner > 0) ? o->tol_inner : (mixed ? 1e-7 : 1e-8);
  max_outer = (o && o->max_outer > 0) ? o->max_outer : 8;
  kmax = (o && o->max_krylov > 0) ? std::min(o->max_krylov, KMAX_LIMIT) : 64;
}
int batch_of(const sfdp_opts* o) { return (o && o->batch > 0) ? std::min(o->batch, NRMAX) : NRMAX; }

sfdp_status check_ready(const Problem* p) {
  if (!p) return fail(SFDP_E_INVALID, "null problem");
  if (!p->factored) return fail(SFDP_E_STATE, "sfdp_set_beta has not been called");
  return SFDP_OK;
}

sfdp_status alloc_rs(Problem& p) {
  if (p.r1) return SFDP_OK;
  size_t n = (size_t)NRMAX * p.n_free;
  size_t nred = RED_HEAD + NRMAX * (size_t)red_pstride(p);
  sfdp_status s;
  if ((s = dalloc(p, (void**)&p.r1, sizeof(double) * n)) || (s = dalloc(p, (void**)&p.r2, sizeof(double) * n)) ||
      (s = dalloc(p, (void**)&p.r3, sizeof(double) * n)) || (s = dalloc(p, (void**)&p.red, sizeof(double) * nred)) ||
      (s = dalloc(p, (void**)&p.cvec, sizeof(cd) * n)) || (s = dalloc(p, (void**)&p.cvec2, sizeof(cd) * n)) ||
      (s = dalloc(p, (void**)&p.cvec3, sizeof(cd) * n)))
    return s;
  return SFDP_OK;
}

}  // namespace

extern "C" {

const char* sfdp_last_error(void) { return g_err.c_str(); }

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
  *out = c;
  return SFDP_OK;
}

void sfdp_ctx_destroy(sfdp_ctx* c) { delete c; }

sfdp_status sfdp_problem_create(sfdp_ctx* ctx, int dim, int n_elem, int sub_elem, sfdp_precision prec,
                                sfdp_problem** out) {
  if (!ctx || !out) return fail(SFDP_E_INVALID, "NULL argument");
  *out = nullptr;
  if (dim != 2) return fail(SFDP_E_INVALID, "only dim = 2 is implemented");
  if (sub_elem < 2 || sub_elem > 32) return fail(SFDP_E_INVALID, "sub_elem must be in [2, 32] for dim 2");
  if (n_elem % sub_elem != 0 || n_elem / sub_elem < 2)
    return fail(SFDP_E_INVALID, "n_elem must be a multiple of sub_elem with at least 2 subdomains per side");
  if (prec != SFDP_FP64 && prec != SFDP_MIXED && prec != SFDP_MIXED_IFACE)
    return fail(SFDP_E_INVALID, "bad precision");
  HIPCHK(hipSetDevice(ctx->device));
  sfdp_problem* p = new (std::nothrow) sfdp_problem();
  if (!p) return fail(SFDP_E_NOMEM, "host allocation");
  p->ctx = ctx;
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
  if (s != SFDP_OK) { sfdp_problem_destroy(p); return s; }
  // solve workspaces
  // per right-hand side (NRMAX r-major copies, strides of Problem::rs())
  size_t nsd = (size_t)NRMAX * p->nsub * p->ND;
  size_t n4 = (size_t)NRMAX * p->nsub * 4;
  size_t nC = (size_t)NRMAX * std::max(p->nC, 1);
  size_t nm = (size_t)NRMAX * p->nmu;
  if ((s = dalloc(*p, (void**)&p->Xd, sizeof(cd) * nsd)) || (s = dalloc(*p, (void**)&p->Ubuf, sizeof(cd) * nsd)) ||
      (s = dalloc(*p, (void**)&p->Abuf, sizeof(cd) * nsd)) || (s = dalloc(*p, (void**)&p->Ybuf, sizeof(cd) * nsd)) ||
      (s = dalloc(*p, (void**)&p->Cbuf, sizeof(cd) * n4)) || (s = dalloc(*p, (void**)&p->Qc, sizeof(cd) * n4)) ||
      (s = dalloc(*p, (void**)&p->fcs, sizeof(cd) * nC)) || (s = dalloc(*p, (void**)&p->u0, sizeof(cd) * nC)) ||
      (s = dalloc(*p, (void**)&p->ymin, sizeof(cd) * nC)) || (s = dalloc(*p, (void**)&p->dvec, sizeof(cd) * nm)) ||
      (s = dalloc(*p, (void**)&p->mu, sizeof(cd) * nm)) || (s = dalloc(*p, (void**)&p->wv, sizeof(cd) * nm)) ||
      (s = dalloc(*p, (void**)&p->dscal, sizeof(double) * 8)) || (s = dalloc(*p, (void**)&p->bar, 4096)) ||
      (s = dalloc(*p, (void**)&p->flags, sizeof(int) * FLAG_WORDS))) {
    sfdp_problem_destroy(p);
    return s;
  }
  p->gmres_blocks = std::min(p->nsub, ctx->num_cu);
  hipError_t ez = launch_fill(p->flags, sizeof(int) * FLAG_WORDS, ctx->stream);
  if (ez == hipSuccess) ez = launch_fill(p->bar, 4096, ctx->stream);
  if (ez == hipSuccess) ez = launch_fill(p->dscal, sizeof(double) * 8, ctx->stream);
  if (ez == hipSuccess) ez = hipStreamSynchronize(ctx->stream);
  if (ez != hipSuccess) {
    sfdp_problem_destroy(p);
    return fail(SFDP_E_DEVICE, std::string("init: ") + hipGetErrorString(ez));
  }
  *out = p;
  return SFDP_OK;
}

sfdp_status sfdp_problem_sizes(const sfdp_problem* p, sfdp_sizes* out) {
  if (!p || !out) return fail(SFDP_E_INVALID, "NULL argument");
  out->n_free = p->n_free;
  out->n_bdry = p->n_bdry;
  out->n_sub = p->nsub;
  out->n_mult = p->nmu;
  out->n_corner = p->nC;
  out->max_delta = 4 * (p->m - 1);
  out->resident_bytes = (int64_t)p->bytes;
  return SFDP_OK;
}

void sfdp_problem_destroy(sfdp_problem* p) {
  if (!p) return;
  hipSetDevice(p->ctx->device);
  hipStreamSynchronize(p->ctx->stream);
  free_factors(*p);
  void* arr[] = {p->dloc, p->dmid, p->dpart, p->nd, p->dsgn, p->cloc, p->cgid, p->muown, p->mufree,
                 p->cown, p->cfree, p->full2bdry, p->Xd, p->Ubuf, p->Abuf, p->Ybuf, p->Cbuf, p->Qc,
                 p->fcs, p->u0, p->ymin, p->dvec, p->mu, p->wv, p->Qk, p->Hk, p->part, p->dscal,
                 p->bar, p->flags, p->r1, p->r2, p->r3, p->red, p->cvec, p->cvec2, p->cvec3, p->Kwork};
  for (void* a : arr)
    if (a) hipFree(a);
  for (hipEvent_t e : p->ev_pool) hipEventDestroy(e);
  p->ctx->used -= std::min(p->ctx->used, p->bytes);
  delete p;
}

sfdp_status sfdp_set_beta(sfdp_problem* p, double beta) {
  if (!p) return fail(SFDP_E_INVALID, "null problem");
  if (!(beta > 0) || !std::isfinite(beta)) return fail(SFDP_E_INVALID, "beta must be positive and finite");
  HIPCHK(hipSetDevice(p->ctx->device));
  hipStream_t st = p->ctx->stream;
  free_factors(*p);
  p->beta = beta;
  p->alpha = 1.0 / std::sqrt(beta);
  const int ml = p->ml, ND = p->ND, nsub = p->nsub;
  size_t es = elem_size(*p);
  size_t nG = (size_t)nsub * ml * ml * ml, nS = (size_t)nsub * ND * ND, nP = (size_t)nsub * ND * 4;
  const size_t nPK = (size_t)nsub * ND * (ND + 1) / 2;
  sfdp_status s;
  if ((s = dalloc(*p, &p->G, g_size(*p) * nG)) || (s = dalloc(*p, &p->Sinv, es * nPK)) ||
      (s = dalloc(*p, &p->Sbb, sizeof(cf) * nPK)) || (s = dalloc(*p, &p->Phi, es * nP)) ||
      (s = dalloc(*p, (void**)&p->Kinv, sizeof(cd) * std::max(p->nC * p->nC, 1))) ||
      (s = dalloc(*p, (void**)&p->Kcc, sizeof(cd) * std::max(p->nC * p->nC, 1))))
    return s;
  // FP64 scratch
  cd *G64 = nullptr, *Sinv64 = nullptr, *S64 = nullptr, *Phi64 = nullptr, *PhiFull = nullptr,
     *scr = nullptr, *Kw = nullptr;
  size_t nF = (size_t)nsub * ml * ml * 4, nScr = (size_t)nsub * ml * ml * 32;
  size_t nK = (size_t)std::max(p->nC * p->nC, 1);
  auto cleanup = [&]() {
    hipStreamSynchronize(st);
    hipFree(G64); hipFree(Sinv64); hipFree(S64); hipFree(Phi64); hipFree(PhiFull); hipFree(scr); hipFree(Kw);
  };
  if (hipMalloc(&G64, sizeof(cd) * nG) || hipMalloc(&Sinv64, sizeof(cd) * nS) ||
      hipMalloc(&S64, sizeof(cd) * nS) || hipMalloc(&Phi64, sizeof(cd) * nP) ||
      hipMalloc(&PhiFull, sizeof(cd) * nF) || hipMalloc(&scr, sizeof(cd) * nScr) ||
      hipMalloc(&Kw, sizeof(cd) * nK)) {
    cleanup();
    return fail(SFDP_E_NOMEM, "setup scratch allocation failed");
  }
  hipError_t e = hipSuccess;
  if (!e) e = launch_fill(Sinv64, sizeof(cd) * nS, st);
  if (!e) e = launch_fill(Phi64, sizeof(cd) * nP, st);
  if (!e) e = launch_factor_lines(*p, G64, st);
  if (!e) e = launch_multi_solve(*p, G64, Sinv64, Phi64, PhiFull, scr, st);
  if (!e) e = hipMemcpyAsync(S64, Sinv64, sizeof(cd) * nS, hipMemcpyDeviceToDevice, st);
  if (!e) e = launch_invert_batched(*p, S64, st);
  if (!e && p->nC > 0) e = launch_zcc_and_coarse(*p, PhiFull, p->Kcc, st);
  if (!e && p->nC > 0)
    e = hipMemcpyAsync(p->Kinv, p->Kcc, sizeof(cd) * p->nC * p->nC, hipMemcpyDeviceToDevice, st);
  if (!e && p->nC > 0) e = launch_invert_dense(p->nC, p->Kinv, Kw, st);
  if (!e) e = launch_store_factors(*p, G64, Sinv64, S64, Phi64, st);
  if (!e) e = hipStreamSynchronize(st);
  cleanup();
  if (e) return fail(SFDP_E_DEVICE, std::string("setup: ") + hipGetErrorString(e));
  p->factored = true;
  return SFDP_OK;
}

sfdp_status sfdp_feti_solve(sfdp_problem* p, int conj_z, int nrhs, const double* f, double* x,
                            const sfdp_opts* opts, int* krylov_its) {
  sfdp_status s = check_ready(p);
  if (s) return s;
  if (nrhs <= 0 || !f || !x) return fail(SFDP_E_INVALID, "bad arguments");
  double tk, ti;
  int mo, kmax;
  defaults(*p, opts, tk, ti, mo, kmax);
  const int bsz = batch_of(opts);
  HIPCHK(hipSetDevice(p->ctx->device));
  if ((s = alloc_workspace(*p, kmax))) return s;
  hipStream_t st = p->ctx->stream;
  HIPCHK(launch_fill(p->flags, sizeof(int) * FLAG_WORDS, st));
  std::vector<int> its(nrhs, 0);
  for (int r0 = 0; r0 < nrhs; r0 += bsz) {
    const int nr = std::min(bsz, nrhs - r0);
    const cd* fr = (const cd*)f + (size_t)r0 * p->n_free;
    cd* xr = (cd*)x + (size_t)r0 * p->n_free;
    if ((s = feti_one(*p, fr, conj_z ? 1 : 0, xr, ti, kmax, nr, nullptr))) return s;
    HIPCHK(hipMemcpyAsync(its.data() + r0, p->flags + 8, sizeof(int) * nr, hipMemcpyDeviceToHost, st));
  }
  int flags[8];
  HIPCHK(hipMemcpyAsync(flags, p->flags, sizeof(flags), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (flags[1]) return fail(SFDP_E_DEVICE, "grid barrier timed out");
  HIPCHK(ev_harvest(*p));
  if (p->timing) { p->it_gmres += flags[3]; p->it_rhs += flags[4]; }
  if (krylov_its)
    for (int r = 0; r < nrhs; ++r) krylov_its[r] = its[r];
  return SFDP_OK;
}

sfdp_status sfdp_apply_operator(sfdp_problem* p, char which, int nrhs, const double* x, const double* xc,
                                double* y) {
  if (!p || !x || !y || nrhs <= 0) return fail(SFDP_E_INVALID, "bad arguments");
  HIPCHK(hipSetDevice(p->ctx->device));
  if (which == 'K') HIPCHK(launch_apply_K(*p, nrhs, x, xc, y, p->ctx->stream));
  else if (which == 'M') HIPCHK(launch_apply_M(*p, nrhs, x, y, p->ctx->stream));
  else return fail(SFDP_E_INVALID, "which must be 'K' or 'M'");
  return SFDP_OK;
}

sfdp_status sfdp_kkt_residual(sfdp_problem* p, int nrhs, const double* ybar, const double* yc,
                              const double* y, const double* u, const double* lam, double* rel) {
  if (!p || !ybar || !y || !u || !lam || !rel || nrhs <= 0) return fail(SFDP_E_INVALID, "bad arguments");
  if (!(p->beta > 0)) return fail(SFDP_E_STATE, "beta not set");
  HIPCHK(hipSetDevice(p->ctx->device));
  sfdp_status s = alloc_rs(*p);
  if (s) return s;
  hipStream_t st = p->ctx->stream;
  const size_t n = p->n_free;
  for (int r0 = 0; r0 < nrhs; r0 += NRMAX) {
    const int nr = std::min(NRMAX, nrhs - r0);
    const unsigned map = 0x03020100u;  // slot c for the c-th right-hand side
    double red[2 * NRMAX];
    HIPCHK(launch_kkt_residual(*p, nr, map, ybar + r0 * n, yc ? yc + r0 * p->n_bdry : nullptr, y + r0 * n,
                               u + r0 * n, lam + r0 * n, p->r1, p->r2, p->r3, p->red, st));
    HIPCHK(hipMemcpyAsync(red, p->red, sizeof(red), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int c = 0; c < nr; ++c) rel[r0 + c] = red[2 * c];
  }
  HIPCHK(hipStreamSynchronize(st));
  return SFDP_OK;
}

// Range-space solves of a group of ng <= NRMAX targets (arrays at the group's
// first RHS, stride n_free / n_bdry).  All unfinished members take each
// two-factor step together: both FETI-DP solves of a step run the group's
// active right-hand sides in one launch sequence.
static sfdp_status range_space_group(sfdp_problem* p, int ng, const double* ybar, const double* yc,
                                     double* y, double* u, double* lam, double tol_kkt, double tol_inner,
                                     int max_outer, int kmax, sfdp_info* info) {
  hipStream_t st = p->ctx->stream;
  const int64_t n = p->n_free;
  HIPCHK(launch_copy(ng * n, ybar, y, st));
  HIPCHK(launch_fill(u, sizeof(double) * ng * n, st));
  HIPCHK(launch_fill(lam, sizeof(double) * ng * n, st));
  HIPCHK(launch_fill(p->flags + ITLOG, sizeof(int) * NRMAX * 16, st));
  sfdp_info loc[NRMAX];
  memset(loc, 0, sizeof(loc));
  bool act[NRMAX] = {false, false, false, false};
  int nfeti[NRMAX] = {0, 0, 0, 0};
  std::string why[NRMAX];
  for (int q = 0; q < ng; ++q) act[q] = true;
  double red[2 * NRMAX];
  for (int step = 0;; ++step) {
    unsigned map = 0;
    int na = 0;
    for (int q = 0; q < ng; ++q)
      if (act[q]) map |= (unsigned)q << (8 * na++);
    if (na == 0) break;
    HIPCHK(launch_kkt_residual(*p, na, map, ybar, yc, y, u, lam, p->r1, p->r2, p->r3, p->red, st));
    HIPCHK(hipMemcpyAsync(red, p->red, sizeof(red), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(ev_harvest(*p));
    unsigned map2 = 0;
    int nb2 = 0;
    for (int c = 0; c < na; ++c) {
      const int q = (map >> (8 * c)) & 255;
      const double rho = red[2 * q];
      loc[q].rel_kkt = rho;
      if (step == 1) loc[q].rel_kkt_first = rho;
      if (step > 0) loc[q].imag_ratio = red[2 * q + 1];
      if (!std::isfinite(rho)) { act[q] = false; why[q] = "non-finite residual"; continue; }
      if (rho <= tol_kkt) { act[q] = false; continue; }
      if (step >= max_outer) { act[q] = false; why[q] = "outer refinement limit reached"; continue; }
      map2 |= (unsigned)q << (8 * nb2++);
    }
    if (nb2 == 0) break;
    int* dst[NRMAX];
    auto set_dst = [&]() {
      for (int c = 0; c < nb2; ++c) {
        const int q = (map2 >> (8 * c)) & 255;
        dst[c] = nfeti[q] < 16 ? p->flags + ITLOG + 16 * q + nfeti[q] : nullptr;
        ++nfeti[q];
      }
    };
    HIPCHK(launch_make_rhs1(*p, nb2, map2, p->r1, p->r3, p->cvec, st));
    set_dst();
    sfdp_status s = feti_one(*p, p->cvec, 0, p->cvec2, tol_inner, kmax, nb2, dst);
    if (s) return s;
    HIPCHK(launch_make_rhs2(*p, nb2, map2, p->r1, p->cvec2, p->cvec3, st));
    set_dst();
    s = feti_one(*p, p->cvec3, 0, p->cvec, tol_inner, kmax, nb2, dst);
    if (s) return s;
    HIPCHK(launch_update(*p, nb2, map2, p->cvec2, p->cvec, y, u, lam, p->red, st));
    for (int c = 0; c < nb2; ++c) loc[(map2 >> (8 * c)) & 255].outer_steps = step + 1;
  }
  int flags[FLAG_WORDS];
  HIPCHK(hipMemcpyAsync(flags, p->flags, sizeof(flags), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (flags[1]) return fail(SFDP_E_DEVICE, "grid barrier timed out");
  sfdp_status status = SFDP_OK;
  for (int q = 0; q < ng; ++q) {
    loc[q].n_feti = nfeti[q];
    for (int i = 0; i < nfeti[q] && i < 16; ++i) {
      loc[q].krylov_its[i] = flags[ITLOG + 16 * q + i];
      loc[q].krylov_total += flags[ITLOG + 16 * q + i];
    }
    if (!why[q].empty()) status = fail(SFDP_E_NOCONV, why[q]);
    if (info) info[q] = loc[q];
  }
  return status;
}

sfdp_status sfdp_solve_range_space(sfdp_problem* p, int nrhs, const double* ybar, const double* yc,
                                   double* y, double* u, double* lam, const sfdp_opts* opts,
                                   sfdp_info* info) {
  sfdp_status s = check_ready(p);
  if (s) return s;
  if (nrhs <= 0 || !ybar || !y || !u || !lam) return fail(SFDP_E_INVALID, "bad arguments");
  double tk, ti;
  int mo, kmax;
  defaults(*p, opts, tk, ti, mo, kmax);
  const int bsz = batch_of(opts);
  HIPCHK(hipSetDevice(p->ctx->device));
  if ((s = alloc_workspace(*p, kmax)) || (s = alloc_rs(*p))) return s;
  HIPCHK(launch_fill(p->flags, sizeof(int) * FLAG_WORDS, p->ctx->stream));
  sfdp_status worst = SFDP_OK;
  const size_t n = p->n_free;
  for (int r0 = 0; r0 < nrhs; r0 += bsz) {
    const int ng = std::min(bsz, nrhs - r0);
    s = range_space_group(p, ng, ybar + r0 * n, yc ? yc + r0 * p->n_bdry : nullptr, y + r0 * n,
                          u + r0 * n, lam + r0 * n, tk, ti, mo, kmax, info ? info + r0 : nullptr);
    if (s == SFDP_E_NOCONV) worst = s;
    else if (s) return s;
  }
  if (p->timing) {
    int f[8];
    HIPCHK(hipMemcpy(f, p->flags, sizeof(f), hipMemcpyDeviceToHost));
    p->it_gmres += f[3];
    p->it_rhs += f[4];
  }
  return worst;
}

sfdp_status sfdp_apply_schur_inv(sfdp_problem* p, int nrhs, const double* r, double* z,
                                 const sfdp_opts* opts, sfdp_info* info) {
  sfdp_status s = check_ready(p);
  if (s) return s;
  if (nrhs <= 0 || !r || !z) return fail(SFDP_E_INVALID, "bad arguments");
  double tk, ti;
  int mo, kmax;
  defaults(*p, opts, tk, ti, mo, kmax);
  const int bsz = batch_of(opts);
  HIPCHK(hipSetDevice(p->ctx->device));
  if ((s = alloc_workspace(*p, kmax)) || (s = alloc_rs(*p))) return s;
  hipStream_t st = p->ctx->stream;
  HIPCHK(launch_fill(p->flags, sizeof(int) * FLAG_WORDS, st));
  const int64_t n = p->n_free;
  // the middle factor needs r1 = 0: v = conj(0 + M w)
  HIPCHK(launch_fill(p->r1, sizeof(double) * NRMAX * n, st));
  std::vector<int> its((size_t)2 * nrhs, 0);
  for (int r0 = 0; r0 < nrhs; r0 += bsz) {
    const int nr = std::min(bsz, nrhs - r0);
    const unsigned map = 0x03020100u;
    // factor 1: w = Z^-1 r ; middle: v = conj(M w) ; factor 2: z = Re conj(Z^-1 v) = Re Z^-1 v
    HIPCHK(launch_copy_real_to_complex(nr * n, r + r0 * n, p->cvec, st));
    if ((s = feti_one(*p, p->cvec, 0, p->cvec2, ti, kmax, nr, nullptr))) return s;
    HIPCHK(hipMemcpyAsync(its.data() + 2 * r0, p->flags + 8, sizeof(int) * nr, hipMemcpyDeviceToHost, st));
    HIPCHK(launch_make_rhs2(*p, nr, map, p->r1, p->cvec2, p->cvec3, st));
    if ((s = feti_one(*p, p->cvec3, 0, p->cvec, ti, kmax, nr, nullptr))) return s;
    HIPCHK(hipMemcpyAsync(its.data() + 2 * r0 + nr, p->flags + 8, sizeof(int) * nr, hipMemcpyDeviceToHost,
                          st));
    HIPCHK(launch_real_part(nr * n, p->cvec, z + r0 * n, st));
  }
  int flags[8];
  HIPCHK(hipMemcpyAsync(flags, p->flags, sizeof(flags), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (flags[1]) return fail(SFDP_E_DEVICE, "grid barrier timed out");
  HIPCHK(ev_harvest(*p));
  if (p->timing) { p->it_gmres += flags[3]; p->it_rhs += flags[4]; }
  if (info) {
    // its holds, per group of nr, the nr factor-1 counts then the nr factor-2 counts
    for (int r0 = 0; r0 < nrhs; r0 += bsz) {
      const int nr = std::min(bsz, nrhs - r0);
      for (int c = 0; c < nr; ++c) {
        sfdp_info& o = info[r0 + c];
        memset(&o, 0, sizeof(o));
        o.n_feti = 2;
        o.krylov_its[0] = its[2 * r0 + c];
        o.krylov_its[1] = its[2 * r0 + nr + c];
        o.krylov_total = o.krylov_its[0] + o.krylov_its[1];
      }
    }
  }
  return SFDP_OK;
}

sfdp_status sfdp_inspect(sfdp_problem* p, sfdp_query what, int sub, double* out, int* rows, int* cols) {
  sfdp_status s = check_ready(p);
  if (s) return s;
  HIPCHK(hipSetDevice(p->ctx->device));
  std::vector<int> ndv(p->nsub), cl(4 * p->nsub);
  HIPCHK(hipMemcpy(ndv.data(), p->nd, sizeof(int) * p->nsub, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(cl.data(), p->cloc, sizeof(int) * 4 * p->nsub, hipMemcpyDeviceToHost));
  int r = 0, c = 0;
  if (what == SFDP_Q_COARSE) {
    r = c = p->nC;
  } else {
    if (sub < 0 || sub >= p->nsub) return fail(SFDP_E_INVALID, "sub out of range");
    r = ndv[sub];
    if (what == SFDP_Q_PHI) {
      c = 0;
      for (int q = 0; q < 4; ++q) c += cl[4 * sub + q] >= 0;
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
  if (what == SFDP_Q_COARSE) {
    HIPCHK(hipMemcpy(host.data(), p->Kcc, sizeof(cd) * host.size(), hipMemcpyDeviceToHost));
  } else if (what == SFDP_Q_PHI) {
    size_t es = elem_size(*p);
    std::vector<char> raw((size_t)p->ND * 4 * es);
    HIPCHK(hipMemcpy(raw.data(), (const char*)p->Phi + (size_t)sub * p->ND * 4 * es, raw.size(),
                     hipMemcpyDeviceToHost));
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < c; ++j) {
        size_t idx = (size_t)i * 4 + j;
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

sfdp_status sfdp_timing_enable(sfdp_problem* p, int enable) {
  if (!p) return fail(SFDP_E_INVALID, "null problem");
  HIPCHK(hipSetDevice(p->ctx->device));
  HIPCHK(hipStreamSynchronize(p->ctx->stream));
  p->ev_pending.clear();
  p->ev_used = 0;
  p->timing = enable != 0;
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
  if (which == 'D') {
    const cd* f = (const cd*)x;
    HIPCHK(launch_local_solve(*p, 0, f, 0, nullptr, 1, st));
    HIPCHK(launch_coarse_rhs(*p, f, 0, 1, st));
    HIPCHK(launch_fetidp_rhs(*p, 1, st));
    HIPCHK(hipMemcpyAsync(y, p->dvec, sizeof(cd) * p->nmu, hipMemcpyDeviceToDevice, st));
    return SFDP_OK;
  }
  if (which != 'F' && which != 'P') return fail(SFDP_E_INVALID, "which must be 'F', 'P' or 'D'");
  HIPCHK(launch_interface_apply(*p, which, (const cd*)x, (cd*)y, st));
  return SFDP_OK;
}

}  // extern "C"

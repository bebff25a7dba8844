// Host side of the linear-elasticity instances (Sec. 6.2 cantilever control):
// the element matrices, the partition and interface maps, the CSR operators,
// the load of the target's forward simulation, and the set-up, FETI-DP,
// range-space and forward-solve drivers behind the C ABI.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "elastic.h"

namespace sfdp {

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

#define ELCHK(call)                                                                        \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return host_fail(SFDP_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

using List = std::vector<std::pair<void*, size_t>>;

template <class T>
sfdp_status take(Problem& p, List& list, T** ptr, size_t count) {
  const size_t bytes = sizeof(T) * std::max<size_t>(count, 1);
  sfdp_status s = dev_alloc(p, (void**)ptr, bytes);
  if (s) return s;
  list.push_back({(void*)*ptr, bytes});
  return SFDP_OK;
}
template <class T>
sfdp_status upload(Problem& p, List& list, T** ptr, const std::vector<T>& v) {
  sfdp_status s = take(p, list, ptr, v.size());
  if (s) return s;
  if (!v.empty()) ELCHK(hipMemcpy(*ptr, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  return SFDP_OK;
}
void release(Problem& p, List& list) {
  for (auto& a : list) dev_free(p, a.first, a.second);
  list.clear();
}

// Element matrices of a cube cell of side h in closed form (trilinear shape
// functions N_v = phi_a(x) phi_b(y) phi_c(z), vertex v = a + 2 b + 4 c): the
// integrals of products of shape functions and their derivatives factor into
// 1D integrals on [0, h]:
//   int phi_i phi_j = h (1 + [i = j]) / 6,  int phi_i' phi_j' = (2 [i = j] - 1) / h,
//   int phi_i' phi_j = (2 i - 1) / 2.
// Stiffness of isotropic linear elasticity between N_v1 e_c1 and N_v2 e_c2
// (the energy lambda div u div w + 2 mu eps(u) : eps(w)):
//   lambda I(c1, c2) + mu I(c2, c1) + mu [c1 = c2] sum_d I(d, d),
//   I(d1, d2) = int d_{d1} N_v1 d_{d2} N_v2.
// Out: [24][24] stiffness (dof 3 v + c), then the [8][8] scalar mass.
std::vector<double> element_matrices(double h, double young, double poisson) {
  const double lam = young * poisson / ((1.0 + poisson) * (1.0 - 2.0 * poisson));
  const double mu = young / (2.0 * (1.0 + poisson));
  auto m1 = [&](int i, int j) { return h * (i == j ? 2.0 : 1.0) / 6.0; };
  auto k1 = [&](int i, int j) { return (i == j ? 1.0 : -1.0) / h; };
  auto g1 = [&](int i) { return i ? 0.5 : -0.5; };  // int phi_i' phi_j, any j
  auto I = [&](int d1, int d2, int v1, int v2) {
    double r = 1.0;
    for (int d = 0; d < 3; ++d) {
      const int i = (v1 >> d) & 1, j = (v2 >> d) & 1;
      if (d == d1 && d == d2) r *= k1(i, j);
      else if (d == d1) r *= g1(i);
      else if (d == d2) r *= g1(j);
      else r *= m1(i, j);
    }
    return r;
  };
  std::vector<double> KM(24 * 24 + 64, 0.0);
  for (int v1 = 0; v1 < 8; ++v1)
    for (int v2 = 0; v2 < 8; ++v2) {
      const double lap = I(0, 0, v1, v2) + I(1, 1, v1, v2) + I(2, 2, v1, v2);
      for (int c1 = 0; c1 < 3; ++c1)
        for (int c2 = 0; c2 < 3; ++c2)
          KM[(3 * v1 + c1) * 24 + 3 * v2 + c2] =
              lam * I(c1, c2, v1, v2) + mu * I(c2, c1, v1, v2) + (c1 == c2 ? mu * lap : 0.0);
      double mm = 1.0;
      for (int d = 0; d < 3; ++d) mm *= m1((v1 >> d) & 1, (v2 >> d) & 1);
      KM[576 + v1 * 8 + v2] = mm;
    }
  return KM;
}

struct Grid {
  int nx, ny, nz;
  int64_t node(int i, int j, int k) const { return i + (int64_t)(nx + 1) * (j + (int64_t)(ny + 1) * k); }
  // free node of an unclamped grid node (i >= 1)
  int64_t free_node(int i, int j, int k) const { return (i - 1) + (int64_t)nx * (j + (int64_t)(ny + 1) * k); }
};

// subdomains sharing a coordinate v on an axis of `top` cells cut every m cells
int share(int v, int m, int top) { return (v % m == 0 && v > 0 && v < top) ? 2 : 1; }

}  // namespace

// ----------------------------------------------------------------- maps --

sfdp_status el_build(Problem& p, int n, int m, int length, double young, double poisson) {
  Elastic& el = *p.el;
  GeoE& g = el.g;
  el.young = young;
  el.poisson = poisson;
  g.n = n;
  g.m = m;
  g.ml = m + 1;
  g.L = length;
  g.nx = length * n;
  g.ny = g.nz = n;
  g.Px = g.nx / m;
  g.Py = g.ny / m;
  g.Pz = g.nz / m;
  g.nsub = g.Px * g.Py * g.Pz;
  g.alpha = 0.0;
  g.rshift = 0;
  const Grid G{g.nx, g.ny, g.nz};
  g.n_free = 3 * (int64_t)g.nx * (g.ny + 1) * (g.nz + 1);
  if (g.n_free > INT32_MAX / 2) return host_fail(SFDP_E_INVALID, "mesh too large");
  const int ml = g.ml, nl = ml * ml * ml, nsub = g.nsub;
  // classify the local nodes of every subdomain
  std::vector<int> ni(nsub), nds(nsub);
  std::vector<std::vector<int>> loc_nodes(nsub), del_nodes(nsub);
  auto coords = [&](int s, int l, int& gi, int& gj, int& gk) {
    const int sx = s % g.Px, sy = (s / g.Px) % g.Py, sz = s / (g.Px * g.Py);
    gi = sx * m + l % ml;
    gj = sy * m + (l / ml) % ml;
    gk = sz * m + l / (ml * ml);
  };
  auto is_vertex = [&](int l) {
    const int a = l % ml, b = (l / ml) % ml, c = l / (ml * ml);
    return (a == 0 || a == m) && (b == 0 || b == m) && (c == 0 || c == m);
  };
  int NR = 0, ND = 0;
  for (int s = 0; s < nsub; ++s) {
    for (int l = 0; l < nl; ++l) {
      int gi, gj, gk;
      coords(s, l, gi, gj, gk);
      if (gi == 0 || is_vertex(l)) continue;
      const int mult = share(gi, m, g.nx) * share(gj, m, g.ny) * share(gk, m, g.nz);
      (mult >= 2 ? del_nodes[s] : loc_nodes[s]).push_back(l);
    }
    ni[s] = 3 * (int)loc_nodes[s].size();
    nds[s] = 3 * (int)del_nodes[s].size();
    NR = std::max(NR, ni[s] + nds[s]);
    ND = std::max(ND, nds[s]);
  }
  g.NR = NR;
  g.ND = ND;
  std::vector<int> rdof((size_t)nsub * NR, -1), rfree((size_t)nsub * NR, -1);
  std::vector<float> rw((size_t)nsub * NR, 0.f), dw((size_t)nsub * ND, 0.f);
  struct Inc {
    int64_t fdof;
    int s, d;
    float w;
  };
  std::vector<Inc> inc;
  std::vector<int> fcor(g.n_free, -1), fown((size_t)g.n_free * 4, -1), fcnt(g.n_free, 0);
  for (int s = 0; s < nsub; ++s) {
    int p = 0;
    for (int part = 0; part < 2; ++part)
      for (int l : part == 0 ? loc_nodes[s] : del_nodes[s]) {
        int gi, gj, gk;
        coords(s, l, gi, gj, gk);
        const int mult = share(gi, m, g.nx) * share(gj, m, g.ny) * share(gk, m, g.nz);
        const int64_t f = G.free_node(gi, gj, gk);
        for (int c = 0; c < 3; ++c, ++p) {
          const size_t at = (size_t)s * NR + p;
          rdof[at] = 3 * l + c;
          rfree[at] = (int)(3 * f + c);
          rw[at] = 1.0f / mult;
          if (part == 1) {
            const int d = p - ni[s];
            dw[(size_t)s * ND + d] = 1.0f / mult;
            inc.push_back({3 * f + c, s, d, 1.0f / mult});
          }
          const int64_t t = 3 * f + c;
          if (fcnt[t] >= 4) return host_fail(SFDP_E_INVALID, "more than four copies of a dof");
          fown[(size_t)t * 4 + fcnt[t]++] = s * NR + p;
        }
      }
  }
  // corners: the three dofs of every unclamped subdomain vertex
  g.nC = 3 * g.Px * (g.Py + 1) * (g.Pz + 1);
  std::vector<int> cdof((size_t)nsub * EQ, -1), cg((size_t)nsub * EQ, -1), cown((size_t)g.nC * 8, -1),
      ccnt(g.nC, 0), cfree(g.nC, -1);
  for (int s = 0; s < nsub; ++s)
    for (int v = 0; v < 8; ++v) {
      const int l = (v & 1) * m + ml * (((v >> 1) & 1) * m) + ml * ml * (((v >> 2) & 1) * m);
      int gi, gj, gk;
      coords(s, l, gi, gj, gk);
      if (gi == 0) continue;
      const int cn = (gi / m - 1) + g.Px * (gj / m + (g.Py + 1) * (gk / m));
      const int64_t f = G.free_node(gi, gj, gk);
      for (int c = 0; c < 3; ++c) {
        const int q = 3 * v + c, id = 3 * cn + c;
        cdof[s * EQ + q] = 3 * l + c;
        cg[s * EQ + q] = id;
        if (ccnt[id] >= 8) return host_fail(SFDP_E_INVALID, "more than eight owners of a corner");
        cown[(size_t)id * 8 + ccnt[id]++] = s * EQ + q;
        cfree[id] = (int)(3 * f + c);
        fcor[3 * f + c] = id;
      }
    }
  std::vector<float> cw(g.nC);
  for (int c = 0; c < g.nC; ++c) {
    if (ccnt[c] == 0) return host_fail(SFDP_E_INVALID, "corner without owner");
    cw[c] = 1.0f / ccnt[c];
  }
  for (int64_t t = 0; t < g.n_free; ++t)
    if (fcor[t] < 0 && fcnt[t] == 0) return host_fail(SFDP_E_INVALID, "dof without subdomain");
  // fully redundant multipliers: by free dof, then by pair (s_a < s_b), +1 on s_a
  std::stable_sort(inc.begin(), inc.end(),
                   [](const Inc& a, const Inc& b) { return a.fdof != b.fdof ? a.fdof < b.fdof : a.s < b.s; });
  std::vector<int> dmu((size_t)nsub * ND * 3, -1), muown;
  std::vector<float> dsg((size_t)nsub * ND * 3, 0.f), muw;
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
    while (i1 < inc.size() && inc[i1].fdof == inc[i0].fdof) ++i1;
    for (size_t a = i0; a < i1; ++a)
      for (size_t b = a + 1; b < i1; ++b) {
        const int k = (int)muw.size();
        muown.push_back(inc[a].s * ND + inc[a].d);
        muown.push_back(inc[b].s * ND + inc[b].d);
        muw.push_back(inc[a].w);
        if (!add(inc[a].s, inc[a].d, k, 1.f) || !add(inc[b].s, inc[b].d, k, -1.f))
          return host_fail(SFDP_E_INVALID, "more than three multipliers on a dof");
      }
    i0 = i1;
  }
  g.nmu = (int)muw.size();
  // CSR of K and M over the free dofs: row (node, c1), columns the neighbour
  // nodes' dofs in increasing free-dof order, entries summed over the shared
  // elements
  const std::vector<double> KM = element_matrices(1.0 / n, young, poisson);
  std::vector<int> rp(g.n_free + 1, 0), ci;
  std::vector<double> kv, mv;
  ci.reserve((size_t)g.n_free * 81);
  kv.reserve((size_t)g.n_free * 81);
  mv.reserve((size_t)g.n_free * 81);
  for (int k = 0; k <= g.nz; ++k)
    for (int j = 0; j <= g.ny; ++j)
      for (int i = 1; i <= g.nx; ++i)
        for (int c1 = 0; c1 < 3; ++c1) {
          const int64_t row = 3 * G.free_node(i, j, k) + c1;
          for (int dk = -1; dk <= 1; ++dk)
            for (int dj = -1; dj <= 1; ++dj)
              for (int di = -1; di <= 1; ++di) {
                const int i2 = i + di, j2 = j + dj, k2 = k + dk;
                if (i2 < 1 || i2 > g.nx || j2 < 0 || j2 > g.ny || k2 < 0 || k2 > g.nz) continue;
                for (int c2 = 0; c2 < 3; ++c2) {
                  double kk = 0.0, mm = 0.0;
                  for (int ek = std::max(std::max(k, k2) - 1, 0); ek <= std::min(std::min(k, k2), g.nz - 1); ++ek)
                    for (int ej = std::max(std::max(j, j2) - 1, 0); ej <= std::min(std::min(j, j2), g.ny - 1); ++ej)
                      for (int ei = std::max(std::max(i, i2) - 1, 0); ei <= std::min(std::min(i, i2), g.nx - 1);
                           ++ei) {
                        const int v1 = (i - ei) + 2 * (j - ej) + 4 * (k - ek);
                        const int v2 = (i2 - ei) + 2 * (j2 - ej) + 4 * (k2 - ek);
                        kk += KM[(3 * v1 + c1) * 24 + 3 * v2 + c2];
                        if (c1 == c2) mm += KM[576 + v1 * 8 + v2];
                      }
                  ci.push_back((int)(3 * G.free_node(i2, j2, k2) + c2));
                  kv.push_back(kk);
                  mv.push_back(mm);
                }
              }
          rp[row + 1] = (int)ci.size();
        }
  el.nnz = (int64_t)ci.size();
  el.h_ni = ni;
  el.h_nds = nds;
  el.h_rdof = rdof;
  el.h_cg = cg;
  sfdp_status s;
  List& o = el.owned;
  if ((s = upload(p, o, &el.rdof, rdof)) || (s = upload(p, o, &el.rfree, rfree)) || (s = upload(p, o, &el.rw, rw)) ||
      (s = upload(p, o, &el.ni, ni)) || (s = upload(p, o, &el.nds, nds)) || (s = upload(p, o, &el.dw, dw)) ||
      (s = upload(p, o, &el.dmu, dmu)) || (s = upload(p, o, &el.dsg, dsg)) || (s = upload(p, o, &el.muown, muown)) ||
      (s = upload(p, o, &el.muw, muw)) || (s = upload(p, o, &el.cdof, cdof)) || (s = upload(p, o, &el.cg, cg)) ||
      (s = upload(p, o, &el.cown, cown)) || (s = upload(p, o, &el.cw, cw)) || (s = upload(p, o, &el.cfree, cfree)) ||
      (s = upload(p, o, &el.fcor, fcor)) || (s = upload(p, o, &el.fown, fown)) || (s = upload(p, o, &el.Ke, KM)) ||
      (s = upload(p, o, &el.rp, rp)) || (s = upload(p, o, &el.ci, ci)) || (s = upload(p, o, &el.Kv, kv)) ||
      (s = upload(p, o, &el.Mv, mv)))
    return s;
  p.nsub = nsub;
  p.nmu = g.nmu;
  p.nC = g.nC;
  p.nK = g.nC;
  p.nE = 0;
  p.ND = ND;
  p.ndmax = ND;
  p.n_free = g.n_free;
  p.n_bdry = 0;
  return SFDP_OK;
}

namespace {

void free_twin(Problem& p, Elastic& el) {
  if (!el.fwd) return;
  release(p, el.fwd->owned);
  delete el.fwd;
  el.fwd = nullptr;
}

void free_krylov(Problem& p, Elastic& el) {
  release(p, el.kowned);
  if (el.kb.gih) hipHostFree(el.kb.gih);
  el.kb = KBuf{};
}

}  // namespace

void el_destroy(Problem& p) {
  Elastic* el = p.el;
  if (!el) return;
  free_twin(p, *el);
  free_krylov(p, *el);
  if (el->sumh) hipHostFree(el->sumh);
  el->sumh = nullptr;
  release(p, el->owned);
  delete el;
  p.el = nullptr;
}

// ---------------------------------------------------------------- set-up --

namespace {

size_t el_es(bool s32) { return s32 ? sizeof(cf) : sizeof(cd); }

// factors of el (allocated once, reused by every set-up)
sfdp_status alloc_factors(Problem& p, Elastic& el, bool s32) {
  if (el.Zinv) return SFDP_OK;
  const GeoE& g = el.g;
  const size_t es = el_es(s32), ns = g.nsub, nc2 = (size_t)std::max(g.nC, 1) * std::max(g.nC, 1);
  List& o = el.owned;
  sfdp_status s;
  char *zi = nullptr, *si = nullptr, *sb = nullptr, *ph = nullptr;
  if ((s = take(p, o, &zi, es * ns * g.NR * g.NR)) || (s = take(p, o, &si, es * ns * g.ND * g.ND)) ||
      (s = take(p, o, &sb, es * ns * g.ND * g.ND)) || (s = take(p, o, &ph, es * ns * g.ND * EQ)) ||
      (s = take(p, o, &el.PhiFull, ns * g.NR * EQ)) || (s = take(p, o, &el.Zrc, ns * g.NR * EQ)) ||
      (s = take(p, o, &el.Zcc, ns * EQ * EQ)) || (s = take(p, o, &el.Kcc, nc2)) || (s = take(p, o, &el.Kinv, nc2)))
    return s;
  el.Zinv = zi;
  el.Sinv = si;
  el.Sbb = sb;
  el.Phi = ph;
  return SFDP_OK;
}

sfdp_status setup_factors(Problem& p, Elastic& el, bool s32) {
  sfdp_status s = alloc_factors(p, el, s32);
  if (s) return s;
  const GeoE& g = el.g;
  const size_t eb = sizeof(cd) * (size_t)g.nsub * g.NR * g.NR, e2b = sizeof(cd) * (size_t)g.nsub * g.ND * g.ND,
               wb = sizeof(cd) * (size_t)g.nsub * 2 * 32 * 32;
  void *E = nullptr, *E2 = nullptr, *W = nullptr;
  if ((s = dev_alloc(p, &E, eb)) || (s = dev_alloc(p, &E2, e2b)) || (s = dev_alloc(p, &W, wb))) {
    dev_free(p, E, eb);
    dev_free(p, E2, e2b);
    return s;
  }
  hipStream_t st = p.ctx->stream;
  hipError_t e = el_launch_setup(el, s32, el.Kcc, el.Kinv, (cd*)E, (cd*)E2, (cd*)W, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  dev_free(p, E, eb);
  dev_free(p, E2, e2b);
  dev_free(p, W, wb);
  if (e != hipSuccess) return host_fail(SFDP_E_DEVICE, std::string("elastic setup: ") + hipGetErrorString(e));
  return SFDP_OK;
}

}  // namespace

sfdp_status el_setup(Problem& p) {
  Elastic& el = *p.el;
  el.g.alpha = p.alpha;
  el.g.rshift = p.rshift ? 1 : 0;
  p.factored = false;
  const double t0 = now_ms();
  sfdp_status s = setup_factors(p, el, p.s32());
  if (s) return s;
  p.t_setup_ms = now_ms() - t0;
  p.factored = true;
  return SFDP_OK;
}

// ------------------------------------------------------------ workspaces --

namespace {

constexpr int EL_KMAX_DEFAULT = 300;
constexpr int EL_KMAX_LIMIT = 400;

// FETI-DP workspaces (NRMAX copies) and the Krylov buffers for kmax iterations
sfdp_status ensure_ws(Problem& p, Elastic& el, int kmax) {
  const GeoE& g = el.g;
  const size_t R = NRMAX;
  sfdp_status s;
  if (!el.T) {
    List& o = el.owned;
    const size_t nc = std::max(g.nC, 1);
    if ((s = take(p, o, &el.T, R * g.nsub * g.NR)) || (s = take(p, o, &el.Y, R * g.nsub * g.ND)) ||
        (s = take(p, o, &el.Wc, R * g.nsub * EQ)) || (s = take(p, o, &el.fcs, R * nc)) ||
        (s = take(p, o, &el.uc, R * nc)) || (s = take(p, o, &el.gc, R * nc)))
      return s;
  }
  if (el.kb.kalloc >= kmax) return SFDP_OK;
  free_krylov(p, el);
  const size_t nm = std::max(g.nmu, 1), nb = (nm + 255) / 256, kk = kmax + 1;
  KBuf& kb = el.kb;
  List& o = el.kowned;
  if ((s = take(p, o, &kb.V, R * kk * nm)) || (s = take(p, o, &kb.part, R * kk * 4 * nb)) ||
      (s = take(p, o, &kb.hd, R * (2 * kk + 1))) || (s = take(p, o, &kb.d, R * nm)) ||
      (s = take(p, o, &kb.z, R * nm)) || (s = take(p, o, &kb.w, R * nm)) || (s = take(p, o, &kb.mu, R * nm)) ||
      (s = take(p, o, &kb.npart, R * nb)) || (s = take(p, o, &kb.nvd, R)) ||
      (s = take(p, o, &kb.gs, R * gs_len(kmax))) || (s = take(p, o, &kb.gi, (size_t)GI_WORDS)))
    return s;
  if (hipHostMalloc((void**)&kb.gih, sizeof(int) * GI_WORDS) != hipSuccess) {
    kb.gih = nullptr;
    return host_fail(SFDP_E_NOMEM, "pinned host allocation");
  }
  kb.kalloc = kmax;
  return SFDP_OK;
}

// range-space vectors (NRMAX copies) and the partial-sum buffers
sfdp_status ensure_rs(Problem& p, Elastic& el) {
  if (el.r1) return SFDP_OK;
  const size_t R = NRMAX, n = el.g.n_free, nb = (n + 15) / 16;  // workgroups of the KKT kernel (16 rows each)
  List& o = el.owned;
  sfdp_status s;
  if ((s = take(p, o, &el.r1, R * n)) || (s = take(p, o, &el.r3, R * n)) || (s = take(p, o, &el.c1, R * n)) ||
      (s = take(p, o, &el.c2, R * n)) || (s = take(p, o, &el.c3, R * n)) ||
      (s = take(p, o, &el.part, R * nb * EL_SUMS)) || (s = take(p, o, &el.sums, 2 * R * EL_SUMS)))
    return s;
  if (hipHostMalloc((void**)&el.sumh, sizeof(double) * 2 * R * EL_SUMS) != hipSuccess) {
    el.sumh = nullptr;
    return host_fail(SFDP_E_NOMEM, "pinned host allocation");
  }
  return SFDP_OK;
}

struct Ctl {
  double tol_kkt, tol_inner, tol_first;
  int max_outer, kmax, batch;
  bool single;
};

// Defaults of the elasticity drivers.  The stopping test is on the blockwise
// backward error (eta_blk): the KKT right-hand side (M ybar, 0, 0) is some
// eps E / h^2 smaller than the stiffness terms of the residual, so even the
// exact solution's relative KKT residual sits near 1e-7 at these meshes.
Ctl controls(const Problem& p, const sfdp_opts* o) {
  Ctl c;
  const bool mixed = p.prec != SFDP_FP64;
  c.tol_kkt = (o && o->tol_kkt > 0) ? o->tol_kkt : (mixed ? 1e-10 : 1e-12);
  c.tol_inner = (o && o->tol_inner > 0) ? o->tol_inner : (mixed ? 3e-7 : 1e-8);
  c.tol_first = (o && o->tol_inner_first > 0) ? o->tol_inner_first : c.tol_inner;
  c.max_outer = (o && o->max_outer > 0) ? o->max_outer : 8;
  c.kmax = (o && o->max_krylov > 0) ? std::min(o->max_krylov, EL_KMAX_LIMIT) : EL_KMAX_DEFAULT;
  c.batch = (o && o->batch > 0) ? std::min(o->batch, NRMAX) : NRMAX;
  c.single = o && o->factors == 1;
  return c;
}

sfdp_status check_factored(const Problem& p) {
  if (!p.factored) return host_fail(SFDP_E_STATE, "sfdp_set_beta has not been called");
  return SFDP_OK;
}

// One group of FETI-DP solves (nr <= NRMAX right-hand sides of stride n_free).
sfdp_status feti_group(Problem& p, Elastic& el, bool s32, int nr, const cd* f, cd* x, int conj, double tol,
                       int kmax, int* its) {
  hipError_t e = el_launch_feti(el, s32, el.Kinv, nr, f, x, conj, tol, kmax, its, p.ctx->stream);
  if (e != hipSuccess) return host_fail(SFDP_E_DEVICE, std::string("elastic FETI-DP: ") + hipGetErrorString(e));
  return SFDP_OK;
}

}  // namespace

// ------------------------------------------------------------- FETI-DP --

sfdp_status el_feti(Problem& p, int conj, int nrhs, const cd* f, cd* x, const sfdp_opts* o, int* its) {
  sfdp_status s = check_factored(p);
  if (s) return s;
  Elastic& el = *p.el;
  const Ctl c = controls(p, o);
  if ((s = ensure_ws(p, el, c.kmax))) return s;
  const int64_t n = el.g.n_free;
  int loc[NRMAX];
  for (int r0 = 0; r0 < nrhs; r0 += c.batch) {
    const int nr = std::min(c.batch, nrhs - r0);
    if ((s = feti_group(p, el, p.s32(), nr, f + r0 * n, x + r0 * n, conj, c.tol_inner, c.kmax, loc))) return s;
    if (its)
      for (int r = 0; r < nr; ++r) its[r0 + r] = loc[r];
  }
  ELCHK(hipStreamSynchronize(p.ctx->stream));
  return SFDP_OK;
}

sfdp_status el_interface(Problem& p, char which, const cd* x, cd* y) {
  sfdp_status s = check_factored(p);
  if (s) return s;
  Elastic& el = *p.el;
  if ((s = ensure_ws(p, el, 1))) return s;
  ELCHK(el_launch_interface(el, p.s32(), el.Kinv, which, x, y, p.ctx->stream));
  ELCHK(hipStreamSynchronize(p.ctx->stream));
  return SFDP_OK;
}

// --------------------------------------------------- KKT and range space --

namespace {

struct Metrics {
  double rel, eta, viol;
};

// rel = ||r|| / ||M ybar||, eta = blockwise backward error, viol = ||K y - M u|| / ||K y||
Metrics metrics(const double* s, double beta) {
  double nrm[EL_SUMS];
  for (int e = 0; e < EL_SUMS; ++e) nrm[e] = std::sqrt(s[e]);
  Metrics m;
  const double rn = std::sqrt(s[0] + s[1] + s[2]);
  m.rel = nrm[6] > 0.0 ? rn / nrm[6] : rn;
  m.viol = nrm[3] > 0.0 ? nrm[2] / nrm[3] : nrm[2];
  const double den[3] = {nrm[4] + nrm[5] + nrm[6], beta * nrm[7] + nrm[8], nrm[9] + nrm[7]};
  m.eta = 0.0;
  for (int b = 0; b < 3; ++b)
    if (nrm[b] > 0.0) m.eta = std::max(m.eta, den[b] > 0.0 ? nrm[b] / den[b] : INFINITY);
  return m;
}

SlotE slots(int64_t n, int nr, const double* ybar, double* y, double* u, double* lam) {
  SlotE sl{};
  for (int i = 0; i < nr; ++i) {
    sl.ybar[i] = ybar + i * n;
    sl.y[i] = y + i * n;
    sl.u[i] = u + i * n;
    sl.lam[i] = lam + i * n;
  }
  return sl;
}

// KKT sums of nr targets to the host (el.sumh[i * EL_SUMS + e])
sfdp_status kkt_sums(Problem& p, Elastic& el, int nr, const SlotE& sl, bool keep) {
  hipStream_t st = p.ctx->stream;
  ELCHK(el_launch_kkt(el, nr, sl, p.beta, keep, st));
  ELCHK(hipMemcpyAsync(el.sumh, el.sums, sizeof(double) * 2 * NRMAX * EL_SUMS, hipMemcpyDeviceToHost, st));
  ELCHK(hipStreamSynchronize(st));
  return SFDP_OK;
}

}  // namespace

sfdp_status el_kkt(Problem& p, int nrhs, const double* ybar, const double* y, const double* u, const double* lam,
                   double* rel, double* eta, double* viol) {
  if (!(p.beta > 0)) return host_fail(SFDP_E_STATE, "beta not set");
  Elastic& el = *p.el;
  sfdp_status s = ensure_rs(p, el);
  if (s) return s;
  const int64_t n = el.g.n_free;
  for (int r0 = 0; r0 < nrhs; r0 += NRMAX) {
    const int nr = std::min(NRMAX, nrhs - r0);
    const SlotE sl = slots(n, nr, ybar + r0 * n, (double*)y + r0 * n, (double*)u + r0 * n, (double*)lam + r0 * n);
    if ((s = kkt_sums(p, el, nr, sl, false))) return s;
    for (int i = 0; i < nr; ++i) {
      const Metrics m = metrics(el.sumh + i * EL_SUMS, p.beta);
      if (rel) rel[r0 + i] = m.rel;
      if (eta) eta[r0 + i] = m.eta;
      if (viol) viol[r0 + i] = m.viol;
    }
  }
  return SFDP_OK;
}

// The range-space refinement of Sec. 3.1 with the two complex factors of
// Sec. 4 on the elasticity KKT system (right-hand side (M ybar, 0, 0): the
// clamp is homogeneous).  Each step, on the current FP64 residual (r1, r2, r3):
//   dw = Z^-1 (-r3 - i alpha r1);  v = r1 + M dw;  z = Z^-1 conj(v);
//   y -= Re dw;  lam += Re z;  u = lam / beta
// Each target stops on its own test.
sfdp_status el_range_space(Problem& p, int nrhs, const double* ybar, double* y, double* u, double* lam,
                           const sfdp_opts* o, sfdp_info* info) {
  sfdp_status s = check_factored(p);
  if (s) return s;
  Elastic& el = *p.el;
  const Ctl c = controls(p, o);
  if (c.single) return host_fail(SFDP_E_INVALID, "elasticity problems take the two-factor step");
  if ((s = ensure_ws(p, el, c.kmax)) || (s = ensure_rs(p, el))) return s;
  hipStream_t st = p.ctx->stream;
  const int64_t n = el.g.n_free;
  const double t0 = now_ms();
  sfdp_status worst = SFDP_OK;
  for (int r0 = 0; r0 < nrhs; r0 += c.batch) {
    const int nr = std::min(c.batch, nrhs - r0);
    const SlotE sl = slots(n, nr, ybar + r0 * n, y + r0 * n, u + r0 * n, lam + r0 * n);
    for (int i = 0; i < nr; ++i) {
      ELCHK(hipMemcpyAsync(sl.y[i], sl.ybar[i], sizeof(double) * n, hipMemcpyDeviceToDevice, st));
      ELCHK(el_launch_fill(sl.u[i], sizeof(double) * n, st));
      ELCHK(el_launch_fill(sl.lam[i], sizeof(double) * n, st));
    }
    std::vector<sfdp_info> loc(nr);
    std::vector<int> done(nr, 0);
    for (auto& inf : loc) {
      inf = sfdp_info{};
      inf.t_setup_ms = p.t_setup_ms;
    }
    for (int step = 0;; ++step) {
      p.yield_point();
      if ((s = kkt_sums(p, el, nr, sl, true))) return s;
      ActE a{};
      for (int i = 0; i < nr; ++i) {
        const Metrics m = metrics(el.sumh + i * EL_SUMS, p.beta);
        sfdp_info& inf = loc[i];
        inf.rel_kkt = m.rel;
        inf.eta_blk = m.eta;
        inf.constr_viol = m.viol;
        if (step == 1) inf.rel_kkt_first = m.rel;
        if (done[i]) continue;
        if (!std::isfinite(m.eta) || !std::isfinite(m.rel)) {
          done[i] = 1;
          worst = host_fail(SFDP_E_NOCONV, "non-finite residual");
          continue;
        }
        if (m.eta <= c.tol_kkt) {
          done[i] = 1;
          continue;
        }
        if (step >= c.max_outer) {
          done[i] = 1;
          worst = host_fail(SFDP_E_NOCONV, "outer refinement limit reached");
          continue;
        }
        a.idx[a.n++] = i;
      }
      if (a.n == 0) break;
      const double tin = step == 0 ? c.tol_first : c.tol_inner;
      int its[NRMAX] = {};
      auto log = [&](int ci) {
        sfdp_info& inf = loc[a.idx[ci]];
        if (inf.n_feti < 16) inf.krylov_its[inf.n_feti] = its[ci];
        inf.n_feti++;
        inf.krylov_total += its[ci];
      };
      ELCHK(el_launch_rhs1(el, a, p.alpha, st));
      if ((s = feti_group(p, el, p.s32(), a.n, el.c1, el.c2, 0, tin, c.kmax, its))) return s;
      for (int ci = 0; ci < a.n; ++ci) log(ci);
      ELCHK(el_launch_rhs2(el, a, st));
      if ((s = feti_group(p, el, p.s32(), a.n, el.c3, el.c1, 0, tin, c.kmax, its))) return s;
      for (int ci = 0; ci < a.n; ++ci) log(ci);
      ELCHK(el_launch_update(el, a, sl, p.beta, st));
      ELCHK(hipMemcpyAsync(el.sumh + NRMAX * EL_SUMS, el.sums + NRMAX * EL_SUMS, sizeof(double) * NRMAX * EL_SUMS,
                           hipMemcpyDeviceToHost, st));
      ELCHK(hipStreamSynchronize(st));
      for (int ci = 0; ci < a.n; ++ci) {
        sfdp_info& inf = loc[a.idx[ci]];
        const double im = el.sumh[(NRMAX + ci) * EL_SUMS], re = el.sumh[(NRMAX + ci) * EL_SUMS + 1];
        inf.imag_ratio = re > 0.0 ? std::sqrt(im / re) : std::sqrt(im);
        inf.outer_steps = step + 1;
      }
    }
    if (info)
      for (int i = 0; i < nr; ++i) info[r0 + i] = loc[i];
  }
  if (info)
    for (int r = 0; r < nrhs; ++r) info[r].t_solve_ms = now_ms() - t0;
  return worst;
}

// z = S^-1 r = Re conj(Z^-1 conj(M Z^-1 r)) (Sec. 4), real r
sfdp_status el_schur_inv(Problem& p, int nrhs, const double* r, double* z, const sfdp_opts* o, sfdp_info* info) {
  sfdp_status s = check_factored(p);
  if (s) return s;
  Elastic& el = *p.el;
  const Ctl c = controls(p, o);
  if (c.single) return host_fail(SFDP_E_INVALID, "elasticity problems take the two-factor form");
  if (o && o->schur_block) return host_fail(SFDP_E_INVALID, "elasticity problems apply the exact S");
  if ((s = ensure_ws(p, el, c.kmax)) || (s = ensure_rs(p, el))) return s;
  hipStream_t st = p.ctx->stream;
  const int64_t n = el.g.n_free;
  const double t0 = now_ms();
  for (int r0 = 0; r0 < nrhs; r0 += c.batch) {
    const int nr = std::min(c.batch, nrhs - r0);
    ActE a{};
    a.n = nr;
    for (int i = 0; i < nr; ++i) {
      a.idx[i] = i;
      ELCHK(el_launch_r2c(n, r + (r0 + i) * n, el.c1 + i * n, st));
      ELCHK(el_launch_fill(el.r1 + i * n, sizeof(double) * n, st));
    }
    int its1[NRMAX] = {}, its2[NRMAX] = {};
    if ((s = feti_group(p, el, p.s32(), nr, el.c1, el.c2, 0, c.tol_inner, c.kmax, its1))) return s;
    ELCHK(el_launch_rhs2(el, a, st));  // c3 = conj(0 + M c2)
    if ((s = feti_group(p, el, p.s32(), nr, el.c3, el.c1, 0, c.tol_inner, c.kmax, its2))) return s;
    for (int i = 0; i < nr; ++i) ELCHK(el_launch_c2r(n, el.c1 + i * n, 0, 1.0, z + (r0 + i) * n, st));
    if (info)
      for (int i = 0; i < nr; ++i) {
        sfdp_info& inf = info[r0 + i];
        inf = sfdp_info{};
        inf.constr_viol = inf.eta_blk = -1.0;
        inf.n_feti = 2;
        inf.krylov_its[0] = its1[i];
        inf.krylov_its[1] = its2[i];
        inf.krylov_total = its1[i] + its2[i];
        inf.t_setup_ms = p.t_setup_ms;
      }
  }
  ELCHK(hipStreamSynchronize(st));
  if (info)
    for (int i = 0; i < nrhs; ++i) info[i].t_solve_ms = now_ms() - t0;
  return SFDP_OK;
}

sfdp_status el_apply(Problem& p, char which, int nrhs, const double* x, double* y) {
  if (which != 'K' && which != 'M') return host_fail(SFDP_E_INVALID, "elasticity problems apply 'K' or 'M'");
  ELCHK(el_launch_spmv(*p.el, which, nrhs, x, y, p.ctx->stream));
  return SFDP_OK;
}

// ---------------------------------------------------------- inspection --

sfdp_status el_inspect(Problem& p, sfdp_query what, int sub, double* out, int* rows, int* cols) {
  sfdp_status s = check_factored(p);
  if (s) return s;
  const Elastic& el = *p.el;
  const GeoE& g = el.g;
  int r = 0, c = 0;
  std::vector<int> qcols;
  if (what == SFDP_Q_COARSE || what == SFDP_Q_COARSE_INV) {
    r = c = g.nC;
  } else {
    if (sub < 0 || sub >= g.nsub) return host_fail(SFDP_E_INVALID, "sub out of range");
    r = el.h_nds[sub];
    if (what == SFDP_Q_PHI) {
      for (int q = 0; q < EQ; ++q)
        if (el.h_cg[sub * EQ + q] >= 0) qcols.push_back(q);
      c = (int)qcols.size();
    } else if (what == SFDP_Q_SINV || what == SFDP_Q_SBB) {
      c = r;
    } else {
      return host_fail(SFDP_E_INVALID, "unknown query");
    }
  }
  if (rows) *rows = r;
  if (cols) *cols = c;
  if (!out) return SFDP_OK;
  ELCHK(hipStreamSynchronize(p.ctx->stream));
  std::vector<cd> host((size_t)r * c);
  const size_t es = el_es(p.s32());
  auto get = [&](const std::vector<char>& raw, size_t idx) {
    if (es == sizeof(cf)) {
      const cf v = ((const cf*)raw.data())[idx];
      return cd{v.x, v.y};
    }
    return ((const cd*)raw.data())[idx];
  };
  if (what == SFDP_Q_COARSE || what == SFDP_Q_COARSE_INV) {
    ELCHK(hipMemcpy(host.data(), what == SFDP_Q_COARSE ? el.Kcc : el.Kinv, sizeof(cd) * host.size(),
                    hipMemcpyDeviceToHost));
  } else if (what == SFDP_Q_PHI) {
    std::vector<char> raw((size_t)g.ND * EQ * es);
    ELCHK(hipMemcpy(raw.data(), (const char*)el.Phi + (size_t)sub * raw.size(), raw.size(), hipMemcpyDeviceToHost));
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < c; ++j) host[(size_t)i * c + j] = get(raw, (size_t)i * EQ + qcols[j]);
  } else {
    std::vector<char> raw((size_t)g.ND * g.ND * es);
    const char* base = (const char*)(what == SFDP_Q_SINV ? el.Sinv : el.Sbb);
    ELCHK(hipMemcpy(raw.data(), base + (size_t)sub * raw.size(), raw.size(), hipMemcpyDeviceToHost));
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < c; ++j) host[(size_t)i * c + j] = get(raw, (size_t)i * g.ND + j);
  }
  ELCHK(hipMemcpy(out, host.data(), sizeof(cd) * host.size(), hipMemcpyHostToDevice));
  return SFDP_OK;
}

// ------------------------------------------------- target: forward solve --

// Consistent nodal forces of a uniform pressure on the bottom face z = 0,
// pushing in -z: every bottom face cell gives each of its four vertices
// -pressure h^2 / 4 (a bilinear shape function integrates to a quarter of the
// face); clamped vertices take none.
sfdp_status el_pressure(Problem& p, double pressure, double* f) {
  const GeoE& g = p.el->g;
  const Grid G{g.nx, g.ny, g.nz};
  const double h = 1.0 / g.n, q = -pressure * h * h / 4.0;
  std::vector<double> v(g.n_free, 0.0);
  for (int ey = 0; ey < g.ny; ++ey)
    for (int ex = 0; ex < g.nx; ++ex)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          const int i = ex + a, j = ey + b;
          if (i == 0) continue;
          v[3 * G.free_node(i, j, 0) + 2] += q;
        }
  ELCHK(hipMemcpy(f, v.data(), sizeof(double) * v.size(), hipMemcpyHostToDevice));
  return SFDP_OK;
}

// u = K^-1 f (real, nrhs right-hand sides) by FETI-DP on K alone: a twin of
// the partition (sharing its maps and workspaces) holds the factors of K,
// built on the first call and kept; complex128 storage whatever the problem's
// precision (the target of the control problem).
sfdp_status el_forward(Problem& p, int nrhs, const double* f, double* u, const sfdp_opts* o, int* its) {
  Elastic& el = *p.el;
  const Ctl c = controls(p, o);
  sfdp_status s;
  if ((s = ensure_ws(p, el, c.kmax)) || (s = ensure_rs(p, el))) return s;
  if (!el.fwd) {
    Elastic* tw = new (std::nothrow) Elastic();
    if (!tw) return host_fail(SFDP_E_NOMEM, "host allocation");
    tw->g = el.g;
    tw->g.alpha = 0.0;
    tw->g.rshift = 1;
    tw->rdof = el.rdof; tw->rfree = el.rfree; tw->rw = el.rw; tw->ni = el.ni; tw->nds = el.nds; tw->dw = el.dw;
    tw->dmu = el.dmu; tw->dsg = el.dsg; tw->muown = el.muown; tw->muw = el.muw; tw->cdof = el.cdof;
    tw->cg = el.cg; tw->cown = el.cown; tw->cw = el.cw; tw->cfree = el.cfree; tw->fcor = el.fcor;
    tw->fown = el.fown; tw->Ke = el.Ke;
    el.fwd = tw;
    if ((s = setup_factors(p, *tw, false))) {
      free_twin(p, el);
      return s;
    }
  }
  Elastic& tw = *el.fwd;
  // the twin works in the parent's workspaces
  tw.T = el.T; tw.Y = el.Y; tw.Wc = el.Wc; tw.fcs = el.fcs; tw.uc = el.uc; tw.gc = el.gc; tw.kb = el.kb;
  hipStream_t st = p.ctx->stream;
  const int64_t n = el.g.n_free;
  int loc[NRMAX];
  for (int r0 = 0; r0 < nrhs; r0 += c.batch) {
    const int nr = std::min(c.batch, nrhs - r0);
    for (int i = 0; i < nr; ++i) ELCHK(el_launch_r2c(n, f + (r0 + i) * n, el.c1 + i * n, st));
    if ((s = feti_group(p, tw, false, nr, el.c1, el.c2, 0, c.tol_inner, c.kmax, loc))) return s;
    for (int i = 0; i < nr; ++i) ELCHK(el_launch_c2r(n, el.c2 + i * n, 0, 1.0, u + (r0 + i) * n, st));
    if (its)
      for (int i = 0; i < nr; ++i) its[r0 + i] = loc[i];
  }
  ELCHK(hipStreamSynchronize(st));
  return SFDP_OK;
}

}  // namespace sfdp

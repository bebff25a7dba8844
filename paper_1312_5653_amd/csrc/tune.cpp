// Launch-variant autotuning.  Some kernels come in variants that compute the
// same results with different launch shapes (one workgroup per subdomain for
// all right-hand sides or one per right-hand side; the depth of the load
// pipeline of a streamed product).  Which is faster depends on the shape of
// the problem and on the device, so the first time a kernel runs for a key
// (kernel family, shape, storage precision, right-hand sides) every candidate
// is launched on the real operands -- the candidate kernels only read their
// inputs and overwrite their outputs, so running them again is harmless --
// and the one with the smallest median of three timed launches is kept for
// the rest of the process.  With tuning switched off (sfdp_set_tuning) the
// fixed default candidate runs.
#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "common.h"

namespace sfdp {

namespace {
std::mutex g_mu;
std::map<TuneKey, int> g_table;
bool g_enabled = true;
int g_force = -1;  // >= 0: run this candidate wherever a family has it (tests)
}  // namespace

bool TuneKey::operator<(const TuneKey& o) const {
  const int a[6] = {family, device, k0, k1, k2, k3}, b[6] = {o.family, o.device, o.k0, o.k1, o.k2, o.k3};
  return std::lexicographical_compare(a, a + 6, b, b + 6);
}

int tune_choice(const TuneKey& key, int ncand, int fallback, hipStream_t st, const std::function<void(int)>& launch,
                const float* weight) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_force >= 0) return g_force < ncand ? g_force : fallback;
    if (!g_enabled || ncand <= 1) return fallback;
    auto it = g_table.find(key);
    if (it != g_table.end()) return it->second;
  }
  hipEvent_t ev[4];
  for (hipEvent_t& e : ev)
    if (hipEventCreate(&e) != hipSuccess) return fallback;
  int best = fallback;
  float best_ms = 0.f;
  bool ok = true;
  for (int c = 0; c < ncand && ok; ++c) {
    launch(c);  // first run: code load, caches
    std::vector<float> t;
    for (int rep = 0; rep < 3 && ok; ++rep) {
      ok = hipEventRecord(ev[0], st) == hipSuccess;
      launch(c);
      ok = ok && hipEventRecord(ev[1], st) == hipSuccess && hipEventSynchronize(ev[1]) == hipSuccess;
      float ms = 0.f;
      ok = ok && hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess && hipGetLastError() == hipSuccess;
      t.push_back(ms);
    }
    if (!ok) break;
    std::sort(t.begin(), t.end());
    const float ms = t[1] * (weight ? weight[c] : 1.f);
    if (c == 0 || ms < best_ms) {
      best = c;
      best_ms = ms;
    }
  }
  for (hipEvent_t& e : ev) hipEventDestroy(e);
  if (!ok) return fallback;
  std::lock_guard<std::mutex> lk(g_mu);
  g_table[key] = best;
  return best;
}

std::atomic<unsigned> g_gen{0};

void tune_set_mode(bool on, int force) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_enabled = on;
  g_force = force;
  g_table.clear();
  g_gen++;
}

unsigned tune_generation() { return g_gen.load(); }

int tune_table(TuneEntry* out, int cap) {
  std::lock_guard<std::mutex> lk(g_mu);
  int n = 0;
  for (const auto& kv : g_table) {
    if (n < cap && out) out[n] = TuneEntry{kv.first, kv.second};
    ++n;
  }
  return n;
}

}  // namespace sfdp

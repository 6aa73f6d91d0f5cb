// Project-written schedule autotuner: times every registered column schedule
// of each (H, W) group of a plan and keeps the fastest, in the plan and in an
// in-process cache keyed by the group's size, coil count and slice count (the
// slice count sets the grid, so the best schedule depends on it).
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "api_internal.h"

using namespace mrx;

// Each candidate is timed on what it runs in practice: four CG iterations
// over the whole plan (operator plus CG update, with this group's candidate
// and the other groups' current choices) when the workspace is set, else
// (and for variational-network plans, whose stages apply the plain
// operator) five operator applications of the group.
extern "C" mrx_status mrx_plan_autotune(mrx_plan p, const float* S, const float* mask, float* a, float* b,
                                        void* stream) {
  if (!p) return fail(MRX_EINVAL, "autotune: null plan");
  if (!S || !mask || !a || !b) return fail(MRX_EINVAL, "autotune: null data pointer");
  if (p->toep) return MRX_OK;  // one Toeplitz schedule per padded length: nothing to choose
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(MRX_EHIP, "autotune: event create");
  // plans for the variational network use the plain operator, the others CG
  const bool use_cg = p->ws != nullptr && !(p->flags & MRX_PLAN_VN);
  // With several size groups running concurrently, coil-split schedules on
  // 8-column tiles (half a 128-byte row segment; the pairs of workgroups
  // that share a segment are not guaranteed to run together) are left out
  // where the length has a 16-column split: timed in four CG iterations they
  // can come out ahead, yet the 64-slice batch's reconstruction graph ran
  // 11% slower with one (384 x 320) than with the 16-column split.
  const bool several = p->groups.size() > 1;
  for (auto& g : p->groups) {
    const ColVariant* best = g.col;
    float best_ms = 1e30f;
    bool wide_split = false;
    for (const ColVariant* v : col_variants(g.H)) wide_split = wide_split || (v->kspl > 1 && v->WT >= 16);
    for (const ColVariant* v : col_variants(g.H)) {
      if (several && wide_split && v->kspl > 1 && v->WT < 16) continue;
      g.col = v;
      if (refresh_desc(p, true) != MRX_OK) continue;
      auto run = [&]() -> bool {
        if (use_cg)
          return cg_impl(p, (const float2*)a, nullptr, (const float2*)S, mask, nullptr, 4, (float2*)b, nullptr, s) ==
                 MRX_OK;
        // the operator application as normal_impl runs it (with the
        // schedule's coil split where the scratch allows)
        bool ok = true;
        for (int it = 0; it < 5; ++it)
          ok = ok && normal_group(p, g, (const float2*)a, (const float2*)S, mask, nullptr, (float2*)b, s) ==
                         hipSuccess;
        return ok;
      };
      if (!run()) continue;  // warm-up
      // the fastest of five timed pairs: robust against a slow outlier
      bool ok = true;
      float ms = 1e30f;
      for (int trial = 0; trial < 5 && ok; ++trial) {
        ok = hipEventRecord(e0, s) == hipSuccess;
        for (int rep = 0; rep < 2; ++rep) ok = ok && run();
        ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float t = 0.f;
        ok = ok && hipEventElapsedTime(&t, e0, e1) == hipSuccess;
        if (ok) ms = t < ms ? t : ms;
      }
      if (ok && ms < best_ms) { best_ms = ms; best = v; }
    }
    g.col = best;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[{g.H, g.W, g.maxC, (int)g.slices.size()}] = best->name;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // the timing solves may have raised status bits; they are not the caller's
  if (use_cg && clear_status(p, s) != hipSuccess) return fail(MRX_EHIP, "autotune: status reset");
  if (hipGetLastError() != hipSuccess) return fail(MRX_EHIP, "autotune: launch failed");
  return refresh_desc(p, true);
}

// Text form of the cache, one entry a line: "H W C slices schedule_name".
extern "C" mrx_status mrx_tune_cache_save(const char* path) {
  if (!path) return fail(MRX_EINVAL, "tune_cache_save: null path");
  FILE* f = fopen(path, "w");
  if (!f) return fail(MRX_EINVAL, std::string("tune_cache_save: cannot open ") + path);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : g_tune_cache)
      fprintf(f, "%d %d %d %d %s\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
              std::get<3>(kv.first), kv.second.c_str());
  }
  return fclose(f) == 0 ? MRX_OK : fail(MRX_EINVAL, std::string("tune_cache_save: write failed: ") + path);
}

extern "C" mrx_status mrx_tune_cache_load(const char* path, int32_t* n_loaded) {
  if (!path) return fail(MRX_EINVAL, "tune_cache_load: null path");
  FILE* f = fopen(path, "r");
  if (!f) return fail(MRX_EINVAL, std::string("tune_cache_load: cannot open ") + path);
  std::map<std::tuple<int, int, int, int>, std::string> entries;
  char line[512];
  int lineno = 0;
  while (fgets(line, sizeof line, f)) {
    ++lineno;
    int H = 0, W = 0, C = 0, n = 0;
    char name[256] = {0};
    if (line[0] == '\n' || line[0] == '#') continue;
    if (sscanf(line, "%d %d %d %d %255s", &H, &W, &C, &n, name) != 5 || !find_col(H, name) || W <= 0 || C <= 0 ||
        n <= 0) {
      fclose(f);
      return fail(MRX_EINVAL, std::string("tune_cache_load: bad entry at line ") + std::to_string(lineno) +
                                  " of " + path);
    }
    entries[{H, W, C, n}] = name;
  }
  fclose(f);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& kv : entries) g_tune_cache[kv.first] = kv.second;
  if (n_loaded) *n_loaded = (int32_t)entries.size();
  return MRX_OK;
}

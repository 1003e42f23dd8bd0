// Autotuner: times every legal (exchange depth, workgroups per CU) pair of a circuit's fused
// Maxwell step, and the dense-block path where the call may take it, with HIP events on the
// context stream and keeps the fastest.  The key is
// (arch, n, rounds, fused gates, entangler kinds) plus a point-count bucket; results persist as
// JSON lines in the file named by QP_TUNE_CACHE (if set; later lines override earlier ones).
// Each tuning also records its choice under the bucket "any", which circuit compilation looks up
// so that a cached choice applies from the first evaluation on.
#include "tune.hpp"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "fused.hpp"

namespace qp {

namespace {
std::mutex g_mu;
std::map<std::string, TuneEntry> g_cache;
bool g_loaded = false;

void load_file() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = std::getenv("QP_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[1024];
  while (std::fgets(line, sizeof(line), f)) {
    char key[512];
    TuneEntry e{};
    int dense = 0;   // lines without the field: the fused path
    const int got = std::sscanf(line, "{\"key\": \"%511[^\"]\", \"exs\": %d, \"wg_per_cu\": %d, \"ms\": %lf, \"dense\": %d}",
                                key, &e.exs, &e.wg_per_cu, &e.ms, &dense);
    if (got >= 4) {
      e.dense = got == 5 ? (dense != 0) : 0;
      g_cache[key] = e;
    }
  }
  std::fclose(f);
}

void append_file(const std::string& key, const TuneEntry& e) {
  const char* path = std::getenv("QP_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "{\"key\": \"%s\", \"exs\": %d, \"wg_per_cu\": %d, \"ms\": %.6f, \"dense\": %d}\n", key.c_str(), e.exs,
               e.wg_per_cu, e.ms, e.dense);
  std::fclose(f);
}
}  // namespace

std::string tune_key(const qp_ctx* ctx, const qp_circuit* c) {
  int ncnot = 0, ncz = 0;
  for (const auto& g : c->hp.gates) {
    ncnot += g.kind == QP_CNOT;
    ncz += g.kind == QP_CZ;
  }
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s/n%d/r%zu/f%zu/cx%d/cz%d/e%d", ctx->arch.c_str(), c->hp.n, c->hp.rounds.size(),
                c->hp.fused.size(), ncnot, ncz, c->hp.enc_kind);
  return buf;
}

static std::string pkey(const std::string& k, int64_t P) {
  const int b = P > 0 ? (int)std::floor(std::log2((double)P)) : 0;
  return k + "/p" + std::to_string(b);
}

const TuneEntry* tune_lookup(const qp_ctx* ctx, const qp_circuit* c) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_file();
  auto it = g_cache.find(tune_key(ctx, c) + "/any");
  return it == g_cache.end() ? nullptr : &it->second;
}

void tune_circuit(qp_ctx* ctx, qp_circuit* c, const float* params, const float* points, const float* angles,
                  const float* jac, int64_t P, const qp_maxwell_desc* ld, void* ws, bool dense_ok) {
  const std::string key = pkey(tune_key(ctx, c), P);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    load_file();
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      c->exs = it->second.exs;
      c->wg_per_cu = it->second.wg_per_cu;
      c->use_dense = it->second.dense != 0 && c->hp.dense_ok;
      return;
    }
  }
  const int n = c->hp.n;
  const int F = (int)c->hp.fused.size();
  const size_t cap = 160 * 1024;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  TuneEntry best{c->exs, c->wg_per_cu, 1e30};
  const int max_wg = fused_max_wg_per_cu(n);
  const int NM = n_moments(c);
  for (int exs : {2, 4}) {
    if (exs == 4 && NM > 0) continue;   // phase stages run on the unpipelined kernel
    const size_t lds = fused_lds_bytes(n, exs, F, NM);
    if (lds > cap) continue;
    for (int wg = 1; wg <= max_wg; ++wg) {
      if (lds * wg > cap) break;
      const int grid = ctx->cu_count * wg;
      double best_ms = 1e30;
      for (int rep = 0; rep < 3; ++rep) {   // first run warms up; the main kernel only
        hipEventRecord(e0, ctx->stream);
        run_fused(ctx, c, kModeMaxwell, params, points, angles, jac, P, ld, nullptr, nullptr, nullptr, nullptr,
                  nullptr, nullptr, nullptr, nullptr, ws, 0, exs, grid);
        hipEventRecord(e1, ctx->stream);
        hipEventSynchronize(e1);
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) best_ms = std::min(best_ms, (double)ms);
      }
      if (best_ms < best.ms) best = TuneEntry{exs, wg, best_ms};
    }
  }
  if (dense_ok) {   // fusion width: the dense-block path keeps the fused path's launch shape
    double best_ms = 1e30;
    for (int rep = 0; rep < 3; ++rep) {
      hipEventRecord(e0, ctx->stream);
      run_dense(ctx, c, kModeMaxwell, params, points, angles, jac, P, ld, nullptr, nullptr, nullptr, nullptr, nullptr,
                nullptr, ws, 0);
      hipEventRecord(e1, ctx->stream);
      hipEventSynchronize(e1);
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) best_ms = std::min(best_ms, (double)ms);
    }
    if (best_ms < best.ms) { best.ms = best_ms; best.dense = 1; }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  c->exs = best.exs;
  c->wg_per_cu = best.wg_per_cu;
  c->use_dense = best.dense != 0;
  std::lock_guard<std::mutex> lk(g_mu);
  const std::string any = tune_key(ctx, c) + "/any";
  g_cache[key] = best;
  g_cache[any] = best;
  append_file(key, best);
  append_file(any, best);
}

}  // namespace qp

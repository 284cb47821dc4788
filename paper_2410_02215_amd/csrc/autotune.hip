// Tile-shape autotuner of the grouped GEMM.
//
// A grouped GEMM plan is classified by a shape key (GEMM kind, the binary
// orders of magnitude of the largest M, N and K and of the group count, and
// whether any group is a symmetric product or a block scatter). In tuning
// mode the first plan of an unseen key is timed, on scratch operands of its
// own extents, with every tile configuration of the kernel (64 x 64,
// 128 x 128, 256 x 16, 256 x 32, 16 x 256, 32 x 256) whose padded tiles do not
// exceed four times the useful area, each with and without the heuristic
// split-K factor; the fastest (median of three timed runs after one warm-up)
// is kept for the key. Plans of a known key take the stored choice; without
// an entry, or with the tuner off, the built-in heuristic decides. The
// choices are kept in a process-wide table that can be saved to and loaded
// from a small JSON file (one entry per key: configuration, split factor,
// measured microseconds).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "common.h"

namespace ftn {

namespace {
struct Choice {
  int cfg = -1;
  int split = -1;
  double us = 0.0;
};
std::mutex g_mu;
std::map<std::string, Choice> g_table;
int g_mode = 0;  // 0 off, 1 use stored choices, 2 also tune unseen keys
int64_t g_tuned = 0, g_hits = 0;

constexpr double TUNE_MAX_BYTES = 2.0 * (1 << 30);
const int TILE_BM[] = {64, 128, 256, 256, 16, 32};
const int TILE_BN[] = {64, 128, 16, 32, 256, 256};

int lg2(int64_t x) {
  int e = 0;
  while ((int64_t(1) << e) < x) ++e;
  return e;
}

std::string shape_key(const std::vector<GemmGroup>& gs, int kind) {
  int64_t mm = 0, mn = 0, mk = 0;
  int sym = 0, sc = 0;
  for (auto& g : gs) {
    mm = std::max(mm, g.M);
    mn = std::max(mn, g.N);
    mk = std::max(mk, g.K);
    sym |= g.sym ? 1 : 0;
    sc |= g.scatter == 1 ? 1 : 0;
  }
  std::ostringstream o;
  o << "k" << kind << "-m" << lg2(mm) << "-n" << lg2(mn) << "-k" << lg2(std::max<int64_t>(mk, 1)) << "-g"
    << lg2((int64_t)gs.size()) << "-s" << sym << "-x" << sc;
  return o.str();
}

// element extents of the operands the groups touch
void extents(const std::vector<GemmGroup>& gs, int64_t& ea, int64_t& eb, int64_t& ec) {
  ea = eb = ec = 1;
  for (auto& g : gs) {
    if (g.K > 0) {
      ea = std::max(ea, g.a_off + (g.transA ? (g.K - 1) * g.lda + g.M : (g.M - 1) * g.lda + g.K));
      eb = std::max(eb, g.b_off + (g.transB ? (g.N - 1) * g.ldb + g.K : (g.K - 1) * g.ldb + g.N));
    }
  }
  int64_t c = 0;
  for (auto& g : gs) c += g.M * g.N;
  ec = std::max<int64_t>(c, 1);
}

Choice tune_now(const std::vector<GemmGroup>& gs0, int kind, hipStream_t s) {
  // scatter outputs are timed as plain outputs (same tiles and K loop)
  std::vector<GemmGroup> gs(gs0);
  int64_t co = 0;
  for (auto& g : gs) {
    if (g.scatter == 1) g.scatter = 0;
    g.c_off = co;
    g.ldc = g.N;
    co += g.M * g.N;
  }
  int64_t ea, eb, ec;
  extents(gs, ea, eb, ec);
  const size_t es = kind == FTN_GEMM_F64 ? 8 : 4;
  const int dtype = kind == FTN_GEMM_F64 ? FTN_F64 : FTN_F32;
  Choice best;
  // plans whose operands span more than TUNE_MAX_BYTES are left to the
  // heuristic (their large tiles fill the chip anyway)
  const double need = (double)(ea + eb + ec) * es;
  static const bool trace = std::getenv("FTN_TRACE_TUNE") != nullptr;
  if (trace)
    std::fprintf(stderr, "[tune] %s extents %lld %lld %lld (%.3g GB)\n", shape_key(gs0, kind).c_str(), (long long)ea,
                 (long long)eb, (long long)ec, need / 1e9);
  if (need > TUNE_MAX_BYTES) return best;
  DBuf<char> A(ea * es, s), B(eb * es, s), C(ec * es, s);
  HIPC(hipMemsetAsync(A.p, 0, ea * es, s));
  HIPC(hipMemsetAsync(B.p, 0, eb * es, s));
  double useful = 0;
  for (auto& g : gs) useful += (double)g.M * g.N;
  hipEvent_t e0, e1;
  HIPC(hipEventCreate(&e0));
  HIPC(hipEventCreate(&e1));
  best.us = 1e300;
  prof_quiet(true);
  try {
    for (int cfg = 0; cfg < gemm_ncfg(); ++cfg) {
      double padded = 0;
      for (auto& g : gs) padded += (double)cdiv(g.M, TILE_BM[cfg]) * TILE_BM[cfg] * cdiv(g.N, TILE_BN[cfg]) * TILE_BN[cfg];
      if (padded > 4.0 * useful) continue;
      int64_t last_split = -2;
      for (int sp : {-1, 1}) {
        GemmPlan p;
        gemm_plan_with(p, gs, kind, s, false, cfg, sp);
        if (p.split == last_split) continue;
        last_split = p.split;
        if ((double)p.ws_elems * es > TUNE_MAX_BYTES) continue;
        DBuf<char> ws(p.ws_elems * es, s);
        run_gemm(p, dtype, A.p, B.p, C.p, nullptr, s, 1.0, 0.0, ws.p);
        float t[3];
        for (int r = 0; r < 3; ++r) {
          HIPC(hipEventRecord(e0, s));
          run_gemm(p, dtype, A.p, B.p, C.p, nullptr, s, 1.0, 0.0, ws.p);
          HIPC(hipEventRecord(e1, s));
          HIPC(hipEventSynchronize(e1));
          HIPC(hipEventElapsedTime(&t[r], e0, e1));
        }
        std::sort(t, t + 3);
        const double us = 1000.0 * t[1];
        if (us < best.us) {
          best.us = us;
          best.cfg = cfg;
          best.split = (int)p.split;
        }
      }
    }
  } catch (...) {
    prof_quiet(false);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  prof_quiet(false);
  HIPC(hipEventDestroy(e0));
  HIPC(hipEventDestroy(e1));
  return best;
}
}  // namespace

void tune_choice(const std::vector<GemmGroup>& gs, int kind, hipStream_t s, int* cfg, int* split) {
  *cfg = -1;
  *split = -1;
  int mode;
  {
    std::lock_guard<std::mutex> g(g_mu);
    mode = g_mode;
  }
  if (mode == 0) return;
  const std::string key = shape_key(gs, kind);
  {
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_table.find(key);
    if (it != g_table.end()) {
      *cfg = it->second.cfg;
      *split = it->second.split;
      ++g_hits;
      return;
    }
  }
  if (mode != 2) return;
  const Choice c = tune_now(gs, kind, s);
  if (c.cfg < 0) return;
  std::lock_guard<std::mutex> g(g_mu);
  g_table[key] = c;
  ++g_tuned;
  *cfg = c.cfg;
  *split = c.split;
}

}  // namespace ftn

using namespace ftn;

template <typename F>
static int guarded_tune(F&& f) {
  try {
    f();
    return FTN_OK;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return FTN_EINVAL;
  }
}

extern "C" int ftn_autotune(int mode) {
  return guarded_tune([&] {
    if (mode < 0 || mode > 2) fail(FTN_EINVAL, "autotune mode must be 0, 1 or 2");
    std::lock_guard<std::mutex> g(g_mu);
    g_mode = mode;
  });
}

extern "C" int ftn_autotune_save(const char* path) {
  return guarded_tune([&] {
    if (!path) fail(FTN_EINVAL, "null path");
    std::ofstream f(path);
    if (!f) fail(FTN_EINVAL, std::string("cannot write ") + path);
    std::lock_guard<std::mutex> g(g_mu);
    f << "{\n \"version\": 1,\n \"arch\": \"gfx950\",\n \"entries\": {";
    bool first = true;
    for (auto& kv : g_table) {
      f << (first ? "\n" : ",\n") << "  \"" << kv.first << "\": [" << kv.second.cfg << ", " << kv.second.split
        << ", " << kv.second.us << "]";
      first = false;
    }
    f << "\n }\n}\n";
    if (!f) fail(FTN_EINVAL, std::string("write failed: ") + path);
  });
}

extern "C" int ftn_autotune_load(const char* path) {
  return guarded_tune([&] {
    if (!path) fail(FTN_EINVAL, "null path");
    std::ifstream f(path);
    if (!f) fail(FTN_EINVAL, std::string("cannot read ") + path);
    std::string line;
    std::map<std::string, Choice> add;
    while (std::getline(f, line)) {
      const size_t q0 = line.find('"'), q1 = q0 == std::string::npos ? q0 : line.find('"', q0 + 1);
      const size_t b = line.find('[');
      if (q0 == std::string::npos || q1 == std::string::npos || b == std::string::npos || b < q1) continue;
      Choice c;
      if (std::sscanf(line.c_str() + b, "[%d, %d, %lf]", &c.cfg, &c.split, &c.us) != 3) continue;
      if (c.cfg < 0 || c.cfg >= gemm_ncfg() || c.split < 1) fail(FTN_EINVAL, "bad tuning entry: " + line);
      add[line.substr(q0 + 1, q1 - q0 - 1)] = c;
    }
    std::lock_guard<std::mutex> g(g_mu);
    for (auto& kv : add) g_table[kv.first] = kv.second;
  });
}

extern "C" int ftn_autotune_stats(int64_t* entries, int64_t* tuned, int64_t* hits) {
  return guarded_tune([&] {
    std::lock_guard<std::mutex> g(g_mu);
    if (entries) *entries = (int64_t)g_table.size();
    if (tuned) *tuned = g_tuned;
    if (hits) *hits = g_hits;
  });
}

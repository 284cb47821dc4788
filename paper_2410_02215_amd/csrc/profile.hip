// Opt-in kernel timing with HIP events on the launching stream. When
// enabled, each instrumented launch carries two events in its dispatch
// (hipExtLaunchKernelGGL), which take the times the kernel starts and ends,
// so that a duration is the kernel's own even while other streams keep the
// device busy; durations, launch counts and the algorithmic work the caller
// attributes to the launch (flops or bytes) are accumulated per kernel
// class until collected.
#include <mutex>

#include "common.h"

namespace ftn {

namespace {
struct Rec {
  hipEvent_t a, b;
  int cls;
  double work;
  double bytes;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
double g_ms[FTN_PROF_NCLASS], g_cnt[FTN_PROF_NCLASS], g_work[FTN_PROF_NCLASS], g_bytes[FTN_PROF_NCLASS];

hipEvent_t take() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPC(hipEventCreate(&e));
  return e;
}

// durations of a batch of records, taken outside the lock (waiting for the
// events must not hold up the other threads' launches). Without `block`,
// only records whose end event has completed are taken; the others go back.
void settle(std::vector<Rec>& recs, bool block) {
  std::vector<float> ms(recs.size(), -1.0f);
  for (size_t i = 0; i < recs.size(); ++i) {
    if (block) {
      HIPC(hipEventSynchronize(recs[i].b));
    } else {
      const hipError_t q = hipEventQuery(recs[i].b);
      if (q == hipErrorNotReady) {
        (void)hipGetLastError();
        continue;
      }
      HIPC(q);
    }
    HIPC(hipEventElapsedTime(&ms[i], recs[i].a, recs[i].b));
  }
  std::lock_guard<std::mutex> g(g_mu);
  for (size_t i = 0; i < recs.size(); ++i) {
    const Rec& r = recs[i];
    if (ms[i] < 0.0f) {
      g_recs.push_back(r);
      continue;
    }
    g_ms[r.cls] += ms[i];
    g_cnt[r.cls] += 1;
    g_work[r.cls] += r.work;
    g_bytes[r.cls] += r.bytes;
    // single-kernel classes also count in their family class
    const int par = (r.cls >= FTN_PROF_K_GEMM_F64_64x64 && r.cls <= FTN_PROF_K_SPLITK_F64) ||
                            r.cls == FTN_PROF_K_SKINNY_F64 || r.cls == FTN_PROF_K_GEMM_F64_TALL
                        ? FTN_PROF_GEMM_F64
                    : r.cls >= FTN_PROF_K_ORTH && r.cls <= FTN_PROF_K_SVD_COLS  ? FTN_PROF_FACTOR
                                                                                : -1;
    if (par >= 0) {
      const bool time_only = r.cls == FTN_PROF_K_SPLITK_F64 || r.cls == FTN_PROF_K_JACOBI_VEC;
      g_ms[par] += ms[i];
      if (!time_only) {
        g_cnt[par] += 1;
        g_work[par] += r.work;
        g_bytes[par] += r.bytes;
      }
    }
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  recs.clear();
}

void drain() {
  std::vector<Rec> recs;
  {
    std::lock_guard<std::mutex> g(g_mu);
    recs.swap(g_recs);
  }
  settle(recs, true);
}
}  // namespace

// Launches made from library worker threads (several host threads submitting
// at once) are never instrumented: every event record of this timer happens
// on a thread that called into the library, under the timer's lock.
thread_local bool t_quiet = false;

bool prof_on() { return g_on && !t_quiet; }

void prof_quiet(bool on) { t_quiet = on; }

void* prof_begin(hipStream_t s) {
  (void)s;
  if (!g_on || t_quiet) return nullptr;
  std::lock_guard<std::mutex> g(g_mu);
  Rec* r = new Rec;
  r->a = take();
  r->b = take();
  return r;
}

hipEvent_t prof_ev(void* tok, int which) {
  if (!tok) return nullptr;
  Rec* r = (Rec*)tok;
  return which ? r->b : r->a;
}

void prof_end(void* tok, hipStream_t s, int cls, double work, double bytes) {
  if (!tok) return;
  Rec* r = (Rec*)tok;
  r->cls = cls;
  r->work = work;
  r->bytes = bytes;
  (void)s;
  std::vector<Rec> full;
  {
    std::lock_guard<std::mutex> g(g_mu);
    g_recs.push_back(*r);
    if (g_recs.size() > 4096) full.swap(g_recs);
  }
  delete r;
  if (!full.empty()) settle(full, false);
}

void prof_enable(int on) {
  drain();
  std::lock_guard<std::mutex> g(g_mu);
  g_on = on != 0;
}

void prof_collect(double* ms, double* count, double* work, double* bytes) {
  drain();
  std::lock_guard<std::mutex> g(g_mu);
  for (int c = 0; c < FTN_PROF_NCLASS; ++c) {
    if (ms) ms[c] = g_ms[c];
    if (count) count[c] = g_cnt[c];
    if (work) work[c] = g_work[c];
    if (bytes) bytes[c] = g_bytes[c];
    g_ms[c] = g_cnt[c] = g_work[c] = g_bytes[c] = 0;
  }
}

}  // namespace ftn

extern "C" int ftn_profile_enable(int on) {
  try {
    ftn::prof_enable(on);
    return FTN_OK;
  } catch (const ftn::Error& e) {
    ftn::set_last_error(e.msg);
    return e.code;
  }
}

extern "C" int ftn_profile_collect(double* ms, double* count, double* work, double* bytes) {
  try {
    ftn::prof_collect(ms, count, work, bytes);
    return FTN_OK;
  } catch (const ftn::Error& e) {
    ftn::set_last_error(e.msg);
    return e.code;
  }
}

// Error reporting, default constants and launch profiling of libgsmi.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "common.h"

namespace gsmi {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

gs_status hip_fail(hipError_t e, const char *what) {
  set_error("%s: %s", what, hipGetErrorString(e));
  return GS_ERR_HIP;
}

// ------------------------------------------------------------ profiling
struct ProfRecord {
  std::string name;
  hipEvent_t start, stop;
};
static bool g_prof_on = false;
static std::vector<std::string> g_prof_sel;  // empty: every kernel
static std::vector<ProfRecord> g_prof;
static std::vector<hipEvent_t> g_free_events;

static hipEvent_t take_event() {
  if (!g_free_events.empty()) {
    hipEvent_t e = g_free_events.back();
    g_free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

static bool selected(const char *n) {
  if (g_prof_sel.empty()) return true;
  for (const auto &x : g_prof_sel)
    if (x == n) return true;
  return false;
}

ProfScope::ProfScope(const char *n, hipStream_t s) : name(n), stream(s), slot(-1) {
  if (!g_prof_on || !selected(n)) return;
  ProfRecord r{n, take_event(), take_event()};
  if (!r.start || !r.stop) return;
  (void)hipEventRecord(r.start, s);
  g_prof.push_back(r);
  slot = (int)g_prof.size() - 1;
}

ProfScope::~ProfScope() {
  if (slot >= 0) (void)hipEventRecord(g_prof[slot].stop, stream);
}

}  // namespace gsmi

using namespace gsmi;

extern "C" {

const char *gs_last_error(void) { return g_err; }

void gs_default_params(gs_raster_params *p) {
  if (!p) return;
  p->eps2d = 0.3f;
  p->alpha_max = 0.99f;
  p->alpha_min = 1.0f / 255.0f;
  p->t_min = 1e-4f;
  p->guard = 1.3f;
  p->mip_filter = 0;
}

void gs_profile_enable(int on) { g_prof_on = on != 0; }

void gs_profile_select(const char *names) {
  g_prof_sel.clear();
  if (!names) return;
  std::string cur;
  for (const char *c = names;; ++c) {
    if (*c == ',' || *c == 0) {
      if (!cur.empty()) g_prof_sel.push_back(cur);
      cur.clear();
      if (*c == 0) break;
    } else {
      cur.push_back(*c);
    }
  }
}

void gs_profile_reset(void) {
  for (auto &r : g_prof) {
    (void)hipEventSynchronize(r.stop);
    g_free_events.push_back(r.start);
    g_free_events.push_back(r.stop);
  }
  g_prof.clear();
}

gs_status gs_profile_read(const char *kernel, double *total_ms, int64_t *launches) {
  GS_REQUIRE(kernel && total_ms && launches, "gs_profile_read: NULL argument");
  double sum = 0.0;
  int64_t cnt = 0;
  for (auto &r : g_prof) {
    if (r.name != kernel) continue;
    GS_CHECK_HIP(hipEventSynchronize(r.stop), "hipEventSynchronize");
    float ms = 0.f;
    GS_CHECK_HIP(hipEventElapsedTime(&ms, r.start, r.stop), "hipEventElapsedTime");
    sum += ms;
    ++cnt;
  }
  *total_ms = sum;
  *launches = cnt;
  return GS_OK;
}

}  // extern "C"

// Opt-in per-launch timing: an event pair around each kernel launch on the
// launching stream, tagged with the kernel family and the launch's algorithmic
// bytes. Events come from a pool so recording costs no allocation once warm.
#include <string>

#include "prof.h"

namespace qsv {

namespace {
struct Rec {
  const char* name;
  int a, b;  // pool indices
  double bytes;
};
bool g_on = false;
std::vector<hipEvent_t> g_pool;
size_t g_used = 0;
std::vector<Rec> g_recs;

int take_event() {
  if (g_used == g_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    g_pool.push_back(e);
  }
  return int(g_used++);
}
}  // namespace

bool prof_on() { return g_on; }

ProfScope::ProfScope(const char* name, double bytes, hipStream_t stream)
    : name_(name), bytes_(bytes), stream_(stream) {
  if (!g_on) return;
  a_ = take_event();
  if (a_ >= 0) (void)hipEventRecord(g_pool[a_], stream_);
}

ProfScope::~ProfScope() {
  if (!g_on || a_ < 0) return;
  const int b = take_event();
  if (b < 0) return;
  (void)hipEventRecord(g_pool[b], stream_);
  g_recs.push_back({name_, a_, b, bytes_});
}

}  // namespace qsv

using namespace qsv;

extern "C" {

int qsv_prof_enable(int on) {
  clear_error();
  if (on) {
    for (hipEvent_t e : g_pool) (void)hipEventSynchronize(e);
    g_recs.clear();
    g_used = 0;
  }
  g_on = on != 0;
  return QSV_OK;
}

int qsv_prof_read(const char* name, int* launches, double* total_ms, double* bytes) {
  clear_error();
  if (!name) return fail(QSV_EINVAL, "null kernel family name");
  int cnt = 0;
  double ms = 0.0, by = 0.0;
  for (const Rec& r : g_recs) {
    if (std::string(r.name) != name) continue;
    QSV_HIP_CHECK(hipEventSynchronize(g_pool[r.b]));
    float t = 0.f;
    QSV_HIP_CHECK(hipEventElapsedTime(&t, g_pool[r.a], g_pool[r.b]));
    ++cnt;
    ms += t;
    by += r.bytes;
  }
  if (launches) *launches = cnt;
  if (total_ms) *total_ms = ms;
  if (bytes) *bytes = by;
  return QSV_OK;
}

}  // extern "C"

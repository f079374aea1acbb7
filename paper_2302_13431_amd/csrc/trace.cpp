// Kernel tracing: HIP events bracket the launches whose kernel name contains
// the filter, on the handle's stream, so a caller can time individual kernels
// inside a larger timed region (pisco_trace_enable / pisco_trace_read).
#include <cstring>
#include <map>

#include "common.hpp"

namespace pisco {

static hipEvent_t next_event(Handle* h) {
  if (h->events_used == h->event_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->event_pool.push_back(e);
  }
  return h->event_pool[h->events_used++];
}

TraceScope::TraceScope(Handle* hh, const char* name) : h(hh) {
  if (!h || !h->trace) return;
  if (!h->trace_filter.empty() && !std::strstr(name, h->trace_filter.c_str())) return;
  rec.name = name;
  rec.begin = next_event(h);
  rec.end = next_event(h);
  if (rec.begin && rec.end) (void)hipEventRecord(rec.begin, h->stream);
}

TraceScope::~TraceScope() {
  if (!rec.name || !rec.begin || !rec.end) return;
  (void)hipEventRecord(rec.end, h->stream);
  h->records.push_back(rec);
}

}  // namespace pisco

using namespace pisco;

extern "C" {

pisco_status_t pisco_trace_enable(pisco_handle_t handle, int32_t enable, const char* filter) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  if (!h) return PISCO_ERR_ARG;
  h->trace = enable != 0;
  h->trace_filter = filter ? filter : "";
  return PISCO_OK;
}

pisco_status_t pisco_trace_read(pisco_handle_t handle, pisco_trace_entry_t* out, int32_t cap,
                                int32_t* count) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  if (!h || !count || (cap > 0 && !out)) return PISCO_ERR_ARG;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_check(h, e, "pisco_trace_read");
  std::map<std::string, std::pair<int, double>> agg;
  for (const TraceRec& r : h->records) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.begin, r.end) != hipSuccess) continue;
    auto& a = agg[r.name];
    a.first += 1;
    a.second += ms;
  }
  h->records.clear();
  h->events_used = 0;
  int n = 0;
  for (const auto& kv : agg) {
    if (n < cap) {
      std::memset(out[n].name, 0, sizeof(out[n].name));
      std::strncpy(out[n].name, kv.first.c_str(), sizeof(out[n].name) - 1);
      out[n].launches = kv.second.first;
      out[n].total_ms = kv.second.second;
    }
    ++n;
  }
  *count = n;
  return PISCO_OK;
}

}  // extern "C"

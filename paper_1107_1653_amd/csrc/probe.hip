// Kernel timing probe: when enabled for a kernel family, every launch of that
// family is bracketed by HIP events recorded on the launch stream, and the
// algorithmic bytes the launch must move are accumulated.  Reading the probe
// synchronises on the recorded events and returns launches, total device
// time and total algorithmic bytes.
#include "probe.hpp"

#include <mutex>

namespace shp {

namespace {
struct Family {
  bool on = false;
  std::vector<hipEvent_t> ev;   // start/stop pairs recorded since the last flush
  std::vector<hipEvent_t> pool; // created events ready for reuse
  int64_t launches = 0;
  double bytes = 0.0;
  double flushed_ms = 0.0;
};
std::mutex g_mu;
Family g_fam[kProbeFamilies];

void flush(Family& f) {
  for (size_t k = 0; k + 1 < f.ev.size(); k += 2) {
    SHP_HIP(hipEventSynchronize(f.ev[k + 1]));
    float ms = 0.f;
    SHP_HIP(hipEventElapsedTime(&ms, f.ev[k], f.ev[k + 1]));
    f.flushed_ms += ms;
  }
  f.pool.insert(f.pool.end(), f.ev.begin(), f.ev.end());
  f.ev.clear();
}

hipEvent_t take(Family& f) {
  if (f.pool.empty()) {
    hipEvent_t e;
    SHP_HIP(hipEventCreate(&e));
    return e;
  }
  hipEvent_t e = f.pool.back();
  f.pool.pop_back();
  return e;
}
}  // namespace

bool probe_on(int fam) { return fam >= 0 && fam < kProbeFamilies && g_fam[fam].on; }

void probe_begin(int fam, hipStream_t s) {
  if (!probe_on(fam)) return;
  std::lock_guard<std::mutex> lk(g_mu);
  Family& f = g_fam[fam];
  if (f.ev.size() >= 4096) flush(f);
  hipEvent_t e = take(f);
  SHP_HIP(hipEventRecord(e, s));
  f.ev.push_back(e);
}

void probe_end(int fam, hipStream_t s, double bytes) {
  if (!probe_on(fam)) return;
  std::lock_guard<std::mutex> lk(g_mu);
  Family& f = g_fam[fam];
  hipEvent_t e = take(f);
  SHP_HIP(hipEventRecord(e, s));
  f.ev.push_back(e);
  f.launches += 1;
  f.bytes += bytes;
}

void probe_add_bytes(int fam, double bytes) {
  if (!probe_on(fam)) return;
  std::lock_guard<std::mutex> lk(g_mu);
  g_fam[fam].bytes += bytes;
}

void probe_enable(int fam, bool on) {
  std::lock_guard<std::mutex> lk(g_mu);
  Family& f = g_fam[fam];
  flush(f);
  f.on = on;
  f.launches = 0;
  f.bytes = 0.0;
  f.flushed_ms = 0.0;
}

void probe_read(int fam, int64_t* launches, double* ms, double* bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  Family& f = g_fam[fam];
  flush(f);
  *launches = f.launches;
  *ms = f.flushed_ms;
  *bytes = f.bytes;
}

}  // namespace shp

extern "C" {

int shapley_probe_enable(int32_t family, int32_t on) {
  if (family < 0 || family >= shp::kProbeFamilies) {
    shp::set_last_error("unknown probe family");
    return SHAPLEY_EINVAL;
  }
  try {
    shp::probe_enable(family, on != 0);
  } catch (const shp::Error& e) {
    shp::set_last_error(e.what());
    return e.code;
  }
  return SHAPLEY_OK;
}

int shapley_probe_read(int32_t family, int64_t* launches, double* total_ms, double* total_bytes) {
  if (family < 0 || family >= shp::kProbeFamilies || !launches || !total_ms || !total_bytes) {
    shp::set_last_error("bad probe arguments");
    return SHAPLEY_EINVAL;
  }
  try {
    shp::probe_read(family, launches, total_ms, total_bytes);
  } catch (const shp::Error& e) {
    shp::set_last_error(e.what());
    return e.code;
  }
  return SHAPLEY_OK;
}

}  // extern "C"

// Kernel timing probe: when enabled for a kernel family, every launch of that
// family is bracketed by HIP events recorded on the launch stream, and the
// algorithmic bytes the launch must move are accumulated.  Reading the probe
// synchronises on the recorded events and returns launches, total device
// time and total algorithmic bytes, over all launches or over the largest
// ones (by algorithmic bytes: the launches on the finest level).
#include "probe.hpp"

#include <algorithm>
#include <mutex>

namespace shp {

namespace {
// per-launch records kept for the largest-launch totals (beyond this many,
// only the totals over all launches are kept)
constexpr size_t kMaxRecords = size_t(1) << 20;

struct Launch {
  double bytes;
  double ms;
};

struct Family {
  bool on = false;
  std::vector<hipEvent_t> ev;   // start/stop pairs recorded since the last flush
  std::vector<double> ev_bytes; // algorithmic bytes of each pair in ev
  std::vector<hipEvent_t> pool; // created events ready for reuse
  std::vector<Launch> rec;      // flushed launches
  bool rec_full = false;        // rec stopped at kMaxRecords
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
    if (f.rec.size() < kMaxRecords)
      f.rec.push_back({f.ev_bytes[k / 2], double(ms)});
    else
      f.rec_full = true;
  }
  f.pool.insert(f.pool.end(), f.ev.begin(), f.ev.end());
  f.ev.clear();
  f.ev_bytes.clear();
}

hipEvent_t take(Family& f) {
  if (f.pool.empty()) {
    // timing only: no system-scope fence (no cache writeback and invalidation
    // at each record, which would slow the work being timed)
    hipEvent_t e;
    SHP_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
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
  f.ev_bytes.push_back(bytes);
  f.launches += 1;
  f.bytes += bytes;
}

void probe_add_bytes(int fam, double bytes) {
  if (!probe_on(fam)) return;
  std::lock_guard<std::mutex> lk(g_mu);
  Family& f = g_fam[fam];
  f.bytes += bytes;
  // the bytes belong to the last launch of the family
  if (!f.ev_bytes.empty())
    f.ev_bytes.back() += bytes;
  else if (!f.rec.empty())
    f.rec.back().bytes += bytes;
}

void probe_enable(int fam, bool on) {
  std::lock_guard<std::mutex> lk(g_mu);
  Family& f = g_fam[fam];
  flush(f);
  f.on = on;
  f.rec.clear();
  f.rec_full = false;
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

bool probe_read_large(int fam, double frac, int64_t* launches, double* ms, double* bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  Family& f = g_fam[fam];
  flush(f);
  if (f.rec_full) return false;
  double top = 0.0;
  for (const Launch& r : f.rec) top = std::max(top, r.bytes);
  *launches = 0;
  *ms = 0.0;
  *bytes = 0.0;
  for (const Launch& r : f.rec)
    if (r.bytes >= frac * top && r.bytes > 0.0) {
      *launches += 1;
      *ms += r.ms;
      *bytes += r.bytes;
    }
  return true;
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

int shapley_probe_read_large(int32_t family, double frac, int64_t* launches, double* total_ms,
                             double* total_bytes) {
  if (family < 0 || family >= shp::kProbeFamilies || !launches || !total_ms || !total_bytes ||
      !(frac > 0.0 && frac <= 1.0)) {
    shp::set_last_error("bad probe arguments");
    return SHAPLEY_EINVAL;
  }
  try {
    if (!shp::probe_read_large(family, frac, launches, total_ms, total_bytes)) {
      shp::set_last_error("too many probed launches to keep per-launch records; read the totals");
      return SHAPLEY_ENOMEM;
    }
  } catch (const shp::Error& e) {
    shp::set_last_error(e.what());
    return e.code;
  }
  return SHAPLEY_OK;
}

}  // extern "C"

// Kernel timing probe (see probe.hip).
#pragma once

#include "internal.hpp"

namespace shp {

// kernel families (values of the C ABI's SHAPLEY_PROBE_* constants)
enum {
  kProbeSmooth = 0,   // weighted-Jacobi relaxation, all levels
  kProbeResid64 = 1,  // FP64 residual of the refinement (finest level)
  kProbeImprove = 2,  // policy improvement + Shapley residual
  kProbeResid = 3,    // cycle residual, all levels
  kProbeRestrict = 4,
  kProbeProlong = 5,
  kProbeRap = 6,
  kProbeInterp = 7,
  kProbeTail = 8,     // V-cycle tail (coarse levels of a game in one workgroup)
  kProbeFamilies = 9
};

bool probe_on(int fam);
void probe_begin(int fam, hipStream_t s);
void probe_end(int fam, hipStream_t s, double bytes);
// bytes of a launch known only after it ran (a launch that loops on the device)
void probe_add_bytes(int fam, double bytes);
void probe_enable(int fam, bool on);
void probe_read(int fam, int64_t* launches, double* ms, double* bytes);
// totals over the launches whose algorithmic bytes are >= frac x the largest
// launch's; false when the per-launch records overflowed
bool probe_read_large(int fam, double frac, int64_t* launches, double* ms, double* bytes);

}  // namespace shp

// The Shapley operator with no allocation: for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, harnesses
// that forbid it).  The reductions of the sweep (max |F(v) - v| and the sum of
// squares) fold into a fixed device array of this file instead of buffers the
// library allocates; the work list of the sweep is computed from the block
// index; the game descriptor travels as a kernel argument.
#include "internal.hpp"

#include <mutex>

namespace shp {

namespace {

// Fixed device scratch of the allocation-free entry point: the stripes of the
// per-call reductions (kStripes copies of 4 values for one game padded to 4,
// doubles then ints) and the two results.  Its size does not depend on the
// game: any n is accepted.  Each device holds its own copy until the process
// ends; every call on a device shares it, so calls that overlap on one device
// race (the caller orders them on one stream or synchronises between them).
constexpr size_t kStripeVals = (size_t)kStripes * 4 * 4;
constexpr size_t kScratchBytes = kStripeVals * sizeof(double) + kStripeVals * sizeof(int) + 2 * sizeof(double);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device

// The device address of this device's copy of the array (looked up once per
// device, with the device current).  The array's name is a host-side stand-in
// in host code: only the address returned here reaches kernels.
unsigned char* scratch_of_current_device() {
  int dev = 0;
  SHP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error(SHAPLEY_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error(SHAPLEY_EDEVICE, std::string("hipGetSymbolAddress of the scratch array failed: ") +
                                       hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  return static_cast<unsigned char*>(g_scratch[dev]);
}

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

}  // namespace shp

using namespace shp;

extern "C" int shapley_apply_operator_noalloc(shapley_game_t gh, const double* v, double* F, int32_t* alpha,
                                              int32_t* beta, double* res, void* stream) {
  try {
    if (!gh || !gh->g || !v) throw Error(SHAPLEY_EINVAL, "null argument");
    if (!alpha || !beta) throw Error(SHAPLEY_EINVAL, "alpha and beta outputs are required");
    Game* g = gh->g->finest();
    if ((int64_t)g->n > INT32_MAX / 2) throw Error(SHAPLEY_EINVAL, "game too large");
    hipStream_t s = stream ? (hipStream_t)stream : g->stream;
    unsigned char* base = scratch_of_current_device();
    double* sd = reinterpret_cast<double*>(base);
    int* si = reinterpret_cast<int*>(base + kStripeVals * sizeof(double));
    double* out = reinterpret_cast<double*>(base + kStripeVals * (sizeof(double) + sizeof(int)));
    // the stripes must start at zero: cleared by fill kernels on the stream
    // (a previous call leaves them cleared, an interrupted one might not)
    fill_async(sd, 0.0, kStripeVals, s);
    fill_async(si, 0, kStripeVals, s);
    GameDesc d{};
    d.rp = g->rp.p; d.ci = g->ci.p; d.w = g->w.p; d.r = g->r.p; d.valid = g->valid.p;
    d.urp = g->urp.p; d.uci = g->uci.p;
    d.v = const_cast<double*>(v);
    d.alpha = nullptr;   // no incumbents: the greedy strategies
    d.beta = nullptr;
    d.beta_in = nullptr;
    d.alpha_c = alpha;
    d.beta_c = beta;
    d.F = F;
    d.bvals = nullptr;
    d.n = g->n; d.m1 = g->m1; d.m2 = g->m2; d.slot = 0; d.mu = g->mu;
    d.x_off = 0; d.a_off = 0;
    const Stripes st{sd, si, stripe_games(1)};
    launch_improve_flat(d, 0.0, st, s);
    launch_fold_finish(st, 1, 2, 2u, 0, res ? res : out, 2, nullptr, 0, s);
    return SHAPLEY_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return SHAPLEY_EDEVICE;
  }
}

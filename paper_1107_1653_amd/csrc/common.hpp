// Internal helpers shared by the HIP translation units of libshapley.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <atomic>
#include <string>
#include <vector>

namespace shp {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

#define SHP_HIP(call)                                                              \
  do {                                                                             \
    hipError_t _e = (call);                                                        \
    if (_e != hipSuccess)                                                          \
      throw ::shp::Error(SHAPLEY_EDEVICE, std::string("HIP error: ") +             \
                                              hipGetErrorString(_e) + " at " +     \
                                              __FILE__ + ":" + std::to_string(__LINE__)); \
  } while (0)

#define SHP_LAUNCH_CHECK() SHP_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------

// Fault injection for tests of the error paths: when armed with k > 0, the
// k-th device allocation from then on fails (shapley_debug_fail_alloc).
extern std::atomic<long long> g_alloc_fault;
inline bool alloc_fault_due() {
  long long k = g_alloc_fault.load(std::memory_order_relaxed);
  while (k > 0) {
    if (g_alloc_fault.compare_exchange_weak(k, k - 1, std::memory_order_relaxed)) return k == 1;
  }
  return false;
}

// Owning device allocation (hipMalloc / hipFree), movable, not copyable.
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  explicit DBuf(size_t count) { alloc(count); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DBuf() { release(); }
  void alloc(size_t count) {
    release();
    n = count;
    if (count) {
      if (alloc_fault_due()) {
        n = 0;
        throw Error(SHAPLEY_ENOMEM, "device allocation failed (injected by shapley_debug_fail_alloc)");
      }
      hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(T));
      if (e != hipSuccess) {
        p = nullptr; n = 0;
        throw Error(SHAPLEY_ENOMEM, std::string("device allocation of ") +
                                        std::to_string(count * sizeof(T)) + " bytes failed");
      }
    }
  }
  // grow-only reallocation (contents not preserved)
  void ensure(size_t count) { if (count > n) alloc(count); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr; n = 0;
  }
  size_t bytes() const { return n * sizeof(T); }
};

template <class T>
inline void h2d(T* dst, const T* src, size_t count, hipStream_t s) {
  if (count) SHP_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, s));
}
template <class T>
inline void d2h(T* dst, const T* src, size_t count, hipStream_t s) {
  if (count) SHP_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyDeviceToHost, s));
}
template <class T>
inline void d2d(T* dst, const T* src, size_t count, hipStream_t s) {
  if (count) SHP_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyDeviceToDevice, s));
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t work, int per_block = kBlock) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > 0x7fffffff) throw Error(SHAPLEY_EINVAL, "launch grid too large");
  return static_cast<unsigned>(g);
}

// Row range [r0, r1) of one game inside a merged (block-diagonal) level.
struct Tile {
  int r0, r1, game;
};

// Builds tiles of at most `rows` rows that never straddle a game boundary.
// off has G+1 entries (prefix offsets); only games with keep[g] != 0 are tiled.
std::vector<Tile> make_tiles(const std::vector<int>& off, const std::vector<char>& keep, int rows);

// ---------------------------------------------------------------------------
// device-side helpers
// ---------------------------------------------------------------------------

// atomic max of a non-negative double (the IEEE bit pattern orders like the value)
__device__ inline void atomic_max_nonneg(double* addr, double v) {
  if (!(v >= 0.0)) v = __longlong_as_double(0x7ff8000000000000LL);  // NaN propagates as max
  atomicMax(reinterpret_cast<unsigned long long*>(addr),
            static_cast<unsigned long long>(__double_as_longlong(v)));
}

// Device fill by a kernel: on this runtime a memset call costs tens of
// microseconds of queue time, a kernel launch a few.
template <class T>
__global__ void k_fill(T* __restrict__ p, T v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
// Workgroups of a launch are dispatched to the 8 XCDs in turn (workgroup b
// runs on XCD b mod 8, and each XCD has its own L2).  The logical index
// gives each XCD one contiguous range of workgroups, so workgroups whose rows
// gather the same neighbours share an L2.  A bijection of [0, gridDim.x).
// Used by the setup's gather-bound kernels (interpolation, Galerkin
// product); the streaming cycle kernels measured faster with the plain
// order, whose concurrent workgroups on the eight XCDs read adjacent memory.
__device__ __forceinline__ unsigned xcd_block() {
  const unsigned n = gridDim.x, b = blockIdx.x;
  if (n < 16) return b;
  const unsigned per = n >> 3, rem = n & 7u, x = b & 7u;
  return x * per + (x < rem ? x : rem) + (b >> 3);
}

// up to four counters set to zero by one launch (null pointers skipped)
template <class T>
__global__ void k_zero4(T* a, T* b, T* c, T* d) {
  if (threadIdx.x == 0) {
    if (a) *a = 0;
    if (b) *b = 0;
    if (c) *c = 0;
    if (d) *d = 0;
  }
}
inline void zero_counters_async(hipStream_t s, int* a, int* b = nullptr, int* c = nullptr, int* d = nullptr) {
  hipLaunchKernelGGL(k_zero4<int>, dim3(1), dim3(64), 0, s, a, b, c, d);
  SHP_LAUNCH_CHECK();
}
template <class T>
inline void fill_async(T* p, T v, size_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, p, v, n);
  SHP_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Striped per-game reductions.  Thousands of workgroups folding a value into
// one address serialise on that address (device-scope atomics); instead each
// 256-thread workgroup combines its four wavefronts in LDS and folds the
// result into one of kStripes copies (workgroup index mod kStripes).  A
// finishing pass combines the copies per game, writes the result and clears
// the copies for the next use.  Layout: [stripe][game (padded to 4)][4].
// Maxima are of non-negative values; a NaN must be mapped to +inf by the
// caller so that it survives the max.
// ---------------------------------------------------------------------------
constexpr int kStripes = 64;
inline int stripe_games(int G) { return ((G > 1 ? G : 1) + 3) & ~3; }
struct Stripes {
  double* d;
  int* i;
  int gp;  // padded game count
};
__host__ __device__ inline size_t stripe_at(const Stripes& st, int stripe, int g, int q) {
  return ((size_t)stripe * st.gp + g) * 4 + q;
}

// Every thread of the (256-thread) workgroup must call this; vd/vi hold the
// values already reduced within each wavefront (lane 0's copy is used).
// Bit q of sum_mask selects a sum for double quantity q, else a maximum.
template <int ND, int NI>
__device__ inline void block_fold(const Stripes& st, int g, const double* vd, unsigned sum_mask,
                                  const int* vi) {
  __shared__ double sd[4][ND > 0 ? ND : 1];
  __shared__ int si[4][NI > 0 ? NI : 1];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    for (int q = 0; q < ND; ++q) sd[w][q] = vd[q];
    for (int q = 0; q < NI; ++q) si[w][q] = vi[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    const int s = blockIdx.x % kStripes;
    for (int q = 0; q < ND; ++q) {
      const bool sum = (sum_mask >> q) & 1u;
      double v = sd[0][q];
      for (int k = 1; k < nw; ++k) v = sum ? v + sd[k][q] : fmax(v, sd[k][q]);
      if (v != 0.0) {
        double* a = st.d + stripe_at(st, s, g, q);
        if (sum) atomicAdd(a, v); else atomic_max_nonneg(a, v);
      }
    }
    for (int q = 0; q < NI; ++q) {
      int v = si[0][q];
      for (int k = 1; k < nw; ++k) v += si[k][q];
      if (v) atomicAdd(st.i + stripe_at(st, s, g, q), v);
    }
  }
}

// 32-bit bijective mixer (murmur3 finaliser) -- deterministic PMIS weights
__host__ __device__ inline uint32_t mix32(uint32_t x) {
  x ^= x >> 16; x *= 0x85ebca6bu;
  x ^= x >> 13; x *= 0xc2b2ae35u;
  x ^= x >> 16;
  return x;
}

}  // namespace shp

// Internal helpers shared by the HIP translation units of libshapley.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <stdexcept>
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

// 32-bit bijective mixer (murmur3 finaliser) -- deterministic PMIS weights
__host__ __device__ inline uint32_t mix32(uint32_t x) {
  x ^= x >> 16; x *= 0x85ebca6bu;
  x ^= x >> 13; x *= 0xc2b2ae35u;
  x ^= x >> 16;
  return x;
}

}  // namespace shp

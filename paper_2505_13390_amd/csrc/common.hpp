// Shared host/device utilities of the MGPBD HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mgpbd.h"

namespace mgpbd {

struct Error : std::runtime_error {
  int status;
  Error(int s, const std::string &m) : std::runtime_error(m), status(s) {}
};

#define MG_HIP(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      throw ::mgpbd::Error(MGPBD_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define MG_REQUIRE(cond, status, msg)                  \
  do {                                                 \
    if (!(cond)) throw ::mgpbd::Error((status), (msg)); \
  } while (0)

constexpr int kWave = 64;
constexpr int kBlock = 256;        // threads per block for streaming kernels
constexpr int kMaxGrid = 2048;     // blocks of a streaming kernel (8 per CU on 256 CUs)
constexpr int kNumXcd = 8;         // MI355X: 8 XCDs, blocks are dealt round-robin
// Most partial sums one block of a reduction writes (partials[k * grid + block],
// k < kMaxBlockSums); the shared partials buffer holds this many per block.
constexpr int kMaxBlockSums = 3;

// Owning device buffer.
template <class T>
struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  // (re)allocate exactly n elements; contents undefined
  void alloc(size_t count) {
    if (count == n && p) return;
    release();
    size_t bytes = (count ? count : 1) * sizeof(T);
    hipError_t e = hipMalloc((void **)&p, bytes);
    if (e != hipSuccess) {
      p = nullptr;
      throw Error(MGPBD_E_OUT_OF_MEMORY,
                  "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    }
    n = count;
  }
  // grow-only allocation
  void reserve(size_t count) {
    if (count > n || !p) alloc(count);
  }
  T *get() const { return p; }
  void upload(const T *h, size_t count, hipStream_t s) {
    alloc(count);
    if (count) MG_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
  }
  void download(T *h, size_t count, hipStream_t s) const {
    if (count) MG_HIP(hipMemcpyAsync(h, p, count * sizeof(T), hipMemcpyDeviceToHost, s));
  }
};

// ------------------------------------------------------------------
// Counter-based random numbers: SplitMix64 (Steele, Lea, Flood 2014).
// mix64(seed, stream, i) = splitmix64(splitmix64(seed << 8 | stream) + i).
// ------------------------------------------------------------------
__host__ __device__ inline uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t stream_salt(uint64_t seed, uint64_t stream) {
  return splitmix64((seed << 8) | stream);
}
__host__ __device__ inline uint64_t mix64_salted(uint64_t salt, uint64_t i) {
  return splitmix64(salt + i);
}
// open-interval uniform in (0, 1): (top 53 bits + 0.5) * 2^-53
__host__ __device__ inline double uniform_open(uint64_t h) {
  return ((double)(h >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}
// visiting priority: high 32 bits random, low 32 bits the index (distinct keys)
__host__ __device__ inline uint64_t prio_key(uint64_t salt, int level, int64_t i) {
  uint64_t h = mix64_salted(salt, ((uint64_t)level << 40) + (uint64_t)i);
  return (h & 0xFFFFFFFF00000000ULL) | (uint64_t)(uint32_t)i;
}

// Random streams drawn by the solver itself.
enum Stream : uint64_t { kStreamNearKernel = 2, kStreamAggPrio = 3, kStreamColorPrio = 4,
                         kStreamPowerStart = 5 };

inline int grid_for(int64_t work_items, int per_block) {
  int64_t g = (work_items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > kMaxGrid) g = kMaxGrid;
  return (int)g;
}
inline unsigned blocks_for(int64_t work_items, int per_block) {
  int64_t g = (work_items + per_block - 1) / per_block;
  return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace mgpbd

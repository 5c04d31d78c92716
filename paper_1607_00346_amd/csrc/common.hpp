// Shared host-side plumbing of the HIF library: status handling, device
// buffers with high-water accounting, launch checks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <atomic>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hif.h"

namespace hif {

// An error that crosses the ABI as a status code plus a thread-local message.
struct Error : std::runtime_error {
  hif_status status;
  Error(hif_status s, const std::string& msg) : std::runtime_error(msg), status(s) {}
};

void set_last_error(const std::string& msg);

#define HIF_HIP(call)                                                                 \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      throw ::hif::Error(e_ == hipErrorOutOfMemory ? HIF_ENOMEM : HIF_EDEVICE,        \
                         std::string(#call) + ": " + hipGetErrorString(e_));          \
    }                                                                                 \
  } while (0)

#define HIF_LAUNCH_CHECK() HIF_HIP(hipGetLastError())

#define HIF_REQUIRE(cond, status, msg)                          \
  do {                                                          \
    if (!(cond)) throw ::hif::Error((status), (msg));           \
  } while (0)

// Bytes of device memory held by the library (per process) and their peak.
struct MemStats {
  std::atomic<int64_t> live{0};
  std::atomic<int64_t> peak{0};
};
MemStats& mem_stats();

// Device memory with a best-fit cache: a released block is kept for reuse by a
// later allocation that fits in it with at most a quarter of the request (or
// 2 MiB) to spare (repeated builds of one problem then allocate nothing new).  The cache holds
// at most three quarters of the device's memory (at least kPoolCap bytes); a
// release that would overflow it first frees the largest cached blocks (a
// quarter of the cap at once, after one device synchronization).
//
// Reuse is stream ordered: a block released while a StreamScope for stream s
// is active on this thread is handed out again, without any synchronization,
// to an allocation made under a scope for the same s (later work on s runs
// after the work that used the block).  Blocks released outside any scope are
// reused after a device synchronization; blocks wanted by another stream only
// when a fresh allocation fails (a device-wide wait would stall that stream).
constexpr int64_t kPoolCap = int64_t(48) << 30;

// Smallest eps > 0 accepted: the ID's rank test on the FP64 Gram diagonal
// needs eps^2 well above the FP64 unit roundoff.
constexpr double kEpsMin = 1e-7;
void* pool_alloc(size_t bytes);
void pool_free(void* p, size_t bytes);
// Returns every cached block to the device (after a device synchronization).
void pool_release_cached();
size_t pool_round(size_t bytes);

// The stream that all device work of the current library call is ordered on.
class StreamScope {
 public:
  explicit StreamScope(hipStream_t s);
  ~StreamScope();
  StreamScope(const StreamScope&) = delete;
  StreamScope& operator=(const StreamScope&) = delete;

 private:
  hipStream_t prev_;
  bool prev_set_;
};

// Pinned host memory through which uploads are staged, so that an upload
// enqueued behind running kernels does not wait for them (a copy from pageable
// memory does).  While a Staging object is alive on this thread, upload_bytes
// on its stream copies the source into pinned chunks and returns at once.  The
// chunks are rewound by synced() (the stream has been synchronized, so every
// staged copy is complete) and returned to a process-wide cache by the
// destructor, which synchronizes the stream first.
class Staging {
 public:
  explicit Staging(hipStream_t s);
  ~Staging();
  Staging(const Staging&) = delete;
  Staging& operator=(const Staging&) = delete;
  void copy(void* dst, const void* src, size_t bytes);
  void synced();
  hipStream_t stream() const { return s_; }

 private:
  struct Chunk {
    char* p;
    size_t cap, used;
  };
  hipStream_t s_;
  Staging* prev_;
  std::vector<Chunk> chunks_;
};

// Host-to-device copy of `bytes` ordered on stream s; the source may be reused
// as soon as the call returns.
void upload_bytes(void* dst, const void* src, size_t bytes, hipStream_t s);

// Stream s has just been synchronized: rewind this thread's staging for s.
void staging_synced(hipStream_t s);

// Owning device allocation.  Move-only; frees on destruction.
template <typename T>
class DevBuf {
 public:
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p_(o.p_), n_(o.n_) { o.p_ = nullptr; o.n_ = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p_ = o.p_; n_ = o.n_; o.p_ = nullptr; o.n_ = 0; }
    return *this;
  }
  ~DevBuf() { release(); }

  void alloc(size_t count) {
    release();
    if (count == 0) return;
    p_ = static_cast<T*>(pool_alloc(count * sizeof(T)));
    n_ = count;
    auto& ms = mem_stats();
    const int64_t now = ms.live.fetch_add((int64_t)(count * sizeof(T))) + (int64_t)(count * sizeof(T));
    int64_t pk = ms.peak.load();
    while (now > pk && !ms.peak.compare_exchange_weak(pk, now)) {
    }
  }
  void release() {
    if (p_) {
      pool_free(p_, n_ * sizeof(T));
      mem_stats().live -= (int64_t)(n_ * sizeof(T));
    }
    p_ = nullptr;
    n_ = 0;
  }
  T* get() const { return p_; }
  size_t size() const { return n_; }
  size_t bytes() const { return n_ * sizeof(T); }

  void upload(const std::vector<T>& h, hipStream_t s) {
    if (h.size() != n_) alloc(h.size());
    if (n_) upload_bytes(p_, h.data(), n_ * sizeof(T), s);
  }
  void download(std::vector<T>& h, hipStream_t s) const {
    h.resize(n_);
    if (n_) HIF_HIP(hipMemcpyAsync(h.data(), p_, n_ * sizeof(T), hipMemcpyDeviceToHost, s));
  }

 private:
  T* p_ = nullptr;
  size_t n_ = 0;
};

// Pointers that came out of memory (batch descriptors) are generic to the
// compiler, which then emits flat accesses; flat loads also count against the
// LDS wait counter, so waiting for LDS operands would wait for the prefetch
// of the next chunk too.  These casts declare them global.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* as_global(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* as_global(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// Element at a 32-bit byte offset from a wave-uniform global base: the base
// stays in scalar registers, the offset in one vector register.
template <typename T>
__device__ __forceinline__ T load_global(const T* base, uint32_t off) {
  return *(const __attribute__((address_space(1))) T*)((const char*)base + off);
}

// Device array whose storage may be shared (the level-0 index arrays of a
// problem are uploaded once and shared by every factor built from it).
template <typename V>
struct DevArr {
  std::shared_ptr<DevBuf<V>> buf;
  V* get() const { return buf ? buf->get() : nullptr; }
  size_t size() const { return buf ? buf->size() : 0; }
};

template <typename V>
DevArr<V> dev_arr(const std::vector<V>& h, hipStream_t s) {
  DevArr<V> a;
  a.buf = std::make_shared<DevBuf<V>>();
  a.buf->upload(h, s);
  return a;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int pad_ld(int rows) { return rows < 1 ? 1 : (int)(ceil_div(rows, 4) * 4); }

}  // namespace hif

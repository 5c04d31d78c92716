// Shared host-side plumbing of the HIF library: status handling, device
// buffers with high-water accounting, launch checks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
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
  int64_t live = 0;
  int64_t peak = 0;
};
MemStats& mem_stats();

// Device memory with a size-exact cache: released blocks are kept for reuse by
// a later allocation of the same rounded size (repeated builds of one problem
// then allocate nothing new).  The cache holds at most kPoolCap bytes.
constexpr int64_t kPoolCap = int64_t(48) << 30;
void* pool_alloc(size_t bytes);
void pool_free(void* p, size_t bytes);
size_t pool_round(size_t bytes);

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
    ms.live += (int64_t)(count * sizeof(T));
    if (ms.live > ms.peak) ms.peak = ms.live;
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
    if (n_) HIF_HIP(hipMemcpyAsync(p_, h.data(), n_ * sizeof(T), hipMemcpyHostToDevice, s));
  }
  void download(std::vector<T>& h, hipStream_t s) const {
    h.resize(n_);
    if (n_) HIF_HIP(hipMemcpyAsync(h.data(), p_, n_ * sizeof(T), hipMemcpyDeviceToHost, s));
  }

 private:
  T* p_ = nullptr;
  size_t n_ = 0;
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int pad_ld(int rows) { return rows < 1 ? 1 : (int)(ceil_div(rows, 4) * 4); }

}  // namespace hif

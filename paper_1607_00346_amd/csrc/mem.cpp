// Device memory cache with stream-ordered reuse, and pinned staging of uploads.
#include <algorithm>
#include <cstring>
#include <iterator>
#include <map>
#include <unordered_map>
#include <mutex>

#include "common.hpp"

namespace hif {

namespace {

thread_local hipStream_t t_stream = nullptr;
thread_local bool t_stream_set = false;
thread_local Staging* t_staging = nullptr;

enum class Tag { kClean, kStream, kUnknown };

struct Block {
  void* p;
  Tag tag;
  hipStream_t s;  // valid for Tag::kStream
};

struct Pool {
  std::mutex mu;
  std::multimap<size_t, Block> free_blocks;  // keyed by block size
  std::unordered_map<void*, size_t> live;    // size of every block handed out
  int64_t cached = 0;
  ~Pool() {
    for (auto& kv : free_blocks) (void)hipFree(kv.second.p);
  }
};

Pool& pool() {
  static Pool p;
  return p;
}

// Pinned chunks kept between library calls.
constexpr size_t kChunk = size_t(32) << 20;
constexpr size_t kPinCacheCap = size_t(1) << 30;

struct PinCache {
  std::mutex mu;
  std::multimap<size_t, char*> chunks;
  size_t total = 0;
  ~PinCache() {
    for (auto& kv : chunks) (void)hipHostFree(kv.second);
  }
};

PinCache& pin_cache() {
  static PinCache c;
  return c;
}

}  // namespace

size_t pool_round(size_t bytes) {
  const size_t g = bytes >= (size_t(1) << 20) ? (size_t(2) << 20) : 256;
  return (bytes + g - 1) / g * g;
}

namespace {

// Frees cached blocks, largest first, until at least `target` bytes are gone
// (after one device synchronization, so no freed block is still in use).
void trim_locked(Pool& P, int64_t target) {
  (void)hipDeviceSynchronize();
  int64_t freed = 0;
  while (freed < target && !P.free_blocks.empty()) {
    auto it = std::prev(P.free_blocks.end());
    (void)hipFree(it->second.p);
    freed += (int64_t)it->first;
    P.cached -= (int64_t)it->first;
    P.free_blocks.erase(it);
  }
  for (auto& kv : P.free_blocks) kv.second.tag = Tag::kClean;
}

// The cache's cap: three quarters of the device's memory (at least
// kPoolCap).  A joint build of many problems frees tens of GB of
// temporaries and factors between its levels and calls; a cap below that
// volume made releases trim (a device synchronization and hipFree calls in
// the middle of a level) and the next level allocate afresh.  An allocation
// that finds the device full still empties the cache and retries.
int64_t pool_cap() {
  static const int64_t cap = [] {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      (void)hipGetLastError();
      return kPoolCap;
    }
    return std::max<int64_t>(kPoolCap, (int64_t)(total_b / 4 * 3));
  }();
  return cap;
}

}  // namespace

void* pool_alloc(size_t bytes) {
  const size_t r = pool_round(bytes);
  // best fit among cached blocks at most a quarter (or 2 MiB) larger
  const size_t slack = std::max(r / 4, size_t(2) << 20);
  Pool& P = pool();
  std::lock_guard<std::mutex> lock(P.mu);
  auto lo = P.free_blocks.lower_bound(r);
  auto hi = P.free_blocks.upper_bound(r + slack);
  auto take = P.free_blocks.end();
  for (auto it = lo; it != hi; ++it) {
    const Block& b = it->second;
    if (b.tag == Tag::kClean || (b.tag == Tag::kStream && t_stream_set && b.s == t_stream)) {
      take = it;
      break;
    }
  }
  if (take == P.free_blocks.end() && lo != hi) {
    // Only blocks that other streams or unknown work (a release outside any
    // call) may still use.  Blocks of other streams: allocate afresh if the
    // device has room, since a wait for the device would stall the other
    // streams.  Otherwise (or without room) wait for the device, after which
    // every cached block is free for anyone.
    bool unknown = false;
    for (auto it = lo; it != hi; ++it) unknown = unknown || it->second.tag == Tag::kUnknown;
    if (!unknown) {
      void* p = nullptr;
      if (hipMalloc(&p, r) == hipSuccess) {
        P.live[p] = r;
        return p;
      }
      (void)hipGetLastError();
    }
    HIF_HIP(hipDeviceSynchronize());
    for (auto& kv : P.free_blocks) kv.second.tag = Tag::kClean;
    take = lo;
  }
  if (take != P.free_blocks.end()) {
    void* p = take->second.p;
    const size_t sz = take->first;
    P.free_blocks.erase(take);
    P.cached -= (int64_t)sz;
    P.live[p] = sz;
    return p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, r);
  if (e == hipErrorOutOfMemory && !P.free_blocks.empty()) {
    (void)hipGetLastError();
    trim_locked(P, P.cached);
    e = hipMalloc(&p, r);
  }
  if (e != hipSuccess)
    throw Error(e == hipErrorOutOfMemory ? HIF_ENOMEM : HIF_EDEVICE,
                std::string("hipMalloc: ") + hipGetErrorString(e));
  P.live[p] = r;
  return p;
}

void pool_release_cached() {
  Pool& P = pool();
  std::lock_guard<std::mutex> lock(P.mu);
  trim_locked(P, P.cached);
}

void pool_free(void* p, size_t bytes) {
  Pool& P = pool();
  std::lock_guard<std::mutex> lock(P.mu);
  size_t sz = pool_round(bytes);
  auto it = P.live.find(p);
  if (it != P.live.end()) {
    sz = it->second;
    P.live.erase(it);
  }
  const int64_t cap = pool_cap();
  if (P.cached + (int64_t)sz > cap) {
    // make room for a quarter of the cache at once, so that a build that
    // overflows it synchronizes once rather than at every release
    trim_locked(P, P.cached + (int64_t)sz - cap + cap / 4);
  }
  Block b{p, t_stream_set ? Tag::kStream : Tag::kUnknown, t_stream};
  P.free_blocks.emplace(sz, b);
  P.cached += (int64_t)sz;
}

StreamScope::StreamScope(hipStream_t s) : prev_(t_stream), prev_set_(t_stream_set) {
  t_stream = s;
  t_stream_set = true;
}

StreamScope::~StreamScope() {
  t_stream = prev_;
  t_stream_set = prev_set_;
}

Staging::Staging(hipStream_t s) : s_(s), prev_(t_staging) { t_staging = this; }

Staging::~Staging() {
  (void)hipStreamSynchronize(s_);
  t_staging = prev_;
  PinCache& C = pin_cache();
  std::lock_guard<std::mutex> lock(C.mu);
  for (const Chunk& c : chunks_) {
    if (C.total + c.cap > kPinCacheCap) {
      (void)hipHostFree(c.p);
    } else {
      C.chunks.emplace(c.cap, c.p);
      C.total += c.cap;
    }
  }
}

void Staging::copy(void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return;
  const size_t need = (bytes + 255) / 256 * 256;
  Chunk* c = nullptr;
  for (Chunk& k : chunks_)
    if (k.cap - k.used >= need) {
      c = &k;
      break;
    }
  if (!c) {
    const size_t cap = std::max(kChunk, (need + kChunk - 1) / kChunk * kChunk);
    char* p = nullptr;
    {
      PinCache& C = pin_cache();
      std::lock_guard<std::mutex> lock(C.mu);
      auto it = C.chunks.lower_bound(cap);
      if (it != C.chunks.end()) {
        p = it->second;
        chunks_.push_back({p, it->first, 0});
        C.total -= it->first;
        C.chunks.erase(it);
      }
    }
    if (!p) {
      HIF_HIP(hipHostMalloc((void**)&p, cap, hipHostMallocDefault));
      chunks_.push_back({p, cap, 0});
    }
    c = &chunks_.back();
  }
  char* stage = c->p + c->used;
  std::memcpy(stage, src, bytes);
  c->used += need;
  HIF_HIP(hipMemcpyAsync(dst, stage, bytes, hipMemcpyHostToDevice, s_));
}

void Staging::synced() {
  for (Chunk& c : chunks_) c.used = 0;
}

void staging_synced(hipStream_t s) {
  if (t_staging && t_staging->stream() == s) t_staging->synced();
}

void upload_bytes(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  if (t_staging && t_staging->stream() == s) {
    t_staging->copy(dst, src, bytes);
    return;
  }
  HIF_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
  HIF_HIP(hipStreamSynchronize(s));  // the source belongs to the caller again
}

}  // namespace hif

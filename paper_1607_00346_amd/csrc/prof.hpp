// Per-kernel-class device timing with HIP events (off unless a caller asks
// for it through hif_profile_begin).  Each instrumented launch records an
// event pair on the stream it runs on, plus the launch's algorithmic flops and
// bytes.  Not thread safe: profile one thread's calls at a time.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

namespace hif {

class Profiler {
 public:
  struct Rec {
    int cls;
    hipEvent_t a, b;
    double flops, bytes;
  };
  bool on = false;
  // When non-empty, only kernel classes whose name (before any "@level")
  // equals one of these are recorded.
  std::vector<std::string> only;
  std::vector<std::string> names;
  std::vector<Rec> recs;

  int class_id(const char* name);
  bool selected(const char* name) const;
  hipEvent_t event();
  void recycle(hipEvent_t e) { pool_.push_back(e); }

 private:
  std::vector<hipEvent_t> pool_;
};

Profiler& profiler();

// The factorization level of the calling thread's launches, appended to class
// names as "@level" when >= 0.
int& prof_level();

// RAII: records a start event now and an end event when it goes out of scope.
class ProfScope {
 public:
  ProfScope(const char* name, hipStream_t s, double flops = 0.0, double bytes = 0.0);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  bool on_ = false;
  hipStream_t s_ = nullptr;
  Profiler::Rec rec_{};
};

}  // namespace hif

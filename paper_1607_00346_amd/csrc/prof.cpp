// Per-kernel-class event timing (see prof.hpp).
#include "prof.hpp"

#include <cstdio>
#include <cstring>

namespace hif {

Profiler& profiler() {
  static Profiler p;
  return p;
}

int& prof_level() {
  thread_local int level = -1;
  return level;
}

int Profiler::class_id(const char* name) {
  for (size_t i = 0; i < names.size(); ++i)
    if (names[i] == name) return (int)i;
  names.emplace_back(name);
  return (int)names.size() - 1;
}

bool Profiler::selected(const char* name) const {
  if (only.empty()) return true;
  for (const std::string& o : only)
    if (o == name) return true;
  return false;
}

hipEvent_t Profiler::event() {
  if (!pool_.empty()) {
    hipEvent_t e = pool_.back();
    pool_.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

ProfScope::ProfScope(const char* name, hipStream_t s, double flops, double bytes) {
  Profiler& p = profiler();
  if (!p.on || !p.selected(name)) return;
  if (prof_level() >= 0) {
    char buf[64];
    snprintf(buf, sizeof(buf), "%s@%d", name, prof_level());
    rec_.cls = p.class_id(buf);
  } else {
    rec_.cls = p.class_id(name);
  }
  rec_.a = p.event();
  rec_.b = p.event();
  rec_.flops = flops;
  rec_.bytes = bytes;
  if (!rec_.a || !rec_.b) return;
  s_ = s;
  on_ = hipEventRecord(rec_.a, s) == hipSuccess;
}

ProfScope::~ProfScope() {
  if (!on_) return;
  if (hipEventRecord(rec_.b, s_) == hipSuccess) profiler().recs.push_back(rec_);
}

}  // namespace hif

// extern "C" entry points of the HIF library: argument checks, status codes,
// thread-local error text.  No exception crosses this boundary.
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>

#include "hif_impl.hpp"
#include "prof.hpp"

namespace hif {

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string& msg) { g_last_error = msg; }

MemStats& mem_stats() {
  static MemStats ms;
  return ms;
}

}  // namespace hif

namespace {

template <typename Fn>
hif_status guarded(Fn&& fn) {
  try {
    hif::set_last_error("");
    fn();
    return HIF_OK;
  } catch (const hif::Error& e) {
    hif::set_last_error(e.what());
    return e.status;
  } catch (const std::bad_alloc&) {
    hif::set_last_error("host allocation failed");
    return HIF_ENOMEM;
  } catch (const std::exception& e) {
    hif::set_last_error(e.what());
    return HIF_EDEVICE;
  } catch (...) {
    hif::set_last_error("unknown error");
    return HIF_EDEVICE;
  }
}

void check_options(const hif_options* o) {
  HIF_REQUIRE(o != nullptr, HIF_EINVAL, "options must not be NULL");
  HIF_REQUIRE(o->n >= 2 && o->n <= 1024, HIF_EINVAL, "n must be in [2, 1024]");
  HIF_REQUIRE(hif::levels_for(o->n, o->leaf) >= 0, HIF_EINVAL,
              "n must equal leaf * 2^L with leaf >= 2");
  HIF_REQUIRE(std::isfinite(o->eps) && (o->eps == 0.0 || (o->eps >= hif::kEpsMin && o->eps < 1.0)),
              HIF_EINVAL, "eps must be 0 or in [1e-7, 1)");
  HIF_REQUIRE(o->precision == HIF_FP64 || o->precision == HIF_MIXED, HIF_EINVAL,
              "precision must be HIF_FP64 or HIF_MIXED");
  HIF_REQUIRE(o->bc == HIF_DIRICHLET || o->bc == HIF_PERIODIC, HIF_EINVAL,
              "bc must be HIF_DIRICHLET or HIF_PERIODIC");
  HIF_REQUIRE(o->bc != HIF_PERIODIC || o->n >= 4, HIF_EINVAL, "periodic grids need n >= 4");
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

extern "C" {

hif_status hif_problem_create(const hif_options* opts, const double* a, const double* b,
                              void* stream, hif_problem_t* out) {
  if (out) *out = nullptr;
  return guarded([&] {
    HIF_REQUIRE(out != nullptr, HIF_EINVAL, "out must not be NULL");
    check_options(opts);
    HIF_REQUIRE(a != nullptr && b != nullptr, HIF_EINVAL, "a and b must not be NULL");
    hif::StreamScope scope(as_stream(stream));
    auto* A = new hif_problem_s();
    try {
      A->opts = *opts;
      A->n = opts->n;
      A->N = (int64_t)opts->n * opts->n * opts->n;
      hif::problem_assemble(A, a, b, as_stream(stream));
    } catch (...) {
      delete A;
      throw;
    }
    *out = A;
  });
}

hif_status hif_build(hif_problem_t A, const hif_options* opts, void* stream, hif_factor_t* out) {
  if (out) *out = nullptr;
  return guarded([&] {
    HIF_REQUIRE(out != nullptr && A != nullptr, HIF_EINVAL, "NULL handle");
    check_options(opts);
    HIF_REQUIRE(opts->n == A->n && opts->bc == A->opts.bc, HIF_EINVAL,
                "options describe another grid than the problem");
    hif::StreamScope scope(as_stream(stream));
    hif::Staging staging(as_stream(stream));  // synchronizes the stream when the build ends
    auto* F = new hif_factor_s();
    try {
      F->opts = *opts;
      if (opts->precision == HIF_MIXED)
        hif::build_factor<float>(A, *opts, as_stream(stream), F);
      else
        hif::build_factor<double>(A, *opts, as_stream(stream), F);
    } catch (...) {
      (void)hipStreamSynchronize(as_stream(stream));
      delete F;
      throw;
    }
    *out = F;
  });
}

hif_status hif_build_batched(int32_t count, const hif_problem_t* A, const hif_options* opts,
                             void* stream, hif_factor_t* out) {
  if (out && count > 0)
    for (int32_t i = 0; i < count; ++i) out[i] = nullptr;
  return guarded([&] {
    HIF_REQUIRE(count >= 1, HIF_EINVAL, "count must be >= 1");
    HIF_REQUIRE(A != nullptr && opts != nullptr && out != nullptr, HIF_EINVAL, "NULL array");
    for (int32_t i = 0; i < count; ++i) {
      HIF_REQUIRE(A[i] != nullptr, HIF_EINVAL, "NULL problem handle");
      check_options(&opts[i]);
      HIF_REQUIRE(opts[i].n == A[i]->n && opts[i].bc == A[i]->opts.bc, HIF_EINVAL,
                  "options describe another grid than the problem");
      HIF_REQUIRE(opts[i].precision == opts[0].precision && opts[i].eps == opts[0].eps,
                  HIF_EINVAL, "the problems of a batch must share precision and eps");
    }
    hif::StreamScope scope(as_stream(stream));
    hif::Staging staging(as_stream(stream));  // synchronizes the stream when the build ends
    std::vector<std::unique_ptr<hif_factor_s>> F(count);
    std::vector<hif::BuildRequest> req(count);
    for (int32_t i = 0; i < count; ++i) {
      F[i].reset(new hif_factor_s());
      F[i]->opts = opts[i];
      req[i] = {A[i], opts[i], F[i].get()};
    }
    try {
      if (opts[0].precision == HIF_MIXED)
        hif::build_factors<float>(req, as_stream(stream));
      else
        hif::build_factors<double>(req, as_stream(stream));
    } catch (...) {
      (void)hipStreamSynchronize(as_stream(stream));
      throw;
    }
    for (int32_t i = 0; i < count; ++i) out[i] = F[i].release();
  });
}

hif_status hif_release_cached_memory(void) {
  return guarded([&] { hif::pool_release_cached(); });
}

hif_status hif_tune_begin(void) {
  return guarded([&] { hif::tune_begin(); });
}

hif_status hif_tune_end(const char* path, int32_t* keys) {
  return guarded([&] {
    const int n = hif::tune_end(path);
    if (keys) *keys = n;
  });
}

hif_status hif_apply(hif_factor_t F, const double* f, double* u, int32_t nrhs, void* stream) {
  return guarded([&] {
    HIF_REQUIRE(F != nullptr && F->impl, HIF_EINVAL, "NULL factor");
    HIF_REQUIRE(nrhs >= 0, HIF_EINVAL, "nrhs must be >= 0");
    if (nrhs == 0) return;
    HIF_REQUIRE(f != nullptr && u != nullptr, HIF_EINVAL, "NULL vector");
    const int64_t N = F->stats.n_dof;
    hif::StreamScope scope(as_stream(stream));
    if (nrhs == 1)
      F->impl->apply(f, u, as_stream(stream));
    else
      F->impl->apply_block(f, u, nrhs, as_stream(stream));
  });
}

hif_status hif_apply_noalloc(hif_factor_t F, const double* f, double* u, void* stream) {
  return guarded([&] {
    HIF_REQUIRE(F != nullptr && F->impl, HIF_EINVAL, "NULL factor");
    HIF_REQUIRE(f != nullptr && u != nullptr, HIF_EINVAL, "NULL vector");
    hif::apply_noalloc(F, f, u, as_stream(stream));
  });
}

hif_status hif_apply_forward(hif_factor_t F, const double* x, double* y, void* stream) {
  return guarded([&] {
    HIF_REQUIRE(F != nullptr && F->impl, HIF_EINVAL, "NULL factor");
    HIF_REQUIRE(x != nullptr && y != nullptr, HIF_EINVAL, "NULL vector");
    hif::StreamScope scope(as_stream(stream));
    F->impl->apply_forward(x, y, as_stream(stream));
  });
}

hif_status hif_matvec(hif_problem_t A, const double* x, double* y, int32_t nrhs, void* stream) {
  return guarded([&] {
    HIF_REQUIRE(A != nullptr, HIF_EINVAL, "NULL problem");
    HIF_REQUIRE(nrhs >= 0, HIF_EINVAL, "nrhs must be >= 0");
    if (nrhs == 0) return;
    HIF_REQUIRE(x != nullptr && y != nullptr && x != y, HIF_EINVAL, "bad vectors");
    hif::StreamScope scope(as_stream(stream));
    for (int c = 0; c < nrhs; ++c)
      hif::stencil_matvec(A->stencil(), x + c * A->N, y + c * A->N, as_stream(stream));
  });
}

hif_status hif_pcg(hif_problem_t A, hif_factor_t F, const double* f, double* u, int32_t nrhs,
                   double tol, int32_t maxit, hif_pcg_info* info, void* stream) {
  return guarded([&] {
    HIF_REQUIRE(A != nullptr && F != nullptr && F->impl, HIF_EINVAL, "NULL handle");
    HIF_REQUIRE(F->stats.n_dof == A->N, HIF_EINVAL, "factor and problem sizes differ");
    HIF_REQUIRE(nrhs >= 0 && maxit >= 1 && std::isfinite(tol) && tol > 0.0, HIF_EINVAL,
                "need nrhs >= 0, maxit >= 1, tol > 0");
    if (nrhs == 0) return;
    HIF_REQUIRE(f != nullptr && u != nullptr && info != nullptr && f != u, HIF_EINVAL,
                "bad vectors");
    hif::StreamScope scope(as_stream(stream));
    if (nrhs == 1)
      hif::pcg_solve(A, F, f, u, tol, maxit, info, as_stream(stream));
    else
      hif::pcg_solve_block(A, F, f, u, nrhs, tol, maxit, info, as_stream(stream));
    bool all = true;
    for (int c = 0; c < nrhs; ++c) all = all && info[c].converged;
    if (!all) throw hif::Error(HIF_ENOCONV, "PCG did not reach tol within maxit");
  });
}

hif_status hif_gmres(hif_problem_t A, hif_factor_t F, const double* f, double* u, double tol,
                     int32_t restart, int32_t maxit, hif_pcg_info* info, void* stream) {
  return guarded([&] {
    HIF_REQUIRE(A != nullptr && F != nullptr && F->impl, HIF_EINVAL, "NULL handle");
    HIF_REQUIRE(F->stats.n_dof == A->N, HIF_EINVAL, "factor and problem sizes differ");
    HIF_REQUIRE(restart >= 1 && restart <= 1024 && maxit >= 1 && std::isfinite(tol) && tol > 0.0,
                HIF_EINVAL, "need 1 <= restart <= 1024, maxit >= 1, tol > 0");
    HIF_REQUIRE(f != nullptr && u != nullptr && info != nullptr && f != u, HIF_EINVAL,
                "bad vectors");
    hif::StreamScope scope(as_stream(stream));
    hif::gmres_solve(A, F, f, u, tol, restart, maxit, info, as_stream(stream));
    if (!info->converged) throw hif::Error(HIF_ENOCONV, "GMRES did not reach tol within maxit");
  });
}

hif_status hif_pcg_batched(int32_t count, const hif_problem_t* A, const hif_factor_t* F,
                           const double* const* f, double* const* u, double tol, int32_t maxit,
                           hif_pcg_info* info, void* stream) {
  return guarded([&] {
    HIF_REQUIRE(count >= 1 && A != nullptr && F != nullptr && f != nullptr && u != nullptr &&
                    info != nullptr,
                HIF_EINVAL, "NULL array or count < 1");
    HIF_REQUIRE(maxit >= 1 && std::isfinite(tol) && tol > 0.0, HIF_EINVAL,
                "need maxit >= 1, tol > 0");
    for (int32_t i = 0; i < count; ++i) {
      HIF_REQUIRE(A[i] != nullptr && F[i] != nullptr && F[i]->impl, HIF_EINVAL, "NULL handle");
      HIF_REQUIRE(F[i]->stats.n_dof == A[i]->N, HIF_EINVAL, "factor and problem sizes differ");
      HIF_REQUIRE(f[i] != nullptr && u[i] != nullptr && f[i] != u[i], HIF_EINVAL, "bad vectors");
      for (int32_t j = 0; j < i; ++j)
        HIF_REQUIRE(F[j] != F[i], HIF_EINVAL, "a factor listed twice (its calls would overlap)");
    }
    hif::pcg_solve_batched(count, A, F, f, u, tol, maxit, info, as_stream(stream));
    bool all = true;
    for (int32_t i = 0; i < count; ++i) all = all && info[i].converged;
    if (!all) throw hif::Error(HIF_ENOCONV, "PCG did not reach tol within maxit");
  });
}

hif_status hif_factor_stats(hif_factor_t F, hif_stats* out) {
  return guarded([&] {
    HIF_REQUIRE(F != nullptr && out != nullptr, HIF_EINVAL, "NULL argument");
    *out = F->stats;
  });
}

hif_status hif_factor_ranks(hif_factor_t F, int32_t level, int32_t* ranks, int32_t* sizes,
                            int32_t cap, int32_t* count) {
  return guarded([&] {
    HIF_REQUIRE(F != nullptr && count != nullptr, HIF_EINVAL, "NULL argument");
    HIF_REQUIRE(level >= 0 && level < (int)F->ranks.size(), HIF_EINVAL, "level out of range");
    const auto& rk = F->ranks[level];
    const auto& sz = F->sizes[level];
    *count = (int32_t)rk.size();
    const int m = std::min<int>(cap, (int)rk.size());
    if (ranks) std::memcpy(ranks, rk.data(), sizeof(int32_t) * std::max(m, 0));
    if (sizes) std::memcpy(sizes, sz.data(), sizeof(int32_t) * std::max(m, 0));
  });
}

hif_status hif_factor_error(hif_problem_t A, hif_factor_t F, const double* x, int32_t power_iters,
                            double* e_s, double* err_norm, void* stream) {
  return guarded([&] {
    HIF_REQUIRE(A != nullptr && F != nullptr && F->impl && x != nullptr, HIF_EINVAL,
                "NULL argument");
    HIF_REQUIRE(F->stats.n_dof == A->N, HIF_EINVAL, "factor and problem sizes differ");
    HIF_REQUIRE(power_iters >= 0, HIF_EINVAL, "power_iters must be >= 0");
    hif::StreamScope scope(as_stream(stream));
    double es = 0.0, nrm = 0.0;
    hif::factor_error(A, F, x, power_iters, &es, &nrm, as_stream(stream));
    F->stats.e_s = es;
    F->stats.err_norm = nrm;
    if (e_s) *e_s = es;
    if (err_norm) *err_norm = nrm;
  });
}

hif_status hif_factor_save(hif_factor_t F, const char* path, void* stream) {
  return guarded([&] {
    HIF_REQUIRE(F != nullptr && F->impl && path != nullptr, HIF_EINVAL, "NULL argument");
    hif::StreamScope scope(as_stream(stream));
    hif::factor_save(F, path, as_stream(stream));
  });
}

hif_status hif_factor_load(const char* path, void* stream, hif_factor_t* out) {
  if (out) *out = nullptr;
  return guarded([&] {
    HIF_REQUIRE(path != nullptr && out != nullptr, HIF_EINVAL, "NULL argument");
    hif::StreamScope scope(as_stream(stream));
    std::unique_ptr<hif_factor_s> F(new hif_factor_s());
    try {
      hif::factor_load(path, as_stream(stream), F.get());
    } catch (...) {
      (void)hipStreamSynchronize(as_stream(stream));
      throw;
    }
    *out = F.release();
  });
}

hif_status hif_factor_active(hif_factor_t F, int32_t level, uint8_t* mask) {
  return guarded([&] {
    HIF_REQUIRE(F != nullptr && mask != nullptr, HIF_EINVAL, "NULL argument");
    HIF_REQUIRE(F->impl, HIF_EINVAL, "NULL factor");
    HIF_REQUIRE(level >= 0 && level < (int)F->redundant_pts.size(), HIF_EINVAL,
                "level out of range");
    std::memset(mask, 1, (size_t)F->stats.n_dof);
    for (int l = 0; l <= level; ++l) {
      const hif::LevelPlan& P = F->impl->level_plan(l);
      for (int c = 0; c < P.ncell; ++c)
        for (int64_t t = P.crow_off[c]; t < P.crow_off[c] + P.cI[c]; ++t) mask[P.rows[t]] = 0;
      for (int p : F->redundant_pts[l]) mask[p] = 0;
    }
  });
}

hif_status hif_profile_begin(void) {
  return guarded([&] {
    hif::Profiler& p = hif::profiler();
    for (auto& r : p.recs) {
      p.recycle(r.a);
      p.recycle(r.b);
    }
    p.recs.clear();
    p.on = true;
  });
}

hif_status hif_profile_select(const char* classes) {
  return guarded([&] {
    hif::Profiler& p = hif::profiler();
    p.only.clear();
    if (!classes) return;
    std::string cur;
    for (const char* c = classes;; ++c) {
      if (*c == ',' || *c == '\0') {
        if (!cur.empty()) p.only.push_back(cur);
        cur.clear();
        if (*c == '\0') break;
      } else if (*c != ' ') {
        cur.push_back(*c);
      }
    }
  });
}

hif_status hif_profile_end(hif_kernel_stat* out, int32_t cap, int32_t* count) {
  return guarded([&] {
    HIF_REQUIRE(count != nullptr, HIF_EINVAL, "count must not be NULL");
    hif::Profiler& p = hif::profiler();
    p.on = false;
    std::vector<hif_kernel_stat> agg(p.names.size());
    for (size_t i = 0; i < p.names.size(); ++i) {
      std::memset(&agg[i], 0, sizeof(hif_kernel_stat));
      std::strncpy(agg[i].name, p.names[i].c_str(), sizeof(agg[i].name) - 1);
    }
    for (auto& r : p.recs) {
      HIF_HIP(hipEventSynchronize(r.b));
      float ms = 0.f;
      HIF_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      hif_kernel_stat& k = agg[r.cls];
      k.launches += 1;
      k.seconds += ms * 1e-3;
      k.flops += r.flops;
      k.bytes += r.bytes;
      p.recycle(r.a);
      p.recycle(r.b);
    }
    p.recs.clear();
    int32_t nz = 0;
    for (auto& k : agg)
      if (k.launches > 0) {
        if (out && nz < cap) out[nz] = k;
        ++nz;
      }
    *count = nz;
  });
}

void hif_factor_destroy(hif_factor_t F) { delete F; }
void hif_problem_destroy(hif_problem_t A) { delete A; }

const char* hif_status_string(hif_status s) {
  switch (s) {
    case HIF_OK: return "HIF_OK";
    case HIF_EINVAL: return "HIF_EINVAL: invalid argument";
    case HIF_ENOMEM: return "HIF_ENOMEM: out of device memory";
    case HIF_ENOTSPD: return "HIF_ENOTSPD: matrix not positive definite";
    case HIF_ENOCONV: return "HIF_ENOCONV: PCG did not converge";
    case HIF_EDEVICE: return "HIF_EDEVICE: device runtime error or failed internal check";
  }
  return "unknown hif_status";
}

const char* hif_last_error(void) { return hif::g_last_error.c_str(); }

}  // extern "C"

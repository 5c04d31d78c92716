// Saving a factorization to a file and loading it back (the stored blocks of
// F, paper Section 2.4 product form, with what is needed to apply them).
//
// The file holds the options, the statistics, and per level the ranks, face
// sizes and redundant points (the ID's outcome), the face points in pivot
// order, and the numeric arenas of the fronts ([L_I^{-1}; L_SI] per cell)
// and of the skeletons (T, L_F̌^{-1}, Y per face), in the factor's
// precision, and the signs of a periodic root's L S L^T.  Everything else -- the cell/face plans, block layouts and
// sweep descriptors -- is a function of the grid, the leaf width, the
// boundary condition and the redundant points, and is rebuilt on load the
// way the build lays it out.
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>

#include "hif_impl.hpp"

namespace hif {
namespace {

constexpr char kMagic[8] = {'H', 'I', 'F', 'F', 'A', 'C', 'T', '1'};
constexpr uint32_t kVersion = 2;

struct File {
  FILE* f = nullptr;
  std::string path;
  File(const char* p, const char* mode) : path(p) {
    f = std::fopen(p, mode);
    HIF_REQUIRE(f != nullptr, HIF_EINVAL, "cannot open " + path);
  }
  ~File() {
    if (f) std::fclose(f);
  }
  void write(const void* p, size_t n) {
    if (n == 0) return;
    HIF_REQUIRE(std::fwrite(p, 1, n, f) == n, HIF_EINVAL, "write failed: " + path);
  }
  void read(void* p, size_t n) {
    if (n == 0) return;
    HIF_REQUIRE(std::fread(p, 1, n, f) == n, HIF_EINVAL, "truncated factor file: " + path);
  }
  template <typename V>
  void put(const V& v) { write(&v, sizeof(V)); }
  template <typename V>
  V get() {
    V v;
    read(&v, sizeof(V));
    return v;
  }
  template <typename V>
  void put_vec(const std::vector<V>& v) {
    put<uint64_t>(v.size());
    write(v.data(), sizeof(V) * v.size());
  }
  template <typename V>
  std::vector<V> get_vec(uint64_t limit) {
    const uint64_t n = get<uint64_t>();
    HIF_REQUIRE(n <= limit, HIF_EINVAL, "corrupt factor file: " + path);
    std::vector<V> v(n);
    read(v.data(), sizeof(V) * n);
    return v;
  }
};

template <typename V>
void put_dev(File& out, const DevBuf<V>& d, hipStream_t s) {
  std::vector<V> h;
  d.download(h, s);
  HIF_HIP(hipStreamSynchronize(s));
  out.put_vec(h);
}

template <typename T>
void save_impl(const hif_factor_s* F, const FactorImpl<T>& I, File& out, hipStream_t s) {
  const int L = I.L;
  out.put<int32_t>(L);
  for (int l = 0; l < L; ++l) {
    out.put_vec(F->ranks[l]);
    out.put_vec(F->sizes[l]);
    out.put_vec(F->redundant_pts[l]);
  }
  for (int l = 0; l <= L; ++l) {
    const Level<T>& lv = I.levels[l];
    if (l < L) put_dev(out, lv.skpts, s);
    put_dev(out, lv.front, s);
    if (l < L) put_dev(out, lv.skel, s);
    else put_dev(out, lv.sign, s);  // the signs of a periodic root's L S L^T (else empty)
  }
}

template <typename T>
std::unique_ptr<FactorImpl<T>> load_impl(hif_factor_s* F, File& in, hipStream_t s) {
  const hif_options& o = F->opts;
  const int n = o.n;
  const int L = levels_for(n, o.leaf);
  const int64_t N = (int64_t)n * n * n;
  HIF_REQUIRE(in.get<int32_t>() == L, HIF_EINVAL, "corrupt factor file: " + in.path);
  auto I = std::make_unique<FactorImpl<T>>();
  I->n = n;
  I->L = L;
  I->N = N;
  I->levels.resize(L + 1);
  F->ranks.resize(L);
  F->sizes.resize(L);
  F->redundant_pts.resize(L);
  for (int l = 0; l < L; ++l) {
    F->ranks[l] = in.get_vec<int>(N);
    F->sizes[l] = in.get_vec<int>(N);
    F->redundant_pts[l] = in.get_vec<int>(N);
  }
  const std::vector<LevelGeom> geom = plan_geometry(n, o.leaf, o.bc == HIF_PERIODIC);
  std::vector<uint8_t> active((size_t)N, 1);
  for (int l = 0; l <= L; ++l) {
    Level<T>& lv = I->levels[l];
    lv.plan = std::make_shared<const LevelPlan>(plan_level(geom[l], active));
    const LevelPlan& P = *lv.plan;
    // cells: the front layout of the build
    lv.rows = dev_arr(P.rows, s);
    lv.crow_off = dev_arr(P.crow_off, s);
    lv.hfd.resize(P.ncell);
    std::vector<int64_t> foff(P.ncell);
    int64_t off = 0;
    lv.hyoff.resize(P.ncell);
    lv.hzoff.resize(P.ncell);
    for (int c = 0; c < P.ncell; ++c) {
      FrontDesc& d = lv.hfd[c];
      foff[c] = off;
      d.nI = P.cI[c];
      d.nR = P.cI[c] + P.cS[c];
      d.ld = pad_ld(d.nR);
      d.id = c;
      off += (int64_t)d.ld * d.nI;
      lv.hyoff[c] = lv.ysum;
      lv.hzoff[c] = lv.zsum;
      lv.ysum += d.nI;
      lv.zsum += P.cS[c];
      lv.maxI = std::max(lv.maxI, d.nI);
      lv.maxS = std::max(lv.maxS, P.cS[c]);
    }
    std::vector<int> skpts;
    if (l < L) {
      skpts = in.get_vec<int>(N);
      HIF_REQUIRE(skpts.size() == std::max<size_t>(P.fpts.size(), 1), HIF_EINVAL,
                  "factor file does not match its grid: " + in.path);
    }
    std::vector<T> front = in.get_vec<T>((uint64_t)off);
    HIF_REQUIRE((int64_t)front.size() == off, HIF_EINVAL,
                "factor file does not match its grid: " + in.path);
    lv.front.upload(front, s);
    for (int c = 0; c < P.ncell; ++c) lv.hfd[c].ptr = lv.front.get() + foff[c];
    lv.fd.upload(lv.hfd, s);
    lv.yoff.upload(lv.hyoff, s);
    lv.zoff.upload(lv.hzoff, s);
    if (l == L) {
      std::vector<T> sign = in.get_vec<T>((uint64_t)lv.ysum);
      HIF_REQUIRE(sign.empty() || (int64_t)sign.size() == lv.ysum, HIF_EINVAL,
                  "factor file does not match its grid: " + in.path);
      lv.sign.upload(sign, s);
      break;
    }
    // faces: the skeleton layout of the build
    lv.fpts = dev_arr(P.fpts, s);
    lv.fpt_off = dev_arr(P.fpt_off, s);
    lv.fN = dev_arr(P.fN, s);
    lv.fcellA = dev_arr(P.fcellA, s);
    lv.fcellB = dev_arr(P.fcellB, s);
    lv.rb_face = dev_arr(P.rb_face, s);
    lv.rb_off = dev_arr(P.rb_off, s);
    lv.rb_sa = dev_arr(P.rb_sa, s);
    lv.rb_sb = dev_arr(P.rb_sb, s);
    for (int f = 0; f < P.nface; ++f) lv.maxF = std::max(lv.maxF, P.fN[f]);
    HIF_REQUIRE(F->ranks[l].size() == (size_t)P.nface && F->sizes[l] == P.fN, HIF_EINVAL,
                "factor file does not match its grid: " + in.path);
    lv.hk = F->ranks[l];
    int64_t ssz = 0;
    for (int f = 0; f < P.nface; ++f) {
      const int k = lv.hk[f], r = P.fN[f] - k;
      HIF_REQUIRE(k >= 0 && r >= 0, HIF_EINVAL, "corrupt factor file: " + in.path);
      if (r == 0) continue;
      SkelDesc d{};
      d.face = f;
      d.k = k;
      d.r = r;
      d.pts_off = P.fpt_off[f];
      d.offT = ssz;
      ssz += (int64_t)k * r;
      d.offL = ssz;
      ssz += (int64_t)r * r;
      d.offY = ssz;
      ssz += (int64_t)r * k;
      d.kofs = lv.ksum;
      d.rofs = lv.rsum;
      lv.ksum += k;
      lv.rsum += r;
      lv.hsk.push_back(d);
      lv.maxk = std::max(lv.maxk, k);
      lv.maxr = std::max(lv.maxr, r);
      lv.redundant += r;
    }
    lv.sk.upload(lv.hsk, s);
    // (a build at eps = 0 keeps no skeleton arena at all)
    std::vector<T> skel = in.get_vec<T>((uint64_t)std::max<int64_t>(ssz, 1));
    HIF_REQUIRE((int64_t)skel.size() == ssz || (ssz == 0 && skel.size() <= 1), HIF_EINVAL,
                "factor file does not match its grid: " + in.path);
    lv.skel.upload(skel, s);
    for (int p : skpts)
      HIF_REQUIRE(p >= 0 && p < N, HIF_EINVAL, "corrupt factor file: " + in.path);
    lv.skpts.upload(skpts, s);
    for (int p : F->redundant_pts[l]) {
      HIF_REQUIRE(p >= 0 && p < N, HIF_EINVAL, "corrupt factor file: " + in.path);
      active[p] = 0;
    }
  }
  I->prepare(s);
  HIF_HIP(hipStreamSynchronize(s));
  return I;
}

}  // namespace

void factor_save(const hif_factor_s* F, const char* path, hipStream_t s) {
  File out(path, "wb");
  out.write(kMagic, sizeof(kMagic));
  out.put<uint32_t>(kVersion);
  out.put<int32_t>(F->opts.n);
  out.put<int32_t>(F->opts.leaf);
  out.put<double>(F->opts.eps);
  out.put<int32_t>(F->opts.precision);
  out.put<int32_t>(F->opts.bc);
  out.put<uint64_t>(sizeof(hif_stats));
  out.put(F->stats);
  if (F->opts.precision == HIF_MIXED)
    save_impl(F, static_cast<const FactorImpl<float>&>(*F->impl), out, s);
  else
    save_impl(F, static_cast<const FactorImpl<double>&>(*F->impl), out, s);
}

void factor_load(const char* path, hipStream_t s, hif_factor_s* F) {
  File in(path, "rb");
  char magic[8];
  in.read(magic, sizeof(magic));
  HIF_REQUIRE(std::memcmp(magic, kMagic, sizeof(kMagic)) == 0, HIF_EINVAL,
              "not a HIF factor file: " + in.path);
  HIF_REQUIRE(in.get<uint32_t>() == kVersion, HIF_EINVAL,
              "unsupported factor file version: " + in.path);
  hif_options& o = F->opts;
  std::memset(&o, 0, sizeof(o));
  o.n = in.get<int32_t>();
  o.leaf = in.get<int32_t>();
  o.eps = in.get<double>();
  o.precision = in.get<int32_t>();
  o.bc = in.get<int32_t>();
  HIF_REQUIRE(o.n >= 2 && o.n <= 1024 && levels_for(o.n, o.leaf) >= 0 &&
                  (o.precision == HIF_FP64 || o.precision == HIF_MIXED) &&
                  (o.bc == HIF_DIRICHLET || o.bc == HIF_PERIODIC),
              HIF_EINVAL, "corrupt factor file header: " + in.path);
  HIF_REQUIRE(in.get<uint64_t>() == sizeof(hif_stats), HIF_EINVAL,
              "factor file from another library version: " + in.path);
  F->stats = in.get<hif_stats>();
  if (o.precision == HIF_MIXED)
    F->impl = load_impl<float>(F, in, s);
  else
    F->impl = load_impl<double>(F, in, s);
}

}  // namespace hif

// Host planner for the HIF cell hierarchy (paper, Section 2.1 and the level
// loop of Section 2.4).
#include "plan.hpp"

#include <algorithm>
#include <stdexcept>

namespace hif {

int levels_for(int n, int leaf) {
  if (leaf < 2 || n < leaf) return -1;
  int L = 0;
  while ((int64_t)leaf << L < n) ++L;
  return ((int64_t)leaf << L) == n ? L : -1;
}

int64_t LevelPlan::sum_I() const {
  int64_t s = 0;
  for (int v : cI) s += v;
  return s;
}
int64_t LevelPlan::sum_S() const {
  int64_t s = 0;
  for (int v : cS) s += v;
  return s;
}

namespace {

inline int face_id(int nc, int d, int plane, int i_lo, int i_hi) {
  // i_lo: cell index along the faster of the two other dimensions.
  return ((d * (nc - 1) + (plane - 1)) * nc + i_hi) * nc + i_lo;
}

inline int cell_id(int nc, int cx, int cy, int cz) { return (cz * nc + cy) * nc + cx; }

}  // namespace

LevelPlan plan_level(int n, int leaf, int level, int L, const std::vector<uint8_t>& active) {
  LevelPlan P;
  P.level = level;
  P.w = leaf << level;
  P.nc = n / P.w;
  P.root = (level == L);
  const int w = P.w, nc = P.nc;
  P.ncell = nc * nc * nc;
  P.nface = 3 * (nc - 1) * nc * nc;
  const int64_t N = (int64_t)n * n * n;

  // Pass 1: classify active points, count per cell / face.
  std::vector<int> owner(N, -1);  // >= 0: cell id; <= -2: -(face id) - 2
  P.cI.assign(P.ncell, 0);
  P.fN.assign(P.nface, 0);
  for (int64_t p = 0; p < N; ++p) {
    if (!active[p]) continue;
    const int c[3] = {(int)(p % n), (int)((p / n) % n), (int)(p / ((int64_t)n * n))};
    int nsep = 0, dsep = -1;
    for (int d = 0; d < 3; ++d)
      if (c[d] % w == 0 && c[d] != 0) { ++nsep; dsep = d; }
    if (nsep == 0) {
      const int id = cell_id(nc, c[0] / w, c[1] / w, c[2] / w);
      owner[p] = id;
      ++P.cI[id];
    } else if (nsep == 1) {
      const int o1 = dsep == 0 ? 1 : 0;
      const int o2 = dsep == 2 ? 1 : 2;
      const int id = face_id(nc, dsep, c[dsep] / w, c[o1] / w, c[o2] / w);
      owner[p] = -id - 2;
      ++P.fN[id];
    }
  }

  // Face point lists (ascending because p is visited in order).
  P.fpt_off.assign(P.nface + 1, 0);
  for (int f = 0; f < P.nface; ++f) P.fpt_off[f + 1] = P.fpt_off[f] + P.fN[f];
  P.fpts.resize(P.fpt_off[P.nface]);
  {
    std::vector<int64_t> cur(P.fpt_off.begin(), P.fpt_off.end() - 1);
    for (int64_t p = 0; p < N; ++p)
      if (owner[p] <= -2) P.fpts[cur[-owner[p] - 2]++] = (int)p;
  }

  // Faces of each cell, S offsets.
  P.cface.assign((size_t)P.ncell * 6, -1);
  P.cface_off.assign((size_t)P.ncell * 6, -1);
  P.cS.assign(P.ncell, 0);
  for (int cz = 0; cz < nc; ++cz)
    for (int cy = 0; cy < nc; ++cy)
      for (int cx = 0; cx < nc; ++cx) {
        const int id = cell_id(nc, cx, cy, cz);
        const int cc[3] = {cx, cy, cz};
        int off = 0;
        for (int d = 0; d < 3; ++d) {
          const int o1 = d == 0 ? 1 : 0;
          const int o2 = d == 2 ? 1 : 2;
          for (int up = 0; up < 2; ++up) {
            const int plane = cc[d] + up;
            if (plane < 1 || plane > nc - 1) continue;
            const int f = face_id(nc, d, plane, cc[o1], cc[o2]);
            P.cface[(size_t)id * 6 + 2 * d + up] = f;
            P.cface_off[(size_t)id * 6 + 2 * d + up] = off;
            off += P.fN[f];
          }
        }
        P.cS[id] = off;
      }

  // Rows of each front: I then S.
  P.crow_off.assign(P.ncell + 1, 0);
  for (int c = 0; c < P.ncell; ++c) P.crow_off[c + 1] = P.crow_off[c] + P.cI[c] + P.cS[c];
  P.rows.resize(P.crow_off[P.ncell]);
  {
    std::vector<int64_t> cur(P.ncell);
    for (int c = 0; c < P.ncell; ++c) cur[c] = P.crow_off[c];
    for (int64_t p = 0; p < N; ++p)
      if (owner[p] >= 0) P.rows[cur[owner[p]]++] = (int)p;
    for (int c = 0; c < P.ncell; ++c) {
      int64_t o = P.crow_off[c] + P.cI[c];
      for (int s = 0; s < 6; ++s) {
        const int f = P.cface[(size_t)c * 6 + s];
        if (f < 0) continue;
        for (int64_t t = P.fpt_off[f]; t < P.fpt_off[f + 1]; ++t) P.rows[o++] = P.fpts[t];
      }
    }
  }

  // Neighbouring cells of each face and the panel row blocks.
  P.fcellA.assign(P.nface, -1);
  P.fcellB.assign(P.nface, -1);
  P.rb_face.assign((size_t)P.nface * kRowBlocks, -1);
  P.rb_off.assign((size_t)P.nface * kRowBlocks, 0);
  P.rb_sa.assign((size_t)P.nface * kRowBlocks, -1);
  P.rb_sb.assign((size_t)P.nface * kRowBlocks, -1);
  P.prow.assign(P.nface, 0);
  for (int d = 0; d < 3; ++d) {
    const int o1 = d == 0 ? 1 : 0;
    const int o2 = d == 2 ? 1 : 2;
    for (int plane = 1; plane < nc; ++plane)
      for (int ihi = 0; ihi < nc; ++ihi)
        for (int ilo = 0; ilo < nc; ++ilo) {
          const int f = face_id(nc, d, plane, ilo, ihi);
          int ca[3], cb[3];
          ca[d] = plane - 1;
          cb[d] = plane;
          ca[o1] = cb[o1] = ilo;
          ca[o2] = cb[o2] = ihi;
          const int A = cell_id(nc, ca[0], ca[1], ca[2]);
          const int B = cell_id(nc, cb[0], cb[1], cb[2]);
          P.fcellA[f] = A;
          P.fcellB[f] = B;
          const int slotA = 2 * d + 1, slotB = 2 * d;
          size_t base = (size_t)f * kRowBlocks;
          int t = 0, ro = 0;
          P.rb_face[base] = f;
          P.rb_off[base] = 0;
          P.rb_sa[base] = P.cface_off[(size_t)A * 6 + slotA];
          P.rb_sb[base] = P.cface_off[(size_t)B * 6 + slotB];
          ro += P.fN[f];
          ++t;
          for (int side = 0; side < 2; ++side) {
            const int cell = side == 0 ? A : B;
            const int skip = side == 0 ? slotA : slotB;
            for (int s = 0; s < 6; ++s) {
              const int g = P.cface[(size_t)cell * 6 + s];
              if (s == skip || g < 0) continue;
              P.rb_face[base + t] = g;
              P.rb_off[base + t] = ro;
              if (side == 0) P.rb_sa[base + t] = P.cface_off[(size_t)cell * 6 + s];
              else P.rb_sb[base + t] = P.cface_off[(size_t)cell * 6 + s];
              ro += P.fN[g];
              ++t;
            }
          }
          P.prow[f] = ro;
        }
  }
  return P;
}

}  // namespace hif

// Host planner for the HIF cell hierarchy (paper, Section 2.1 and the level
// loop of Section 2.4).
#include "plan.hpp"

#include <algorithm>
#include <stdexcept>
#include <string>

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

// Faces per dimension: nc - 1 interior planes (Dirichlet: planes 1..nc-1) or
// nc planes (periodic: planes 0..nc-1, plane 0 between cells nc-1 and 0).
struct Planes {
  int count, first;
};
inline Planes planes_of(int nc, bool periodic) {
  return periodic ? Planes{nc, 0} : Planes{nc - 1, 1};
}

inline int face_id(const Planes& pl, int nc, int d, int plane, int i_lo, int i_hi) {
  // i_lo: cell index along the faster of the two other dimensions.
  return ((d * pl.count + (plane - pl.first)) * nc + i_hi) * nc + i_lo;
}

inline int cell_id(int nc, int cx, int cy, int cz) { return (cz * nc + cy) * nc + cx; }

}  // namespace

std::vector<LevelGeom> plan_geometry(int n, int leaf, bool periodic) {
  const int L = levels_for(n, leaf);
  if (L < 0) throw std::invalid_argument("n must be leaf * 2^L");
  const int64_t N = (int64_t)n * n * n;
  std::vector<LevelGeom> out(L + 1);
  std::vector<int> owner(N);
  std::vector<int> sep(n), cidx(n);
  for (int level = 0; level <= L; ++level) {
    LevelGeom& G = out[level];
    G.level = level;
    G.w = leaf << level;
    G.nc = n / G.w;
    G.root = level == L;
    const int w = G.w, nc = G.nc;
    // the root level (one cell) has no separators in either layout
    const bool per = periodic && !G.root;
    const Planes pl = planes_of(nc, per);
    G.ncell = nc * nc * nc;
    G.nface = G.root ? 0 : 3 * pl.count * nc * nc;
    for (int x = 0; x < n; ++x) {
      sep[x] = G.root ? 0 : (x % w == 0 && (per || x != 0));
      cidx[x] = x / w;
    }
    // candidates: points with no separator coordinate at any earlier level
    // (equivalently at level-1, the separators being nested), classified now
    std::vector<int> cntI(G.ncell, 0), cntF(G.nface, 0);
    const int wp = level > 0 ? (leaf << (level - 1)) : 0;
    for (int z = 0; z < n; ++z)
      for (int y = 0; y < n; ++y) {
        const int64_t row = ((int64_t)z * n + y) * n;
        for (int x = 0; x < n; ++x) {
          const int64_t p = row + x;
          owner[p] = -1;
          if (level > 0) {
            const bool sp = (x % wp == 0 && (periodic || x != 0)) ||
                            (y % wp == 0 && (periodic || y != 0)) ||
                            (z % wp == 0 && (periodic || z != 0));
            if (!sp) continue;  // eliminated as an interior point at an earlier level
          }
          const int ns = sep[x] + sep[y] + sep[z];
          if (ns == 0) {
            const int id = (cidx[z] * nc + cidx[y]) * nc + cidx[x];
            owner[p] = id;
            ++cntI[id];
          } else if (ns == 1) {
            const int c3[3] = {x, y, z};
            const int d = sep[x] ? 0 : (sep[y] ? 1 : 2);
            const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
            const int id = face_id(pl, nc, d, cidx[c3[d]], cidx[c3[o1]], cidx[c3[o2]]);
            owner[p] = -id - 2;
            ++cntF[id];
          }
        }
      }
    G.cand_I_off.assign(G.ncell + 1, 0);
    for (int c = 0; c < G.ncell; ++c) G.cand_I_off[c + 1] = G.cand_I_off[c] + cntI[c];
    G.cand_F_off.assign(G.nface + 1, 0);
    for (int f = 0; f < G.nface; ++f) G.cand_F_off[f + 1] = G.cand_F_off[f] + cntF[f];
    G.cand_I.resize(G.cand_I_off[G.ncell]);
    G.cand_F.resize(G.cand_F_off[G.nface]);
    {
      std::vector<int64_t> ci(G.cand_I_off.begin(), G.cand_I_off.end() - 1);
      std::vector<int64_t> cf(G.cand_F_off.begin(), G.cand_F_off.end() - 1);
      for (int64_t p = 0; p < N; ++p) {
        const int o = owner[p];
        if (o >= 0) G.cand_I[ci[o]++] = (int)p;
        else if (o <= -2) G.cand_F[cf[-o - 2]++] = (int)p;
      }
    }
    G.cface.assign((size_t)G.ncell * 6, -1);
    for (int cz = 0; cz < nc; ++cz)
      for (int cy = 0; cy < nc; ++cy)
        for (int cx = 0; cx < nc; ++cx) {
          const int id = cell_id(nc, cx, cy, cz);
          const int cc[3] = {cx, cy, cz};
          for (int d = 0; d < 3; ++d) {
            const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
            for (int up = 0; up < 2; ++up) {
              int plane = cc[d] + up;
              if (per) plane %= nc;
              else if (G.root || plane < 1 || plane > nc - 1) continue;
              G.cface[(size_t)id * 6 + 2 * d + up] = face_id(pl, nc, d, plane, cc[o1], cc[o2]);
            }
          }
        }
    G.fcellA.assign(G.nface, -1);
    G.fcellB.assign(G.nface, -1);
    G.rb_face.assign((size_t)G.nface * kRowBlocks, -1);
    G.rb_slotA.assign((size_t)G.nface * kRowBlocks, -1);
    G.rb_slotB.assign((size_t)G.nface * kRowBlocks, -1);
    for (int d = 0; d < 3 && !G.root; ++d) {
      const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
      for (int plane = pl.first; plane < pl.first + pl.count; ++plane)
        for (int ihi = 0; ihi < nc; ++ihi)
          for (int ilo = 0; ilo < nc; ++ilo) {
            const int f = face_id(pl, nc, d, plane, ilo, ihi);
            int ca[3], cb[3];
            ca[d] = (plane - 1 + nc) % nc;  // lower neighbour (wraps for plane 0)
            cb[d] = plane;
            ca[o1] = cb[o1] = ilo;
            ca[o2] = cb[o2] = ihi;
            const int A = cell_id(nc, ca[0], ca[1], ca[2]);
            const int B = cell_id(nc, cb[0], cb[1], cb[2]);
            G.fcellA[f] = A;
            G.fcellB[f] = B;
            const int slotA = 2 * d + 1, slotB = 2 * d;
            const size_t base = (size_t)f * kRowBlocks;
            int t = 0;
            G.rb_face[base] = f;
            G.rb_slotA[base] = slotA;
            G.rb_slotB[base] = slotB;
            ++t;
            for (int side = 0; side < 2; ++side) {
              const int cell = side == 0 ? A : B;
              const int skip = side == 0 ? slotA : slotB;
              for (int s = 0; s < 6; ++s) {
                const int g = G.cface[(size_t)cell * 6 + s];
                if (s == skip || g < 0) continue;
                // a face of both cells (periodic with two cells along d: the
                // other plane between them) is one row block fed by both
                int at = -1;
                for (int u = 0; u < t; ++u)
                  if (G.rb_face[base + u] == g) at = u;
                if (at < 0) {
                  at = t++;
                  if (t > kRowBlocks) throw std::logic_error("face panel row blocks overflow");
                  G.rb_face[base + at] = g;
                }
                if (side == 0) G.rb_slotA[base + at] = s;
                else G.rb_slotB[base + at] = s;
              }
            }
          }
    }
  }
  return out;
}

LevelPlan plan_level(const LevelGeom& G, const std::vector<uint8_t>& active) {
  LevelPlan P;
  P.level = G.level;
  P.w = G.w;
  P.nc = G.nc;
  P.root = G.root;
  P.ncell = G.ncell;
  P.nface = G.nface;
  // active face points.  The compactions here write every candidate and
  // advance past the active ones only: no branch on the irregular mask.
  P.fN.assign(P.nface, 0);
  P.fpt_off.assign(P.nface + 1, 0);
  P.fpts.resize(G.cand_F.size());
  int64_t nf = 0;
  for (int f = 0; f < P.nface; ++f) {
    for (int64_t t = G.cand_F_off[f]; t < G.cand_F_off[f + 1]; ++t) {
      const int p = G.cand_F[t];
      P.fpts[nf] = p;
      nf += active[p] != 0;
    }
    P.fpt_off[f + 1] = nf;
    P.fN[f] = (int)(P.fpt_off[f + 1] - P.fpt_off[f]);
  }
  P.fpts.resize(nf);
  // cells: I then S
  P.cface = G.cface;
  P.cface_off.assign((size_t)P.ncell * 6, -1);
  P.cI.assign(P.ncell, 0);
  P.cS.assign(P.ncell, 0);
  P.crow_off.assign(P.ncell + 1, 0);
  // a cell's rows: its active interior, then the points of its up to six faces
  int64_t cap = (int64_t)G.cand_I.size();
  for (size_t q = 0; q < P.cface.size(); ++q)
    if (P.cface[q] >= 0) cap += P.fN[P.cface[q]];
  P.rows.resize(cap);
  int64_t nr = 0;
  for (int c = 0; c < P.ncell; ++c) {
    for (int64_t t = G.cand_I_off[c]; t < G.cand_I_off[c + 1]; ++t) {
      const int p = G.cand_I[t];
      P.rows[nr] = p;
      nr += active[p] != 0;
    }
    P.cI[c] = (int)(nr - P.crow_off[c]);
    int off = 0;
    for (int s = 0; s < 6; ++s) {
      const int f = P.cface[(size_t)c * 6 + s];
      if (f < 0) continue;
      P.cface_off[(size_t)c * 6 + s] = off;
      std::copy(P.fpts.begin() + P.fpt_off[f], P.fpts.begin() + P.fpt_off[f + 1],
                P.rows.begin() + nr);
      nr += P.fN[f];
      off += P.fN[f];
    }
    P.cS[c] = off;
    P.crow_off[c + 1] = nr;
  }
  P.rows.resize(nr);
  // panel row blocks
  P.fcellA = G.fcellA;
  P.fcellB = G.fcellB;
  P.rb_face = G.rb_face;
  P.rb_off.assign((size_t)P.nface * kRowBlocks, 0);
  P.rb_sa.assign((size_t)P.nface * kRowBlocks, -1);
  P.rb_sb.assign((size_t)P.nface * kRowBlocks, -1);
  P.prow.assign(P.nface, 0);
  for (int f = 0; f < P.nface; ++f) {
    const size_t base = (size_t)f * kRowBlocks;
    const int A = P.fcellA[f], B = P.fcellB[f];
    int ro = 0;
    for (int t = 0; t < kRowBlocks; ++t) {
      const int g = P.rb_face[base + t];
      if (g < 0) break;
      P.rb_off[base + t] = ro;
      if (G.rb_slotA[base + t] >= 0) P.rb_sa[base + t] = P.cface_off[(size_t)A * 6 + G.rb_slotA[base + t]];
      if (G.rb_slotB[base + t] >= 0) P.rb_sb[base + t] = P.cface_off[(size_t)B * 6 + G.rb_slotB[base + t]];
      ro += P.fN[g];
    }
    P.prow[f] = ro;
  }
  return P;
}

LevelPlan plan_level(int n, int leaf, int level, int L, const std::vector<uint8_t>& active,
                     bool periodic) {
  (void)L;
  const std::vector<LevelGeom> G = plan_geometry(n, leaf, periodic);
  return plan_level(G[level], active);
}

}  // namespace hif

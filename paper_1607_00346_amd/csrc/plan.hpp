// Host planner: the cell hierarchy of the HIF and the per-level index maps.
//
// Level l cells have width w = leaf * 2^l (paper, Section 2.1).  With zero
// Dirichlet values outside the grid, the separators of level l are the grid
// planes x_d = w * j with j >= 1 (the plane x_d = 0 is not a separator and
// there is none at x_d = n), so every face borders exactly two cells.  With
// periodic boundaries (the paper's setting) every plane x_d = w * j, j >= 0,
// is a separator; the face on x_d = 0 lies between the last and the first
// cell along d, so again every face borders exactly two cells.  A point
// with c separator coordinates is a cell interior point (c = 0), a face point
// (c = 1), an edge point (c = 2) or a corner (c = 3).
//
// Structural facts the maps rely on (7-point stencil, levels processed in
// order): edge and corner points only ever couple to their stencil
// neighbours, so the shell S of a cell interior is exactly the active points
// of the cell's (up to six) faces, and the rows R of a face's interpolative
// decomposition are the other faces of its two cells plus stencil couplings
// to edge points.
#pragma once

#include <cstdint>
#include <vector>

namespace hif {

constexpr int kRowBlocks = 11;  // a face panel holds the face and the other faces of both cells

struct LevelPlan {
  int level = 0, w = 0, nc = 0;  // nc = cells per dimension
  bool root = false;             // level L: one cell, no faces

  // Cells in lexicographic order (x1 fastest).  rows[crow_off[c] ...] lists the
  // interior I (ascending global index) followed by S = the cell's faces in
  // slot order (d = 0 lower, d = 0 upper, d = 1 lower, ...).
  int ncell = 0;
  std::vector<int> cI, cS;
  std::vector<int64_t> crow_off;
  std::vector<int> rows;
  std::vector<int> cface;      // ncell * 6: face id per slot or -1
  std::vector<int> cface_off;  // ncell * 6: offset of that face inside S or -1

  // Faces enumerated by (normal d, plane j_d (>= 1; periodic: >= 0), index of the slower other
  // dimension, index of the faster one).  fpts lists a face's active points
  // ascending.  Cell A is the lower neighbour along d, cell B the upper.
  int nface = 0;
  std::vector<int> fN;
  std::vector<int64_t> fpt_off;
  std::vector<int> fpts;
  std::vector<int> fcellA, fcellB;
  // Panel row blocks per face (kRowBlocks slots, unused = -1): the face id, its
  // row offset in the panel, its offset inside S of cell A / cell B (or -1).
  std::vector<int> rb_face, rb_off, rb_sa, rb_sb;
  std::vector<int> prow;  // panel rows

  int64_t sum_I() const;
  int64_t sum_S() const;
};

// Geometry of one level that does not depend on ranks: the candidate points of
// every cell interior and every face (points not interior at any earlier
// level, ascending), the faces of each cell and the panel row-block faces.
struct LevelGeom {
  int level = 0, w = 0, nc = 0, ncell = 0, nface = 0;
  bool root = false;
  std::vector<int64_t> cand_I_off, cand_F_off;
  std::vector<int> cand_I, cand_F;
  std::vector<int> cface;    // ncell * 6
  std::vector<int> fcellA, fcellB;
  std::vector<int> rb_face;  // nface * kRowBlocks
  std::vector<int> rb_slotA, rb_slotB;  // slot of the block's face in cell A / B, or -1
};

// Geometry of every level 0..L of an n^3 grid with leaf width `leaf`;
// periodic: every plane x_d = w j (j >= 0) below the root is a separator and
// the faces on x_d = 0 join the last and the first cell along d.
std::vector<LevelGeom> plan_geometry(int n, int leaf, bool periodic);

// Plan level `level` from its geometry and the current active mask (1 byte per
// grid point): the candidates that are still active.
LevelPlan plan_level(const LevelGeom& G, const std::vector<uint8_t>& active);

// Plan level `level` of an n^3 grid directly (geometry + filter).
LevelPlan plan_level(int n, int leaf, int level, int L, const std::vector<uint8_t>& active,
                     bool periodic);

// Number of levels L with n = leaf * 2^L, or -1 if n is not of that form.
int levels_for(int n, int leaf);

}  // namespace hif

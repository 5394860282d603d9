// DoF maps of the leaf mesh and of the level meshes (Sec. 2.3, Fig. 1):
// node identity, Dirichlet nodes, hanging-node constraints, first-touch
// numbering, S/I/D level splitting, copy map leaf -> level, and sibling
// family maps used by the transfer operators (Sec. 2.2).
#pragma once
#include <cstdint>
#include <vector>

#include "fe1d.hpp"
#include "forest.hpp"
#include "layout.hpp"
#include "leaftiles.hpp"

namespace gmg {

enum : uint8_t { kFlagS = 0, kFlagI = 1, kFlagD = 2 };

struct LevelData {
  int level = 0;
  int64_t n_cells = 0, n_dofs = 0, n_fam = 0;
  std::vector<Cell> cells;            // canonical order
  std::vector<uint64_t> keys;         // forest keys of the cells
  std::vector<int32_t> leaf_index;    // leaf index of a cell that is a leaf, else -1
  std::vector<int32_t> cellmap;       // [n_cells * npc] level DoF ids
  std::vector<uint8_t> flags;         // [n_dofs]
  std::vector<int32_t> parent;        // [n_fam] parent index among level-1 cells
  std::vector<int32_t> famap;         // [n_fam * mf] level DoF ids of the family nodes
  std::vector<uint32_t> own;          // [n_fam * own_words] family owns node bit
  std::vector<double> coeff;          // [n_cells]
  std::vector<int32_t> edge_cells;    // cells having an I node
  std::vector<int32_t> ilist;         // I node ids
};

struct Maps {
  int dim = 0, k = 0, n = 0, npc = 0, mf = 0, own_words = 0;
  FE1D fe;
  int64_t n_leaves = 0, n_dofs = 0, n_hanging = 0;
  std::vector<int32_t> leaf_cellmap;  // [n_leaves * npc] DoF id or -(h+1)
  // In-cell form of the hanging-node constraints: on a face or edge of a
  // leaf shared with a coarser leaf, the cell holds the DoFs of its parent's
  // nodes at the same local positions and interpolates them with the 1D
  // embedding rows of its child position.
  std::vector<int32_t> leaf_cellmap_parent;  // [n_leaves * npc] DoF ids only
  // bits 0..2 child position (x, y, z) in the parent, 3..5 hanging face
  // normal to x / y / z (on the child's side of the parent), 6..8 hanging
  // edge along x / y / z (at the child's corner edge of the parent)
  std::vector<uint16_t> leaf_mask;
  std::vector<int8_t> leaf_level;
  std::vector<int32_t> leaf_anchor;   // [n_leaves * 3] global anchors (units 2^-20)
  std::vector<double> leaf_coeff;
  std::vector<uint8_t> dirichlet;     // [n_dofs]
  std::vector<int64_t> con_off;       // [n_hanging+1]
  std::vector<int32_t> con_mas;
  std::vector<double> con_w;
  std::vector<int8_t> copy_level;     // [n_dofs]
  std::vector<int32_t> copy_index;    // [n_dofs]
  std::vector<LevelData> levels;
  std::vector<LevelLayout> layouts;  // device layout of levels >= 1
  LeafTiles tiles;                   // tiled leaf operator (empty in 3D at degree >= 3)
};

// threads: host threads for the leaf-mesh phases (0: the hardware's, at
// most 16); the result does not depend on it.
Maps build_maps(const Forest& f, int k, const double* coeff, int threads = 0);

}  // namespace gmg

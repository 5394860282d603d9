// Tiles of the leaf operator (the constrained operator q = C^T A C p of
// Sec. 2.1/2.3 on the leaf mesh): runs of consecutive leaf cells, each run
// processed by one wavefront that gathers the values of all nodes its cells
// touch once into LDS and adds its cells' results per node in LDS (the
// results of constrained positions, owed to the parent's nodes, included).
// A node whose contributions all come from one tile is written by that tile
// directly; the other nodes collect one partial sum per tile that touches
// them and are summed in a second pass in a fixed order.
#pragma once
#include <cstdint>
#include <vector>

namespace gmg {

struct Maps;

struct LeafTiles {
  static constexpr int kCells = 64;  // cells per tile (one wavefront)
  int64_t n_tiles = 0;
  int32_t max_nodes = 0;             // largest node count of a tile
  // per tile: first entry in `node`, numbers of complete and partial nodes,
  // first partial slot
  std::vector<int64_t> node_off;     // [n_tiles + 1]
  std::vector<int32_t> n_complete;   // [n_tiles]
  std::vector<int32_t> n_partial;    // [n_tiles]
  std::vector<int32_t> pbase;        // [n_tiles]
  // DoF of each tile node, complete nodes first (first-touch order), then
  // partial ones; a complete Dirichlet node is stored as ~dof
  std::vector<int32_t> node;
  // per (cell, local position): index of its target in the tile's node list
  std::vector<uint16_t> lmap;        // [n_leaves * npc], cell-major
  int64_t n_part = 0;                // partial slots
  // second pass: nodes summed from partial slots (ascending DoF), their slot
  // lists (ascending slot index)
  std::vector<int32_t> p2_dof;
  std::vector<int32_t> p2_off;       // [n_p2 + 1]
  std::vector<int32_t> p2_slot;
};

// threads: host threads (0: the hardware's, at most 16); the result does not
// depend on it
LeafTiles build_leaf_tiles(const Maps& M, int threads = 0);

}  // namespace gmg

// Tiles of the leaf operator (the constrained operator q = C^T A C p of
// Sec. 2.1/2.3 on the leaf mesh): runs of consecutive leaf cells, each run
// processed by one wavefront that gathers the values of all nodes its cells
// touch once into LDS and adds its cells' results per node in LDS (the
// results of constrained positions, owed to the parent's nodes, included).
//
// The leaf DoFs are numbered by first touch in leaf order, so the DoFs first
// touched by the cells of one tile form a contiguous range: the tile's own
// nodes.  A tile reads and writes its own nodes as that range (no index
// list); it writes its own nodes' sums to q directly.  The other nodes it
// touches (own nodes of other tiles: shared nodes of earlier or later tiles
// and parent nodes reached through hanging-node constraints) are listed; it
// writes their sums to one slot per listed entry, and a second pass adds each
// node's slots to q in ascending slot order.
#pragma once
#include <cstdint>
#include <vector>

namespace gmg {

struct Maps;

struct LeafTiles {
  static constexpr int kCells = 64;  // cells per tile (one wavefront)
  int64_t n_tiles = 0;
  int32_t max_nodes = 0;             // largest node count (own + listed) of a tile
  // per tile: its own DoFs [own[t], own[t+1]) and its listed nodes
  // [list_off[t], list_off[t+1]) in `list`; listed entry i has slot i
  std::vector<int32_t> own;          // [n_tiles + 1]
  std::vector<int64_t> list_off;     // [n_tiles + 1]
  std::vector<int32_t> list;         // listed node DoFs, per tile in first-reference order, and one
                                     // padding entry (0)
  // per (cell, local position): index of its target in the tile's nodes (own
  // nodes at 0..R-1 in DoF order, then the listed ones)
  std::vector<uint16_t> lmap;        // [n_leaves * npc], cell-major
  // second pass: the nodes with listed entries (ascending DoF) and their
  // slots (ascending)
  std::vector<int32_t> p2_dof;
  std::vector<int32_t> p2_off;       // [n_p2 + 1]
  std::vector<int32_t> p2_slot;
  int64_t n_slots() const { return list_off.empty() ? 0 : list_off.back(); }
};

// threads: host threads (0: the hardware's, at most 16); the result does not
// depend on it
LeafTiles build_leaf_tiles(const Maps& M, int threads = 0);

}  // namespace gmg

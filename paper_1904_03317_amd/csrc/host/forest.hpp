// Forest of quad/hex trees over unit coarse cells with isotropic refinement
// (Sec. 2.2), cell levels and leaf mesh (Sec. 2.3) and 2:1 closure (Sec. 3.5:
// leaves that touch differ by at most one level).  Leaves are kept in
// canonical order: coarse cell, then z-order of the anchor.
#pragma once
#include <array>
#include <cstdint>
#include <vector>

#include "common.hpp"

namespace gmg {

constexpr int kDepth = 20;         // anchors in units of 2^-20
constexpr int kMaxLevel = 16;     // key: 7 bits tree, 3 x 16 bits z-order, 5 bits level
constexpr int kMaxCoarse = 128;
constexpr int kMaxExtent = 16;     // bounding box of the coarse mesh, unit cells per axis

inline int64_t side_of(int level) { return int64_t(1) << (kDepth - level); }
inline int64_t floor_to(int64_t v, int64_t s) {
  int64_t q = v / s;
  if (v % s != 0 && v < 0) --q;
  return q * s;
}

struct Cell {
  int8_t level = 0;
  int16_t tree = 0;
  std::array<int32_t, 3> a{};   // global anchor, units 2^-20
};

struct Leaf {
  uint64_t key;
  Cell c;
};

class Forest {
 public:
  Forest(int dim, int n_coarse, const int32_t* origins);

  int dim() const { return dim_; }
  int n_coarse() const { return (int)origins_.size(); }
  const std::vector<Leaf>& leaves() const { return leaves_; }
  // tree containing the unit cube with integer corner u, or -1
  int tree_of_unit(const int64_t* u) const;
  int tree_of_anchor(const int64_t* a) const;
  uint64_t key(int level, const int64_t* a, int tree) const;
  uint64_t key(const Cell& c) const;
  // 0 absent, 1 leaf, 2 refined
  uint8_t status(int level, const int64_t* a) const;
  int64_t refine(const uint8_t* flags);
  const std::array<int32_t, 3>& box_lo() const { return lo_; }
  int max_level() const;
  // neighbour offsets in {-1,0,1}^dim minus 0, in lexicographic order
  const std::vector<std::array<int, 3>>& offsets() const { return offsets_; }

 private:
  void set_children(const Cell& c);
  void emit(const Cell& c, std::vector<Leaf>& out) const;
  int dim_;
  std::vector<std::array<int32_t, 3>> origins_;
  std::array<int32_t, 3> lo_{}, ext_{};
  std::vector<int16_t> unit_tree_;   // dense over the bounding box
  std::vector<Leaf> leaves_;
  CellMap cells_;
  std::vector<std::array<int, 3>> offsets_;
};

}  // namespace gmg

// Device layout of the level vectors on levels >= 1 (families of 2^d
// siblings, Sec. 2.2 / 2.3).  A family's (2k+1)^d node patch splits into
// 3^d entities by the position of each axis coordinate (low face, inside,
// high face): the family interior, its facets, edges (3D) and vertices.  An
// entity with r axes on the patch boundary is shared by at most 2^r
// families, and the family's position around it is the bit pattern of
// those axes.  Level DoFs are renumbered section by section (r = 0, 1, ..);
// inside a section entity by entity, and inside an entity lexicographically
// over its inside axes (x fastest).  A family then needs only the base index
// of each of its 3^d entities; every node index and every operator slot
// follows by arithmetic.
#pragma once
#include <cstdint>
#include <vector>

namespace gmg {

struct Maps;

struct LevelLayout {
  int64_t n_fam = 0, n_dofs = 0;
  // node index where section r begins (r = 0 interiors .. d vertices),
  // sec[d + 1] = n_dofs; unused entries equal n_dofs.  Inside a section the
  // entities shared by two or more families come first.
  int64_t sec[5] = {0, 0, 0, 0, 0};
  int64_t nsh[5] = {0, 0, 0, 0, 0};     // shared entities of section r
  // prefix sums of the shared nodes over the sections (pass 2 ranges):
  // shn[1] = 0, shn[r + 1] = shn[r] + nsh[r] * size_r
  int64_t shn[5] = {0, 0, 0, 0, 0};
  // first shared entity (pmask index) and first operator slot of section r
  // (2^r slots per shared node)
  int64_t entoff[5] = {0, 0, 0, 0, 0};
  int64_t eoff[5] = {0, 0, 0, 0, 0};
  int64_t n_ent = 0, n_slots = 0;       // shared entities, operator slots
  std::vector<int32_t> perm;    // [n_dofs] level DoF id -> device index
  std::vector<int32_t> gbase;   // [n_fam * 3^d] device index of each entity's first node
  std::vector<uint32_t> own;    // [n_fam] bit j: the family owns entity j (transfers)
  std::vector<uint32_t> excl;   // [n_fam] bit j: no other family touches entity j
  std::vector<uint8_t> pmask;   // [n_ent] bit p: the family at position p exists
  std::vector<int32_t> child;   // [n_fam * 2^d] family on the next finer level of each cell, or -1
};

// layouts[l] for l >= 1 (layouts[0] stays empty: level 0 keeps its numbering)
void build_layouts(Maps& M);

}  // namespace gmg

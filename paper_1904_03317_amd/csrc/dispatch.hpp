// Host-side launchers of the degree- and dimension-templated kernels.  One
// translation unit per (dim, k) instantiates them (inst_*.hip) and registers
// a table, so the heavy unrolled kernels compile in parallel.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace gmg {

// Device view of one level, passed to the kernels by value.  Level 0 keeps
// its own numbering and per-cell maps; levels >= 1 use the entity layout of
// their families (host/layout.hpp) and hold no per-node or per-cell maps.
struct LevelView {
  int64_t n_cells = 0, n_dofs = 0, n_fam = 0;
  const double* scale = nullptr;    // per-cell a_K h^{d-2}, or null
  double scale0 = 1.0;              // uniform value when scale is null
  const uint8_t* flags = nullptr;   // [n_dofs] 0 S, 1 I, 2 D
  // level 0: per-cell node map, operator slots of (cell, local node) in a
  // node-major buffer with per-node ranges, and the ranges of the
  // contributions restricted from level 1
  const int32_t* cmap = nullptr;    // SoA [npc][n_cells]
  const int32_t* slot = nullptr;    // SoA [npc][n_cells]
  const int32_t* soff = nullptr;    // [n_dofs + 1]
  const int32_t* roff = nullptr;    // [n_dofs + 1]
  // levels >= 1: entity layout
  const int32_t* gbase = nullptr;   // SoA [3^d][n_fam] device index of each entity's first node
  const uint32_t* own = nullptr;    // [n_fam] bit j: the family owns entity j
  const uint32_t* excl = nullptr;   // [n_fam] bit j: no other family touches entity j
  const uint8_t* pmask = nullptr;   // [entities] present positions
  const int32_t* parent = nullptr;  // [n_fam] parent cell on the next coarser level
  const int32_t* child = nullptr;   // SoA [2^d][n_fam] family of each cell on the next finer level, or -1
  const int32_t* rslot = nullptr;   // level 1: SoA [npc][n_fam] level-0 slots of the parent nodes
  int64_t sec[5] = {0, 0, 0, 0, 0};     // first node of section r (r = boundary axes)
  int64_t shn[5] = {0, 0, 0, 0, 0};     // prefix sums of the shared nodes of the sections
  int64_t entoff[5] = {0, 0, 0, 0, 0};  // first shared entity of section r
  int64_t eoff[5] = {0, 0, 0, 0, 0};    // first slot of section r (2^r slots per shared node)
};

struct LeafView {
  // 3D at degree >= 3: cells with in-cell constraints first, [0, n_con);
  // otherwise n_con = n_cells
  int64_t n_cells = 0, n_dofs = 0, n_con = 0;
  const int32_t* cmap = nullptr;    // SoA [npc][n_cells], parent-arranged DoFs on refinement edges
  const uint16_t* mask = nullptr;   // [n_cells] in-cell constraint mask
  const double* scale = nullptr;    // a_K h^{d-2}
  const double* mscale = nullptr;   // h^d
  const int32_t* slot = nullptr;    // SoA [npc][n_cells] slot in the node-major buffer
  const int32_t* soff = nullptr;    // [n_dofs + 1]
  const uint8_t* dir = nullptr;     // [n_dofs] Dirichlet flag
  // tiles of 64 cells (all but 3D at degree >= 3; host/leaftiles.hpp): per
  // tile its own DoF range and its listed nodes (listed entry i writes slot
  // i); per (position, cell) the tile-local node (own nodes first, then the
  // listed ones); the second-pass nodes and their slot lists
  int64_t n_tiles = 0, n_slots = 0, n_p2 = 0;
  int32_t max_nodes = 0;
  const int32_t* t_own = nullptr;   // [n_tiles + 1]
  const int64_t* t_loff = nullptr;  // [n_tiles + 1]
  const int32_t* t_list = nullptr;  // [n_slots]
  const uint16_t* lmap = nullptr;   // SoA [npc][n_cells]
  const int32_t* p2_dof = nullptr;  // [n_p2]
  const int32_t* p2_off = nullptr;  // [n_p2 + 1]
  const int32_t* p2_slot = nullptr;
};

template <typename T>
struct MatsH {
  T M[25], K[25], E[45];
};

namespace dev {
template <typename T>
struct Epi;
template <typename T>
struct OpItem;
template <typename T>
struct SumItem;
template <typename T>
struct XferItem;
struct LeafItem;
struct EstView;
struct EstMatsD;
}

// kinds of batched transfers (LevelOps::xfer_batch)
enum XferKind { kXRFine = 0, kXRestrict = 1, kXRestrict0 = 2, kXProlong = 3 };

template <typename T>
struct LevelOps {
  // levels >= 1, pass 1 of the operator: interior values through the
  // epilogue epi (dev::kEpi*), shared-entity values into the slots E
  void (*op)(const LevelView&, int epi, const T* x, const dev::Epi<T>&, T* E, const MatsH<T>&, hipStream_t);
  // levels >= 1, pass 2: shared nodes, same epilogue
  void (*sum)(const LevelView&, int epi, const T* E, const dev::Epi<T>&, hipStream_t);
  // restriction of the fine residual r into coarse level >= 1: the
  // restricted values of each fine family's parent cell into rb, then the
  // coarse patches (rstart epilogue on their final nodes, coarse slots for
  // the rest)
  void (*restrict_fc)(const LevelView& fine, const LevelView& coarse, const T* r, const dev::Epi<T>& coarse_ep,
                      T* rb, T* E, const MatsH<T>&, hipStream_t);
  // restriction from level 1 into the level-0 slots
  void (*restrict0)(const LevelView& fine, const T* r, T* E, const MatsH<T>&, hipStream_t);
  // x_f += P x_c
  void (*prolong)(const LevelView& fine, const LevelView& coarse, const T* xc, T* xf, const MatsH<T>&,
                  hipStream_t);
  // level 0, pass 1 of the operator: cell results into the node-major slots
  void (*cell_e)(const LevelView&, const T* x, T* E, const MatsH<T>&, hipStream_t);
  // pass 1 and pass 2 of several levels in one launch (device item tables,
  // b0 set from op_blocks / sum_blocks); op_batch is null where pass 1 has
  // no batched form (3D at k >= 3)
  void (*op_batch)(const dev::OpItem<T>* items, int n, int64_t blocks, int epi, const MatsH<T>&, hipStream_t);
  void (*sum_batch)(const dev::SumItem<T>* items, int n, int64_t blocks, int epi, hipStream_t);
  int64_t (*op_blocks)(const LevelView&);   // pass-1 blocks of a level
  // transfers of several problems in one launch (XferKind; the blocks of an
  // item from xfer_blocks of its fine level, coarse level for kXRestrict);
  // null where they have no batched form (3D at k >= 3)
  void (*xfer_batch)(int kind, const dev::XferItem<T>* items, int n, int64_t blocks, const MatsH<T>&, hipStream_t);
  int64_t (*xfer_blocks)(int kind, const LevelView&);
};

struct KernelTable {
  LevelOps<float> f32;
  LevelOps<double> f64;
  // pass 1 of the leaf operator (or mass matrix): cell results into slots
  // (3D at degree >= 3)
  void (*leaf_e)(const LeafView&, const double* x, double* E, bool mass, const MatsH<double>&, hipStream_t);
  // tiled leaf operator, pass 1: each tile's own nodes into y, its listed
  // nodes into the slots E; with part, one partial sum of x.y per block over
  // the own nodes (pass 2 adds the listed nodes' share); returns the grid
  unsigned (*leaf_t)(const LeafView&, const double* x, double* y, double* E, double* part, bool mass,
                     const MatsH<double>&, hipStream_t);
  // level 0: diagonal of the operator accumulated per node
  void (*diag0)(const LevelView&, double* diag, const MatsH<double>&, hipStream_t);
  // the tiled leaf operator (with partial sums of x.y) of several problems
  // in one launch, lds: the largest dynamic LDS of the items; null for 3D at
  // degree >= 3
  void (*leaf_t_batch)(const dev::LeafItem* items, int n, int64_t blocks, size_t lds, const MatsH<double>&,
                       hipStream_t);
  // residual error estimator (Sec. 4.3): eta[c] for every leaf from the
  // solution u and the nodal right-hand side f (leaf DoF vectors)
  void (*est)(const dev::EstView&, const double* u, const double* f, double* eta, const dev::EstMatsD&, hipStream_t);
};

const KernelTable* kernel_table(int dim, int k);
void register_table(int dim, int k, const KernelTable* t);

}  // namespace gmg

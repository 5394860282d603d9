// Host-side launchers of the degree- and dimension-templated kernels.  One
// translation unit per (dim, k) instantiates them (inst_*.hip) and registers
// a table, so the heavy unrolled kernels compile in parallel.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace gmg {

struct LevelView {
  int64_t n_cells = 0, n_dofs = 0, n_fam = 0, n_edge = 0;
  const int32_t* cmap = nullptr;    // SoA [npc][n_cells]
  const double* scale = nullptr;    // per-cell a_K h^{d-2}, or null
  double scale0 = 1.0;              // uniform value when scale is null
  const uint8_t* flags = nullptr;
  const int32_t* edge = nullptr;
  const int32_t* famap = nullptr;   // SoA [mf][n_fam]
  const uint32_t* own = nullptr;    // SoA [own_words][n_fam]
  const int32_t* parent = nullptr;
  // two-pass operator: slot of (cell, local node) in the node-major buffer,
  // and per-node slot ranges
  const int32_t* slot = nullptr;    // SoA [npc][n_cells] (level 0: per-cell slots)
  const int32_t* fslot = nullptr;   // SoA [mf][n_fam] (levels >= 1: per-family patch slots)
  const int32_t* soff = nullptr;    // [n_dofs + 1]
  // restriction into the next coarser level: slot of (family, parent node)
  const int32_t* rslot = nullptr;   // SoA [npc][n_fam]
  // slot ranges of the contributions restricted from the next finer level
  const int32_t* roff = nullptr;    // [n_dofs + 1]
};

struct LeafView {
  int64_t n_cells = 0, n_dofs = 0;
  const int32_t* cmap = nullptr;    // SoA [npc][n_cells], parent-arranged DoFs on refinement edges
  const uint16_t* mask = nullptr;   // [n_cells] in-cell constraint mask
  const double* scale = nullptr;    // a_K h^{d-2}
  const double* mscale = nullptr;   // h^d
  const int32_t* slot = nullptr;    // SoA [npc][n_cells] slot in the node-major buffer
  const int32_t* soff = nullptr;    // [n_dofs + 1]
  const uint8_t* dir = nullptr;     // [n_dofs] Dirichlet flag
};

template <typename T>
struct MatsH {
  T M[25], K[25], E[45];
};

template <typename T>
struct LevelOps {
  // pass 1 of y = A x over all cells: cell results into the slots E
  void (*apply_e)(const LevelView&, const T* x, T* E, const MatsH<T>&, hipStream_t);
  // y[S] += sign * A^{SI} x^I on the edge cells (atomic scatter; test hook)
  void (*edge)(const LevelView&, const T* x, T* y, T sign, const MatsH<T>&, hipStream_t);
  // x_f += P x_c on owned fine nodes
  void (*prolong)(const LevelView& fine, const LevelView& coarse, const T* xc, T* xf, const MatsH<T>&,
                  hipStream_t);
  // family contributions of R r to the parent-node slots E
  void (*restrict_e)(const LevelView& fine, const T* r, T* E, const MatsH<T>&, hipStream_t);
};

struct KernelTable {
  LevelOps<float> f32;
  LevelOps<double> f64;
  // pass 1 of the leaf operator (or mass matrix): cell results into slots
  void (*leaf_e)(const LeafView&, const double* x, double* E, bool mass, const MatsH<double>&, hipStream_t);
  void (*diag)(const LevelView&, double* diag, const MatsH<double>&, hipStream_t);
};

const KernelTable* kernel_table(int dim, int k);
void register_table(int dim, int k, const KernelTable* t);

}  // namespace gmg

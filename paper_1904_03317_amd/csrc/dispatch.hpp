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
};

struct LeafView {
  int64_t n_cells = 0, n_dofs = 0;
  const int32_t* cmap = nullptr;    // SoA [npc][n_cells], hanging h as n_dofs + h
  const double* scale = nullptr;    // a_K h^{d-2}
  const double* mscale = nullptr;   // h^d
};

template <typename T>
struct MatsH {
  T M[25], K[25], E[45];
};

template <typename T>
struct LevelOps {
  // y += A x over all cells (plain gather/scatter)
  void (*apply)(const LevelView&, const T* x, T* y, const MatsH<T>&, hipStream_t);
  // y[S] += sign * A^{SI} x^I on the edge cells
  void (*edge)(const LevelView&, const T* x, T* y, T sign, const MatsH<T>&, hipStream_t);
  // x_f += P x_c on owned fine nodes
  void (*prolong)(const LevelView& fine, const LevelView& coarse, const T* xc, T* xf, const MatsH<T>&,
                  hipStream_t);
  // d_c += R (g - t) over free owned fine nodes; t := 0 on them
  void (*restrict_)(const LevelView& fine, const LevelView& coarse, const T* g, T* t, T* dc,
                    const MatsH<T>&, hipStream_t);
};

struct KernelTable {
  LevelOps<float> f32;
  LevelOps<double> f64;
  // leaf operator / mass into y (n_dofs) and yh (hanging), both pre-zeroed
  void (*leaf_apply)(const LeafView&, const double* x, const double* xh, double* y, double* yh, bool mass,
                     const MatsH<double>&, hipStream_t);
  void (*diag)(const LevelView&, double* diag, const MatsH<double>&, hipStream_t);
};

const KernelTable* kernel_table(int dim, int k);
void register_table(int dim, int k, const KernelTable* t);

}  // namespace gmg

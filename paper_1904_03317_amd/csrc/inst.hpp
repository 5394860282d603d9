// Instantiation of the kernel table for one (dim, k); included by inst_*.hip.
#pragma once
#include "dispatch.hpp"
#include "gmg.h"
#include "host/common.hpp"
#include "kernels.hpp"

namespace gmg {

template <typename T>
inline dev::Mats<T> to_dev(const MatsH<T>& h) {
  dev::Mats<T> m;
  for (int i = 0; i < 25; ++i) {
    m.M[i] = h.M[i];
    m.K[i] = h.K[i];
  }
  for (int i = 0; i < 45; ++i) m.E[i] = h.E[i];
  return m;
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + dev::kBlock - 1) / dev::kBlock); }

template <int DIM, int K>
struct Inst {
  static constexpr int N = K + 1;

  template <typename T>
  static void apply_e(const LevelView& v, const T* x, T* E, const MatsH<T>& m, hipStream_t s) {
    if (!v.n_cells) return;
    if (v.n_fam > 0 && v.fslot) {
      using S = dev::FamilyShape<DIM, K, T>;
      const unsigned g = (unsigned)((v.n_fam + S::FB - 1) / S::FB);
      hipLaunchKernelGGL((dev::family_to_slots<DIM, K, T>), dim3(g), dim3(S::THREADS), 0, s, v.n_fam, v.famap,
                         v.fslot, v.scale, v.scale0, x, E, to_dev(m));
      return;
    }
    if (!v.slot) fail(GMG_E_STATE, "level operator has neither cell nor family slots");
    hipLaunchKernelGGL((dev::cell_to_slots<DIM, N, T, false, false>), dim3(grid_for(v.n_cells)), dim3(dev::kBlock),
                       0, s, v.n_cells, v.cmap, v.slot, v.scale, v.scale0, x, (const uint16_t*)nullptr, E,
                       to_dev(m));
  }
  template <typename T>
  static void edge(const LevelView& v, const T* x, T* y, T sign, const MatsH<T>& m, hipStream_t s) {
    if (!v.n_edge) return;
    hipLaunchKernelGGL((dev::cell_apply<DIM, N, T, 2, false>), dim3(grid_for(v.n_edge)), dim3(dev::kBlock), 0, s,
                       v.n_edge, v.edge, v.n_cells, v.cmap, v.scale, v.scale0, x, (const T*)nullptr, y,
                       (T*)nullptr, (int64_t)0, v.flags, sign, to_dev(m));
  }
  template <typename T>
  static void prolong(const LevelView& f, const LevelView& c, const T* xc, T* xf, const MatsH<T>& m,
                      hipStream_t s) {
    if (!f.n_fam) return;
    hipLaunchKernelGGL((dev::prolongate<DIM, K, T>), dim3(grid_for(f.n_fam)), dim3(dev::kBlock), 0, s, f.n_fam,
                       f.famap, f.own, f.parent, c.n_cells, c.cmap, xc, xf, to_dev(m));
  }
  template <typename T>
  static void restrict_e(const LevelView& f, const T* r, T* E, const MatsH<T>& m, hipStream_t s) {
    if (!f.n_fam) return;
    hipLaunchKernelGGL((dev::restrict_to_slots<DIM, K, T>), dim3(grid_for(f.n_fam)), dim3(dev::kBlock), 0, s,
                       f.n_fam, f.famap, f.own, r, f.rslot, E, to_dev(m));
  }
  static void leaf_e(const LeafView& v, const double* x, double* E, bool mass, const MatsH<double>& m,
                     hipStream_t s) {
    if (!v.n_cells) return;
    if (mass)
      hipLaunchKernelGGL((dev::cell_to_slots<DIM, N, double, true, true>), dim3(grid_for(v.n_cells)),
                         dim3(dev::kBlock), 0, s, v.n_cells, v.cmap, v.slot, v.mscale, 1.0, x, v.mask, E, to_dev(m));
    else
      hipLaunchKernelGGL((dev::cell_to_slots<DIM, N, double, true, false>), dim3(grid_for(v.n_cells)),
                         dim3(dev::kBlock), 0, s, v.n_cells, v.cmap, v.slot, v.scale, 1.0, x, v.mask, E, to_dev(m));
  }
  static void diag(const LevelView& v, double* d, const MatsH<double>& m, hipStream_t s) {
    if (!v.n_cells) return;
    hipLaunchKernelGGL((dev::cell_diag<DIM, N>), dim3(grid_for(v.n_cells)), dim3(dev::kBlock), 0, s, v.n_cells,
                       v.cmap, v.scale, v.scale0, d, to_dev(m));
  }

  static const KernelTable* table() {
    static KernelTable t = {
        {&apply_e<float>, &edge<float>, &prolong<float>, &restrict_e<float>},
        {&apply_e<double>, &edge<double>, &prolong<double>, &restrict_e<double>},
        &leaf_e,
        &diag,
    };
    return &t;
  }
};

}  // namespace gmg

#define GMG_INSTANTIATE(DIM, K)                                                        \
  namespace {                                                                          \
  struct Reg##DIM##K {                                                                 \
    Reg##DIM##K() { gmg::register_table(DIM, K, gmg::Inst<DIM, K>::table()); }         \
  } reg_##DIM##K;                                                                      \
  }

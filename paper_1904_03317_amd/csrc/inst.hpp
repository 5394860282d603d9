// Instantiation of the kernel table for one (dim, k); included by inst_*.hip.
#pragma once
#include "dispatch.hpp"
#include "gmg.h"
#include "host/common.hpp"
#include "estkernels.hpp"
#include "famkernels.hpp"
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

  template <typename T, int EPI>
  static void op_launch(const LevelView& v, const T* x, const dev::Epi<T>& ep, T* E, const MatsH<T>& m,
                        hipStream_t s) {
    if constexpr (dev::kCoopOp<DIM, K>) {
      using S = dev::CoopShape<DIM, K, T>;
      const unsigned g = (unsigned)((v.n_fam + S::FB - 1) / S::FB);
      hipLaunchKernelGGL((dev::fam_op_coop<DIM, K, T, EPI>), dim3(g), dim3(S::THREADS), 0, s, v, x, ep, E,
                         to_dev(m));
    } else {
      using S = dev::FamShape<DIM, K, T>;
      const unsigned g = (unsigned)((v.n_fam + S::FB - 1) / S::FB);
      hipLaunchKernelGGL((dev::fam_op<DIM, K, T, EPI>), dim3(g), dim3(S::THREADS), 0, s, v, x, ep, E,
                         to_dev(m));
    }
  }
  template <typename T>
  static void op(const LevelView& v, int epi, const T* x, const dev::Epi<T>& ep, T* E, const MatsH<T>& m,
                 hipStream_t s) {
    if (!v.n_fam) return;
    if (!v.gbase) fail(GMG_E_STATE, "level operator called on a level without families");
    switch (epi) {
      case dev::kEpiPlain:
        return op_launch<T, dev::kEpiPlain>(v, x, ep, E, m, s);
      case dev::kEpiCheb:
        return op_launch<T, dev::kEpiCheb>(v, x, ep, E, m, s);
      case dev::kEpiResid:
        return op_launch<T, dev::kEpiResid>(v, x, ep, E, m, s);
      case dev::kEpiDiag:
        if constexpr (sizeof(T) == 8) return op_launch<T, dev::kEpiDiag>(v, x, ep, E, m, s);
        break;
      default:
        break;
    }
    fail(GMG_E_INVAL, "unsupported operator epilogue");
  }
  template <typename T>
  static void sum(const LevelView& v, int epi, const T* E, const dev::Epi<T>& ep, hipStream_t s) {
    const int64_t nb = v.shn[DIM + 1];
    if (nb <= 0) return;
    const dim3 g(grid_for(nb)), b(dev::kBlock);
    switch (epi) {
      case dev::kEpiPlain:
      case dev::kEpiDiag:
        hipLaunchKernelGGL((dev::fam_sum<DIM, K, T, dev::kEpiPlain>), g, b, 0, s, v, E, ep);
        return;
      case dev::kEpiCheb:
        hipLaunchKernelGGL((dev::fam_sum<DIM, K, T, dev::kEpiCheb>), g, b, 0, s, v, E, ep);
        return;
      case dev::kEpiResid:
        hipLaunchKernelGGL((dev::fam_sum<DIM, K, T, dev::kEpiResid>), g, b, 0, s, v, E, ep);
        return;
      case dev::kEpiRStart:
        hipLaunchKernelGGL((dev::fam_sum<DIM, K, T, dev::kEpiRStart>), g, b, 0, s, v, E, ep);
        return;
      default:
        break;
    }
    fail(GMG_E_INVAL, "unsupported operator epilogue");
  }
  template <typename T>
  static void restrict_fc(const LevelView& f, const LevelView& c, const T* r, const dev::Epi<T>& ep, T* rb, T* E,
                          const MatsH<T>& m, hipStream_t s) {
    if constexpr (dev::kCoopOp<DIM, K>) {
      using S = dev::CoopShape<DIM, K, T>;
      if (f.n_fam) {
        const unsigned g = (unsigned)((f.n_fam + S::FB - 1) / S::FB);
        hipLaunchKernelGGL((dev::fam_rfine_coop<DIM, K, T>), dim3(g), dim3(S::THREADS), 0, s, f, r, rb, to_dev(m));
      }
      if (!c.n_fam) return;
      const unsigned g = (unsigned)((c.n_fam + S::FB - 1) / S::FB);
      hipLaunchKernelGGL((dev::fam_restrict_coop<DIM, K, T>), dim3(g), dim3(S::THREADS), 0, s, c, (const T*)rb, ep,
                         E, to_dev(m));
    } else {
      using S = dev::FamShape<DIM, K, T>;
      if (f.n_fam) {
        const unsigned g = (unsigned)((f.n_fam + S::FB - 1) / S::FB);
        hipLaunchKernelGGL((dev::fam_rfine<DIM, K, T>), dim3(g), dim3(S::THREADS), 0, s, f, r, rb, to_dev(m));
      }
      if (!c.n_fam) return;
      const unsigned g = (unsigned)((c.n_fam + S::FB - 1) / S::FB);
      hipLaunchKernelGGL((dev::fam_restrict<DIM, K, T>), dim3(g), dim3(S::THREADS), 0, s, c, (const T*)rb, ep, E,
                         to_dev(m));
    }
  }
  template <typename T>
  static void restrict0(const LevelView& f, const T* r, T* E, const MatsH<T>& m, hipStream_t s) {
    if (!f.n_fam) return;
    hipLaunchKernelGGL((dev::fam_restrict0<DIM, K, T>), dim3(grid_for(f.n_fam)), dim3(dev::kBlock), 0, s, f, r, E,
                       to_dev(m));
  }
  template <typename T>
  static void prolong(const LevelView& f, const LevelView& c, const T* xc, T* xf, const MatsH<T>& m,
                      hipStream_t s) {
    if (!f.n_fam) return;
    if constexpr (dev::kCoopOp<DIM, K>) {
      using S = dev::CoopShape<DIM, K, T>;
      const unsigned g = (unsigned)((f.n_fam + S::FB - 1) / S::FB);
      hipLaunchKernelGGL((dev::fam_prolong_coop<DIM, K, T>), dim3(g), dim3(S::THREADS), 0, s, f, c, xc, xf,
                         to_dev(m));
    } else {
      using S = dev::FamShape<DIM, K, T>;
      const unsigned g = (unsigned)((f.n_fam + S::FB - 1) / S::FB);
      hipLaunchKernelGGL((dev::fam_prolong<DIM, K, T>), dim3(g), dim3(S::THREADS), 0, s, f, c, xc, xf, to_dev(m));
    }
  }
  template <typename T>
  static void cell_e(const LevelView& v, const T* x, T* E, const MatsH<T>& m, hipStream_t s) {
    if (!v.n_cells) return;
    if (!v.slot || !v.cmap) fail(GMG_E_STATE, "per-cell operator called on a level without cell maps");
    hipLaunchKernelGGL((dev::cell_to_slots<DIM, N, T, false, false>), dim3(grid_for(v.n_cells)), dim3(dev::kBlock),
                       0, s, v.n_cells, v.n_cells, v.cmap, v.slot, v.scale, v.scale0, x, (const uint16_t*)nullptr,
                       E, to_dev(m));
  }
  static void leaf_e(const LeafView& v, const double* x, double* E, bool mass, const MatsH<double>& m,
                     hipStream_t s) {
    if (!v.n_cells) return;
    // 3D, degree >= 3: the cooperative kernel, on the constrained cells
    // (first) with the in-cell constraint steps and on the rest without;
    // otherwise every cell lane by lane
    if constexpr (DIM == 3 && K >= 3) {
      using LC = dev::LeafCoop<N>;
      const dim3 b(LC::THREADS);
      const double* sc = mass ? v.mscale : v.scale;
      if (v.n_con) {
        const unsigned g = (unsigned)((v.n_con + LC::CB - 1) / LC::CB);
        if (mass)
          hipLaunchKernelGGL((dev::leaf_coop<N, true, true>), dim3(g), b, 0, s, v.n_cells, (int64_t)0, v.n_con,
                             v.cmap, v.slot, sc, 1.0, x, v.mask, E, to_dev(m));
        else
          hipLaunchKernelGGL((dev::leaf_coop<N, false, true>), dim3(g), b, 0, s, v.n_cells, (int64_t)0, v.n_con,
                             v.cmap, v.slot, sc, 1.0, x, v.mask, E, to_dev(m));
      }
      const int64_t nr = v.n_cells - v.n_con;
      if (nr) {
        const unsigned g = (unsigned)((nr + LC::CB - 1) / LC::CB);
        if (mass)
          hipLaunchKernelGGL((dev::leaf_coop<N, true, false>), dim3(g), b, 0, s, v.n_cells, v.n_con, v.n_cells,
                             v.cmap, v.slot, sc, 1.0, x, v.mask, E, to_dev(m));
        else
          hipLaunchKernelGGL((dev::leaf_coop<N, false, false>), dim3(g), b, 0, s, v.n_cells, v.n_con, v.n_cells,
                             v.cmap, v.slot, sc, 1.0, x, v.mask, E, to_dev(m));
      }
    } else {
      if (mass)
        hipLaunchKernelGGL((dev::cell_to_slots<DIM, N, double, true, true>), dim3(grid_for(v.n_cells)),
                           dim3(dev::kBlock), 0, s, v.n_cells, v.n_cells, v.cmap, v.slot, v.mscale, 1.0, x, v.mask,
                           E, to_dev(m));
      else
        hipLaunchKernelGGL((dev::cell_to_slots<DIM, N, double, true, false>), dim3(grid_for(v.n_cells)),
                           dim3(dev::kBlock), 0, s, v.n_cells, v.n_cells, v.cmap, v.slot, v.scale, 1.0, x, v.mask,
                           E, to_dev(m));
    }
  }
  static unsigned leaf_t(const LeafView& v, const double* x, double* y, double* E, double* part, bool mass,
                         const MatsH<double>& m, hipStream_t s) {
    if constexpr (DIM == 3 && K >= 3) {
      fail(GMG_E_STATE, "tiled leaf operator not built for 3D degree >= 3");
    } else {
      if (!v.n_tiles) return 0;
      const unsigned g = (unsigned)std::min<int64_t>(v.n_tiles, dev::kLeafBlocks);
      const size_t lds = size_t(v.max_nodes) * sizeof(double);
      if (mass)
        hipLaunchKernelGGL((dev::leaf_tiles<DIM, N, true, false>), dim3(g), dim3(64), lds, s, v, x, y, E, part,
                           to_dev(m));
      else if (part)
        hipLaunchKernelGGL((dev::leaf_tiles<DIM, N, false, true>), dim3(g), dim3(64), lds, s, v, x, y, E, part,
                           to_dev(m));
      else
        hipLaunchKernelGGL((dev::leaf_tiles<DIM, N, false, false>), dim3(g), dim3(64), lds, s, v, x, y, E, part,
                           to_dev(m));
      return g;
    }
  }
  static void diag0(const LevelView& v, double* d, const MatsH<double>& m, hipStream_t s) {
    if (!v.n_cells) return;
    hipLaunchKernelGGL((dev::cell_diag<DIM, N>), dim3(grid_for(v.n_cells)), dim3(dev::kBlock), 0, s, v.n_cells,
                       v.cmap, v.scale, v.scale0, d, to_dev(m));
  }

  template <typename T>
  static void op_batch(const dev::OpItem<T>* items, int n, int64_t blocks, int epi, const MatsH<T>& m,
                       hipStream_t s) {
    if constexpr (dev::kCoopOp<DIM, K>) {
      fail(GMG_E_STATE, "no batched level operator at this degree");
    } else {
      using S = dev::FamShape<DIM, K, T>;
      if (blocks <= 0) return;
      const dim3 g((unsigned)blocks), b(S::THREADS);
      switch (epi) {
        case dev::kEpiPlain:
          hipLaunchKernelGGL((dev::fam_op_batch<DIM, K, T, dev::kEpiPlain>), g, b, 0, s, items, n, to_dev(m));
          return;
        case dev::kEpiCheb:
          hipLaunchKernelGGL((dev::fam_op_batch<DIM, K, T, dev::kEpiCheb>), g, b, 0, s, items, n, to_dev(m));
          return;
        case dev::kEpiResid:
          hipLaunchKernelGGL((dev::fam_op_batch<DIM, K, T, dev::kEpiResid>), g, b, 0, s, items, n, to_dev(m));
          return;
        default:
          break;
      }
      fail(GMG_E_INVAL, "unsupported batched operator epilogue");
    }
  }
  template <typename T>
  static void sum_batch(const dev::SumItem<T>* items, int n, int64_t blocks, int epi, hipStream_t s) {
    if (blocks <= 0) return;
    const dim3 g((unsigned)blocks), b(dev::kBlock);
    switch (epi) {
      case dev::kEpiPlain:
        hipLaunchKernelGGL((dev::fam_sum_batch<DIM, K, T, dev::kEpiPlain>), g, b, 0, s, items, n);
        return;
      case dev::kEpiCheb:
        hipLaunchKernelGGL((dev::fam_sum_batch<DIM, K, T, dev::kEpiCheb>), g, b, 0, s, items, n);
        return;
      case dev::kEpiResid:
        hipLaunchKernelGGL((dev::fam_sum_batch<DIM, K, T, dev::kEpiResid>), g, b, 0, s, items, n);
        return;
      case dev::kEpiRStart:
        hipLaunchKernelGGL((dev::fam_sum_batch<DIM, K, T, dev::kEpiRStart>), g, b, 0, s, items, n);
        return;
      default:
        break;
    }
    fail(GMG_E_INVAL, "unsupported batched epilogue");
  }
  template <typename T>
  static int64_t op_blocks(const LevelView& v) {
    if constexpr (dev::kCoopOp<DIM, K>) {
      using S = dev::CoopShape<DIM, K, T>;
      return (v.n_fam + S::FB - 1) / S::FB;
    } else {
      using S = dev::FamShape<DIM, K, T>;
      return (v.n_fam + S::FB - 1) / S::FB;
    }
  }

  template <typename T>
  static void xfer_batch(int kind, const dev::XferItem<T>* items, int n, int64_t blocks, const MatsH<T>& m,
                         hipStream_t s) {
    if constexpr (dev::kCoopOp<DIM, K>) {
      fail(GMG_E_STATE, "no batched transfers at this degree");
    } else {
      using S = dev::FamShape<DIM, K, T>;
      if (blocks <= 0) return;
      const dim3 g((unsigned)blocks), b(S::THREADS);
      switch (kind) {
        case kXRFine:
          hipLaunchKernelGGL((dev::fam_rfine_batch<DIM, K, T>), g, b, 0, s, items, n, to_dev(m));
          return;
        case kXRestrict:
          hipLaunchKernelGGL((dev::fam_restrict_batch<DIM, K, T>), g, b, 0, s, items, n, to_dev(m));
          return;
        case kXRestrict0:
          hipLaunchKernelGGL((dev::fam_restrict0_batch<DIM, K, T>), g, dim3(dev::kBlock), 0, s, items, n, to_dev(m));
          return;
        case kXProlong:
          hipLaunchKernelGGL((dev::fam_prolong_batch<DIM, K, T>), g, b, 0, s, items, n, to_dev(m));
          return;
        default:
          break;
      }
      fail(GMG_E_INVAL, "unknown transfer kind");
    }
  }
  // blocks of one transfer launch (as restrict_fc, restrict0, prolong)
  template <typename T>
  static int64_t xfer_blocks(int kind, const LevelView& v) {
    if (kind == kXRestrict0) return grid_for(v.n_fam);
    if constexpr (dev::kCoopOp<DIM, K>) {
      using S = dev::CoopShape<DIM, K, T>;
      return (v.n_fam + S::FB - 1) / S::FB;
    } else {
      using S = dev::FamShape<DIM, K, T>;
      return (v.n_fam + S::FB - 1) / S::FB;
    }
  }
  static void leaf_t_batch(const dev::LeafItem* items, int n, int64_t blocks, size_t lds, const MatsH<double>& m,
                           hipStream_t s) {
    if constexpr (DIM == 3 && K >= 3) {
      fail(GMG_E_STATE, "tiled leaf operator not built for 3D degree >= 3");
    } else {
      if (blocks <= 0) return;
      hipLaunchKernelGGL((dev::leaf_tiles_batch<DIM, N>), dim3((unsigned)blocks), dim3(64), lds, s, items, n,
                         to_dev(m));
    }
  }

  static void est(const dev::EstView& v, const double* u, const double* f, double* eta, const dev::EstMatsD& m,
                  hipStream_t s) {
    if (!v.n_cells) return;
    hipLaunchKernelGGL((dev::est_cells<DIM, N>), dim3((unsigned)((v.n_cells + 63) / 64)), dim3(64), 0, s, v, u, f,
                       eta, m);
  }

  template <typename T>
  static constexpr LevelOps<T> ops() {
    return LevelOps<T>{&op<T>,        &sum<T>,   &restrict_fc<T>,
                       &restrict0<T>, &prolong<T>, &cell_e<T>,
                       dev::kCoopOp<DIM, K> ? nullptr : &op_batch<T>, &sum_batch<T>, &op_blocks<T>,
                       dev::kCoopOp<DIM, K> ? nullptr : &xfer_batch<T>, &xfer_blocks<T>};
  }
  static const KernelTable* table() {
    static KernelTable t = {ops<float>(), ops<double>(), &leaf_e, &leaf_t, &diag0,
                            (DIM == 3 && K >= 3) ? nullptr : &leaf_t_batch, &est};
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

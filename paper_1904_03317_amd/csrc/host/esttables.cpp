// Face tables of the residual error estimator (see esttables.hpp).
#include "esttables.hpp"

#include <algorithm>

#include "common.hpp"
#include "maps.hpp"

namespace gmg {

namespace {

// (level, anchor) -> leaf index, open addressing on the exact pair of words
// (level, a0) and (a1, a2)
class LeafIndex {
 public:
  explicit LeafIndex(const Maps& M) {
    size_t cap = 16;
    while (cap < 2 * size_t(M.n_leaves) + 16) cap <<= 1;
    k1_.assign(cap, kEmpty);
    k2_.assign(cap, 0);
    vals_.assign(cap, -1);
    mask_ = cap - 1;
    for (int64_t i = 0; i < M.n_leaves; ++i) put(M.leaf_level[i], &M.leaf_anchor[size_t(i) * 3], (int32_t)i);
  }
  int32_t find(int level, const int32_t* a) const {
    if (level < 0) return -1;
    const uint64_t w1 = word1(level, a), w2 = word2(a);
    size_t i = mix64(w1 ^ mix64(w2)) & mask_;
    while (k1_[i] != kEmpty) {
      if (k1_[i] == w1 && k2_[i] == w2) return vals_[i];
      i = (i + 1) & mask_;
    }
    return -1;
  }

 private:
  static constexpr uint64_t kEmpty = ~uint64_t(0);
  static uint64_t word1(int level, const int32_t* a) { return (uint64_t)(uint32_t)level << 32 | (uint32_t)a[0]; }
  static uint64_t word2(const int32_t* a) { return (uint64_t)(uint32_t)a[1] << 32 | (uint32_t)a[2]; }
  void put(int level, const int32_t* a, int32_t v) {
    const uint64_t w1 = word1(level, a), w2 = word2(a);
    size_t i = mix64(w1 ^ mix64(w2)) & mask_;
    while (k1_[i] != kEmpty) {
      if (k1_[i] == w1 && k2_[i] == w2) fail(-8, "estimator tables: a leaf twice");
      i = (i + 1) & mask_;
    }
    k1_[i] = w1;
    k2_[i] = w2;
    vals_[i] = v;
  }
  std::vector<uint64_t> k1_, k2_;
  std::vector<int32_t> vals_;
  size_t mask_ = 0;
};

}  // namespace

EstTables build_est_tables(const Maps& M) {
  EstTables T;
  const int dim = M.dim;
  T.dim = dim;
  T.nf = 2 * dim;
  T.nsub = 1 << (dim - 1);
  const int64_t nl = M.n_leaves;
  T.kind.assign(size_t(nl) * T.nf, kFaceBoundary);
  T.off.assign(size_t(nl) * T.nf, 0);
  T.nb.assign(size_t(nl) * T.nf * T.nsub, -1);
  T.con_off = M.con_off;
  if (T.con_off.empty()) T.con_off.push_back(0);
  LeafIndex idx(M);
  for (int64_t i = 0; i < nl; ++i) {
    const int lv = M.leaf_level[i];
    const int32_t* a = &M.leaf_anchor[size_t(i) * 3];
    const int32_t s = (int32_t)side_of(lv);
    for (int ax = 0; ax < dim; ++ax) {
      int tang[2] = {0, 0}, nt = 0;
      for (int b = 0; b < dim; ++b)
        if (b != ax) tang[nt++] = b;
      for (int hi = 0; hi < 2; ++hi) {
        const size_t f = size_t(i) * T.nf + 2 * ax + hi;
        int32_t na[3] = {a[0], a[1], a[2]};
        na[ax] += hi ? s : -s;
        int32_t* nbf = &T.nb[f * T.nsub];
        const int32_t j = idx.find(lv, na);
        if (j >= 0) {
          T.kind[f] = kFaceSame;
          nbf[0] = j;
          continue;
        }
        // coarser: the parent-level cell containing the neighbour position
        if (lv >= 1) {
          const int32_t ps = (int32_t)side_of(lv - 1);
          int32_t pa[3] = {0, 0, 0};
          for (int d = 0; d < dim; ++d) pa[d] = (int32_t)floor_to(na[d], ps);
          const int32_t jc = idx.find(lv - 1, pa);
          if (jc >= 0) {
            T.kind[f] = kFaceCoarser;
            nbf[0] = jc;
            uint8_t bits = 0;
            for (int t = 0; t < nt; ++t)
              if (a[tang[t]] != pa[tang[t]]) bits |= (uint8_t)(1u << t);
            T.off[f] = bits;
            continue;
          }
        }
        // finer: the children of the neighbour position touching the face
        const int32_t cs = s / 2;
        int found = 0;
        for (int b = 0; b < T.nsub; ++b) {
          int32_t ca[3] = {na[0], na[1], na[2]};
          ca[ax] = hi ? na[ax] : na[ax] + cs;
          for (int t = 0; t < nt; ++t)
            if ((b >> t) & 1) ca[tang[t]] += cs;
          const int32_t jf = idx.find(lv + 1, ca);
          nbf[b] = jf;
          found += jf >= 0;
        }
        if (found == T.nsub) {
          T.kind[f] = kFaceFiner;
        } else if (found != 0) {
          fail(-8, "estimator tables: a face with some but not all finer neighbours (2:1 balance)");
        } else {
          std::fill(nbf, nbf + T.nsub, -1);  // domain boundary
        }
      }
    }
  }
  return T;
}

EstMats est_mats(const Maps& M) {
  EstMats E{};
  const FE1D& fe = M.fe;
  const int n = fe.n, nq = n;
  double qx[5], qw[5];
  gauss_01(nq, qx, qw);
  for (int q = 0; q < nq; ++q) {
    E.w[q] = qw[q];
    lagrange_values(fe, qx[q], &E.V[q * n]);
    lagrange_second_derivs(fe, qx[q], &E.S[q * n]);
    lagrange_values(fe, 0.5 * qx[q], &E.VH[0][q * n]);
    lagrange_values(fe, 0.5 * (1.0 + qx[q]), &E.VH[1][q * n]);
  }
  lagrange_derivs(fe, 0.0, E.DE[0]);
  lagrange_derivs(fe, 1.0, E.DE[1]);
  return E;
}

}  // namespace gmg

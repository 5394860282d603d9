// Tables of the residual error estimator of the adaptive loop (Sec. 4.3) on
// the leaf mesh: for every leaf and face its neighbour(s) across the face,
// and the one-dimensional evaluation matrices at the (k+1)-point Gauss
// points.
#pragma once
#include <cstdint>
#include <vector>

namespace gmg {

struct Maps;

// face f = 2 axis + side (side 1: the face at the upper end of the axis)
enum EstFaceKind : uint8_t { kFaceBoundary = 0, kFaceSame = 1, kFaceCoarser = 2, kFaceFiner = 3 };

struct EstTables {
  int dim = 0, nf = 0, nsub = 0;   // 2 dim faces per leaf, 2^(dim-1) sub-faces per face
  std::vector<uint8_t> kind;       // [n_leaves * nf]
  // coarser neighbour: bit t set when the leaf lies in the upper half of the
  // neighbour's face along the t-th tangential axis (ascending axis order)
  std::vector<uint8_t> off;        // [n_leaves * nf]
  // neighbour leaves: same or coarser in entry 0; finer: the nsub leaves
  // touching the face, entry b with bit t of b = upper half along the t-th
  // tangential axis; -1 unused
  std::vector<int32_t> nb;         // [n_leaves * nf * nsub]
  // the constraint offsets of the leaf mesh, with at least one entry
  std::vector<int64_t> con_off;
};

// the face tables of the leaf mesh of M (fails if a face has no consistent
// neighbour, which 2:1 balance excludes)
EstTables build_est_tables(const Maps& M);

// one-dimensional matrices on [0, 1] for the nodes of M's element and its
// nq = k+1 Gauss points: values V[q n + j] = l_j(x_q), second derivatives
// S, values at the Gauss points of the lower and upper half (x_q / 2 and
// (1 + x_q) / 2) VH[h], first derivatives at the end points DE[e][j] =
// l_j'(e), Gauss weights w[q]
struct EstMats {
  double V[25], S[25], VH[2][25], DE[2][5], w[5];
};
EstMats est_mats(const Maps& M);

}  // namespace gmg

// HIP kernels for gfx950 (MI355X).  Matrix-free tensor-product operators on
// axis-aligned cells (Sec. 3.2 matrix-free evaluation, here re-designed for
// 64-wide wavefronts: one lane per cell, the whole cell tensor in registers),
// the leaf operator with in-cell hanging-node constraints, level-0 kernels,
// vector kernels of the smoother and the V-cycle (Sec. 4.1) and the FP64 CG.
// The level kernels of levels >= 1 are in famkernels.hpp.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dispatch.hpp"

namespace gmg {
namespace dev {

constexpr int kBlock = 256;

// 1D reference matrices passed by value (kernel arguments, read as scalars)
template <typename T>
struct Mats {
  T M[25];
  T K[25];
  T E[45];   // (2k+1) x (k+1), row-major
};

// The 1D matrices of degrees 1 and 2, whose Gauss-Lobatto nodes are the
// equidistant ones, as compile-time constants (the rationals the host's
// quadrature computes up to rounding): mass M_ij = int l_i l_j and
// stiffness K_ij = int l_i' l_j' on [0, 1], embedding rows E (2k+1 child
// nodes of the two halves by k+1 parent nodes).  Kernels that take them
// keep no matrix entries in registers.
template <int N>
struct Exact1D;
template <>
struct Exact1D<2> {
  static constexpr double M[4] = {2.0 / 6, 1.0 / 6, 1.0 / 6, 2.0 / 6};
  static constexpr double K[4] = {1.0, -1.0, -1.0, 1.0};
  static constexpr double E[6] = {1.0, 0.0, 0.5, 0.5, 0.0, 1.0};
};
template <>
struct Exact1D<3> {
  static constexpr double M[9] = {4.0 / 30, 2.0 / 30, -1.0 / 30, 2.0 / 30, 16.0 / 30, 2.0 / 30, -1.0 / 30, 2.0 / 30, 4.0 / 30};
  static constexpr double K[9] = {7.0 / 3, -8.0 / 3, 1.0 / 3, -8.0 / 3, 16.0 / 3, -8.0 / 3, 1.0 / 3, -8.0 / 3, 7.0 / 3};
  static constexpr double E[15] = {1.0,  0.0,    0.0,   0.375, 0.75, -0.125, 0.0, 1.0,
                                   0.0, -0.125, 0.75, 0.375, 0.0,  0.0,    1.0};
};

// Consecutive hardware dispatch goes round-robin over the 8 XCDs, each with
// its own L2.  Give each XCD one contiguous range of the logical block space
// so that neighbouring cells (which share nodes) hit the same L2.
__device__ __forceinline__ int64_t xcd_block_of(int64_t b, int64_t nb) {
  const int64_t q = nb / 8, r = nb % 8, x = b % 8, i = b / 8;
  return x * q + (x < r ? x : r) + i;
}
__device__ __forceinline__ int64_t xcd_block() { return xcd_block_of(blockIdx.x, gridDim.x); }
__device__ __forceinline__ int64_t xcd_tid() { return xcd_block() * blockDim.x + threadIdx.x; }

// ------------------------------------------------------------------ batched launches
// Kernel bodies below take their block index b and grid size nb as
// arguments, so that one launch can run the same body for several problems:
// item i of a batched launch covers the blocks [b0_i, b0_i + nb_i) of the
// grid and runs its body with b = blockIdx.x - b0_i.  Each item's blocks do
// exactly what the blocks of its own launch would do (same results bit for
// bit).

// the item of this block (items in ascending b0, the first at 0)
template <typename Item>
__device__ __forceinline__ int batch_item(const Item* items, int n) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (items[mid].b0 <= (int64_t)blockIdx.x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// a body (a device function object called with (b, nb)) and its blocks
template <class F>
struct LaunchItem {
  F f;
  int64_t b0, nb;
};

template <class F, int TH>
__global__ void __launch_bounds__(TH) run_items(const LaunchItem<F>* __restrict__ items, int n) {
  const int i = batch_item(items, n);
  const F f = items[i].f;
  f((int64_t)blockIdx.x - items[i].b0, items[i].nb);
}

template <typename T>
__device__ __forceinline__ void atomic_add(T* p, T v) {
  unsafeAtomicAdd(p, v);
}

// ------------------------------------------------------------------ sweeps
// 1D contraction along the axis with stride ST of an array of extent
// N_IN along that axis: out[i] = sum_j A[i*N_IN + j] in[j].
// The tensor of a cell is stored x fastest.

// y = (sum over directions of K in that direction, M elsewhere) x, 3D
template <int N, typename T, typename MT>
__device__ __forceinline__ void laplace3(const MT& m, const T (&u)[N * N * N], T (&out)[N * N * N]) {
  T a[N * N * N], b[N * N * N];
#pragma unroll
  for (int zy = 0; zy < N * N; ++zy) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T sa = 0, sb = 0;
#pragma unroll
      for (int j = 0; j < N; ++j) {
        sa += m.M[i * N + j] * u[zy * N + j];
        sb += m.K[i * N + j] * u[zy * N + j];
      }
      a[zy * N + i] = sa;
      b[zy * N + i] = sb;
    }
  }
  // y direction: c = M_y a, e = K_y a + M_y b (in place per line)
#pragma unroll
  for (int z = 0; z < N; ++z) {
#pragma unroll
    for (int x = 0; x < N; ++x) {
      T la[N], lb[N];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        la[j] = a[(z * N + j) * N + x];
        lb[j] = b[(z * N + j) * N + x];
      }
#pragma unroll
      for (int i = 0; i < N; ++i) {
        T sc = 0, se = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
          sc += m.M[i * N + j] * la[j];
          se += m.K[i * N + j] * la[j] + m.M[i * N + j] * lb[j];
        }
        a[(z * N + i) * N + x] = sc;
        b[(z * N + i) * N + x] = se;
      }
    }
  }
  // z direction: out = M_z e + K_z c
#pragma unroll
  for (int yx = 0; yx < N * N; ++yx) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T s = 0;
#pragma unroll
      for (int j = 0; j < N; ++j) s += m.M[i * N + j] * b[j * N * N + yx] + m.K[i * N + j] * a[j * N * N + yx];
      out[i * N * N + yx] = s;
    }
  }
}

template <int N, typename T, typename MT>
__device__ __forceinline__ void laplace2(const MT& m, const T (&u)[N * N], T (&out)[N * N]) {
  T a[N * N], b[N * N];
#pragma unroll
  for (int y = 0; y < N; ++y)
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T sa = 0, sb = 0;
#pragma unroll
      for (int j = 0; j < N; ++j) {
        sa += m.M[i * N + j] * u[y * N + j];
        sb += m.K[i * N + j] * u[y * N + j];
      }
      a[y * N + i] = sa;
      b[y * N + i] = sb;
    }
#pragma unroll
  for (int x = 0; x < N; ++x)
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T s = 0;
#pragma unroll
      for (int j = 0; j < N; ++j) s += m.K[i * N + j] * a[j * N + x] + m.M[i * N + j] * b[j * N + x];
      out[i * N + x] = s;
    }
}

// mass: out = (M x M [x M]) u
template <int DIM, int N, typename T, typename MT>
__device__ __forceinline__ void mass_nd(const MT& m, T* u, T* out) {
  constexpr int NP = DIM == 3 ? N * N * N : N * N;
  T a[NP];
#pragma unroll
  for (int r = 0; r < NP / N; ++r)
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T s = 0;
#pragma unroll
      for (int j = 0; j < N; ++j) s += m.M[i * N + j] * u[r * N + j];
      a[r * N + i] = s;
    }
  // y
#pragma unroll
  for (int z = 0; z < NP / (N * N); ++z)
#pragma unroll
    for (int x = 0; x < N; ++x)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        T s = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) s += m.M[i * N + j] * a[(z * N + j) * N + x];
        out[(z * N + i) * N + x] = s;
      }
  if (DIM == 3) {
#pragma unroll
    for (int yx = 0; yx < N * N; ++yx) {
      T l[N];
#pragma unroll
      for (int j = 0; j < N; ++j) l[j] = out[j * N * N + yx];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        T s = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) s += m.M[i * N + j] * l[j];
        out[i * N * N + yx] = s;
      }
    }
  }
}

// ------------------------------------------------------------------ in-cell constraints
// A leaf on the fine side of a refinement face or edge holds, at the
// positions of that face/edge, the values of its parent's nodes at the same
// local indices; the child's values there are the parent's polynomial at the
// child's nodes: per tangential axis the 1D embedding rows of the child
// position b (rows b*k .. b*k+k of E).  The transpose applies the columns,
// each fine position counted once.
template <int N, typename T>
__device__ __forceinline__ T emb(const Mats<T>& m, int b, int j, int J) {
  return b ? m.E[(N - 1 + j) * N + J] : m.E[j * N + J];
}

template <int DIM, int N>
__device__ constexpr int lidx(int jx, int jy, int jz) {
  return DIM == 3 ? jx + N * (jy + N * jz) : jx + N * jy;
}

// position with j_A = JA, j_P = p, j_Q = q (3D) or j_A = JA, j_P = p (2D)
template <int DIM, int N, int A, int JA>
__device__ constexpr int fpos(int p, int q) {
  if (DIM == 2) return A == 0 ? lidx<2, N>(JA, p, 0) : lidx<2, N>(p, JA, 0);
  return A == 0 ? lidx<3, N>(JA, p, q) : (A == 1 ? lidx<3, N>(p, JA, q) : lidx<3, N>(p, q, JA));
}

template <int DIM, int N, int A, int JA, typename T>
__device__ __forceinline__ void face_fwd(const Mats<T>& m, const int* bb, const T* uc, T* u) {
  constexpr int P = A == 0 ? 1 : 0;
  constexpr int Q = A == 2 ? 1 : 2;
  if (DIM == 2) {
#pragma unroll
    for (int jp = 0; jp < N; ++jp) {
      T s = 0;
#pragma unroll
      for (int J = 0; J < N; ++J) s += emb<N>(m, bb[P], jp, J) * uc[fpos<DIM, N, A, JA>(J, 0)];
      u[fpos<DIM, N, A, JA>(jp, 0)] = s;
    }
    return;
  }
  T t[N * N];
#pragma unroll
  for (int jp = 0; jp < N; ++jp)
#pragma unroll
    for (int Jq = 0; Jq < N; ++Jq) {
      T s = 0;
#pragma unroll
      for (int Jp = 0; Jp < N; ++Jp) s += emb<N>(m, bb[P], jp, Jp) * uc[fpos<DIM, N, A, JA>(Jp, Jq)];
      t[jp * N + Jq] = s;
    }
#pragma unroll
  for (int jp = 0; jp < N; ++jp)
#pragma unroll
    for (int jq = 0; jq < N; ++jq) {
      T s = 0;
#pragma unroll
      for (int Jq = 0; Jq < N; ++Jq) s += emb<N>(m, bb[Q], jq, Jq) * t[jp * N + Jq];
      u[fpos<DIM, N, A, JA>(jp, jq)] = s;
    }
}

template <int DIM, int N, int A, int JA, typename T>
__device__ __forceinline__ void face_bwd(const Mats<T>& m, const int* bb, const T* t, T* v, uint32_t* used) {
  constexpr int P = A == 0 ? 1 : 0;
  constexpr int Q = A == 2 ? 1 : 2;
  constexpr int NQ = DIM == 3 ? N : 1;
  T w[N * NQ];
#pragma unroll
  for (int jp = 0; jp < N; ++jp)
#pragma unroll
    for (int jq = 0; jq < NQ; ++jq) {
      constexpr int dummy = 0;
      (void)dummy;
      const int p = fpos<DIM, N, A, JA>(jp, jq);
      const bool u = (used[p >> 5] >> (p & 31)) & 1u;
      w[jp * NQ + jq] = u ? T(0) : t[p];
      if (!u) v[p] -= t[p];
      used[p >> 5] |= 1u << (p & 31);
    }
  T c[N * NQ];
#pragma unroll
  for (int Jp = 0; Jp < N; ++Jp)
#pragma unroll
    for (int jq = 0; jq < NQ; ++jq) {
      T s = 0;
#pragma unroll
      for (int jp = 0; jp < N; ++jp) s += emb<N>(m, bb[P], jp, Jp) * w[jp * NQ + jq];
      c[Jp * NQ + jq] = s;
    }
  if (DIM == 2) {
#pragma unroll
    for (int Jp = 0; Jp < N; ++Jp) v[fpos<DIM, N, A, JA>(Jp, 0)] += c[Jp];
    return;
  }
#pragma unroll
  for (int Jp = 0; Jp < N; ++Jp)
#pragma unroll
    for (int Jq = 0; Jq < N; ++Jq) {
      T s = 0;
#pragma unroll
      for (int jq = 0; jq < N; ++jq) s += emb<N>(m, bb[Q], jq, Jq) * c[Jp * NQ + jq];
      v[fpos<DIM, N, A, JA>(Jp, Jq)] += s;
    }
}

// edge along axis A at j_P = JP, j_Q = JQ (3D)
template <int N, int A, int JP, int JQ>
__device__ constexpr int epos(int ja) {
  return A == 0 ? lidx<3, N>(ja, JP, JQ) : (A == 1 ? lidx<3, N>(JP, ja, JQ) : lidx<3, N>(JP, JQ, ja));
}

template <int N, int A, int JP, int JQ, typename T>
__device__ __forceinline__ void edge_fwd(const Mats<T>& m, int b, const T* uc, T* u) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    T s = 0;
#pragma unroll
    for (int J = 0; J < N; ++J) s += emb<N>(m, b, j, J) * uc[epos<N, A, JP, JQ>(J)];
    u[epos<N, A, JP, JQ>(j)] = s;
  }
}

template <int N, int A, int JP, int JQ, typename T>
__device__ __forceinline__ void edge_bwd(const Mats<T>& m, int b, const T* t, T* v, uint32_t* used) {
  T w[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const int p = epos<N, A, JP, JQ>(j);
    const bool u = (used[p >> 5] >> (p & 31)) & 1u;
    w[j] = u ? T(0) : t[p];
    if (!u) v[p] -= t[p];
    used[p >> 5] |= 1u << (p & 31);
  }
#pragma unroll
  for (int J = 0; J < N; ++J) {
    T s = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) s += emb<N>(m, b, j, J) * w[j];
    v[epos<N, A, JP, JQ>(J)] += s;
  }
}

template <int N, int A, typename T>
__device__ __forceinline__ void edge_dispatch(const Mats<T>& m, const int* bb, const T* in, T* out, uint32_t* used,
                                              bool fwd) {
  constexpr int P = A == 0 ? 1 : 0;
  constexpr int Q = A == 2 ? 1 : 2;
  constexpr int K = N - 1;
  const int sel = bb[P] + 2 * bb[Q];
  if (fwd) {
    if (sel == 0) edge_fwd<N, A, 0, 0>(m, bb[A], in, out);
    else if (sel == 1) edge_fwd<N, A, K, 0>(m, bb[A], in, out);
    else if (sel == 2) edge_fwd<N, A, 0, K>(m, bb[A], in, out);
    else edge_fwd<N, A, K, K>(m, bb[A], in, out);
  } else {
    if (sel == 0) edge_bwd<N, A, 0, 0>(m, bb[A], in, out, used);
    else if (sel == 1) edge_bwd<N, A, K, 0>(m, bb[A], in, out, used);
    else if (sel == 2) edge_bwd<N, A, 0, K>(m, bb[A], in, out, used);
    else edge_bwd<N, A, K, K>(m, bb[A], in, out, used);
  }
}

template <int DIM, int N, int A, typename T>
__device__ __forceinline__ void face_dispatch(const Mats<T>& m, const int* bb, const T* in, T* out, uint32_t* used,
                                              bool fwd) {
  constexpr int K = N - 1;
  if (fwd) {
    if (bb[A]) face_fwd<DIM, N, A, K>(m, bb, in, out);
    else face_fwd<DIM, N, A, 0>(m, bb, in, out);
  } else {
    if (bb[A]) face_bwd<DIM, N, A, K>(m, bb, in, out, used);
    else face_bwd<DIM, N, A, 0>(m, bb, in, out, used);
  }
}

// u <- C_K u (fwd) or v <- C_K^T v (bwd) for the mask of a leaf, with c a
// copy of the input (registers, or LDS in the cooperative kernels)
template <int DIM, int N, typename T>
__device__ __forceinline__ void constrain_from(const Mats<T>& m, uint32_t mask, const T* c, T* u, bool fwd) {
  constexpr int NP = DIM == 3 ? N * N * N : N * N;
  const int bb[3] = {(int)(mask & 1u), (int)((mask >> 1) & 1u), (int)((mask >> 2) & 1u)};
  uint32_t used[(NP + 31) / 32];
#pragma unroll
  for (int w = 0; w < (NP + 31) / 32; ++w) used[w] = 0u;
  if ((mask >> 3) & 1u) face_dispatch<DIM, N, 0>(m, bb, c, u, used, fwd);
  if ((mask >> 4) & 1u) face_dispatch<DIM, N, 1>(m, bb, c, u, used, fwd);
  if (DIM == 3) {
    if ((mask >> 5) & 1u) face_dispatch<DIM, N, 2>(m, bb, c, u, used, fwd);
    if ((mask >> 6) & 1u) edge_dispatch<N, 0>(m, bb, c, u, used, fwd);
    if ((mask >> 7) & 1u) edge_dispatch<N, 1>(m, bb, c, u, used, fwd);
    if ((mask >> 8) & 1u) edge_dispatch<N, 2>(m, bb, c, u, used, fwd);
  }
}

template <int DIM, int N, typename T>
__device__ __forceinline__ void constrain(const Mats<T>& m, uint32_t mask, T* u, bool fwd) {
  constexpr int NP = DIM == 3 ? N * N * N : N * N;
  T c[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) c[j] = u[j];
  constrain_from<DIM, N, T>(m, mask, c, u, fwd);
}

// ------------------------------------------------------------------ canonical in-cell constraints
// The same in-cell constraints after a reflection of the cell that moves its
// child position to 0 along every axis (lane-per-cell kernels).  The
// constrained faces and edges of a leaf lie on its parent's boundary on the
// child's side, so after the reflection they are the faces j_a = 0 and the
// edges through the corner 0; the embedding rows of child position 0 are
// then fixed (compile-time indices, no per-coefficient selects), which holds
// because the 1D matrices of symmetric nodes are centro-symmetric:
// E[2K - i][K - J] = E[i][J], and the cell operator and mass matrix are
// invariant under reflections of the node order.

// c ? a : b by bit masks (no select of addresses, which would move a
// register array to scratch memory)
__device__ __forceinline__ double bsel(bool c, double a, double b) {
  const long long m = -(long long)c;
  return __longlong_as_double((__double_as_longlong(a) & m) | (__double_as_longlong(b) & ~m));
}

// reverse the node order along every axis a with bit a of r set
template <int DIM, int N>
__device__ __forceinline__ void reflect_cell(uint32_t r, double* u) {
  constexpr int K = N - 1;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const bool f = (r >> a) & 1u;
    const int st = a == 0 ? 1 : a == 1 ? N : N * N;
#pragma unroll
    for (int p = 0; p < (DIM == 3 ? N * N * N : N * N); ++p) {
      const int ja = (p / st) % N;
      if (2 * ja < K) {
        const int q = p + (K - 2 * ja) * st;
        const double x = u[p], y = u[q];
        u[p] = bsel(f, y, x);
        u[q] = bsel(f, x, y);
      }
    }
  }
}

// local index of position (ja, jb, jc) given along axes a, b, c
template <int DIM, int N>
__device__ constexpr int pos3(int a, int ja, int b, int jb, int c, int jc) {
  int j[3] = {0, 0, 0};
  j[a] = ja;
  j[b] = jb;
  if (DIM == 3) j[c] = jc;
  return DIM == 3 ? j[0] + N * (j[1] + N * j[2]) : j[0] + N * j[1];
}

// Number of the canonical entities containing position p (zero
// coordinates): faces a (j_a = 0, entity a, mask bit 3 + a), then in 3D
// edges along a (the other two coordinates 0, entity 3 + a, bit 6 + a).
template <int DIM, int N>
__device__ constexpr bool on_entity(int e, int p) {
  const int j0 = p % N, j1 = (p / N) % N, j2 = DIM == 3 ? p / (N * N) : 0;
  const int j[3] = {j0, j1, j2};
  if (e < DIM) return j[e] == 0;
  const int a = e - 3;
  return (a != 0 ? j[0] == 0 : true) && (a != 1 ? j[1] == 0 : true) && (a != 2 ? j[2] == 0 : true);
}

// u <- C u on a reflected cell (act: mask bits 3..8, entity order faces x,
// y, z then edges x, y, z, the last active entity containing a position
// giving its value, every entity reading the gathered values)
template <int DIM, int N, typename MT>
__device__ __forceinline__ void con_fwd_canon(const MT& m, uint32_t act, double* u) {
  constexpr int K = N - 1, NP = DIM == 3 ? N * N * N : N * N, NE = DIM == 3 ? 6 : 2;
  // gathered values of the positions on more than one entity
  double o[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    int cnt = 0;
#pragma unroll
    for (int e = 0; e < DIM; ++e) cnt += on_entity<DIM, N>(e, p) ? 1 : 0;
    if (cnt >= 2) o[p] = u[p];
  }
  auto src = [&](int p) -> double {
    int cnt = 0;
#pragma unroll
    for (int e = 0; e < DIM; ++e) cnt += on_entity<DIM, N>(e, p) ? 1 : 0;
    return cnt >= 2 ? o[p] : u[p];
  };
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    if (!((act >> e) & 1u)) continue;
    if (e < DIM) {
      const int a = e, b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
      constexpr int NC = DIM == 3 ? N : 1;
      double g[N * NC], t[N * NC];
#pragma unroll
      for (int jb = 0; jb < N; ++jb)
#pragma unroll
        for (int jc = 0; jc < NC; ++jc) g[jb * NC + jc] = src(pos3<DIM, N>(a, 0, b, jb, c, jc));
#pragma unroll
      for (int jb = 0; jb < N; ++jb)
#pragma unroll
        for (int jc = 0; jc < NC; ++jc) {
          double s = 0.0;
#pragma unroll
          for (int J = 0; J < N; ++J) s += m.E[jb * N + J] * g[J * NC + jc];
          t[jb * NC + jc] = s;
        }
#pragma unroll
      for (int jb = 0; jb < N; ++jb)
#pragma unroll
        for (int jc = 0; jc < NC; ++jc) {
          double s = t[jb * NC + jc];
          if (DIM == 3) {
            s = 0.0;
#pragma unroll
            for (int J = 0; J < N; ++J) s += m.E[jc * N + J] * t[jb * NC + J];
          }
          u[pos3<DIM, N>(a, 0, b, jb, c, jc)] = s;
        }
    } else {
      const int a = e - 3, b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
      double g[N];
#pragma unroll
      for (int J = 0; J < N; ++J) g[J] = src(pos3<DIM, N>(a, J, b, 0, c, 0));
#pragma unroll
      for (int ja = 0; ja < N; ++ja) {
        double s = 0.0;
#pragma unroll
        for (int J = 0; J < N; ++J) s += m.E[ja * N + J] * g[J];
        u[pos3<DIM, N>(a, ja, b, 0, c, 0)] = s;
      }
    }
  }
  (void)K;
}

// v <- C^T v on a reflected cell: every position of an active entity is
// claimed by the first active entity containing it, whose transposed
// embedding moves the claimed values to the entity's parent positions
template <int DIM, int N, typename MT>
__device__ __forceinline__ void con_bwd_canon(const MT& m, uint32_t act, double* v) {
  constexpr int NP = DIM == 3 ? N * N * N : N * N, NE = DIM == 3 ? 6 : 2;
  // the operator values of the positions on more than one entity
  double o[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    int cnt = 0;
#pragma unroll
    for (int e = 0; e < DIM; ++e) cnt += on_entity<DIM, N>(e, p) ? 1 : 0;
    if (cnt >= 2) o[p] = v[p];
  }
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    if (!((act >> e) & 1u)) continue;
    // claimed here: on this entity, on no earlier active one
    auto claim = [&](int p) -> bool {
      bool earlier = false;
#pragma unroll
      for (int f = 0; f < e; ++f)
        if (on_entity<DIM, N>(f, p)) earlier = earlier || ((act >> f) & 1u);
      return !earlier;
    };
    auto val = [&](int p) -> double {
      int cnt = 0;
#pragma unroll
      for (int f = 0; f < DIM; ++f) cnt += on_entity<DIM, N>(f, p) ? 1 : 0;
      return cnt >= 2 ? o[p] : v[p];
    };
    if (e < DIM) {
      const int a = e, b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
      constexpr int NC = DIM == 3 ? N : 1;
      double w[N * NC], t[N * NC];
#pragma unroll
      for (int jb = 0; jb < N; ++jb)
#pragma unroll
        for (int jc = 0; jc < NC; ++jc) {
          const int p = pos3<DIM, N>(a, 0, b, jb, c, jc);
          const bool cl = claim(p);
          const double x = val(p);
          w[jb * NC + jc] = bsel(cl, x, 0.0);
          v[p] -= w[jb * NC + jc];
        }
#pragma unroll
      for (int Jb = 0; Jb < N; ++Jb)
#pragma unroll
        for (int jc = 0; jc < NC; ++jc) {
          double s = 0.0;
#pragma unroll
          for (int jb = 0; jb < N; ++jb) s += m.E[jb * N + Jb] * w[jb * NC + jc];
          t[Jb * NC + jc] = s;
        }
#pragma unroll
      for (int Jb = 0; Jb < N; ++Jb)
#pragma unroll
        for (int Jc = 0; Jc < NC; ++Jc) {
          double s = t[Jb * NC + Jc];
          if (DIM == 3) {
            s = 0.0;
#pragma unroll
            for (int jc = 0; jc < N; ++jc) s += m.E[jc * N + Jc] * t[Jb * NC + jc];
          }
          v[pos3<DIM, N>(a, 0, b, Jb, c, Jc)] += s;
        }
    } else {
      const int a = e - 3, b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
      double w[N];
#pragma unroll
      for (int ja = 0; ja < N; ++ja) {
        const int p = pos3<DIM, N>(a, ja, b, 0, c, 0);
        const bool cl = claim(p);
        const double x = val(p);
        w[ja] = bsel(cl, x, 0.0);
        v[p] -= w[ja];
      }
#pragma unroll
      for (int J = 0; J < N; ++J) {
        double s = 0.0;
#pragma unroll
        for (int ja = 0; ja < N; ++ja) s += m.E[ja * N + J] * w[ja];
        v[pos3<DIM, N>(a, J, b, 0, c, 0)] += s;
      }
    }
  }
}

// Two-pass operator, pass 1: every (cell, local node) owns one slot of the
// node-major buffer E (the slots of a node are contiguous), so the cell
// results are written with plain stores and no two lanes ever write the same
// address.  Pass 2 (seg_*) sums the slots of each node in a fixed order:
// deterministic and free of atomics.  LEAF: cells carry in-cell
// constraint masks.  Cells [0, c_end) of n_cells (the stride of the maps).
template <int DIM, int N, typename T, bool LEAF, bool MASS>
__global__ void __launch_bounds__(kBlock) cell_to_slots(
    int64_t n_cells, int64_t c_end, const int32_t* __restrict__ cmap, const int32_t* __restrict__ slot,
    const double* __restrict__ scale, double scale0, const T* __restrict__ x,
    const uint16_t* __restrict__ mask, T* __restrict__ E, Mats<T> m) {
  constexpr int NP = DIM == 3 ? N * N * N : N * N;
  const int64_t c = xcd_tid();
  if (c >= c_end) return;
  T u[NP], v[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) u[j] = x[cmap[(int64_t)j * n_cells + c]];
  const uint32_t mk = LEAF ? (uint32_t)mask[c] : 0u;
  if (LEAF && (mk >> 3)) constrain<DIM, N, T>(m, mk, u, true);
  if (MASS) {
    mass_nd<DIM, N, T>(m, u, v);
  } else if (DIM == 3) {
    laplace3<N, T>(m, *reinterpret_cast<const T(*)[N * N * N]>(u), *reinterpret_cast<T(*)[N * N * N]>(v));
  } else {
    laplace2<N, T>(m, *reinterpret_cast<const T(*)[N * N]>(u), *reinterpret_cast<T(*)[N * N]>(v));
  }
  if (LEAF && (mk >> 3)) constrain<DIM, N, T>(m, mk, v, false);
  const T s = T(scale ? scale[c] : scale0);
#pragma unroll
  for (int j = 0; j < NP; ++j) E[slot[(int64_t)j * n_cells + c]] = s * v[j];
}

// Leaf operator q = C^T A C p (or the mass matrix) on tiles of 64
// consecutive leaf cells, one wavefront (block) per tile at a time, the
// tiles of a block contiguous.  Per tile: the values of all nodes the cells
// touch are gathered once into LDS, the tile's own DoFs (a contiguous range)
// first, then its listed nodes; each lane takes one cell (in-cell
// constraints forward, operator, constraints transposed) and adds its
// results into LDS position by position, the results of constrained
// positions into the parent's nodes.  Only this wave adds into the tile's
// LDS, its adds issue in a fixed order, and same-address adds within one
// instruction are resolved by the LDS unit in a fixed order, so every sum is
// formed in the same order on every run.  Then the own nodes' sums are
// written to q (Dirichlet rows zero) and the listed nodes' sums to their
// slots, which leaf_pass2 adds to q.  DOT: one partial sum of p.q per block
// over the own nodes' sums (leaf_pass2 adds p.q over the slots).

// one leaf cell: in-cell constraints on the cell reflected to child
// position 0 (a cell without constrained entities is neither reflected nor
// constrained), operator or mass matrix, constraints transposed, reflected
// back
template <int DIM, int N, bool MASS, typename MT>
__device__ __forceinline__ void leaf_cell(const MT& m, uint32_t mk, double* u, double* w) {
  const uint32_t ce = (mk >> 3) & 0x3fu;
  const uint32_t refl = ce ? (mk & 7u) : 0u;
  if (ce) {
    reflect_cell<DIM, N>(refl, u);
    con_fwd_canon<DIM, N>(m, ce, u);
  }
  if (MASS)
    mass_nd<DIM, N, double>(m, u, w);
  else if (DIM == 3)
    laplace3<N, double>(m, *reinterpret_cast<const double(*)[N * N * N]>(u), *reinterpret_cast<double(*)[N * N * N]>(w));
  else
    laplace2<N, double>(m, *reinterpret_cast<const double(*)[N * N]>(u), *reinterpret_cast<double(*)[N * N]>(w));
  if (ce) {
    con_bwd_canon<DIM, N>(m, ce, w);
    reflect_cell<DIM, N>(refl, w);
  }
}

constexpr int kLeafBlocks = 32768;  // grid of leaf_tiles at most (128 one-wave blocks per CU)
constexpr int kLeafGB = 16;        // tile nodes per lane whose loads are issued together
constexpr int kLeafOwn = 8;        // own nodes per lane per write-out round

// LDS ordering between the lanes of a one-wavefront block: the wave's LDS
// accesses are performed in program order, so the block needs no hardware
// barrier (which would also wait for its outstanding global stores), only
// fences that keep the compiler from moving memory accesses across this
// point
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Every global load below reads a valid address on every lane (indices
// clamped into their arrays; the listed-node array has one padding entry),
// and the lanes without a node drop the value: loads under a lane mask were
// compiled into branches that waited for each load before issuing the next.
template <int DIM, int N, bool MASS, bool DOT>
__device__ __forceinline__ void leaf_tiles_at(const LeafView& v, const double* __restrict__ x,
                                              double* __restrict__ y, double* __restrict__ E,
                                              double* __restrict__ part, const Mats<double>& m, int64_t b,
                                              int64_t G) {
  constexpr int NP = DIM == 3 ? N * N * N : N * N;
  HIP_DYNAMIC_SHARED(double, lds)
  const int lane = threadIdx.x;
  const int64_t lb = xcd_block_of(b, G);
  const int64_t t0 = v.n_tiles * lb / G, t1 = v.n_tiles * (lb + 1) / G;
  const int64_t nlast = v.n_dofs - 1;
  double dot = 0.0;
  for (int64_t t = t0; t < t1; ++t) {
    const int32_t lo = v.t_own[t];
    const int R = v.t_own[t + 1] - lo;
    const int64_t l0 = v.t_loff[t];
    const int L = (int)(v.t_loff[t + 1] - l0);
    const int nt = R + L;
    const int64_t c = t * 64 + lane;
    const bool live = c < v.n_cells;
    const int64_t cc = live ? c : v.n_cells - 1;
    // the cells' local indices, constraint masks and scales first: their
    // latency passes during the gather
    uint32_t lu[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) lu[j] = v.lmap[(int64_t)j * v.n_cells + cc];
    const uint32_t mk = v.mask[cc];
    const double sc = live ? (MASS ? v.mscale[cc] : v.scale[cc]) : 0.0;
    // gather, in rounds of kLeafGB nodes per lane: the listed node ids, then
    // all values, then the LDS stores
    for (int i0 = 0; i0 < nt; i0 += 64 * kLeafGB) {
      int32_t li[kLeafGB];
      double xv[kLeafGB];
#pragma unroll
      for (int k = 0; k < kLeafGB; ++k) {
        const int i = i0 + lane + 64 * k;
        li[k] = v.t_list[l0 + (i < R ? 0 : i - R < L ? i - R : L)];
      }
#pragma unroll
      for (int k = 0; k < kLeafGB; ++k) {
        const int i = i0 + lane + 64 * k;
        const int64_t d = i < R ? (int64_t)lo + i : i < nt ? (int64_t)li[k] : 0;
        xv[k] = x[d];
      }
#pragma unroll
      for (int k = 0; k < kLeafGB; ++k) {
        const int i = i0 + lane + 64 * k;
        if (i < nt) lds[i] = xv[k];
      }
    }
    wave_lds_sync();
    double w[NP];
    {
      double u[NP];
#pragma unroll
      for (int j = 0; j < NP; ++j) u[j] = lds[lu[j]];
      if constexpr (N <= 3)
        leaf_cell<DIM, N, MASS>(Exact1D<N>{}, mk, u, w);
      else
        leaf_cell<DIM, N, MASS>(m, mk, u, w);
#pragma unroll
      for (int j = 0; j < NP; ++j) w[j] *= sc;
    }
    // the local indices again (cached) rather than held in registers through
    // the operator; not scheduled above this point, and the cell index passed
    // through an empty asm statement so that the compiler cannot merge this
    // read with the first one
    __builtin_amdgcn_sched_barrier(0);
    int64_t cr = cc;
    asm volatile("" : "+v"(cr));
    uint32_t lm[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) lm[j] = v.lmap[(int64_t)j * v.n_cells + cr];
    // the first write-out round's Dirichlet flags and p values, loaded now so
    // that their latency passes during the LDS phase
    uint8_t dr[kLeafOwn];
    double xd[kLeafOwn];
#pragma unroll
    for (int k = 0; k < kLeafOwn; ++k) {
      const int64_t d = (int64_t)lo + lane + 64 * k < nlast ? (int64_t)lo + lane + 64 * k : nlast;
      dr[k] = v.dir[d];
      if (DOT) xd[k] = x[d];
    }
    wave_lds_sync();
    for (int i = lane; i < nt; i += 64) lds[i] = 0.0;
    wave_lds_sync();
    if (live) {
#pragma unroll
      for (int j = 0; j < NP; ++j) atomicAdd(&lds[lm[j]], w[j]);
    }
    wave_lds_sync();
    // write-out: own nodes to y (Dirichlet rows zero) in rounds of kLeafOwn
    // per lane, then the listed ones to their slots
    for (int i0 = 0; i0 < R; i0 += 64 * kLeafOwn) {
      if (i0 > 0) {
#pragma unroll
        for (int k = 0; k < kLeafOwn; ++k) {
          const int64_t d = (int64_t)lo + i0 + lane + 64 * k < nlast ? (int64_t)lo + i0 + lane + 64 * k : nlast;
          dr[k] = v.dir[d];
          if (DOT) xd[k] = x[d];
        }
      }
#pragma unroll
      for (int k = 0; k < kLeafOwn; ++k) {
        const int i = i0 + lane + 64 * k;
        if (i < R) {
          const double qk = dr[k] ? 0.0 : lds[i];
          y[lo + i] = qk;
          if (DOT) dot += xd[k] * qk;
        }
      }
    }
    double* lslot = E + l0 - R;
    for (int i0 = R; i0 < nt; i0 += 64 * kLeafGB) {
      double q[kLeafGB];
#pragma unroll
      for (int k = 0; k < kLeafGB; ++k) q[k] = lds[i0 + lane + 64 * k < nt ? i0 + lane + 64 * k : nt - 1];
#pragma unroll
      for (int k = 0; k < kLeafGB; ++k) {
        const int i = i0 + lane + 64 * k;
        if (i < nt) lslot[i] = q[k];
      }
    }
    wave_lds_sync();
  }
  if (DOT) {
    for (int o = 32; o > 0; o >>= 1) dot += __shfl_down(dot, o, 64);
    if (lane == 0) part[b] = dot;
  }
}
template <int DIM, int N, bool MASS, bool DOT>
__global__ void __launch_bounds__(64) leaf_tiles(LeafView v, const double* __restrict__ x, double* __restrict__ y,
                                                 double* __restrict__ E, double* __restrict__ part, Mats<double> m) {
  leaf_tiles_at<DIM, N, MASS, DOT>(v, x, y, E, part, m, blockIdx.x, gridDim.x);
}

// the tiled leaf operator of several problems in one launch (q = A p with
// the partial sums of p.q, as leaf_tiles<DIM, N, false, true>)
struct LeafItem {
  LeafView v;
  const double* x;
  double* y;
  double* E;
  double* part;
  int64_t b0, nb;
};
template <int DIM, int N>
__global__ void __launch_bounds__(64) leaf_tiles_batch(const LeafItem* __restrict__ items, int n, Mats<double> m) {
  const LeafItem& it = items[batch_item(items, n)];
  leaf_tiles_at<DIM, N, false, true>(it.v, it.x, it.y, it.E, it.part, m, (int64_t)blockIdx.x - it.b0, it.nb);
}

// In-cell constraints of one node, gathered (3D, used by the cooperative
// leaf kernel, one thread per node of a cell).  The constraint entities of
// a leaf with mask mk are the faces normal to axis e (mask bit 3 + e) and
// the edges along axis e (bit 6 + e) on the side of its child position
// bits; with c the cell's values:
//  forward:   u_j = the interpolation of the last active entity (faces x, y,
//             z, then edges x, y, z) containing node j, else c_j (the
//             order in which constrain_from overwrites);
//  transpose: v_J = (J claimed ? 0 : c_J) + the sum, over the active
//             entities containing J, of the embedding weights times c_p of
//             the nodes p each entity claims (the first active entity
//             containing p, as the used-mask of constrain_from).
// sE holds the 1D embedding rows E (2k+1 rows of k+1) in LDS: run-time
// indices into a kernel argument would move it to scratch memory.
template <int N>
struct CellCon {
  static constexpr int K = N - 1;
  uint32_t mk;
  int bb[3], JB[3];
  __device__ __forceinline__ explicit CellCon(uint32_t m) : mk(m) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      bb[a] = (int)((m >> a) & 1u);
      JB[a] = bb[a] * K;
    }
  }
  static constexpr int P(int a) { return a == 0 ? 1 : 0; }
  static constexpr int Q(int a) { return a == 2 ? 1 : 2; }
  static __device__ __forceinline__ int lid(const int (&q)[3]) { return q[0] + N * (q[1] + N * q[2]); }
  __device__ __forceinline__ bool active(int e) const { return (mk >> (3 + e)) & 1u; }
  // e is a compile-time constant wherever these are called (unrolled loops)
  __device__ __forceinline__ bool contains(int e, const int (&p)[3]) const {
    if (e < 3) return p[e] == JB[e];
    return p[P(e - 3)] == JB[P(e - 3)] && p[Q(e - 3)] == JB[Q(e - 3)];
  }
  __device__ __forceinline__ int claim(const int (&p)[3]) const {
    int c = -1;
#pragma unroll
    for (int e = 5; e >= 0; --e)
      if (active(e) && contains(e, p)) c = e;
    return c;
  }
  static __device__ __forceinline__ double emb(const double* sE, int b, int j, int J) {
    return sE[(b * K + j) * N + J];
  }
  // interpolation of entity e at node p from the cell's values c
  __device__ __forceinline__ double interp(int e, const double* sE, const double* c, const int (&p)[3]) const {
    double s = 0.0;
    if (e < 3) {
      const int A = e, Pa = P(A), Qa = Q(A);
      double wp[N], wq[N];
#pragma unroll
      for (int J = 0; J < N; ++J) {
        wp[J] = emb(sE, bb[Pa], p[Pa], J);
        wq[J] = emb(sE, bb[Qa], p[Qa], J);
      }
#pragma unroll
      for (int Jq = 0; Jq < N; ++Jq) {
        double t = 0.0;
#pragma unroll
        for (int Jp = 0; Jp < N; ++Jp) {
          int q[3];
          q[A] = JB[A];
          q[Pa] = Jp;
          q[Qa] = Jq;
          t += wp[Jp] * c[lid(q)];
        }
        s += wq[Jq] * t;
      }
    } else {
      const int A = e - 3;
#pragma unroll
      for (int J = 0; J < N; ++J) {
        int q[3];
        q[A] = J;
        q[P(A)] = JB[P(A)];
        q[Q(A)] = JB[Q(A)];
        s += emb(sE, bb[A], p[A], J) * c[lid(q)];
      }
    }
    return s;
  }
  __device__ __forceinline__ double forward(const double* sE, const double* c, int j) const {
    const int p[3] = {j % N, (j / N) % N, j / (N * N)};
    int last = -1;
#pragma unroll
    for (int e = 0; e < 6; ++e)
      if (active(e) && contains(e, p)) last = e;
    double s = c[j];
#pragma unroll
    for (int e = 0; e < 6; ++e)
      if (e == last) s = interp(e, sE, c, p);
    return s;
  }
  __device__ __forceinline__ double transpose(const double* sE, const double* c, int jj) const {
    const int J[3] = {jj % N, (jj / N) % N, jj / (N * N)};
    double s = claim(J) < 0 ? c[jj] : 0.0;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      if (!active(e) || !contains(e, J)) continue;
      if (e < 3) {
        const int A = e, Pa = P(A), Qa = Q(A);
        double wp[N], wq[N];
#pragma unroll
        for (int a = 0; a < N; ++a) {
          wp[a] = emb(sE, bb[Pa], a, J[Pa]);
          wq[a] = emb(sE, bb[Qa], a, J[Qa]);
        }
#pragma unroll
        for (int b = 0; b < N; ++b) {
          double t = 0.0;
#pragma unroll
          for (int a = 0; a < N; ++a) {
            int q[3];
            q[A] = JB[A];
            q[Pa] = a;
            q[Qa] = b;
            if (claim(q) == e) t += wp[a] * c[lid(q)];
          }
          s += wq[b] * t;
        }
      } else {
        const int A = e - 3;
#pragma unroll
        for (int a = 0; a < N; ++a) {
          int q[3];
          q[A] = a;
          q[P(A)] = JB[P(A)];
          q[Q(A)] = JB[Q(A)];
          if (claim(q) == e) s += emb(sE, bb[A], a, J[A]) * c[lid(q)];
        }
      }
    }
    return s;
  }
};

// Leaf pass 1 in 3D at degree >= 3 on cells [c_first, n_cells) (otherwise
// the contract of cell_to_slots): the cells' (k+1)^3 values do not fit one
// lane's registers, so a workgroup stages CB cells in LDS and its threads
// share the work: the gather, the in-cell constraints (CON) and the slot
// stores one thread per (node, cell), the sum-factorized contractions one
// thread per line of a cell and direction (as in the cooperative level
// operator: a = M u, b = K u along z; c = M a, f = K a + M b along y;
// K c + M f along x; the mass matrix is M M M).
template <int N>
struct LeafCoop {
  static constexpr int NP = N * N * N, NL = N * N, THREADS = 256;
  static constexpr int CB = 32768 / (2 * NP * 8);
  static constexpr int ITG = (CB * NP + THREADS - 1) / THREADS;
  static constexpr int ITL = (CB * NL + THREADS - 1) / THREADS;
};

template <int N, bool MASS, bool CON>
__global__ void __launch_bounds__(LeafCoop<N>::THREADS) __attribute__((amdgpu_waves_per_eu(5)))
    leaf_coop(int64_t n_cells, int64_t c_first, int64_t c_end, const int32_t* __restrict__ cmap,
              const int32_t* __restrict__ slot, const double* __restrict__ scale, double scale0,
              const double* __restrict__ x, const uint16_t* __restrict__ mask, double* __restrict__ E,
              Mats<double> m) {
  using S = LeafCoop<N>;
  constexpr int NP = S::NP, NL = S::NL, CB = S::CB, TH = S::THREADS;
  // input values (tu), then the second intermediate in the same space
  __shared__ double tu[CB * NP];
  __shared__ double ta[CB * NP];
  __shared__ double sE[(2 * N - 1) * N];
  __shared__ uint32_t smk[CB];
  double* tb = tu;
  const int64_t c0 = c_first + xcd_block() * CB;
  const int nc = (int)(c_end - c0 < CB ? c_end - c0 : CB);
  const int tid = threadIdx.x;
  if (CON) {
    if (tid == 0) {
#pragma unroll
      for (int e = 0; e < (2 * N - 1) * N; ++e) sE[e] = m.E[e];
    }
    if (tid < nc) smk[tid] = mask[c0 + tid];
  }
  {
    double g[S::ITG];
#pragma unroll
    for (int it = 0; it < S::ITG; ++it) {
      const int e = tid + it * TH, j = e / CB, cl = e % CB;
      g[it] = e < CB * NP && cl < nc ? x[cmap[(int64_t)j * n_cells + c0 + cl]] : 0.0;
    }
#pragma unroll
    for (int it = 0; it < S::ITG; ++it) {
      const int e = tid + it * TH, j = e / CB, cl = e % CB;
      if (e < CB * NP && cl < nc) tu[cl * NP + j] = g[it];
    }
  }
  __syncthreads();
  const double* src = tu;
  if (CON) {
    // u <- C u, into ta
#pragma unroll
    for (int it = 0; it < S::ITG; ++it) {
      const int e = tid + it * TH, cl = e / NP, j = e % NP;
      if (cl < nc) ta[e] = CellCon<N>(smk[cl]).forward(sE, tu + cl * NP, j);
    }
    __syncthreads();
    src = ta;
  }
  const int nline = nc * NL;
  // lines along z
#pragma unroll
  for (int it = 0; it < S::ITL; ++it) {
    const int u = tid + it * TH;
    if (u < nline) {
      const int cl = u / NL, p = u % NL;
      const int o = cl * NP + p;  // (px, py, z = 0)
      double v[N];
#pragma unroll
      for (int z = 0; z < N; ++z) v[z] = src[o + z * NL];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int z = 0; z < N; ++z) {
          a += m.M[i * N + z] * v[z];
          if (!MASS) b += m.K[i * N + z] * v[z];
        }
        ta[o + i * NL] = a;
        if (!MASS) tb[o + i * NL] = b;
      }
    }
  }
  __syncthreads();
  // lines along y, in place
#pragma unroll
  for (int it = 0; it < S::ITL; ++it) {
    const int u = tid + it * TH;
    if (u < nline) {
      const int cl = u / NL, p = u % NL, px = p % N, pz = p / N;
      const int o = cl * NP + px + pz * NL;
      double a[N], b[N];
#pragma unroll
      for (int y = 0; y < N; ++y) {
        a[y] = ta[o + y * N];
        if (!MASS) b[y] = tb[o + y * N];
      }
#pragma unroll
      for (int i = 0; i < N; ++i) {
        double c = 0.0, f = 0.0;
#pragma unroll
        for (int y = 0; y < N; ++y) {
          c += m.M[i * N + y] * a[y];
          if (!MASS) f += m.K[i * N + y] * a[y] + m.M[i * N + y] * b[y];
        }
        ta[o + i * N] = c;
        if (!MASS) tb[o + i * N] = f;
      }
    }
  }
  __syncthreads();
  // lines along x, in place
#pragma unroll
  for (int it = 0; it < S::ITL; ++it) {
    const int u = tid + it * TH;
    if (u < nline) {
      const int cl = u / NL, p = u % NL;
      const int o = cl * NP + p * N;
      double c[N], f[N];
#pragma unroll
      for (int xx = 0; xx < N; ++xx) {
        c[xx] = ta[o + xx];
        if (!MASS) f[xx] = tb[o + xx];
      }
#pragma unroll
      for (int i = 0; i < N; ++i) {
        double r = 0.0;
#pragma unroll
        for (int xx = 0; xx < N; ++xx) {
          if (MASS)
            r += m.M[i * N + xx] * c[xx];
          else
            r += m.K[i * N + xx] * c[xx] + m.M[i * N + xx] * f[xx];
        }
        ta[o + i] = r;
      }
    }
  }
  __syncthreads();
  const double* res = ta;
  if (CON) {
    // v <- C^T v, into tb
#pragma unroll
    for (int it = 0; it < S::ITG; ++it) {
      const int e = tid + it * TH, cl = e / NP, j = e % NP;
      if (cl < nc) tb[e] = CellCon<N>(smk[cl]).transpose(sE, ta + cl * NP, j);
    }
    __syncthreads();
    res = tb;
  }
#pragma unroll
  for (int it = 0; it < S::ITG; ++it) {
    const int e = tid + it * TH, j = e / CB, cl = e % CB;
    if (e < CB * NP && cl < nc) {
      const int64_t c = c0 + cl;
      E[slot[(int64_t)j * n_cells + c]] = (scale ? scale[c] : scale0) * res[cl * NP + j];
    }
  }
}

// diagonal of the cell Laplacian, accumulated per node (FP64)
template <int DIM, int N>
__global__ void __launch_bounds__(kBlock) cell_diag(int64_t n_cells, const int32_t* __restrict__ cmap,
                                                    const double* __restrict__ scale, double scale0,
                                                    double* __restrict__ diag, Mats<double> m) {
  constexpr int NP = DIM == 3 ? N * N * N : N * N;
  const int64_t c = xcd_tid();
  if (c >= n_cells) return;
  const double s = scale ? scale[c] : scale0;
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    const int jx = j % N, jy = (j / N) % N, jz = j / (N * N);
    double mx = m.M[jx * N + jx], my = m.M[jy * N + jy], kx = m.K[jx * N + jx], ky = m.K[jy * N + jy];
    double v;
    if (DIM == 3) {
      double mz = m.M[jz * N + jz], kz = m.K[jz * N + jz];
      v = kx * my * mz + mx * ky * mz + mx * my * kz;
    } else {
      v = kx * my + mx * ky;
    }
    atomic_add(&diag[cmap[(int64_t)j * n_cells + c]], s * v);
  }
}

template <typename T>
__global__ void make_dinv(int64_t n, const double* __restrict__ diag, const uint8_t* __restrict__ flags,
                          T* __restrict__ dinv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dinv[i] = flags[i] == 0 ? T(1.0 / diag[i]) : T(0);
}

// ------------------------------------------------------------------ vectors
template <typename T>
__device__ __forceinline__ void fill_at(int64_t n, T* __restrict__ p, T v, int64_t b, int64_t nb) {
  for (int64_t i = b * blockDim.x + threadIdx.x; i < n; i += nb * blockDim.x) p[i] = v;
}
template <typename T>
__global__ void fill(int64_t n, T* __restrict__ p, T v) {
  fill_at(n, p, v, blockIdx.x, gridDim.x);
}

// t = x on the rows whose flag is want, 0 elsewhere (t may alias x)
template <typename T>
__global__ void mask_rows(int64_t n, const uint8_t* __restrict__ flags, int want, const T* x, T* t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t[i] = flags[i] == want ? x[i] : T(0);
}

// Chebyshev step (Sec. 4.1 smoother): d = c1 d + c2 D^{-1} (g - t); x += d;
// t = 0.  zero_start: d = c2 D^{-1} g; x = d (first step from x = 0).
// Rows that are not smoothed have D^{-1} = 0 and keep d = 0.
template <typename T>
__device__ __forceinline__ void cheb_step_at(int64_t n, T* __restrict__ x, T* __restrict__ d,
                                             const T* __restrict__ g, T* __restrict__ t,
                                             const T* __restrict__ dinv, T c1, T c2, int zero_start, int64_t b) {
  const int64_t i = b * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T di = dinv[i];
  if (zero_start) {
    const T v = c2 * di * g[i];
    d[i] = v;
    x[i] = v;
  } else {
    const T v = c1 * d[i] + c2 * di * (g[i] - t[i]);
    d[i] = v;
    x[i] += v;
    t[i] = T(0);
  }
}
template <typename T>
__global__ void cheb_step(int64_t n, T* __restrict__ x, T* __restrict__ d, const T* __restrict__ g,
                          T* __restrict__ t, const T* __restrict__ dinv, T c1, T c2, int zero_start) {
  cheb_step_at(n, x, d, g, t, dinv, c1, c2, zero_start, blockIdx.x);
}

template <typename T>
__device__ __forceinline__ void copy_to_levels_at(int64_t n, const int32_t* __restrict__ copy,
                                                  const double* __restrict__ r, T* __restrict__ lg, int64_t b) {
  const int64_t i = b * blockDim.x + threadIdx.x;
  if (i < n) lg[copy[i]] = T(r[i]);
}
template <typename T>
__global__ void copy_to_levels(int64_t n, const int32_t* __restrict__ copy, const double* __restrict__ r,
                               T* __restrict__ lg) {
  copy_to_levels_at(n, copy, r, lg, blockIdx.x);
}

template <typename T>
__device__ __forceinline__ void copy_from_levels_at(int64_t n, const int32_t* __restrict__ copy,
                                                    const T* __restrict__ lx, double* __restrict__ z, int64_t b) {
  const int64_t i = b * blockDim.x + threadIdx.x;
  if (i < n) z[i] = double(lx[copy[i]]);
}
template <typename T>
__global__ void copy_from_levels(int64_t n, const int32_t* __restrict__ copy, const T* __restrict__ lx,
                                 double* __restrict__ z) {
  copy_from_levels_at(n, copy, lx, z, blockIdx.x);
}

// z = level solution read back through the copy map, fused with the partial
// sums of r.z (kFuseNPT nodes per thread, one partial per block)
template <typename T>
__global__ void __launch_bounds__(kBlock) copy_from_levels_dot(int64_t n, const int32_t* __restrict__ copy,
                                                               const T* __restrict__ lx, double* __restrict__ z,
                                                               const double* __restrict__ r,
                                                               double* __restrict__ part);

// exact coarse solve: x0[S] = A0^{-1} d0[S] (FP64), other rows of x0 zero
template <typename T>
__device__ __forceinline__ void coarse_solve_at(int n_nodes, int n0, const double* __restrict__ ainv,
                                                const int32_t* __restrict__ idx, const T* __restrict__ d0,
                                                T* __restrict__ x0) {
  HIP_DYNAMIC_SHARED(double, sd)
  for (int i = threadIdx.x; i < n_nodes; i += blockDim.x) x0[i] = T(0);
  for (int i = threadIdx.x; i < n0; i += blockDim.x) sd[i] = double(d0[idx[i]]);
  __syncthreads();
  for (int i = threadIdx.x; i < n0; i += blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < n0; ++j) s += ainv[(int64_t)i * n0 + j] * sd[j];
    x0[idx[i]] = T(s);
  }
}
template <typename T>
__global__ void __launch_bounds__(kBlock) coarse_solve(int n_nodes, int n0, const double* __restrict__ ainv,
                                                       const int32_t* __restrict__ idx, const T* __restrict__ d0,
                                                       T* __restrict__ x0) {
  coarse_solve_at(n_nodes, n0, ainv, idx, d0, x0);
}

// ------------------------------------------------------------------ pass 2
// sum of the slots of node i, four independent loads at a time (fixed order)
template <typename T>
__device__ __forceinline__ T seg_sum(const int32_t* __restrict__ off, const T* __restrict__ E, int64_t i) {
  T y = 0;
  int32_t p = off[i];
  const int32_t e = off[i + 1];
  for (; p + 4 <= e; p += 4) {
    const T a0 = E[p], a1 = E[p + 1], a2 = E[p + 2], a3 = E[p + 3];
    y += (a0 + a1) + (a2 + a3);
  }
  for (; p < e; ++p) y += E[p];
  return y;
}

// residual r = g - A x on free rows, 0 on Dirichlet rows (use_e = 0: A x = 0)
template <typename T>
__device__ __forceinline__ void seg_residual_at(int64_t n, const int32_t* __restrict__ off, const T* __restrict__ E,
                                                const T* __restrict__ g, const uint8_t* __restrict__ flags,
                                                T* __restrict__ r, int use_e, int64_t b) {
  const int64_t i = b * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T y = use_e ? seg_sum(off, E, i) : T(0);
  r[i] = flags[i] == 2 ? T(0) : g[i] - y;
}
template <typename T>
__global__ void seg_residual(int64_t n, const int32_t* __restrict__ off, const T* __restrict__ E,
                             const T* __restrict__ g, const uint8_t* __restrict__ flags, T* __restrict__ r,
                             int use_e) {
  seg_residual_at(n, off, E, g, flags, r, use_e, blockIdx.x);
}

template <typename T>
__global__ void seg_plain(int64_t n, const int32_t* __restrict__ off, const T* __restrict__ E, T* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = seg_sum(off, E, i);
}

// g += restricted contributions; then the first Chebyshev step from x = 0:
// d = c2 D^{-1} g, x = d
template <typename T>
__device__ __forceinline__ void seg_restrict_start_at(int64_t n, const int32_t* __restrict__ off,
                                                      const T* __restrict__ E, T* __restrict__ g, T* __restrict__ x,
                                                      T* __restrict__ d, const T* __restrict__ dinv, T c2,
                                                      int smooth, int64_t b) {
  const int64_t i = b * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T gi = g[i] + seg_sum(off, E, i);
  g[i] = gi;
  if (smooth) {
    const T v = c2 * dinv[i] * gi;
    d[i] = v;
    x[i] = v;
  }
}
template <typename T>
__global__ void seg_restrict_start(int64_t n, const int32_t* __restrict__ off, const T* __restrict__ E,
                                   T* __restrict__ g, T* __restrict__ x, T* __restrict__ d,
                                   const T* __restrict__ dinv, T c2, int smooth) {
  seg_restrict_start_at(n, off, E, g, x, d, dinv, c2, smooth, blockIdx.x);
}

#ifdef GMG_SOLVER_TU
// Non-template kernels: compiled in the solver translation unit only.

// leaf operator, pass 2: per-DoF sums, Dirichlet rows zero
__global__ void seg_dir(int64_t n, const int32_t* __restrict__ off, const double* __restrict__ E,
                        const uint8_t* __restrict__ dir, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = seg_sum(off, E, i);
  y[i] = dir[i] ? 0.0 : s;
}

// ------------------------------------------------------------------ CG (FP64)
constexpr int kDotBlocks = 1024;

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kBlock / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBlock / 64; ++i) s += red[i];
  return s;
}

// deterministic two-stage dot: fixed grid, fixed order
__global__ void __launch_bounds__(kBlock) dot_partial(int64_t n, const double* __restrict__ a,
                                                      const double* __restrict__ b, double* __restrict__ part) {
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += a[i] * b[i];
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

enum ScalarSlot { kRho = 0, kRhoOld, kAlpha, kBeta, kPq, kRr, kBb, kFirst, kNumScalars };

// sums the partials (fixed order) and updates the CG scalars
__device__ __forceinline__ void cg_scalars_at(int nparts, const double* __restrict__ part,
                                              double* __restrict__ sc, int op) {
  // each thread adds its strided partials in ascending order, eight loads
  // issued at a time (the order of the additions is that of one at a time)
  double v = 0.0;
  const int st = blockDim.x;
  int i = threadIdx.x;
  for (; i + 7 * st < nparts; i += 8 * st) {
    double a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = part[i + k * st];
#pragma unroll
    for (int k = 0; k < 8; ++k) v += a[k];
  }
  for (; i < nparts; i += st) v += part[i];
  v = block_sum(v);
  if (threadIdx.x != 0) return;
  if (op == 0) {  // rho = r.z ; beta
    sc[kBeta] = sc[kFirst] != 0.0 ? 0.0 : v / sc[kRhoOld];
    sc[kRho] = v;
  } else if (op == 1) {  // pq = p.Ap ; alpha
    sc[kPq] = v;
    sc[kAlpha] = sc[kRho] / v;
  } else if (op == 2) {  // rr ; shift rho
    sc[kRr] = v;
    sc[kRhoOld] = sc[kRho];
    sc[kFirst] = 0.0;
  } else if (op == 3) {
    sc[kBb] = v;
  }
}
__global__ void __launch_bounds__(kBlock) cg_scalars(int nparts, const double* __restrict__ part,
                                                     double* __restrict__ sc, int op) {
  cg_scalars_at(nparts, part, sc, op);
}

__device__ __forceinline__ void update_p_at(int64_t n, double* __restrict__ p, const double* __restrict__ z,
                                            const double* __restrict__ sc, int64_t b) {
  const int64_t i = b * blockDim.x + threadIdx.x;
  const double beta = sc[kBeta];
  if (i < n) p[i] = z[i] + beta * p[i];
}
__global__ void update_p(int64_t n, double* __restrict__ p, const double* __restrict__ z,
                         const double* __restrict__ sc) {
  update_p_at(n, p, z, sc, blockIdx.x);
}

// x += alpha p ; r -= alpha q ; partial sums of r.r with the dot's grid
__device__ __forceinline__ void update_xr_at(int64_t n, double* __restrict__ x, double* __restrict__ r,
                                             const double* __restrict__ p, const double* __restrict__ q,
                                             const double* __restrict__ sc, double* __restrict__ part, int64_t b,
                                             int64_t nb) {
  const double alpha = sc[kAlpha];
  const int64_t st = nb * blockDim.x;
  double s = 0.0;
  int64_t i = b * blockDim.x + threadIdx.x;
  // four strided nodes per step, their loads issued together (the fixed grid
  // otherwise has too few loads in flight to reach the copy rate); the sum of
  // r.r is formed in the same order as one node at a time
  for (; i + 3 * st < n; i += 4 * st) {
    double xv[4], pv[4], rv[4], qv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      xv[k] = x[i + k * st];
      pv[k] = p[i + k * st];
      rv[k] = r[i + k * st];
      qv[k] = q[i + k * st];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      x[i + k * st] = xv[k] + alpha * pv[k];
      const double ri = rv[k] - alpha * qv[k];
      r[i + k * st] = ri;
      s += ri * ri;
    }
  }
  for (; i < n; i += st) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    s += ri * ri;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[b] = s;
}
__global__ void __launch_bounds__(kBlock) update_xr(int64_t n, double* __restrict__ x, double* __restrict__ r,
                                                    const double* __restrict__ p, const double* __restrict__ q,
                                                    const double* __restrict__ sc, double* __restrict__ part) {
  update_xr_at(n, x, r, p, q, sc, part, blockIdx.x, gridDim.x);
}

// nodes per thread of the kernels fused with a dot product (kFuseNPT
// consecutive block-strided nodes, unrolled so that their loads issue
// together; one partial per block, summed in fixed order by cg_scalars)
constexpr int kFuseNPT = 8;
// nodes per thread of the leaf operator's second pass
constexpr int kP2NPT = 4;

// tiled leaf operator, pass 2: the listed nodes' slots (sums of the tiles
// listing them, in ascending slot order) added to q, which holds the owning
// tile's sum; Dirichlet rows stay zero; DOT: partial sums of p.q over the
// added parts per block
template <bool DOT>
__device__ __forceinline__ void leaf_pass2_at(const LeafView& v, const double* __restrict__ E,
                                              const double* __restrict__ x, double* __restrict__ y,
                                              double* __restrict__ part, int64_t b) {
  // kP2NPT nodes per thread, the first kP2S slots of each unrolled so that
  // the loads of all of them issue together; longer lists continue in a
  // loop.  Every load reads a valid address (node index clamped to the last
  // node, slot index to the node's last slot: every node has one) and the
  // unused values are dropped, since loads under a lane mask were compiled
  // into branches that waited for each load before issuing the next.
  constexpr int kP2S = 2;
  const int64_t base = b * blockDim.x * kP2NPT + threadIdx.x;
  const int64_t last = v.n_p2 - 1;
  bool in[kP2NPT];
  int32_t d[kP2NPT], o0[kP2NPT], o1[kP2NPT];
#pragma unroll
  for (int k = 0; k < kP2NPT; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    in[k] = i <= last;
    const int64_t ic = in[k] ? i : last;
    d[k] = v.p2_dof[ic];
    o0[k] = v.p2_off[ic];
    o1[k] = v.p2_off[ic + 1];
  }
  int32_t sl[kP2NPT][kP2S];
#pragma unroll
  for (int k = 0; k < kP2NPT; ++k)
#pragma unroll
    for (int j = 0; j < kP2S; ++j) sl[k][j] = v.p2_slot[o0[k] + j < o1[k] ? o0[k] + j : o1[k] - 1];
  double y0[kP2NPT], xd[kP2NPT];
  uint8_t dr[kP2NPT];
#pragma unroll
  for (int k = 0; k < kP2NPT; ++k) {
    y0[k] = y[d[k]];
    dr[k] = v.dir[d[k]];
    if (DOT) xd[k] = x[d[k]];
  }
  double ev[kP2NPT][kP2S];
#pragma unroll
  for (int k = 0; k < kP2NPT; ++k)
#pragma unroll
    for (int j = 0; j < kP2S; ++j) ev[k][j] = E[sl[k][j]];
  double q[kP2NPT];
#pragma unroll
  for (int k = 0; k < kP2NPT; ++k) {
    q[k] = 0.0;
#pragma unroll
    for (int j = 0; j < kP2S; ++j) q[k] += o0[k] + j < o1[k] ? ev[k][j] : 0.0;
    for (int32_t o = o0[k] + kP2S; o < o1[k]; ++o) q[k] += E[v.p2_slot[o]];
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kP2NPT; ++k) {
    if (in[k] && !dr[k]) {
      y[d[k]] = y0[k] + q[k];
      if (DOT) s += xd[k] * q[k];
    }
  }
  if (DOT) {
    s = block_sum(s);
    if (threadIdx.x == 0) part[b] = s;
  }
}
template <bool DOT>
__global__ void __launch_bounds__(kBlock) leaf_pass2(LeafView v, const double* __restrict__ E,
                                                     const double* __restrict__ x, double* __restrict__ y,
                                                     double* __restrict__ part) {
  leaf_pass2_at<DOT>(v, E, x, y, part, blockIdx.x);
}

// leaf operator, pass 2, fused with the partial sums of p.q
__global__ void __launch_bounds__(kBlock) seg_dir_dot(int64_t n, const int32_t* __restrict__ off,
                                                      const double* __restrict__ E, const uint8_t* __restrict__ dir,
                                                      double* __restrict__ q, const double* __restrict__ p,
                                                      double* __restrict__ part) {
  const int64_t base = (int64_t)blockIdx.x * blockDim.x * kFuseNPT + threadIdx.x;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kFuseNPT; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    if (i < n) {
      const double v = dir[i] ? 0.0 : seg_sum(off, E, i);
      q[i] = v;
      s += p[i] * v;
    }
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename T>
__device__ __forceinline__ void copy_from_levels_dot_at(int64_t n, const int32_t* __restrict__ copy,
                                                        const T* __restrict__ lx, double* __restrict__ z,
                                                        const double* __restrict__ r, double* __restrict__ part,
                                                        int64_t b) {
  // every load reads a valid address (index clamped to the last node; the
  // lanes past the end drop their values), so that the loads of all nodes of
  // a thread issue together instead of one masked branch after another
  const int64_t base = b * blockDim.x * kFuseNPT + threadIdx.x;
  int32_t cp[kFuseNPT];
  double rv[kFuseNPT], v[kFuseNPT];
#pragma unroll
  for (int k = 0; k < kFuseNPT; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    const int64_t ic = i < n ? i : n - 1;
    cp[k] = copy[ic];
    rv[k] = r[ic];
  }
#pragma unroll
  for (int k = 0; k < kFuseNPT; ++k) v[k] = double(lx[cp[k]]);
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kFuseNPT; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    if (i < n) {
      z[i] = v[k];
      s += rv[k] * v[k];
    }
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[b] = s;
}
template <typename T>
__global__ void __launch_bounds__(kBlock) copy_from_levels_dot(int64_t n, const int32_t* __restrict__ copy,
                                                               const T* __restrict__ lx, double* __restrict__ z,
                                                               const double* __restrict__ r,
                                                               double* __restrict__ part) {
  copy_from_levels_dot_at(n, copy, lx, z, r, part, blockIdx.x);
}

__global__ void copy_vec(int64_t n, const double* __restrict__ a, double* __restrict__ b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// eigenvalue-estimate helpers (FP64, level vectors)
// start vector r (set on the host, zero off the S rows): z = p = D^{-1} r
__global__ void eig_init(int64_t n, const double* __restrict__ dinv, const double* __restrict__ r,
                         double* __restrict__ z, double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = r[i];
  z[i] = dinv[i] * v;
  p[i] = dinv[i] * v;
}

__global__ void axpy_zr(int64_t n, double alpha, const double* __restrict__ q, double* __restrict__ r,
                        const double* __restrict__ dinv, double* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double ri = r[i] - alpha * q[i];
  r[i] = ri;
  z[i] = dinv[i] * ri;
}

__global__ void xpby(int64_t n, const double* __restrict__ z, double beta, double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = z[i] + beta * p[i];
}

#endif  // GMG_SOLVER_TU

}  // namespace dev
}  // namespace gmg

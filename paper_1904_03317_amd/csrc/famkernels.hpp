// Level kernels on the entity layout of levels >= 1 (families of 2^d
// siblings; the layout is described in host/layout.hpp).  Operator, smoother
// update, residual and transfers (Sec. 2.2, 2.3, 4.1) without stored node
// maps: a family holds the base index of each of its 3^d entities, and the
// node index and operator slot of every patch position follow from the
// position's entity and its offset inside it.
//
// Operator, two passes.  Pass 1 (fam_op): a workgroup stages the node
// patches of FB families in LDS (interiors, contiguous in memory, by
// coalesced loads; entity nodes through the entity bases), one lane computes
// one cell, siblings combine by lane shuffles (floating-point atomics in LDS
// measured several times slower for FP32).  Values at nodes no other family
// touches (the family interior, and level-boundary entities) are final and
// go straight through the epilogue (Chebyshev update, residual, or plain
// output); values at shared entities go to the entity's slot for this
// family's position.  Pass 2 (fam_sum) runs over the shared nodes only:
// each sums its present position slots in a fixed order and applies the
// same epilogue.  No atomics in global memory, no index arrays per node;
// all loads of an epilogue are issued before their values are used.
//
// In 3D at k >= 3 a cell's values no longer fit one lane: the cooperative
// kernels (*_coop) share each cell's 1D line contractions among the threads
// of a workgroup through LDS and keep the same patch epilogues and slots.
#pragma once
#include "dispatch.hpp"
#include "kernels.hpp"

namespace gmg {
namespace dev {

enum { kEpiPlain = 0, kEpiCheb = 1, kEpiResid = 2, kEpiDiag = 3, kEpiRStart = 4 };

// Vectors of one level for the epilogues (pointers already offset to the level).
//   plain / diag: y = A x (or diag A)
//   cheb:  d = c1 d + c2 D^{-1} (g - A x), x += d    (Sec. 4.1 smoother step)
//   resid: y = g - A x, 0 on Dirichlet rows
//   rstart: g += restricted contribution; if smooth: d = c2 D^{-1} g, x = d
template <typename T>
struct Epi {
  T* x = nullptr;
  T* d = nullptr;
  T* y = nullptr;
  T* g = nullptr;
  const T* dinv = nullptr;
  const uint8_t* flags = nullptr;
  T c1 = 0, c2 = 0;
  int smooth = 0;
};

// Patch geometry of a family: (2k+1)^d positions, 3^d entities.
template <int DIM, int K>
struct Geo {
  static constexpr int N = K + 1, M2 = 2 * K + 1, S1 = 2 * K - 1;
  static constexpr int MF = DIM == 3 ? M2 * M2 * M2 : M2 * M2;
  static constexpr int NP = DIM == 3 ? N * N * N : N * N;
  static constexpr int NJ = DIM == 3 ? 27 : 9;
  static constexpr int CPF = 1 << DIM;
  static constexpr int NI = DIM == 3 ? S1 * S1 * S1 : S1 * S1;  // interior positions
  static constexpr int NB = MF - NI;                             // entity positions
  static constexpr int INTERIOR = DIM == 3 ? 13 : 4;             // entity index of the interior
  // patch position of interior offset loc
  __host__ __device__ static constexpr int iq(int loc) {
    const int lx = loc % S1, ly = (loc / S1) % S1, lz = DIM == 3 ? loc / (S1 * S1) : 0;
    return (lx + 1) + M2 * ((ly + 1) + M2 * (DIM == 3 ? lz + 1 : 0));
  }
  // index of an entity position among the entity positions (ascending q)
  __host__ __device__ static constexpr int bidx(int q) {
    const int qx = q % M2, qy = (q / M2) % M2, qz = DIM == 3 ? q / (M2 * M2) : 0;
    auto cnt = [](int a) { return a <= 0 ? 0 : a - 1 > S1 ? S1 : a - 1; };
    auto in = [](int a) { return a >= 1 && a <= S1; };
    int before = DIM == 3 ? cnt(qz) * S1 * S1 : 0;
    if (DIM == 2 || in(qz)) {
      before += cnt(qy) * S1;
      if (in(qy)) before += cnt(qx);
    }
    return q - before;
  }
  // code of position q: entity j (bits 0-4), offset in the entity (5-19),
  // boundary axes r (20-21), position around the entity (23-25)
  __host__ __device__ static constexpr uint32_t code(int q) {
    int j = 0, loc = 0, r = 0, pos = 0, mul = 1, st = 1, t = q;
    for (int a = 0; a < DIM; ++a) {
      const int qa = t % M2;
      t /= M2;
      const int c = qa == 0 ? 0 : qa == 2 * K ? 2 : 1;
      j += c * mul;
      mul *= 3;
      if (c == 1) {
        loc += (qa - 1) * st;
        st *= S1;
      } else {
        pos |= (c == 2 ? 1 : 0) << r;
        ++r;
      }
    }
    return (uint32_t)j | ((uint32_t)loc << 5) | ((uint32_t)r << 20) | ((uint32_t)pos << 23);
  }
  __host__ __device__ static constexpr int size_r(int r) {
    int s = 1;
    for (int i = 0; i < DIM - r; ++i) s *= S1;
    return s;
  }
  static __device__ __forceinline__ int cj(uint32_t c) { return (int)(c & 31u); }
  static __device__ __forceinline__ int cloc(uint32_t c) { return (int)((c >> 5) & 0x7fffu); }
  static __device__ __forceinline__ int cr(uint32_t c) { return (int)((c >> 20) & 3u); }
  static __device__ __forceinline__ int cpos(uint32_t c) { return (int)((c >> 23) & 7u); }
};

// Families per workgroup of the lane-per-cell kernels (k <= 2, and 2D): LDS
// holds the input and output patches, the entity bases of FB families and
// the position codes (at most 80 KB at k <= 2, 160 KB at k >= 3 in 2D, of the
// 160 KB of a gfx950 CU).
template <int DIM, int K, typename T>
struct FamShape {
  using G = Geo<DIM, K>;
  static constexpr int MF = G::MF, CPF = G::CPF, NJ = G::NJ;
  // padded patch length: odd in 4-byte words so that families fall on
  // different LDS banks
  static constexpr int MFP = sizeof(T) == 4 ? (MF % 2 ? MF + 2 : MF + 1) : MF + 1;
  // LDS budget per workgroup: two workgroups per CU at k <= 2 (FP64 half
  // that: its register count allows two waves per SIMD anyway, and smaller
  // workgroups overlap their memory phases better), one at k >= 3
  static constexpr int budget = K >= 3 ? 163840 : sizeof(T) == 8 ? 40960 : 81920;
  static constexpr int fixed = G::NB * 14 + 256;
  static constexpr int fb_lds = (budget - fixed) / (2 * MFP * (int)sizeof(T) + NJ * 4 + 4);
  static constexpr int fb_cap = 256 / CPF;
  static constexpr int fb_raw = fb_lds < fb_cap ? fb_lds : fb_cap;
  static constexpr int FB = fb_raw >= 64 ? 64 : fb_raw >= 32 ? 32 : fb_raw >= 16 ? 16 : fb_raw >= 8 ? 8 : 4;
  static constexpr int THREADS = FB * CPF;
  // entity positions handled per round of the output epilogue (registers)
  static constexpr int CH = 5;
  static constexpr int ITI = (G::NI * FB + THREADS - 1) / THREADS;
  static constexpr int ITB = (G::NB * FB + THREADS - 1) / THREADS;
};

// Operator shape in 3D at k >= 3, where a cell's (k+1)^3 values and their
// products no longer fit one lane's registers: the threads of a workgroup
// share the sum-factorized contractions of all cells of its families, one
// thread per 1D line of a cell and direction, through two LDS arrays of
// per-cell intermediates; each patch position then sums the values of the
// cells containing it, in ascending child order.
template <int DIM, int K>
inline constexpr bool kCoopOp = DIM == 3 && K >= 3;

template <int DIM, int K, typename T>
struct CoopShape {
  using G = Geo<DIM, K>;
  static constexpr int N = G::N, MF = G::MF, CPF = G::CPF, NJ = G::NJ;
  static constexpr int MFP = FamShape<DIM, K, T>::MFP;
  // per-cell intermediates, x fastest, rows padded to an odd length so that
  // the lines along x of consecutive threads fall on different LDS banks
  static constexpr int NXP = N % 2 ? N : N + 1;
  static constexpr int CS = NXP * N * N;
  static constexpr int FS = CPF * CS;  // per family; the output patch reuses the second array
  static constexpr int THREADS = 256;
  // LDS per workgroup: small, so that several workgroups per CU overlap
  // their memory phases (with waves_per_eu below; measured best among
  // budgets of 27-160 KB and 128-512 threads)
  static constexpr int budget = 32768;
  static constexpr int fixed = G::NB * 14 + 256;
  static constexpr int FB = (budget - fixed) / ((MFP + 2 * FS) * (int)sizeof(T) + NJ * 4 + 4);
  static constexpr int CH = 5;
  static constexpr int ITI = (G::NI * FB + THREADS - 1) / THREADS;
  static constexpr int ITB = (G::NB * FB + THREADS - 1) / THREADS;
  static constexpr int NL = N * N;  // lines per cell and direction
  static constexpr int ITL = (FB * CPF * NL + THREADS - 1) / THREADS;
  static constexpr int ITQ = (FB * MF + THREADS - 1) / THREADS;
  static_assert(FB >= 1 && FS >= MFP, "cooperative operator shape");
};

// Operator slot of a shared-entity position (r >= 1) of a family whose
// entity base is gb: eoff[r] + (gb - sec[r]) 2^r + pos size_r + loc.  All
// terms but gb 2^r depend on the position only and are tabulated per
// workgroup (bo, from stage_bases), so that the per-section offsets of the
// view are not indexed at run time in the hot loops.
template <int DIM, int K>
__device__ __forceinline__ int64_t slot_part(const LevelView& v, uint32_t c) {
  using G = Geo<DIM, K>;
  const int r = G::cr(c);
  const int sz = r == 1 ? G::size_r(1) : r == 2 ? G::size_r(2) : G::size_r(3);
  return v.eoff[r] - (v.sec[r] << r) + (int64_t)G::cpos(c) * sz + G::cloc(c);
}

// Epilogue on IT nodes (node < 0: nothing), split into the loads of its
// operands (epi_load, at a valid index — node 0 of the level — when the node
// is skipped) and the arithmetic plus predicated stores (epi_apply), so that
// the loads can be issued early and no control flow sits between a load and
// its use; stores share the wait counter with loads.
// FLAGS: the nodes may be interface or Dirichlet nodes (residual rows of D
// nodes are zero); family-interior nodes are always smoothed nodes.
// xo: the node's x before this operator application (Chebyshev update).
template <typename T, int IT>
struct EpiOps {
  T d[IT], g[IT], di[IT];
  uint8_t fl[IT];
};

template <typename T, int EPI, int IT, bool FLAGS>
__device__ __forceinline__ void epi_load(const Epi<T>& ep, const int32_t (&node)[IT], EpiOps<T, IT>& o) {
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int32_t i = node[it] >= 0 ? node[it] : 0;
    if (EPI == kEpiCheb) {
      o.d[it] = ep.d[i];
      o.g[it] = ep.g[i];
      o.di[it] = ep.dinv[i];
    } else if (EPI == kEpiResid) {
      o.g[it] = ep.g[i];
      o.fl[it] = FLAGS ? ep.flags[i] : 0;
    } else if (EPI == kEpiRStart) {
      o.g[it] = ep.g[i];
      o.di[it] = ep.smooth ? ep.dinv[i] : T(0);
    }
  }
}

template <typename T, int EPI, int IT>
__device__ __forceinline__ void epi_apply(const Epi<T>& ep, const int32_t (&node)[IT], const T (&ax)[IT],
                                          const T (&xo)[IT], EpiOps<T, IT>& o) {
  if (EPI == kEpiPlain || EPI == kEpiDiag) {
#pragma unroll
    for (int it = 0; it < IT; ++it)
      if (node[it] >= 0) ep.y[node[it]] = ax[it];
  } else if (EPI == kEpiCheb) {
#pragma unroll
    for (int it = 0; it < IT; ++it) o.d[it] = ep.c1 * o.d[it] + ep.c2 * o.di[it] * (o.g[it] - ax[it]);
#pragma unroll
    for (int it = 0; it < IT; ++it)
      if (node[it] >= 0) {
        ep.d[node[it]] = o.d[it];
        ep.x[node[it]] = xo[it] + o.d[it];
      }
  } else if (EPI == kEpiResid) {
#pragma unroll
    for (int it = 0; it < IT; ++it) o.g[it] = o.fl[it] == 2 ? T(0) : o.g[it] - ax[it];
#pragma unroll
    for (int it = 0; it < IT; ++it)
      if (node[it] >= 0) ep.y[node[it]] = o.g[it];
  } else {  // kEpiRStart
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      o.g[it] += ax[it];
      o.di[it] = ep.c2 * o.di[it] * o.g[it];
    }
#pragma unroll
    for (int it = 0; it < IT; ++it)
      if (node[it] >= 0) {
        ep.g[node[it]] = o.g[it];
        if (ep.smooth) {
          ep.d[node[it]] = o.di[it];
          ep.x[node[it]] = o.di[it];
        }
      }
  }
}

template <typename T, int EPI, int IT, bool FLAGS>
__device__ __forceinline__ void epi_batch(const Epi<T>& ep, const int32_t (&node)[IT], const T (&ax)[IT],
                                          const T (&xo)[IT]) {
  EpiOps<T, IT> o;
  epi_load<T, EPI, IT, FLAGS>(ep, node, o);
  epi_apply<T, EPI, IT>(ep, node, ax, xo, o);
}

// interior nodes of the workgroup's families: node f0 NI + e for e < nf NI
// (contiguous), else -1
template <int DIM, int K, typename T, typename S = FamShape<DIM, K, T>>
__device__ __forceinline__ void interior_nodes(int64_t f0, int nf, int32_t (&node)[S::ITI]) {
  constexpr int NI = Geo<DIM, K>::NI;
#pragma unroll
  for (int it = 0; it < S::ITI; ++it) {
    const int e = threadIdx.x + it * S::THREADS;
    node[it] = e < nf * NI ? (int32_t)(f0 * NI + e) : -1;
  }
}

// single shared node (pass 2)
template <typename T, int EPI>
__device__ __forceinline__ void epi_shared(const Epi<T>& ep, int64_t i, T ax) {
  if (EPI == kEpiPlain || EPI == kEpiDiag) {
    ep.y[i] = ax;
  } else if (EPI == kEpiCheb) {
    const T dn = ep.c1 * ep.d[i] + ep.c2 * ep.dinv[i] * (ep.g[i] - ax);
    ep.d[i] = dn;
    ep.x[i] += dn;
  } else if (EPI == kEpiResid) {
    ep.y[i] = ep.flags[i] == 2 ? T(0) : ep.g[i] - ax;
  } else {
    const T gi = ep.g[i] + ax;
    ep.g[i] = gi;
    if (ep.smooth) {
      const T dn = ep.c2 * ep.dinv[i] * gi;
      ep.d[i] = dn;
      ep.x[i] = dn;
    }
  }
}

// stage the entity bases and exclusivity bits of the workgroup's families
// and the table of entity positions (position, code, slot part)
template <int DIM, int K, typename T, typename S = FamShape<DIM, K, T>>
__device__ __forceinline__ void stage_bases(const LevelView& v, int64_t f0, int32_t* sgb, uint32_t* sex,
                                            uint16_t* bq, uint32_t* bc, int64_t* bo) {
  using G = Geo<DIM, K>;
  for (int e = threadIdx.x; e < S::FB * G::NJ; e += S::THREADS) {
    const int j = e / S::FB, fl = e % S::FB;
    sgb[fl * G::NJ + j] = f0 + fl < v.n_fam ? v.gbase[(int64_t)j * v.n_fam + f0 + fl] : 0;
  }
  for (int fl = threadIdx.x; fl < S::FB; fl += S::THREADS) sex[fl] = f0 + fl < v.n_fam ? v.excl[f0 + fl] : 0u;
  for (int q = threadIdx.x; q < G::MF; q += S::THREADS) {
    const uint32_t c = G::code(q);
    if (G::cr(c) != 0) {
      const int b = G::bidx(q);
      bq[b] = (uint16_t)q;
      bc[b] = c;
      bo[b] = slot_part<DIM, K>(v, c);
    }
  }
}

// cell k of a family (child position bits x, y, z): offset of its node
// (jx, jy, jz) in the family patch
template <int DIM, int K>
__device__ __forceinline__ int cell_patch_pos(int cid, int j) {
  using G = Geo<DIM, K>;
  constexpr int N = G::N, M2 = G::M2;
  const int bx = (cid & 1) * K, by = ((cid >> 1) & 1) * K, bz = DIM == 3 ? ((cid >> 2) & 1) * K : 0;
  const int jx = j % N, jy = (j / N) % N, jz = DIM == 3 ? j / (N * N) : 0;
  return ((bz + jz) * M2 + (by + jy)) * M2 + (bx + jx);
}

// Value of the lane whose index differs in bit B (B = 0, 1, 2) from this
// lane's, by data-parallel moves inside each group of 8 lanes (no LDS):
// xor 1 and xor 2 are quad permutations, xor 4 is the mirror inside each
// half row followed by the reversal inside each quad.
template <int B>
__device__ __forceinline__ int32_t lane_xor(int32_t v) {
  constexpr int kQuadXor1 = 0xB1, kQuadXor2 = 0x4E, kQuadRev = 0x1B, kHalfMirror = 0x141;
  if (B == 0) return __builtin_amdgcn_mov_dpp(v, kQuadXor1, 0xF, 0xF, false);
  if (B == 1) return __builtin_amdgcn_mov_dpp(v, kQuadXor2, 0xF, 0xF, false);
  return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, kHalfMirror, 0xF, 0xF, false), kQuadRev, 0xF, 0xF,
                                  false);
}
template <int B>
__device__ __forceinline__ float lane_xor(float v) {
  return __int_as_float(lane_xor<B>(__float_as_int(v)));
}
template <int B>
__device__ __forceinline__ double lane_xor(double v) {
  const long long u = __double_as_longlong(v);
  const int32_t lo = lane_xor<B>((int32_t)(u & 0xffffffffLL)), hi = lane_xor<B>((int32_t)(u >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(uint32_t)lo);
}

// c ? a : b by bit masks: a value select the compiler cannot turn into a
// select of addresses (which would index the cell array at run time and move
// it from registers to scratch memory)
__device__ __forceinline__ float sel(bool c, float a, float b) {
  const int32_t m = -(int32_t)c;
  return __int_as_float((__float_as_int(a) & m) | (__float_as_int(b) & ~m));
}
__device__ __forceinline__ double sel(bool c, double a, double b) {
  const long long m = -(long long)c;
  return __longlong_as_double((__double_as_longlong(a) & m) | (__double_as_longlong(b) & ~m));
}

// Sum over the 2^d sibling cells of a family of their per-node values.  The
// cells of a family sit in 2^d consecutive lanes of one wave (lane bits =
// child position bits x, y, z).  Axis by axis, the two cells on either side
// of the family's middle plane exchange their values on that plane and keep
// the sum (the same sum in both lanes: addition is commutative); after d
// stages every lane holds, for each of its nodes, the sum over all cells of
// the family that contain the node.  Every lane of the wave must take part.
template <int DIM, int N, int A, typename T>
__device__ __forceinline__ void family_sum_axis(int cid, T (&w)[DIM == 3 ? N * N * N : N * N]) {
  constexpr int K = N - 1;
  constexpr int NZ = DIM == 3 ? N : 1;
  const bool hi = (cid >> A) & 1;
#pragma unroll
  for (int s = 0; s < N * NZ; ++s) {
    // the two other local indices of a node on the plane normal to A
    const int u = s % N, v = s / N;
    const int i0 = A == 0 ? (v * N + u) * N : A == 1 ? v * N * N + u : v * N + u;  // index 0 along A
    const int iK = i0 + K * (A == 0 ? 1 : A == 1 ? N : N * N);                    // index K along A
    const T a = w[i0], b = w[iK];
    T t = sel(hi, a, b);
    t += lane_xor<A>(t);
    w[i0] = sel(hi, t, a);
    w[iK] = sel(hi, b, t);
  }
}
template <int DIM, int N, typename T>
__device__ __forceinline__ void family_sum(int cid, T (&w)[DIM == 3 ? N * N * N : N * N]) {
  family_sum_axis<DIM, N, 0, T>(cid, w);
  family_sum_axis<DIM, N, 1, T>(cid, w);
  if (DIM == 3) family_sum_axis<DIM, N, 2, T>(cid, w);
}

// lane cid writes its local node j to the family patch iff no sibling with
// a lower child position contains the node
template <int DIM, int N>
__device__ __forceinline__ bool family_owner(int cid, int j) {
  const int jx = j % N, jy = (j / N) % N, jz = DIM == 3 ? j / (N * N) : 0;
  const int m = (jx == 0 ? 1 : 0) | (jy == 0 ? 2 : 0) | (DIM == 3 && jz == 0 ? 4 : 0);
  return (cid & m) == 0;
}

// ------------------------------------------------------------------ pass 1
// Output of a family patch held in LDS (sout): interior nodes and nodes of
// exclusive entities through the epilogue, shared entities to their slots.
// xo from sin (CHEB only).
template <int DIM, int K, typename T, int EPI, typename S = FamShape<DIM, K, T>>
__device__ __forceinline__ void patch_out(const LevelView& v, int64_t f0, int nf, const T* sout, const T* sin,
                                          const int32_t* sgb, const uint32_t* sex, const uint16_t* bq,
                                          const uint32_t* bc, const int64_t* bo, const Epi<T>& ep,
                                          T* __restrict__ E, const int32_t (&inode)[S::ITI],
                                          EpiOps<T, S::ITI>& iops) {
  using G = Geo<DIM, K>;
  constexpr int MFP = S::MFP, NJ = G::NJ, NI = G::NI, NB = G::NB;
  const int tid = threadIdx.x;
  {
    // interior nodes: operands were loaded before the compute
    T ax[S::ITI], xo[S::ITI];
#pragma unroll
    for (int it = 0; it < S::ITI; ++it) {
      const int e = tid + it * S::THREADS;
      ax[it] = xo[it] = T(0);
      if (inode[it] >= 0) {
        const int fl = e / NI, q = G::iq(e % NI);
        ax[it] = sout[fl * MFP + q];
        if (EPI == kEpiCheb) xo[it] = sin[fl * MFP + q];
      }
    }
    epi_apply<T, EPI, S::ITI>(ep, inode, ax, xo, iops);
  }
  // entity positions, in rounds of CH: values and targets from LDS, the slot
  // stores of shared entities, then the epilogue of exclusive ones
#pragma unroll
  for (int c0 = 0; c0 < S::ITB; c0 += S::CH) {
    int32_t node[S::CH], slot[S::CH];
    T ax[S::CH], xo[S::CH];
#pragma unroll
    for (int k = 0; k < S::CH; ++k) {
      const int it = c0 + k;
      const int e = tid + it * S::THREADS;
      node[k] = slot[k] = -1;
      ax[k] = xo[k] = T(0);
      if (it < S::ITB && e < nf * NB) {
        const int fl = e / NB, b = e % NB;
        const int q = bq[b];
        const uint32_t c = bc[b];
        const int j = G::cj(c);
        const int32_t gb = sgb[fl * NJ + j];
        ax[k] = sout[fl * MFP + q];
        if ((sex[fl] >> j) & 1u) {
          node[k] = gb + G::cloc(c);
          if (EPI == kEpiCheb) xo[k] = sin[fl * MFP + q];
        } else {
          slot[k] = (int32_t)(bo[b] + ((int64_t)gb << G::cr(c)));
        }
      }
    }
#pragma unroll
    for (int k = 0; k < S::CH; ++k)
      if (slot[k] >= 0) E[slot[k]] = ax[k];
    epi_batch<T, EPI, S::CH, true>(ep, node, ax, xo);
  }
}

// node patches of the workgroup's families into LDS (sin[fl MFP + q]):
// interiors by coalesced loads of a contiguous block, entity positions
// through the staged entity bases; all loads issued before the LDS stores
template <int DIM, int K, typename T, typename S = FamShape<DIM, K, T>>
__device__ __forceinline__ void gather_patch(int64_t f0, int nf, const T* __restrict__ xin, const int32_t* sgb,
                                             const uint16_t* bq, const uint32_t* bc, T* sin) {
  using G = Geo<DIM, K>;
  constexpr int MFP = S::MFP, NJ = G::NJ, NI = G::NI, NB = G::NB;
  const int tid = threadIdx.x;
  T vi[S::ITI], vb[S::ITB];
#pragma unroll
  for (int it = 0; it < S::ITI; ++it) {
    const int e = tid + it * S::THREADS;
    vi[it] = e < nf * NI ? xin[f0 * NI + e] : T(0);
  }
#pragma unroll
  for (int it = 0; it < S::ITB; ++it) {
    const int e = tid + it * S::THREADS;
    const int ee = e < nf * NB ? e : 0;  // a valid position when out of range
    const int fl = ee / NB;
    const uint32_t c = bc[ee % NB];
    vb[it] = xin[sgb[fl * NJ + G::cj(c)] + G::cloc(c)];
  }
#pragma unroll
  for (int it = 0; it < S::ITI; ++it) {
    const int e = tid + it * S::THREADS;
    if (e < nf * NI) sin[(e / NI) * MFP + G::iq(e % NI)] = vi[it];
  }
#pragma unroll
  for (int it = 0; it < S::ITB; ++it) {
    const int e = tid + it * S::THREADS;
    if (e < nf * NB) sin[(e / NB) * MFP + bq[e % NB]] = vb[it];
  }
}

// pass 1 for the families of logical block blk
template <int DIM, int K, typename T, int EPI>
__device__ __forceinline__ void fam_op_body(const LevelView& v, const T* __restrict__ xin, const Epi<T>& ep,
                                            T* __restrict__ E, const Mats<T>& m, int64_t blk) {
  using S = FamShape<DIM, K, T>;
  using G = Geo<DIM, K>;
  constexpr int N = G::N, MFP = S::MFP, FB = S::FB, CPF = G::CPF, NJ = G::NJ, NP = G::NP;
  constexpr int NI = G::NI, NB = G::NB;
  __shared__ T sin[FB * MFP];
  __shared__ T sout[FB * MFP];
  __shared__ int32_t sgb[FB * NJ];
  __shared__ uint32_t sex[FB];
  __shared__ uint16_t bq[NB];
  __shared__ uint32_t bc[NB];
  __shared__ int64_t bo[NB];
  const int64_t f0 = blk * FB;
  const int nf = (int)(v.n_fam - f0 < FB ? v.n_fam - f0 : FB);
  const int tid = threadIdx.x;
  // interior epilogue operands: contiguous, known before anything else
  int32_t inode[S::ITI];
  interior_nodes<DIM, K, T>(f0, nf, inode);
  EpiOps<T, S::ITI> iops;
  epi_load<T, EPI, S::ITI, false>(ep, inode, iops);
  stage_bases<DIM, K, T>(v, f0, sgb, sex, bq, bc, bo);
  __syncthreads();
  if (EPI != kEpiDiag) {
    gather_patch<DIM, K, T>(f0, nf, xin, sgb, bq, bc, sin);
    __syncthreads();
  }
  {
    // one lane per cell (all lanes take part in the family sum; lanes of
    // families beyond the level compute on zeros)
    const int fl = tid / CPF, cid = tid % CPF;
    const int64_t f = f0 + fl;
    T w[NP];
    if (EPI == kEpiDiag) {
#pragma unroll
      for (int j = 0; j < NP; ++j) {
        const int jx = j % N, jy = (j / N) % N, jz = DIM == 3 ? j / (N * N) : 0;
        const T mx = m.M[jx * N + jx], my = m.M[jy * N + jy], kx = m.K[jx * N + jx], ky = m.K[jy * N + jy];
        if (DIM == 3) {
          const T mz = m.M[jz * N + jz], kz = m.K[jz * N + jz];
          w[j] = kx * my * mz + mx * ky * mz + mx * my * kz;
        } else {
          w[j] = kx * my + mx * ky;
        }
      }
    } else {
      T u[NP];
#pragma unroll
      for (int j = 0; j < NP; ++j) u[j] = sin[fl * MFP + cell_patch_pos<DIM, K>(cid, j)];
      if (DIM == 3)
        laplace3<N, T>(m, *reinterpret_cast<const T(*)[N * N * N]>(u), *reinterpret_cast<T(*)[N * N * N]>(w));
      else
        laplace2<N, T>(m, *reinterpret_cast<const T(*)[N * N]>(u), *reinterpret_cast<T(*)[N * N]>(w));
    }
    const T sc = fl < nf ? T(v.scale ? v.scale[f * CPF + cid] : v.scale0) : T(0);
#pragma unroll
    for (int j = 0; j < NP; ++j) w[j] *= sc;
    // sibling sum by lane moves (floating-point atomic adds in LDS measured
    // several times slower)
    family_sum<DIM, N, T>(cid, w);
    // every lane holds the family totals of its nodes (bit for bit the same
    // in all lanes sharing a node), so all of them may write
#pragma unroll
    for (int j = 0; j < NP; ++j) sout[fl * MFP + cell_patch_pos<DIM, K>(cid, j)] = w[j];
  }
  __syncthreads();
  patch_out<DIM, K, T, EPI>(v, f0, nf, sout, sin, sgb, sex, bq, bc, bo, ep, E, inode, iops);
}

template <int DIM, int K, typename T, int EPI>
__global__ void __launch_bounds__((FamShape<DIM, K, T>::THREADS)) fam_op(LevelView v, const T* __restrict__ xin,
                                                                          Epi<T> ep, T* __restrict__ E, Mats<T> m) {
  fam_op_body<DIM, K, T, EPI>(v, xin, ep, E, m, xcd_block());
}

// Several levels (of several problems) in one launch: item i covers the
// blocks [b0_i, b0_{i+1}) of the grid, each item a level with its input,
// epilogue and slots.  A level's families get the same logical blocks as in
// a launch of their own, so every result is the same bit for bit.
template <typename T>
struct OpItem {
  LevelView v;
  Epi<T> ep;
  const T* x;
  T* E;
  int64_t b0;
};

template <int DIM, int K, typename T, int EPI>
__global__ void __launch_bounds__((FamShape<DIM, K, T>::THREADS)) fam_op_batch(const OpItem<T>* __restrict__ items,
                                                                                int n, Mats<T> m) {
  const OpItem<T> it = items[batch_item(items, n)];
  fam_op_body<DIM, K, T, EPI>(it.v, it.x, it.ep, it.E, m, (int64_t)blockIdx.x - it.b0);
}

// Pass 1 in 3D at k >= 3 (same contract as fam_op).  Per cell, with the
// cell scale s (coefficient times h): a = M u and b = K u along z; c = M a
// and f = K a + M b along y; s (K c + M f) along x, which is s times
// (K x M x M + M x K x M + M x M x K) u (Sec. 4.1, sum factorization).
template <int DIM, int K, typename T, int EPI>
__global__ void __launch_bounds__((CoopShape<DIM, K, T>::THREADS)) __attribute__((amdgpu_waves_per_eu(5)))
    fam_op_coop(LevelView v, const T* __restrict__ xin, Epi<T> ep, T* __restrict__ E, Mats<T> m) {
  using S = CoopShape<DIM, K, T>;
  using G = Geo<DIM, K>;
  constexpr int N = G::N, M2 = G::M2, MF = G::MF, MFP = S::MFP, FB = S::FB, CPF = G::CPF, NJ = G::NJ;
  constexpr int NB = G::NB, NXP = S::NXP, CS = S::CS, FS = S::FS, NL = S::NL, TH = S::THREADS;
  static_assert(DIM == 3, "cooperative operator is 3D");
  __shared__ T sin[FB * MFP];
  __shared__ T ta[FB * FS];
  __shared__ T tb[FB * FS];
  __shared__ int32_t sgb[FB * NJ];
  __shared__ uint32_t sex[FB];
  __shared__ uint16_t bq[NB];
  __shared__ uint32_t bc[NB];
  __shared__ int64_t bo[NB];
  T* sout = tb;  // family patches of the output, once tb is no longer needed
  const int64_t f0 = xcd_block() * FB;
  const int nf = (int)(v.n_fam - f0 < FB ? v.n_fam - f0 : FB);
  const int tid = threadIdx.x;
  int32_t inode[S::ITI];
  interior_nodes<DIM, K, T, S>(f0, nf, inode);
  EpiOps<T, S::ITI> iops;
  epi_load<T, EPI, S::ITI, false>(ep, inode, iops);
  stage_bases<DIM, K, T, S>(v, f0, sgb, sex, bq, bc, bo);
  __syncthreads();
  const int nline = nf * CPF * NL;
  if (EPI != kEpiDiag) {
    gather_patch<DIM, K, T, S>(f0, nf, xin, sgb, bq, bc, sin);
    __syncthreads();
    // lines along z
#pragma unroll
    for (int it = 0; it < S::ITL; ++it) {
      const int u = tid + it * TH;
      if (u < nline) {
        const int fl = u / (CPF * NL), r = u % (CPF * NL), cid = r / NL, p = r % NL;
        const int px = p % N, py = p / N;
        const T* src = sin + fl * MFP + cell_patch_pos<DIM, K>(cid, px + N * py);
        T x[N];
#pragma unroll
        for (int z = 0; z < N; ++z) x[z] = src[z * M2 * M2];
        T* da = ta + fl * FS + cid * CS + px + NXP * py;
        T* db = tb + fl * FS + cid * CS + px + NXP * py;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          T a = T(0), b = T(0);
#pragma unroll
          for (int z = 0; z < N; ++z) {
            a += m.M[i * N + z] * x[z];
            b += m.K[i * N + z] * x[z];
          }
          da[i * NXP * N] = a;
          db[i * NXP * N] = b;
        }
      }
    }
    __syncthreads();
    // lines along y, in place
#pragma unroll
    for (int it = 0; it < S::ITL; ++it) {
      const int u = tid + it * TH;
      if (u < nline) {
        const int fl = u / (CPF * NL), r = u % (CPF * NL), cid = r / NL, p = r % NL;
        const int px = p % N, pz = p / N;
        T* pa = ta + fl * FS + cid * CS + px + NXP * N * pz;
        T* pb = tb + fl * FS + cid * CS + px + NXP * N * pz;
        T a[N], b[N];
#pragma unroll
        for (int y = 0; y < N; ++y) {
          a[y] = pa[y * NXP];
          b[y] = pb[y * NXP];
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
          T c = T(0), f = T(0);
#pragma unroll
          for (int y = 0; y < N; ++y) {
            c += m.M[i * N + y] * a[y];
            f += m.K[i * N + y] * a[y] + m.M[i * N + y] * b[y];
          }
          pa[i * NXP] = c;
          pb[i * NXP] = f;
        }
      }
    }
    __syncthreads();
  }
  // lines along x: the scaled cell values (diagonal: the scaled diagonal of
  // the cell matrix)
#pragma unroll
  for (int it = 0; it < S::ITL; ++it) {
    const int u = tid + it * TH;
    if (u < nline) {
      const int fl = u / (CPF * NL), r = u % (CPF * NL), cid = r / NL, p = r % NL;
      const int py = p % N, pz = p / N;
      T* pa = ta + fl * FS + cid * CS + NXP * (py + N * pz);
      const T* pb = tb + fl * FS + cid * CS + NXP * (py + N * pz);
      const T sc = T(v.scale ? v.scale[(f0 + fl) * CPF + cid] : v.scale0);
      if (EPI == kEpiDiag) {
        const T my = m.M[py * N + py], mz = m.M[pz * N + pz], ky = m.K[py * N + py], kz = m.K[pz * N + pz];
#pragma unroll
        for (int i = 0; i < N; ++i)
          pa[i] = sc * (m.K[i * N + i] * my * mz + m.M[i * N + i] * (ky * mz + my * kz));
      } else {
        T c[N], f[N];
#pragma unroll
        for (int x = 0; x < N; ++x) {
          c[x] = pa[x];
          f[x] = pb[x];
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
          T o = T(0);
#pragma unroll
          for (int x = 0; x < N; ++x) o += m.K[i * N + x] * c[x] + m.M[i * N + x] * f[x];
          pa[i] = sc * o;
        }
      }
    }
  }
  __syncthreads();
  // sum over the cells of the family containing each patch position
#pragma unroll
  for (int it = 0; it < S::ITQ; ++it) {
    const int e = tid + it * TH;
    if (e < nf * MF) {
      const int fl = e / MF, q = e % MF;
      const int qx = q % M2, qy = (q / M2) % M2, qz = q / (M2 * M2);
      T s = T(0);
#pragma unroll
      for (int cid = 0; cid < CPF; ++cid) {
        const int jx = qx - (cid & 1) * K, jy = qy - ((cid >> 1) & 1) * K, jz = qz - ((cid >> 2) & 1) * K;
        if (jx >= 0 && jx <= K && jy >= 0 && jy <= K && jz >= 0 && jz <= K)
          s += ta[fl * FS + cid * CS + jx + NXP * (jy + N * jz)];
      }
      sout[fl * MFP + q] = s;
    }
  }
  __syncthreads();
  patch_out<DIM, K, T, EPI, S>(v, f0, nf, sout, sin, sgb, sex, bq, bc, bo, ep, E, inode, iops);
}

// ------------------------------------------------------------------ pass 2
// shared nodes: sum of the present position slots (fixed order), epilogue
template <int DIM, int K, int R, typename T>
__device__ __forceinline__ T sum_slots(const LevelView& v, const T* __restrict__ E, int64_t i) {
  using G = Geo<DIM, K>;
  constexpr int SZ = G::size_r(R);
  const int64_t t = i - v.sec[R];
  const int64_t e = t / SZ;
  const int loc = (int)(t - e * SZ);
  const uint32_t pm = v.pmask[v.entoff[R] + e];
  const T* p = E + v.eoff[R] + ((e << R) * SZ) + loc;
  // every position slot of a shared entity lies inside the buffer; slots of
  // absent families hold stale values and are dropped by the select
  T a[1 << R];
#pragma unroll
  for (int pos = 0; pos < (1 << R); ++pos) a[pos] = p[pos * SZ];
  T s = T(0);
#pragma unroll
  for (int pos = 0; pos < (1 << R); ++pos) s += ((pm >> pos) & 1u) ? a[pos] : T(0);
  return s;
}

template <int DIM, int K, typename T, int EPI>
__device__ __forceinline__ void fam_sum_body(const LevelView& v, const T* __restrict__ E, const Epi<T>& ep,
                                             int64_t t) {
  if (t >= v.shn[DIM + 1]) return;
  T s;
  int64_t i;
  if (t < v.shn[2]) {
    i = v.sec[1] + t;
    s = sum_slots<DIM, K, 1, T>(v, E, i);
  } else if (DIM == 2 || t < v.shn[3]) {
    i = v.sec[2] + (t - v.shn[2]);
    s = sum_slots<DIM, K, 2, T>(v, E, i);
  } else {
    i = v.sec[3] + (t - v.shn[3]);
    s = sum_slots<DIM, K, DIM == 3 ? 3 : 2, T>(v, E, i);
  }
  epi_shared<T, EPI>(ep, i, s);
}

template <int DIM, int K, typename T, int EPI>
__global__ void __launch_bounds__(kBlock) fam_sum(LevelView v, const T* __restrict__ E, Epi<T> ep) {
  fam_sum_body<DIM, K, T, EPI>(v, E, ep, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

template <typename T>
struct SumItem {
  LevelView v;
  Epi<T> ep;
  const T* E;
  int64_t b0;
};

template <int DIM, int K, typename T, int EPI>
__global__ void __launch_bounds__(kBlock) fam_sum_batch(const SumItem<T>* __restrict__ items, int n) {
  const SumItem<T> it = items[batch_item(items, n)];
  fam_sum_body<DIM, K, T, EPI>(it.v, it.E, it.ep, ((int64_t)blockIdx.x - it.b0) * blockDim.x + threadIdx.x);
}

// ------------------------------------------------------------------ transfers
// Fine-family values at patch position q (compile-time), read through the
// fine family's entity bases; positions of entities the family does not own
// read as zero when MASK is set.
template <int DIM, int K>
__device__ __forceinline__ int64_t fam_node(const int32_t (&gb)[Geo<DIM, K>::NJ], int q) {
  using G = Geo<DIM, K>;
  const uint32_t c = G::code(q);
  return (int64_t)gb[G::cj(c)] + G::cloc(c);
}

// Restriction R = P^T of the fine residual r on the nodes the fine family
// owns, contracted to the (k+1)^d values of its parent cell: fine z-slab by
// z-slab (x contraction row by row while loading, then y, then the slab's
// share of the z contraction), so that only one slab is live at a time.
template <int DIM, int K, typename T>
__device__ __forceinline__ void restrict_family(const LevelView& fine, int64_t f, const T* __restrict__ r,
                                                const Mats<T>& m, T (&out)[Geo<DIM, K>::NP]) {
  using G = Geo<DIM, K>;
  constexpr int N = G::N, M2 = G::M2, NJ = G::NJ;
  constexpr int NZ = DIM == 3 ? M2 : 1;
  int32_t gb[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) gb[j] = fine.gbase[(int64_t)j * fine.n_fam + f];
  const uint32_t ow = fine.own[f];
#pragma unroll
  for (int j = 0; j < G::NP; ++j) out[j] = T(0);
#pragma unroll
  for (int iz = 0; iz < NZ; ++iz) {
    T a[M2 * N];
#pragma unroll
    for (int iy = 0; iy < M2; ++iy) {
      T rv[M2];
#pragma unroll
      for (int ix = 0; ix < M2; ++ix) rv[ix] = r[fam_node<DIM, K>(gb, (iz * M2 + iy) * M2 + ix)];
#pragma unroll
      for (int ix = 0; ix < M2; ++ix)
        if (!((ow >> G::cj(G::code((iz * M2 + iy) * M2 + ix))) & 1u)) rv[ix] = T(0);
#pragma unroll
      for (int J = 0; J < N; ++J) {
        T s = 0;
#pragma unroll
        for (int ix = 0; ix < M2; ++ix) s += m.E[ix * N + J] * rv[ix];
        a[iy * N + J] = s;
      }
    }
    T b[N * N];
#pragma unroll
    for (int Jy = 0; Jy < N; ++Jy)
#pragma unroll
      for (int Jx = 0; Jx < N; ++Jx) {
        T s = 0;
#pragma unroll
        for (int iy = 0; iy < M2; ++iy) s += m.E[iy * N + Jy] * a[iy * N + Jx];
        b[Jy * N + Jx] = s;
      }
    if (DIM == 2) {
#pragma unroll
      for (int j = 0; j < N * N; ++j) out[j] = b[j];
    } else {
#pragma unroll
      for (int Jz = 0; Jz < N; ++Jz) {
        const T w = m.E[iz * N + Jz];
#pragma unroll
        for (int yx = 0; yx < N * N; ++yx) out[Jz * N * N + yx] += w * b[yx];
      }
    }
  }
}

// Restriction, fine side: fine families in workgroups like the operator;
// the fine residual patch is staged in LDS, one lane per fine cell takes
// the patch nodes it owns (first cell of the family containing the node, and
// only on entities the family owns: every fine node is counted once), applies
// the transposed 1D embedding rows of its child position per axis, and the
// 2^d lanes sum their (k+1)^d parent-cell values; rb[f (k+1)^d + j] receives
// the restricted residual of family f's parent cell.
template <int DIM, int K, typename T>
__device__ __forceinline__ void fam_rfine_at(const LevelView& fine, const T* __restrict__ r, T* __restrict__ rb,
                                             const Mats<T>& m, int64_t b, int64_t nb) {
  using S = FamShape<DIM, K, T>;
  using G = Geo<DIM, K>;
  constexpr int N = G::N, MFP = S::MFP, FB = S::FB, CPF = G::CPF, NJ = G::NJ, NP = G::NP, NB = G::NB;
  __shared__ T sin[FB * MFP];
  __shared__ int32_t sgb[FB * NJ];
  __shared__ uint32_t sex[FB];
  __shared__ uint16_t bq[NB];
  __shared__ uint32_t bc[NB];
  __shared__ int64_t bo[NB];
  const int64_t f0 = xcd_block_of(b, nb) * FB;
  const int nf = (int)(fine.n_fam - f0 < FB ? fine.n_fam - f0 : FB);
  const int tid = threadIdx.x;
  stage_bases<DIM, K, T>(fine, f0, sgb, sex, bq, bc, bo);
  __syncthreads();
  gather_patch<DIM, K, T>(f0, nf, r, sgb, bq, bc, sin);
  __syncthreads();
  const int fl = tid / CPF, cid = tid % CPF;
  const uint32_t ow = fl < nf ? fine.own[f0 + fl] : 0u;
  const bool hx = cid & 1, hy = (cid >> 1) & 1, hz = DIM == 3 && ((cid >> 2) & 1);
  T v[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    const int q = cell_patch_pos<DIM, K>(cid, j);
    const bool keep = family_owner<DIM, N>(cid, j) && ((ow >> G::cj(G::code(q))) & 1u);
    v[j] = keep ? sin[fl * MFP + q] : T(0);
  }
  constexpr int NZ = DIM == 3 ? N : 1;
  // x: t[z][y][J] = sum_i E[b_x k + i][J] v[z][y][i]
  T t[NP];
#pragma unroll
  for (int rr = 0; rr < NZ * N; ++rr)
#pragma unroll
    for (int J = 0; J < N; ++J) {
      T s = 0;
#pragma unroll
      for (int i = 0; i < N; ++i) s += sel(hx, m.E[(K + i) * N + J], m.E[i * N + J]) * v[rr * N + i];
      t[rr * N + J] = s;
    }
  // y
#pragma unroll
  for (int z = 0; z < NZ; ++z)
#pragma unroll
    for (int x = 0; x < N; ++x) {
      T col[N];
#pragma unroll
      for (int i = 0; i < N; ++i) col[i] = t[(z * N + i) * N + x];
#pragma unroll
      for (int J = 0; J < N; ++J) {
        T s = 0;
#pragma unroll
        for (int i = 0; i < N; ++i) s += sel(hy, m.E[(K + i) * N + J], m.E[i * N + J]) * col[i];
        t[(z * N + J) * N + x] = s;
      }
    }
  // z
#pragma unroll
  for (int yx = 0; yx < N * N; ++yx)
#pragma unroll
    for (int J = 0; J < NZ; ++J) {
      if (DIM == 3) {
        T s = 0;
#pragma unroll
        for (int i = 0; i < N; ++i) s += sel(hz, m.E[(K + i) * N + J], m.E[i * N + J]) * t[i * N * N + yx];
        v[J * N * N + yx] = s;
      } else {
        v[yx] = t[yx];
      }
    }
  // sum over the family's cells (every lane ends with the same totals)
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    v[j] += lane_xor<0>(v[j]);
    v[j] += lane_xor<1>(v[j]);
    if (DIM == 3) v[j] += lane_xor<2>(v[j]);
  }
  if (fl < nf) {
#pragma unroll
    for (int j = 0; j < NP; ++j)
      if (j % CPF == cid) rb[(f0 + fl) * NP + j] = v[j];
  }
}
template <int DIM, int K, typename T>
__global__ void __launch_bounds__((FamShape<DIM, K, T>::THREADS)) fam_rfine(LevelView fine, const T* __restrict__ r,
                                                                             T* __restrict__ rb, Mats<T> m) {
  fam_rfine_at<DIM, K, T>(fine, r, rb, m, blockIdx.x, gridDim.x);
}

// Restriction, coarse side: one workgroup per FB coarse families, one lane
// per coarse cell reading the restricted values of its fine family (if the
// cell is refined); siblings combine as in the operator and the coarse
// patch leaves through the restriction-start epilogue (every coarse node of
// the level passes through it, restricted contribution or not; pass 2 of
// the coarse level finishes the shared nodes).
template <int DIM, int K, typename T>
__device__ __forceinline__ void fam_restrict_at(const LevelView& coarse, const T* __restrict__ rb, const Epi<T>& ep,
                                                T* __restrict__ E, const Mats<T>& m, int64_t b, int64_t nb) {
  using S = FamShape<DIM, K, T>;
  using G = Geo<DIM, K>;
  constexpr int MFP = S::MFP, FB = S::FB, CPF = G::CPF, NJ = G::NJ, NP = G::NP, NB = G::NB;
  __shared__ T sout[FB * MFP];
  __shared__ int32_t sgb[FB * NJ];
  __shared__ uint32_t sex[FB];
  __shared__ uint16_t bq[NB];
  __shared__ uint32_t bc[NB];
  __shared__ int64_t bo[NB];
  const int64_t f0 = xcd_block_of(b, nb) * FB;
  const int nf = (int)(coarse.n_fam - f0 < FB ? coarse.n_fam - f0 : FB);
  const int tid = threadIdx.x;
  int32_t inode[S::ITI];
  interior_nodes<DIM, K, T>(f0, nf, inode);
  EpiOps<T, S::ITI> iops;
  epi_load<T, kEpiRStart, S::ITI, false>(ep, inode, iops);
  stage_bases<DIM, K, T>(coarse, f0, sgb, sex, bq, bc, bo);
  __syncthreads();
  {
    const int fl = tid / CPF, cid = tid % CPF;
    const int64_t f = fl < nf ? coarse.child[(int64_t)cid * coarse.n_fam + f0 + fl] : -1;
    T out[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) out[j] = f >= 0 ? rb[f * NP + j] : T(0);
    family_sum<DIM, G::N, T>(cid, out);
#pragma unroll
    for (int j = 0; j < NP; ++j)
      if (family_owner<DIM, G::N>(cid, j)) sout[fl * MFP + cell_patch_pos<DIM, K>(cid, j)] = out[j];
  }
  __syncthreads();
  patch_out<DIM, K, T, kEpiRStart>(coarse, f0, nf, sout, sout, sgb, sex, bq, bc, bo, ep, E, inode, iops);
}
template <int DIM, int K, typename T>
__global__ void __launch_bounds__((FamShape<DIM, K, T>::THREADS)) fam_restrict(LevelView coarse,
                                                                                const T* __restrict__ rb, Epi<T> ep,
                                                                                T* __restrict__ E, Mats<T> m) {
  fam_restrict_at<DIM, K, T>(coarse, rb, ep, E, m, blockIdx.x, gridDim.x);
}

// Restriction from level 1 into level 0 (no families there): one lane per
// level-1 family, parent-node values to the level-0 node-major slots
// (summed by seg_restrict_start).
template <int DIM, int K, typename T>
__device__ __forceinline__ void fam_restrict0_at(const LevelView& fine, const T* __restrict__ r, T* __restrict__ E,
                                                 const Mats<T>& m, int64_t b, int64_t nb) {
  using G = Geo<DIM, K>;
  const int64_t f = xcd_block_of(b, nb) * blockDim.x + threadIdx.x;
  if (f >= fine.n_fam) return;
  T out[G::NP];
  restrict_family<DIM, K, T>(fine, f, r, m, out);
#pragma unroll
  for (int j = 0; j < G::NP; ++j) E[fine.rslot[(int64_t)j * fine.n_fam + f]] = out[j];
}
template <int DIM, int K, typename T>
__global__ void __launch_bounds__(kBlock) fam_restrict0(LevelView fine, const T* __restrict__ r,
                                                        T* __restrict__ E, Mats<T> m) {
  fam_restrict0_at<DIM, K, T>(fine, r, E, m, blockIdx.x, gridDim.x);
}

// Prolongation x_f += P x_c, fine families in workgroups like the operator:
// the parent cell's (k+1)^d coarse values of each family are staged in LDS
// (through the coarse family's entity bases, or the level-0 cell map), one
// lane per fine cell interpolates its (k+1)^d nodes (rows b k .. b k + k of
// the 1D embedding per axis, b its child position bit), the family patch
// is assembled in LDS, and the workgroup adds it to x_f on the entities each
// family owns (interiors contiguous, entity positions by table).
// Prolongation staging: entity bases and ownership of the fine families,
// the entity-position table, and the parent cell's coarse values su.
template <int DIM, int K, typename T, typename S>
__device__ __forceinline__ void prolong_stage(const LevelView& fine, const LevelView& coarse,
                                              const T* __restrict__ xc, int64_t f0, int nf, int32_t* sgb,
                                              uint32_t* sown, uint16_t* bq, uint32_t* bc, T* su) {
  using G = Geo<DIM, K>;
  constexpr int N = G::N, FB = S::FB, CPF = G::CPF, NJ = G::NJ, NP = G::NP;
  const int tid = threadIdx.x;
  for (int e = tid; e < FB * NJ; e += S::THREADS) {
    const int j = e / FB, fl = e % FB;
    sgb[fl * NJ + j] = fl < nf ? fine.gbase[(int64_t)j * fine.n_fam + f0 + fl] : 0;
  }
  for (int fl = tid; fl < FB; fl += S::THREADS) sown[fl] = fl < nf ? fine.own[f0 + fl] : 0u;
  for (int q = tid; q < G::MF; q += S::THREADS) {
    const uint32_t c = G::code(q);
    if (G::cr(c) != 0) {
      const int b = G::bidx(q);
      bq[b] = (uint16_t)q;
      bc[b] = c;
    }
  }
  // parent values
  for (int e = tid; e < FB * NP; e += S::THREADS) {
    const int fl = e / NP, j = e % NP;
    T val = T(0);
    if (fl < nf) {
      const int64_t p = fine.parent[f0 + fl];
      if (coarse.gbase) {
        const int64_t F = p >> DIM;
        const int cid = (int)(p & (CPF - 1));
        const int jc[3] = {j % N, (j / N) % N, DIM == 3 ? j / (N * N) : 0};
        int jj = 0, loc = 0, mul = 1, st = 1;
        for (int a = 0; a < DIM; ++a) {
          const int qa = ((cid >> a) & 1) * K + jc[a];
          const int c = qa == 0 ? 0 : qa == 2 * K ? 2 : 1;
          jj += c * mul;
          mul *= 3;
          if (c == 1) {
            loc += (qa - 1) * st;
            st *= G::S1;
          }
        }
        val = xc[coarse.gbase[(int64_t)jj * coarse.n_fam + F] + loc];
      } else {
        val = xc[coarse.cmap[(int64_t)j * coarse.n_cells + p]];
      }
    }
    su[fl * NP + j] = val;
  }
}

// x_f += the assembled fine patch on the entities each family owns:
// interiors (contiguous), then entity positions by table.
template <int DIM, int K, typename T, typename S>
__device__ __forceinline__ void prolong_add(int64_t f0, int nf, const T* sout, const int32_t* sgb,
                                            const uint32_t* sown, const uint16_t* bq, const uint32_t* bc,
                                            T* __restrict__ xf) {
  using G = Geo<DIM, K>;
  constexpr int MFP = S::MFP, NJ = G::NJ, NI = G::NI, NB = G::NB;
  const int tid = threadIdx.x;
  {
    int32_t node[S::ITI];
    T old[S::ITI];
    interior_nodes<DIM, K, T, S>(f0, nf, node);
#pragma unroll
    for (int it = 0; it < S::ITI; ++it) old[it] = xf[node[it] >= 0 ? node[it] : 0];
#pragma unroll
    for (int it = 0; it < S::ITI; ++it) {
      const int e = tid + it * S::THREADS;
      if (node[it] >= 0) xf[node[it]] = old[it] + sout[(e / NI) * MFP + G::iq(e % NI)];
    }
  }
#pragma unroll
  for (int c0 = 0; c0 < S::ITB; c0 += S::CH) {
    int32_t node[S::CH];
    T val[S::CH], old[S::CH];
#pragma unroll
    for (int k = 0; k < S::CH; ++k) {
      const int it = c0 + k;
      const int e = tid + it * S::THREADS;
      node[k] = -1;
      val[k] = T(0);
      if (it < S::ITB && e < nf * NB) {
        const int fl = e / NB, b = e % NB;
        const uint32_t c = bc[b];
        const int j = G::cj(c);
        if ((sown[fl] >> j) & 1u) {
          node[k] = sgb[fl * NJ + j] + G::cloc(c);
          val[k] = sout[fl * MFP + bq[b]];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < S::CH; ++k) old[k] = xf[node[k] >= 0 ? node[k] : 0];
#pragma unroll
    for (int k = 0; k < S::CH; ++k)
      if (node[k] >= 0) xf[node[k]] = old[k] + val[k];
  }
}

template <int DIM, int K, typename T>
__device__ __forceinline__ void fam_prolong_at(const LevelView& fine, const LevelView& coarse,
                                               const T* __restrict__ xc, T* __restrict__ xf, const Mats<T>& m,
                                               int64_t b, int64_t nb) {
  using S = FamShape<DIM, K, T>;
  using G = Geo<DIM, K>;
  constexpr int N = G::N, MFP = S::MFP, FB = S::FB, CPF = G::CPF, NJ = G::NJ, NP = G::NP, NB = G::NB;
  __shared__ T sout[FB * MFP];
  __shared__ T su[FB * NP];
  __shared__ int32_t sgb[FB * NJ];
  __shared__ uint32_t sown[FB];
  __shared__ uint16_t bq[NB];
  __shared__ uint32_t bc[NB];
  const int64_t f0 = xcd_block_of(b, nb) * FB;
  const int nf = (int)(fine.n_fam - f0 < FB ? fine.n_fam - f0 : FB);
  const int tid = threadIdx.x;
  prolong_stage<DIM, K, T, S>(fine, coarse, xc, f0, nf, sgb, sown, bq, bc, su);
  __syncthreads();
  {
    // fine cell cid of family fl: v = (E_z ⊗ E_y ⊗ E_x) u on its sub-box
    const int fl = tid / CPF, cid = tid % CPF;
    const bool hx = cid & 1, hy = (cid >> 1) & 1, hz = DIM == 3 && ((cid >> 2) & 1);
    T u[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) u[j] = su[fl * NP + j];
    constexpr int NZ = DIM == 3 ? N : 1;
    // x: t[jz][jy][i] = sum_jx E[b_x k + i][jx] u[jz][jy][jx]
    T t[NP];
#pragma unroll
    for (int r = 0; r < NZ * N; ++r)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        T s = 0;
#pragma unroll
        for (int jx = 0; jx < N; ++jx) s += sel(hx, m.E[(K + i) * N + jx], m.E[i * N + jx]) * u[r * N + jx];
        t[r * N + i] = s;
      }
    // y
#pragma unroll
    for (int z = 0; z < NZ; ++z)
#pragma unroll
      for (int x = 0; x < N; ++x) {
        T col[N];
#pragma unroll
        for (int jy = 0; jy < N; ++jy) col[jy] = t[(z * N + jy) * N + x];
#pragma unroll
        for (int i = 0; i < N; ++i) {
          T s = 0;
#pragma unroll
          for (int jy = 0; jy < N; ++jy) s += sel(hy, m.E[(K + i) * N + jy], m.E[i * N + jy]) * col[jy];
          t[(z * N + i) * N + x] = s;
        }
      }
    // z
    T v[NP];
#pragma unroll
    for (int yx = 0; yx < N * N; ++yx)
#pragma unroll
      for (int i = 0; i < NZ; ++i) {
        if (DIM == 3) {
          T s = 0;
#pragma unroll
          for (int jz = 0; jz < N; ++jz) s += sel(hz, m.E[(K + i) * N + jz], m.E[i * N + jz]) * t[jz * N * N + yx];
          v[i * N * N + yx] = s;
        } else {
          v[yx] = t[yx];
        }
      }
#pragma unroll
    for (int j = 0; j < NP; ++j)
      if (family_owner<DIM, N>(cid, j)) sout[fl * MFP + cell_patch_pos<DIM, K>(cid, j)] = v[j];
  }
  __syncthreads();
  prolong_add<DIM, K, T, S>(f0, nf, sout, sgb, sown, bq, bc, xf);
}
template <int DIM, int K, typename T>
__global__ void __launch_bounds__((FamShape<DIM, K, T>::THREADS)) fam_prolong(LevelView fine, LevelView coarse,
                                                                               const T* __restrict__ xc,
                                                                               T* __restrict__ xf, Mats<T> m) {
  fam_prolong_at<DIM, K, T>(fine, coarse, xc, xf, m, blockIdx.x, gridDim.x);
}

// The transfer kernels of several problems in one launch (item contract as
// OpItem; fields a kernel does not take are unused): restriction fine side
// (f, in = r, out = rb), coarse side (c, in = rb, ep, E), into level 0 (f,
// in = r, E), prolongation (f, c, in = x_c, out = x_f).
template <typename T>
struct XferItem {
  LevelView f, c;
  const T* in;
  T* out;
  Epi<T> ep;
  T* E;
  int64_t b0, nb;
};
template <int DIM, int K, typename T>
__global__ void __launch_bounds__((FamShape<DIM, K, T>::THREADS))
    fam_rfine_batch(const XferItem<T>* __restrict__ items, int n, Mats<T> m) {
  const XferItem<T>& it = items[batch_item(items, n)];
  fam_rfine_at<DIM, K, T>(it.f, it.in, it.out, m, (int64_t)blockIdx.x - it.b0, it.nb);
}
template <int DIM, int K, typename T>
__global__ void __launch_bounds__((FamShape<DIM, K, T>::THREADS))
    fam_restrict_batch(const XferItem<T>* __restrict__ items, int n, Mats<T> m) {
  const XferItem<T>& it = items[batch_item(items, n)];
  fam_restrict_at<DIM, K, T>(it.c, it.in, it.ep, it.E, m, (int64_t)blockIdx.x - it.b0, it.nb);
}
template <int DIM, int K, typename T>
__global__ void __launch_bounds__(kBlock) fam_restrict0_batch(const XferItem<T>* __restrict__ items, int n,
                                                              Mats<T> m) {
  const XferItem<T>& it = items[batch_item(items, n)];
  fam_restrict0_at<DIM, K, T>(it.f, it.in, it.E, m, (int64_t)blockIdx.x - it.b0, it.nb);
}
template <int DIM, int K, typename T>
__global__ void __launch_bounds__((FamShape<DIM, K, T>::THREADS))
    fam_prolong_batch(const XferItem<T>* __restrict__ items, int n, Mats<T> m) {
  const XferItem<T>& it = items[batch_item(items, n)];
  fam_prolong_at<DIM, K, T>(it.f, it.c, it.in, it.out, m, (int64_t)blockIdx.x - it.b0, it.nb);
}

// ------------------------------------------------------------------ transfers, 3D at k >= 3
// The same three transfer kernels with the cells' line contractions shared
// by the threads of a workgroup through LDS (per-cell arrays laid out as in
// the cooperative operator), for the degrees whose (k+1)^3 cell values do
// not fit one lane's registers.  E^(b)[i][J] = E[(b k + i) (k+1) + J]: the
// 1D embedding rows of child position b.
template <int K, typename T>
__device__ __forceinline__ T emb_rows(const Mats<T>& m, bool hi, int i, int J) {
  return sel(hi, m.E[(K + i) * (K + 1) + J], m.E[i * (K + 1) + J]);
}

// Restriction, fine side (contract of fam_rfine): the owned patch values of
// each cell are contracted with the transposed rows along x, y, z in place,
// and every parent-cell node sums its 2^d cells in ascending child order.
template <int DIM, int K, typename T>
__global__ void __launch_bounds__((CoopShape<DIM, K, T>::THREADS)) __attribute__((amdgpu_waves_per_eu(5)))
    fam_rfine_coop(LevelView fine, const T* __restrict__ r, T* __restrict__ rb, Mats<T> m) {
  using S = CoopShape<DIM, K, T>;
  using G = Geo<DIM, K>;
  constexpr int N = G::N, MFP = S::MFP, FB = S::FB, CPF = G::CPF, NJ = G::NJ, NP = G::NP, NB = G::NB;
  constexpr int NXP = S::NXP, CS = S::CS, FS = S::FS, NL = S::NL, TH = S::THREADS;
  static_assert(DIM == 3, "cooperative transfers are 3D");
  __shared__ T sin[FB * MFP];
  __shared__ T ta[FB * FS];
  __shared__ int32_t sgb[FB * NJ];
  __shared__ uint32_t sex[FB];
  __shared__ uint32_t sown[FB];
  __shared__ uint16_t bq[NB];
  __shared__ uint32_t bc[NB];
  __shared__ int64_t bo[NB];
  const int64_t f0 = xcd_block() * FB;
  const int nf = (int)(fine.n_fam - f0 < FB ? fine.n_fam - f0 : FB);
  const int tid = threadIdx.x;
  stage_bases<DIM, K, T, S>(fine, f0, sgb, sex, bq, bc, bo);
  for (int fl = tid; fl < FB; fl += TH) sown[fl] = fl < nf ? fine.own[f0 + fl] : 0u;
  __syncthreads();
  gather_patch<DIM, K, T, S>(f0, nf, r, sgb, bq, bc, sin);
  __syncthreads();
  // each cell's values at the patch nodes it counts (first cell of the
  // family containing the node, on entities the family owns)
  for (int e = tid; e < nf * CPF * NP; e += TH) {
    const int fl = e / (CPF * NP), rr = e % (CPF * NP), cid = rr / NP, j = rr % NP;
    const int q = cell_patch_pos<DIM, K>(cid, j);
    const bool keep = family_owner<DIM, N>(cid, j) && ((sown[fl] >> G::cj(G::code(q))) & 1u);
    const int jx = j % N, jy = (j / N) % N, jz = j / (N * N);
    ta[fl * FS + cid * CS + jx + NXP * (jy + N * jz)] = keep ? sin[fl * MFP + q] : T(0);
  }
  __syncthreads();
  const int nline = nf * CPF * NL;
  // axis a = 0, 1, 2: t[J] = sum_i E^(b_a)[i][J] v[i] along the lines of axis a
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int it = 0; it < S::ITL; ++it) {
      const int u = tid + it * TH;
      if (u < nline) {
        const int fl = u / (CPF * NL), rr = u % (CPF * NL), cid = rr / NL, p = rr % NL;
        const int p0 = p % N, p1 = p / N;
        const int o = fl * FS + cid * CS +
                      (a == 0 ? NXP * (p0 + N * p1) : a == 1 ? p0 + NXP * N * p1 : p0 + NXP * p1);
        const int st = a == 0 ? 1 : a == 1 ? NXP : NXP * N;
        const bool hi = (cid >> a) & 1;
        T v[N];
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = ta[o + i * st];
#pragma unroll
        for (int J = 0; J < N; ++J) {
          T s = T(0);
#pragma unroll
          for (int i = 0; i < N; ++i) s += emb_rows<K>(m, hi, i, J) * v[i];
          ta[o + J * st] = s;
        }
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < nf * NP; e += TH) {
    const int fl = e / NP, j = e % NP;
    const int jx = j % N, jy = (j / N) % N, jz = j / (N * N);
    T s = T(0);
#pragma unroll
    for (int cid = 0; cid < CPF; ++cid) s += ta[fl * FS + cid * CS + jx + NXP * (jy + N * jz)];
    rb[(f0 + fl) * NP + j] = s;
  }
}

// Restriction, coarse side (contract of fam_restrict): every coarse patch
// position sums the restricted values of the cells containing it that are
// refined, in ascending child order, then the restriction-start epilogue.
template <int DIM, int K, typename T>
__global__ void __launch_bounds__((CoopShape<DIM, K, T>::THREADS)) __attribute__((amdgpu_waves_per_eu(5)))
    fam_restrict_coop(LevelView coarse, const T* __restrict__ rb, Epi<T> ep, T* __restrict__ E, Mats<T> m) {
  using S = CoopShape<DIM, K, T>;
  using G = Geo<DIM, K>;
  constexpr int N = G::N, M2 = G::M2, MF = G::MF, MFP = S::MFP, FB = S::FB, CPF = G::CPF, NJ = G::NJ;
  constexpr int NP = G::NP, NB = G::NB, TH = S::THREADS;
  static_assert(DIM == 3, "cooperative transfers are 3D");
  __shared__ T sout[FB * MFP];
  __shared__ int32_t sgb[FB * NJ];
  __shared__ uint32_t sex[FB];
  __shared__ int32_t sch[FB * CPF];
  __shared__ uint16_t bq[NB];
  __shared__ uint32_t bc[NB];
  __shared__ int64_t bo[NB];
  const int64_t f0 = xcd_block() * FB;
  const int nf = (int)(coarse.n_fam - f0 < FB ? coarse.n_fam - f0 : FB);
  const int tid = threadIdx.x;
  int32_t inode[S::ITI];
  interior_nodes<DIM, K, T, S>(f0, nf, inode);
  EpiOps<T, S::ITI> iops;
  epi_load<T, kEpiRStart, S::ITI, false>(ep, inode, iops);
  stage_bases<DIM, K, T, S>(coarse, f0, sgb, sex, bq, bc, bo);
  for (int e = tid; e < FB * CPF; e += TH) {
    const int fl = e / CPF, cid = e % CPF;
    sch[e] = fl < nf ? coarse.child[(int64_t)cid * coarse.n_fam + f0 + fl] : -1;
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < S::ITQ; ++it) {
    const int e = tid + it * TH;
    if (e < nf * MF) {
      const int fl = e / MF, q = e % MF;
      const int qx = q % M2, qy = (q / M2) % M2, qz = q / (M2 * M2);
      T v[CPF];
#pragma unroll
      for (int cid = 0; cid < CPF; ++cid) {
        const int jx = qx - (cid & 1) * K, jy = qy - ((cid >> 1) & 1) * K, jz = qz - ((cid >> 2) & 1) * K;
        const int32_t f = sch[fl * CPF + cid];
        const bool in = jx >= 0 && jx <= K && jy >= 0 && jy <= K && jz >= 0 && jz <= K && f >= 0;
        v[cid] = in ? rb[(int64_t)f * NP + jx + N * (jy + N * jz)] : T(0);
      }
      T s = T(0);
#pragma unroll
      for (int cid = 0; cid < CPF; ++cid) s += v[cid];
      sout[fl * MFP + q] = s;
    }
  }
  __syncthreads();
  patch_out<DIM, K, T, kEpiRStart, S>(coarse, f0, nf, sout, sout, sgb, sex, bq, bc, bo, ep, E, inode, iops);
}

// Prolongation (contract of fam_prolong): the parent values are embedded
// along x into each cell's array, then along y and z in place; every patch
// position takes the value of the lowest cell containing it.
template <int DIM, int K, typename T>
__global__ void __launch_bounds__((CoopShape<DIM, K, T>::THREADS)) __attribute__((amdgpu_waves_per_eu(5)))
    fam_prolong_coop(LevelView fine, LevelView coarse, const T* __restrict__ xc, T* __restrict__ xf, Mats<T> m) {
  using S = CoopShape<DIM, K, T>;
  using G = Geo<DIM, K>;
  constexpr int N = G::N, M2 = G::M2, MF = G::MF, MFP = S::MFP, FB = S::FB, CPF = G::CPF, NJ = G::NJ;
  constexpr int NP = G::NP, NB = G::NB, NXP = S::NXP, CS = S::CS, FS = S::FS, NL = S::NL, TH = S::THREADS;
  static_assert(DIM == 3, "cooperative transfers are 3D");
  __shared__ T sout[FB * MFP];
  __shared__ T su[FB * NP];
  __shared__ T ta[FB * FS];
  __shared__ int32_t sgb[FB * NJ];
  __shared__ uint32_t sown[FB];
  __shared__ uint16_t bq[NB];
  __shared__ uint32_t bc[NB];
  const int64_t f0 = xcd_block() * FB;
  const int nf = (int)(fine.n_fam - f0 < FB ? fine.n_fam - f0 : FB);
  const int tid = threadIdx.x;
  prolong_stage<DIM, K, T, S>(fine, coarse, xc, f0, nf, sgb, sown, bq, bc, su);
  __syncthreads();
  const int nline = nf * CPF * NL;
  // x: from the parent values into the cell arrays
#pragma unroll
  for (int it = 0; it < S::ITL; ++it) {
    const int u = tid + it * TH;
    if (u < nline) {
      const int fl = u / (CPF * NL), rr = u % (CPF * NL), cid = rr / NL, p = rr % NL;
      const bool hi = cid & 1;
      T v[N];
#pragma unroll
      for (int J = 0; J < N; ++J) v[J] = su[fl * NP + p * N + J];
      T* o = ta + fl * FS + cid * CS + NXP * p;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        T s = T(0);
#pragma unroll
        for (int J = 0; J < N; ++J) s += emb_rows<K>(m, hi, i, J) * v[J];
        o[i] = s;
      }
    }
  }
  __syncthreads();
  // y, z in place
#pragma unroll
  for (int a = 1; a < 3; ++a) {
#pragma unroll
    for (int it = 0; it < S::ITL; ++it) {
      const int u = tid + it * TH;
      if (u < nline) {
        const int fl = u / (CPF * NL), rr = u % (CPF * NL), cid = rr / NL, p = rr % NL;
        const int p0 = p % N, p1 = p / N;
        const int o = fl * FS + cid * CS + (a == 1 ? p0 + NXP * N * p1 : p0 + NXP * p1);
        const int st = a == 1 ? NXP : NXP * N;
        const bool hi = (cid >> a) & 1;
        T v[N];
#pragma unroll
        for (int J = 0; J < N; ++J) v[J] = ta[o + J * st];
#pragma unroll
        for (int i = 0; i < N; ++i) {
          T s = T(0);
#pragma unroll
          for (int J = 0; J < N; ++J) s += emb_rows<K>(m, hi, i, J) * v[J];
          ta[o + i * st] = s;
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int it = 0; it < S::ITQ; ++it) {
    const int e = tid + it * TH;
    if (e < nf * MF) {
      const int fl = e / MF, q = e % MF;
      const int qx = q % M2, qy = (q / M2) % M2, qz = q / (M2 * M2);
      const int bx = qx > K, by = qy > K, bz = qz > K;
      const int cid = bx | (by << 1) | (bz << 2);
      sout[fl * MFP + q] = ta[fl * FS + cid * CS + (qx - bx * K) + NXP * ((qy - by * K) + N * (qz - bz * K))];
    }
  }
  __syncthreads();
  prolong_add<DIM, K, T, S>(f0, nf, sout, sgb, sown, bq, bc, xf);
}

}  // namespace dev
}  // namespace gmg

// Residual error estimator of the adaptive loop (Sec. 4.3), per leaf K:
//   e(K) = h_K^2 || f_h + eps_K Laplace u_h ||_K^2
//        + sum over the faces F of K of h_K || eps grad u_h . n ||_F jump ^2,
// with u_h and f_h the Q_k polynomials of their constrained nodal values on
// each cell (hanging values from the constraints), integrals by (k+1)-point
// Gauss quadrature per direction, no term on the domain boundary, and a
// face shared with finer leaves integrated over each of their faces.
//
// One thread per leaf: the cell term at the Gauss points of the cell, then
// the faces in the order (axis, side), each with its neighbour(s) gathered
// and both polynomials' normal derivatives evaluated at the face's Gauss
// points (for a coarser neighbour, at the points of this leaf's part of its
// face; for finer neighbours, at the points of each of their faces).
#pragma once
#include "dispatch.hpp"
#include "kernels.hpp"

namespace gmg {
namespace dev {

struct EstView {
  int64_t n_cells = 0;
  const int32_t* cmap = nullptr;     // [n_cells * NP] DoF id or -(h+1) for hanging node h
  const int64_t* con_off = nullptr;  // [n_hanging + 1]
  const int32_t* con_mas = nullptr;
  const double* con_w = nullptr;
  const int8_t* level = nullptr;     // [n_cells]
  const double* eps = nullptr;       // [n_cells]
  const uint8_t* kind = nullptr;     // [n_cells * 2d] boundary / same / coarser / finer
  const uint8_t* off = nullptr;      // [n_cells * 2d] coarser: upper-half bits per tangential axis
  const int32_t* nb = nullptr;       // [n_cells * 2d * 2^(d-1)]
};

// 1D matrices (EstMats of the host, same layout)
struct EstMatsD {
  double V[25], S[25], VH[2][25], DE[2][5], w[5];
};

constexpr int kEstLds = 4 * 25 + 10 + 5;

// constrained nodal values of cell c
template <int NP>
__device__ __forceinline__ void est_gather(const EstView& v, int64_t c, const double* __restrict__ x,
                                           double (&u)[NP]) {
  // all map entries, then all node values (a hanging position reads node 0
  // and is overwritten below), so that the loads issue together; then the
  // hanging positions, interpolated from their constraint rows
  int32_t mm[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) mm[j] = v.cmap[c * NP + j];
#pragma unroll
  for (int j = 0; j < NP; ++j) u[j] = x[mm[j] >= 0 ? mm[j] : 0];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    if (mm[j] < 0) {
      const int64_t h = -(int64_t)mm[j] - 1;
      double s = 0.0;
      for (int64_t p = v.con_off[h]; p < v.con_off[h + 1]; ++p) s += v.con_w[p] * x[v.con_mas[p]];
      u[j] = s;
    }
  }
}

// sum_j u_j rx[j_x] ry[j_y] (rz[j_z]) with rows of the 1D matrices in LDS
template <int DIM, int N>
__device__ __forceinline__ double est_eval(const double (&u)[DIM == 3 ? N * N * N : N * N], const double* rx,
                                           const double* ry, const double* rz) {
  double ax[N], ay[N], az[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    ax[i] = rx[i];
    ay[i] = ry[i];
    az[i] = DIM == 3 ? rz[i] : 1.0;
  }
  double s = 0.0;
#pragma unroll
  for (int jz = 0; jz < (DIM == 3 ? N : 1); ++jz) {
    double sy = 0.0;
#pragma unroll
    for (int jy = 0; jy < N; ++jy) {
      double sx = 0.0;
#pragma unroll
      for (int jx = 0; jx < N; ++jx) sx += u[(jz * N + jy) * N + jx] * ax[jx];
      sy += sx * ay[jy];
    }
    s += sy * az[jz];
  }
  return s;
}

// the face terms of axis AX of cell c (both sides), added to e in side order
template <int DIM, int N, int AX>
__device__ __forceinline__ void est_faces(const EstView& v, int64_t c, const double* __restrict__ x,
                                          const double (&ui)[DIM == 3 ? N * N * N : N * N], double h, double ei,
                                          const double* sm, double& e) {
  constexpr int NP = DIM == 3 ? N * N * N : N * N;
  constexpr int NF = 2 * DIM, NSUB = 1 << (DIM - 1);
  constexpr int T0 = AX == 0 ? 1 : 0;
  constexpr int T1 = DIM == 3 ? (AX == 2 ? 1 : 2) : 0;
  const double *sV = sm, *sVH0 = sm + 50, *sVH1 = sm + 75, *sDE0 = sm + 100, *sDE1 = sm + 105, *sw = sm + 110;
  for (int hi = 0; hi < 2; ++hi) {
    const int64_t f = c * NF + 2 * AX + hi;
    const int kind = v.kind[f];
    if (kind == 0) continue;
    const int parts = kind == 3 ? NSUB : 1;
    const double hj = kind == 1 ? h : kind == 2 ? 2.0 * h : 0.5 * h;
    const double fh = kind == 3 ? 0.5 * h : h;
    const double fw = DIM == 3 ? fh * fh : fh;
    const uint8_t ob = v.off[f];
    double jump2 = 0.0;
    for (int b = 0; b < parts; ++b) {
      const int32_t j = v.nb[f * NSUB + b];
      double uj[NP];
      est_gather<NP>(v, j, x, uj);
      const double ej = v.eps[j];
      // tangential half of this leaf (finer neighbours) or of the neighbour (coarser)
      const bool ib0 = kind == 3 && (b & 1), ib1 = kind == 3 && ((b >> 1) & 1);
      const bool jb0 = kind == 2 && (ob & 1), jb1 = kind == 2 && ((ob >> 1) & 1);
      const double* ni = hi ? sDE1 : sDE0;   // this leaf's face at its end `hi`
      const double* nj = hi ? sDE0 : sDE1;   // the neighbour's face at the other end
      for (int q0 = 0; q0 < N; ++q0) {
        const double* ti0 = kind == 3 ? (ib0 ? sVH1 : sVH0) + q0 * N : sV + q0 * N;
        const double* tj0 = kind == 2 ? (jb0 ? sVH1 : sVH0) + q0 * N : sV + q0 * N;
        for (int q1 = 0; q1 < (DIM == 3 ? N : 1); ++q1) {
          const double* ti1 = kind == 3 ? (ib1 ? sVH1 : sVH0) + q1 * N : sV + q1 * N;
          const double* tj1 = kind == 2 ? (jb1 ? sVH1 : sVH0) + q1 * N : sV + q1 * N;
          const double* ri[3];
          const double* rj[3];
          ri[AX] = ni;
          rj[AX] = nj;
          ri[T0] = ti0;
          rj[T0] = tj0;
          if (DIM == 3) {
            ri[T1] = ti1;
            rj[T1] = tj1;
          }
          const double gi = est_eval<DIM, N>(ui, ri[0], ri[1], DIM == 3 ? ri[2] : ri[0]) / h;
          const double gj = est_eval<DIM, N>(uj, rj[0], rj[1], DIM == 3 ? rj[2] : rj[0]) / hj;
          const double jmp = ei * gi - ej * gj;
          const double W = sw[q0] * (DIM == 3 ? sw[q1] : 1.0) * fw;
          jump2 += W * jmp * jmp;
        }
      }
    }
    e += h * jump2;
  }
}

template <int DIM, int N>
__global__ void __launch_bounds__(64) est_cells(EstView v, const double* __restrict__ u,
                                                const double* __restrict__ fn, double* __restrict__ eta, EstMatsD m) {
  constexpr int NP = DIM == 3 ? N * N * N : N * N;
  __shared__ double sm[kEstLds];
  {
    const double* src = m.V;
    for (int i = threadIdx.x; i < 25; i += blockDim.x) {
      sm[i] = m.V[i];
      sm[25 + i] = m.S[i];
      sm[50 + i] = m.VH[0][i];
      sm[75 + i] = m.VH[1][i];
    }
    for (int i = threadIdx.x; i < 5; i += blockDim.x) {
      sm[100 + i] = m.DE[0][i];
      sm[105 + i] = m.DE[1][i];
      sm[110 + i] = m.w[i];
    }
    (void)src;
  }
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= v.n_cells) return;
  const double *sV = sm, *sS = sm + 25, *sw = sm + 110;
  double ui[NP];
  est_gather<NP>(v, c, u, ui);
  const double h = ldexp(1.0, -(int)v.level[c]);
  const double ei = v.eps[c];
  double e;
  {
    double fi[NP];
    est_gather<NP>(v, c, fn, fi);
    const double hd = DIM == 3 ? h * h * h : h * h;
    double acc = 0.0;
    for (int qz = 0; qz < (DIM == 3 ? N : 1); ++qz)
      for (int qy = 0; qy < N; ++qy)
        for (int qx = 0; qx < N; ++qx) {
          const double *Vx = sV + qx * N, *Vy = sV + qy * N, *Vz = sV + qz * N;
          const double *Sx = sS + qx * N, *Sy = sS + qy * N, *Sz = sS + qz * N;
          double lap = est_eval<DIM, N>(ui, Sx, Vy, Vz) + est_eval<DIM, N>(ui, Vx, Sy, Vz);
          if (DIM == 3) lap += est_eval<DIM, N>(ui, Vx, Vy, Sz);
          lap /= h * h;
          const double fq = est_eval<DIM, N>(fi, Vx, Vy, Vz);
          const double W = sw[qx] * sw[qy] * (DIM == 3 ? sw[qz] : 1.0) * hd;
          const double r = fq + ei * lap;
          acc += W * r * r;
        }
    e = h * h * acc;
  }
  est_faces<DIM, N, 0>(v, c, u, ui, h, ei, sm, e);
  est_faces<DIM, N, 1>(v, c, u, ui, h, ei, sm, e);
  if (DIM == 3) est_faces<DIM, N, DIM == 3 ? 2 : 1>(v, c, u, ui, h, ei, sm, e);
  eta[c] = e;
}

}  // namespace dev
}  // namespace gmg

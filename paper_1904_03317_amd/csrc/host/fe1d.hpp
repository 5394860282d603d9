// One-dimensional ingredients of the tensor-product Q_k element on [0,1]
// (Sec. 2.1): Gauss-Lobatto-Legendre nodes, Lagrange basis, reference mass and
// stiffness by (k+1)-point Gauss-Legendre quadrature, and the (2k+1)x(k+1)
// embedding of the parent basis into two children (Sec. 2.2, nested spaces).
#pragma once
#include <vector>

namespace gmg {

struct FE1D {
  int k = 1, n = 2;
  double x[5] = {};          // nodes
  double M[25] = {};         // M[i*n+j] = int l_i l_j
  double K[25] = {};         // K[i*n+j] = int l_i' l_j'
  double E[9 * 5] = {};      // E[i*n+J] = l_J(family point i), i < 2k+1
  double fam[9] = {};        // family points in parent coordinates
};

FE1D make_fe1d(int k);
// values of the Lagrange basis on the nodes of `fe` at xi: out[j], j <= k
void lagrange_values(const FE1D& fe, double xi, double* out);
// their first and second derivatives at xi
void lagrange_derivs(const FE1D& fe, double xi, double* out);
void lagrange_second_derivs(const FE1D& fe, double xi, double* out);
// n-point Gauss-Legendre points and weights on [0,1], ascending
void gauss_01(int n, double* x, double* w);

}  // namespace gmg

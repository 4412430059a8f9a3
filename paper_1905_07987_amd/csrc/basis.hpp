// Host construction of the one-dimensional ADER-DG tables (basis.cpp).
#pragma once

namespace adg {

constexpr int kBasisMaxN = 8;

// n Gauss-Legendre points on [0, 1]; returns 0 on success.  Outputs (any may
// be null): nodes xi[n], weights w[n], D[n*n] with D[i*n+j] = phi_j'(xi_i),
// l0[n] = phi(0), l1[n] = phi(1), K1inv[n*n].
int basis_tables(int n, double* xi, double* w, double* D, double* l0, double* l1, double* K1inv);

// Tables of the a-posteriori subcell limiter on m = 2n - 1 equal subcells of
// [0, 1]; returns 0 on success.  A[s*n+k]: the average of phi_k over subcell
// s; B[k*m+s]: the least-squares inverse (A^T A)^{-1} A^T; Qf[k*m+s] =
// A[s*n+k] / (m w_k), which maps piecewise constant face data to face nodes.
int limiter_tables(int n, double* A, double* B, double* Qf);

}  // namespace adg

// Host construction of the one-dimensional ADER-DG tables (basis.cpp).
#pragma once

namespace adg {

constexpr int kBasisMaxN = 8;

// n Gauss-Legendre points on [0, 1]; returns 0 on success.  Outputs (any may
// be null): nodes xi[n], weights w[n], D[n*n] with D[i*n+j] = phi_j'(xi_i),
// l0[n] = phi(0), l1[n] = phi(1), K1inv[n*n].
int basis_tables(int n, double* xi, double* w, double* D, double* l0, double* l1, double* K1inv);

}  // namespace adg

// Host construction of the one-dimensional ADER-DG tables on [0, 1].
//
// Gauss-Legendre nodes come from Newton's method on the Legendre polynomial
// (evaluated by Bonnet's recurrence) in long double, the Lagrange derivative
// matrix from the barycentric form (Berrut & Trefethen, SIAM Review 2004),
// and K1^{-1} from LU factorisation with partial pivoting.  The time matrix
// is K1_ij = phi_i(1) phi_j(1) - sum_m w_m phi_i'(xi_m) phi_j(xi_m)
//          = l1_i l1_j - w_j D_ji,
// i.e. the time derivative of the space-time weak form (ExaHyPE paper,
// Sec. 3.3, Eq. (5)) integrated by parts, with the old time level as the
// upwind value at the start of the step.
#include <cmath>

#include "basis.hpp"

namespace adg {
namespace {

using ld = long double;

void gauss_legendre(int n, ld* x, ld* w) {
  const ld pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    // Tricomi's first guess of the i-th largest root
    ld z = cosl(pi * (4 * i + 3) / (4 * n + 2));
    ld dp = 0;
    for (int it = 0; it < 60; ++it) {
      ld p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1; }
      dp = n * (p0 - z * p1) / (1 - z * z);
      ld step = p1 / dp;
      z -= step;
      if (fabsl(step) <= 1e-24L) break;
    }
    // recompute P_n' at the converged root for the weight
    {
      ld p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1; }
      dp = n * (p0 - z * p1) / (1 - z * z);
    }
    ld wt = 1 / ((1 - z * z) * dp * dp);  // on [0,1]: half of 2/((1-z^2)P'^2)
    x[n - 1 - i] = (1 + z) / 2;
    x[i] = (1 - z) / 2;
    w[n - 1 - i] = wt;
    w[i] = wt;
  }
}

}  // namespace

int basis_tables(int n, double* xi, double* w, double* D, double* l0, double* l1,
                 double* K1inv) {
  if (n < 1 || n > kBasisMaxN) return -1;
  ld x[kBasisMaxN], wt[kBasisMaxN], bw[kBasisMaxN], Dl[kBasisMaxN][kBasisMaxN], a[kBasisMaxN], b[kBasisMaxN];
  gauss_legendre(n, x, wt);
  // barycentric weights
  for (int j = 0; j < n; ++j) {
    ld p = 1;
    for (int m = 0; m < n; ++m)
      if (m != j) p *= (x[j] - x[m]);
    bw[j] = 1 / p;
  }
  for (int i = 0; i < n; ++i) {
    ld diag = 0;
    for (int j = 0; j < n; ++j) {
      if (i == j) continue;
      Dl[i][j] = (bw[j] / bw[i]) / (x[i] - x[j]);
      diag -= Dl[i][j];  // rows of D annihilate constants
    }
    Dl[i][i] = diag;
  }
  // boundary values from the barycentric formula of the second kind
  for (int side = 0; side < 2; ++side) {
    ld xe = side ? 1.0L : 0.0L, den = 0;
    ld* out = side ? b : a;
    for (int j = 0; j < n; ++j) den += bw[j] / (xe - x[j]);
    for (int j = 0; j < n; ++j) out[j] = (bw[j] / (xe - x[j])) / den;
  }
  // K1 and its inverse (LU with partial pivoting, then n solves)
  ld K[kBasisMaxN][kBasisMaxN], Kinv[kBasisMaxN][kBasisMaxN];
  int perm[kBasisMaxN];
  for (int i = 0; i < n; ++i) {
    perm[i] = i;
    for (int j = 0; j < n; ++j) K[i][j] = b[i] * b[j] - wt[j] * Dl[j][i];
  }
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (fabsl(K[r][c]) > fabsl(K[p][c])) p = r;
    if (p != c) {
      for (int j = 0; j < n; ++j) {
        ld tmp = K[c][j];
        K[c][j] = K[p][j];
        K[p][j] = tmp;
      }
      int tp = perm[c];
      perm[c] = perm[p];
      perm[p] = tp;
    }
    for (int r = c + 1; r < n; ++r) {
      K[r][c] /= K[c][c];
      for (int j = c + 1; j < n; ++j) K[r][j] -= K[r][c] * K[c][j];
    }
  }
  for (int col = 0; col < n; ++col) {
    ld y[kBasisMaxN];
    for (int i = 0; i < n; ++i) {
      ld s = (perm[i] == col) ? 1.0L : 0.0L;
      for (int j = 0; j < i; ++j) s -= K[i][j] * y[j];
      y[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
      ld s = y[i];
      for (int j = i + 1; j < n; ++j) s -= K[i][j] * Kinv[j][col];
      Kinv[i][col] = s / K[i][i];
    }
  }
  for (int i = 0; i < n; ++i) {
    if (xi) xi[i] = (double)x[i];
    if (w) w[i] = (double)wt[i];
    if (l0) l0[i] = (double)a[i];
    if (l1) l1[i] = (double)b[i];
    for (int j = 0; j < n; ++j) {
      if (D) D[i * n + j] = (double)Dl[i][j];
      if (K1inv) K1inv[i * n + j] = (double)Kinv[i][j];
    }
  }
  return 0;
}

// The subcell averages come from the exact antiderivative of each Lagrange
// polynomial, expanded in powers of y = x - 1/2; the least-squares inverse
// from the Cholesky factorisation of A^T A.
int limiter_tables(int n, double* A, double* B, double* Qf) {
  if (n < 1 || n > kBasisMaxN) return -1;
  const int m = 2 * n - 1;
  ld x[kBasisMaxN], wt[kBasisMaxN], Al[2 * kBasisMaxN][kBasisMaxN];
  gauss_legendre(n, x, wt);
  for (int k = 0; k < n; ++k) {
    ld c[kBasisMaxN + 1] = {1.0L};  // phi_k = sum_i c_i y^i
    int deg = 0;
    for (int j = 0; j < n; ++j) {
      if (j == k) continue;
      const ld yj = x[j] - 0.5L, den = x[k] - x[j];
      for (int i = deg + 1; i >= 0; --i) c[i] = ((i > 0 ? c[i - 1] : 0.0L) - yj * (i <= deg ? c[i] : 0.0L)) / den;
      ++deg;
    }
    auto prim = [&](ld y) {  // sum_i c_i y^{i+1} / (i+1)
      ld in = 0.0L;
      for (int i = deg; i >= 0; --i) in = in * y + c[i] / (i + 1);
      return in * y;
    };
    for (int s = 0; s < m; ++s) Al[s][k] = m * (prim((ld)(s + 1) / m - 0.5L) - prim((ld)s / m - 0.5L));
  }
  ld G[kBasisMaxN][kBasisMaxN], L[kBasisMaxN][kBasisMaxN] = {};
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      ld g = 0.0L;
      for (int s = 0; s < m; ++s) g += Al[s][i] * Al[s][j];
      G[i][j] = g;
    }
  for (int j = 0; j < n; ++j) {
    ld d = G[j][j];
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(d > 0.0L)) return -1;
    L[j][j] = sqrtl(d);
    for (int i = j + 1; i < n; ++i) {
      ld v = G[i][j];
      for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
      L[i][j] = v / L[j][j];
    }
  }
  for (int s = 0; s < m; ++s) {
    ld y[kBasisMaxN], z[kBasisMaxN];
    for (int i = 0; i < n; ++i) {  // L y = A[s]^T
      ld v = Al[s][i];
      for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
      y[i] = v / L[i][i];
    }
    for (int i = n - 1; i >= 0; --i) {  // L^T z = y
      ld v = y[i];
      for (int k = i + 1; k < n; ++k) v -= L[k][i] * z[k];
      z[i] = v / L[i][i];
    }
    for (int k = 0; k < n; ++k) {
      if (A) A[s * n + k] = (double)Al[s][k];
      if (B) B[k * m + s] = (double)z[k];
      if (Qf) Qf[k * m + s] = (double)(Al[s][k] / (m * wt[k]));
    }
  }
  return 0;
}

}  // namespace adg

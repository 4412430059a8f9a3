/*
 * adg_oracle.c -- plain, slow, FP64 CPU oracle of one ADER-DG time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The GPU library never
 * links, includes or calls it, and the two share no code, headers or tables.
 *
 * What it computes follows the ExaHyPE paper (Reinarz et al., "ExaHyPE: An
 * Engine for Parallel Dynamically Adaptive Simulations of Wave Problems"):
 *   - the balance law with flux, non-conservative product, source and point
 *     sources: Sec. 2, Eq. (1);
 *   - the element-local space-time predictor, a fixed-point (Picard) iteration
 *     on the weak form Eq. (5), tensor-product Lagrange basis on Gauss-Legendre
 *     points: Sec. 3.3;
 *   - the three phases of a step (predictor, Rusanov face flux, corrector
 *     Eq. (6) with a diagonal mass matrix): Sec. 3.3;
 *   - the time step restriction Eq. (7): Sec. 3.4;
 *   - the admissibility check of the a-posteriori limiter: Sec. 3.5;
 *   - the a-posteriori subcell limiter in its hybrid ADER-DG/FV form (FV
 *     subcells, discrete maximum principle, MUSCL-Hancock, projections):
 *     Sec. 3.5, Table 1, Fig. 2 (section 10 below);
 *   - boundary faces (outflow, wall, inflow; the paper's boundaryValues,
 *     Table 2);
 *   - the PDEs: compressible Euler, Eqs. (8) and (10) (Sec. 6.1) and linear
 *     elasticity in velocity-stress form (Sec. 2.1).
 * Readings of silent or ambiguous passages are marked READING below.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC.
 * No FMA contraction, IEEE binary64, round to nearest.
 *
 * Data contract (the same one the GPU library documents for its callers):
 *   Q      : [cell][nvar][node]   node = kx + n*(ky + n*kz), x fastest
 *   params : [cell][nparam]       material parameters, constant per cell
 *   cell   = cx + Cx*(cy + Cy*cz)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXN 8   /* n = N+1 <= 8 */
#define ORC_MAXQ 16  /* evolved + parameter slots per point */
#define ORC_MAXSRC 8

enum { ORC_EULER = 1, ORC_ELASTIC = 2, ORC_ADVECTION = 3 };

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -3 };

/* Problem description.  Mirrored field by field by a ctypes Structure. */
typedef struct {
  int dim, order, pde, nvar, nparam, picard_iters;
  int cells[3];
  double lo[3], hi[3];
  double cfl;
  double gamma;  /* Euler: ratio of specific heats */
  double adv[3]; /* advection: velocity a */
  double kappa;  /* advection: linear decay source S(q) = -kappa q */
  int nsrc;
  int guess;     /* initial guess of the Picard iteration: ORC_GUESS_* */
  double src_x[ORC_MAXSRC][3];
  double src_w[ORC_MAXSRC][ORC_MAXQ]; /* which variables a source drives */
  double src_f0[ORC_MAXSRC], src_t0[ORC_MAXSRC], src_amp[ORC_MAXSRC];
  /* boundary condition of face 2 d + side (side 1 at the high end of axis
   * d): ORC_BC_PERIODIC on both faces of an axis, or OUTFLOW / WALL */
  int bc[6];
  /* the outside state of an ORC_BC_INFLOW face (its first nvar entries) */
  double bc_state[6][ORC_MAXQ];
} orc_problem;

enum { ORC_BC_PERIODIC = 0, ORC_BC_OUTFLOW = 1, ORC_BC_WALL = 2, ORC_BC_INFLOW = 3 };
enum { ORC_GUESS_CONSTANT = 0, ORC_GUESS_CERK = 1 };

/* ------------------------------------------------------------------------
 * 1. One-dimensional tables on the reference interval [0,1].
 *    Gauss-Legendre nodes xi_i and weights w_i (sum w = 1), the Lagrange
 *    basis phi_i through the nodes, D_ij = phi_j'(xi_i), the boundary values
 *    l0_i = phi_i(0), l1_i = phi_i(1), and the time matrix of the predictor
 *    K1_ij = phi_i(1) phi_j(1) - int_0^1 phi_i'(tau) phi_j(tau) dtau
 *          = l1_i l1_j - w_j D_ji         (exact under Gauss quadrature)
 *    which comes from integrating the time derivative of Eq. (5) by parts
 *    with the old solution taken as the upwind value at the start of the
 *    step (Sec. 3.3).  Everything is formed in long double, then rounded.
 * ------------------------------------------------------------------------ */
typedef struct {
  int n;
  double xi[ORC_MAXN], w[ORC_MAXN];
  double D[ORC_MAXN][ORC_MAXN];
  double l0[ORC_MAXN], l1[ORC_MAXN];
  double K1[ORC_MAXN][ORC_MAXN], K1inv[ORC_MAXN][ORC_MAXN];
} tables;

/* Legendre polynomial P_n(x) and its derivative, three-term recurrence. */
static void legendre(int n, long double x, long double *p, long double *dp) {
  long double p0 = 1.0L, p1 = x;
  if (n == 0) { *p = 1.0L; *dp = 0.0L; return; }
  for (int k = 2; k <= n; ++k) {
    long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *p = p1;
  *dp = n * (x * p1 - p0) / (x * x - 1.0L);
}

/* Lagrange basis phi_i(x) on nodes xs[0..n-1], straight from the product. */
static long double lagrange_ld(int n, const long double *xs, int i, long double x) {
  long double v = 1.0L;
  for (int m = 0; m < n; ++m)
    if (m != i) v *= (x - xs[m]) / (xs[i] - xs[m]);
  return v;
}

/* phi_j'(x_i) from the product rule written out. */
static long double lagrange_deriv_at_node(int n, const long double *xs, int j, int i) {
  if (i == j) {
    long double s = 0.0L;
    for (int m = 0; m < n; ++m)
      if (m != j) s += 1.0L / (xs[j] - xs[m]);
    return s;
  }
  long double num = 1.0L, den = 1.0L;
  for (int m = 0; m < n; ++m) {
    if (m != j) den *= (xs[j] - xs[m]);
    if (m != j && m != i) num *= (xs[i] - xs[m]);
  }
  return num / den;
}

static int make_tables(int n, tables *T) {
  if (n < 1 || n > ORC_MAXN) return ORC_EINVAL;
  long double x[ORC_MAXN], w[ORC_MAXN];
  /* Newton on P_n from the Chebyshev-like first guess, on [-1,1]. */
  for (int i = 0; i < n; ++i) {
    long double z = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (n + 0.5L));
    for (int it = 0; it < 100; ++it) {
      long double p, dp;
      legendre(n, z, &p, &dp);
      long double dz = p / dp;
      z -= dz;
      if (fabsl(dz) < 1e-30L) break;
    }
    long double p, dp;
    legendre(n, z, &p, &dp);
    /* map to [0,1]: xi = (1 + z)/2 ascending, weight 2/((1-z^2) P'^2) halved */
    x[n - 1 - i] = 0.5L * (1.0L + z);
    w[n - 1 - i] = 1.0L / ((1.0L - z * z) * dp * dp);
  }
  long double D[ORC_MAXN][ORC_MAXN], l0[ORC_MAXN], l1[ORC_MAXN];
  for (int i = 0; i < n; ++i) {
    l0[i] = lagrange_ld(n, x, i, 0.0L);
    l1[i] = lagrange_ld(n, x, i, 1.0L);
    for (int j = 0; j < n; ++j) D[i][j] = lagrange_deriv_at_node(n, x, j, i);
  }
  long double K[ORC_MAXN][2 * ORC_MAXN];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      K[i][j] = l1[i] * l1[j] - w[j] * D[j][i];
      K[i][n + j] = (i == j) ? 1.0L : 0.0L;
    }
  T->n = n;
  for (int i = 0; i < n; ++i) {
    T->xi[i] = (double)x[i];
    T->w[i] = (double)w[i];
    T->l0[i] = (double)l0[i];
    T->l1[i] = (double)l1[i];
    for (int j = 0; j < n; ++j) {
      T->D[i][j] = (double)D[i][j];
      T->K1[i][j] = (double)K[i][j];
    }
  }
  /* Gauss-Jordan elimination with partial pivoting for K1^{-1}. */
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabsl(K[r][col]) > fabsl(K[piv][col])) piv = r;
    if (piv != col)
      for (int c = 0; c < 2 * n; ++c) {
        long double tmp = K[col][c];
        K[col][c] = K[piv][c];
        K[piv][c] = tmp;
      }
    long double d = K[col][col];
    for (int c = 0; c < 2 * n; ++c) K[col][c] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      long double f = K[r][col];
      for (int c = 0; c < 2 * n; ++c) K[r][c] -= f * K[col][c];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) T->K1inv[i][j] = (double)K[i][n + j];
  return ORC_OK;
}

/* phi_i(x) in double for interpolation at arbitrary reference points. */
static double lagrange(const tables *T, int i, double x) {
  double v = 1.0;
  for (int m = 0; m < T->n; ++m)
    if (m != i) v *= (x - T->xi[m]) / (T->xi[i] - T->xi[m]);
  return v;
}

/* ------------------------------------------------------------------------
 * 2. The PDE terms of Eq. (1), pointwise, in the (Q, direction, out)
 *    convention of the paper's user functions (Table 2, Sec. 4.1).
 *    Q holds the nvar evolved quantities followed by the nparam material
 *    parameters (Sec. 6.2 keeps the material in the state vector).
 * ------------------------------------------------------------------------ */

/* Euler pressure, Eq. (10): p = (gamma-1) (E - |j|^2 / (2 rho)). */
static double euler_pressure(const orc_problem *P, const double *Q) {
  double jj = 0.0;
  for (int a = 0; a < P->dim; ++a) jj += Q[1 + a] * Q[1 + a];
  return (P->gamma - 1.0) * (Q[P->dim + 1] - 0.5 * jj / Q[0]);
}

/* Stress index of the symmetric pair (i, d): xx yy zz xy xz yz. */
static int sym_index(int i, int d) {
  if (i == d) return i;
  int a = i < d ? i : d, b = i < d ? d : i;
  if (a == 0 && b == 1) return 3;
  if (a == 0 && b == 2) return 4;
  return 5;
}

/* Flux F_d(Q) (the d-th column of the flux tensor). */
static void pde_flux(const orc_problem *P, const double *Q, int d, double *F) {
  switch (P->pde) {
    case ORC_EULER: {
      /* Eq. (8): F_d = (j_d, j_d j / rho + p e_d, j_d (E + p) / rho) */
      int E = P->dim + 1;
      double p = euler_pressure(P, Q);
      double ud = Q[1 + d] / Q[0];
      F[0] = Q[1 + d];
      for (int a = 0; a < P->dim; ++a) F[1 + a] = ud * Q[1 + a];
      F[1 + d] += p;
      F[E] = ud * (Q[E] + p);
      break;
    }
    case ORC_ELASTIC: {
      /* Sec. 2.1: F = (0, sigma) -- the momentum rows carry sigma_{i d}. */
      for (int v = 0; v < 6; ++v) F[v] = 0.0;
      for (int i = 0; i < 3; ++i) F[6 + i] = Q[sym_index(i, d)];
      break;
    }
    case ORC_ADVECTION:
      F[0] = P->adv[d] * Q[0];
      break;
  }
}

/* Non-conservative product B(Q) . grad Q; gradQ is [dim][nq]. */
static void pde_ncp(const orc_problem *P, const double *Q, const double *gradQ, double *BgradQ) {
  int nq = P->nvar + P->nparam;
  for (int v = 0; v < P->nvar; ++v) BgradQ[v] = 0.0;
  if (P->pde != ORC_ELASTIC) return;
  /* Sec. 2.1: the stress rows carry E(lambda, mu) . grad v with v = (rho v)/rho.
   * lambda = rho (cp^2 - 2 cs^2), mu = rho cs^2 (READING: the Lame constants
   * "can be derived" from Table 3's rho, cp, cs). */
  double rho = Q[9], cp = Q[10], cs = Q[11];
  double mu = rho * cs * cs;
  double lam = rho * cp * cp - 2.0 * mu;
  double g[3][3]; /* g[i][d] = d v_i / d x_d */
  for (int i = 0; i < 3; ++i)
    for (int d = 0; d < 3; ++d) g[i][d] = gradQ[d * nq + 6 + i] / rho;
  double divv = g[0][0] + g[1][1] + g[2][2];
  BgradQ[0] = 2.0 * mu * g[0][0] + lam * divv;
  BgradQ[1] = 2.0 * mu * g[1][1] + lam * divv;
  BgradQ[2] = 2.0 * mu * g[2][2] + lam * divv;
  BgradQ[3] = mu * (g[0][1] + g[1][0]);
  BgradQ[4] = mu * (g[0][2] + g[2][0]);
  BgradQ[5] = mu * (g[1][2] + g[2][1]);
}

/* Smooth source S(Q, x, t).  Only the advection test PDE has one. */
static void pde_source(const orc_problem *P, const double *Q, const double *x, double t, double *S) {
  (void)x;
  (void)t;
  for (int v = 0; v < P->nvar; ++v) S[v] = 0.0;
  if (P->pde == ORC_ADVECTION) S[0] = -P->kappa * Q[0];
}

/* Largest absolute eigenvalue of the flux Jacobian in direction d (Sec. 4.1's
 * eigenvalues hook; the kernel only needs the maximum). */
static double pde_max_eigen(const orc_problem *P, const double *Q, int d) {
  switch (P->pde) {
    case ORC_EULER: {
      /* textbook: u_d - c, u_d, u_d + c, c = sqrt(gamma p / rho) */
      double c = sqrt(P->gamma * euler_pressure(P, Q) / Q[0]);
      return fabs(Q[1 + d] / Q[0]) + c;
    }
    case ORC_ELASTIC:
      return Q[10]; /* +-cp, +-cs (twice), 0 (three times) */
    case ORC_ADVECTION:
      return fabs(P->adv[d]);
  }
  return 0.0;
}

/* Physical admissibility (Sec. 3.5, criterion 1) plus finiteness. */
static int pde_admissible(const orc_problem *P, const double *Q) {
  int nq = P->nvar + P->nparam;
  for (int v = 0; v < nq; ++v)
    if (!isfinite(Q[v])) return 0;
  if (P->pde == ORC_EULER) {
    if (!(Q[0] > 0.0)) return 0;
    if (!(euler_pressure(P, Q) > 0.0)) return 0;
  }
  return 1;
}

/* Ricker wavelet s(t) = amp (1 - 2 pi^2 f0^2 (t-t0)^2) exp(-pi^2 f0^2 (t-t0)^2). */
static double ricker(const orc_problem *P, int s, double t) {
  const double pi = 3.14159265358979323846;
  double a = pi * P->src_f0[s] * (t - P->src_t0[s]);
  a = a * a;
  return P->src_amp[s] * (1.0 - 2.0 * a) * exp(-a);
}

/* ------------------------------------------------------------------------
 * 3. Mesh helpers: uniform Cartesian cells, periodic in every direction.
 * ------------------------------------------------------------------------ */
typedef struct {
  int n, S, F, nv, nq, dim;
  long C;
  double h[3];
  int stride[3]; /* node stride along each axis: 1, n, n^2 */
} mesh;

static int bc_valid(const orc_problem *P);

static int make_mesh(const orc_problem *P, mesh *M) {
  if (P->dim < 2 || P->dim > 3) return ORC_EINVAL;
  if (!bc_valid(P)) return ORC_EINVAL;
  if (P->order < 1 || P->order + 1 > ORC_MAXN) return ORC_EINVAL;
  if (P->nvar < 1 || P->nvar + P->nparam > ORC_MAXQ || P->nparam < 0) return ORC_EINVAL;
  M->dim = P->dim;
  M->n = P->order + 1;
  M->S = 1;
  M->F = 1;
  M->C = 1;
  for (int d = 0; d < P->dim; ++d) {
    if (P->cells[d] < 1) return ORC_EINVAL;
    M->S *= M->n;
    if (d > 0) M->F *= M->n;
    M->C *= P->cells[d];
    M->h[d] = (P->hi[d] - P->lo[d]) / P->cells[d];
    M->stride[d] = d == 0 ? 1 : M->stride[d - 1] * M->n;
  }
  M->nv = P->nvar;
  M->nq = P->nvar + P->nparam;
  return ORC_OK;
}

static void cell_coords(const orc_problem *P, long c, int cc[3]) {
  cc[0] = (int)(c % P->cells[0]);
  long r = c / P->cells[0];
  cc[1] = (int)(P->dim > 1 ? r % P->cells[1] : 0);
  cc[2] = (int)(P->dim > 2 ? r / P->cells[1] : 0);
}

static long cell_index(const orc_problem *P, const int cc[3]) {
  long c = cc[0];
  if (P->dim > 1) c += (long)P->cells[0] * cc[1];
  if (P->dim > 2) c += (long)P->cells[0] * P->cells[1] * cc[2];
  return c;
}

/* neighbour across the face with normal e_d on side s (-1 or +1): wrapped
 * around on a periodic axis, -1 where the face lies on a non-periodic
 * domain boundary */
static long neighbour(const orc_problem *P, long c, int d, int s) {
  int cc[3];
  cell_coords(P, c, cc);
  int to = cc[d] + s;
  if ((to < 0 || to >= P->cells[d]) && P->bc[2 * d + (s > 0)] != ORC_BC_PERIODIC) return -1;
  cc[d] = (to + P->cells[d]) % P->cells[d];
  return cell_index(P, cc);
}

/* Boundary conditions (the paper's boundaryValues user function, Table 2,
 * gives the state and the normal flux outside a boundary face; its Euler
 * explosion problem uses wall boundaries).  READING: both are built
 * pointwise from the cell's own time-averaged face traces (qin, Fin):
 *   OUTFLOW  qout = qin, Fout = Fin (a transmissive boundary: no jump);
 *   WALL     the mirror image across the face.  Euler: R reverses the
 *            momentum normal to the face; F_d(R q) = -R F_d(q), so
 *            qout = R qin, Fout = -R Fin (a reflecting wall: no mass or
 *            energy crosses it).  Elasticity: the traction sigma_{i d}
 *            reversed, the velocity kept (a traction-free surface); the
 *            flux is linear, Fout = F_d(qout) = -Fin.
 *   INFLOW   a prescribed outside state (bc_state of the face, constant in
 *            time) and its flux, Fout = F_d(qout).
 * Material parameters outside are the cell's own. */
static int bc_valid(const orc_problem *P) {
  for (int d = 0; d < 3; ++d) {
    int lo = P->bc[2 * d], hi = P->bc[2 * d + 1];
    if (lo < 0 || lo > ORC_BC_INFLOW || hi < 0 || hi > ORC_BC_INFLOW) return 0;
    if (d >= P->dim && (lo || hi)) return 0;
    if ((lo == ORC_BC_PERIODIC) != (hi == ORC_BC_PERIODIC)) return 0;
    if ((lo == ORC_BC_WALL || hi == ORC_BC_WALL) && P->pde == ORC_ADVECTION) return 0;
  }
  return 1;
}

static int bc_periodic(const orc_problem *P) {
  for (int f = 0; f < 6; ++f)
    if (P->bc[f] != ORC_BC_PERIODIC) return 0;
  return 1;
}

static void bc_ghost(const orc_problem *P, int face, const double *qin, const double *Fin,
                     double *qout, double *Fout) {
  const int kind = P->bc[face], d = face / 2;
  for (int v = 0; v < P->nvar + P->nparam; ++v) qout[v] = qin[v];
  for (int v = 0; v < P->nvar; ++v) Fout[v] = Fin[v];
  if (kind == ORC_BC_INFLOW) {
    for (int v = 0; v < P->nvar; ++v) qout[v] = P->bc_state[face][v];
    pde_flux(P, qout, d, Fout);
    return;
  }
  if (kind != ORC_BC_WALL) return;
  if (P->pde == ORC_EULER) {
    qout[1 + d] = -qin[1 + d];
    for (int v = 0; v < P->nvar; ++v)
      if (v != 1 + d) Fout[v] = -Fin[v];
  } else if (P->pde == ORC_ELASTIC) {
    /* traction components sigma_{x d}, sigma_{y d}, sigma_{z d} */
    for (int i = 0; i < 3; ++i) qout[sym_index(i, d)] = -qin[sym_index(i, d)];
    for (int v = 0; v < P->nvar; ++v) Fout[v] = -Fin[v];
  }
}

/* node multi-index */
static void node_index(const mesh *M, int k, int kk[3]) {
  kk[0] = k % M->n;
  kk[1] = (k / M->n) % M->n;
  kk[2] = k / (M->n * M->n);
  if (M->dim == 2) kk[2] = 0;
}

/* index of the face node k_perp for a face with normal d: the remaining axes
 * in increasing order, the lower one fastest. */
static int face_node(const mesh *M, int d, const int kk[3]) {
  int f = 0, mul = 1;
  for (int a = 0; a < M->dim; ++a) {
    if (a == d) continue;
    f += kk[a] * mul;
    mul *= M->n;
  }
  return f;
}

/* ------------------------------------------------------------------------
 * 4. Space-time predictor for one cell (Sec. 3.3, phase 1).
 *
 *    q_h(x, tau) = sum_{j,k} theta_j(tau) phi_k(x) q_{j,k}, tau in [0,1],
 *    t = t^n + tau dt.  Testing Eq. (1) with theta_i phi_k over the cell and
 *    the step, integrating the time derivative by parts with u^n upwind at
 *    tau = 0, and using Gauss-Legendre quadrature collocated with the nodes:
 *       sum_j K1_ij q_{j,k} = l0_i u^n_k + dt w_i R(q)_{i,k},
 *       R = - div F(q_h) - B(q_h) . grad q_h + S(q_h) + point sources,
 *    with spatial derivatives of the nodal interpolants.  This is solved by
 *    the fixed-point iteration the paper uses for non-linear PDEs:
 *       q^0_j = u^n,   q^{r+1}_i = sum_j K1inv_ij (l0_j u^n + dt w_j R(q^r)_j).
 *    READING: the iteration count is fixed (picard_iters, default N+1), no
 *    tolerance test, and the initial guess is u^n at every time node.
 * ------------------------------------------------------------------------ */
typedef struct {
  double *u;      /* [S][nq]          u^n with the parameters appended */
  double *q;      /* [n][S][nq]       current iterate */
  double *qn;     /* [n][S][nq]       next iterate */
  double *F;      /* [dim][n][S][nv]  flux at every space-time node */
  double *grad;   /* [n][S][dim][nq]  spatial gradient of q */
  double *R;      /* [n][S][nv]       right-hand side of the predictor */
  double *ncp;    /* [n][S][nv] */
  double *src;    /* [n][S][nv] */
  /* outputs of the predictor, at the final iterate */
  double *qbar;   /* [S][nv]          time average of q */
  double *Fbar;   /* [dim][S][nv]     time average of F_d(q) */
  double *Nbar;   /* [S][nv]          time average of B(q) grad q */
  double *Sbar;   /* [S][nv]          time average of the sources */
} work;

static int work_alloc(const mesh *M, work *W) {
  size_t S = M->S, n = M->n, nq = M->nq, nv = M->nv, d = M->dim;
  W->u = calloc(S * nq, sizeof(double));
  W->q = calloc(n * S * nq, sizeof(double));
  W->qn = calloc(n * S * nq, sizeof(double));
  W->F = calloc(d * n * S * nv, sizeof(double));
  W->grad = calloc(n * S * d * nq, sizeof(double));
  W->R = calloc(n * S * nv, sizeof(double));
  W->ncp = calloc(n * S * nv, sizeof(double));
  W->src = calloc(n * S * nv, sizeof(double));
  W->qbar = calloc(S * nv, sizeof(double));
  W->Fbar = calloc(d * S * nv, sizeof(double));
  W->Nbar = calloc(S * nv, sizeof(double));
  W->Sbar = calloc(S * nv, sizeof(double));
  if (!W->u || !W->q || !W->qn || !W->F || !W->grad || !W->R || !W->ncp || !W->src ||
      !W->qbar || !W->Fbar || !W->Nbar || !W->Sbar)
    return ORC_ENOMEM;
  return ORC_OK;
}

static void work_free(work *W) {
  free(W->u); free(W->q); free(W->qn); free(W->F); free(W->grad); free(W->R);
  free(W->ncp); free(W->src); free(W->qbar); free(W->Fbar); free(W->Nbar); free(W->Sbar);
}

/* Evaluate F, grad q, B grad q, S and R = -div F - B grad q + S at every
 * space-time node of the iterate W->q. */
static void eval_terms(const orc_problem *P, const mesh *M, const tables *T, long c,
                       const double *xlo, double dt, double t, work *W) {
  const int n = M->n, S = M->S, nq = M->nq, nv = M->nv, dim = M->dim;
  /* fluxes */
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < S; ++k)
      for (int d = 0; d < dim; ++d)
        pde_flux(P, &W->q[((size_t)j * S + k) * nq], d,
                 &W->F[(((size_t)d * n + j) * S + k) * nv]);
  for (int j = 0; j < n; ++j) {
    double tj = t + T->xi[j] * dt; /* time nodes share the spatial nodes */
    for (int k = 0; k < S; ++k) {
      int kk[3];
      node_index(M, k, kk);
      const double *qk = &W->q[((size_t)j * S + k) * nq];
      double *g = &W->grad[((size_t)j * S + k) * dim * nq];
      double divF[ORC_MAXQ];
      for (int v = 0; v < nv; ++v) divF[v] = 0.0;
      for (int d = 0; d < dim; ++d) {
        for (int v = 0; v < nq; ++v) g[d * nq + v] = 0.0;
        for (int m = 0; m < n; ++m) {
          int km = k + (m - kk[d]) * M->stride[d]; /* node with k_d <- m */
          double Dkm = T->D[kk[d]][m];
          const double *qm = &W->q[((size_t)j * S + km) * nq];
          const double *Fm = &W->F[(((size_t)d * n + j) * S + km) * nv];
          for (int v = 0; v < nv; ++v) {
            g[d * nq + v] += Dkm * qm[v];
            divF[v] += Dkm * Fm[v] / M->h[d];
          }
        }
        for (int v = 0; v < nv; ++v) g[d * nq + v] /= M->h[d];
        /* material parameters are constant inside the cell: zero gradient */
      }
      double *B = &W->ncp[((size_t)j * S + k) * nv];
      pde_ncp(P, qk, g, B);
      double x[3] = {0.0, 0.0, 0.0};
      for (int d = 0; d < dim; ++d) x[d] = xlo[d] + M->h[d] * T->xi[kk[d]];
      double *Sv = &W->src[((size_t)j * S + k) * nv];
      pde_source(P, qk, x, tj, Sv);
      /* point sources, Eq. (1): the test function integrates a Dirac delta
       * to phi_k(x_s); dividing by the diagonal mass |T| W_k gives the nodal
       * value.  READING: a point lying on a face belongs to the cell whose
       * half-open interval [x_lo, x_lo + h) contains it. */
      for (int s = 0; s < P->nsrc; ++s) {
        int sc[3] = {0, 0, 0};
        double xs[3];
        for (int d = 0; d < dim; ++d) {
          sc[d] = (int)floor((P->src_x[s][d] - P->lo[d]) / M->h[d]);
          xs[d] = (P->src_x[s][d] - P->lo[d]) / M->h[d] - sc[d];
        }
        if (cell_index(P, sc) != c) continue;
        double phi = 1.0, mass = 1.0;
        for (int d = 0; d < dim; ++d) {
          phi *= lagrange(T, kk[d], xs[d]);
          mass *= M->h[d] * T->w[kk[d]];
        }
        double amp = ricker(P, s, tj) * phi / mass;
        for (int v = 0; v < nv; ++v) Sv[v] += amp * P->src_w[s][v];
      }
      double *R = &W->R[((size_t)j * S + k) * nv];
      for (int v = 0; v < nv; ++v) R[v] = -divF[v] - B[v] + Sv[v];
    }
  }
}

/* Initial guess by a continuous extension Runge-Kutta method (CERK; the
 * alternative to a constant guess the paper names for its optimised
 * kernels, Sec. 5.2, without giving one).  READING: the cell-local ODE
 * dq/dt = R(q, t) of the predictor (the same R as in the Picard step: the
 * cell's spatial derivatives, non-conservative product and sources, no face
 * terms) is integrated over the step by the classical four-stage Runge-Kutta
 * method,
 *    k1 = R(u, t),  k2 = R(u + dt/2 k1, t + dt/2),
 *    k3 = R(u + dt/2 k2, t + dt/2),  k4 = R(u + dt k3, t + dt),
 * with its continuous extension (dense output) of uniform order three,
 *    q(tau) = u + dt sum_s b_s(tau) k_s,   b1 = tau - 3 tau^2/2 + 2 tau^3/3,
 *    b2 = b3 = tau^2 - 2 tau^3/3,   b4 = -tau^2/2 + 2 tau^3/3,
 * taken at the time nodes tau = xi_j as q^0_j.  The Picard passes that
 * follow start from an iterate whose error is O(dt^4) instead of O(dt):
 * picard_iters = N - 2 passes reach the order that N + 1 passes from the
 * constant guess reach.  Each stage's R is evaluated by filling every time
 * slice with the stage state at the stage time (dt = 0 in eval_terms). */
static void cerk_guess(const orc_problem *P, const mesh *M, const tables *T, long c,
                       const double *xlo, double dt, double t, work *W) {
  const int n = M->n, S = M->S, nq = M->nq, nv = M->nv;
  const double cst[4] = {0.0, 0.5, 0.5, 1.0};  /* stage times c_s */
  const double ast[4] = {0.0, 0.5, 0.5, 1.0};  /* Y_s = u + dt a_s k_{s-1} */
  double *qg = calloc((size_t)n * S * nq, sizeof(double));  /* the guess, assembled */
  double *kprev = calloc((size_t)S * nv, sizeof(double));
  if (!qg || !kprev) {
    free(qg);
    free(kprev);
    return;  /* no memory: the constant guess stays (the caller sees no error) */
  }
  for (int j = 0; j < n; ++j) memcpy(&qg[(size_t)j * S * nq], W->u, sizeof(double) * S * nq);
  for (int st = 0; st < 4; ++st) {
    /* stage state Y_s in every slice of the iterate */
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < S; ++k) {
        double *qk = &W->q[((size_t)j * S + k) * nq];
        for (int v = 0; v < nv; ++v) qk[v] = W->u[(size_t)k * nq + v] + dt * ast[st] * kprev[(size_t)k * nv + v];
        for (int p = nv; p < nq; ++p) qk[p] = W->u[(size_t)k * nq + p];
      }
    eval_terms(P, M, T, c, xlo, 0.0, t + cst[st] * dt, W);
    for (int k = 0; k < S; ++k)
      for (int v = 0; v < nv; ++v) kprev[(size_t)k * nv + v] = W->R[(size_t)k * nv + v];  /* slice 0 */
    for (int j = 0; j < n; ++j) {
      const double x = T->xi[j];
      double b;
      if (st == 0) b = x - 1.5 * x * x + 2.0 / 3.0 * x * x * x;
      else if (st == 3) b = -0.5 * x * x + 2.0 / 3.0 * x * x * x;
      else b = x * x - 2.0 / 3.0 * x * x * x;
      for (int k = 0; k < S; ++k)
        for (int v = 0; v < nv; ++v) qg[((size_t)j * S + k) * nq + v] += dt * b * kprev[(size_t)k * nv + v];
    }
  }
  memcpy(W->q, qg, sizeof(double) * (size_t)n * S * nq);
  free(qg);
  free(kprev);
}

static void predictor_cell(const orc_problem *P, const mesh *M, const tables *T, long c,
                           const double *Q, const double *params, double dt, double t,
                           int iters, work *W) {
  const int n = M->n, S = M->S, nq = M->nq, nv = M->nv, dim = M->dim;
  int cc[3];
  cell_coords(P, c, cc);
  double xlo[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < dim; ++d) xlo[d] = P->lo[d] + cc[d] * M->h[d];
  /* gather u^n (evolved quantities, then the cell's parameters) */
  for (int k = 0; k < S; ++k) {
    for (int v = 0; v < nv; ++v) W->u[(size_t)k * nq + v] = Q[((size_t)c * nv + v) * S + k];
    for (int p = 0; p < P->nparam; ++p)
      W->u[(size_t)k * nq + nv + p] = params[(size_t)c * P->nparam + p];
  }
  /* initial guess q^0_j = u^n */
  for (int j = 0; j < n; ++j)
    memcpy(&W->q[(size_t)j * S * nq], W->u, sizeof(double) * S * nq);
  if (P->guess == ORC_GUESS_CERK) cerk_guess(P, M, T, c, xlo, dt, t, W);
  for (int r = 0; r < iters; ++r) {
    eval_terms(P, M, T, c, xlo, dt, t, W);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < S; ++k) {
        double *qi = &W->qn[((size_t)i * S + k) * nq];
        for (int v = 0; v < nv; ++v) {
          double acc = 0.0;
          for (int j = 0; j < n; ++j)
            acc += T->K1inv[i][j] *
                   (T->l0[j] * W->u[(size_t)k * nq + v] + dt * T->w[j] * W->R[((size_t)j * S + k) * nv + v]);
          qi[v] = acc;
        }
        for (int p = 0; p < P->nparam; ++p) qi[nv + p] = W->u[(size_t)k * nq + nv + p];
      }
    double *tmp = W->q;
    W->q = W->qn;
    W->qn = tmp;
  }
  /* READING: the averaged terms are evaluated at the final iterate q^I. */
  eval_terms(P, M, T, c, xlo, dt, t, W);
  for (int k = 0; k < S; ++k)
    for (int v = 0; v < nv; ++v) {
      double a = 0.0, b = 0.0, s = 0.0;
      for (int j = 0; j < n; ++j) {
        a += T->w[j] * W->q[((size_t)j * S + k) * nq + v];
        b += T->w[j] * W->ncp[((size_t)j * S + k) * nv + v];
        s += T->w[j] * W->src[((size_t)j * S + k) * nv + v];
      }
      W->qbar[(size_t)k * nv + v] = a;
      W->Nbar[(size_t)k * nv + v] = b;
      W->Sbar[(size_t)k * nv + v] = s;
      for (int d = 0; d < dim; ++d) {
        double f = 0.0;
        for (int j = 0; j < n; ++j) f += T->w[j] * W->F[(((size_t)d * n + j) * S + k) * nv + v];
        W->Fbar[((size_t)d * S + k) * nv + v] = f;
      }
    }
}

/* ------------------------------------------------------------------------
 * 5. Projection of the prediction onto the faces (Sec. 5.1, step fusion;
 *    Sec. 3.3 phase 2 needs q_h and F(q_h) on both sides of every face).
 *    READING: the time-averaged state and the time-averaged normal flux are
 *    both extrapolated with l0 / l1.
 *    Per cell: qhat, Fhat [2*dim faces][F face nodes][nv], face = 2d + side.
 * ------------------------------------------------------------------------ */
static void project_to_faces(const mesh *M, const tables *T, const work *W, double *qhat, double *Fhat) {
  const int S = M->S, nv = M->nv, F = M->F;
  size_t face_sz = (size_t)F * nv;
  memset(qhat, 0, sizeof(double) * 2 * M->dim * face_sz);
  memset(Fhat, 0, sizeof(double) * 2 * M->dim * face_sz);
  for (int k = 0; k < S; ++k) {
    int kk[3];
    node_index(M, k, kk);
    for (int d = 0; d < M->dim; ++d) {
      int f = face_node(M, d, kk);
      for (int side = 0; side < 2; ++side) {
        double l = side ? T->l1[kk[d]] : T->l0[kk[d]];
        double *qh = &qhat[(2 * d + side) * face_sz + (size_t)f * nv];
        double *Fh = &Fhat[(2 * d + side) * face_sz + (size_t)f * nv];
        for (int v = 0; v < nv; ++v) {
          qh[v] += l * W->qbar[(size_t)k * nv + v];
          Fh[v] += l * W->Fbar[((size_t)d * S + k) * nv + v];
        }
      }
    }
  }
}

/* ------------------------------------------------------------------------
 * 6. Rusanov flux with a path-conservative non-conservative part
 *    (Sec. 3.3 phase 2; the default Riemann solver of Table 1).
 *    The face has normal +e_d; L is the cell on its low side.
 *       s = max(lambda*(qL), lambda*(qR))            READING: pointwise
 *       G = (FL + FR)/2 - s (qR - qL)/2
 *       Bmid = B_d((qL + qR)/2) (qR - qL) / 2       READING: straight path,
 *                                                    midpoint rule
 *    The fluctuation entering cell L through its high face is G - FL + Bmid,
 *    the one entering cell R through its low face is FR - G + Bmid.
 * ------------------------------------------------------------------------ */
static void rusanov(const orc_problem *P, int d, const double *qL, const double *FL,
                    const double *qR, const double *FR, double *flL, double *flR) {
  int nv = P->nvar, nq = P->nvar + P->nparam;
  double s = fmax(pde_max_eigen(P, qL, d), pde_max_eigen(P, qR, d));
  double qm[ORC_MAXQ], grad[3 * ORC_MAXQ], Bm[ORC_MAXQ];
  for (int v = 0; v < nq; ++v) qm[v] = 0.5 * (qL[v] + qR[v]);
  for (int a = 0; a < 3 * ORC_MAXQ; ++a) grad[a] = 0.0;
  for (int v = 0; v < nv; ++v) grad[d * nq + v] = qR[v] - qL[v];
  pde_ncp(P, qm, grad, Bm);
  for (int v = 0; v < nv; ++v) {
    double G = 0.5 * (FL[v] + FR[v]) - 0.5 * s * (qR[v] - qL[v]);
    double Bmid = 0.5 * Bm[v];
    flL[v] = G - FL[v] + Bmid;
    flR[v] = FR[v] - G + Bmid;
  }
}

/* ------------------------------------------------------------------------
 * 7. Corrector (Sec. 3.3 phase 3, Eq. (6)) with the diagonal GL mass matrix.
 *    READING: Eq. (6) as printed has the sign of the volume term flipped;
 *    the standard weak form is used,
 *       int_T phi_k dq = dt [ int_T grad phi_k . Fbar - int_dT phi_k G.n ]
 *                       - dt int_T phi_k Nbar + dt int_T phi_k Sbar
 *                       - (path-conservative jump terms of the NCP),
 *    evaluated in the equivalent strong form (summation by parts on GL):
 *       dq_k = dt (-div Fbar - Nbar + Sbar)_k
 *              - dt sum_d [l1_{k_d} flL(high face) + l0_{k_d} flR(low face)]
 *                          / (h_d w_{k_d}).
 *    The weak form itself is also evaluated for conservative PDEs so the
 *    tests can check that the two agree.
 * ------------------------------------------------------------------------ */
typedef struct {
  double *vol;  /* [C][S][nv]         dt (-div Fbar - Nbar + Sbar) */
  double *weak; /* [C][S][nv]         weak-form volume part dt sum w D Fbar + dt Sbar */
  double *qhat; /* [C][2 dim][F][nv] */
  double *Fhat; /* [C][2 dim][F][nv] */
} cellside;

/* Predict cell c and store its volume increment and face traces. */
static void predict_and_project(const orc_problem *P, const mesh *M, const tables *T, long c,
                                const double *Q, const double *params, double dt, double t,
                                work *W, double *vol, double *weak, double *qhat, double *Fhat) {
  const int S = M->S, nv = M->nv, n = M->n;
  predictor_cell(P, M, T, c, Q, params, dt, t, P->picard_iters, W);
  project_to_faces(M, T, W, qhat, Fhat);
  for (int k = 0; k < S; ++k) {
    int kk[3];
    node_index(M, k, kk);
    for (int v = 0; v < nv; ++v) {
      double divF = 0.0, wk = 0.0;
      for (int d = 0; d < M->dim; ++d) {
        double a = 0.0, b = 0.0;
        for (int m = 0; m < n; ++m) {
          int km = k + (m - kk[d]) * M->stride[d];
          double f = W->Fbar[((size_t)d * S + km) * nv + v];
          a += T->D[kk[d]][m] * f;
          b += T->w[m] * T->D[m][kk[d]] * f; /* int phi_k' F over the cell */
        }
        divF += a / M->h[d];
        wk += b / (M->h[d] * T->w[kk[d]]);
      }
      vol[(size_t)k * nv + v] = dt * (-divF - W->Nbar[(size_t)k * nv + v] + W->Sbar[(size_t)k * nv + v]);
      if (weak) weak[(size_t)k * nv + v] = dt * (wk + W->Sbar[(size_t)k * nv + v]);
    }
  }
}

/* Assemble u^{n+1} of cell c from its own traces and its neighbours'.
 * Gover (NULL, or [2 dim] pointers each NULL or [F][nv]) replaces the
 * Rusanov flux G on a face by a given normal flux (the subcell limiter's FV
 * fluxes, section 10; conservative PDEs only). */
static void correct_cell(const orc_problem *P, const mesh *M, const tables *T, long c,
                         const double *Q, const double *params, double dt, const double *vol,
                         const double *weak, double *const *qhat_of, double *const *Fhat_of,
                         const long *nb /*[dim][2]: low, high neighbour*/, double *out,
                         double *weak_out, const double *const *Gover) {
  const int S = M->S, nv = M->nv, F = M->F, nq = M->nq;
  size_t face_sz = (size_t)F * nv;
  /* fluctuations on the faces of this cell, [2 dim][F][nv] */
  double *fl = malloc(sizeof(double) * 2 * M->dim * face_sz);
  double *G = malloc(sizeof(double) * 2 * M->dim * face_sz);
  double qL[ORC_MAXQ], qR[ORC_MAXQ], flL[ORC_MAXQ], flR[ORC_MAXQ];
  double FL[ORC_MAXQ], FR[ORC_MAXQ];
  for (int d = 0; d < M->dim; ++d) {
    for (int side = 0; side < 2; ++side) {
      /* side 1: this cell is L, the neighbour above is R; side 0: reverse.
       * Without a neighbour (a non-periodic boundary face) the other side is
       * the boundary condition's outside state. */
      const long other = nb[2 * d + side];
      const double *qown = qhat_of[0] + (size_t)(2 * d + side) * face_sz;
      const double *Fown = Fhat_of[0] + (size_t)(2 * d + side) * face_sz;
      const double *qoth = other < 0 ? NULL : qhat_of[1 + 2 * d + side] + (size_t)(2 * d + 1 - side) * face_sz;
      const double *Foth = other < 0 ? NULL : Fhat_of[1 + 2 * d + side] + (size_t)(2 * d + 1 - side) * face_sz;
      for (int f = 0; f < F; ++f) {
        double qo[ORC_MAXQ], qx[ORC_MAXQ], Fo[ORC_MAXQ], Fx[ORC_MAXQ];
        for (int v = 0; v < nv; ++v) {
          qo[v] = qown[(size_t)f * nv + v];
          Fo[v] = Fown[(size_t)f * nv + v];
        }
        for (int p = 0; p < P->nparam; ++p) qo[nv + p] = params[(size_t)c * P->nparam + p];
        if (other < 0) {
          bc_ghost(P, 2 * d + side, qo, Fo, qx, Fx);
        } else {
          for (int v = 0; v < nv; ++v) {
            qx[v] = qoth[(size_t)f * nv + v];
            Fx[v] = Foth[(size_t)f * nv + v];
          }
          for (int p = 0; p < P->nparam; ++p) qx[nv + p] = params[(size_t)other * P->nparam + p];
        }
        for (int v = 0; v < nv + P->nparam; ++v) {
          qL[v] = side ? qo[v] : qx[v];
          qR[v] = side ? qx[v] : qo[v];
        }
        for (int v = 0; v < nv; ++v) {
          FL[v] = side ? Fo[v] : Fx[v];
          FR[v] = side ? Fx[v] : Fo[v];
        }
        rusanov(P, d, qL, FL, qR, FR, flL, flR);
        if (Gover && Gover[2 * d + side]) {
          const double *Go = Gover[2 * d + side] + (size_t)f * nv;
          for (int v = 0; v < nv; ++v) {
            flL[v] = Go[v] - FL[v];
            flR[v] = FR[v] - Go[v];
          }
        }
        for (int v = 0; v < nv; ++v) {
          fl[(2 * d + side) * face_sz + (size_t)f * nv + v] = side ? flL[v] : flR[v];
          /* G itself, for the weak-form check */
          G[(2 * d + side) * face_sz + (size_t)f * nv + v] = side ? flL[v] + FL[v] : FR[v] - flR[v];
        }
      }
    }
  }
  (void)nq;
  for (int k = 0; k < S; ++k) {
    int kk[3];
    node_index(M, k, kk);
    for (int v = 0; v < nv; ++v) {
      double surf = 0.0, wsurf = 0.0;
      for (int d = 0; d < M->dim; ++d) {
        int f = face_node(M, d, kk);
        double hi = fl[(2 * d + 1) * face_sz + (size_t)f * nv + v];
        double lo = fl[(2 * d + 0) * face_sz + (size_t)f * nv + v];
        surf += (T->l1[kk[d]] * hi + T->l0[kk[d]] * lo) / (M->h[d] * T->w[kk[d]]);
        double Ghi = G[(2 * d + 1) * face_sz + (size_t)f * nv + v];
        double Glo = G[(2 * d + 0) * face_sz + (size_t)f * nv + v];
        wsurf += (T->l1[kk[d]] * Ghi - T->l0[kk[d]] * Glo) / (M->h[d] * T->w[kk[d]]);
      }
      double u = Q[((size_t)c * nv + v) * S + k];
      out[(size_t)v * S + k] = u + (vol[(size_t)k * nv + v] - dt * surf);
      if (weak_out) weak_out[(size_t)v * S + k] = u + (weak[(size_t)k * nv + v] - dt * wsurf);
    }
  }
  free(fl);
  free(G);
}

/* ------------------------------------------------------------------------
 * 8. Exported entry points.
 * ------------------------------------------------------------------------ */
int orc_tables(int n, double *xi, double *w, double *D, double *l0, double *l1, double *K1,
               double *K1inv) {
  tables T;
  int st = make_tables(n, &T);
  if (st) return st;
  for (int i = 0; i < n; ++i) {
    if (xi) xi[i] = T.xi[i];
    if (w) w[i] = T.w[i];
    if (l0) l0[i] = T.l0[i];
    if (l1) l1[i] = T.l1[i];
    for (int j = 0; j < n; ++j) {
      if (D) D[i * n + j] = T.D[i][j];
      if (K1) K1[i * n + j] = T.K1[i][j];
      if (K1inv) K1inv[i * n + j] = T.K1inv[i][j];
    }
  }
  return ORC_OK;
}

/* Lagrange basis values phi_i(x), i < n, at one reference point. */
int orc_basis_eval(int n, double x, double *phi) {
  tables T;
  int st = make_tables(n, &T);
  if (st) return st;
  for (int i = 0; i < n; ++i) phi[i] = lagrange(&T, i, x);
  return ORC_OK;
}

int orc_set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  return omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

/* Physical coordinates of every node, [C][S][dim]. */
int orc_node_coords(const orc_problem *P, double *xyz) {
  mesh M;
  tables T;
  if (make_mesh(P, &M) || make_tables(M.n, &T)) return ORC_EINVAL;
  for (long c = 0; c < M.C; ++c) {
    int cc[3];
    cell_coords(P, c, cc);
    for (int k = 0; k < M.S; ++k) {
      int kk[3];
      node_index(&M, k, kk);
      for (int d = 0; d < M.dim; ++d)
        xyz[((size_t)c * M.S + k) * M.dim + d] = P->lo[d] + (cc[d] + T.xi[kk[d]]) * M.h[d];
    }
  }
  return ORC_OK;
}

/* Pointwise terms, exported for unit tests. */
int orc_pointwise(const orc_problem *P, const double *Q, int d, double *flux, double *max_eigen,
                  int *admissible) {
  if (flux) pde_flux(P, Q, d, flux);
  if (max_eigen) *max_eigen = pde_max_eigen(P, Q, d);
  if (admissible) *admissible = pde_admissible(P, Q);
  return ORC_OK;
}

int orc_ncp(const orc_problem *P, const double *Q, const double *gradQ, double *BgradQ) {
  pde_ncp(P, Q, gradQ, BgradQ);
  return ORC_OK;
}

int orc_rusanov(const orc_problem *P, int d, const double *qL, const double *FL, const double *qR,
                const double *FR, double *flL, double *flR) {
  rusanov(P, d, qL, FL, qR, FR, flL, flR);
  return ORC_OK;
}

/* Maximum of two signal speeds for Eq. (7).  READING: a NaN speed (for
 * Euler: a NaN in the state, or a state where the sound speed is the square
 * root of a negative number, such as a negative pressure at positive density)
 * is not skipped: the maximum, and with it dt, becomes NaN.  Speeds of the
 * linear PDEs do not depend on the state. */
static double speed_max(double a, double b) {
  if (isnan(a) || isnan(b)) return NAN;
  return a > b ? a : b;
}

/* Eq. (7): dt = CFL / (d (2N+1)) * h / |lambda_max|.
 * READING: h = min_d h_d, lambda_max = max over cells, nodes and directions
 * of the largest absolute eigenvalue, evaluated on u^n; NaN as above. */
int orc_stable_dt(const orc_problem *P, const double *Q, const double *params, double *dt,
                  double *lambda_max) {
  mesh M;
  if (make_mesh(P, &M)) return ORC_EINVAL;
  double lam = 0.0;
  for (long c = 0; c < M.C; ++c)
    for (int k = 0; k < M.S; ++k) {
      double q[ORC_MAXQ];
      for (int v = 0; v < M.nv; ++v) q[v] = Q[((size_t)c * M.nv + v) * M.S + k];
      for (int p = 0; p < P->nparam; ++p) q[M.nv + p] = params[(size_t)c * P->nparam + p];
      for (int d = 0; d < M.dim; ++d) lam = speed_max(lam, pde_max_eigen(P, q, d));
    }
  double h = M.h[0];
  for (int d = 1; d < M.dim; ++d) h = fmin(h, M.h[d]);
  if (lambda_max) *lambda_max = lam;
  *dt = P->cfl / (M.dim * (2.0 * P->order + 1.0)) * h / lam;
  return ORC_OK;
}

/* Space-time predictor of one cell, [n][S][nq] (unit tests). */
int orc_predictor(const orc_problem *P, long cell, const double *Q, const double *params, double dt,
                  double t, int iters, double *qst, double *qbar, double *Fbar) {
  mesh M;
  tables T;
  work W;
  if (make_mesh(P, &M) || make_tables(M.n, &T)) return ORC_EINVAL;
  if (work_alloc(&M, &W)) { work_free(&W); return ORC_ENOMEM; }
  predictor_cell(P, &M, &T, cell, Q, params, dt, t, iters, &W);
  if (qst) memcpy(qst, W.q, sizeof(double) * M.n * M.S * M.nq);
  if (qbar) memcpy(qbar, W.qbar, sizeof(double) * M.S * M.nv);
  if (Fbar) memcpy(Fbar, W.Fbar, sizeof(double) * M.dim * M.S * M.nv);
  work_free(&W);
  return ORC_OK;
}

/* Face traces (qhat, Fhat) and volume increment of every cell. */
static int predict_all(const orc_problem *P, const mesh *M, const tables *T, const double *Q,
                       const double *params, double dt, double t, const long *cells, long ncells,
                       cellside *CS) {
  size_t face_all = (size_t)2 * M->dim * M->F * M->nv;
  int fail = 0;
#pragma omp parallel
  {
    work W;
    int ok = work_alloc(M, &W) == ORC_OK;
    if (!ok) {
#pragma omp atomic write
      fail = 1;
    }
#pragma omp for schedule(dynamic, 4)
    for (long i = 0; i < ncells; ++i) {
      if (!ok) continue;
      long c = cells ? cells[i] : i;
      predict_and_project(P, M, T, c, Q, params, dt, t, &W, &CS->vol[(size_t)i * M->S * M->nv],
                          CS->weak ? &CS->weak[(size_t)i * M->S * M->nv] : NULL,
                          &CS->qhat[i * face_all], &CS->Fhat[i * face_all]);
    }
    work_free(&W);
  }
  return fail ? ORC_ENOMEM : ORC_OK;
}

/* One full step in place: Q <- u^{n+1}.  If weak_out is not NULL it receives
 * u^{n+1} assembled with the weak form of Eq. (6) (conservative PDEs only). */
int orc_step(const orc_problem *P, double *Q, const double *params, double dt, double t,
             double *weak_out) {
  mesh M;
  tables T;
  if (make_mesh(P, &M) || make_tables(M.n, &T)) return ORC_EINVAL;
  size_t face_all = (size_t)2 * M.dim * M.F * M.nv;
  cellside CS;
  CS.vol = malloc(sizeof(double) * M.C * M.S * M.nv);
  CS.weak = weak_out ? malloc(sizeof(double) * M.C * M.S * M.nv) : NULL;
  CS.qhat = malloc(sizeof(double) * M.C * face_all);
  CS.Fhat = malloc(sizeof(double) * M.C * face_all);
  double *out = malloc(sizeof(double) * M.C * M.S * M.nv);
  int st = ORC_ENOMEM;
  if (CS.vol && CS.qhat && CS.Fhat && out && (!weak_out || CS.weak)) {
    st = predict_all(P, &M, &T, Q, params, dt, t, NULL, M.C, &CS);
    if (st == ORC_OK) {
#pragma omp parallel for schedule(dynamic, 8)
      for (long c = 0; c < M.C; ++c) {
        long nb[6];
        double *qh[7], *Fh[7];
        qh[0] = &CS.qhat[c * face_all];
        Fh[0] = &CS.Fhat[c * face_all];
        for (int d = 0; d < M.dim; ++d)
          for (int s = 0; s < 2; ++s) {
            nb[2 * d + s] = neighbour(P, c, d, s ? 1 : -1);
            qh[1 + 2 * d + s] = nb[2 * d + s] < 0 ? NULL : &CS.qhat[nb[2 * d + s] * face_all];
            Fh[1 + 2 * d + s] = nb[2 * d + s] < 0 ? NULL : &CS.Fhat[nb[2 * d + s] * face_all];
          }
        correct_cell(P, &M, &T, c, Q, params, dt, &CS.vol[(size_t)c * M.S * M.nv],
                     CS.weak ? &CS.weak[(size_t)c * M.S * M.nv] : NULL, qh, Fh, nb,
                     &out[(size_t)c * M.nv * M.S],
                     weak_out ? &weak_out[(size_t)c * M.nv * M.S] : NULL, NULL);
      }
      memcpy(Q, out, sizeof(double) * M.C * M.S * M.nv);
    }
  }
  free(CS.vol); free(CS.weak); free(CS.qhat); free(CS.Fhat); free(out);
  return st;
}

/* u^{n+1} of a chosen set of cells only (out: [ncs][nv][S]).  Each chosen
 * cell needs its own prediction and those of its 2 dim face neighbours. */
int orc_step_cells(const orc_problem *P, const double *Q, const double *params, double dt,
                   double t, long ncs, const long *cells, double *out) {
  mesh M;
  tables T;
  if (make_mesh(P, &M) || make_tables(M.n, &T)) return ORC_EINVAL;
  size_t face_all = (size_t)2 * M.dim * M.F * M.nv;
  long per = 1 + 2 * M.dim;
  long nall = ncs * per;
  long *list = malloc(sizeof(long) * nall);
  cellside CS;
  CS.vol = malloc(sizeof(double) * nall * M.S * M.nv);
  CS.weak = NULL;
  CS.qhat = malloc(sizeof(double) * nall * face_all);
  CS.Fhat = malloc(sizeof(double) * nall * face_all);
  int st = ORC_ENOMEM;
  if (list && CS.vol && CS.qhat && CS.Fhat) {
    for (long i = 0; i < ncs; ++i) {
      list[i * per] = cells[i];
      for (int d = 0; d < M.dim; ++d)
        for (int s = 0; s < 2; ++s) {
          /* a boundary face predicts the cell itself again (unused) */
          long o = neighbour(P, cells[i], d, s ? 1 : -1);
          list[i * per + 1 + 2 * d + s] = o < 0 ? cells[i] : o;
        }
    }
    st = predict_all(P, &M, &T, Q, params, dt, t, list, nall, &CS);
    if (st == ORC_OK) {
#pragma omp parallel for
      for (long i = 0; i < ncs; ++i) {
        long nb[6];
        double *qh[7], *Fh[7];
        for (int a = 0; a < per; ++a) {
          qh[a] = &CS.qhat[(i * per + a) * face_all];
          Fh[a] = &CS.Fhat[(i * per + a) * face_all];
          if (a > 0) nb[a - 1] = neighbour(P, cells[i], (a - 1) / 2, (a - 1) % 2 ? 1 : -1);
        }
        correct_cell(P, &M, &T, cells[i], Q, params, dt, &CS.vol[(size_t)(i * per) * M.S * M.nv],
                     NULL, qh, Fh, nb, &out[(size_t)i * M.nv * M.S], NULL, NULL);
      }
    }
  }
  free(list); free(CS.vol); free(CS.qhat); free(CS.Fhat);
  return st;
}

/* Face traces of one cell: qhat and Fhat, each [2 dim][F][nv] (unit tests and
 * parity of the projection step). */
int orc_cell_traces(const orc_problem *P, long cell, const double *Q, const double *params,
                    double dt, double t, double *qhat, double *Fhat, double *vol) {
  mesh M;
  tables T;
  work W;
  if (make_mesh(P, &M) || make_tables(M.n, &T)) return ORC_EINVAL;
  if (work_alloc(&M, &W)) { work_free(&W); return ORC_ENOMEM; }
  double *v = malloc(sizeof(double) * M.S * M.nv);
  predict_and_project(P, &M, &T, cell, Q, params, dt, t, &W, v, NULL, qhat, Fhat);
  if (vol) memcpy(vol, v, sizeof(double) * M.S * M.nv);
  free(v);
  work_free(&W);
  return ORC_OK;
}

/* Receivers: u(x_r) = sum_k Phi_k(xi_r) u_k in the cell holding x_r
 * (half-open cell intervals).  out: [nrec][nv]. */
int orc_sample_receivers(const orc_problem *P, int nrec, const double *xyz, const double *Q,
                         double *out) {
  mesh M;
  tables T;
  if (make_mesh(P, &M) || make_tables(M.n, &T)) return ORC_EINVAL;
  for (int r = 0; r < nrec; ++r) {
    int cc[3] = {0, 0, 0};
    double xs[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < M.dim; ++d) {
      double s = (xyz[r * 3 + d] - P->lo[d]) / M.h[d];
      cc[d] = (int)floor(s);
      if (cc[d] < 0 || cc[d] >= P->cells[d]) return ORC_EINVAL;
      xs[d] = s - cc[d];
    }
    long c = cell_index(P, cc);
    for (int v = 0; v < M.nv; ++v) {
      double acc = 0.0;
      for (int k = 0; k < M.S; ++k) {
        int kk[3];
        node_index(&M, k, kk);
        double phi = 1.0;
        for (int d = 0; d < M.dim; ++d) phi *= lagrange(&T, kk[d], xs[d]);
        acc += phi * Q[((size_t)c * M.nv + v) * M.S + k];
      }
      out[r * M.nv + v] = acc;
    }
  }
  return ORC_OK;
}

/* Admissibility of every cell (Sec. 3.5, physical criterion plus finiteness):
 * flags[c] = 1 if any node of c fails; *count = number of flagged cells. */
int orc_check_admissible(const orc_problem *P, const double *Q, const double *params,
                         unsigned char *flags, int *count) {
  mesh M;
  if (make_mesh(P, &M)) return ORC_EINVAL;
  int cnt = 0;
  for (long c = 0; c < M.C; ++c) {
    int bad = 0;
    for (int k = 0; k < M.S && !bad; ++k) {
      double q[ORC_MAXQ];
      for (int v = 0; v < M.nv; ++v) q[v] = Q[((size_t)c * M.nv + v) * M.S + k];
      for (int p = 0; p < P->nparam; ++p) q[M.nv + p] = params[(size_t)c * P->nparam + p];
      bad = !pde_admissible(P, q);
    }
    flags[c] = (unsigned char)bad;
    cnt += bad;
  }
  *count = cnt;
  return ORC_OK;
}

/* ========================================================================
 * 9. Discrete adjoint of one step, for the PDEs that are linear in Q
 *    (elasticity, advection), with dt frozen.
 *
 *    The step maps (u^n, m) -> u^{n+1}, m the per-cell material parameters.
 *    Given lam = dJ/du^{n+1} it returns dJ/du^n (in place) and adds
 *    dJ/dm to gparams, by running the forward step of Sections 4-7 and then
 *    every operation of it in reverse order, transposed.  All inner products
 *    are the plain Euclidean ones over nodal arrays (a discrete adjoint).
 *    READING: the derivative of max() in the Rusanov speed is split half and
 *    half between the two sides on a tie; the step size is held fixed.
 * ======================================================================== */
static int pde_is_linear(const orc_problem *P) {
  return P->pde == ORC_ELASTIC || P->pde == ORC_ADVECTION;
}

/* lamQ += (dF_d/dQ)^T lamF */
static void flux_T(const orc_problem *P, int d, const double *lamF, double *lamQ) {
  if (P->pde == ORC_ELASTIC) {
    for (int i = 0; i < 3; ++i) lamQ[sym_index(i, d)] += lamF[6 + i];
  } else if (P->pde == ORC_ADVECTION) {
    lamQ[0] += P->adv[d] * lamF[0];
  }
}

/* lamQ += (dS/dQ)^T lamS for the smooth source */
static void source_T(const orc_problem *P, const double *lamS, double *lamQ) {
  if (P->pde == ORC_ADVECTION) lamQ[0] += -P->kappa * lamS[0];
}

/* lamG += (dB/dgradQ)^T lamB, lamG is [dim][nq] */
static void ncp_T(const orc_problem *P, const double *Q, const double *lamB, double *lamG) {
  if (P->pde != ORC_ELASTIC) return;
  int nq = P->nvar + P->nparam;
  double rho = Q[9], cp = Q[10], cs = Q[11];
  double mu = rho * cs * cs;
  double lam = rho * cp * cp - 2.0 * mu;
  double lg[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double ldiv = lam * (lamB[0] + lamB[1] + lamB[2]);
  for (int i = 0; i < 3; ++i) lg[i][i] += 2.0 * mu * lamB[i] + ldiv;
  lg[0][1] += mu * lamB[3];
  lg[1][0] += mu * lamB[3];
  lg[0][2] += mu * lamB[4];
  lg[2][0] += mu * lamB[4];
  lg[1][2] += mu * lamB[5];
  lg[2][1] += mu * lamB[5];
  for (int i = 0; i < 3; ++i)
    for (int d = 0; d < 3; ++d) lamG[d * nq + 6 + i] += lg[i][d] / rho;
}

/* gp[0..2] += (dB/d(rho, cp, cs))^T lamB, with B = ncp(Q, gradQ) */
static void ncp_dparams_T(const orc_problem *P, const double *Q, const double *gradQ,
                          const double *lamB, double *gp) {
  if (P->pde != ORC_ELASTIC) return;
  int nq = P->nvar + P->nparam;
  double rho = Q[9], cp = Q[10], cs = Q[11];
  double mu = rho * cs * cs;
  double lam = rho * cp * cp - 2.0 * mu;
  double g[3][3];
  for (int i = 0; i < 3; ++i)
    for (int d = 0; d < 3; ++d) g[i][d] = gradQ[d * nq + 6 + i] / rho;
  double divv = g[0][0] + g[1][1] + g[2][2];
  /* derivatives of (mu, lam, g) with respect to rho, cp, cs */
  double dmu[3] = {cs * cs, 0.0, 2.0 * rho * cs};
  double dlam[3] = {cp * cp - 2.0 * cs * cs, 2.0 * rho * cp, -4.0 * rho * cs};
  double dgs[3] = {-1.0 / rho, 0.0, 0.0}; /* dg/dp = dgs * g */
  for (int p = 0; p < 3; ++p) {
    double dB[6];
    for (int i = 0; i < 3; ++i)
      dB[i] = 2.0 * dmu[p] * g[i][i] + dlam[p] * divv + dgs[p] * (2.0 * mu * g[i][i] + lam * divv);
    dB[3] = dmu[p] * (g[0][1] + g[1][0]) + dgs[p] * mu * (g[0][1] + g[1][0]);
    dB[4] = dmu[p] * (g[0][2] + g[2][0]) + dgs[p] * mu * (g[0][2] + g[2][0]);
    dB[5] = dmu[p] * (g[1][2] + g[2][1]) + dgs[p] * mu * (g[1][2] + g[2][1]);
    double s = 0.0;
    for (int v = 0; v < 6; ++v) s += lamB[v] * dB[v];
    gp[p] += s;
  }
}

/* Reverse of rusanov() for one face node.  lamflL / lamflR are the adjoints
 * of the two fluctuations; the adjoints of the traces of both sides and of
 * the parameters of both sides are accumulated. */
static void rusanov_T(const orc_problem *P, int d, const double *qL, const double *qR,
                      const double *lamflL, const double *lamflR, double *lqL, double *lFL,
                      double *lqR, double *lFR, double *gpL, double *gpR) {
  int nv = P->nvar, nq = P->nvar + P->nparam;
  double sL = pde_max_eigen(P, qL, d), sR = pde_max_eigen(P, qR, d);
  double s = fmax(sL, sR);
  double lamG[ORC_MAXQ], ld[ORC_MAXQ], lamBm[ORC_MAXQ];
  double ls = 0.0;
  for (int v = 0; v < nv; ++v) {
    lamG[v] = lamflL[v] - lamflR[v];
    lFL[v] += -lamflL[v] + 0.5 * lamG[v];
    lFR[v] += lamflR[v] + 0.5 * lamG[v];
    ld[v] = -0.5 * s * lamG[v];
    ls += -0.5 * (qR[v] - qL[v]) * lamG[v];
    lamBm[v] = 0.5 * (lamflL[v] + lamflR[v]); /* Bmid = 0.5 * ncp(...) */
  }
  if (P->pde == ORC_ELASTIC) {
    /* s = max(cp_L, cp_R) */
    if (sL > sR) gpL[1] += ls;
    else if (sR > sL) gpR[1] += ls;
    else { gpL[1] += 0.5 * ls; gpR[1] += 0.5 * ls; }
    double qm[ORC_MAXQ], grad[3 * ORC_MAXQ], lgrad[3 * ORC_MAXQ], gpm[3] = {0.0, 0.0, 0.0};
    for (int v = 0; v < nq; ++v) qm[v] = 0.5 * (qL[v] + qR[v]);
    for (int a = 0; a < 3 * ORC_MAXQ; ++a) grad[a] = lgrad[a] = 0.0;
    for (int v = 0; v < nv; ++v) grad[d * nq + v] = qR[v] - qL[v];
    ncp_T(P, qm, lamBm, lgrad);
    for (int v = 0; v < nv; ++v) ld[v] += lgrad[d * nq + v];
    ncp_dparams_T(P, qm, grad, lamBm, gpm);
    for (int p = 0; p < 3; ++p) {
      gpL[p] += 0.5 * gpm[p];
      gpR[p] += 0.5 * gpm[p];
    }
  }
  for (int v = 0; v < nv; ++v) {
    lqR[v] += ld[v];
    lqL[v] -= ld[v];
  }
}

/* Forward predictor of one cell that also keeps every iterate q^0..q^I. */
static void predictor_history(const orc_problem *P, const mesh *M, const tables *T, long c,
                              const double *Q, const double *params, double dt, double t,
                              work *W, double *hist /*[I+1][n][S][nq]*/) {
  const int n = M->n, S = M->S, nq = M->nq, nv = M->nv, I = P->picard_iters;
  size_t it_sz = (size_t)n * S * nq;
  int cc[3];
  cell_coords(P, c, cc);
  double xlo[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < M->dim; ++d) xlo[d] = P->lo[d] + cc[d] * M->h[d];
  for (int k = 0; k < S; ++k) {
    for (int v = 0; v < nv; ++v) W->u[(size_t)k * nq + v] = Q[((size_t)c * nv + v) * S + k];
    for (int p = 0; p < P->nparam; ++p) W->u[(size_t)k * nq + nv + p] = params[(size_t)c * P->nparam + p];
  }
  for (int j = 0; j < n; ++j) memcpy(&W->q[(size_t)j * S * nq], W->u, sizeof(double) * S * nq);
  memcpy(hist, W->q, sizeof(double) * it_sz);
  for (int r = 0; r < I; ++r) {
    eval_terms(P, M, T, c, xlo, dt, t, W);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < S; ++k) {
        double *qi = &W->qn[((size_t)i * S + k) * nq];
        for (int v = 0; v < nv; ++v) {
          double acc = 0.0;
          for (int j = 0; j < n; ++j)
            acc += T->K1inv[i][j] *
                   (T->l0[j] * W->u[(size_t)k * nq + v] + dt * T->w[j] * W->R[((size_t)j * S + k) * nv + v]);
          qi[v] = acc;
        }
        for (int p = 0; p < P->nparam; ++p) qi[nv + p] = W->u[(size_t)k * nq + nv + p];
      }
    double *tmp = W->q;
    W->q = W->qn;
    W->qn = tmp;
    memcpy(&hist[(size_t)(r + 1) * it_sz], W->q, sizeof(double) * it_sz);
  }
}

/* gradient of one time slice of an iterate: grad[k][d][nq] (evolved only) */
static void slice_gradient(const mesh *M, const tables *T, const double *qs /*[S][nq]*/, double *grad) {
  const int n = M->n, S = M->S, nq = M->nq, nv = M->nv, dim = M->dim;
  for (int k = 0; k < S; ++k) {
    int kk[3];
    node_index(M, k, kk);
    double *g = &grad[(size_t)k * dim * nq];
    for (int a = 0; a < dim * nq; ++a) g[a] = 0.0;
    for (int d = 0; d < dim; ++d) {
      for (int m = 0; m < n; ++m) {
        int km = k + (m - kk[d]) * M->stride[d];
        for (int v = 0; v < nv; ++v) g[d * nq + v] += T->D[kk[d]][m] * qs[(size_t)km * nq + v];
      }
      for (int v = 0; v < nv; ++v) g[d * nq + v] /= M->h[d];
    }
  }
}

/* Reverse of R(q_j) = -div F(q_j) - B(q_j) grad q_j + S(q_j) for one slice:
 * lamR [S][nv] -> lamq [S][nq] (+=), gp (+=, the cell's parameters). */
static void rhs_T(const orc_problem *P, const mesh *M, const tables *T, const double *qs,
                  const double *lamR, double *lamq, double *gp) {
  const int n = M->n, S = M->S, nq = M->nq, nv = M->nv, dim = M->dim;
  double *grad = malloc(sizeof(double) * S * dim * nq);
  double *lamF = calloc((size_t)dim * S * nv, sizeof(double));
  double *lamG = calloc((size_t)S * dim * nq, sizeof(double));
  slice_gradient(M, T, qs, grad);
  for (int k = 0; k < S; ++k) {
    int kk[3];
    node_index(M, k, kk);
    const double *lr = &lamR[(size_t)k * nv];
    /* -div F: divF[k] = sum_d (1/h_d) sum_m D[k_d][m] F_d(q_km) */
    for (int d = 0; d < dim; ++d)
      for (int m = 0; m < n; ++m) {
        int km = k + (m - kk[d]) * M->stride[d];
        for (int v = 0; v < nv; ++v)
          lamF[((size_t)d * S + km) * nv + v] += -T->D[kk[d]][m] * lr[v] / M->h[d];
      }
    /* -B grad q */
    double lamB[ORC_MAXQ];
    for (int v = 0; v < nv; ++v) lamB[v] = -lr[v];
    ncp_T(P, &qs[(size_t)k * nq], lamB, &lamG[(size_t)k * dim * nq]);
    if (gp) ncp_dparams_T(P, &qs[(size_t)k * nq], &grad[(size_t)k * dim * nq], lamB, gp);
    /* + S(q) */
    source_T(P, lr, &lamq[(size_t)k * nq]);
  }
  /* transpose of the flux evaluation */
  for (int d = 0; d < dim; ++d)
    for (int k = 0; k < S; ++k) flux_T(P, d, &lamF[((size_t)d * S + k) * nv], &lamq[(size_t)k * nq]);
  /* transpose of the gradient: g[k][d] = (1/h_d) sum_m D[k_d][m] q(k:k_d<-m) */
  for (int k = 0; k < S; ++k) {
    int kk[3];
    node_index(M, k, kk);
    for (int d = 0; d < dim; ++d)
      for (int m = 0; m < n; ++m) {
        int km = k + (m - kk[d]) * M->stride[d];
        for (int v = 0; v < nv; ++v)
          lamq[(size_t)km * nq + v] += T->D[kk[d]][m] * lamG[((size_t)k * dim + d) * nq + v] / M->h[d];
      }
  }
  free(grad);
  free(lamF);
  free(lamG);
}

int orc_step_adjoint(const orc_problem *P, const double *Q, const double *params, double dt,
                     double t, double *lam, double *gparams) {
  mesh M;
  tables T;
  /* the adjoint is that of the periodic step */
  if (!pde_is_linear(P) || !bc_periodic(P) || make_mesh(P, &M) || make_tables(M.n, &T)) return ORC_EINVAL;
  const int n = M.n, S = M.S, nv = M.nv, nq = M.nq, F = M.F, dim = M.dim, I = P->picard_iters;
  const size_t face_all = (size_t)2 * dim * F * nv;
  const long C = M.C;
  const int np = P->nparam;
  /* 1. forward traces of every cell */
  double *qhat = malloc(sizeof(double) * C * face_all);
  double *Fhat = malloc(sizeof(double) * C * face_all);
  double *lamfl = calloc(C * face_all, sizeof(double));
  double *lqh = calloc(C * face_all, sizeof(double));
  double *lFh = calloc(C * face_all, sizeof(double));
  double *lam_out = malloc(sizeof(double) * C * nv * S);
  if (!qhat || !Fhat || !lamfl || !lqh || !lFh || !lam_out) return ORC_ENOMEM;
#pragma omp parallel
  {
    work W;
    work_alloc(&M, &W);
    double *vol = malloc(sizeof(double) * S * nv);
#pragma omp for schedule(dynamic, 4)
    for (long c = 0; c < C; ++c)
      predict_and_project(P, &M, &T, c, Q, params, dt, t, &W, vol, NULL, &qhat[c * face_all],
                          &Fhat[c * face_all]);
    free(vol);
    work_free(&W);
  }
  /* 2. adjoints of the fluctuations each cell uses:
   *    u^{n+1}_k = u_k + vol_k - dt sum_d (l1 fl_hi + l0 fl_lo) / (h_d w_{k_d}) */
  for (long c = 0; c < C; ++c)
    for (int k = 0; k < S; ++k) {
      int kk[3];
      node_index(&M, k, kk);
      for (int d = 0; d < dim; ++d) {
        int f = face_node(&M, d, kk);
        for (int v = 0; v < nv; ++v) {
          double l = lam[((size_t)c * nv + v) * S + k];
          double sc = -dt / (M.h[d] * T.w[kk[d]]);
          lamfl[c * face_all + (size_t)(2 * d + 1) * F * nv + (size_t)f * nv + v] += sc * T.l1[kk[d]] * l;
          lamfl[c * face_all + (size_t)(2 * d + 0) * F * nv + (size_t)f * nv + v] += sc * T.l0[kk[d]] * l;
        }
      }
    }
  /* 3. Rusanov in reverse: each cell collects the adjoints of its own traces
   *    and parameters from both fluctuations of each of its faces */
  for (long c = 0; c < C; ++c) {
    for (int d = 0; d < dim; ++d)
      for (int side = 0; side < 2; ++side) {
        long nb = neighbour(P, c, d, side ? 1 : -1);
        long cl = side ? c : nb, cr = side ? nb : c;
        const double *qhL = &qhat[cl * face_all + (size_t)(2 * d + 1) * F * nv];
        const double *qhR = &qhat[cr * face_all + (size_t)(2 * d + 0) * F * nv];
        const double *lfL = &lamfl[cl * face_all + (size_t)(2 * d + 1) * F * nv];
        const double *lfR = &lamfl[cr * face_all + (size_t)(2 * d + 0) * F * nv];
        for (int f = 0; f < F; ++f) {
          double qL[ORC_MAXQ], qR[ORC_MAXQ], lqL[ORC_MAXQ] = {0}, lqR[ORC_MAXQ] = {0};
          double lFL[ORC_MAXQ] = {0}, lFR[ORC_MAXQ] = {0}, gpL[3] = {0, 0, 0}, gpR[3] = {0, 0, 0};
          for (int v = 0; v < nv; ++v) {
            qL[v] = qhL[(size_t)f * nv + v];
            qR[v] = qhR[(size_t)f * nv + v];
          }
          for (int p = 0; p < np; ++p) {
            qL[nv + p] = params[(size_t)cl * np + p];
            qR[nv + p] = params[(size_t)cr * np + p];
          }
          rusanov_T(P, d, qL, qR, &lfL[(size_t)f * nv], &lfR[(size_t)f * nv], lqL, lFL, lqR, lFR, gpL, gpR);
          double *oq = &lqh[c * face_all + (size_t)(2 * d + side) * F * nv + (size_t)f * nv];
          double *oF = &lFh[c * face_all + (size_t)(2 * d + side) * F * nv + (size_t)f * nv];
          for (int v = 0; v < nv; ++v) {
            oq[v] += side ? lqL[v] : lqR[v];
            oF[v] += side ? lFL[v] : lFR[v];
          }
          for (int p = 0; p < np; ++p) gparams[(size_t)c * np + p] += side ? gpL[p] : gpR[p];
        }
      }
  }
  /* 4. predictor in reverse, per cell */
  int fail = 0;
#pragma omp parallel
  {
    work W;
    int ok = work_alloc(&M, &W) == ORC_OK;
    size_t it_sz = (size_t)n * S * nq;
    double *hist = malloc(sizeof(double) * (I + 1) * it_sz);
    double *lq = malloc(sizeof(double) * it_sz);   /* adjoint of an iterate [n][S][nq] */
    double *lqn = malloc(sizeof(double) * it_sz);
    double *lR = malloc(sizeof(double) * S * nv);
    double *lqbar = malloc(sizeof(double) * S * nv);
    double *lFbar = malloc(sizeof(double) * dim * S * nv);
    double *lu = malloc(sizeof(double) * S * nv);
    if (!ok || !hist || !lq || !lqn || !lR || !lqbar || !lFbar || !lu) {
#pragma omp atomic write
      fail = 1;
    }
    double gcell[3];
#pragma omp for schedule(dynamic, 4)
    for (long c = 0; c < C; ++c) {
      if (fail) continue;
      gcell[0] = gcell[1] = gcell[2] = 0.0;
      predictor_history(P, &M, &T, c, Q, params, dt, t, &W, hist);
      const double *qI = &hist[(size_t)I * it_sz];
      for (size_t a = 0; a < (size_t)S * nv; ++a) lu[a] = 0.0;
      /* u^{n+1} = u + vol - surf: identity part */
      for (int k = 0; k < S; ++k)
        for (int v = 0; v < nv; ++v) lu[(size_t)k * nv + v] = lam[((size_t)c * nv + v) * S + k];
      /* vol = dt (-div Fbar - Nbar + Sbar) with Fbar, Nbar, Sbar time averages
       * of F, B grad q, S at the final iterate: reverse through the time
       * average into per-slice adjoints of R-like terms (weight w_j) */
      for (size_t a = 0; a < (size_t)dim * S * nv; ++a) lFbar[a] = 0.0;
      for (size_t a = 0; a < (size_t)S * nv; ++a) lqbar[a] = 0.0;
      /* traces: qhat = sum_m l_m qbar, Fhat = sum_m l_m Fbar_d */
      for (int k = 0; k < S; ++k) {
        int kk[3];
        node_index(&M, k, kk);
        for (int d = 0; d < dim; ++d) {
          int f = face_node(&M, d, kk);
          for (int side = 0; side < 2; ++side) {
            double l = side ? T.l1[kk[d]] : T.l0[kk[d]];
            const double *a1 = &lqh[c * face_all + (size_t)(2 * d + side) * F * nv + (size_t)f * nv];
            const double *a2 = &lFh[c * face_all + (size_t)(2 * d + side) * F * nv + (size_t)f * nv];
            for (int v = 0; v < nv; ++v) {
              lqbar[(size_t)k * nv + v] += l * a1[v];
              lFbar[((size_t)d * S + k) * nv + v] += l * a2[v];
            }
          }
        }
      }
      /* the volume term: -dt div Fbar adds to lFbar; -dt Nbar and +dt Sbar act
       * per slice with weight w_j (handled below with the slices) */
      for (int k = 0; k < S; ++k) {
        int kk[3];
        node_index(&M, k, kk);
        for (int d = 0; d < dim; ++d)
          for (int m = 0; m < n; ++m) {
            int km = k + (m - kk[d]) * M.stride[d];
            for (int v = 0; v < nv; ++v)
              lFbar[((size_t)d * S + km) * nv + v] +=
                  -dt * T.D[kk[d]][m] * lu[(size_t)k * nv + v] / M.h[d];
          }
      }
      /* adjoint of the final iterate, slice by slice:
       * qbar = sum_j w_j q_j;  Fbar_d = sum_j w_j F_d(q_j);
       * Nbar = sum_j w_j B(q_j) grad q_j;  Sbar = sum_j w_j S(q_j) */
      for (size_t a = 0; a < it_sz; ++a) lq[a] = 0.0;
      for (int j = 0; j < n; ++j) {
        const double *qs = &qI[(size_t)j * S * nq];
        double *lqs = &lq[(size_t)j * S * nq];
        for (int k = 0; k < S; ++k) {
          for (int v = 0; v < nv; ++v) lqs[(size_t)k * nq + v] += T.w[j] * lqbar[(size_t)k * nv + v];
          for (int d = 0; d < dim; ++d) {
            double lf[ORC_MAXQ];
            for (int v = 0; v < nv; ++v) lf[v] = T.w[j] * lFbar[((size_t)d * S + k) * nv + v];
            flux_T(P, d, lf, &lqs[(size_t)k * nq]);
          }
        }
        /* -dt Nbar + dt Sbar is w_j dt (-B grad q_j + S(q_j)): the same map as
         * R without its flux part; reuse rhs_T with the flux adjoint zero by
         * passing an R-adjoint whose divergence part is handled separately */
        for (int k = 0; k < S; ++k)
          for (int v = 0; v < nv; ++v) lR[(size_t)k * nv + v] = T.w[j] * dt * lu[(size_t)k * nv + v];
        {
          /* B grad q and S parts only */
          double *grad = malloc(sizeof(double) * S * dim * nq);
          double *lamG = calloc((size_t)S * dim * nq, sizeof(double));
          slice_gradient(&M, &T, qs, grad);
          for (int k = 0; k < S; ++k) {
            double lamB[ORC_MAXQ];
            for (int v = 0; v < nv; ++v) lamB[v] = -lR[(size_t)k * nv + v];
            ncp_T(P, &qs[(size_t)k * nq], lamB, &lamG[(size_t)k * dim * nq]);
            ncp_dparams_T(P, &qs[(size_t)k * nq], &grad[(size_t)k * dim * nq], lamB, gcell);
            source_T(P, &lR[(size_t)k * nv], &lqs[(size_t)k * nq]);
          }
          for (int k = 0; k < S; ++k) {
            int kk[3];
            node_index(&M, k, kk);
            for (int d = 0; d < dim; ++d)
              for (int m = 0; m < n; ++m) {
                int km = k + (m - kk[d]) * M.stride[d];
                for (int v = 0; v < nv; ++v)
                  lqs[(size_t)km * nq + v] += T.D[kk[d]][m] * lamG[((size_t)k * dim + d) * nq + v] / M.h[d];
              }
          }
          free(grad);
          free(lamG);
        }
      }
      /* Picard in reverse: q^{r+1}_i = sum_j K1inv_ij (l0_j u + dt w_j R(q^r)_j) */
      for (int r = I - 1; r >= 0; --r) {
        const double *qr = &hist[(size_t)r * it_sz];
        for (size_t a = 0; a < it_sz; ++a) lqn[a] = 0.0;
        for (int j = 0; j < n; ++j) {
          for (int k = 0; k < S; ++k)
            for (int v = 0; v < nv; ++v) {
              double sR = 0.0, sU = 0.0;
              for (int i = 0; i < n; ++i) {
                double a = lq[((size_t)i * S + k) * nq + v];
                sR += T.K1inv[i][j] * a;
                sU += T.K1inv[i][j] * a;
              }
              lR[(size_t)k * nv + v] = dt * T.w[j] * sR;
              lu[(size_t)k * nv + v] += T.l0[j] * sU;
            }
          rhs_T(P, &M, &T, &qr[(size_t)j * S * nq], lR, &lqn[(size_t)j * S * nq], gcell);
        }
        double *tmp = lq;
        lq = lqn;
        lqn = tmp;
      }
      /* q^0_j = u for every j */
      for (int j = 0; j < n; ++j)
        for (int k = 0; k < S; ++k)
          for (int v = 0; v < nv; ++v) lu[(size_t)k * nv + v] += lq[((size_t)j * S + k) * nq + v];
      for (int k = 0; k < S; ++k)
        for (int v = 0; v < nv; ++v) lam_out[((size_t)c * nv + v) * S + k] = lu[(size_t)k * nv + v];
      for (int p = 0; p < np; ++p) gparams[(size_t)c * np + p] += gcell[p];
    }
    free(hist); free(lq); free(lqn); free(lR); free(lqbar); free(lFbar); free(lu);
    work_free(&W);
  }
  if (!fail) memcpy(lam, lam_out, sizeof(double) * C * nv * S);
  free(qhat); free(Fhat); free(lamfl); free(lqh); free(lFh); free(lam_out);
  return fail ? ORC_ENOMEM : ORC_OK;
}

/* Transpose of orc_sample_receivers: lam[c_r][v][k] += Phi_k(xi_r) lamrec[r][v]. */
int orc_sample_receivers_T(const orc_problem *P, int nrec, const double *xyz, const double *lamrec,
                           double *lam) {
  mesh M;
  tables T;
  if (make_mesh(P, &M) || make_tables(M.n, &T)) return ORC_EINVAL;
  for (int r = 0; r < nrec; ++r) {
    int cc[3] = {0, 0, 0};
    double xs[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < M.dim; ++d) {
      double s = (xyz[r * 3 + d] - P->lo[d]) / M.h[d];
      cc[d] = (int)floor(s);
      if (cc[d] < 0 || cc[d] >= P->cells[d]) return ORC_EINVAL;
      xs[d] = s - cc[d];
    }
    long c = cell_index(P, cc);
    for (int k = 0; k < M.S; ++k) {
      int kk[3];
      node_index(&M, k, kk);
      double phi = 1.0;
      for (int d = 0; d < M.dim; ++d) phi *= lagrange(&T, kk[d], xs[d]);
      for (int v = 0; v < M.nv; ++v) lam[((size_t)c * M.nv + v) * M.S + k] += phi * lamrec[r * M.nv + v];
    }
  }
  return ORC_OK;
}

/* ========================================================================
 * 10. A-posteriori subcell limiter for the Euler equations (Sec. 3.5, the
 *     FV, limiter and projection kernels of Table 1, the status stencil of
 *     Fig. 2).  One limited step:
 *       1. the unlimited ADER-DG step gives a candidate u* in every cell;
 *       2. a cell is troubled if u* fails the physical admissibility test
 *          (at every node and every subcell average) or the relaxed discrete
 *          maximum principle;
 *       3. troubled cells and their face neighbours are recomputed from u^n
 *          with a second-order FV scheme on (2N+1)^d subcells, and the FV
 *          result is projected back to the DG space;
 *       4. DG cells that share a face with a recomputed cell take, on that
 *          face, the FV fluxes in place of the Rusanov flux of step 1, so
 *          that what leaves one cell enters the other.
 *    READINGS (the paper names these pieces but gives no formulas):
 *    - projectOnFVLimiterSpace gives exact subcell averages,
 *        v_s = sum_k prod_d A[s_d][k_d] u_k,
 *        A[s][k] = m * integral of phi_k over [s/m, (s+1)/m],  m = 2N+1;
 *    - projectOnDGSpace is the least-squares inverse, u = (B x .. x B) v,
 *      B = (A^T A)^{-1} A^T: a projected polynomial comes back unchanged and
 *      the cell mean is kept;
 *    - relaxed DMP: with lo_v, hi_v the smallest and largest subcell average
 *      of u^n over the cell and its face neighbours, every subcell average of
 *      the candidate must lie in [lo_v - delta_v, hi_v + delta_v],
 *      delta_v = max(1e-4, 1e-3 (hi_v - lo_v)) (the constants of the MOOD
 *      subcell-limiter work the paper cites);
 *    - the FV scheme is MUSCL-Hancock with the minmod limiter (Table 1's
 *      defaults): unsplit; minmod slopes of the conserved variables along
 *      each axis; the values extrapolated to the 2d subcell faces are moved
 *      half a step with the flux differences of all axes; Rusanov at every
 *      subcell face; a subcell whose extrapolated or moved values are not
 *      admissible uses its average on all faces (first order);
 *    - FV ghost subcells outside the domain mirror the inside ones (wall:
 *      the normal momentum reversed; outflow: unchanged);
 *    - hybrid ADER-DG/FV (the paper's variant of the method): a cell that
 *      was FV in the previous step keeps its FV subcell averages as its
 *      solution, and its DG polynomial (their projection) only serves its
 *      neighbours; in the next step its FV data, not the projection of that
 *      polynomial, is where its FV step starts and what the DMP and the
 *      neighbours' ghost subcells see (projecting a shock profile to a
 *      polynomial and back is not positive).  Every cell's DG candidate is
 *      computed each step; a cell is DG again as soon as its candidate
 *      passes both tests;
 *    - the flux a DG neighbour takes at a node of the shared face is the L2
 *      projection, with the GL face mass, of the piecewise constant subface
 *      fluxes: G_f = sum_t prod_{a != d} Qf[f_a][t_a] Fsub_t,
 *      Qf[j][s] = A[s][j] / (m w_j); the face's total flux is then the FV
 *      one.
 * ======================================================================== */
#define ORC_MAXM (2 * ORC_MAXN - 1)

typedef struct {
  int m;
  double A[ORC_MAXM][ORC_MAXN];  /* subcell averages of phi_k */
  double B[ORC_MAXN][ORC_MAXM];  /* least-squares inverse of A */
  double Qf[ORC_MAXN][ORC_MAXM]; /* piecewise constant face data -> face nodes */
} lim_tables;

static int make_lim_tables(const tables *T, lim_tables *L) {
  const int n = T->n, m = 2 * n - 1;
  long double A[ORC_MAXM][ORC_MAXN], xs[ORC_MAXN];
  L->m = m;
  for (int i = 0; i < n; ++i) xs[i] = T->xi[i];
  for (int s = 0; s < m; ++s)
    for (int k = 0; k < n; ++k) {
      /* n-point Gauss quadrature on the subinterval is exact for degree N;
       * m times (1/m) sum_q w_q phi_k(x_q) */
      long double sum = 0.0L;
      for (int q = 0; q < n; ++q) sum += (long double)T->w[q] * lagrange_ld(n, xs, k, ((long double)s + xs[q]) / m);
      A[s][k] = sum;
      L->A[s][k] = (double)sum;
    }
  /* B = (A^T A)^{-1} A^T by Gauss-Jordan on the normal equations */
  long double N[ORC_MAXN][2 * ORC_MAXN];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      long double a = 0.0L;
      for (int s = 0; s < m; ++s) a += A[s][i] * A[s][j];
      N[i][j] = a;
      N[i][n + j] = i == j ? 1.0L : 0.0L;
    }
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabsl(N[r][col]) > fabsl(N[piv][col])) piv = r;
    if (piv != col)
      for (int c = 0; c < 2 * n; ++c) {
        long double tmp = N[col][c];
        N[col][c] = N[piv][c];
        N[piv][c] = tmp;
      }
    long double d = N[col][col];
    if (d == 0.0L) return ORC_EINVAL;
    for (int c = 0; c < 2 * n; ++c) N[col][c] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      long double f = N[r][col];
      for (int c = 0; c < 2 * n; ++c) N[r][c] -= f * N[col][c];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int s = 0; s < m; ++s) {
      long double b = 0.0L;
      for (int j = 0; j < n; ++j) b += N[i][n + j] * A[s][j];
      L->B[i][s] = (double)b;
      L->Qf[i][s] = (double)(A[s][i] / ((long double)m * (long double)T->w[i]));
    }
  return ORC_OK;
}

static int ipow_i(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

static void sub_multi(int m, int s, int ss[3]) {
  ss[0] = s % m;
  ss[1] = (s / m) % m;
  ss[2] = s / (m * m);
}

/* v[var][s] = subcell averages of one cell's nodal values u[var][k] */
static void lim_project(const mesh *M, const lim_tables *L, const double *u, double *v) {
  const int m = L->m, ns = ipow_i(m, M->dim);
  for (int s = 0; s < ns; ++s) {
    int ss[3];
    sub_multi(m, s, ss);
    for (int var = 0; var < M->nv; ++var) {
      double sum = 0.0;
      for (int k = 0; k < M->S; ++k) {
        int kk[3];
        node_index(M, k, kk);
        double a = 1.0;
        for (int d = 0; d < M->dim; ++d) a *= L->A[ss[d]][kk[d]];
        sum += a * u[(size_t)var * M->S + k];
      }
      v[(size_t)var * ns + s] = sum;
    }
  }
}

/* u[var][k] = least-squares DG polynomial of subcell averages v[var][s] */
static void lim_reconstruct(const mesh *M, const lim_tables *L, const double *v, double *u) {
  const int m = L->m, ns = ipow_i(m, M->dim);
  for (int k = 0; k < M->S; ++k) {
    int kk[3];
    node_index(M, k, kk);
    for (int var = 0; var < M->nv; ++var) {
      double sum = 0.0;
      for (int s = 0; s < ns; ++s) {
        int ss[3];
        sub_multi(m, s, ss);
        double b = 1.0;
        for (int d = 0; d < M->dim; ++d) b *= L->B[kk[d]][ss[d]];
        sum += b * v[(size_t)var * ns + s];
      }
      u[(size_t)var * M->S + k] = sum;
    }
  }
}

/* Subcell average of u^n at global subcell index g (up to two subcells
 * outside the domain); V is [C][nv][m^dim]. */
static void lim_value(const orc_problem *P, const mesh *M, int m, const double *V, const int gin[3],
                      double *out) {
  int g[3] = {gin[0], gin[1], gin[2]}, flip[3] = {0, 0, 0}, cc[3] = {0, 0, 0}, ss[3] = {0, 0, 0};
  for (int d = 0; d < M->dim; ++d) {
    const int G = m * P->cells[d];
    if (g[d] < 0 || g[d] >= G) {
      const int side = g[d] >= G, kind = P->bc[2 * d + side];
      if (kind == ORC_BC_PERIODIC) {
        g[d] = ((g[d] % G) + G) % G;
      } else {
        g[d] = side ? 2 * G - 1 - g[d] : -1 - g[d];
        flip[d] = kind == ORC_BC_WALL;
      }
    }
    cc[d] = g[d] / m;
    ss[d] = g[d] % m;
  }
  const int ns = ipow_i(m, M->dim);
  const int si = ss[0] + m * (ss[1] + m * ss[2]);
  const long c = cell_index(P, cc);
  for (int var = 0; var < M->nv; ++var) out[var] = V[((size_t)c * M->nv + var) * ns + si];
  for (int d = 0; d < M->dim; ++d)
    if (flip[d]) out[1 + d] = -out[1 + d];
}

static double minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return fmin(a, b);
  if (a < 0.0 && b < 0.0) return fmax(a, b);
  return 0.0;
}

/* MUSCL-Hancock: the average of subcell g extrapolated to its 2 dim faces
 * with minmod slopes and moved half a step; out[d][side][var]. */
static void lim_evolved(const orc_problem *P, const mesh *M, int m, const double *V, const int g[3],
                        double dt, const double *hs, double out[3][2][ORC_MAXQ]) {
  const int nv = M->nv;
  double w[ORC_MAXQ], ext[3][2][ORC_MAXQ], corr[ORC_MAXQ];
  int ok = 1;
  lim_value(P, M, m, V, g, w);
  for (int d = 0; d < M->dim; ++d) {
    double wl[ORC_MAXQ], wr[ORC_MAXQ];
    int gl[3] = {g[0], g[1], g[2]}, gr[3] = {g[0], g[1], g[2]};
    gl[d] -= 1;
    gr[d] += 1;
    lim_value(P, M, m, V, gl, wl);
    lim_value(P, M, m, V, gr, wr);
    for (int v = 0; v < nv; ++v) {
      double slope = minmod(w[v] - wl[v], wr[v] - w[v]);
      ext[d][0][v] = w[v] - 0.5 * slope;
      ext[d][1][v] = w[v] + 0.5 * slope;
    }
    ok = ok && pde_admissible(P, ext[d][0]) && pde_admissible(P, ext[d][1]);
  }
  for (int v = 0; v < nv; ++v) corr[v] = 0.0;
  for (int d = 0; d < M->dim; ++d) {
    double Fl[ORC_MAXQ], Fr[ORC_MAXQ];
    pde_flux(P, ext[d][0], d, Fl);
    pde_flux(P, ext[d][1], d, Fr);
    for (int v = 0; v < nv; ++v) corr[v] += 0.5 * dt / hs[d] * (Fl[v] - Fr[v]);
  }
  for (int d = 0; d < M->dim; ++d)
    for (int side = 0; side < 2; ++side) {
      for (int v = 0; v < nv; ++v) out[d][side][v] = ext[d][side][v] + corr[v];
      ok = ok && pde_admissible(P, out[d][side]);
    }
  if (!ok)
    for (int d = 0; d < M->dim; ++d)
      for (int side = 0; side < 2; ++side)
        for (int v = 0; v < nv; ++v) out[d][side][v] = w[v];
}

/* Rusanov flux between the states a (low side) and b (high side) along d */
static void lim_rusanov(const orc_problem *P, int d, const double *a, const double *b, double *G) {
  double Fa[ORC_MAXQ], Fb[ORC_MAXQ];
  pde_flux(P, a, d, Fa);
  pde_flux(P, b, d, Fb);
  double s = fmax(pde_max_eigen(P, a, d), pde_max_eigen(P, b, d));
  for (int v = 0; v < P->nvar; ++v) G[v] = 0.5 * (Fa[v] + Fb[v]) - 0.5 * s * (b[v] - a[v]);
}

/* index of a subface (or face node) across the axes other than d, lower
 * axis fastest */
static int transverse_index(int dim, int d, int m, const int ss[3]) {
  int t = 0, mul = 1;
  for (int a = 0; a < dim; ++a) {
    if (a == d) continue;
    t += ss[a] * mul;
    mul *= m;
  }
  return t;
}

/* FV step of cell c from the u^n subcell averages V: vnew [nv][m^dim] and
 * the fluxes through the cell's faces, frec [2 dim][m^(dim-1)][nv]. */
static void lim_fv_cell(const orc_problem *P, const mesh *M, const lim_tables *L, const double *V, long c,
                        double dt, double *vnew, double *frec) {
  const int m = L->m, nv = M->nv, ns = ipow_i(m, M->dim), nsf = ipow_i(m, M->dim - 1);
  double hs[3];
  int cc[3];
  for (int d = 0; d < M->dim; ++d) hs[d] = M->h[d] / m;
  cell_coords(P, c, cc);
  for (int s = 0; s < ns; ++s) {
    int ss[3], g[3] = {0, 0, 0};
    sub_multi(m, s, ss);
    for (int d = 0; d < M->dim; ++d) g[d] = cc[d] * m + ss[d];
    double w[ORC_MAXQ], acc[ORC_MAXQ], E[3][2][ORC_MAXQ];
    lim_value(P, M, m, V, g, w);
    lim_evolved(P, M, m, V, g, dt, hs, E);
    for (int v = 0; v < nv; ++v) acc[v] = 0.0;
    for (int d = 0; d < M->dim; ++d) {
      double En[3][2][ORC_MAXQ], Glo[ORC_MAXQ], Ghi[ORC_MAXQ];
      int gn[3] = {g[0], g[1], g[2]};
      gn[d] = g[d] + 1;
      lim_evolved(P, M, m, V, gn, dt, hs, En);
      lim_rusanov(P, d, E[d][1], En[d][0], Ghi);
      gn[d] = g[d] - 1;
      lim_evolved(P, M, m, V, gn, dt, hs, En);
      lim_rusanov(P, d, En[d][1], E[d][0], Glo);
      for (int v = 0; v < nv; ++v) acc[v] += (Ghi[v] - Glo[v]) / hs[d];
      const int t = transverse_index(M->dim, d, m, ss);
      if (ss[d] == m - 1)
        for (int v = 0; v < nv; ++v) frec[((size_t)(2 * d + 1) * nsf + t) * nv + v] = Ghi[v];
      if (ss[d] == 0)
        for (int v = 0; v < nv; ++v) frec[((size_t)(2 * d) * nsf + t) * nv + v] = Glo[v];
    }
    for (int v = 0; v < nv; ++v) vnew[(size_t)v * ns + s] = w[v] - dt * acc[v];
  }
}

/* Subface fluxes of one face [m^(dim-1)][nv] -> face-node fluxes [F][nv] */
static void lim_face_to_nodes(const mesh *M, const lim_tables *L, const double *fsub, double *G) {
  const int m = L->m, nsf = ipow_i(m, M->dim - 1);
  for (int f = 0; f < M->F; ++f) {
    int ff[2] = {f % M->n, f / M->n};
    for (int v = 0; v < M->nv; ++v) {
      double sum = 0.0;
      for (int t = 0; t < nsf; ++t) {
        int tt[2] = {t % m, t / m};
        double q = 1.0;
        for (int a = 0; a < M->dim - 1; ++a) q *= L->Qf[ff[a]][tt[a]];
        sum += q * fsub[(size_t)t * M->nv + v];
      }
      G[(size_t)f * M->nv + v] = sum;
    }
  }
}

/* One limited step in place (Euler only).
 * status [C], in and out: 0 DG, 1 DG taking FV fluxes on some face, 2 FV as
 *   a neighbour of a troubled cell, 3 troubled (FV); all zero before the
 *   first step.
 * sub [C][nv][m^dim], in and out: the FV subcell averages of the cells with
 *   status >= 2 (the other cells' entries are neither read nor written).
 * counts[3] (may be NULL): troubled cells, FV cells (status 2 or 3), DG
 *   cells with FV faces. */
int orc_step_limited(const orc_problem *P, double *Q, const double *params, double dt, double t,
                     double *sub, unsigned char *status, int *counts) {
  mesh M;
  tables T;
  lim_tables L;
  if (P->pde != ORC_EULER || !sub || !status) return ORC_EINVAL;
  for (int f = 0; f < 6; ++f)
    if (P->bc[f] == ORC_BC_INFLOW) return ORC_EINVAL; /* FV ghosts: mirror faces only */
  if (make_mesh(P, &M) || make_tables(M.n, &T) || make_lim_tables(&T, &L)) return ORC_EINVAL;
  const int m = L.m, nv = M.nv, S = M.S, ns = ipow_i(m, M.dim), nsf = ipow_i(m, M.dim - 1);
  const long C = M.C;
  for (long c = 0; c < C; ++c)
    if (status[c] > 3) return ORC_EINVAL;
  const size_t face_all = (size_t)2 * M.dim * M.F * nv, cell_sz = (size_t)nv * S;
  const size_t rec_sz = (size_t)2 * M.dim * nsf * nv;
  cellside CS;
  CS.vol = malloc(sizeof(double) * C * S * nv);
  CS.weak = NULL;
  CS.qhat = malloc(sizeof(double) * C * face_all);
  CS.Fhat = malloc(sizeof(double) * C * face_all);
  double *Qn = malloc(sizeof(double) * C * cell_sz);
  double *Qc = malloc(sizeof(double) * C * cell_sz);
  double *Vn = malloc(sizeof(double) * C * nv * ns);
  double *lo = malloc(sizeof(double) * C * nv), *hi = malloc(sizeof(double) * C * nv);
  double *frec = malloc(sizeof(double) * C * rec_sz);
  unsigned char *st = malloc(C);
  int rc = ORC_ENOMEM;
  if (!CS.vol || !CS.qhat || !CS.Fhat || !Qn || !Qc || !Vn || !lo || !hi || !frec || !st) goto done;
  memcpy(Qn, Q, sizeof(double) * C * cell_sz);

  /* 1. the unlimited candidate */
  rc = predict_all(P, &M, &T, Qn, params, dt, t, NULL, C, &CS);
  if (rc != ORC_OK) goto done;
#pragma omp parallel for schedule(dynamic, 8)
  for (long c = 0; c < C; ++c) {
    long nb[6];
    double *qh[7], *Fh[7];
    qh[0] = &CS.qhat[c * face_all];
    Fh[0] = &CS.Fhat[c * face_all];
    for (int d = 0; d < M.dim; ++d)
      for (int s = 0; s < 2; ++s) {
        nb[2 * d + s] = neighbour(P, c, d, s ? 1 : -1);
        qh[1 + 2 * d + s] = nb[2 * d + s] < 0 ? NULL : &CS.qhat[nb[2 * d + s] * face_all];
        Fh[1 + 2 * d + s] = nb[2 * d + s] < 0 ? NULL : &CS.Fhat[nb[2 * d + s] * face_all];
      }
    correct_cell(P, &M, &T, c, Qn, params, dt, &CS.vol[(size_t)c * S * nv], NULL, qh, Fh, nb,
                 &Qc[(size_t)c * cell_sz], NULL, NULL);
  }

  /* 2. subcell averages at t^n (FV cells: their own) and their ranges */
#pragma omp parallel for schedule(dynamic, 8)
  for (long c = 0; c < C; ++c) {
    double *v = &Vn[(size_t)c * nv * ns];
    if (status[c] >= 2)
      memcpy(v, &sub[(size_t)c * nv * ns], sizeof(double) * nv * ns);
    else
      lim_project(&M, &L, &Qn[(size_t)c * cell_sz], v);
    for (int var = 0; var < nv; ++var) {
      double a = v[(size_t)var * ns], b = a;
      for (int s = 1; s < ns; ++s) {
        a = fmin(a, v[(size_t)var * ns + s]);
        b = fmax(b, v[(size_t)var * ns + s]);
      }
      lo[c * nv + var] = a;
      hi[c * nv + var] = b;
    }
  }

  /* 3. troubled cells: physical admissibility, then the relaxed DMP */
#pragma omp parallel for schedule(dynamic, 8)
  for (long c = 0; c < C; ++c) {
    const double *u = &Qc[(size_t)c * cell_sz];
    double *v = NULL;
    int bad = 0;
    for (int k = 0; k < S && !bad; ++k) {
      double q[ORC_MAXQ];
      for (int var = 0; var < nv; ++var) q[var] = u[(size_t)var * S + k];
      bad = !pde_admissible(P, q);
    }
    v = malloc(sizeof(double) * nv * ns);
    lim_project(&M, &L, u, v);
    for (int s = 0; s < ns && !bad; ++s) {
      double q[ORC_MAXQ];
      for (int var = 0; var < nv; ++var) q[var] = v[(size_t)var * ns + s];
      bad = !pde_admissible(P, q);
    }
    for (int var = 0; var < nv && !bad; ++var) {
      double a = lo[c * nv + var], b = hi[c * nv + var];
      for (int d = 0; d < M.dim; ++d)
        for (int sd = -1; sd <= 1; sd += 2) {
          long o = neighbour(P, c, d, sd);
          if (o < 0) continue;
          a = fmin(a, lo[o * nv + var]);
          b = fmax(b, hi[o * nv + var]);
        }
      double delta = fmax(1e-4, 1e-3 * (b - a));
      for (int s = 0; s < ns && !bad; ++s) {
        double x = v[(size_t)var * ns + s];
        bad = !(x >= a - delta && x <= b + delta);
      }
    }
    free(v);
    st[c] = bad ? 3 : 0;
  }

  /* 4. FV set: troubled cells and their face neighbours; DG cells next to it */
  for (long c = 0; c < C; ++c) {
    if (st[c] == 3) continue;
    int near = 0;
    for (int d = 0; d < M.dim; ++d)
      for (int sd = -1; sd <= 1; sd += 2) {
        long o = neighbour(P, c, d, sd);
        if (o >= 0 && st[o] == 3) near = 1;
      }
    if (near) st[c] = 2;
  }
  for (long c = 0; c < C; ++c) {
    if (st[c] >= 2) continue;
    for (int d = 0; d < M.dim; ++d)
      for (int sd = -1; sd <= 1; sd += 2) {
        long o = neighbour(P, c, d, sd);
        if (o >= 0 && st[o] >= 2) st[c] = 1;
      }
  }

  /* 5. FV cells, from the subcell averages at t^n */
#pragma omp parallel for schedule(dynamic, 1)
  for (long c = 0; c < C; ++c) {
    if (st[c] < 2) continue;
    double *vnew = &sub[(size_t)c * nv * ns];
    lim_fv_cell(P, &M, &L, Vn, c, dt, vnew, &frec[(size_t)c * rec_sz]);
    lim_reconstruct(&M, &L, vnew, &Q[(size_t)c * cell_sz]);
  }

  /* 6. DG cells: the candidate, with FV fluxes on faces shared with FV cells */
#pragma omp parallel for schedule(dynamic, 8)
  for (long c = 0; c < C; ++c) {
    if (st[c] >= 2) continue;
    if (st[c] == 0) {
      memcpy(&Q[(size_t)c * cell_sz], &Qc[(size_t)c * cell_sz], sizeof(double) * cell_sz);
      continue;
    }
    long nb[6];
    double *qh[7], *Fh[7], *Gbuf = malloc(sizeof(double) * 2 * M.dim * M.F * nv);
    const double *Gover[6] = {NULL, NULL, NULL, NULL, NULL, NULL};
    qh[0] = &CS.qhat[c * face_all];
    Fh[0] = &CS.Fhat[c * face_all];
    for (int d = 0; d < M.dim; ++d)
      for (int s = 0; s < 2; ++s) {
        long o = neighbour(P, c, d, s ? 1 : -1);
        nb[2 * d + s] = o;
        qh[1 + 2 * d + s] = o < 0 ? NULL : &CS.qhat[o * face_all];
        Fh[1 + 2 * d + s] = o < 0 ? NULL : &CS.Fhat[o * face_all];
        if (o >= 0 && st[o] >= 2) {
          /* the neighbour's record of the same face: its opposite side */
          double *G = &Gbuf[(size_t)(2 * d + s) * M.F * nv];
          lim_face_to_nodes(&M, &L, &frec[(size_t)o * rec_sz + (size_t)(2 * d + 1 - s) * nsf * nv], G);
          Gover[2 * d + s] = G;
        }
      }
    correct_cell(P, &M, &T, c, Qn, params, dt, &CS.vol[(size_t)c * S * nv], NULL, qh, Fh, nb,
                 &Q[(size_t)c * cell_sz], NULL, Gover);
    free(Gbuf);
  }

  if (counts) {
    counts[0] = counts[1] = counts[2] = 0;
    for (long c = 0; c < C; ++c) {
      counts[0] += st[c] == 3;
      counts[1] += st[c] >= 2;
      counts[2] += st[c] == 1;
    }
  }
  memcpy(status, st, C);
  rc = ORC_OK;
done:
  free(CS.vol); free(CS.qhat); free(CS.Fhat); free(Qn); free(Qc); free(Vn); free(lo); free(hi);
  free(frec); free(st);
  return rc;
}

/* Limiter tables for the tests: A [m][n], B [n][m], Qf [n][m]. */
int orc_limiter_tables(int n, double *A, double *B, double *Qf) {
  tables T;
  lim_tables L;
  if (make_tables(n, &T) || make_lim_tables(&T, &L)) return ORC_EINVAL;
  const int m = L.m;
  for (int s = 0; s < m; ++s)
    for (int k = 0; k < n; ++k) {
      A[s * n + k] = L.A[s][k];
      B[k * m + s] = L.B[k][s];
      Qf[k * m + s] = L.Qf[k][s];
    }
  return ORC_OK;
}

/* The FV scheme alone on every cell (status forced to FV everywhere):
 * Q <- projectOnDG(MUSCL-Hancock(projectOnFV(Q))).  For the tests. */
int orc_fv_step(const orc_problem *P, double *Q, double dt, double *subcells_out) {
  mesh M;
  tables T;
  lim_tables L;
  if (P->pde != ORC_EULER) return ORC_EINVAL;
  if (make_mesh(P, &M) || make_tables(M.n, &T) || make_lim_tables(&T, &L)) return ORC_EINVAL;
  const int m = L.m, nv = M.nv, S = M.S, ns = ipow_i(m, M.dim), nsf = ipow_i(m, M.dim - 1);
  const size_t cell_sz = (size_t)nv * S, rec_sz = (size_t)2 * M.dim * nsf * nv;
  double *Vn = malloc(sizeof(double) * M.C * nv * ns);
  if (!Vn) return ORC_ENOMEM;
#pragma omp parallel for
  for (long c = 0; c < M.C; ++c) lim_project(&M, &L, &Q[(size_t)c * cell_sz], &Vn[(size_t)c * nv * ns]);
#pragma omp parallel for schedule(dynamic, 1)
  for (long c = 0; c < M.C; ++c) {
    double *vnew = malloc(sizeof(double) * nv * ns), *frec = malloc(sizeof(double) * rec_sz);
    lim_fv_cell(P, &M, &L, Vn, c, dt, vnew, frec);
    if (subcells_out) memcpy(&subcells_out[(size_t)c * nv * ns], vnew, sizeof(double) * nv * ns);
    lim_reconstruct(&M, &L, vnew, &Q[(size_t)c * cell_sz]);
    free(vnew);
    free(frec);
  }
  free(Vn);
  return ORC_OK;
}

/* Eq. (7) for a run with the subcell limiter.  READING: the solution of an
 * FV cell (status >= 2) is its subcell averages, so its signal speed is
 * taken over those; DG cells use their nodal values as in orc_stable_dt.
 * (The least-squares polynomial of an FV cell is not its solution and can
 * hold non-physical values at nodes.) */
int orc_stable_dt_limited(const orc_problem *P, const double *Q, const double *sub,
                          const unsigned char *status, double *dt, double *lambda_max) {
  mesh M;
  if (P->pde != ORC_EULER || make_mesh(P, &M)) return ORC_EINVAL;
  const int m = 2 * P->order + 1, ns = ipow_i(m, M.dim);
  double lam = 0.0;
  for (long c = 0; c < M.C; ++c) {
    const int fv = status[c] >= 2;
    const int npts = fv ? ns : M.S;
    for (int k = 0; k < npts; ++k) {
      double q[ORC_MAXQ];
      for (int v = 0; v < M.nv; ++v)
        q[v] = fv ? sub[((size_t)c * M.nv + v) * ns + k] : Q[((size_t)c * M.nv + v) * M.S + k];
      for (int d = 0; d < M.dim; ++d) lam = speed_max(lam, pde_max_eigen(P, q, d));
    }
  }
  double h = M.h[0];
  for (int d = 1; d < M.dim; ++d) h = fmin(h, M.h[d]);
  if (lambda_max) *lambda_max = lam;
  *dt = P->cfl / (M.dim * (2.0 * P->order + 1.0)) * h / lam;
  return ORC_OK;
}

// Pointwise PDE terms of Eq. (1) of the ExaHyPE paper for the built-in
// systems, written as device functors templated on the arithmetic type.
//
// Each PDE type provides
//   DIM, NV (evolved quantities), NP (material parameters)
//   flux_nonzero(d, v)  compile-time sparsity of F_d (which components the
//                       kernels must differentiate)
//   grad_needed(v)      which evolved quantities the non-conservative
//                       product reads the gradient of
//   kHasNcp, kHasSource
//   fluxes(Q, P, F)     all directions at once, F[d][v] (only nonzero ones
//                       are read)
//   ncp(Q, P, g, B)     B(Q) . grad Q with g[d][v] = dQ_v/dx_d
//   source(Q, P, S)     smooth source term S(Q)
//   max_eigen(Q, P, d)  largest |eigenvalue| of the direction-d system
//   admissible(Q, P)    physical admissibility (Sec. 3.5) incl. finiteness
// Q points to NV evolved values, P to NP parameter values.
//
// PDEs that are linear in Q (kLinear) also provide the transposes the
// discrete adjoint of the step needs (all accumulate with +=):
//   flux_T(d, pc, lamF, lamQ)        lamQ += (dF_d/dQ)^T lamF
//   ncp_T(P, lamB, lamG)             lamG[d][v] += (dB/d(dQ_v/dx_d))^T lamB
//   ncp_dparams_T(P, g, lamB, gp)    gp += (dB/dP)^T lamB at gradient g
//   source_T(lamS, lamQ)             lamQ += (dS/dQ)^T lamS
//   max_eigen_dparams(P, d, s, gp)   gp += s * d max_eigen(d) / dP
#pragma once

#if !defined(__HIPCC_RTC__)
#include <hip/hip_runtime.h>
#endif

#include "adg_internal.hpp"

namespace adg {

template <class R>
__device__ __forceinline__ R rdiv(R a, R b) {
  return a / b;
}

template <class R>
__device__ __forceinline__ bool finite_val(R x) {
  return __builtin_isfinite(x);
}

// Compressible Euler, Eqs. (8) and (10): Q = (rho, j, E).
template <int DIM_>
struct Euler {
  static constexpr int DIM = DIM_, NV = DIM_ + 2, NP = 0;
  static constexpr bool kHasNcp = false, kHasSource = false, kLinear = false;
  static constexpr bool flux_nonzero(int, int) { return true; }
  static constexpr bool grad_needed(int) { return false; }

  template <class R>
  __device__ static __forceinline__ void fluxes(const R* Q, const R*, const PdeConsts& pc,
                                                R (*F)[NV]) {
    const R gm1 = R(pc.gamma) - R(1);
    const R irho = R(1) / Q[0];
    R jj = R(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) jj += Q[1 + a] * Q[1 + a];
    const R p = gm1 * (Q[DIM + 1] - R(0.5) * jj * irho);
    const R Ep = Q[DIM + 1] + p;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const R ud = Q[1 + d] * irho;
      F[d][0] = Q[1 + d];
#pragma unroll
      for (int a = 0; a < DIM; ++a) F[d][1 + a] = ud * Q[1 + a];
      F[d][1 + d] += p;
      F[d][DIM + 1] = ud * Ep;
    }
  }

  // F_d alone (the same arithmetic as fluxes() for that direction): kernels
  // that store the fluxes one direction at a time keep fewer values live
  template <class R>
  __device__ static __forceinline__ void flux_dir(const R* Q, const R*, const PdeConsts& pc, int d, R* F) {
    const R gm1 = R(pc.gamma) - R(1);
    const R irho = R(1) / Q[0];
    R jj = R(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) jj += Q[1 + a] * Q[1 + a];
    const R p = gm1 * (Q[DIM + 1] - R(0.5) * jj * irho);
    const R Ep = Q[DIM + 1] + p;
    const R ud = Q[1 + d] * irho;
    F[0] = Q[1 + d];
#pragma unroll
    for (int a = 0; a < DIM; ++a) F[1 + a] = ud * Q[1 + a];
    F[1 + d] += p;
    F[DIM + 1] = ud * Ep;
  }

  template <class R>
  __device__ static __forceinline__ void ncp(const R*, const R*, const PdeConsts&,
                                             const R (*)[NV], R* B) {
#pragma unroll
    for (int v = 0; v < NV; ++v) B[v] = R(0);
  }

  template <class R>
  __device__ static __forceinline__ void source(const R*, const R*, const PdeConsts&, R* S) {
#pragma unroll
    for (int v = 0; v < NV; ++v) S[v] = R(0);
  }

  template <class R>
  __device__ static __forceinline__ R pressure(const R* Q, const PdeConsts& pc) {
    R jj = R(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) jj += Q[1 + a] * Q[1 + a];
    return (R(pc.gamma) - R(1)) * (Q[DIM + 1] - R(0.5) * jj / Q[0]);
  }

  // u_d -+ c and u_d: the largest modulus is |u_d| + c, c = sqrt(gamma p / rho)
  template <class R>
  __device__ static __forceinline__ R max_eigen(const R* Q, const R*, const PdeConsts& pc, int d) {
    const R c = sqrt(R(pc.gamma) * pressure(Q, pc) / Q[0]);
    return fabs(Q[1 + d] / Q[0]) + c;
  }

  template <class R>
  __device__ static __forceinline__ bool admissible(const R* Q, const R*, const PdeConsts& pc) {
    bool ok = true;
#pragma unroll
    for (int v = 0; v < NV; ++v) ok = ok && finite_val(Q[v]);
    return ok && Q[0] > R(0) && pressure(Q, pc) > R(0);
  }
};

// Linear elasticity, velocity-stress form of Sec. 2.1:
//   Q = (sxx, syy, szz, sxy, sxz, syz, rho vx, rho vy, rho vz), params (rho, cp, cs)
//   d/dt sigma + E(lambda, mu) grad v = 0,   d/dt (rho v) + div sigma = 0.
struct Elastic3 {
  static constexpr int DIM = 3, NV = 9, NP = 3;
  static constexpr bool kHasNcp = true, kHasSource = false, kLinear = true;
  static constexpr bool flux_nonzero(int, int v) { return v >= 6; }
  static constexpr bool grad_needed(int v) { return v >= 6; }
  static constexpr int sym(int i, int d) {
    return i == d ? i : ((i + d == 1) ? 3 : ((i + d == 2) ? 4 : 5));
  }

  template <class R>
  __device__ static __forceinline__ void fluxes(const R* Q, const R*, const PdeConsts&,
                                                R (*F)[NV]) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
      for (int v = 0; v < 6; ++v) F[d][v] = R(0);
#pragma unroll
      for (int i = 0; i < 3; ++i) F[d][6 + i] = Q[sym(i, d)];
    }
  }

  template <class R>
  __device__ static __forceinline__ void ncp(const R*, const R* P, const PdeConsts&,
                                             const R (*g)[NV], R* B) {
    const R rho = P[0], cp = P[1], cs = P[2];
    const R mu = rho * cs * cs;
    const R lam = rho * cp * cp - R(2) * mu;
    const R ir = R(1) / rho;
    R gv[3][3];  // gv[i][d] = d v_i / d x_d
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int d = 0; d < 3; ++d) gv[i][d] = g[d][6 + i] * ir;
    const R divv = gv[0][0] + gv[1][1] + gv[2][2];
    B[0] = R(2) * mu * gv[0][0] + lam * divv;
    B[1] = R(2) * mu * gv[1][1] + lam * divv;
    B[2] = R(2) * mu * gv[2][2] + lam * divv;
    B[3] = mu * (gv[0][1] + gv[1][0]);
    B[4] = mu * (gv[0][2] + gv[2][0]);
    B[5] = mu * (gv[1][2] + gv[2][1]);
    B[6] = B[7] = B[8] = R(0);
  }

  template <class R>
  __device__ static __forceinline__ void source(const R*, const R*, const PdeConsts&, R* S) {
#pragma unroll
    for (int v = 0; v < NV; ++v) S[v] = R(0);
  }

  // +-cp, +-cs (twice), 0 (three times)
  template <class R>
  __device__ static __forceinline__ R max_eigen(const R*, const R* P, const PdeConsts&, int) {
    return P[1];
  }

  // --- transposes for the adjoint ---------------------------------------
  __device__ static __forceinline__ void flux_T(int d, const PdeConsts&, const double* lamF,
                                                double* lamQ) {
#pragma unroll
    for (int i = 0; i < 3; ++i) lamQ[sym(i, d)] += lamF[6 + i];
  }

  // B = E(lambda, mu) grad(rho v) / rho: the adjoint of the velocity
  // gradient, lamG[d][6 + i] = (E^T lamB)_{i d} / rho.
  __device__ static __forceinline__ void ncp_T(const double* P, const PdeConsts&,
                                               const double* lamB, double (*lamG)[NV]) {
    const double rho = P[0], cp = P[1], cs = P[2];
    const double mu = rho * cs * cs;
    const double lam = rho * cp * cp - 2.0 * mu;
    const double ir = 1.0 / rho;
    const double ldiv = lam * (lamB[0] + lamB[1] + lamB[2]);
    double lg[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) lg[i][i] = 2.0 * mu * lamB[i] + ldiv;
    lg[0][1] = lg[1][0] = mu * lamB[3];
    lg[0][2] = lg[2][0] = mu * lamB[4];
    lg[1][2] = lg[2][1] = mu * lamB[5];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int i = 0; i < 3; ++i) lamG[d][6 + i] += lg[i][d] * ir;
  }

  // derivatives of B with respect to (rho, cp, cs) through mu, lambda and 1/rho
  __device__ static __forceinline__ void ncp_dparams_T(const double* P, const PdeConsts&,
                                                       const double (*g)[NV], const double* lamB,
                                                       double* gp) {
    const double rho = P[0], cp = P[1], cs = P[2];
    const double mu = rho * cs * cs;
    const double lam = rho * cp * cp - 2.0 * mu;
    const double ir = 1.0 / rho;
    double gv[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int d = 0; d < 3; ++d) gv[i][d] = g[d][6 + i] * ir;
    const double divv = gv[0][0] + gv[1][1] + gv[2][2];
    // a = lamB . E(1, 0) gv (the lambda part), b = lamB . E(0, 1) gv (the mu part)
    const double a = (lamB[0] + lamB[1] + lamB[2]) * divv;
    const double b = 2.0 * (lamB[0] * gv[0][0] + lamB[1] * gv[1][1] + lamB[2] * gv[2][2]) +
                     lamB[3] * (gv[0][1] + gv[1][0]) + lamB[4] * (gv[0][2] + gv[2][0]) +
                     lamB[5] * (gv[1][2] + gv[2][1]);
    // d/d rho: dmu = cs^2, dlam = cp^2 - 2 cs^2, and gv scales with -1/rho
    gp[0] += cs * cs * b + (cp * cp - 2.0 * cs * cs) * a - ir * (mu * b + lam * a);
    gp[1] += 2.0 * rho * cp * a;
    gp[2] += 2.0 * rho * cs * b - 4.0 * rho * cs * a;
  }

  __device__ static __forceinline__ void source_T(const PdeConsts&, const double*, double*) {}

  __device__ static __forceinline__ void max_eigen_dparams(const double*, int, double s, double* gp) {
    gp[1] += s;
  }

  template <class R>
  __device__ static __forceinline__ bool admissible(const R* Q, const R* P, const PdeConsts&) {
    bool ok = true;
#pragma unroll
    for (int v = 0; v < NV; ++v) ok = ok && finite_val(Q[v]);
#pragma unroll
    for (int p = 0; p < NP; ++p) ok = ok && finite_val(P[p]);
    return ok;
  }
};

// Scalar advection with linear decay (a test PDE with a closed-form solution).
template <int DIM_>
struct Advection {
  static constexpr int DIM = DIM_, NV = 1, NP = 0;
  static constexpr bool kHasNcp = false, kHasSource = true, kLinear = true;
  static constexpr bool flux_nonzero(int, int) { return true; }
  static constexpr bool grad_needed(int) { return false; }

  template <class R>
  __device__ static __forceinline__ void fluxes(const R* Q, const R*, const PdeConsts& pc,
                                                R (*F)[NV]) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) F[d][0] = R(pc.adv[d]) * Q[0];
  }
  template <class R>
  __device__ static __forceinline__ void ncp(const R*, const R*, const PdeConsts&,
                                             const R (*)[NV], R* B) {
    B[0] = R(0);
  }
  template <class R>
  __device__ static __forceinline__ void source(const R* Q, const R*, const PdeConsts& pc, R* S) {
    S[0] = -R(pc.kappa) * Q[0];
  }
  template <class R>
  __device__ static __forceinline__ R max_eigen(const R*, const R*, const PdeConsts& pc, int d) {
    return fabs(R(pc.adv[d]));
  }

  __device__ static __forceinline__ void flux_T(int d, const PdeConsts& pc, const double* lamF,
                                                double* lamQ) {
    lamQ[0] += pc.adv[d] * lamF[0];
  }
  __device__ static __forceinline__ void ncp_T(const double*, const PdeConsts&, const double*,
                                               double (*)[NV]) {}
  __device__ static __forceinline__ void ncp_dparams_T(const double*, const PdeConsts&,
                                                       const double (*)[NV], const double*, double*) {}
  __device__ static __forceinline__ void source_T(const PdeConsts& pc, const double* lamS,
                                                  double* lamQ) {
    lamQ[0] += -pc.kappa * lamS[0];
  }
  __device__ static __forceinline__ void max_eigen_dparams(const double*, int, double, double*) {}
  template <class R>
  __device__ static __forceinline__ bool admissible(const R* Q, const R*, const PdeConsts&) {
    return finite_val(Q[0]);
  }
};

// Wall boundary condition per PDE: the outside state and normal flux of a
// wall face with normal e_d from the inside traces (qin, Fin).
template <class PDE>
struct Wall;

// Euler: the mirror image, R = normal momentum reversed; qout = R qin and,
// as F_d(R q) = -R F_d(q), Fout = -R Fin (a reflecting wall).
template <int DIM_>
struct Wall<Euler<DIM_>> {
  static constexpr int NV = Euler<DIM_>::NV;
  __device__ static __forceinline__ void apply(int d, const double* qin, const double* Fin, double* qout,
                                               double* Fout) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const bool normal = v == 1 + d;
      qout[v] = normal ? -qin[v] : qin[v];
      Fout[v] = normal ? Fin[v] : -Fin[v];
    }
  }
};

// Elasticity: the traction sigma_{i d} reversed, the velocity kept (a
// traction-free surface); the flux is linear, Fout = -Fin.
template <>
struct Wall<Elastic3> {
  static constexpr int NV = Elastic3::NV;
  __device__ static __forceinline__ void apply(int d, const double* qin, const double* Fin, double* qout,
                                               double* Fout) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const bool traction = v == Elastic3::sym(0, d) || v == Elastic3::sym(1, d) || v == Elastic3::sym(2, d);
      qout[v] = traction ? -qin[v] : qin[v];
      Fout[v] = -Fin[v];
    }
  }
};

// The advection PDE has no wall condition (refused at context creation).
template <int DIM_>
struct Wall<Advection<DIM_>> {
  __device__ static __forceinline__ void apply(int, const double* qin, const double* Fin, double* qout,
                                               double* Fout) {
    qout[0] = qin[0];
    Fout[0] = Fin[0];
  }
};

}  // namespace adg

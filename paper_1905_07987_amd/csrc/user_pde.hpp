// A PDE supplied at run time as HIP source text (adg_create_user), adapted
// to the kernels' PDE concept.  The user writes the pointwise terms of
// Eq. (1) the way the paper's Table 2 lists them, with the (Q, direction,
// out) convention of its printed eigenvalues signature, as static member
// templates of a struct named AdgUserPDE:
//
//   struct AdgUserPDE {
//     static constexpr int DIM = 2 or 3, NV = evolved quantities,
//                          NP = material parameters per cell;
//     static constexpr bool LINEAR = flux, ncp and source linear and
//                                    homogeneous in the evolved quantities,
//                           HAS_NCP, HAS_SOURCE;
//     template <class R> __device__ static void flux(const R* Q, int d, R* F);
//     template <class R> __device__ static void eigenvalues(const R* Q, int d, R* lam);
//     template <class R> __device__ static void ncp(const R* Q, const R* gradQ, R* BgradQ);
//     template <class R> __device__ static void source(const R* Q, R* S);
//     template <class R> __device__ static bool admissible(const R* Q);
//     // optional, for ADG_BC_USER faces (the paper's boundaryValues):
//     static constexpr bool HAS_BOUNDARY = true;
//     __device__ static void boundary_values(const double* x, double t, double dt, int face,
//                                            const double* Qin, const double* Fin,
//                                            double* Qout, double* Fout);
//   };
//
// Q holds the NV evolved quantities followed by the cell's NP parameters;
// F (the flux along axis d), lam (the NV eigenvalues along d), BgradQ and S
// have NV entries; gradQ is [DIM][NV] (gradQ[d * NV + v] = dQ_v / dx_d).
// R is double, or float in the mixed-precision predictor.  The kernels use
// the largest absolute eigenvalue; admissible() is checked after finiteness.
// boundary_values gets, at a node of a boundary face 2 d + side, the node's
// position x[DIM], the step's start time t and size dt, the cell's own
// time-averaged state (Qin, NV values and the NP parameters) and normal
// flux (Fin, NV values) there, and returns the outside state and normal
// flux (NV values each).
#pragma once

#include "kernels.hpp"

namespace adg {

template <class... T>
using adg_void_t = void;

template <class U, class = void>
struct UserHasBoundary {
  static constexpr bool value = false;
};
template <class U>
struct UserHasBoundary<U, adg_void_t<decltype(U::HAS_BOUNDARY)>> {
  static constexpr bool value = U::HAS_BOUNDARY;
};

template <class U>
struct UserTerms {
  static_assert(U::DIM == 2 || U::DIM == 3, "AdgUserPDE::DIM must be 2 or 3");
  static_assert(U::NV >= 1 && U::NP >= 0 && U::NV + U::NP <= kMaxVar,
                "AdgUserPDE: NV + NP must be in 1..16");
  static constexpr int DIM = U::DIM, NV = U::NV, NP = U::NP;
  static constexpr bool kHasNcp = U::HAS_NCP, kHasSource = U::HAS_SOURCE, kLinear = U::LINEAR;
  static constexpr bool kUserBoundary = UserHasBoundary<U>::value;
  static constexpr bool flux_nonzero(int, int) { return true; }
  static constexpr bool grad_needed(int) { return U::HAS_NCP; }

  template <class R>
  __device__ static __forceinline__ void gather(const R* Q, const R* P, R (&q)[NV + NP]) {
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = Q[v];
#pragma unroll
    for (int p = 0; p < NP; ++p) q[NV + p] = P[p];
  }

  template <class R>
  __device__ static __forceinline__ void fluxes(const R* Q, const R* P, const PdeConsts&, R (*F)[NV]) {
    R q[NV + NP];
    gather(Q, P, q);
#pragma unroll
    for (int d = 0; d < DIM; ++d) U::flux(q, d, F[d]);
  }

  template <class R>
  __device__ static __forceinline__ void ncp(const R* Q, const R* P, const PdeConsts&, const R (*g)[NV],
                                             R* B) {
    if constexpr (U::HAS_NCP) {
      R q[NV + NP];
      gather(Q, P, q);
      U::ncp(q, &g[0][0], B);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) B[v] = R(0);
    }
  }

  template <class R>
  __device__ static __forceinline__ void source(const R* Q, const R* P, const PdeConsts&, R* S) {
    if constexpr (U::HAS_SOURCE) {
      R q[NV + NP];
      gather(Q, P, q);
      U::source(q, S);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) S[v] = R(0);
    }
  }

  template <class R>
  __device__ static __forceinline__ R max_eigen(const R* Q, const R* P, const PdeConsts&, int d) {
    R q[NV + NP], lam[NV];
    gather(Q, P, q);
    U::eigenvalues(q, d, lam);
    // the largest |eigenvalue|; a NaN eigenvalue is kept (fmax would drop it)
    R m = R(0);
    bool nan = false;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const R x = fabs(lam[v]);
      nan = nan || x != x;
      m = fmax(m, x);
    }
    return nan ? R(__builtin_nan("")) : m;
  }

  __device__ static __forceinline__ void boundary(const double* x, double t, double dt, int face,
                                                  const double* qin, const double* P, const double* Fin,
                                                  double* qout, double* Fout) {
    if constexpr (kUserBoundary) {
      double q[NV + NP];
      gather(qin, P, q);
      U::boundary_values(x, t, dt, face, q, Fin, qout, Fout);
    }
  }

  template <class R>
  __device__ static __forceinline__ bool admissible(const R* Q, const R* P, const PdeConsts&) {
    bool ok = true;
#pragma unroll
    for (int v = 0; v < NV; ++v) ok = ok && finite_val(Q[v]);
    if (!ok) return false;
    R q[NV + NP];
    gather(Q, P, q);
    return U::admissible(q);
  }
};

// Walls are not defined for a user PDE (refused at context creation); the
// corrector's wall branch is never taken.
template <class U>
struct Wall<UserTerms<U>> {
  __device__ static __forceinline__ void apply(int, const double* qin, const double* Fin, double* qout,
                                               double* Fout) {
#pragma unroll
    for (int v = 0; v < U::NV; ++v) {
      qout[v] = qin[v];
      Fout[v] = Fin[v];
    }
  }
};

}  // namespace adg

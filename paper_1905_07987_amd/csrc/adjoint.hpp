// Discrete adjoint of one ADER-DG step for the PDEs that are linear in Q
// (elasticity and the advection test PDE), with the step size held fixed.
// Included by kernels.hpp after the forward kernels, whose helpers it uses.
//
// The step maps (u^n, m) to u^{n+1}, m the per-cell material parameters.
// Given lam = dJ/du^{n+1}, the adjoint step overwrites lam with
// dJ/du^n = (du^{n+1}/du^n)^T lam and adds (du^{n+1}/dm)^T lam to the
// parameter gradient.  Inner products are the plain Euclidean ones over the
// nodal arrays.  Linearity in Q gives three exact identities (up to rounding)
// that shape the kernels:
//  - the corrector's time averages depend on the predictor only through
//    qbar = sum_j w_j q_j: Fbar_d = F_d(qbar), the averaged non-conservative
//    product is B grad qbar and Sbar = S(qbar) plus the point sources, which
//    depend on neither u nor m;
//  - the face trace of Fbar_d is F_d of the face trace of qbar, so the adjoint
//    of the flux trace folds into the adjoint of the state trace;
//  - the Rusanov flux is linear in the traces with coefficients that depend
//    on the parameters only (max_eigen does not read Q for these PDEs); its
//    transpose needs no traces, its parameter derivative does.
// Reading: the derivative of the max() in the Rusanov speed is split half
// and half between the two cells on a tie.
//
// Launch sequence on the caller's stream; work holds two face arrays
// A and B of [C][2 dim][NV][F] doubles (face = 2 d + side, side 1 = high):
//  1. adj_face_project_kernel: A = sum_m l_side(m) / w_m lam(line f, m), the
//     face projections of lam that the surface integral's transpose needs.
//  2. adj_rusanov_kernel<true, false>: B = adjoint of each cell's own face
//     traces (state trace plus folded flux trace) from the fluctuation
//     adjoints of both cells of the face.
//  3. adj_predict_lin_kernel: per cell, the linear predictor's Horner sweep
//     forward from u^n (keeping the iterates' gradient quantities), then the
//     transposes of the face projection, the volume term and the Horner
//     steps in reverse order; lam <- lam^n, gparams += the cell's volume
//     terms, B <- face traces of qbar (after B's adjoints have been read).
//  4. adj_rusanov_kernel<false, true> (PDEs with parameters): gparams += the
//     Rusanov flux's parameter derivative at every face of the cell.
// From a kept forward step (KArgs::keep: the Horner quantities and, behind
// them, the step's face traces of qbar) the sequence is 1; then
// adj_rusanov_kernel<true, true>, which writes B and each cell's face terms
// of the parameter gradient (gface, C x nparam doubles behind A and B) in
// one pass, the qbar traces being the kept ones; then 3 without the forward
// sweep and without B's qbar traces, adding gface after the cell's volume
// terms (the state path's order of the two sums).
#pragma once

namespace adg {

// Value of f(i) for a lane-dependent index i < n, built from compile-time
// constants (a select chain; no memory access).
template <int n, class Fn>
__device__ __forceinline__ double ct_pick(int i, Fn f) {
  double r = f(0);
#pragma unroll
  for (int ii = 1; ii < n; ++ii) r = (i == ii) ? f(ii) : r;
  return r;
}

// Face kernels: one thread per (cell, face, face node); CPB_R cells per block.
template <class PDE, int N>
struct GeoAdjR {
  using G = Geo<PDE, N>;
  static constexpr int TPF = 2 * G::DIM * G::F;  // tasks per cell
  static constexpr int CPB = TPF >= 256 ? 1 : 256 / TPF;
  static constexpr int BLOCK = cmin(256, (CPB * TPF + 63) / 64 * 64);  // no idle wave
};

// face node f of the faces normal to d, position m along d -> node index
template <int DIM, int n>
__device__ __forceinline__ int face_line_node(int d, int f, int m) {
  if (DIM == 2) return d == 0 ? f * n + m : f + n * m;
  return d == 0 ? n * f + m : (d == 1 ? (f % n) + n * m + n * n * (f / n) : f + n * n * m);
}

// ---------------------------------------------------------------------------
// 1. Face projections of lam: A[c][face][v][f] = sum_m l_side(m) / w_m lam.
// Each lam value lies on the lines of 2 DIM faces; a block stages its cells'
// lam in LDS with contiguous loads (each value read from HBM once) and
// writes the projections in A's order (contiguous stores).
// ---------------------------------------------------------------------------
template <class PDE, int N>
struct GeoAdjP {
  using G = Geo<PDE, N>;
  static constexpr int CELL = G::NV * G::S;                // lam values per cell
  static constexpr int OUT = 2 * G::DIM * G::NV * G::F;    // projections per cell
  static constexpr int CPB = cmax(1, cmin(8, 1152 / CELL));
  static constexpr int BLOCK = 256;
};

template <class PDE, int N>
__global__ void __launch_bounds__(256)
adj_face_project_kernel(const KArgs a, const double* __restrict__ lam, double* __restrict__ A) {
  using G = Geo<PDE, N>;
  using GP = GeoAdjP<PDE, N>;
  using T = CT<double, G::n>;
  constexpr int n = G::n, S = G::S, F = G::F, NV = G::NV, DIM = G::DIM;
  constexpr int CELL = GP::CELL, OUT = GP::OUT, CPB = GP::CPB;
  __shared__ double sl[CPB * CELL];
  const long long cell0 = (long long)blockIdx.x * CPB;
  const int here = (int)(a.ncells - cell0 < CPB ? a.ncells - cell0 : CPB);
  const double* src = lam + cell0 * CELL;
  for (int i = threadIdx.x; i < here * CELL; i += GP::BLOCK) sl[i] = src[i];
  __syncthreads();
  for (int c2 = 0; c2 < here; ++c2) {
    double* dst = A + (cell0 + c2) * OUT;
    for (int r = threadIdx.x; r < OUT; r += GP::BLOCK) {
      const int f = r % F, v = (r / F) % NV, face = r / (F * NV);
      const int d = face >> 1, side = face & 1;
      const double* row = sl + c2 * CELL + v * S;
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < n; ++m)
        acc += (side ? T::l1(m) : T::l0(m)) * (1.0 / T::w(m)) * row[face_line_node<DIM, n>(d, f, m)];
      dst[r] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// 2./4. Rusanov flux in reverse.  OUT: B <- adjoint of the cell's own face
// traces.  GRAD: the flux's parameter derivative, the face traces of qbar
// read from tq (face stride tq_face doubles: NV F for B, 2 NV F for the
// forward trace array), added to gp (GRAD only) or written to gp (OUT and
// GRAD: the per-cell face terms that the predictor adjoint adds).
//
// Forward, at the face with normal e_d between L (low) and R (high):
//   s = max(lambda*(pL), lambda*(pR)), G = (FL + FR)/2 - s (qR - qL)/2,
//   Bm = B_d(pm) (qR - qL) / 2 with pm = (pL + pR)/2,
//   flL = G - FL + Bm (into L's high face), flR = FR - G + Bm (into R's low
//   face), each scaled by dt / h_d in the update u -= l flL / w ...
// ---------------------------------------------------------------------------
template <class PDE, int N, bool OUT, bool GRAD>
__global__ void __launch_bounds__(256)
adj_rusanov_kernel(const KArgs a, const double* __restrict__ params, const double* __restrict__ clock,
                   const double* __restrict__ A, const double* __restrict__ tq, int tq_face,
                   double* __restrict__ B, double* __restrict__ gp_out) {
  using G = Geo<PDE, N>;
  using GR = GeoAdjR<PDE, N>;
  constexpr int F = G::F, NV = G::NV, NP = G::NP, DIM = G::DIM;
  constexpr int NPX = NP > 0 ? NP : 1;
  constexpr int TPF = GR::TPF, CPB = GR::CPB;
  __shared__ double contrib[GRAD ? CPB * TPF * NPX : 1];
  const int tid = threadIdx.x;
  const long long cell0 = (long long)xcd_block(blockIdx.x, a.nblocks) * CPB;
  const double dt = clock[1];
  const int C0 = a.cells[0], C1 = a.cells[1];

  for (int task = tid; task < CPB * TPF; task += GR::BLOCK) {
    const int f = task % F;
    const int face = (task / F) % (2 * DIM);
    const int c2 = task / TPF;
    const long long c = cell0 + c2;
    double gp[NPX];
#pragma unroll
    for (int p = 0; p < NPX; ++p) gp[p] = 0.0;
    if (c < a.ncells) {
      const int d = face >> 1, side = face & 1;
      long long cc[3];
      cc[0] = c % C0;
      cc[1] = (c / C0) % C1;
      cc[2] = DIM == 3 ? c / ((long long)C0 * C1) : 0;
      cc[d] += side ? 1 : -1;
      if (cc[d] < 0) cc[d] += a.cells[d];
      if (cc[d] >= a.cells[d]) cc[d] -= a.cells[d];
      const long long nb = cc[0] + C0 * (cc[1] + (long long)C1 * cc[2]);
      const long long cL = side ? c : nb, cR = side ? nb : c;
      const double scale = -dt * a.inv_h[d];
      const double* aL = A + ((cL * (2 * DIM) + 2 * d + 1) * NV) * F + f;
      const double* aR = A + ((cR * (2 * DIM) + 2 * d + 0) * NV) * F + f;
      double lL[NV], lR[NV], lG[NV], lBm[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        lL[v] = scale * aL[v * F];
        lR[v] = scale * aR[v * F];
        lG[v] = lL[v] - lR[v];
        lBm[v] = 0.5 * (lL[v] + lR[v]);
      }
      double pL[NPX] = {}, pR[NPX] = {}, pm[NPX] = {}, qz[NV];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        pL[p] = params[cL * NP + p];
        pR[p] = params[cR * NP + p];
        pm[p] = 0.5 * (pL[p] + pR[p]);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) qz[v] = 0.0;
      const double sL = PDE::max_eigen(qz, pL, a.pde, d), sR = PDE::max_eigen(qz, pR, a.pde, d);
      if constexpr (OUT) {
        const double s = fmax(sL, sR);
        double ld[NV], lF[NV], out[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          ld[v] = -0.5 * s * lG[v];
          lF[v] = side ? (-lL[v] + 0.5 * lG[v]) : (lR[v] + 0.5 * lG[v]);
        }
        if constexpr (PDE::kHasNcp) {
          double lg[DIM][NV];
#pragma unroll
          for (int e = 0; e < DIM; ++e)
#pragma unroll
            for (int v = 0; v < NV; ++v) lg[e][v] = 0.0;
          PDE::ncp_T(pm, a.pde, lBm, lg);
#pragma unroll
          for (int e = 0; e < DIM; ++e)
            if (e == d) {
#pragma unroll
              for (int v = 0; v < NV; ++v) ld[v] += lg[e][v];
            }
        }
        // qR enters with +ld, qL with -ld
#pragma unroll
        for (int v = 0; v < NV; ++v) out[v] = side ? -ld[v] : ld[v];
        PDE::flux_T(d, a.pde, lF, out);
        double* o = B + ((c * (2 * DIM) + face) * NV) * F + f;
#pragma unroll
        for (int v = 0; v < NV; ++v) o[v * F] = out[v];
      }
      if constexpr (GRAD) {
        const double* tL = tq + (cL * (2 * DIM) + 2 * d + 1) * tq_face + f;
        const double* tR = tq + (cR * (2 * DIM) + 2 * d + 0) * tq_face + f;
        double jump[NV], ls = 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          jump[v] = tR[v * F] - tL[v * F];
          ls += -0.5 * jump[v] * lG[v];
        }
        const double mine = side ? sL : sR, other = side ? sR : sL;
        const double share = mine > other ? 1.0 : (mine == other ? 0.5 : 0.0);
        PDE::max_eigen_dparams(side ? pL : pR, d, share * ls, gp);
        if constexpr (PDE::kHasNcp) {
          double g[DIM][NV], gpm[NPX];
#pragma unroll
          for (int e = 0; e < DIM; ++e)
#pragma unroll
            for (int v = 0; v < NV; ++v) g[e][v] = e == d ? jump[v] : 0.0;
#pragma unroll
          for (int p = 0; p < NPX; ++p) gpm[p] = 0.0;
          PDE::ncp_dparams_T(pm, a.pde, g, lBm, gpm);
#pragma unroll
          for (int p = 0; p < NP; ++p) gp[p] += 0.5 * gpm[p];
        }
      }
    }
    if constexpr (GRAD) {
#pragma unroll
      for (int p = 0; p < NPX; ++p) contrib[task * NPX + p] = gp[p];
    }
  }
  if constexpr (GRAD) {
    __syncthreads();
    // fixed-order sum per (cell, parameter): deterministic
    if (tid < CPB * NP) {
      const int c2 = tid / NP, p = tid - c2 * NP;
      const long long c = cell0 + c2;
      if (c < a.ncells) {
        double s = 0.0;
        for (int i = 0; i < TPF; ++i) s += contrib[(c2 * TPF + i) * NPX + p];
        if constexpr (OUT) gp_out[c * NP + p] = s;
        else gp_out[c * NP + p] += s;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 3. Predictor adjoint in the polynomial form of the linear predictor: the
// forward step's time average is t_0 of Horner's scheme
//   t_I = c_I u;  t_k = c_k u + dt e_{k+1} w + dt L(m) t_{k+1},
// and the volume term dt (L qbar + e_0 w).  Its transpose runs the same
// recursion backwards with L^T:
//   mu_0 = E^T hat + dt L^T lam       (E = extrapolation to the faces)
//   for k = 0..I-1:  lam_u += c_k mu_k;  gp += (d(L t_{k+1})/dm)^T (dt mu_k);
//                    mu_{k+1} = dt L^T mu_k
//   lam_u += c_I mu_I;  lam^n = lam + lam_u
// plus gp += (d(L qbar)/dm)^T (dt lam).  A forward sweep recomputes the t_k
// and keeps, in registers, the quantities whose gradient the parameter
// terms read (those of the non-conservative product); each L^T application
// differentiates them in the same LDS round.  One thread per node; the
// adjoint's Picard count is at most n, so the sweeps unroll.
// ---------------------------------------------------------------------------
template <class PDE, int N>
struct GeoAdjL {
  using G = Geo<PDE, N>;
  using C = Chan<PDE>;
  // rows of L^T with the forward-gradient channels, qbar, gradient partials
  static constexpr int CELL_ELEMS = cmax(cmax((C::NCH + G::DIM * C::ngrad()) * LinLayout<G>::SP, G::NV * G::S),
                                         G::S * (G::NP > 0 ? G::NP : 1));
  static constexpr int by_threads = G::S >= 256 ? 1 : 256 / G::S;
  static constexpr int by_lds = cmax(1, (76 * 1024) / (CELL_ELEMS * 8));
  static constexpr int CPB = cmin(by_threads, by_lds);
  static constexpr int BLOCK = CPB * G::S;
  static constexpr bool supported = PDE::kLinear && C::uniform() && BLOCK >= 64 && BLOCK <= 1024 &&
                                    CPB * CELL_ELEMS * 8 <= 150 * 1024;
  static constexpr int MIN_WAVES = 2;
};

template <class PDE, int N>
__global__ void __launch_bounds__((GeoAdjL<PDE, N>::BLOCK), (GeoAdjL<PDE, N>::MIN_WAVES))
adj_predict_lin_kernel(const KArgs a, const double* __restrict__ Q, const double* __restrict__ params,
                       const double* __restrict__ clock, double* __restrict__ lam,
                       double* __restrict__ gparams, double* __restrict__ hat,
                       const double* __restrict__ gface) {
  using G = Geo<PDE, N>;
  using C = Chan<PDE>;
  using GA = GeoAdjL<PDE, N>;
  using T = CT<double, G::n>;
  using Op = LinOp<PDE, N, double, GA::CPB, GA::BLOCK, GA::CELL_ELEMS>;
  static_assert(GA::supported, "adjoint not available for this PDE and order");
  constexpr int n = G::n, S = G::S, F = G::F, NV = G::NV, NP = G::NP, DIM = G::DIM;
  constexpr int CPB = GA::CPB, BLOCK = GA::BLOCK;
  constexpr int NGR = C::ngrad(), NGX = NGR > 0 ? NGR : 1, NPX = NP > 0 ? NP : 1;
  constexpr int IMAX = n;  // the adjoint step takes at most n Picard iterations
  __shared__ double lds[GA::CPB * GA::CELL_ELEMS];
  __shared__ double src_e[kMaxSources][kMaxLin + 1];

  const int tid = threadIdx.x;
  const int lc = tid / S, k = tid - lc * S;
  int kk3[3] = {0, 0, 0};
  node_coords<DIM>(k, n, kk3);
  int ln[DIM], pk[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    ln[d] = G::line_of(d, kk3[0], kk3[1], DIM == 3 ? kk3[2] : 0);
    pk[d] = LinLayout<G>::addr(d, ln[d], kk3[d]);
  }
  const long long cell0 = (long long)xcd_block(blockIdx.x, a.nblocks) * CPB;
  const long long cell = cell0 + lc;
  const bool active = cell < a.ncells;
  const long long cl = active ? cell : a.ncells - 1;  // clamp loads of the ragged tail
  double* const mine = lds + lc * GA::CELL_ELEMS;

  const double t_n = clock[0], dt = clock[1];
  const int I = a.picard_iters;
  // a.keep: the forward step's quantities (Horner's iterates' gradient
  // channels and qbar) were kept by that step; Q is not read
  using KG = KeepGeo<PDE, N>;
  const double* const keep = a.keep ? a.keep + cl * (long long)(KG::SLOTS * S) + k : nullptr;
  double P[NPX], u[NV], inv_h[3];
#pragma unroll
  for (int p = 0; p < NPX; ++p) P[p] = p < NP ? params[cl * NP + p] : 0.0;
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = keep ? 0.0 : Q[(cl * NV + v) * S + k];
#pragma unroll
  for (int d = 0; d < 3; ++d) inv_h[d] = a.inv_h[d];

  bool src_here = false;
  for (int s = 0; s < a.nsrc; ++s)
    src_here = src_here || (a.src[s].cell >= cell0 && a.src[s].cell < cell0 + CPB);
  if (src_here && tid < a.nsrc) lin_source_weights<n>(a, tid, t_n, dt, I, src_e[tid]);
  if (src_here) __syncthreads();  // src_e for every wave of the block
  auto add_sources = [&](int kk, double scale, double* t) {
    if (!src_here) return;
    for (int s = 0; s < a.nsrc; ++s) {
      if (a.src[s].cell != cell) continue;
      const double e = scale * src_e[s][kk];
      const double* wsk = a.src_w + ((long long)s * S + k) * NV;
#pragma unroll
      for (int v = 0; v < NV; ++v) t[v] += e * wsk[v];
    }
  };
  // gp += (dB/dm at gradient gq)^T (-nu): the parameter derivative of L t
  // for the gradients gq of t
  auto param_terms = [&](const double (&gq)[DIM][NV], const double (&nu)[NV], double (&gp)[NPX]) {
    if constexpr (PDE::kHasNcp) {
      double lB[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) lB[v] = -nu[v];
      PDE::ncp_dparams_T(P, a.pde, gq, lB, gp);
    }
  };

  // ---- forward sweep: t_k, keeping the gradient quantities of t_{k+1} ----
  double fwv[IMAX][NGX];
  double t[NV];
  if (keep) {
#pragma unroll
    for (int kk = 0; kk < IMAX; ++kk)
#pragma unroll
      for (int c = 0; c < NGX; ++c) fwv[kk][c] = c < NGR && kk < I ? keep[(kk * KG::NGR + c) * S] : 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) t[v] = keep[(KG::QBAR + v) * S];
  } else {
    const double cI = a.lin_c[I];
#pragma unroll
    for (int v = 0; v < NV; ++v) t[v] = cI * u[v];
#pragma unroll
    for (int kk = IMAX - 1; kk >= 0; --kk) {
      if (kk < I) {
#pragma unroll
        for (int c = 0; c < NGX; ++c) fwv[kk][c] = c < NGR ? t[C::grad_var(c)] : 0.0;
        double Lt[NV], g[DIM][NV];
        Op::apply(a, lds, mine, pk, tid, t, P, inv_h, Lt, g);
        const double ck = a.lin_c[kk];
#pragma unroll
        for (int v = 0; v < NV; ++v) t[v] = ck * u[v] + dt * Lt[v];
        add_sources(kk + 1, dt, t);
      }
    }
  }

  // ---- adjoint of the face traces (read hat before it is overwritten) ----
  double tseed[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) tseed[v] = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d)
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const double l = ct_pick<n>(kk3[d], [&](int i) { return side ? T::l1(i) : T::l0(i); });
      const double* h = hat + ((cl * (2 * DIM) + 2 * d + side) * NV) * F + ln[d];
#pragma unroll
      for (int v = 0; v < NV; ++v) tseed[v] += l * h[v * F];
    }

  // ---- face traces of qbar = t into hat (for the Rusanov parameter
  // derivative; a kept step's are the forward step's own) ----
  if (NP > 0 && !keep) {
    Op::sync();  // the forward sweep's last read-backs are done
#pragma unroll
    for (int v = 0; v < NV; ++v) mine[v * S + k] = t[v];
    Op::sync();  // also: every read of hat above is done
    Op::template cell_tasks<DIM * NV * F>(tid, [&](int c2, int it) {
      const int f = it % F, v = (it / F) % NV, d = it / (F * NV);
      const long long tcell = cell0 + c2;
      if (tcell >= a.ncells) return;
      const int st = face_line_node<DIM, n>(d, 0, 1) - face_line_node<DIM, n>(d, 0, 0);
      double e0, e1;
      line_ends<double, n>(lds + c2 * GA::CELL_ELEMS + v * S + face_line_node<DIM, n>(d, f, 0), st, e0, e1);
      double* h = hat + tcell * (2 * DIM * NV * F) + v * F + f;
      h[(2 * d) * NV * F] = e0;
      h[(2 * d + 1) * NV * F] = e1;
    });
    Op::sync();
  }

  // ---- volume term: mu_0 = dt L^T lam + E^T hat; parameter term at qbar ----
  double nu[NV], mu[NV], gp[NPX], lu[NV];
#pragma unroll
  for (int p = 0; p < NPX; ++p) gp[p] = 0.0;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    nu[v] = dt * lam[(cl * NV + v) * S + k];
    lu[v] = 0.0;
  }
  {
    double fq[NGX], gq[DIM][NV];
#pragma unroll
    for (int c = 0; c < NGX; ++c) fq[c] = c < NGR ? t[C::grad_var(c)] : 0.0;
    Op::template apply_T<true>(a, lds, mine, pk, tid, nu, P, inv_h, mu, fq, gq);
    param_terms(gq, nu, gp);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) mu[v] += tseed[v];

  // ---- reverse sweep ----
#pragma unroll
  for (int kk = 0; kk < IMAX; ++kk) {
    if (kk < I) {
      const double ck = a.lin_c[kk];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        lu[v] += ck * mu[v];
        nu[v] = dt * mu[v];
      }
      double gq[DIM][NV];
      Op::template apply_T<true>(a, lds, mine, pk, tid, nu, P, inv_h, mu, fwv[kk], gq);
      param_terms(gq, nu, gp);
    }
  }
  {
    const double cI = a.lin_c[I];
#pragma unroll
    for (int v = 0; v < NV; ++v) lu[v] += cI * mu[v];
  }

  // ---- lam^n = lam^{n+1} + lam_u; the cell's parameter terms ----
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) lam[(cell * NV + v) * S + k] += lu[v];
  }
  if constexpr (NP > 0) {
    Op::sync();  // the reverse sweep's last read-backs are done
#pragma unroll
    for (int p = 0; p < NP; ++p) mine[k * NP + p] = gp[p];
    Op::sync();
    if (k < NP && active) {
      double s = 0.0;
      for (int i = 0; i < S; ++i) s += mine[i * NP + k];
      double g = gparams[cell * NP + k] + s;
      if (gface) g += gface[cell * NP + k];  // the face terms after the volume terms
      gparams[cell * NP + k] = g;
    }
  }
}

#if !defined(__HIPCC_RTC__)
// Launch sequence of one adjoint step.
template <class PDE, int N>
struct AdjLaunch {
  using G = Geo<PDE, N>;
  using GR = GeoAdjR<PDE, N>;
  static hipError_t run(const KArgs& a0, const double* Q, const double* params, const double* clock,
                        double* lam, double* gparams, double* work, hipStream_t st) {
    constexpr long long face_elems = 2LL * G::DIM * G::NV * G::F;
    constexpr int NP = G::NP;
    double* A = work;
    double* B = work + a0.ncells * face_elems;
    // kept step: its face traces of qbar follow the keep buffer's node slots
    const bool kept = a0.keep != nullptr;
    const double* tq = kept ? a0.keep + a0.ncells * (long long)(KeepGeo<PDE, N>::SLOTS * G::S) : B;
    double* gface = kept && NP > 0 ? work + 2 * a0.ncells * face_elems : nullptr;
    KArgs a = a0;
    using GPj = GeoAdjP<PDE, N>;
    hipLaunchKernelGGL((adj_face_project_kernel<PDE, N>), dim3((unsigned)((a0.ncells + GPj::CPB - 1) / GPj::CPB)),
                       dim3(GPj::BLOCK), 0, st, a, lam, A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    a.nblocks = (int)((a0.ncells + GR::CPB - 1) / GR::CPB);
    bool fused = false;
    if constexpr (NP > 0) {
      if (kept) {
        hipLaunchKernelGGL((adj_rusanov_kernel<PDE, N, true, true>), dim3(a.nblocks), dim3(GR::BLOCK), 0, st,
                           a, params, clock, A, tq, (int)(2 * G::NV * G::F), B, gface);
        fused = true;
      }
    }
    if (!fused)
      hipLaunchKernelGGL((adj_rusanov_kernel<PDE, N, true, false>), dim3(a.nblocks), dim3(GR::BLOCK), 0, st,
                         a, params, clock, A, nullptr, 0, B, nullptr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    KArgs ap = a0;
    using GL = GeoAdjL<PDE, N>;
    ap.nblocks = (int)((a0.ncells + GL::CPB - 1) / GL::CPB);
    hipLaunchKernelGGL((adj_predict_lin_kernel<PDE, N>), dim3(ap.nblocks), dim3(GL::BLOCK), 0, st, ap, Q,
                       params, clock, lam, gparams, B, gface);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if constexpr (NP > 0) {
      if (!kept) {
        hipLaunchKernelGGL((adj_rusanov_kernel<PDE, N, false, true>), dim3(a.nblocks), dim3(GR::BLOCK), 0, st,
                           a, params, clock, A, tq, (int)(G::NV * G::F), nullptr, gparams);
        e = hipGetLastError();
      }
    }
    return e;
  }
};
#endif

}  // namespace adg

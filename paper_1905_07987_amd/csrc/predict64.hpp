// FP64 space-time predictor with one thread per spatial node and the whole
// time history of the node in that thread's registers (ExaHyPE paper,
// Sec. 3.3, Eq. (5): q^{r+1}_i = u^n + dt sum_j (K1^{-1})_ij w_j R(q^r)_j).
//
// Because every lane of a wave owns all n time slices, the coefficients of
// the time operator are the same for every lane: they are compile-time
// constants and live in scalar registers, and the Picard update needs no
// exchange between lanes.  A cell of n^3 <= 256 nodes is one block of at most
// four waves; several blocks share a compute unit (three at n = 6, where the
// LDS rows and 168 registers per lane set the bound) so that one block's
// barriers are covered by the others' work.
//
// Spatial derivatives go through LDS: the node threads write the fluxes (and
// the quantities the non-conservative product differentiates) of two time
// slices as one 16-byte element per (channel, node) into line-major rows
// (one slice in 8-byte elements for 3-D cells of 4^3 nodes, whose waves are
// bounded by LDS), one thread per (direction, channel, line) differentiates
// its line in place, and the node threads read their derivatives back.
#pragma once

namespace adg {

#ifndef N64_SINGLE_WAVES
#define N64_SINGLE_WAVES 4
#endif

template <class PDE, int N>
struct GeoN64 {
  using G = Geo<PDE, N>;
  using C = Chan<PDE>;
  static constexpr int n = G::n, S = G::S, F = G::F, DIM = G::DIM, NV = G::NV;
  // Cells of fewer than 64 nodes share a wave.
  static constexpr int CPB = S >= 64 ? 1 : 64 / S;
  static constexpr int LANES = CPB * S;
  static constexpr int BLOCK = (LANES + 63) / 64 * 64;
  // LDS rows: line-major with the odd line stride of Geo in general (a
  // line's points contiguous, lines LS elements apart).  For 3-D n = 6 the
  // odd stride leaves room for only two blocks per compute unit, and
  // unpadded line-major rows (6 elements per line) give the line tasks'
  // 16-byte accesses two-way bank conflicts (gfx950 serves such an access
  // 16 lanes at a time, conflict-free when their 16-byte units differ
  // mod 16).  There (PM) the rows are position-major: point m of line l at
  // l + F m in the final phase, and in the Picard rounds position-major
  // across all of a round's rows at once (GPM, below): row r, line l,
  // point m at F r + l + EI m, EI = F times the rows, so that consecutive
  // line tasks touch consecutive units, also across row boundaries.
  static constexpr bool PM = n == 6 && DIM == 3;
  static constexpr int LS = PM ? 1 : (n == 6 ? 6 : G::LS);  // elements between lines
  static constexpr int ES = PM ? F : 1;                      // elements between a line's points
  static constexpr int SP = PM ? n * F : F * LS;
  __host__ __device__ static constexpr int slot(int line, int pos) { return line * LS + pos * ES; }
  // PAIR: two time slices per LDS round in 16-byte elements.  A 3-D cell of
  // 4^3 nodes is one wave, which needs few registers; there LDS bounds the
  // waves per CU, so the rounds take one slice (8-byte elements) and the
  // final phase one direction at a time: half and a third of the LDS, twice
  // the waves per CU.
  static constexpr bool PAIR = !(DIM == 3 && n == 4 && !PDE::kHasNcp && NV <= 5);
  static constexpr bool FINDIR = !PAIR;
  // Picard rounds' rows: RS elements between rows, EI between a line's points
  static constexpr bool GPM = PM && PAIR;
  // (EI one more than the rows' elements: EI = 13 mod 16 spreads a line's
  // points over distinct banks)
  static constexpr int EI = GPM ? C::NCH * F + 1 : ES, RS = GPM ? F : SP;
  __host__ __device__ static constexpr int islot(int line, int pos) { return GPM ? line + pos * EI : slot(line, pos); }
  static constexpr int ITER_ELEMS = GPM ? 2 * n * EI : (PAIR ? 2 : 1) * C::NCH * SP;
  static constexpr int FIN_ELEMS = (FINDIR ? 1 : DIM) * (NV + C::NFLUX) * SP;
  static constexpr int CELL_ELEMS = cmax(ITER_ELEMS, FIN_ELEMS);
  static constexpr int ELEMS = CPB * CELL_ELEMS;
  // The Ricker amplitudes of the point sources (n + 3 time entries per
  // source) live in the slots past the n points of each line (LS > n), which
  // no round and no final phase touches, where there are enough of them;
  // else in an array of their own.
  static constexpr int NAMP = kMaxSources * (n + 3);
  static constexpr bool AMP_IN_PAD = !PM && !PAIR && CPB == 1 && (LS - n) * F * (CELL_ELEMS / SP) >= NAMP;
  // Single-slice geometry: the rows the final phase leaves free hold each
  // node's time-averaged source S-bar through the final phase (fewer
  // registers live there)
  static constexpr bool STASH = FINDIR && CPB == 1 && CELL_ELEMS - FIN_ELEMS >= NV * BLOCK;
  static constexpr bool fits = ELEMS * 8 <= 80 * 1024 && BLOCK <= 256;
  // Waves per SIMD the register allocator aims at: as many as the blocks
  // whose LDS fits a compute unit (160 KiB) provide, at most WMAX (3: <= 168
  // registers per lane; fewer spill).
  static constexpr int WMAX = PAIR ? 3 : N64_SINGLE_WAVES;
  static constexpr int LDS_BLOCKS = (156 * 1024) / (ELEMS * 8 + (AMP_IN_PAD ? 0 : NAMP * 8));
  static constexpr int MIN_WAVES = cmax(1, cmin(WMAX, LDS_BLOCKS * (BLOCK / 64) / 4));
};

// Line numbering of the Picard rounds' rows for 3-D n = 6 (GPM): a
// permutation of each direction's 36 lines, chosen by a search over the
// node threads' 16-lane access groups (lane k = kx + 6 ky + 36 kz) so that,
// with EI = 541, their 16-byte units fall on distinct banks as far as
// possible (x: 15 cycles per 14 groups, y: 20, z: 18, against 28, 26 and
// 18 with the natural numbering and EI = 540).  Any permutation is correct:
// a line task differentiates whichever line its index names.
static __constant__ const signed char kN64LinePerm[3][36] = {
    {11, 29, 25, 17, 15, 7, 3, 5, 22, 8, 4, 2, 26, 32, 12, 30, 9, 27, 23, 34, 16, 21, 35, 1, 24, 10, 6, 18, 20, 0, 28, 14, 31, 33, 13, 19},
    {30, 21, 28, 13, 19, 20, 5, 18, 10, 27, 3, 32, 35, 11, 9, 2, 33, 26, 17, 25, 24, 0, 7, 31, 1, 8, 15, 22, 29, 23, 4, 34, 16, 12, 14, 6},
    {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26, 27, 28, 29, 30, 31, 32, 33, 34, 35}};
template <bool GPM>
__device__ __forceinline__ int n64_line_perm(int d, int line) {
  if constexpr (GPM) return kN64LinePerm[d][line];
  return line;
}

// PDEs that provide flux_dir(Q, P, pc, d, F), the flux of one direction
template <class... T>
using n64_void_t = void;
template <class PDE, class = void>
struct HasFluxDir : std::false_type {};
template <class PDE>
struct HasFluxDir<PDE, n64_void_t<decltype(&PDE::template flux_dir<double>)>> : std::true_type {};

template <class PDE, int N>
__global__ void __launch_bounds__((GeoN64<PDE, N>::BLOCK), (GeoN64<PDE, N>::MIN_WAVES))
predict_kernel_n64(const KArgs a, const double* Q, const double* __restrict__ params,
                   const double* __restrict__ clock, double* Qout, double* __restrict__ traces) {
  // Q and Qout may be the same array (in-place step): each element is read
  // at the start and written at the end by the thread of its node.
  using GN = GeoN64<PDE, N>;
  using C = Chan<PDE>;
  using T = CT<double, GN::n>;
  constexpr int n = GN::n, S = GN::S, F = GN::F, NV = GN::NV, NP = PDE::NP, DIM = GN::DIM;
  constexpr int CPB = GN::CPB, BLOCK = GN::BLOCK, SP = GN::SP, LS = GN::LS, ES = GN::ES, RS = GN::RS, EI = GN::EI;
  constexpr int NCHD = C::NCHD, NFL = C::NFLUX, NGR = C::ngrad();
  static_assert(C::uniform(), "flux sparsity must be the same in every direction");
  static_assert(GN::fits, "predictor block exceeds its LDS or thread budget");
  __shared__ double lds[GN::ELEMS];

  const int tid = threadIdx.x;
  const int lc = tid / S;  // local cell (CPB means idle lanes in the last wave)
  const int k = tid - lc * S;
  const bool node = lc < CPB;
  const long long cell0 = (long long)xcd_block(blockIdx.x, a.nblocks) * CPB;
  const long long cell = cell0 + (node ? lc : 0);
  const bool active = node && cell < a.ncells;
  const long long cl = cell < a.ncells ? cell : a.ncells - 1;  // clamp loads of the ragged tail

  // this node's slot in the LDS rows of each direction; idle lanes take
  // node 0 of cell 0, so that every lane reads back valid slots (the writes
  // stay with the node lanes) and the read-back sums need no zero start
  int pk[DIM], pki[DIM];  // final phase's rows, Picard rounds' rows
  const int lcr = node ? lc : 0;
  {
    const int kr = node ? k : 0;
    const int kx = kr % n, ky = (kr / n) % n, kz = DIM == 3 ? kr / (n * n) : 0;
    const int kd[3] = {kx, ky, kz};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      pk[d] = GN::slot(GN::G::line_of(d, kx, ky, kz), kd[d]);
      pki[d] = GN::islot(n64_line_perm<GN::GPM>(d, GN::G::line_of(d, kx, ky, kz)), kd[d]);
    }
  }

  // u^n is read from Q where it is used (an L2 hit after the first read;
  // Q is only written at the end, by this thread) rather than kept in
  // registers through the Picard loop
  auto load_u = [&](double (&uu)[NV]) {
#pragma unroll
    for (int v = 0; v < NV; ++v) uu[v] = Q[(cl * NV + v) * S + k];
  };
  double P[NP > 0 ? NP : 1];
#pragma unroll
  for (int p = 0; p < NP; ++p) P[p] = params[cl * NP + p];
  const double t_n = clock[0], dt = clock[1];

  // Point sources: the Ricker amplitude at the n time nodes of this step
  // and at the stage times 0, 1/2, 1 of the CERK guess (entries n .. n+2),
  // once per block; only blocks holding a source cell use them.
  constexpr int NA = n + 3;
  __shared__ double src_amp_own[GN::AMP_IN_PAD ? 1 : kMaxSources * NA];
  auto src_amp = [&](int e) -> double& {
    if constexpr (GN::AMP_IN_PAD) {
      constexpr int PADL = LS - n;  // free slots per line
      const int r = e / (F * PADL), l = (e / PADL) % F, o = e % PADL;
      return lds[r * SP + l * LS + n + o];
    } else {
      return src_amp_own[e];
    }
  };
  bool src_here = false;
  for (int s = 0; s < a.nsrc; ++s)
    src_here = src_here || (a.src[s].cell >= cell0 && a.src[s].cell < cell0 + CPB);
  if (src_here && tid < a.nsrc * NA) {
    const int s = tid / NA, j = tid - s * NA;
    const double tau = j < n ? a.t64.xi[j] : 0.5 * (j - n);
    src_amp(tid) = ricker(a.src[s].f0, a.src[s].t0, a.src[s].amp, t_n + tau * dt);
  }
  // (made visible by the first barrier below)
  auto add_point_sources = [&](int j, double* Sv, double sgn = 1.0) {
    if (!src_here || !node) return;
    for (int s = 0; s < a.nsrc; ++s) {
      if (a.src[s].cell != cell) continue;
      const double amp = src_amp(s * NA + j);
      const double* wsk = a.src_w + ((long long)s * S + k) * NV;
#pragma unroll
      for (int v = 0; v < NV; ++v) Sv[v] += (sgn * amp) * wsk[v];
    }
  };

  // PDEs with neither source nor non-conservative product carry -R (= div F
  // minus the point sources) through the Picard passes; the update and the
  // CERK stages take the sign (no negation of every right-hand side)
  constexpr bool NEG_R = !PDE::kHasNcp && !PDE::kHasSource;
  constexpr double RSGN = NEG_R ? -1.0 : 1.0;

  double q[n][NV];  // iterate at the n time nodes of node k; R_j replaces q_j
  double Fbar[DIM][NV], Nbar[NV], Sbar[NV], qbar[NV];  // final pass: time averages

  // One LDS round for two states qa and qb of the node (two time slices of
  // the iterate, or one state twice): the two share one 16-byte element per
  // (channel, node), so the node threads' writes and read-backs and the line
  // tasks all move 16 bytes per access.  FIN: only the gradients the
  // non-conservative product reads (the final pass averages the fluxes and
  // differentiates their average once).
  using P2 = Pair<double>;
  P2* const lds2 = reinterpret_cast<P2*>(lds);
  // Single-slice geometry (!PAIR): the same round for qa alone, 8-byte
  // elements (qb, div1 and g1 are not used).
  auto round1 = [&](auto fin_tag, const double (&qa)[NV], double (&div0)[NV], double (&g0)[DIM][NV]) {
    constexpr bool FIN = decltype(fin_tag)::value;
    double* const mine = lds + lc * GN::CELL_ELEMS;
    if (node) {
      if constexpr (!FIN) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          double Fa[NV];
          if constexpr (HasFluxDir<PDE>::value) {
            PDE::flux_dir(qa, P, a.pde, d, Fa);
          } else {
            double Fall[DIM][NV];
            PDE::fluxes(qa, P, a.pde, Fall);
#pragma unroll
            for (int v = 0; v < NV; ++v) Fa[v] = Fall[d][v];
          }
#pragma unroll
          for (int cc = 0; cc < NFL; ++cc) mine[(d * NCHD + cc) * RS + pki[d]] = Fa[C::flux_var(d, cc)];
        }
      }
#pragma unroll
      for (int d = 0; d < DIM; ++d)
#pragma unroll
        for (int cc = 0; cc < NGR; ++cc) mine[(d * NCHD + NFL + cc) * RS + pki[d]] = qa[C::grad_var(cc)];
    }
    __syncthreads();
    constexpr int CH0 = FIN ? NFL : 0;
    constexpr int NCT = NCHD - CH0;
    for (int task = tid; task < CPB * DIM * NCT * F; task += BLOCK) {
      const int l = task % F;
      const int ch = CH0 + (task / F) % NCT;
      const int d = (task / (F * NCT)) % DIM;
      const int c2 = task / (F * NCT * DIM);
      double* row = lds + c2 * GN::CELL_ELEMS + (d * NCHD + ch) * RS + GN::islot(l, 0);
      double x[n], y[n];
#pragma unroll
      for (int m = 0; m < n; ++m) x[m] = row[m * EI];
      line_deriv<double, n>(x, y, 1.0);
#pragma unroll
      for (int i = 0; i < n; ++i) row[i * EI] = y[i];
    }
    __syncthreads();
    const double* const rmine = lds + lcr * GN::CELL_ELEMS;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double ih = a.inv_h[d];
#pragma unroll
      for (int cc = 0; cc < NFL; ++cc) {
        if constexpr (FIN) break;
        const int v = C::flux_var(d, cc);
        const double t = rmine[(d * NCHD + cc) * RS + pki[d]];
        div0[v] = C::first_flux_dir(v) == d ? t * ih : fma_r(t, ih, div0[v]);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) g0[d][v] = 0.0;
#pragma unroll
      for (int cc = 0; cc < NGR; ++cc) g0[d][C::grad_var(cc)] = rmine[(d * NCHD + NFL + cc) * RS + pki[d]] * ih;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (FIN || C::first_flux_dir(v) < 0) div0[v] = 0.0;
    // No barrier here: a node thread reads back only its own slots and the
    // next round's writes go to the same slots of the same thread (an idle
    // lane's read of node 0's slots may see either round's values; its sums
    // are never used); the final phase, which uses another layout, starts
    // with a barrier.
  };

  auto round = [&](auto fin_tag, const double (&qa)[NV], const double (&qb)[NV], double (&div0)[NV],
                   double (&g0)[DIM][NV], double (&div1)[NV], double (&g1)[DIM][NV]) {
    constexpr bool FIN = decltype(fin_tag)::value;
    if constexpr (!GN::PAIR) {
      round1(fin_tag, qa, div0, g0);
      return;
    }
    P2* const mine = lds2 + lc * (GN::CELL_ELEMS / 2);
    if (node) {
      if constexpr (!FIN) {
        if constexpr (HasFluxDir<PDE>::value) {
          // one direction at a time (fewer values live)
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
            double Fa[NV], Fb[NV];
            PDE::flux_dir(qa, P, a.pde, d, Fa);
            PDE::flux_dir(qb, P, a.pde, d, Fb);
#pragma unroll
            for (int cc = 0; cc < NFL; ++cc)
              mine[(d * NCHD + cc) * RS + pki[d]] = P2{Fa[C::flux_var(d, cc)], Fb[C::flux_var(d, cc)]};
          }
        } else {
          double Fa[DIM][NV], Fb[DIM][NV];
          PDE::fluxes(qa, P, a.pde, Fa);
          PDE::fluxes(qb, P, a.pde, Fb);
#pragma unroll
          for (int d = 0; d < DIM; ++d)
#pragma unroll
            for (int cc = 0; cc < NFL; ++cc)
              mine[(d * NCHD + cc) * RS + pki[d]] = P2{Fa[d][C::flux_var(d, cc)], Fb[d][C::flux_var(d, cc)]};
        }
      }
#pragma unroll
      for (int d = 0; d < DIM; ++d)
#pragma unroll
        for (int cc = 0; cc < NGR; ++cc)
          mine[(d * NCHD + NFL + cc) * RS + pki[d]] = P2{qa[C::grad_var(cc)], qb[C::grad_var(cc)]};
    }
    __syncthreads();
    constexpr int CH0 = FIN ? NFL : 0;
    constexpr int NCT = NCHD - CH0;
    constexpr int NT = CPB * DIM * NCT * F;
    // Whole tasks (both slices of a line) while every lane has one; the rest
    // split by slice, one slice per lane, so the last round costs half a task.
    constexpr int NWHOLE = NT / BLOCK * BLOCK;
    auto row_of = [&](int task, int& d) {
      const int l = task % F;
      const int ch = CH0 + (task / F) % NCT;
      d = (task / (F * NCT)) % DIM;
      const int c2 = task / (F * NCT * DIM);
      return lds2 + c2 * (GN::CELL_ELEMS / 2) + (d * NCHD + ch) * RS + GN::islot(l, 0);
    };
    auto whole = [&](P2* row, const P2 (&xr)[n]) {
      double x0[n], x1[n], y0[n], y1[n];
#pragma unroll
      for (int m = 0; m < n; ++m) {
        x0[m] = xr[m].x;
        x1[m] = xr[m].y;
      }
      line_deriv<double, n>(x0, y0, 1.0);
      line_deriv<double, n>(x1, y1, 1.0);
#pragma unroll
      for (int i = 0; i < n; ++i) row[i * EI] = P2{y0[i], y1[i]};
    };
    if constexpr (NWHOLE == 2 * BLOCK) {
      // two whole tasks per lane: both lines are loaded before either is
      // differentiated
      int d;
      P2* ra = row_of(tid, d);
      P2* rb = row_of(tid + BLOCK, d);
      P2 xa[n], xb[n];
#pragma unroll
      for (int m = 0; m < n; ++m) xa[m] = ra[m * EI];
#pragma unroll
      for (int m = 0; m < n; ++m) xb[m] = rb[m * EI];
      whole(ra, xa);
      whole(rb, xb);
    } else {
      for (int task = tid; task < NWHOLE; task += BLOCK) {
        int d;
        P2* row = row_of(task, d);
        P2 xr[n];
#pragma unroll
        for (int m = 0; m < n; ++m) xr[m] = row[m * EI];
        whole(row, xr);
      }
    }
    for (int h = tid; h < 2 * (NT - NWHOLE); h += BLOCK) {
      int d;
      double* half = reinterpret_cast<double*>(row_of(NWHOLE + (h >> 1), d)) + (h & 1);
      double x[n], y[n];
#pragma unroll
      for (int m = 0; m < n; ++m) x[m] = half[2 * m * EI];
      line_deriv<double, n>(x, y, 1.0);
#pragma unroll
      for (int i = 0; i < n; ++i) half[2 * i * EI] = y[i];
    }
    __syncthreads();
    const P2* const rmine = lds2 + lcr * (GN::CELL_ELEMS / 2);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double ih = a.inv_h[d];
#pragma unroll
      for (int cc = 0; cc < NFL; ++cc) {
        if constexpr (FIN) break;
        const int v = C::flux_var(d, cc);
        const P2 t = rmine[(d * NCHD + cc) * RS + pki[d]];
        div0[v] = C::first_flux_dir(v) == d ? t.x * ih : fma_r(t.x, ih, div0[v]);
        div1[v] = C::first_flux_dir(v) == d ? t.y * ih : fma_r(t.y, ih, div1[v]);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) g0[d][v] = g1[d][v] = 0.0;
#pragma unroll
      for (int cc = 0; cc < NGR; ++cc) {
        const P2 t = rmine[(d * NCHD + NFL + cc) * RS + pki[d]];
        g0[d][C::grad_var(cc)] = t.x * ih;
        g1[d][C::grad_var(cc)] = t.y * ih;
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (FIN || C::first_flux_dir(v) < 0) div0[v] = div1[v] = 0.0;
    // No barrier here: a node thread reads back only its own slots and the
    // next round's writes go to the same slots of the same thread (an idle
    // lane's read of node 0's slots may see either round's values; its sums
    // are never used); the final phase, which uses another layout, starts
    // with a barrier.
  };

  // One LDS round of a single state in the two-slice rows (the first pass
  // from the constant guess, the CERK stages): the first slice of each
  // element only, one slice per line task, half the LDS traffic and line
  // work of a round of two states.  (Single-slice geometry: round1.)
  auto round_one = [&](const double (&qa)[NV], double (&div0)[NV], double (&g0)[DIM][NV]) {
    if constexpr (!GN::PAIR) {
      round1(std::false_type{}, qa, div0, g0);
      return;
    }
    double* const mine1 = reinterpret_cast<double*>(lds2 + lc * (GN::CELL_ELEMS / 2));
    if (node) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        double Fa[NV];
        if constexpr (HasFluxDir<PDE>::value) {
          PDE::flux_dir(qa, P, a.pde, d, Fa);
        } else {
          double Fall[DIM][NV];
          PDE::fluxes(qa, P, a.pde, Fall);
#pragma unroll
          for (int v = 0; v < NV; ++v) Fa[v] = Fall[d][v];
        }
#pragma unroll
        for (int cc = 0; cc < NFL; ++cc) mine1[2 * ((d * NCHD + cc) * RS + pki[d])] = Fa[C::flux_var(d, cc)];
#pragma unroll
        for (int cc = 0; cc < NGR; ++cc) mine1[2 * ((d * NCHD + NFL + cc) * RS + pki[d])] = qa[C::grad_var(cc)];
      }
    }
    __syncthreads();
    for (int task = tid; task < CPB * DIM * NCHD * F; task += BLOCK) {
      const int l = task % F;
      const int ch = (task / F) % NCHD;
      const int d = (task / (F * NCHD)) % DIM;
      const int c2 = task / (F * NCHD * DIM);
      double* half = reinterpret_cast<double*>(lds2 + c2 * (GN::CELL_ELEMS / 2) + (d * NCHD + ch) * RS + GN::islot(l, 0));
      double x[n], y[n];
#pragma unroll
      for (int m = 0; m < n; ++m) x[m] = half[2 * m * EI];
      line_deriv<double, n>(x, y, 1.0);
#pragma unroll
      for (int i = 0; i < n; ++i) half[2 * i * EI] = y[i];
    }
    __syncthreads();
    const double* const rmine1 = reinterpret_cast<const double*>(lds2 + lcr * (GN::CELL_ELEMS / 2));
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double ih = a.inv_h[d];
#pragma unroll
      for (int cc = 0; cc < NFL; ++cc) {
        const int v = C::flux_var(d, cc);
        const double t = rmine1[2 * ((d * NCHD + cc) * RS + pki[d])];
        div0[v] = C::first_flux_dir(v) == d ? t * ih : fma_r(t, ih, div0[v]);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) g0[d][v] = 0.0;
#pragma unroll
      for (int cc = 0; cc < NGR; ++cc) g0[d][C::grad_var(cc)] = rmine1[2 * ((d * NCHD + NFL + cc) * RS + pki[d])] * ih;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (C::first_flux_dir(v) < 0) div0[v] = 0.0;
    // (no barrier after the read-backs, as in round)
  };

  // right-hand side R = S - div F - B grad q of the state qj (+ the point
  // sources at time entry j of src_amp)
  auto rhs = [&](const double (&qj)[NV], int j, const double (&div)[NV], const double (&g)[DIM][NV],
                 double (&Rv)[NV], double (&B)[NV], double (&Sv)[NV], bool sources) {
    if constexpr (NEG_R) {
      // -R = div F, minus the point sources where the block has one (S
      // holds them for the final pass's average)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Rv[v] = div[v];
        B[v] = Sv[v] = 0.0;
      }
      if (sources && src_here && node) {
        add_point_sources(j, Sv);
#pragma unroll
        for (int v = 0; v < NV; ++v) Rv[v] -= Sv[v];
      }
      return;
    }
    if constexpr (PDE::kHasNcp) {
      PDE::ncp(qj, P, a.pde, g, B);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) B[v] = 0.0;
    }
    PDE::source(qj, P, a.pde, Sv);
    if (sources) add_point_sources(j, Sv);
#pragma unroll
    for (int v = 0; v < NV; ++v) Rv[v] = Sv[v] - div[v] - B[v];
  };

  // q^{r+1}_i = u + dt sum_j KW_ij R_j, R_j held in q[j]
  auto update = [&]() {
    double u[NV];
    load_u(u);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double t[n];
#pragma unroll
      for (int i = 0; i < n; ++i) {
        double s = 0.0;
#pragma unroll
        for (int jj = 0; jj < n; ++jj) s += T::KW(i, jj) * q[jj][v];
        t[i] = s;
      }
#pragma unroll
      for (int i = 0; i < n; ++i) q[i][v] = u[v] + (RSGN * dt) * t[i];
    }
  };

  const int I = a.picard_iters;
  int r0 = 0;  // Picard passes taken before the loop below
  if (a.guess == ADG_GUESS_CERK) {
    // CERK guess (READING of the paper's alternative initial guess): the
    // cell-local ODE dq/dt = R(q, t) by the classical four-stage Runge-Kutta
    // method, whose continuous extension of uniform order three,
    // q(tau) = u + dt sum_s b_s(tau) k_s, is taken at the time nodes.  Each
    // stage is one LDS round of one state; the passes that follow are
    // ordinary Picard passes.
    double Y[NV];
    load_u(Y);
#pragma unroll
    for (int j = 0; j < n; ++j)
#pragma unroll
      for (int v = 0; v < NV; ++v) q[j][v] = Y[v];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      double div[NV], g[DIM][NV], kk[NV], B[NV], Sv[NV];
      round_one(Y, div, g);
      rhs(Y, n + (st == 0 ? 0 : (st == 3 ? 2 : 1)), div, g, kk, B, Sv, true);
#pragma unroll
      for (int j = 0; j < n; ++j) {
        const double b = (RSGN * dt) * T::cerk_b(st, j);
#pragma unroll
        for (int v = 0; v < NV; ++v) q[j][v] += b * kk[v];
      }
      const double as = st == 2 ? 1.0 : 0.5;  // Y_{s+1} = u + dt a_{s+1} k_s
      load_u(Y);
#pragma unroll
      for (int v = 0; v < NV; ++v) Y[v] += (RSGN * dt) * as * kk[v];
    }
  } else {
    // First Picard step: q^0 = u^n at every time node, so every slice has
    // the same right-hand side apart from point sources; one round suffices.
    load_u(q[0]);
    double div[NV], g[DIM][NV], R0[NV], B[NV], Sv[NV];
    round_one(q[0], div, g);
    rhs(q[0], 0, div, g, R0, B, Sv, false);
#pragma unroll
    for (int jj = 0; jj < n; ++jj) {
#pragma unroll
      for (int v = 0; v < NV; ++v) q[jj][v] = R0[v];
      add_point_sources(jj, q[jj], RSGN);
    }
    update();
    r0 = 1;
  }
  constexpr int SLICES = GN::PAIR ? 2 : 1;  // time slices per LDS round
  for (int r = r0; r < I; ++r) {
#pragma unroll
    for (int j = 0; j < n; j += SLICES) {
      const int j1 = j + SLICES - 1 < n ? j + SLICES - 1 : j;
      double div0[NV], g0[DIM][NV], div1[NV], g1[DIM][NV], Rv[NV], B[NV], Sv[NV];
      round(std::false_type{}, q[j], q[j1], div0, g0, div1, g1);
      rhs(q[j], j, div0, g0, Rv, B, Sv, true);
      if (j1 != j) {
        double Rw[NV];
        rhs(q[j1], j1, div1, g1, Rw, B, Sv, true);
#pragma unroll
        for (int v = 0; v < NV; ++v) q[j1][v] = Rw[v];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) q[j][v] = Rv[v];
    }
    update();
  }

  // Final pass at the last iterate (READING: the averaged terms use the
  // final iterate): time averages of q, F, B grad q and S.  Without a
  // non-conservative product the final pass needs no LDS round, so qbar goes
  // to its rows of the final phase at once (fewer registers live).
  __syncthreads();  // every read-back of the last round is done
  constexpr int FIN_D = (NV + NFL) * SP;
  constexpr int NDG = GN::FINDIR ? DIM : 1;  // direction groups of the final phase
  constexpr int DPG = DIM / NDG;             // directions per group
  auto fin_off = [](int d) { return GN::FINDIR ? 0 : d * FIN_D; };
  double* const fin_mine = lds + lc * GN::CELL_ELEMS;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    Nbar[v] = Sbar[v] = qbar[v] = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) Fbar[d][v] = 0.0;
  }
  if constexpr (!PDE::kHasNcp) {
#pragma unroll
    for (int j = 0; j < n; ++j)
#pragma unroll
      for (int v = 0; v < NV; ++v) qbar[v] += T::w(j) * q[j][v];
    if (node && !GN::FINDIR) {
#pragma unroll
      for (int d = 0; d < DIM; ++d)
#pragma unroll
        for (int v = 0; v < NV; ++v) fin_mine[d * FIN_D + v * SP + pk[d]] = qbar[v];
    }
  }
#pragma unroll
  for (int j = 0; j < n; ++j) {
    double div[NV], g[DIM][NV], Rv[NV], B[NV], Sv[NV];
    if constexpr (PDE::kHasNcp) {
      double div1[NV], g1[DIM][NV];
      round(std::true_type{}, q[j], q[j], div, g, div1, g1);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        div[v] = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) g[d][v] = 0.0;
      }
    }
    rhs(q[j], j, div, g, Rv, B, Sv, true);
    const double wj = T::w(j);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if constexpr (PDE::kHasNcp) qbar[v] += wj * q[j][v];
      Nbar[v] += wj * B[v];
      Sbar[v] += wj * Sv[v];
    }
    if constexpr (GN::FINDIR) {
      // Fbar_d is formed direction by direction in the final phase below
    } else if constexpr (HasFluxDir<PDE>::value) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        double Fl[NV];
        PDE::flux_dir(q[j], P, a.pde, d, Fl);
#pragma unroll
        for (int v = 0; v < NV; ++v) Fbar[d][v] += wj * Fl[v];
      }
    } else {
      double Fl[DIM][NV];
      PDE::fluxes(q[j], P, a.pde, Fl);
#pragma unroll
      for (int d = 0; d < DIM; ++d)
#pragma unroll
        for (int v = 0; v < NV; ++v) Fbar[d][v] += wj * Fl[d][v];
    }
  }

  // Volume term and face projection, all directions at once (or one at a
  // time, FINDIR): direction d's region of the cell's LDS holds qbar (NV
  // rows) and the nonzero components of Fbar_d (NFL rows) in d's layout.
  if constexpr (PDE::kHasNcp) __syncthreads();  // the final pass's rounds are done
  double* const stash = lds + GN::FIN_ELEMS;  // GN::STASH: [NV][BLOCK], untouched by the final phase
  if constexpr (GN::STASH) {
#pragma unroll
    for (int v = 0; v < NV; ++v) stash[v * BLOCK + tid] = Sbar[v];
  }
  double divF[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) divF[v] = 0.0;
#pragma unroll
  for (int dg = 0; dg < NDG; ++dg) {
    if (dg > 0) __syncthreads();  // the previous direction's read-backs are done
    if constexpr (GN::FINDIR) {
      // Fbar_d = sum_j w_j F_d(q_j) for this group's direction only (the
      // iterate is still in registers): fewer values live than all of Fbar
#pragma unroll
      for (int d = dg * DPG; d < (dg + 1) * DPG; ++d) {
#pragma unroll
        for (int j = 0; j < n; ++j) {
          double Fl[NV];
          if constexpr (HasFluxDir<PDE>::value) {
            PDE::flux_dir(q[j], P, a.pde, d, Fl);
          } else {
            double Fall[DIM][NV];
            PDE::fluxes(q[j], P, a.pde, Fall);
#pragma unroll
            for (int v = 0; v < NV; ++v) Fl[v] = Fall[d][v];
          }
#pragma unroll
          for (int v = 0; v < NV; ++v) Fbar[d][v] += T::w(j) * Fl[v];
        }
      }
    }
    if (node) {
#pragma unroll
      for (int d = dg * DPG; d < (dg + 1) * DPG; ++d) {
        if constexpr (PDE::kHasNcp || GN::FINDIR) {
#pragma unroll
          for (int v = 0; v < NV; ++v) fin_mine[fin_off(d) + v * SP + pk[d]] = qbar[v];
        }
#pragma unroll
        for (int cc = 0; cc < NFL; ++cc)
          fin_mine[fin_off(d) + (NV + cc) * SP + pk[d]] = Fbar[d][C::flux_var(d, cc)];
      }
    }
    __syncthreads();
    // One task per (cell, direction of the group, quantity v, line l): the
    // traces of qbar_v and of the normal flux Fbar_{d,v} at both faces of
    // the line, and the derivative of Fbar_{d,v} along it, in place.  The
    // direction and the quantity are runtime indices, so every task takes
    // the same code path and a wave runs one task body per pass.
    for (int task = tid; task < CPB * DPG * NV * F; task += BLOCK) {
      const int l = task % F;
      const int v = (task / F) % NV;
      const int d = dg * DPG + (task / (F * NV)) % DPG;
      const int c2 = task / (F * NV * DPG);
      const long long tcell = cell0 + c2;
      const bool tact = tcell < a.ncells;
      double* rows = lds + c2 * GN::CELL_ELEMS + fin_off(d) + GN::slot(l, 0);
      double* tr = traces + ((tcell * (2 * DIM) + 2 * d) * 2) * (long long)NV * F + v * F + l;
      double e0 = 0.0, e1 = 0.0;
#pragma unroll
      for (int m = 0; m < n; ++m) {
        const double x = rows[v * SP + m * ES];
        e0 += T::l0(m) * x;
        e1 += T::l1(m) * x;
      }
      // the flux row of v in d's layout (-1: F_d has no component v)
      int cc = -1;
#pragma unroll
      for (int dd = dg * DPG; dd < (dg + 1) * DPG; ++dd)
#pragma unroll
        for (int c = 0; c < NFL; ++c)
          if (dd == d && C::flux_var(dd, c) == v) cc = c;
      double f0 = 0.0, f1 = 0.0;
      if (cc >= 0) {
        double x[n], y[n];
#pragma unroll
        for (int m = 0; m < n; ++m) x[m] = rows[(NV + cc) * SP + m * ES];
#pragma unroll
        for (int m = 0; m < n; ++m) {
          f0 += T::l0(m) * x[m];
          f1 += T::l1(m) * x[m];
        }
        line_deriv<double, n>(x, y, a.inv_h[d]);
#pragma unroll
        for (int i = 0; i < n; ++i) rows[(NV + cc) * SP + i * ES] = y[i];
      }
      if (tact) {
        tr[0 * NV * F] = e0;  // face 2d,   state
        tr[1 * NV * F] = f0;  // face 2d,   normal flux
        tr[2 * NV * F] = e1;  // face 2d+1, state
        tr[3 * NV * F] = f1;  // face 2d+1, normal flux
      }
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int d = dg * DPG; d < (dg + 1) * DPG; ++d)
#pragma unroll
        for (int cc = 0; cc < NFL; ++cc) divF[C::flux_var(d, cc)] += fin_mine[fin_off(d) + (NV + cc) * SP + pk[d]];
    }
  }
  if (active) {
    // u^n again from memory (not kept in registers through the final pass;
    // Q is only written here, by this thread)
    if constexpr (GN::STASH) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Sbar[v] = stash[v * BLOCK + tid];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double un = Q[(cell * NV + v) * S + k];
      Qout[(cell * NV + v) * S + k] = un + dt * (Sbar[v] - divF[v] - Nbar[v]);
    }
  }
}

}  // namespace adg

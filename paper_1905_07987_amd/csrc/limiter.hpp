// A-posteriori subcell limiter for the Euler equations (ExaHyPE paper,
// Sec. 3.5; the FV, limiter and projection kernels of Table 1; the hybrid
// ADER-DG/FV status stencil of Fig. 2).  A limited step on the device:
//   prepare   u^n copied, the previous status kept, the range of each
//             cell's subcell averages at t^n (FV cells: their own FV data);
//   (the unlimited ADER-DG step in place: the candidate)
//   detect    physical admissibility at every node and subcell average of
//             the candidate, then the relaxed discrete maximum principle;
//   classify  troubled (3), FV as a neighbour of a troubled cell (2), DG
//             with an FV face (1), DG (0); FV cells and DG cells with an FV
//             face are appended to two lists;
//   fv        MUSCL-Hancock with minmod on the (2N+1)^d subcells of each FV
//             cell from the subcell averages at t^n, projected back to the
//             DG space; the fluxes through the cell's faces are kept as
//             face-node values for the DG neighbours;
//   faces     a DG cell with an FV face exchanges the Rusanov flux of that
//             face in its update for the FV one (what leaves one cell
//             enters the other).
// Readings where the paper gives no formula: subcell averages are exact
// averages of the nodal polynomial; the way back is their least-squares
// inverse; the DMP range is the cell's and its face neighbours' subcell
// averages at t^n widened by max(1e-4, 1e-3 (max - min)); a subcell whose
// extrapolated or half-step values are not admissible uses its average on
// all faces; ghost subcells beyond a wall or outflow face mirror the inside
// ones (the wall reverses the normal momentum); FV cells keep their subcell
// averages from step to step and a cell returns to DG once its candidate
// passes both tests.
#pragma once

namespace adg {

template <class PDE>
struct LimiterPDE {
  static constexpr bool value = false;
};
template <int D>
struct LimiterPDE<Euler<D>> {
  static constexpr bool value = true;
};

template <class PDE, int N>
struct GeoLim {
  static constexpr int DIM = PDE::DIM, NV = PDE::NV, n = N + 1, m = 2 * N + 1;
  static constexpr int S = ipow(n, DIM), F = ipow(n, DIM - 1);
  static constexpr int NS = ipow(m, DIM), NSF = ipow(m, DIM - 1);
  static constexpr int EB = m + 4, NB = ipow(EB, DIM);  // subcells of the cell and two ghost layers
  static constexpr int EC = m + 2, NC = ipow(EC, DIM);  // subcells whose face values are moved
  static constexpr int NTAB = 3 * m * n;                // A [m][n], B [n][m], Qf [n][m]
  static constexpr int BLOCK = 512;                     // threads of the FV kernel
  static constexpr int VPT = (NS + BLOCK - 1) / BLOCK;  // subcells per thread in the update
  static constexpr int NOWN = DIM == 3 ? 19 : 9;        // the cell, its face and edge neighbours
  // fv: tables, the subcell box, then either the owners' nodal values (while
  // the box is filled) or the half-step corrections and the subface fluxes
  static constexpr int FV_D = NTAB + NV * NB + cmax(NV * (NC + 2 * DIM * NSF), NOWN * NV * S);
  static constexpr bool built = LimiterPDE<PDE>::value && FV_D * 8 + NC <= 120 * 1024;
};

template <int DIM>
__device__ __forceinline__ void lim_multi(int idx, int e, int (&x)[3]) {
  x[0] = idx % e;
  x[1] = (idx / e) % e;
  x[2] = DIM == 3 ? idx / (e * e) : 0;
}

// face neighbour along d on side s (-1, +1); -1 on a non-periodic boundary
template <int DIM>
__device__ __forceinline__ long long lim_neighbour(const KArgs& a, long long c, int d, int s) {
  const int C0 = a.cells[0], C1 = a.cells[1];
  int cc[3] = {(int)(c % C0), (int)((c / C0) % C1), DIM == 3 ? (int)(c / ((long long)C0 * C1)) : 0};
  int to = cc[d] + s;
  if (to < 0 || to >= a.cells[d]) {
    if (a.bc[2 * d + (s > 0)] != ADG_BC_PERIODIC) return -1;
    to = (to + a.cells[d]) % a.cells[d];
  }
  cc[d] = to;
  return cc[0] + (long long)C0 * (cc[1] + (long long)C1 * cc[2]);
}

__device__ __forceinline__ void lim_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-wave LDS of the prepare and detect kernels: one group of variables'
// nodal values and the contraction stages of the projection onto the
// subcells (the last stage is evaluated in registers, one column of subcells
// per lane).  Region A holds the nodal values, later the second stage
// (3-D); region B the first stage.  The variables go in two groups, so a
// wave needs half the LDS and more waves share a CU.  The subcell averages
// of the basis, LimConst<n>::A, are compile-time constants.
template <class PDE, int N>
struct GeoLimW {
  using GL = GeoLim<PDE, N>;
  static constexpr int WPB = 4;                   // cells (waves) per block
  static constexpr int VG = (GL::NV + 1) / 2;     // variables of the first group
  static constexpr int P1 = VG * GL::m * ipow(GL::n, GL::DIM - 1);
  static constexpr int P2 = GL::DIM == 3 ? VG * GL::m * GL::m * GL::n : 0;
  static constexpr int RA = cmax(VG * GL::S, P2), RB = P1;
  static constexpr int RN = (GL::NV - VG) * GL::S;  // nodal values of the second group
  static constexpr int PW = RA + RB + RN;
  // columns of subcells along the last axis: one per lane
  static constexpr int LAST = ipow(GL::m, GL::DIM - 1);
  static_assert(LAST <= 64, "one column of subcells per lane");
};

// The leading stages for NVS variables, one line per lane and step: along x
// (nodal values in A, [v][kz][ky][kx], to B, [v][kz][ky][sx]); in 3-D then
// along y (B to A, [v][kz][sy][sx]).
template <class PDE, int N, int NVS>
__device__ __forceinline__ void lim_stages_wave(const double* src, double* ra, double* rb, int lane) {
  using GL = GeoLim<PDE, N>;
  using LC = LimConst<GL::n>;
  constexpr int n = GL::n, m = GL::m;
  constexpr int L1 = NVS * ipow(n, GL::DIM - 1);
  for (int line = lane; line < L1; line += 64) {
    double in[n];
#pragma unroll
    for (int k = 0; k < n; ++k) in[k] = src[line * n + k];
#pragma unroll
    for (int s = 0; s < m; ++s) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < n; ++k) acc += LC::A[s][k] * in[k];
      rb[line * m + s] = acc;
    }
  }
  lim_wave_sync();
  if constexpr (GL::DIM == 3) {
    constexpr int L2 = NVS * n * m;
    for (int line = lane; line < L2; line += 64) {
      const int sx = line % m, vk = line / m;  // vk = v n + kz
      double in[n];
#pragma unroll
      for (int k = 0; k < n; ++k) in[k] = rb[(vk * n + k) * m + sx];
#pragma unroll
      for (int s = 0; s < m; ++s) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < n; ++k) acc += LC::A[s][k] * in[k];
        ra[(vk * m + s) * m + sx] = acc;
      }
    }
    lim_wave_sync();
  }
}

// Variables V0 .. V0 + NVS - 1 of a cell through the projection, from
// their nodal values at src (LDS, [v][S]): out[V0 + v][j] = the average of
// variable V0 + v over the j-th subcell of this lane's column (subcell index
// lane + j m^(dim-1)), for lanes below the column count.
template <class PDE, int N, int V0, int NVS>
__device__ __forceinline__ void lim_group_wave(const double* src, double* ra, double* rb, int lane,
                                               double (&out)[PDE::NV][2 * N + 1]) {
  using GL = GeoLim<PDE, N>;
  using LC = LimConst<GL::n>;
  constexpr int n = GL::n, m = GL::m;
  lim_stages_wave<PDE, N, NVS>(src, ra, rb, lane);
  if (lane < GeoLimW<PDE, N>::LAST) {
#pragma unroll
    for (int v = 0; v < NVS; ++v) {
      double in[n];
#pragma unroll
      for (int k = 0; k < n; ++k)
        in[k] = GL::DIM == 2 ? rb[(v * n + k) * m + lane] : ra[(v * n + k) * m * m + lane];
#pragma unroll
      for (int j = 0; j < m; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < n; ++k) acc += LC::A[j][k] * in[k];
        out[V0 + v][j] = acc;
      }
    }
  }
  lim_wave_sync();  // the next group overwrites the stages
}

// The cell's nodal values from registers (lane k < S: node k) to the wave's
// LDS: the first group where the projection's first stage reads it, the
// second group in a region of its own.
template <class PDE, int N>
__device__ __forceinline__ void lim_stage_nodes(const double (&x)[PDE::NV], double* ra, double* rn, int lane) {
  constexpr int S = GeoLim<PDE, N>::S, VG = GeoLimW<PDE, N>::VG;
  if (lane < S) {
#pragma unroll
    for (int v = 0; v < PDE::NV; ++v) (v < VG ? ra + v * S : rn + (v - VG) * S)[lane] = x[v];
  }
  lim_wave_sync();
}

__device__ __forceinline__ double lim_wave_min(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fmin(x, __shfl_xor(x, off, 64));
  return x;
}
__device__ __forceinline__ double lim_wave_max(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
  return x;
}

// The prepare and detect kernels issue every global load of a cell at once
// (all nodal values into registers, and in detect the DMP ranges, one
// (variable, cell) per lane) before the chain of dependent LDS stages of
// the projection, so that a cell waits for one HBM round trip instead of
// one per variable group and neighbour.
template <class PDE, int N>
struct GeoLimSeq {
  static unsigned grid(long long ncells) {
    return (unsigned)((ncells + GeoLimW<PDE, N>::WPB - 1) / GeoLimW<PDE, N>::WPB);
  }
};

// nodal values of cell c (lane k < S: node k), zero past the grid
template <class PDE, int N>
__device__ __forceinline__ void lim_load_nodes(const double* __restrict__ Q, long long c, long long ncells, int lane,
                                               double (&x)[PDE::NV]) {
  constexpr int NV = PDE::NV, S = GeoLim<PDE, N>::S;
  const bool ok = c < ncells && lane < S;
  const long long cl = ok ? c : 0;
#pragma unroll
  for (int v = 0; v < NV; ++v) x[v] = ok ? Q[(cl * NV + v) * S + lane] : 0.0;
}

// One wave per cell: u^n copied, status kept, range of the subcell
// averages at t^n (w.reuse: for a DG cell of status 0, whose u^n is the
// previous step's candidate, the range that step's detect stored).  Block 0
// clears the counters of the step.
template <class PDE, int N>
__global__ void __launch_bounds__(256)
lim_prepare_kernel(const KArgs a, const double* __restrict__ Q, const double* __restrict__ sub_in,
                   const uint8_t* __restrict__ status, const LimWork w) {
  using GL = GeoLim<PDE, N>;
  using GW = GeoLimW<PDE, N>;
  constexpr int NV = GL::NV, S = GL::S, NS = GL::NS, m = GL::m;
  __shared__ double buf[GW::WPB][GW::PW];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (blockIdx.x == 0 && tid < 4) w.counters[tid] = 0;
  const long long c = (long long)blockIdx.x * GW::WPB + wv;
  if (c >= a.ncells) return;
  double* ra = buf[wv];
  double* rb = ra + GW::RA;
  double* rn = rb + GW::RB;
  const uint8_t st = status[c];
  double x[NV];
  lim_load_nodes<PDE, N>(Q, c, a.ncells, lane, x);
  if (lane == 0) w.st_prev[c] = st;
  if (lane < S)
#pragma unroll
    for (int v = 0; v < NV; ++v) w.Qold[(c * NV + v) * S + lane] = x[v];
  double lo[NV], hi[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    lo[v] = INFINITY;
    hi[v] = -INFINITY;
  }
  if (w.reuse && st == 0) {
    if (lane < NV) {
      w.lohi[(c * NV + lane) * 2] = w.lohi_next[(c * NV + lane) * 2];
      w.lohi[(c * NV + lane) * 2 + 1] = w.lohi_next[(c * NV + lane) * 2 + 1];
    }
    return;
  }
  if (st >= 2) {
    for (int s = lane; s < NS; s += 64)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double y = sub_in[(c * NV + v) * NS + s];
        lo[v] = fmin(lo[v], y);
        hi[v] = fmax(hi[v], y);
      }
  } else {
    lim_stage_nodes<PDE, N>(x, ra, rn, lane);
    double q[NV][m];
    lim_group_wave<PDE, N, 0, GW::VG>(ra, ra, rb, lane, q);
    lim_group_wave<PDE, N, GW::VG, NV - GW::VG>(rn, ra, rb, lane, q);
    if (lane < GW::LAST)
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int j = 0; j < m; ++j) {
          lo[v] = fmin(lo[v], q[v][j]);
          hi[v] = fmax(hi[v], q[v][j]);
        }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double l = lim_wave_min(lo[v]), h = lim_wave_max(hi[v]);
    if (lane == 0) {
      w.lohi[(c * NV + v) * 2] = l;
      w.lohi[(c * NV + v) * 2 + 1] = h;
    }
  }
}

// The DMP ranges of cell c and its face neighbours, one (cell, variable)
// per lane: lane v 8 + j holds (lo, hi) of variable v of cell j (j = 0 the
// cell itself, 1 .. 2 dim its face neighbours; an empty range past a
// non-periodic boundary and on the spare lanes).
template <class PDE, int N>
__device__ __forceinline__ void lim_load_ranges(const KArgs& a, const double* lohi, long long c, int lane,
                                                double& lo, double& hi) {
  constexpr int DIM = PDE::DIM, NV = PDE::NV;
  static_assert(NV * 8 <= 64 && 2 * DIM + 1 <= 8, "one lane per (variable, cell)");
  const int v = lane >> 3, j = lane & 7;
  long long o = -1;
  if (c < a.ncells && v < NV && j <= 2 * DIM)
    o = j == 0 ? c : lim_neighbour<DIM>(a, c, (j - 1) >> 1, ((j - 1) & 1) ? 1 : -1);
  lo = INFINITY;
  hi = -INFINITY;
  if (o >= 0) {
    lo = lohi[(o * NV + v) * 2];
    hi = lohi[(o * NV + v) * 2 + 1];
  }
}

// One wave per cell: is the candidate troubled?  (w.store_next: also the
// range of the candidate's subcell averages, as prepare computes it, for
// the next step's prepare.)
template <class PDE, int N>
__global__ void __launch_bounds__(256)
lim_detect_kernel(const KArgs a, const double* __restrict__ Q, const LimWork w) {
  using GL = GeoLim<PDE, N>;
  using GW = GeoLimW<PDE, N>;
  constexpr int NV = GL::NV, S = GL::S, m = GL::m;
  __shared__ double buf[GW::WPB][GW::PW];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const long long c = (long long)blockIdx.x * GW::WPB + wv;
  if (c >= a.ncells) return;
  double* ra = buf[wv];
  double* rb = ra + GW::RA;
  double* rn = rb + GW::RB;
  double x[NV], rlo, rhi;
  lim_load_nodes<PDE, N>(Q, c, a.ncells, lane, x);
  lim_load_ranges<PDE, N>(a, w.lohi, c, lane, rlo, rhi);
  bool bad = lane < S && !PDE::admissible(x, x, a.pde);
  lim_stage_nodes<PDE, N>(x, ra, rn, lane);
  // DMP range: the cell's and its face neighbours' subcell averages at t^n
#pragma unroll
  for (int off = 1; off < 8; off <<= 1) {
    rlo = fmin(rlo, __shfl_xor(rlo, off, 64));
    rhi = fmax(rhi, __shfl_xor(rhi, off, 64));
  }
  double lo[NV], hi[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    lo[v] = __shfl(rlo, v * 8, 64);
    hi[v] = __shfl(rhi, v * 8, 64);
  }
  double qv[NV][m];
  lim_group_wave<PDE, N, 0, GW::VG>(ra, ra, rb, lane, qv);
  lim_group_wave<PDE, N, GW::VG, NV - GW::VG>(rn, ra, rb, lane, qv);
  if (lane < GW::LAST) {
#pragma unroll
    for (int j = 0; j < m; ++j) {
      double q[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) q[v] = qv[v][j];
      bad = bad || !PDE::admissible(q, q, a.pde);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double delta = fmax(1e-4, 1e-3 * (hi[v] - lo[v]));
        bad = bad || !(q[v] >= lo[v] - delta && q[v] <= hi[v] + delta);
      }
    }
  }
  if (w.store_next) {
    double l2[NV], h2[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      l2[v] = INFINITY;
      h2[v] = -INFINITY;
    }
    if (lane < GW::LAST)
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int j = 0; j < m; ++j) {
          l2[v] = fmin(l2[v], qv[v][j]);
          h2[v] = fmax(h2[v], qv[v][j]);
        }
    if constexpr (2 * NV * 71 <= GW::PW) {
      // the lanes' partial ranges through the wave's stage buffer (free once
      // the projection is done; rows 65 apart, so the folding lanes take
      // distinct banks), then one lane per (variable, bound) folds the 64
      // (the minima stored negated: one max loop)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        ra[(2 * v) * 65 + lane] = -l2[v];
        ra[(2 * v + 1) * 65 + lane] = h2[v];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (lane < 2 * NV * 6) {  // six lanes per (variable, bound), 11 values each
        const int slot = lane / 6, part = lane - slot * 6;
        const double* col = ra + slot * 65 + part * 11;
        double r = -INFINITY;
#pragma unroll
        for (int i = 0; i < 11; ++i)
          if (part * 11 + i < 64) r = fmax(r, col[i]);
        ra[2 * NV * 65 + lane] = r;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (lane < 2 * NV) {
        const double* pr = ra + 2 * NV * 65 + lane * 6;
        double r = pr[0];
#pragma unroll
        for (int i = 1; i < 6; ++i) r = fmax(r, pr[i]);
        w.lohi_next[c * NV * 2 + lane] = (lane & 1) ? r : -r;
      }
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double l = lim_wave_min(l2[v]), h = lim_wave_max(h2[v]);
        if (lane == 0) {
          w.lohi_next[(c * NV + v) * 2] = l;
          w.lohi_next[(c * NV + v) * 2 + 1] = h;
        }
      }
    }
  }
  bad = __ballot(bad) != 0;
  if (lane == 0) {
    w.trb[c] = bad ? 1 : 0;
    if (bad) atomicAdd(&w.counters[0], 1);
  }
}

// One thread per cell: status of the step and the two cell lists.
template <int DIM>
__global__ void __launch_bounds__(256) lim_classify_kernel(const KArgs a, uint8_t* __restrict__ status, const LimWork w) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.ncells) return;
  uint8_t s = 0;
  if (w.trb[c]) {
    s = 3;
  } else {
    bool near_troubled = false, near_fv = false;
    for (int d = 0; d < DIM; ++d)
      for (int sd = -1; sd <= 1; sd += 2) {
        const long long o = lim_neighbour<DIM>(a, c, d, sd);
        if (o < 0) continue;
        if (w.trb[o]) {
          near_troubled = true;
          continue;
        }
        for (int d2 = 0; d2 < DIM; ++d2)
          for (int s2 = -1; s2 <= 1; s2 += 2) {
            const long long o2 = lim_neighbour<DIM>(a, o, d2, s2);
            if (o2 >= 0 && w.trb[o2]) near_fv = true;
          }
      }
    s = near_troubled ? 2 : (near_fv ? 1 : 0);
  }
  status[c] = s;
  if (s >= 2) w.fv_list[atomicAdd(&w.counters[1], 1)] = (int)c;
  if (s == 1) w.y_list[atomicAdd(&w.counters[2], 1)] = (int)c;
}

__device__ __forceinline__ double lim_minmod(double x, double y) {
  if (x > 0.0 && y > 0.0) return fmin(x, y);
  if (x < 0.0 && y < 0.0) return fmax(x, y);
  return 0.0;
}

// Rusanov flux along d between the states qa (low side) and qb (high side).
template <class PDE>
__device__ __forceinline__ void lim_rusanov(const PdeConsts& pc, int d, const double* qa, const double* qb,
                                            double* G) {
  constexpr int NV = PDE::NV, DIM = PDE::DIM;
  double Fa[DIM][NV], Fb[DIM][NV];
  PDE::fluxes(qa, qa, pc, Fa);
  PDE::fluxes(qb, qb, pc, Fb);
  const double s = fmax(PDE::max_eigen(qa, qa, pc, d), PDE::max_eigen(qb, qb, pc, d));
#pragma unroll
  for (int v = 0; v < NV; ++v) G[v] = 0.5 * (Fa[d][v] + Fb[d][v]) - 0.5 * s * (qb[v] - qa[v]);
}

// The value of box position p extrapolated to its face (d, side) and moved
// half a step (its average where the subcell falls back to first order).
template <class PDE, int N>
__device__ __forceinline__ void lim_moved(const double* box, const double* corr, const uint8_t* okf, int p, int q,
                                          int d, int side, double (&out)[PDE::NV]) {
  using GL = GeoLim<PDE, N>;
  constexpr int NV = GL::NV, NB = GL::NB, NC = GL::NC, EB = GL::EB;
  const int sd = d == 0 ? 1 : (d == 1 ? EB : EB * EB);
  const bool ok = okf[q] != 0;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double wv = box[v * NB + p];
    if (ok) {
      const double slope = lim_minmod(wv - box[v * NB + p - sd], box[v * NB + p + sd] - wv);
      out[v] = (side ? wv + 0.5 * slope : wv - 0.5 * slope) + corr[v * NC + q];
    } else {
      out[v] = wv;
    }
  }
}

// FV cells, a persistent grid over the FV list.
template <class PDE, int N>
__global__ void __launch_bounds__(512)
lim_fv_kernel(const KArgs a, const double* __restrict__ clock, const double* __restrict__ sub_in, double* __restrict__ Q,
              double* __restrict__ sub_out, const LimWork w) {
  using GL = GeoLim<PDE, N>;
  constexpr int DIM = GL::DIM, NV = GL::NV, S = GL::S, NS = GL::NS, NSF = GL::NSF, F = GL::F;
  constexpr int m = GL::m, n = GL::n, EB = GL::EB, NB = GL::NB, EC = GL::EC, NC = GL::NC, BLOCK = GL::BLOCK;
  __shared__ double lds[GL::FV_D];
  __shared__ uint8_t okf[NC];
  __shared__ long long owner[GL::NOWN];  // owner cell of each slot, -1 beyond a non-periodic face
  __shared__ uint8_t fvdata[GL::NOWN];   // the owner was FV at t^n: its subcell data is read
  double* T = lds;
  double* box = T + GL::NTAB;
  double* corr = box + NV * NB;
  double* fsub = corr + NV * NC;
  double* ou = corr;  // the owners' nodal values, only while the box is filled
  const double* A = T;
  const double* B = T + m * n;
  const double* Qf = T + 2 * m * n;
  const int tid = threadIdx.x;
  for (int i = tid; i < GL::NTAB; i += BLOCK) T[i] = w.tab[i];
  const double dt = clock[1];
  double hs[3] = {1.0, 1.0, 1.0};
#pragma unroll
  for (int d = 0; d < DIM; ++d) hs[d] = a.h[d] / m;
  const int count = w.counters[1];
  for (int it = blockIdx.x; it < count; it += gridDim.x) {
    const long long c = w.fv_list[it];
    const int C0 = a.cells[0], C1 = a.cells[1];
    const int cc[3] = {(int)(c % C0), (int)((c / C0) % C1), DIM == 3 ? (int)(c / ((long long)C0 * C1)) : 0};
    __syncthreads();  // the previous cell's LDS reads are done
    // 1. the subcell box: the cell, two ghost layers across each face, one
    //    across each edge (corners are never read).  Every position belongs
    //    to the cell or to a face or edge neighbour (beyond a non-periodic
    //    face it mirrors a subcell of the cell on this side, the wall
    //    reversing the normal momentum).  The owners' nodal values are
    //    staged in LDS first (owner slot: the offset's rank among the
    //    offsets in {-1,0,1}^dim with at most two nonzero entries).
    // one thread per offset k in {-1,0,1}^dim: its owner cell and whether
    // that owner was FV at t^n
    if (tid < ipow(3, DIM)) {
      const int k = tid;
      const int off[3] = {k % 3 - 1, (k / 3) % 3 - 1, DIM == 3 ? k / 9 - 1 : 0};
      if ((off[0] != 0) + (off[1] != 0) + (off[2] != 0) <= 2) {
        const int slot = DIM == 2 ? k
                                  : k - ((k > 0) + (k > 2) + (k > 6) + (k > 8) + (k > 18) + (k > 20) + (k > 24));
        int oc[3] = {cc[0], cc[1], cc[2]};
        bool exists = true;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          oc[d] += off[d];
          if (oc[d] < 0 || oc[d] >= a.cells[d]) {
            if (a.bc[2 * d + (off[d] > 0)] != ADG_BC_PERIODIC) exists = false;
            oc[d] = (oc[d] + a.cells[d]) % a.cells[d];
          }
        }
        const long long o = exists ? oc[0] + (long long)C0 * (oc[1] + (long long)C1 * oc[2]) : -1;
        owner[slot] = o;
        fvdata[slot] = (exists && w.st_prev[o] >= 2) ? 1 : 0;
      }
    }
    __syncthreads();
    for (int i = tid; i < GL::NOWN * NV * S; i += BLOCK) {
      const int slot = i / (NV * S), j = i - slot * NV * S;
      if (owner[slot] >= 0 && !fvdata[slot]) ou[i] = w.Qold[owner[slot] * NV * S + j];
    }
    __syncthreads();
    for (int p = tid; p < NB; p += BLOCK) {
      int x[3];
      lim_multi<DIM>(p, EB, x);
      int outside = 0, far = 0, po[3] = {0, 0, 0}, ss[3] = {0, 0, 0};
      bool flip[3] = {false, false, false};
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int r = x[d] - 2;
        if (r < 0 || r >= m) {
          ++outside;
          const int side = r >= m, to = cc[d] + (side ? 1 : -1);
          if ((to < 0 || to >= a.cells[d]) && a.bc[2 * d + side] != ADG_BC_PERIODIC) {
            ss[d] = side ? 2 * m - 1 - r : -1 - r;
            flip[d] = a.bc[2 * d + side] == ADG_BC_WALL;
          } else {
            po[d] = side ? 1 : -1;
            ss[d] = r - po[d] * m;
          }
        } else {
          ss[d] = r;
        }
        if (r < -1 || r > m) ++far;
      }
      if (outside > 2 || (outside == 2 && far > 0)) continue;
      // slot of the offset po
      const int kpo = (po[0] + 1) + 3 * (po[1] + 1) + (DIM == 3 ? 9 * (po[2] + 1) : 0);
      // rank of kpo among the offsets with at most two nonzero entries: in
      // 3-D the eight corners k = 0, 2, 6, 8, 18, 20, 24, 26 are left out
      const int slot = DIM == 2 ? kpo
                                : kpo - ((kpo > 0) + (kpo > 2) + (kpo > 6) + (kpo > 8) + (kpo > 18) + (kpo > 20) +
                                         (kpo > 24));
      const long long o = owner[slot];
      double val[NV];
      if (fvdata[slot]) {
        const int si = ss[0] + m * (ss[1] + m * ss[2]);
#pragma unroll
        for (int v = 0; v < NV; ++v) val[v] = sub_in[(o * NV + v) * NS + si];
      } else {
        const double* uo = ou + slot * NV * S;
#pragma unroll
        for (int v = 0; v < NV; ++v) val[v] = 0.0;
        for (int kk = 0; kk < S; ++kk) {
          const int kx = kk % n, ky = (kk / n) % n, kz = DIM == 3 ? kk / (n * n) : 0;
          double cf = A[ss[0] * n + kx] * A[ss[1] * n + ky];
          if (DIM == 3) cf *= A[ss[2] * n + kz];
#pragma unroll
          for (int v = 0; v < NV; ++v) val[v] += cf * uo[v * S + kk];
        }
      }
#pragma unroll
      for (int d = 0; d < DIM; ++d)
        if (flip[d]) val[1 + d] = -val[1 + d];
#pragma unroll
      for (int v = 0; v < NV; ++v) box[v * NB + p] = val[v];
    }
    __syncthreads();
    // 2. minmod slopes, extrapolated values and their half-step correction
    //    for the cell's subcells and the first ghost layer across each face
    for (int q = tid; q < NC; q += BLOCK) {
      int x[3];
      lim_multi<DIM>(q, EC, x);
      int outside = 0, p = 0, mul = 1;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int r = x[d] - 1;
        if (r < 0 || r >= m) ++outside;
        p += (r + 2) * mul;
        mul *= EB;
      }
      if (outside > 1) continue;
      double ext[DIM][2][NV], cv[NV];
      bool ok = true;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int sd = d == 0 ? 1 : (d == 1 ? EB : EB * EB);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double wv = box[v * NB + p];
          const double slope = lim_minmod(wv - box[v * NB + p - sd], box[v * NB + p + sd] - wv);
          ext[d][0][v] = wv - 0.5 * slope;
          ext[d][1][v] = wv + 0.5 * slope;
        }
        ok = ok && PDE::admissible(ext[d][0], ext[d][0], a.pde) && PDE::admissible(ext[d][1], ext[d][1], a.pde);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) cv[v] = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        double Fl[DIM][NV], Fr[DIM][NV];
        PDE::fluxes(ext[d][0], ext[d][0], a.pde, Fl);
        PDE::fluxes(ext[d][1], ext[d][1], a.pde, Fr);
#pragma unroll
        for (int v = 0; v < NV; ++v) cv[v] += 0.5 * dt / hs[d] * (Fl[d][v] - Fr[d][v]);
      }
#pragma unroll
      for (int d = 0; d < DIM; ++d)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          double mv[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) mv[v] = ext[d][side][v] + cv[v];
          ok = ok && PDE::admissible(mv, mv, a.pde);
        }
#pragma unroll
      for (int v = 0; v < NV; ++v) corr[v * NC + q] = cv[v];
      okf[q] = ok ? 1 : 0;
    }
    __syncthreads();
    // 3. Rusanov at the subcell faces and the update of the cell's subcells
    double vnew[GL::VPT][NV];
#pragma unroll
    for (int j = 0; j < GL::VPT; ++j) {
      const int s = tid + j * BLOCK;
      if (s >= NS) break;
      int x[3];
      lim_multi<DIM>(s, m, x);
      int p = 0, q = 0, mb = 1, mc = 1;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        p += (x[d] + 2) * mb;
        q += (x[d] + 1) * mc;
        mb *= EB;
        mc *= EC;
      }
      double acc[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int sd = d == 0 ? 1 : (d == 1 ? EB : EB * EB), cd = d == 0 ? 1 : (d == 1 ? EC : EC * EC);
        double e0[NV], e1[NV], Ghi[NV], Glo[NV];
        lim_moved<PDE, N>(box, corr, okf, p, q, d, 1, e0);
        lim_moved<PDE, N>(box, corr, okf, p + sd, q + cd, d, 0, e1);
        lim_rusanov<PDE>(a.pde, d, e0, e1, Ghi);
        lim_moved<PDE, N>(box, corr, okf, p - sd, q - cd, d, 1, e0);
        lim_moved<PDE, N>(box, corr, okf, p, q, d, 0, e1);
        lim_rusanov<PDE>(a.pde, d, e0, e1, Glo);
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += (Ghi[v] - Glo[v]) / hs[d];
        // subface index across the other axes, lower axis fastest
        const int t = DIM == 2 ? x[1 - d] : (d == 0 ? x[1] + m * x[2] : (d == 1 ? x[0] + m * x[2] : x[0] + m * x[1]));
        if (x[d] == m - 1)
#pragma unroll
          for (int v = 0; v < NV; ++v) fsub[((2 * d + 1) * NSF + t) * NV + v] = Ghi[v];
        if (x[d] == 0)
#pragma unroll
          for (int v = 0; v < NV; ++v) fsub[((2 * d) * NSF + t) * NV + v] = Glo[v];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        vnew[j][v] = box[v * NB + p] - dt * acc[v];
        sub_out[(c * NV + v) * NS + s] = vnew[j][v];
      }
    }
    __syncthreads();
    // 4. back to the DG space, and the face-node fluxes for DG neighbours
    double* vn = box;
#pragma unroll
    for (int j = 0; j < GL::VPT; ++j) {
      const int s = tid + j * BLOCK;
      if (s < NS)
#pragma unroll
        for (int v = 0; v < NV; ++v) vn[v * NS + s] = vnew[j][v];
    }
    __syncthreads();
    // least-squares fit, one axis at a time: x (vn -> r1), y (r1 -> r2,
    // 3-D), the last axis into Q
    {
      using LC = LimConst<n>;
      double* r1 = box + NV * NS;  // [v][(sz)][sy][kx]
      double* r2 = corr;           // 3-D: [v][sz][ky][kx]
      constexpr int L1 = NV * ipow(m, DIM - 1);
      for (int line = tid; line < L1; line += BLOCK) {
        double in[m];
#pragma unroll
        for (int j = 0; j < m; ++j) in[j] = vn[line * m + j];
#pragma unroll
        for (int k = 0; k < n; ++k) {
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < m; ++j) acc += LC::B[k][j] * in[j];
          r1[line * n + k] = acc;
        }
      }
      __syncthreads();
      const double* rl = r1;
      if constexpr (DIM == 3) {
        for (int line = tid; line < NV * m * n; line += BLOCK) {
          const int kx = line % n, vz = line / n;  // vz = v m + sz
          double in[m];
#pragma unroll
          for (int j = 0; j < m; ++j) in[j] = r1[(vz * m + j) * n + kx];
#pragma unroll
          for (int k = 0; k < n; ++k) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < m; ++j) acc += LC::B[k][j] * in[j];
            r2[(vz * n + k) * n + kx] = acc;
          }
        }
        __syncthreads();
        rl = r2;
      }
      constexpr int RL = ipow(n, DIM - 1);  // lines per variable of the last stage
      for (int line = tid; line < NV * RL; line += BLOCK) {
        const int v = line / RL, r = line - v * RL;
        double in[m];
#pragma unroll
        for (int j = 0; j < m; ++j) in[j] = rl[(v * m + j) * RL + r];
#pragma unroll
        for (int k = 0; k < n; ++k) {
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < m; ++j) acc += LC::B[k][j] * in[j];
          Q[c * NV * S + v * S + k * RL + r] = acc;
        }
      }
    }
    for (int i = tid; i < 2 * DIM * NV * F; i += BLOCK) {
      const int f = i % F, v = (i / F) % NV, face = i / (F * NV);
      const int f0 = f % n, f1 = f / n;
      double acc = 0.0;
      for (int t = 0; t < NSF; ++t) {
        const int t0 = t % m, t1 = t / m;
        double qv = Qf[f0 * m + t0];
        if (DIM == 3) qv *= Qf[f1 * m + t1];
        acc += qv * fsub[(face * NSF + t) * NV + v];
      }
      w.gfv[((c * 2 * DIM + face) * NV + v) * F + f] = acc;
    }
  }
}

// DG cells with an FV face: the Rusanov flux of that face in the
// candidate's update exchanged for the FV one.  Persistent grid over the
// list.
template <class PDE, int N>
__global__ void __launch_bounds__(256)
lim_faces_kernel(const KArgs a, const double* __restrict__ clock, const double* __restrict__ traces,
                 const uint8_t* __restrict__ status, double* __restrict__ Q, const LimWork w) {
  using GL = GeoLim<PDE, N>;
  constexpr int DIM = GL::DIM, NV = GL::NV, S = GL::S, F = GL::F, n = GL::n, BLOCK = 256;
  const Tables<double>& T = a.t64;
  const double dt = clock[1];
  const int count = w.counters[2];
  for (int it = blockIdx.x; it < count; it += gridDim.x) {
    const long long c = w.y_list[it];
    for (int i = threadIdx.x; i < NV * S; i += BLOCK) {
      const int v = i / S, k = i - v * S;
      const int kk[3] = {k % n, (k / n) % n, DIM == 3 ? k / (n * n) : 0};
      double delta = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          const long long o = lim_neighbour<DIM>(a, c, d, side ? 1 : -1);
          if (o < 0 || status[o] < 2) continue;
          const int f = DIM == 2 ? kk[1 - d] : (d == 0 ? kk[1] + n * kk[2] : (d == 1 ? kk[0] + n * kk[2] : kk[0] + n * kk[1]));
          const long long cL = side ? c : o, cR = side ? o : c;
          const double* tL = traces + ((cL * (2 * DIM) + 2 * d + 1) * 2) * NV * F;
          const double* tR = traces + ((cR * (2 * DIM) + 2 * d) * 2) * NV * F;
          double qL[NV], qR[NV];
#pragma unroll
          for (int u = 0; u < NV; ++u) {
            qL[u] = tL[u * F + f];
            qR[u] = tR[u * F + f];
          }
          const double s = fmax(PDE::max_eigen(qL, qL, a.pde, d), PDE::max_eigen(qR, qR, a.pde, d));
          const double G = 0.5 * (tL[(NV + v) * F + f] + tR[(NV + v) * F + f]) - 0.5 * s * (qR[v] - qL[v]);
          const double Gfv = w.gfv[((o * 2 * DIM + 2 * d + 1 - side) * NV + v) * F + f];
          const double dG = (Gfv - G) * T.invw[kk[d]] * a.inv_h[d];
          delta += side ? T.l1[kk[d]] * dG : -T.l0[kk[d]] * dG;
        }
      Q[c * NV * S + i] -= dt * delta;
    }
  }
}

// Eq. (7) after a limited step: the largest signal speed over the nodal
// values of DG cells and the subcell averages of FV cells (an FV cell's
// solution; its least-squares polynomial can hold non-physical nodes).  One
// wave per cell; block maxima into the reduction slots.
template <class PDE, int N>
__global__ void __launch_bounds__(256)
lim_lambda_kernel(const KArgs a, const double* __restrict__ Q, const double* __restrict__ sub,
                  const uint8_t* __restrict__ status) {
  using GL = GeoLim<PDE, N>;
  constexpr int DIM = GL::DIM, NV = GL::NV, S = GL::S, NS = GL::NS;
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const long long c = (long long)blockIdx.x * 4 + wv;
  double lam = 0.0;
  if (c < a.ncells) {
    const bool fv = status[c] >= 2;
    const int npts = fv ? NS : S;
    const double* base = fv ? sub + c * NV * NS : Q + c * NV * S;
    for (int k = lane; k < npts; k += 64) {
      double q[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) q[v] = base[v * npts + k];
#pragma unroll
      for (int d = 0; d < DIM; ++d) lam = lam_max(lam, PDE::max_eigen(q, q, a.pde, d));
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) lam = lam_max(lam, __shfl_xor(lam, off, 64));
  if (lane == 0) red[wv] = lam;
  __syncthreads();
  if (tid == 0) slot_max(a.slots, blockIdx.x, lam_max(lam_max(red[0], red[1]), lam_max(red[2], red[3])));
}

template <class PDE, int N>
struct LimLaunch {
  using GL = GeoLim<PDE, N>;
  static constexpr int kFvGrid = 512, kFaceGrid = 1024;
  // prepare; the caller's DG step follows
  static hipError_t before(const KArgs& a, const double* Q, const double* sub_in, const uint8_t* status,
                           const LimWork& w, hipStream_t st) {
    const unsigned grid = GeoLimSeq<PDE, N>::grid(a.ncells);
    hipLaunchKernelGGL((lim_prepare_kernel<PDE, N>), dim3(grid), dim3(64 * GeoLimW<PDE, N>::WPB), 0, st, a, Q,
                       sub_in, status, w);
    return hipGetLastError();
  }
  // detect, classify, FV cells, DG cells with FV faces
  static hipError_t after(const KArgs& a, double* Q, double* clock, const double* traces,
                          const double* sub_in, double* sub_out, uint8_t* status, const LimWork& w,
                          int next_dt, hipStream_t st) {
    const unsigned grid = GeoLimSeq<PDE, N>::grid(a.ncells);
    hipLaunchKernelGGL((lim_detect_kernel<PDE, N>), dim3(grid), dim3(64 * GeoLimW<PDE, N>::WPB), 0, st, a, Q, w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((lim_classify_kernel<GL::DIM>), dim3((unsigned)((a.ncells + 255) / 256)), dim3(256), 0, st,
                       a, status, w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((lim_fv_kernel<PDE, N>), dim3(kFvGrid), dim3(GL::BLOCK), 0, st, a, clock, sub_in, Q,
                       sub_out, w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((lim_faces_kernel<PDE, N>), dim3(kFaceGrid), dim3(256), 0, st, a, clock, traces,
                       status, Q, w);
    if ((e = hipGetLastError()) != hipSuccess || !next_dt) return e;
    hipLaunchKernelGGL((lim_lambda_kernel<PDE, N>), dim3((unsigned)((a.ncells + 3) / 4)), dim3(256), 0, st, a, Q,
                       sub_out, status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kSlots), 0, st, a.slots, a.dt_factor, 1, clock);
    return hipGetLastError();
  }
};

}  // namespace adg

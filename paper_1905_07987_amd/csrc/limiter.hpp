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
  static constexpr int BLOCK = 256;
  static constexpr int VPT = (NS + BLOCK - 1) / BLOCK;  // subcells per thread in the update
  // prepare and detect: tables, nodal values, the contraction stages
  static constexpr int PJ1 = NV * m * ipow(n, DIM - 1), PJ2 = DIM == 3 ? NV * m * m * n : 0;
  static constexpr int PJ_D = NTAB + NV * S + PJ1 + PJ2 + NV * NS;
  // fv: tables, the subcell box, the half-step corrections, the subface fluxes
  static constexpr int FV_D = NTAB + NV * (NB + NC + 2 * DIM * NSF);
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

// One contraction stage of the projection onto the subcells: axis ax of the
// tensor in[NV][e2][e1][e0] (x fastest) goes from extent ein to mo through
// M[mo][ein].
template <int BLOCK>
__device__ __forceinline__ void lim_stage(const double* in, double* out, int nv, int e0, int e1, int e2, int ax,
                                          int mo, const double* M, int tid) {
  const int ein = ax == 0 ? e0 : (ax == 1 ? e1 : e2);
  const int o0 = ax == 0 ? mo : e0, o1 = ax == 1 ? mo : e1, o2 = ax == 2 ? mo : e2;
  const int per = o0 * o1 * o2, stride = ax == 0 ? 1 : (ax == 1 ? e0 : e0 * e1);
  for (int i = tid; i < nv * per; i += BLOCK) {
    const int v = i / per, r = i - v * per;
    const int x0 = r % o0, x1 = (r / o0) % o1, x2 = r / (o0 * o1);
    const int xo = ax == 0 ? x0 : (ax == 1 ? x1 : x2);
    const double* src = in + v * (e0 * e1 * e2) + (ax == 0 ? 0 : x0) + e0 * ((ax == 1 ? 0 : x1) + e1 * (ax == 2 ? 0 : x2));
    double acc = 0.0;
    for (int k = 0; k < ein; ++k) acc += M[xo * ein + k] * src[k * stride];
    out[i] = acc;
  }
}

// Subcell averages of the nodal values u[NV][S] (LDS) into out[NV][NS].
template <class PDE, int N>
__device__ __forceinline__ void lim_project_block(const double* T, const double* u, double* t1, double* t2,
                                                  double* out, int tid) {
  using GL = GeoLim<PDE, N>;
  constexpr int n = GL::n, m = GL::m, NV = GL::NV;
  if constexpr (GL::DIM == 2) {
    lim_stage<GL::BLOCK>(u, t1, NV, n, n, 1, 0, m, T, tid);
    __syncthreads();
    lim_stage<GL::BLOCK>(t1, out, NV, m, n, 1, 1, m, T, tid);
  } else {
    lim_stage<GL::BLOCK>(u, t1, NV, n, n, n, 0, m, T, tid);
    __syncthreads();
    lim_stage<GL::BLOCK>(t1, t2, NV, m, n, n, 1, m, T, tid);
    __syncthreads();
    lim_stage<GL::BLOCK>(t2, out, NV, m, m, n, 2, m, T, tid);
  }
  __syncthreads();
}

// Block-wide min and max of (lo, hi); the result is valid in thread 0.
template <int BLOCK>
__device__ __forceinline__ void lim_minmax(double& lo, double& hi, double* red) {
  red[threadIdx.x] = lo;
  red[BLOCK + threadIdx.x] = hi;
  __syncthreads();
  for (int off = BLOCK / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + off]);
      red[BLOCK + threadIdx.x] = fmax(red[BLOCK + threadIdx.x], red[BLOCK + threadIdx.x + off]);
    }
    __syncthreads();
  }
  lo = red[0];
  hi = red[BLOCK];
  __syncthreads();
}

// One block per cell: u^n copied, status kept, range of the subcell
// averages at t^n.  Block 0 clears the counters of the step.
template <class PDE, int N>
__global__ void __launch_bounds__(256)
lim_prepare_kernel(const KArgs a, const double* __restrict__ Q, const double* __restrict__ sub_in,
                   const uint8_t* __restrict__ status, const LimWork w) {
  using GL = GeoLim<PDE, N>;
  constexpr int NV = GL::NV, S = GL::S, NS = GL::NS, BLOCK = GL::BLOCK;
  __shared__ double lds[GL::PJ_D];
  __shared__ double red[2 * BLOCK];
  double* T = lds;
  double* u = T + GL::NTAB;
  double* t1 = u + NV * S;
  double* t2 = t1 + GL::PJ1;
  double* pv = t2 + GL::PJ2;
  const int tid = threadIdx.x;
  const long long c = blockIdx.x;
  if (c == 0 && tid < 4) w.counters[tid] = 0;
  for (int i = tid; i < GL::NTAB; i += BLOCK) T[i] = w.tab[i];
  for (int i = tid; i < NV * S; i += BLOCK) {
    const double x = Q[c * NV * S + i];
    u[i] = x;
    w.Qold[c * NV * S + i] = x;
  }
  const uint8_t st = status[c];
  if (tid == 0) w.st_prev[c] = st;
  __syncthreads();
  const double* W = pv;
  if (st >= 2) W = sub_in + c * NV * NS;
  else lim_project_block<PDE, N>(T, u, t1, t2, pv, tid);
  for (int v = 0; v < NV; ++v) {
    double lo = INFINITY, hi = -INFINITY;
    for (int s = tid; s < NS; s += BLOCK) {
      lo = fmin(lo, W[v * NS + s]);
      hi = fmax(hi, W[v * NS + s]);
    }
    lim_minmax<BLOCK>(lo, hi, red);
    if (tid == 0) {
      w.lohi[(c * NV + v) * 2] = lo;
      w.lohi[(c * NV + v) * 2 + 1] = hi;
    }
  }
}

// One block per cell: is the candidate troubled?
template <class PDE, int N>
__global__ void __launch_bounds__(256)
lim_detect_kernel(const KArgs a, const double* __restrict__ Q, const LimWork w) {
  using GL = GeoLim<PDE, N>;
  constexpr int DIM = GL::DIM, NV = GL::NV, S = GL::S, NS = GL::NS, BLOCK = GL::BLOCK;
  __shared__ double lds[GL::PJ_D];
  __shared__ double bounds[NV][2];
  double* T = lds;
  double* u = T + GL::NTAB;
  double* t1 = u + NV * S;
  double* t2 = t1 + GL::PJ1;
  double* pv = t2 + GL::PJ2;
  const int tid = threadIdx.x;
  const long long c = blockIdx.x;
  for (int i = tid; i < GL::NTAB; i += BLOCK) T[i] = w.tab[i];
  for (int i = tid; i < NV * S; i += BLOCK) u[i] = Q[c * NV * S + i];
  if (tid < NV) {
    double lo = w.lohi[(c * NV + tid) * 2], hi = w.lohi[(c * NV + tid) * 2 + 1];
    for (int d = 0; d < DIM; ++d)
      for (int s = -1; s <= 1; s += 2) {
        const long long o = lim_neighbour<DIM>(a, c, d, s);
        if (o < 0) continue;
        lo = fmin(lo, w.lohi[(o * NV + tid) * 2]);
        hi = fmax(hi, w.lohi[(o * NV + tid) * 2 + 1]);
      }
    bounds[tid][0] = lo;
    bounds[tid][1] = hi;
  }
  __syncthreads();
  bool bad = false;
  for (int k = tid; k < S; k += BLOCK) {
    double q[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = u[v * S + k];
    bad = bad || !PDE::admissible(q, q, a.pde);
  }
  lim_project_block<PDE, N>(T, u, t1, t2, pv, tid);
  for (int s = tid; s < NS; s += BLOCK) {
    double q[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = pv[v * NS + s];
    bad = bad || !PDE::admissible(q, q, a.pde);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double lo = bounds[v][0], hi = bounds[v][1];
      const double delta = fmax(1e-4, 1e-3 * (hi - lo));
      bad = bad || !(q[v] >= lo - delta && q[v] <= hi + delta);
    }
  }
  bad = __syncthreads_or(bad);
  if (tid == 0) {
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

// The subcell average at t^n of a subcell box position whose global subcell
// index is g: the owner's FV data, or the projection of its DG polynomial.
template <class PDE, int N>
__device__ __forceinline__ void lim_ghost_value(const KArgs& a, const double* T, const double* __restrict__ Qold,
                                                const double* __restrict__ sub_in,
                                                const uint8_t* __restrict__ st_prev, const int (&gin)[3],
                                                double (&out)[PDE::NV]) {
  using GL = GeoLim<PDE, N>;
  constexpr int DIM = GL::DIM, NV = GL::NV, S = GL::S, NS = GL::NS, m = GL::m, n = GL::n;
  int g[3] = {gin[0], gin[1], gin[2]}, cc[3] = {0, 0, 0}, ss[3] = {0, 0, 0};
  bool flip[3] = {false, false, false};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int G = m * a.cells[d];
    if (g[d] < 0 || g[d] >= G) {
      const int side = g[d] >= G, kind = a.bc[2 * d + side];
      if (kind == ADG_BC_PERIODIC) {
        g[d] = ((g[d] % G) + G) % G;
      } else {
        g[d] = side ? 2 * G - 1 - g[d] : -1 - g[d];
        flip[d] = kind == ADG_BC_WALL;
      }
    }
    cc[d] = g[d] / m;
    ss[d] = g[d] - cc[d] * m;
  }
  const long long o = cc[0] + (long long)a.cells[0] * (cc[1] + (long long)a.cells[1] * cc[2]);
  if (st_prev[o] >= 2) {
    const int si = ss[0] + m * (ss[1] + m * ss[2]);
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = sub_in[(o * NV + v) * NS + si];
  } else {
    const double* u = Qold + o * NV * S;
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = 0.0;
    for (int k = 0; k < S; ++k) {
      const int kx = k % n, ky = (k / n) % n, kz = DIM == 3 ? k / (n * n) : 0;
      double c = T[ss[0] * n + kx] * T[ss[1] * n + ky];
      if (DIM == 3) c *= T[ss[2] * n + kz];
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v] += c * u[v * S + k];
    }
  }
#pragma unroll
  for (int d = 0; d < DIM; ++d)
    if (flip[d]) out[1 + d] = -out[1 + d];
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
__global__ void __launch_bounds__(256)
lim_fv_kernel(const KArgs a, const double* __restrict__ clock, const double* __restrict__ sub_in, double* __restrict__ Q,
              double* __restrict__ sub_out, const LimWork w) {
  using GL = GeoLim<PDE, N>;
  constexpr int DIM = GL::DIM, NV = GL::NV, S = GL::S, NS = GL::NS, NSF = GL::NSF, F = GL::F;
  constexpr int m = GL::m, n = GL::n, EB = GL::EB, NB = GL::NB, EC = GL::EC, NC = GL::NC, BLOCK = GL::BLOCK;
  __shared__ double lds[GL::FV_D];
  __shared__ uint8_t okf[NC];
  double* T = lds;
  double* box = T + GL::NTAB;
  double* corr = box + NV * NB;
  double* fsub = corr + NV * NC;
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
    //    across each edge (corners are never read)
    for (int p = tid; p < NB; p += BLOCK) {
      int x[3];
      lim_multi<DIM>(p, EB, x);
      int outside = 0, far = 0, g[3] = {0, 0, 0};
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int r = x[d] - 2;
        if (r < 0 || r >= m) ++outside;
        if (r < -1 || r > m) ++far;
        g[d] = cc[d] * m + r;
      }
      if (outside > 2 || (outside == 2 && far > 0)) continue;
      double val[NV];
      lim_ghost_value<PDE, N>(a, T, w.Qold, sub_in, w.st_prev, g, val);
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
    for (int i = tid; i < NV * S; i += BLOCK) {
      const int v = i / S, k = i - v * S;
      const int kx = k % n, ky = (k / n) % n, kz = DIM == 3 ? k / (n * n) : 0;
      double acc = 0.0;
      for (int s = 0; s < NS; ++s) {
        const int sx = s % m, sy = (s / m) % m, sz = DIM == 3 ? s / (m * m) : 0;
        double b = B[kx * m + sx] * B[ky * m + sy];
        if (DIM == 3) b *= B[kz * m + sz];
        acc += b * vn[v * NS + s];
      }
      Q[c * NV * S + i] = acc;
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
  constexpr int DIM = GL::DIM, NV = GL::NV, S = GL::S, F = GL::F, n = GL::n, BLOCK = GL::BLOCK;
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

template <class PDE, int N>
struct LimLaunch {
  using GL = GeoLim<PDE, N>;
  static constexpr int kFvGrid = 512, kFaceGrid = 1024;
  // prepare; the caller's DG step follows
  static hipError_t before(const KArgs& a, const double* Q, const double* sub_in, const uint8_t* status,
                           const LimWork& w, hipStream_t st) {
    hipLaunchKernelGGL((lim_prepare_kernel<PDE, N>), dim3((unsigned)a.ncells), dim3(GL::BLOCK), 0, st, a, Q,
                       sub_in, status, w);
    return hipGetLastError();
  }
  // detect, classify, FV cells, DG cells with FV faces
  static hipError_t after(const KArgs& a, double* Q, const double* clock, const double* traces,
                          const double* sub_in, double* sub_out, uint8_t* status, const LimWork& w,
                          hipStream_t st) {
    hipLaunchKernelGGL((lim_detect_kernel<PDE, N>), dim3((unsigned)a.ncells), dim3(GL::BLOCK), 0, st, a, Q, w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((lim_classify_kernel<GL::DIM>), dim3((unsigned)((a.ncells + 255) / 256)), dim3(256), 0, st,
                       a, status, w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((lim_fv_kernel<PDE, N>), dim3(kFvGrid), dim3(GL::BLOCK), 0, st, a, clock, sub_in, Q,
                       sub_out, w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((lim_faces_kernel<PDE, N>), dim3(kFaceGrid), dim3(GL::BLOCK), 0, st, a, clock, traces,
                       status, Q, w);
    return hipGetLastError();
  }
};

}  // namespace adg

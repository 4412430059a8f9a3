// HIP kernels of one ADER-DG step for gfx950, templated on the PDE, the
// polynomial degree N and (for the predictor) the arithmetic type.
//
// Work mapping: one cell per group of S = n^dim threads, one thread per
// spatial node k; CPB cells share a block so that blocks hold ~256 lanes.
// The thread of node k keeps the whole time history q[j][v] (j = 0..N) of its
// node in registers, so the predictor's time operator (ExaHyPE paper,
// Sec. 3.3, Eq. (5): q^{r+1}_i = u + dt sum_j (K1^{-1})_ij w_j R_j) is
// thread-local.  Spatial derivatives need whole lines of a cell: fluxes (and
// the quantities whose gradient the non-conservative product reads) of a
// chunk of time slices are written to LDS, one thread per (slice, direction,
// line) differentiates its line in place, and every node thread reads its
// derivatives back.  Face traces and the volume term come from the same line
// tasks applied to the time averages.
#pragma once

#include <hip/hip_runtime.h>

#include "adg_internal.hpp"
#include "pde.hpp"

namespace adg {

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int cmin(int a, int b) { return a < b ? a : b; }

template <class PDE, int N>
struct Geo {
  static constexpr int DIM = PDE::DIM;
  static constexpr int n = N + 1;
  static constexpr int S = ipow(n, DIM);   // nodes per cell
  static constexpr int F = S / n;          // nodes per face == lines per direction
  static constexpr int NV = PDE::NV, NP = PDE::NP;
  static constexpr int CPB = S >= 256 ? 1 : 256 / S;  // cells per block
  static constexpr int BLOCK = CPB * S;
  static constexpr int SP = S + S / n;     // LDS row: one pad slot per x-row
  static_assert(BLOCK >= 64 && BLOCK <= 1024, "block must hold one full wave");
  __host__ __device__ static constexpr int pidx(int k) { return k + k / n; }
};

// Derivative channels per direction: the nonzero flux components, then the
// quantities whose gradient feeds the non-conservative product.
template <class PDE>
struct Chan {
  static constexpr int nflux(int d) {
    int c = 0;
    for (int v = 0; v < PDE::NV; ++v) c += PDE::flux_nonzero(d, v) ? 1 : 0;
    return c;
  }
  static constexpr int flux_var(int d, int c) {
    for (int v = 0; v < PDE::NV; ++v)
      if (PDE::flux_nonzero(d, v) && c-- == 0) return v;
    return -1;
  }
  static constexpr int ngrad() {
    int c = 0;
    for (int v = 0; v < PDE::NV; ++v) c += PDE::grad_needed(v) ? 1 : 0;
    return c;
  }
  static constexpr int grad_var(int c) {
    for (int v = 0; v < PDE::NV; ++v)
      if (PDE::grad_needed(v) && c-- == 0) return v;
    return -1;
  }
  static constexpr int NCHD = nflux(0) + ngrad();  // channels per direction
  static constexpr int NCH = PDE::DIM * NCHD;
  static constexpr int NFLUX = nflux(0);
  static constexpr bool uniform() {
    for (int d = 0; d < PDE::DIM; ++d)
      if (nflux(d) != nflux(0)) return false;
    return true;
  }
};

// Time slices per LDS chunk: enough line tasks for the block, within 64 KiB.
template <class PDE, int N, class R>
struct Chunk {
  using G = Geo<PDE, N>;
  using C = Chan<PDE>;
  static constexpr int want = (G::n + G::DIM - 1) / G::DIM;
  static constexpr int per_slot = G::CPB * C::NCH * G::SP * (int)sizeof(R);
  static constexpr int fit = (64 * 1024) / per_slot;
  static constexpr int TC = cmax(1, cmin(want, fit));
  static constexpr int ITER_ELEMS = G::CPB * TC * C::NCH * G::SP;
  static constexpr int FIN_ELEMS = G::CPB * (G::NV + C::NFLUX) * G::SP;
  static constexpr int ELEMS = cmax(ITER_ELEMS, FIN_ELEMS);
};

template <class R>
__device__ __forceinline__ const Tables<R>& tables(const KArgs& a);
template <>
__device__ __forceinline__ const Tables<double>& tables<double>(const KArgs& a) {
  return a.t64;
}
template <>
__device__ __forceinline__ const Tables<float>& tables<float>(const KArgs& a) {
  return a.t32;
}

// Block -> cell-block map that gives each of the 8 XCDs (blocks are dealt to
// XCDs round-robin) one contiguous range of cells, so face neighbours along x
// and y mostly share an L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

template <int DIM>
__device__ __forceinline__ void node_coords(int k, int n, int* kk) {
  kk[0] = k % n;
  kk[1] = (k / n) % n;
  if (DIM == 3) kk[2] = k / (n * n);
}

// First node and stride of line l (the face-node index) along direction d.
template <int DIM>
__device__ __forceinline__ void line_geom(int d, int l, int n, int& base, int& stride) {
  if (DIM == 2) {
    base = d == 0 ? l * n : l;
    stride = d == 0 ? 1 : n;
  } else {
    const int a = l % n, b = l / n;  // remaining axes, lower one first
    if (d == 0) { base = n * a + n * n * b; stride = 1; }
    else if (d == 1) { base = a + n * n * b; stride = n; }
    else { base = a + n * b; stride = n * n; }
  }
}

// Block-level max of non-negative doubles; returns the block max in thread 0.
// Every thread stores its value in LDS; the first wave (always complete:
// BLOCK >= 64) folds the block and reduces across its lanes, so no shuffle
// ever reads a lane that does not exist in a partial last wave.
template <int BLOCK>
__device__ __forceinline__ double block_max(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  double m = 0.0;
  if (threadIdx.x < 64) {
    for (int i = threadIdx.x; i < BLOCK; i += 64) m = fmax(m, red[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  }
  return m;
}

// Grid-wide completion: returns true in thread 0 of the last block to finish.
__device__ __forceinline__ bool last_block(unsigned int* counter, bool* flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned prev = atomicAdd(counter, 1u);
    *flag = (prev == gridDim.x - 1);
  }
  __syncthreads();
  return *flag && threadIdx.x == 0;
}

__device__ __forceinline__ double ricker(double f0, double t0, double amp, double t) {
  const double pi = 3.14159265358979323846;
  double x = pi * f0 * (t - t0);
  x = x * x;
  return amp * (1.0 - 2.0 * x) * exp(-x);
}

// ---------------------------------------------------------------------------
// Kernel A: predictor, time averages, volume term and face projection.
// ---------------------------------------------------------------------------
template <class PDE, int N, class R>
__global__ void __launch_bounds__((Geo<PDE, N>::BLOCK))
predict_kernel(const KArgs a, const double* Q, const double* __restrict__ params,
               const double* __restrict__ clock, double* Qout, double* __restrict__ traces) {
  // Q and Qout may be the same array (in-place step): each element is read
  // once at the start and written once at the end by the same thread.
  using G = Geo<PDE, N>;
  using C = Chan<PDE>;
  using K = Chunk<PDE, N, R>;
  constexpr int n = G::n, S = G::S, F = G::F, NV = G::NV, NP = G::NP, DIM = G::DIM;
  constexpr int CPB = G::CPB, BLOCK = G::BLOCK, SP = G::SP, TC = K::TC;
  constexpr int NCH = C::NCH, NCHD = C::NCHD, NFL = C::NFLUX, NGR = C::ngrad();
  static_assert(C::uniform(), "flux sparsity must be the same in every direction");
  __shared__ R lds[K::ELEMS];

  const Tables<R>& T = tables<R>(a);
  const int tid = threadIdx.x;
  const int lc = tid / S, k = tid - lc * S;
  const long long cell0 = (long long)xcd_block(blockIdx.x, a.nblocks) * CPB;
  const long long cell = cell0 + lc;
  const bool active = cell < a.ncells;
  const long long cl = active ? cell : a.ncells - 1;  // clamp loads of the ragged tail

  int kk[3] = {0, 0, 0};
  node_coords<DIM>(k, n, kk);

  double u64[NV];
  R u[NV], P[NP > 0 ? NP : 1];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    u64[v] = Q[(cl * NV + v) * S + k];
    u[v] = R(u64[v]);
  }
#pragma unroll
  for (int p = 0; p < NP; ++p) P[p] = R(params[cl * NP + p]);
  const double t_n = clock[0], dt64 = clock[1];
  const R dt = R(dt64);
  R inv_h[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) inv_h[d] = R(a.inv_h[d]);

  R q[n][NV];
#pragma unroll
  for (int j = 0; j < n; ++j)
#pragma unroll
    for (int v = 0; v < NV; ++v) q[j][v] = u[v];

  R Fbar[DIM][NV], Nbar[NV], Sbar[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    Nbar[v] = Sbar[v] = R(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) Fbar[d][v] = R(0);
  }

  R* const mine = lds + lc * (TC * NCH * SP);  // this cell's chunk region
  const int I = a.picard_iters;

  for (int r = 0; r <= I; ++r) {
    const bool fin = (r == I);  // final pass: averages at the last iterate
    R acc[n][NV];
#pragma unroll
    for (int i = 0; i < n; ++i)
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[i][v] = R(0);

#pragma unroll
    for (int c0 = 0; c0 < n; c0 += TC) {
      const int cnt = cmin(TC, n - c0);
      // (1) fluxes and gradient inputs of the chunk's slices -> LDS
#pragma unroll
      for (int jj = 0; jj < TC; ++jj) {
        if (c0 + jj >= n) break;
        const int j = c0 + jj;
        R Fl[DIM][NV];
        PDE::fluxes(q[j], P, a.pde, Fl);
        if (fin) {
#pragma unroll
          for (int d = 0; d < DIM; ++d)
#pragma unroll
            for (int v = 0; v < NV; ++v) Fbar[d][v] += T.w[j] * Fl[d][v];
        }
        if (!fin || PDE::kHasNcp) {
          R* slot = mine + jj * NCH * SP;
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
#pragma unroll
            for (int c = 0; c < NFL; ++c)
              slot[(d * NCHD + c) * SP + G::pidx(k)] = Fl[d][C::flux_var(d, c)];
#pragma unroll
            for (int c = 0; c < NGR; ++c)
              slot[(d * NCHD + NFL + c) * SP + G::pidx(k)] = q[j][C::grad_var(c)];
          }
        }
      }
      if (!fin || PDE::kHasNcp) {
        __syncthreads();
        // (2) one task per (cell, slice, direction, line): differentiate in place
        const int ntask = CPB * cnt * DIM * F;
        for (int task = tid; task < ntask; task += BLOCK) {
          const int l = task % F;
          const int rest = task / F;
          const int d = rest % DIM;
          const int rest2 = rest / DIM;
          const int jj = rest2 % cnt;
          const int c2 = rest2 / cnt;
          int base, stride;
          line_geom<DIM>(d, l, n, base, stride);
          R* row = lds + c2 * (TC * NCH * SP) + (jj * NCH + d * NCHD) * SP;
          const R s = inv_h[d];
#pragma unroll
          for (int c = 0; c < NCHD; ++c) {
            R x[n];
#pragma unroll
            for (int m = 0; m < n; ++m) x[m] = row[c * SP + G::pidx(base + m * stride)];
#pragma unroll
            for (int i = 0; i < n; ++i) {
              R y = R(0);
#pragma unroll
              for (int m = 0; m < n; ++m) y += T.D[i][m] * x[m];
              row[c * SP + G::pidx(base + i * stride)] = y * s;
            }
          }
        }
        __syncthreads();
      }
      // (3) right-hand side of every slice at this node
#pragma unroll
      for (int jj = 0; jj < TC; ++jj) {
        if (c0 + jj >= n) break;
        const int j = c0 + jj;
        const R* slot = mine + jj * NCH * SP;
        R divF[NV], g[DIM][NV], B[NV], Sv[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          divF[v] = R(0);
#pragma unroll
          for (int d = 0; d < DIM; ++d) g[d][v] = R(0);
        }
        if (!fin || PDE::kHasNcp) {
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
            if (!fin) {
#pragma unroll
              for (int c = 0; c < NFL; ++c)
                divF[C::flux_var(d, c)] += slot[(d * NCHD + c) * SP + G::pidx(k)];
            }
#pragma unroll
            for (int c = 0; c < NGR; ++c)
              g[d][C::grad_var(c)] = slot[(d * NCHD + NFL + c) * SP + G::pidx(k)];
          }
        }
        if (PDE::kHasNcp) {
          PDE::ncp(q[j], P, a.pde, g, B);
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) B[v] = R(0);
        }
        PDE::source(q[j], P, a.pde, Sv);
        if (a.nsrc > 0) {
          const double tj = t_n + (double)a.t64.xi[j] * dt64;
          for (int s = 0; s < a.nsrc; ++s) {
            if (a.src[s].cell != cell) continue;
            const R amp = R(ricker(a.src[s].f0, a.src[s].t0, a.src[s].amp, tj));
            const double* wsk = a.src_w + ((long long)s * S + k) * NV;
#pragma unroll
            for (int v = 0; v < NV; ++v) Sv[v] += amp * R(wsk[v]);
          }
        }
        if (!fin) {
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const R Rv = Sv[v] - divF[v] - B[v];
#pragma unroll
            for (int i = 0; i < n; ++i) acc[i][v] += T.KW[i][j] * Rv;
          }
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            Nbar[v] += T.w[j] * B[v];
            Sbar[v] += T.w[j] * Sv[v];
          }
        }
      }
      if (!fin || PDE::kHasNcp) __syncthreads();
    }
    if (!fin) {
#pragma unroll
      for (int i = 0; i < n; ++i)
#pragma unroll
        for (int v = 0; v < NV; ++v) q[i][v] = u[v] + dt * acc[i][v];
    }
  }

  // time average of the final iterate
  R qbar[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    R s = R(0);
#pragma unroll
    for (int j = 0; j < n; ++j) s += T.w[j] * q[j][v];
    qbar[v] = s;
  }

  // Volume term and face projection, one direction at a time.  Region A of
  // the cell's LDS holds qbar (NV rows), region B the nonzero components of
  // Fbar_d (NFL rows).
  R divF[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) divF[v] = R(0);
  R* const fin_mine = lds + lc * ((NV + NFL) * SP);
#pragma unroll
  for (int v = 0; v < NV; ++v) fin_mine[v * SP + G::pidx(k)] = qbar[v];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
#pragma unroll
    for (int c = 0; c < NFL; ++c) fin_mine[(NV + c) * SP + G::pidx(k)] = Fbar[d][C::flux_var(d, c)];
    __syncthreads();
    for (int task = tid; task < CPB * F; task += BLOCK) {
      const int l = task % F, c2 = task / F;
      const long long tcell = cell0 + c2;
      int base, stride;
      line_geom<DIM>(d, l, n, base, stride);
      R* rows = lds + c2 * ((NV + NFL) * SP);
      double* tr = traces + ((tcell * (2 * DIM) + 2 * d) * 2) * (long long)NV * F;
      const bool tact = tcell < a.ncells;
      // qbar traces at both ends
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        R e0 = R(0), e1 = R(0);
#pragma unroll
        for (int m = 0; m < n; ++m) {
          const R x = rows[v * SP + G::pidx(base + m * stride)];
          e0 += T.l0[m] * x;
          e1 += T.l1[m] * x;
        }
        if (tact) {
          tr[(0 * NV + v) * F + l] = double(e0);          // face 2d,   state
          tr[(2 * NV + v) * F + l] = double(e1);          // face 2d+1, state
        }
      }
      // normal-flux traces; derivative of Fbar_d in place
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (!PDE::flux_nonzero(d, v) && tact) {
          tr[(1 * NV + v) * F + l] = 0.0;
          tr[(3 * NV + v) * F + l] = 0.0;
        }
      }
#pragma unroll
      for (int c = 0; c < NFL; ++c) {
        const int v = C::flux_var(d, c);
        R x[n];
#pragma unroll
        for (int m = 0; m < n; ++m) x[m] = rows[(NV + c) * SP + G::pidx(base + m * stride)];
        R e0 = R(0), e1 = R(0);
#pragma unroll
        for (int m = 0; m < n; ++m) {
          e0 += T.l0[m] * x[m];
          e1 += T.l1[m] * x[m];
        }
        if (tact) {
          tr[(1 * NV + v) * F + l] = double(e0);
          tr[(3 * NV + v) * F + l] = double(e1);
        }
        const R s = inv_h[d];
#pragma unroll
        for (int i = 0; i < n; ++i) {
          R y = R(0);
#pragma unroll
          for (int m = 0; m < n; ++m) y += T.D[i][m] * x[m];
          rows[(NV + c) * SP + G::pidx(base + i * stride)] = y * s;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NFL; ++c) divF[C::flux_var(d, c)] += fin_mine[(NV + c) * SP + G::pidx(k)];
    __syncthreads();
  }

  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const R vol = dt * (Sbar[v] - divF[v] - Nbar[v]);
      Qout[(cell * NV + v) * S + k] = u64[v] + double(vol);
    }
  }
}

// ---------------------------------------------------------------------------
// Kernel B: Rusanov flux on every face of the cell, surface integral and
// update; optionally the Eq. (7) maximum of the new state for the next step.
// ---------------------------------------------------------------------------
template <class PDE, int N>
__global__ void __launch_bounds__((Geo<PDE, N>::BLOCK))
correct_kernel(const KArgs a, double* __restrict__ Q, const double* __restrict__ params,
               double* __restrict__ clock, const double* __restrict__ traces, int next_dt) {
  using G = Geo<PDE, N>;
  constexpr int n = G::n, S = G::S, F = G::F, NV = G::NV, NP = G::NP, DIM = G::DIM;
  constexpr int CPB = G::CPB, BLOCK = G::BLOCK;
  __shared__ double fl[CPB * 2 * DIM * NV * F];
  __shared__ double red[BLOCK];
  __shared__ bool last;

  const Tables<double>& T = a.t64;
  const int tid = threadIdx.x;
  const long long cell0 = (long long)xcd_block(blockIdx.x, a.nblocks) * CPB;
  const double dt = clock[1];

  // fluctuations, one task per (cell, face, face node)
  for (int task = tid; task < CPB * 2 * DIM * F; task += BLOCK) {
    const int f = task % F;
    const int face = (task / F) % (2 * DIM);
    const int c2 = task / (F * 2 * DIM);
    const long long c = cell0 + c2;
    if (c >= a.ncells) continue;
    const int d = face >> 1, side = face & 1;
    // periodic neighbour across this face
    long long cc[3];
    cc[0] = c % a.cells[0];
    cc[1] = (c / a.cells[0]) % a.cells[1];
    cc[2] = DIM == 3 ? c / ((long long)a.cells[0] * a.cells[1]) : 0;
    cc[d] += side ? 1 : -1;
    if (cc[d] < 0) cc[d] += a.cells[d];
    if (cc[d] >= a.cells[d]) cc[d] -= a.cells[d];
    const long long nb = cc[0] + (long long)a.cells[0] * (cc[1] + (long long)a.cells[1] * cc[2]);
    const long long cL = side ? c : nb, cR = side ? nb : c;
    const double* tL = traces + ((cL * (2 * DIM) + 2 * d + 1) * 2) * (long long)NV * F;
    const double* tR = traces + ((cR * (2 * DIM) + 2 * d + 0) * 2) * (long long)NV * F;
    double qL[NV], qR[NV], FL[NV], FR[NV], pL[NP > 0 ? NP : 1], pR[NP > 0 ? NP : 1], pm[NP > 0 ? NP : 1];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      qL[v] = tL[v * F + f];
      FL[v] = tL[(NV + v) * F + f];
      qR[v] = tR[v * F + f];
      FR[v] = tR[(NV + v) * F + f];
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      pL[p] = params[cL * NP + p];
      pR[p] = params[cR * NP + p];
      pm[p] = 0.5 * (pL[p] + pR[p]);
    }
    const double s = fmax(PDE::max_eigen(qL, pL, a.pde, d), PDE::max_eigen(qR, pR, a.pde, d));
    double B[NV];
    if (PDE::kHasNcp) {
      double qm[NV], g[DIM][NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        qm[v] = 0.5 * (qL[v] + qR[v]);
#pragma unroll
        for (int e = 0; e < DIM; ++e) g[e][v] = e == d ? qR[v] - qL[v] : 0.0;
      }
      PDE::ncp(qm, pm, a.pde, g, B);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) B[v] = 0.0;
    }
    const double scale = dt * a.inv_h[d];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double G = 0.5 * (FL[v] + FR[v]) - 0.5 * s * (qR[v] - qL[v]);
      const double Bm = 0.5 * B[v];
      const double flv = side ? (G - FL[v] + Bm) : (FR[v] - G + Bm);
      fl[((c2 * 2 * DIM + face) * NV + v) * F + f] = flv * scale;
    }
  }
  __syncthreads();

  const int lc = tid / S, k = tid - lc * S;
  const long long cell = cell0 + lc;
  double lam = 0.0;
  if (cell < a.ncells) {
    int kk[3] = {0, 0, 0};
    node_coords<DIM>(k, n, kk);
    int fidx[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      // face-node index of node k on the faces normal to d
      if (DIM == 2) fidx[d] = kk[1 - d];
      else fidx[d] = d == 0 ? kk[1] + n * kk[2] : (d == 1 ? kk[0] + n * kk[2] : kk[0] + n * kk[1]);
    }
    double qn[NV], P[NP > 0 ? NP : 1];
#pragma unroll
    for (int p = 0; p < NP; ++p) P[p] = params[cell * NP + p];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double surf = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const double hi = fl[((lc * 2 * DIM + 2 * d + 1) * NV + v) * F + fidx[d]];
        const double lo = fl[((lc * 2 * DIM + 2 * d) * NV + v) * F + fidx[d]];
        surf += (T.l1[kk[d]] * hi + T.l0[kk[d]] * lo) * T.invw[kk[d]];
      }
      const long long idx = (cell * NV + v) * S + k;
      qn[v] = Q[idx] - surf;
      Q[idx] = qn[v];
    }
    if (next_dt) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) lam = fmax(lam, PDE::max_eigen(qn, P, a.pde, d));
    }
  }
  if (next_dt) {
    const double m = block_max<BLOCK>(lam, red);
    if (tid == 0) atomicMax(a.red_max, (unsigned long long)__double_as_longlong(m));
  }
  if (last_block(a.red_count, &last)) {
    __threadfence();
    if (next_dt) {
      const double lmax = __longlong_as_double((long long)atomicAdd(a.red_max, 0ull));
      clock[1] = a.dt_factor / lmax;
      atomicExch(a.red_max, 0ull);
    }
    clock[0] = clock[0] + dt;
    atomicExch(a.red_count, 0u);
  }
}

// ---------------------------------------------------------------------------
// Eq. (7) on a given state.
// ---------------------------------------------------------------------------
template <class PDE, int N>
__global__ void __launch_bounds__((Geo<PDE, N>::BLOCK))
stable_dt_kernel(const KArgs a, const double* __restrict__ Q, const double* __restrict__ params,
                 double* __restrict__ clock) {
  using G = Geo<PDE, N>;
  constexpr int S = G::S, NV = G::NV, NP = G::NP, DIM = G::DIM, CPB = G::CPB;
  __shared__ double red[G::BLOCK];
  __shared__ bool last;
  const int tid = threadIdx.x;
  const int lc = tid / S, k = tid - lc * S;
  const long long cell = (long long)xcd_block(blockIdx.x, a.nblocks) * CPB + lc;
  double lam = 0.0;
  if (cell < a.ncells) {
    double q[NV], P[NP > 0 ? NP : 1];
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = Q[(cell * NV + v) * S + k];
#pragma unroll
    for (int p = 0; p < NP; ++p) P[p] = params[cell * NP + p];
#pragma unroll
    for (int d = 0; d < DIM; ++d) lam = fmax(lam, PDE::max_eigen(q, P, a.pde, d));
  }
  const double m = block_max<G::BLOCK>(lam, red);
  if (tid == 0) atomicMax(a.red_max, (unsigned long long)__double_as_longlong(m));
  if (last_block(a.red_count, &last)) {
    __threadfence();
    const double lmax = __longlong_as_double((long long)atomicAdd(a.red_max, 0ull));
    clock[1] = a.dt_factor / lmax;
    atomicExch(a.red_max, 0ull);
    atomicExch(a.red_count, 0u);
  }
}

// ---------------------------------------------------------------------------
// Physical admissibility per cell (Sec. 3.5).
// ---------------------------------------------------------------------------
template <class PDE, int N>
__global__ void __launch_bounds__((Geo<PDE, N>::BLOCK))
admissible_kernel(const KArgs a, const double* __restrict__ Q, const double* __restrict__ params,
                  uint8_t* __restrict__ troubled, int32_t* __restrict__ count) {
  using G = Geo<PDE, N>;
  constexpr int S = G::S, NV = G::NV, NP = G::NP, CPB = G::CPB;
  __shared__ int bad[CPB];
  __shared__ bool last;
  const int tid = threadIdx.x;
  const int lc = tid / S, k = tid - lc * S;
  const long long cell = (long long)xcd_block(blockIdx.x, a.nblocks) * CPB + lc;
  if (tid < CPB) bad[tid] = 0;
  __syncthreads();
  if (cell < a.ncells) {
    double q[NV], P[NP > 0 ? NP : 1];
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = Q[(cell * NV + v) * S + k];
#pragma unroll
    for (int p = 0; p < NP; ++p) P[p] = params[cell * NP + p];
    if (!PDE::admissible(q, P, a.pde)) bad[lc] = 1;
  }
  __syncthreads();
  if (k == 0 && cell < a.ncells) {
    troubled[cell] = (uint8_t)bad[lc];
    if (bad[lc]) atomicAdd(a.red_sum, 1);
  }
  if (last_block(a.red_count, &last)) {
    __threadfence();
    *count = atomicAdd(a.red_sum, 0);
    atomicExch(a.red_sum, 0);
    atomicExch(a.red_count, 0u);
  }
}

// ---------------------------------------------------------------------------
// Launchers and the per-(PDE, N) kernel set.
// ---------------------------------------------------------------------------
template <class PDE, int N>
struct Launch {
  using G = Geo<PDE, N>;
  static int blocks(const KArgs& a) { return (int)((a.ncells + G::CPB - 1) / G::CPB); }

  static hipError_t predict(const KArgs& a0, int precision, const double* Q, const double* params,
                            const double* clock, double* Qout, double* traces, hipStream_t st) {
    KArgs a = a0;
    a.nblocks = blocks(a);
    if (precision == ADG_MIXED_FP32)
      hipLaunchKernelGGL((predict_kernel<PDE, N, float>), dim3(a.nblocks), dim3(G::BLOCK), 0, st, a,
                         Q, params, clock, Qout, traces);
    else
      hipLaunchKernelGGL((predict_kernel<PDE, N, double>), dim3(a.nblocks), dim3(G::BLOCK), 0, st,
                         a, Q, params, clock, Qout, traces);
    return hipGetLastError();
  }
  static hipError_t correct(const KArgs& a0, double* Q, const double* params, double* clock,
                            const double* traces, int next_dt, hipStream_t st) {
    KArgs a = a0;
    a.nblocks = blocks(a);
    hipLaunchKernelGGL((correct_kernel<PDE, N>), dim3(a.nblocks), dim3(G::BLOCK), 0, st, a, Q, params,
                       clock, traces, next_dt);
    return hipGetLastError();
  }
  static hipError_t stable_dt(const KArgs& a0, const double* Q, const double* params, double* clock,
                              hipStream_t st) {
    KArgs a = a0;
    a.nblocks = blocks(a);
    hipLaunchKernelGGL((stable_dt_kernel<PDE, N>), dim3(a.nblocks), dim3(G::BLOCK), 0, st, a, Q, params,
                       clock);
    return hipGetLastError();
  }
  static hipError_t admissible(const KArgs& a0, const double* Q, const double* params,
                               uint8_t* troubled, int32_t* count, hipStream_t st) {
    KArgs a = a0;
    a.nblocks = blocks(a);
    hipLaunchKernelGGL((admissible_kernel<PDE, N>), dim3(a.nblocks), dim3(G::BLOCK), 0, st, a, Q,
                       params, troubled, count);
    return hipGetLastError();
  }
  static const KernelSet* set() {
    static const KernelSet ks = {G::BLOCK, G::CPB, &predict, &correct, &stable_dt, &admissible};
    return &ks;
  }
};

}  // namespace adg

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

#if !defined(__HIPCC_RTC__)
#include <hip/hip_runtime.h>
#endif

#include <type_traits>

#include "adg_internal.hpp"
#include "pde.hpp"
#include "tables_gen.hpp"

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
  // LDS rows are stored line-major per direction: node k of a row for
  // direction d sits at line_d(k) * LS + k_d, with the line stride LS odd so
  // that 16 consecutive lanes touching consecutive lines, or consecutive
  // nodes of a line, fall into distinct banks.
  static constexpr int LS = (n % 2 == 0) ? n + 1 : n + 2;
  static constexpr int SP = F * LS;        // LDS row length (elements)
  static_assert(BLOCK >= 64 && BLOCK <= 1024, "block must hold one full wave");
  // line index of node (kx, ky, kz) for direction d: the other axes, lower first
  __host__ __device__ static constexpr int line_of(int d, int kx, int ky, int kz) {
    return DIM == 2 ? (d == 0 ? ky : kx)
                    : (d == 0 ? ky + n * kz : (d == 1 ? kx + n * kz : kx + n * ky));
  }
};

// a * b + c with one rounding, in the precision of the operands
__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }

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
  // the first direction whose flux has a nonzero component v (-1: none)
  static constexpr int first_flux_dir(int v) {
    for (int d = 0; d < PDE::DIM; ++d)
      if (PDE::flux_nonzero(d, v)) return d;
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

// Layout of the FP32 predictor (one thread per node).  Time slices are processed in pairs; the two slices of
// a pair share one 16-byte LDS element per (channel, node), so every LDS
// access of the iteration is 128-bit wide.  Cells per block: ~256 lanes,
// limited so the block's LDS stays within 64 KiB.
template <class R>
struct alignas(2 * sizeof(R)) Pair {
  R x, y;
};

template <class PDE, int N, class R, bool MF = false>
struct GeoA1 {
  using G = Geo<PDE, N>;
  using C = Chan<PDE>;
  static constexpr int ITER_ELEMS = C::NCH * G::SP * 2;          // per cell, in R
  static constexpr int FIN_ELEMS = (G::NV + C::NFLUX) * G::SP;   // per cell, in R
  static constexpr int CELL_ELEMS = cmax(ITER_ELEMS, FIN_ELEMS);
  static constexpr int by_threads = G::S >= 256 ? 1 : 256 / G::S;
  static constexpr int by_lds = cmax(1, (64 * 1024) / (CELL_ELEMS * (int)sizeof(R)));
  static constexpr int CPB = cmin(by_threads, by_lds);
  // MF (split-BF16 MFMA line derivatives): matrix instructions read every
  // lane of a wave, so the block is padded to whole waves
  static constexpr int BLOCK = MF ? (CPB * G::S + 63) / 64 * 64 : CPB * G::S;
  static constexpr int ELEMS = CPB * CELL_ELEMS;
  static_assert(BLOCK >= 64 && BLOCK <= 1024, "block must hold one full wave");
  // Occupancy target (waves per SIMD) handed to the register allocator:
  // three 4-wave blocks per CU at FP32.
  static constexpr int MIN_WAVES = 3;
  static_assert(ELEMS * (int)sizeof(R) <= 64 * 1024, "predictor LDS exceeds 64 KiB");
};

// Layout of the FP64 predictor (two threads per node).  A lane pair shares each spatial node; the
// even lane owns time slices 0..H-1 and the odd lane slices H..n-1
// (H = ceil(n/2)).  A chunk step handles one slice per lane, i.e. the slice
// pair (c, H+c) of every node, and the two slices share one 16-byte LDS
// element per (channel, node), so the line tasks use 128-bit LDS accesses.
// Cells per block: up to 512 lanes, limited so the block's LDS stays within
// 64 KiB.
template <class PDE, int N, class R>
struct GeoA2 {
  using G = Geo<PDE, N>;
  using C = Chan<PDE>;
  static constexpr int H = (G::n + 1) / 2;                       // slices per lane
  static constexpr int TPC = 2 * G::S;                           // threads per cell
  // LDS row layout of direction d: position x of line L (both in 0..n-1 and
  // 0..F-1) sits at A_d L + L / P_d + B_d x.  In 3-D, for n = 4, 5, 6 the
  // coefficients come from a search over this family that minimises the
  // bank collisions of the node lanes' 8-byte writes and read-backs (a wave
  // holds 32 consecutive nodes) while the line tasks' 16-byte reads (one
  // line per lane, consecutive lines) stay collision-free; otherwise the odd
  // line stride LS with contiguous lines.
  static constexpr bool kTuned = G::DIM == 3 && G::n >= 4 && G::n <= 6;
  static constexpr int lay_A(int d) {
    return !kTuned ? G::LS : (G::n == 6 ? (d == 0 ? 6 : 1) : (G::n == 5 ? (d == 0 ? 5 : 1) : 1));
  }
  static constexpr int lay_B(int d) {
    return !kTuned ? 1
                   : (G::n == 6 ? (d == 0 ? 1 : (d == 1 ? 38 : 36))
                                : (G::n == 5 ? (d == 0 ? 1 : (d == 1 ? 27 : 25)) : (d == 2 ? 16 : 20)));
  }
  static constexpr int lay_P(int d) { return (kTuned && G::n == 6 && d == 0) ? 8 : 0; }
  __host__ __device__ static constexpr int addr(int d, int L, int x) {
    return lay_A(d) * L + (lay_P(d) ? L / lay_P(d) : 0) + lay_B(d) * x;
  }
  static constexpr int row_len(int d) { return addr(d, G::F - 1, G::n - 1) + 1; }
  static constexpr int SP = cmax(row_len(0), cmax(row_len(1), row_len(G::DIM - 1)));  // elements per row
  static constexpr int ITER_ELEMS = C::NCH * SP * 2;             // per cell, in R
  static constexpr int FIN_ELEMS = (G::NV + C::NFLUX) * SP;      // per cell, in R
  static constexpr int CELL_ELEMS = cmax(ITER_ELEMS, FIN_ELEMS);
  // Blocks of about 512 threads; cells of at most 128 threads (N <= 3 in
  // 3-D) go two to a block of 256, so that three blocks, not one, fill a CU
  // at this kernel's register count and their barriers overlap.
  static constexpr int by_threads = TPC >= 512 ? 1 : (TPC <= 128 ? 256 : 512) / TPC;
  static constexpr int by_lds = cmax(1, (64 * 1024) / (CELL_ELEMS * (int)sizeof(R)));
  static constexpr int CPB = cmin(by_threads, by_lds);
  static constexpr int BLOCK = CPB * TPC;
  static constexpr int ELEMS = CPB * CELL_ELEMS;
  static_assert(BLOCK >= 64 && BLOCK <= 1024, "block must hold one full wave");
  static_assert(ELEMS * (int)sizeof(R) <= 64 * 1024, "predictor LDS exceeds 64 KiB");
  // A one-cell block of seven or more waves runs one block per CU at the register
  // counts of this kernel (at most 3 waves/SIMD), so they can afford a
  // second LDS buffer (gfx950: 160 KiB per CU): chunk steps alternate
  // buffers, and the barrier between one chunk's read-back and the next
  // chunk's writes goes away.
  static constexpr int NBUF = (CPB == 1 && BLOCK > 384 && 2 * ELEMS * (int)sizeof(R) <= 156 * 1024) ? 2 : 1;
  // Occupancy target (waves per SIMD) handed to the register allocator: half
  // the time history per lane keeps the FP64 kernel within 256 registers at
  // two waves per SIMD without spilling (one thread per node needs ~320).
  static constexpr int MIN_WAVES = 2;
};

// Exchange a value with the other lane of the pair (lanes 2k and 2k+1).
__device__ __forceinline__ double pair_swap(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0xB1, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float pair_swap(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, false));
}

// Compile-time one-dimensional tables of order n in precision R (generated at
// build time from the same host construction as adg_basis_tables); every use
// sits in a fully unrolled loop, so the constants fold into the instructions.
template <class R, int n>
struct CT {
  using B = BasisConst<n>;
  __device__ static constexpr R D(int i, int m) { return R(B::D[i][m]); }
  __device__ static constexpr R KW(int i, int j) { return R(B::KW[i][j]); }
  __device__ static constexpr R w(int j) { return R(B::w[j]); }
  __device__ static constexpr R l0(int j) { return R(B::l0[j]); }
  __device__ static constexpr R l1(int j) { return R(B::l1[j]); }
  // weights b_s(tau_j) of the third-order continuous extension of the
  // classical four-stage Runge-Kutta method at time node j
  __device__ static constexpr R cerk_b(int s, int j) {
    const double x = B::xi[j];
    return R(s == 0 ? x - 1.5 * x * x + (2.0 / 3.0) * x * x * x
                    : (s == 3 ? -0.5 * x * x + (2.0 / 3.0) * x * x * x : x * x - (2.0 / 3.0) * x * x * x));
  }
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

// Maximum of two signal speeds (non-negative doubles) for Eq. (7) that keeps
// a NaN: a NaN operand gives the positive quiet NaN, whose bit pattern ranks
// above +inf in the ordered-bits atomic max of the reduction slots, so one
// NaN speed anywhere makes the step size NaN (fmax would drop it).
__device__ __forceinline__ double lam_max(double a, double b) {
  const double m = fmax(a, b);
  return (a != a || b != b) ? __longlong_as_double(0x7ff8000000000000LL) : m;
}

// Block-level maximum of signal speeds (lam_max); returns the block maximum
// in thread 0.  Every thread stores its value in LDS; the first wave (always
// complete: BLOCK >= 64) folds the block and reduces across its lanes, so no
// shuffle ever reads a lane that does not exist in a partial last wave.
template <int BLOCK>
__device__ __forceinline__ double block_max(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  double m = 0.0;
  if (threadIdx.x < 64) {
    for (int i = threadIdx.x; i < BLOCK; i += 64) m = lam_max(m, red[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = lam_max(m, __shfl_xor(m, off, 64));
  }
  return m;
}

// Reductions over blocks go through kSlots slots kSlotStride words apart
// (one 64-byte line each): block b folds its maximum into slot b % kSlots
// with an atomic max on the bit pattern (ordered like the value for
// non-negative doubles), so contention per address stays low.
__device__ __forceinline__ void slot_max(unsigned long long* slots, int b, double m) {
  atomicMax(slots + (b % kSlots) * kSlotStride, (unsigned long long)__double_as_longlong(m));
}

// true if local cell c of block b exists (ragged last block)
__device__ __forceinline__ bool cell0_valid(const KArgs& a, int b, int cpb, int c) {
  return (long long)xcd_block(b, a.nblocks) * cpb + c < a.ncells;
}

__device__ __forceinline__ double ricker(double f0, double t0, double amp, double t) {
  const double pi = 3.14159265358979323846;
  double x = pi * f0 * (t - t0);
  x = x * x;
  return amp * (1.0 - 2.0 * x) * exp(-x);
}

// ---------------------------------------------------------------------------
// Split-BF16 line derivatives on the matrix cores (ADG_MIXED_BF16X3).
//
// A float is the exact sum of three BF16 terms h + m + l (8 significant bits
// each).  The product of D and x keeps the six partial products whose size
// is at least 2^-16 of the whole, hh, hm, mh, hl, mm, lh (the three dropped
// ones are below 2^-24), each a BF16 x BF16 product accumulated in FP32 by
// v_mfma_f32_16x16x32_bf16: rows i = output node (n of 16 used), columns =
// 16 (line, slice) pairs, K = (partial product, input node), one product per
// 8-entry group of K, so two instructions cover the six.
// ---------------------------------------------------------------------------
typedef __bf16 adg_bf16x8 __attribute__((ext_vector_type(8)));
typedef float adg_f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split_bf16x3(float x, __bf16& h, __bf16& m, __bf16& l) {
  h = static_cast<__bf16>(x);
  const float r1 = x - static_cast<float>(h);  // exact
  m = static_cast<__bf16>(r1);
  l = static_cast<__bf16>(r1 - static_cast<float>(m));  // exact: at most 8 bits left
}

// part of the matrix (A) and of the data (B) in partial product p = 0..5
__device__ __forceinline__ constexpr int bf_apart(int p) { return p == 2 || p == 4 ? 1 : (p == 5 ? 2 : 0); }
__device__ __forceinline__ constexpr int bf_bpart(int p) { return p == 1 || p == 4 ? 1 : (p == 3 ? 2 : 0); }

// The A operands of the two instructions for this lane: D's split parts,
// row i = lane % 16, K group g = lane / 16 holds partial product 4 s + g.
template <int n>
__device__ __forceinline__ void bf16x3_matrix(adg_bf16x8 (&A)[2]) {
  const int lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
#pragma unroll
  for (int st = 0; st < 2; ++st) {
    const int p = 4 * st + g;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      __bf16 part[3] = {static_cast<__bf16>(0.0f), static_cast<__bf16>(0.0f), static_cast<__bf16>(0.0f)};
      if (p < 6 && i < n && m < n) split_bf16x3(float(BasisConst<n>::D[i][m]), part[0], part[1], part[2]);
      A[st][m] = p < 6 ? part[bf_apart(p < 6 ? p : 0)] : static_cast<__bf16>(0.0f);
    }
  }
}

// Differentiate, in place, NLINES lines of n two-slice elements: line t of
// the list starts at row_of(t) (a Pair<float> pointer, stride 1 along the
// line) and is scaled by scale_of(t).  Every wave of the block takes tiles of
// 16 (line, slice) columns in turn; all 64 lanes of a wave execute the
// matrix instructions.
template <int n, class RowOf, class ScaleOf>
__device__ __forceinline__ void bf16x3_line_derivs(int NLINES, RowOf row_of, ScaleOf scale_of, int nwaves,
                                                   const adg_bf16x8 (&A)[2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, g = lane >> 4;
  const int ntiles = (2 * NLINES + 15) / 16;
  for (int tile = wave; tile < ntiles; tile += nwaves) {
    const int c = tile * 16 + col;  // (line, slice) column, slice fastest
    const int t = c >> 1, sl = c & 1;
    const bool valid = t < NLINES;
    float* xp = valid ? reinterpret_cast<float*>(row_of(t)) + sl : nullptr;
    float x[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) x[m] = (valid && m < n) ? xp[2 * m] : 0.0f;
    __bf16 xs[3][8];
#pragma unroll
    for (int m = 0; m < 8; ++m) split_bf16x3(x[m], xs[0][m], xs[1][m], xs[2][m]);
    adg_f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      const int p = 4 * st + g;
      const int bp = bf_bpart(p < 6 ? p : 0);
      adg_bf16x8 B;
#pragma unroll
      for (int m = 0; m < 8; ++m)
        B[m] = p < 6 ? (bp == 0 ? xs[0][m] : (bp == 1 ? xs[1][m] : xs[2][m])) : static_cast<__bf16>(0.0f);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[st], B, acc, 0, 0, 0);
    }
    // lane (g, col) holds output nodes i = 4 g + r of column col
    if (valid) {
      const float s = scale_of(t);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * g + r;
        if (i < n) xp[2 * i] = acc[r] * s;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Kernel A, one thread per node (used for the FP32 predictor).
// ---------------------------------------------------------------------------
template <class PDE, int N, class R, bool MF = false>
__global__ void __launch_bounds__((GeoA1<PDE, N, R, MF>::BLOCK), (GeoA1<PDE, N, R, MF>::MIN_WAVES))
predict_kernel_node(const KArgs a, const double* Q, const double* __restrict__ params,
               const double* __restrict__ clock, double* Qout, double* __restrict__ traces) {
  // MF: the derivative contractions of the Picard passes in split BF16 on
  // the matrix cores (ADG_MIXED_BF16X3), everything else as in FP32.
  // Q and Qout may be the same array (in-place step): each element is read
  // once at the start and written once at the end by the same thread.
  using G = Geo<PDE, N>;
  using C = Chan<PDE>;
  using GA = GeoA1<PDE, N, R, MF>;
  using T = CT<R, G::n>;
  using P2 = Pair<R>;
  constexpr int n = G::n, S = G::S, F = G::F, NV = G::NV, NP = G::NP, DIM = G::DIM;
  constexpr int CPB = GA::CPB, BLOCK = GA::BLOCK, SP = G::SP;
  constexpr int NCH = C::NCH, NCHD = C::NCHD, NFL = C::NFLUX, NGR = C::ngrad();
  static_assert(C::uniform(), "flux sparsity must be the same in every direction");
  __shared__ P2 lds2[GA::ELEMS / 2];
  R* const lds = reinterpret_cast<R*>(lds2);

  const int tid = threadIdx.x;
  // lanes past the block's nodes (a block padded to whole waves) only take
  // part in the line derivatives
  const bool node = !MF || tid < CPB * S;
  const int lc = node ? tid / S : 0, k = node ? tid - lc * S : 0;
  int pk[DIM];  // this node's slot in the LDS rows of each direction
  {
    const int kx = k % n, ky = (k / n) % n, kz = DIM == 3 ? k / (n * n) : 0;
    const int kd[3] = {kx, ky, kz};
#pragma unroll
    for (int d = 0; d < DIM; ++d) pk[d] = G::line_of(d, kx, ky, kz) * G::LS + kd[d];
  }
  const long long cell0 = (long long)xcd_block(blockIdx.x, a.nblocks) * CPB;
  const long long cell = cell0 + lc;
  const bool active = node && cell < a.ncells;
  const long long cl = active ? cell : a.ncells - 1;  // clamp loads of the ragged tail

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

  // Point sources: the Ricker amplitude at the n time nodes of this step is
  // evaluated once per block; only blocks holding a source cell use them.
  __shared__ double src_amp[kMaxSources * n];
  bool src_here = false;
  for (int s = 0; s < a.nsrc; ++s)
    src_here = src_here || (a.src[s].cell >= cell0 && a.src[s].cell < cell0 + CPB);
  if (src_here && tid < a.nsrc * n) {
    const int s = tid / n, j = tid - s * n;
    src_amp[tid] = ricker(a.src[s].f0, a.src[s].t0, a.src[s].amp, t_n + a.t64.xi[j] * dt64);
  }
  // (made visible by the first barrier below)

  P2* const mine = lds2 + lc * (GA::CELL_ELEMS / 2);  // this cell's pairs [NCH][SP]
  adg_bf16x8 Amf[2];  // MF: this lane's split-BF16 operands of D
  if constexpr (MF) bf16x3_matrix<n>(Amf);
  R q[n][NV];     // current iterate at the n time nodes of node k
  R Fbar[DIM][NV], Nbar[NV], Sbar[NV];  // final pass: time averages

  // point-source term of slice j at this node, added to Sv
  auto add_point_sources = [&](int j, R* Sv) {
    if (!src_here) return;
    for (int s = 0; s < a.nsrc; ++s) {
      if (a.src[s].cell != cell) continue;
      const R amp = R(src_amp[s * n + j]);
      const double* wsk = a.src_w + ((long long)s * S + k) * NV;
#pragma unroll
      for (int v = 0; v < NV; ++v) Sv[v] += amp * R(wsk[v]);
    }
  };

  // One pass over the time slices of the current iterate, two at a time.
  //  KIND 0: first Picard step.  q^0 = u^n at every time node, so every slice
  //          has the same right-hand side apart from point sources: one
  //          slice is evaluated and copied to all n.
  //  KIND 1: Picard step.
  //  Both leave R_j in q[j]; the caller then forms sum_j KW_ij R_j.
  //  KIND 2: final pass at the last iterate: time averages of F, B grad q
  //          and S (READING: the averaged terms use the final iterate).
  auto pass = [&](auto kind_tag) {
    constexpr int KIND = decltype(kind_tag)::value;
    constexpr bool FIN = KIND == 2;
    constexpr bool USE_LDS = !FIN || PDE::kHasNcp;
    constexpr int NSL = KIND == 0 ? 1 : n;  // slices evaluated
#pragma unroll
    for (int c0 = 0; c0 < NSL; c0 += 2) {
      const bool two = c0 + 1 < NSL;  // compile-time after unrolling
      const int j0 = c0, j1 = two ? c0 + 1 : c0;
      // (1) fluxes and gradient inputs of slices j0, j1 -> LDS pairs
      R Fa[DIM][NV], Fb[DIM][NV];
      PDE::fluxes(q[j0], P, a.pde, Fa);
      if (two) PDE::fluxes(q[j1], P, a.pde, Fb);
      if constexpr (FIN) {
#pragma unroll
        for (int d = 0; d < DIM; ++d)
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            Fbar[d][v] += T::w(j0) * Fa[d][v];
            if (two) Fbar[d][v] += T::w(j1) * Fb[d][v];
          }
      }
      if constexpr (USE_LDS) {
        if (node) {
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
            if constexpr (!FIN) {
#pragma unroll
              for (int c = 0; c < NFL; ++c) {
                const int v = C::flux_var(d, c);
                mine[(d * NCHD + c) * SP + pk[d]] = P2{Fa[d][v], two ? Fb[d][v] : R(0)};
              }
            }
#pragma unroll
            for (int c = 0; c < NGR; ++c) {
              const int v = C::grad_var(c);
              mine[(d * NCHD + NFL + c) * SP + pk[d]] = P2{q[j0][v], two ? q[j1][v] : R(0)};
            }
          }
        }
        __syncthreads();
        // (2) line tasks (cell, direction, channel half, line): differentiate
        //     both slices of every channel in place
        constexpr int CH0 = FIN ? NFL : 0;  // the final pass only needs gradients
        constexpr int CHM = (CH0 + NCHD + 1) / 2;
        if constexpr (MF) {
          constexpr int NCT = NCHD - CH0;
          bf16x3_line_derivs<n>(
              CPB * DIM * NCT * F,
              [&](int t) {
                const int l = t % F, ch = CH0 + (t / F) % NCT, d = (t / (F * NCT)) % DIM, c2 = t / (F * NCT * DIM);
                return lds2 + c2 * (GA::CELL_ELEMS / 2) + (d * NCHD + ch) * SP + l * G::LS;
              },
              [&](int) { return 1.0f; }, BLOCK / 64, Amf);
        } else
        for (int task = tid; task < CPB * DIM * 2 * F; task += BLOCK) {
          const int l = task % F;
          const int hf = (task / F) & 1;
          const int d = (task / (2 * F)) % DIM;
          const int c2 = task / (2 * F * DIM);
          P2* row = lds2 + c2 * (GA::CELL_ELEMS / 2) + d * NCHD * SP + l * G::LS;
          const int cb = hf ? CHM : CH0, ce = hf ? NCHD : CHM;
          for (int c = cb; c < ce; ++c) {
            P2 x[n];
#pragma unroll
            for (int m = 0; m < n; ++m) x[m] = row[c * SP + m];
#pragma unroll
            for (int i = 0; i < n; ++i) {
              R y0 = R(0), y1 = R(0);
#pragma unroll
              for (int m = 0; m < n; ++m) {
                y0 += T::D(i, m) * x[m].x;
                y1 += T::D(i, m) * x[m].y;
              }
              row[c * SP + i] = P2{y0, y1};
            }
          }
        }
        __syncthreads();
      }
      // (3) right-hand sides of slices j0, j1 at this node; the line tasks
      // leave the 1/h of each direction to this read-back, whose sums start
      // from the first direction's values
      R divA[NV], divB[NV], gA[DIM][NV], gB[DIM][NV];
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int d = 0; d < DIM; ++d) gA[d][v] = gB[d][v] = R(0);
      if constexpr (USE_LDS) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const R ih = inv_h[d];
#pragma unroll
          for (int c = 0; c < NFL; ++c) {
            if constexpr (FIN) break;
            const int v = C::flux_var(d, c);
            const P2 t = mine[(d * NCHD + c) * SP + pk[d]];
            divA[v] = C::first_flux_dir(v) == d ? t.x * ih : fma_r(t.x, ih, divA[v]);
            divB[v] = C::first_flux_dir(v) == d ? t.y * ih : fma_r(t.y, ih, divB[v]);
          }
#pragma unroll
          for (int c = 0; c < NGR; ++c) {
            const P2 t = mine[(d * NCHD + NFL + c) * SP + pk[d]];
            gA[d][C::grad_var(c)] = t.x * ih;
            gB[d][C::grad_var(c)] = t.y * ih;
          }
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v)
        if (!USE_LDS || FIN || C::first_flux_dir(v) < 0) divA[v] = divB[v] = R(0);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h == 1 && !two) break;
        const int j = h ? j1 : j0;
        R B[NV], Sv[NV];
        if constexpr (PDE::kHasNcp) {
          PDE::ncp(q[j], P, a.pde, h ? gB : gA, B);
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) B[v] = R(0);
        }
        PDE::source(q[j], P, a.pde, Sv);
        if constexpr (KIND == 0) {
          // identical slices: R_j = R (plus the point sources of slice j)
          R Rv[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) Rv[v] = Sv[v] - divA[v] - B[v];
#pragma unroll
          for (int jj = 0; jj < n; ++jj) {
            R Sp[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) Sp[v] = R(0);
            add_point_sources(jj, Sp);
#pragma unroll
            for (int v = 0; v < NV; ++v) q[jj][v] = Rv[v] + Sp[v];
          }
        } else if constexpr (KIND == 1 && !PDE::kHasNcp && !PDE::kHasSource) {
          // R_j = -div F (+ the point sources, added to R_j itself) in the
          // place of q_j, which is no longer needed
#pragma unroll
          for (int v = 0; v < NV; ++v) q[j][v] = -(h ? divB[v] : divA[v]);
          add_point_sources(j, q[j]);
        } else {
          add_point_sources(j, Sv);
          if constexpr (KIND == 1) {
            // q_j is no longer needed once R_j is known: keep R_j in its place
#pragma unroll
            for (int v = 0; v < NV; ++v) q[j][v] = Sv[v] - (h ? divB[v] : divA[v]) - B[v];
          } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              Nbar[v] += T::w(j) * B[v];
              Sbar[v] += T::w(j) * Sv[v];
            }
          }
        }
      }
      // no barrier after the read-backs: a node thread reads back and next
      // writes only its own slots (the final phase starts with a barrier)
    }
  };

  const int I = a.picard_iters;
#pragma unroll
  for (int j = 0; j < n; ++j)
#pragma unroll
    for (int v = 0; v < NV; ++v) q[j][v] = u[v];
  for (int r = 0; r < I; ++r) {
    if (r == 0)
      pass(std::integral_constant<int, 0>{});
    else
      pass(std::integral_constant<int, 1>{});
    // q holds R_j at every time node: q^{r+1}_i = u + dt sum_j KW_ij R_j
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      R t[n];
#pragma unroll
      for (int i = 0; i < n; ++i) {
        R s = R(0);
#pragma unroll
        for (int j = 0; j < n; ++j) s += T::KW(i, j) * q[j][v];
        t[i] = s;
      }
#pragma unroll
      for (int i = 0; i < n; ++i) q[i][v] = u[v] + dt * t[i];
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    Nbar[v] = Sbar[v] = R(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) Fbar[d][v] = R(0);
  }
  pass(std::integral_constant<int, 2>{});

  // time average of the final iterate
  R qbar[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    R s = R(0);
#pragma unroll
    for (int j = 0; j < n; ++j) s += T::w(j) * q[j][v];
    qbar[v] = s;
  }

  // Volume term and face projection, all directions at once: direction d's
  // region of the cell's LDS holds qbar (NV rows) and the nonzero components
  // of Fbar_d (NFL rows) in d's line-major layout.
  constexpr int FIN_D = (NV + NFL) * SP;
  static_assert(DIM * FIN_D <= GA::CELL_ELEMS, "final-phase rows exceed the cell's LDS");
  R divF[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) divF[v] = R(0);
  R* const fin_mine = lds + lc * GA::CELL_ELEMS;
  __syncthreads();  // every read-back of the passes is done
  if (node) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
#pragma unroll
      for (int v = 0; v < NV; ++v) fin_mine[d * FIN_D + v * SP + pk[d]] = qbar[v];
#pragma unroll
      for (int c = 0; c < NFL; ++c)
        fin_mine[d * FIN_D + (NV + c) * SP + pk[d]] = Fbar[d][C::flux_var(d, c)];
    }
  }
  __syncthreads();
  // one task per (cell, direction, quantity v, line l), runtime indices, one
  // code path: traces of qbar_v and Fbar_{d,v}, derivative of Fbar_{d,v}
  for (int task = tid; task < CPB * DIM * NV * F; task += BLOCK) {
    const int l = task % F;
    const int v = (task / F) % NV;
    const int d = (task / (F * NV)) % DIM;
    const int c2 = task / (F * NV * DIM);
    const long long tcell = cell0 + c2;
    const bool tact = tcell < a.ncells;
    R* rows = lds + c2 * GA::CELL_ELEMS + d * FIN_D + l * G::LS;
    double* tr = traces + ((tcell * (2 * DIM) + 2 * d) * 2) * (long long)NV * F + v * F + l;
    R e0 = R(0), e1 = R(0);
#pragma unroll
    for (int m = 0; m < n; ++m) {
      const R x = rows[v * SP + m];
      e0 += T::l0(m) * x;
      e1 += T::l1(m) * x;
    }
    int cc = -1;  // the flux row of v in d's layout (-1: F_d has no component v)
#pragma unroll
    for (int dd = 0; dd < DIM; ++dd)
#pragma unroll
      for (int c = 0; c < NFL; ++c)
        if (dd == d && C::flux_var(dd, c) == v) cc = c;
    R f0 = R(0), f1 = R(0);
    if (cc >= 0) {
      R x[n];
#pragma unroll
      for (int m = 0; m < n; ++m) x[m] = rows[(NV + cc) * SP + m];
#pragma unroll
      for (int m = 0; m < n; ++m) {
        f0 += T::l0(m) * x[m];
        f1 += T::l1(m) * x[m];
      }
      R s = inv_h[0];  // 1/h of direction d (a select chain: inv_h stays in registers)
#pragma unroll
      for (int dd = 1; dd < DIM; ++dd)
        if (d == dd) s = inv_h[dd];
#pragma unroll
      for (int i = 0; i < n; ++i) {
        R y = R(0);
#pragma unroll
        for (int m = 0; m < n; ++m) y += T::D(i, m) * x[m];
        rows[(NV + cc) * SP + i] = y * s;
      }
    }
    if (tact) {
      tr[0 * NV * F] = double(e0);  // face 2d,   state
      tr[1 * NV * F] = double(f0);  // face 2d,   normal flux
      tr[2 * NV * F] = double(e1);  // face 2d+1, state
      tr[3 * NV * F] = double(f1);  // face 2d+1, normal flux
    }
  }
  __syncthreads();
#pragma unroll
  for (int d = 0; d < DIM; ++d)
#pragma unroll
    for (int c = 0; c < NFL; ++c) divF[C::flux_var(d, c)] += fin_mine[d * FIN_D + (NV + c) * SP + pk[d]];

  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const R vol = dt * (Sbar[v] - divF[v] - Nbar[v]);
      Qout[(cell * NV + v) * S + k] = u64[v] + double(vol);
    }
  }
}

// y = s D x along one line of n nodes.  D is centro-antisymmetric on the
// symmetric GL nodes (D[n-1-i][n-1-m] = -D[i][m]): with sums and
// differences of mirrored inputs, rows i and n-1-i share half the products
// and half the constants.
template <class R, int n>
__device__ __forceinline__ void line_deriv(const R (&x)[n], R (&y)[n], R s) {
  using T = CT<R, n>;
  constexpr int HF = n / 2;
  R sm[HF > 0 ? HF : 1], dm[HF > 0 ? HF : 1];
#pragma unroll
  for (int m = 0; m < HF; ++m) {
    sm[m] = x[m] + x[n - 1 - m];
    dm[m] = x[m] - x[n - 1 - m];
  }
#pragma unroll
  for (int i = 0; i < HF; ++i) {
    R p = R(0), q = R(0);
#pragma unroll
    for (int m = 0; m < HF; ++m) {
      p += R(0.5 * (BasisConst<n>::D[i][m] + BasisConst<n>::D[i][n - 1 - m])) * sm[m];
      q += R(0.5 * (BasisConst<n>::D[i][m] - BasisConst<n>::D[i][n - 1 - m])) * dm[m];
    }
    if constexpr (n % 2 == 1) p += T::D(i, HF) * x[HF];
    y[i] = (q + p) * s;
    y[n - 1 - i] = (q - p) * s;
  }
  if constexpr (n % 2 == 1) {
    R c = R(0);
#pragma unroll
    for (int m = 0; m < HF; ++m) c += T::D(HF, m) * dm[m];
    y[HF] = c * s;
  }
}

// ---------------------------------------------------------------------------
// Kernel A, a lane pair per node (used for the FP64 predictor).
// ---------------------------------------------------------------------------
template <class PDE, int N, class R>
__global__ void __launch_bounds__((GeoA2<PDE, N, R>::BLOCK), (GeoA2<PDE, N, R>::MIN_WAVES))
predict_kernel_pair(const KArgs a, const double* Q, const double* __restrict__ params,
               const double* __restrict__ clock, double* Qout, double* __restrict__ traces) {
  // Q and Qout may be the same array (in-place step): each element is read
  // at the start and written at the end by the even lane of its node.
  using G = Geo<PDE, N>;
  using C = Chan<PDE>;
  using GA = GeoA2<PDE, N, R>;
  using T = CT<R, G::n>;
  using P2 = Pair<R>;
  constexpr int n = G::n, S = G::S, F = G::F, NV = G::NV, NP = G::NP, DIM = G::DIM;
  constexpr int CPB = GA::CPB, BLOCK = GA::BLOCK, SP = GA::SP, H = GA::H, TPC = GA::TPC;
  constexpr int NCHD = C::NCHD, NFL = C::NFLUX, NGR = C::ngrad();
  static_assert(C::uniform(), "flux sparsity must be the same in every direction");
  __shared__ P2 lds_all[GA::NBUF * GA::ELEMS / 2];
  P2* lds2 = lds_all;  // the buffer of the current chunk step
  R* const lds = reinterpret_cast<R*>(lds_all);

  const int tid = threadIdx.x;
  const int lc = tid / TPC;
  const int rr = tid - lc * TPC;
  const int k = rr >> 1;   // spatial node
  const int h = rr & 1;    // time half owned by this lane
  const long long cell0 = (long long)xcd_block(blockIdx.x, a.nblocks) * CPB;
  const long long cell = cell0 + lc;
  const bool active = cell < a.ncells;
  const long long cl = active ? cell : a.ncells - 1;  // clamp loads of the ragged tail

  int pk[DIM];  // this node's slot in the LDS rows of each direction
  {
    const int kx = k % n, ky = (k / n) % n, kz = DIM == 3 ? k / (n * n) : 0;
    const int kd[3] = {kx, ky, kz};
#pragma unroll
    for (int d = 0; d < DIM; ++d) pk[d] = GA::addr(d, G::line_of(d, kx, ky, kz), kd[d]);
  }

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

  // Per-lane coefficients of the time operator for the output slices this
  // lane owns (i = h H + il): Kown over its own slices, Kpar over the
  // partner's, zero where a slice index reaches n (odd n).
  // Per-lane coefficients of the time operator for the output slices this
  // lane owns (i = h H + il): Kown over its own slices, Kpar over the
  // partner's, zero where a slice index reaches n (odd n).  One LDS table per
  // half, read by broadcast.
  auto kw = [](int i, int j) { return (i < n && j < n) ? T::KW(i, j) : R(0); };
  __shared__ R ktab[2][2 * H * H + H];
  if (tid < 2) {
    const int hh = tid;
#pragma unroll
    for (int il = 0; il < H; ++il)
#pragma unroll
      for (int c = 0; c < H; ++c) {
        ktab[hh][il * H + c] = hh ? kw(H + il, H + c) : kw(il, c);
        ktab[hh][H * H + il * H + c] = hh ? kw(H + il, c) : kw(il, H + c);
      }
#pragma unroll
    for (int c = 0; c < H; ++c) ktab[hh][2 * H * H + c] = hh ? (H + c < n ? T::w(H + c) : R(0)) : T::w(c);
  }
  const R* const kt = ktab[h];
  auto Kown = [&](int il, int c) { return kt[il * H + c]; };
  auto Kpar = [&](int il, int c) { return kt[H * H + il * H + c]; };
  auto wown = [&](int c) { return kt[2 * H * H + c]; };

  // Point sources: the Ricker amplitude at the n time nodes of this step is
  // evaluated once per block; only blocks holding a source cell use them.
  __shared__ double src_amp[kMaxSources * n];
  bool src_here = false;
  for (int s = 0; s < a.nsrc; ++s)
    src_here = src_here || (a.src[s].cell >= cell0 && a.src[s].cell < cell0 + CPB);
  if (src_here && tid < a.nsrc * n) {
    const int s = tid / n, j = tid - s * n;
    src_amp[tid] = ricker(a.src[s].f0, a.src[s].t0, a.src[s].amp, t_n + a.t64.xi[j] * dt64);
  }
  // (made visible by the first barrier below)

  // point-source term of slice j at this node, added to Sv
  auto add_point_sources = [&](int j, R* Sv) {
    if (!src_here) return;
    for (int s = 0; s < a.nsrc; ++s) {
      if (a.src[s].cell != cell) continue;
      const R amp = R(src_amp[s * n + j]);
      const double* wsk = a.src_w + ((long long)s * S + k) * NV;
#pragma unroll
      for (int v = 0; v < NV; ++v) Sv[v] += amp * R(wsk[v]);
    }
  };

  R q[H][NV];     // current iterate at the slices this lane owns
  R Fbar[DIM][NV], Nbar[NV], Sbar[NV];  // final pass: time averages (own slices)

  // One pass over the time slices of the current iterate; chunk step c
  // handles slice hH + c on this lane.
  //  KIND 0: first Picard step.  q^0 = u^n at every time node, so every slice
  //          has the same right-hand side apart from point sources; one
  //          chunk step suffices.
  //  KIND 1: Picard step; R_j replaces q_j, which is no longer needed.
  //  KIND 2: final pass at the last iterate: time averages of F, B grad q
  //          and S over the lane's slices (READING: the averaged terms use the
  //          final iterate).
  R R0[NV];  // KIND 0 right-hand side
  auto pass = [&](auto kind_tag) {
    constexpr int KIND = decltype(kind_tag)::value;
    constexpr bool FIN = KIND == 2;
    constexpr bool USE_LDS = !FIN || PDE::kHasNcp;
    constexpr int STEPS = KIND == 0 ? 1 : H;
#pragma unroll
    for (int c = 0; c < STEPS; ++c) {
      const int j = h * H + c;
      const bool valid = j < n;
      if constexpr (GA::NBUF == 2 && USE_LDS) lds2 = (lds2 == lds_all) ? lds_all + GA::ELEMS / 2 : lds_all;
      P2* const mine = lds2 + lc * (GA::CELL_ELEMS / 2);  // this cell's pairs [NCH][SP]
      R* const mine_h = reinterpret_cast<R*>(mine) + h;   // this lane's half of each pair
      // (1) flux and gradient inputs of slice j -> this lane's half of the pairs
      R Fl[DIM][NV];
      PDE::fluxes(q[c], P, a.pde, Fl);
      if constexpr (FIN) {
#pragma unroll
        for (int d = 0; d < DIM; ++d)
#pragma unroll
          for (int v = 0; v < NV; ++v) Fbar[d][v] += wown(c) * Fl[d][v];
      }
      if constexpr (USE_LDS) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          if constexpr (!FIN) {
#pragma unroll
            for (int cc = 0; cc < NFL; ++cc)
              mine_h[2 * ((d * NCHD + cc) * SP + pk[d])] = Fl[d][C::flux_var(d, cc)];
          }
#pragma unroll
          for (int cc = 0; cc < NGR; ++cc)
            mine_h[2 * ((d * NCHD + NFL + cc) * SP + pk[d])] = q[c][C::grad_var(cc)];
        }
        __syncthreads();
        // (2) line tasks (cell, direction, channel, line): differentiate both
        //     slices of the pair in place
        constexpr int CH0 = FIN ? NFL : 0;  // the final pass only needs gradients
        constexpr int NCT = NCHD - CH0;
        // Tasks that fill whole rounds of the block differentiate both slices
        // of the pair; if the remaining tasks fit half a round, they are split
        // by slice, so the last round costs half a task instead of a whole one.
        constexpr int NT = CPB * DIM * NCT * F;
        constexpr int REM = NT % BLOCK;
        constexpr bool SPLIT = REM > 0 && 2 * REM <= BLOCK;
        constexpr int NWHOLE = SPLIT ? NT - REM : NT;
          auto task_row = [&](int task) {
          const int l = task % F;
          const int ch = CH0 + (task / F) % NCT;
          const int d = (task / (F * NCT)) % DIM;
          const int c2 = task / (F * NCT * DIM);
          return lds2 + c2 * (GA::CELL_ELEMS / 2) + (d * NCHD + ch) * SP + GA::addr(d, l, 0);
        };
        // element stride along a line of the task's direction
        auto task_stride = [&](int task) { return GA::lay_B((task / (F * NCT)) % DIM); };
        for (int task = tid; task < NWHOLE; task += BLOCK) {
          P2* row = task_row(task);
          const int st = task_stride(task);
          const R s = inv_h[(task / (F * NCT)) % DIM];
          R x0[n], x1[n], y0[n], y1[n];
#pragma unroll
          for (int m = 0; m < n; ++m) {
            const P2 t = row[m * st];
            x0[m] = t.x;
            x1[m] = t.y;
          }
          line_deriv<R, n>(x0, y0, s);
          line_deriv<R, n>(x1, y1, s);
#pragma unroll
          for (int i = 0; i < n; ++i) row[i * st] = P2{y0[i], y1[i]};
        }
        if constexpr (SPLIT) {
          if (tid < 2 * REM) {
            const int task = NWHOLE + (tid >> 1);
            R* row = reinterpret_cast<R*>(task_row(task)) + (tid & 1);  // one half of each pair
            const int st = 2 * task_stride(task);
            const R s = inv_h[(task / (F * NCT)) % DIM];
            R x[n], y[n];
#pragma unroll
            for (int m = 0; m < n; ++m) x[m] = row[m * st];
            line_deriv<R, n>(x, y, s);
#pragma unroll
            for (int i = 0; i < n; ++i) row[i * st] = y[i];
          }
        }
        __syncthreads();
      }
      // (3) right-hand side of slice j at this node
      R divF[NV], g[DIM][NV], B[NV], Sv[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        divF[v] = R(0);
#pragma unroll
        for (int d = 0; d < DIM; ++d) g[d][v] = R(0);
      }
      if constexpr (USE_LDS) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          if constexpr (!FIN) {
#pragma unroll
            for (int cc = 0; cc < NFL; ++cc)
              divF[C::flux_var(d, cc)] += mine_h[2 * ((d * NCHD + cc) * SP + pk[d])];
          }
#pragma unroll
          for (int cc = 0; cc < NGR; ++cc)
            g[d][C::grad_var(cc)] = mine_h[2 * ((d * NCHD + NFL + cc) * SP + pk[d])];
        }
      }
      if constexpr (PDE::kHasNcp) {
        PDE::ncp(q[c], P, a.pde, g, B);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) B[v] = R(0);
      }
      PDE::source(q[c], P, a.pde, Sv);
      if constexpr (KIND == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) R0[v] = Sv[v] - divF[v] - B[v];
      } else {
        if (valid) add_point_sources(j, Sv);
        if constexpr (KIND == 1) {
#pragma unroll
          for (int v = 0; v < NV; ++v) q[c][v] = valid ? Sv[v] - divF[v] - B[v] : R(0);
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            Nbar[v] += wown(c) * B[v];
            Sbar[v] += wown(c) * Sv[v];
          }
        }
      }
      if constexpr (USE_LDS && GA::NBUF == 1) __syncthreads();
    }
  };

  // q^{r+1}_i = u + dt sum_j KW_ij R_j for the lane's own i, with R_j of the
  // own slices in q and those of the partner exchanged across the pair.
  auto update = [&]() {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      R Rp[H], t[H];
#pragma unroll
      for (int c = 0; c < H; ++c) Rp[c] = pair_swap(q[c][v]);
#pragma unroll
      for (int il = 0; il < H; ++il) {
        R s = R(0);
#pragma unroll
        for (int c = 0; c < H; ++c) s += Kown(il, c) * q[c][v] + Kpar(il, c) * Rp[c];
        t[il] = s;
      }
#pragma unroll
      for (int il = 0; il < H; ++il) q[il][v] = u[v] + dt * t[il];
    }
  };

  const int I = a.picard_iters;
#pragma unroll
  for (int c = 0; c < H; ++c)
#pragma unroll
    for (int v = 0; v < NV; ++v) q[c][v] = u[v];
  for (int r = 0; r < I; ++r) {
    if (r == 0) {
      pass(std::integral_constant<int, 0>{});
      // every slice has R0 (+ its point sources)
#pragma unroll
      for (int c = 0; c < H; ++c) {
        const int j = h * H + c;
        R Sp[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) Sp[v] = R(0);
        if (j < n) add_point_sources(j, Sp);
#pragma unroll
        for (int v = 0; v < NV; ++v) q[c][v] = j < n ? R0[v] + Sp[v] : R(0);
      }
    } else {
      pass(std::integral_constant<int, 1>{});
    }
    update();
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    Nbar[v] = Sbar[v] = R(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) Fbar[d][v] = R(0);
  }
  pass(std::integral_constant<int, 2>{});

  // time averages: own half plus the partner's half
  R qbar[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    R s = R(0);
#pragma unroll
    for (int c = 0; c < H; ++c) s += wown(c) * q[c][v];
    qbar[v] = s + pair_swap(s);
    Nbar[v] += pair_swap(Nbar[v]);
    Sbar[v] += pair_swap(Sbar[v]);
#pragma unroll
    for (int d = 0; d < DIM; ++d) Fbar[d][v] += pair_swap(Fbar[d][v]);
  }

  // Volume term and face projection, all directions at once: direction d's
  // region of the cell's LDS holds qbar (NV rows) and the nonzero components
  // of Fbar_d (NFL rows) in d's line-major layout; the even lane of each node
  // writes them.
  constexpr int FIN_D = (NV + NFL) * SP;
  static_assert(DIM * FIN_D <= GA::CELL_ELEMS, "final-phase rows exceed the cell's LDS");
  R divF[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) divF[v] = R(0);
  R* const fin_mine = lds + lc * GA::CELL_ELEMS;
  if constexpr (GA::NBUF == 2) __syncthreads();  // last read-backs done
  if (h == 0) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
#pragma unroll
      for (int v = 0; v < NV; ++v) fin_mine[d * FIN_D + v * SP + pk[d]] = qbar[v];
#pragma unroll
      for (int cc = 0; cc < NFL; ++cc)
        fin_mine[d * FIN_D + (NV + cc) * SP + pk[d]] = Fbar[d][C::flux_var(d, cc)];
    }
  }
  __syncthreads();
  for (int task = tid; task < CPB * DIM * F * (NFL + 1); task += BLOCK) {
    // task kind 0: qbar traces of line l; kind 1 + cc: flux channel cc
    const int l = task % F;
    const int kind = (task / F) % (NFL + 1);
    const int dt_ = (task / (F * (NFL + 1))) % DIM;
    const int c2 = task / (F * (NFL + 1) * DIM);
    const long long tcell = cell0 + c2;
    const bool tact = tcell < a.ncells;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      if (d != dt_) continue;
      R* rows = lds + c2 * GA::CELL_ELEMS + d * FIN_D + GA::addr(d, l, 0);
      const int st = GA::lay_B(d);
      double* tr = traces + ((tcell * (2 * DIM) + 2 * d) * 2) * (long long)NV * F;
      if (kind == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          R e0 = R(0), e1 = R(0);
#pragma unroll
          for (int m = 0; m < n; ++m) {
            const R x = rows[v * SP + m * st];
            e0 += T::l0(m) * x;
            e1 += T::l1(m) * x;
          }
          if (tact) {
            tr[(0 * NV + v) * F + l] = double(e0);  // face 2d,   state
            tr[(2 * NV + v) * F + l] = double(e1);  // face 2d+1, state
          }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          if (!PDE::flux_nonzero(d, v) && tact) {
            tr[(1 * NV + v) * F + l] = 0.0;
            tr[(3 * NV + v) * F + l] = 0.0;
          }
        }
      } else {
        // normal-flux traces; derivative of Fbar_d in place
#pragma unroll
        for (int cc = 0; cc < NFL; ++cc) {
          if (cc != kind - 1) continue;
          const int v = C::flux_var(d, cc);
          R x[n], y[n];
#pragma unroll
          for (int m = 0; m < n; ++m) x[m] = rows[(NV + cc) * SP + m * st];
          R e0 = R(0), e1 = R(0);
#pragma unroll
          for (int m = 0; m < n; ++m) {
            e0 += T::l0(m) * x[m];
            e1 += T::l1(m) * x[m];
          }
          if (tact) {
            tr[(1 * NV + v) * F + l] = double(e0);
            tr[(3 * NV + v) * F + l] = double(e1);
          }
          line_deriv<R, n>(x, y, inv_h[d]);
#pragma unroll
          for (int i = 0; i < n; ++i) rows[(NV + cc) * SP + i * st] = y[i];
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int d = 0; d < DIM; ++d)
#pragma unroll
    for (int cc = 0; cc < NFL; ++cc)
      divF[C::flux_var(d, cc)] += fin_mine[d * FIN_D + (NV + cc) * SP + pk[d]];

  if (active && h == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const R vol = dt * (Sbar[v] - divF[v] - Nbar[v]);
      Qout[(cell * NV + v) * S + k] = u64[v] + double(vol);
    }
  }
}

// ---------------------------------------------------------------------------
// Kernel A for PDEs linear in Q (flux, non-conservative product and source
// linear and homogeneous in Q, with per-cell coefficients), one thread per
// node.  With R(q) = L q + s(t) and the element operator L acting on space
// only, the Picard update q^{r+1} = 1 u + dt (KW amp) w + dt (KW (x) L) q^r
// (Sec. 3.3, Eq. 5; amp = point-source amplitudes at the time nodes, w =
// their nodal weights) unrolls exactly, and the time average of the I-th
// iterate is
//   qbar = sum_{k=0..I} c_k (dt L)^k u + sum_{k=0..I-1} dt e_{k+1} (dt L)^k w,
//   c_k = w_t^T KW^k 1,  e_k = w_t^T KW^k amp.
// Horner's scheme evaluates it with I applications of L:
//   t_I = c_I u;  t_k = c_k u + dt e_{k+1} w + dt L t_{k+1};  qbar = t_0.
// The averaged terms of the volume term and of the traces are those of
// qbar by linearity: vol = dt (L qbar + e_0 w), traces qhat = trace of qbar
// and Fhat_d = F_d(qhat) (the flux traces only where KArgs::flux_traces asks
// for them).  The result equals the Picard form up to the
// order of rounding, at I + 1 applications of L instead of about n I.
// ---------------------------------------------------------------------------
// LDS row layout of the linear-PDE kernels: position x of line L of
// direction d at A_d L + B_d x.  In 3-D at n = 5 the lines are contiguous
// (A = n): 32 consecutive node lanes then write and read back 32 distinct
// bank pairs for x-lines, and consecutive lines keep an odd stride for the
// line tasks (a bank model of one L application: ~35 % fewer conflict
// cycles than the odd stride n + 2; the C3 predictor 1.39 -> 1.24 ms).
// Otherwise the odd line stride LS.  (A layout searched the same way for
// n = 4 measured 9 % slower and is not used.)
template <class G>
struct LinLayout {
  static constexpr int n = G::n;
  static constexpr bool k5 = G::DIM == 3 && n == 5;
  __host__ __device__ static constexpr int lay_A(int) { return k5 ? n : G::LS; }
  __host__ __device__ static constexpr int lay_B(int) { return 1; }
  __host__ __device__ static constexpr int addr(int d, int L, int x) { return lay_A(d) * L + lay_B(d) * x; }
  static constexpr int SP = G::F * lay_A(0);  // elements per row (every line, A_d the same)
};

template <class PDE, int N, class R>
struct GeoL {
  using G = Geo<PDE, N>;
  using C = Chan<PDE>;
  static constexpr int ROW_ELEMS = C::NCH * LinLayout<G>::SP;  // every derivative channel of one field
  static constexpr int AVG_ELEMS = G::NV * G::S;    // the time average in node order
  static constexpr int CELL_ELEMS = cmax(ROW_ELEMS, AVG_ELEMS);
  static constexpr int by_threads = G::S >= 256 ? 1 : 256 / G::S;
  static constexpr int by_lds = cmax(1, (52 * 1024) / (CELL_ELEMS * (int)sizeof(R)));
  // at least one full wave per block
  static constexpr int CPB = cmax(cmin(by_threads, by_lds), (64 + G::S - 1) / G::S);
  static constexpr int BLOCK = CPB * G::S;
  static constexpr int ELEMS = CPB * CELL_ELEMS;
  static_assert(BLOCK >= 64 && BLOCK <= 1024, "block must hold one full wave");
  static_assert(ELEMS * (int)sizeof(R) <= 150 * 1024, "linear predictor LDS exceeds the CU");
  static constexpr int MIN_WAVES = 3;
};

// node index of position m on line l of direction d
template <class G>
__device__ __forceinline__ int line_node(int d, int l, int m) {
  constexpr int n = G::n;
  if constexpr (G::DIM == 2) return d == 0 ? m + n * l : l + n * m;
  return d == 0 ? m + n * l : (d == 1 ? (l % n) + n * m + n * n * (l / n) : l + n * n * m);
}

// y = s D^T x along one line.  D^T is centro-antisymmetric too
// (D^T[n-1-i][n-1-m] = -D^T[i][m]), so rows i and n-1-i share the products
// of mirrored sums and differences as in line_deriv.
template <class R, int n>
__device__ __forceinline__ void line_deriv_T(const R (&x)[n], R (&y)[n], R s) {
  using B = BasisConst<n>;
  constexpr int HF = n / 2;
  R sm[HF > 0 ? HF : 1], dm[HF > 0 ? HF : 1];
#pragma unroll
  for (int m = 0; m < HF; ++m) {
    sm[m] = x[m] + x[n - 1 - m];
    dm[m] = x[m] - x[n - 1 - m];
  }
#pragma unroll
  for (int i = 0; i < HF; ++i) {
    R p = R(0), q = R(0);
#pragma unroll
    for (int m = 0; m < HF; ++m) {
      p += R(0.5 * (B::D[m][i] + B::D[n - 1 - m][i])) * sm[m];
      q += R(0.5 * (B::D[m][i] - B::D[n - 1 - m][i])) * dm[m];
    }
    if constexpr (n % 2 == 1) p += R(B::D[HF][i]) * x[HF];
    y[i] = (q + p) * s;
    y[n - 1 - i] = (q - p) * s;
  }
  if constexpr (n % 2 == 1) {
    R c = R(0);
#pragma unroll
    for (int m = 0; m < HF; ++m) c += R(B::D[m][HF]) * dm[m];
    y[HF] = c * s;
  }
}

// The element operator L of a PDE linear in Q on the LDS rows of a block of
// CPB cells (CELL_ELEMS elements each, NCH channel rows of SP elements in
// the per-direction line-major layout).  Every thread of the block calls
// these together (they hold three barriers); a thread's own node sits at
// pk[d] in the rows of direction d of its cell's region `mine`.
template <class PDE, int N, class R, int CPB, int BLOCK, int CELL_ELEMS>
struct LinOp {
  using G = Geo<PDE, N>;
  using C = Chan<PDE>;
  using LL = LinLayout<G>;
  static constexpr int n = G::n, F = G::F, NV = G::NV, DIM = G::DIM, SP = LL::SP;
  static constexpr int NCH = C::NCH, NCHD = C::NCHD, NFL = C::NFLUX, NGR = C::ngrad();
  // A cell of 64 nodes is one wave: its rows are written, differentiated and
  // read back by that wave alone, so the line tasks of a cell stay on its
  // wave and a wave-level fence replaces the block barrier (LDS accesses of
  // one wave complete in order).
  static constexpr bool kWave = G::S == 64;

  __device__ static __forceinline__ void sync() {
    if constexpr (kWave) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      __syncthreads();
    }
  }

  // f(cell in block, task in cell) over the NT tasks of every cell of the
  // block: on the cell's own wave (kWave) or spread over the block
  template <int NT, class Fn>
  __device__ static __forceinline__ void cell_tasks(int tid, Fn f) {
    if constexpr (kWave) {
      for (int t = tid & 63; t < NT; t += 64) f(tid >> 6, t);
    } else {
      for (int task = tid; task < CPB * NT; task += BLOCK) f(task / NT, task % NT);
    }
  }

  // out = L t = S(t) - div F(t) - B(t) grad t at this node; g = the gradients
  // the non-conservative product reads (zero elsewhere)
  __device__ static __forceinline__ void apply(const KArgs& a, R* lds, R* mine, const int (&pk)[DIM],
                                               int tid, const R (&t)[NV], const R* P,
                                               const R (&inv_h)[3], R (&out)[NV], R (&g)[DIM][NV]) {
    R Fl[DIM][NV];
    PDE::fluxes(t, P, a.pde, Fl);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
#pragma unroll
      for (int cc = 0; cc < NFL; ++cc) mine[(d * NCHD + cc) * SP + pk[d]] = Fl[d][C::flux_var(d, cc)];
#pragma unroll
      for (int cc = 0; cc < NGR; ++cc) mine[(d * NCHD + NFL + cc) * SP + pk[d]] = t[C::grad_var(cc)];
    }
    sync();
    cell_tasks<NCH * F>(tid, [&](int c2, int t) {
      const int l = t % F, ch = t / F;
      const int d = ch / NCHD, st = LL::lay_B(d);
      R* row = lds + c2 * CELL_ELEMS + ch * SP + LL::addr(d, l, 0);
      R x[n], y[n];
#pragma unroll
      for (int m = 0; m < n; ++m) x[m] = row[m * st];
      line_deriv<R, n>(x, y, R(1));
#pragma unroll
      for (int i = 0; i < n; ++i) row[i * st] = y[i];
    });
    sync();
    // the 1/h of each direction is applied here; the divergence starts at
    // the first direction with a flux in v
    R divF[NV], B[NV], Sv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int d = 0; d < DIM; ++d) g[d][v] = R(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const R ih = inv_h[d];
#pragma unroll
      for (int cc = 0; cc < NFL; ++cc) {
        const int v = C::flux_var(d, cc);
        const R x = mine[(d * NCHD + cc) * SP + pk[d]];
        divF[v] = C::first_flux_dir(v) == d ? x * ih : fma_r(x, ih, divF[v]);
      }
#pragma unroll
      for (int cc = 0; cc < NGR; ++cc) g[d][C::grad_var(cc)] = mine[(d * NCHD + NFL + cc) * SP + pk[d]] * ih;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (C::first_flux_dir(v) < 0) divF[v] = R(0);
    if constexpr (PDE::kHasNcp) {
      PDE::ncp(t, P, a.pde, g, B);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) B[v] = R(0);
    }
    if constexpr (PDE::kHasSource) {
      PDE::source(t, P, a.pde, Sv);
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v] = Sv[v] - divF[v] - B[v];
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v] = -divF[v] - B[v];
    }
    // No barrier here: a thread reads back only its own slots, which only it
    // writes in the next application; a caller that uses the rows otherwise
    // next calls sync() first.
  }

  // mu = L^T nu at this node (FP64; the PDE's transposes): the flux part
  // through D^T of nu's flux components, the non-conservative part through
  // D^T of the gradient adjoints, plus the source's transpose.  With FW, the
  // same round also differentiates the forward values fw (the quantities
  // whose gradient the non-conservative product reads) into gq.  Rows: the
  // NCHD adjoint channels of every direction, then (FW) NGR forward
  // channels of every direction.
  template <bool FW>
  __device__ static __forceinline__ void apply_T(const KArgs& a, double* lds, double* mine,
                                                 const int (&pk)[DIM], int tid, const double (&nu)[NV],
                                                 const double* P, const double (&inv_h)[3],
                                                 double (&mu)[NV], const double* fw,
                                                 double (&gq)[DIM][NV]) {
    constexpr int NF = FW ? NGR : 0;
    double lB[NV], lG[DIM][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      lB[v] = -nu[v];
#pragma unroll
      for (int d = 0; d < DIM; ++d) lG[d][v] = 0.0;
    }
    if constexpr (PDE::kHasNcp) PDE::ncp_T(P, a.pde, lB, lG);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
#pragma unroll
      for (int cc = 0; cc < NFL; ++cc) mine[(d * NCHD + cc) * SP + pk[d]] = nu[C::flux_var(d, cc)];
#pragma unroll
      for (int cc = 0; cc < NGR; ++cc) mine[(d * NCHD + NFL + cc) * SP + pk[d]] = lG[d][C::grad_var(cc)];
#pragma unroll
      for (int cc = 0; cc < NF; ++cc) mine[(NCH + d * NGR + cc) * SP + pk[d]] = fw[cc];
    }
    sync();
    // per cell: adjoint channels (D^T) first, forward channels (D) after
    // them, so that waves mostly take one kind
    constexpr int NTA = NCH * F, NTF = DIM * NF * F;
    auto task = [&](int c2, int t) {
      double x[n], y[n];
      if (t < NTA) {
        const int l = t % F, ch = t / F;
        const int d = ch / NCHD, st = LL::lay_B(d);
        double* row = lds + c2 * CELL_ELEMS + ch * SP + LL::addr(d, l, 0);
#pragma unroll
        for (int m = 0; m < n; ++m) x[m] = row[m * st];
        line_deriv_T<double, n>(x, y, inv_h[d]);
#pragma unroll
        for (int i = 0; i < n; ++i) row[i * st] = y[i];
      } else if constexpr (NF > 0) {
        const int tf = t - NTA;
        const int l = tf % F, ch = tf / F;
        const int d = ch / NF, st = LL::lay_B(d);
        double* row = lds + c2 * CELL_ELEMS + (NCH + ch) * SP + LL::addr(d, l, 0);
#pragma unroll
        for (int m = 0; m < n; ++m) x[m] = row[m * st];
        line_deriv<double, n>(x, y, inv_h[d]);
#pragma unroll
        for (int i = 0; i < n; ++i) row[i * st] = y[i];
      }
    };
    if constexpr (kWave) {
      cell_tasks<NTA + NTF>(tid, task);
    } else {
      // all cells' adjoint tasks, then all cells' forward tasks
      for (int i = tid; i < CPB * (NTA + NTF); i += BLOCK) {
        if (i < CPB * NTA) task(i / NTA, i % NTA);
        else task((i - CPB * NTA) / (NTF > 0 ? NTF : 1), NTA + (i - CPB * NTA) % (NTF > 0 ? NTF : 1));
      }
    }
    sync();
#pragma unroll
    for (int v = 0; v < NV; ++v) mu[v] = 0.0;
    PDE::source_T(a.pde, nu, mu);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      double lF[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        lF[v] = 0.0;
        gq[d][v] = 0.0;
      }
#pragma unroll
      for (int cc = 0; cc < NFL; ++cc) lF[C::flux_var(d, cc)] = -mine[(d * NCHD + cc) * SP + pk[d]];
      PDE::flux_T(d, a.pde, lF, mu);
#pragma unroll
      for (int cc = 0; cc < NGR; ++cc) mu[C::grad_var(cc)] += mine[(d * NCHD + NFL + cc) * SP + pk[d]];
#pragma unroll
      for (int cc = 0; cc < NF; ++cc) gq[d][C::grad_var(cc)] = mine[(NCH + d * NGR + cc) * SP + pk[d]];
    }
    // no barrier here (see apply)
  }
};

// e_k = w_t^T KW^k amp for k = 0..I, amp = the source's Ricker amplitudes
// at the n time nodes of the step (t_n + xi_j dt).
template <int n>
__device__ inline void lin_source_weights(const KArgs& a, int s, double t_n, double dt, int I, double* e) {
  double v[n], t[n];
#pragma unroll
  for (int j = 0; j < n; ++j) v[j] = ricker(a.src[s].f0, a.src[s].t0, a.src[s].amp, t_n + a.t64.xi[j] * dt);
  for (int kk = 0; kk <= I; ++kk) {
    if (kk > 0) {
#pragma unroll
      for (int i = 0; i < n; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < n; ++j) acc += a.t64.KW[i][j] * v[j];
        t[i] = acc;
      }
#pragma unroll
      for (int i = 0; i < n; ++i) v[i] = t[i];
    }
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < n; ++j) acc += a.t64.w[j] * v[j];
    e[kk] = acc;
  }
}

// The values at both ends of a line of n nodes x[m st]: e0 = sum_m l0(m) x,
// e1 = sum_m l1(m) x (the linear predictor's face traces and, in the same
// arithmetic, the adjoint's).
template <class R, int n>
__device__ __forceinline__ void line_ends(const R* __restrict__ x, int st, R& e0, R& e1) {
  using T = CT<R, n>;
  R s0 = R(0), s1 = R(0);
#pragma unroll
  for (int m = 0; m < n; ++m) {
    const R y = x[m * st];
    s0 += T::l0(m) * y;
    s1 += T::l1(m) * y;
  }
  e0 = s0;
  e1 = s1;
}

// Slots per node of KArgs::keep ([C][SLOTS][S] doubles): for k < n (the
// adjoint's most Picard iterations), the channels of Horner's iterate
// t_{k+1} whose gradient the non-conservative product reads; then all of
// t_0 = qbar.  A step's keep buffer continues with its face traces (the
// trace array's layout), which the step's predictor writes there.
template <class PDE, int N>
struct KeepGeo {
  static constexpr int NGR = Chan<PDE>::ngrad(), IMAX = N + 1;
  static constexpr int QBAR = IMAX * NGR;       // first slot of qbar
  static constexpr int SLOTS = QBAR + PDE::NV;
};

// The linear predictor for the CPB cells of a block from cell0 on: this
// thread's node starts from u64 (with its cell's parameters P); the face
// traces go to traces and u + dt vol to Qout (active nodes only).  t_n is
// the start of the step (point sources), dt64 its size.  With a.keep set
// (FP64), the quantities the step's adjoint reads go there too.
template <class PDE, int N, class R>
__device__ __forceinline__ void lin_predict_block(const KArgs& a, R* lds, double (*src_e)[kMaxLin + 1],
                                                  int tid, long long cell0, const double (&u64)[PDE::NV],
                                                  const R* P, const double* __restrict__ params, double t_n,
                                                  double dt64, double* Qout, double* __restrict__ traces) {
  using G = Geo<PDE, N>;
  using GL = GeoL<PDE, N, R>;
  using T = CT<R, G::n>;
  using Op = LinOp<PDE, N, R, GL::CPB, GL::BLOCK, GL::CELL_ELEMS>;
  constexpr int n = G::n, S = G::S, F = G::F, NV = G::NV, NP = G::NP, DIM = G::DIM;
  constexpr int CPB = GL::CPB;
  const int lc = tid / S, k = tid - lc * S;
  const long long cell = cell0 + lc;
  const bool active = cell < a.ncells;
  int pk[DIM];  // this node's slot in the LDS rows of each direction
  {
    const int kx = k % n, ky = (k / n) % n, kz = DIM == 3 ? k / (n * n) : 0;
    const int kd[3] = {kx, ky, kz};
#pragma unroll
    for (int d = 0; d < DIM; ++d) pk[d] = LinLayout<G>::addr(d, G::line_of(d, kx, ky, kz), kd[d]);
  }
  R u[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = R(u64[v]);
  const R dt = R(dt64);
  const int I = a.picard_iters;
  R inv_h[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) inv_h[d] = R(a.inv_h[d]);

  // point sources of this block
  bool src_here = false;
  for (int s = 0; s < a.nsrc; ++s)
    src_here = src_here || (a.src[s].cell >= cell0 && a.src[s].cell < cell0 + CPB);
  if (src_here && tid < a.nsrc) lin_source_weights<n>(a, tid, t_n, dt64, I, src_e[tid]);
  if (src_here) __syncthreads();  // src_e for every wave of the block
  // t[v] += scale * e_kk * w at this node for every source in this cell
  auto add_sources = [&](int kk, R scale, R* t) {
    if (!src_here) return;
    for (int s = 0; s < a.nsrc; ++s) {
      if (a.src[s].cell != cell) continue;
      const R e = scale * R(src_e[s][kk]);
      const double* wsk = a.src_w + ((long long)s * S + k) * NV;
#pragma unroll
      for (int v = 0; v < NV; ++v) t[v] += e * R(wsk[v]);
    }
  };

  R* const mine = lds + lc * GL::CELL_ELEMS;
  // Horner's scheme for the time average of the I-th Picard iterate
  R t[NV];
  {
    const R cI = R(a.lin_c[I]);
#pragma unroll
    for (int v = 0; v < NV; ++v) t[v] = cI * u[v];
  }
  using KG = KeepGeo<PDE, N>;
  constexpr bool KEEP = std::is_same<R, double>::value;
  double* const keep = KEEP && a.keep && active ? a.keep + cell * (long long)(KG::SLOTS * S) + k : nullptr;
  for (int kk = I - 1; kk >= 0; --kk) {
    if (keep && kk < KG::IMAX) {
#pragma unroll
      for (int c = 0; c < KG::NGR; ++c) keep[(kk * KG::NGR + c) * S] = double(t[Chan<PDE>::grad_var(c)]);
    }
    R Lt[NV], g[DIM][NV];
    Op::apply(a, lds, mine, pk, tid, t, P, inv_h, Lt, g);
    const R ck = R(a.lin_c[kk]);
#pragma unroll
    for (int v = 0; v < NV; ++v) t[v] = ck * u[v] + dt * Lt[v];
    add_sources(kk + 1, dt, t);
  }
  if (keep) {
#pragma unroll
    for (int v = 0; v < NV; ++v) keep[(KG::QBAR + v) * S] = double(t[v]);
  }

  // volume term
  R vol[NV];
  {
    R g[DIM][NV];
    Op::apply(a, lds, mine, pk, tid, t, P, inv_h, vol, g);
    add_sources(0, R(1), vol);
  }

  // face traces: qhat = trace of qbar, Fhat_d = F_d(qhat); one task per
  // (cell, direction, line) extrapolates every quantity to both ends
  Op::sync();  // the operator's last read-backs are done
#pragma unroll
  for (int v = 0; v < NV; ++v) mine[v * S + k] = t[v];
  Op::sync();
  // (the direction is a runtime index: every task takes the same code path)
  Op::template cell_tasks<DIM * F>(tid, [&](int c2, int task) {
    const int l = task % F;
    const int d = task / F;
    const long long tcell = cell0 + c2;
    if (tcell >= a.ncells) return;
    const R* rows = lds + c2 * GL::CELL_ELEMS + line_node<G>(d, l, 0);
    const int st = line_node<G>(d, 0, 1) - line_node<G>(d, 0, 0);  // node stride along d
    R e0[NV], e1[NV], Pt[NP > 0 ? NP : 1];
#pragma unroll
    for (int p = 0; p < NP; ++p) Pt[p] = R(params[tcell * NP + p]);
#pragma unroll
    for (int v = 0; v < NV; ++v) line_ends<R, n>(rows + v * S, st, e0[v], e1[v]);
    double* tr = traces + ((tcell * (2 * DIM) + 2 * d) * 2) * (long long)NV * F;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      tr[(0 * NV + v) * F + l] = double(e0[v]);  // face 2d,   state
      tr[(2 * NV + v) * F + l] = double(e1[v]);  // face 2d+1, state
    }
    if (a.flux_traces) {
      // F_d at both faces (all directions' fluxes, d's picked by a select
      // chain so that Fa stays in registers)
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        R Fa[DIM][NV];
        PDE::fluxes(side ? e1 : e0, Pt, a.pde, Fa);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          R fv = Fa[0][v];
#pragma unroll
          for (int dd = 1; dd < DIM; ++dd)
            if (d == dd) fv = Fa[dd][v];
          tr[((side ? 3 : 1) * NV + v) * F + l] = double(fv);
        }
      }
    }
  });

  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Qout[(cell * NV + v) * S + k] = u64[v] + double(dt * vol[v]);
  }
}

template <class PDE, int N, class R>
__global__ void __launch_bounds__((GeoL<PDE, N, R>::BLOCK), (GeoL<PDE, N, R>::MIN_WAVES))
predict_kernel_lin(const KArgs a, const double* Q, const double* __restrict__ params,
                   const double* __restrict__ clock, double* Qout, double* __restrict__ traces) {
  // Q and Qout may be the same array (in-place step): each element is read
  // at the start and written at the end by the thread of its node.
  using G = Geo<PDE, N>;
  using GL = GeoL<PDE, N, R>;
  static_assert(PDE::kLinear, "the linear predictor needs a PDE linear in Q");
  static_assert(Chan<PDE>::uniform(), "flux sparsity must be the same in every direction");
  constexpr int S = G::S, NV = G::NV, NP = G::NP;
  __shared__ R lds[GL::ELEMS];
  __shared__ double src_e[kMaxSources][kMaxLin + 1];

  const int tid = threadIdx.x;
  const int lc = tid / S, k = tid - lc * S;
  const long long cell0 = (long long)xcd_block(blockIdx.x, a.nblocks) * GL::CPB;
  const long long cell = cell0 + lc;
  const long long cl = cell < a.ncells ? cell : a.ncells - 1;  // clamp loads of the ragged tail
  double u64[NV];
  R P[NP > 0 ? NP : 1];
#pragma unroll
  for (int v = 0; v < NV; ++v) u64[v] = Q[(cl * NV + v) * S + k];
#pragma unroll
  for (int p = 0; p < NP; ++p) P[p] = R(params[cl * NP + p]);
  lin_predict_block<PDE, N, R>(a, lds, src_e, tid, cell0, u64, P, params, clock[0], clock[1], Qout, traces);
}

// ---------------------------------------------------------------------------
// Kernel B: Rusanov flux on every face of the cell, surface integral and
// update; optionally the per-block Eq. (7) maximum of the new state (reduced
// over blocks by finalize_kernel, which also advances the clock).
// ---------------------------------------------------------------------------
template <class PDE, int N>
struct GeoB {
  using G = Geo<PDE, N>;
  static constexpr int FL_PER_CELL = 2 * G::DIM * G::NV * G::F;  // doubles
  // cells of 128 nodes or more one per block (C2, N = 5: 2.54 -> 2.44 ms per
  // launch against two per block), smaller ones up to 512 threads (N = 3:
  // 3.01 ms, against 3.07 and 3.16 ms with 128- and 256-thread blocks)
  static constexpr int by_threads = G::S >= 128 ? 1 : 512 / G::S;
  static constexpr int by_lds = cmax(1, (48 * 1024) / (FL_PER_CELL * 8));
  // at least one full wave per block
  static constexpr int CPB = cmax(cmin(by_threads, by_lds), (64 + G::S - 1) / G::S);
  static constexpr int BLOCK = CPB * G::S;
  static_assert(BLOCK >= 64 && BLOCK <= 1024, "block must hold one full wave");
};

// First cell of the corrector's logical block lb (CPB consecutive cells).
// In 3-D meshes whose extents are multiples of 8 the blocks walk bricks of
// 8 x 8 x 8 cells (x fastest inside a brick and from brick to brick), so a
// cell's y and z neighbours are visited within 64 cells of it and the face
// traces it shares with them are still in L2 (in cell order the z
// neighbours are C0 C1 cells apart); otherwise the cells in order.
template <int DIM, int CPB>
__device__ __forceinline__ int corr_cell0(const KArgs& a, int lb) {
  const int first = lb * CPB;
  if constexpr (DIM == 3 && 8 % CPB == 0) {
    const int C0 = a.cells[0], C1 = a.cells[1], C2 = a.cells[2];
    if (((C0 | C1 | C2) & 7) == 0) {
      const int o = first & 511, bi = first >> 9, nbx = C0 >> 3, nby = C1 >> 3;
      const int bx = bi % nbx, by = (bi / nbx) % nby, bz = bi / (nbx * nby);
      return (bx * 8 + (o & 7)) + C0 * ((by * 8 + ((o >> 3) & 7)) + C1 * (bz * 8 + (o >> 6)));
    }
  }
  return first;
}

// PDEs with a boundary_values function for ADG_BC_USER faces (run-time PDEs
// that define one)
template <class... T>
using kern_void_t = void;
template <class P, class = void>
struct HasUserBoundary {
  static constexpr bool value = false;
};
template <class P>
struct HasUserBoundary<P, kern_void_t<decltype(P::kUserBoundary)>> {
  static constexpr bool value = P::kUserBoundary;
};

// Corrector phase 1: the fluctuation of each cell's side at every face node
// of the CPB cells from cell0 on (block-wide tasks, one per (cell, face,
// face node)), scaled by dt / h_d, into fl[CPB][2 dim][NV][F].
template <class PDE, int N, int CPB, int BLOCK>
__device__ __forceinline__ void face_fluctuations(const KArgs& a, const double* __restrict__ params,
                                                  const double* __restrict__ traces, double t, double dt,
                                                  int cell0, int tid, double* fl) {
  using G = Geo<PDE, N>;
  constexpr int F = G::F, NV = G::NV, NP = G::NP, DIM = G::DIM;
  const int C0 = a.cells[0], C1 = a.cells[1];
  const int ncells = (int)a.ncells;
  for (int task = tid; task < CPB * 2 * DIM * F; task += BLOCK) {
    const int f = task % F;
    const int face = (task / F) % (2 * DIM);
    const int c2 = task / (F * 2 * DIM);
    const int c = cell0 + c2;
    if (c >= ncells) continue;
    const int d = face >> 1, side = face & 1;
    const int c_own[3] = {c % C0, (c / C0) % C1, DIM == 3 ? c / (C0 * C1) : 0};
    // neighbour across this face: wrapped around on a periodic axis; on a
    // boundary face of a non-periodic axis the outside state and normal flux
    // come from this cell's own traces (outflow: a copy, wall: the mirror
    // image)
    int cc[3];
    cc[0] = c % C0;
    cc[1] = (c / C0) % C1;
    cc[2] = DIM == 3 ? c / (C0 * C1) : 0;
    cc[d] += side ? 1 : -1;
    const int bc = (cc[d] < 0 || cc[d] >= a.cells[d]) ? a.bc[face] : ADG_BC_PERIODIC;
    if (cc[d] < 0) cc[d] += a.cells[d];
    if (cc[d] >= a.cells[d]) cc[d] -= a.cells[d];
    const int nb = bc == ADG_BC_PERIODIC ? cc[0] + C0 * (cc[1] + C1 * cc[2]) : c;
    const int cL = side ? c : nb, cR = side ? nb : c;
    // the two traces that meet at this face; on a boundary face both are
    // this cell's own trace of the face
    const int fL = bc != ADG_BC_PERIODIC ? face : 2 * d + 1;
    const int fR = bc != ADG_BC_PERIODIC ? face : 2 * d;
    const double* tL = traces + ((long long)(cL * (2 * DIM) + fL) * 2) * NV * F;
    const double* tR = traces + ((long long)(cR * (2 * DIM) + fR) * 2) * NV * F;
    // an inflow face: the outside trace is the prescribed state and its flux
    if (bc == ADG_BC_INFLOW) (side ? tR : tL) = a.bc_trace + face * 2 * NV * F;
    double qL[NV], qR[NV], FL[NV], FR[NV], pL[NP > 0 ? NP : 1], pR[NP > 0 ? NP : 1], pm[NP > 0 ? NP : 1];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      pL[p] = params[cL * NP + p];
      pR[p] = params[cR * NP + p];
      pm[p] = 0.5 * (pL[p] + pR[p]);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      qL[v] = tL[v * F + f];
      qR[v] = tR[v * F + f];
    }
    if constexpr (PDE::kLinear) {
      // linear flux: the trace of the averaged flux is the flux of the
      // averaged state's trace, so only the state traces are read
      double Fa[DIM][NV], Fb[DIM][NV];
      PDE::fluxes(qL, pL, a.pde, Fa);
      PDE::fluxes(qR, pR, a.pde, Fb);
#pragma unroll
      for (int v = 0; v < NV; ++v) FL[v] = FR[v] = 0.0;
#pragma unroll
      for (int e = 0; e < DIM; ++e) {
        if (e != d) continue;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          if (!PDE::flux_nonzero(e, v)) continue;
          FL[v] = Fa[e][v];
          FR[v] = Fb[e][v];
        }
      }
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        FL[v] = tL[(NV + v) * F + f];
        FR[v] = tR[(NV + v) * F + f];
      }
    }
    if (bc == ADG_BC_WALL) {
      // both sides hold this cell's trace: replace the outside one
      double qx[NV], Fx[NV];
      Wall<PDE>::apply(d, side ? qL : qR, side ? FL : FR, qx, Fx);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (side) {
          qR[v] = qx[v];
          FR[v] = Fx[v];
        } else {
          qL[v] = qx[v];
          FL[v] = Fx[v];
        }
      }
    }
    if constexpr (HasUserBoundary<PDE>::value) {
      if (bc == ADG_BC_USER) {
        // the user's boundaryValues at this face node
        const int fa = DIM == 2 ? f : f % Geo<PDE, N>::n, fb = DIM == 2 ? 0 : f / Geo<PDE, N>::n;
        double x[3] = {0.0, 0.0, 0.0};
        int in_face = 0;
#pragma unroll
        for (int e = 0; e < DIM; ++e) {
          if (e == d) {
            x[e] = a.lo[e] + (c_own[e] + side) * a.h[e];
          } else {
            const int ke = in_face++ == 0 ? fa : fb;
            x[e] = a.lo[e] + (c_own[e] + a.t64.xi[ke]) * a.h[e];
          }
        }
        double qx[NV], Fx[NV];
        PDE::boundary(x, t, dt, face, side ? qL : qR, side ? pL : pR, side ? FL : FR, qx, Fx);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          if (side) {
            qR[v] = qx[v];
            FR[v] = Fx[v];
          } else {
            qL[v] = qx[v];
            FL[v] = Fx[v];
          }
        }
      }
    }
    const double s = fmax(PDE::max_eigen(qL, pL, a.pde, d), PDE::max_eigen(qR, pR, a.pde, d));
    double B[NV];
    if constexpr (PDE::kHasNcp) {
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
}

// Corrector phase 2 at node k of local cell lc: the surface term of Eq. (6),
// from the fluctuations of its 2 dim faces in fl.
template <class PDE, int N>
__device__ __forceinline__ void surface_terms(const KArgs& a, const double* fl, int lc, int k,
                                              double (&surf)[PDE::NV]) {
  using G = Geo<PDE, N>;
  constexpr int n = G::n, F = G::F, NV = G::NV, DIM = G::DIM;
  const Tables<double>& T = a.t64;
  int kk[3] = {0, 0, 0};
  node_coords<DIM>(k, n, kk);
  int fidx[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    // face-node index of node k on the faces normal to d
    if (DIM == 2) fidx[d] = kk[1 - d];
    else fidx[d] = d == 0 ? kk[1] + n * kk[2] : (d == 1 ? kk[0] + n * kk[2] : kk[0] + n * kk[1]);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double sv = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double hi = fl[((lc * 2 * DIM + 2 * d + 1) * NV + v) * F + fidx[d]];
      const double lo = fl[((lc * 2 * DIM + 2 * d) * NV + v) * F + fidx[d]];
      sv += (T.l1[kk[d]] * hi + T.l0[kk[d]] * lo) * T.invw[kk[d]];
    }
    surf[v] = sv;
  }
}

template <class PDE, int N>
__global__ void __launch_bounds__((GeoB<PDE, N>::BLOCK))
correct_kernel(const KArgs a, double* __restrict__ Q, const double* __restrict__ params,
               const double* __restrict__ clock, const double* __restrict__ traces, int next_dt) {
  using G = Geo<PDE, N>;
  using GB = GeoB<PDE, N>;
  constexpr int S = G::S, NV = G::NV, NP = G::NP, DIM = G::DIM;
  constexpr int CPB = GB::CPB, BLOCK = GB::BLOCK;
  __shared__ double fl[CPB * GB::FL_PER_CELL];
  __shared__ double red[BLOCK];

  const int tid = threadIdx.x;
  const int cell0 = corr_cell0<DIM, CPB>(a, xcd_block(blockIdx.x, a.nblocks));
  const double dt = clock[1];
  const int ncells = (int)a.ncells;

  // this thread's node of the update; for PDEs linear in Q (few registers
  // in the face phase) its state is loaded now, so that the loads overlap
  // the face phase (measured: -2 to -3 % on elasticity, +5 % on Euler)
  const int lc = tid / S, k = tid - lc * S;
  const int cell = cell0 + lc;
  double qold[NV];
  if constexpr (PDE::kLinear) {
    if (cell < ncells) {
#pragma unroll
      for (int v = 0; v < NV; ++v) qold[v] = Q[((long long)cell * NV + v) * S + k];
    }
  }

  face_fluctuations<PDE, N, CPB, BLOCK>(a, params, traces, clock[0], dt, cell0, tid, fl);
  __syncthreads();

  double lam = 0.0;
  if (cell < ncells) {
    double surf[NV], qn[NV], P[NP > 0 ? NP : 1];
    surface_terms<PDE, N>(a, fl, lc, k, surf);
#pragma unroll
    for (int p = 0; p < NP; ++p) P[p] = params[cell * NP + p];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const long long idx = ((long long)cell * NV + v) * S + k;
      qn[v] = (PDE::kLinear ? qold[v] : Q[idx]) - surf[v];
      Q[idx] = qn[v];
    }
    if (next_dt) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) lam = lam_max(lam, PDE::max_eigen(qn, P, a.pde, d));
    }
  }
  if (next_dt) {
    const double m = block_max<BLOCK>(lam, red);
    if (tid == 0) slot_max(a.slots, blockIdx.x, m);
  }
}

// ---------------------------------------------------------------------------
// Step fusion (Sec. 5.1) for PDEs linear in Q with the step size held
// fixed: the corrector of step n (Rusanov, surface integral, update; from
// the traces tr_in of step n's prediction and Q = u^n + dt vol^n) and the
// predictor of step n + 1 from the resulting u^{n+1}, in one pass over the
// cells, with the traces of step n + 1 in tr_out.  Saves the state's write
// and re-read between the two phases.  clock = {t^n, dt}; the predictor
// uses t^n + dt.  rec_out (when the context has receivers): u^{n+1} at the
// receivers, [nrec][NV].
// ---------------------------------------------------------------------------
template <class PDE, int N, class R>
struct GeoStep {
  using GL = GeoL<PDE, N, R>;
  // doubles of LDS: the predictor's rows (R), the fluctuations, u^{n+1}
  static constexpr int LDS_D = cmax(cmax((GL::ELEMS * (int)sizeof(R) + 7) / 8, GL::CPB * GeoB<PDE, N>::FL_PER_CELL),
                                    GL::CPB * Geo<PDE, N>::NV * Geo<PDE, N>::S);
  static constexpr bool built = PDE::kLinear && LDS_D * 8 <= 150 * 1024;
};

template <class PDE, int N, class R>
__global__ void __launch_bounds__((GeoL<PDE, N, R>::BLOCK), (GeoL<PDE, N, R>::MIN_WAVES))
step_kernel_lin(const KArgs a, double* Q, const double* __restrict__ params, const double* __restrict__ clock,
                const double* __restrict__ tr_in, double* __restrict__ tr_out, double* __restrict__ rec_out) {
  using G = Geo<PDE, N>;
  using GL = GeoL<PDE, N, R>;
  static_assert(GeoStep<PDE, N, R>::built, "step fusion is built for PDEs linear in Q");
  constexpr int S = G::S, NV = G::NV, NP = G::NP, CPB = GL::CPB, BLOCK = GL::BLOCK;
  __shared__ double lds[GeoStep<PDE, N, R>::LDS_D];
  __shared__ double src_e[kMaxSources][kMaxLin + 1];

  const int tid = threadIdx.x;
  const int lc = tid / S, k = tid - lc * S;
  const long long cell0 = (long long)xcd_block(blockIdx.x, a.nblocks) * CPB;
  const long long cell = cell0 + lc;
  const bool active = cell < a.ncells;
  const long long cl = active ? cell : a.ncells - 1;
  const double t_n = clock[0], dt = clock[1];

  // corrector of step n
  double u1[NV];
  R P[NP > 0 ? NP : 1];
#pragma unroll
  for (int v = 0; v < NV; ++v) u1[v] = Q[(cl * NV + v) * S + k];
#pragma unroll
  for (int p = 0; p < NP; ++p) P[p] = R(params[cl * NP + p]);
  face_fluctuations<PDE, N, CPB, BLOCK>(a, params, tr_in, t_n, dt, (int)cell0, tid, lds);
  __syncthreads();
  if (active) {
    double surf[NV];
    surface_terms<PDE, N>(a, lds, lc, k, surf);
#pragma unroll
    for (int v = 0; v < NV; ++v) u1[v] -= surf[v];
  }
  __syncthreads();  // the fluctuations are read; the rows are free

  // receivers: u^{n+1} interpolated, a fixed-order sum per (receiver, quantity)
  if (a.nrec > 0 && rec_out) {
#pragma unroll
    for (int v = 0; v < NV; ++v) lds[(lc * NV + v) * S + k] = u1[v];
    __syncthreads();
    for (int i = tid; i < a.nrec * NV; i += BLOCK) {
      const int r = i / NV, v = i - r * NV;
      const long long c = a.rec_cell[r];
      if (c < cell0 || c >= cell0 + CPB || c >= a.ncells) continue;
      const double* w = a.rec_w + (long long)r * S;
      const double* uq = lds + ((c - cell0) * NV + v) * S;
      double acc = 0.0;
      for (int kk = 0; kk < S; ++kk) acc += w[kk] * uq[kk];
      rec_out[(long long)r * NV + v] = acc;
    }
    __syncthreads();
  }

  // predictor of step n + 1
  lin_predict_block<PDE, N, R>(a, reinterpret_cast<R*>(lds), src_e, tid, cell0, u1, P, params, t_n + dt, dt, Q,
                               tr_out);
}

// ---------------------------------------------------------------------------
// Eq. (7) on a given state: per-block maxima of the largest |eigenvalue|.
// ---------------------------------------------------------------------------
template <class PDE, int N>
__global__ void __launch_bounds__((GeoB<PDE, N>::BLOCK))
lambda_kernel(const KArgs a, const double* __restrict__ Q, const double* __restrict__ params) {
  using G = Geo<PDE, N>;
  using GB = GeoB<PDE, N>;
  constexpr int S = G::S, NV = G::NV, NP = G::NP, DIM = G::DIM, CPB = GB::CPB;
  __shared__ double red[GB::BLOCK];
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
    for (int d = 0; d < DIM; ++d) lam = lam_max(lam, PDE::max_eigen(q, P, a.pde, d));
  }
  const double m = block_max<GB::BLOCK>(lam, red);
  if (tid == 0) slot_max(a.slots, blockIdx.x, m);
}

namespace {  // one copy per translation unit

// One block folds the reduction slots, clears them for the next use, and
// updates the clock {t, dt}:
// mode & 1: dt <- dt_factor / max(slots)      (Eq. (7))
// mode & 2: t <- t + dt (the dt the step used, read before it is replaced)
__global__ void __launch_bounds__(kSlots)
finalize_kernel(unsigned long long* __restrict__ slots, double dt_factor, int mode,
                double* __restrict__ clock) {
  __shared__ double red[kSlots];
  double m = 0.0;
  if (mode & 1) {
    m = __longlong_as_double((long long)slots[threadIdx.x * kSlotStride]);
    slots[threadIdx.x * kSlotStride] = 0ull;
  }
  m = block_max<kSlots>(m, red);
  if (threadIdx.x == 0) {
    const double dt_used = clock[1];
    if (mode & 2) clock[0] = clock[0] + dt_used;
    if (mode & 1) clock[1] = dt_factor / m;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Physical admissibility per cell (Sec. 3.5); per-block counts summed by
// count_kernel.
// ---------------------------------------------------------------------------
template <class PDE, int N>
__global__ void __launch_bounds__((GeoB<PDE, N>::BLOCK))
admissible_kernel(const KArgs a, const double* __restrict__ Q, const double* __restrict__ params,
                  uint8_t* __restrict__ troubled) {
  using G = Geo<PDE, N>;
  using GB = GeoB<PDE, N>;
  constexpr int S = G::S, NV = G::NV, NP = G::NP, CPB = GB::CPB;
  __shared__ int bad[CPB];
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
  if (k == 0 && cell < a.ncells) troubled[cell] = (uint8_t)bad[lc];
  if (tid == 0) {
    int cnt = 0;
    for (int c = 0; c < CPB; ++c) cnt += (cell0_valid(a, blockIdx.x, CPB, c) ? bad[c] : 0);
    if (cnt) atomicAdd(reinterpret_cast<int*>(a.slots + (blockIdx.x % kSlots) * kSlotStride), cnt);
  }
}

namespace {

__global__ void __launch_bounds__(kSlots)
count_kernel(unsigned long long* __restrict__ slots, int32_t* __restrict__ count) {
  __shared__ int red[kSlots];
  int* const sl = reinterpret_cast<int*>(slots + threadIdx.x * kSlotStride);
  red[threadIdx.x] = *sl;
  *sl = 0;
  __syncthreads();
  for (int off = kSlots / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = red[0];
}

}  // namespace

}  // namespace adg

#include "predict64.hpp"
#include "adjoint.hpp"

#if !defined(__HIPCC_RTC__)
namespace adg {

// ---------------------------------------------------------------------------
// Launchers and the per-(PDE, N) kernel set.
// ---------------------------------------------------------------------------
}  // namespace adg

#include "limiter.hpp"

namespace adg {

// The flux half of each inflow face's outside trace: F_d(q_out) at every
// face node (the built-in fluxes do not depend on the material parameters).
template <class PDE, int N>
__global__ void __launch_bounds__(64) bc_flux_kernel(const KArgs a, double* __restrict__ tr) {
  constexpr int NV = PDE::NV, NP = PDE::NP, DIM = PDE::DIM, F = Geo<PDE, N>::F;
  const int f = threadIdx.x;
  if (f >= 2 * DIM || a.bc[f] != ADG_BC_INFLOW) return;
  const int d = f / 2;
  double q[NV], P[NP > 0 ? NP : 1], Fx[DIM][NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) q[v] = tr[(f * 2 * NV + v) * F];
#pragma unroll
  for (int p = 0; p < (NP > 0 ? NP : 1); ++p) P[p] = 1.0;
  PDE::fluxes(q, P, a.pde, Fx);
  for (int v = 0; v < NV; ++v)
    for (int k = 0; k < F; ++k) tr[((f * 2 + 1) * NV + v) * F + k] = PDE::flux_nonzero(d, v) ? Fx[d][v] : 0.0;
}

// The FP64 predictor of PDEs that are not linear in Q: one thread per node
// (predict_kernel_n64) where a cell fits one block of at most four waves,
// else the lane-pair kernel.
template <class PDE, int N>
struct UseN64 {
#if defined(ADG_PAIR_PREDICTOR)
  static constexpr bool value = false;
#else
  static constexpr bool value = GeoN64<PDE, N>::fits;
#endif
};

template <class PDE, int N>
struct Launch {
  using G = Geo<PDE, N>;
  using GB = GeoB<PDE, N>;
  using GP = std::conditional_t<UseN64<PDE, N>::value, GeoN64<PDE, N>, GeoA2<PDE, N, double>>;
  template <class GA>
  static int blocks_a(const KArgs& a) {
    return (int)((a.ncells + GA::CPB - 1) / GA::CPB);
  }
  static int blocks_b(const KArgs& a) { return (int)((a.ncells + GB::CPB - 1) / GB::CPB); }

  static hipError_t predict(const KArgs& a0, int precision, const double* Q, const double* params,
                            const double* clock, double* Qout, double* traces, int flux_traces,
                            hipStream_t st) {
    KArgs a = a0;
    a.flux_traces = flux_traces;
    if constexpr (PDE::kLinear) {
      if (a.picard_iters <= kMaxLin) {
        if (precision == ADG_MIXED_FP32) {
          using GL = GeoL<PDE, N, float>;
          a.nblocks = blocks_a<GL>(a);
          hipLaunchKernelGGL((predict_kernel_lin<PDE, N, float>), dim3(a.nblocks), dim3(GL::BLOCK), 0,
                             st, a, Q, params, clock, Qout, traces);
        } else {
          using GL = GeoL<PDE, N, double>;
          a.nblocks = blocks_a<GL>(a);
          hipLaunchKernelGGL((predict_kernel_lin<PDE, N, double>), dim3(a.nblocks), dim3(GL::BLOCK), 0,
                             st, a, Q, params, clock, Qout, traces);
        }
        return hipGetLastError();
      }
    }
    if (precision == ADG_MIXED_FP32) {
      using GA = GeoA1<PDE, N, float>;
      a.nblocks = blocks_a<GA>(a);
      hipLaunchKernelGGL((predict_kernel_node<PDE, N, float>), dim3(a.nblocks), dim3(GA::BLOCK), 0,
                         st, a, Q, params, clock, Qout, traces);
    } else if (precision == ADG_MIXED_BF16X3) {
      if constexpr (PDE::kLinear) {
        return hipErrorNotSupported;  // refused when the context is created
      } else {
        using GA = GeoA1<PDE, N, float, true>;
        a.nblocks = blocks_a<GA>(a);
        hipLaunchKernelGGL((predict_kernel_node<PDE, N, float, true>), dim3(a.nblocks), dim3(GA::BLOCK), 0,
                           st, a, Q, params, clock, Qout, traces);
      }
    } else if constexpr (UseN64<PDE, N>::value) {
      using GA = GeoN64<PDE, N>;
      a.nblocks = blocks_a<GA>(a);
      hipLaunchKernelGGL((predict_kernel_n64<PDE, N>), dim3(a.nblocks), dim3(GA::BLOCK), 0, st, a, Q,
                         params, clock, Qout, traces);
    } else {
      using GA = GeoA2<PDE, N, double>;
      a.nblocks = blocks_a<GA>(a);
      hipLaunchKernelGGL((predict_kernel_pair<PDE, N, double>), dim3(a.nblocks), dim3(GA::BLOCK), 0,
                         st, a, Q, params, clock, Qout, traces);
    }
    return hipGetLastError();
  }
  static hipError_t correct(const KArgs& a0, double* Q, const double* params, double* clock,
                            const double* traces, int next_dt, hipStream_t st) {
    KArgs a = a0;
    a.nblocks = blocks_b(a);
    hipLaunchKernelGGL((correct_kernel<PDE, N>), dim3(a.nblocks), dim3(GB::BLOCK), 0, st, a, Q,
                       params, clock, traces, next_dt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kSlots), 0, st, a.slots, a.dt_factor,
                       next_dt ? 3 : 2, clock);
    return hipGetLastError();
  }
  static hipError_t stable_dt(const KArgs& a0, const double* Q, const double* params, double* clock,
                              hipStream_t st) {
    KArgs a = a0;
    a.nblocks = blocks_b(a);
    hipLaunchKernelGGL((lambda_kernel<PDE, N>), dim3(a.nblocks), dim3(GB::BLOCK), 0, st, a, Q, params);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kSlots), 0, st, a.slots, a.dt_factor, 1, clock);
    return hipGetLastError();
  }
  static hipError_t admissible(const KArgs& a0, const double* Q, const double* params,
                               uint8_t* troubled, int32_t* count, hipStream_t st) {
    KArgs a = a0;
    a.nblocks = blocks_b(a);
    hipLaunchKernelGGL((admissible_kernel<PDE, N>), dim3(a.nblocks), dim3(GB::BLOCK), 0, st, a, Q,
                       params, troubled);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(count_kernel, dim3(1), dim3(kSlots), 0, st, a.slots, count);
    return hipGetLastError();
  }
  // corrector of step n fused with the predictor of step n + 1, then t += dt
  template <class R>
  static hipError_t step_fused_r(const KArgs& a0, double* Q, const double* params, double* clock,
                                 const double* tr_in, double* tr_out, double* rec_out, hipStream_t st) {
    using GL = GeoL<PDE, N, R>;
    KArgs a = a0;
    a.flux_traces = 0;
    a.nblocks = blocks_a<GL>(a);
    hipLaunchKernelGGL((step_kernel_lin<PDE, N, R>), dim3(a.nblocks), dim3(GL::BLOCK), 0, st, a, Q, params,
                       clock, tr_in, tr_out, rec_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kSlots), 0, st, a.slots, a.dt_factor, 2, clock);
    return hipGetLastError();
  }
  static hipError_t step_fused(const KArgs& a, int precision, double* Q, const double* params, double* clock,
                               const double* tr_in, double* tr_out, double* rec_out, hipStream_t st) {
    if constexpr (GeoStep<PDE, N, double>::built && GeoStep<PDE, N, float>::built) {
      if (precision == ADG_MIXED_FP32) return step_fused_r<float>(a, Q, params, clock, tr_in, tr_out, rec_out, st);
      return step_fused_r<double>(a, Q, params, clock, tr_in, tr_out, rec_out, st);
    } else {
      return hipErrorNotSupported;
    }
  }
  static constexpr decltype(KernelSet::step_fused) step_fused_entry() {
    if constexpr (GeoStep<PDE, N, double>::built && GeoStep<PDE, N, float>::built) return &step_fused;
    else return nullptr;
  }
  static constexpr decltype(KernelSet::adjoint) adjoint_entry() {
    if constexpr (GeoAdjL<PDE, N>::supported) return &AdjLaunch<PDE, N>::run;
    else return nullptr;
  }
  static constexpr decltype(KernelSet::lim_before) lim_before_entry() {
    if constexpr (GeoLim<PDE, N>::built) return &LimLaunch<PDE, N>::before;
    else return nullptr;
  }
  static constexpr decltype(KernelSet::lim_after) lim_after_entry() {
    if constexpr (GeoLim<PDE, N>::built) return &LimLaunch<PDE, N>::after;
    else return nullptr;
  }
  static hipError_t bc_flux(const KArgs& a, double* tr, hipStream_t st) {
    hipLaunchKernelGGL((bc_flux_kernel<PDE, N>), dim3(1), dim3(64), 0, st, a, tr);
    return hipGetLastError();
  }
  static const KernelSet* set() {
    static const KernelSet ks = {GP::BLOCK, GP::CPB, GB::CPB,
                                 &predict, &correct, &stable_dt, &admissible, adjoint_entry(),
                                 step_fused_entry(), lim_before_entry(), lim_after_entry(), &bc_flux,
                                 GeoAdjL<PDE, N>::supported ? KeepGeo<PDE, N>::SLOTS : 0};
    return &ks;
  }
};

}  // namespace adg
#endif

// Internal declarations shared by the host API and the kernel translation
// units of libadg.  Not part of the ABI.
#pragma once

// The device part (constants, tables, KArgs) is also compiled at run time by
// hiprtc for user-supplied PDEs (__HIPCC_RTC__), which brings its own HIP
// device runtime and no host headers.
#if !defined(__HIPCC_RTC__)
#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>
#endif
#include <cstdint>

#include "../../include/adg.h"
#include "basis.hpp"

namespace adg {

constexpr int kMaxN = 8;       // n = N + 1 points per axis
constexpr int kMaxSources = 16;
constexpr int kMaxVar = 16;
constexpr int kSlots = 256;       // reduction slots
constexpr int kSlotStride = 8;    // words between slots (64 bytes)
constexpr int kMaxLin = 16;       // Picard iterations the linear-PDE predictor takes

// One-dimensional tables on [0, 1] (see adg_basis_tables).  KW = K1^{-1} W is
// the time operator of the Picard update, invw = 1 / w.
template <class R>
struct Tables {
  R xi[kMaxN], w[kMaxN], invw[kMaxN], l0[kMaxN], l1[kMaxN];
  R D[kMaxN][kMaxN];   // D[i][j] = phi_j'(xi_i)
  R KW[kMaxN][kMaxN];  // (K1^{-1})_ij w_j
};

struct PdeConsts {
  double gamma;
  double adv[3];
  double kappa;
};

// Point source as the kernels see it: the owning cell, the Ricker
// parameters and the nodal weights phi_k(xi_s) / (|T| W_k) * weight[v] live in
// a device table of [nsrc][S][nvar] doubles.
struct SourceDev {
  long long cell;
  double f0, t0, amp;
};

// Everything a kernel needs besides the data pointers; passed by value.
struct KArgs {
  int cells[3];
  int bc[6];  // ADG_BC_* per face 2 d + side
  // ADG_BC_INFLOW faces (device): an outside trace per face in the layout of
  // a cell's face trace, [6][2][nvar][F]: the prescribed state and its
  // normal flux at every face node (filled once per context)
  const double* bc_trace;
  int picard_iters;
  int guess;  // ADG_GUESS_*: initial guess of the Picard iteration
  long long ncells;
  double lo[3], h[3], inv_h[3];  // lower corner of the domain, cell sizes
  double dt_factor;  // cfl / (dim (2N+1)) * min_d h_d
  PdeConsts pde;
  Tables<double> t64;
  Tables<float> t32;
  // lin_c[k] = w^T KW^k 1 (k = 0..kMaxLin): the weights of the time average
  // of the Picard iterate as a polynomial in dt L for PDEs linear in Q
  double lin_c[kMaxLin + 1];
  // 0: the linear-PDE predictor leaves the flux traces unwritten (the
  // corrector of a PDE with a linear flux evaluates the flux of the state
  // trace); set per launch
  int flux_traces;
  int nsrc;
  int nblocks;  // grid size of the cell kernels (for the block -> cell map)
  const SourceDev* src;
  const double* src_w;  // [nsrc][S][nvar]
  // receivers (set for the fused multi-step launches): cell and nodal
  // weights [nrec][S]
  int nrec;
  const long long* rec_cell;
  const double* rec_w;
  // reduction slots (workspace, zero between uses): kSlots words, each on
  // its own 64-byte line
  unsigned long long* slots;
  // the forward quantities of one step that its discrete adjoint reads
  // (linear-PDE predictor, FP64): written by the forward step when set, read
  // by the adjoint step instead of recomputing them; [C][keep slots][S]
  // doubles (see adg_keep_size).  Null in every other launch.
  double* keep;
};

// Workspace of a step with the a-posteriori subcell limiter (owned by the
// context, allocated on first use).
struct LimWork {
  const double* tab;  // A [m][n], B [n][m], Qf [n][m] of the order (limiter_tables)
  double* Qold;       // [C][nv][S]   u^n
  uint8_t* st_prev;   // [C]          status at the start of the step
  uint8_t* trb;       // [C]          troubled flags of this step
  double* lohi;       // [C][nv][2]   range of the subcell averages at t^n
  double* lohi_next;  // [C][nv][2]   range of the candidate's subcell averages (detect)
  int reuse;          // prepare takes lohi_next of DG cells (status 0) instead of projecting
  int store_next;     // detect writes lohi_next
  int* fv_list;       // [C]
  int* y_list;        // [C]
  int* counters;      // [4]: troubled cells, FV cells, DG cells with FV faces
  double* gfv;        // [C][2 dim][nv][F] FV fluxes at the face nodes of FV cells
};

#if !defined(__HIPCC_RTC__)
// Kernel entry points of one (PDE, dim, order) instantiation set.
struct KernelSet {
  int block;  // threads per block of the predictor
  int cells_per_block;    // predictor
  int cells_per_block_b;  // corrector and reductions
  hipError_t (*predict)(const KArgs&, int precision, const double* Q, const double* params,
                        const double* clock, double* Qout, double* traces, int flux_traces,
                        hipStream_t);
  hipError_t (*correct)(const KArgs&, double* Q, const double* params, double* clock,
                        const double* traces, int next_dt, hipStream_t);
  hipError_t (*stable_dt)(const KArgs&, const double* Q, const double* params, double* clock,
                          hipStream_t);
  hipError_t (*admissible)(const KArgs&, const double* Q, const double* params,
                           uint8_t* troubled, int32_t* count, hipStream_t);
  // Discrete adjoint of one FP64 step (nullptr where not built: PDEs that
  // are not linear in Q, orders whose kernel does not fit).  work holds
  // 2 C 2dim nvar F + C nparam doubles (the trace workspace).  With
  // KArgs::keep (a kept forward step) Q is not read.
  hipError_t (*adjoint)(const KArgs&, const double* Q, const double* params, const double* clock,
                        double* lam, double* gparams, double* work, hipStream_t);
  // Corrector of step n and predictor of step n + 1 in one kernel (the
  // predictor in the context's precision), fixed step size; then t += dt
  // (nullptr where not built: PDEs not linear in Q).  rec_out: [nrec][nvar]
  // samples of u^{n+1}, or null.
  hipError_t (*step_fused)(const KArgs&, int precision, double* Q, const double* params, double* clock,
                           const double* tr_in, double* tr_out, double* rec_out, hipStream_t);
  // The a-posteriori subcell limiter around an unlimited step (nullptr
  // where not built): lim_before ahead of the step, lim_after behind it.
  hipError_t (*lim_before)(const KArgs&, const double* Q, const double* sub_in, const uint8_t* status,
                           const LimWork&, hipStream_t);
  hipError_t (*lim_after)(const KArgs&, double* Q, double* clock, const double* traces, const double* sub_in,
                          double* sub_out, uint8_t* status, const LimWork&, int next_dt, hipStream_t);
  // the flux half of KArgs::bc_trace from its state half (inflow faces)
  hipError_t (*bc_flux)(const KArgs&, double* bc_trace, hipStream_t);
  // doubles per node of KArgs::keep (0 where the adjoint is not built)
  int keep_slots;
};

// Registries implemented by the per-PDE translation units; return nullptr if
// the order is not built.
const KernelSet* kernels_euler2(int order);
const KernelSet* kernels_euler3(int order);
const KernelSet* kernels_elastic3(int order);
const KernelSet* kernels_advection2(int order);
const KernelSet* kernels_advection3(int order);
int max_order_euler2();
int max_order_euler3();
int max_order_elastic3();
int max_order_advection2();
int max_order_advection3();

// PDEs compiled at run time (user.hip).
struct UserTraits {
  int dim, nv, np, linear, has_ncp, has_source, has_boundary;
};
struct UserModule;
adg_status user_traits(const char* source, const std::string& arch, UserTraits* t, std::string* err);
adg_status user_module_create(const char* source, const std::string& arch, int order, int precision,
                              bool linear_predictor, UserModule** out, std::string* err);
void user_module_destroy(UserModule* u);
hipError_t user_predict(const UserModule* u, const KArgs& a, const double* Q, const double* params,
                        const double* clock, double* Qout, double* traces, int flux_traces, hipStream_t st);
hipError_t user_correct(const UserModule* u, const KArgs& a, double* Q, const double* params, double* clock,
                        const double* traces, int next_dt, hipStream_t st);
hipError_t user_stable_dt(const UserModule* u, const KArgs& a, const double* Q, const double* params,
                          double* clock, hipStream_t st);
hipError_t user_admissible(const UserModule* u, const KArgs& a, const double* Q, const double* params,
                           uint8_t* troubled, int32_t* count, hipStream_t st);
#endif


}  // namespace adg

// C ABI of libadg (declared in include/adg.h): argument checking, context
// set-up, and the launch sequence of one step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "adg_internal.hpp"

using namespace adg;

struct adg_ctx {
  adg_config cfg;
  int n = 0, S = 0, F = 0, nv = 0, np = 0, dim = 0;
  long long C = 0;
  int device = 0;
  const KernelSet* ks = nullptr;
  KArgs args{};
  double* traces = nullptr;  // [C][2 dim][2][nv][F]
  double* traces2 = nullptr; // the second trace array of fused runs (adg_run_reserve)
  size_t trace_elems = 0;
  size_t trace_alloc = 0;    // doubles per trace array: also the adjoint's C x np face terms
  void* red = nullptr;       // reduction slots
  size_t red_bytes = 0;
  SourceDev* d_src = nullptr;
  double* d_src_w = nullptr;
  int nsrc = 0;
  long long* d_rec_cell = nullptr;
  double* d_rec_w = nullptr;  // [nrec][S]
  int nrec = 0;
  bool traces_ready = false;  // workspace holds traces of a predict call
  UserModule* user = nullptr;  // kernels of a run-time PDE (ks is null then)
  // subcell limiter workspace (allocated on the first limited step)
  LimWork lim{};
  void* lim_block = nullptr;
  size_t lim_bytes = 0;  // size of lim_block
  bool lim_ranges_stored = false;  // the last adg_step_limited stored its candidate's ranges
  double* d_bc_state = nullptr;  // [6][2][nvar][F] outside traces of inflow faces
  void* scratch = nullptr;       // this device's copy of the static scratch array
};

// Device scratch of adg_step_noalloc (callers that cannot allocate: graph
// capture, serving loops): the reduction slots and the face traces of one
// step.  Every GPU the library runs on holds its own copy for the life of
// the process; host code uses the per-device address from
// hipGetSymbolAddress, never the array's name.
constexpr size_t kScratchSlotBytes = sizeof(unsigned long long) * adg::kSlots * adg::kSlotStride;  // 16 KiB
constexpr size_t kScratchTraceBytes = size_t(32) << 20;                                          // 32 MiB
static __device__ __align__(256) unsigned char scratch[kScratchSlotBytes + kScratchTraceBytes];

namespace {

thread_local std::string g_err;

adg_status fail(adg_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

adg_status hip_fail(hipError_t e, const char* what) {
  return fail(ADG_ERR_HIP, std::string(what) + ": " + hipGetErrorName(e) + " (" +
                               hipGetErrorString(e) + ")");
}

#define ADG_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return hip_fail(e_, #call);   \
  } while (0)

constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices];  // scratch address per device, set once
std::mutex g_scratch_mu;

// The address of this device's scratch array (the current device's), looked
// up once per device.
hipError_t scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = p;
  }
  *out = g_scratch[device];
  return hipSuccess;
}

// zero the reduction slots (a kernel, not a memset node, so the call can be
// captured in a graph)
__global__ void clear_slots_kernel(unsigned long long* __restrict__ slots, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) slots[i] = 0ull;
}

const KernelSet* find_kernels(int pde, int dim, int order) {
  if (pde == ADG_PDE_EULER && dim == 2) return kernels_euler2(order);
  if (pde == ADG_PDE_EULER && dim == 3) return kernels_euler3(order);
  if (pde == ADG_PDE_ELASTIC && dim == 3) return kernels_elastic3(order);
  if (pde == ADG_PDE_ADVECTION && dim == 2) return kernels_advection2(order);
  if (pde == ADG_PDE_ADVECTION && dim == 3) return kernels_advection3(order);
  return nullptr;
}

int pde_nvar(int pde, int dim) {
  if (pde == ADG_PDE_EULER) return dim + 2;
  if (pde == ADG_PDE_ELASTIC) return 9;
  if (pde == ADG_PDE_ADVECTION) return 1;
  return 0;
}

int pde_nparam(int pde) { return pde == ADG_PDE_ELASTIC ? 3 : 0; }

// phi_i(x) of the Lagrange basis through the GL nodes.
double lagrange(const double* xi, int n, int i, double x) {
  double v = 1.0;
  for (int m = 0; m < n; ++m)
    if (m != i) v *= (x - xi[m]) / (xi[i] - xi[m]);
  return v;
}

// Cell and reference coordinates of a physical point (half-open cells).
bool locate(const adg_ctx* c, const double* x, long long* cell, double* ref) {
  long long idx = 0, mul = 1;
  for (int d = 0; d < c->dim; ++d) {
    const double h = (c->cfg.hi[d] - c->cfg.lo[d]) / c->cfg.cells[d];
    const double s = (x[d] - c->cfg.lo[d]) / h;
    const double fl = std::floor(s);
    if (!(fl >= 0.0 && fl < c->cfg.cells[d])) return false;
    ref[d] = s - fl;
    idx += (long long)fl * mul;
    mul *= c->cfg.cells[d];
  }
  *cell = idx;
  return true;
}

// out[r][v] = sum_k Phi_k(xi_r) Q[c_r][v][k], one thread per (receiver,
// quantity), the nodes summed in order: the same sum, bit for bit, as the
// receivers sampled inside the fused step kernel.
__global__ void sample_kernel(const double* __restrict__ Q, const long long* __restrict__ rcell,
                              const double* __restrict__ rw, double* __restrict__ out, int nrec, int nv,
                              int S) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrec * nv) return;
  const int r = i / nv, v = i - r * nv;
  const long long c = rcell[r];
  const double* w = rw + (long long)r * S;
  const double* uq = Q + (c * nv + v) * S;
  double acc = 0.0;
  for (int k = 0; k < S; ++k) acc += w[k] * uq[k];
  out[(long long)r * nv + v] = acc;
}

// lam[c_r][v][k] += Phi_k(xi_r) lamrec[r][v], the transpose of sample_kernel.
// One thread per (receiver, quantity, node); the thread of the first
// receiver in a cell adds, in receiver order, the terms of every receiver of
// that cell (a fixed order of the sums; the others return).
__global__ void sample_adjoint_kernel(const double* __restrict__ lamrec,
                                      const long long* __restrict__ rcell,
                                      const double* __restrict__ rw, double* __restrict__ lam,
                                      int nrec, int nv, int S) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)nrec * nv * S) return;
  const int r = (int)(i / ((long long)nv * S));
  const int j = (int)(i - (long long)r * nv * S), v = j / S, k = j - v * S;
  const long long c = rcell[r];
  for (int q = 0; q < r; ++q)
    if (rcell[q] == c) return;  // an earlier receiver's thread owns this cell
  double* x = lam + (c * nv + v) * S + k;
  double acc = *x;
  for (int q = r; q < nrec; ++q)
    if (rcell[q] == c) acc += rw[(long long)q * S + k] * lamrec[(long long)q * nv + v];
  *x = acc;
}

}  // namespace

extern "C" {

const char* adg_last_error(void) { return g_err.c_str(); }

int adg_max_order(int pde, int dim) {
  if (pde == ADG_PDE_EULER && dim == 2) return max_order_euler2();
  if (pde == ADG_PDE_EULER && dim == 3) return max_order_euler3();
  if (pde == ADG_PDE_ELASTIC && dim == 3) return max_order_elastic3();
  if (pde == ADG_PDE_ADVECTION && dim == 2) return max_order_advection2();
  if (pde == ADG_PDE_ADVECTION && dim == 3) return max_order_advection3();
  return 0;
}

adg_status adg_basis_tables(int order, double* xi, double* w, double* D, double* l0, double* l1,
                            double* K1inv) {
  if (order < 0 || order + 1 > kMaxN) return fail(ADG_ERR_INVALID_ARG, "order out of range 0..7");
  if (basis_tables(order + 1, xi, w, D, l0, l1, K1inv) != 0)
    return fail(ADG_ERR_INVALID_ARG, "basis construction failed");
  return ADG_OK;
}

adg_status adg_limiter_tables(int order, double* A, double* B, double* Qf) {
  if (order < 0 || order + 1 > kBasisMaxN) return fail(ADG_ERR_INVALID_ARG, "order out of range");
  if (!A || !B || !Qf) return fail(ADG_ERR_INVALID_ARG, "null output");
  if (limiter_tables(order + 1, A, B, Qf)) return fail(ADG_ERR_INVALID_ARG, "limiter tables failed");
  return ADG_OK;
}

}  // extern "C"

namespace {

// Shared by adg_create (built-in PDEs) and adg_create_user (source != null).
adg_status create_ctx(const adg_config* cfg, const char* source, adg_ctx** out) {
  if (!cfg || !out) return fail(ADG_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  const adg_config& c = *cfg;
  if (c.dim != 2 && c.dim != 3) return fail(ADG_ERR_INVALID_ARG, "dim must be 2 or 3");
  if (c.order < 1) return fail(ADG_ERR_INVALID_ARG, "order must be >= 1");
  if (source ? c.pde != ADG_PDE_USER : pde_nvar(c.pde, c.dim) == 0)
    return fail(ADG_ERR_INVALID_ARG, source ? "adg_create_user needs pde = ADG_PDE_USER" : "unknown pde");
  if (c.precision != ADG_FP64 && c.precision != ADG_MIXED_FP32 && c.precision != ADG_MIXED_BF16X3)
    return fail(ADG_ERR_INVALID_ARG, "unknown precision");
  if (c.precision == ADG_MIXED_BF16X3 && (source || c.pde != ADG_PDE_EULER))
    return fail(ADG_ERR_UNSUPPORTED, "the split-BF16 predictor is built for the Euler equations");
  if (!(c.cfl > 0.0) || !std::isfinite(c.cfl)) return fail(ADG_ERR_INVALID_ARG, "cfl must be > 0");
  if (c.picard_iters < 0 || c.picard_iters > 64)
    return fail(ADG_ERR_INVALID_ARG, "picard_iters must be in 0..64");
  if (c.initial_guess != ADG_GUESS_CONSTANT && c.initial_guess != ADG_GUESS_CERK)
    return fail(ADG_ERR_INVALID_ARG, "unknown initial_guess");
  if (c.initial_guess == ADG_GUESS_CERK &&
      (source || c.pde != ADG_PDE_EULER || c.precision != ADG_FP64))
    return fail(ADG_ERR_UNSUPPORTED,
                "the CERK initial guess is built for the FP64 predictor of the Euler equations");
  if (c.pde == ADG_PDE_EULER && !(c.gamma > 1.0)) return fail(ADG_ERR_INVALID_ARG, "gamma must be > 1");
  for (int d = 0; d < 3; ++d) {
    const int blo = c.bc[2 * d], bhi = c.bc[2 * d + 1];
    if (blo < ADG_BC_PERIODIC || blo > ADG_BC_USER || bhi < ADG_BC_PERIODIC || bhi > ADG_BC_USER)
      return fail(ADG_ERR_INVALID_ARG, "unknown boundary condition");
    if ((blo == ADG_BC_USER || bhi == ADG_BC_USER) && !source)
      return fail(ADG_ERR_INVALID_ARG, "ADG_BC_USER needs a run-time PDE with boundary_values");
    if (d >= c.dim && (blo || bhi)) return fail(ADG_ERR_INVALID_ARG, "boundary condition on a missing axis");
    if ((blo == ADG_BC_PERIODIC) != (bhi == ADG_BC_PERIODIC))
      return fail(ADG_ERR_INVALID_ARG, "an axis is periodic on both faces or on neither");
    if ((blo == ADG_BC_WALL || bhi == ADG_BC_WALL) && (c.pde == ADG_PDE_ADVECTION || c.pde == ADG_PDE_USER))
      return fail(ADG_ERR_INVALID_ARG, "no wall condition for this PDE");
    if ((blo == ADG_BC_INFLOW || bhi == ADG_BC_INFLOW) && c.pde == ADG_PDE_USER)
      return fail(ADG_ERR_INVALID_ARG, "no inflow condition for a run-time PDE");
    for (int side = 0; side < 2; ++side)
      if (c.bc[2 * d + side] == ADG_BC_INFLOW)
        for (int v = 0; v < 16; ++v)
          if (!std::isfinite(c.bc_state[2 * d + side][v]))
            return fail(ADG_ERR_INVALID_ARG, "inflow state must be finite");
  }
  long long C = 1;
  for (int d = 0; d < c.dim; ++d) {
    if (c.cells[d] < 1) return fail(ADG_ERR_INVALID_ARG, "cells must be >= 1");
    if (!(c.hi[d] > c.lo[d])) return fail(ADG_ERR_INVALID_ARG, "hi must exceed lo");
    C *= c.cells[d];
  }
  const KernelSet* ks = nullptr;
  UserModule* um = nullptr;
  int nv = 0, np = 0;
  if (source) {
    // the kernels for the user's struct, compiled for the current device
    if (c.order + 1 > kMaxN) return fail(ADG_ERR_UNSUPPORTED, "order above 7");
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "device properties");
    const std::string arch = prop.gcnArchName;
    std::string err;
    UserTraits t{};
    adg_status st = user_traits(source, arch, &t, &err);
    if (st) return fail(st, err);
    if (t.dim != c.dim) return fail(ADG_ERR_INVALID_ARG, "AdgUserPDE::DIM differs from cfg->dim");
    for (int f = 0; f < 6; ++f)
      if (c.bc[f] == ADG_BC_USER && !t.has_boundary)
        return fail(ADG_ERR_INVALID_ARG, "ADG_BC_USER needs AdgUserPDE::HAS_BOUNDARY and boundary_values");
    if (t.nv < 1 || t.np < 0 || t.nv + t.np > kMaxVar)
      return fail(ADG_ERR_INVALID_ARG, "AdgUserPDE: NV + NP must be in 1..16");
    const int I = c.picard_iters ? c.picard_iters : c.order + 1;
    st = user_module_create(source, arch, c.order, c.precision, t.linear && I <= kMaxLin, &um, &err);
    if (st) return fail(st, err);
    nv = t.nv;
    np = t.np;
  } else {
    ks = find_kernels(c.pde, c.dim, c.order);
    if (!ks) {
      char buf[128];
      snprintf(buf, sizeof buf, "order %d not built for pde %d in %dD (max %d)", c.order, c.pde,
               c.dim, adg_max_order(c.pde, c.dim));
      return fail(ADG_ERR_UNSUPPORTED, buf);
    }
    if ((C + ks->cells_per_block - 1) / ks->cells_per_block > 0x7fffffffLL)
      return fail(ADG_ERR_UNSUPPORTED, "too many cells for one launch");
    nv = pde_nvar(c.pde, c.dim);
    np = pde_nparam(c.pde);
  }

  adg_ctx* x = new (std::nothrow) adg_ctx;
  if (!x) {
    user_module_destroy(um);
    return fail(ADG_ERR_NOMEM, "host allocation failed");
  }
  x->cfg = c;
  x->dim = c.dim;
  x->n = c.order + 1;
  x->S = c.dim == 2 ? x->n * x->n : x->n * x->n * x->n;
  x->F = x->S / x->n;
  x->nv = nv;
  x->np = np;
  x->C = C;
  x->ks = ks;
  x->user = um;
  hipError_t e = hipGetDevice(&x->device);
  if (e != hipSuccess) {
    user_module_destroy(um);
    delete x;
    return hip_fail(e, "hipGetDevice");
  }

  e = scratch_address(x->device, &x->scratch);
  if (e != hipSuccess) {
    user_module_destroy(um);
    delete x;
    return hip_fail(e, "hipGetSymbolAddress(scratch)");
  }

  KArgs& a = x->args;
  for (int f = 0; f < 6; ++f) a.bc[f] = c.bc[f];
  for (int d = 0; d < 3; ++d) {
    a.lo[d] = d < c.dim ? c.lo[d] : 0.0;
    a.cells[d] = d < c.dim ? c.cells[d] : 1;
    a.h[d] = d < c.dim ? (c.hi[d] - c.lo[d]) / c.cells[d] : 1.0;
    a.inv_h[d] = 1.0 / a.h[d];
  }
  a.ncells = C;
  a.guess = c.initial_guess;
  a.picard_iters = c.picard_iters ? c.picard_iters
                                  : (c.initial_guess == ADG_GUESS_CERK ? (c.order > 3 ? c.order - 2 : 1) : c.order + 1);
  double hmin = a.h[0];
  for (int d = 1; d < c.dim; ++d) hmin = std::fmin(hmin, a.h[d]);
  a.dt_factor = c.cfl / (c.dim * (2.0 * c.order + 1.0)) * hmin;
  a.pde.gamma = c.gamma;
  for (int d = 0; d < 3; ++d) a.pde.adv[d] = c.adv[d];
  a.pde.kappa = c.kappa;
  {
    const int n = x->n;
    double xi[kMaxN], w[kMaxN], D[kMaxN * kMaxN], l0[kMaxN], l1[kMaxN], Ki[kMaxN * kMaxN];
    basis_tables(n, xi, w, D, l0, l1, Ki);
    std::memset(&a.t64, 0, sizeof a.t64);
    std::memset(&a.t32, 0, sizeof a.t32);
    for (int i = 0; i < n; ++i) {
      a.t64.xi[i] = xi[i];
      a.t64.w[i] = w[i];
      a.t64.invw[i] = 1.0 / w[i];
      a.t64.l0[i] = l0[i];
      a.t64.l1[i] = l1[i];
      for (int j = 0; j < n; ++j) {
        a.t64.D[i][j] = D[i * n + j];
        a.t64.KW[i][j] = Ki[i * n + j] * w[j];
      }
    }
    {
      double v[kMaxN];
      for (int i = 0; i < n; ++i) v[i] = 1.0;
      for (int k = 0; k <= kMaxLin; ++k) {
        if (k > 0) {
          double t[kMaxN];
          for (int i = 0; i < n; ++i) {
            t[i] = 0.0;
            for (int j = 0; j < n; ++j) t[i] += a.t64.KW[i][j] * v[j];
          }
          for (int i = 0; i < n; ++i) v[i] = t[i];
        }
        double c = 0.0;
        for (int i = 0; i < n; ++i) c += w[i] * v[i];
        a.lin_c[k] = c;
      }
    }
    for (int i = 0; i < n; ++i) {
      a.t32.xi[i] = (float)a.t64.xi[i];
      a.t32.w[i] = (float)a.t64.w[i];
      a.t32.invw[i] = (float)a.t64.invw[i];
      a.t32.l0[i] = (float)a.t64.l0[i];
      a.t32.l1[i] = (float)a.t64.l1[i];
      for (int j = 0; j < n; ++j) {
        a.t32.D[i][j] = (float)a.t64.D[i][j];
        a.t32.KW[i][j] = (float)a.t64.KW[i][j];
      }
    }
  }
  x->trace_elems = (size_t)C * 2 * c.dim * 2 * x->nv * x->F;
  x->trace_alloc = x->trace_elems + (ks && ks->adjoint ? (size_t)C * np : 0);
  e = hipMalloc((void**)&x->traces, x->trace_alloc * sizeof(double));
  if (e != hipSuccess) {
    user_module_destroy(um);
    delete x;
    return fail(ADG_ERR_NOMEM, std::string("trace workspace: ") + hipGetErrorString(e));
  }
  x->red_bytes = sizeof(unsigned long long) * kSlots * kSlotStride;
  e = hipMalloc(&x->red, x->red_bytes);
  if (e == hipSuccess) e = hipMemset(x->red, 0, x->red_bytes);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    (void)hipFree(x->traces);
    user_module_destroy(um);
    delete x;
    return fail(ADG_ERR_NOMEM, std::string("reduction slots: ") + hipGetErrorString(e));
  }
  a.slots = (unsigned long long*)x->red;
  {
    // inflow faces: the prescribed state at every face node; the flux half
    // is filled on the device
    const size_t nbt = (size_t)6 * 2 * nv * x->F;
    std::vector<double> bt(nbt, 0.0);
    bool inflow = false;
    for (int f = 0; f < 6; ++f) {
      if (c.bc[f] != ADG_BC_INFLOW) continue;
      inflow = true;
      for (int v = 0; v < nv; ++v)
        for (int k = 0; k < x->F; ++k) bt[((size_t)f * 2 * nv + v) * x->F + k] = c.bc_state[f][v];
    }
    e = hipMalloc((void**)&x->d_bc_state, sizeof(double) * nbt);
    if (e == hipSuccess) e = hipMemcpy(x->d_bc_state, bt.data(), sizeof(double) * nbt, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
      a.bc_trace = x->d_bc_state;
      if (inflow && ks) e = ks->bc_flux(a, x->d_bc_state, nullptr);
      if (e == hipSuccess) e = hipDeviceSynchronize();
    }
  }
  if (e != hipSuccess) {
    (void)hipFree(x->d_bc_state);
    (void)hipFree(x->red);
    (void)hipFree(x->traces);
    user_module_destroy(um);
    delete x;
    return fail(ADG_ERR_NOMEM, std::string("boundary states: ") + hipGetErrorString(e));
  }
  a.nsrc = 0;
  a.src = nullptr;
  a.src_w = nullptr;
  *out = x;
  return ADG_OK;
}

// The kernels of a context: the built-in set or the run-time module.
hipError_t k_predict(const adg_ctx* x, const double* Q, const double* params, const double* clock,
                     double* Qout, double* traces, int flux_traces, hipStream_t st) {
  if (x->user) return user_predict(x->user, x->args, Q, params, clock, Qout, traces, flux_traces, st);
  return x->ks->predict(x->args, x->cfg.precision, Q, params, clock, Qout, traces, flux_traces, st);
}
hipError_t k_correct(const adg_ctx* x, double* Q, const double* params, double* clock, int next_dt,
                     hipStream_t st) {
  if (x->user) return user_correct(x->user, x->args, Q, params, clock, x->traces, next_dt, st);
  return x->ks->correct(x->args, Q, params, clock, x->traces, next_dt, st);
}
hipError_t k_stable_dt(const adg_ctx* x, const double* Q, const double* params, double* clock,
                       hipStream_t st) {
  if (x->user) return user_stable_dt(x->user, x->args, Q, params, clock, st);
  return x->ks->stable_dt(x->args, Q, params, clock, st);
}
hipError_t k_admissible(const adg_ctx* x, const double* Q, const double* params, uint8_t* troubled,
                        int32_t* count, hipStream_t st) {
  if (x->user) return user_admissible(x->user, x->args, Q, params, troubled, count, st);
  return x->ks->admissible(x->args, Q, params, troubled, count, st);
}

}  // namespace

extern "C" {

adg_status adg_create(const adg_config* cfg, adg_ctx** out) { return create_ctx(cfg, nullptr, out); }

adg_status adg_create_user(const adg_config* cfg, const char* source, adg_ctx** out) {
  if (!source) return fail(ADG_ERR_INVALID_ARG, "null source");
  return create_ctx(cfg, source, out);
}

adg_status adg_destroy(adg_ctx* ctx) {
  if (!ctx) return ADG_OK;
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(ctx->traces);
  (void)hipFree(ctx->traces2);
  (void)hipFree(ctx->red);
  (void)hipFree(ctx->d_src);
  (void)hipFree(ctx->d_src_w);
  (void)hipFree(ctx->d_rec_cell);
  (void)hipFree(ctx->d_rec_w);
  (void)hipFree(ctx->lim_block);
  (void)hipFree(ctx->d_bc_state);
  user_module_destroy(ctx->user);
  (void)hipSetDevice(dev);
  delete ctx;
  return ADG_OK;
}

adg_status adg_query(const adg_ctx* ctx, adg_info* info) {
  if (!ctx || !info) return fail(ADG_ERR_INVALID_ARG, "null argument");
  info->nvar = ctx->nv;
  info->nparam = ctx->np;
  info->nodes_per_cell = ctx->S;
  info->face_nodes = ctx->F;
  info->ncells = ctx->C;
  info->state_elems = ctx->C * ctx->nv * ctx->S;
  info->trace_elems = ctx->trace_elems;
  info->workspace_bytes = ctx->trace_alloc * sizeof(double) * (ctx->traces2 ? 2 : 1) + ctx->red_bytes +
                          ctx->lim_bytes;
  return ADG_OK;
}

adg_status adg_node_coords(const adg_ctx* ctx, double* xyz) {
  if (!ctx || !xyz) return fail(ADG_ERR_INVALID_ARG, "null argument");
  const int n = ctx->n, dim = ctx->dim;
  for (long long c = 0; c < ctx->C; ++c) {
    long long cc[3] = {c % ctx->cfg.cells[0], (c / ctx->cfg.cells[0]) % (dim > 1 ? ctx->cfg.cells[1] : 1),
                       dim == 3 ? c / ((long long)ctx->cfg.cells[0] * ctx->cfg.cells[1]) : 0};
    for (int k = 0; k < ctx->S; ++k) {
      int kk[3] = {k % n, (k / n) % n, k / (n * n)};
      for (int d = 0; d < dim; ++d)
        xyz[((size_t)c * ctx->S + k) * dim + d] =
            ctx->cfg.lo[d] + (cc[d] + ctx->args.t64.xi[kk[d]]) * ctx->args.h[d];
    }
  }
  return ADG_OK;
}

static adg_status check_state(adg_ctx* ctx, const void* Q, const void* params) {
  if (!ctx) return fail(ADG_ERR_INVALID_ARG, "null context");
  if (!Q) return fail(ADG_ERR_INVALID_ARG, "null state");
  if (ctx->np > 0 && !params) return fail(ADG_ERR_INVALID_ARG, "this PDE needs material parameters");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != ctx->device)
    return fail(ADG_ERR_STATE, "current HIP device differs from the context's device");
  return ADG_OK;
}

adg_status adg_stable_dt(adg_ctx* ctx, const double* Q, const double* params, double* clock,
                         void* stream) {
  adg_status st = check_state(ctx, Q, params);
  if (st) return st;
  if (!clock) return fail(ADG_ERR_INVALID_ARG, "null clock");
  hipError_t e = k_stable_dt(ctx, Q, params, clock, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "stable_dt launch");
  return ADG_OK;
}

adg_status adg_read_clock_host(const double* clock, double* host, void* stream) {
  if (!clock || !host) return fail(ADG_ERR_INVALID_ARG, "null argument");
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e == hipSuccess) e = hipMemcpy(host, clock, 2 * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "read clock");
  return ADG_OK;
}

adg_status adg_predict(adg_ctx* ctx, const double* Q, const double* params, const double* clock,
                       double* Qvol, double* traces, void* stream) {
  adg_status st = check_state(ctx, Q, params);
  if (st) return st;
  if (!clock || !Qvol) return fail(ADG_ERR_INVALID_ARG, "null clock or output");
  // the caller's trace array gets both fields; the workspace only what the
  // corrector reads
  hipError_t e = k_predict(ctx, Q, params, clock, Qvol, traces ? traces : ctx->traces, traces ? 1 : 0,
                           (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "predict launch");
  if (!traces) ctx->traces_ready = true;
  return ADG_OK;
}

adg_status adg_correct(adg_ctx* ctx, double* Q, const double* params, double* clock, int flags,
                       void* stream) {
  adg_status st = check_state(ctx, Q, params);
  if (st) return st;
  if (!clock) return fail(ADG_ERR_INVALID_ARG, "null clock");
  if (flags & ~ADG_STEP_NEXT_DT) return fail(ADG_ERR_INVALID_ARG, "unknown flags");
  if (!ctx->traces_ready) return fail(ADG_ERR_STATE, "adg_correct needs a preceding adg_predict");
  hipError_t e = k_correct(ctx, Q, params, clock, (flags & ADG_STEP_NEXT_DT) ? 1 : 0, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "correct launch");
  return ADG_OK;
}

adg_status adg_step(adg_ctx* ctx, double* Q, const double* params, double* clock, int flags,
                    void* stream) {
  adg_status st = check_state(ctx, Q, params);
  if (st) return st;
  if (!clock) return fail(ADG_ERR_INVALID_ARG, "null clock");
  if (flags & ~ADG_STEP_NEXT_DT) return fail(ADG_ERR_INVALID_ARG, "unknown flags");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = k_predict(ctx, Q, params, clock, Q, ctx->traces, 0, s);
  if (e != hipSuccess) return hip_fail(e, "predict launch");
  ctx->traces_ready = true;
  e = k_correct(ctx, Q, params, clock, (flags & ADG_STEP_NEXT_DT) ? 1 : 0, s);
  if (e != hipSuccess) return hip_fail(e, "correct launch");
  return ADG_OK;
}

adg_status adg_step_noalloc(adg_ctx* ctx, double* Q, const double* params, double* clock, int flags,
                            void* stream) {
  adg_status st = check_state(ctx, Q, params);
  if (st) return st;
  if (!clock) return fail(ADG_ERR_INVALID_ARG, "null clock");
  if (flags & ~ADG_STEP_NEXT_DT) return fail(ADG_ERR_INVALID_ARG, "unknown flags");
  const size_t tbytes = ctx->trace_elems * sizeof(double);
  if (tbytes > kScratchTraceBytes) {
    char buf[200];
    snprintf(buf, sizeof buf,
             "adg_step_noalloc: the face traces of this mesh take %zu bytes, the static scratch holds %zu",
             tbytes, kScratchTraceBytes);
    return fail(ADG_ERR_UNSUPPORTED, buf);
  }
  hipStream_t s = (hipStream_t)stream;
  unsigned long long* slots = static_cast<unsigned long long*>(ctx->scratch);
  double* traces = reinterpret_cast<double*>(static_cast<unsigned char*>(ctx->scratch) + kScratchSlotBytes);
  KArgs a = ctx->args;
  a.slots = slots;
  const int nslot = kSlots * kSlotStride;
  hipLaunchKernelGGL(clear_slots_kernel, dim3((nslot + 255) / 256), dim3(256), 0, s, slots, nslot);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "clear launch");
  const int next = (flags & ADG_STEP_NEXT_DT) ? 1 : 0;
  if (ctx->user) {
    e = user_predict(ctx->user, a, Q, params, clock, Q, traces, 0, s);
    if (e == hipSuccess) e = user_correct(ctx->user, a, Q, params, clock, traces, next, s);
  } else {
    e = ctx->ks->predict(a, ctx->cfg.precision, Q, params, clock, Q, traces, 0, s);
    if (e == hipSuccess) e = ctx->ks->correct(a, Q, params, clock, traces, next, s);
  }
  if (e != hipSuccess) return hip_fail(e, "step launch");
  return ADG_OK;
}

adg_status adg_limiter_reserve(adg_ctx* ctx) {
  if (!ctx) return fail(ADG_ERR_INVALID_ARG, "null context");
  if (!ctx->ks || !ctx->ks->lim_before || !ctx->ks->lim_after)
    return fail(ADG_ERR_UNSUPPORTED,
                "the subcell limiter is built for the Euler equations (2-D: N <= 7, 3-D: N <= 3)");
  for (int f = 0; f < 6; ++f)
    if (ctx->args.bc[f] == ADG_BC_INFLOW) return fail(ADG_ERR_UNSUPPORTED, "the subcell limiter has no inflow faces");
  if (ctx->C > 0x7fffffffLL) return fail(ADG_ERR_UNSUPPORTED, "the subcell limiter indexes cells with 32-bit lists");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != ctx->device)
    return fail(ADG_ERR_STATE, "current HIP device differs from the context's device");
  const long long C = ctx->C;
  const int nv = ctx->nv, S = ctx->S, n = ctx->n, m = 2 * n - 1;
  if (!ctx->lim_block) {
    // one allocation, each array on a 256-byte boundary
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t ntab = (size_t)3 * m * n;
    const size_t sz[10] = {up(ntab * 8), up((size_t)C * nv * S * 8), up((size_t)C), up((size_t)C),
                           up((size_t)C * nv * 2 * 8), up((size_t)C * 4), up((size_t)C * 4), up(4 * 4),
                           up((size_t)C * 2 * ctx->dim * nv * ctx->F * 8), up((size_t)C * nv * 2 * 8)};
    size_t total = 0;
    for (size_t b : sz) total += b;
    void* blk = nullptr;
    if (hipMalloc(&blk, total) != hipSuccess) return fail(ADG_ERR_NOMEM, "limiter workspace");
    std::vector<double> tab(ntab);
    if (limiter_tables(n, tab.data(), tab.data() + m * n, tab.data() + 2 * m * n)) {
      (void)hipFree(blk);
      return fail(ADG_ERR_INVALID_ARG, "limiter tables failed");
    }
    hipError_t e = hipMemcpy(blk, tab.data(), ntab * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(blk);
      return hip_fail(e, "limiter tables upload");
    }
    char* p = (char*)blk;
    LimWork& w = ctx->lim;
    w.tab = (const double*)p;   p += sz[0];
    w.Qold = (double*)p;        p += sz[1];
    w.st_prev = (uint8_t*)p;    p += sz[2];
    w.trb = (uint8_t*)p;        p += sz[3];
    w.lohi = (double*)p;        p += sz[4];
    w.fv_list = (int*)p;        p += sz[5];
    w.y_list = (int*)p;         p += sz[6];
    w.counters = (int*)p;       p += sz[7];
    w.gfv = (double*)p;         p += sz[8];
    w.lohi_next = (double*)p;
    ctx->lim_block = blk;
    ctx->lim_ranges_stored = false;
    ctx->lim_bytes = total;
  }
  return ADG_OK;
}

adg_status adg_step_limited(adg_ctx* ctx, double* Q, double* clock, const double* sub_in, double* sub_out,
                            uint8_t* status, int32_t* counts, int flags, void* stream) {
  if (!ctx) return fail(ADG_ERR_INVALID_ARG, "null context");
  if (!ctx->ks || !ctx->ks->lim_before || !ctx->ks->lim_after)
    return fail(ADG_ERR_UNSUPPORTED,
                "the subcell limiter is built for the Euler equations (2-D: N <= 7, 3-D: N <= 3)");
  for (int f = 0; f < 6; ++f)
    if (ctx->args.bc[f] == ADG_BC_INFLOW) return fail(ADG_ERR_UNSUPPORTED, "the subcell limiter has no inflow faces");
  if (ctx->C > 0x7fffffffLL) return fail(ADG_ERR_UNSUPPORTED, "the subcell limiter indexes cells with 32-bit lists");
  adg_status st = check_state(ctx, Q, nullptr);
  if (st) return st;
  if (!clock || !sub_in || !sub_out || !status) return fail(ADG_ERR_INVALID_ARG, "null argument");
  if (sub_in == sub_out) return fail(ADG_ERR_INVALID_ARG, "sub_in and sub_out must be different arrays");
  if (flags & ~(ADG_STEP_NEXT_DT | ADG_STEP_REUSE_RANGES)) return fail(ADG_ERR_INVALID_ARG, "unknown flags");
  if (!ctx->lim_block) return fail(ADG_ERR_STATE, "adg_step_limited needs adg_limiter_reserve first");
  hipStream_t s = (hipStream_t)stream;
  // ranges of the previous call's candidate: taken only if that call stored
  // them and this one says its state continues from there
  const bool reuse_flag = (flags & ADG_STEP_REUSE_RANGES) != 0;
  LimWork w = ctx->lim;
  w.reuse = reuse_flag && ctx->lim_ranges_stored ? 1 : 0;
  w.store_next = reuse_flag ? 1 : 0;
  ctx->lim_ranges_stored = false;
  hipError_t e = ctx->ks->lim_before(ctx->args, Q, sub_in, status, w, s);
  if (e != hipSuccess) return hip_fail(e, "limiter prepare launch");
  e = k_predict(ctx, Q, nullptr, clock, Q, ctx->traces, 0, s);
  if (e != hipSuccess) return hip_fail(e, "predict launch");
  ctx->traces_ready = true;
  e = k_correct(ctx, Q, nullptr, clock, 0, s);
  if (e != hipSuccess) return hip_fail(e, "correct launch");
  e = ctx->ks->lim_after(ctx->args, Q, clock, ctx->traces, sub_in, sub_out, status, w,
                         (flags & ADG_STEP_NEXT_DT) ? 1 : 0, s);
  if (e != hipSuccess) return hip_fail(e, "limiter launch");
  ctx->lim_ranges_stored = reuse_flag;
  if (counts) ADG_HIP(hipMemcpyAsync(counts, ctx->lim.counters, 3 * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  return ADG_OK;
}

adg_status adg_check_admissible(adg_ctx* ctx, const double* Q, const double* params,
                                uint8_t* troubled, int32_t* count, void* stream) {
  adg_status st = check_state(ctx, Q, params);
  if (st) return st;
  if (!troubled || !count) return fail(ADG_ERR_INVALID_ARG, "null output");
  hipError_t e = k_admissible(ctx, Q, params, troubled, count, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "admissible launch");
  return ADG_OK;
}

adg_status adg_set_point_sources(adg_ctx* ctx, int n, const adg_point_source* src) {
  if (!ctx) return fail(ADG_ERR_INVALID_ARG, "null context");
  if (n < 0 || n > kMaxSources) return fail(ADG_ERR_INVALID_ARG, "0 <= n <= 16 sources");
  if (n > 0 && !src) return fail(ADG_ERR_INVALID_ARG, "null sources");
  const int S = ctx->S, nv = ctx->nv, nd = ctx->n;
  SourceDev hs[kMaxSources];
  double* hw = new (std::nothrow) double[(size_t)(n > 0 ? n : 1) * S * nv];
  if (!hw) return fail(ADG_ERR_NOMEM, "host allocation failed");
  const double* xi = ctx->args.t64.xi;
  const double* w = ctx->args.t64.w;
  double vol = 1.0;
  for (int d = 0; d < ctx->dim; ++d) vol *= ctx->args.h[d];
  for (int s = 0; s < n; ++s) {
    long long cell;
    double ref[3] = {0, 0, 0};
    if (!locate(ctx, src[s].x, &cell, ref)) {
      delete[] hw;
      return fail(ADG_ERR_INVALID_ARG, "point source outside the domain");
    }
    hs[s] = SourceDev{cell, src[s].f0, src[s].t0, src[s].amp};
    for (int k = 0; k < S; ++k) {
      int kk[3] = {k % nd, (k / nd) % nd, k / (nd * nd)};
      double phi = 1.0, mass = vol;
      for (int d = 0; d < ctx->dim; ++d) {
        phi *= lagrange(xi, nd, kk[d], ref[d]);
        mass *= w[kk[d]];
      }
      for (int v = 0; v < nv; ++v) hw[((size_t)s * S + k) * nv + v] = phi / mass * src[s].weight[v];
    }
  }
  (void)hipDeviceSynchronize();
  (void)hipFree(ctx->d_src);
  (void)hipFree(ctx->d_src_w);
  ctx->d_src = nullptr;
  ctx->d_src_w = nullptr;
  ctx->nsrc = 0;
  ctx->args.nsrc = 0;
  ctx->args.src = nullptr;
  ctx->args.src_w = nullptr;
  if (n > 0) {
    hipError_t e = hipMalloc((void**)&ctx->d_src, sizeof(SourceDev) * n);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_src_w, sizeof(double) * n * S * nv);
    if (e == hipSuccess) e = hipMemcpy(ctx->d_src, hs, sizeof(SourceDev) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(ctx->d_src_w, hw, sizeof(double) * n * S * nv, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      delete[] hw;
      return hip_fail(e, "source upload");
    }
    ctx->nsrc = n;
    ctx->args.nsrc = n;
    ctx->args.src = ctx->d_src;
    ctx->args.src_w = ctx->d_src_w;
  }
  delete[] hw;
  return ADG_OK;
}

adg_status adg_set_receivers(adg_ctx* ctx, int n, const double* xyz) {
  if (!ctx) return fail(ADG_ERR_INVALID_ARG, "null context");
  if (n < 0 || (n > 0 && !xyz)) return fail(ADG_ERR_INVALID_ARG, "bad receiver list");
  const int S = ctx->S, nd = ctx->n;
  long long* hc = new (std::nothrow) long long[n > 0 ? n : 1];
  double* hw = new (std::nothrow) double[(size_t)(n > 0 ? n : 1) * S];
  if (!hc || !hw) {
    delete[] hc;
    delete[] hw;
    return fail(ADG_ERR_NOMEM, "host allocation failed");
  }
  for (int r = 0; r < n; ++r) {
    double ref[3] = {0, 0, 0};
    if (!locate(ctx, xyz + 3 * r, &hc[r], ref)) {
      delete[] hc;
      delete[] hw;
      return fail(ADG_ERR_INVALID_ARG, "receiver outside the domain");
    }
    for (int k = 0; k < S; ++k) {
      int kk[3] = {k % nd, (k / nd) % nd, k / (nd * nd)};
      double phi = 1.0;
      for (int d = 0; d < ctx->dim; ++d) phi *= lagrange(ctx->args.t64.xi, nd, kk[d], ref[d]);
      hw[(size_t)r * S + k] = phi;
    }
  }
  (void)hipDeviceSynchronize();
  (void)hipFree(ctx->d_rec_cell);
  (void)hipFree(ctx->d_rec_w);
  ctx->d_rec_cell = nullptr;
  ctx->d_rec_w = nullptr;
  ctx->nrec = 0;
  if (n > 0) {
    hipError_t e = hipMalloc((void**)&ctx->d_rec_cell, sizeof(long long) * n);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_rec_w, sizeof(double) * n * S);
    if (e == hipSuccess) e = hipMemcpy(ctx->d_rec_cell, hc, sizeof(long long) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->d_rec_w, hw, sizeof(double) * n * S, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      delete[] hc;
      delete[] hw;
      return hip_fail(e, "receiver upload");
    }
    ctx->nrec = n;
  }
  delete[] hc;
  delete[] hw;
  return ADG_OK;
}

adg_status adg_sample_receivers(adg_ctx* ctx, const double* Q, double* out, void* stream) {
  adg_status st = check_state(ctx, Q, (const void*)1);
  if (st) return st;
  if (ctx->nrec == 0) return fail(ADG_ERR_STATE, "no receivers set");
  if (!out) return fail(ADG_ERR_INVALID_ARG, "null output");
  hipLaunchKernelGGL(sample_kernel, dim3((ctx->nrec * ctx->nv + 63) / 64), dim3(64), 0, (hipStream_t)stream, Q,
                     ctx->d_rec_cell, ctx->d_rec_w, out, ctx->nrec, ctx->nv, ctx->S);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "sample launch");
  return ADG_OK;
}

static bool run_fuses(const adg_ctx* ctx) {
  return ctx->ks && ctx->ks->step_fused && ctx->args.picard_iters <= kMaxLin;
}

adg_status adg_run_reserve(adg_ctx* ctx) {
  if (!ctx) return fail(ADG_ERR_INVALID_ARG, "null context");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != ctx->device)
    return fail(ADG_ERR_STATE, "current HIP device differs from the context's device");
  if (!run_fuses(ctx) || ctx->traces2) return ADG_OK;
  double* p = nullptr;
  hipError_t e = hipMalloc((void**)&p, ctx->trace_alloc * sizeof(double));
  if (e != hipSuccess) return fail(ADG_ERR_NOMEM, std::string("second trace array: ") + hipGetErrorString(e));
  ctx->traces2 = p;
  return ADG_OK;
}

// a step's keep buffer: the per-node slots, then the step's face traces
static long long keep_elems(const adg_ctx* ctx) {
  return ctx->C * (long long)ctx->S * ctx->ks->keep_slots + (long long)ctx->trace_elems;
}
static double* keep_traces(const adg_ctx* ctx, double* keep) {
  return keep + ctx->C * (long long)ctx->S * ctx->ks->keep_slots;
}

// nsteps fixed-dt steps (fused corrector/predictor kernels where built and
// nsteps > 1; the caller has checked adg_run_reserve then).  rec_out: the
// receiver samples after every step, or null.  keeps: step n's kept
// quantities for its adjoint at keeps + n keep_n, or null; step n's traces
// are then those of its keep buffer.
static hipError_t run_steps(adg_ctx* ctx, double* Q, const double* params, double* clock, int nsteps,
                            double* rec_out, double* keeps, long long keep_n, hipStream_t s) {
  auto ktr = [&](int n) { return keep_traces(ctx, keeps + n * keep_n); };
  const long long rec_stride = (long long)ctx->nrec * ctx->nv;
  auto sample = [&](int n) -> hipError_t {
    if (!rec_out) return hipSuccess;
    hipLaunchKernelGGL(sample_kernel, dim3((ctx->nrec * ctx->nv + 63) / 64), dim3(64), 0, s, Q, ctx->d_rec_cell,
                       ctx->d_rec_w, rec_out + n * rec_stride, ctx->nrec, ctx->nv, ctx->S);
    return hipGetLastError();
  };
  auto predict = [&](int n) -> hipError_t {  // the (unfused) predictor of step n
    if (!keeps) return k_predict(ctx, Q, params, clock, Q, ctx->traces, 0, s);
    KArgs a = ctx->args;
    a.keep = keeps + n * keep_n;
    return ctx->ks->predict(a, ctx->cfg.precision, Q, params, clock, Q, ktr(n), 0, s);
  };
  auto correct = [&](int n) -> hipError_t {  // the (unfused) corrector of step n
    if (!keeps) return k_correct(ctx, Q, params, clock, 0, s);
    return ctx->ks->correct(ctx->args, Q, params, clock, ktr(n), 0, s);
  };
  hipError_t e = hipSuccess;
  if (!(run_fuses(ctx) && nsteps > 1)) {
    for (int n = 0; n < nsteps && e == hipSuccess; ++n) {
      e = predict(n);
      if (e == hipSuccess) e = correct(n);
      if (e == hipSuccess) e = sample(n);
    }
  } else {
    KArgs a = ctx->args;
    a.nrec = rec_out ? ctx->nrec : 0;
    a.rec_cell = ctx->d_rec_cell;
    a.rec_w = ctx->d_rec_w;
    e = predict(0);  // predictor of the first step
    for (int n = 0; n + 1 < nsteps && e == hipSuccess; ++n) {
      double* rec = rec_out ? rec_out + n * rec_stride : nullptr;
      if (keeps) {
        a.keep = keeps + (n + 1) * keep_n;  // the fused predictor is step n + 1's
        e = ctx->ks->step_fused(a, ctx->cfg.precision, Q, params, clock, ktr(n), ktr(n + 1), rec, s);
      } else {
        e = ctx->ks->step_fused(a, ctx->cfg.precision, Q, params, clock, ctx->traces, ctx->traces2, rec, s);
        std::swap(ctx->traces, ctx->traces2);  // the newest traces are the workspace
      }
    }
    if (e == hipSuccess) e = correct(nsteps - 1);  // corrector of the last step
    if (e == hipSuccess) e = sample(nsteps - 1);
  }
  ctx->traces_ready = false;
  return e;
}

adg_status adg_run(adg_ctx* ctx, double* Q, const double* params, double* clock, int nsteps,
                   double* rec_out, void* stream) {
  adg_status st = check_state(ctx, Q, params);
  if (st) return st;
  if (!clock) return fail(ADG_ERR_INVALID_ARG, "null clock");
  if (nsteps < 0) return fail(ADG_ERR_INVALID_ARG, "nsteps must be >= 0");
  if (rec_out && ctx->nrec == 0) return fail(ADG_ERR_STATE, "no receivers set");
  if (nsteps == 0) return ADG_OK;
  if (run_fuses(ctx) && nsteps > 1 && !ctx->traces2)
    return fail(ADG_ERR_STATE, "adg_run needs adg_run_reserve first (fused steps)");
  hipError_t e = run_steps(ctx, Q, params, clock, nsteps, rec_out, nullptr, 0, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "run launch");
  return ADG_OK;
}

adg_status adg_sample_receivers_adjoint(adg_ctx* ctx, const double* lamrec, double* lam,
                                        void* stream) {
  adg_status st = check_state(ctx, lam, (const void*)1);
  if (st) return st;
  if (ctx->nrec == 0) return fail(ADG_ERR_STATE, "no receivers set");
  if (!lamrec) return fail(ADG_ERR_INVALID_ARG, "null receiver adjoint");
  const long long nthreads = (long long)ctx->nrec * ctx->nv * ctx->S;
  hipLaunchKernelGGL(sample_adjoint_kernel, dim3((unsigned)((nthreads + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, lamrec,
                     ctx->d_rec_cell, ctx->d_rec_w, lam, ctx->nrec, ctx->nv, ctx->S);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "sample adjoint launch");
  return ADG_OK;
}

adg_status adg_step_adjoint(adg_ctx* ctx, const double* Q, const double* params,
                            const double* clock, double* lam, double* gparams, void* stream) {
  adg_status st = check_state(ctx, Q, params);
  if (st) return st;
  if (!clock || !lam) return fail(ADG_ERR_INVALID_ARG, "null clock or adjoint");
  if (ctx->np > 0 && !gparams) return fail(ADG_ERR_INVALID_ARG, "null parameter gradient");
  for (int f = 0; f < 6; ++f)
    if (ctx->args.bc[f] != ADG_BC_PERIODIC) return fail(ADG_ERR_UNSUPPORTED, "the adjoint needs a periodic mesh");
  if (!ctx->ks || !ctx->ks->adjoint)
    return fail(ADG_ERR_UNSUPPORTED, "the adjoint is built for the PDEs linear in Q (elastic, advection)");
  if (ctx->args.picard_iters > ctx->cfg.order + 1)
    return fail(ADG_ERR_UNSUPPORTED, "the adjoint supports at most order + 1 Picard iterations");
  hipError_t e = ctx->ks->adjoint(ctx->args, Q, params, clock, lam, gparams, ctx->traces,
                                  (hipStream_t)stream);
  ctx->traces_ready = false;  // the adjoint reuses the trace workspace
  if (e != hipSuccess) return hip_fail(e, "adjoint launch");
  return ADG_OK;
}

// the checks of adg_step_adjoint for the kept-quantity pair below
static adg_status check_keep(adg_ctx* ctx, const void* keep) {
  if (!keep) return fail(ADG_ERR_INVALID_ARG, "null keep buffer");
  for (int f = 0; f < 6; ++f)
    if (ctx->args.bc[f] != ADG_BC_PERIODIC) return fail(ADG_ERR_UNSUPPORTED, "the adjoint needs a periodic mesh");
  if (ctx->user || !ctx->ks || !ctx->ks->adjoint || ctx->ks->keep_slots <= 0)
    return fail(ADG_ERR_UNSUPPORTED, "the adjoint is built for the PDEs linear in Q (elastic, advection)");
  if (ctx->cfg.precision != ADG_FP64) return fail(ADG_ERR_UNSUPPORTED, "the adjoint is that of the FP64 step");
  if (ctx->args.picard_iters > ctx->cfg.order + 1)
    return fail(ADG_ERR_UNSUPPORTED, "the adjoint supports at most order + 1 Picard iterations");
  return ADG_OK;
}

adg_status adg_keep_size(const adg_ctx* ctx, long long* n) {
  if (!ctx || !n) return fail(ADG_ERR_INVALID_ARG, "null context or output");
  if (ctx->user || !ctx->ks || !ctx->ks->adjoint || ctx->ks->keep_slots <= 0)
    return fail(ADG_ERR_UNSUPPORTED, "the adjoint is built for the PDEs linear in Q (elastic, advection)");
  *n = keep_elems(ctx);
  return ADG_OK;
}

adg_status adg_step_keep(adg_ctx* ctx, double* Q, const double* params, double* clock, double* keep,
                         void* stream) {
  adg_status st = check_state(ctx, Q, params);
  if (st) return st;
  if (!clock) return fail(ADG_ERR_INVALID_ARG, "null clock");
  st = check_keep(ctx, keep);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  KArgs a = ctx->args;
  a.keep = keep;
  double* tr = keep_traces(ctx, keep);  // the step's traces stay in its keep buffer
  hipError_t e = ctx->ks->predict(a, ctx->cfg.precision, Q, params, clock, Q, tr, 0, s);
  if (e != hipSuccess) return hip_fail(e, "predict launch");
  e = ctx->ks->correct(ctx->args, Q, params, clock, tr, 0, s);
  if (e != hipSuccess) return hip_fail(e, "correct launch");
  return ADG_OK;
}

adg_status adg_run_keep(adg_ctx* ctx, double* Q, const double* params, double* clock, int nsteps,
                        double* rec_out, double* keeps, void* stream) {
  adg_status st = check_state(ctx, Q, params);
  if (st) return st;
  if (!clock) return fail(ADG_ERR_INVALID_ARG, "null clock");
  if (nsteps < 0) return fail(ADG_ERR_INVALID_ARG, "nsteps must be >= 0");
  if (rec_out && ctx->nrec == 0) return fail(ADG_ERR_STATE, "no receivers set");
  st = check_keep(ctx, keeps);
  if (st) return st;
  if (nsteps == 0) return ADG_OK;
  if (run_fuses(ctx) && nsteps > 1 && !ctx->traces2)
    return fail(ADG_ERR_STATE, "adg_run_keep needs adg_run_reserve first (fused steps)");
  const long long keep_n = keep_elems(ctx);
  hipError_t e = run_steps(ctx, Q, params, clock, nsteps, rec_out, keeps, keep_n, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "run launch");
  return ADG_OK;
}

adg_status adg_step_adjoint_kept(adg_ctx* ctx, const double* params, const double* clock,
                                 const double* keep, double* lam, double* gparams, void* stream) {
  adg_status st = check_state(ctx, lam, params);
  if (st) return st;
  if (!clock) return fail(ADG_ERR_INVALID_ARG, "null clock");
  if (ctx->np > 0 && !gparams) return fail(ADG_ERR_INVALID_ARG, "null parameter gradient");
  st = check_keep(ctx, keep);
  if (st) return st;
  KArgs a = ctx->args;
  a.keep = const_cast<double*>(keep);  // read only by the adjoint kernels
  hipError_t e = ctx->ks->adjoint(a, nullptr, params, clock, lam, gparams, ctx->traces, (hipStream_t)stream);
  ctx->traces_ready = false;  // the adjoint reuses the trace workspace
  if (e != hipSuccess) return hip_fail(e, "adjoint launch");
  return ADG_OK;
}

}  // extern "C"

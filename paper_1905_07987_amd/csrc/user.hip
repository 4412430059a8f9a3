// PDEs supplied at run time as HIP source text (adg_create_user): the
// library's own kernel templates (embedded at build time as header texts)
// are compiled by hiprtc for the user's struct AdgUserPDE, through the
// adapter in user_pde.hpp, and launched from the loaded module.  Two
// compilations: a small one that reads the struct's traits (DIM, NV, NP,
// LINEAR, ...), then one of the kernels the configuration needs, which also
// exports their launch geometry as a __constant__ array.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cstring>
#include <string>
#include <vector>

#include "adg_internal.hpp"

namespace adg {

// Generated at build time from the kernel headers (rtc_headers.cpp).
extern const int kRtcHeaderCount;
extern const char* const kRtcHeaderNames[];
extern const char* const kRtcHeaderTexts[];

struct UserModule {
  hipModule_t mod = nullptr;
  hipFunction_t predict = nullptr, correct = nullptr, lambda = nullptr, admissible = nullptr;
  hipFunction_t finalize = nullptr, count = nullptr;
  int pred_block = 0, pred_cpb = 0, b_block = 0, b_cpb = 0;
};

namespace {

struct Compiled {
  std::vector<char> code;
  std::vector<std::string> lowered;
};

adg_status rtc_compile(const std::string& src, const std::vector<std::string>& names, const std::string& arch,
                       Compiled* out, std::string* err) {
  hiprtcProgram p;
  hiprtcResult r = hiprtcCreateProgram(&p, src.c_str(), "adg_user.hip", kRtcHeaderCount, kRtcHeaderTexts,
                                       kRtcHeaderNames);
  if (r != HIPRTC_SUCCESS) {
    *err = std::string("hiprtcCreateProgram: ") + hiprtcGetErrorString(r);
    return ADG_ERR_COMPILE;
  }
  for (const std::string& n : names) hiprtcAddNameExpression(p, n.c_str());
  const std::string arch_opt = "--offload-arch=" + arch;
  const char* opts[] = {arch_opt.c_str(), "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                        "-packed-fp32-ops"};
  r = hiprtcCompileProgram(p, (int)(sizeof opts / sizeof opts[0]), opts);
  size_t ls = 0;
  hiprtcGetProgramLogSize(p, &ls);
  std::string log(ls, '\0');
  if (ls) hiprtcGetProgramLog(p, &log[0]);
  if (r != HIPRTC_SUCCESS) {
    *err = std::string("hiprtc: ") + hiprtcGetErrorString(r) + "\n" + log;
    hiprtcDestroyProgram(&p);
    return ADG_ERR_COMPILE;
  }
  size_t cs = 0;
  hiprtcGetCodeSize(p, &cs);
  out->code.resize(cs);
  hiprtcGetCode(p, out->code.data());
  out->lowered.clear();
  for (const std::string& n : names) {
    const char* low = nullptr;
    if (hiprtcGetLoweredName(p, n.c_str(), &low) != HIPRTC_SUCCESS || !low) {
      *err = "hiprtc: no kernel for " + n;
      hiprtcDestroyProgram(&p);
      return ADG_ERR_COMPILE;
    }
    out->lowered.emplace_back(low);
  }
  hiprtcDestroyProgram(&p);
  return ADG_OK;
}

adg_status hip_err(hipError_t e, const char* what, std::string* err) {
  *err = std::string(what) + ": " + hipGetErrorName(e);
  return ADG_ERR_HIP;
}

// Read an int array exported by a loaded module.
adg_status read_ints(hipModule_t m, const char* name, int* out, int n, std::string* err) {
  hipDeviceptr_t p = nullptr;
  size_t bytes = 0;
  hipError_t e = hipModuleGetGlobal(&p, &bytes, m, name);
  if (e != hipSuccess) return hip_err(e, "hipModuleGetGlobal", err);
  if (bytes != sizeof(int) * (size_t)n) {
    *err = std::string("unexpected size of ") + name;
    return ADG_ERR_COMPILE;
  }
  e = hipMemcpyDtoH(out, p, bytes);
  if (e != hipSuccess) return hip_err(e, "hipMemcpyDtoH", err);
  return ADG_OK;
}

std::string prelude(const char* source) {
  return std::string("#include \"user_pde.hpp\"\n#line 1 \"AdgUserPDE\"\n") + source + "\n";
}

}  // namespace

adg_status user_traits(const char* source, const std::string& arch, UserTraits* t, std::string* err) {
  const std::string src = prelude(source) +
                          "extern \"C\" __constant__ int adg_user_traits[7] = {AdgUserPDE::DIM, "
                          "AdgUserPDE::NV, AdgUserPDE::NP, (int)AdgUserPDE::LINEAR, "
                          "(int)AdgUserPDE::HAS_NCP, (int)AdgUserPDE::HAS_SOURCE, "
                          "(int)adg::UserHasBoundary<AdgUserPDE>::value};\n";
  Compiled c;
  adg_status st = rtc_compile(src, {}, arch, &c, err);
  if (st) return st;
  hipModule_t m = nullptr;
  hipError_t e = hipModuleLoadData(&m, c.code.data());
  if (e != hipSuccess) return hip_err(e, "hipModuleLoadData", err);
  int v[7];
  st = read_ints(m, "adg_user_traits", v, 7, err);
  (void)hipModuleUnload(m);
  if (st) return st;
  t->dim = v[0];
  t->nv = v[1];
  t->np = v[2];
  t->linear = v[3];
  t->has_ncp = v[4];
  t->has_source = v[5];
  t->has_boundary = v[6];
  return ADG_OK;
}

adg_status user_module_create(const char* source, const std::string& arch, int order, int precision,
                              bool linear_predictor, UserModule** out, std::string* err) {
  *out = nullptr;
  const std::string N = std::to_string(order);
  const std::string UP = "adg::UserTerms<::AdgUserPDE>";
  std::string pred, geo;
  if (linear_predictor) {
    const char* R = precision == ADG_MIXED_FP32 ? "float" : "double";
    pred = "adg::predict_kernel_lin<" + UP + ", " + N + ", " + R + ">";
    geo = "adg::GeoL<" + UP + ", " + N + ", " + R + ">";
  } else if (precision == ADG_MIXED_FP32) {
    pred = "adg::predict_kernel_node<" + UP + ", " + N + ", float>";
    geo = "adg::GeoA1<" + UP + ", " + N + ", float>";
  } else {
    pred = "adg::predict_kernel_pair<" + UP + ", " + N + ", double>";
    geo = "adg::GeoA2<" + UP + ", " + N + ", double>";
  }
  const std::string gb = "adg::GeoB<" + UP + ", " + N + ">";
  const std::string src = prelude(source) + "extern \"C\" __constant__ int adg_user_geo[4] = {" + geo +
                          "::BLOCK, " + geo + "::CPB, " + gb + "::BLOCK, " + gb + "::CPB};\n";
  const std::vector<std::string> names = {"&" + pred,
                                          "&adg::correct_kernel<" + UP + ", " + N + ">",
                                          "&adg::lambda_kernel<" + UP + ", " + N + ">",
                                          "&adg::admissible_kernel<" + UP + ", " + N + ">",
                                          "&adg::finalize_kernel",
                                          "&adg::count_kernel"};
  Compiled c;
  adg_status st = rtc_compile(src, names, arch, &c, err);
  if (st) return st;
  UserModule* u = new UserModule;
  hipError_t e = hipModuleLoadData(&u->mod, c.code.data());
  if (e != hipSuccess) {
    delete u;
    return hip_err(e, "hipModuleLoadData", err);
  }
  hipFunction_t* fs[] = {&u->predict, &u->correct, &u->lambda, &u->admissible, &u->finalize, &u->count};
  for (size_t i = 0; i < names.size(); ++i) {
    e = hipModuleGetFunction(fs[i], u->mod, c.lowered[i].c_str());
    if (e != hipSuccess) {
      user_module_destroy(u);
      return hip_err(e, "hipModuleGetFunction", err);
    }
  }
  int g[4];
  st = read_ints(u->mod, "adg_user_geo", g, 4, err);
  if (st) {
    user_module_destroy(u);
    return st;
  }
  u->pred_block = g[0];
  u->pred_cpb = g[1];
  u->b_block = g[2];
  u->b_cpb = g[3];
  *out = u;
  return ADG_OK;
}

void user_module_destroy(UserModule* u) {
  if (!u) return;
  if (u->mod) (void)hipModuleUnload(u->mod);
  delete u;
}

namespace {
hipError_t launch(hipFunction_t f, long long blocks, int block, hipStream_t st, void** args) {
  return hipModuleLaunchKernel(f, (unsigned)blocks, 1, 1, (unsigned)block, 1, 1, 0, st, args, nullptr);
}
}  // namespace

hipError_t user_predict(const UserModule* u, const KArgs& a0, const double* Q, const double* params,
                        const double* clock, double* Qout, double* traces, int flux_traces, hipStream_t st) {
  KArgs a = a0;
  a.flux_traces = flux_traces;
  a.nblocks = (int)((a.ncells + u->pred_cpb - 1) / u->pred_cpb);
  void* args[] = {&a, &Q, &params, &clock, &Qout, &traces};
  return launch(u->predict, a.nblocks, u->pred_block, st, args);
}

hipError_t user_correct(const UserModule* u, const KArgs& a0, double* Q, const double* params, double* clock,
                        const double* traces, int next_dt, hipStream_t st) {
  KArgs a = a0;
  a.nblocks = (int)((a.ncells + u->b_cpb - 1) / u->b_cpb);
  void* args[] = {&a, &Q, &params, &clock, &traces, &next_dt};
  hipError_t e = launch(u->correct, a.nblocks, u->b_block, st, args);
  if (e != hipSuccess) return e;
  unsigned long long* slots = a.slots;
  double dt_factor = a.dt_factor;
  int mode = next_dt ? 3 : 2;
  void* fargs[] = {&slots, &dt_factor, &mode, &clock};
  return launch(u->finalize, 1, kSlots, st, fargs);
}

hipError_t user_stable_dt(const UserModule* u, const KArgs& a0, const double* Q, const double* params,
                          double* clock, hipStream_t st) {
  KArgs a = a0;
  a.nblocks = (int)((a.ncells + u->b_cpb - 1) / u->b_cpb);
  void* args[] = {&a, &Q, &params};
  hipError_t e = launch(u->lambda, a.nblocks, u->b_block, st, args);
  if (e != hipSuccess) return e;
  unsigned long long* slots = a.slots;
  double dt_factor = a.dt_factor;
  int mode = 1;
  void* fargs[] = {&slots, &dt_factor, &mode, &clock};
  return launch(u->finalize, 1, kSlots, st, fargs);
}

hipError_t user_admissible(const UserModule* u, const KArgs& a0, const double* Q, const double* params,
                           uint8_t* troubled, int32_t* count, hipStream_t st) {
  KArgs a = a0;
  a.nblocks = (int)((a.ncells + u->b_cpb - 1) / u->b_cpb);
  void* args[] = {&a, &Q, &params, &troubled};
  hipError_t e = launch(u->admissible, a.nblocks, u->b_block, st, args);
  if (e != hipSuccess) return e;
  unsigned long long* slots = a.slots;
  void* cargs[] = {&slots, &count};
  return launch(u->count, 1, kSlots, st, cargs);
}

}  // namespace adg

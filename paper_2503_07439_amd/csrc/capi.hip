// C ABI of the event-parallel tree-level matrix-element library (see
// include/nlome.h): argument validation, context state and dispatch to the
// per-process kernel units.  Host code only.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "generated/index.hpp"
#include "launch.hpp"
#include "nlome.h"

using namespace nlo;

namespace {

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
thread_local std::string g_err;

nlo_status fail(nlo_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
nlo_status fail(nlo_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

constexpr int NPROC_ = NPROC;

}  // namespace

struct nlo_ctx {
  nlo_params params;
  std::mutex mu;
  nlo_kernel_config cfg[NPROC_][5];
};

namespace {

nlo_proc_info info_of(int pid) {
  const ProcStatic& P = PROC_STATIC[pid];
  nlo_proc_info r;
  r.name = P.name;
  r.npart = P.npart;
  r.ninitial = P.nin;
  r.ncolour = P.nflow;
  r.nhel = P.nhel;
  r.ngood_hel = P.ngood;
  r.ndiagrams = P.ndiag;
  r.nterms = P.nterm;
  r.ncurrents = P.ncur;
  r.avg_factor = P.avg;
  r.ident_factor = P.ident;
  r.gs_pow = P.gs_pow;
  r.e_pow = P.e_pow;
  return r;
}

// average factor times g_s^(2 gs_pow) e^(2 e_pow), applied to the FP64 helicity sum
double coupling_scale(int pid, const nlo_params& p) {
  const ProcStatic& P = PROC_STATIC[pid];
  const double gs2 = 4.0 * M_PI * p.alpha_s, e2 = 4.0 * M_PI * p.alpha;
  return P.avg * std::pow(gs2, P.gs_pow) * std::pow(e2, P.e_pow);
}

nlo_status launch_me2(nlo_ctx* ctx, int pid, int64_t n, int64_t ld, const double* mom, double* out, nlo_prec prec,
                      hipStream_t st) {
  const nlo_kernel_config& kc = ctx->cfg[pid][prec];
  int var;
  if (prec == NLO_FP64) {
    var = VAR_F64;
  } else {
    int mode = kc.colour_mode;
    if (mode == 0) mode = (prec == NLO_MIXED) ? 2 : 1;
    var = (mode == 2) ? VAR_MFMA : VAR_F32;
  }
  LaunchArgs a{n, ld, mom, out, coupling_scale(pid, ctx->params), ctx->params.m_top, kc.block, st};
  hipError_t err = ME2_LAUNCH[pid][var](a);
  if (err != hipSuccess) return fail(NLO_EDEVICE, "nlo_me2: launch failed: %s", hipGetErrorString(err));
  return NLO_OK;
}

nlo_status check_ctx(const nlo_ctx* ctx, int proc_id, const char* fn) {
  if (!ctx) return fail(NLO_EINVAL, "%s: ctx is NULL", fn);
  if (proc_id < 0 || proc_id >= NPROC_) return fail(NLO_EPROC, "%s: unknown process id %d", fn, proc_id);
  return NLO_OK;
}

nlo_status use_device(const nlo_ctx* ctx, const char* fn) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(NLO_EDEVICE, "%s: hipGetDevice failed", fn);
  if (cur != ctx->params.device && hipSetDevice(ctx->params.device) != hipSuccess)
    return fail(NLO_EDEVICE, "%s: hipSetDevice(%d) failed", fn, ctx->params.device);
  return NLO_OK;
}

}  // namespace

extern "C" {

uint32_t nlo_abi_version(void) { return NLO_ABI_VERSION; }

const char* nlo_last_error(void) { return g_err.c_str(); }

int nlo_num_processes(void) { return NPROC_; }

nlo_status nlo_create(nlo_ctx** out, const nlo_params* params) {
  if (!out || !params) return fail(NLO_EINVAL, "nlo_create: NULL argument");
  *out = nullptr;
  if (!(params->alpha > 0) || !(params->alpha_s > 0) || !(params->m_top > 0))
    return fail(NLO_EINVAL, "nlo_create: couplings and top mass must be positive");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(NLO_EDEVICE, "nlo_create: no HIP device");
  if (params->device < 0 || params->device >= ndev)
    return fail(NLO_EINVAL, "nlo_create: device %d out of range [0, %d)", params->device, ndev);
  nlo_ctx* c = new (std::nothrow) nlo_ctx;
  if (!c) return fail(NLO_ENOMEM, "nlo_create: out of host memory");
  c->params = *params;
  for (auto& row : c->cfg)
    for (auto& k : row) k = nlo_kernel_config{256, 0};
  *out = c;
  return NLO_OK;
}

nlo_status nlo_destroy(nlo_ctx* ctx) {
  delete ctx;
  return NLO_OK;
}

nlo_status nlo_process_info(const nlo_ctx* ctx, int proc_id, nlo_proc_info* out) {
  (void)ctx;
  if (!out) return fail(NLO_EINVAL, "nlo_process_info: out is NULL");
  if (proc_id < 0 || proc_id >= NPROC_) return fail(NLO_EPROC, "nlo_process_info: unknown process id %d", proc_id);
  *out = info_of(proc_id);
  return NLO_OK;
}

nlo_status nlo_set_kernel_config(nlo_ctx* ctx, int proc_id, nlo_prec prec, const nlo_kernel_config* cfg) {
  nlo_status st = check_ctx(ctx, proc_id, "nlo_set_kernel_config");
  if (st) return st;
  if (!cfg) return fail(NLO_EINVAL, "nlo_set_kernel_config: cfg is NULL");
  if ((int)prec < 0 || (int)prec > NLO_MIXED) return fail(NLO_EINVAL, "nlo_set_kernel_config: bad precision");
  if (cfg->block < 64 || cfg->block > NLO_MAX_BLOCK || cfg->block % 64)
    return fail(NLO_EINVAL, "nlo_set_kernel_config: block %d must be a multiple of 64 in [64, %d]", cfg->block,
                NLO_MAX_BLOCK);
  if (cfg->colour_mode < 0 || cfg->colour_mode > 2) return fail(NLO_EINVAL, "nlo_set_kernel_config: bad colour_mode");
  if (cfg->colour_mode == 2 && prec == NLO_FP64)
    return fail(NLO_EUNSUPPORTED, "nlo_set_kernel_config: matrix-core colour contraction is FP32 only");
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->cfg[proc_id][prec] = *cfg;
  return NLO_OK;
}

nlo_status nlo_get_kernel_config(const nlo_ctx* ctx, int proc_id, nlo_prec prec, nlo_kernel_config* cfg) {
  nlo_status st = check_ctx(ctx, proc_id, "nlo_get_kernel_config");
  if (st) return st;
  if (!cfg) return fail(NLO_EINVAL, "nlo_get_kernel_config: cfg is NULL");
  if ((int)prec < 0 || (int)prec > NLO_MIXED) return fail(NLO_EINVAL, "nlo_get_kernel_config: bad precision");
  *cfg = ctx->cfg[proc_id][prec];
  return NLO_OK;
}

nlo_status nlo_me2(nlo_ctx* ctx, int proc_id, int64_t n, int64_t ld, const double* mom, double* me2, nlo_prec prec,
                   void* hip_stream) {
  nlo_status st = check_ctx(ctx, proc_id, "nlo_me2");
  if (st) return st;
  if (n < 0) return fail(NLO_EINVAL, "nlo_me2: n = %lld < 0", (long long)n);
  if (ld < n) return fail(NLO_EINVAL, "nlo_me2: ld = %lld < n = %lld", (long long)ld, (long long)n);
  if (prec != NLO_FP64 && prec != NLO_FP32 && prec != NLO_MIXED)
    return fail(NLO_EUNSUPPORTED, "nlo_me2: precision %d not supported (FP64, FP32, MIXED)", (int)prec);
  if (n == 0) return NLO_OK;
  if (!mom || !me2) return fail(NLO_EINVAL, "nlo_me2: NULL device pointer");
  if ((int64_t)((n + 1023) / 64) > (int64_t)0x7fffffff) return fail(NLO_EINVAL, "nlo_me2: n too large");
  std::lock_guard<std::mutex> g(ctx->mu);
  st = use_device(ctx, "nlo_me2");
  if (st) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  return launch_me2(ctx, proc_id, n, ld, mom, me2, prec, s);
}

}  // extern "C"

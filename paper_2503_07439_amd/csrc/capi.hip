// C ABI of the event-parallel tree-level matrix-element library (see
// include/nlome.h): argument validation, context state and dispatch to the
// per-process kernel units.  Host code only.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "generated/index.hpp"
#include "launch.hpp"
#include "phase_space.hpp"
#include "checks.hpp"
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
// Automatic colour unit: the vector ALU for every process.  Measured on
// MI355X with the nested helicity schedule, the matrix-core variant stages
// each helicity's flow vectors through LDS behind two barriers and is slower
// at 6 flows (gg -> t tbar g: 2.70 against 1.83 ms per 2^22 events) and at
// 24 (gg -> t tbar g g); nlo_set_kernel_config selects it explicitly.
int auto_colour_mode(int pid, nlo_prec prec) {
  (void)pid;
  (void)prec;
  return 1;
}

}  // namespace

#ifndef NLO_BUILD_ID
#define NLO_BUILD_ID "unversioned"
#endif

struct nlo_ctx {
  nlo_params params;
  std::mutex mu;
  nlo_kernel_config cfg[NPROC_][5];
  nlo_fks_config fks_cfg[NFKS][5];   // per FKS sector (FKS_TABLE order) and precision
  std::string tuning_path;           // JSON tuning cache that autotune results are merged into
  // MIXED routes an FKS event to FP64 when kappa = xi (1-y) (or xi (1-y^2)
  // for the beams) is below this: measured on the stress sets, FP32 keeps
  // |dW|/|W| below 1e-4 for every event with kappa >= 0.1
  double fks_thr = 0.1;
  int fks_compact = 0;   // 1: skip the real |M|^2 of events whose R cut fails
  // workspace of the evaluation calls (FKS buckets, half-width fallback
  // list, cross-section chunks), sized by nlo_reserve for up to ws_events
  // events; evaluation calls never allocate
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int64_t ws_events = 0;
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
  r.nschedules = ME2_LAUNCH[pid][VAR_F64_ALT] != ME2_LAUNCH[pid][VAR_F64] ? 2 : 1;
  return r;
}

// average factor times g_s^(2 gs_pow) e^(2 e_pow), applied to the FP64 helicity sum
double coupling_scale(int pid, const nlo_params& p) {
  const ProcStatic& P = PROC_STATIC[pid];
  const double gs2 = 4.0 * M_PI * p.alpha_s, e2 = 4.0 * M_PI * p.alpha;
  return P.avg * std::pow(gs2, P.gs_pow) * std::pow(e2, P.e_pow);
}

bool half_prec(nlo_prec p) { return p == NLO_FP16 || p == NLO_BF16; }

// workspace of a half-width |M|^2 launch: the FP32 fallback list (n entries)
// and its counter
size_t half_ws_bytes(int64_t n) { return (size_t)n * sizeof(unsigned) + 128; }

nlo_status launch_me2(nlo_ctx* ctx, int pid, int64_t n, int64_t ld, const double* mom, double* out, nlo_prec prec,
                      hipStream_t st, void* ws = nullptr) {
  const nlo_kernel_config& kc = ctx->cfg[pid][prec];
  int var;
  if (prec == NLO_FP64) {
    var = kc.schedule ? VAR_F64_ALT : VAR_F64;
  } else if (prec == NLO_FP16) {
    var = VAR_F16;
  } else if (prec == NLO_BF16) {
    var = VAR_BF16;
  } else {
    const int mode = kc.colour_mode ? kc.colour_mode : auto_colour_mode(pid, prec);
    var = (mode == 2) ? VAR_MFMA : (kc.schedule ? VAR_F32_ALT : VAR_F32);
  }
  LaunchArgs a{n, ld, mom, out, coupling_scale(pid, ctx->params), ctx->params.m_top, kc.block, st};
  if (half_prec(prec)) {
    if (!ws) return fail(NLO_EINVAL, "nlo_me2: internal: no workspace for a half-width launch");
    a.fb_list = static_cast<unsigned*>(ws);
    const uintptr_t c = reinterpret_cast<uintptr_t>(a.fb_list + n);
    a.fb_cnt = reinterpret_cast<unsigned*>((c + 63) & ~uintptr_t(63));
    a.fb_launch = ME2_LAUNCH[pid][VAR_F32];
  }
  hipError_t err = ME2_LAUNCH[pid][var](a);
  if (err != hipSuccess) return fail(NLO_EDEVICE, "nlo_me2: launch failed: %s", hipGetErrorString(err));
  return NLO_OK;
}

// the reserved workspace must hold need bytes (evaluation calls never
// allocate: nlo_reserve sizes it); caller holds ctx->mu
nlo_status check_ws(const nlo_ctx* ctx, size_t need, int64_t n, const char* fn) {
  if (need <= ctx->ws_bytes) return NLO_OK;
  return fail(NLO_EINVAL, "%s: %lld events need a workspace of %zu bytes, %zu reserved; call nlo_reserve(ctx, %lld)",
              fn, (long long)n, need, ctx->ws_bytes, (long long)n);
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

// ---------------------------------------------------------------------------
// allocation-free FKS evaluation (nlo_subtracted_static)
// ---------------------------------------------------------------------------
// The workspace of up to SCRATCH_EVENTS events of any FKS sector lives in a
// file-scope device array: (4 NR + 3) doubles and 2 indices per event (NR <= 6
// particles) plus the bucket counters.  Each GPU holds its own copy at its own
// address, found once per device by hipGetSymbolAddress at nlo_create; host
// code uses that address, never the array's name.
constexpr int64_t SCRATCH_EVENTS = 65536;
constexpr size_t SCRATCH_BYTES = (size_t)SCRATCH_EVENTS * ((6 * 4 + 3) * sizeof(double) + 3 * sizeof(unsigned)) + 256 +
                                 FKS_SUM_PARTS * sizeof(double);
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// device address of this GPU's scratch array (called with no device change
// visible to the caller: the previous current device is restored)
nlo_status scratch_setup(int dev, const char* fn) {
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(NLO_EUNSUPPORTED, "%s: device %d beyond %d", fn, dev, SCRATCH_MAX_DEVICES);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[dev]) return NLO_OK;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(NLO_EDEVICE, "%s: hipGetDevice failed", fn);
  if (cur != dev && hipSetDevice(dev) != hipSuccess) return fail(NLO_EDEVICE, "%s: hipSetDevice(%d) failed", fn, dev);
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != dev) (void)hipSetDevice(cur);
  if (e != hipSuccess || !p)
    return fail(NLO_EDEVICE, "%s: address of the scratch array on device %d: %s", fn, dev, hipGetErrorString(e));
  g_scratch_ptr[dev] = p;
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
  nlo_status sst = scratch_setup(params->device, "nlo_create");
  if (sst) return sst;
  nlo_ctx* c = new (std::nothrow) nlo_ctx;
  if (!c) return fail(NLO_ENOMEM, "nlo_create: out of host memory");
  c->params = *params;
  for (auto& row : c->cfg)
    for (auto& k : row) k = nlo_kernel_config{256, 0, 0};
  for (auto& row : c->fks_cfg)
    for (auto& k : row) k = nlo_fks_config{256, 0, 256};
  *out = c;
  return NLO_OK;
}

nlo_status nlo_destroy(nlo_ctx* ctx) {
  if (ctx && ctx->ws) (void)hipFree(ctx->ws);
  delete ctx;
  return NLO_OK;
}

nlo_status nlo_set_fks_threshold(nlo_ctx* ctx, double threshold) {
  if (!ctx) return fail(NLO_EINVAL, "nlo_set_fks_threshold: ctx is NULL");
  if (!(threshold >= 0.0) || !(threshold <= 1.0))
    return fail(NLO_EINVAL, "nlo_set_fks_threshold: threshold must be in [0, 1]");
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->fks_thr = threshold;
  return NLO_OK;
}

nlo_status nlo_set_fks_mask_mode(nlo_ctx* ctx, int mode) {
  if (!ctx) return fail(NLO_EINVAL, "nlo_set_fks_mask_mode: ctx is NULL");
  if (mode != 0 && mode != 1) return fail(NLO_EINVAL, "nlo_set_fks_mask_mode: mode must be 0 or 1");
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->fks_compact = mode;
  return NLO_OK;
}

}  // extern "C"

namespace {

// validation shared by the direct call and batch items
nlo_status check_subtracted(const nlo_ctx* ctx, int real_proc, int fks_i, int fks_j, int64_t n, int64_t ld,
                            const double* born_mom, const double* xi_tilde, const double* y, const double* phi,
                            nlo_prec prec, const nlo_fks_out* out, const FksSector** sec_out, const char* fn) {
  nlo_status st = check_ctx(ctx, real_proc, fn);
  if (st) return st;
  const FksSector* sec = nullptr;
  for (const FksSector& f : FKS_TABLE)
    if (f.real == real_proc && f.i == fks_i && f.j == fks_j) sec = &f;
  if (!sec)
    return fail(NLO_EUNSUPPORTED, "%s: no FKS sector (%d, %d) for process %s", fn, fks_i, fks_j,
                PROC_STATIC[real_proc].name);
  if (n < 0) return fail(NLO_EINVAL, "%s: n = %lld < 0", fn, (long long)n);
  if (ld < n) return fail(NLO_EINVAL, "%s: ld = %lld < n = %lld", fn, (long long)ld, (long long)n);
  if (n > 0x7fffffffLL) return fail(NLO_EINVAL, "%s: n too large", fn);
  if (prec != NLO_FP64 && prec != NLO_FP32 && prec != NLO_MIXED)
    return fail(NLO_EUNSUPPORTED, "%s: precision %d not supported (FP64, FP32, MIXED)", fn, (int)prec);
  if (!out) return fail(NLO_EINVAL, "%s: out is NULL", fn);
  if (n > 0 && (!born_mom || !xi_tilde || !y || !phi || !out->W))
    return fail(NLO_EINVAL, "%s: NULL device pointer", fn);
  *sec_out = sec;
  return NLO_OK;
}

size_t fks_ws_bytes(int real_proc, int64_t n) {
  const int nr = PROC_STATIC[real_proc].npart;
  return (size_t)n * (nr * 4 + 3) * sizeof(double) + 3 * (size_t)n * sizeof(unsigned) + 128 +
         FKS_SUM_PARTS * sizeof(double);
}

// cross-section chunk of m events: momenta, weights, |M|^2, partial sums,
// accumulator, then the half-width fallback list
size_t xs_ws_bytes(int npart, int64_t m) {
  return ((size_t)npart * 4 * m + 2 * (size_t)m + XS_PART_DOUBLES + 8) * sizeof(double) + half_ws_bytes(m);
}

constexpr int64_t XS_CHUNK = (int64_t)1 << 20;

// the sectors of a real process, in table order
int fks_sectors(int real_proc, const FksSector** out, int max) {
  int k = 0;
  for (const FksSector& f : FKS_TABLE)
    if (f.real == real_proc && k < max) out[k++] = &f;
  return k;
}

// nlo_integrate_subtracted with n points per iteration and niter iterations:
// the FKS workspace, then Born momenta, weights, radiation variables, one
// dsig and one W array per sector, f, bin indices, histogram partials, the
// grid, partial sums, per-iteration sums and a counter
size_t int_ws_bytes(int real_proc, int64_t n, int niter) {
  const FksSector* secs[8];
  const int ns = fks_sectors(real_proc, secs, 8);
  if (!ns) return 0;
  const int nb = PROC_STATIC[secs[0]->born].npart;
  const int D = 4 * (nb - 2) + 3;
  const size_t dbl = (size_t)n * (nb * 4 + 4 + 2 * ns + 1) + (size_t)(VEGAS_HIST_BLOCKS + VEGAS_HIST_SEG) * D * VEGAS_BINS +
                     (size_t)D * (VEGAS_BINS + 1) + XS_PART_DOUBLES + 2 * (size_t)niter + 64;
  return fks_ws_bytes(real_proc, n) + 256 + dbl * sizeof(double) + (size_t)n * D + 256;
}

constexpr int INT_MAX_ITER = 64;

// nlo_generate_passing: block counts and offsets of one chunk, its total and
// the trial count
size_t gen_ws_bytes() { return 2 * (size_t)(GEN_CHUNK / 256) * sizeof(unsigned) + 256; }

// final-state leg classes of a process for the cuts
CutLegs legs_of(int pid) {
  const ProcStatic& P = PROC_STATIC[pid];
  const int nf = P.npart - P.nin;
  const unsigned all = (1u << nf) - 1u;
  const unsigned top = (P.top_legs >> P.nin) & all, lep = (P.lep_legs >> P.nin) & all;
  return CutLegs{all & ~top & ~lep, top, lep};
}

nlo_status check_cuts(const nlo_cuts* c, const char* fn) {
  if (!c) return fail(NLO_EINVAL, "%s: cuts is NULL", fn);
  const double v[7] = {c->jet_r, c->jet_ptmin, c->jet_ymax, c->top_ptmin, c->top_ymax, c->lep_ptmin, c->lep_ymax};
  for (double x : v)
    if (std::isnan(x)) return fail(NLO_EINVAL, "%s: a cut is NaN", fn);
  if (!(c->jet_r > 0.0)) return fail(NLO_EINVAL, "%s: jet_r must be positive", fn);
  if (c->njet_min < 0) return fail(NLO_EINVAL, "%s: njet_min < 0", fn);
  return NLO_OK;
}

// workspace that serves every evaluation call of up to n events: the largest
// FKS sector, a half-width |M|^2 launch, a cross-section chunk and an
// integration of up to min(n, 2^20) points per iteration
size_t ws_bytes_for(int64_t n) {
  size_t b = half_ws_bytes(n);
  for (const FksSector& f : FKS_TABLE) b = std::max(b, fks_ws_bytes(f.real, n));
  for (int p = 0; p < NPROC_; ++p) b = std::max(b, xs_ws_bytes(PROC_STATIC[p].npart, std::min(n, XS_CHUNK)));
  for (const FksSector& f : FKS_TABLE) b = std::max(b, int_ws_bytes(f.real, std::min(n, XS_CHUNK), INT_MAX_ITER));
  return std::max(b, gen_ws_bytes());
}

// the launch sequence of one FKS sector on stream s with workspace ws
hipError_t launch_subtracted(const nlo_ctx* ctx, const FksSector* sec, int real_proc, int64_t n, int64_t ld,
                             const double* born_mom, const double* xi_tilde, const double* y, const double* phi,
                             const uint8_t* mask, nlo_prec prec, const nlo_fks_out* out, void* ws, hipStream_t s,
                             bool force_compact = false) {
  const int nr = PROC_STATIC[real_proc].npart;
  char* base = static_cast<char*>(ws);
  FksArgs a{};
  a.n = n;
  a.ld = ld;
  a.born = born_mom;
  a.xit = xi_tilde;
  a.y = y;
  a.phi = phi;
  a.mask = mask;
  a.real = reinterpret_cast<double*>(base);
  a.me2r = a.real + (size_t)n * nr * 4;
  a.pinv = a.me2r + n;
  a.inv = reinterpret_cast<unsigned*>(a.pinv + 2 * (size_t)n);
  a.skip_inv = a.inv + n;
  a.redo = a.skip_inv + n;
  uintptr_t c = reinterpret_cast<uintptr_t>(a.redo + n);
  a.cnt = reinterpret_cast<unsigned*>((c + 63) & ~uintptr_t(63));
  a.compact = ((ctx->fks_compact || force_compact) && mask) ? 1 : 0;
  a.thr = ctx->fks_thr;
  a.mode = prec == NLO_FP64 ? 1 : (prec == NLO_FP32 ? 0 : 2);
  a.scale_b = coupling_scale(sec->born, ctx->params);
  a.scale_bm = coupling_scale(sec->bornm, ctx->params);
  a.g2 = 4.0 * M_PI * ctx->params.alpha_s;
  a.mt = ctx->params.m_top;
  a.xi_out = out->xi;
  a.born_out = out->born;
  a.gR = out->g_R;
  a.gS = out->g_S;
  a.gC = out->g_C;
  a.gCm = out->g_Cm;
  a.gSC = out->g_SC;
  a.gSCm = out->g_SCm;
  a.W = out->W;
  a.dsig = out->dsig;
  a.jac = out->jac;
  a.status = out->status;
  a.real_out = out->real_mom;
  const nlo_fks_config& fc = ctx->fks_cfg[sec - FKS_TABLE][prec];
  const int block = fc.ct_block;
  hipError_t err = sec->map(a, block, s);
  // real |M|^2 per bucket: FP32 from the front, FP64 from the back
  LaunchArgs la{n, n, a.real, a.me2r, coupling_scale(real_proc, ctx->params), ctx->params.m_top, fc.real_block, s,
                a.cnt, 0};
  // the real |M|^2 takes the FKS pair's invariants from the radiation variables
  if (sec->j >= 0) {
    la.ovp.a0 = std::min(sec->i, sec->j);
    la.ovp.b0 = std::max(sec->i, sec->j);
  } else {
    la.ovp.a0 = 0;
    la.ovp.b0 = sec->i;
    la.ovp.a1 = 1;
    la.ovp.b1 = sec->i;
  }
  la.ovv = a.pinv;
  const bool mfma = (fc.colour_mode ? fc.colour_mode : auto_colour_mode(real_proc, prec)) == 2;
  // FP32 bucket first (real |M|^2, then counterterms and W, which list the
  // events whose W came out unresolved or non-finite), then one FP64 launch of
  // each kernel over the FP64 bucket followed by that list (MIXED; a launch
  // that has any event at all takes at least one wave's time for one event's
  // whole helicity sum, about 1.7 ms in FP64 for g g -> t tbar g g, so the
  // re-evaluation gets no launch of its own)
  if (err == hipSuccess && a.mode != 1) err = ME2_LAUNCH[real_proc][mfma ? VAR_MFMA : VAR_F32](la);
  if (err == hipSuccess && a.mode != 1) err = sec->born_fn[1](a, 0, block, s);
  // compact mode: counterterms of the events that skipped the real |M|^2
  if (err == hipSuccess && a.compact && a.mode != 1) err = sec->born_fn[1](a, 2, block, s);
  if (err == hipSuccess && a.mode != 0) {
    la.which = a.mode == 2 ? 3 : 1;
    la.list = a.redo;
    err = ME2_LAUNCH[real_proc][VAR_F64](la);
  }
  if (err == hipSuccess && a.mode != 0) err = sec->born_fn[0](a, a.mode == 2 ? 9 : 1, block, s);
  if (err == hipSuccess && a.compact && a.mode != 0) err = sec->born_fn[0](a, a.mode == 2 ? 11 : 3, block, s);
  if (err == hipSuccess && out->w_sum) {
    // partial sums after the bucket counters (which take the first 64 bytes)
    double* part = reinterpret_cast<double*>(a.cnt + 16);
    hipLaunchKernelGGL(k_sum_part, dim3(FKS_SUM_PARTS), dim3(256), 0, s, n, (const double*)out->W, part);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, (const double*)part, out->w_sum);
    err = hipGetLastError();
  }
  return err;
}

}  // namespace

struct nlo_plan {
  nlo_ctx* ctx = nullptr;
  std::vector<void*> ws;
  std::vector<hipStream_t> streams;   // [0] capture origin, then the branches
  std::vector<hipEvent_t> events;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

// ---------------------------------------------------------------------------
// tuning cache: a JSON object {"format": ..., "entries": [{...}, ...]} of flat
// entries (string and number values), written and read here only
// ---------------------------------------------------------------------------
const char* const PREC_NAME[5] = {"fp64", "fp32", "fp16", "bf16", "mixed"};
const char* const KEY_FIELDS[5] = {"arch", "cus", "runtime", "driver", "build"};

struct TuneEntry {
  std::vector<std::string> k, v;
  std::vector<bool> str;   // value was a JSON string
  const std::string* get(const char* key) const {
    for (size_t i = 0; i < k.size(); ++i)
      if (k[i] == key) return &v[i];
    return nullptr;
  }
  void put(const char* key, const std::string& val, bool is_str) {
    for (size_t i = 0; i < k.size(); ++i)
      if (k[i] == key) {
        v[i] = val;
        str[i] = is_str;
        return;
      }
    k.emplace_back(key);
    v.push_back(val);
    str.push_back(is_str);
  }
};

// the identity of this device, runtime and build
TuneEntry tuning_identity(int device) {
  hipDeviceProp_t p{};
  int rt = 0, drv = 0;
  TuneEntry e;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) p.gcnArchName[0] = 0;
  (void)hipRuntimeGetVersion(&rt);
  (void)hipDriverGetVersion(&drv);
  e.put("arch", p.gcnArchName, true);
  e.put("cus", std::to_string(p.multiProcessorCount), false);
  e.put("runtime", std::to_string(rt), false);
  e.put("driver", std::to_string(drv), false);
  e.put("build", NLO_BUILD_ID, true);
  return e;
}

bool same_fields(const TuneEntry& a, const TuneEntry& b, const char* const* keys, int nk) {
  for (int i = 0; i < nk; ++i) {
    const std::string *x = a.get(keys[i]), *y = b.get(keys[i]);
    if (!x || !y || *x != *y) return false;
  }
  return true;
}

bool parse_tuning(const std::string& t, std::vector<TuneEntry>& out) {
  size_t i = t.find("\"entries\"");
  if (i == std::string::npos) return false;
  i = t.find('[', i);
  if (i == std::string::npos) return false;
  ++i;
  auto ws = [&]() { while (i < t.size() && (t[i] == ' ' || t[i] == '\n' || t[i] == '\r' || t[i] == '\t' || t[i] == ',')) ++i; };
  auto str = [&](std::string& o) {
    if (i >= t.size() || t[i] != '"') return false;
    ++i;
    o.clear();
    while (i < t.size() && t[i] != '"') {
      if (t[i] == '\\' && i + 1 < t.size()) ++i;
      o += t[i++];
    }
    if (i >= t.size()) return false;
    ++i;
    return true;
  };
  for (;;) {
    ws();
    if (i >= t.size()) return false;
    if (t[i] == ']') return true;
    if (t[i] != '{') return false;
    ++i;
    TuneEntry e;
    for (;;) {
      ws();
      if (i >= t.size()) return false;
      if (t[i] == '}') {
        ++i;
        break;
      }
      std::string key, val;
      if (!str(key)) return false;
      ws();
      if (i >= t.size() || t[i] != ':') return false;
      ++i;
      while (i < t.size() && t[i] == ' ') ++i;
      if (i < t.size() && t[i] == '"') {
        if (!str(val)) return false;
        e.put(key.c_str(), val, true);
      } else {
        const size_t b = i;
        while (i < t.size() && t[i] != ',' && t[i] != '}' && t[i] != ' ' && t[i] != '\n') ++i;
        val = t.substr(b, i - b);
        char* end = nullptr;
        (void)std::strtod(val.c_str(), &end);
        if (val.empty() || end != val.c_str() + val.size()) return false;
        e.put(key.c_str(), val, false);
      }
    }
    out.push_back(std::move(e));
  }
}

std::string format_tuning(const std::vector<TuneEntry>& es) {
  std::string o = "{\"format\": \"nlome-tuning-1\",\n \"entries\": [\n";
  for (size_t n = 0; n < es.size(); ++n) {
    o += "  {";
    for (size_t i = 0; i < es[n].k.size(); ++i) {
      if (i) o += ", ";
      o += "\"" + es[n].k[i] + "\": ";
      if (es[n].str[i]) {
        o += "\"";
        for (char c : es[n].v[i]) {
          if (c == '"' || c == '\\') o += '\\';
          o += c;
        }
        o += "\"";
      } else {
        o += es[n].v[i];
      }
    }
    o += n + 1 < es.size() ? "},\n" : "}\n";
  }
  return o + " ]}\n";
}

// read a cache file: missing = empty; false when it does not parse
bool read_tuning(const std::string& path, std::vector<TuneEntry>& out) {
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return true;
  std::string t;
  char buf[4096];
  size_t r;
  while ((r = std::fread(buf, 1, sizeof buf, f)) > 0) t.append(buf, r);
  std::fclose(f);
  if (t.find_first_not_of(" \n\r\t") == std::string::npos) return true;
  return parse_tuning(t, out);
}

int proc_by_name(const std::string& name) {
  for (int p = 0; p < NPROC_; ++p)
    if (name == PROC_STATIC[p].name) return p;
  return -1;
}

int prec_by_name(const std::string& name) {
  for (int p = 0; p < 5; ++p)
    if (name == PREC_NAME[p]) return p;
  return -1;
}

bool valid_block(long b) { return b >= 64 && b <= NLO_MAX_BLOCK && b % 64 == 0; }

// apply one entry of this device's key to the context; false if it names
// nothing this build has or holds an invalid configuration
bool apply_entry(nlo_ctx* ctx, const TuneEntry& e) {
  const std::string *kind = e.get("kind"), *proc = e.get("proc"), *prec = e.get("prec");
  if (!kind || !proc || !prec) return false;
  const int pid = proc_by_name(*proc), pr = prec_by_name(*prec);
  if (pid < 0 || pr < 0) return false;
  auto num = [&](const char* k, long& v) {
    const std::string* x = e.get(k);
    if (!x) return false;
    v = std::strtol(x->c_str(), nullptr, 10);
    return true;
  };
  long cm = 0;
  if (!num("colour_mode", cm) || cm < 0 || cm > 2 || (cm == 2 && pr != NLO_FP32 && pr != NLO_MIXED)) return false;
  if (*kind == "me2") {
    long b = 0, sc = 0;
    if (!num("block", b) || !valid_block(b)) return false;
    if (e.get("schedule") && (!num("schedule", sc) || sc < 0 || sc > 1)) return false;
    if (sc == 1 && (ME2_LAUNCH[pid][VAR_F64_ALT] == ME2_LAUNCH[pid][VAR_F64] || cm == 2)) return false;
    ctx->cfg[pid][pr] = nlo_kernel_config{(int)b, (int)cm, (int)sc};
    return true;
  }
  if (*kind == "subtracted") {
    long fi = 0, fj = 0, rb = 0, cb = 0;
    if (!num("i", fi) || !num("j", fj) || !num("real_block", rb) || !num("ct_block", cb)) return false;
    if (!valid_block(rb) || !valid_block(cb)) return false;
    for (int k = 0; k < NFKS; ++k)
      if (FKS_TABLE[k].real == pid && FKS_TABLE[k].i == fi && FKS_TABLE[k].j == fj) {
        ctx->fks_cfg[k][pr] = nlo_fks_config{(int)rb, (int)cm, (int)cb};
        return true;
      }
  }
  return false;
}

// merge one result into the context's cache file (no-op without one)
nlo_status merge_tuning(const nlo_ctx* ctx, TuneEntry e, const char* fn) {
  if (ctx->tuning_path.empty()) return NLO_OK;
  std::vector<TuneEntry> es;
  if (!read_tuning(ctx->tuning_path, es)) return fail(NLO_EINVAL, "%s: tuning cache %s does not parse", fn,
                                                      ctx->tuning_path.c_str());
  const TuneEntry id = tuning_identity(ctx->params.device);
  TuneEntry full = id;
  for (size_t i = 0; i < e.k.size(); ++i) full.put(e.k[i].c_str(), e.v[i], e.str[i]);
  static const char* const ident[10] = {"arch", "cus", "runtime", "driver", "build", "kind", "proc", "prec", "i", "j"};
  bool replaced = false;
  for (TuneEntry& x : es)
    if (same_fields(x, full, ident, 8) && (x.get("i") == nullptr) == (full.get("i") == nullptr) &&
        (!full.get("i") || same_fields(x, full, ident + 8, 2))) {
      x = full;
      replaced = true;
    }
  if (!replaced) es.push_back(full);
  const std::string tmp = ctx->tuning_path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return fail(NLO_EINVAL, "%s: cannot write %s", fn, tmp.c_str());
  const std::string text = format_tuning(es);
  const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
  if (std::fclose(f) != 0 || !ok || std::rename(tmp.c_str(), ctx->tuning_path.c_str()) != 0)
    return fail(NLO_EINVAL, "%s: cannot write %s", fn, ctx->tuning_path.c_str());
  return NLO_OK;
}

std::string fmt_double(double v) {
  char b[64];
  std::snprintf(b, sizeof b, "%.6g", v);
  return b;
}

}  // namespace

extern "C" {

nlo_status nlo_subtracted(nlo_ctx* ctx, int real_proc, int fks_i, int fks_j, int64_t n, int64_t ld,
                          const double* born_mom, const double* xi_tilde, const double* y, const double* phi,
                          const uint8_t* mask, nlo_prec prec, const nlo_fks_out* out, void* hip_stream) {
  const FksSector* sec = nullptr;
  nlo_status st = check_subtracted(ctx, real_proc, fks_i, fks_j, n, ld, born_mom, xi_tilde, y, phi, prec, out, &sec,
                                   "nlo_subtracted");
  if (st) return st;
  if (n == 0) return NLO_OK;
  std::lock_guard<std::mutex> g(ctx->mu);
  st = use_device(ctx, "nlo_subtracted");
  if (st) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  st = check_ws(ctx, fks_ws_bytes(real_proc, n), n, "nlo_subtracted");
  if (st) return st;
  hipError_t err = launch_subtracted(ctx, sec, real_proc, n, ld, born_mom, xi_tilde, y, phi, mask, prec, out,
                                     ctx->ws, s);
  if (err != hipSuccess) return fail(NLO_EDEVICE, "nlo_subtracted: launch failed: %s", hipGetErrorString(err));
  return NLO_OK;
}

nlo_status nlo_subtracted_static(nlo_ctx* ctx, int real_proc, int fks_i, int fks_j, int64_t n, int64_t ld,
                                 const double* born_mom, const double* xi_tilde, const double* y, const double* phi,
                                 const uint8_t* mask, nlo_prec prec, const nlo_fks_out* out, void* hip_stream) {
  const FksSector* sec = nullptr;
  nlo_status st = check_subtracted(ctx, real_proc, fks_i, fks_j, n, ld, born_mom, xi_tilde, y, phi, prec, out, &sec,
                                   "nlo_subtracted_static");
  if (st) return st;
  if (n > SCRATCH_EVENTS)
    return fail(NLO_EINVAL, "nlo_subtracted_static: n = %lld exceeds the static scratch (%lld events)", (long long)n,
                (long long)SCRATCH_EVENTS);
  if (fks_ws_bytes(real_proc, n) > SCRATCH_BYTES)
    return fail(NLO_EINVAL, "nlo_subtracted_static: %zu bytes needed, scratch holds %zu", fks_ws_bytes(real_proc, n),
                SCRATCH_BYTES);
  if (n == 0) return NLO_OK;
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    const int dev = ctx->params.device;
    ws = (dev >= 0 && dev < SCRATCH_MAX_DEVICES) ? g_scratch_ptr[dev] : nullptr;
  }
  if (!ws) return fail(NLO_EDEVICE, "nlo_subtracted_static: no scratch address for device %d", ctx->params.device);
  std::lock_guard<std::mutex> g(ctx->mu);
  st = use_device(ctx, "nlo_subtracted_static");
  if (st) return st;
  hipError_t err = launch_subtracted(ctx, sec, real_proc, n, ld, born_mom, xi_tilde, y, phi, mask, prec, out, ws,
                                     (hipStream_t)hip_stream);
  if (err != hipSuccess) return fail(NLO_EDEVICE, "nlo_subtracted_static: launch failed: %s", hipGetErrorString(err));
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
  if (cfg->colour_mode == 2 && prec != NLO_FP32 && prec != NLO_MIXED)
    return fail(NLO_EUNSUPPORTED, "nlo_set_kernel_config: matrix-core colour contraction is FP32 only");
  if (cfg->schedule < 0 || cfg->schedule > 1) return fail(NLO_EINVAL, "nlo_set_kernel_config: bad schedule");
  if (cfg->schedule == 1 && ME2_LAUNCH[proc_id][VAR_F64_ALT] == ME2_LAUNCH[proc_id][VAR_F64])
    return fail(NLO_EUNSUPPORTED, "nlo_set_kernel_config: %s has one helicity schedule", PROC_STATIC[proc_id].name);
  if (cfg->schedule == 1 && (cfg->colour_mode == 2 || (prec != NLO_FP64 && prec != NLO_FP32 && prec != NLO_MIXED)))
    return fail(NLO_EUNSUPPORTED, "nlo_set_kernel_config: the alternative schedule is for the vector-ALU FP64/FP32 "
                "kernels");
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

}  // extern "C"

namespace {

// nlo_me2 and nlo_me2_checked: validation, then (under the context lock) the
// |M|^2 launch and, with a status array, the status kernels
nlo_status me2_call(nlo_ctx* ctx, int proc_id, int64_t n, int64_t ld, const double* mom, double* me2, uint8_t* status,
                    nlo_prec prec, void* hip_stream, const char* fn) {
  nlo_status st = check_ctx(ctx, proc_id, fn);
  if (st) return st;
  if (n < 0) return fail(NLO_EINVAL, "%s: n = %lld < 0", fn, (long long)n);
  if (ld < n) return fail(NLO_EINVAL, "%s: ld = %lld < n = %lld", fn, (long long)ld, (long long)n);
  if ((int)prec < 0 || (int)prec > NLO_MIXED) return fail(NLO_EINVAL, "%s: bad precision %d", fn, (int)prec);
  if (n == 0) return NLO_OK;
  if (!mom || !me2) return fail(NLO_EINVAL, "%s: NULL device pointer", fn);
  if ((int64_t)((n + 1023) / 64) > (int64_t)0x7fffffff) return fail(NLO_EINVAL, "%s: n too large", fn);
  if (half_prec(prec) && n > 0x7fffffffLL) return fail(NLO_EINVAL, "%s: n too large for FP16/BF16 (event list)", fn);
  std::lock_guard<std::mutex> g(ctx->mu);
  st = use_device(ctx, fn);
  if (st) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  if (half_prec(prec)) {
    st = check_ws(ctx, half_ws_bytes(n), n, fn);
    if (st) return st;
  }
  st = launch_me2(ctx, proc_id, n, ld, mom, me2, prec, s, ctx->ws);
  if (st || !status) return st;
  hipError_t e = launch_me2_status(n, ld, PROC_STATIC[proc_id].npart, mom, me2, status, s);
  if (e == hipSuccess && half_prec(prec)) {
    // the events the half-width pass listed for FP32 (list and counter as
    // launch_me2 lays them out in the workspace)
    const unsigned* list = static_cast<const unsigned*>(ctx->ws);
    const uintptr_t c = reinterpret_cast<uintptr_t>(list + n);
    const unsigned* cnt = reinterpret_cast<const unsigned*>((c + 63) & ~uintptr_t(63));
    e = launch_mark_list(n, cnt, list, 4, status, s);
  }
  if (e != hipSuccess) return fail(NLO_EDEVICE, "%s: launch failed: %s", fn, hipGetErrorString(e));
  return NLO_OK;
}

}  // namespace

extern "C" {

nlo_status nlo_me2(nlo_ctx* ctx, int proc_id, int64_t n, int64_t ld, const double* mom, double* me2, nlo_prec prec,
                   void* hip_stream) {
  return me2_call(ctx, proc_id, n, ld, mom, me2, nullptr, prec, hip_stream, "nlo_me2");
}

nlo_status nlo_me2_checked(nlo_ctx* ctx, int proc_id, int64_t n, int64_t ld, const double* mom, double* me2,
                           uint8_t* status, nlo_prec prec, void* hip_stream) {
  if (n > 0 && !status) return fail(NLO_EINVAL, "nlo_me2_checked: status is NULL");
  return me2_call(ctx, proc_id, n, ld, mom, me2, status, prec, hip_stream, "nlo_me2_checked");
}

nlo_status nlo_reserve(nlo_ctx* ctx, int64_t n) {
  if (!ctx) return fail(NLO_EINVAL, "nlo_reserve: ctx is NULL");
  if (n < 0 || n > 0x7fffffffLL) return fail(NLO_EINVAL, "nlo_reserve: n = %lld out of [0, 2^31)", (long long)n);
  std::lock_guard<std::mutex> g(ctx->mu);
  if (n <= ctx->ws_events) return NLO_OK;
  nlo_status st = use_device(ctx, "nlo_reserve");
  if (st) return st;
  const size_t need = ws_bytes_for(n);
  if (ctx->ws) {
    // work already queued on any stream may still use the old workspace
    if (hipDeviceSynchronize() != hipSuccess) return fail(NLO_EDEVICE, "nlo_reserve: device sync failed");
    (void)hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    ctx->ws_events = 0;
  }
  if (hipMalloc(&ctx->ws, need) != hipSuccess) {
    ctx->ws = nullptr;
    return fail(NLO_ENOMEM, "nlo_reserve: workspace of %zu bytes", need);
  }
  ctx->ws_bytes = need;
  ctx->ws_events = n;
  return NLO_OK;
}

nlo_status nlo_colour_unit(const nlo_ctx* ctx, int proc_id, nlo_prec prec, int* unit) {
  nlo_status st = check_ctx(ctx, proc_id, "nlo_colour_unit");
  if (st) return st;
  if (!unit) return fail(NLO_EINVAL, "nlo_colour_unit: unit is NULL");
  if ((int)prec < 0 || (int)prec > NLO_MIXED) return fail(NLO_EINVAL, "nlo_colour_unit: bad precision %d", (int)prec);
  if (prec != NLO_FP32 && prec != NLO_MIXED) {
    *unit = 1;
    return NLO_OK;
  }
  const int mode = ctx->cfg[proc_id][prec].colour_mode;
  *unit = mode ? mode : auto_colour_mode(proc_id, prec);
  return NLO_OK;
}

nlo_status nlo_autotune(nlo_ctx* ctx, int proc_id, nlo_prec prec, int64_t n, int64_t ld, const double* mom,
                        double* me2, void* hip_stream, nlo_kernel_config* best, double* ns_per_event) {
  nlo_status st = check_ctx(ctx, proc_id, "nlo_autotune");
  if (st) return st;
  if (n <= 0 || ld < n) return fail(NLO_EINVAL, "nlo_autotune: need 0 < n <= ld");
  if (!mom || !me2) return fail(NLO_EINVAL, "nlo_autotune: NULL device pointer");
  if ((int)prec < 0 || (int)prec > NLO_MIXED) return fail(NLO_EINVAL, "nlo_autotune: bad precision %d", (int)prec);
  std::lock_guard<std::mutex> g(ctx->mu);
  st = use_device(ctx, "nlo_autotune");
  if (st) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  if (half_prec(prec)) {
    st = check_ws(ctx, half_ws_bytes(n), n, "nlo_autotune");
    if (st) return st;
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(NLO_EDEVICE, "nlo_autotune: event");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(NLO_EDEVICE, "nlo_autotune: event");
  }
  const nlo_kernel_config saved = ctx->cfg[proc_id][prec];
  nlo_kernel_config win = saved;
  float win_ms = -1.0f;
  nlo_status result = NLO_OK;
  const bool fp32 = prec == NLO_FP32 || prec == NLO_MIXED;
  const bool alt = ME2_LAUNCH[proc_id][VAR_F64_ALT] != ME2_LAUNCH[proc_id][VAR_F64] && !half_prec(prec);
  // (colour unit, schedule) pairs: vector ALU with each schedule, the matrix cores with schedule 0
  int cand[3][2], ncand = 0;
  cand[ncand][0] = 1, cand[ncand][1] = 0, ++ncand;
  if (alt) cand[ncand][0] = 1, cand[ncand][1] = 1, ++ncand;
  if (fp32) cand[ncand][0] = 2, cand[ncand][1] = 0, ++ncand;
  for (int block = 64; block <= NLO_MAX_BLOCK && result == NLO_OK; block += 64) {
    for (int m = 0; m < ncand && result == NLO_OK; ++m) {
      ctx->cfg[proc_id][prec] = nlo_kernel_config{block, cand[m][0], cand[m][1]};
      // one warm-up, then three timed launches
      for (int rep = 0; rep < 4 && result == NLO_OK; ++rep) {
        if (rep == 1 && hipEventRecord(e0, s) != hipSuccess) result = fail(NLO_EDEVICE, "nlo_autotune: record");
        if (result == NLO_OK) result = launch_me2(ctx, proc_id, n, ld, mom, me2, prec, s, ctx->ws);
      }
      if (result != NLO_OK) break;
      float ms = 0.0f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        result = fail(NLO_EDEVICE, "nlo_autotune: timing failed");
        break;
      }
      if (win_ms < 0.0f || ms < win_ms) {
        win_ms = ms;
        win = ctx->cfg[proc_id][prec];
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->cfg[proc_id][prec] = result == NLO_OK ? win : saved;
  if (result != NLO_OK) return result;
  const double ns = (double)win_ms * 1e6 / 3.0 / (double)n;
  if (best) *best = win;
  if (ns_per_event) *ns_per_event = ns;
  TuneEntry e;
  e.put("kind", "me2", true);
  e.put("proc", PROC_STATIC[proc_id].name, true);
  e.put("prec", PREC_NAME[prec], true);
  e.put("block", std::to_string(win.block), false);
  e.put("colour_mode", std::to_string(win.colour_mode), false);
  e.put("schedule", std::to_string(win.schedule), false);
  e.put("ns_per_event", fmt_double(ns), false);
  return merge_tuning(ctx, e, "nlo_autotune");
}

nlo_status nlo_set_fks_config(nlo_ctx* ctx, int real_proc, int fks_i, int fks_j, nlo_prec prec,
                              const nlo_fks_config* cfg) {
  const char* fn = "nlo_set_fks_config";
  nlo_status st = check_ctx(ctx, real_proc, fn);
  if (st) return st;
  if (!cfg) return fail(NLO_EINVAL, "%s: cfg is NULL", fn);
  if (prec != NLO_FP64 && prec != NLO_FP32 && prec != NLO_MIXED)
    return fail(NLO_EUNSUPPORTED, "%s: precision %d not supported (FP64, FP32, MIXED)", fn, (int)prec);
  int k = 0;
  while (k < NFKS && !(FKS_TABLE[k].real == real_proc && FKS_TABLE[k].i == fks_i && FKS_TABLE[k].j == fks_j)) ++k;
  if (k == NFKS) return fail(NLO_EUNSUPPORTED, "%s: no FKS sector (%d, %d) for %s", fn, fks_i, fks_j,
                             PROC_STATIC[real_proc].name);
  if (!valid_block(cfg->real_block) || !valid_block(cfg->ct_block))
    return fail(NLO_EINVAL, "%s: blocks must be multiples of 64 in [64, %d]", fn, NLO_MAX_BLOCK);
  if (cfg->colour_mode < 0 || cfg->colour_mode > 2 || (cfg->colour_mode == 2 && prec == NLO_FP64))
    return fail(NLO_EINVAL, "%s: bad colour_mode %d for this precision", fn, cfg->colour_mode);
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->fks_cfg[k][prec] = *cfg;
  return NLO_OK;
}

nlo_status nlo_get_fks_config(const nlo_ctx* ctx, int real_proc, int fks_i, int fks_j, nlo_prec prec,
                              nlo_fks_config* cfg) {
  const char* fn = "nlo_get_fks_config";
  nlo_status st = check_ctx(ctx, real_proc, fn);
  if (st) return st;
  if (!cfg) return fail(NLO_EINVAL, "%s: cfg is NULL", fn);
  if (prec != NLO_FP64 && prec != NLO_FP32 && prec != NLO_MIXED)
    return fail(NLO_EUNSUPPORTED, "%s: precision %d not supported (FP64, FP32, MIXED)", fn, (int)prec);
  for (int k = 0; k < NFKS; ++k)
    if (FKS_TABLE[k].real == real_proc && FKS_TABLE[k].i == fks_i && FKS_TABLE[k].j == fks_j) {
      *cfg = ctx->fks_cfg[k][prec];
      return NLO_OK;
    }
  return fail(NLO_EUNSUPPORTED, "%s: no FKS sector (%d, %d) for %s", fn, fks_i, fks_j, PROC_STATIC[real_proc].name);
}

nlo_status nlo_autotune_subtracted(nlo_ctx* ctx, int real_proc, int fks_i, int fks_j, int64_t n, int64_t ld,
                                   const double* born_mom, const double* xi_tilde, const double* y,
                                   const double* phi, nlo_prec prec, double* w_scratch, void* hip_stream,
                                   nlo_fks_config* best, double* ns_per_event) {
  const char* fn = "nlo_autotune_subtracted";
  nlo_fks_out out{};
  out.W = w_scratch;
  const FksSector* sec = nullptr;
  nlo_status st = check_subtracted(ctx, real_proc, fks_i, fks_j, n, ld, born_mom, xi_tilde, y, phi, prec, &out, &sec,
                                   fn);
  if (st) return st;
  if (n <= 0) return fail(NLO_EINVAL, "%s: need n > 0", fn);
  std::lock_guard<std::mutex> g(ctx->mu);
  st = use_device(ctx, fn);
  if (st) return st;
  st = check_ws(ctx, fks_ws_bytes(real_proc, n), n, fn);
  if (st) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(NLO_EDEVICE, "%s: event", fn);
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(NLO_EDEVICE, "%s: event", fn);
  }
  nlo_fks_config& cur = ctx->fks_cfg[sec - FKS_TABLE][prec];
  const nlo_fks_config saved = cur;
  nlo_fks_config win = saved;
  float win_ms = -1.0f;
  nlo_status result = NLO_OK;
  // one warm-up and three timed calls of the configuration in cur
  auto time_cur = [&]() {
    float ms = -1.0f;
    for (int rep = 0; rep < 4 && result == NLO_OK; ++rep) {
      if (rep == 1 && hipEventRecord(e0, s) != hipSuccess) result = fail(NLO_EDEVICE, "%s: record", fn);
      if (result == NLO_OK) {
        hipError_t err = launch_subtracted(ctx, sec, real_proc, n, ld, born_mom, xi_tilde, y, phi, nullptr, prec,
                                           &out, ctx->ws, s);
        if (err != hipSuccess) result = fail(NLO_EDEVICE, "%s: launch failed: %s", fn, hipGetErrorString(err));
      }
    }
    if (result == NLO_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      result = fail(NLO_EDEVICE, "%s: timing failed", fn);
    if (result == NLO_OK && (win_ms < 0.0f || ms < win_ms)) {
      win_ms = ms;
      win = cur;
    }
  };
  const bool fp32 = prec != NLO_FP64;
  for (int rb = 64; rb <= NLO_MAX_BLOCK && result == NLO_OK; rb += 64)
    for (int m = 1; m <= (fp32 ? 2 : 1) && result == NLO_OK; ++m) {
      cur = nlo_fks_config{rb, m, saved.ct_block};
      time_cur();
    }
  const nlo_fks_config real_win = win;
  for (int cb = 64; cb <= NLO_MAX_BLOCK && result == NLO_OK; cb += 64) {
    if (cb == real_win.ct_block) continue;
    cur = nlo_fks_config{real_win.real_block, real_win.colour_mode, cb};
    time_cur();
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  cur = result == NLO_OK ? win : saved;
  if (result != NLO_OK) return result;
  const double ns = (double)win_ms * 1e6 / 3.0 / (double)n;
  if (best) *best = win;
  if (ns_per_event) *ns_per_event = ns;
  TuneEntry e;
  e.put("kind", "subtracted", true);
  e.put("proc", PROC_STATIC[real_proc].name, true);
  e.put("i", std::to_string(fks_i), false);
  e.put("j", std::to_string(fks_j), false);
  e.put("prec", PREC_NAME[prec], true);
  e.put("real_block", std::to_string(win.real_block), false);
  e.put("colour_mode", std::to_string(win.colour_mode), false);
  e.put("ct_block", std::to_string(win.ct_block), false);
  e.put("ns_per_event", fmt_double(ns), false);
  return merge_tuning(ctx, e, fn);
}

nlo_status nlo_tuning_cache(nlo_ctx* ctx, const char* path, int* loaded) {
  const char* fn = "nlo_tuning_cache";
  if (!ctx) return fail(NLO_EINVAL, "%s: ctx is NULL", fn);
  if (loaded) *loaded = 0;
  std::lock_guard<std::mutex> g(ctx->mu);
  if (!path || !*path) {
    ctx->tuning_path.clear();
    return NLO_OK;
  }
  std::vector<TuneEntry> es;
  if (!read_tuning(path, es)) return fail(NLO_EINVAL, "%s: %s does not parse as a tuning cache", fn, path);
  const TuneEntry id = tuning_identity(ctx->params.device);
  int n = 0;
  for (const TuneEntry& e : es)
    if (same_fields(e, id, KEY_FIELDS, 5) && apply_entry(ctx, e)) ++n;
  ctx->tuning_path = path;
  if (loaded) *loaded = n;
  return NLO_OK;
}

nlo_status nlo_plan_destroy(nlo_plan* plan) {
  if (!plan) return NLO_OK;
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  for (hipEvent_t e : plan->events) (void)hipEventDestroy(e);
  for (hipStream_t s : plan->streams) (void)hipStreamDestroy(s);
  for (void* w : plan->ws) (void)hipFree(w);
  delete plan;
  return NLO_OK;
}

nlo_status nlo_batch_plan(nlo_ctx* ctx, const nlo_work_item* items, int nitems, int nbranches, nlo_plan** out) {
  if (!out) return fail(NLO_EINVAL, "nlo_batch_plan: out is NULL");
  *out = nullptr;
  if (!ctx) return fail(NLO_EINVAL, "nlo_batch_plan: ctx is NULL");
  if (nitems < 0 || (nitems > 0 && !items)) return fail(NLO_EINVAL, "nlo_batch_plan: bad item list");
  if (nbranches == 0) nbranches = 4;
  if (nbranches < 1 || nbranches > 16) return fail(NLO_EINVAL, "nlo_batch_plan: nbranches must be in [1, 16]");
  // validate every item as the direct calls would
  std::vector<const FksSector*> secs(nitems, nullptr);
  std::vector<double> cost(nitems, 0.0);
  for (int k = 0; k < nitems; ++k) {
    const nlo_work_item& it = items[k];
    nlo_status st;
    if (it.kind == NLO_ITEM_ME2) {
      st = check_ctx(ctx, it.proc_id, "nlo_batch_plan");
      if (st) return st;
      if (it.n < 0 || it.ld < it.n) return fail(NLO_EINVAL, "nlo_batch_plan: item %d: bad n/ld", k);
      if ((int)it.prec < 0 || (int)it.prec > NLO_MIXED)
        return fail(NLO_EINVAL, "nlo_batch_plan: item %d: bad precision %d", k, (int)it.prec);
      if (half_prec(it.prec) && it.n > 0x7fffffffLL)
        return fail(NLO_EINVAL, "nlo_batch_plan: item %d: n too large for FP16/BF16", k);
      if (it.n > 0 && (!it.mom || !it.me2)) return fail(NLO_EINVAL, "nlo_batch_plan: item %d: NULL device pointer", k);
    } else if (it.kind == NLO_ITEM_SUBTRACTED) {
      st = check_subtracted(ctx, it.proc_id, it.fks_i, it.fks_j, it.n, it.ld, it.mom, it.xi_tilde, it.y, it.phi,
                            it.prec, &it.fks_out, &secs[k], "nlo_batch_plan");
      if (st) return st;
    } else {
      return fail(NLO_EINVAL, "nlo_batch_plan: item %d: unknown kind %d", k, (int)it.kind);
    }
    const ProcStatic& P = PROC_STATIC[it.proc_id];
    cost[k] = (double)it.n * P.ngood * (P.nterm + P.ncur) * (it.kind == NLO_ITEM_SUBTRACTED ? 1.3 : 1.0) *
              (it.prec == NLO_FP64 ? 4.0 : (it.prec == NLO_FP16 ? 0.6 : (it.prec == NLO_BF16 ? 1.5 : 1.0)));
  }
  std::lock_guard<std::mutex> g(ctx->mu);
  nlo_status st = use_device(ctx, "nlo_batch_plan");
  if (st) return st;
  nlo_plan* plan = new (std::nothrow) nlo_plan;
  if (!plan) return fail(NLO_ENOMEM, "nlo_batch_plan: out of host memory");
  plan->ctx = ctx;
  auto bail = [&](nlo_status code, const char* what, hipError_t e) {
    nlo_plan_destroy(plan);
    return fail(code, "nlo_batch_plan: %s: %s", what, hipGetErrorString(e));
  };
  hipError_t e = hipSuccess;
  // per-item workspaces of FKS and half-width items (items run concurrently)
  std::vector<void*> item_ws(nitems, nullptr);
  for (int k = 0; k < nitems; ++k) {
    const bool sub = items[k].kind == NLO_ITEM_SUBTRACTED, half = !sub && half_prec(items[k].prec);
    if ((!sub && !half) || items[k].n == 0) continue;
    void* w = nullptr;
    e = hipMalloc(&w, sub ? fks_ws_bytes(items[k].proc_id, items[k].n) : half_ws_bytes(items[k].n));
    if (e != hipSuccess) return bail(NLO_ENOMEM, "workspace", e);
    plan->ws.push_back(w);
    item_ws[k] = w;
  }
  for (int b = 0; b <= nbranches; ++b) {
    hipStream_t s;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(NLO_EDEVICE, "stream", e);
    plan->streams.push_back(s);
  }
  for (int b = 0; b <= nbranches; ++b) {
    hipEvent_t ev;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return bail(NLO_EDEVICE, "event", e);
    plan->events.push_back(ev);
  }
  // largest first onto the least-loaded branch
  std::vector<int> idx(nitems);
  for (int k = 0; k < nitems; ++k) idx[k] = k;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<double> load(nbranches, 0.0);
  hipStream_t origin = plan->streams[0];
  e = hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return bail(NLO_EDEVICE, "begin capture", e);
  hipError_t cap_err = hipEventRecord(plan->events[0], origin);
  for (int b = 1; b <= nbranches && cap_err == hipSuccess; ++b) cap_err = hipStreamWaitEvent(plan->streams[b], plan->events[0], 0);
  for (int q = 0; q < nitems && cap_err == hipSuccess; ++q) {
    const int k = idx[q];
    const nlo_work_item& it = items[k];
    if (it.n == 0) continue;
    int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[b] += cost[k];
    hipStream_t s = plan->streams[1 + b];
    if (it.kind == NLO_ITEM_ME2) {
      nlo_status ls = launch_me2(ctx, it.proc_id, it.n, it.ld, it.mom, it.me2, it.prec, s, item_ws[k]);
      if (ls) cap_err = hipErrorLaunchFailure;
    } else {
      cap_err = launch_subtracted(ctx, secs[k], it.proc_id, it.n, it.ld, it.mom, it.xi_tilde, it.y, it.phi, it.mask,
                                  it.prec, &it.fks_out, item_ws[k], s);
    }
  }
  for (int b = 1; b <= nbranches && cap_err == hipSuccess; ++b) {
    cap_err = hipEventRecord(plan->events[b], plan->streams[b]);
    if (cap_err == hipSuccess) cap_err = hipStreamWaitEvent(origin, plan->events[b], 0);
  }
  e = hipStreamEndCapture(origin, &plan->graph);
  if (cap_err != hipSuccess) return bail(NLO_EDEVICE, "capture", cap_err);
  if (e != hipSuccess) return bail(NLO_EDEVICE, "end capture", e);
  e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return bail(NLO_EDEVICE, "instantiate", e);
  *out = plan;
  return NLO_OK;
}

nlo_status nlo_batch_run(nlo_plan* plan, void* hip_stream) {
  if (!plan || !plan->exec) return fail(NLO_EINVAL, "nlo_batch_run: plan is NULL");
  std::lock_guard<std::mutex> g(plan->ctx->mu);
  nlo_status st = use_device(plan->ctx, "nlo_batch_run");
  if (st) return st;
  hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)hip_stream);
  if (e != hipSuccess) return fail(NLO_EDEVICE, "nlo_batch_run: graph launch failed: %s", hipGetErrorString(e));
  return NLO_OK;
}

nlo_status nlo_uniforms(nlo_ctx* ctx, int64_t n, uint32_t seed, uint32_t stream, uint64_t first, uint32_t slot,
                        double* out, void* hip_stream) {
  if (!ctx) return fail(NLO_EINVAL, "nlo_uniforms: ctx is NULL");
  if (n < 0) return fail(NLO_EINVAL, "nlo_uniforms: n = %lld < 0", (long long)n);
  if (n == 0) return NLO_OK;
  if (!out) return fail(NLO_EINVAL, "nlo_uniforms: NULL device pointer");
  if (n > 0x7fffffffLL * 256) return fail(NLO_EINVAL, "nlo_uniforms: n too large");
  std::lock_guard<std::mutex> g(ctx->mu);
  nlo_status st = use_device(ctx, "nlo_uniforms");
  if (st) return st;
  hipError_t e = launch_uniforms(n, seed, stream, first, slot, out, (hipStream_t)hip_stream);
  if (e != hipSuccess) return fail(NLO_EDEVICE, "nlo_uniforms: launch failed: %s", hipGetErrorString(e));
  return NLO_OK;
}

nlo_status nlo_phase_space(nlo_ctx* ctx, int proc_id, int64_t n, int64_t ld, uint32_t seed, uint32_t stream,
                           uint64_t first, double sqrt_s_lo, double sqrt_s_hi, double* mom, double* weight,
                           void* hip_stream) {
  nlo_status st = check_ctx(ctx, proc_id, "nlo_phase_space");
  if (st) return st;
  const ProcStatic& P = PROC_STATIC[proc_id];
  if (n < 0 || ld < n) return fail(NLO_EINVAL, "nlo_phase_space: need 0 <= n <= ld");
  if (n == 0) return NLO_OK;
  if (!mom) return fail(NLO_EINVAL, "nlo_phase_space: NULL device pointer");
  if (n > 0x7fffffffLL * 256) return fail(NLO_EINVAL, "nlo_phase_space: n too large");
  if (P.nin != 2 || P.npart - 2 < 2 || P.npart - 2 > 4)
    return fail(NLO_EUNSUPPORTED, "nlo_phase_space: process %s has no 2 -> 2..4 generator", P.name);
  double msum = 0.0;
  PsArgs a{};
  a.n = n;
  a.ld = ld;
  a.seed = seed;
  a.stream = stream;
  a.first = first;
  a.rs_lo = sqrt_s_lo;
  a.rs_hi = sqrt_s_hi;
  for (int k = 2; k < P.npart; ++k) {
    a.mass[k - 2] = (P.top_legs >> k) & 1u ? ctx->params.m_top : 0.0;
    msum += a.mass[k - 2];
  }
  if (!(sqrt_s_lo > msum) || !(sqrt_s_hi >= sqrt_s_lo) || !std::isfinite(sqrt_s_hi))
    return fail(NLO_EINVAL, "nlo_phase_space: need %g < sqrt_s_lo <= sqrt_s_hi < inf", msum);
  a.mom = mom;
  a.weight = weight;
  std::lock_guard<std::mutex> g(ctx->mu);
  st = use_device(ctx, "nlo_phase_space");
  if (st) return st;
  hipError_t e = launch_rambo(P.npart - 2, a, (hipStream_t)hip_stream);
  if (e != hipSuccess) return fail(NLO_EDEVICE, "nlo_phase_space: launch failed: %s", hipGetErrorString(e));
  return NLO_OK;
}

nlo_status nlo_fks_variables(nlo_ctx* ctx, int64_t n, uint32_t seed, uint32_t stream, uint64_t first,
                             int initial_state, double* xi_tilde, double* y, double* phi, void* hip_stream) {
  if (!ctx) return fail(NLO_EINVAL, "nlo_fks_variables: ctx is NULL");
  if (n < 0) return fail(NLO_EINVAL, "nlo_fks_variables: n = %lld < 0", (long long)n);
  if (n == 0) return NLO_OK;
  if (!xi_tilde || !y || !phi) return fail(NLO_EINVAL, "nlo_fks_variables: NULL device pointer");
  if (n > 0x7fffffffLL * 256) return fail(NLO_EINVAL, "nlo_fks_variables: n too large");
  std::lock_guard<std::mutex> g(ctx->mu);
  nlo_status st = use_device(ctx, "nlo_fks_variables");
  if (st) return st;
  hipError_t e = launch_fks_variables(n, seed, stream, first, initial_state ? 1 : 0, xi_tilde, y, phi,
                                      (hipStream_t)hip_stream);
  if (e != hipSuccess) return fail(NLO_EDEVICE, "nlo_fks_variables: launch failed: %s", hipGetErrorString(e));
  return NLO_OK;
}

nlo_status nlo_cross_section(nlo_ctx* ctx, int proc_id, int64_t n, uint32_t seed, uint32_t stream, double sqrt_s,
                             nlo_prec prec, double* sigma_pb, double* error_pb, void* hip_stream) {
  nlo_status st = check_ctx(ctx, proc_id, "nlo_cross_section");
  if (st) return st;
  const ProcStatic& P = PROC_STATIC[proc_id];
  if (n < 2 || n > (int64_t)1 << 40) return fail(NLO_EINVAL, "nlo_cross_section: need 2 <= n <= 2^40");
  if ((int)prec < 0 || (int)prec > NLO_MIXED) return fail(NLO_EINVAL, "nlo_cross_section: bad precision");
  if (!sigma_pb) return fail(NLO_EINVAL, "nlo_cross_section: sigma_pb is NULL");
  if (P.nin != 2 || P.npart - 2 < 2 || P.npart - 2 > 4)
    return fail(NLO_EUNSUPPORTED, "nlo_cross_section: process %s has no 2 -> 2..4 generator", P.name);
  PsArgs a{};
  double msum = 0.0;
  for (int k = 2; k < P.npart; ++k) {
    a.mass[k - 2] = (P.top_legs >> k) & 1u ? ctx->params.m_top : 0.0;
    msum += a.mass[k - 2];
  }
  if (!(sqrt_s > msum) || !std::isfinite(sqrt_s))
    return fail(NLO_EINVAL, "nlo_cross_section: need %g < sqrt_s < inf", msum);
  std::lock_guard<std::mutex> g(ctx->mu);
  st = use_device(ctx, "nlo_cross_section");
  if (st) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t chunk = std::min<int64_t>(n, XS_CHUNK);
  // workspace: momenta, weights, |M|^2, partial sums, accumulator, then the
  // half-width fallback list
  const size_t mom_d = (size_t)P.npart * 4 * chunk;
  st = check_ws(ctx, xs_ws_bytes(P.npart, chunk), chunk, "nlo_cross_section");
  if (st) return st;
  double* base = static_cast<double*>(ctx->ws);
  double *mom = base, *w = mom + mom_d, *me2 = w + chunk, *part = me2 + chunk, *acc = part + XS_PART_DOUBLES;
  void* hws = static_cast<void*>(acc + 8);
  // f = w |M|^2 ident / (2 s) in pb (1 GeV^-2 = 0.3893793721e9 pb)
  const double conv = 0.3893793721e9;
  const double scale = P.ident * conv / (2.0 * sqrt_s * sqrt_s);
  a.ld = chunk;
  a.seed = seed;
  a.stream = stream;
  a.rs_lo = sqrt_s;
  a.rs_hi = sqrt_s;
  a.mom = mom;
  a.weight = w;
  for (int64_t off = 0; off < n; off += chunk) {
    const int64_t m = std::min(chunk, n - off);
    a.n = m;
    a.first = (uint64_t)off;
    hipError_t e = launch_rambo(P.npart - 2, a, s);
    if (e != hipSuccess) return fail(NLO_EDEVICE, "nlo_cross_section: generation failed: %s", hipGetErrorString(e));
    st = launch_me2(ctx, proc_id, m, chunk, mom, me2, prec, s, hws);
    if (st) return st;
    e = launch_xs_sums(m, w, me2, scale, part, acc, off == 0, s);
    if (e != hipSuccess) return fail(NLO_EDEVICE, "nlo_cross_section: reduction failed: %s", hipGetErrorString(e));
  }
  double h[2];
  if (hipMemcpyAsync(h, acc, sizeof h, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return fail(NLO_EDEVICE, "nlo_cross_section: result copy failed");
  const double mean = h[0] / (double)n;
  *sigma_pb = mean;
  if (error_pb) *error_pb = std::sqrt(std::max(0.0, h[1] / (double)n - mean * mean) / (double)(n - 1));
  return NLO_OK;
}

nlo_status nlo_integrate_subtracted(nlo_ctx* ctx, int real_proc, double sqrt_s_born, int64_t n, int niter,
                                    int nadapt, uint32_t seed, uint32_t stream, nlo_prec prec, double* sigma_pb,
                                    double* error_pb, double* chi2_dof, double* iterations, void* hip_stream) {
  const char* fn = "nlo_integrate_subtracted";
  nlo_status st = check_ctx(ctx, real_proc, fn);
  if (st) return st;
  const FksSector* secs[8];
  const int ns = fks_sectors(real_proc, secs, 8);
  if (!ns) return fail(NLO_EUNSUPPORTED, "%s: process %s has no FKS sectors", fn, PROC_STATIC[real_proc].name);
  if (n < 2 || n > XS_CHUNK) return fail(NLO_EINVAL, "%s: need 2 <= n <= 2^20 points per iteration", fn);
  if (niter < 1 || niter > INT_MAX_ITER || nadapt < 0 || nadapt >= niter)
    return fail(NLO_EINVAL, "%s: need 0 <= nadapt < niter <= %d", fn, INT_MAX_ITER);
  if (prec != NLO_FP64 && prec != NLO_FP32 && prec != NLO_MIXED)
    return fail(NLO_EUNSUPPORTED, "%s: precision %d not supported (FP64, FP32, MIXED)", fn, (int)prec);
  if (!sigma_pb) return fail(NLO_EINVAL, "%s: sigma_pb is NULL", fn);
  const int born = secs[0]->born;
  const ProcStatic& B = PROC_STATIC[born];
  const int nf = B.npart - 2, D = 4 * nf + 3;
  if (nf < 2 || nf > 3) return fail(NLO_EUNSUPPORTED, "%s: Born %s not supported", fn, B.name);
  VegasArgs va{};
  double msum = 0.0;
  for (int k = 2; k < B.npart; ++k) {
    va.mass[k - 2] = (B.top_legs >> k) & 1u ? ctx->params.m_top : 0.0;
    msum += va.mass[k - 2];
  }
  if (!(sqrt_s_born > msum) || !std::isfinite(sqrt_s_born))
    return fail(NLO_EINVAL, "%s: need %g < sqrt_s_born < inf", fn, msum);
  std::lock_guard<std::mutex> g(ctx->mu);
  st = use_device(ctx, fn);
  if (st) return st;
  st = check_ws(ctx, int_ws_bytes(real_proc, n, niter), n, fn);
  if (st) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  // carve the workspace: the FKS part first (nlo_subtracted's layout), then ours
  char* base = static_cast<char*>(ctx->ws);
  const size_t fks_b = (fks_ws_bytes(real_proc, n) + 255) & ~size_t(255);
  double* dp = reinterpret_cast<double*>(base + fks_b);
  double* mom = dp;            dp += (size_t)n * B.npart * 4;
  double* w = dp;              dp += n;
  double* xit = dp;            dp += n;
  double* yv = dp;             dp += n;
  double* phi = dp;            dp += n;
  double* dsig = dp;           dp += (size_t)n * ns;
  double* wsc = dp;            dp += (size_t)n * ns;
  double* f = dp;              dp += n;
  double* part = dp;           dp += (size_t)(VEGAS_HIST_BLOCKS + VEGAS_HIST_SEG) * D * VEGAS_BINS;
  double* edges = dp;          dp += (size_t)D * (VEGAS_BINS + 1);
  double* xs_part = dp;        dp += XS_PART_DOUBLES;
  double* acc = dp;            dp += 2 * (size_t)niter;
  unsigned* dropped = reinterpret_cast<unsigned*>(dp);
  dp += 8;
  uint8_t* bins = reinterpret_cast<uint8_t*>(dp);
  va.n = n;
  va.seed = seed;
  va.stream = stream;
  va.rs = sqrt_s_born;
  va.edges = edges;
  va.mom = mom;
  va.w = w;
  va.xit = xit;
  va.y = yv;
  va.phi = phi;
  va.bins = bins;
  const double conv = 0.3893793721e9;   // GeV^-2 -> pb
  hipError_t e = launch_vegas_init(D, edges, dropped, s);
  for (int it = 0; it < niter && e == hipSuccess; ++it) {
    va.first = (uint64_t)it * (uint64_t)n;
    e = launch_vegas_points(nf, va, s);
    for (int k = 0; k < ns && e == hipSuccess; ++k) {
      nlo_fks_out o{};
      o.W = wsc + (size_t)k * n;
      o.dsig = dsig + (size_t)k * n;
      e = launch_subtracted(ctx, secs[k], real_proc, n, n, mom, xit, yv, phi, nullptr, prec, &o, ctx->ws, s);
    }
    if (e == hipSuccess)
      e = launch_vegas_update(n, D, ns, dsig, w, conv, f, dropped, bins, part, xs_part, acc + 2 * it,
                              it + 1 < niter, 1.5, edges, s);
  }
  if (e != hipSuccess) return fail(NLO_EDEVICE, "%s: launch failed: %s", fn, hipGetErrorString(e));
  std::vector<double> h(2 * (size_t)niter);
  unsigned nd = 0;
  if (hipMemcpyAsync(h.data(), acc, h.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&nd, dropped, sizeof nd, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(NLO_EDEVICE, "%s: result copy failed", fn);
  // iterations from nadapt on, combined with inverse-variance weights
  double sw = 0.0, swi = 0.0;
  std::vector<double> mean(niter), var(niter);
  for (int it = 0; it < niter; ++it) {
    mean[it] = h[2 * it] / (double)n;
    var[it] = std::max(0.0, h[2 * it + 1] / (double)n - mean[it] * mean[it]) / (double)(n - 1);
    if (iterations) {
      iterations[2 * it] = mean[it];
      iterations[2 * it + 1] = std::sqrt(var[it]);
    }
    if (it >= nadapt && var[it] > 0.0) {
      sw += 1.0 / var[it];
      swi += mean[it] / var[it];
    }
  }
  const double res = sw > 0.0 ? swi / sw : mean[niter - 1];
  double chi = 0.0;
  for (int it = nadapt; it < niter; ++it)
    if (var[it] > 0.0) chi += (mean[it] - res) * (mean[it] - res) / var[it];
  *sigma_pb = res;
  if (error_pb) *error_pb = sw > 0.0 ? 1.0 / std::sqrt(sw) : 0.0;
  if (chi2_dof) *chi2_dof = niter - nadapt > 1 ? chi / (niter - nadapt - 1) : 0.0;
  if (nd) return fail(NLO_EDEVICE, "%s: %u points gave a non-finite integrand", fn, nd);
  return NLO_OK;
}

nlo_status nlo_cut_mask(nlo_ctx* ctx, int proc_id, int64_t n, int64_t ld, const double* mom, const nlo_cuts* cuts,
                        uint8_t* pass, void* hip_stream) {
  const char* fn = "nlo_cut_mask";
  nlo_status st = check_ctx(ctx, proc_id, fn);
  if (st) return st;
  st = check_cuts(cuts, fn);
  if (st) return st;
  if (n < 0 || ld < n) return fail(NLO_EINVAL, "%s: need 0 <= n <= ld", fn);
  if (n == 0) return NLO_OK;
  if (!mom || !pass) return fail(NLO_EINVAL, "%s: NULL device pointer", fn);
  const ProcStatic& P = PROC_STATIC[proc_id];
  std::lock_guard<std::mutex> g(ctx->mu);
  st = use_device(ctx, fn);
  if (st) return st;
  hipError_t e = launch_cut_mask(P.npart - P.nin, n, ld, P.nin, mom, legs_of(proc_id), *cuts, pass,
                                 (hipStream_t)hip_stream);
  if (e != hipSuccess) return fail(NLO_EDEVICE, "%s: launch failed: %s", fn, hipGetErrorString(e));
  return NLO_OK;
}

nlo_status nlo_fks_cut_masks(nlo_ctx* ctx, int real_proc, int fks_i, int fks_j, int64_t n, int64_t ld,
                             const double* born_mom, const double* xi_tilde, const double* y, const double* phi,
                             const nlo_cuts* cuts, uint8_t* mask, void* hip_stream) {
  const char* fn = "nlo_fks_cut_masks";
  nlo_status st = check_ctx(ctx, real_proc, fn);
  if (st) return st;
  st = check_cuts(cuts, fn);
  if (st) return st;
  const FksSector* sec = nullptr;
  for (const FksSector& f : FKS_TABLE)
    if (f.real == real_proc && f.i == fks_i && f.j == fks_j) sec = &f;
  if (!sec) return fail(NLO_EUNSUPPORTED, "%s: no FKS sector (%d, %d) for %s", fn, fks_i, fks_j,
                        PROC_STATIC[real_proc].name);
  if (n < 0 || ld < n) return fail(NLO_EINVAL, "%s: need 0 <= n <= ld", fn);
  if (n == 0) return NLO_OK;
  if (!born_mom || !xi_tilde || !y || !phi || !mask) return fail(NLO_EINVAL, "%s: NULL device pointer", fn);
  std::lock_guard<std::mutex> g(ctx->mu);
  st = use_device(ctx, fn);
  if (st) return st;
  FksCutArgs a{};
  a.n = n;
  a.ld = ld;
  a.born = born_mom;
  a.xit = xi_tilde;
  a.y = y;
  a.phi = phi;
  a.mt = ctx->params.m_top;
  a.cuts = *cuts;
  a.mask = mask;
  hipError_t e = sec->cuts(a, (hipStream_t)hip_stream);
  if (e != hipSuccess) return fail(NLO_EDEVICE, "%s: launch failed: %s", fn, hipGetErrorString(e));
  return NLO_OK;
}

nlo_status nlo_generate_passing(nlo_ctx* ctx, int proc_id, int64_t n, int64_t ld, uint32_t seed, uint32_t stream,
                                uint64_t first, double sqrt_s_lo, double sqrt_s_hi, const nlo_cuts* cuts,
                                double* mom, double* weight, uint64_t* trials, void* hip_stream) {
  const char* fn = "nlo_generate_passing";
  nlo_status st = check_ctx(ctx, proc_id, fn);
  if (st) return st;
  st = check_cuts(cuts, fn);
  if (st) return st;
  if (n < 0 || ld < n || n > 0x7fffffffLL) return fail(NLO_EINVAL, "%s: need 0 <= n <= ld, n < 2^31", fn);
  if (!trials) return fail(NLO_EINVAL, "%s: trials is NULL", fn);
  *trials = 0;
  if (n == 0) return NLO_OK;
  if (!mom) return fail(NLO_EINVAL, "%s: mom is NULL", fn);
  const ProcStatic& P = PROC_STATIC[proc_id];
  const int nf = P.npart - P.nin;
  if (P.nin != 2 || nf < 2 || nf > 4) return fail(NLO_EUNSUPPORTED, "%s: %s not supported", fn, P.name);
  GenArgs a{};
  double msum = 0.0;
  for (int k = 0; k < nf; ++k) {
    a.mass[k] = (P.top_legs >> (k + 2)) & 1u ? ctx->params.m_top : 0.0;
    msum += a.mass[k];
  }
  if (!(sqrt_s_lo > msum) || !(sqrt_s_hi >= sqrt_s_lo) || !std::isfinite(sqrt_s_hi))
    return fail(NLO_EINVAL, "%s: need %g < sqrt_s_lo <= sqrt_s_hi < inf", fn, msum);
  std::lock_guard<std::mutex> g(ctx->mu);
  st = use_device(ctx, fn);
  if (st) return st;
  st = check_ws(ctx, gen_ws_bytes(), 1, fn);
  if (st) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  unsigned* base = static_cast<unsigned*>(ctx->ws);
  a.bcount = base;
  a.boff = base + GEN_CHUNK / 256;
  uintptr_t c = reinterpret_cast<uintptr_t>(a.boff + GEN_CHUNK / 256);
  c = (c + 63) & ~uintptr_t(63);
  a.total = reinterpret_cast<unsigned*>(c);
  a.trials = reinterpret_cast<uint64_t*>(c + 64);
  a.n = n;
  a.ld = ld;
  a.seed = seed;
  a.stream = stream;
  a.first0 = first;
  a.rs_lo = sqrt_s_lo;
  a.rs_hi = sqrt_s_hi;
  a.legs = legs_of(proc_id);
  a.cuts = *cuts;
  a.mom = mom;
  a.weight = weight;
  uint64_t cand = first, dry = 0;
  int64_t have = 0;
  while (have < n) {
    // as many candidates as the acceptance so far suggests, at least 2^16
    int64_t m = GEN_CHUNK;
    if (have > 0) {
      const double acc = (double)have / (double)(cand - first);
      m = std::min<int64_t>(GEN_CHUNK, std::max<int64_t>(65536, (int64_t)(1.2 * (double)(n - have) / acc) + 1));
    } else if (cand == first) {
      m = std::min<int64_t>(GEN_CHUNK, std::max<int64_t>(65536, 2 * n));
    }
    a.m = m;
    a.have = have;
    a.first = cand;
    hipError_t e = launch_generate_chunk(nf, a, s);
    unsigned tot = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&tot, a.total, sizeof tot, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(NLO_EDEVICE, "%s: %s", fn, hipGetErrorString(e));
    have += tot;
    cand += (uint64_t)m;
    dry = tot ? 0 : dry + (uint64_t)m;
    if (dry >= ((uint64_t)1 << 26))
      return fail(NLO_EINVAL, "%s: no candidate passed the cuts in %llu in a row", fn, (unsigned long long)dry);
  }
  hipError_t e = hipMemcpyAsync(trials, a.trials, sizeof *trials, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(NLO_EDEVICE, "%s: %s", fn, hipGetErrorString(e));
  return NLO_OK;
}

nlo_status nlo_virtual_integrated(nlo_ctx* ctx, int born_proc, int64_t n, int64_t ld, const double* mom,
                                  nlo_prec prec, double* born, double* vi, void* hip_stream) {
  const char* fn = "nlo_virtual_integrated";
  nlo_status st = check_ctx(ctx, born_proc, fn);
  if (st) return st;
  if (std::strcmp(PROC_STATIC[born_proc].name, "ee_uu") != 0)
    return fail(NLO_EUNSUPPORTED, "%s: %s: only a Born with two massless coloured partons (ee_uu)", fn,
                PROC_STATIC[born_proc].name);
  if (prec != NLO_FP64 && prec != NLO_FP32 && prec != NLO_MIXED)
    return fail(NLO_EUNSUPPORTED, "%s: precision %d not supported (FP64, FP32, MIXED)", fn, (int)prec);
  if (n < 0 || ld < n) return fail(NLO_EINVAL, "%s: need 0 <= n <= ld", fn);
  if (n == 0) return NLO_OK;
  if (!mom || !born || !vi) return fail(NLO_EINVAL, "%s: NULL device pointer", fn);
  std::lock_guard<std::mutex> g(ctx->mu);
  st = use_device(ctx, fn);
  if (st) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  st = launch_me2(ctx, born_proc, n, ld, mom, born, prec, s);
  if (st) return st;
  const double cf = 4.0 / 3.0;
  const double c = ctx->params.alpha_s * cf / (2.0 * M_PI) * (5.0 - 2.0 * M_PI * M_PI / 3.0);
  hipError_t e = launch_scale(n, born, c, vi, s);
  if (e != hipSuccess) return fail(NLO_EDEVICE, "%s: launch failed: %s", fn, hipGetErrorString(e));
  return NLO_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// buffered FKS evaluation: cut-class queues that fill across calls
// ---------------------------------------------------------------------------
struct nlo_fks_buffer {
  nlo_ctx* ctx = nullptr;
  const FksSector* sec = nullptr;
  int real = 0;
  nlo_prec prec = NLO_FP64;
  int64_t threshold = 0, cap = 0;
  double* w_out = nullptr;
  FksQueue q[2] = {};
  unsigned* cnt = nullptr;
  int64_t host_cnt[2] = {0, 0};
  double* wq = nullptr;     // W of one queue evaluation [cap]
  void* ws = nullptr;       // FKS workspace for cap events
  void* block = nullptr;    // the one device allocation holding all of the above
};

namespace {

// evaluate queue c (its events' own terms only) and add the results to their slots
nlo_status buffer_eval(nlo_fks_buffer* b, int c, hipStream_t s, const char* fn) {
  const int64_t m = b->host_cnt[c];
  if (m == 0) return NLO_OK;
  nlo_fks_out o{};
  o.W = b->wq;
  hipError_t e = launch_subtracted(b->ctx, b->sec, b->real, m, b->cap, b->q[c].born, b->q[c].xit, b->q[c].y,
                                   b->q[c].phi, b->q[c].mask, b->prec, &o, b->ws, s, true);
  if (e == hipSuccess) e = launch_queue_scatter(m, b->q[c].slot, b->wq, b->w_out, s);
  if (e == hipSuccess) e = launch_queue_reset(b->cnt, c, s);
  if (e != hipSuccess) return fail(NLO_EDEVICE, "%s: %s", fn, hipGetErrorString(e));
  b->host_cnt[c] = 0;
  return NLO_OK;
}

}  // namespace

extern "C" {

nlo_status nlo_fks_buffer_create(nlo_ctx* ctx, int real_proc, int fks_i, int fks_j, nlo_prec prec,
                                 int64_t threshold, double* w_out, nlo_fks_buffer** out) {
  const char* fn = "nlo_fks_buffer_create";
  if (!out) return fail(NLO_EINVAL, "%s: out is NULL", fn);
  *out = nullptr;
  nlo_status st = check_ctx(ctx, real_proc, fn);
  if (st) return st;
  const FksSector* sec = nullptr;
  for (const FksSector& f : FKS_TABLE)
    if (f.real == real_proc && f.i == fks_i && f.j == fks_j) sec = &f;
  if (!sec) return fail(NLO_EUNSUPPORTED, "%s: no FKS sector (%d, %d) for %s", fn, fks_i, fks_j,
                        PROC_STATIC[real_proc].name);
  if (prec != NLO_FP64 && prec != NLO_FP32 && prec != NLO_MIXED)
    return fail(NLO_EUNSUPPORTED, "%s: precision %d not supported (FP64, FP32, MIXED)", fn, (int)prec);
  if (threshold < 1 || threshold > ((int64_t)1 << 24)) return fail(NLO_EINVAL, "%s: threshold in [1, 2^24]", fn);
  if (!w_out) return fail(NLO_EINVAL, "%s: w_out is NULL", fn);
  std::lock_guard<std::mutex> g(ctx->mu);
  st = use_device(ctx, fn);
  if (st) return st;
  nlo_fks_buffer* b = new (std::nothrow) nlo_fks_buffer;
  if (!b) return fail(NLO_ENOMEM, "%s: out of host memory", fn);
  b->ctx = ctx;
  b->sec = sec;
  b->real = real_proc;
  b->prec = prec;
  b->threshold = threshold;
  b->cap = 2 * threshold;
  b->w_out = w_out;
  const int nb = PROC_STATIC[sec->born].npart;
  const size_t cap = (size_t)b->cap;
  const size_t per_q = cap * (nb * 4 + 3) * sizeof(double) + cap * sizeof(unsigned) + 4 * cap + 256;
  const size_t ws_b = (fks_ws_bytes(real_proc, b->cap) + 255) & ~size_t(255);
  const size_t total = 2 * per_q + cap * sizeof(double) + 256 + ws_b + 256;
  if (hipMalloc(&b->block, total) != hipSuccess) {
    delete b;
    return fail(NLO_ENOMEM, "%s: device allocation of %zu bytes failed", fn, total);
  }
  char* p = static_cast<char*>(b->block);
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 255) & ~size_t(255);
    return r;
  };
  for (int c = 0; c < 2; ++c) {
    b->q[c].born = reinterpret_cast<double*>(take(cap * nb * 4 * sizeof(double)));
    b->q[c].xit = reinterpret_cast<double*>(take(cap * sizeof(double)));
    b->q[c].y = reinterpret_cast<double*>(take(cap * sizeof(double)));
    b->q[c].phi = reinterpret_cast<double*>(take(cap * sizeof(double)));
    b->q[c].slot = reinterpret_cast<unsigned*>(take(cap * sizeof(unsigned)));
    b->q[c].mask = reinterpret_cast<uint8_t*>(take(4 * cap));
  }
  b->wq = reinterpret_cast<double*>(take(cap * sizeof(double)));
  b->cnt = reinterpret_cast<unsigned*>(take(256));
  b->ws = take(ws_b);
  hipError_t e = launch_queue_reset(b->cnt, 0, nullptr);
  if (e == hipSuccess) e = launch_queue_reset(b->cnt, 1, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    (void)hipFree(b->block);
    delete b;
    return fail(NLO_EDEVICE, "%s: %s", fn, hipGetErrorString(e));
  }
  *out = b;
  return NLO_OK;
}

nlo_status nlo_fks_buffer_push(nlo_fks_buffer* b, int64_t n, int64_t ld, const double* born_mom,
                               const double* xi_tilde, const double* y, const double* phi, const uint8_t* mask,
                               const uint32_t* slot, void* hip_stream) {
  const char* fn = "nlo_fks_buffer_push";
  if (!b) return fail(NLO_EINVAL, "%s: buffer is NULL", fn);
  if (n < 0 || ld < n) return fail(NLO_EINVAL, "%s: need 0 <= n <= ld", fn);
  if (n == 0) return NLO_OK;
  if (!born_mom || !xi_tilde || !y || !phi || !slot) return fail(NLO_EINVAL, "%s: NULL device pointer", fn);
  std::lock_guard<std::mutex> g(b->ctx->mu);
  nlo_status st = use_device(b->ctx, fn);
  if (st) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  const int nb = PROC_STATIC[b->sec->born].npart;
  int64_t off = 0;
  while (off < n) {
    const int64_t room = b->cap - std::max(b->host_cnt[0], b->host_cnt[1]);
    if (room < b->threshold) {        // cannot happen after the evaluations below; kept as a guard
      for (int c = 0; c < 2; ++c)
        if ((st = buffer_eval(b, c, s, fn))) return st;
      continue;
    }
    const int64_t m = std::min(n - off, room);
    // inputs of events off .. off + m - 1: pointers shifted by off, same leading dimension
    hipError_t e = launch_queue_push(m, ld, nb, born_mom + off, xi_tilde + off, y + off, phi + off,
                                     mask ? mask + off : nullptr, slot + off, b->q[0], b->q[1], b->cap, b->cnt, s);
    unsigned h[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(h, b->cnt, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(NLO_EDEVICE, "%s: %s", fn, hipGetErrorString(e));
    b->host_cnt[0] = h[0];
    b->host_cnt[1] = h[1];
    for (int c = 0; c < 2; ++c)
      if (b->host_cnt[c] >= b->threshold && (st = buffer_eval(b, c, s, fn))) return st;
    off += m;
  }
  return NLO_OK;
}

nlo_status nlo_fks_buffer_flush(nlo_fks_buffer* b, void* hip_stream) {
  const char* fn = "nlo_fks_buffer_flush";
  if (!b) return fail(NLO_EINVAL, "%s: buffer is NULL", fn);
  std::lock_guard<std::mutex> g(b->ctx->mu);
  nlo_status st = use_device(b->ctx, fn);
  if (st) return st;
  for (int c = 0; c < 2; ++c)
    if ((st = buffer_eval(b, c, (hipStream_t)hip_stream, fn))) return st;
  return NLO_OK;
}

nlo_status nlo_fks_buffer_destroy(nlo_fks_buffer* b) {
  if (!b) return NLO_OK;
  if (b->block) (void)hipFree(b->block);
  delete b;
  return NLO_OK;
}

}  // extern "C"

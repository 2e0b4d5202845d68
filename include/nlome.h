/* nlome.h -- C ABI of the event-parallel tree-level matrix-element library
 * for AMD MI355X (gfx950).
 *
 * The library evaluates, for large batches of phase-space points, the
 * quantities the paper's branch-free NLO event loop (its second algorithm)
 * needs at every point: tree-level squared matrix elements of Born and
 * real-emission processes (helicity- and colour-summed |M|^2, the paper's
 * Born and real equations) and, for real emissions, the FKS-subtracted
 * real-minus-counterterm weight.  One event is one GPU lane.
 *
 * Conventions shared by every entry point
 *  - All functions return nlo_status; none throws, aborts or exits.  On a
 *    non-zero status nlo_last_error() describes the failure.
 *  - Pointers named "device" are HIP device pointers owned by the caller
 *    (e.g. torch.Tensor.data_ptr()); the library never frees them.
 *  - Momenta are float64, GeV, structure of arrays:
 *        mom[(ip * 4 + mu) * ld + e],   ip = particle, mu = 0:E 1:px 2:py 3:pz,
 *    e = event in [0, n), ld >= n the leading dimension.  Incoming particles
 *    come first, in the order of the process name, in their centre-of-mass
 *    frame; then the outgoing particles in the order of the name.
 *  - Evaluation calls are asynchronous on the given HIP stream (NULL = the
 *    default stream); host-detectable argument errors return before any
 *    launch.  n == 0 is a valid no-op.
 *  - One context may be used from several threads; calls are serialised
 *    internally.  Distinct contexts are independent.
 *  - Device memory is allocated only by nlo_reserve (the context workspace),
 *    nlo_batch_plan (its own workspaces) and nlo_create (nothing beyond HIP's
 *    context).  Evaluation calls never allocate or synchronise the device; one
 *    that needs more workspace than reserved returns NLO_EINVAL.  Calls that
 *    overlap on different streams with the same context share its workspace
 *    and race on it: order them on one stream, or use one context per stream.
 */
#ifndef NLOME_H
#define NLOME_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NLO_ABI_VERSION 2u

typedef struct nlo_ctx nlo_ctx;   /* opaque, library-owned */

typedef enum {
  NLO_OK = 0,
  NLO_EINVAL = 1,        /* bad argument (null pointer, n < 0, ld < n, ...) */
  NLO_EPROC = 2,         /* unknown process id */
  NLO_EDEVICE = 3,       /* HIP runtime error */
  NLO_ENOMEM = 4,        /* device allocation failed */
  NLO_EUNSUPPORTED = 5   /* valid but unsupported combination */
} nlo_status;

/* Arithmetic of the amplitude evaluation.  Inputs and outputs are always
 * float64.  NLO_FP64: everything in double.  NLO_FP32: spinors, currents,
 * vertices and the colour contraction in float; helicity-independent
 * quantities (internal momenta, propagator denominators, external-state
 * set-up) and the per-event helicity sum in double.  NLO_MIXED for |M|^2 is
 * NLO_FP32; for subtracted weights it routes events near soft/collinear
 * limits to FP64.  In both, the colour contraction runs on the vector ALU
 * unless nlo_set_kernel_config selects the matrix cores (measured slower at 6
 * and at 24 colour flows; nlo_colour_unit reports the unit in use).
 * NLO_FP16 / NLO_BF16 (nlo_me2 and ME2 batch items only): amplitudes in
 * half-width floats on packed pairs of events, with momenta and masses
 * divided by sqrt(s_hat) of the event first (|M|^2 of N particles is
 * s_hat^(4-N) times that of the scaled momenta, applied in double); FP64
 * prologue, colour contraction in float, helicity sum in double.  The
 * external wavefunctions of each event are also scaled by a power of two set
 * by its largest propagator denominator, which keeps the intermediate values
 * inside the FP16 range.  Events whose largest denominator exceeds 2^14/s_hat
 * (close to a soft or collinear pole, where the diagrams cancel beyond what
 * a half-width significand resolves) are listed and evaluated again in FP32
 * by a second launch; this uses the context workspace (nlo_reserve).  BF16 has no native
 * arithmetic on this GPU: every operation rounds through FP32.
 * These are accuracy studies, not production precisions. */
typedef enum { NLO_FP64 = 0, NLO_FP32 = 1, NLO_FP16 = 2, NLO_BF16 = 3, NLO_MIXED = 4 } nlo_prec;

/* Physics parameters: fixed couplings (no running), top mass, zero widths,
 * all other masses zero; device = HIP device ordinal. */
typedef struct {
  double alpha;      /* e^2/(4 pi), e.g. 1/132.507 */
  double alpha_s;    /* g_s^2/(4 pi), e.g. 0.118 */
  double m_top;      /* GeV, e.g. 173 */
  int device;
} nlo_params;

typedef struct {
  const char* name;      /* e.g. "gg_ttg"; static storage */
  int npart, ninitial;
  int ncolour;           /* colour flows */
  int nhel, ngood_hel;   /* helicity combinations, structurally non-zero ones */
  int ndiagrams;         /* Feynman diagrams */
  int nterms;            /* amplitude terms (a four-gluon diagram gives three) */
  int ncurrents;         /* off-shell currents evaluated per helicity */
  double avg_factor;     /* initial spin x colour average, applied by nlo_me2 */
  double ident_factor;   /* identical final-state factor, NOT applied */
  int gs_pow, e_pow;     /* |M|^2 is proportional to g_s^(2 gs_pow) e^(2 e_pow) */
  int nschedules;        /* helicity schedules of the FP64/FP32 kernels (1 or 2) */
} nlo_proc_info;

/* Kernel launch configuration of one (process, precision) pair. */
typedef struct {
  int block;        /* threads per block: 64, 128, 192 or 256 */
  int colour_mode;  /* 0 = automatic, 1 = vector ALU, 2 = matrix cores (FP32 family only) */
  int schedule;     /* helicity schedule of the vector-ALU FP64/FP32 kernels: 0 = the
                       generator's choice for the precision, 1 = the alternative lazy
                       depth (sub-currents evaluated once per helicity of their own
                       legs where the default evaluates some of them inside the
                       deepest loop, else one level of them inside it: fewer flops or
                       fewer live registers), where the process has one
                       (nlo_process_info: nschedules = 2) */
} nlo_kernel_config;

/* Launch configuration of one FKS sector's subtracted evaluation in one
 * precision: the real-emission |M|^2 kernels (real_block threads per block,
 * colour unit as in nlo_kernel_config) and the map and counterterm kernels
 * (ct_block threads per block).  Defaults {256, 0, 256}. */
typedef struct {
  int real_block;   /* 64, 128, 192 or 256 */
  int colour_mode;  /* 0 = automatic, 1 = vector ALU, 2 = matrix cores (FP32/MIXED only) */
  int ct_block;     /* 64, 128, 192 or 256 */
} nlo_fks_config;

uint32_t nlo_abi_version(void);

/* Create a context on params->device; *out receives it.  Allocates nothing on
 * the device beyond HIP's own context. */
nlo_status nlo_create(nlo_ctx** out, const nlo_params* params);

/* Destroy a context (NULL is a no-op).  Waits for nothing: the caller must
 * have synchronised the streams it used. */
nlo_status nlo_destroy(nlo_ctx* ctx);

/* Thread-local description of the last failure on this thread; valid until
 * the next call from the same thread.  Never NULL. */
const char* nlo_last_error(void);

/* Number of processes; ids are 0 .. n-1:
 *   0 ee_mumu  e+e- -> mu+mu- (photon)     5 gg_ttg   g g -> t tbar g
 *   1 ee_uu    e+e- -> u ubar (photon)     6 uu_ttg   u ubar -> t tbar g
 *   2 ee_uug   e+e- -> u ubar g (photon)   7 ug_ttu   u g -> t tbar u
 *   3 gg_tt    g g -> t tbar               8 gg_ttgg  g g -> t tbar g g
 *   4 uu_tt    u ubar -> t tbar                                          */
int nlo_num_processes(void);

/* Static description of process proc_id. */
nlo_status nlo_process_info(const nlo_ctx* ctx, int proc_id, nlo_proc_info* out);

/* Override the launch configuration used for (proc_id, prec). */
nlo_status nlo_set_kernel_config(nlo_ctx* ctx, int proc_id, nlo_prec prec, const nlo_kernel_config* cfg);
nlo_status nlo_get_kernel_config(const nlo_ctx* ctx, int proc_id, nlo_prec prec, nlo_kernel_config* cfg);

/* The colour-contraction unit an evaluation of (proc_id, prec) uses with the
 * context's configuration: *unit = 1 vector ALU, 2 matrix cores (FP32 and
 * MIXED only; FP64, FP16 and BF16 always report 1). */
nlo_status nlo_colour_unit(const nlo_ctx* ctx, int proc_id, nlo_prec prec, int* unit);

/* Size the context workspace for evaluation calls of up to n events (any
 * process, FKS sector or precision; a cross section needs min(n, 2^20)).  The
 * only evaluation-side allocation: it waits for the device to be idle before
 * freeing a smaller workspace, so call it outside stream capture and before
 * the evaluation calls it serves.  A smaller n than already reserved is a
 * no-op.  n in [0, 2^31). */
nlo_status nlo_reserve(nlo_ctx* ctx, int64_t n);

/* Autotuner: times every launch configuration of (proc_id, prec) -- block of
 * 64/128/192/256 threads (FP16/BF16 blocks cover two events per thread),
 * for FP64/FP32/MIXED both helicity schedules where the process has two, and
 * for FP32/MIXED the colour contraction on the vector ALU or the matrix cores
 * (the matrix-core kernel with schedule 0) -- on the caller's sample batch (device
 * momenta, n events, scratch output me2 of n doubles) with HIP events on the
 * given stream, keeps the fastest for this context and returns it in *best
 * (may be NULL) and its time per event in *ns_per_event (may be NULL).
 * Synchronises the stream; allocates nothing (FP16/BF16 use the context
 * workspace, which must hold n events: nlo_reserve).  With a tuning cache set
 * (nlo_tuning_cache), the result is merged into it. */
nlo_status nlo_autotune(nlo_ctx* ctx, int proc_id, nlo_prec prec, int64_t n, int64_t ld, const double* mom,
                        double* me2, void* hip_stream, nlo_kernel_config* best, double* ns_per_event);

/* Per-sector launch configuration of nlo_subtracted (sector as there). */
nlo_status nlo_set_fks_config(nlo_ctx* ctx, int real_proc, int fks_i, int fks_j, nlo_prec prec,
                              const nlo_fks_config* cfg);
nlo_status nlo_get_fks_config(const nlo_ctx* ctx, int real_proc, int fks_i, int fks_j, nlo_prec prec,
                              nlo_fks_config* cfg);

/* Autotuner for one FKS sector's subtracted evaluation (the launch
 * configuration of the paper's per-sector event loop, section "A data
 * parallel algorithm"): times, with HIP events on the given stream, the real
 * |M|^2 block size x colour unit (FP32/MIXED: vector ALU or matrix cores)
 * with the default counterterm block, then the counterterm block with the
 * winner, each by one warm-up and three timed nlo_subtracted calls on the
 * caller's sample (Born momenta, radiation variables as nlo_subtracted; W
 * scratch output of n doubles); keeps the fastest for this context, returns it
 * in *best and its time per event in *ns_per_event (either may be NULL).
 * Uses the context workspace (nlo_reserve(ctx, n)); synchronises the stream.
 * With a tuning cache set (nlo_tuning_cache), the result is merged into it. */
nlo_status nlo_autotune_subtracted(nlo_ctx* ctx, int real_proc, int fks_i, int fks_j, int64_t n, int64_t ld,
                                   const double* born_mom, const double* xi_tilde, const double* y,
                                   const double* phi, nlo_prec prec, double* w_scratch, void* hip_stream,
                                   nlo_fks_config* best, double* ns_per_event);

/* Tuning cache: a JSON file of autotune results, each entry keyed by the
 * device architecture (gcnArchName), its compute-unit count, the HIP runtime
 * and driver versions and the library build (a hash of its sources).  This
 * call reads path (a missing file is an empty cache), applies to the context
 * every entry whose key matches the current device and build (*loaded, may be
 * NULL, receives their number; entries of other keys are kept but ignored),
 * and remembers path: every later nlo_autotune / nlo_autotune_subtracted on
 * this context merges its result into the file (replacing the entry of the
 * same key, process, sector and precision; written to a temporary file and
 * renamed).  path NULL or "" stops the merging.  Host I/O only; a malformed
 * file returns NLO_EINVAL and changes nothing. */
nlo_status nlo_tuning_cache(nlo_ctx* ctx, const char* path, int* loaded);

/* Squared matrix elements (the paper's Born and real equations):
 *   me2[e] = avg_factor * sum_{helicities} sum_{colours} |M(mom_e)|^2
 * for e in [0, n).  mom: device, layout above, npart particles.  me2: device
 * float64 [n].  prec: any nlo_prec.  Per-event values are written only;
 * nothing is accumulated.  An event whose momenta put an internal propagator
 * exactly on shell has no finite |M|^2; its output is then unspecified (the
 * kernels are compiled without IEEE NaN/infinity guarantees, so it need not
 * be inf or NaN). */
nlo_status nlo_me2(nlo_ctx* ctx, int proc_id, int64_t n, int64_t ld, const double* mom, double* me2,
                   nlo_prec prec, void* hip_stream);

/* nlo_me2 followed by a per-event status (the paper's event loop keeps
 * every point on the device; the status says which results to trust):
 *   status: device uint8 [n], written: bit0 me2[e] is not a finite
 *   non-negative number, bit1 a momentum component of event e is not finite,
 *   bit2 (FP16/BF16) the event was evaluated again in FP32 near a pole.
 * The tests read exponent bits, so they hold whatever the arithmetic rules
 * of the |M|^2 kernels.  One extra launch reading the momenta and |M|^2. */
nlo_status nlo_me2_checked(nlo_ctx* ctx, int proc_id, int64_t n, int64_t ld, const double* mom, double* me2,
                           uint8_t* status, nlo_prec prec, void* hip_stream);

/* Outputs of nlo_subtracted: device arrays owned by the caller.  W is
 * required; every other pointer may be NULL (not written). */
typedef struct {
  double* W;          /* [n] subtracted weight (g_R - g_S - g_C + g_SC)/(xi (1-y)), or the
                         two-sided initial-state form */
  double* xi;         /* [n] xi = xi_tilde * xi_max */
  double* born;       /* [n] Born |M|^2 at the Born point (with its average factor) */
  double *g_R, *g_S;  /* [n] real and soft terms */
  double *g_C, *g_Cm; /* [n] collinear terms, y -> +1 and (initial state only) y -> -1 */
  double *g_SC, *g_SCm; /* [n] soft-collinear terms */
  uint8_t* status;    /* [n] bit0 non-finite W, bit1 evaluated in FP64, bit2 a mask zeroed a term,
                          bit3 W not resolved to 1e-3 in its working precision (its rounding
                          bound, 1e-12 D in FP64 and 32 eps_32 (1 + 1/sqrt(1-|y|)) D in FP32
                          with D = sum|g_X| / kappa, exceeds 1e-3 |W|), bit4 (MIXED) evaluated
                          in FP32 first and again in FP64 because W came out unresolved or
                          non-finite (bit1 is then set too) */
  double* real_mom;   /* [npart_real][4][ld] real-emission momenta in event order */
  double* w_sum;      /* [1] fixed-order FP64 sum of W over the batch */
  /* [n] the subtracted cross section per unit Born phase space and per unit
   * xi_tilde, y, phi, in GeV^-2 (the integrand of nlo_integrate_subtracted):
   *   dsig = xi_max / (2 s_B) [j g_R - j(0,y) g_S - j(xi,1) g_C + j(0,1) g_SC] / (xi (1-y))
   * (initial state: both collinear ends as in W), where the map's phase-space
   * factor j enters every term at its own kinematics.  Final-state emitter:
   *   dPhi_{n+1} = dPhi_n xi j dxi dy dphi,  j = s E_j / (64 pi^3 Ebar_j (1 - xi (1-y)/2)),
   * j(0,y) = s/(64 pi^3), j(xi,1) = z s/(64 pi^3).  Beams: at fixed real energy
   * dPhi_{n+1}(s_R) = s_R xi/(64 pi^3) dxi dy dphi dPhi_n(s_R (1-xi)); with the
   * real flux 1/(2 s_R) and incoming momentum fractions x_1 x_2 = xbar_1 xbar_2/(1-xi)
   * at fixed Born kinematics, j = s_B/(64 pi^3 (1-xi)), j(0,y) = s_B/(64 pi^3). */
  double* dsig;
  double* jac;        /* [n] xi_max j: dPhi_{n+1} = dPhi_n xi jac dxi_tilde dy dphi (beams: as above) */
} nlo_fks_out;

/* FKS-subtracted real emission for one FKS sector (the paper's FKS
 * subtraction; its branch-free loop evaluates Born, real, soft and collinear
 * terms at every point, then zeroes those whose cuts fail).
 *   real_proc: ee_uug (pairs (4,2), (4,3)), gg_ttg (4,-1), uu_ttg (4,-1),
 *              ug_ttu (4,-1), gg_ttgg ((4,5), (5,4), (4,-1), (5,-1));
 *              fks_j = -1: both beams.  In ug_ttu the FKS parton is the final
 *              quark: g_S = g_SC = 0, g_C uses the g g -> t tbar Born (beam 1
 *              quark turned gluon) and g_Cm the u ubar -> t tbar Born (beam 2
 *              gluon turned antiquark); born_mom are then the common t tbar
 *              kinematics and `born` reports the g g -> t tbar Born.
 *   born_mom:  device, Born momenta (the real process without particle
 *              fks_i), layout above, in the Born centre-of-mass frame.
 *   xi_tilde, y, phi: device [n] radiation variables: xi = xi_tilde * xi_max
 *              is the energy fraction 2 k_i^0/sqrt(s_R) of parton fks_i, y the
 *              cosine of its angle to parton fks_j (to beam 1 if fks_j = -1),
 *              phi its azimuth about that axis.
 *   mask:      device [4][ld] bytes for B, R, S, C (non-zero = passes its cuts)
 *              or NULL (all pass).  A failed cut zeroes its term after
 *              evaluation; the soft-collinear terms need both S and C.  A C
 *              byte with bit 1 set gives the beams' two collinear ends
 *              separately: bit 2 the y = +1 end (g_C, g_SC), bit 3 the
 *              y = -1 end (g_Cm, g_SCm) (nlo_fks_cut_masks writes these).
 *   prec:      NLO_FP64, NLO_FP32 (real amplitudes in float, kinematics and
 *              assembly in double) or NLO_MIXED (float unless the event is
 *              near a singular limit, see nlo_set_fks_threshold).
 * The Born point is on shell and conserves momentum by definition: the
 * final-state three-momenta are shifted by a common amount to sum to zero,
 * their energies put on the mass shell, and the beams (along +-z) carry half
 * the total energy each; the FKS pair's invariant (2 k_i.k_j, or 2 p_a.k_i
 * for the beams) enters the real |M|^2 from the radiation variables.  W is a
 * difference of terms growing like 1/kappa (kappa = xi (1-y), or
 * xi (1-y^2) for the beams): in FP64 its error stays within 1e-12 of
 * D = sum|g_X| / kappa (measured against a binary128 evaluation).
 * Uses the context workspace, which must hold n events (nlo_reserve). */
/* How nlo_subtracted treats the cut masks (a context setting; batch plans
 * take the one in force when they are made).
 *   0 (default): branch-free, as in the paper's Algorithm 2 -- every term is
 *      evaluated at every point and failed cuts zero it afterwards;
 *   1: compact -- events whose R cut fails are set aside by the map kernel
 *      and skip the real |M|^2 evaluation, and events none of whose B, S and
 *      C cuts passes skip the Born amplitudes (the paper's "smarter" variant
 *      that evaluates only points passing a cut).  Results are bit for bit
 *      those of mode 0. */
nlo_status nlo_set_fks_mask_mode(nlo_ctx* ctx, int mode);

nlo_status nlo_subtracted(nlo_ctx* ctx, int real_proc, int fks_i, int fks_j, int64_t n, int64_t ld,
                          const double* born_mom, const double* xi_tilde, const double* y, const double* phi,
                          const uint8_t* mask, nlo_prec prec, const nlo_fks_out* out, void* hip_stream);

/* nlo_subtracted without any allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results, with the workspace in
 * a static device array (about 14.7 MB per GPU, held until the process ends)
 * instead of the context workspace.  n <= 65536 events of any sector, else
 * NLO_EINVAL with no launch.  Every call on one GPU shares that GPU's array
 * (the kernels clear the counters they need): calls that overlap on one GPU,
 * from any context or stream, race on it. */
nlo_status nlo_subtracted_static(nlo_ctx* ctx, int real_proc, int fks_i, int fks_j, int64_t n, int64_t ld,
                                 const double* born_mom, const double* xi_tilde, const double* y, const double* phi,
                                 const uint8_t* mask, nlo_prec prec, const nlo_fks_out* out, void* hip_stream);

/* Routing threshold of NLO_MIXED subtracted weights: an event is evaluated in
 * FP64 when kappa = xi (1-y) (final-state fks_j) or xi (1-y^2) (beams) is below
 * it, in FP32 otherwise.  Default 0.1: the FP32 rounding of the real |M|^2
 * reaches W amplified by about 1/kappa, and at kappa >= 0.1 FP32 keeps
 * |dW|/|W| below 1e-4 on every event measured.  An FP32 event whose W comes
 * out unresolved or non-finite (status bits 3, 0) is evaluated again in FP64
 * within the same call (status bit 4), so MIXED flags bit 3 on the events FP64
 * flags.  threshold in [0, 1]. */
nlo_status nlo_set_fks_threshold(nlo_ctx* ctx, double threshold);

/* ---- batched mixes: one graph launch for many (process, contribution) items ----
 * The paper notes that Born amplitudes are evaluated at several kinematics per
 * NLO event and that parallelism should run over FKS sectors; a batch gathers
 * the Born, real and subtracted evaluations of several subprocesses with
 * uneven event counts.  nlo_batch_plan validates the items, allocates the
 * FKS workspaces, and captures every item's launch sequence into one HIP
 * graph whose independent items run concurrently (items are spread over
 * forked capture streams, largest first).  nlo_batch_run is a single
 * hipGraphLaunch on the caller's stream.  Items keep pointing at the caller's
 * device arrays: refill them between runs, do not free them while the plan
 * lives. */
typedef enum { NLO_ITEM_ME2 = 0, NLO_ITEM_SUBTRACTED = 1 } nlo_item_kind;

typedef struct {
  nlo_item_kind kind;
  int proc_id;                       /* process (ME2) or real process (SUBTRACTED) */
  int fks_i, fks_j;                  /* SUBTRACTED only */
  int64_t n, ld;
  const double* mom;                 /* ME2: momenta; SUBTRACTED: Born momenta (device) */
  const double *xi_tilde, *y, *phi;  /* SUBTRACTED only (device [n]) */
  const uint8_t* mask;               /* SUBTRACTED only, or NULL */
  nlo_prec prec;
  double* me2;                       /* ME2 output (device [n]) */
  nlo_fks_out fks_out;               /* SUBTRACTED outputs (device arrays) */
} nlo_work_item;

typedef struct nlo_plan nlo_plan;   /* opaque, library-owned (holds the graph) */

/* Build a plan; nbranches = concurrent branches (1..16, 0 = 4). */
nlo_status nlo_batch_plan(nlo_ctx* ctx, const nlo_work_item* items, int nitems, int nbranches, nlo_plan** out);
nlo_status nlo_batch_run(nlo_plan* plan, void* hip_stream);
nlo_status nlo_plan_destroy(nlo_plan* plan);

/* ---- on-device phase-space generation: the point-sampling step that opens
 * each iteration of the paper's event loop (Algorithm 2), batched ----
 * Every draw is a pure function of (seed, stream, event index, slot): the
 * counter-based Philox4x32-10 generator with key (seed, stream) and counter
 * (event low word, event high word, slot, 0); its four words give two doubles
 * (53 random bits each, plus half a unit of the last place, so in (0, 1)).
 * Event indices are first, first + 1, ...: any sub-range of a batch can be
 * regenerated on its own, whatever the launch shape. */

/* out: device float64 [n][2], the two uniforms of (event first + i, slot). */
nlo_status nlo_uniforms(nlo_ctx* ctx, int64_t n, uint32_t seed, uint32_t stream, uint64_t first, uint32_t slot,
                        double* out, void* hip_stream);

/* RAMBO phase-space points for process proc_id (2 -> 2, 3 or 4), in the
 * partonic centre-of-mass frame with the beams along +z and -z:
 *   sqrt(s_hat) = sqrt_s_lo + (sqrt_s_hi - sqrt_s_lo) u (slot 64; equal
 *   bounds give a fixed energy); final-state particle k from slots 2k, 2k+1;
 *   top quarks at the context's m_top, everything else massless.
 * mom: device, layout above ([npart][4][ld]); weight: device [n] RAMBO weight
 * (the phase-space volume factor, (2 pi)^(4-3n) included) or NULL.
 * Requires sqrt_s_lo > the sum of the final-state masses. */
nlo_status nlo_phase_space(nlo_ctx* ctx, int proc_id, int64_t n, int64_t ld, uint32_t seed, uint32_t stream,
                           uint64_t first, double sqrt_s_lo, double sqrt_s_hi, double* mom, double* weight,
                           void* hip_stream);

/* FKS radiation variables of nlo_subtracted: xi_tilde and 1 - |y|
 * log-uniform in [1e-6, 1] (slot 65), phi uniform in [0, 2 pi) and, if
 * initial_state, a random sign of y (slot 66).  Outputs: device [n] each. */
nlo_status nlo_fks_variables(nlo_ctx* ctx, int64_t n, uint32_t seed, uint32_t stream, uint64_t first,
                             int initial_state, double* xi_tilde, double* y, double* phi, void* hip_stream);

/* Buffered FKS evaluation: the paper's "smarter" alternative to branch-free
 * masking (end of section "A data parallel algorithm") -- points are stored
 * per cut class and evaluated once enough of them pass, across calls.  Two
 * class queues per buffer: the real emission (events whose R cut passes) and
 * the counterterms (events whose S cut or either collinear cut passes).  A
 * queue is evaluated (its own terms only: the real |M|^2 without Born
 * amplitudes, or the Born-level counterterms without the real |M|^2) when it
 * holds at least `threshold` events, and by nlo_fks_buffer_flush; each
 * evaluation adds its contribution to W to w_out[slot] (device float64,
 * caller-owned, zeroed by the caller; one slot per event), so that after the
 * flush w_out[slot] = W of nlo_subtracted with the same masks (up to the
 * rounding of the two-part sum, within 1e-12 of D in FP64; in MIXED a queue
 * sees the real and counterterm parts apart, not their cancellation, so the
 * events that nlo_subtracted evaluates again in FP64 keep FP32 parts here,
 * within the FP32 rounding bound).  Each slot
 * receives at most one contribution per queue, added in stream order, so the
 * result does not depend on how events were pushed.  create allocates the
 * queues and their own FKS workspace (2 threshold events); push and flush
 * allocate nothing and synchronise the stream once per pushed piece (to read
 * the queue sizes).  One buffer serves one stream at a time. */
typedef struct nlo_fks_buffer nlo_fks_buffer;
nlo_status nlo_fks_buffer_create(nlo_ctx* ctx, int real_proc, int fks_i, int fks_j, nlo_prec prec,
                                 int64_t threshold, double* w_out, nlo_fks_buffer** out);
/* born_mom, xi_tilde, y, phi, mask: as nlo_subtracted (mask may be NULL: all
 * pass); slot: device uint32 [n], the w_out index of each event */
nlo_status nlo_fks_buffer_push(nlo_fks_buffer* buf, int64_t n, int64_t ld, const double* born_mom,
                               const double* xi_tilde, const double* y, const double* phi, const uint8_t* mask,
                               const uint32_t* slot, void* hip_stream);
nlo_status nlo_fks_buffer_flush(nlo_fks_buffer* buf, void* hip_stream);
nlo_status nlo_fks_buffer_destroy(nlo_fks_buffer* buf);

/* Born and the finite part of virtual + integrated counterterms, per event
 * (the paper's NLO section: the virtual correction and the FKS counterterms
 * added back, integrated in d = 4 - 2 eps dimensions, where their poles
 * cancel).  For a Born with exactly two massless coloured partons (e+e- ->
 * u ubar, the Born of the sectors (4,2) and (4,3) of e+e- -> u ubar g) every
 * piece is proportional to the Born: with the subtraction of nlo_subtracted
 * (always subtract, xi_c = 1, delta = 2, these sector functions) the
 * counterterms integrate to (alpha_s C_F / 2 pi) c_Gamma (4 pi mu^2 / s)^eps
 * [2/eps^2 + 3/eps + 13 - 5 pi^2 / 3] B and the one-loop quark form factor to
 * [-2/eps^2 - 3/eps - 8 + pi^2] B, so
 *   vi[e] = B (alpha_s C_F / 2 pi) (5 - 2 pi^2 / 3),   B = born[e] (as nlo_me2),
 * independent of the renormalisation scale.  With the subtracted real
 * emission integrated (nlo_integrate_subtracted) the total is
 * sigma_B (1 + alpha_s / pi).  prec: FP64, FP32 or MIXED (of the Born).
 * Other Borns: NLO_EUNSUPPORTED (their integrated soft counterterms need
 * colour-linked Borns with massive eikonal integrals, and beam collinear
 * remnants need parton densities). */
nlo_status nlo_virtual_integrated(nlo_ctx* ctx, int born_proc, int64_t n, int64_t ld, const double* mom,
                                  nlo_prec prec, double* born, double* vi, void* hip_stream);

/* ---- cuts: the passCuts / passAnyCuts predicates of the paper's Algorithm 2
 * (the paper defines no cuts; these are infrared safe, so that the
 * subtraction still cancels) ----
 * Jets are the final-state massless coloured partons clustered by the
 * anti-kT algorithm with radius jet_r in (rapidity, azimuth), four-momentum
 * recombination; a parton exactly along the beam (pT = 0) is not clustered.
 * An event passes when at least njet_min jets have pT >= jet_ptmin and
 * |y| <= jet_ymax, every top quark has pT >= top_ptmin and |y| <= top_ymax,
 * and every charged lepton pT >= lep_ptmin and |y| <= lep_ymax (GeV; use 0
 * and a large number to switch a cut off). */
typedef struct {
  double jet_r;
  double jet_ptmin, jet_ymax;
  int njet_min;
  double top_ptmin, top_ymax;
  double lep_ptmin, lep_ymax;
} nlo_cuts;

/* pass: device uint8 [n], 1 where event e of mom (layout above, process
 * proc_id) passes the cuts, else 0. */
nlo_status nlo_cut_mask(nlo_ctx* ctx, int proc_id, int64_t n, int64_t ld, const double* mom, const nlo_cuts* cuts,
                        uint8_t* pass, void* hip_stream);

/* The mask argument of nlo_subtracted for one FKS sector, every term at its
 * own kinematics (Algorithm 2: passCuts(a, p_a)): B and S at the Born point
 * as given (the soft limit adds a zero-energy parton, which is not
 * clustered); R at the real point of the FKS map; C at the map's collinear
 * end: for a final-state emitter the y = 1 point, whose collinear pair the jet
 * algorithm merges back into the Born jet (C = B); for the beams the y = +1
 * and y = -1 points separately, encoded as 2 | 4 (y = +1 passes) | 8 (y = -1
 * passes), which nlo_subtracted reads per end.  mask: device [4][ld] bytes. */
nlo_status nlo_fks_cut_masks(nlo_ctx* ctx, int real_proc, int fks_i, int fks_j, int64_t n, int64_t ld,
                             const double* born_mom, const double* xi_tilde, const double* y, const double* phi,
                             const nlo_cuts* cuts, uint8_t* mask, void* hip_stream);

/* Algorithm 2's "regenerate until a cut passes" loop as stream compaction:
 * RAMBO candidates of proc_id (exactly as nlo_phase_space: candidate c is
 * event first + c of (seed, stream)) are generated and cut in chunks of up to
 * 2^20, and the passing ones written, in candidate order, to mom (layout
 * above, [npart][4][ld]) and weight ([n], or NULL) until n have passed.
 * *trials (host) receives the number of candidates used, i.e. one past the
 * index of the n-th passing one, so that a Monte Carlo estimate over the cut
 * region is (1/trials) sum over the n outputs.  Candidates are generated twice
 * (count, then scatter) instead of stored; a block's count and its position
 * among the passing candidates come from fixed-order scans, so the output is
 * the same for any chunking.  Synchronises the stream once per chunk.  Fails
 * with NLO_EINVAL when 2^26 candidates in a row pass nothing. */
nlo_status nlo_generate_passing(nlo_ctx* ctx, int proc_id, int64_t n, int64_t ld, uint32_t seed, uint32_t stream,
                                uint64_t first, double sqrt_s_lo, double sqrt_s_hi, const nlo_cuts* cuts,
                                double* mom, double* weight, uint64_t* trials, void* hip_stream);

/* Partonic cross section of proc_id at fixed sqrt(s_hat) by plain Monte Carlo
 * integration (the paper's section "Monte-Carlo integration": the mean of the
 * integrand times the volume of the measure) over n RAMBO points generated on
 * the device (seed, stream; events 0..n-1), with |M|^2 in precision prec:
 *   sigma = (1/n) sum_e w_e |M|^2_e ident / (2 s_hat),  in pb (GeV^-2 x 0.3893793721e9),
 * error = the standard error of that mean.  Sums are accumulated in FP64 in a
 * fixed order (reproducible for a given n).  Processes min(n, 2^20) events
 * per chunk in the context workspace (nlo_reserve of that many events) and
 * synchronises the stream before returning.  error_pb may be NULL. */
nlo_status nlo_cross_section(nlo_ctx* ctx, int proc_id, int64_t n, uint32_t seed, uint32_t stream, double sqrt_s,
                             nlo_prec prec, double* sigma_pb, double* error_pb, void* hip_stream);

/* Subtracted real-emission cross section of real_proc at fixed Born energy,
 * summed over its FKS sectors, by adaptive Monte Carlo on the device (the
 * paper's fixed-order integration, section "Monte-Carlo integration", with
 * importance sampling):
 *   sigma = sum_sectors int dPhi_B(s_B) int dxi_tilde dy dphi dsig,   in pb,
 * dsig as in nlo_fks_out (the subtracted weight with the map's phase-space
 * factor), dPhi_B the Born phase space at sqrt(s_B) = sqrt_s_born (beams along
 * +-z).  Integration variables: the 4 RAMBO uniforms of every Born final-state
 * particle and xi_tilde, (1+y)/2, phi/(2 pi), each on its own VEGAS grid
 * (Lepage's algorithm, 50 bins, damping alpha = 1.5), refined after every
 * iteration from the per-bin sums of f^2.  n points per iteration (2 <= n <=
 * 2^20), niter iterations; the first nadapt only shape the grid, the others
 * are combined with inverse-variance weights (error_pb: its standard error,
 * chi2_dof: their chi^2 per degree of freedom).  Uniforms: Philox (seed,
 * stream), point k of iteration t at counter t n + k, slot d/2 for variable d.
 * Every reduction runs in a fixed order, so a result is reproducible bit for
 * bit.  iterations (host, may be NULL): [niter][2] per-iteration estimate and
 * standard error.  Uses the context workspace (nlo_reserve(ctx, n) covers it)
 * and synchronises the stream before returning.  prec: FP64, FP32 or MIXED.
 * A point whose integrand is not finite counts as zero and makes the call
 * return NLO_EDEVICE after filling the outputs. */
nlo_status nlo_integrate_subtracted(nlo_ctx* ctx, int real_proc, double sqrt_s_born, int64_t n, int niter,
                                    int nadapt, uint32_t seed, uint32_t stream, nlo_prec prec, double* sigma_pb,
                                    double* error_pb, double* chi2_dof, double* iterations, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* NLOME_H */

/*
 * tor.h -- C ABI of the MI355X Torontonian library.
 *
 * The library evaluates the Torontonian (Sec. 3.1, Eq. 2 of "Benchmarking
 * 50-Photon Gaussian Boson Sampling on the Sunway TaihuLight"):
 *
 *     Tor(O) = sum over Z subset of {1..n} of (-1)^(n-|Z|) / sqrt(det(I - O_Z)),
 *
 * where O is the 2n x 2n sampling matrix of an n-click pattern (Eq. 1: the
 * paper's A_{S}, with A = I - Sigma^{-1}) and O_Z keeps rows and columns i
 * and i+n for every i in Z.  It is the probability of the click pattern
 * divided by the vacuum probability (Eq. 1), so GBS samplers need many of
 * them.
 *
 * Conventions for every entry point:
 *   - O is complex128 (interleaved re, im), row-major, leading dimension
 *     `ld` >= 2n in complex elements, in the paper's block order
 *     [[O00, O01], [O10, O11]] (all a-modes, then all a^dagger-modes).
 *   - Only the lower triangle (row >= column) is read.  The input must be
 *     exactly Hermitian, with I - O positive definite (then every I - O_Z
 *     is, Sec. 4.2); a pivot that is not > 0 is reported as TOR_ENOTPD.
 *   - n = 0 gives Tor = 1 (the empty set is the one term).
 *   - Pointers marked "device" are HIP device pointers; the caller owns all
 *     input and output buffers.  The library owns a per-device workspace,
 *     allocated on first use and released by tor_shutdown().
 *   - `stream` is a hipStream_t (NULL: the default stream).  Work is
 *     enqueued on it; synchronous entry points also wait for it.
 *   - Every call returns TOR_OK (0) or a negative TOR_E* code; nothing
 *     throws or aborts across the ABI.  Calls on one device are not
 *     thread-safe with respect to each other.
 */
#ifndef TOR_H
#define TOR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define TOR_OK 0
#define TOR_EINVAL (-1)       /* n out of range, null pointer, bad ld, unknown tier/algo */
#define TOR_ENOTPD (-2)       /* a pivot was not > 0: I - O is not positive definite */
#define TOR_EHIP (-3)         /* a HIP runtime error */
#define TOR_ENOMEM (-4)       /* device allocation failed */
#define TOR_EUNSUPPORTED (-5) /* tier x n does not fit the kernel's storage plan, or the library was compiled without the facility */
#define TOR_EINPUT (-6)       /* TOR_FLAG_CHECK_INPUT: O is not finite, not Hermitian, or lacks the block structure of Eq. 3 */

/* Largest n accepted: the paper's largest instance (N = 50, a 100 x 100
 * matrix, Sec. 7).  Subset masks are 64-bit.  The Schur path keeps a
 * frontier and chunks sized for it (at n = 50 about 10 GB in FP64, 26 GB in
 * DD, 80 GB in QD of device memory); the bordered kernel keeps the factor in
 * LDS and answers TOR_EUNSUPPORTED where a tier x n does not fit (DD beyond
 * n = 49, QD beyond n = 34). */
#define TOR_NMAX 50

/* Precision tiers (Sec. 5.1-5.4; the paper's 128-bit tier corresponds to
 * TOR_DD and its 256-bit tier to TOR_QD, as in Table 5). */
typedef enum {
  TOR_FP64 = 0, /* binary64 arithmetic, double-double accumulation of terms */
  TOR_DD = 1,   /* double-double (~106-bit significand) throughout */
  TOR_QD = 2,   /* quad-double (~212-bit significand) throughout */
  TOR_AUTO = -1 /* the library picks per instance (precision selector) */
} tor_tier_t;

/* Subset-tree algorithms.  Both enumerate the 2^n subsets as depth-first
 * subtrees hanging off prefixes of the first d modes (Sec. 4.1 splits the
 * same enumeration by subset size instead) and carry one factorisation
 * along each path. */
typedef enum {
  TOR_ALGO_AUTO = 0,
  TOR_ALGO_BORDER = 1, /* bordered Cholesky: appending a mode adds two rows to
                          the factor, O(|Z|^2) per subset (Sec. 4.2's
                          elimination made incremental) */
  TOR_ALGO_SCHUR = 2   /* right-looking: each state carries the Schur
                          complement of the undecided modes, in the real
                          quadrature basis; taking a mode in is a rank-2
                          update, about 12 of them per subset amortised */
} tor_algo_t;

/* Result of one Torontonian. 64 bytes. */
typedef struct tor_result {
  double tor[4];     /* Tor as a non-overlapping expansion, largest first:
                        FP64 and DD fill [0..1], QD fills [0..3]; rest 0 */
  double abs_sum[2]; /* S_abs = sum of |terms|, double-double; the
                        cancellation ratio is abs_sum / |tor| */
  double err_bound;  /* a-priori estimate of |Tor - computed| (absolute):
                        c * (2n)^2 * u_tier * S_abs */
  int32_t tier_used; /* tier the value was computed in */
  int32_t status;    /* TOR_OK or TOR_ENOTPD for this instance */
} tor_result_t;

/* Optional knobs; pass NULL for defaults. */
typedef struct tor_options {
  int32_t algo;         /* tor_algo_t */
  int32_t split_depth;  /* TOR_ALGO_BORDER: d, the number of leading modes
                           whose subsets form the work items (2^d of them);
                           -1 = automatic */
  int32_t grid;         /* persistent workgroups; 0 = from occupancy */
  int32_t flags;        /* TOR_FLAG_* bits */
  int32_t bottom_modes; /* TOR_ALGO_SCHUR: modes each lane finishes in
                           registers (s_b); 0 = the tier's default */
  int32_t reserved[3];
} tor_options_t;

/* Record HIP events around the subset-tree kernel (on the caller's stream);
 * read the duration back with tor_last_kernel_ms(). */
#define TOR_FLAG_TIME_KERNEL 1
/* tor_eval_batched: capture the batch's launches in a HIP graph on first
 * use and replay it when the same batch (same pointers, sizes, offsets and
 * tiers) comes again. */
#define TOR_FLAG_GRAPH 2
/* tor_eval, tor_eval_part, tor_eval_batched: first check on the device that
 * every O is what the kernels assume (they read the lower triangle and the
 * O00 / O01 blocks only): all entries finite, O Hermitian, O11 = conj(O00)
 * and O10 = conj(O01) (the block structure of the sampling matrix, Eq. 3),
 * compared exactly.  On a violation the call evaluates nothing and returns
 * TOR_EINPUT.  The check is one small kernel and a copy of one flag per
 * instance, synchronous; without the flag nothing is checked. */
#define TOR_FLAG_CHECK_INPUT 4

/* Library version string. */
const char* tor_version(void);

/* Text for an error code. */
const char* tor_strerror(int code);

/* Optional: set up the workspace of the current device ahead of time. */
int tor_init(void);

/* Release the workspaces of all devices (the library re-creates them on
 * the next call). */
int tor_shutdown(void);

/* Tor(O) for one instance (Sec. 3.1, Eq. 2).
 *   O      device, complex128, 2n x 2n, block order, lower triangle read
 *   n      0 <= n <= TOR_NMAX
 *   ld     leading dimension of O in complex elements (>= 2n)
 *   tier   TOR_FP64, TOR_DD or TOR_QD
 *   opt    NULL or knobs
 *   stream hipStream_t or NULL
 *   out    host; filled on return
 * Synchronous: enqueues on `stream` and waits for it. */
int tor_eval(const void* O, int32_t n, int64_t ld, int32_t tier, const tor_options_t* opt,
             void* stream, tor_result_t* out);

/* A share of one Torontonian (Sec. 3.1, Eq. 2), for evaluations split over
 * calls (checkpoint and resume: keep the finished parts' results) or over
 * devices (the paper splits the 2^N subsets over its processes, Alg. 1).
 * Part `part` of `nparts` covers the subsets Z whose decisions on the first
 * k modes, k = ceil(log2 nparts), read as a binary number with mode 0 as its
 * most significant bit (bit set = mode in Z), lie in
 * [part 2^k / nparts, (part + 1) 2^k / nparts) (floor divisions): the parts
 * are disjoint, cover every subset, and differ in size by at most a factor
 * of two.  The definition does not depend on the tier or the options.
 *   O, n, ld, tier, opt, stream   as tor_eval (opt->algo AUTO or SCHUR)
 *   part, nparts   0 <= part < nparts; nparts <= 2^d where d is the depth at
 *                  which the evaluation keeps its frontier (10 for most n;
 *                  fewer below n = 22; one more per mode from n = 42 in
 *                  FP64, 40 in DD and 38 in QD, up to 18 at n = 50 in FP64
 *                  and DD and 19 in QD), else TOR_EINVAL; n = 0 allows
 *                  nparts = 1
 *   out            host: tor = the part's signed sum, abs_sum its sum of
 *                  magnitudes, err_bound and status as tor_eval
 * Synchronous. */
int tor_eval_part(const void* O, int32_t n, int64_t ld, int32_t tier, const tor_options_t* opt,
                  void* stream, int32_t part, int32_t nparts, tor_result_t* out);

/* Tor from the results of all nparts parts of one instance (tor_eval_part,
 * any order of evaluation), added in part order in the tier's arithmetic
 * (double-double, quad-double for TOR_QD).  parts: host, nparts results, all
 * with tier_used == tier; out: host.  status is the first part's non-OK
 * status, if any.  Host only; no GPU needed. */
int tor_combine_parts(int32_t tier, int32_t n, const tor_result_t* parts, int32_t nparts,
                      tor_result_t* out);

/* Torontonians of many instances of uneven n (the click patterns a sampler
 * scores, Sec. 7.1.1: about a hundred per sample), enqueued on `stream`.
 * Instances are grouped by (n, tier); each group's states are expanded
 * together and the whole batch is one fixed sequence of launches, which
 * TOR_FLAG_GRAPH captures once and replays.
 *   O_packed  device; instance k's O (2n_k x 2n_k complex128, row-major,
 *             leading dimension 2n_k, block order, lower triangle read)
 *             starts at O_packed + offsets[k] complex elements
 *   offsets   host, batch int64
 *   n         host, batch int32, each 0..TOR_NMAX
 *   tiers     host, batch int32 (TOR_FP64 / TOR_DD / TOR_QD / TOR_AUTO), or
 *             NULL for all TOR_AUTO; TOR_AUTO instances get the cheapest
 *             tier the precision selector expects to meet `tau`
 *   tau       forward relative accuracy target |dTor| / |Tor| for TOR_AUTO
 *   opt       NULL or knobs (algo must be TOR_ALGO_AUTO or TOR_ALGO_SCHUR)
 *   out       device, batch results; status TOR_ENOTPD marks an instance
 *             whose I - O is not positive definite
 * With fixed tiers the call is stream-ordered: it enqueues the plan's
 * upload (from pinned memory, into one of four plan slots that are reused
 * once the batch that last used them has finished) and the evaluation on
 * `stream` and returns without waiting; a replay of a captured batch
 * (TOR_FLAG_GRAPH) is one graph launch.  The device workspace is shared by
 * every call on a device, so calls on different streams must be ordered by
 * the caller.  With TOR_AUTO instances it is synchronous: the tiers are
 * chosen first, and a
 * sample of the network's FP64 and DD choices whose predicted error lies
 * within 4 decades of tau (1/32 of them, at least one per tier;
 * TOR_SPOT_FRACTION and TOR_SPOT_WINDOW override) is re-evaluated one tier
 * up within the same launch sequence (the re-evaluations join the groups
 * of their n and tier); when a sample misses tau, every instance of that
 * tier predicted at least as hard is re-evaluated one tier up
 * (tor_last_select_stats reports the counts). */
int tor_eval_batched(const void* O_packed, const int64_t* offsets, const int32_t* n, int32_t batch,
                     const int32_t* tiers, double tau, const tor_options_t* opt, void* stream,
                     tor_result_t* out);

/* Markov chains over N-click patterns: the independence Metropolis sampler
 * the paper scores candidate patterns with, about a hundred per sample
 * (Sec. 7.1.1), on the pattern probabilities of Eq. 1,
 * p(S) = Tor(O_S) / sqrt(det Sigma_Q), where O_S keeps rows and columns k
 * and M+k of the M-mode O for every clicked mode k.
 * `chains` chains run side by side for `steps` steps.  Step t offers chain b
 * the candidate proposals[t][b][0..N-1]; step 0 takes it, and at a later step
 * a chain at pattern x moves to the candidate c when
 *     uniforms[t][b] * Tor(O_x) < Tor(O_c),
 * with both Torontonians' leading binary64 words and the product rounded to
 * binary64 (the vacuum factor of Eq. 1 is common to every pattern and
 * cancels).  With candidates drawn uniformly and u uniform in [0, 1) a chain
 * moves with probability min(1, p(c)/p(x)).  The candidates do not depend
 * on the chains, so all steps x chains of them are scored first, in batched
 * evaluations (as tor_eval_batched, in chunks of at most 1 GiB of packed
 * O_S; the environment variable TOR_MCMC_CHUNK caps the candidates per
 * chunk further), and then one lane per chain takes its decisions in order.
 *   O_full     device, complex128, 2M x 2M of the M-mode state, block order,
 *              leading dimension ld >= 2M; only the lower triangle is read
 *   M, N       1 <= M; 0 <= N <= min(M, TOR_NMAX) clicks per pattern
 *   chains, steps  >= 1, chains * steps < 2^31
 *   proposals  device, int32 [steps][chains][N]: each row's modes strictly
 *              increasing in [0, M) (may be NULL when N = 0)
 *   uniforms   device, double [steps][chains], each in [0, 1]
 *   tier       TOR_FP64 / TOR_DD / TOR_QD, or TOR_AUTO with target `tau`
 *   opt        NULL or knobs as tor_eval_batched (TOR_FLAG_GRAPH is ignored)
 *   cand_out   device, tor_result_t [steps][chains]: each candidate's Tor
 *   state_step device, int32 [steps][chains]: after step t chain b holds the
 *              candidate of step state_step[t][b] (<= t)
 * The library allocates the packed candidates and frees them before it
 * returns.  Synchronous.  TOR_EINVAL when a candidate row or variate is out
 * of range (checked on the device before anything is scored), TOR_ENOTPD when
 * some I - O_S was not positive definite (outputs still written). */
int tor_mcmc(const void* O_full, int32_t M, int64_t ld, int32_t N, int32_t chains, int32_t steps,
             const int32_t* proposals, const double* uniforms, int32_t tier, double tau,
             const tor_options_t* opt, void* stream, tor_result_t* cand_out, int32_t* state_step);

/* Per-level sums L_m = sum over |Z| = m of det(I - O_Z)^(-1/2), m = 0..n
 * (the pieces Alg. 1's level loop adds up, each unsigned).
 *   out_levels  host, 4*(n+1) doubles: level m as an expansion at [4m..4m+3]
 *   out         host, the Torontonian of the same run
 * Synchronous. */
int tor_debug_level_sums(const void* O, int32_t n, int64_t ld, int32_t tier, void* stream,
                         double* out_levels, tor_result_t* out);

/* The same per-level sums through the Schur path's own kernels (the
 * breadth-first top levels and the middle + bottom kernel in a level-sum
 * mode: one wavefront per workgroup, bottoms of at most 4 / 3 / 2 modes in
 * FP64 / DD / QD, every lane keeping one run per subset size and every
 * wavefront adding its lanes' runs in lane order); arguments and output as
 * tor_debug_level_sums, any n up to TOR_NMAX.  Synchronous. */
int tor_debug_level_sums_schur(const void* O, int32_t n, int64_t ld, int32_t tier, void* stream,
                               double* out_levels, tor_result_t* out);

/* Where the middle + bottom kernel's time goes: the shader-clock cycles its
 * wavefronts spent in each phase, summed over all wavefronts since the last
 * reset, TOR_NPHASE values in this order: the expansion's middle levels in
 * LDS (with the next state's prefetch), each lane's own last middle level,
 * the barrier after the expansion, the bottom level, the wave totals and
 * the partial's store, the barrier after the bottom, set-up and tail.  The
 * paper times its elimination kernels the same way, per kernel and per
 * instruction schedule (Sec. 6, Table 3).  Only a library built with
 * TOR_PHASE_CLOCKS counts (the in-tree build writes it beside the regular
 * one, as libtor_hip_phase.so); the regular library answers
 * TOR_EUNSUPPORTED.
 *   reset  nonzero: zero the totals after reading them
 *   out    host, TOR_NPHASE uint64
 * Reads the current device's totals; synchronous. */
#define TOR_NPHASE 7
int tor_debug_phase_clocks(int32_t reset, uint64_t* out);

/* det(I - O_Z)^(-1/2) with its sign (-1)^(n-|Z|) for k explicit subsets
 * (one term of Eq. 2 each).
 *   masks      device, k uint64 (bit i <=> mode i in Z, i < n)
 *   out_terms  device, 4*k doubles: term i as an expansion at [4i..4i+3]
 * Enqueued on `stream`; returns without waiting. */
int tor_debug_sampled_terms(const void* O, int32_t n, int64_t ld, int32_t tier,
                            const uint64_t* masks, int64_t k, void* stream, double* out_terms);

/* Time of the dominant kernel in the last synchronous evaluation on the
 * current device that set TOR_FLAG_TIME_KERNEL: the sum, in milliseconds,
 * of HIP-event durations recorded on the caller's stream around each launch
 * of the bordered kernel (TOR_ALGO_BORDER) or of the middle+bottom kernel
 * (TOR_ALGO_SCHUR).  *launches receives the number of launches, *split_depth
 * the split depth (border) or the middle-level depth n - s_m (Schur),
 * *grid the workgroups per launch.  Any pointer may be NULL.  -1 if none. */
double tor_last_kernel_ms(int32_t* split_depth, int32_t* grid, int32_t* launches);

/* ---- Autotuner -------------------------------------------------------------
 * The Schur path's only shape choice with a real trade-off is s_b, the modes
 * each lane finishes in registers (more registers per lane vs. fewer middle
 * levels in LDS).  The tuner times every compiled s_b for (n, tier) in the
 * shape such evaluations run in: for n <= 24 a batch group of 256 instances
 * (the batched workloads), for larger n one instance timed on a share of
 * about 2^28 subsets of its kept frontier and scaled to the whole (so
 * tuning at n = 50 takes seconds, not hours); the work does not depend on
 * the values, so the instances are synthetic.  The fastest becomes the
 * default for that (n, tier) in this process.  A table shipped beside the
 * library (data/autotune_default.txt in its directory, written by tuning
 * n = 1..40 on an MI355X) is read before the first evaluation; the
 * environment variable TOR_AUTOTUNE_TABLE names another file (empty: none). */

/* best_bottom: host, the chosen s_b; ms: host, 6 doubles (s_b = 1..6, -1
 * where not compiled for the tier), the measured or scaled milliseconds, may
 * be NULL.  Synchronous; 1 <= n <= TOR_NMAX. */
int tor_autotune(int32_t n, int32_t tier, void* stream, int32_t* best_bottom, double* ms);
/* Save / load the tuned table as text lines "n tier s_b". */
int tor_autotune_save(const char* path);
int tor_autotune_load(const char* path);

/* ---- Precision selector (TOR_AUTO) --------------------------------------
 * The paper picks its precision once per run from bounds on the largest and
 * smallest intermediate values (Sec. 5.4, Eq. 5-7).  Here a small network
 * predicts, from cheap features, either each instance's cancellation ratio
 * kappa = S_abs / |Tor| or directly an upper quantile of the FP64 tier's
 * forward error, and the cheapest tier expected to meet the accuracy target
 * is picked; outside the network's training range the bound estimate
 * decides. */

#define TOR_NFEAT 20      /* features per instance (see tor_features) */
#define TOR_MLP_H1 32     /* network: TOR_NFEAT -> 32 -> 32 -> 1, tanh hidden */
#define TOR_MLP_H2 32
#define TOR_MLP_PARAMS 1761

/* Features of `batch` instances (all n >= 1), binary64, on the device.
 * R is the real quadrature form of I - O (same principal minors), Q its
 * inverse (sigma_Q in the same basis), q_k = det(R_kk)^(1/2):
 *   f0 n; f1 -1/2 log det R (log of the largest term, the level-n sum
 *   L_n); f2 sum_k log((1+q_k)/(1-q_k)) (log kappa if the modes were
 *   independent); f3 mean_k -log q_k; f4 a = mean Re O_kk; f5 Eq. 5's
 *   k = ((1-a)^2 - det(R)^(1/n))/n; f6 sum_{i<j} log(det_ij/(det_i det_j));
 *   f7 max q_k; f8 min q_k; f9, f10 log of the smallest and largest
 *   Cholesky pivot of R; f11 log mean_{i<j} det_ij^(-1/2) (level 2).
 *   Spectrum of R: f12 the Gershgorin lower bound min_i (R_ii - sum_j!=i
 *   |R_ij|), f13 log of the Gershgorin upper bound, f14 and f15 log of the
 *   smallest and largest Ritz value of 12 Lanczos steps (fewer when 2n < 12)
 *   from the normalised all-ones vector.
 *   Top levels (their terms over the largest term, t_k = det(Q_kk)^(-1/2)
 *   for the level-(n-1) subset without mode k, t_kl likewise with the 4x4
 *   block of modes k, l for level n-2): f16 log mean_k t_k, f17 log max_k
 *   t_k, f18 log mean_{k<l} t_kl, f19 log max_{k<l} t_kl (0 when n = 1).
 * Inputs as tor_eval_batched (offsets, n on the host); feats device,
 * batch x TOR_NFEAT.  Enqueued on `stream`. */
int tor_features(const void* O_packed, const int64_t* offsets, const int32_t* n, int32_t batch,
                 void* stream, double* feats);

/* Network forward pass: Y[b] = net(theta; (X[b] - mean) / std).  All device
 * pointers; X is B x TOR_NFEAT.  Enqueued on `stream`. */
int tor_mlp_forward(const double* theta, const double* mean, const double* std, const double* X,
                    int32_t B, void* stream, double* Y);

/* Gradient of the mean asymmetric squared loss
 *   L = (1/B) sum_b w_b (y_b - net(x_b))^2,  w_b = under if y_b > net(x_b) else over
 * (under > over penalises under-predicting kappa).  grad: device,
 * TOR_MLP_PARAMS; loss: device, 1 (or NULL).  Per-sample gradients are
 * summed in sample order.  Enqueued on `stream`. */
int tor_mlp_grad(const double* theta, const double* mean, const double* std, const double* X,
                 const double* y, int32_t B, double under, double over, void* stream, double* grad,
                 double* loss);

/* Gradient of the mean quantile (pinball) loss at level q in (0, 1),
 *   L = (1/B) sum_b max(q r_b, (q - 1) r_b),  r_b = y_b - net(x_b),
 * whose minimiser is the conditional q-quantile of y (an upper quantile of
 * the error for q near 1).  Arguments as tor_mlp_grad. */
int tor_mlp_grad_quantile(const double* theta, const double* mean, const double* std, const double* X,
                          const double* y, int32_t B, double q, void* stream, double* grad,
                          double* loss);

/* One Adam step (moments m, v, step >= 1) on theta in place; device. */
int tor_mlp_adam(double* theta, const double* grad, double* m, double* v, double lr, double beta1,
                 double beta2, double eps, int32_t step, void* stream);

/* What the network predicts. */
#define TOR_TARGET_KAPPA 0 /* y = log10 kappa; tier t's predicted error is
                              log10_c[t] + slope[t] (y + margin) + log10 u_t */
#define TOR_TARGET_ERR64 1 /* y = an upper quantile of log10 of the FP64 tier's
                              relative forward error; tier t's predicted error
                              is y + margin + log10_c[t] */

/* The selector used by TOR_AUTO (one per process).  A tier is chosen when
 * its predicted error is at most log10 tau; the cheapest such tier wins. */
typedef struct tor_selector {
  double theta[TOR_MLP_PARAMS];
  double mean[TOR_NFEAT], std[TOR_NFEAT]; /* input standardisation */
  double fmin[TOR_NFEAT], fmax[TOR_NFEAT]; /* training range; outside it the
                                              bound estimate decides */
  double log10_c[3]; /* per tier: the error model's offset (see target) */
  double slope[3];   /* per tier, in (0, 2]; TOR_TARGET_KAPPA only */
  double margin;     /* extra log10 safety margin on the prediction */
  int32_t nmin, nmax; /* training range of n */
  int32_t trained;    /* 0: no network, the bound estimate decides */
  int32_t target;     /* TOR_TARGET_KAPPA or TOR_TARGET_ERR64 */
} tor_selector_t;

int tor_selector_set(const tor_selector_t* sel); /* NULL clears it */
int tor_selector_get(tor_selector_t* sel);
int tor_selector_save(const char* path);
int tor_selector_load(const char* path);

/* ---- Selector training (Sec. 5.4's precision choice, learned) ----------- */

/* Labels of `count` instances from the library's own evaluations: the
 * reference tier (TOR_QD, or TOR_DD where QD would be slow) gives Tor and
 * S_abs, and the cheaper tiers are evaluated beside it.
 *   O_packed, offsets, n  as tor_eval_batched (offsets, n host)
 *   ref_tier   TOR_QD or TOR_DD
 *   labels     host, count x 4: [0] log10 kappa = log10(S_abs / |Tor|)
 *              (60 when Tor is exactly 0); [1], [2] log10 of the FP64 and DD
 *              values' relative forward errors |T_t - T_ref| / |T_ref| (at
 *              least log10 u_t - 2; the DD one NaN when DD is the
 *              reference); [3] NaN.  NaN rows for n = 0 or a failed
 *              reference.
 * Synchronous; allocates a result buffer for the call. */
int tor_selector_label(const void* O_packed, const int64_t* offsets, const int32_t* n, int32_t count,
                       int32_t ref_tier, void* stream, double* labels);

#define TOR_LOSS_ASYM_SQUARED 0 /* tor_mlp_grad's loss (under, over) */
#define TOR_LOSS_QUANTILE 1     /* tor_mlp_grad_quantile's loss (quantile) */

typedef struct tor_train_options {
  int32_t target;     /* TOR_TARGET_KAPPA or TOR_TARGET_ERR64 */
  int32_t loss;       /* TOR_LOSS_ASYM_SQUARED or TOR_LOSS_QUANTILE */
  int32_t epochs;     /* passes over the samples */
  int32_t batch_size; /* samples per Adam step */
  double lr, beta1, beta2, eps; /* Adam */
  double under, over; /* asymmetric squared loss weights */
  double quantile;    /* quantile loss level */
  double slack;       /* decades added to each tier's calibrated offset */
  double margin;      /* tor_selector_t.margin of the result */
  uint64_t seed;      /* initial weights and sample order */
} tor_train_options_t;

/* Train the selector network on the GPU by the library's kernels
 * (tor_mlp_grad / tor_mlp_grad_quantile per minibatch, fixed-order sums,
 * tor_mlp_adam) and calibrate its per-tier error model on the training
 * samples (Sec. 5.4's choice of precision from an error estimate).
 *   feats   host, count x TOR_NFEAT (tor_features)
 *   labels  host, count x 4 (tor_selector_label); rows whose target or
 *           features are not finite are skipped
 *   n       host, count
 *   opt     options (all fields used)
 *   out     host: the trained selector (not installed: tor_selector_set)
 *   losses  host, opt->epochs mean losses, or NULL
 * Weights start normal with standard deviation 1/sqrt(fan in) from a
 * splitmix64 stream of opt->seed, biases at 0; every epoch visits the samples
 * in a new order from the same stream.  Calibration, per tier t in {FP64, DD}
 * over the samples where its error is measured: TOR_TARGET_ERR64: log10_c[t]
 * = max (log10 err_t - y_pred) + slack; TOR_TARGET_KAPPA: for each slope in
 * [0.3, 1] the intercept is the upper envelope of log10(err_t / u_t) - s
 * log10 kappa, and the slope whose envelope is lowest on average is kept
 * (+ slack).  QD takes DD's model scaled by their unit roundoffs.  The same
 * inputs and options give the same selector bit for bit.  Synchronous;
 * allocates device memory for the call. */
int tor_selector_train(const double* feats, const double* labels, const int32_t* n, int32_t count,
                       const tor_train_options_t* opt, void* stream, tor_selector_t* out, double* losses);

/* Bound-based estimate of the significand bits an instance needs (Eq. 7 read
 * for floating tiers): log2 of the rigorous S_abs <= 2^n det(I-O)^(-1/2) over
 * the Eq. 6 estimate of |Tor| (with a and k of Eq. 5), plus log2(1/tau)
 * (the wanted digits) and log2(0.5 2^n n^2) (accumulated error).  feats:
 * host, one instance's TOR_NFEAT features.  No GPU needed. */
double tor_fallback_bits(const double* feats, double tau);

/* Tiers TOR_AUTO would pick for each instance, without evaluating them.
 *   tiers, log10_kappa, source: host, batch entries each (the last two may
 *   be NULL); source[k] = 0 network, 1 bound estimate.  Synchronous. */
int tor_select_tiers(const void* O_packed, const int64_t* offsets, const int32_t* n, int32_t batch,
                     double tau, void* stream, int32_t* tiers, double* log10_kappa,
                     int32_t* source);

/* What the last TOR_AUTO batch did. */
typedef struct tor_select_stats {
  int32_t n_fp64, n_dd, n_qd;  /* tiers chosen */
  int32_t n_fallback;          /* decided by the bound estimate */
  int32_t n_spot;              /* re-evaluated at the next tier as a check */
  int32_t n_violations;        /* spot checks that missed tau */
  int32_t n_escalated;         /* instances moved up a tier afterwards */
  int32_t reserved;
} tor_select_stats_t;
int tor_last_select_stats(tor_select_stats_t* out);

/* ---- Host-side scheduling helpers (no GPU needed) ----------------------
 * Alg. 2's mask functions, used to order the work items by subset size. */

/* Next N-bit mask with the same number of ones, in decreasing numeric order
 * (Alg. 2, get_next_mask: the trailing block of ones moves down under the
 * lowest remaining one).  Returns 0 after the last mask of that popcount. */
uint64_t tor_next_mask(uint64_t mask);

/* The k-th (0-based) N-bit mask with c ones, in the same decreasing order
 * (Alg. 2, get_kth_mask: bits decided from the top, skipping blocks of
 * C(remaining positions, remaining ones) masks).  N <= 63, 0 <= c <= N,
 * k < C(N, c); returns 0 for out-of-range arguments. */
uint64_t tor_kth_mask(int32_t N, int32_t c, uint64_t k);

/* The 2^d work items of an n-mode evaluation split at depth d: every subset
 * of modes [0, d) exactly once, largest subsets first (their subtrees carry
 * the largest factors), each size class in decreasing numeric order.
 *   out   host, 2^d uint64
 * 0 <= d <= min(n, 30). */
int tor_plan_items(int32_t n, int32_t d, uint64_t* out);

/* ---- Evaluation without device allocation -------------------------------
 * For callers that cannot call hipMalloc: code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation.  The library holds
 * one fixed buffer of TOR_NOALLOC_SCRATCH_BYTES on every device it runs on,
 * from the moment its code is loaded there until the process ends. */
#define TOR_NOALLOC_SCRATCH_BYTES ((uint64_t)256 << 20)

/* Tor(O) as tor_eval computes it through the Schur path (Sec. 3.1, Eq. 2),
 * with every intermediate in the fixed buffer: no device or host memory is
 * allocated (the first call on a device, or tor_init, looks up the
 * buffer's device address).  Enqueued on `stream`; returns without waiting.
 *   O, n, ld, tier  as tor_eval (default options: library's bottom size)
 *   out             device, one tor_result_t, written by the last kernel
 * n above tor_noalloc_nmax(tier) gives TOR_EUNSUPPORTED.  Where the plan
 * tor_eval uses fits in the buffer the result is bit-for-bit tor_eval's;
 * larger n run the same kernels in smaller chunks (same value within the
 * tier's error bound).  Every call on a device shares that device's buffer,
 * which keeps the last call's contents (what must start at zero is cleared
 * by a kernel in the sequence): calls that overlap on one device (other
 * streams, other threads) race and must be ordered by the caller.  Usable
 * inside stream capture. */
int tor_eval_noalloc(const void* O, int32_t n, int64_t ld, int32_t tier, void* stream,
                     tor_result_t* out);

/* Largest n tor_eval_noalloc accepts in `tier` (the plan must fit in
 * TOR_NOALLOC_SCRATCH_BYTES); TOR_EINVAL for an unknown tier.  Host only. */
int32_t tor_noalloc_nmax(int32_t tier);

/* Device workspace that one evaluation of an n-mode instance (tor_eval,
 * tor_eval_part) needs in `tier`: the Schur path's kept frontier of the
 * subset tree (Eq. 2), its per-chunk level buffers and partial sums
 * (the paper sizes its per-process storage in Sec. 4.2; here it is the
 * plan the library allocates by, rounded up to 2 MiB: the workspace grows
 * to exactly this for the largest evaluation it has run).  Host only, no
 * GPU needed.
 *   bottom_modes  0 (the library's choice) or as tor_options_t
 *   bytes         host, out
 * TOR_EINVAL for n outside 0..TOR_NMAX, an unknown tier or bottom_modes < 0. */
int tor_workspace_bytes(int32_t n, int32_t tier, int32_t bottom_modes, uint64_t* bytes);

/* Device workspace tor_eval_batched (and tor_mcmc) needs for `count`
 * instances of n modes in one tier: a group whose plan would pass 4 GiB runs
 * as sub-groups of equal size, so this is the largest sub-group's plan (a
 * single instance needs its own plan, as tor_workspace_bytes).  Host only. */
int tor_batch_workspace_bytes(int32_t n, int32_t tier, int32_t count, int32_t bottom_modes,
                              uint64_t* bytes);

#ifdef __cplusplus
}
#endif

#endif /* TOR_H */

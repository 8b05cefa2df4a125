// tor_internal.hpp -- declarations shared by the C-ABI layer (tor_abi.cpp)
// and the kernel launchers (tor_border.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tor.h"

namespace tor {

// Kernel modes of the subset-tree kernels.
enum KernelMode : int {
  MODE_SUM = 0,     // signed sum and |sum| per work item
  MODE_LEVELS = 1,  // ... plus per-level sums of |term|
  MODE_MASKS = 2,   // one explicit subset per item: its own term
};

// Per-item accumulator size in bytes for a tier (DD for F64/DD, QD for QD).
size_t acc_bytes(int tier);

// Stage O (block order, lower triangle read, leading dimension ld in complex
// elements) into Oi: 2n x 2n, row-major, interleaved mode order
// (row 2a+u <-> block row a + u n), both triangles filled.
hipError_t launch_stage(const double2* O, int n, int64_t ld, double2* Oi, hipStream_t s);

// Check the input conventions of ninst instances (finite, Hermitian, the
// block structure of Eq. 3): offs == nullptr for one instance at O (n1, ld1),
// else device offs / ns per instance.  bad[k] (zeroed by the caller) becomes
// 1 where instance k violates them.
hipError_t launch_check_input(const double2* O, const int64_t* offs, const int32_t* ns, int ninst, int n1, int64_t ld1,
                              int32_t* bad, hipStream_t s);

// Zero `count` 32-bit words (a kernel, so the call is safe inside a captured graph).
hipError_t launch_zero_words(uint32_t* p, int count, hipStream_t s);

// Bordered-Cholesky subset-tree kernel.  items: prefix masks (MODE_SUM /
// MODE_LEVELS, over modes [0, d)) or full subsets (MODE_MASKS).  partials:
// [nitems][ncols] accumulators, ncols = 2 (+ n+1 for MODE_LEVELS).
struct BorderLaunch {
  int tier, mode, n, d, nitems, grid;
  const double2* Oi;
  const uint64_t* items;
  uint32_t* queue;
  void* partials;
  int32_t* status;
};
size_t border_lds_bytes(int tier, int mode, int n);
hipError_t border_occupancy(int tier, int mode, int n, int* blocks_per_cu);
hipError_t launch_border(const BorderLaunch& a, hipStream_t s);

// Fixed-order reduction of partials [nitems][ncols] into red [ncols]; for
// more than 4096 items a first pass per 4096-item segment goes to scratch
// (reduce_scratch_bytes).  The order never depends on the launch shape.
size_t reduce_scratch_bytes(int tier, int nitems, int ncols);
hipError_t launch_reduce_cols(int tier, const void* partials, int nitems, int ncols, void* red,
                              void* scratch, hipStream_t s);

// Fixed-order sums of nseg contiguous segments of seg_len items of
// part[][2] into out[nseg][2].
hipError_t launch_seg_reduce(int tier, const void* part, int nseg, int seg_len, void* out,
                             hipStream_t s);

// One tor_result_t per instance from red[ninst][2]; an instance whose sums
// are not finite (a pivot was not > 0) gets status TOR_ENOTPD.
hipError_t launch_finalize_batch(int tier, const void* red, int ninst, const int32_t* out_index,
                                 int n, double err_rel, tor_result_t* out, hipStream_t s);

// out[idx[k]] = the n = 0 result (Tor = 1) with tier tiers[k], k < count.
hipError_t launch_fill_trivial(tor_result_t* out, const int32_t* idx, const int32_t* tiers,
                               int count, hipStream_t s);

// Build the tor_result_t from the two reduced columns (signed sum, |sum|).
hipError_t launch_finalize(int tier, const void* red, const int32_t* status, double err_rel,
                           tor_result_t* out, hipStream_t s);

// Copy column 0 of partials [nitems][2] into out4 (4 doubles per item).
hipError_t launch_expand_terms(int tier, const void* partials, int nitems, double* out4,
                               hipStream_t s);

// ---- right-looking Schur-complement kernels (tor_schur.hip) ----
size_t schur_value_bytes(int tier);
// middle-level (s_m) and bottom-level (s_b) mode counts for a tier and n
void schur_levels(int tier, int n, int sb_req, int* s_m, int* s_b);
// Root states of ninst instances of n modes: instance k's O starts at
// O + offs[k] (offs NULL: one instance at O), leading dimension ld.
hipError_t launch_real_root(int tier, const double2* O, const int64_t* offs, int ninst, int n,
                            int64_t ld, void* mat, void* g, int32_t* m, hipStream_t s);
hipError_t launch_expand(int tier, const void* in_mat, const void* in_g, const int32_t* in_m,
                         int s, int nst, void* out_mat, void* out_g, int32_t* out_m,
                         int32_t* status, hipStream_t st);
// K = 2 or 3 expansions in one launch (the levels in between in LDS): nst
// states of s modes -> nst * 2^K states of s - K modes, numbered as K
// launch_expand calls would number them, with the same values.  0 bytes:
// not available for these arguments; launches need bytes <= EXPAND_MULTI_LDS_MAX.
constexpr size_t EXPAND_MULTI_LDS_MAX = 48 * 1024;
// with the staged input state (three workgroups per 160 KiB CU)
constexpr size_t EXPAND_MULTI_STAGE_LDS_MAX = 53 * 1024;
size_t expand_multi_lds_bytes(int tier, int s, int K);
hipError_t launch_expand_multi(int tier, const void* in_mat, const void* in_g, const int32_t* in_m,
                               int s, int K, int nst, void* out_mat, void* out_g, int32_t* out_m,
                               int32_t* status, hipStream_t st);
// Level-sum debug mode of the middle + bottom kernel: as launch_leaf, and
// every workgroup (one wavefront) writes its level sums of |terms| by subset
// size, lvpart[block][0..n] (accumulators), for the states it took.  Bottom
// sizes 1..level_sb_max(tier).
int level_sb_max(int tier);
hipError_t launch_leaf_levels(int tier, int s_m, int s_b, const void* mat, const void* g, const int32_t* m,
                              int nst, int n, void* partials, int32_t* status, int grid, void* lvpart,
                              hipStream_t st);
hipError_t leaf_levels_occupancy(int tier, int s_b, int* blocks_per_cu);
hipError_t launch_leaf(int tier, int s_m, int s_b, const void* mat, const void* g, const int32_t* m,
                       int nst, int n, void* partials, int32_t* status, int grid, hipStream_t st);
hipError_t leaf_occupancy(int tier, int s_b, int* blocks_per_cu);
// The middle + bottom kernel's per-phase clock totals (TOR_NPHASE values;
// reset: zero them after reading).  hipErrorNotSupported unless the kernels
// were built with TOR_PHASE_CLOCKS.
hipError_t phase_clocks(bool reset, uint64_t* out);

// ---- selector kernels (tor_select.hip) ----
size_t features_lds_bytes(int nmax);
hipError_t launch_features(const double2* O, const int64_t* offs, const int32_t* ns, int batch,
                           int nmax, double* feats, hipStream_t s);
hipError_t launch_mlp_forward(const double* th, const double* mean, const double* sd,
                              const double* X, int B, double* Y, hipStream_t s);
// kind 0: asymmetric squared loss (under, over); kind 1: quantile loss at
// level q = under.  G: B x TOR_MLP_PARAMS scratch, lossb: B scratch.
hipError_t launch_mlp_grad(const double* th, const double* mean, const double* sd, const double* X,
                           const double* y, int B, int kind, double under, double over, double* G,
                           double* lossb, double* grad, double* loss, hipStream_t s);
// Minibatch rows idx[0..B) of X (TOR_NFEAT columns) and y into Xo, yo.
hipError_t launch_gather_samples(const double* X, const double* y, const int32_t* idx, int B, double* Xo,
                                 double* yo, hipStream_t s);
hipError_t launch_adam(double* th, const double* grad, double* m, double* v, double lr, double b1,
                       double b2, double eps, int step, hipStream_t s);

// The fixed device buffer of tor_eval_noalloc (TOR_NOALLOC_SCRATCH_BYTES per
// device): its device address on the current device and the device's
// compute units, looked up on the first call on each device.
hipError_t noalloc_buffer(void** ptr, int* cus);
// One trivial result (Tor = 1, the n = 0 case) written by a kernel.
hipError_t launch_trivial_one(tor_result_t* out, int tier, hipStream_t s);

}  // namespace tor

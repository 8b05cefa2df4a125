// tor_mcmc.hip -- device side of the Markov-chain sampler entry point
// (tor_mcmc): checking the caller's candidates, cutting each candidate's O_S
// out of the M-mode O (Eq. 1), and every chain's move decisions in order.
//
// The chains are independence Metropolis chains over N-click patterns, the
// sampler the paper scores candidate patterns with (Sec. 7.1.1).  Their
// candidates do not depend on the chains' states, so all of them are scored
// first, by the batched evaluator, and the decisions only read the scores.
#include <algorithm>

#include "tor_internal.hpp"
#include "tor_mcmc.hpp"

namespace tor {
namespace {

// bit 0: a candidate row that is not strictly increasing inside [0, M);
// bit 1: an acceptance variate outside [0, 1] (or NaN)
__global__ void mcmc_check_kernel(const int32_t* __restrict__ prop, const double* __restrict__ u,
                                  int64_t count, int N, int M, int32_t* flag) {
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t* r = prop + i * N;
    int prev = -1;
    for (int j = 0; j < N; ++j) {
      const int m = r[j];
      if (m <= prev || m >= M) bad |= 1;
      prev = m;
    }
    const double v = u[i];
    if (!(v >= 0.0 && v <= 1.0)) bad |= 2;
  }
  if (bad) atomicOr(flag, bad);
}

// One workgroup per candidate: O_S (2N x 2N, leading dimension 2N, block
// order) with row/column j < N taken from mode m_j and j >= N from M + m_{j-N}.
// The index list ascends, so the lower triangle of O_S comes from the lower
// triangle of O; the upper triangle is written as its conjugate.  Indices are
// clamped into [0, M) (the host has already rejected candidates outside it).
__global__ void mcmc_gather_kernel(const double2* __restrict__ O, int64_t ld, int M,
                                   const int32_t* __restrict__ prop, int N, int64_t first,
                                   double2* __restrict__ out) {
  __shared__ int idx[2 * TOR_NMAX];
  const int32_t* r = prop + (first + blockIdx.x) * N;
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    int m = r[j];
    m = m < 0 ? 0 : (m >= M ? M - 1 : m);
    idx[j] = m;
    idx[N + j] = M + m;
  }
  __syncthreads();
  const int n2 = 2 * N;
  double2* dst = out + (int64_t)blockIdx.x * n2 * n2;
  for (int e = threadIdx.x; e < n2 * n2; e += blockDim.x) {
    const int a = e / n2, b = e - a * n2;
    double2 v;
    if (a >= b) {
      v = O[(int64_t)idx[a] * ld + idx[b]];
    } else {
      v = O[(int64_t)idx[b] * ld + idx[a]];
      v.y = -v.y;
    }
    dst[e] = v;
  }
}

// One lane per chain, steps in order: step 0 takes its candidate; later the
// chain at x moves to candidate c when u * Tor(O_x) < Tor(O_c), on the
// Torontonians' leading binary64 words (the vacuum factor of Eq. 1 is common
// to all patterns and cancels).  Bit 2 of flag: a candidate whose
// evaluation did not return TOR_OK.
__global__ void mcmc_scan_kernel(const tor_result_t* __restrict__ cand, const double* __restrict__ u,
                                 int chains, int steps, int32_t* __restrict__ state_step,
                                 int32_t* flag) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= chains) return;
  int cur = 0;
  double tx = cand[b].tor[0];
  int bad = cand[b].status != TOR_OK;
  state_step[b] = 0;
  for (int t = 1; t < steps; ++t) {
    const int64_t i = (int64_t)t * chains + b;
    const double tc = cand[i].tor[0];
    bad |= cand[i].status != TOR_OK;
    if (u[i] * tx < tc) {
      cur = t;
      tx = tc;
    }
    state_step[i] = cur;
  }
  if (bad) atomicOr(flag, 4);
}

}  // namespace

hipError_t launch_mcmc_check(const int32_t* prop, const double* u, int64_t count, int N, int M,
                             int32_t* flag, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(mcmc_check_kernel, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, s,
                     prop, u, count, N, M, flag);
  return hipGetLastError();
}

hipError_t launch_mcmc_gather(const double2* O, int64_t ld, int M, const int32_t* prop, int N,
                              int64_t first, int count, double2* out, hipStream_t s) {
  if (count <= 0 || N <= 0) return hipSuccess;
  hipLaunchKernelGGL(mcmc_gather_kernel, dim3(count), dim3(256), 0, s, O, ld, M, prop, N, first, out);
  return hipGetLastError();
}

hipError_t launch_mcmc_scan(const tor_result_t* cand, const double* u, int chains, int steps,
                            int32_t* state_step, int32_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(mcmc_scan_kernel, dim3((chains + 255) / 256), dim3(256), 0, s, cand, u, chains,
                     steps, state_step, flag);
  return hipGetLastError();
}

}  // namespace tor

// tor_mcmc.hpp -- launchers of the Markov-chain sampler kernels
// (tor_mcmc.hip), used by the C-ABI layer.  Not part of the public ABI.
#pragma once

#include "tor_internal.hpp"

namespace tor {

// flag |= 1 for a candidate row not strictly increasing in [0, M), 2 for a
// variate outside [0, 1]; count rows of N int32 and count variates.
hipError_t launch_mcmc_check(const int32_t* prop, const double* u, int64_t count, int N, int M,
                             int32_t* flag, hipStream_t s);
// O_S of candidates first .. first+count-1 into out (2N x 2N each, packed).
hipError_t launch_mcmc_gather(const double2* O, int64_t ld, int M, const int32_t* prop, int N,
                              int64_t first, int count, double2* out, hipStream_t s);
// Move decisions of `chains` chains over `steps` steps; flag |= 4 when a
// candidate's status is not TOR_OK.
hipError_t launch_mcmc_scan(const tor_result_t* cand, const double* u, int chains, int steps,
                            int32_t* state_step, int32_t* flag, hipStream_t s);

}  // namespace tor

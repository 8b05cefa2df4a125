/* A plain C client of libtor_hip.so: no Python, no PyTorch, only the HIP
 * runtime for device memory and a stream.  It reads k instances from a
 * file (each O as 2n x 2n little-endian complex128, block order, one after
 * another), evaluates each with tor_eval in FP64, DD and QD, then all of
 * them in one tor_eval_batched call in DD on its own stream, and prints one
 * line per result:
 *   eval <k> <tier> <status> <tor[0..3]> <abs_sum[0..1]>      (hex floats)
 *   batched <k> <tier_used> <status> <tor[0..3]> <abs_sum[0..1]>
 * usage: tor_client FILE n_1 ... n_k
 * Exit status 0 on success, 1 on a usage or file error, 2 on a library or
 * HIP error (the message names the call). */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "tor.h"

static void print_result(const char* kind, int k, int tier, const tor_result_t* r) {
  printf("%s %d %d %d %a %a %a %a %a %a\n", kind, k, tier, r->status, r->tor[0], r->tor[1], r->tor[2], r->tor[3],
         r->abs_sum[0], r->abs_sum[1]);
}

#define HIP_OR_DIE(x)                                                      \
  do {                                                                     \
    hipError_t e_ = (x);                                                   \
    if (e_ != hipSuccess) {                                                \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));              \
      return 2;                                                            \
    }                                                                      \
  } while (0)
#define TOR_OR_DIE(x)                                                      \
  do {                                                                     \
    int rc_ = (x);                                                         \
    if (rc_ != TOR_OK) {                                                   \
      fprintf(stderr, "%s: %s (%d)\n", #x, tor_strerror(rc_), rc_);        \
      return 2;                                                            \
    }                                                                      \
  } while (0)

int main(int argc, char** argv) {
  if (argc < 3) {
    fprintf(stderr, "usage: %s FILE n_1 ... n_k\n", argv[0]);
    return 1;
  }
  const int k = argc - 2;
  int32_t* n = (int32_t*)malloc(sizeof(int32_t) * k);
  int64_t* offsets = (int64_t*)malloc(sizeof(int64_t) * k);
  int32_t* tiers = (int32_t*)malloc(sizeof(int32_t) * k);
  int64_t total = 0; /* complex elements */
  for (int i = 0; i < k; ++i) {
    n[i] = atoi(argv[2 + i]);
    if (n[i] < 1 || n[i] > TOR_NMAX) {
      fprintf(stderr, "bad n %s\n", argv[2 + i]);
      return 1;
    }
    offsets[i] = total;
    total += 4 * (int64_t)n[i] * n[i];
    tiers[i] = TOR_DD;
  }
  double* host = (double*)malloc(sizeof(double) * 2 * total);
  FILE* f = fopen(argv[1], "rb");
  if (!f || fread(host, sizeof(double) * 2, (size_t)total, f) != (size_t)total) {
    fprintf(stderr, "cannot read %lld complex values from %s\n", (long long)total, argv[1]);
    return 1;
  }
  fclose(f);
  void* dO = NULL;
  HIP_OR_DIE(hipMalloc(&dO, sizeof(double) * 2 * total));
  HIP_OR_DIE(hipMemcpy(dO, host, sizeof(double) * 2 * total, hipMemcpyHostToDevice));
  TOR_OR_DIE(tor_init());
  const int tier_list[3] = {TOR_FP64, TOR_DD, TOR_QD};
  for (int i = 0; i < k; ++i)
    for (int t = 0; t < 3; ++t) {
      tor_result_t r;
      TOR_OR_DIE(tor_eval((const double*)dO + 2 * offsets[i], n[i], 2 * (int64_t)n[i], tier_list[t], NULL, NULL, &r));
      print_result("eval", i, tier_list[t], &r);
    }
  hipStream_t s;
  HIP_OR_DIE(hipStreamCreate(&s));
  tor_result_t* dres = NULL;
  HIP_OR_DIE(hipMalloc((void**)&dres, sizeof(tor_result_t) * k));
  TOR_OR_DIE(tor_eval_batched(dO, offsets, n, k, tiers, 1e-3, NULL, (void*)s, dres));
  tor_result_t* res = (tor_result_t*)malloc(sizeof(tor_result_t) * k);
  HIP_OR_DIE(hipMemcpyAsync(res, dres, sizeof(tor_result_t) * k, hipMemcpyDeviceToHost, s));
  HIP_OR_DIE(hipStreamSynchronize(s));
  for (int i = 0; i < k; ++i) print_result("batched", i, res[i].tier_used, &res[i]);
  HIP_OR_DIE(hipStreamDestroy(s));
  HIP_OR_DIE(hipFree(dres));
  HIP_OR_DIE(hipFree(dO));
  TOR_OR_DIE(tor_shutdown());
  free(res);
  free(host);
  free(tiers);
  free(offsets);
  free(n);
  return 0;
}

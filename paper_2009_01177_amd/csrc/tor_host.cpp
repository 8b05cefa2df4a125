// tor_host.cpp -- host-side work planning: the mask functions of Alg. 2 and
// the ordering of work items by cost class.
#include <stdint.h>

#include "tor_host.h"

namespace {

// C(a, b) for 0 <= b <= a <= 63 (exact in 64 bits).
uint64_t binom(int a, int b) {
  if (b < 0 || a < 0 || b > a) return 0;
  if (b > a - b) b = a - b;
  uint64_t r = 1;
  for (int i = 1; i <= b; ++i) r = r * (uint64_t)(a - b + i) / (uint64_t)i;
  return r;
}

}  // namespace

extern "C" {

uint64_t tor_next_mask(uint64_t mask) {
  if (mask == 0) return 0;
  const int cto = __builtin_ctzll(~mask);  // trailing ones
  if (cto >= 64) return 0;
  const uint64_t x = mask - ((((uint64_t)1) << cto) - 1);
  if (x == 0) return 0;  // the ones were all packed at the bottom: last mask
  const int ctz = __builtin_ctzll(x);
  return x - (((uint64_t)1) << (ctz - cto - 1));
}

uint64_t tor_kth_mask(int32_t N, int32_t c, uint64_t k) {
  if (N < 0 || N > 63 || c < 0 || c > N) return 0;
  if (k >= binom(N, c)) return 0;
  uint64_t mask = 0;
  int l = -1;  // position (from the top, 0-based) of the last one placed
  for (int i = 0; i < c; ++i) {
    // candidate positions for the i-th one, leaving room for the rest
    for (int j = l + 1; j <= N - c + i; ++j) {
      const uint64_t cnt = binom(N - j - 1, c - i - 1);  // masks with this one at j
      if (k < cnt) {
        mask |= ((uint64_t)1) << (N - j - 1);
        l = j;
        break;
      }
      k -= cnt;
    }
  }
  return mask;
}

int tor_plan_items(int32_t n, int32_t d, uint64_t* out) {
  if (out == nullptr || d < 0 || d > 30 || n < 0 || d > n) return TOR_EINVAL;
  uint64_t w = 0;
  for (int c = d; c >= 0; --c) {
    uint64_t m = tor_kth_mask(d, c, 0);
    const uint64_t cnt = binom(d, c);
    for (uint64_t i = 0; i < cnt; ++i) {
      out[w++] = m;
      m = tor_next_mask(m);
    }
  }
  return w == ((uint64_t)1 << d) ? TOR_OK : TOR_EINVAL;
}

}  // extern "C"

// tor_select.hip -- the learned precision selector's GPU kernels: per
// instance features, and the forward pass, per-sample gradients, fixed-order
// gradient reduction and Adam update of a small MLP (all binary64).
//
// The selector predicts log10 of the cancellation ratio S_abs / |Tor| of an
// instance, the quantity that decides how many of a tier's bits survive the
// alternating sum (Sec. 5.1: Tor is tiny while every term exceeds 1).  The
// paper fixes its precision once per run from bounds (Sec. 5.4, Eq. 5-7);
// here a network makes the call per instance, with the bound estimate as the
// fallback outside the network's training range.
#include <hip/hip_runtime.h>

#include "tor_internal.hpp"

namespace tor {

// --------------------------------------------------------------------------
// Features (one workgroup of 256 threads per instance).  R is the real
// quadrature form of I - O (rows interleaved per mode), full square in LDS;
// Q = R^-1 (sigma_Q in the same basis) replaces it in the same array.
//   f0  n
//   f1  -1/2 log det(I - O)           (log of the largest term)
//   f2  sum_k log((1 + q_k)/(1 - q_k)), q_k = det(I - O)_{kk}^(1/2)
//       (log S_abs/|Tor| if the modes were independent)
//   f3  mean_k -log q_k
//   f4  a = mean_k Re O_kk            (Eq. 5's representative diagonal)
//   f5  k = ((1 - a)^2 - det(I - O)^(1/n)) / n   (Eq. 5 solved at |Z| = n)
//   f6  sum_{i<j} log(det_{ij} / (det_i det_j))  (pairwise coupling, <= 0)
//   f7  max_k q_k,  f8  min_k q_k
//   f9  log of the smallest, f10 of the largest Cholesky pivot of R
//   f11 log of the mean pair term, mean_{i<j} det_{ij}^(-1/2)
//   f12 Gershgorin lower bound of R's spectrum, f13 log of the upper one
//   f14, f15 log of the smallest / largest Ritz value of 12 Lanczos steps
//       on R from the normalised all-ones vector (fewer when 2n < 12)
//   f16, f17 log of the mean / largest det(Q_kk)^(-1/2): the level n-1
//       terms over the level-n term (det R_{-k} / det R = det Q_kk)
//   f18, f19 the same for the 4x4 blocks of mode pairs (level n-2)
// --------------------------------------------------------------------------

constexpr int LANCZOS_STEPS = 12;

__device__ inline double o_lower(const double2* O, int64_t ld, int r, int c, bool imag) {
  // element (r, c) of O in block order, read from the lower triangle
  if (r >= c) {
    const double2 v = O[(int64_t)r * ld + c];
    return imag ? v.y : v.x;
  }
  const double2 v = O[(int64_t)c * ld + r];
  return imag ? -v.y : v.x;
}

// Wavefront reductions by butterfly: lane results can differ in the last
// bit for sums (each lane associates differently), so the sum is taken from
// lane 0; min / max are exact in any order.
__device__ inline double wave_sum(double x) {
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
  return __shfl(x, 0);
}
__device__ inline double wave_min(double x) {
  for (int o = 32; o >= 1; o >>= 1) x = fmin(x, __shfl_xor(x, o));
  return x;
}
__device__ inline double wave_max(double x) {
  for (int o = 32; o >= 1; o >>= 1) x = fmax(x, __shfl_xor(x, o));
  return x;
}
__device__ inline int wave_min_int(int x) {
  for (int o = 32; o >= 1; o >>= 1) x = min(x, __shfl_xor(x, o));
  return x;
}

// Sum over the workgroup's 256 threads in a fixed order (the four
// wavefronts' sums, then (w0 + w1) + (w2 + w3)); every thread gets it.
// red: 8 doubles of LDS, the two halves used alternately (`phase`), so one
// barrier per call suffices as long as calls alternate phases.
__device__ inline double block_sum(double x, double* red, int phase) {
  const double ws = wave_sum(x);
  double* r = red + 4 * phase;
  if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = ws;
  __syncthreads();
  return (r[0] + r[1]) + (r[2] + r[3]);
}

// Number of eigenvalues below x of the k x k symmetric tridiagonal matrix
// with diagonal al and off-diagonal be (Sturm sequence of the LDL^T pivots).
__device__ inline int sturm_count(const double* al, const double* be, int k, double x) {
  int cnt = 0;
  double d = 1.0;
  for (int i = 0; i < k; ++i) {
    const double b2 = i > 0 ? be[i - 1] * be[i - 1] : 0.0;
    d = (al[i] - x) - (i > 0 ? b2 / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0.0) ++cnt;
  }
  return cnt;
}

// The j-th smallest eigenvalue of the tridiagonal matrix, by multisection
// inside its Gershgorin interval: in each round the 256 threads evaluate the
// Sturm count at 256 interior points and the interval shrinks to the gap
// where the count passes j (a factor of 257 per round).  Every thread
// returns the same value.  cnt: 8 ints of LDS.
__device__ inline double tridiag_eig(const double* al, const double* be, int k, int j, int* cnt) {
  const int tid = threadIdx.x;
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? fabs(be[i - 1]) : 0.0) + (i + 1 < k ? fabs(be[i]) : 0.0);
    lo = fmin(lo, al[i] - r);
    hi = fmax(hi, al[i] + r);
  }
  for (int round = 0; round < 8 && hi - lo > 1e-15 * fmax(fabs(lo), fabs(hi)); ++round) {
    const double w = (hi - lo) / 257.0;
    const int m = wave_min_int(sturm_count(al, be, k, lo + w * (tid + 1)) > j ? tid : 256);
    int* c = cnt + 4 * (round & 1);
    if ((tid & 63) == 0) c[tid >> 6] = m;
    __syncthreads();
    const int t = min(min(c[0], c[1]), min(c[2], c[3]));  // first point above eigenvalue j (256: none)
    const double nlo = lo + w * t, nhi = t < 256 ? lo + w * (t + 1) : hi;
    lo = nlo;
    hi = nhi;
  }
  __syncthreads();  // cnt is free for the next call
  return 0.5 * (lo + hi);
}

// Row-major lower-triangle index e = r (r + 1) / 2 + c, c <= r  ->  (r, c).
__device__ inline void tri_rc(int e, int* r, int* c) {
  int rr = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
  while (rr * (rr + 1) / 2 > e) --rr;
  while ((rr + 1) * (rr + 2) / 2 <= e) ++rr;
  *r = rr;
  *c = e - rr * (rr + 1) / 2;
}

// det of the 4x4 block of modes (i, j), i < j, of a symmetric matrix of
// which only the lower triangle (with the diagonal) is stored
__device__ inline double det_pair_lower(const double* A, int N2, int i, int j) {
  const int idx[4] = {2 * i, 2 * i + 1, 2 * j, 2 * j + 1};
  double a[4][4];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) a[r][c] = r >= c ? A[idx[r] * N2 + idx[c]] : A[idx[c] * N2 + idx[r]];
  double det = 1.0;
  for (int k = 0; k < 4; ++k) {
    const double d = a[k][k];
    det *= d;
    for (int r = k + 1; r < 4; ++r) {
      const double f = a[r][k] / d;
      for (int c = k + 1; c < 4; ++c) a[r][c] -= f * a[k][c];
    }
  }
  return det;
}

// p -> (i, j), i < j, lexicographic over the n modes
__device__ inline void pair_ij(int p, int n, int* i, int* j) {
  int ii = 0, rem = p;
  while (rem >= n - 1 - ii) {
    rem -= n - 1 - ii;
    ++ii;
  }
  *i = ii;
  *j = ii + 1 + rem;
}

__global__ __launch_bounds__(256) void features_kernel(const double2* __restrict__ Obase,
                                                       const int64_t* __restrict__ offs,
                                                       const int32_t* __restrict__ ns,
                                                       double* __restrict__ feats) {
  extern __shared__ double sh[];
  const int inst = blockIdx.x;
  const int n = ns[inst];
  const int N2 = 2 * n;
  const int64_t ld = 2 * n;
  const double2* O = Obase + offs[inst];
  double* R = sh;                   // N2 x N2: R, then its factor, then Q (lower)
  double* piv = R + N2 * N2;        // N2
  double* q = piv + N2;             // n
  double* pr = q + n;               // 2 * npairs: log ratio, det^(-1/2)
  const int npairs = n * (n - 1) / 2;
  double* red = pr + 2 * npairs;    // 256: reductions
  double* lz = red + 256;           // Lanczos: v_prev, v, w (N2 each), alpha, beta
  double* vp = lz, *vc = lz + N2, *wv = lz + 2 * N2;
  double* al = lz + 3 * N2, *be = al + LANCZOS_STEPS;
  double* gl = be + LANCZOS_STEPS;  // Gershgorin per row: lo, hi (N2 each)
  double* tq = gl + 2 * N2;         // n + npairs: det(Q_k)^(-1/2), then det(Q_kl)^(-1/2)
  const int tid = threadIdx.x;
  // R, one mode pair (its 2 x 2 block, four reads of O) per thread
  for (int pp = tid; pp < n * n; pp += 256) {
    const int i = pp / n, j = pp - (pp / n) * n;
    const double xr = o_lower(O, ld, i, j, false), xi = o_lower(O, ld, i, j, true);
    const double yr = o_lower(O, ld, i, j + n, false), yi = o_lower(O, ld, i, j + n, true);
    const double dlt = i == j ? 1.0 : 0.0;
    R[(2 * i) * N2 + 2 * j] = (dlt - xr) - yr;
    R[(2 * i) * N2 + 2 * j + 1] = xi - yi;
    R[(2 * i + 1) * N2 + 2 * j] = -xi - yi;
    R[(2 * i + 1) * N2 + 2 * j + 1] = (dlt - xr) + yr;
  }
  __syncthreads();
  for (int k = tid; k < n; k += 256) {
    const double d = R[(2 * k) * N2 + 2 * k] * R[(2 * k + 1) * N2 + 2 * k + 1] -
                     R[(2 * k + 1) * N2 + 2 * k] * R[(2 * k + 1) * N2 + 2 * k];
    q[k] = sqrt(d);
  }
  // Gershgorin discs
  for (int r = tid; r < N2; r += 256) {
    double off = 0.0;
    for (int c = 0; c < N2; ++c)
      if (c != r) off += fabs(R[r * N2 + c]);
    gl[r] = R[r * N2 + r] - off;
    gl[N2 + r] = R[r * N2 + r] + off;
  }
  __syncthreads();
  for (int p = tid; p < npairs; p += 256) {
    int i, j;
    pair_ij(p, n, &i, &j);
    const double dij = det_pair_lower(R, N2, i, j);
    pr[2 * p] = log(dij / (q[i] * q[i] * q[j] * q[j]));
    pr[2 * p + 1] = 1.0 / sqrt(dij);
  }
  // Lanczos on R (before it is factorised): v_0 = ones / sqrt(N2)
  const int ksteps = N2 < LANCZOS_STEPS ? N2 : LANCZOS_STEPS;
  int kdone = 0;
  for (int r = tid; r < N2; r += 256) {
    vp[r] = 0.0;
    vc[r] = 1.0 / sqrt((double)N2);
  }
  __syncthreads();
  // w = R v in nsplit column slices (thread (slice, row)), the slices'
  // partial products in red[8..) summed in slice order per row
  const int nsplit = N2 <= 62 ? 4 : (N2 <= 82 ? 3 : 2);
  double* mv = red + 8;
  const int mrow = tid % N2, mpart = tid / N2;
  const int mc0 = mpart * N2 / nsplit, mc1 = (mpart + 1) * N2 / nsplit;
  for (int j = 0; j < ksteps; ++j) {
    if (mpart < nsplit) {
      double s0 = 0.0, s1 = 0.0;
      int c = mc0;
      for (; c + 1 < mc1; c += 2) {
        s0 = fma(R[mrow * N2 + c], vc[c], s0);
        s1 = fma(R[mrow * N2 + c + 1], vc[c + 1], s1);
      }
      if (c < mc1) s0 = fma(R[mrow * N2 + c], vc[c], s0);
      mv[mpart * N2 + mrow] = s0 + s1;
    }
    __syncthreads();
    double part = 0.0;
    for (int r = tid; r < N2; r += 256) {
      double sr = mv[r];
      for (int q2 = 1; q2 < nsplit; ++q2) sr += mv[q2 * N2 + r];
      wv[r] = sr;
      part = fma(sr, vc[r], part);
    }
    const double a = block_sum(part, red, 0);
    const double bprev = j > 0 ? be[j - 1] : 0.0;
    part = 0.0;
    for (int r = tid; r < N2; r += 256) {
      const double w = wv[r] - a * vc[r] - bprev * vp[r];
      wv[r] = w;
      part = fma(w, w, part);
    }
    const double b = sqrt(block_sum(part, red, 1));
    if (tid == 0) {
      al[j] = a;
      be[j] = b;
    }
    kdone = j + 1;
    if (!(b > 1e-12 * fabs(a))) break;  // invariant subspace: T_j is exact
    for (int r = tid; r < N2; r += 256) {
      vp[r] = vc[r];
      vc[r] = wv[r] / b;
    }
    __syncthreads();
  }
  __syncthreads();
  // Cholesky of R in place, lower triangle, unscaled (R = L D L^T: piv = D,
  // the eliminated column below the pivot is D_j L_rj).  Step j updates the
  // triangle of rows and columns > j, four entries per thread per pass with
  // their loads issued first (column j is not written in step j, so it is
  // read without a barrier before the update).
  for (int j = 0; j < N2; ++j) {
    const double d = R[j * N2 + j];
    if (tid == 0) piv[j] = d;
    const double rd = 1.0 / d;
    const int m = N2 - j - 1, cnt = m * (m + 1) / 2;
    for (int e0 = tid; e0 < cnt; e0 += 1024) {
      int ro[4], co[4];
      double t[4], x[4], y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + 256 * u;
        if (e < cnt) {
          tri_rc(e, &ro[u], &co[u]);
          ro[u] += j + 1;
          co[u] += j + 1;
          x[u] = R[ro[u] * N2 + j];
          y[u] = R[co[u] * N2 + j];
          t[u] = R[ro[u] * N2 + co[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e0 + 256 * u < cnt) R[ro[u] * N2 + co[u]] = t[u] - x[u] * y[u] * rd;
    }
    __syncthreads();
  }
  // Q = R^-1 = X^T D^-1 X with X = L^-1 (unit lower), in R's own array:
  // the unit factor L formed in the lower triangle (column j of the
  // eliminated part over its pivot; reciprocal pivots in wv), X below its
  // unit diagonal kept transposed in the upper triangle (X_ic at (c, i)),
  // built by right-looking elimination (step j subtracts L_ij times row j
  // of X from every row i > j), then Q into the lower triangle and the
  // diagonal
  for (int j = tid; j < N2; j += 256) wv[j] = 1.0 / piv[j];
  __syncthreads();
  for (int e = tid; e < N2 * N2; e += 256) {
    const int r = e / N2, c = e - (e / N2) * N2;
    if (r > c) R[e] *= wv[c];
    if (r < c) R[e] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j + 1 < N2; ++j) {
    // (i, c), j < i < N2, 0 <= c <= j: X_ic -= L_ij X_jc (X_jj = 1)
    const int w = j + 1, cnt = (N2 - 1 - j) * w;
    for (int e0 = tid; e0 < cnt; e0 += 1024) {
      int io[4], co[4];
      double t[4], l[4], xj[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + 256 * u;
        if (e < cnt) {
          io[u] = j + 1 + e / w;
          co[u] = e - (e / w) * w;
          l[u] = R[io[u] * N2 + j];
          xj[u] = co[u] == j ? 1.0 : R[co[u] * N2 + j];
          t[u] = R[co[u] * N2 + io[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e0 + 256 * u < cnt) R[co[u] * N2 + io[u]] = t[u] - l[u] * xj[u];
    }
    __syncthreads();
  }
  // Q_ab = sum_{k >= a} X_ka X_kb / d_k for a >= b (X_ka = 0 for k < a):
  // reads the upper triangle only, writes the lower one and the diagonal
  for (int e = tid; e < N2 * (N2 + 1) / 2; e += 256) {
    int a, b;
    tri_rc(e, &a, &b);
    double s0 = (a == b ? 1.0 : R[b * N2 + a]) * wv[a], s1 = 0.0;
    int k = a + 1;
    for (; k + 1 < N2; k += 2) {
      s0 = fma(R[a * N2 + k] * wv[k], R[b * N2 + k], s0);
      s1 = fma(R[a * N2 + k + 1] * wv[k + 1], R[b * N2 + k + 1], s1);
    }
    if (k < N2) s0 = fma(R[a * N2 + k] * wv[k], R[b * N2 + k], s0);
    R[a * N2 + b] = s0 + s1;
  }
  __syncthreads();
  // the top levels' term ratios, one mode or pair per thread
  for (int k = tid; k < n; k += 256) {
    const double* Qk = R + (2 * k) * N2 + 2 * k;
    tq[k] = 1.0 / sqrt(Qk[0] * Qk[N2 + 1] - Qk[N2] * Qk[N2]);
  }
  for (int p = tid; p < npairs; p += 256) {
    int i, j;
    pair_ij(p, n, &i, &j);
    tq[n + p] = 1.0 / sqrt(det_pair_lower(R, N2, i, j));
  }
  __syncthreads();
  // extreme Ritz values (all threads take part in the multisection)
  const double ritz_lo = tridiag_eig(al, be, kdone, 0, (int*)red);
  const double ritz_hi = tridiag_eig(al, be, kdone, kdone - 1, (int*)red);
  // the rest: per-thread partial sums, minima and maxima, then per
  // wavefront, then the four wavefronts in a fixed order
  const double inf = __builtin_inf();
  double sm[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // logdet f2 f3 asum f6 pt s1 s2
  double mn[3] = {inf, inf, inf};                           // pmin qmin glo
  double mx[5] = {-inf, -inf, -inf, 0.0, 0.0};              // pmax qmax ghi m1 m2
  for (int j = tid; j < N2; j += 256) {
    sm[0] += log(piv[j]);
    mn[0] = fmin(mn[0], piv[j]);
    mx[0] = fmax(mx[0], piv[j]);
    mn[2] = fmin(mn[2], gl[j]);
    mx[2] = fmax(mx[2], gl[N2 + j]);
  }
  for (int k = tid; k < n; k += 256) {
    sm[1] += log((1.0 + q[k]) / (1.0 - q[k]));
    sm[2] += -log(q[k]);
    sm[3] += O[(int64_t)k * ld + k].x;
    mn[1] = fmin(mn[1], q[k]);
    mx[1] = fmax(mx[1], q[k]);
    sm[6] += tq[k];
    mx[3] = fmax(mx[3], tq[k]);
  }
  for (int p = tid; p < npairs; p += 256) {
    sm[4] += pr[2 * p];
    sm[5] += pr[2 * p + 1];
    sm[7] += tq[n + p];
    mx[4] = fmax(mx[4], tq[n + p]);
  }
  double* wr = red + 16 * (tid >> 6);
  {
    double v[16];
    for (int i = 0; i < 8; ++i) v[i] = wave_sum(sm[i]);
    for (int i = 0; i < 3; ++i) v[8 + i] = wave_min(mn[i]);
    for (int i = 0; i < 5; ++i) v[11 + i] = wave_max(mx[i]);
    if ((tid & 63) == 0)
      for (int i = 0; i < 16; ++i) wr[i] = v[i];
  }
  __syncthreads();
  if (tid == 0) {
    double v[16];
    for (int i = 0; i < 8; ++i) v[i] = (red[i] + red[16 + i]) + (red[32 + i] + red[48 + i]);
    for (int i = 8; i < 11; ++i) v[i] = fmin(fmin(red[i], red[16 + i]), fmin(red[32 + i], red[48 + i]));
    for (int i = 11; i < 16; ++i) v[i] = fmax(fmax(red[i], red[16 + i]), fmax(red[32 + i], red[48 + i]));
    const double logdet = v[0], f2 = v[1], f3 = v[2], asum = v[3], f6 = v[4], pt = v[5], s1 = v[6], s2 = v[7];
    const double pmin = v[8], qmin = v[9], glo = v[10];
    const double pmax = v[11], qmax = v[12], ghi = v[13], m1 = v[14], m2 = v[15];
    const double a = asum / n;
    double* f = feats + (size_t)inst * TOR_NFEAT;
    f[0] = n;
    f[1] = -0.5 * logdet;
    f[2] = f2;
    f[3] = f3 / n;
    f[4] = a;
    f[5] = ((1.0 - a) * (1.0 - a) - exp(logdet / n)) / n;
    f[6] = f6;
    f[7] = qmax;
    f[8] = qmin;
    f[9] = log(pmin);
    f[10] = log(pmax);
    f[11] = npairs > 0 ? log(pt / npairs) : 0.0;
    f[12] = glo;
    f[13] = log(ghi);
    f[14] = log(ritz_lo);
    f[15] = log(ritz_hi);
    f[16] = log(s1 / n);
    f[17] = log(m1);
    f[18] = npairs > 0 ? log(s2 / npairs) : 0.0;
    f[19] = npairs > 0 ? log(m2) : 0.0;
  }
}

// LDS of the features kernel for instances of up to nmax modes (R and its
// inverse share one N2 x N2 array: every n up to TOR_NMAX fits).
size_t features_lds_bytes(int nmax) {
  const size_t N2 = 2 * (size_t)nmax;
  return sizeof(double) * (N2 * N2 + N2 + nmax + (size_t)nmax * (nmax - 1) + 256 + 3 * N2 +
                           2 * LANCZOS_STEPS + 2 * N2 + nmax + (size_t)nmax * (nmax - 1) / 2);
}

hipError_t launch_features(const double2* O, const int64_t* offs, const int32_t* ns, int batch,
                           int nmax, double* feats, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  const size_t lds = features_lds_bytes(nmax);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&features_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(features_kernel, dim3(batch), dim3(256), lds, s, O, offs, ns, feats);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// MLP: TOR_NFEAT -> H1 -> H2 -> 1, tanh hidden layers, parameters packed as
// [W1 (H1 x F), b1, W2 (H2 x H1), b2, W3 (1 x H2), b3], W row-major (out, in).
// Inputs are standardised: x = (f - mean) / std.
// --------------------------------------------------------------------------

constexpr int F = TOR_NFEAT, H1 = TOR_MLP_H1, H2 = TOR_MLP_H2;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + H1 * F, OFF_W2 = OFF_B1 + H1, OFF_B2 = OFF_W2 + H2 * H1,
              OFF_W3 = OFF_B2 + H2, OFF_B3 = OFF_W3 + H2, NPARAM = OFF_B3 + 1;
static_assert(NPARAM == TOR_MLP_PARAMS, "parameter layout");

__device__ inline void mlp_fwd_one(const double* __restrict__ th, const double* x, double* h1,
                                   double* h2, double& out) {
  for (int o = 0; o < H1; ++o) {
    double z = th[OFF_B1 + o];
    for (int i = 0; i < F; ++i) z = fma(th[OFF_W1 + o * F + i], x[i], z);
    h1[o] = tanh(z);
  }
  for (int o = 0; o < H2; ++o) {
    double z = th[OFF_B2 + o];
    for (int i = 0; i < H1; ++i) z = fma(th[OFF_W2 + o * H1 + i], h1[i], z);
    h2[o] = tanh(z);
  }
  double z = th[OFF_B3];
  for (int i = 0; i < H2; ++i) z = fma(th[OFF_W3 + i], h2[i], z);
  out = z;
}

__global__ void mlp_forward_kernel(const double* __restrict__ th, const double* __restrict__ mean,
                                   const double* __restrict__ sd, const double* __restrict__ X,
                                   int B, double* __restrict__ Y) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double x[F], h1[H1], h2[H2], out;
  for (int i = 0; i < F; ++i) x[i] = (X[(size_t)b * F + i] - mean[i]) / sd[i];
  mlp_fwd_one(th, x, h1, h2, out);
  Y[b] = out;
}

// Per-sample gradient of the mean loss over the B samples, kind 0: the
// asymmetric squared loss
//   L = (1/B) sum_b w_b (y_b - pred_b)^2,  w_b = under if y_b > pred_b else over;
// kind 1: the quantile (pinball) loss at level q = under
//   L = (1/B) sum_b max(q r_b, (q - 1) r_b),  r_b = y_b - pred_b,
// whose minimiser is the q-quantile of y given the features.
__global__ void mlp_sample_grad_kernel(const double* __restrict__ th, const double* __restrict__ mean,
                                       const double* __restrict__ sd, const double* __restrict__ X,
                                       const double* __restrict__ y, int B, int kind, double under,
                                       double over, double* __restrict__ G,
                                       double* __restrict__ lossb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double x[F], h1[H1], h2[H2], out;
  for (int i = 0; i < F; ++i) x[i] = (X[(size_t)b * F + i] - mean[i]) / sd[i];
  mlp_fwd_one(th, x, h1, h2, out);
  const double err = y[b] - out;
  double d3;  // dL/dout
  if (kind == 0) {
    const double w = err > 0.0 ? under : over;
    lossb[b] = w * err * err / B;
    d3 = -2.0 * w * err / B;
  } else {
    const double q = under;
    lossb[b] = (err > 0.0 ? q * err : (q - 1.0) * err) / B;
    d3 = (err > 0.0 ? -q : 1.0 - q) / B;
  }
  double* g = G + (size_t)b * NPARAM;
  g[OFF_B3] = d3;
  double d2[H2];
  for (int i = 0; i < H2; ++i) {
    g[OFF_W3 + i] = d3 * h2[i];
    d2[i] = d3 * th[OFF_W3 + i] * (1.0 - h2[i] * h2[i]);
  }
  for (int o = 0; o < H2; ++o) {
    g[OFF_B2 + o] = d2[o];
    for (int i = 0; i < H1; ++i) g[OFF_W2 + o * H1 + i] = d2[o] * h1[i];
  }
  for (int i = 0; i < H1; ++i) {
    double s = 0.0;
    for (int o = 0; o < H2; ++o) s = fma(d2[o], th[OFF_W2 + o * H1 + i], s);
    const double d1 = s * (1.0 - h1[i] * h1[i]);
    g[OFF_B1 + i] = d1;
    for (int k = 0; k < F; ++k) g[OFF_W1 + i * F + k] = d1 * x[k];
  }
}

// grad[p] = sum_b G[b][p], in increasing b; loss = sum_b lossb[b] likewise.
__global__ void mlp_reduce_kernel(const double* __restrict__ G, const double* __restrict__ lossb,
                                  int B, double* __restrict__ grad, double* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NPARAM) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += G[(size_t)b * NPARAM + p];
    grad[p] = s;
  } else if (p == NPARAM && loss) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += lossb[b];
    *loss = s;
  }
}

__global__ void adam_kernel(double* __restrict__ th, const double* __restrict__ grad,
                            double* __restrict__ m, double* __restrict__ v, double lr, double b1,
                            double b2, double eps, int step) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const double g = grad[p];
  const double mm = b1 * m[p] + (1.0 - b1) * g;
  const double vv = b2 * v[p] + (1.0 - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  const double mh = mm / (1.0 - pow(b1, (double)step));
  const double vh = vv / (1.0 - pow(b2, (double)step));
  th[p] -= lr * mh / (sqrt(vh) + eps);
}

hipError_t launch_mlp_forward(const double* th, const double* mean, const double* sd,
                              const double* X, int B, double* Y, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((B + 63) / 64), dim3(64), 0, s, th, mean, sd, X, B, Y);
  return hipGetLastError();
}

// Rows idx[0..B) of X (F columns) gathered into out (B x F).
__global__ void gather_rows_kernel(const double* __restrict__ X, const int32_t* __restrict__ idx, int B,
                                   double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * F) return;
  const int b = e / F, i = e - b * F;
  out[e] = X[(size_t)idx[b] * F + i];
}

__global__ void gather_vals_kernel(const double* __restrict__ y, const int32_t* __restrict__ idx, int B,
                                   double* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) out[b] = y[idx[b]];
}

hipError_t launch_gather_samples(const double* X, const double* y, const int32_t* idx, int B, double* Xo,
                                 double* yo, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_rows_kernel, dim3((B * F + 255) / 256), dim3(256), 0, s, X, idx, B, Xo);
  hipLaunchKernelGGL(gather_vals_kernel, dim3((B + 255) / 256), dim3(256), 0, s, y, idx, B, yo);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const double* th, const double* mean, const double* sd, const double* X,
                           const double* y, int B, int kind, double under, double over, double* G,
                           double* lossb, double* grad, double* loss, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_sample_grad_kernel, dim3((B + 63) / 64), dim3(64), 0, s, th, mean, sd, X, y,
                     B, kind, under, over, G, lossb);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((NPARAM + 1 + 255) / 256), dim3(256), 0, s, G, lossb, B,
                     grad, loss);
  return hipGetLastError();
}

hipError_t launch_adam(double* th, const double* grad, double* m, double* v, double lr, double b1,
                       double b2, double eps, int step, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, s, th, grad, m, v, lr,
                     b1, b2, eps, step);
  return hipGetLastError();
}

}  // namespace tor

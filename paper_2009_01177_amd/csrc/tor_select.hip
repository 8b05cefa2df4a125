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
// Q = R^-1 (sigma_Q in the same basis) where it fits beside R.
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

__device__ inline double r_entry(const double2* O, int64_t ld, int n, int r, int c) {
  const int i = r >> 1, j = c >> 1, qi = r & 1, qj = c & 1;
  const double xr = o_lower(O, ld, i, j, false), xi = o_lower(O, ld, i, j, true);
  const double yr = o_lower(O, ld, i, j + n, false), yi = o_lower(O, ld, i, j + n, true);
  const double dlt = (i == j && qi == qj) ? 1.0 : 0.0;
  if (qi == 0 && qj == 0) return (dlt - xr) - yr;
  if (qi == 0 && qj == 1) return xi - yi;
  if (qi == 1 && qj == 0) return -xi - yi;
  return (dlt - xr) + yr;
}

// det of the 4x4 symmetric block of modes (i, j) of a full N2 x N2 matrix,
// by elimination without pivoting
__device__ inline double det_pair(const double* R, int N2, int i, int j) {
  int idx[4] = {2 * i, 2 * i + 1, 2 * j, 2 * j + 1};
  double a[4][4];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) a[r][c] = R[idx[r] * N2 + idx[c]];
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

// sum of v[0..256) over the workgroup in a fixed order (every thread gets it)
__device__ inline double block_sum(double x, double* red) {
  const int tid = threadIdx.x;
  red[tid] = x;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double v = red[0];
  __syncthreads();
  return v;
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
// returns the same value.  cnt: 256 ints of LDS.
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
    cnt[tid] = sturm_count(al, be, k, lo + w * (tid + 1)) > j ? tid : 256;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
      if (tid < h) cnt[tid] = min(cnt[tid], cnt[tid + h]);
      __syncthreads();
    }
    const int t = cnt[0];  // first point above eigenvalue j (256: none)
    __syncthreads();
    const double nlo = lo + w * t, nhi = t < 256 ? lo + w * (t + 1) : hi;
    lo = nlo;
    hi = nhi;
  }
  return 0.5 * (lo + hi);
}

__global__ __launch_bounds__(256) void features_kernel(const double2* __restrict__ Obase,
                                                       const int64_t* __restrict__ offs,
                                                       const int32_t* __restrict__ ns, int nq,
                                                       double* __restrict__ feats) {
  extern __shared__ double sh[];
  const int inst = blockIdx.x;
  const int n = ns[inst];
  const int N2 = 2 * n;
  const int64_t ld = 2 * n;
  const double2* O = Obase + offs[inst];
  double* R = sh;                   // N2 x N2
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
  double* Q = tq + n + npairs;      // N2 x N2 (instances of up to nq modes)
  const bool with_q = n <= nq;
  const int tid = threadIdx.x;
  for (int e = tid; e < N2 * N2; e += 256) R[e] = r_entry(O, ld, n, e / N2, e % N2);
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
    // p -> (i, j), i < j, lexicographic
    int i = 0, rem = p;
    while (rem >= n - 1 - i) {
      rem -= n - 1 - i;
      ++i;
    }
    const int j = i + 1 + rem;
    const double dij = det_pair(R, N2, i, j);
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
  for (int j = 0; j < ksteps; ++j) {
    double part = 0.0;
    for (int r = tid; r < N2; r += 256) {
      double s = 0.0;
      for (int c = 0; c < N2; ++c) s = fma(R[r * N2 + c], vc[c], s);
      wv[r] = s;
      part = fma(s, vc[r], part);
    }
    const double a = block_sum(part, red);
    const double bprev = j > 0 ? be[j - 1] : 0.0;
    part = 0.0;
    for (int r = tid; r < N2; r += 256) {
      const double w = wv[r] - a * vc[r] - bprev * vp[r];
      wv[r] = w;
      part = fma(w, w, part);
    }
    const double b = sqrt(block_sum(part, red));
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
  // Cholesky of R in place, unscaled (R = L D L^T: piv = D, the eliminated
  // column below the pivot is D_j L_rj)
  for (int j = 0; j < N2; ++j) {
    const double d = R[j * N2 + j];
    if (tid == 0) piv[j] = d;
    __syncthreads();
    const double rd = 1.0 / d;
    for (int e = tid; e < (N2 - j - 1) * (N2 - j - 1); e += 256) {
      const int r = j + 1 + e / (N2 - j - 1), c = j + 1 + e % (N2 - j - 1);
      if (c <= r) R[r * N2 + c] -= R[r * N2 + j] * R[c * N2 + j] * rd;
    }
    __syncthreads();
  }
  // Q = R^-1, one column per thread: L y = e_c, then L^T x = D^-1 y, with
  // the unit lower factor L formed in place first (column j of the
  // eliminated part over its pivot) and the pivots' reciprocals kept in wv
  if (with_q) {
    for (int j = tid; j < N2; j += 256) wv[j] = 1.0 / piv[j];
    __syncthreads();
    for (int e = tid; e < N2 * N2; e += 256) {
      const int r = e / N2, c = e - r * N2;
      if (r > c) R[e] *= wv[c];
    }
    __syncthreads();
    for (int c = tid; c < N2; c += 256) {
      double* x = Q;  // column c of Q: Q[i * N2 + c]
      for (int i = 0; i < N2; ++i) {
        double y = (i == c) ? 1.0 : 0.0;
        for (int j = c; j < i; ++j) y = fma(-R[i * N2 + j], x[j * N2 + c], y);
        x[i * N2 + c] = i < c ? 0.0 : y;
      }
      for (int i = N2 - 1; i >= 0; --i) {
        double z = x[i * N2 + c] * wv[i];
        for (int j = i + 1; j < N2; ++j) z = fma(-R[j * N2 + i], x[j * N2 + c], z);
        x[i * N2 + c] = z;
      }
    }
    __syncthreads();
    // the top levels' term ratios, one mode or pair per thread
    for (int k = tid; k < n; k += 256) {
      const double* Qk = Q + (2 * k) * N2 + 2 * k;
      tq[k] = 1.0 / sqrt(Qk[0] * Qk[N2 + 1] - Qk[N2] * Qk[N2]);
    }
    for (int p = tid; p < npairs; p += 256) {
      int i = 0, rem = p;
      while (rem >= n - 1 - i) {
        rem -= n - 1 - i;
        ++i;
      }
      tq[n + p] = 1.0 / sqrt(det_pair(Q, N2, i, i + 1 + rem));
    }
    __syncthreads();
  }
  // extreme Ritz values (all threads take part in the multisection)
  const double ritz_lo = tridiag_eig(al, be, kdone, 0, (int*)red);
  const double ritz_hi = tridiag_eig(al, be, kdone, kdone - 1, (int*)red);
  if (tid == 0) {
    double logdet = 0.0, pmin = piv[0], pmax = piv[0];
    for (int j = 0; j < N2; ++j) {
      logdet += log(piv[j]);
      pmin = fmin(pmin, piv[j]);
      pmax = fmax(pmax, piv[j]);
    }
    double f2 = 0.0, f3 = 0.0, qmax = q[0], qmin = q[0], asum = 0.0;
    for (int k = 0; k < n; ++k) {
      f2 += log((1.0 + q[k]) / (1.0 - q[k]));
      f3 += -log(q[k]);
      qmax = fmax(qmax, q[k]);
      qmin = fmin(qmin, q[k]);
      asum += O[(int64_t)k * ld + k].x;
    }
    double f6 = 0.0, pt = 0.0;
    for (int p = 0; p < npairs; ++p) {
      f6 += pr[2 * p];
      pt += pr[2 * p + 1];
    }
    double glo = gl[0], ghi = gl[N2];
    for (int r = 1; r < N2; ++r) {
      glo = fmin(glo, gl[r]);
      ghi = fmax(ghi, gl[N2 + r]);
    }
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
    if (with_q) {
      double s1 = 0.0, m1 = 0.0;
      for (int k = 0; k < n; ++k) {
        s1 += tq[k];
        m1 = fmax(m1, tq[k]);
      }
      double s2 = 0.0, m2 = 0.0;
      for (int p = 0; p < npairs; ++p) {
        s2 += tq[n + p];
        m2 = fmax(m2, tq[n + p]);
      }
      f[16] = log(s1 / n);
      f[17] = log(m1);
      f[18] = npairs > 0 ? log(s2 / npairs) : 0.0;
      f[19] = npairs > 0 ? log(m2) : 0.0;
    } else {
      const double nan = __builtin_nan("");
      f[16] = f[17] = f[18] = f[19] = nan;
    }
  }
}

// LDS of the features kernel for instances of up to nmax modes, with or
// without the inverse Q.
size_t features_lds_bytes(int nmax, bool with_q) {
  const size_t N2 = 2 * (size_t)nmax;
  const size_t base = N2 * N2 + N2 + nmax + (size_t)nmax * (nmax - 1) + 256 + 3 * N2 + 2 * LANCZOS_STEPS + 2 * N2 +
                      nmax + (size_t)nmax * (nmax - 1) / 2;
  return sizeof(double) * (base + (with_q ? N2 * N2 : 0));
}

constexpr size_t FEATURES_LDS_MAX = 160 * 1024;

// Largest n whose instances get Q beside R (the top-level features f16..f19).
int features_nq() {
  int nq = 0;
  while (nq < TOR_NMAX && features_lds_bytes(nq + 1, true) <= FEATURES_LDS_MAX) ++nq;
  return nq;
}

size_t features_lds_bytes(int nmax) {
  const int nq = features_nq();
  const size_t a = features_lds_bytes(nmax < nq ? nmax : nq, true), b = features_lds_bytes(nmax, false);
  return a > b ? a : b;
}

hipError_t launch_features(const double2* O, const int64_t* offs, const int32_t* ns, int batch,
                           int nmax, double* feats, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  const size_t lds = features_lds_bytes(nmax);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&features_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(features_kernel, dim3(batch), dim3(256), lds, s, O, offs, ns, features_nq(), feats);
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

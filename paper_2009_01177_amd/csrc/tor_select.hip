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
// quadrature form of I - O (rows interleaved per mode), full square in LDS.
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
// --------------------------------------------------------------------------

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

// det of the 4x4 symmetric block of modes (i, j) by Cholesky
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
  double* R = sh;                   // N2 x N2
  double* piv = R + N2 * N2;        // N2
  double* q = piv + N2;             // n
  double* pr = q + n;               // 2 * npairs: log ratio, det^(-1/2)
  const int npairs = n * (n - 1) / 2;
  const int tid = threadIdx.x;
  for (int e = tid; e < N2 * N2; e += 256) R[e] = r_entry(O, ld, n, e / N2, e % N2);
  __syncthreads();
  for (int k = tid; k < n; k += 256) {
    const double d = R[(2 * k) * N2 + 2 * k] * R[(2 * k + 1) * N2 + 2 * k + 1] -
                     R[(2 * k + 1) * N2 + 2 * k] * R[(2 * k + 1) * N2 + 2 * k];
    q[k] = sqrt(d);
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
  __syncthreads();
  // Cholesky of R in place (pivots only are kept)
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
  }
}

size_t features_lds_bytes(int nmax) {
  const int N2 = 2 * nmax;
  return sizeof(double) * ((size_t)N2 * N2 + N2 + nmax + (size_t)nmax * (nmax - 1));
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

// Per-sample gradient of the mean asymmetric squared loss
//   L = (1/B) sum_b w_b (y_b - pred_b)^2,  w_b = under if y_b > pred_b else over.
__global__ void mlp_sample_grad_kernel(const double* __restrict__ th, const double* __restrict__ mean,
                                       const double* __restrict__ sd, const double* __restrict__ X,
                                       const double* __restrict__ y, int B, double under,
                                       double over, double* __restrict__ G,
                                       double* __restrict__ lossb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double x[F], h1[H1], h2[H2], out;
  for (int i = 0; i < F; ++i) x[i] = (X[(size_t)b * F + i] - mean[i]) / sd[i];
  mlp_fwd_one(th, x, h1, h2, out);
  const double err = y[b] - out;
  const double w = err > 0.0 ? under : over;
  lossb[b] = w * err * err / B;
  double* g = G + (size_t)b * NPARAM;
  const double d3 = -2.0 * w * err / B;  // dL/dout
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

hipError_t launch_mlp_grad(const double* th, const double* mean, const double* sd, const double* X,
                           const double* y, int B, double under, double over, double* G,
                           double* lossb, double* grad, double* loss, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_sample_grad_kernel, dim3((B + 63) / 64), dim3(64), 0, s, th, mean, sd, X, y,
                     B, under, over, G, lossb);
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

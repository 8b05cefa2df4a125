// tor_train.cpp -- labelling and training of the learned precision selector
// (the C ABI's tor_selector_label / tor_selector_train): the labels come
// from the library's own evaluations, the network is trained by its own
// kernels (per-sample gradients, fixed-order sums, Adam), and the per-tier
// error model is calibrated on the host.  The paper fixes its precision once
// per run from bounds (Sec. 5.4, Eq. 5-7); this selector chooses per
// instance and keeps the bound estimate as its fallback.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/tor.h"
#include "prec.hpp"
#include "tor_internal.hpp"

namespace tor {
namespace {

inline int hip_rc(hipError_t e) { return e == hipSuccess ? TOR_OK : (e == hipErrorOutOfMemory ? TOR_ENOMEM : TOR_EHIP); }

#define TT_TRY(expr)                  \
  do {                                \
    int rc__ = (expr);                \
    if (rc__ != TOR_OK) return rc__;  \
  } while (0)
#define TT_HIP(expr) TT_TRY(hip_rc(expr))

constexpr double LOG10_2 = 0.30102999566398120;
constexpr double KAPPA_CAP = 60.0;  // log10 kappa when Tor is exactly 0

double unit_log10(int t) { return -(t == TOR_FP64 ? 53.0 : (t == TOR_DD ? 104.0 : 208.0)) * LOG10_2; }

// a tor_result_t's value as a quad-double (the FP64 and DD tiers fill two words)
prec::qd value_of(const tor_result_t& r) { return prec::qd{{r.tor[0], r.tor[1], r.tor[2], r.tor[3]}}; }

// splitmix64: seeds, minibatch order and the initial weights
struct Rng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }  // [0, 1)
  double normal() {                                                // Box-Muller
    double u1 = uniform();
    while (u1 <= 0.0) u1 = uniform();
    const double u2 = uniform();
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
};

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  int alloc(size_t bytes) { return hip_rc(hipMalloc(&p, bytes)); }
  template <class T>
  T* as() const {
    return (T*)p;
  }
};

}  // namespace
}  // namespace tor

using namespace tor;

extern "C" {

int tor_selector_label(const void* O_packed, const int64_t* offsets, const int32_t* n, int32_t count,
                       int32_t ref_tier, void* stream, double* labels) {
  if (count < 0 || !labels || (ref_tier != TOR_DD && ref_tier != TOR_QD)) return TOR_EINVAL;
  if (count == 0) return TOR_OK;
  if (!O_packed || !offsets || !n) return TOR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  // results: reference tier, FP64, and DD when QD is the reference
  const int nt = ref_tier == TOR_QD ? 3 : 2;
  DevBuf dres;
  TT_TRY(dres.alloc(sizeof(tor_result_t) * (size_t)count * nt));
  tor_result_t* res = dres.as<tor_result_t>();
  std::vector<int32_t> tiers((size_t)count);
  const int order[3] = {ref_tier, TOR_FP64, TOR_DD};
  for (int k = 0; k < nt; ++k) {
    std::fill(tiers.begin(), tiers.end(), order[k]);
    TT_TRY(tor_eval_batched(O_packed, offsets, n, count, tiers.data(), 1.0, nullptr, stream,
                            res + (size_t)k * count));
  }
  std::vector<tor_result_t> h((size_t)count * nt);
  TT_HIP(hipMemcpyAsync(h.data(), res, sizeof(tor_result_t) * h.size(), hipMemcpyDeviceToHost, s));
  TT_HIP(hipStreamSynchronize(s));
  const double nan = std::nan("");
  for (int i = 0; i < count; ++i) {
    double* L = labels + 4 * (size_t)i;
    L[0] = L[1] = L[2] = L[3] = nan;
    if (n[i] == 0) continue;
    const tor_result_t& rr = h[i];
    if (rr.status != TOR_OK) continue;
    const prec::qd tref = prec::qd_nonoverlapping(value_of(rr));
    const double aref = fabs(tref.x[0]);
    const double sabs = rr.abs_sum[0] + rr.abs_sum[1];
    L[0] = aref > 0.0 ? std::min(KAPPA_CAP, log10(sabs / aref)) : KAPPA_CAP;
    const double den = aref > 0.0 ? aref : sabs;
    for (int k = 1; k < nt; ++k) {
      const tor_result_t& rt = h[(size_t)k * count + i];
      if (rt.status != TOR_OK) continue;
      const int t = order[k];
      // |T_t - T_ref| exactly enough: the difference of the expansions in
      // quad-double, relative to |T_ref|; an error below a hundredth of the
      // tier's unit roundoff reads as that floor
      const prec::qd d = prec::qd_nonoverlapping(prec::qd_sub(value_of(rt), tref));
      const double e = fabs(d.x[0]) / den;
      L[1 + t] = std::max(e > 0.0 ? log10(e) : -400.0, unit_log10(t) - 2.0);
    }
  }
  return TOR_OK;
}

int tor_selector_train(const double* feats, const double* labels, const int32_t* n, int32_t count,
                       const tor_train_options_t* opt, void* stream, tor_selector_t* out, double* losses) {
  if (count < 1 || !feats || !labels || !n || !opt || !out) return TOR_EINVAL;
  if (opt->target != TOR_TARGET_KAPPA && opt->target != TOR_TARGET_ERR64) return TOR_EINVAL;
  if (opt->epochs < 1 || opt->batch_size < 1 || !(opt->lr > 0.0)) return TOR_EINVAL;
  if (opt->loss != TOR_LOSS_ASYM_SQUARED && opt->loss != TOR_LOSS_QUANTILE) return TOR_EINVAL;
  if (opt->loss == TOR_LOSS_QUANTILE && !(opt->quantile > 0.0 && opt->quantile < 1.0)) return TOR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  constexpr int F = TOR_NFEAT, P = TOR_MLP_PARAMS;
  // samples with a finite target (column 0: log10 kappa, 1: log10 FP64 error)
  const int col = opt->target == TOR_TARGET_KAPPA ? 0 : 1;
  std::vector<int32_t> keep;
  for (int i = 0; i < count; ++i) {
    bool ok = std::isfinite(labels[4 * (size_t)i + col]) && n[i] >= 1;
    for (int j = 0; j < F && ok; ++j) ok = std::isfinite(feats[(size_t)i * F + j]);
    if (ok) keep.push_back(i);
  }
  const int B = (int)keep.size();
  if (B < 2) return TOR_EINVAL;
  std::vector<double> X((size_t)B * F), y(B);
  for (int b = 0; b < B; ++b) {
    memcpy(&X[(size_t)b * F], feats + (size_t)keep[b] * F, sizeof(double) * F);
    y[b] = labels[4 * (size_t)keep[b] + col];
  }
  // standardisation, sample order
  double mean[F], sd[F], fmin[F], fmax[F];
  for (int j = 0; j < F; ++j) {
    double m = 0.0;
    for (int b = 0; b < B; ++b) m += X[(size_t)b * F + j];
    m /= B;
    double v = 0.0;
    fmin[j] = fmax[j] = X[j];
    for (int b = 0; b < B; ++b) {
      const double d = X[(size_t)b * F + j] - m;
      v += d * d;
      fmin[j] = std::min(fmin[j], X[(size_t)b * F + j]);
      fmax[j] = std::max(fmax[j], X[(size_t)b * F + j]);
    }
    mean[j] = m;
    sd[j] = sqrt(v / B);
    if (sd[j] < 1e-12) sd[j] = 1.0;
  }
  // initial weights: normal with standard deviation 1/sqrt(fan in), biases 0
  Rng rng{opt->seed * 0x2545f4914f6cdd1dull + 1};
  std::vector<double> th(P, 0.0);
  {
    const int sizes[4] = {F, TOR_MLP_H1, TOR_MLP_H2, 1};
    size_t off = 0;
    for (int l = 0; l < 3; ++l) {
      const int fi = sizes[l], fo = sizes[l + 1];
      for (int e = 0; e < fo * fi; ++e) th[off + e] = rng.normal() / sqrt((double)fi);
      off += (size_t)fo * fi + fo;
    }
  }
  const int bs = std::min(opt->batch_size, B);
  const int nb = (B + bs - 1) / bs;
  // device: X, y, theta, m, v, grad, minibatch X and y, order, per-sample
  // gradients and losses, per-step losses, predictions, mean, std
  const size_t steps = (size_t)opt->epochs * nb;
  DevBuf d;
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return o;
  };
  const size_t oX = carve(sizeof(double) * X.size()), oy = carve(sizeof(double) * B);
  const size_t oth = carve(sizeof(double) * P), om = carve(sizeof(double) * P), ov = carve(sizeof(double) * P);
  const size_t og = carve(sizeof(double) * P), oXb = carve(sizeof(double) * bs * F), oyb = carve(sizeof(double) * bs);
  const size_t oidx = carve(sizeof(int32_t) * B), oG = carve(sizeof(double) * (size_t)bs * P);
  const size_t olb = carve(sizeof(double) * bs), olos = carve(sizeof(double) * steps);
  const size_t opred = carve(sizeof(double) * B), omean = carve(sizeof(double) * F), osd = carve(sizeof(double) * F);
  TT_TRY(d.alloc(off));
  char* base = d.as<char>();
  auto dp = [&](size_t o) { return (double*)(base + o); };
  TT_HIP(hipMemcpyAsync(dp(oX), X.data(), sizeof(double) * X.size(), hipMemcpyHostToDevice, s));
  TT_HIP(hipMemcpyAsync(dp(oy), y.data(), sizeof(double) * B, hipMemcpyHostToDevice, s));
  TT_HIP(hipMemcpyAsync(dp(oth), th.data(), sizeof(double) * P, hipMemcpyHostToDevice, s));
  TT_HIP(hipMemcpyAsync(dp(omean), mean, sizeof(double) * F, hipMemcpyHostToDevice, s));
  TT_HIP(hipMemcpyAsync(dp(osd), sd, sizeof(double) * F, hipMemcpyHostToDevice, s));
  TT_HIP(hipMemsetAsync(dp(om), 0, sizeof(double) * P, s));
  TT_HIP(hipMemsetAsync(dp(ov), 0, sizeof(double) * P, s));
  const int kind = opt->loss == TOR_LOSS_QUANTILE ? 1 : 0;
  const double a1 = kind == 1 ? opt->quantile : opt->under, a2 = kind == 1 ? 0.0 : opt->over;
  std::vector<int32_t> perm(B);
  int step = 0;
  for (int ep = 0; ep < opt->epochs; ++ep) {
    for (int b = 0; b < B; ++b) perm[b] = b;
    for (int b = B - 1; b > 0; --b) std::swap(perm[b], perm[(size_t)(rng.next() % (uint64_t)(b + 1))]);
    // the order of this epoch goes up behind the previous epoch's steps
    TT_HIP(hipMemcpyAsync(base + oidx, perm.data(), sizeof(int32_t) * B, hipMemcpyHostToDevice, s));
    for (int i = 0; i < B; i += bs) {
      const int cnt = std::min(bs, B - i);
      TT_HIP(launch_gather_samples(dp(oX), dp(oy), (const int32_t*)(base + oidx) + i, cnt, dp(oXb), dp(oyb), s));
      TT_HIP(launch_mlp_grad(dp(oth), dp(omean), dp(osd), dp(oXb), dp(oyb), cnt, kind, a1, a2, dp(oG), dp(olb),
                             dp(og), dp(olos) + step, s));
      ++step;
      TT_HIP(launch_adam(dp(oth), dp(og), dp(om), dp(ov), opt->lr, opt->beta1, opt->beta2, opt->eps, step, s));
    }
    // the host copy of the order is rewritten next epoch: wait for the upload
    TT_HIP(hipStreamSynchronize(s));
  }
  TT_HIP(launch_mlp_forward(dp(oth), dp(omean), dp(osd), dp(oX), B, dp(opred), s));
  std::vector<double> pred(B), sl(steps);
  TT_HIP(hipMemcpyAsync(th.data(), dp(oth), sizeof(double) * P, hipMemcpyDeviceToHost, s));
  TT_HIP(hipMemcpyAsync(pred.data(), dp(opred), sizeof(double) * B, hipMemcpyDeviceToHost, s));
  TT_HIP(hipMemcpyAsync(sl.data(), dp(olos), sizeof(double) * steps, hipMemcpyDeviceToHost, s));
  TT_HIP(hipStreamSynchronize(s));
  if (losses) {
    // mean loss per epoch: each step's mean loss weighted by its sample count
    for (int ep = 0; ep < opt->epochs; ++ep) {
      double tot = 0.0;
      for (int k = 0; k < nb; ++k) {
        const int cnt = std::min(bs, B - k * bs);
        tot += sl[(size_t)ep * nb + k] * cnt;
      }
      losses[ep] = tot / B;
    }
  }
  // error model per tier, calibrated on the training samples
  tor_selector_t sel;
  memset(&sel, 0, sizeof(sel));
  memcpy(sel.theta, th.data(), sizeof(double) * P);
  memcpy(sel.mean, mean, sizeof(mean));
  memcpy(sel.std, sd, sizeof(sd));
  memcpy(sel.fmin, fmin, sizeof(fmin));
  memcpy(sel.fmax, fmax, sizeof(fmax));
  sel.nmin = TOR_NMAX;
  sel.nmax = 0;
  for (int b = 0; b < B; ++b) {
    sel.nmin = std::min(sel.nmin, (int32_t)n[keep[b]]);
    sel.nmax = std::max(sel.nmax, (int32_t)n[keep[b]]);
  }
  sel.target = opt->target;
  sel.margin = opt->margin;
  for (int t = TOR_FP64; t <= TOR_DD; ++t) {
    // residuals of the tier's measured error against the model, samples
    // with a measured error only
    std::vector<double> kap, lerr, pr;
    for (int b = 0; b < B; ++b) {
      const double* L = labels + 4 * (size_t)keep[b];
      if (!std::isfinite(L[1 + t])) continue;
      kap.push_back(L[0]);
      lerr.push_back(L[1 + t]);
      pr.push_back(pred[b]);
    }
    if (kap.empty()) {
      sel.log10_c[t] = t == TOR_FP64 ? 0.0 : sel.log10_c[TOR_FP64] + unit_log10(TOR_DD) - unit_log10(TOR_FP64);
      sel.slope[t] = 1.0;
      continue;
    }
    if (opt->target == TOR_TARGET_ERR64) {
      // log10 err_t <= prediction + c_t: the upper envelope of the residuals
      double c = -1e300;
      for (size_t k = 0; k < pr.size(); ++k) c = std::max(c, lerr[k] - pr[k]);
      sel.log10_c[t] = c + opt->slack;
      sel.slope[t] = 1.0;
    } else {
      // log10(err_t / u_t) <= c_t + s_t log10 kappa: for each slope in
      // [0.3, 1] the intercept is the upper envelope of the samples; keep the
      // slope whose envelope lies lowest on average over them
      double best_h = 1e300, best_c = 0.0, best_s = 1.0;
      for (int si = 0; si <= 70; ++si) {
        const double sl_ = 0.30 + 0.01 * si;
        double c = -1e300, h = 0.0;
        for (size_t k = 0; k < kap.size(); ++k) c = std::max(c, lerr[k] - unit_log10(t) - sl_ * kap[k]);
        for (size_t k = 0; k < kap.size(); ++k) h += c + sl_ * kap[k];
        h /= (double)kap.size();
        if (h < best_h) {
          best_h = h;
          best_c = c;
          best_s = sl_;
        }
      }
      sel.log10_c[t] = best_c + opt->slack;
      sel.slope[t] = best_s;
    }
  }
  // quad-double: double-double's model shifted by the ratio of the unit roundoffs
  sel.log10_c[TOR_QD] = sel.log10_c[TOR_DD] +
                        (opt->target == TOR_TARGET_ERR64 ? unit_log10(TOR_QD) - unit_log10(TOR_DD) : 0.0);
  sel.slope[TOR_QD] = sel.slope[TOR_DD];
  sel.trained = 1;
  *out = sel;
  return TOR_OK;
}

}  // extern "C"

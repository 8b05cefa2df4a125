// prec.hpp -- extended precision built from binary64 error-free transforms.
//
// The paper runs the Torontonian in 128- and 256-bit fixed point (Sec. 5.2,
// 5.3) because binary64 cannot hold the ~25 significant digits that the
// alternating sum needs (Sec. 5.1).  This library instead builds floating
// tiers on binary64 hardware, the same pairing Table 5 makes between the
// 128-bit tier and double-double (106 bits) and the 256-bit tier and
// quad-double (212 bits):
//
//   F64  plain binary64 with fused multiply-add;
//   DD   double-double  (hi + lo, |lo| <= ulp(hi)/2);
//   QD   quad-double    (x0 + x1 + x2 + x3, a non-overlapping expansion).
//
// Error-free transforms (round to nearest-even, no reassociation, no
// contraction: this file must be compiled with -ffp-contract=off and
// without fast-math):
//   two_sum       Knuth: s + e == a + b exactly.
//   fast_two_sum  Dekker: same, valid when |a| >= |b| or a == 0.
//   two_prod      p + e == a * b exactly, e = fma(a, b, -p).
//
// Double-double operations follow Joldes, Muller and Popescu, "Tight and
// rigorous error bounds for basic building blocks of double-word arithmetic"
// (ACM TOMS 2017): DWPlusFP, AccurateDWPlusDW, DWTimesFP (FMA form) and
// DWTimesDW (FMA form), with relative error bounds 2u^2, 3u^2 + 13u^3, 2u^2
// and 4u^2 (u = 2^-53).  Reciprocal, square root and reciprocal square root
// take one Newton step from the binary64 approximation with the residual
// formed in double-double.
//
// Quad-double values are kept as 4-term expansions.  Every operation forms
// an exact multi-term intermediate (with two_sum / two_prod) and compresses
// it back to four terms by repeated distillation: a bottom-up chain of
// two_sums yields the rounded total and the exact list of its rounding
// errors; the chain is run again on those errors to give the next term, and
// so on four times.  The value kept differs from the exact intermediate by
// about u^4 of the sum of the magnitudes involved.  This is branch-free,
// which suits 64-wide wavefronts.
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define PREC_HD __host__ __device__ __forceinline__
#else
#define PREC_HD inline
#endif

namespace prec {

// ---------------------------------------------------------------------------
// Error-free transforms
// ---------------------------------------------------------------------------

PREC_HD void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

PREC_HD void fast_two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  e = b - (s - a);
}

PREC_HD void two_prod(double a, double b, double& p, double& e) {
  p = a * b;
  e = fma(a, b, -p);
}

// ---------------------------------------------------------------------------
// Double-double
// ---------------------------------------------------------------------------

// 16-byte aligned, so that a value moves through LDS and memory as one
// 128-bit access
struct alignas(16) dd {
  double hi, lo;
};

PREC_HD dd dd_make(double x) { return dd{x, 0.0}; }

PREC_HD dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }

// DWPlusFP
PREC_HD dd dd_add_d(dd a, double b) {
  double sh, sl;
  two_sum(a.hi, b, sh, sl);
  double v = a.lo + sl;
  dd z;
  fast_two_sum(sh, v, z.hi, z.lo);
  return z;
}

// AccurateDWPlusDW
PREC_HD dd dd_add(dd x, dd y) {
  double sh, sl, th, tl;
  two_sum(x.hi, y.hi, sh, sl);
  two_sum(x.lo, y.lo, th, tl);
  double c = sl + th;
  double vh, vl;
  fast_two_sum(sh, c, vh, vl);
  double w = tl + vl;
  dd z;
  fast_two_sum(vh, w, z.hi, z.lo);
  return z;
}

PREC_HD dd dd_sub(dd x, dd y) { return dd_add(x, dd_neg(y)); }

// DWTimesFP (FMA form)
PREC_HD dd dd_mul_d(dd x, double y) {
  double ch, cl1;
  two_prod(x.hi, y, ch, cl1);
  double cl3 = fma(x.lo, y, cl1);
  dd z;
  fast_two_sum(ch, cl3, z.hi, z.lo);
  return z;
}

// DWTimesDW (FMA form)
PREC_HD dd dd_mul(dd x, dd y) {
  double ch, cl1;
  two_prod(x.hi, y.hi, ch, cl1);
  double tl0 = x.lo * y.lo;
  double tl1 = fma(x.hi, y.lo, tl0);
  double cl2 = fma(x.lo, y.hi, tl1);
  double cl3 = cl1 + cl2;
  dd z;
  fast_two_sum(ch, cl3, z.hi, z.lo);
  return z;
}

// Exact product of two binary64 values as a double-double.
PREC_HD dd dd_prod_dd(double a, double b) {
  dd z;
  two_prod(a, b, z.hi, z.lo);
  return z;
}

// 1/y: Newton step r1 = r0 + r0 (1 - y r0), residual in double-double.
PREC_HD dd dd_recip(dd y) {
  double r0 = 1.0 / y.hi;
  // e = 1 - y*r0: 1 - yh*r0 is exact through fma; subtract yl*r0.
  double eh = fma(-y.hi, r0, 1.0);
  double e = eh - y.lo * r0;
  dd z;
  fast_two_sum(r0, r0 * e, z.hi, z.lo);
  return z;
}

PREC_HD dd dd_div(dd x, dd y) {
  // q0 = x.hi / y.hi; remainder x - y*q0 in double-double; one correction.
  double q0 = x.hi / y.hi;
  dd p = dd_mul_d(y, q0);
  dd r = dd_sub(x, p);
  double q1 = r.hi / y.hi;
  dd z;
  fast_two_sum(q0, q1, z.hi, z.lo);
  return z;
}

// sqrt: s1 = s0 + (x - s0^2) / (2 s0), with s0^2 exact through two_prod.
PREC_HD dd dd_sqrt(dd x) {
  if (!(x.hi > 0.0)) return dd{x.hi == 0.0 ? 0.0 : sqrt(x.hi), 0.0};
  double s0 = sqrt(x.hi);
  double p, e;
  two_prod(s0, s0, p, e);
  double r = ((x.hi - p) - e) + x.lo;
  dd z;
  fast_two_sum(s0, r * (0.5 / s0), z.hi, z.lo);
  return z;
}

// Binary64 1/sqrt(a), within about 1.5 ulp.  On the device: the hardware
// estimate (v_rsq_f64) refined by one Newton step y + y (1 - a y^2) / 2, so
// the estimate's own error e leaves 1.5 e^2 + 1.5 u; on the host: the library
// square root and a division.  Not for a <= 0 (the callers test the pivot
// sign first).
PREC_HD double rsqrt_d(double a) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double y = __builtin_amdgcn_rsq(a);
  const double r = a * y;
  const double h = fma(-r, y, 1.0);
  return fma(0.5 * y, h, y);
#else
  return 1.0 / sqrt(a);
#endif
}

// 1/sqrt(x): y1 = y0 + y0 h / 2 with h = 1 - x y0^2.  x.hi y0 = r + re
// exactly (two_prod); h = 1 - r y0 - re y0 - x.lo y0^2 by three fmas, each
// rounding a value of the order of h ~ u, so h carries about 3 u^2 of
// absolute error; with the Newton term 1.5 e^2 of a seed error e the result
// is within about 7 u^2 (measured 6.8 u^2 worst over 1e5 arguments).
PREC_HD dd dd_rsqrt(dd x) {
  const double y0 = rsqrt_d(x.hi);
  const double r = x.hi * y0;
  const double re = fma(x.hi, y0, -r);
  double h = fma(-r, y0, 1.0);
  h = fma(-re, y0, h);
  h = fma(-(x.lo * y0), y0, h);
  dd z;
  fast_two_sum(y0, (0.5 * y0) * h, z.hi, z.lo);
  return z;
}

PREC_HD double dd_to_d(dd a) { return a.hi + a.lo; }

// Fused Schur-complement updates  t - a b  and  t - a b - c d.
//
// Composing DWTimesDW and AccurateDWPlusDW costs 29 binary64 operations per
// product-and-subtract.  These evaluate the whole expression at once: the
// leading products exactly (two_prod), their cross terms by fma, the
// leading parts  t.hi - p - q  exactly by a two_sum chain, every low-order
// piece (t.lo, cross terms, two_sum errors) summed in binary64 into l, and
// one final fast_two_sum(s, l).  With u = 2^-53 and inputs normalised
// (|x.lo| <= u |x.hi|), the low-order sum is within 4 u^2 of its exact
// value times the magnitudes and |l| <= 4 u (|t| + |a b| + |c d|); the final
// step is exact when |s| >= |l| and otherwise adds at most u |l| (this only
// happens when the result has cancelled to order u of the magnitudes).  The
// absolute error is at most
//     15 u^2 (|t| + |a b|)               (dd_fms)
//     26 u^2 (|t| + |a b| + |c d|)       (dd_fms2),
// against 7 u^2 and 14 u^2 for the composed JMP operations: the same
// u^2-times-magnitudes form that Cholesky's backward error already has, at
// 15 and 27 operations.  The dropped a.lo b.lo is part of the bound.
// (Over 4e5 random and cancelling cases: at most 3.3 u^2 and 4.0 u^2.)
PREC_HD dd dd_fms(dd t, dd a, dd b) {
  double p, pe;
  two_prod(a.hi, b.hi, p, pe);
  const double x = fma(a.lo, b.hi, fma(a.hi, b.lo, pe));
  double s, e;
  two_sum(t.hi, -p, s, e);
  const double l = (t.lo - x) + e;
  dd z;
  fast_two_sum(s, l, z.hi, z.lo);
  return z;
}

PREC_HD dd dd_fms2(dd t, dd a, dd b, dd c, dd d) {
  double p, pe, q, qe;
  two_prod(a.hi, b.hi, p, pe);
  two_prod(c.hi, d.hi, q, qe);
  const double x = fma(a.lo, b.hi, fma(a.hi, b.lo, pe));
  const double y = fma(c.lo, d.hi, fma(c.hi, d.lo, qe));
  double s1, e1, s, e2;
  two_sum(t.hi, -p, s1, e1);
  two_sum(s1, -q, s, e2);
  const double l = (((t.lo - x) - y) + e1) + e2;
  dd z;
  fast_two_sum(s, l, z.hi, z.lo);
  return z;
}

// ---------------------------------------------------------------------------
// Quad-double
// ---------------------------------------------------------------------------

struct alignas(16) qd {
  double x[4];
};

PREC_HD qd qd_make(double a) { return qd{{a, 0.0, 0.0, 0.0}}; }
PREC_HD qd qd_from_dd(dd a) { return qd{{a.hi, a.lo, 0.0, 0.0}}; }
PREC_HD qd qd_neg(qd a) { return qd{{-a.x[0], -a.x[1], -a.x[2], -a.x[3]}}; }

// One distillation pass over t[0..k-1] (k >= 1), largest-expected first:
// returns the rounded total; t[1..k-1] receive the exact rounding errors
// (t[0] is left unspecified).  sum(before) == total + sum(t[1..k-1]) exactly.
template <int K>
PREC_HD double distill(double* t) {
  double s = t[K - 1];
#pragma unroll
  for (int i = K - 2; i >= 0; --i) {
    double e;
    two_sum(t[i], s, s, e);
    t[i + 1] = e;
  }
  return s;
}

// Compress an exact K-term list into a 4-term expansion.
template <int K>
PREC_HD qd qd_compress(double* t) {
  qd r;
  r.x[0] = distill<K>(t);
  r.x[1] = distill<K - 1>(t + 1);
  r.x[2] = distill<K - 2>(t + 2);
  // the last term only needs the rounded total of what is left
  double s = 0.0;
#pragma unroll
  for (int i = K - 1; i >= 3; --i) s += t[i];
  r.x[3] = s;
  return r;
}

PREC_HD qd qd_add(qd a, qd b) {
  double t[8] = {a.x[0], b.x[0], a.x[1], b.x[1], a.x[2], b.x[2], a.x[3], b.x[3]};
  return qd_compress<8>(t);
}

PREC_HD qd qd_sub(qd a, qd b) { return qd_add(a, qd_neg(b)); }

// The words of a quad-double rewritten as a non-overlapping expansion with
// the same exact sum, largest first (zeros last): each word lies below the
// lowest set bit of the one before.  The arithmetic above keeps sums exact
// but, after heavy cancellation, may leave overlapping words; an output
// value is put in this form so that its leading word is within an ulp of
// the sum.  Shewchuk's Grow-Expansion ("Adaptive precision
// floating-point arithmetic", 1997): adding a double to a non-overlapping
// expansion by a chain of two_sums gives a non-overlapping expansion of the
// exact sum, components in increasing magnitude.
PREC_HD qd qd_nonoverlapping(qd a) {
  double e[4] = {a.x[3], 0.0, 0.0, 0.0};
  int m = 1;
  for (int k = 2; k >= 0; --k) {
    double q = a.x[k];
    for (int i = 0; i < m; ++i) {
      double h;
      two_sum(q, e[i], q, h);
      e[i] = h;
    }
    e[m++] = q;
  }
  qd z{{0.0, 0.0, 0.0, 0.0}};
  int j = 0;
  for (int i = 3; i >= 0; --i)
    if (e[i] != 0.0) z.x[j++] = e[i];
  return z;
}

PREC_HD qd qd_add_d(qd a, double b) {
  double t[5] = {a.x[0], b, a.x[1], a.x[2], a.x[3]};
  return qd_compress<5>(t);
}

PREC_HD qd qd_add_dd(qd a, dd b) {
  double t[6] = {a.x[0], b.hi, a.x[1], b.lo, a.x[2], a.x[3]};
  return qd_compress<6>(t);
}

PREC_HD qd qd_mul_d(qd a, double b) {
  double t[8];
  two_prod(a.x[0], b, t[0], t[1]);
  two_prod(a.x[1], b, t[2], t[3]);
  two_prod(a.x[2], b, t[4], t[5]);
  t[6] = a.x[3] * b;
  t[7] = 0.0;
  return qd_compress<7>(t);
}

PREC_HD qd qd_mul(qd a, qd b) {
  // products a_i b_j with i + j <= 2 exactly (two_prod), i + j == 3 rounded;
  // the dropped part is below u^4 of |a b|.
  double t[16];
  two_prod(a.x[0], b.x[0], t[0], t[1]);
  two_prod(a.x[0], b.x[1], t[2], t[4]);
  two_prod(a.x[1], b.x[0], t[3], t[5]);
  two_prod(a.x[0], b.x[2], t[6], t[9]);
  two_prod(a.x[1], b.x[1], t[7], t[10]);
  two_prod(a.x[2], b.x[0], t[8], t[11]);
  t[12] = a.x[0] * b.x[3];
  t[13] = a.x[1] * b.x[2];
  t[14] = a.x[2] * b.x[1];
  t[15] = a.x[3] * b.x[0];
  return qd_compress<16>(t);
}

// The terms of a b down to third order, largest-expected first: the exact
// products a_i b_j with i + j <= 2 (TwoProd: value and error), and one
// binary64 sum of everything of third order (the products with i + j == 3
// and the errors of the second-order products).  Their exact sum is a b up
// to about u^4 |a| |b| (the rounding of the third-order sum and the dropped
// fourth-order products).  s = +1 or -1 multiplies every term (exact).
PREC_HD void qd_prod_terms(qd a, qd b, double s, double* t) {
  double p00, e00, p01, e01, p10, e10, p02, e02, p11, e11, p20, e20;
  two_prod(a.x[0], b.x[0], p00, e00);
  two_prod(a.x[0], b.x[1], p01, e01);
  two_prod(a.x[1], b.x[0], p10, e10);
  two_prod(a.x[0], b.x[2], p02, e02);
  two_prod(a.x[1], b.x[1], p11, e11);
  two_prod(a.x[2], b.x[0], p20, e20);
  const double r3 = ((a.x[0] * b.x[3] + a.x[3] * b.x[0]) + (a.x[1] * b.x[2] + a.x[2] * b.x[1])) +
                    ((e02 + e11) + e20);
  t[0] = s * p00;
  t[1] = s * e00;
  t[2] = s * p01;
  t[3] = s * p10;
  t[4] = s * e01;
  t[5] = s * e10;
  t[6] = s * p02;
  t[7] = s * p11;
  t[8] = s * p20;
  t[9] = s * r3;
}

// a b from its ten terms: three distillation passes and a rounded remainder.
PREC_HD qd qd_mul_fast(qd a, qd b) {
  double t[10];
  qd_prod_terms(a, b, 1.0, t);
  return qd_compress<10>(t);
}

// Fused Schur updates in quad-double: t - a b and t - a b - c d as one
// compression of all their terms (the third-order tails of the products and
// t's last word summed in binary64 into one term), in place of a product
// compression followed by an addition compression each.  Error of the order
// of u^4 times |t| + |a b| (+ |c d|), the same form as the composed
// operations'; measured constants are in the tests.
PREC_HD qd qd_fms(qd t, qd a, qd b) {
  double p[10];
  qd_prod_terms(a, b, -1.0, p);
  // last: third order, t's last word and the product's tail
  double y[13] = {t.x[0], p[0], t.x[1], p[1], p[2], p[3], t.x[2], p[4], p[5], p[6], p[7], p[8],
                  t.x[3] + p[9]};
  return qd_compress<13>(y);
}

PREC_HD qd qd_fms2(qd t, qd a, qd b, qd c, qd d) {
  double p[10], q[10];
  qd_prod_terms(a, b, -1.0, p);
  qd_prod_terms(c, d, -1.0, q);
  double y[22] = {t.x[0], p[0], q[0], t.x[1], p[1], p[2], p[3], q[1], q[2], q[3], t.x[2],
                  p[4], p[5], p[6], p[7], p[8], q[4], q[5], q[6], q[7], q[8], 0.0};
  y[21] = (t.x[3] + p[9]) + q[9];
  return qd_compress<22>(y);
}

PREC_HD double qd_to_d(qd a) { return a.x[0] + (a.x[1] + (a.x[2] + a.x[3])); }

// 1/y by Newton from the double-double reciprocal: r <- r + r (1 - y r).
PREC_HD qd qd_recip(qd y) {
  dd r0 = dd_recip(dd{y.x[0], y.x[1]});
  qd r = qd_from_dd(r0);
  qd e = qd_add_d(qd_neg(qd_mul(y, r)), 1.0);
  return qd_add(r, qd_mul(r, e));
}

PREC_HD qd qd_div(qd x, qd y) { return qd_mul(x, qd_recip(y)); }

// 1/sqrt(x) by one Newton step from double-double, y <- y + y (1 - x y^2) / 2:
// y0 has two words, so y0^2 is exact as six terms (TwoProds of the words);
// x y0^2 is one quad-double product; h = 1 - x y0^2 is of order u^2 and
// accurate to about u^4, so the correction y0 h / 2 needs only a
// double-double product.
PREC_HD qd qd_rsqrt(qd x) {
  const dd y0 = dd_rsqrt(dd{x.x[0], x.x[1]});
  double t[6];
  two_prod(y0.hi, y0.hi, t[0], t[2]);
  two_prod(2.0 * y0.hi, y0.lo, t[1], t[3]);
  two_prod(y0.lo, y0.lo, t[4], t[5]);
  const qd y2 = qd_compress<6>(t);
  const qd h = qd_add_d(qd_neg(qd_mul_fast(x, y2)), 1.0);
  // h's words need not be normalised after that cancellation (its first
  // word is often exactly 0): add them up as a double-double
  const dd hd = dd_add_d(dd_add_d(dd_add_d(dd{h.x[0], 0.0}, h.x[1]), h.x[2]), h.x[3]);
  const dd c = dd_mul(y0, hd);
  return qd_add_dd(qd_from_dd(y0), dd{0.5 * c.hi, 0.5 * c.lo});
}

// sqrt(x) = x * rsqrt(x), then one Newton correction s + (x - s^2)/(2s).
PREC_HD qd qd_sqrt(qd x) {
  if (!(x.x[0] > 0.0)) return qd_make(x.x[0] == 0.0 ? 0.0 : sqrt(x.x[0]));
  qd r = qd_rsqrt(x);
  qd s = qd_mul(x, r);
  qd res = qd_add(x, qd_neg(qd_mul(s, s)));
  return qd_add(s, qd_mul_d(qd_mul(res, r), 0.5));
}

}  // namespace prec

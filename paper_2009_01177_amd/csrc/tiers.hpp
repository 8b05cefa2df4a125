// tiers.hpp -- device-side arithmetic for the three precision tiers, in one
// interface the kernels are templated on.
//
//   tier F64: values binary64, fused multiply-add; subset terms accumulated
//             in double-double.
//   tier DD : values double-double; terms accumulated in double-double.
//   tier QD : values quad-double; terms accumulated in quad-double.
//
// The staged input (-O in interleaved mode order) is binary64; entries of
// I - O off the diagonal are exactly -O, and the diagonal 1 - O_ii is formed
// exactly in DD and QD (two_sum) and rounded once in F64.
#pragma once

#include <hip/hip_runtime.h>

#include "prec.hpp"

namespace tor {

using prec::dd;
using prec::qd;

template <class R>
struct cx {
  R re, im;
};

// --------------------------------------------------------------------------
// Real operations per value type
// --------------------------------------------------------------------------

__device__ __forceinline__ double r_add(double a, double b) { return a + b; }
__device__ __forceinline__ double r_sub(double a, double b) { return a - b; }
__device__ __forceinline__ double r_mul(double a, double b) { return a * b; }
__device__ __forceinline__ double r_neg(double a) { return -a; }
__device__ __forceinline__ double r_from(double a) { return a; }
__device__ __forceinline__ double r_lead(double a) { return a; }
__device__ __forceinline__ double r_rsqrt(double a) { return prec::rsqrt_d(a); }
__device__ __forceinline__ double r_one_minus(double o) { return 1.0 - o; }
// c - a*b and c + a*b with one rounding
__device__ __forceinline__ double r_fms(double c, double a, double b) { return fma(-a, b, c); }
__device__ __forceinline__ double r_fma(double c, double a, double b) { return fma(a, b, c); }
// t - a*b - c*d (a Schur-update entry)
__device__ __forceinline__ double r_fms2(double t, double a, double b, double c, double d) {
  return fma(-c, d, fma(-a, b, t));
}

__device__ __forceinline__ dd r_add(dd a, dd b) { return prec::dd_add(a, b); }
__device__ __forceinline__ dd r_sub(dd a, dd b) { return prec::dd_sub(a, b); }
__device__ __forceinline__ dd r_mul(dd a, dd b) { return prec::dd_mul(a, b); }
__device__ __forceinline__ dd r_neg(dd a) { return prec::dd_neg(a); }
__device__ __forceinline__ double r_lead(dd a) { return a.hi; }
__device__ __forceinline__ dd r_rsqrt(dd a) { return prec::dd_rsqrt(a); }
__device__ __forceinline__ dd r_fms(dd c, dd a, dd b) { return prec::dd_fms(c, a, b); }
__device__ __forceinline__ dd r_fma(dd c, dd a, dd b) { return prec::dd_fms(c, prec::dd_neg(a), b); }
__device__ __forceinline__ dd r_fms2(dd t, dd a, dd b, dd c, dd d) { return prec::dd_fms2(t, a, b, c, d); }

__device__ __forceinline__ qd r_add(qd a, qd b) { return prec::qd_add(a, b); }
__device__ __forceinline__ qd r_sub(qd a, qd b) { return prec::qd_sub(a, b); }
__device__ __forceinline__ qd r_mul(qd a, qd b) { return prec::qd_mul_fast(a, b); }
__device__ __forceinline__ qd r_neg(qd a) { return prec::qd_neg(a); }
__device__ __forceinline__ double r_lead(qd a) { return a.x[0]; }
__device__ __forceinline__ qd r_rsqrt(qd a) { return prec::qd_rsqrt(a); }
__device__ __forceinline__ qd r_fms(qd c, qd a, qd b) { return prec::qd_fms(c, a, b); }
__device__ __forceinline__ qd r_fma(qd c, qd a, qd b) { return prec::qd_fms(c, prec::qd_neg(a), b); }
__device__ __forceinline__ qd r_fms2(qd t, qd a, qd b, qd c, qd d) { return prec::qd_fms2(t, a, b, c, d); }

template <class R>
__device__ __forceinline__ R r_zero();
template <>
__device__ __forceinline__ double r_zero<double>() { return 0.0; }
template <>
__device__ __forceinline__ dd r_zero<dd>() { return dd{0.0, 0.0}; }
template <>
__device__ __forceinline__ qd r_zero<qd>() { return qd{{0.0, 0.0, 0.0, 0.0}}; }

template <class R>
__device__ __forceinline__ R r_of(double x);
template <>
__device__ __forceinline__ double r_of<double>(double x) { return x; }
template <>
__device__ __forceinline__ dd r_of<dd>(double x) { return dd{x, 0.0}; }
template <>
__device__ __forceinline__ qd r_of<qd>(double x) { return qd{{x, 0.0, 0.0, 0.0}}; }

// 1 - o, exact in DD and QD
template <class R>
__device__ __forceinline__ R r_one_minus_t(double o);
template <>
__device__ __forceinline__ double r_one_minus_t<double>(double o) { return 1.0 - o; }
template <>
__device__ __forceinline__ dd r_one_minus_t<dd>(double o) {
  dd z;
  prec::two_sum(1.0, -o, z.hi, z.lo);
  return z;
}
template <>
__device__ __forceinline__ qd r_one_minus_t<qd>(double o) {
  double s, e;
  prec::two_sum(1.0, -o, s, e);
  return qd{{s, e, 0.0, 0.0}};
}

// --------------------------------------------------------------------------
// Complex helpers
// --------------------------------------------------------------------------

template <class R>
__device__ __forceinline__ cx<R> c_of(double re, double im) {
  return cx<R>{r_of<R>(re), r_of<R>(im)};
}

template <class R>
__device__ __forceinline__ cx<R> c_conj(cx<R> a) {
  return cx<R>{a.re, r_neg(a.im)};
}

// c - a*b
template <class R>
__device__ __forceinline__ cx<R> c_fms(cx<R> c, cx<R> a, cx<R> b) {
  cx<R> z;
  z.re = r_fma(r_fms(c.re, a.re, b.re), a.im, b.im);
  z.im = r_fms(r_fms(c.im, a.re, b.im), a.im, b.re);
  return z;
}

template <class R>
__device__ __forceinline__ cx<R> c_scale(cx<R> a, R s) {
  return cx<R>{r_mul(a.re, s), r_mul(a.im, s)};
}

// |a|^2
template <class R>
__device__ __forceinline__ R c_abs2(cx<R> a) {
  return r_fma(r_mul(a.re, a.re), a.im, a.im);
}

// conj(a) * b
template <class R>
__device__ __forceinline__ cx<R> c_conj_mul(cx<R> a, cx<R> b) {
  cx<R> z;
  z.re = r_fma(r_mul(a.re, b.re), a.im, b.im);
  z.im = r_fms(r_mul(a.re, b.im), a.im, b.re);
  return z;
}

// --------------------------------------------------------------------------
// Cross-lane moves (wave64)
// --------------------------------------------------------------------------

__device__ __forceinline__ double lane_bcast(double x, int lane) {
  // lane must be wave-uniform
  int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ dd lane_bcast(dd x, int lane) {
  return dd{lane_bcast(x.hi, lane), lane_bcast(x.lo, lane)};
}
__device__ __forceinline__ qd lane_bcast(qd x, int lane) {
  return qd{{lane_bcast(x.x[0], lane), lane_bcast(x.x[1], lane), lane_bcast(x.x[2], lane),
             lane_bcast(x.x[3], lane)}};
}
template <class R>
__device__ __forceinline__ cx<R> lane_bcast(cx<R> x, int lane) {
  return cx<R>{lane_bcast(x.re, lane), lane_bcast(x.im, lane)};
}

__device__ __forceinline__ double lane_xor(double x, int m) { return __shfl_xor(x, m, 64); }
__device__ __forceinline__ dd lane_xor(dd x, int m) { return dd{lane_xor(x.hi, m), lane_xor(x.lo, m)}; }
__device__ __forceinline__ qd lane_xor(qd x, int m) {
  return qd{{lane_xor(x.x[0], m), lane_xor(x.x[1], m), lane_xor(x.x[2], m), lane_xor(x.x[3], m)}};
}

// DPP moves within rows of 16 lanes; every lane has a source, so no bound
// control is needed.  CTRL: 0xB1 quad_perm [1,0,3,2], 0x4E quad_perm
// [2,3,0,1], 0x141 row_half_mirror, 0x140 row_mirror.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ dd dpp_mov(dd x) {
  return dd{dpp_mov<CTRL>(x.hi), dpp_mov<CTRL>(x.lo)};
}
template <int CTRL>
__device__ __forceinline__ qd dpp_mov(qd x) {
  return qd{{dpp_mov<CTRL>(x.x[0]), dpp_mov<CTRL>(x.x[1]), dpp_mov<CTRL>(x.x[2]), dpp_mov<CTRL>(x.x[3])}};
}

// Total over the 64 lanes in a fixed order: pairs, quads, groups of 8 and
// rows of 16 by DPP moves, then the four row totals read from lanes 0, 16,
// 32 and 48 and added as (r0 + r1) + (r2 + r3).  Every lane returns the same
// value.
template <class TT>
__device__ __forceinline__ typename TT::Acc wave_total(typename TT::Acc v) {
  v = TT::acc_merge(v, dpp_mov<0xB1>(v));
  v = TT::acc_merge(v, dpp_mov<0x4E>(v));
  v = TT::acc_merge(v, dpp_mov<0x141>(v));
  v = TT::acc_merge(v, dpp_mov<0x140>(v));
  const typename TT::Acc r0 = lane_bcast(v, 0), r1 = lane_bcast(v, 16);
  const typename TT::Acc r2 = lane_bcast(v, 32), r3 = lane_bcast(v, 48);
  return TT::acc_merge(TT::acc_merge(r0, r1), TT::acc_merge(r2, r3));
}

// Sum over the 64 lanes in a fixed butterfly order; every lane gets the sum.
template <class R>
__device__ __forceinline__ R wave_sum(R v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = r_add(v, lane_xor(v, m));
  return v;
}

// --------------------------------------------------------------------------
// Tier descriptors
// --------------------------------------------------------------------------

// acc_add: accumulate one term, normalised.  acc_run / acc_fix: the same
// for a run of k terms summed by one lane: the leading parts through
// two_sum, every low-order part (the terms' and the two_sum errors) added
// into the low word in binary64, and one renormalisation at the end.  The
// extra error is within k^2 u^2 of the sum of the magnitudes involved
// (k <= 32 in the Schur bottom).
struct TierF64 {
  using R = double;
  using Acc = dd;
  static constexpr int id = 0;
  __device__ static Acc acc_zero() { return dd{0.0, 0.0}; }
  __device__ static Acc acc_add(Acc a, R t) { return prec::dd_add_d(a, t); }
  __device__ static Acc acc_merge(Acc a, Acc b) { return prec::dd_add(a, b); }
  __device__ static Acc acc_run(Acc a, R t) {
    double s, e;
    prec::two_sum(a.hi, t, s, e);
    return dd{s, a.lo + e};
  }
  __device__ static Acc acc_fix(Acc a) {
    dd z;
    prec::two_sum(a.hi, a.lo, z.hi, z.lo);
    return z;
  }
};

struct TierDD {
  using R = dd;
  using Acc = dd;
  static constexpr int id = 1;
  __device__ static Acc acc_zero() { return dd{0.0, 0.0}; }
  __device__ static Acc acc_add(Acc a, R t) { return prec::dd_add(a, t); }
  __device__ static Acc acc_merge(Acc a, Acc b) { return prec::dd_add(a, b); }
  __device__ static Acc acc_run(Acc a, R t) {
    double s, e;
    prec::two_sum(a.hi, t.hi, s, e);
    return dd{s, a.lo + (t.lo + e)};
  }
  __device__ static Acc acc_fix(Acc a) {
    dd z;
    prec::two_sum(a.hi, a.lo, z.hi, z.lo);
    return z;
  }
};

struct TierQD {
  using R = qd;
  using Acc = qd;
  static constexpr int id = 2;
  __device__ static Acc acc_zero() { return qd{{0.0, 0.0, 0.0, 0.0}}; }
  __device__ static Acc acc_add(Acc a, R t) { return prec::qd_add(a, t); }
  __device__ static Acc acc_merge(Acc a, Acc b) { return prec::qd_add(a, b); }
  __device__ static Acc acc_run(Acc a, R t) { return prec::qd_add(a, t); }
  __device__ static Acc acc_fix(Acc a) { return a; }
};

// |x| of a value whose sign is carried by its leading component
__device__ __forceinline__ double r_abs(double a) { return fabs(a); }
__device__ __forceinline__ dd r_abs(dd a) { return a.hi < 0.0 ? prec::dd_neg(a) : a; }
__device__ __forceinline__ qd r_abs(qd a) { return a.x[0] < 0.0 ? prec::qd_neg(a) : a; }

}  // namespace tor

"""The extended-precision arithmetic of the HIP path (csrc/prec.hpp, which is
host-compatible), compiled for the host and checked against exact rational
arithmetic: the fused Schur updates t - ab and t - ab - cd within their
stated bounds (15 u^2 and 26 u^2 of the magnitudes), results normalised,
and the composed double-double operations within their published ones.
CPU only."""
import os
import subprocess
from fractions import Fraction as F

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
U = F(1, 2 ** 53)

HARNESS = r"""
#include "prec.hpp"
#include <cstdio>
#include <cstdlib>
#include <random>
using namespace prec;
int main(int argc, char** argv) {
  std::mt19937_64 g(atoi(argv[1]));
  const int count = atoi(argv[2]);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  std::uniform_int_distribution<int> E(-30, 30);
  auto mk = [&](double scale) {
    const double h = ldexp(U(g), E(g) / 10) * scale;
    const double l = U(g) * 0x1p-54 * h;
    dd z;
    fast_two_sum(h, l, z.hi, z.lo);
    return z;
  };
  for (int i = 0; i < count; ++i) {
    const int mode = i % 4;
    dd a = mk(1), b = mk(1), c = mk(1), d = mk(1), t = mk(1);
    if (mode == 1) t = dd_add(dd_mul(a, b), dd_mul(c, d));   // near-total cancellation
    if (mode == 2) t = dd_mul(a, b);                          // t - ab ~ 0
    if (mode == 3) { c = a; d = b; }                          // repeated product
    const dd z1 = dd_fms(t, a, b), z2 = dd_fms2(t, a, b, c, d);
    const dd m = dd_mul(a, b), s = dd_add(t, c);
    printf("%a %a %a %a %a %a %a %a %a %a %a %a %a %a %a %a %a %a\n", t.hi, t.lo, a.hi, a.lo, b.hi, b.lo,
           c.hi, c.lo, d.hi, d.lo, z1.hi, z1.lo, z2.hi, z2.lo, m.hi, m.lo, s.hi, s.lo);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def cases(tmp_path_factory):
    d = tmp_path_factory.mktemp("prec")
    src, exe = d / "h.cpp", d / "h"
    src.write_text(HARNESS)
    r = subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-I",
                        os.path.join(ROOT, "paper_2009_01177_amd", "csrc"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe), "7", "6000"], capture_output=True, text=True, check=True).stdout
    rows = []
    for line in out.splitlines():
        v = [F(float.fromhex(x)) for x in line.split()]
        rows.append([(v[2 * k], v[2 * k + 1]) for k in range(9)])
    return rows


def _val(p):
    return p[0] + p[1]


def _normalised(p):
    hi, lo = p
    return hi == 0 and lo == 0 or abs(lo) <= U * abs(hi)


def test_fused_update_t_minus_ab(cases):
    worst = F(0)
    for t, a, b, c, d, z1, z2, m, s in cases:
        mag = abs(_val(t)) + abs(_val(a) * _val(b))
        err = abs(_val(z1) - (_val(t) - _val(a) * _val(b)))
        assert err <= 15 * U * U * mag
        assert _normalised(z1)
        worst = max(worst, err / (U * U * mag) if mag else F(0))
    assert worst > 0  # the cases do exercise rounding


def test_fused_update_t_minus_ab_minus_cd(cases):
    for t, a, b, c, d, z1, z2, m, s in cases:
        ab, cd = _val(a) * _val(b), _val(c) * _val(d)
        mag = abs(_val(t)) + abs(ab) + abs(cd)
        err = abs(_val(z2) - (_val(t) - ab - cd))
        assert err <= 26 * U * U * mag
        assert _normalised(z2)


def test_composed_operations_meet_their_published_bounds(cases):
    # DWTimesDW (FMA form) 4u^2, AccurateDWPlusDW 3u^2 + 13u^3, relative
    for t, a, b, c, d, z1, z2, m, s in cases:
        ab = _val(a) * _val(b)
        if ab != 0:
            assert abs(_val(m) - ab) <= 4 * U * U * abs(ab)
        tc = _val(t) + _val(c)
        if tc != 0:
            assert abs(_val(s) - tc) <= (3 * U * U + 13 * U ** 3) * abs(tc)


QD_HARNESS = r"""
#include "prec.hpp"
#include <cstdio>
#include <cstdlib>
#include <random>
using namespace prec;
static std::mt19937_64 g;
static std::uniform_real_distribution<double> U(-1.0, 1.0);
qd mk() {
  double t[4];
  t[0] = ldexp(U(g), (int)(U(g) * 8));
  t[1] = U(g) * 0x1p-53 * t[0];
  t[2] = U(g) * 0x1p-106 * t[0];
  t[3] = U(g) * 0x1p-159 * t[0];
  return qd_compress<4>(t);
}
void pr(qd a) { printf(" %a %a %a %a", a.x[0], a.x[1], a.x[2], a.x[3]); }
int main(int argc, char** argv) {
  g.seed(atoi(argv[1]));
  const int count = atoi(argv[2]);
  for (int i = 0; i < count; ++i) {
    const int mode = i % 4;
    qd a = mk(), b = mk(), c = mk(), d = mk(), t = mk();
    if (mode == 1) t = qd_add(qd_mul(a, b), qd_mul(c, d));  // near-total cancellation
    if (mode == 2) t = qd_mul(a, b);                          // t - ab ~ 0
    if (mode == 3) { c = a; d = b; }
    pr(t); pr(a); pr(b); pr(c); pr(d);
    pr(qd_mul_fast(a, b)); pr(qd_fms(t, a, b)); pr(qd_fms2(t, a, b, c, d));
    qd x = a.x[0] < 0.0 ? qd_neg(a) : a;
    pr(x); pr(qd_rsqrt(x));
    printf("\n");
  }
  return 0;
}
"""

U4 = F(1, 2 ** 212)


@pytest.fixture(scope="module")
def qd_cases(tmp_path_factory):
    d = tmp_path_factory.mktemp("qdprec")
    src, exe = d / "q.cpp", d / "q"
    src.write_text(QD_HARNESS)
    r = subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-I",
                        os.path.join(ROOT, "paper_2009_01177_amd", "csrc"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe), "11", "2000"], capture_output=True, text=True, check=True).stdout
    rows = []
    for line in out.splitlines():
        v = [F(float.fromhex(x)) for x in line.split()]
        rows.append([sum(v[4 * k:4 * k + 4]) for k in range(10)])
    return rows


def test_quad_double_fused_operations_within_their_bounds(qd_cases):
    # product, t - ab and t - ab - cd from one compression each: within
    # 4 u^4 of the magnitudes (1.0 to 1.3 u^4 measured)
    worst = [F(0)] * 3
    for t, a, b, c, d, m, f1, f2, x, r in qd_cases:
        ab, cd = a * b, c * d
        for k, (val, ref, mag) in enumerate(((m, ab, abs(ab)), (f1, t - ab, abs(t) + abs(ab)),
                                              (f2, t - ab - cd, abs(t) + abs(ab) + abs(cd)))):
            if mag:
                err = abs(val - ref)
                assert err <= 4 * U4 * mag, (k, float(err / (U4 * mag)))
                worst[k] = max(worst[k], err / (U4 * mag))
    assert all(w > 0 for w in worst)  # the cases do exercise rounding


def test_quad_double_rsqrt_within_its_bound(qd_cases):
    # one Newton step from the double-double estimate (about 7 u^2): the
    # quadratic term 1.5 (7 u^2)^2 dominates; 128 u^4 relative is the pin
    import mpmath
    mpmath.mp.prec = 400
    u4 = mpmath.mpf(2) ** -212
    worst = mpmath.mpf(0)
    for *_, x, r in qd_cases:
        ref = 1 / mpmath.sqrt(mpmath.mpf(x.numerator) / x.denominator)
        got = mpmath.mpf(r.numerator) / r.denominator
        rel = abs(got - ref) / (u4 * ref)
        assert rel <= 128, float(rel)
        worst = max(worst, rel)
    assert worst > 0


NONOVERLAP_HARNESS = r"""
#include "prec.hpp"
#include <cstdio>
#include <cstdlib>
#include <random>
using namespace prec;
int main(int argc, char** argv) {
  std::mt19937_64 g(atoi(argv[1]));
  const int count = atoi(argv[2]);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  for (int i = 0; i < count; ++i) {
    // a quad-double, and a nearby one cancelling it to 1e-3 .. 1e-30 of its size
    qd a{{U(g) * 8.0, 0.0, 0.0, 0.0}};
    a.x[1] = U(g) * 0x1p-54 * a.x[0];
    a.x[2] = U(g) * 0x1p-54 * a.x[1];
    a.x[3] = U(g) * 0x1p-54 * a.x[2];
    const double rel = ldexp(U(g), -10 - (int)(i % 90));
    qd b = qd_add(a, qd{{a.x[0] * rel, 0.0, 0.0, 0.0}});
    if (i % 3 == 1) b = qd{{b.x[0], b.x[1], 0.0, 0.0}};
    const qd d = qd_sub(b, a);
    const qd z = qd_nonoverlapping(d);
    printf("%a %a %a %a %a %a %a %a\n", d.x[0], d.x[1], d.x[2], d.x[3], z.x[0], z.x[1], z.x[2], z.x[3]);
  }
  return 0;
}
"""


def lowest_bit(x: float) -> F:
    """The value of the lowest set bit of a nonzero double."""
    f = abs(F(x))
    if f.denominator > 1:
        return F(1, f.denominator)
    m = f.numerator
    return F(m & -m)


def test_quad_double_output_is_non_overlapping(tmp_path):
    """qd_nonoverlapping keeps the exact sum of the words and returns them
    largest first and non-overlapping (each word smaller than the lowest set
    bit of the one before, Shewchuk's definition), so the leading word is the
    sum to within an ulp, also after the heavy cancellation where the
    arithmetic leaves overlapping words."""
    import math
    src, exe = tmp_path / "n.cpp", tmp_path / "n"
    src.write_text(NONOVERLAP_HARNESS)
    r = subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-I",
                        os.path.join(ROOT, "paper_2009_01177_amd", "csrc"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe), "3", "3000"], capture_output=True, text=True, check=True).stdout
    overlapped = 0
    for line in out.splitlines():
        v = [float.fromhex(x) for x in line.split()]
        d, z = v[:4], v[4:]
        exact = sum(F(x) for x in d)
        assert sum(F(x) for x in z) == exact
        for i in range(3):
            if z[i + 1] != 0.0:
                assert z[i] != 0.0 and F(abs(z[i + 1])) < lowest_bit(z[i])
        if exact != 0:
            assert abs(F(z[0]) - exact) <= F(math.ulp(z[0]))
            if abs(F(d[0]) - exact) > F(math.ulp(abs(float(exact)))):
                overlapped += 1
    assert overlapped > 0  # the cases this exists for occur

"""GPU parity: the HIP path against the float128 oracle on the same seeded
inputs, through the C ABI.

Tolerance reading (the stated targets are relative errors of 1e-12 for the
FP64 tier and 1e-25 for double-double; the alternating sum cancels, so the
error of any tier scales with S_abs = sum |terms|, not with |Tor|):
    |Tor_gpu - Tor_oracle| <= tol_tier * S_abs,
    tol = 1e-12 (FP64), 1e-25 (DD), 1e-30 (QD: the oracle's own binary128
    limit; QD's 1e-50 is checked against 80-digit brute force instead).
"""
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import gbs_inputs as g
import oracle

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "dd": 1e-25, "qd": 1e-30}
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def tor():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_01177_amd as t
    t.tor_init()
    return t


_REF_CACHE = {}


def ladder(n):
    """The n=30 workload's state with n clicked modes, and its oracle value
    (cached: the binary128 oracle takes tens of seconds at n = 20)."""
    if n not in _REF_CACHE:
        O, _ = g.workload("n30_lossy", n=n)
        _REF_CACHE[n] = (O, oracle.tor(O))
    return _REF_CACHE[n]


def err_rel(res, ref):
    return float(abs(res.exact - ref["tor"]) / ref["abs_sum"])


def check(tor, O, tier, ref=None, **kw):
    print(f"[parity] n={O.shape[0] // 2} tier={tier} {kw}", flush=True)
    ref = oracle.tor(O) if ref is None else ref
    res = tor.tor_eval(O, tier=tier, **kw)
    assert res.status == 0
    assert res.tier_used == {"fp64": 0, "dd": 1, "qd": 2}[tier]
    e = err_rel(res, ref)
    assert e <= TOL[tier], (tier, e)
    # S_abs is a sum of positive terms: relative agreement
    assert abs(float(res.abs_exact / ref["abs_sum"]) - 1.0) < max(TOL[tier], 1e-28) * 10
    return res, ref


@pytest.mark.parametrize("algo", ["border", "schur"])
@pytest.mark.parametrize("tier", ["fp64", "dd", "qd"])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 8, 11, 13])
def test_small_random_instances(tor, tier, n, algo):
    check(tor, g.random_instance(n, 1000 + n), tier, algo=algo)


@pytest.mark.parametrize("algo", ["border", "schur"])
@pytest.mark.parametrize("tier", ["fp64", "dd", "qd"])
def test_workload_n16_all_tiers(tor, tier, algo):
    O, _ = g.workload("n16_lossless")
    check(tor, O, tier, algo=algo)


@pytest.mark.parametrize("algo", ["border", "schur"])
@pytest.mark.parametrize("tier", ["fp64", "dd"])
@pytest.mark.parametrize("n", [18, 20])
def test_same_state_ladder(tor, tier, n, algo):
    """The n=30 workload's state, fewer clicked modes: several thousand work
    items, ragged subtrees."""
    O, ref = ladder(n)
    check(tor, O, tier, ref=ref, algo=algo)


def test_schur_qd_n20_against_oracle(tor):
    """QD through the Schur path with its top level running (n > 12)."""
    O, ref = ladder(20)
    check(tor, O, "qd", ref=ref, algo="schur")


@pytest.mark.parametrize("d", [0, 1, 4, 7, 11, 13])
def test_split_depth_does_not_change_the_result(tor, d):
    O = g.random_instance(13, 77)
    ref = oracle.tor(O)
    res, _ = check(tor, O, "dd", ref=ref, split_depth=d, algo="border")
    # and a second run is bitwise identical (fixed-order reduction)
    res2 = tor.tor_eval(O, tier="dd", split_depth=d, algo="border")
    assert res2.expansion == res.expansion


@pytest.mark.parametrize("algo", ["border", "schur"])
def test_grid_size_does_not_change_bits(tor, algo):
    O = g.random_instance(19, 5)
    a = tor.tor_eval(O, tier="dd", split_depth=8, grid=1, algo=algo)
    b = tor.tor_eval(O, tier="dd", split_depth=8, grid=97, algo=algo)
    c = tor.tor_eval(O, tier="dd", split_depth=8, algo=algo)
    assert a.expansion == b.expansion == c.expansion


# ---- closed forms through the GPU path --------------------------------------

@pytest.mark.parametrize("algo", ["border", "schur"])
@pytest.mark.parametrize("tier", ["fp64", "dd", "qd"])
def test_closed_forms(tor, tier, algo):
    r = 0.9
    res = tor.tor_eval(g.squeezed_o(r, 0.4), tier=tier, algo=algo)
    with mpmath.workdps(40):
        assert abs(res.value - float(mpmath.cosh(r) - 1)) < 1e-14
        res = tor.tor_eval(g.tmsv_o(r), tier=tier, algo=algo)
        assert abs(res.value - float(mpmath.sinh(r) ** 2)) < 1e-14 * res.value
    assert tor.tor_eval(g.click_submatrix(g.tmsv_o(r), [0]), tier=tier, algo=algo).exact == 0
    res = tor.tor_eval(np.zeros((0, 0), dtype=np.complex128), tier=tier, algo=algo)
    assert res.value == 1.0


@pytest.mark.parametrize("algo", ["border", "schur"])
@pytest.mark.parametrize("tier", ["fp64", "dd", "qd"])
def test_thermal_product_n20(tor, tier, algo):
    rng = np.random.default_rng(20)
    O = g.thermal_o(rng.uniform(0.05, 3.0, size=20))
    exact = Fraction(1)
    sabs = Fraction(1)
    for i in range(20):
        d = Fraction(O[i, i].real)
        exact *= d / (1 - d)
        sabs *= 1 / (1 - d) + 1
    res = tor.tor_eval(O, tier=tier, algo=algo)
    assert float(abs(res.exact - exact) / sabs) <= TOL[tier]


def _block_state(n, seed):
    """A product of 1- and 2-mode states, relabelled and phase-rotated; its
    Torontonian is the product of the blocks' (each by 60-digit brute force)."""
    rng = np.random.default_rng(seed)
    blocks, sizes = [], 0
    while sizes < n:
        k = 1 if (n - sizes == 1 or rng.random() < 0.5) else 2
        if k == 1:
            blocks.append(g.lossy_squeezed_o(rng.uniform(0.6, 1.4), rng.uniform(0.3, 0.9)))
        else:
            blocks.append(g.random_instance(2, int(rng.integers(1 << 30)), M=4))
        sizes += k
    O = g.direct_sum_o(blocks)
    perm = rng.permutation(n)
    O = g.permute_and_phase_o(O, perm, rng.uniform(0, 2 * np.pi, size=n))
    inv = np.argsort(perm)
    off = 0
    prod = Fraction(1)
    sabs = Fraction(1)
    with mpmath.workdps(60):
        for b in blocks:
            k = b.shape[0] // 2
            modes = sorted(inv[off:off + k])
            off += k
            sub = g.click_submatrix(O, modes)
            t, sa = _mp_tor(sub)
            prod *= t
            sabs *= sa
    return O, prod, sabs


def _mp_tor(O):
    n = O.shape[0] // 2
    M = mpmath.matrix(2 * n, 2 * n)
    for i in range(2 * n):
        for j in range(2 * n):
            v = O[i, j]
            M[i, j] = (1 if i == j else 0) - mpmath.mpc(float(v.real), float(v.imag))
    tot, sabs = mpmath.mpf(0), mpmath.mpf(0)
    for z in range(1 << n):
        Z = [i for i in range(n) if (z >> i) & 1]
        idx = Z + [i + n for i in Z]
        if idx:
            sub = mpmath.matrix(len(idx), len(idx))
            for a, ia in enumerate(idx):
                for b, ib in enumerate(idx):
                    sub[a, b] = M[ia, ib]
            d = mpmath.re(mpmath.det(sub))
        else:
            d = mpmath.mpf(1)
        t = 1 / mpmath.sqrt(d)
        sabs += t
        tot += t if (n - len(Z)) % 2 == 0 else -t
    f = lambda x: Fraction(mpmath.nstr(x, 70, min_fixed=-1e9, max_fixed=1e9))
    return f(tot), f(sabs)


@pytest.mark.parametrize("algo", ["border", "schur"])
@pytest.mark.parametrize("tier", ["fp64", "dd"])
def test_block_diagonal_closed_form_n24(tor, tier, algo):
    O, prod, sabs = _block_state(24, 24)
    res = tor.tor_eval(O, tier=tier, algo=algo)
    assert float(abs(res.exact - prod) / sabs) <= TOL[tier]


@pytest.mark.parametrize("tier", ["fp64", "dd"])
def test_block_diagonal_closed_form_n30_schur(tor, tier):
    """The full n = 30 size through the Schur path: a product state whose
    Torontonian is known exactly (product of 60-digit block values)."""
    O, prod, sabs = _block_state(30, 30)
    res = tor.tor_eval(O, tier=tier, algo="schur")
    assert float(abs(res.exact - prod) / sabs) <= TOL[tier]


def test_qd_against_80_digit_brute_force(tor):
    for n, seed in [(3, 1), (4, 2), (5, 3)]:
        O = g.random_instance(n, seed)
        with mpmath.workdps(80):
            t, sa = _mp_tor(O)
        for algo in ("border", "schur"):
            res = tor.tor_eval(O, tier="qd", algo=algo)
            assert float(abs(res.exact - t) / sa) < 1e-50, (n, algo)


# ---- debug entry points -----------------------------------------------------

@pytest.mark.parametrize("tier", ["fp64", "dd", "qd"])
def test_level_sums(tor, tier):
    O = g.random_instance(12, 31)
    ref = oracle.tor(O, level_sums=True)
    levels, res = tor.tor_debug_level_sums(O, tier=tier)
    for m in range(13):
        assert float(abs(levels[m] - ref["levels"][m]) / ref["levels"][m]) < max(TOL[tier], 1e-30)
    assert err_rel(res, ref) <= TOL[tier]


@pytest.mark.parametrize("tier", ["fp64", "dd", "qd"])
@pytest.mark.parametrize("n,seed", [(1, 3), (5, 8), (12, 31), (15, 32)])
def test_level_sums_through_the_schur_kernels(tor, tier, n, seed):
    """Per-level sums L_m from the Schur path's own kernels (level-sum mode)
    against the binary128 oracle's, every level; the signed total against
    the oracle's Torontonian."""
    O = g.random_instance(n, seed)
    ref = oracle.tor(O, level_sums=True)
    levels, res = tor.tor_debug_level_sums(O, tier=tier, algo="schur")
    for m in range(n + 1):
        assert float(abs(levels[m] - ref["levels"][m]) / ref["levels"][m]) < max(TOL[tier], 1e-30), m
    assert err_rel(res, ref) <= TOL[tier]


@pytest.mark.parametrize("tier", ["fp64", "dd", "qd"])
def test_sampled_terms_at_n30(tor, tier):
    """Per-subset terms at the full n = 30 against the oracle's binary128
    determinants (the bordered update on a generic coupled state)."""
    O, _ = g.workload("n30_lossy")
    rng = np.random.default_rng(3)
    masks = rng.integers(0, 1 << 30, size=400, dtype=np.uint64)
    masks[:4] = [0, 1, (1 << 30) - 1, 1 << 29]
    got = tor.tor_debug_sampled_terms(O, masks, tier=tier)
    _, want, st = oracle.terms_exact(O, masks)
    assert (st == 0).all()
    tol = {"fp64": 1e-13, "dd": 1e-28, "qd": 1e-31}[tier]
    for i in range(len(masks)):
        g_ = sum((Fraction(x) for x in got[i]), Fraction(0))
        assert float(abs(g_ - want[i]) / abs(want[i])) < tol, (i, int(masks[i]))


# ---- invariants and errors ----------------------------------------------------

def test_permutation_and_phase_invariance(tor):
    O, _ = g.workload("n16_lossless")
    rng = np.random.default_rng(1)
    O2 = g.permute_and_phase_o(O, rng.permutation(16), rng.uniform(0, 6.3, size=16))
    for algo in ("border", "schur"):
        a = tor.tor_eval(O, tier="dd", algo=algo)
        b = tor.tor_eval(O2, tier="dd", algo=algo)
        assert float(abs(a.exact - b.exact) / a.abs_exact) < 1e-14


@pytest.mark.parametrize("algo", ["border", "schur"])
def test_not_positive_definite(tor, algo):
    from paper_2009_01177_amd import TorError
    O = (2.0 * np.eye(8)).astype(np.complex128)
    with pytest.raises(TorError) as e:
        tor.tor_eval(O, tier="dd", algo=algo)
    assert e.value.code == -2


def test_leading_dimension(tor):
    import torch
    O = g.random_instance(9, 3)
    big = np.zeros((18, 25), dtype=np.complex128)
    big[:, :18] = O
    t = torch.from_numpy(big).cuda()[:, :18]
    assert t.stride(0) == 25
    a = tor.tor_eval(t, tier="dd")
    b = tor.tor_eval(O, tier="dd")
    assert a.expansion == b.expansion


def test_library_before_torch_keeps_torch_on_the_gpu(tor):
    """Regression: initialising the library before PyTorch has touched the
    GPU used to leave PyTorch without a device in that process.  Runs in a
    fresh interpreter, library first."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_2009_01177_amd as t\n"
            "t.tor_init()\n"
            "import numpy as np, torch, gbs_inputs as g\n"
            "O = g.random_instance(6, 5)\n"
            "r = t.tor_eval(torch.from_numpy(O).cuda(), tier='fp64')\n"
            "print('ok', r.status, torch.cuda.device_count())\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.split()[:2] == ["ok", "0"], out.stdout


# every compiled bottom size, at n just above its middle depth (two and eight
# middle states), one to three workgroups: the two-wavefront alternation with
# short and uneven rounds
@pytest.mark.parametrize("tier,sb", [("fp64", s) for s in range(1, 7)] + [("dd", s) for s in range(1, 6)]
                         + [("qd", s) for s in range(1, 4)])
@pytest.mark.parametrize("extra", [1, 3])
def test_every_bottom_size_and_small_grids(tor, tier, sb, extra):
    n = sb + 6 + extra
    O = g.random_instance(n, 700 + 10 * sb + extra)
    print(f"[parity] bottom size {sb} tier {tier} n={n}", flush=True)
    ref = oracle.tor(O)
    runs = [tor.tor_eval(O, tier=tier, algo="schur", bottom_modes=sb, grid=gr) for gr in (1, 3, 0)]
    for r in runs:
        assert r.status == 0
        assert err_rel(r, ref) <= TOL[tier]
    assert runs[0].expansion == runs[1].expansion == runs[2].expansion

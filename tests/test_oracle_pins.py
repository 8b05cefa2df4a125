"""Pins of the float128 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formula: each compares it with a closed
form, an independent route (different matrices, a library determinant,
high-precision arithmetic on tiny inputs) or an exact invariant.
"""
from fractions import Fraction
import itertools

import mpmath
import numpy as np
import pytest

import gbs_inputs as g
import oracle

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def rel(a, b):
    a, b = Fraction(a), Fraction(b)
    return float(abs(a - b) / abs(b)) if b != 0 else float(abs(a - b))


def mp_tor_bruteforce(O, dps=60):
    """Eq. 2 by brute force at `dps` digits: mpmath determinant of every
    principal submatrix (I - O)_Z in block order."""
    with mpmath.workdps(dps):
        n = O.shape[0] // 2
        M = mpmath.matrix(2 * n, 2 * n)
        for i in range(2 * n):
            for j in range(2 * n):
                v = O[i, j]
                M[i, j] = (1 if i == j else 0) - mpmath.mpc(float(v.real), float(v.imag))
        tot = mpmath.mpf(0)
        sabs = mpmath.mpf(0)
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
        return tot, sabs


def mp_to_frac(x):
    return Fraction(mpmath.nstr(x, 70, min_fixed=-1e9, max_fixed=1e9)) if x != 0 else Fraction(0)


# ---- P1: the empty product -------------------------------------------------

def test_n0_is_one():
    r = oracle.tor(np.zeros((0, 0), dtype=np.complex128))
    assert r["tor"] == 1 and r["abs_sum"] == 1


# ---- P2: one mode ------------------------------------------------------------

@pytest.mark.parametrize("r", [0.1, 0.5, 1.0, 1.6])
def test_single_mode_squeezed_is_cosh_minus_one(r):
    res = oracle.tor(g.squeezed_o(r, phi=0.3))
    # closed form from the physics: p(click) = 1 - 1/cosh r, Tor = cosh r - 1
    with mpmath.workdps(40):
        closed = mp_to_frac(mpmath.cosh(r) - 1)
    assert rel(res["tor"], closed) < 1e-14
    # exact from the FP64 input value b: det(I - O) = 1 - |b|^2
    b = np.tanh(r)  # |e^{i phi} tanh r| differs from tanh r only by rounding
    O = g.squeezed_o(r, phi=0.0)
    res0 = oracle.tor(O)
    bb = Fraction(O[1, 0].real) ** 2
    with mpmath.workdps(60):
        exact = 1 / mpmath.sqrt(mpmath.mpf(1) - mpmath.mpf(bb.numerator) / bb.denominator) - 1
    assert rel(res0["tor"], mp_to_frac(exact)) < 1e-31


@pytest.mark.parametrize("nbar", [0.01, 0.3, 2.5, 40.0])
def test_single_mode_thermal_is_nbar(nbar):
    O = g.thermal_o([nbar])
    d = Fraction(O[0, 0].real)
    # Tor = det(I-O)^(-1/2) - 1 = 1/(1-d) - 1 = d/(1-d), and d = nbar/(nbar+1)
    assert rel(oracle.tor(O)["tor"], d / (1 - d)) < 1e-32
    assert rel(oracle.tor(O)["tor"], nbar) < 1e-14


# ---- P3: two-mode squeezed vacuum ---------------------------------------------

@pytest.mark.parametrize("r", [0.2, 0.9, 1.5])
def test_tmsv(r):
    O = g.tmsv_o(r)
    t = Fraction(O[2, 1].real)
    res = oracle.tor(O)
    # both-click probability 1 - 1/cosh^2 r over the vacuum probability
    with mpmath.workdps(40):
        closed = mp_to_frac(mpmath.sinh(r) ** 2)
    assert rel(res["tor"], closed) < 1e-14
    assert rel(res["tor"], t * t / (1 - t * t)) < 1e-32
    # one mode clicks, its partner is dark: probability 0, exactly
    O1 = g.click_submatrix(O, [0])
    assert oracle.tor(O1)["tor"] == 0
    assert oracle.tor(g.click_submatrix(O, [1]))["tor"] == 0


# ---- P4: thermal product --------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 5, 9, 12])
def test_thermal_product(n):
    rng = np.random.default_rng(n)
    O = g.thermal_o(rng.uniform(0.05, 3.0, size=n))
    exact = Fraction(1)
    for i in range(n):
        d = Fraction(O[i, i].real)
        exact *= d / (1 - d)
    res = oracle.tor(O)
    # the alternating sum cancels: its error scales with S_abs, not |Tor|
    u128 = 2.0 ** -113
    assert float(abs(res["tor"] - exact) / res["abs_sum"]) < 8 * (3 * n + 2) * u128
    # S_abs = prod (1/(1-d) + 1) for a product state (independent modes)
    sabs = Fraction(1)
    for i in range(n):
        d = Fraction(O[i, i].real)
        sabs *= 1 / (1 - d) + 1
    assert rel(res["abs_sum"], sabs) < (n + 2) * 1e-33


def test_thermal_equals_eq6_with_k_zero():
    # Eq. 6 with k = 0 reads Tor ~ (1/(1-a) - 1)^N, exact for O = a I
    a, n = 0.16, 10
    O = (a * np.eye(2 * n)).astype(np.complex128)
    fa = Fraction(a)
    res = oracle.tor(O)
    err = abs(res["tor"] - (1 / (1 - fa) - 1) ** n)
    assert float(err / res["abs_sum"]) < 8 * (3 * n + 2) * 2.0 ** -113


# ---- P5: product states, relabelled and phase-rotated -------------------------------

def _block(kind, rng):
    if kind == "sq":
        return g.lossy_squeezed_o(rng.uniform(0.3, 1.5), rng.uniform(0.2, 1.0))
    if kind == "th":
        return g.thermal_o([rng.uniform(0.1, 2.0)])
    if kind == "two":
        return g.random_instance(2, int(rng.integers(1 << 30)), M=3)
    raise ValueError(kind)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_block_diagonal_factorises(seed):
    rng = np.random.default_rng(100 + seed)
    kinds = ["sq", "th", "two", "sq", "two", "th", "sq"]
    blocks = [_block(k, rng) for k in kinds]
    O = g.direct_sum_o(blocks)
    n = O.shape[0] // 2
    perm = rng.permutation(n)
    O = g.permute_and_phase_o(O, perm, rng.uniform(0, 2 * np.pi, size=n))
    # each block by brute force at 60 digits (Eq. 2 over its 2 or 4 subsets),
    # on the block exactly as it sits in the relabelled, rotated matrix
    inv = np.argsort(perm)
    off = 0
    prod = mpmath.mpf(1)
    with mpmath.workdps(60):
        for b in blocks:
            k = b.shape[0] // 2
            modes = sorted(inv[off:off + k])
            off += k
            sub = g.click_submatrix(O, modes)
            t, _ = mp_tor_bruteforce(sub)
            prod *= t
        res = oracle.tor(O)
        assert rel(res["tor"], mp_to_frac(prod)) < 1e-28


# ---- P6 and P7: click probabilities --------------------------------------------------

def _state(M, seed, eta=0.6):
    rng = np.random.Generator(np.random.PCG64(seed))
    U = g.haar_unitary(M, rng)
    r = rng.uniform(0.3, 1.2, size=M)
    sq = g.gbs_sigma_q(U, r, eta)
    return sq, g.o_from_sigma_q(sq)


def test_probabilities_sum_to_one():
    M = 7
    sq, O = _state(M, 7)
    pvac = np.sqrt(np.linalg.det(np.eye(2 * M) - O).real)
    tot = Fraction(0)
    for z in range(1 << M):
        S = [k for k in range(M) if (z >> k) & 1]
        tot += oracle.tor(g.click_submatrix(O, S))["tor"] * Fraction(pvac)
    assert abs(float(tot) - 1.0) < 1e-12


def test_jacobi_route_probabilities():
    """p(S) from determinants of sigma_Q's principal submatrices (no
    inverse): det(M_Z)^(-1/2) / sqrt(det sigma_Q) = det(sigma_Q[Z^c])^(-1/2),
    so p(S) = sum_{Z subset S} (-1)^{|S|-|Z|} det(sigma_Q[Z^c])^(-1/2)."""
    M = 6
    sq, O = _state(M, 11, eta=0.5)
    dsq = np.linalg.det(sq).real
    rng = np.random.default_rng(3)
    for _ in range(6):
        S = sorted(rng.choice(M, size=int(rng.integers(1, M + 1)), replace=False).tolist())
        with mpmath.workdps(40):
            p = mpmath.mpf(0)
            for r_ in range(len(S) + 1):
                for Z in itertools.combinations(S, r_):
                    comp = [k for k in range(M) if k not in Z]
                    idx = comp + [k + M for k in comp]
                    if idx:
                        sub = mpmath.matrix(sq[np.ix_(idx, idx)].tolist())
                        d = mpmath.re(mpmath.det(sub))
                    else:
                        d = mpmath.mpf(1)
                    s = 1 if (len(S) - r_) % 2 == 0 else -1
                    p += s / mpmath.sqrt(d)
            p_or = float(oracle.tor(g.click_submatrix(O, S))["tor"]) / np.sqrt(dsq)
            assert abs(p_or - float(p)) <= 1e-12 * max(1.0, abs(float(p)))


# ---- P9 / P10: brute force -----------------------------------------------------------

def test_terms_match_library_determinants():
    """Every subset's det against numpy's LAPACK slogdet (binary64), n = 9."""
    O = g.random_instance(9, 5)
    n = 9
    masks = np.arange(1 << n, dtype=np.uint64)
    det, term, st = oracle.terms(O, masks)
    assert (st == 0).all()
    Mfull = np.eye(2 * n) - O
    for z in range(1 << n):
        Z = [i for i in range(n) if (z >> i) & 1]
        idx = Z + [i + n for i in Z]
        d = np.linalg.det(Mfull[np.ix_(idx, idx)]).real if idx else 1.0
        assert abs(det[z] - d) <= 1e-12 * d
        sgn = 1 if (n - len(Z)) % 2 == 0 else -1
        assert abs(term[z] - sgn / np.sqrt(d)) <= 1e-12 / np.sqrt(d)
    # the full sum and the level sums agree with the per-term values
    res = oracle.tor(O, level_sums=True)
    pops = np.array([bin(z).count("1") for z in range(1 << n)])
    for m in range(n + 1):
        lm = np.abs(term[pops == m]).sum()
        assert abs(float(res["levels"][m]) - lm) <= 1e-13 * lm
    assert abs(float(res["tor"]) - term.sum()) <= 1e-13 * float(res["abs_sum"])


@pytest.mark.parametrize("n,seed", [(3, 1), (4, 2), (5, 3)])
def test_full_sum_against_mpmath(n, seed):
    O = g.random_instance(n, seed)
    t, sabs = mp_tor_bruteforce(O, dps=60)
    res = oracle.tor(O)
    err = abs(res["tor"] - mp_to_frac(t))
    assert float(err / mp_to_frac(sabs)) < 1e-31
    assert rel(res["abs_sum"], mp_to_frac(sabs)) < 1e-31


def test_level_sums_function_matches_full_run():
    O = g.random_instance(10, 9)
    full = oracle.tor(O, level_sums=True)
    lv = oracle.level_sums(O, list(range(11)))
    for m in range(11):
        assert rel(lv[m], full["levels"][m]) < 1e-30


def test_terms_exact_match_full_run_extremes():
    O = g.random_instance(8, 4)
    n = 8
    dets, ts, st = oracle.terms_exact(O, np.arange(256, dtype=np.uint64))
    full = oracle.tor(O)
    assert rel(sum(ts), full["tor"]) < 1e-30
    assert min(dets) == full["min_det"]
    assert max(abs(t) for t in ts) == full["max_term"]
    # every reciprocal square root exceeds 1 and det shrinks under inclusion
    for z in range(256):
        assert abs(ts[z]) >= 1
        for i in range(n):
            if not (z >> i) & 1:
                assert dets[z | (1 << i)] <= dets[z]


# ---- invariants and errors ----------------------------------------------------------

def test_permutation_and_phase_invariance():
    O = g.random_instance(8, 21)
    rng = np.random.default_rng(0)
    O2 = g.permute_and_phase_o(O, rng.permutation(8), rng.uniform(0, 6.3, size=8))
    a, b = oracle.tor(O), oracle.tor(O2)
    assert float(abs(a["tor"] - b["tor"]) / a["abs_sum"]) < 1e-14


def test_not_positive_definite_is_reported():
    O = (2.0 * np.eye(6)).astype(np.complex128)
    with pytest.raises(oracle.OracleError) as e:
        oracle.tor(O)
    assert e.value.code == oracle.ENOTPD


def test_threads_do_not_change_the_result_beyond_rounding():
    O = g.random_instance(12, 3)
    a = oracle.tor(O, threads=1)
    b = oracle.tor(O, threads=5)
    assert float(abs(a["tor"] - b["tor"]) / a["abs_sum"]) < 1e-32


def test_input_symmetries_hold_exactly():
    O, _ = g.workload("n16_lossless")
    n = O.shape[0] // 2
    assert np.array_equal(O, O.conj().T)
    assert np.array_equal(O[n:, n:], O[:n, :n].conj())
    assert np.array_equal(O[:n, n:], O[:n, n:].T)


def test_asymmetry_is_reported_not_repaired():
    """The oracle reports O's deviations from Hermitian and from the block
    structure of Eq. 3 (O11 = conj O00, O10 = conj O01); it does not repair
    them.  Built inputs report zeros; a planted deviation in one block is
    reported at its own size in the blocks it breaks and nowhere else."""
    O, _ = g.workload("n16_lossless")
    n = O.shape[0] // 2
    r = oracle.tor(g.random_instance(6, 11))
    assert r["asymmetry"] == dict(hermitian=0.0, o11=0.0, o10=0.0)
    assert oracle.asymmetry(O) == dict(hermitian=0.0, o11=0.0, o10=0.0)
    P = O.copy()
    P[0, 1] += 3e-9                                   # inside O00 only
    a = oracle.asymmetry(P)
    assert a["hermitian"] == pytest.approx(3e-9, rel=1e-6)
    assert a["o11"] == pytest.approx(3e-9, rel=1e-6) and a["o10"] == 0.0
    P = O.copy()
    P[n + 2, 1] += 5e-7j                              # inside O10 only
    a = oracle.asymmetry(P)
    assert a["hermitian"] == pytest.approx(5e-7, rel=1e-6)
    assert a["o10"] == pytest.approx(5e-7, rel=1e-6) and a["o11"] == 0.0
    # the input itself is left as it was
    assert P[n + 2, 1] != O[n + 2, 1]

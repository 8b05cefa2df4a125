"""tor_eval_part / tor_combine_parts: every part's signed sum and sum of
magnitudes against the binary128 oracle summed over exactly that part's
subsets, and the combined parts against the oracle and against tor_eval.
Parts are evaluated in any order (a resumed run)."""
from fractions import Fraction

import numpy as np
import pytest

import gbs_inputs as g
import oracle

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "dd": 1e-25, "qd": 1e-30}


@pytest.fixture(scope="module")
def tor():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_01177_amd as t
    t.tor_init()
    return t


_REF = {}


def _reference(n, seed):
    """Instance and the oracle's per-mask terms as exact Fractions."""
    key = (n, seed)
    if key not in _REF:
        O = g.random_instance(n, seed)
        masks = np.arange(1 << n, dtype=np.uint64)
        d3, t3, st = oracle._terms3(O, masks)
        assert (st == 0).all()
        terms = [Fraction(t3[i, 0]) + Fraction(t3[i, 1]) + Fraction(t3[i, 2]) for i in range(1 << n)]
        _REF[key] = (O, terms)
    return _REF[key]


def _part_of(mask, k, nparts):
    code = 0
    for i in range(k):
        code = (code << 1) | ((mask >> i) & 1)
    codes = 1 << k
    for p in range(nparts):
        if p * codes // nparts <= code < (p + 1) * codes // nparts:
            return p
    raise AssertionError


@pytest.mark.parametrize("tier", ["fp64", "dd", "qd"])
@pytest.mark.parametrize("nparts", [1, 2, 3, 5, 8])
def test_parts_match_the_oracle(tor, tier, nparts):
    n = 16
    O, terms = _reference(n, 4242)
    k = max(0, (nparts - 1).bit_length())
    want = [Fraction(0)] * nparts
    want_abs = [Fraction(0)] * nparts
    for m, t in enumerate(terms):
        p = _part_of(m, k, nparts)
        want[p] += t
        want_abs[p] += abs(t)
    print(f"[parts] n={n} tier={tier} nparts={nparts}", flush=True)
    res = []
    for p in reversed(range(nparts)):  # any order
        r = tor.tor_eval_part(O, p, nparts, tier=tier)
        assert r.status == 0
        assert float(abs(r.exact - want[p]) / want_abs[p]) <= TOL[tier], p
        assert abs(r.abs_exact - want_abs[p]) <= 1e-12 * want_abs[p]
        res.append(r)
    res.reverse()
    total = tor.tor_combine_parts(tier, n, res)
    S = sum(want_abs)
    assert float(abs(total.exact - sum(want)) / S) <= TOL[tier]
    whole = tor.tor_eval(O, tier=tier, algo="schur")
    assert float(abs(total.exact - whole.exact) / S) <= TOL[tier]
    if nparts == 1:
        assert total.exact == whole.exact


def test_benchmark_instance_in_parts(tor):
    # the n = 30 instance in 16 parts, evaluated last to first, against one
    # whole evaluation
    O, _ = g.workload("n30_lossy")
    print("[parts] n=30 dd nparts=16", flush=True)
    res = [tor.tor_eval_part(O, p, 16, tier="dd") for p in reversed(range(16))][::-1]
    total = tor.tor_combine_parts("dd", 30, res)
    whole = tor.tor_eval(O, tier="dd")
    assert total.status == 0
    assert float(abs(total.exact - whole.exact) / whole.abs_exact) <= 1e-25
    assert abs(total.abs_exact - whole.abs_exact) <= 1e-25 * whole.abs_exact


def test_too_many_parts_are_refused(tor):
    O = g.random_instance(12, 7)
    with pytest.raises(tor.TorError):
        tor.tor_eval_part(O, 0, 4096, tier="dd")


def test_interrupted_run_resumes_from_its_checkpoint(tor, tmp_path):
    from paper_2009_01177_amd import parts
    O = g.random_instance(22, 99)
    ck = str(tmp_path / "run.json")
    print("[parts] n=22 dd: 3 of 8 parts, then resume", flush=True)
    assert parts.evaluate_in_parts(O, 8, "dd", checkpoint=ck, stop_after=3) is None
    seen = []
    total = parts.evaluate_in_parts(O, 8, "dd", checkpoint=ck, progress=lambda p, r: seen.append(p))
    assert seen == [3, 4, 5, 6, 7]
    straight = parts.evaluate_in_parts(O, 8, "dd")
    assert total.exact == straight.exact
    whole = tor.tor_eval(O, tier="dd")
    assert float(abs(total.exact - whole.exact) / whole.abs_exact) <= 1e-25


def _share_against_the_oracle(tor, O, code, k, tiers=("dd", "fp64", "qd")):
    """The share `code` of 2^k of instance O through the timed kernels (the
    default bottom sizes and launch shape) against the binary128 oracle's
    terms for exactly the subsets whose decisions on modes 0..k-1 spell
    `code` (mode 0 the most significant bit)."""
    import math
    n = O.shape[0] // 2
    pre = 0
    for i in range(k):
        if (code >> (k - 1 - i)) & 1:
            pre |= 1 << i
    masks = np.uint64(pre) | (np.arange(1 << (n - k), dtype=np.uint64) << np.uint64(k))
    print(f"[parts] n={n} share {code} of {1 << k}: oracle terms for 2^{n - k} subsets", flush=True)
    d3, t3, st = oracle._terms3(O, masks)
    assert (st == 0).all()
    want = sum(map(Fraction, t3.ravel()))
    sabs = math.fsum(np.abs(t3[:, 0]))
    for tier in tiers:
        r = tor.tor_eval_part(O, code, 1 << k, tier=tier)
        assert r.status == 0
        assert float(abs(r.exact - want)) <= TOL[tier] * sabs, tier
        assert abs(float(r.abs_exact) - sabs) <= 1e-12 * sabs


@pytest.mark.parametrize("code", [0b1000000001, "seed-1", "seed-2"])
def test_a_share_of_the_benchmark_instance_against_the_oracle(tor, code):
    # the n = 30 benchmark instance: the share "in, out x8, in" of 1024 and
    # two seeded shares with three modes in (2^20 subsets each)
    O, _ = g.workload("n30_lossy")
    if isinstance(code, str):
        rng = np.random.default_rng(int(code[-1]))
        bits = rng.choice(10, size=3, replace=False)
        code = int(sum(1 << int(b) for b in bits))
    _share_against_the_oracle(tor, O, code, 10)


def test_the_all_in_share_of_the_benchmark_state(tor):
    # the largest terms: every subset containing modes 0..9 (the all-in share
    # of 1024), on 26 clicked modes of the benchmark's state (2^16 subsets;
    # at n = 30 the oracle needs minutes for this share)
    O, _ = g.workload("n30_lossy", n=26)
    _share_against_the_oracle(tor, O, (1 << 10) - 1, 10)


@pytest.mark.parametrize("tier", ["fp64", "dd", "qd"])
def test_a_part_at_the_largest_n(tor, tier):
    # n = 50 (the paper's largest instance size) through the Schur path: the
    # part of 2^17 whose decisions on modes 0..16 are a seeded code (2^33
    # subsets), of a product of 1- and 2-mode states whose first 17 modes are
    # whole blocks, against its closed form (prefix blocks' terms times the
    # other blocks' Torontonians, each at 60 digits)
    from test_parts_host import part_closed_form, product_state_in_order
    n, k = 50, 17
    O, spans = product_state_in_order(n, k, 5017)
    code = int(np.random.default_rng(k).integers(1 << k))
    want, sabs = part_closed_form(O, spans, k, code)
    print(f"[parts] n=50 tier={tier} part {code} of 2^{k}", flush=True)
    r = tor.tor_eval_part(O, code, 1 << k, tier=tier)
    assert r.status == 0
    assert float(abs(r.exact - want) / sabs) <= TOL[tier]
    assert abs(float(r.abs_exact) - float(sabs)) <= 1e-12 * float(sabs)

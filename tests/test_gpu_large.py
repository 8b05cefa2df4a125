"""Full-size checks of the benchmark workloads (n = 30, 36, 40) and the
largest n the library accepts: sampled terms against the binary128 oracle,
closed forms of product states at the full size, agreement between tiers,
and the autotuner."""
from fractions import Fraction

import numpy as np
import pytest

import gbs_inputs as g
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tor():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_01177_amd as t
    t.tor_init()
    return t


def _sampled(tor, O, n, tier, k, seed, tol):
    rng = np.random.default_rng(seed)
    masks = rng.integers(0, 1 << n, size=k, dtype=np.uint64)
    masks[:3] = [0, (1 << n) - 1, 1 << (n - 1)]
    print(f"[large] sampled terms n={n} tier={tier} k={k}", flush=True)
    got = tor.tor_debug_sampled_terms(O, masks, tier=tier)
    _, want, st = oracle.terms_exact(O, masks)
    assert (st == 0).all()
    for i in range(k):
        gv = sum((Fraction(x) for x in got[i]), Fraction(0))
        assert float(abs(gv - want[i]) / abs(want[i])) < tol, (i, int(masks[i]))


@pytest.mark.parametrize("name,n", [("n36_stress", 36), ("n40_lossy", 40)])
@pytest.mark.parametrize("tier,tol", [("fp64", 1e-12), ("dd", 1e-27)])
def test_sampled_terms_full_size(tor, name, n, tier, tol):
    O, _ = g.workload(name)
    _sampled(tor, O, n, tier, 120, n, tol)


def test_sampled_terms_qd_largest_factor_in_lds(tor):
    """QD single-subset terms use the bordered kernel, whose quad-double factor
    fits LDS up to n = 34; larger n is refused with TOR_EUNSUPPORTED."""
    O, _ = g.workload("n40_lossy", n=34)
    _sampled(tor, O, 34, "qd", 60, 34, 1e-31)
    O36, _ = g.workload("n36_stress")
    with pytest.raises(tor.TorError) as e:
        tor.tor_debug_sampled_terms(O36, np.array([1], dtype=np.uint64), tier="qd")
    assert e.value.code == -5


@pytest.mark.parametrize("tier,tol", [("fp64", 1e-12), ("dd", 1e-27)])
def test_sampled_terms_at_n48(tor, tier, tol):
    O = g.random_instance(48, 4848, M=60)
    _sampled(tor, O, 48, tier, 40, 48, tol)


def test_sampled_terms_at_the_largest_n(tor):
    """n = 50 (TOR_NMAX): FP64 single-subset terms against the oracle; the
    double-double factor of a 100 x 100 matrix (164 KB) does not fit the
    bordered kernel's LDS and is refused with TOR_EUNSUPPORTED."""
    import paper_2009_01177_amd._lib as L
    assert L.TOR_NMAX == 50
    O = g.random_instance(50, 5050, M=60)
    _sampled(tor, O, 50, "fp64", 40, 50, 1e-12)
    with pytest.raises(tor.TorError) as e:
        tor.tor_debug_sampled_terms(O, np.array([1], dtype=np.uint64), tier="dd")
    assert e.value.code == -5


def _block_state(n, seed):
    from test_gpu_parity import _block_state as bs
    return bs(n, seed)


@pytest.mark.parametrize("n", [36, 40])
def test_block_diagonal_closed_form_full_size(tor, n):
    """Product states at the full sizes through the Schur path (DD), against
    the exact product of 60-digit block values."""
    O, prod, sabs = _block_state(n, 1000 + n)
    print(f"[large] block-diagonal n={n} dd", flush=True)
    res = tor.tor_eval(O, tier="dd")
    assert float(abs(res.exact - prod) / sabs) <= 1e-25


_ORACLE_LEVELS = {}


@pytest.mark.parametrize("name,ms,tier,tol", [
    (name, ms, tier, tol)
    for name, ms in (("n30_lossy", [0, 1, 2, 3, 4, 26, 27, 28, 29, 30]),
                     ("n36_stress", [0, 1, 2, 3, 33, 34, 35, 36]),
                     ("n40_lossy", [0, 1, 2, 3, 37, 38, 39, 40]))
    for tier, tol in (("dd", 1e-27), ("fp64", 1e-12))
    if not (name == "n40_lossy" and tier == "fp64")  # about a minute each at n = 40: DD only
])
def test_extreme_level_sums_through_the_schur_kernels(tor, name, ms, tier, tol):
    """P14 at the full size on generic coupled instances: the per-level sums
    L_m of the extreme levels (the benchmark's n = 30 instance: m <= 4 and
    m >= 26, 63,862 subsets; the n = 36 stress instance: m <= 3 and
    m >= 33, 15,614 subsets; the n = 40 instance: m <= 3 and m >= 37,
    21,402 subsets, DD only), from the Schur path's kernels in their
    level-sum mode against the binary128 oracle's level sums of the same
    subsets.  Level sums add positive terms, so each is held relative to
    itself."""
    O, _ = g.workload(name)
    print(f"[large] {name} level sums {ms} via schur, tier={tier}", flush=True)
    levels, res = tor.tor_debug_level_sums(O, tier=tier, algo="schur")
    if name not in _ORACLE_LEVELS:  # both tiers check against one oracle run
        _ORACLE_LEVELS[name] = oracle.level_sums(O, ms)
    want = _ORACLE_LEVELS[name]
    for m, w in zip(ms, want):
        assert float(abs(levels[m] - w) / w) <= tol, m
    assert res.status == 0


def test_extreme_level_sums_at_n30_in_quad_double(tor):
    """The same P14 check in quad-double (bottoms of at most two modes in the
    level-sum mode), held to the binary128 oracle's own accuracy."""
    name, ms = "n30_lossy", [0, 1, 2, 3, 4, 26, 27, 28, 29, 30]
    O, _ = g.workload(name)
    print(f"[large] {name} level sums {ms} via schur, tier=qd", flush=True)
    levels, res = tor.tor_debug_level_sums(O, tier="qd", algo="schur")
    if name not in _ORACLE_LEVELS:
        _ORACLE_LEVELS[name] = oracle.level_sums(O, ms)
    for m, w in zip(ms, _ORACLE_LEVELS[name]):
        assert float(abs(levels[m] - w) / w) <= 1e-30, m
    assert res.status == 0


def test_tiers_agree_on_the_n30_workload(tor):
    """FP64 and DD against QD on the benchmark's own instance (kappa 2.6e21)."""
    O, _ = g.workload("n30_lossy")
    q = tor.tor_eval(O, tier="qd")
    d = tor.tor_eval(O, tier="dd")
    f = tor.tor_eval(O, tier="fp64")
    sabs = q.abs_exact
    print(f"[large] n30 kappa={q.kappa:.3e}", flush=True)
    assert float(abs(d.exact - q.exact) / sabs) <= 1e-25
    assert float(abs(f.exact - q.exact) / sabs) <= 1e-12
    # DD keeps about kappa * n * 2^-104 of relative accuracy: 8 digits here
    assert float(abs(d.exact - q.exact) / abs(q.exact)) < 1e-6


def test_tiers_agree_on_the_n36_stress_workload(tor):
    O, _ = g.workload("n36_stress")
    d = tor.tor_eval(O, tier="dd")
    f = tor.tor_eval(O, tier="fp64")
    assert float(abs(f.exact - d.exact) / d.abs_exact) <= 1e-12


def test_autotuner(tor, tmp_path):
    # n = 20 is tuned as a batch group of 256 instances (the batched shape)
    best, ms = tor.tor_autotune(20, "dd")
    print(f"[large] autotune n=20 dd best={best} ms={ms}", flush=True)
    assert 1 <= best <= 5 and ms[best - 1] > 0
    assert ms[best - 1] == min(x for x in ms if x > 0)
    # n = 46 on a share of its frontier, scaled to the whole evaluation
    # (about 20 minutes in DD): seconds
    import time
    t = time.time()
    b46, ms46 = tor.tor_autotune(46, "dd")
    print(f"[large] autotune n=46 dd best={b46} in {time.time() - t:.1f} s, projected ms {ms46}", flush=True)
    assert time.time() - t < 60 and 1 <= b46 <= 5 and ms46[b46 - 1] > 6e5
    p = str(tmp_path / "tune.txt")
    tor.tor_autotune_save(p)
    tor.tor_autotune_load(p)
    assert f"20 1 {best}" in open(p).read()
    # the tuned default still matches the oracle
    from test_gpu_parity import ladder
    O, ref = ladder(20)
    res = tor.tor_eval(O, tier="dd")
    assert float(abs(res.exact - ref["tor"]) / ref["abs_sum"]) <= 1e-25

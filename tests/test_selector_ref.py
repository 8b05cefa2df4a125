"""Pins of the selector's binary64 reference (oracle/selector_ref.py) and the
library's host-side selector pieces (fallback estimate, model file), CPU only."""
import itertools
import math
import os

import numpy as np
import pytest

import gbs_inputs as g
import oracle
from oracle import selector_ref as ref


def test_real_form_keeps_every_principal_minor():
    O = g.random_instance(6, 3)
    n = 6
    R = ref.real_form(O)
    assert np.allclose(R, R.T, atol=0, rtol=0) or np.max(np.abs(R - R.T)) < 1e-15
    M = np.eye(2 * n) - O
    for r in range(1, n + 1):
        for Z in itertools.combinations(range(n), r):
            iz = list(Z) + [k + n for k in Z]
            ir = [x for k in Z for x in (2 * k, 2 * k + 1)]
            dm = np.linalg.det(M[np.ix_(iz, iz)]).real
            dr = np.linalg.det(R[np.ix_(ir, ir)])
            assert abs(dm - dr) <= 1e-13 * abs(dm)


def test_independent_mode_feature_is_exact_for_product_states():
    """For a product state kappa = prod (1 + q_k)/(1 - q_k) exactly, so
    feature f2 equals log(S_abs/|Tor|) of the oracle; the pair coupling f6
    vanishes."""
    rng = np.random.default_rng(2)
    blocks = [g.lossy_squeezed_o(rng.uniform(0.3, 1.4), rng.uniform(0.3, 0.9)) for _ in range(5)]
    blocks += [g.thermal_o([rng.uniform(0.1, 2.0)]) for _ in range(3)]
    O = g.direct_sum_o(blocks)
    O = g.permute_and_phase_o(O, rng.permutation(8), rng.uniform(0, 6.3, size=8))
    f = ref.features(O)
    r = oracle.tor(O)
    assert abs(f[2] - math.log(r["kappa"])) < 1e-9
    assert abs(f[6]) < 1e-12
    # and f1 is the log of the largest term
    assert abs(f[1] - math.log(float(r["max_term"]))) < 1e-12


def test_features_basic_identities():
    O = g.random_instance(7, 12)
    f = ref.features(O)
    assert f[0] == 7
    assert 0 < f[8] <= f[7] < 1
    assert f[6] <= 1e-12  # Fischer: det of a PD block matrix <= product of its diagonal blocks
    n = 7
    M = np.eye(2 * n) - O
    assert abs(f[1] + 0.5 * np.linalg.slogdet(M)[1]) < 1e-12
    assert abs(f[4] - np.mean(O.real.diagonal()[:n])) < 1e-15


def test_spectrum_features_bracket_the_eigenvalues():
    """Gershgorin's interval contains the spectrum of R, and Lanczos Ritz
    values lie inside [lambda_min, lambda_max] (Cauchy interlacing): LAPACK's
    eigenvalues of R pin f12..f15 from both sides; when 12 steps cover the
    whole space (2n <= 12) the Ritz values are the extreme eigenvalues."""
    for n, seed in ((3, 5), (6, 7), (11, 9)):
        O = g.random_instance(n, seed)
        f = ref.features(O)
        ev = np.linalg.eigvalsh(ref.real_form(O))
        assert f[12] <= ev[0] * (1 + 1e-12)
        assert math.log(ev[-1]) <= f[13] + 1e-12
        assert math.log(ev[0]) <= f[14] + 1e-9 and f[15] <= math.log(ev[-1]) + 1e-9
        assert f[14] <= f[15]
        if 2 * n <= ref.LANCZOS_STEPS:
            assert abs(f[14] - math.log(ev[0])) < 1e-8 and abs(f[15] - math.log(ev[-1])) < 1e-8


def test_top_level_features_are_the_oracles_term_ratios():
    """f16..f19 are the level-(n-1) and level-(n-2) terms over the level-n
    term; the binary128 oracle's terms of those subsets (determinants of
    I - O_Z, no inverse) give the same means and maxima."""
    n = 7
    O = g.random_instance(n, 21)
    f = ref.features(O)
    full = float(oracle.terms(O, [(1 << n) - 1])[1][0])
    m1 = [(1 << n) - 1 - (1 << k) for k in range(n)]
    m2 = [(1 << n) - 1 - (1 << i) - (1 << j) for i in range(n) for j in range(i + 1, n)]
    t1 = np.abs(oracle.terms(O, m1)[1]) / abs(full)
    t2 = np.abs(oracle.terms(O, m2)[1]) / abs(full)
    assert abs(f[16] - math.log(t1.mean())) < 1e-10 and abs(f[17] - math.log(t1.max())) < 1e-10
    assert abs(f[18] - math.log(t2.mean())) < 1e-10 and abs(f[19] - math.log(t2.max())) < 1e-10
    # every term is at most the largest one (det R_Z grows as Z shrinks)
    assert f[17] <= 1e-12 and f[19] <= 1e-12


def test_quantile_loss_gradient_against_finite_differences():
    rng = np.random.default_rng(4)
    P = ref.n_params()
    theta = rng.normal(0, 0.3, size=P)
    X = rng.normal(0, 1, size=(19, ref.NFEAT))
    y = rng.normal(0, 1, size=19)
    mean, std = np.zeros(ref.NFEAT), np.ones(ref.NFEAT)
    loss, grad = ref.mlp_loss_and_grad(theta, X, y, mean, std, quantile=0.9)
    pred = ref.mlp_forward(theta, X, mean, std)
    r = y - pred
    assert abs(loss - np.mean(np.maximum(0.9 * r, -0.1 * r))) < 1e-14
    for p in rng.choice(P, size=40, replace=False):
        h = 1e-7
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        lp, _ = ref.mlp_loss_and_grad(tp, X, y, mean, std, quantile=0.9)
        lm, _ = ref.mlp_loss_and_grad(tm, X, y, mean, std, quantile=0.9)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[p]) <= 1e-6 * max(1.0, abs(fd)), p


@pytest.mark.parametrize("n,seed", [(6, 1), (8, 2), (10, 3)])
def test_fallback_bits_cover_the_actual_cancellation(n, seed):
    """The bound estimate must ask for at least the bits the alternating sum
    actually loses plus the wanted digits."""
    O = g.random_instance(n, seed)
    r = oracle.tor(O)
    tau = 1e-3
    bits = ref.fallback_bits(O, tau)
    assert bits >= math.log2(r["kappa"]) + math.log2(1 / tau)


def test_fallback_bits_thermal_matches_eq6():
    # O = a I: Eq. 6 with k = 0 is exact; the estimate is then the rigorous
    # S_abs bound over the exact Tor
    a, n, tau = 0.2, 9, 1e-3
    O = (a * np.eye(2 * n)).astype(np.complex128)
    bits = ref.fallback_bits(O, tau)
    want = (n - n * math.log2(1 - a)) - n * math.log2(a / (1 - a)) + math.log2(1 / tau) \
        + math.log2(0.5 * 2 ** n * n * n)
    assert abs(bits - want) < 1e-9


def test_library_fallback_matches_reference():
    from paper_2009_01177_amd import tor_fallback_bits
    for seed in range(4):
        O = g.random_instance(5 + seed, 40 + seed)
        f = ref.features(O)
        for tau in (1e-3, 1e-6):
            assert abs(tor_fallback_bits(f, tau) - ref.fallback_bits(O, tau)) < 1e-9


def test_mlp_gradient_against_finite_differences():
    rng = np.random.default_rng(0)
    P = ref.n_params()
    theta = rng.normal(0, 0.3, size=P)
    X = rng.normal(0, 1, size=(17, ref.NFEAT))
    y = rng.normal(0, 1, size=17)
    mean, std = np.zeros(ref.NFEAT), np.ones(ref.NFEAT)
    loss, grad = ref.mlp_loss_and_grad(theta, X, y, mean, std, under=3.0, over=1.0)
    # the loss is the forward pass's
    pred = ref.mlp_forward(theta, X, mean, std)
    err = y - pred
    assert abs(loss - np.mean(np.where(err > 0, 3.0, 1.0) * err ** 2)) < 1e-14
    for p in rng.choice(P, size=40, replace=False):
        h = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        lp, _ = ref.mlp_loss_and_grad(tp, X, y, mean, std, under=3.0, over=1.0)
        lm, _ = ref.mlp_loss_and_grad(tm, X, y, mean, std, under=3.0, over=1.0)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[p]) <= 1e-6 * max(1.0, abs(fd)), p


def test_selector_file_round_trip(tmp_path):
    import paper_2009_01177_amd as tor
    from paper_2009_01177_amd import _lib
    sel = _lib.TorSelectorC()
    rng = np.random.default_rng(1)
    for i in range(_lib.TOR_MLP_PARAMS):
        sel.theta[i] = rng.normal()
    for i in range(_lib.TOR_NFEAT):
        sel.mean[i], sel.std[i] = rng.normal(), 1.0 + rng.random()
        sel.fmin[i], sel.fmax[i] = -1.0 - i, 1.0 + i
    sel.log10_c[0], sel.log10_c[1], sel.log10_c[2] = 1.5, 2.0, 2.5
    sel.slope[0], sel.slope[1], sel.slope[2] = 0.55, 0.8, 1.0
    sel.margin = 0.7
    sel.nmin, sel.nmax, sel.trained, sel.target = 6, 24, 1, _lib.TOR_TARGET_ERR64
    old = tor.tor_selector_get()
    try:
        tor.tor_selector_set(sel)
        p = os.path.join(tmp_path, "sel.txt")
        tor.tor_selector_save(p)
        tor.tor_selector_set(None)
        assert tor.tor_selector_get().trained == 0
        tor.tor_selector_load(p)
        back = tor.tor_selector_get()
        assert list(back.theta) == list(sel.theta)
        assert list(back.std) == list(sel.std) and back.margin == sel.margin
        assert list(back.slope) == list(sel.slope) and list(back.log10_c) == list(sel.log10_c)
        assert (back.nmin, back.nmax, back.trained, back.target) == (6, 24, 1, _lib.TOR_TARGET_ERR64)
    finally:
        tor.tor_selector_set(old)


def test_selector_files_of_the_12_feature_networks_are_refused(tmp_path):
    """Version 3 files hold the 20-feature network and its target; files of
    earlier versions (12-feature networks) are refused, as are a slope
    outside (0, 2] for a kappa-target selector and an unknown target."""
    import paper_2009_01177_amd as tor
    from paper_2009_01177_amd import _lib
    old = tor.tor_selector_get()
    try:
        sel = _lib.TorSelectorC()
        for i in range(_lib.TOR_NFEAT):
            sel.std[i], sel.fmax[i] = 1.0, 1.0
        for t in range(3):
            sel.slope[t] = 0.5
        sel.nmin, sel.nmax, sel.trained, sel.target = 6, 24, 1, _lib.TOR_TARGET_KAPPA
        tor.tor_selector_set(sel)
        p = os.path.join(tmp_path, "v3.txt")
        tor.tor_selector_save(p)
        lines = open(p).read().splitlines()
        assert lines[0] == "tor_selector 3"
        for v in (1, 2):
            pv = os.path.join(tmp_path, f"v{v}.txt")
            open(pv, "w").write("\n".join([f"tor_selector {v}"] + lines[1:]) + "\n")
            with pytest.raises(tor.TorError):
                tor.tor_selector_load(pv)
        sel.slope[0] = 0.0
        with pytest.raises(tor.TorError):
            tor.tor_selector_set(sel)
        sel.slope[0] = 0.5
        sel.target = 7
        with pytest.raises(tor.TorError):
            tor.tor_selector_set(sel)
    finally:
        tor.tor_selector_set(old)

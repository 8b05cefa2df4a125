"""Precision selector on the GPU: feature kernel and MLP kernels against the
binary64 reference, training, the TOR_AUTO path's accuracy, the gain of the
trained network over the bound estimate alone, and spot re-evaluation."""
import math
import os

import numpy as np
import pytest

import gbs_inputs as g
from oracle import selector_ref as ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tor():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_01177_amd as t
    t.tor_init()
    return t


def test_features_kernel_matches_reference(tor):
    Os = [g.random_instance(n, 300 + n) for n in [1, 2, 3, 5, 8, 13, 17, 21, 30, 40]]
    f = tor.tor_features(tor.Batch(Os)).cpu().numpy()
    for k, O in enumerate(Os):
        want = ref.features(O)
        print(f"[features] n={O.shape[0] // 2}", flush=True)
        assert np.allclose(f[k], want, rtol=1e-10, atol=1e-10), (k, f[k] - want)


def test_features_at_the_largest_n(tor):
    """R and its inverse share one array in LDS, so every feature is
    defined up to n = TOR_NMAX; instances of 47 and 50 modes match the
    reference, and a small instance in the same launch keeps its features."""
    Os = [g.random_instance(47, 77), g.random_instance(9, 78), g.random_instance(50, 79)]
    f = tor.tor_features(tor.Batch(Os)).cpu().numpy()
    for k in range(3):
        assert np.all(np.isfinite(f[k]))
        assert np.allclose(f[k], ref.features(Os[k]), rtol=1e-10, atol=1e-10), (k, f[k] - ref.features(Os[k]))


def test_mlp_kernels_match_reference(tor):
    import torch
    rng = np.random.default_rng(5)
    P = ref.n_params()
    theta = rng.normal(0, 0.4, size=P)
    X = rng.normal(0, 2, size=(300, ref.NFEAT))
    y = rng.normal(0, 3, size=300)
    mean = rng.normal(0, 1, size=ref.NFEAT)
    std = 0.5 + rng.random(ref.NFEAT)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    Y = tor.tor_mlp_forward(d(theta), d(mean), d(std), d(X)).cpu().numpy()
    assert np.allclose(Y, ref.mlp_forward(theta, X, mean, std), rtol=1e-12, atol=1e-12)
    grad, loss = tor.tor_mlp_grad(d(theta), d(mean), d(std), d(X), d(y), under=4.0, over=1.0)
    lw, gw = ref.mlp_loss_and_grad(theta, X, y, mean, std, under=4.0, over=1.0)
    assert abs(loss.item() - lw) <= 1e-12 * abs(lw)
    assert np.allclose(grad.cpu().numpy(), gw, rtol=1e-10, atol=1e-13)
    grad, loss = tor.tor_mlp_grad_quantile(d(theta), d(mean), d(std), d(X), d(y), q=0.9)
    lw, gw = ref.mlp_loss_and_grad(theta, X, y, mean, std, quantile=0.9)
    assert abs(loss.item() - lw) <= 1e-12 * abs(lw)
    assert np.allclose(grad.cpu().numpy(), gw, rtol=1e-10, atol=1e-13)


def test_adam_step_matches_reference(tor):
    import torch
    rng = np.random.default_rng(6)
    P = ref.n_params()
    th, gr = rng.normal(size=P), rng.normal(size=P)
    m, v = rng.normal(size=P) * 0.1, rng.random(P) * 0.1
    lr, b1, b2, eps, step = 1e-2, 0.9, 0.999, 1e-8, 3
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    tt, mm, vv = d(th), d(m), d(v)
    tor.tor_mlp_adam(tt, d(gr), mm, vv, lr, step, b1, b2, eps)
    m2 = b1 * m + (1 - b1) * gr
    v2 = b2 * v + (1 - b2) * gr * gr
    th2 = th - lr * (m2 / (1 - b1 ** step)) / (np.sqrt(v2 / (1 - b2 ** step)) + eps)
    assert np.allclose(tt.cpu().numpy(), th2, rtol=1e-14, atol=1e-15)
    assert np.allclose(mm.cpu().numpy(), m2, rtol=1e-15, atol=0)


def _reference_qd(tor, Os):
    return tor.tor_eval_batched(tor.Batch(Os), tiers="qd")


def _meets(res, ref_, tau):
    bad = []
    for k, (r, q) in enumerate(zip(res, ref_)):
        tq = q.exact
        if tq == 0:
            continue
        if float(abs(r.exact - tq) / abs(tq)) > tau:
            bad.append(k)
    return bad


def test_auto_with_bound_estimate_only_meets_tau(tor):
    tor.tor_selector_set(None)
    Os = [O for O in g.batched_workload(batch=200) if O.shape[0] // 2 <= 18][:120]
    b = tor.Batch(Os)
    res = tor.tor_eval_batched(b, tau=1e-3)
    st = tor.tor_last_select_stats()
    assert st["n_fallback"] == len(Os)
    assert not _meets(res, _reference_qd(tor, Os), 1e-3)


def test_labels_are_the_reference_evaluations(tor):
    """tor_selector_label: log10 kappa and the FP64 / DD forward errors
    against the quad-double evaluation of the same instance, recomputed here
    from the exact expansions of the same batched evaluations."""
    Os = [g.random_instance(n, 600 + n) for n in (4, 9, 14)] + [np.zeros((0, 0), np.complex128)]
    b = tor.Batch(Os)
    L = tor.tor_selector_label(b, "qd")
    assert np.all(np.isnan(L[3]))
    res = {t: tor.tor_eval_batched(b, tiers=t) for t in ("qd", "fp64", "dd")}
    for k, O in enumerate(Os[:3]):
        q = res["qd"][k]
        assert abs(L[k, 0] - math.log10(float(q.abs_exact / abs(q.exact)))) < 1e-12
        for col, tier, u in ((1, "fp64", 2.0 ** -53), (2, "dd", 2.0 ** -104)):
            r = res[tier][k]
            e = float(abs(r.exact - q.exact) / abs(q.exact))
            want = max(math.log10(e) if e > 0 else -400.0, math.log10(u) - 2.0)
            assert abs(L[k, col] - want) < 1e-9, (k, col, L[k, col], want)
        assert np.isnan(L[k, 3])


@pytest.fixture(scope="module")
def trained(tor, tmp_path_factory):
    """A selector trained through tor_selector_train on a quickly labelled
    set: 8 states of the batched workload's family (other seeds), n 6..18."""
    from paper_2009_01177_amd import selector
    path = str(tmp_path_factory.mktemp("sel") / "selector.txt")
    X, L, n = selector.label(selector.family_instances(8, 60, 7000, 6, 18))
    sel, losses = selector.fit(X, L, n, epochs=150)
    tor.tor_selector_set(sel)
    tor.tor_selector_save(path)
    return sel, (X, L, n), losses, path


def test_training_reduces_the_loss(trained):
    _, _, losses, _ = trained
    assert losses[-1] < 0.25 * losses[0]


def test_training_is_reproducible(tor, trained):
    """The same samples and options give the same selector bit for bit."""
    from paper_2009_01177_amd import selector
    sel, (X, L, n), _, _ = trained
    again, _ = selector.fit(X, L, n, epochs=150)
    assert bytes(again) == bytes(sel)


def test_shipped_selector_retrains_from_its_training_set(tor):
    """Retraining through tor_selector_train from the shipped training set
    with the shipped options gives the shipped selector bit for bit, so its
    tiers on the whole 4096-pattern benchmark batch at tau = 1e-3 are the
    same."""
    from paper_2009_01177_amd import selector
    X, L, n = selector.load_training_set()
    sel, _ = selector.fit(X, L, n)
    tor.tor_selector_load(selector.DEFAULT_PATH)
    shipped = tor.tor_selector_get()
    assert bytes(sel) == bytes(shipped)
    b = tor.Batch(g.batched_workload(batch=4096))
    t_shipped, _, _ = tor.tor_select_tiers(b, 1e-3)
    tor.tor_selector_set(sel)
    t_new, _, _ = tor.tor_select_tiers(b, 1e-3)
    selector.load_default()
    assert np.array_equal(t_new, t_shipped)


def test_trained_selector_meets_tau_and_gains_over_bounds(tor, trained):
    """The trained network's tiers meet tau on a held-out batch from the
    batched workload's state, and route more instances to the FP64 tier
    than the bound estimate alone would."""
    sel, _, _, path = trained
    tor.tor_selector_load(path)
    Os = [O for O in g.batched_workload(batch=600) if 6 <= O.shape[0] // 2 <= 18][:200]
    b = tor.Batch(Os)
    refq = _reference_qd(tor, Os)
    for tau in (1e-3, 1e-6):
        res = tor.tor_eval_batched(b, tau=tau)
        st = tor.tor_last_select_stats()
        print(f"[selector] tau={tau} {st}", flush=True)
        assert not _meets(res, refq, tau)
        t_net, _, src = tor.tor_select_tiers(b, tau)
        tor.tor_selector_set(None)
        t_fb, _, _ = tor.tor_select_tiers(b, tau)
        tor.tor_selector_load(path)
        cheap_net = int((t_net == 0).sum())
        cheap_fb = int((t_fb == 0).sum())
        print(f"[selector] tau={tau} fp64 picks: network {cheap_net}, bounds {cheap_fb}", flush=True)
        assert cheap_net >= cheap_fb
    assert cheap_net > cheap_fb or cheap_net == len(Os)


def test_spot_check_escalates_a_wrong_choice(tor, trained):
    """A selector whose FP64 error factor is set far too low picks FP64 where
    it cannot meet tau; with every such instance spot-checked, the misses are
    found and moved up a tier."""
    from paper_2009_01177_amd import _lib
    _, _, _, path = trained
    tor.tor_selector_load(path)
    sel = tor.tor_selector_get()
    sel.log10_c[0] = -30.0
    tor.tor_selector_set(sel)
    Os = [O for O in g.batched_workload(batch=300) if 12 <= O.shape[0] // 2 <= 18][:40]
    b = tor.Batch(Os)
    old = {k: os.environ.get(k) for k in ("TOR_SPOT_FRACTION", "TOR_SPOT_WINDOW")}
    os.environ["TOR_SPOT_FRACTION"] = "1"
    os.environ["TOR_SPOT_WINDOW"] = "100"  # the doctored factor puts every prediction far below tau
    try:
        res = tor.tor_eval_batched(b, tau=1e-6)
        st = tor.tor_last_select_stats()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
        tor.tor_selector_load(path)
    print(f"[spot] {st}", flush=True)
    assert st["n_fp64"] > 0 and st["n_violations"] > 0 and st["n_escalated"] > 0
    assert not _meets(res, _reference_qd(tor, Os), 1e-6)


def test_spot_samples_ride_in_the_batch(tor, trained):
    """Every network choice sampled (TOR_SPOT_FRACTION = 1, a wide window):
    the re-evaluations one tier up run in the batch's own launch sequence,
    into slots after the batch's.  Each instance's result (fixed tiers, n = 0
    and TOR_AUTO mixed) is its own evaluation at the tier it reports, within
    that tier's tolerance of S_abs; graph replays give the same bits."""
    _, _, _, path = trained
    tor.tor_selector_load(path)
    Os = [O for O in g.batched_workload(batch=200) if 6 <= O.shape[0] // 2 <= 16][:48]
    Os = Os[:20] + [np.zeros((0, 0), dtype=np.complex128)] + Os[20:]
    tiers = ["auto"] * len(Os)
    tiers[3], tiers[7], tiers[30] = "dd", "fp64", "qd"
    b = tor.Batch(Os)
    old = {k: os.environ.get(k) for k in ("TOR_SPOT_FRACTION", "TOR_SPOT_WINDOW")}
    os.environ["TOR_SPOT_FRACTION"] = "1"
    os.environ["TOR_SPOT_WINDOW"] = "100"
    try:
        res = tor.tor_eval_batched(b, tiers=tiers, tau=1e-3)
        st = tor.tor_last_select_stats()
        again = tor.tor_eval_batched(b, tiers=tiers, tau=1e-3, graph=True)
        again = tor.tor_eval_batched(b, tiers=tiers, tau=1e-3, graph=True)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    print(f"[spot] {st}", flush=True)
    _, _, src = tor.tor_select_tiers(b, 1e-3)
    n_net = sum(1 for k, O in enumerate(Os) if tiers[k] == "auto" and O.shape[0] > 0 and src[k] == 0)
    assert n_net > 0 and st["n_spot"] == n_net
    assert st["n_violations"] > 0 or st["n_escalated"] == 0
    tol = {0: 1e-12, 1: 1e-25, 2: 1e-30}
    for k, (O, r) in enumerate(zip(Os, res)):
        if O.shape[0] == 0:
            assert r.exact == 1
            continue
        if tiers[k] != "auto":
            assert r.tier_used == tor.tier_id(tiers[k])
        one = tor.tor_eval(O, tier=r.tier_used)
        assert abs(r.exact - one.exact) <= tol[r.tier_used] * one.abs_exact, k
    assert [(r.expansion, r.tier_used) for r in again] == [(r.expansion, r.tier_used) for r in res]


@pytest.mark.parametrize("learned", [False, True])
def test_auto_graph_replays_survive_spot_checks(tor, trained, learned):
    """Regression: TOR_AUTO with graph capture, called repeatedly.  Each call
    runs spot re-evaluations, which evaluate other plans between replays of
    the captured graph; every replay must equal the uncaptured result."""
    _, _, _, path = trained
    if learned:
        tor.tor_selector_load(path)
    else:
        tor.tor_selector_set(None)
    Os = [O for O in g.batched_workload(batch=400) if 8 <= O.shape[0] // 2 <= 20][:150]
    b = tor.Batch(Os)
    base = tor.tor_eval_batched(b, tau=1e-3)
    for rep in range(3):
        b.out.zero_()
        got = tor.tor_eval_batched(b, tau=1e-3, graph=True)
        assert [r.expansion for r in got] == [r.expansion for r in base], rep
    tor.tor_selector_load(path)

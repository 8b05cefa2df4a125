"""Batched path (many instances of uneven n, one launch sequence, optional
HIP graph) against the float128 oracle and against single evaluations."""
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


def _mixed(count, nlo, nhi, seed):
    rng = np.random.default_rng(seed)
    Os = []
    for i in range(count):
        n = int(rng.integers(nlo, nhi + 1))
        Os.append(g.random_instance(n, seed * 1000 + i) if n > 0 else np.zeros((0, 0), np.complex128))
    return Os


@pytest.mark.parametrize("tier", ["fp64", "dd", "qd"])
def test_batch_matches_oracle(tor, tier):
    Os = _mixed(40, 0, 13, 7)
    print(f"[batched] tier={tier} ns={[o.shape[0] // 2 for o in Os]}", flush=True)
    b = tor.Batch(Os)
    res = tor.tor_eval_batched(b, tiers=tier)
    for O, r in zip(Os, res):
        ref = oracle.tor(O)
        assert r.status == 0
        assert float(abs(r.exact - ref["tor"]) / ref["abs_sum"]) <= TOL[tier]


def test_batch_mixed_tiers_and_single_agreement(tor):
    Os = _mixed(30, 1, 18, 11)
    tiers = ["fp64", "dd", "qd"] * 10
    b = tor.Batch(Os)
    res = tor.tor_eval_batched(b, tiers=tiers)
    for O, t, r in zip(Os, tiers, res):
        one = tor.tor_eval(O, tier=t, algo="schur")
        assert r.tier_used == one.tier_used
        assert float(abs(r.exact - one.exact) / one.abs_exact) <= TOL[t]


def test_graph_replay_is_bitwise_identical(tor):
    import torch
    Os = _mixed(64, 4, 16, 3)
    b = tor.Batch(Os)
    eager = tor.tor_eval_batched(b, tiers="dd")
    for rep in range(3):
        b.out.zero_()
        # unrelated eager work on the same stream between replays
        x = torch.randn(1000, device="cuda").sum().item()
        got = tor.tor_eval_batched(b, tiers="dd", graph=True)
        assert [r.expansion for r in got] == [r.expansion for r in eager], rep
        assert np.isfinite(x)


def test_not_positive_definite_instance_is_flagged(tor):
    Os = _mixed(6, 3, 6, 5)
    Os[2] = (2.0 * np.eye(8)).astype(np.complex128)
    b = tor.Batch(Os)
    res = tor.tor_eval_batched(b, tiers="dd")
    assert [r.status for r in res] == [0, 0, -2, 0, 0, 0]


def test_config3_like_batch(tor):
    """The batched workload's generator (one 100-mode lossy state, uneven
    click patterns), cut to 96 instances of n <= 14 for the oracle."""
    Os = [O for O in g.batched_workload(batch=400) if O.shape[0] // 2 <= 14][:96]
    b = tor.Batch(Os)
    res = tor.tor_eval_batched(b, tiers="dd", graph=True)
    for O, r in zip(Os, res):
        ref = oracle.tor(O)
        assert float(abs(r.exact - ref["tor"]) / ref["abs_sum"]) <= 1e-25


def test_the_full_benchmark_batch_sampled(tor):
    """The whole 4096-pattern batch (n ~ U{8..24}) in one graph-captured
    launch sequence, as bench.py times it, in fixed DD and with selected
    tiers at tau = 1e-3: 40 instances with n <= 14 against the binary128
    oracle, 8 with n >= 22 against their single quad-double evaluation."""
    from paper_2009_01177_amd import selector
    Os = g.batched_workload(batch=4096)
    ns = np.array([O.shape[0] // 2 for O in Os])
    b = tor.Batch(Os)
    print("[batched] full 4096 batch, dd and auto", flush=True)
    dd = tor.tor_eval_batched(b, tiers="dd", graph=True)
    selector.load_default()
    auto = tor.tor_eval_batched(b, tau=1e-3, graph=True)
    small = np.flatnonzero(ns <= 14)[:40]
    large = np.flatnonzero(ns >= 22)[:8]
    assert len(small) == 40 and len(large) == 8
    for k in small:
        ref = oracle.tor(Os[k])
        assert float(abs(dd[k].exact - ref["tor"]) / ref["abs_sum"]) <= 1e-25, k
        if ref["tor"] != 0:
            assert float(abs(auto[k].exact - ref["tor"]) / abs(ref["tor"])) <= 1e-3, k
    for k in large:
        q = tor.tor_eval(Os[k], tier="qd")
        assert float(abs(dd[k].exact - q.exact) / q.abs_exact) <= 1e-25, k
        assert float(abs(auto[k].exact - q.exact) / abs(q.exact)) <= 1e-3, k


def _results_equal(a, b):
    return [r.expansion for r in a] == [r.expansion for r in b]


@pytest.mark.parametrize("graph", [False, True])
def test_fixed_tier_batches_return_before_their_work_ends(tor, graph):
    """A fixed-tier batch is stream-ordered: the call returns while its
    kernels still run (an event recorded right after it is not yet
    complete), and the results are those of a synchronous call.  With
    graph=True the second call is a replay of the cached graph."""
    import torch
    Os = [g.random_instance(26, 900 + i) for i in range(12)]
    b = tor.Batch(Os)
    ref = tor.tor_eval_batched(b, tiers="dd", graph=graph)
    torch.cuda.synchronize()
    b.out.zero_()
    torch.cuda.synchronize()
    tor.tor_eval_batched(b, tiers="dd", graph=graph, sync=False)
    ev = torch.cuda.Event()
    ev.record()
    pending = not ev.query()
    torch.cuda.synchronize()
    from paper_2009_01177_amd.api import _results_from
    got = _results_from(b.out[:b.batch].cpu().numpy())
    print(f"[batched] graph={graph} returned before completion: {pending}", flush=True)
    assert pending
    assert _results_equal(got, ref)


def test_back_to_back_eager_batches_keep_their_plans(tor):
    """More eager batches in flight on one stream than there are plan slots,
    each with its own plan and output: every result matches the batch's
    synchronous evaluation bit for bit (a slot is reused only after the batch
    that last used it has finished)."""
    import torch
    from paper_2009_01177_amd.api import _results_from
    batches = [tor.Batch(_mixed(6 + k, 4, 14, 40 + k)) for k in range(9)]
    refs = [tor.tor_eval_batched(bk, tiers="dd") for bk in batches]
    for bk in batches:
        bk.out.zero_()
    torch.cuda.synchronize()
    for bk in batches:
        tor.tor_eval_batched(bk, tiers="dd", sync=False)
    torch.cuda.synchronize()
    for k, bk in enumerate(batches):
        assert _results_equal(_results_from(bk.out[:bk.batch].cpu().numpy()), refs[k]), k

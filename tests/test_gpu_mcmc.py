"""Markov-chain sampler entry point (tor_mcmc) against the reference chains
of oracle/sampler_ref.py: the same candidates and variates give the same
chain states, and every candidate's Torontonian meets the tier's tolerance
(|dTor| <= tol * S_abs).  At the throughput workload's full size, properties
that hold at any size plus one candidate scored by the oracle."""
import os

import numpy as np
import pytest

import gbs_inputs as gi
from oracle import sampler_ref as sr

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


def _reference(name, chains, steps):
    key = (name, chains, steps)
    if key not in _REF:
        sq, O = gi.mcmc_state(name)
        P = gi.mcmc_proposals(name, chains, steps)
        U = gi.mcmc_uniforms(name, chains, steps)
        _REF[key] = (O, P, U, sr.mcmc(O, P, U))
    return _REF[key]


def _check_against_reference(tor, name, chains, steps, tier):
    O, P, U, ref = _reference(name, chains, steps)
    print(f"[mcmc] {name} chains={chains} steps={steps} tier={tier}", flush=True)
    state, cand = tor.tor_mcmc(O, P, U, tier=tier)
    res = tor.results_of(cand)
    for k, r in enumerate(res):
        t, b = divmod(k, chains)
        key = tuple(int(m) for m in P[t, b])
        exact, sabs = ref["exact"][key]
        assert r.status == 0 and r.tier_used == tor.tier_id(tier)
        assert float(abs(r.exact - exact) / sabs) <= TOL[tier], (t, b)
    # decisions agree unless the reference's u Tor(x) and Tor(c) lie closer
    # than the tier's error (tol * S_abs on each score) can move them; the
    # seeded inputs have no such near-tie, so the chains must be identical
    kap = {k: float(v[1] / v[0]) for k, v in ref["exact"].items()}
    S = ref["state_step"]
    for t in range(1, steps):
        for b in range(chains):
            kx = kap[tuple(int(m) for m in P[S[t - 1, b], b])]
            kc = kap[tuple(int(m) for m in P[t, b])]
            assert ref["margin"][t, b] > TOL[tier] * (kx + kc) + 1e-15, (t, b)
    assert np.array_equal(state.cpu().numpy(), S)


@pytest.mark.parametrize("tier", ["fp64", "dd", "qd"])
def test_chains_match_reference_n8(tor, tier):
    _check_against_reference(tor, "mcmc_m24_n8", 64, 24, tier)


def test_chains_match_reference_n14_several_tiles(tor):
    _check_against_reference(tor, "mcmc_m24_n14", 8, 6, "dd")


def test_chains_with_selected_tiers(tor):
    # TOR_AUTO: each candidate gets the cheapest tier the selector expects to
    # meet tau (relative to |Tor|); the seeded decisions are further from a
    # tie than 1e-4, so tau = 1e-8 leaves the chains unchanged
    tau = 1e-8
    O, P, U, ref = _reference("mcmc_m24_n8", 64, 24)
    print("[mcmc] mcmc_m24_n8 chains=64 steps=24 tier=auto", flush=True)
    state, cand = tor.tor_mcmc(O, P, U, tier="auto", tau=tau)
    used = set()
    for k, r in enumerate(tor.results_of(cand)):
        t, b = divmod(k, 64)
        exact = ref["exact"][tuple(int(m) for m in P[t, b])][0]
        assert r.status == 0
        used.add(r.tier_used)
        assert float(abs(r.exact - exact) / abs(exact)) <= 10 * tau
    assert used <= {tor.TOR_FP64, tor.TOR_DD, tor.TOR_QD}
    assert float(np.min(ref["margin"][1:])) > 1e-4
    assert np.array_equal(state.cpu().numpy(), ref["state_step"])


def test_chunked_scoring_gives_the_same_chains(tor, monkeypatch):
    O, P, U, ref = _reference("mcmc_m24_n8", 64, 24)
    state0, cand0 = tor.tor_mcmc(O, P, U, tier="dd")
    monkeypatch.setenv("TOR_MCMC_CHUNK", "100")
    print("[mcmc] chunks of 100 candidates", flush=True)
    state1, cand1 = tor.tor_mcmc(O, P, U, tier="dd")
    assert np.array_equal(state1.cpu().numpy(), state0.cpu().numpy())
    a = np.array([r.exact for r in tor.results_of(cand0)], dtype=object)
    b = np.array([r.exact for r in tor.results_of(cand1)], dtype=object)
    assert (a == b).all()


def test_no_clicks_and_certain_moves(tor):
    sq, O = gi.mcmc_state("mcmc_m5_n2")
    steps, chains = 5, 3
    P = np.zeros((steps, chains, 0), dtype=np.int32)
    U = gi.mcmc_uniforms("mcmc_m5_n2", chains, steps)
    state, cand = tor.tor_mcmc(O, P, U, tier="dd")
    assert all(r.value == 1.0 for r in tor.results_of(cand))
    assert (state.cpu().numpy() == np.arange(steps)[:, None]).all()
    # one chain, one step
    P = gi.mcmc_proposals("mcmc_m5_n2", 1, 1)
    state, cand = tor.tor_mcmc(O, P, np.zeros((1, 1)), tier="fp64")
    assert state.cpu().numpy().tolist() == [[0]]
    want = sr.pattern_tor(O, P[0, 0])
    assert abs(tor.results_of(cand)[0].exact - want) <= 1e-12 * abs(want)


def test_bad_candidates_are_rejected(tor):
    sq, O = gi.mcmc_state("mcmc_m5_n2")
    P = gi.mcmc_proposals("mcmc_m5_n2", 4, 3)
    U = gi.mcmc_uniforms("mcmc_m5_n2", 4, 3)
    for bad in ([1, 1], [3, 2], [0, 5], [-1, 2]):
        Q = P.copy()
        Q[2, 1] = bad
        with pytest.raises(tor.TorError) as e:
            tor.tor_mcmc(O, Q, U, tier="dd")
        assert e.value.code == -1
    V = U.copy()
    V[1, 3] = 1.5
    with pytest.raises(tor.TorError):
        tor.tor_mcmc(O, P, V, tier="dd")
    V[1, 3] = np.nan
    with pytest.raises(tor.TorError):
        tor.tor_mcmc(O, P, V, tier="dd")


def test_throughput_workload_properties_and_one_sampled_candidate(tor):
    # the sampler workload the benchmark times: 100 modes, 20 clicks,
    # 1024 chains x 16 steps in double-double
    name, chains, steps = "mcmc_m100_n20", 1024, 16
    sq, O = gi.mcmc_state(name)
    P = gi.mcmc_proposals(name, chains, steps)
    U = gi.mcmc_uniforms(name, chains, steps)
    print(f"[mcmc] {name} chains={chains} steps={steps} dd", flush=True)
    state, cand = tor.tor_mcmc(O, P, U, tier="dd")
    S = state.cpu().numpy()
    C = cand.cpu().numpy()
    status = C.reshape(-1, 8).view(np.int32)[:, 15].reshape(steps, chains)
    tc = C[:, :, 0]
    assert (status == 0).all() and (tc > 0).all() and np.isfinite(tc).all()
    # the decisions follow the rule on the returned scores
    cur = np.zeros(chains, dtype=np.int64)
    assert (S[0] == 0).all()
    for t in range(1, steps):
        move = np.array([sr.accepts(U[t, b], tc[cur[b], b], tc[t, b]) for b in range(chains)])
        cur = np.where(move, t, cur)
        assert np.array_equal(S[t], cur)
    # one candidate scored by the oracle (2^20 subsets in binary128)
    t, b = 11, 517
    exact, sabs = sr.pattern_tor_abs(O, P[t, b])
    r = tor.results_of(cand[t, b])[0]
    assert float(abs(r.exact - exact) / sabs) <= TOL["dd"]

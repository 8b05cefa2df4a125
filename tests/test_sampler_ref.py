"""Pins of the reference Markov-chain sampler (oracle/sampler_ref.py) to
facts it does not compute itself: the pattern probabilities of Eq. 1 summing
to one over all click patterns, the product-state factorisation with the
textbook vacuum probability of a squeezed mode, the move rule on hand-made
cases, and the chain's stationary law on a state small enough to
enumerate.  CPU only."""
import itertools
import math

import numpy as np
import pytest

import gbs_inputs as gi
from oracle import sampler_ref as sr


def _all_patterns(M):
    for k in range(M + 1):
        yield from itertools.combinations(range(M), k)


def test_probabilities_of_all_patterns_sum_to_one():
    sq, O = gi.mcmc_state("mcmc_m5_n2")
    total = math.fsum(sr.pattern_probability(O, sq, S) for S in _all_patterns(5))
    assert abs(total - 1.0) < 1e-12


@pytest.mark.parametrize("eta", [1.0, 0.55])
def test_product_state_factorises_with_single_mode_vacuum_probability(eta):
    # no interferometer: the modes are independent squeezed vacua, each after
    # a loss channel of transmission eta.  Its vacuum probability is
    # 1/sqrt(det sigma_Q) of the mode, which in closed form is
    # 2 / sqrt(eta^2 + 2 eta (2 - eta) cosh 2r + (2 - eta)^2)  (sech r when eta = 1).
    r = np.array([0.3, 0.7, 1.1, 0.5])
    M = r.size
    sq = gi.gbs_sigma_q(np.eye(M, dtype=np.complex128), r, eta)
    O = gi.o_from_sigma_q(sq)
    c = np.cosh(2 * r)
    v = 2.0 / np.sqrt(eta ** 2 + 2 * eta * (2 - eta) * c + (2 - eta) ** 2)
    if eta == 1.0:
        assert np.allclose(v, 1.0 / np.cosh(r), rtol=1e-14)
    for S in _all_patterns(M):
        want = math.prod((1 - v[k]) if k in S else v[k] for k in range(M))
        got = sr.pattern_probability(O, sq, S)
        assert abs(got - want) <= 1e-12 * want, (S, got, want)


def test_move_rule_cases():
    assert sr.accepts(0.5, 1.0, 0.6)
    assert not sr.accepts(0.5, 1.0, 0.4)
    assert sr.accepts(0.0, 1.0, 1e-300)
    assert sr.accepts(0.999999, 2.5, 2.5)  # equal probabilities always move
    assert not sr.accepts(0.25, 4.0, 1.0)  # exactly a tie: u p(x) = p(c) stays


def test_repeated_candidate_always_moves_and_state_steps_are_valid():
    sq, O = gi.mcmc_state("mcmc_m5_n2")
    P = np.tile(np.array([1, 3], dtype=np.int32), (6, 3, 1))
    U = gi.mcmc_uniforms("mcmc_m5_n2", 3, 6)
    r = sr.mcmc(O, P, U)
    assert (r["state_step"] == np.arange(6)[:, None]).all()
    P = gi.mcmc_proposals("mcmc_m5_n2", 50, 20)
    U = gi.mcmc_uniforms("mcmc_m5_n2", 50, 20)
    r = sr.mcmc(O, P, U)
    S = r["state_step"]
    assert (S[0] == 0).all()
    for t in range(1, 20):
        assert np.all((S[t] == S[t - 1]) | (S[t] == t))
    pats = sr.chain_patterns(P, S)
    assert pats.shape == P.shape and (pats[0] == P[0]).all()


def test_chains_reach_the_n_click_law():
    # 10 two-click patterns of 5 modes; uniform candidates; after 30 steps
    # the 4000 independent chains' end states follow p(S | N = 2)
    name, chains, steps = "mcmc_m5_n2", 4000, 30
    sq, O = gi.mcmc_state(name)
    pats = list(itertools.combinations(range(5), 2))
    p = np.array([sr.pattern_probability(O, sq, S) for S in pats])
    law = p / p.sum()
    # the law is far from uniform (so a wrong rule shows) and the
    # independence chain mixes at rate 1 - q/max(law) per step
    assert 0.5 * np.abs(law - 0.1).sum() > 0.15
    assert (1 - 0.1 / law.max()) ** steps < 1e-3
    P = gi.mcmc_proposals(name, chains, steps)
    U = gi.mcmc_uniforms(name, chains, steps)
    r = sr.mcmc(O, P, U)
    end = sr.chain_patterns(P, r["state_step"])[-1]
    idx = {S: i for i, S in enumerate(pats)}
    counts = np.bincount([idx[tuple(int(m) for m in row)] for row in end], minlength=10)
    expect = chains * law
    chi2 = float(((counts - expect) ** 2 / expect).sum())
    assert chi2 < 40.0, (chi2, counts, expect)  # 9 degrees of freedom
    # the inverted rule's law (proportional to 1/p) is rejected by the same counts
    inv = (1 / p) / (1 / p).sum()
    chi2_inv = float(((counts - chains * inv) ** 2 / (chains * inv)).sum())
    assert chi2_inv > 400.0

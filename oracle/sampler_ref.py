"""Reference Markov-chain sampler over N-click patterns (Sec. 7.1.1 with
Sec. 3.1, Eq. 1-2).

TEST INFRASTRUCTURE ONLY: used by the test suite and the benchmark's CPU
leg, never by the library.  It shares no code with the GPU path; its
Torontonians come from the binary128 oracle (oracle.tor).

The paper scores about a hundred candidate click patterns per sample with a
Markov chain Monte Carlo sampler (Sec. 7.1.1).  The chain here is an
independence Metropolis sampler over patterns with exactly N clicks:

  - the probability of pattern S is p(S) = Tor(O_S) / sqrt(det sigma_Q)
    (Eq. 1), where O_S keeps rows and columns k and M+k of the M-mode O for
    every clicked mode k;
  - candidates are drawn without regard to the chain's state (the caller
    passes them in, one N-subset per step and chain), and so are the
    acceptance variates u in [0, 1);
  - step 0 takes its candidate; at a later step a chain at x moves to the
    candidate c when u * Tor(O_x) < Tor(O_c).  Both Torontonians are rounded
    to binary64 and the product is formed in binary64.  The vacuum factor
    1/sqrt(det sigma_Q) is the same for every pattern of a state, so it
    cancels; with a symmetric proposal the chain moves with probability
    min(1, p(c) / p(x)) and p restricted to N-click patterns is its
    stationary law.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from . import tor as _oracle_tor


def pattern_o(O_full, modes) -> np.ndarray:
    """O_S of the clicked modes (ascending), block order kept (Eq. 1)."""
    O_full = np.asarray(O_full, dtype=np.complex128)
    M = O_full.shape[0] // 2
    k = np.sort(np.asarray(modes, dtype=np.int64))
    rows = np.concatenate([k, k + M])
    return np.ascontiguousarray(O_full[rows][:, rows])


def pattern_tor(O_full, modes, threads: int = 0) -> Fraction:
    """Tor(O_S) exactly as a Fraction (Eq. 2); Tor of no clicks is 1."""
    return pattern_tor_abs(O_full, modes, threads)[0]


def pattern_tor_abs(O_full, modes, threads: int = 0):
    """(Tor(O_S), S_abs) as Fractions, S_abs the sum of the terms' magnitudes."""
    if len(modes) == 0:
        return Fraction(1), Fraction(1)
    r = _oracle_tor(pattern_o(O_full, modes), threads=threads)
    return r["tor"], r["abs_sum"]


def pattern_probability(O_full, sigma_q, modes) -> float:
    """p(S) = Tor(O_S) / sqrt(det sigma_Q) (Eq. 1), in binary64."""
    sign, logdet = np.linalg.slogdet(np.asarray(sigma_q, dtype=np.complex128))
    return float(pattern_tor(O_full, modes)) * float(np.exp(-0.5 * logdet.real))


def accepts(u: float, tor_x: float, tor_c: float) -> bool:
    """The move rule: u * Tor(O_x) < Tor(O_c) in binary64."""
    return float(u) * float(tor_x) < float(tor_c)


def mcmc(O_full, proposals, uniforms, threads: int = 0, cache: dict | None = None) -> dict:
    """Run chains side by side.

    proposals  steps x chains x N mode indices (each row ascending)
    uniforms   steps x chains acceptance variates
    Returns dict with
      state_step  steps x chains int32: after step t chain b holds the
                  candidate of step state_step[t, b] (<= t)
      tor         steps x chains float64: Tor of each candidate, rounded
      margin      steps x chains float64: |u Tor(O_x) - Tor(O_c)| / Tor(O_c)
                  of each decision (inf at step 0), how far it was from a tie
      exact       {pattern tuple: (Tor, S_abs) as Fractions} of every
                  candidate scored
    A pattern seen twice is scored once (cache, same layout as exact).
    """
    P = np.asarray(proposals)
    U = np.asarray(uniforms, dtype=np.float64)
    steps, chains = P.shape[0], P.shape[1]
    assert U.shape == (steps, chains)
    exact = {} if cache is None else cache
    tor = np.empty((steps, chains), dtype=np.float64)
    for t in range(steps):
        for b in range(chains):
            key = tuple(int(m) for m in P[t, b])
            if key not in exact:
                exact[key] = pattern_tor_abs(O_full, key, threads=threads)
            tor[t, b] = float(exact[key][0])
    state_step = np.zeros((steps, chains), dtype=np.int32)
    margin = np.full((steps, chains), np.inf)
    for b in range(chains):
        cur = 0
        for t in range(1, steps):
            tx, tc = tor[cur, b], tor[t, b]
            if tc != 0.0:
                margin[t, b] = abs(U[t, b] * tx - tc) / abs(tc)
            if accepts(U[t, b], tx, tc):
                cur = t
            state_step[t, b] = cur
    return dict(state_step=state_step, tor=tor, margin=margin, exact=exact)


def chain_patterns(proposals, state_step) -> np.ndarray:
    """steps x chains x N: the pattern each chain holds after each step."""
    P = np.asarray(proposals)
    S = np.asarray(state_step)
    b = np.arange(P.shape[1])[None, :]
    return P[S, b]

"""Seeded synthetic Gaussian-boson-sampling inputs.

This module builds the matrices that the Torontonian is evaluated on and
nothing else: it holds no part of the Torontonian arithmetic (no subset
enumeration, no determinant, no summation).  Both the float128 oracle's
tests and the GPU path's tests and benchmark draw their inputs from here.

Conventions (Sec. 3.1, Eq. 1):
  * A Gaussian state of M modes is described in the complex (a, a^dagger)
    basis by a 2M x 2M covariance matrix; vacuum is I/2.
  * sigma_Q = sigma + I/2 (so the vacuum has det sigma_Q = 1, and the
    vacuum probability of any state is det(sigma_Q)^(-1/2)).
  * The sampling matrix is O = I - sigma_Q^{-1}  (the paper calls it A).
  * A click pattern S selects rows/columns k and M+k for every clicked k
    (Eq. 1), kept in block order [a-modes..., a^dagger-modes...].

Exactness: the oracle and the GPU path read different triangles of O (each
reads the lower triangle of its own row ordering), so O is made exactly
Hermitian with the block symmetries of Eq. 3 (O11 = conj(O00), O10 =
conj(O01), O01 symmetric) before it is handed out.  All of these operations
are exact in binary64.

Recipe for the benchmark states (Haar unitary by Mezzadri's QR method,
single-mode squeezing, a uniform-transmission loss channel):
  sigma_in  = 1/2 [[C, S], [S, C]],  C = diag(cosh 2r), S = diag(sinh 2r)
  sigma_out = W sigma_in W^H,        W = diag(U, conj(U))
  sigma     = eta sigma_out + (1 - eta) I/2
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "haar_unitary", "gbs_sigma_q", "o_from_sigma_q", "symmetrize_o",
    "click_submatrix", "workload", "batched_workload", "random_instance",
    "thermal_o", "squeezed_o", "lossy_squeezed_o", "tmsv_o", "direct_sum_o",
    "permute_and_phase_o", "interleave_perm", "WORKLOADS",
    "MCMC", "mcmc_state", "mcmc_proposals", "mcmc_uniforms",
]


def haar_unitary(m: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random m x m unitary (Mezzadri): QR of a complex Ginibre matrix,
    with the phases of R's diagonal moved into Q."""
    z = (rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return q * (d / np.abs(d))[None, :]


def gbs_sigma_q(U: np.ndarray, r: np.ndarray, eta: float) -> np.ndarray:
    """sigma_Q of squeezed vacua (squeezing r) sent through the interferometer
    U and a uniform loss channel of transmission eta."""
    m = U.shape[0]
    r = np.asarray(r, dtype=np.float64)
    c = np.diag(np.cosh(2.0 * r)).astype(np.complex128)
    s = np.diag(np.sinh(2.0 * r)).astype(np.complex128)
    sig_in = 0.5 * np.block([[c, s], [s, c]])
    W = np.block([[U, np.zeros_like(U)], [np.zeros_like(U), U.conj()]])
    sig_out = W @ sig_in @ W.conj().T
    eye = np.eye(2 * m, dtype=np.complex128)
    sig = eta * sig_out + (1.0 - eta) * 0.5 * eye
    sq = sig + 0.5 * eye
    return 0.5 * (sq + sq.conj().T)


def symmetrize_o(O: np.ndarray) -> np.ndarray:
    """Make O exactly Hermitian with the Eq. 3 block symmetries (exact in
    binary64: only averages of two values, which commute)."""
    n2 = O.shape[0]
    assert O.shape == (n2, n2) and n2 % 2 == 0
    n = n2 // 2
    X = O[:n, :n]
    Y = O[:n, n:]
    Xh = 0.5 * (X + X.conj().T)
    Ys = 0.5 * (Y + Y.T)
    out = np.empty_like(O, dtype=np.complex128)
    out[:n, :n] = Xh
    out[:n, n:] = Ys
    out[n:, :n] = Ys.conj()
    out[n:, n:] = Xh.conj()
    return np.ascontiguousarray(out)


def o_from_sigma_q(sigma_q: np.ndarray) -> np.ndarray:
    """O = I - sigma_Q^{-1}, symmetrised."""
    n2 = sigma_q.shape[0]
    O = np.eye(n2, dtype=np.complex128) - np.linalg.inv(sigma_q)
    return symmetrize_o(O)


def click_submatrix(O_full: np.ndarray, modes) -> np.ndarray:
    """O_S: rows/columns k and M+k for the clicked modes k (ascending),
    block order kept (Eq. 1)."""
    M = O_full.shape[0] // 2
    modes = np.sort(np.asarray(modes, dtype=np.int64))
    idx = np.concatenate([modes, modes + M])
    return np.ascontiguousarray(O_full[np.ix_(idx, idx)])


def interleave_perm(n: int) -> np.ndarray:
    """Row order (0, n, 1, n+1, ...) that pairs each mode's a and a^dagger
    rows; a symmetric permutation, so it leaves every principal minor's
    determinant unchanged."""
    p = np.empty(2 * n, dtype=np.int64)
    p[0::2] = np.arange(n)
    p[1::2] = np.arange(n) + n
    return p


# ---------------------------------------------------------------------------
# Closed-form test states
# ---------------------------------------------------------------------------

def thermal_o(nbar) -> np.ndarray:
    """Product of thermal modes: sigma_Q = diag(nbar+1, nbar+1) per mode, so
    O = diag(nbar/(nbar+1)) on both halves."""
    nbar = np.atleast_1d(np.asarray(nbar, dtype=np.float64))
    d = nbar / (nbar + 1.0)
    return np.diag(np.concatenate([d, d])).astype(np.complex128)


def squeezed_o(r: float, phi: float = 0.0) -> np.ndarray:
    """Single-mode squeezed vacuum (pure): O = [[0, conj(b)], [b, 0]] with
    b = e^{i phi} tanh r."""
    b = np.exp(1j * phi) * np.tanh(r)
    return np.array([[0.0, np.conj(b)], [b, 0.0]], dtype=np.complex128)


def lossy_squeezed_o(r: float, eta: float) -> np.ndarray:
    """Single-mode squeezed vacuum after loss, through sigma_Q."""
    return o_from_sigma_q(gbs_sigma_q(np.eye(1, dtype=np.complex128), np.array([r]), eta))


def tmsv_o(r: float) -> np.ndarray:
    """Two-mode squeezed vacuum (pure): O = [[0, conj(B)], [B, 0]] with
    B = tanh r [[0, 1], [1, 0]] (real, so conj(B) = B)."""
    t = np.tanh(r)
    B = np.array([[0.0, t], [t, 0.0]], dtype=np.complex128)
    Z = np.zeros((2, 2), dtype=np.complex128)
    return np.block([[Z, B.conj()], [B, Z]])


def direct_sum_o(blocks) -> np.ndarray:
    """O of a product state: each block is a 2k x 2k O (block order) of k
    modes; the result is in block order for all sum(k) modes."""
    sizes = [b.shape[0] // 2 for b in blocks]
    n = int(sum(sizes))
    O = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    off = 0
    for b, k in zip(blocks, sizes):
        a = np.arange(off, off + k)
        idx = np.concatenate([a, a + n])
        O[np.ix_(idx, idx)] = b
        off += k
    return O


def permute_and_phase_o(O: np.ndarray, perm, phases) -> np.ndarray:
    """Relabel modes by perm and rotate each mode's phase (a_k -> e^{i phi_k}
    a_k).  Neither changes any click probability; the rotation is
    D O D^H with D = diag(e^{i phi}, e^{-i phi})."""
    n = O.shape[0] // 2
    perm = np.asarray(perm, dtype=np.int64)
    idx = np.concatenate([perm, perm + n])
    P = O[np.ix_(idx, idx)]
    ph = np.exp(1j * np.asarray(phases, dtype=np.float64))
    d = np.concatenate([ph, ph.conj()])
    P = d[:, None] * P * d.conj()[None, :]
    return symmetrize_o(P)


# ---------------------------------------------------------------------------
# Benchmark workloads
# ---------------------------------------------------------------------------

# name -> (modes M, squeezing spec, transmission, clicked modes n, state seed,
# pattern seed).  squeezing spec: ("uniform", lo, hi) or ("const", r).
WORKLOADS = {
    "n16_lossless": dict(M=16, sq=("uniform", 0.5, 1.0), eta=1.0, n=16, seed=1, pseed=101),
    "n30_lossy": dict(M=100, sq=("uniform", 0.8, 1.6), eta=0.3, n=30, seed=2, pseed=102),
    "batch4096_n8_24": dict(M=100, sq=("uniform", 0.8, 1.6), eta=0.3, n=None, seed=2, pseed=103,
                            batch=4096, nlo=8, nhi=24),
    "n36_stress": dict(M=100, sq=("const", 1.5), eta=0.5, n=36, seed=4, pseed=104),
    "n40_lossy": dict(M=100, sq=("uniform", 1.0, 1.6), eta=0.3, n=40, seed=5, pseed=105),
}


def _state(spec):
    rng = np.random.Generator(np.random.PCG64(spec["seed"]))
    M = spec["M"]
    U = haar_unitary(M, rng)
    kind = spec["sq"][0]
    if kind == "uniform":
        r = rng.uniform(spec["sq"][1], spec["sq"][2], size=M)
    else:
        r = np.full(M, float(spec["sq"][1]))
    sq = gbs_sigma_q(U, r, spec["eta"])
    return sq, o_from_sigma_q(sq)


_STATE_CACHE: dict = {}


def state(name: str):
    """(sigma_Q, O_full) of a named workload's GBS state (cached)."""
    spec = WORKLOADS[name]
    key = (spec["M"], spec["sq"], spec["eta"], spec["seed"])
    if key not in _STATE_CACHE:
        _STATE_CACHE[key] = _state(spec)
    return _STATE_CACHE[key]


def workload(name: str, n: int | None = None):
    """(O, modes) for a single-instance workload; n overrides the number of
    clicked modes (same state, same pattern draw)."""
    spec = WORKLOADS[name]
    _, O_full = state(name)
    M = spec["M"]
    n = spec["n"] if n is None else int(n)
    if n == M:
        modes = np.arange(M)
    else:
        prng = np.random.Generator(np.random.PCG64(spec["pseed"]))
        modes = np.sort(prng.choice(M, size=n, replace=False))
    return click_submatrix(O_full, modes), modes


def batched_workload(name: str = "batch4096_n8_24", batch: int | None = None):
    """List of O matrices for the batched workload: click patterns with n
    drawn uniformly from {nlo..nhi} and modes uniformly without replacement."""
    spec = WORKLOADS[name]
    _, O_full = state(name)
    B = spec["batch"] if batch is None else int(batch)
    prng = np.random.Generator(np.random.PCG64(spec["pseed"]))
    out = []
    for _ in range(B):
        n = int(prng.integers(spec["nlo"], spec["nhi"] + 1))
        modes = np.sort(prng.choice(spec["M"], size=n, replace=False))
        out.append(click_submatrix(O_full, modes))
    return out


def random_instance(n: int, seed: int, M: int | None = None, r=(0.8, 1.6), eta=0.3):
    """A small random lossy GBS instance of n clicked modes out of M."""
    rng = np.random.Generator(np.random.PCG64(seed))
    M = max(n, 2 * n) if M is None else M
    U = haar_unitary(M, rng)
    rr = rng.uniform(r[0], r[1], size=M)
    sq = gbs_sigma_q(U, rr, eta)
    O_full = o_from_sigma_q(sq)
    modes = np.sort(rng.choice(M, size=n, replace=False))
    return click_submatrix(O_full, modes)


# --------------------------------------------------------------------------
# Markov-chain sampler inputs.  A chain walks over N-click patterns of an
# M-mode state; its proposals (uniform N-subsets of the modes, drawn without
# regard to the chain) and its acceptance variates are random numbers the
# sampler consumes, so they are generated here and passed in.
# --------------------------------------------------------------------------

MCMC = {
    # 5 modes, 2 clicks: 10 patterns, small enough to enumerate
    "mcmc_m5_n2": dict(M=5, N=2, sq=("uniform", 0.4, 1.2), eta=0.6, seed=21, pseed=121),
    # 24 modes, 8 clicks: parity runs
    "mcmc_m24_n8": dict(M=24, N=8, sq=("uniform", 0.6, 1.2), eta=0.4, seed=22, pseed=122),
    # 24 modes, 14 clicks: several middle-level tiles per Torontonian
    "mcmc_m24_n14": dict(M=24, N=14, sq=("uniform", 0.6, 1.2), eta=0.4, seed=22, pseed=123),
    # 100 modes, 20 clicks: the throughput workload
    "mcmc_m100_n20": dict(M=100, N=20, sq=("uniform", 0.8, 1.6), eta=0.3, seed=2, pseed=124),
}


def mcmc_state(name: str):
    """(sigma_Q, O_full) of a named sampler workload's M-mode state."""
    spec = MCMC[name]
    key = (spec["M"], spec["sq"], spec["eta"], spec["seed"])
    if key not in _STATE_CACHE:
        _STATE_CACHE[key] = _state(spec)
    return _STATE_CACHE[key]


def mcmc_proposals(name: str, chains: int, steps: int) -> np.ndarray:
    """steps x chains x N int32: for every step and chain an N-subset of the
    M modes drawn uniformly, ascending."""
    spec = MCMC[name]
    M, N = spec["M"], spec["N"]
    rng = np.random.Generator(np.random.PCG64(spec["pseed"]))
    out = np.empty((int(steps), int(chains), N), dtype=np.int32)
    for t in range(int(steps)):
        keys = rng.random((int(chains), M))
        out[t] = np.sort(np.argsort(keys, axis=1)[:, :N], axis=1)
    return out


def mcmc_uniforms(name: str, chains: int, steps: int) -> np.ndarray:
    """steps x chains float64 in [0, 1): the acceptance variates."""
    spec = MCMC[name]
    rng = np.random.Generator(np.random.PCG64(spec["pseed"] + 1000))
    return rng.random((int(steps), int(chains)))

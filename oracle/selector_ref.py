"""Reference (binary64, numpy) for the precision selector.

TEST INFRASTRUCTURE ONLY, like the rest of oracle/: it shares no code with
the GPU path and is only used to check the selector's kernels.

Three pieces:
  features(O)        the per-instance features, each a plain definition
                     (determinants by numpy's LAPACK routines);
  fallback_bits(...) the bound-based precision estimate of Eq. 5-7, adapted
                     to floating tiers (readings listed below);
  mlp_forward / mlp_backward
                     the selector network and its exact gradient, written
                     out layer by layer.

Readings of Sec. 5.1 and 5.4 used by the fallback:
  * a is the mean of Re O_ii over the a-modes (the diagonal blocks are
    conjugates of each other, so either half gives the same mean);
  * the paper gives no formula for k; solving Eq. 5 at |Z| = N with the exact
    det(I - O) gives k = ((1 - a)^2 - det(I - O)^(1/N)) / N;
  * Eq. 7 names B_lower "from the upper bound"; read as a typo: B_upper comes
    from the upper bound (Eq. 5) and B_lower from the lower bound (Eq. 6);
  * for floating tiers the range bits are not needed, only the bits lost to
    cancellation: log2(S_abs / |Tor|) with the rigorous
    S_abs <= 2^n det(I - O)^(-1/2) and Eq. 6 as the estimate of |Tor|, plus
    B_sgn = log2(1/tau) and B_accum = log2(alpha 2^n n^2), alpha = 0.5.
"""
from __future__ import annotations

import math

import numpy as np

NFEAT = 20
LANCZOS_STEPS = 12


def real_form(O):
    """R = W^H (I - O) W with W mapping each mode's (a, a^dagger) pair to its
    (q, p) quadratures, rows interleaved per mode.  Same principal minors."""
    O = np.asarray(O, dtype=np.complex128)
    n = O.shape[0] // 2
    M = np.eye(2 * n) - O
    W = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    s = 1.0 / np.sqrt(2.0)
    for k in range(n):
        # columns (q_k, p_k); rows a_k = k, a^dagger_k = k + n
        W[k, 2 * k] = s
        W[k, 2 * k + 1] = 1j * s
        W[k + n, 2 * k] = s
        W[k + n, 2 * k + 1] = -1j * s
    R = W.conj().T @ M @ W
    return R.real


def _mode_idx(modes):
    return [r for k in modes for r in (2 * k, 2 * k + 1)]


def lanczos_ritz_extremes(R, steps=LANCZOS_STEPS):
    """Smallest and largest Ritz value of `steps` Lanczos steps on the
    symmetric R from the normalised all-ones vector (the textbook three-term
    recurrence, no reorthogonalisation; stops early on an invariant
    subspace); the tridiagonal's eigenvalues by LAPACK."""
    N = R.shape[0]
    k = min(N, steps)
    v_prev = np.zeros(N)
    v = np.ones(N) / math.sqrt(N)
    al, be = [], []
    for j in range(k):
        w = R @ v
        a = float(w @ v)
        w = w - a * v - (be[-1] if be else 0.0) * v_prev
        b = float(np.linalg.norm(w))
        al.append(a)
        be.append(b)
        if not b > 1e-12 * abs(a):
            break
        v_prev, v = v, w / b
    T = np.diag(al) + np.diag(be[:len(al) - 1], 1) + np.diag(be[:len(al) - 1], -1)
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1])


def features(O) -> np.ndarray:
    """The selector's 20 features of one instance (n >= 1)."""
    O = np.asarray(O, dtype=np.complex128)
    n = O.shape[0] // 2
    R = real_form(O)
    L = np.linalg.cholesky(R)
    piv = np.diag(L) ** 2
    logdet = float(np.sum(np.log(piv)))
    q = np.empty(n)
    for k in range(n):
        idx = _mode_idx([k])
        q[k] = math.sqrt(np.linalg.det(R[np.ix_(idx, idx)]))
    pair_mi = 0.0
    pair_terms = []
    for i in range(n):
        for j in range(i + 1, n):
            idx = _mode_idx([i, j])
            dij = np.linalg.det(R[np.ix_(idx, idx)])
            pair_mi += math.log(dij / (q[i] ** 2 * q[j] ** 2))
            pair_terms.append(dij ** -0.5)
    a = float(np.mean(O.real.diagonal()[:n]))
    kpap = ((1.0 - a) ** 2 - math.exp(logdet / n)) / n
    f = np.zeros(NFEAT)
    f[0] = n
    f[1] = -0.5 * logdet
    f[2] = float(np.sum(np.log((1.0 + q) / (1.0 - q))))
    f[3] = float(np.mean(-np.log(q)))
    f[4] = a
    f[5] = kpap
    f[6] = pair_mi
    f[7] = float(np.max(q))
    f[8] = float(np.min(q))
    f[9] = float(np.log(np.min(piv)))
    f[10] = float(np.log(np.max(piv)))
    f[11] = float(math.log(np.mean(pair_terms))) if pair_terms else 0.0
    # spectrum of R: Gershgorin discs and Lanczos Ritz values
    off = np.sum(np.abs(R), axis=1) - np.abs(np.diag(R))
    f[12] = float(np.min(np.diag(R) - off))
    f[13] = float(math.log(np.max(np.diag(R) + off)))
    lo, hi = lanczos_ritz_extremes(R)
    f[14] = math.log(lo)
    f[15] = math.log(hi)
    # top levels: det R_{-Z} / det R = det Q_Z for Q = R^-1 (Jacobi), so a
    # level-(n - |Z|) term over the largest term is det(Q_Z)^(-1/2)
    Q = np.linalg.inv(R)
    t1 = [np.linalg.det(Q[np.ix_(_mode_idx([k]), _mode_idx([k]))]) ** -0.5 for k in range(n)]
    t2 = [np.linalg.det(Q[np.ix_(_mode_idx([i, j]), _mode_idx([i, j]))]) ** -0.5
          for i in range(n) for j in range(i + 1, n)]
    f[16] = math.log(np.mean(t1))
    f[17] = math.log(np.max(t1))
    f[18] = math.log(np.mean(t2)) if t2 else 0.0
    f[19] = math.log(np.max(t2)) if t2 else 0.0
    return f


def fallback_bits(O, tau: float, alpha: float = 0.5) -> float:
    """Significand bits the bound-based estimate asks for (Eq. 5-7 reading)."""
    O = np.asarray(O, dtype=np.complex128)
    n = O.shape[0] // 2
    M = np.eye(2 * n) - O
    sign, logdet = np.linalg.slogdet(M)
    det = math.exp(logdet)
    a = float(np.mean(O.real.diagonal()[:n]))
    k = ((1.0 - a) ** 2 - det ** (1.0 / n)) / n
    # Eq. 6: Tor ~ (((1 - a) - k N / (1 - a))^-1 - 1)^N
    base = 1.0 / ((1.0 - a) - k * n / (1.0 - a)) - 1.0
    log2_tor_lower = n * math.log2(base) if base > 0 else -1e300
    log2_sabs_upper = n - 0.5 * logdet / math.log(2.0)
    b_cancel = max(0.0, log2_sabs_upper - log2_tor_lower)
    b_sgn = math.log2(1.0 / tau)
    b_accum = math.log2(alpha * 2.0 ** n * n * n)
    return b_cancel + b_sgn + b_accum


# ---- network: 20 -> 32 -> 32 -> 1, tanh hidden layers ----------------------

SIZES = (NFEAT, 32, 32, 1)


def n_params(sizes=SIZES) -> int:
    return sum(sizes[i + 1] * sizes[i] + sizes[i + 1] for i in range(len(sizes) - 1))


def unpack(theta, sizes=SIZES):
    """Flat parameters -> [(W, b), ...]; W is (out, in), row-major."""
    out, off = [], 0
    for i in range(len(sizes) - 1):
        fi, fo = sizes[i], sizes[i + 1]
        W = theta[off:off + fo * fi].reshape(fo, fi)
        off += fo * fi
        b = theta[off:off + fo]
        off += fo
        out.append((W, b))
    return out


def mlp_forward(theta, X, mean, std):
    """Predictions (B,) for raw features X (B, NFEAT)."""
    h = (np.asarray(X, dtype=np.float64) - mean) / std
    layers = unpack(np.asarray(theta, dtype=np.float64))
    for li, (W, b) in enumerate(layers):
        h = h @ W.T + b
        if li < len(layers) - 1:
            h = np.tanh(h)
    return h[:, 0]


def loss_weights(err, under: float, over: float):
    """Asymmetric squared loss: under-predicting the target (err > 0) costs
    `under`, over-predicting costs `over`."""
    return np.where(err > 0, under, over)


def pinball(r, q: float):
    """Quantile loss of residuals r = y - prediction at level q."""
    return np.where(r > 0, q * r, (q - 1.0) * r)


def mlp_loss_and_grad(theta, X, y, mean, std, under=4.0, over=1.0, quantile=None):
    """Mean loss and its exact gradient w.r.t. theta: the asymmetric squared
    loss (under, over), or with `quantile` = q the pinball loss at level q."""
    theta = np.asarray(theta, dtype=np.float64)
    layers = unpack(theta)
    B = X.shape[0]
    acts = [(np.asarray(X, dtype=np.float64) - mean) / std]
    pre = []
    h = acts[0]
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        pre.append(z)
        h = np.tanh(z) if li < len(layers) - 1 else z
        acts.append(h)
    pred = acts[-1][:, 0]
    err = y - pred
    if quantile is None:
        w = loss_weights(err, under, over)
        loss = float(np.mean(w * err * err))
        # dL/dpred = -2 w err / B
        delta = (-2.0 * w * err / B)[:, None]
    else:
        loss = float(np.mean(pinball(err, quantile)))
        # dL/dpred = -q / B above the prediction, (1 - q) / B below
        delta = (np.where(err > 0, -quantile, 1.0 - quantile) / B)[:, None]
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        gW = delta.T @ acts[li]
        gb = delta.sum(axis=0)
        grads.append((gW, gb))
        if li > 0:
            delta = (delta @ W) * (1.0 - acts[li] ** 2)
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat

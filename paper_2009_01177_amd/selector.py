"""Training the learned precision selector on the GPU.

The network reads the TOR_NFEAT features of tor_features and predicts an
upper quantile of log10 of the FP64 tier's relative forward error (or, for
TOR_TARGET_KAPPA, log10 of the cancellation ratio S_abs / |Tor| that decides
how many of a tier's bits survive the alternating sum, Sec. 5.1).  Labels,
training and calibration run inside the library (tor_selector_label,
tor_selector_train: the library's evaluations, its gradient and Adam
kernels, its calibration); this module generates the training instances and
marshals arguments.
"""
from __future__ import annotations

import math
import os

import numpy as np

from .api import Batch, tor_features, tor_selector_label, tor_selector_set, tor_selector_train, train_options


def family_instances(states: int, per: int, seed: int, nlo: int, nhi: int, M: int = 100,
                     r=(0.8, 1.6), eta: float = 0.3):
    """Click patterns of `states` lossy GBS states of one family (Haar U on
    M modes, squeezing r ~ U[r], transmission eta), each state from its own
    seed (seed, seed + 1, ...), `per` patterns each with n ~ U{nlo..nhi}
    modes chosen uniformly."""
    import gbs_inputs as g
    out = []
    for k in range(states):
        rng = np.random.Generator(np.random.PCG64(seed + k))
        U = g.haar_unitary(M, rng)
        rr = rng.uniform(r[0], r[1], size=M)
        Of = g.o_from_sigma_q(g.gbs_sigma_q(U, rr, eta))
        prng = np.random.Generator(np.random.PCG64(seed + k + 77777))
        for _ in range(per):
            n = int(prng.integers(nlo, nhi + 1))
            out.append(g.click_submatrix(Of, np.sort(prng.choice(M, size=n, replace=False))))
    return out


def training_instances(count: int, nlo: int, nhi: int, seed: int, M: int = 60):
    """Click-pattern matrices from many seeded lossy GBS states: r ~ U[0.4, 1.7],
    transmission ~ U[0.15, 0.7], n ~ U{nlo..nhi} modes chosen uniformly."""
    import gbs_inputs as g
    rng = np.random.default_rng(seed)
    out = []
    states = max(1, count // 16)
    per = int(math.ceil(count / states))
    for s in range(states):
        srng = np.random.Generator(np.random.PCG64(int(rng.integers(1 << 62))))
        U_ = g.haar_unitary(M, srng)
        lo = rng.uniform(0.4, 1.2)
        r = srng.uniform(lo, lo + 0.5, size=M)
        eta = rng.uniform(0.15, 0.7)
        Ofull = g.o_from_sigma_q(g.gbs_sigma_q(U_, r, eta))
        for _ in range(per):
            if len(out) >= count:
                break
            n = int(rng.integers(nlo, nhi + 1))
            modes = np.sort(rng.choice(M, size=n, replace=False))
            out.append(g.click_submatrix(Ofull, modes))
    return out


def label(Os, ref: str = "qd", chunk: int = 2048):
    """(features, labels, n) of instances: features by tor_features, labels
    by tor_selector_label against the reference tier."""
    Xs, Ls, ns = [], [], []
    for i in range(0, len(Os), chunk):
        b = Batch(Os[i:i + chunk])
        Xs.append(tor_features(b).cpu().numpy())
        Ls.append(tor_selector_label(b, ref))
        ns.append(b.n.copy())
    return np.concatenate(Xs), np.concatenate(Ls), np.concatenate(ns)


def training_set(seed: int = 11):
    """The shipped selector's training data: 32 states of the 100-mode lossy
    family of the batched workload (r ~ U[0.8, 1.6], transmission 0.3; seeds
    5000.., never the benchmark's own state) with 400 patterns each,
    n ~ U{6..26}; 4000 patterns of diverse 60-mode states (n 6..26); both
    labelled against quad-double; 400 diverse patterns with n 27..36 labelled
    against double-double."""
    parts = [label(family_instances(32, 400, 5000, 6, 26)),
             label(training_instances(4000, 6, 26, seed)),
             label(training_instances(400, 27, 36, seed + 1), ref="dd", chunk=64)]
    return tuple(np.concatenate([p[i] for p in parts]) for i in range(3))


DEFAULT_OPTIONS = dict(target="err64", loss="quantile", quantile=0.9, epochs=400, batch_size=512, lr=3e-3,
                       slack=0.3, margin=0.0, seed=11)


def fit(X, L, n, **kw):
    """Train and calibrate through tor_selector_train; returns (selector, losses)."""
    o = dict(DEFAULT_OPTIONS)
    o.update(kw)
    return tor_selector_train(X, L, n, train_options(**o))


def fit_and_install(path: str | None = None, **kw):
    """Label the training set, train, calibrate; install the selector (and
    save it)."""
    X, L, n = training_set()
    sel, losses = fit(X, L, n, **kw)
    tor_selector_set(sel)
    if path:
        from .api import tor_selector_save
        tor_selector_save(path)
    return sel, (X, L, n), losses


DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")
DEFAULT_PATH = os.path.join(DATA, "selector_default.txt")
# the labelled training set the shipped selector was trained on (written by
# `--train`): retraining from it with DEFAULT_OPTIONS gives the shipped
# selector bit for bit
TRAIN_SET_PATH = os.path.join(DATA, "selector_train.npz")


def load_training_set(path: str = TRAIN_SET_PATH):
    d = np.load(path)
    return d["X"], d["L"], d["n"]


def load_default() -> bool:
    """Install the selector shipped with the library (trained by
    `python -m paper_2009_01177_amd.selector --train`); False if absent."""
    from .api import tor_selector_load
    if not os.path.exists(DEFAULT_PATH):
        return False
    tor_selector_load(DEFAULT_PATH)
    return True


if __name__ == "__main__":
    import argparse
    import sys
    import time
    ap = argparse.ArgumentParser(description="train the precision selector on the GPU")
    ap.add_argument("--train", action="store_true", help="label the training set, train, save both")
    ap.add_argument("--from-labels", action="store_true", help="retrain from the saved training set")
    ap.add_argument("--out", default=DEFAULT_PATH)
    ap.add_argument("--labels", default=TRAIN_SET_PATH)
    a = ap.parse_args()
    if not (a.train or a.from_labels):
        ap.print_help()
        sys.exit(0)
    t0 = time.time()
    if a.train:
        X, L, n = training_set()
        print(f"[selector] {len(n)} instances labelled in {time.time() - t0:.1f} s", flush=True)
        np.savez_compressed(a.labels, X=X, L=L, n=n.astype(np.int32))
    else:
        X, L, n = load_training_set(a.labels)
    sel, losses = fit(X, L, n)
    tor_selector_set(sel)
    from .api import tor_selector_save
    tor_selector_save(a.out)
    print(f"[selector] loss {losses[0]:.4f} -> {losses[-1]:.4f}; log10_c {list(sel.log10_c)}; saved {a.out} "
          f"({time.time() - t0:.1f} s)", flush=True)

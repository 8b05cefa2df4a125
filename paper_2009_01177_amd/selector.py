"""Training the learned precision selector on the GPU.

The selector predicts y = log10(S_abs / |Tor|), the cancellation ratio that
decides how many of a tier's bits survive the alternating sum (Sec. 5.1),
from the 12 features of tor_features.  Labels come from the library's own
quad-double evaluations, and for larger n (where quad-double is slow) from
double-double ones, which resolve kappa far below their 1e25 or so; the
per-tier error model |dTor|/|Tor| <= C_t kappa^s_t u_t is calibrated from
FP64 and double-double evaluations of the same instances (FP64 against the
reference tier; double-double only where quad-double is the reference).  Forward passes, gradients and Adam steps
run in the library's HIP kernels (tor_mlp_forward / tor_mlp_grad /
tor_mlp_adam); this module only drives them.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass

import numpy as np

from . import _lib
from .api import (Batch, tor_eval_batched, tor_features, tor_mlp_adam, tor_mlp_forward, tor_mlp_grad,
                  tor_selector_set)

U = {0: 2.0 ** -53, 1: 2.0 ** -104, 2: 2.0 ** -208}
YMAX = 60.0  # cap of log10 kappa (Tor == 0 exactly gives kappa = inf)


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


@dataclass
class Labels:
    X: np.ndarray        # (B, 12) features
    y: np.ndarray        # log10 kappa from the reference tier
    err: dict            # tier -> relative forward error |T_t - T_ref| / |T_ref| (nan: no reference)
    n: np.ndarray

    def __add__(self, o: "Labels") -> "Labels":
        return Labels(np.concatenate([self.X, o.X]), np.concatenate([self.y, o.y]),
                      {t: np.concatenate([self.err[t], o.err[t]]) for t in self.err},
                      np.concatenate([self.n, o.n]))


def label(Os, chunk: int = 1024, ref: str = "qd") -> Labels:
    """Features and labels of instances, all on the GPU.  ref: the tier whose
    value and S_abs give kappa, "qd" or (for large n) "dd"."""
    Xs, ys, e0, e1, ns = [], [], [], [], []
    for i in range(0, len(Os), chunk):
        part = Os[i:i + chunk]
        b = Batch(part)
        X = tor_features(b).cpu().numpy()
        rr = tor_eval_batched(b, tiers=ref)
        r0 = tor_eval_batched(b, tiers="fp64")
        r1 = tor_eval_batched(b, tiers="dd") if ref == "qd" else None
        for k in range(len(part)):
            tq = rr[k].exact
            sa = rr[k].abs_exact
            y = float(math.log10(sa / abs(tq))) if tq != 0 else YMAX
            ys.append(min(y, YMAX))
            den = abs(tq) if tq != 0 else sa
            e0.append(float(abs(r0[k].exact - tq) / den))
            e1.append(float(abs(r1[k].exact - tq) / den) if r1 is not None else float("nan"))
        Xs.append(X)
        ns.append(b.n.copy())
    return Labels(np.concatenate(Xs), np.array(ys), {0: np.array(e0), 1: np.array(e1)},
                  np.concatenate(ns))


def init_theta(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    sizes = (_lib.TOR_NFEAT, 32, 32, 1)
    parts = []
    for i in range(3):
        fi, fo = sizes[i], sizes[i + 1]
        parts.append(rng.normal(0.0, 1.0 / math.sqrt(fi), size=fo * fi))
        parts.append(np.zeros(fo))
    return np.concatenate(parts)


def train(X, y, epochs: int = 400, lr: float = 3e-3, batch_size: int = 512, under: float = 4.0,
          over: float = 1.0, seed: int = 0, log_every: int = 0):
    """Adam on the GPU kernels.  Returns (theta, mean, std, losses)."""
    import torch
    dev = "cuda"
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std[std < 1e-12] = 1.0
    th = torch.from_numpy(init_theta(seed)).to(dev)
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    tm = torch.from_numpy(mean).to(dev)
    ts = torch.from_numpy(std).to(dev)
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to(dev)
    yd = torch.from_numpy(np.ascontiguousarray(y)).to(dev)
    rng = np.random.default_rng(seed)
    B = X.shape[0]
    step = 0
    losses = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(B)).to(dev)
        tot = 0.0
        for i in range(0, B, batch_size):
            idx = perm[i:i + batch_size]
            xb = Xd[idx].contiguous()
            yb = yd[idx].contiguous()
            grad, loss = tor_mlp_grad(th, tm, ts, xb, yb, under, over)
            step += 1
            tor_mlp_adam(th, grad, m, v, lr, step)
            tot += float(loss.item()) * len(idx)
        losses.append(tot / B)
        if log_every and ep % log_every == 0:
            print(f"[selector] epoch {ep} loss {losses[-1]:.4f}", flush=True)
    return th.cpu().numpy(), mean, std, losses


def predict(theta, mean, std, X) -> np.ndarray:
    import torch
    dev = "cuda"
    return tor_mlp_forward(torch.from_numpy(np.ascontiguousarray(theta)).to(dev),
                           torch.from_numpy(mean).to(dev), torch.from_numpy(std).to(dev),
                           torch.from_numpy(np.ascontiguousarray(X)).to(dev)).cpu().numpy()


def calibrate(lab: Labels, slack: float = 0.3):
    """The per-tier error model log10(err_t / u_t) <= c_t + s_t log10 kappa:
    for each slope s_t in [0.3, 1] the intercept is the upper envelope of the
    training points; the slope kept is the one whose envelope lies lowest on
    average over them (rounding errors of the alternating sum grow more
    slowly than kappa); the intercept gets `slack` decades on top.
    Returns (log10_c, slopes), three entries each (QD shares DD's)."""
    cs, ss = [], []
    for t in (0, 1):
        e = lab.err[t]
        ok = np.isfinite(e) & (e > 0)
        if not ok.any():
            cs.append(0.0)
            ss.append(1.0)
            continue
        y = lab.y[ok]
        r = np.log10(e[ok]) - math.log10(U[t])
        best = None
        for s in np.arange(0.30, 1.0001, 0.01):
            c = float(np.max(r - s * y))
            height = float(np.mean(c + s * y))
            if best is None or height < best[0]:
                best = (height, c, float(s))
        cs.append(best[1] + slack)
        ss.append(best[2])
    cs.append(cs[-1])
    ss.append(ss[-1])
    return cs, ss


def make_selector(theta, mean, std, lab: Labels, log10_c, slopes=(1.0, 1.0, 1.0), margin: float = 0.5):
    sel = _lib.TorSelectorC()
    for i, v in enumerate(theta):
        sel.theta[i] = float(v)
    for i in range(_lib.TOR_NFEAT):
        sel.mean[i] = float(mean[i])
        sel.std[i] = float(std[i])
        sel.fmin[i] = float(lab.X[:, i].min())
        sel.fmax[i] = float(lab.X[:, i].max())
    for t in range(3):
        sel.log10_c[t] = float(log10_c[t])
        sel.slope[t] = float(slopes[t])
    sel.margin = float(margin)
    sel.nmin = int(lab.n.min())
    sel.nmax = int(lab.n.max())
    sel.trained = 1
    return sel


def fit_and_install(count: int = 3000, nlo: int = 6, nhi: int = 24, seed: int = 7, epochs: int = 300,
                    path: str | None = None, verbose: bool = False, count_dd: int = 0, nhi_dd: int = 0):
    """Generate, label, train, calibrate; install the selector (and save it).
    count_dd instances with n in (nhi, nhi_dd] are labelled by the DD tier."""
    Os = training_instances(count, nlo, nhi, seed)
    lab = label(Os)
    if count_dd > 0 and nhi_dd > nhi:
        lab = lab + label(training_instances(count_dd, nhi + 1, nhi_dd, seed + 1), chunk=64, ref="dd")
    theta, mean, std, losses = train(lab.X, lab.y, epochs=epochs, seed=seed,
                                     log_every=50 if verbose else 0)
    log10_c, slopes = calibrate(lab)
    sel = make_selector(theta, mean, std, lab, log10_c, slopes)
    tor_selector_set(sel)
    if path:
        from .api import tor_selector_save
        tor_selector_save(path)
    return sel, lab, losses


DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "selector_default.txt")


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
    ap.add_argument("--train", action="store_true")
    ap.add_argument("--count", type=int, default=4000)
    ap.add_argument("--nlo", type=int, default=6)
    ap.add_argument("--nhi", type=int, default=26)
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--count-dd", type=int, default=0,
                    help="further instances with n in (nhi, nhi-dd], labelled by the DD tier")
    ap.add_argument("--nhi-dd", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_PATH)
    a = ap.parse_args()
    if not a.train:
        ap.print_help()
        sys.exit(0)
    t0 = time.time()
    Os = training_instances(a.count, a.nlo, a.nhi, a.seed)
    print(f"[selector] {len(Os)} instances, n {a.nlo}..{a.nhi}", flush=True)
    lab = label(Os)
    if a.count_dd > 0 and a.nhi_dd > a.nhi:
        Od = training_instances(a.count_dd, a.nhi + 1, a.nhi_dd, a.seed + 1)
        print(f"[selector] {len(Od)} instances, n {a.nhi + 1}..{a.nhi_dd} (DD reference)", flush=True)
        lab = lab + label(Od, chunk=64, ref="dd")
    print(f"[selector] labelled in {time.time() - t0:.1f} s; log10 kappa "
          f"{lab.y.min():.2f}..{lab.y.max():.2f}", flush=True)
    theta, mean, std, losses = train(lab.X, lab.y, epochs=a.epochs, seed=a.seed, log_every=50)
    log10_c, slopes = calibrate(lab)
    pred = predict(theta, mean, std, lab.X)
    under = float(np.mean(pred < lab.y))
    print(f"[selector] loss {losses[0]:.3f} -> {losses[-1]:.4f}; log10 C = {log10_c}; slopes = {slopes}; "
          f"fraction under-predicted {under:.3f}", flush=True)
    sel = make_selector(theta, mean, std, lab, log10_c, slopes)
    tor_selector_set(sel)
    from .api import tor_selector_save
    tor_selector_save(a.out)
    print(f"[selector] saved {a.out} ({time.time() - t0:.1f} s)", flush=True)

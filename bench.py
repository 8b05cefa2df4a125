#!/usr/bin/env python3
"""Benchmark: Torontonian subset-terms/s at n = 30 on one MI355X.

A step is one full evaluation Tor(O) of the n = 30 workload (100-mode lossy
GBS state, Haar unitary, r ~ U[0.8, 1.6], transmission 0.3, 30 clicked modes;
synthetic, seeded) with O already resident in HBM: staging, every subset-tree
kernel over all 2^30 subsets, the fixed-order reductions and the copy of the
result to the host.  The timed tier is double-double (the paper's 128-bit
tier); the FP64 tier is measured on the same input and reported beside it.

Prints one JSON line.  `value` = 2^30 / seconds per step.  `roofline` is for
the dominant kernel (the middle+bottom kernel of the Schur path, or the
bordered kernel): algorithmic FP64 operations per launch over that kernel's
average launch duration, measured by HIP events the library records on the
stream it launches on, against the 78.6 TFLOP/s FP64 vector peak.  The
operation counts are those of the arithmetic the method performs (one count
per FP64 add, multiply, square root or division; a fused multiply-add counts
two), per subset, in each tier:
  Schur path, a subset whose largest mode leaves s undecided modes:
      s(2s+1) updated entries (two multiply-subtracts each), 2s scaled
      pivot-column entries, one 2x2 pivot (two reciprocal square roots) and
      the running det^(-1/2) product; plus two compensated accumulations of
      every term.
  Bordered path, a subset of m modes: 4(m-1)^2 + 6(m-1) complex
      multiply-adds.
`cpu_baseline` is the float128 oracle timed on the host's cores over a
bounded random sample of the same workload's subsets.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6  # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 flop/clk/CU
# FP64 operations per complex multiply-add in each tier's arithmetic:
#   FP64: 4 fused multiply-adds = 8 flops;
#   DD  : 4 fused double-double multiply-adds t - ab (18 flops each:
#         exact leading product, fma cross terms, an error-free sum and a
#         renormalisation) = 72.
FLOPS_PER_CFMA = {"fp64": 8, "dd": 72}


def kernel_flops(n, tier, algo, dmid):
    """Algorithmic flops of the dominant kernel over one evaluation."""
    if algo == "border":
        return cfma_bordered(n) * FLOPS_PER_CFMA[tier]
    return schur_flops(n, tier, dmid) + (1 << n) * acc_flops(tier)


def schur_node_flops(sp: int, tier: str) -> int:
    """One include producing a child with sp undecided modes (flops: add and
    multiply 1, fma 2, the hardware reciprocal square root estimate 1)."""
    ent, rows = sp * (2 * sp + 1), 2 * sp
    if tier == "fp64":
        # entry: 2 FMA; row: mul, FMA, mul; pivot: 2 rsqrt (estimate and a
        # Newton step, 7), mul, FMA, 2 mul for g
        return 4 * ent + 4 * rows + 19
    # DD: entry t - ab - cd fused (33); row: 2 DWTimesDW (12 each) and one
    # fused t - ab (18); pivot: 2 DD rsqrt (22 each: estimate, binary64 and
    # double-double Newton steps), a DWTimesDW, a fused t - ab, 2 DWTimesDW
    # for g
    return 33 * ent + 42 * rows + 98


def acc_flops(tier: str) -> int:
    """Accumulation of one term into its lane's run for the term's size
    parity (two_sum of the leading parts, low parts added in binary64); the
    two runs give both the signed sum and the sum of magnitudes."""
    return 7 if tier == "fp64" else 8


def schur_flops(n: int, tier: str, dmin: int = 0) -> int:
    """Algorithmic flops of the includes at depth >= dmin (2^k subsets have
    largest mode k), plus every term's accumulation when dmin covers the
    kernel that emits them."""
    return sum((1 << k) * schur_node_flops(n - 1 - k, tier) for k in range(dmin, n))


def cfma_bordered(n: int) -> int:
    """Complex multiply-adds of the bordered update over all non-empty subsets."""
    tot = 0
    for m in range(1, n + 1):
        t = m - 1
        tot += math.comb(n, m) * (4 * t * t + 6 * t)
    return tot


def paper_eq9_flops(n: int) -> float:
    """Eq. 9: the paper's count for per-subset elimination."""
    return sum(math.comb(n, i) * (32.0 / 3 * i ** 3 + 4 * i * i - 8.0 / 3 * i) for i in range(1, n + 1))


KERNEL_SOURCES = ("tor_schur.hip", "tiers.hpp", "prec.hpp", "tor_internal.hpp")


def kernel_code_hash(texts=None) -> str:
    """sha256 prefix of the Schur kernels' code: tor_schur.hip and the headers
    it compiles from, with // comments, trailing blanks and empty lines
    removed, so that a comment edit does not invalidate a measurement of the
    same code.  `texts` (file name -> text) overrides reading the files."""
    import hashlib
    import re
    lines = []
    for name in KERNEL_SOURCES:
        if texts is not None:
            text = texts[name]
        else:
            text = open(os.path.join(ROOT, "paper_2009_01177_amd", "csrc", name)).read()
        for line in text.splitlines():
            line = re.sub(r"//.*$", "", line).rstrip()
            if line:
                lines.append(line)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()[:16]


def measured_traffic(tier: str, n: int, algo: str):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel code."""
    path = os.path.join(ROOT, "profiles", "leaf_kernel_n30_traffic.txt")
    if algo != "schur" or n != 30 or not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            kv[k] = v
    if kv.get("code_sha256_prefix") != kernel_code_hash():
        return None
    v = kv.get(f"{tier}_traffic_bytes")
    return int(v) if v else None


def time_tier(tor, Od, tier, steps, warmup, algo="auto", split=-1, sb=0):
    import torch
    for _ in range(warmup):
        tor.tor_eval(Od, tier=tier, algo=algo, split_depth=split, time_kernel=True, bottom_modes=sb)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    kms = []
    res = None
    t0.record()
    for _ in range(steps):
        res = tor.tor_eval(Od, tier=tier, algo=algo, split_depth=split, time_kernel=True,
                           bottom_modes=sb)
        kms.append(tor.tor_last_kernel_ms())
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    return ms, kms, res


def cpu_baseline(O, n, seconds: float):
    """float128 oracle terms/s on a bounded uniform sample of subsets."""
    import numpy as np
    import oracle
    threads = oracle.max_threads()
    rng = np.random.default_rng(12345)
    k = 64
    while True:
        masks = rng.integers(0, 1 << n, size=k, dtype=np.uint64)
        t = time.perf_counter()
        oracle.terms(O, masks, threads=threads)
        dt = time.perf_counter() - t
        if dt > seconds / 4 or k >= 1 << 22:
            break
        k = int(k * min(16.0, max(2.0, (seconds / 4) / max(dt, 1e-3))))
    # final timed sample of about `seconds`
    k2 = max(k, int(k * seconds / max(dt, 1e-6)))
    masks = rng.integers(0, 1 << n, size=k2, dtype=np.uint64)
    t = time.perf_counter()
    oracle.terms(O, masks, threads=threads)
    dt = time.perf_counter() - t
    return dict(value=k2 / dt, unit="terms/s", cores=threads, kind="oracle",
                sample=f"{k2} uniformly random subsets of the n={n} workload, "
                       f"binary128 per-subset Cholesky, {dt:.1f} s on {threads} threads")


def batched_leg(tor, count: int, tau: float, steps: int, check: bool, extra_taus=()):
    """Batched workload: `count` click patterns (n ~ U{8..24}) of one 100-mode
    lossy state; solves/s for fixed DD (graph replay) and for the learned
    selector (TOR_AUTO: features, network, evaluation, spot re-evaluation)."""
    import numpy as np
    import torch
    import gbs_inputs as g
    from paper_2009_01177_amd import selector
    Os = g.batched_workload(batch=count)
    b = tor.Batch(Os)
    terms = float(sum(2 ** (O.shape[0] // 2) for O in Os))
    out = {"workload": f"{count} Torontonians from one 100-mode lossy GBS state (Haar U, "
                       f"r~U[0.8,1.6], eta=0.3), n~U{{8..24}}", "instances": count, "terms": terms,
           "tau": tau}

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    s_dd = timed(lambda: tor.tor_eval_batched(b, tiers="dd", graph=True, sync=False), steps)
    out["fixed_dd"] = {"s": s_dd, "solves_per_s": count / s_dd, "terms_per_s": terms / s_dd}
    print(f"[bench] batched fixed DD: {s_dd * 1e3:.1f} ms, {count / s_dd:.0f} solves/s", file=sys.stderr,
          flush=True)
    tor.tor_selector_set(None)
    s_fb = timed(lambda: tor.tor_eval_batched(b, tau=tau, graph=True, sync=False), steps)
    st_fb = tor.tor_last_select_stats()
    out["auto_bounds_only"] = {"s": s_fb, "solves_per_s": count / s_fb, "stats": st_fb}
    have = selector.load_default()
    s_ml = timed(lambda: tor.tor_eval_batched(b, tau=tau, graph=True, sync=False), steps)
    st_ml = tor.tor_last_select_stats()
    out["auto_learned"] = {"s": s_ml, "solves_per_s": count / s_ml, "stats": st_ml,
                           "selector": "paper_2009_01177_amd/data/selector_default.txt" if have else None}
    out["gain_learned_vs_fixed_dd"] = s_dd / s_ml
    out["select_ms"] = timed(lambda: tor.tor_select_tiers(b, tau), steps) * 1e3
    # the learned tiers evaluated on their own (no selection, no spot checks)
    chosen, _, _ = tor.tor_select_tiers(b, tau)
    chosen = [int(x) for x in chosen]
    s_ev = timed(lambda: tor.tor_eval_batched(b, tiers=chosen, graph=True, sync=False), steps)
    out["auto_learned"]["eval_only_s"] = s_ev
    out["gain_learned_eval_only_vs_fixed_dd"] = s_dd / s_ev
    out["gain_learned_vs_bounds_only"] = s_fb / s_ml
    print(f"[bench] batched auto: bounds-only {s_fb * 1e3:.1f} ms, learned {s_ml * 1e3:.1f} ms "
          f"({st_ml}); its tiers alone {s_ev * 1e3:.1f} ms, selection {out['select_ms']:.2f} ms",
          file=sys.stderr, flush=True)
    ref = None
    if check:
        res = tor.tor_eval_batched(b, tau=tau)
        ref = tor.tor_eval_batched(b, tiers="qd")
        dd = tor.tor_eval_batched(b, tiers="dd")
        worst = 0.0
        worst_dd = 0.0
        for r, q, d in zip(res, ref, dd):
            tq = q.exact
            if tq != 0:
                worst = max(worst, float(abs(r.exact - tq) / abs(tq)))
                worst_dd = max(worst_dd, float(abs(d.exact - tq) / abs(tq)))
        out["max_rel_err_vs_qd"] = {"auto_learned": worst, "fixed_dd": worst_dd}
        # the ideal per-instance choice: FP64 wherever it meets tau against
        # QD, DD elsewhere (needs the QD values, so it bounds what any
        # selector can gain on this workload)
        f64 = tor.tor_eval_batched(b, tiers="fp64")
        ideal = ["fp64" if q.exact != 0 and abs(f.exact - q.exact) <= tau * abs(q.exact) else "dd"
                 for f, q in zip(f64, ref)]
        s_id = timed(lambda: tor.tor_eval_batched(b, tiers=ideal, graph=True, sync=False), steps)
        nf = sum(1 for x in ideal if x == "fp64")
        out["ideal_choice"] = {"s": s_id, "n_fp64": nf, "n_dd": count - nf,
                               "gain_vs_fixed_dd": s_dd / s_id}
        print(f"[bench] batched ideal choice: {s_id * 1e3:.1f} ms ({nf} FP64)", file=sys.stderr,
              flush=True)
    # the same comparison at further accuracy targets (one timed call of the
    # bound-estimate-only selector each: it is the slow one)
    for t2 in extra_taus:
        tor.tor_selector_set(None)
        s_fb2 = timed(lambda: tor.tor_eval_batched(b, tau=t2, graph=True, sync=False), 1)
        st_fb2 = tor.tor_last_select_stats()
        selector.load_default()
        s_ml2 = timed(lambda: tor.tor_eval_batched(b, tau=t2, graph=True, sync=False), steps)
        st_ml2 = tor.tor_last_select_stats()
        row = {"auto_bounds_only": {"s": s_fb2, "stats": st_fb2},
               "auto_learned": {"s": s_ml2, "solves_per_s": count / s_ml2, "stats": st_ml2},
               "gain_learned_vs_fixed_dd": s_dd / s_ml2, "gain_learned_vs_bounds_only": s_fb2 / s_ml2}
        if check:
            res2 = tor.tor_eval_batched(b, tau=t2)
            row["max_rel_err_vs_qd"] = max(float(abs(r.exact - q.exact) / abs(q.exact))
                                           for r, q in zip(res2, ref) if q.exact != 0)
        out.setdefault("by_tau", {})[repr(t2)] = row
        print(f"[bench] batched tau={t2:g}: learned {s_ml2 * 1e3:.1f} ms ({st_ml2}), bounds-only "
              f"{s_fb2 * 1e3:.1f} ms", file=sys.stderr, flush=True)
    return out


def mcmc_leg(tor, chains: int, steps: int, reps: int):
    """Sampler workload: `chains` independence Metropolis chains over
    20-click patterns of a 100-mode lossy state, `steps` steps each (every
    step scores one candidate per chain), through tor_mcmc in double-double
    with the state, candidates and variates resident on the device."""
    import numpy as np
    import torch
    import gbs_inputs as g
    name = "mcmc_m100_n20"
    spec = g.MCMC[name]
    sq, O = g.mcmc_state(name)
    Od = torch.from_numpy(O).to("cuda:0")
    P = torch.from_numpy(g.mcmc_proposals(name, chains, steps)).to("cuda:0")
    U = torch.from_numpy(g.mcmc_uniforms(name, chains, steps)).to("cuda:0")
    tor.tor_mcmc(Od, P, U, tier="dd")  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        state, cand = tor.tor_mcmc(Od, P, U, tier="dd")
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t) / reps
    S = state.cpu().numpy()
    moves = float((S[1:] == np.arange(1, steps)[:, None]).mean()) if steps > 1 else 0.0
    ncand = chains * steps
    out = {"workload": f"{chains} chains x {steps} steps over {spec['N']}-click patterns of a "
                       f"{spec['M']}-mode lossy GBS state (Haar U, r~U[0.8,1.6], eta=0.3), "
                       f"uniform candidates", "tier": "dd", "chains": chains, "steps": steps,
           "candidates": ncand, "s": sec, "candidates_per_s": ncand / sec,
           "terms_per_s": ncand * float(1 << spec["N"]) / sec,
           "samples_per_s_at_100_candidates": ncand / sec / 100.0, "move_fraction": moves}
    print(f"[bench] mcmc: {sec * 1e3:.1f} ms for {ncand} candidates, {ncand / sec:.0f} candidates/s",
          file=sys.stderr, flush=True)
    return out


def small_leg(tor, reps: int = 20):
    """The 16-mode lossless instance (65,536 subsets; launch-latency bound):
    ms per evaluation in FP64 and DD, and the binary128 oracle's full
    evaluation on the host beside it, with both errors over S_abs."""
    import numpy as np
    import torch
    import gbs_inputs as g
    import oracle
    O, _ = g.workload("n16_lossless")
    Od = torch.from_numpy(O).to("cuda:0")
    out = {"workload": "single Torontonian n=16: 16-mode lossless GBS (Haar U, r~U[0.5,1.0]), "
                       "all modes clicked, O 32x32 complex128"}
    t = time.perf_counter()
    ref = oracle.tor(O)
    out["oracle_s"] = time.perf_counter() - t
    out["oracle_threads"] = ref["threads"]
    b1 = tor.Batch([O])
    for tier in ("fp64", "dd"):
        ms, _, res = time_tier(tor, Od, tier, reps, 2)
        out[tier] = {"ms": ms, "err_over_sabs": float(abs(res.exact - ref["tor"]) / ref["abs_sum"])}
        # the same evaluation captured once as a HIP graph and replayed back
        # to back, its result left on the device (no host round trip)
        for _ in range(2):
            tor.tor_eval_batched(b1, tiers=tier, graph=True, sync=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            tor.tor_eval_batched(b1, tiers=tier, graph=True, sync=False)
        torch.cuda.synchronize()
        out[tier]["graph_replay_ms"] = (time.perf_counter() - t) / reps * 1e3
        # each replay on its own: device time between events around the call,
        # and the host time the call takes to return
        dev, host = [], []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            h = time.perf_counter()
            tor.tor_eval_batched(b1, tiers=tier, graph=True, sync=False)
            host.append((time.perf_counter() - h) * 1e3)
            e1.record()
            torch.cuda.synchronize()
            dev.append(e0.elapsed_time(e1))
        out[tier]["graph_replay_device_ms"] = {"median": float(np.median(dev)), "max": float(np.max(dev))}
        out[tier]["graph_call_host_ms"] = {"median": float(np.median(host)), "max": float(np.max(host))}
        rg = tor.tor_eval_batched(b1, tiers=tier, graph=True)[0]
        out[tier]["graph_err_over_sabs"] = float(abs(rg.exact - ref["tor"]) / ref["abs_sum"])
    print(f"[bench] n=16: fp64 {out['fp64']['ms']:.3f} ms, dd {out['dd']['ms']:.3f} ms (graph replay "
          f"{out['fp64']['graph_replay_ms']:.3f} / {out['dd']['graph_replay_ms']:.3f} ms), oracle "
          f"{out['oracle_s']:.2f} s", file=sys.stderr, flush=True)
    return out


def stress_leg(tor, taus=(1e-3, 1e-6)):
    """Precision-stress workload: n = 36 of a 100-mode state with r = 1.5 and
    transmission 0.5, in FP64, DD and QD (QD as the reference), and what the
    precision selector picks and costs for it at each accuracy target."""
    import torch
    import gbs_inputs as g
    from paper_2009_01177_amd import selector
    selector.load_default()
    O, _ = g.workload("n36_stress")
    Od = torch.from_numpy(O).to("cuda:0")
    out = {"workload": "single Torontonian n=36: 100-mode GBS (Haar U, r=1.5, eta=0.5), 36 clicked "
                       "modes, O 72x72 complex128"}
    res = {}
    n = O.shape[0] // 2
    for tier in ("fp64", "dd", "qd"):
        if tier != "qd":
            tor.tor_eval(Od, tier=tier)
        torch.cuda.synchronize()
        t = time.perf_counter()
        res[tier] = tor.tor_eval(Od, tier=tier, time_kernel=True)
        torch.cuda.synchronize()
        out[tier] = {"s": time.perf_counter() - t, "terms_per_s": float(1 << n) / (time.perf_counter() - t)}
        kms, d_used, _, launches = tor.tor_last_kernel_ms()
        if tier != "qd":
            fl = kernel_flops(n, tier, "schur", d_used)
            out[tier].update({"kernel_s": kms / 1e3, "launches": launches,
                              "frac_fp64_peak": fl / (kms / 1e3) / 1e12 / PEAK_FP64_TFLOPS})
        print(f"[bench] n=36 {tier}: {out[tier]['s']:.3f} s", file=sys.stderr, flush=True)
    q = res["qd"]
    out["kappa"] = q.kappa
    for tier in ("fp64", "dd"):
        out[tier]["rel_err_vs_qd"] = float(abs(res[tier].exact - q.exact) / abs(q.exact))
        out[tier]["err_vs_qd_over_sabs"] = float(abs(res[tier].exact - q.exact) / q.abs_exact)
    b = tor.Batch([O])
    out["selector"] = {}
    for tau in taus:
        tiers, k, src = tor.tor_select_tiers(b, tau)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = tor.tor_eval_batched(b, tau=tau)[0]
        sec = time.perf_counter() - t
        out["selector"][repr(tau)] = {
            "tier": ["fp64", "dd", "qd"][int(tiers[0])],
            "prediction": float(k[0]), "prediction_is": "log10 of the FP64 tier's forward error (upper quantile)"
            if tor.tor_selector_get().target == 1 else "log10 kappa",
            "source": "network" if int(src[0]) == 0 else "bound estimate", "s": sec,
            "rel_err_vs_qd": float(abs(r.exact - q.exact) / abs(q.exact))}
        print(f"[bench] n=36 tau={tau:g}: {out['selector'][repr(tau)]}", file=sys.stderr, flush=True)
    return out


def n40_leg(tor):
    """The largest one-GPU workload: n = 40 of a 100-mode lossy state
    (r ~ U[1.0, 1.6], transmission 0.3), 2^40 subsets in double-double, one
    evaluation (after a one-time n = 40 FP64 warm-up of the workspace)."""
    import torch
    import gbs_inputs as g
    O, _ = g.workload("n40_lossy")
    Od = torch.from_numpy(O).to("cuda:0")
    n = O.shape[0] // 2
    tor.tor_eval(Od, tier="fp64")  # grows the workspace to the n = 40 plan
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = tor.tor_eval(Od, tier="dd", time_kernel=True)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t
    kms, d_used, grid, launches = tor.tor_last_kernel_ms()
    fl = kernel_flops(n, "dd", "schur", d_used)
    out = {"workload": "single Torontonian n=40: 100-mode lossy GBS (Haar U, r~U[1.0,1.6], eta=0.3), "
                       "40 clicked modes, O 80x80 complex128", "tier": "dd", "s": sec,
           "terms": 1 << n, "terms_per_s": float(1 << n) / sec, "kernel_s": kms / 1e3,
           "launches": launches, "frac_fp64_peak": fl / (kms / 1e3) / 1e12 / PEAK_FP64_TFLOPS,
           "tor": r.value, "kappa": r.kappa, "err_bound_over_tor": r.err_bound / abs(r.value)}
    print(f"[bench] n=40 dd: {sec:.2f} s, {out['terms_per_s']:.3e} terms/s, frac {out['frac_fp64_peak']:.3f}",
          file=sys.stderr, flush=True)
    return out


def large_leg(tor):
    """Opt-in figures beyond the default legs: one quad-double evaluation of
    the n = 30 workload, and parts of an n = 50 instance (the paper's
    largest size) of the n = 40 workload's state (50 clicked modes): part 0
    of 2^12 (2^38 subsets) in double-double and in binary64."""
    import torch
    import gbs_inputs as g
    out = {}
    O, _ = g.workload("n30_lossy")
    Od = torch.from_numpy(O).to("cuda:0")
    tor.tor_eval(Od, tier="qd")  # warm-up: workspace and code
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = tor.tor_eval(Od, tier="qd")
    torch.cuda.synchronize()
    sec = time.perf_counter() - t
    out["qd_n30"] = {"s": sec, "terms_per_s": float(1 << 30) / sec, "tor": r.value}
    print(f"[bench] n=30 qd: {sec:.3f} s", file=sys.stderr, flush=True)
    O, _ = g.workload("n40_lossy", n=50)
    nparts = 1 << 12
    for tier in ("fp64", "dd"):
        tor.tor_eval_part(O, 1, nparts, tier=tier)  # warm-up: grows the workspace to the n = 50 plan
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = tor.tor_eval_part(O, 0, nparts, tier=tier)
        sec = time.perf_counter() - t
        terms = float(1 << 50) / nparts
        out[f"n50_part_{tier}"] = {"part": 0, "nparts": nparts, "terms": terms, "s": sec,
                                   "terms_per_s": terms / sec, "whole_instance_h": sec * nparts / 3600}
        print(f"[bench] n=50 {tier} part of 2^38 subsets: {sec:.2f} s, {terms / sec:.3e} terms/s, "
              f"whole instance {sec * nparts / 3600:.2f} h", file=sys.stderr, flush=True)
    return out


def phase_leg(tor, steps: int):
    """Where the middle + bottom kernel's time goes, from the phase-clock
    build (per wavefront, shader-clock cycles between marks in the kernel):
    the n = 30 workload in DD, FP64 and QD, per middle state and as
    fractions of the wavefronts' time."""
    import torch
    import gbs_inputs as g
    O, _ = g.workload("n30_lossy")
    Od = torch.from_numpy(O).to("cuda:0")
    n = O.shape[0] // 2
    out = {}
    for tier in ("dd", "fp64", "qd"):
        tor.tor_eval(Od, tier=tier, algo="schur")
        torch.cuda.synchronize()
        tor.tor_debug_phase_clocks(reset=True)
        kms = 0.0
        for _ in range(steps):
            tor.tor_eval(Od, tier=tier, algo="schur", time_kernel=True)
            k, d_used, grid, launches = tor.tor_last_kernel_ms()
            kms += k
        ph = tor.tor_debug_phase_clocks(reset=True)
        states = steps * (1 << d_used)
        tot = sum(ph.values())
        out[tier] = {"middle_states": states, "kernel_ms": kms, "grid": grid,
                     "cycles_per_state": {k: v / states for k, v in ph.items()},
                     "fraction": {k: v / tot for k, v in ph.items()},
                     "wave_cycles_per_kernel_s": tot / (kms / 1e3)}
        print(f"[bench] phases {tier}: " + " ".join(f"{k}={v / states:.0f}" for k, v in ph.items())
              + f" cycles per middle state ({steps} evaluations, {states} states)", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--tier", default="dd", choices=["dd", "fp64"])
    ap.add_argument("--algo", default="auto")
    ap.add_argument("--split", type=int, default=-1)
    ap.add_argument("--sb", type=int, default=0, help="Schur path: bottom modes per lane (0 = default)")
    ap.add_argument("--sb-other", type=int, default=0)
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=4096, help="batched leg instances (0: skip)")
    ap.add_argument("--tau", type=float, default=1e-3)
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--no-batch-check", action="store_true",
                    help="skip checking the batched leg against QD (and timing the ideal tier choice)")
    ap.add_argument("--batch-taus", default="1e-4,1e-6",
                    help="further accuracy targets for the batched leg, comma-separated ('' for none)")
    ap.add_argument("--mcmc-chains", type=int, default=1024, help="sampler leg chains (0: skip)")
    ap.add_argument("--mcmc-steps", type=int, default=16)
    ap.add_argument("--mcmc-reps", type=int, default=2)
    ap.add_argument("--no-small", action="store_true", help="skip the n = 16 leg")
    ap.add_argument("--no-stress", action="store_true",
                    help="skip the n = 36 precision-stress leg (about 35 s: QD reference)")
    ap.add_argument("--no-n40", action="store_true", help="skip the n = 40 double-double leg (about 25 s)")
    ap.add_argument("--phase-clocks", action="store_true",
                    help="only the per-phase clocks of the middle + bottom kernel (loads the phase-clock build)")
    ap.add_argument("--large", action="store_true",
                    help="add the quad-double n = 30 evaluation and n = 50 parts (about 20 s)")
    ap.add_argument("--mcmc-only", action="store_true",
                    help="run only the sampler leg and print its JSON object (for profiling)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched leg and print its JSON object (for profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="first copy this many bytes device-to-device (a known-size kernel for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library evaluates a Torontonian on a single "
              "MI355X (--gpus 1); multi-GPU sharding of the subset tree is not implemented.",
              file=sys.stderr)
        sys.exit(2)

    if args.phase_clocks:
        os.environ.setdefault("TOR_LIBRARY", os.path.join(ROOT, "paper_2009_01177_amd", "libtor_hip_phase.so"))
    import numpy as np
    import torch
    import gbs_inputs as g
    import paper_2009_01177_amd as tor
    if args.phase_clocks:
        print(json.dumps({"phase_clocks": phase_leg(tor, max(args.steps, 1))}), flush=True)
        return

    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.mcmc_only:
        print(json.dumps({"mcmc": mcmc_leg(tor, max(args.mcmc_chains, 1), args.mcmc_steps,
                                           args.mcmc_reps)}), flush=True)
        return
    if args.batch_only:
        extra = [float(x) for x in args.batch_taus.split(",") if x.strip()]
        print(json.dumps({"batched": batched_leg(tor, max(args.batch, 1), args.tau, args.batch_steps,
                                                 not args.no_batch_check, extra)}), flush=True)
        return

    n = args.n
    O, modes = g.workload("n30_lossy", n=n)
    Od = torch.from_numpy(O).to("cuda:0")
    torch.cuda.synchronize()
    print(f"[bench] n={n} tier={args.tier} steps={args.steps} warmup={args.warmup}", file=sys.stderr,
          flush=True)

    algo = "border" if args.algo == "border" else "schur"
    ms, kms, res = time_tier(tor, Od, args.tier, args.steps, args.warmup, algo, args.split, args.sb)
    terms = float(1 << n)
    value = terms / (ms / 1e3)
    kernel_ms = float(np.mean([k[0] for k in kms]))  # sum over the step's launches
    d_used, grid_used, launches = kms[-1][1], kms[-1][2], kms[-1][3]
    flops = kernel_flops(n, args.tier, algo, d_used)
    achieved = flops / (kernel_ms / 1e3) / 1e12
    print(f"[bench] {args.tier}: {ms:.3f} ms/step, kernel {kernel_ms:.3f} ms over {launches} launches, "
          f"{value:.3e} terms/s, {achieved:.2f} TFLOP/s", file=sys.stderr, flush=True)

    other = "fp64" if args.tier == "dd" else "dd"
    oms, okms, ores = time_tier(tor, Od, other, args.fp64_steps, 1, algo, args.split, args.sb_other)
    okernel = float(np.mean([k[0] for k in okms]))
    oflops = kernel_flops(n, other, algo, okms[-1][1])
    print(f"[bench] {other}: {oms:.3f} ms/step, kernel {okernel:.3f} ms", file=sys.stderr, flush=True)

    line = {
        "metric": f"Torontonian subset-terms/s at n={n} ({args.tier.upper()} tier)",
        "value": value,
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64x2" if args.tier == "dd" else "f64",
        "data": "synthetic",
        "config": {"workload": f"single Torontonian n={n}: 100-mode lossy GBS (Haar U, r~U[0.8,1.6], "
                               f"eta=0.3), {n} clicked modes, O {2 * n}x{2 * n} complex128",
                   "n": n, "terms": int(terms), "tier": args.tier, "algo": algo,
                   "split_depth": d_used, "grid": grid_used},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": measured_traffic(args.tier, n, algo),
                     "kernel": "leaf_kernel" if algo == "schur" else "border_kernel",
                     "launches_per_step": launches,
                     "kernel_ms_per_launch": kernel_ms / max(launches, 1),
                     "algorithmic_flops_per_launch": flops / max(launches, 1)},
        "tiers": {
            args.tier: {"terms_per_s": value, "ms_per_step": ms, "kernel_ms": kernel_ms,
                        "tflops": achieved, "frac_fp64_peak": achieved / PEAK_FP64_TFLOPS,
                        "tor": res.value, "kappa": res.kappa},
            other: {"terms_per_s": terms / (oms / 1e3), "ms_per_step": oms, "kernel_ms": okernel,
                    "tflops": oflops / (okernel / 1e3) / 1e12,
                    "frac_fp64_peak": oflops / (okernel / 1e3) / 1e12 / PEAK_FP64_TFLOPS,
                    "tor": ores.value},
        },
        "paper_eq9_equivalent_pflops": paper_eq9_flops(n) / (ms / 1e3) / 1e15,
        "algorithmic_flops_all_kernels": (schur_flops(n, args.tier) + (1 << n) * acc_flops(args.tier))
        if algo == "schur" else flops,
    }
    # forward error of the FP64 value against the DD one (DD's own error is
    # far below it at this kappa)
    r64, rdd = (ores, res) if other == "fp64" else (res, ores)
    line["tiers"]["fp64"]["rel_err_vs_dd"] = float(abs(r64.exact - rdd.exact) / abs(rdd.exact))
    line["tiers"]["fp64"]["err_vs_dd_over_sabs"] = float(abs(r64.exact - rdd.exact) / rdd.abs_exact)
    if args.batch > 0:
        extra = [float(x) for x in args.batch_taus.split(",") if x.strip()]
        line["batched"] = batched_leg(tor, args.batch, args.tau, args.batch_steps, not args.no_batch_check, extra)
    if args.mcmc_chains > 0:
        line["mcmc"] = mcmc_leg(tor, args.mcmc_chains, args.mcmc_steps, args.mcmc_reps)
    if not args.no_small:
        line["small_n16"] = small_leg(tor)
    if not args.no_stress:
        line["stress_n36"] = stress_leg(tor)
    if not args.no_n40:
        line["n40"] = n40_leg(tor)
    if args.large:
        line["large"] = large_leg(tor)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(O, n, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

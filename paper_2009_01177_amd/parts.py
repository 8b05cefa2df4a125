"""Evaluations in parts with a checkpoint file (tor_eval_part /
tor_combine_parts in include/tor.h).

A long evaluation (N = 50 is hours on one GPU) is split into parts; each
finished part's result is recorded in a JSON file at once, so a run that is
interrupted resumes with the parts still missing.  The file also records
the instance's shape, tier, number of parts and a hash of O, and a resume
against a different instance is refused.  Host-side orchestration only: the
parts run in the library's kernels.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from .api import TorResult, tor_combine_parts, tor_eval_part


def instance_hash(O) -> str:
    """sha256 of O's complex128 bytes (row-major)."""
    a = np.ascontiguousarray(O.cpu().numpy() if hasattr(O, "cpu") else np.asarray(O), dtype=np.complex128)
    return hashlib.sha256(a.tobytes()).hexdigest()


def result_to_json(r: TorResult) -> dict:
    """Exact: every word as its binary64 hex string."""
    return {"tor": [float(x).hex() for x in r.expansion], "abs_sum": [float(x).hex() for x in r.abs_sum],
            "err_bound": float(r.err_bound).hex(), "tier_used": int(r.tier_used), "status": int(r.status)}


def result_from_json(d: dict) -> TorResult:
    return TorResult(tuple(float.fromhex(x) for x in d["tor"]), tuple(float.fromhex(x) for x in d["abs_sum"]),
                     float.fromhex(d["err_bound"]), int(d["tier_used"]), int(d["status"]))


def evaluate_in_parts(O, nparts: int, tier="dd", checkpoint: str | None = None, progress=None,
                      stop_after: int | None = None) -> TorResult | None:
    """Tor(O) as `nparts` parts, resuming from `checkpoint` (a JSON file,
    written after every part) when given.  `progress(part, result)` is
    called after each part evaluated here.  stop_after: evaluate at most
    that many parts in this call and return None if any remain."""
    n = (O.shape[0]) // 2
    key = {"n": int(n), "tier": str(tier), "nparts": int(nparts), "o_sha256": instance_hash(O)}
    done = {}
    if checkpoint and os.path.exists(checkpoint):
        with open(checkpoint) as f:
            state = json.load(f)
        if state.get("key") != key:
            raise ValueError("checkpoint %s belongs to another evaluation" % checkpoint)
        done = {int(p): result_from_json(r) for p, r in state["parts"].items()}
    ran = 0
    for p in range(nparts):
        if p in done:
            continue
        if stop_after is not None and ran >= stop_after:
            return None
        r = tor_eval_part(O, p, nparts, tier=tier)
        done[p] = r
        ran += 1
        if checkpoint:
            tmp = checkpoint + ".tmp"
            with open(tmp, "w") as f:
                json.dump({"key": key, "parts": {str(q): result_to_json(v) for q, v in sorted(done.items())}}, f)
            os.replace(tmp, checkpoint)
        if progress:
            progress(p, r)
    return tor_combine_parts(tier, n, [done[p] for p in range(nparts)])

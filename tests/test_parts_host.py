"""The checkpoint driver of evaluations in parts (paper_2009_01177_amd/parts.py),
host side: exact JSON round trip of results, resume from a complete
checkpoint (only the host-side combination runs), refusal of a checkpoint
of another instance.  No GPU."""
import json
from fractions import Fraction

import numpy as np
import pytest

import gbs_inputs as g
from paper_2009_01177_amd import parts
from paper_2009_01177_amd.api import TorResult


def _res(hi, lo, a):
    return TorResult((hi, lo, 0.0, 0.0), (a, 0.0), 1e-30, 1, 0)


def test_results_round_trip_exactly():
    r = _res(0.1, 2.0 ** -60 / 3, 7.5)
    back = parts.result_from_json(json.loads(json.dumps(parts.result_to_json(r))))
    assert back.expansion == r.expansion and back.abs_sum == r.abs_sum
    assert back.err_bound == r.err_bound and back.tier_used == 1 and back.status == 0


def test_resume_from_a_complete_checkpoint(tmp_path):
    O = g.random_instance(12, 5)
    ck = tmp_path / "ck.json"
    vals = [_res(1.0 + k, 2.0 ** -70 * k, 2.0 + k) for k in range(4)]
    key = {"n": 12, "tier": "dd", "nparts": 4, "o_sha256": parts.instance_hash(O)}
    ck.write_text(json.dumps({"key": key, "parts": {str(k): parts.result_to_json(v) for k, v in enumerate(vals)}}))
    total = parts.evaluate_in_parts(O, 4, "dd", checkpoint=str(ck))
    want = sum(Fraction(v.expansion[0]) + Fraction(v.expansion[1]) for v in vals)
    assert total.exact == want
    assert total.abs_sum[0] == sum(v.abs_sum[0] for v in vals)


def test_checkpoint_of_another_instance_is_refused(tmp_path):
    O = g.random_instance(12, 5)
    ck = tmp_path / "ck.json"
    key = {"n": 12, "tier": "dd", "nparts": 4, "o_sha256": parts.instance_hash(O + 1e-3)}
    ck.write_text(json.dumps({"key": key, "parts": {}}))
    with pytest.raises(ValueError):
        parts.evaluate_in_parts(O, 4, "dd", checkpoint=str(ck))

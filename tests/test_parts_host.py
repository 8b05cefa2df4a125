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


# --- a closed form for one part of a product state -------------------------
# For O = a direct sum of blocks in mode order, every term factorises over
# the blocks (the sign (-1)^(n-|Z|) and det(I - O_Z) both do).  A part fixes
# the decisions on modes 0..k-1 (mode 0 the most significant bit of the
# part's code); when those modes are whole blocks, the part's sum is the
# product of the prefix blocks' terms for their decisions and of the other
# blocks' Torontonians, each block by brute force at 60 digits.

def product_state_in_order(n, k, seed):
    """A product of lossy 1-mode and coupled 2-mode states in mode order,
    its first k modes whole blocks; returns O and the blocks' (first mode,
    size)."""
    rng = np.random.default_rng(seed)
    blocks, spans, pos = [], [], 0
    while pos < n:
        left = (k - pos) if pos < k else (n - pos)
        size = 1 if (left == 1 or rng.random() < 0.5) else 2
        if size == 1:
            blocks.append(g.lossy_squeezed_o(rng.uniform(0.6, 1.4), rng.uniform(0.3, 0.9)))
        else:
            blocks.append(g.random_instance(2, int(rng.integers(1 << 30)), M=4))
        spans.append((pos, size))
        pos += size
    return g.direct_sum_o(blocks), spans


def _block_term(Ob, z):
    """(-1)^(s-|z|) det(I - Ob_z)^(-1/2) of a block of s modes, at 60 digits."""
    import mpmath
    s = Ob.shape[0] // 2
    idx = list(z) + [i + s for i in z]
    if not idx:
        return mpmath.mpf(-1) ** s
    M = mpmath.matrix(len(idx), len(idx))
    for a, ia in enumerate(idx):
        for b, ib in enumerate(idx):
            v = Ob[ia, ib]
            M[a, b] = (1 if ia == ib else 0) - mpmath.mpc(float(v.real), float(v.imag))
    t = 1 / mpmath.sqrt(mpmath.re(mpmath.det(M)))
    return t if (s - len(z)) % 2 == 0 else -t


def part_closed_form(O, spans, k, code):
    """(sum, sum of magnitudes) of part `code` of 2^k, as Fractions."""
    import mpmath
    n = O.shape[0] // 2
    with mpmath.workdps(60):
        val, sabs = mpmath.mpf(1), mpmath.mpf(1)
        for p, size in spans:
            Ob = g.click_submatrix(O, list(range(p, p + size)))
            if p < k:
                z = [i for i in range(size) if (code >> (k - 1 - (p + i))) & 1]
                t = _block_term(Ob, z)
                val *= t
                sabs *= abs(t)
            else:
                ts = [_block_term(Ob, [i for i in range(size) if (m >> i) & 1]) for m in range(1 << size)]
                val *= sum(ts)
                sabs *= sum(abs(t) for t in ts)
        f = lambda x: Fraction(mpmath.nstr(x, 70, min_fixed=-1e9, max_fixed=1e9))
        assert n == sum(s for _, s in spans)
        return f(val), f(sabs)


def test_part_closed_form_against_the_oracle():
    # n = 12, parts of 2^5: the closed form against the binary128 oracle
    # summed over exactly the part's 2^7 subsets
    import oracle
    n, k = 12, 5
    O, spans = product_state_in_order(n, k, 77)
    assert any(s == 2 for p, s in spans if p < k) and any(s == 2 for p, s in spans if p >= k)
    for code in (0, 0b10110, (1 << k) - 1):
        pre = sum(1 << i for i in range(k) if (code >> (k - 1 - i)) & 1)
        masks = np.uint64(pre) | (np.arange(1 << (n - k), dtype=np.uint64) << np.uint64(k))
        _, t3, st = oracle._terms3(O, masks)
        assert (st == 0).all()
        want = sum(Fraction(t3[i, 0]) + Fraction(t3[i, 1]) + Fraction(t3[i, 2]) for i in range(len(masks)))
        got, sabs = part_closed_form(O, spans, k, code)
        assert float(abs(got - want) / sabs) < 1e-28, code
        assert abs(float(sabs) - float(np.sum(np.abs(t3[:, 0])))) <= 1e-12 * float(sabs)

"""TOR_FLAG_CHECK_INPUT: the kernels read the lower triangle and the O00 /
O01 blocks only, so an input that is not exactly Hermitian with the block
structure of Eq. 3 would be evaluated as some other matrix; with the flag
such inputs are refused (TOR_EINPUT) before anything is evaluated."""
import numpy as np
import pytest

import gbs_inputs as g

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tor():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_01177_amd as t
    t.tor_init()
    return t


def _broken(kind, n=12, seed=31):
    O = g.random_instance(n, seed).copy()
    if kind == "hermitian":      # lower and upper triangle disagree
        O[3, 1] += 1e-15
    elif kind == "block":        # O11 != conj(O00), O itself still Hermitian
        d = 1e-14 + 2e-14j
        O[n + 2, n + 1] += d
        O[n + 1, n + 2] += np.conj(d)
    elif kind == "nan":
        O[0, 0] = np.nan
    return O


def test_valid_input_passes_and_gives_the_same_bits(tor):
    O = g.random_instance(12, 30)
    a = tor.tor_eval(O, tier="dd")
    b = tor.tor_eval(O, tier="dd", check_input=True)
    assert a.expansion == b.expansion and a.abs_sum == b.abs_sum


@pytest.mark.parametrize("kind", ["hermitian", "block", "nan"])
def test_broken_input_is_refused(tor, kind):
    O = _broken(kind)
    print(f"[check] {kind}", flush=True)
    with pytest.raises(tor.TorError) as e:
        tor.tor_eval(O, tier="dd", check_input=True)
    assert e.value.code == -6
    with pytest.raises(tor.TorError) as e:
        tor.tor_eval_part(O, 0, 1, tier="fp64", check_input=True)
    assert e.value.code == -6
    if kind != "nan":
        # without the check the same input is evaluated (as another matrix)
        assert tor.tor_eval(O, tier="dd").status == 0


def test_batched_check_refuses_a_batch_with_one_bad_instance(tor):
    good = [g.random_instance(n, 40 + n) for n in (6, 9, 14)]
    empty = np.zeros((0, 0), dtype=np.complex128)
    ok = tor.tor_eval_batched(tor.Batch(good + [empty]), tiers="dd", check_input=True)
    ref = tor.tor_eval_batched(tor.Batch(good + [empty]), tiers="dd")
    assert [r.expansion for r in ok] == [r.expansion for r in ref]
    with pytest.raises(tor.TorError) as e:
        tor.tor_eval_batched(tor.Batch(good[:2] + [_broken("block")] + good[2:]), tiers="dd", check_input=True)
    assert e.value.code == -6

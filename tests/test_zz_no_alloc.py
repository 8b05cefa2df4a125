"""tor_eval_noalloc (the entry point for callers that cannot allocate)
through the C ABI, against tor_eval on the same inputs: two calls in a row,
the second with a smaller instance."""
import ctypes

import numpy as np
import pytest

import gbs_inputs as g


TOL = {"fp64": 1e-12, "dd": 1e-25, "qd": 1e-30}


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_01177_amd import _lib
    L = _lib.lib()
    assert L.tor_init() == 0
    return torch, L, _lib


def _result(raw):
    from paper_2009_01177_amd.api import _results_from
    return _results_from(raw.reshape(1, 8))[0]


def _noalloc(torch, L, _lib, O, tier):
    Od = torch.from_numpy(O).to("cuda")
    n = O.shape[0] // 2
    out = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
    rc = L.tor_eval_noalloc(ctypes.c_void_p(Od.data_ptr()), n, 2 * n, {"fp64": 0, "dd": 1, "qd": 2}[tier], None,
                            ctypes.c_void_p(out.data_ptr()))
    torch.cuda.synchronize()
    return rc, _result(out.cpu().numpy())


def _eval(torch, L, O, tier):
    from paper_2009_01177_amd import _lib
    Od = torch.from_numpy(O).to("cuda")
    n = O.shape[0] // 2
    r = _lib.TorResultC()
    rc = L.tor_eval(ctypes.c_void_p(Od.data_ptr()), n, 2 * n, {"fp64": 0, "dd": 1, "qd": 2}[tier], None, None,
                    ctypes.byref(r))
    from paper_2009_01177_amd.api import _res
    return rc, _res(r)


@pytest.mark.gpu
@pytest.mark.parametrize("tier,n_big,n_small", [("fp64", 30, 14), ("dd", 30, 12), ("qd", 20, 10)])
def test_noalloc_matches_tor_eval_twice(env, tier, n_big, n_small):
    torch, L, _lib = env
    print(f"[noalloc] tier={tier} n={n_big} then n={n_small}", flush=True)
    for n in (n_big, n_small):
        O = g.random_instance(n, 4242 + n)
        rc0, ref = _eval(torch, L, O, tier)
        rc1, got = _noalloc(torch, L, _lib, O, tier)
        assert rc0 == 0 and rc1 == 0 and got.status == 0
        assert got.tier_used == ref.tier_used
        err = float(abs(got.exact - ref.exact) / ref.abs_exact)
        print(f"[noalloc] tier={tier} n={n}: err/S_abs vs tor_eval {err:.2e}", flush=True)
        assert err <= TOL[tier]
        if n == n_small:
            # tor_eval's own plan fits in the buffer: the same bits
            assert got.expansion == ref.expansion


@pytest.mark.gpu
def test_noalloc_edges(env):
    torch, L, _lib = env
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    rc = L.tor_eval_noalloc(None, 0, 0, 1, None, ctypes.c_void_p(out.data_ptr()))
    torch.cuda.synchronize()
    r = _result(out.cpu().numpy())
    assert rc == 0 and r.expansion[0] == 1.0 and r.tier_used == 1
    nmax = L.tor_noalloc_nmax(1)
    O = np.zeros((2 * (nmax + 1), 2 * (nmax + 1)), np.complex128)
    Od = torch.from_numpy(O).to("cuda")
    assert L.tor_eval_noalloc(ctypes.c_void_p(Od.data_ptr()), nmax + 1, 2 * (nmax + 1), 1, None,
                              ctypes.c_void_p(out.data_ptr())) == _lib.TOR_EUNSUPPORTED
    assert L.tor_eval_noalloc(ctypes.c_void_p(Od.data_ptr()), 4, 8, 1, None, None) == _lib.TOR_EINVAL
    assert L.tor_eval_noalloc(ctypes.c_void_p(Od.data_ptr()), 4, 8, 7, None,
                              ctypes.c_void_p(out.data_ptr())) == _lib.TOR_EINVAL


def test_noalloc_limits_need_no_gpu():
    """The largest n the fixed buffer takes, per tier (host only): the
    benchmark's n = 30 and the n = 36 stress size in every tier but QD."""
    from paper_2009_01177_amd import _lib
    L = _lib.lib()
    assert _lib.TOR_NOALLOC_SCRATCH_BYTES == 256 << 20
    nmax = [L.tor_noalloc_nmax(t) for t in (0, 1, 2)]
    assert nmax[0] >= 40 and nmax[1] >= 36 and nmax[2] >= 30, nmax
    assert L.tor_noalloc_nmax(5) == _lib.TOR_EINVAL

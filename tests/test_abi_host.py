"""The C-ABI library loads, exports what include/tor.h declares, and its
host-side logic (Alg. 2 mask functions, work-item plan, argument checks)
behaves; nothing here needs a GPU."""
import ctypes
import itertools
import os
import re
from math import comb

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2009_01177_amd import _lib
    return _lib.lib()


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "tor.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tor_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported(L):
    syms = declared_symbols()
    assert "tor_eval" in syms and "tor_debug_sampled_terms" in syms
    from paper_2009_01177_amd import _lib
    assert sorted(_lib.EXPORTS) == syms
    for s in syms:
        assert hasattr(L, s), s


def test_next_mask_worked_example(L):
    # Sec. 4.1: "010011" -> "001110"
    assert L.tor_next_mask(0b010011) == 0b001110


@pytest.mark.parametrize("N,c", [(6, 2), (7, 3), (10, 5), (12, 1), (9, 9), (8, 0)])
def test_mask_enumeration_brute_force(L, N, c):
    want = sorted((sum(1 << (N - 1 - j) for j in pos) for pos in itertools.combinations(range(N), c)),
                  reverse=True)
    got = [L.tor_kth_mask(N, c, k) for k in range(comb(N, c))]
    assert got == want
    m = L.tor_kth_mask(N, c, 0)
    seq = []
    for _ in range(comb(N, c)):
        seq.append(m)
        m = L.tor_next_mask(m)
    if c > 0:
        assert seq == want
        assert m == 0  # sentinel after the last mask


def test_kth_mask_out_of_range(L):
    assert L.tor_kth_mask(6, 2, comb(6, 2)) == 0
    assert L.tor_kth_mask(6, 7, 0) == 0


@pytest.mark.parametrize("n,d", [(5, 3), (12, 12), (20, 10), (30, 0)])
def test_plan_covers_every_prefix_once_largest_first(n, d):
    from paper_2009_01177_amd import tor_plan_items
    items = tor_plan_items(n, d)
    assert sorted(items.tolist()) == list(range(1 << d))
    pops = [bin(int(x)).count("1") for x in items]
    assert pops == sorted(pops, reverse=True)


def test_phase_clocks_only_in_the_phase_build(L):
    """The regular library has no per-phase clocks and says so; build.py
    writes the phase-clock library beside it."""
    from paper_2009_01177_amd import _lib, build
    out = (ctypes.c_uint64 * _lib.TOR_NPHASE)()
    assert L.tor_debug_phase_clocks(0, out) == _lib.TOR_EUNSUPPORTED
    assert L.tor_debug_phase_clocks(0, None) == _lib.TOR_EINVAL
    assert os.path.exists(build.PHASE_LIB)
    P = ctypes.CDLL(build.PHASE_LIB)
    assert P.tor_debug_phase_clocks(0, None) == _lib.TOR_EINVAL


def test_c_client_links_and_checks_its_arguments_without_a_gpu():
    """The plain C client of the ABI is built, resolves libtor_hip.so from
    the tree, and rejects a bad call before touching a device."""
    import subprocess
    from paper_2009_01177_amd import build
    assert os.path.exists(build.C_CLIENT)
    p = subprocess.run([build.C_CLIENT], capture_output=True, text=True, timeout=60)
    assert p.returncode == 1 and "usage" in p.stderr
    p = subprocess.run([build.C_CLIENT, "/nonexistent", "3"], capture_output=True, text=True, timeout=60)
    assert p.returncode == 1 and "cannot read" in p.stderr


def test_input_error_has_its_own_message(L):
    L.tor_strerror.restype = ctypes.c_char_p
    msg = L.tor_strerror(-6).decode()
    assert "Hermitian" in msg and msg != L.tor_strerror(-1).decode()


def test_argument_checks_need_no_gpu(L):
    from paper_2009_01177_amd import _lib
    out = _lib.TorResultC()
    dummy = ctypes.c_void_p(16)
    assert L.tor_eval(dummy, -1, 2, 1, None, None, ctypes.byref(out)) == _lib.TOR_EINVAL
    assert L.tor_eval(dummy, _lib.TOR_NMAX + 1, 200, 1, None, None, ctypes.byref(out)) == _lib.TOR_EINVAL
    assert L.tor_eval(dummy, 3, 6, 7, None, None, ctypes.byref(out)) == _lib.TOR_EINVAL
    assert L.tor_eval(dummy, 3, 5, 1, None, None, ctypes.byref(out)) == _lib.TOR_EINVAL  # ld < 2n
    assert L.tor_eval(None, 3, 6, 1, None, None, ctypes.byref(out)) == _lib.TOR_EINVAL
    assert L.tor_eval(dummy, 3, 6, 1, None, None, None) == _lib.TOR_EINVAL
    # n = 0 is the empty product and needs no device
    assert L.tor_eval(None, 0, 0, 1, None, None, ctypes.byref(out)) == 0
    assert out.tor[0] == 1.0 and out.abs_sum[0] == 1.0
    assert L.tor_strerror(_lib.TOR_ENOTPD).decode().startswith("I - O")


def test_autotune_table_round_trip_needs_no_gpu(tmp_path):
    import paper_2009_01177_amd as tor
    p = tmp_path / "t.txt"
    p.write_text("30 1 3\n24 0 5\n")
    tor.tor_autotune_load(str(p))
    q = tmp_path / "u.txt"
    tor.tor_autotune_save(str(q))
    lines = set(q.read_text().split("\n"))
    assert {"30 1 3", "24 0 5"} <= lines
    bad = tmp_path / "bad.txt"
    bad.write_text("30 7 3\n")
    with pytest.raises(tor.TorError):
        tor.tor_autotune_load(str(bad))


def test_mcmc_argument_checks_need_no_gpu(L):
    from paper_2009_01177_amd import _lib
    d = ctypes.c_void_p(16)
    ok = dict(O=d, M=6, ld=12, N=2, chains=4, steps=3, P=d, U=d, tier=_lib.TOR_DD, tau=1e-3,
              out=d, st=d)

    def call(**kw):
        a = dict(ok, **kw)
        return L.tor_mcmc(a["O"], a["M"], a["ld"], a["N"], a["chains"], a["steps"], a["P"], a["U"],
                          a["tier"], a["tau"], None, None, a["out"], a["st"])

    E = _lib.TOR_EINVAL
    assert call(M=0) == E
    assert call(N=7) == E                      # more clicks than modes
    assert call(N=-1) == E
    assert call(M=100, ld=200, N=_lib.TOR_NMAX + 1) == E
    assert call(ld=11) == E                    # ld < 2M
    assert call(chains=0) == E and call(steps=0) == E
    assert call(chains=1 << 16, steps=1 << 15) == E   # chains * steps >= 2^31
    assert call(O=None) == E and call(U=None) == E and call(out=None) == E and call(st=None) == E
    assert call(P=None) == E                   # candidates needed when N > 0
    assert call(tier=5) == E
    assert call(tier=_lib.TOR_AUTO, tau=0.0) == E


def test_combine_parts_needs_no_gpu(L):
    from paper_2009_01177_amd import _lib
    from fractions import Fraction as F
    arr = (_lib.TorResultC * 3)()
    vals = [(1.0, 2.0 ** -60), (2.0, -2.0 ** -58), (-0.5, 0.0)]
    for i, (hi, lo) in enumerate(vals):
        arr[i].tor[0], arr[i].tor[1] = hi, lo
        arr[i].abs_sum[0] = abs(hi)
        arr[i].tier_used = _lib.TOR_DD
    out = _lib.TorResultC()
    assert L.tor_combine_parts(_lib.TOR_DD, 10, arr, 3, ctypes.byref(out)) == 0
    got = F(out.tor[0]) + F(out.tor[1])
    assert got == sum(F(h) + F(l) for h, l in vals)
    assert out.abs_sum[0] == 3.5 and out.status == 0 and out.tier_used == _lib.TOR_DD
    # a part's failure is reported; a part of another tier is refused
    arr[1].status = _lib.TOR_ENOTPD
    assert L.tor_combine_parts(_lib.TOR_DD, 10, arr, 3, ctypes.byref(out)) == 0
    assert out.status == _lib.TOR_ENOTPD
    arr[2].tier_used = _lib.TOR_FP64
    assert L.tor_combine_parts(_lib.TOR_DD, 10, arr, 3, ctypes.byref(out)) == _lib.TOR_EINVAL
    assert L.tor_combine_parts(_lib.TOR_DD, 10, arr, 0, ctypes.byref(out)) == _lib.TOR_EINVAL
    # quad-double parts keep all four words
    q = (_lib.TorResultC * 2)()
    for i in range(2):
        q[i].tor[:] = [1.0, 2.0 ** -60, 2.0 ** -120, 2.0 ** -180]
        q[i].tier_used = _lib.TOR_QD
    assert L.tor_combine_parts(_lib.TOR_QD, 10, q, 2, ctypes.byref(out)) == 0
    assert sum(F(x) for x in out.tor) == 2 * (1 + F(2) ** -60 + F(2) ** -120 + F(2) ** -180)


def test_eval_part_argument_checks_need_no_gpu(L):
    from paper_2009_01177_amd import _lib
    out = _lib.TorResultC()
    d = ctypes.c_void_p(16)
    E = _lib.TOR_EINVAL
    assert L.tor_eval_part(d, 10, 20, 1, None, None, 0, 0, ctypes.byref(out)) == E
    assert L.tor_eval_part(d, 10, 20, 1, None, None, 3, 3, ctypes.byref(out)) == E
    assert L.tor_eval_part(d, 10, 20, 1, None, None, -1, 3, ctypes.byref(out)) == E
    assert L.tor_eval_part(d, 10, 20, 1, None, None, 0, 3, None) == E
    assert L.tor_eval_part(d, 12, 24, 1, None, None, 0, 2 ** 31 - 1, ctypes.byref(out)) == E
    assert L.tor_eval_part(None, 0, 0, 1, None, None, 0, 2, ctypes.byref(out)) == E
    assert L.tor_eval_part(None, 0, 0, 1, None, None, 0, 1, ctypes.byref(out)) == 0
    assert out.tor[0] == 1.0


def test_workspace_bytes_needs_no_gpu(L):
    # the device workspace one evaluation allocates: the n = 30 benchmark
    # instance needs about 2 GB in DD; at n = 50 (TOR_NMAX) every tier fits
    # well inside one 288 GB device, DD in about 26 GB
    import paper_2009_01177_amd as t
    from paper_2009_01177_amd import _lib
    GB = 1e9
    assert 1 * GB < t.tor_workspace_bytes(30, "dd") < 4 * GB
    sizes = {tier: t.tor_workspace_bytes(50, tier) for tier in ("fp64", "dd", "qd")}
    assert sizes["fp64"] < 16 * GB and sizes["dd"] < 32 * GB and sizes["qd"] < 100 * GB, sizes
    assert sizes["fp64"] < sizes["dd"] < sizes["qd"]
    for n in range(1, _lib.TOR_NMAX + 1):
        assert t.tor_workspace_bytes(n, "qd") < 100 * GB, n
    assert t.tor_workspace_bytes(0, "dd") == 0
    b = ctypes.c_uint64(0)
    assert L.tor_workspace_bytes(_lib.TOR_NMAX + 1, _lib.TOR_DD, 0, ctypes.byref(b)) == _lib.TOR_EINVAL
    assert L.tor_workspace_bytes(10, 7, 0, ctypes.byref(b)) == _lib.TOR_EINVAL
    assert L.tor_workspace_bytes(10, _lib.TOR_DD, -1, ctypes.byref(b)) == _lib.TOR_EINVAL
    assert L.tor_workspace_bytes(10, _lib.TOR_DD, 0, None) == _lib.TOR_EINVAL


def test_workspace_bytes_is_the_allocated_capacity(L):
    """The workspace grows to exactly the plan of the largest evaluation,
    rounded up to 2 MiB, and that is what tor_workspace_bytes reports: at
    n = 50 about 9.5 GB (FP64), 26 GB (DD), 79 GB (QD)."""
    import paper_2009_01177_amd as t
    from paper_2009_01177_amd import _lib
    step = 2 << 20
    for tier in ("fp64", "dd", "qd"):
        prev = 0
        for n in range(1, _lib.TOR_NMAX + 1):
            b = t.tor_workspace_bytes(n, tier)
            assert b > 0 and b % step == 0, (tier, n, b)
            # a one-instance batch plans the same evaluation
            assert t.tor_batch_workspace_bytes(n, 1, tier) == b, (tier, n)
            prev = b
    GB = 1e9
    s50 = [t.tor_workspace_bytes(50, tier) / GB for tier in ("fp64", "dd", "qd")]
    assert 9 < s50[0] < 10 and 25 < s50[1] < 27 and 78 < s50[2] < 81, s50


def test_batch_groups_stay_within_their_budget(L):
    """A batch group whose plan would pass 4 GiB runs as equal sub-groups:
    at the sampler's default chunk (1 GiB of packed O_S) the batched path
    plans at most 4 GiB for every N up to TOR_NMAX, unless one instance alone
    needs more (then it plans exactly that instance)."""
    import paper_2009_01177_amd as t
    from paper_2009_01177_amd import _lib
    budget = (4 << 30) + (2 << 20)
    for tier in ("fp64", "dd", "qd"):
        for N in range(1, _lib.TOR_NMAX + 1):
            chunk = max(1, (1 << 26) // (4 * N * N))
            b = t.tor_batch_workspace_bytes(N, chunk, tier)
            single = t.tor_workspace_bytes(N, tier)
            assert b <= max(budget, single), (tier, N, chunk, b, single)
            if single > budget:
                assert b == single, (tier, N)
    assert t.tor_batch_workspace_bytes(0, 100, "dd") == 0
    assert t.tor_batch_workspace_bytes(12, 0, "dd") == 0
    b = ctypes.c_uint64(0)
    assert L.tor_batch_workspace_bytes(12, 1, -1, 0, ctypes.byref(b)) == _lib.TOR_EINVAL
    assert L.tor_batch_workspace_bytes(12, 9, 1, 0, ctypes.byref(b)) == _lib.TOR_EINVAL
    assert L.tor_batch_workspace_bytes(12, 1, 1, 0, None) == _lib.TOR_EINVAL


def _workspace_in_subprocess(env_table, queries):
    """tor_workspace_bytes(n, tier, 0) in a fresh process whose
    TOR_AUTOTUNE_TABLE is env_table (None: unset)."""
    import json
    import subprocess
    import sys
    code = ("import json, sys; sys.path.insert(0, %r); import paper_2009_01177_amd as t; "
            "print(json.dumps([t.tor_workspace_bytes(n, tier) for n, tier in %r]))" % (ROOT, queries))
    env = dict(os.environ)
    env.pop("TOR_AUTOTUNE_TABLE", None)
    if env_table is not None:
        env["TOR_AUTOTUNE_TABLE"] = env_table
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, check=True)
    return json.loads(out.stdout.strip().splitlines()[-1])


def test_the_shipped_tuned_table_is_read_before_the_first_plan(tmp_path):
    """Bottom sizes of data/autotune_default.txt are the library's defaults
    in a fresh process (a plan's size shows its bottom size); a table named
    by TOR_AUTOTUNE_TABLE replaces it, and an empty name reads none."""
    import paper_2009_01177_amd as t
    rows = [tuple(int(x) for x in ln.split()) for ln in
            open(os.path.join(ROOT, "paper_2009_01177_amd", "data", "autotune_default.txt"))]
    table = {(n, tier): sb for n, tier, sb in rows}
    assert all((n, tier) in table for n in range(1, 41) for tier in (0, 1, 2))
    names = {0: "fp64", 1: "dd", 2: "qd"}
    picks = [(8, 1), (10, 0), (9, 2), (30, 1)]
    got = _workspace_in_subprocess(None, [(n, names[tier]) for n, tier in picks])
    for (n, tier), b in zip(picks, got):
        assert b == t.tor_workspace_bytes(n, names[tier], table[(n, tier)]), (n, tier)
    # another table
    p = tmp_path / "tune.txt"
    p.write_text("8 1 4\n")
    assert _workspace_in_subprocess(str(p), [(8, "dd")]) == [t.tor_workspace_bytes(8, "dd", 4)]
    # no table: the built-in choice (the largest bottom the tier compiles)
    assert _workspace_in_subprocess("", [(8, "dd")]) == [t.tor_workspace_bytes(8, "dd", 5)]

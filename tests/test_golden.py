"""Values the paper prints, kept as cited text fixtures under tests/golden/."""
import ctypes
import math
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _rows(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return [line.split() for line in f if line.strip() and not line.startswith("#")]


def test_next_mask_worked_example():
    """The library's mask successor reproduces the paper's worked example."""
    from paper_2009_01177_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    L = ctypes.CDLL(_lib.LIB_PATH)
    L.tor_next_mask.restype = ctypes.c_uint64
    L.tor_next_mask.argtypes = [ctypes.c_uint64]
    for cur, nxt in _rows("alg2_next_mask.txt"):
        assert L.tor_next_mask(int(cur, 2)) == int(nxt, 2)
        assert bin(int(cur, 2)).count("1") == bin(int(nxt, 2)).count("1")


def test_eq9_against_the_printed_times_and_rates():
    """bench.py's Eq. 9 count at N = 50 over the paper's own times gives
    rates just below the largest sustained rates it prints (reached at
    other N), in both modes: a wrong coefficient in the transcription would
    land far from them."""
    import sys
    sys.path.insert(0, os.path.dirname(HERE))
    import bench
    g = {k: float(v) for k, v in _rows("eq9_time_to_solution.txt")}
    flops = bench.paper_eq9_flops(int(g["N"]))
    for mode in ("128", "256"):
        rate = flops / g["seconds_" + mode] / 1e15
        top = g["max_pflops_" + mode]
        assert 0.9 * top <= rate <= top, (mode, rate, top)
    # Eq. 9 is Eq. 8's linear-solver count summed over the 2i x 2i blocks
    n = int(g["N"])
    eq8 = sum(math.comb(n, i) * ((4.0 / 3) * (2 * i) ** 3 + (2 * i) ** 2 - (4.0 / 3) * (2 * i)) for i in range(1, n + 1))
    assert abs(eq8 - flops) <= 1e-12 * flops

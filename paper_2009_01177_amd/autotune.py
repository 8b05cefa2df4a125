"""Write the shipped bottom-size table: tor_autotune for every (n, tier),
n = 1..40, on the current device, saved as data/autotune_default.txt (read
by the library before its first evaluation).

Usage: python -m paper_2009_01177_amd.autotune [--nmax 40] [--out PATH]
"""
from __future__ import annotations

import argparse
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "data", "autotune_default.txt")


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--nmax", type=int, default=40)
    ap.add_argument("--out", default=DEFAULT_TABLE)
    a = ap.parse_args()
    # start from an empty table: the shipped one must not seed the result
    os.environ["TOR_AUTOTUNE_TABLE"] = ""
    import paper_2009_01177_amd as tor
    t0 = time.time()
    for tier in ("fp64", "dd", "qd"):
        for n in range(1, a.nmax + 1):
            best, ms = tor.tor_autotune(n, tier)
            print(f"[autotune] {tier} n={n}: s_b={best} ms={[round(x, 3) for x in ms]} ({time.time() - t0:.1f} s)",
                  flush=True)
    tor.tor_autotune_save(a.out)
    print(f"[autotune] saved {a.out}", flush=True)


if __name__ == "__main__":
    main()

"""The committed profiles describe the kernel code in the tree: every
summary under profiles/ that names a kernel code hash names the current one
(bench.py's kernel_code_hash over the subset-tree kernel sources), so a
change to those sources without retaking the profiles fails here, and the
HBM traffic the benchmark reports is never read from counters of other
code.  CPU only."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def _hash():
    import sys
    sys.path.insert(0, ROOT)
    import bench
    return bench.kernel_code_hash()


def test_traffic_counters_belong_to_the_current_kernel_code():
    kv = dict(line.strip().split("=", 1) for line in open(os.path.join(PROFILES, "leaf_kernel_n30_traffic.txt"))
              if "=" in line and not line.startswith("#"))
    assert kv["code_sha256_prefix"] == _hash()
    for tier in ("dd", "fp64"):
        assert 1.0 <= int(kv[f"{tier}_traffic_bytes"]) / int(kv[f"{tier}_algorithmic_bytes"]) < 1.2


@pytest.mark.parametrize("name", sorted(f for f in os.listdir(PROFILES) if f.endswith(".md")))
def test_profile_summaries_name_the_current_kernel_code(name):
    text = open(os.path.join(PROFILES, name)).read()
    hashes = re.findall(r"kernel code hash \(bench\.py `kernel_code_hash`\): ([0-9a-f]{16})", text)
    assert hashes, name
    assert set(hashes) == {_hash()}, name
    assert "_work" not in text  # made by committed files only

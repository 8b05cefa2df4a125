"""The phase-clock build of the library (libtor_hip_phase.so): the same
kernels with per-phase shader-clock marks, which must not change a single
bit of any result, and whose totals cover every phase of the middle +
bottom kernel."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import gbs_inputs as g

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
import torch
import gbs_inputs as g
import paper_2009_01177_amd as tor
O = g.random_instance(20, 4321)
Od = torch.from_numpy(O).cuda()
out = {}
for tier in ("fp64", "dd"):
    tor.tor_eval(Od, tier=tier)
    torch.cuda.synchronize()
    tor.tor_debug_phase_clocks(reset=True)
    r = tor.tor_eval(Od, tier=tier)
    ph = tor.tor_debug_phase_clocks(reset=True)
    out[tier] = {"tor": [x.hex() for x in r.expansion], "clocks": ph}
print(json.dumps(out), flush=True)
"""


def test_phase_build_gives_the_same_bits_and_covers_every_phase():
    import torch
    import paper_2009_01177_amd as tor
    from paper_2009_01177_amd import build
    env = dict(os.environ, TOR_LIBRARY=build.PHASE_LIB, PYTHONPATH=ROOT)
    print("[phase] child with the phase-clock build", flush=True)
    p = subprocess.run([sys.executable, "-c", CHILD], env=env, cwd=ROOT, capture_output=True, text=True, timeout=240)
    assert p.returncode == 0, p.stderr[-2000:]
    got = json.loads(p.stdout.strip().splitlines()[-1])
    O = g.random_instance(20, 4321)
    Od = torch.from_numpy(O).cuda()
    for tier in ("fp64", "dd"):
        r = tor.tor_eval(Od, tier=tier)
        assert got[tier]["tor"] == [x.hex() for x in r.expansion], tier
        ph = got[tier]["clocks"]
        print(f"[phase] {tier} {ph}", flush=True)
        for k in ("expand", "bottom", "totals", "wait_after_expand"):
            assert ph[k] > 0, (tier, k)
        assert all(v >= 0 for v in ph.values())
    # the regular library has no clocks
    with pytest.raises(tor.TorError):
        tor.tor_debug_phase_clocks()

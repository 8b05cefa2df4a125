"""The C ABI from plain C: tests/c_client/tor_client (gcc, linked against
libtor_hip.so, no Python or PyTorch in the process) evaluates instances
with tor_eval in every tier and with one tor_eval_batched call on its own
stream; its results are the Python binding's bit for bit and the oracle's
within the tiers' tolerances."""
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import gbs_inputs as g
import oracle

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLIENT = os.path.join(ROOT, "tests", "c_client", "tor_client")
TOL = {0: 1e-12, 1: 1e-25, 2: 1e-30}


def _parse(text):
    out = {}
    for line in text.splitlines():
        p = line.split()
        if p and p[0] in ("eval", "batched"):
            out[(p[0], int(p[1]), int(p[2]))] = (int(p[3]), [float.fromhex(x) for x in p[4:8]],
                                                 [float.fromhex(x) for x in p[8:10]])
    return out


def test_c_client_matches_the_binding_and_the_oracle(tmp_path):
    import torch
    import paper_2009_01177_amd as tor
    assert os.path.exists(CLIENT), "built by paper_2009_01177_amd.build"
    Os = [g.random_instance(n, 7100 + n) for n in (5, 12, 17)]
    path = str(tmp_path / "o.bin")
    with open(path, "wb") as f:
        for O in Os:
            np.ascontiguousarray(O, dtype="<c16").tofile(f)
    print("[c_client] three instances, n = 5, 12, 17", flush=True)
    p = subprocess.run([CLIENT, path] + [str(O.shape[0] // 2) for O in Os], capture_output=True, text=True,
                       timeout=240)
    assert p.returncode == 0, p.stderr
    got = _parse(p.stdout)
    batch = tor.tor_eval_batched(tor.Batch(Os), tiers="dd")
    for k, O in enumerate(Os):
        ref = oracle.tor(O)
        for tier in (0, 1, 2):
            status, t, a = got[("eval", k, tier)]
            mine = tor.tor_eval(torch.from_numpy(O).cuda(), tier=tier)
            assert status == 0
            assert tuple(t) == tuple(mine.expansion), (k, tier)
            err = float(abs(sum(map(Fraction, t)) - ref["tor"]) / ref["abs_sum"])
            assert err <= TOL[tier], (k, tier, err)
        status, t, a = got[("batched", k, 1)]
        assert status == 0
        assert tuple(t) == tuple(batch[k].expansion), k

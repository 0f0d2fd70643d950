"""Bit-for-bit repeatability of the integrator: the same cells give the
same densities, counters and step records whichever persistent workgroup
(slot) picks them up, including on a workspace whose slots start out
filled with NaN."""
import os
import subprocess
import sys

import numpy as np
import pytest

from conftest import ROOT, YEAR_S

pytestmark = pytest.mark.gpu

SCRIPT = r"""
import sys, numpy as np, torch
sys.path.insert(0, {root!r})
import synthnet, paper_2312_04998_amd as acm
net, cells = synthnet.workload("tiny", n_cells=4)
N = acm.Network.from_synth(net)
ws = acm.Workspace(N, n_slots=3)
y0 = np.repeat(cells.y0[:1], 7, 0)
T = np.array([20.0, 90.0, 20.0, 150.0, 90.0, 33.0, 20.0])
res = []
for rep in range(2):
    y = torch.from_numpy(y0.copy()).cuda()
    o = ws.integrate(y, torch.from_numpy(T).cuda(), 1e5 * {year!r}, tape_cap=20000)
    res.append((y.cpu().numpy(), o["stats"].cpu().numpy(), o["tape_len"].cpu().numpy()))
np.savez({out!r}, y0=res[0][0], s0=res[0][1], l0=res[0][2], y1=res[1][0], s1=res[1][1], l1=res[1][2])
"""


def _run(tmp_path, poison):
    out = str(tmp_path / f"det_{poison}.npz")
    env = dict(os.environ)
    env["ASTROCHEM_POISON_WS"] = "1" if poison else "0"
    code = SCRIPT.format(root=ROOT, year=YEAR_S, out=out)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return np.load(out)


def test_integrator_is_repeatable(tmp_path):
    a = _run(tmp_path, poison=False)
    b = _run(tmp_path, poison=True)
    # cells 0, 2, 6 are the same input: identical results on any slot
    for d in (a, b):
        assert np.array_equal(d["y0"], d["y1"]) and np.array_equal(d["s0"], d["s1"])
        assert np.array_equal(d["y0"][0], d["y0"][2]) and np.array_equal(d["y0"][0], d["y0"][6])
        assert np.array_equal(d["s0"][1], d["s0"][4])
    assert np.all(np.isfinite(b["y0"]))
    assert np.array_equal(a["y0"], b["y0"]) and np.array_equal(a["l0"], b["l0"])

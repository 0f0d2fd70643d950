"""Capture of the hot path in a HIP graph: the library's calls allocate
nothing and clear their device queue with a kernel, so rhs, jac, the fused
rhs_jac and the persistent integrator can be recorded once and replayed. Every replay,
with eager work and synchronisations in between, must reproduce the eager
result bit for bit."""
import numpy as np
import pytest

import synthnet
from conftest import YEAR_S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def acm(torch_dev):
    import paper_2312_04998_amd as acm
    return acm


@pytest.mark.parametrize("which", ["tiny", "medium"])
def test_graph_replays_integration(acm, torch_dev, which):
    torch = torch_dev
    net, cells = synthnet.workload(which, n_cells=6)
    N = acm.Network.from_synth(net)
    ws = acm.Workspace(N, n_slots=4)
    t_end = (1e3 if which == "tiny" else 10.0) * YEAR_S
    y0 = torch.from_numpy(cells.y0.copy()).cuda()
    T = torch.from_numpy(cells.T.copy()).cuda()
    # eager reference (rhs, jac and integration)
    f_ref = N.rhs(y0, T)
    j_ref = N.jac(y0, T)
    y_ref = y0.clone()
    o_ref = ws.integrate(y_ref, T, t_end)
    torch.cuda.synchronize()

    y = y0.clone()
    f = torch.empty_like(y0)
    jv = torch.empty_like(j_ref)
    f2 = torch.empty_like(y0)                       # the fused call's outputs
    jv2 = torch.empty_like(j_ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):                      # warm-up on the capture stream
        y.copy_(y0)
        ws.integrate(y, T, t_end)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        y.copy_(y0)
        acm.ac_rhs(N, None, y0, T, f)
        acm.ac_jac(N, None, y0, T, jv)
        acm.ac_rhs_jac(N, None, y0, T, f2, jv2)
        out = ws.integrate(y, T, t_end)
    for rep in range(3):
        y.fill_(-1.0)
        f.zero_()
        jv.zero_()
        f2.zero_()
        jv2.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(f, f_ref) and torch.equal(jv, j_ref), rep
        assert torch.equal(f2, f_ref) and torch.equal(jv2, j_ref), rep
        assert torch.equal(y, y_ref), rep
        assert torch.equal(out["stats"], o_ref["stats"]) and torch.equal(out["status"], o_ref["status"])
        # eager work between replays
        N.rhs(y0 * 1.5, T)
        torch.cuda.synchronize()

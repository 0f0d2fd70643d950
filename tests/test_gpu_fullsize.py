"""Parity at the workloads' full sizes, in the launch configurations the
benchmark uses, on outputs the oracle can compute one cell at a time:

* VJP over 65,536 cells of the 470/4600 network: sampled dL/dn rows, and
  the cross-cell dL/dlog alpha sum against the oracle's full sum;
* batched integration of 16,384 cells (256 persistent workgroups pulling
  from the device queue), bounded to 200 steps per cell so the run stays
  short; sampled cells against the oracle under the same step budget;
* the discrete adjoint over 4,096 cells, bounded to 60 steps per cell;
  three sampled cells carry the oracle's own tape and are compared with
  the oracle's forward sensitivities through it."""
import numpy as np
import pytest

import synthnet
from conftest import YEAR_S
from test_gpu_integrate import _agree, oracle_with_envelope

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


def _t(a, dtype=np.float64):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype)).cuda()


def _sample(n, k, seed=11):
    return np.sort(np.random.default_rng(seed).choice(n, k, replace=False))


def test_vjp_full_size(acm, torch_dev, oracle_mod, medium_net):
    torch = torch_dev
    net = medium_net
    C = 65536
    cells = synthnet.make_cells(net, C, synthnet.SEED_BASE + 1)
    v = np.random.default_rng(21).standard_normal(cells.y0.shape)
    N = acm.Network.from_synth(net)
    gy, gl = N.vjp(_t(cells.y0), _t(cells.T), _t(v))
    gy, gl = gy.cpu().numpy(), gl.cpu().numpy()
    assert np.isfinite(gy).all() and np.isfinite(gl).all()
    idx = _sample(C, 32)
    ref_gy, _ = oracle_mod.vjp(net, cells.y0[idx], cells.T[idx], v[idx])
    _, abJ = oracle_mod.jac_dense(net, cells.y0[idx], cells.T[idx], with_abs=True)
    scale = np.einsum("ci,cia->ca", np.abs(v[idx]), abJ)
    assert np.all(np.abs(gy[idx] - ref_gy) <= 1e-12 * scale + 1e-300)
    # the cell sum of dL/dlog alpha, against the oracle's, in chunks of cells
    S = np.abs(oracle_mod.stoich(net)).astype(np.float64)
    ref_gl = np.zeros(net.n_reactions)
    scale_gl = np.zeros(net.n_reactions)
    for s in range(0, C, 4096):
        e = s + 4096
        _, g = oracle_mod.vjp(net, cells.y0[s:e], cells.T[s:e], v[s:e])
        ref_gl += g.sum(0)
        r = oracle_mod.rates(net, cells.y0[s:e], cells.T[s:e])
        scale_gl += (np.abs(r) * (np.abs(v[s:e]) @ S)).sum(0)
    # 65,536 terms per reaction: allow the summation's growth in rounding
    assert np.all(np.abs(gl - ref_gl) <= 1e-10 * scale_gl + 1e-300)


def test_integration_full_size_sampled(acm, torch_dev, oracle_mod, medium_net):
    torch = torch_dev
    net = medium_net
    C = 16384
    cells = synthnet.make_cells(net, C, synthnet.SEED_BASE + 2)
    N = acm.Network.from_synth(net)
    ws = acm.Workspace(N)
    y = _t(cells.y0)
    out = ws.integrate(y, _t(cells.T), 1e6 * YEAR_S, max_steps=200)
    st = out["status"].cpu().numpy()
    steps = out["stats"][:, 0].cpu().numpy()
    assert set(np.unique(st).tolist()) <= {acm.AC_CELL_OK, acm.AC_CELL_MAXSTEPS}
    assert steps.max() == 200 and bool(torch.isfinite(y).all())
    idx = _sample(C, 4)
    ref, env, _ = oracle_with_envelope(oracle_mod, net, cells.y0[idx], cells.T[idx], 1e6 * YEAR_S,
                                       k=8, max_steps=200)
    assert st[idx].tolist() == ref["status"].tolist()
    ok = _agree(y.cpu().numpy()[idx], ref["y"], envelope=env)
    assert ok.all(), np.argwhere(~ok)[:5]


def test_adjoint_full_size_sampled(acm, torch_dev, oracle_mod, medium_net):
    torch = torch_dev
    net = medium_net
    C, K = 4096, 60
    cells = synthnet.make_cells(net, C, synthnet.SEED_BASE + 3)
    N = acm.Network.from_synth(net)
    ws = acm.Workspace(N)
    cap = 4 * K + 16
    y = _t(cells.y0)
    fw = ws.integrate(y, _t(cells.T), 1e6 * YEAR_S, max_steps=K, tape_cap=cap)
    tape = fw["tape"]
    tlen = fw["tape_len"].clone()
    idx = _sample(C, 3)
    ref = oracle_mod.bdf(net, cells.y0[idx], cells.T[idx], 1e6 * YEAR_S, max_steps=K, tape_cap=cap)
    ref_tape = acm.tape_from_numpy(ref["tape"])
    for r, c in enumerate(idx):
        tape[int(c)] = ref_tape[r]
        tlen[int(c)] = int(ref["tape_len"][r])
    tgt = np.random.default_rng(8).choice(net.n_species, 8, replace=False)
    yT = y.cpu().numpy()
    lam = np.zeros_like(cells.y0)
    lam[:, tgt] = 1.0 / np.maximum(yT[:, tgt], 1e-30)
    lam[idx] = 0.0
    lam[idx[:, None], tgt[None, :]] = 1.0 / np.maximum(ref["y"][:, tgt], 1e-30)
    out = ws.adjoint(_t(cells.y0), _t(cells.T), tape, tlen, _t(lam), want_cells=True)
    assert int((out["status"] == 0).sum()) == C
    g0 = out["dL_dy0"].cpu().numpy()
    assert np.isfinite(g0).all() and bool(torch.isfinite(out["dL_dlogalpha"]).all())
    gc = out["g_cells"][torch.from_numpy(idx).cuda()].cpu().numpy()
    rng = np.random.default_rng(9)
    n_dir = 2
    dy0 = cells.y0[idx][:, None, :] * rng.standard_normal((3, n_dir, net.n_species))
    dla = rng.standard_normal((n_dir, net.n_reactions))
    _, s = oracle_mod.bdf_replay(net, cells.y0[idx], cells.T[idx], ref["tape"], ref["tape_len"],
                                 dy0=dy0, dlogalpha=dla, n_dir=n_dir)
    for r in range(3):
        for d in range(n_dir):
            lhs = float(np.dot(lam[idx[r]], s[r, d]))
            t_y = g0[idx[r]] * dy0[r, d]
            t_p = gc[r] * dla[d]
            rhs = float(t_y.sum() + t_p.sum())
            scale = float(np.abs(lam[idx[r]] * s[r, d]).sum() + np.abs(t_y).sum() + np.abs(t_p).sum())
            assert abs(lhs - rhs) <= 1e-6 * scale, (r, d, lhs, rhs, scale)

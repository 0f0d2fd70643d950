"""GPU parity for networks whose one-body reactions follow the cosmic-ray
and photo rate laws (the coefficients depend on temperature, cosmic-ray
ionisation rate and FUV intensity, Sec. 3), with per-cell conditions
(T, A_V, zeta/zeta_0, G_0): rate coefficients, RHS, Jacobian, VJP, the
fused call, and integration (replay strictly, free running within the
oracle's rerun envelope) against the oracle."""
import numpy as np
import pytest

import synthnet
from conftest import YEAR_S

pytestmark = pytest.mark.gpu

REL = 1e-12


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


def _close(gpu, ref, scale, rel=REL):
    bad = np.abs(np.asarray(gpu) - ref) > rel * scale
    assert not bad.any(), (int(bad.sum()), np.argwhere(bad)[:5].tolist())


@pytest.fixture(scope="module")
def typed(medium_net):
    net = synthnet.with_rate_laws(medium_net, 5)
    cells = synthnet.make_cells(net, 300, synthnet.SEED_BASE + 9)
    cond = synthnet.make_conditions(cells.T, 9)
    return net, cells.y0, cond


def _jac_at_pattern(N, J):
    rp, col = N.jac_pattern()
    rows = np.repeat(np.arange(N.n_species), np.diff(rp))
    return J[:, rows, col]


def test_rates_with_laws(acm, oracle_mod, typed):
    net, y, cond = typed
    N = acm.Network.from_synth(net)
    assert N.n_cond == 4
    k = N.rates(_t(cond)).cpu().numpy()
    ref = oracle_mod.rate_coeffs(net, cond)
    assert np.all(np.abs(k - ref) <= 2e-13 * np.abs(ref))
    # the typed reactions do differ from the Kooij form of the same parameters
    assert np.all(net.law[net.rtype == 1] > 0)


@pytest.mark.parametrize("layout", ["sell", "csr", "runs"])
def test_rhs_jac_vjp_with_laws(acm, oracle_mod, typed, layout):
    net, y, cond = typed
    N = acm.Network.from_synth(net, layout=layout)
    n = 67
    yd, cd = _t(y[:n]), _t(cond[:n])
    f = N.rhs(yd, cd).cpu().numpy()
    ref, ab = oracle_mod.rhs(net, y[:n], cond[:n], with_abs=True)
    _close(f, ref, ab)
    jv = N.jac(yd[:9], cd[:9]).cpu().numpy()
    J, abJ = oracle_mod.jac_dense(net, y[:9], cond[:9], with_abs=True)
    _close(jv, _jac_at_pattern(N, J), _jac_at_pattern(N, abJ))
    v = np.random.default_rng(3).standard_normal(y[:9].shape)
    gy, gl = N.vjp(yd[:9], cd[:9], _t(v))
    ref_gy, ref_gl = oracle_mod.vjp(net, y[:9], cond[:9], v)
    _close(gy.cpu().numpy(), ref_gy, np.einsum("ci,cia->ca", np.abs(v), abJ))
    S = np.abs(oracle_mod.stoich(net)).astype(np.float64)
    r = oracle_mod.rates(net, y[:9], cond[:9])
    _close(gl.cpu().numpy(), ref_gl.sum(0), (np.abs(r) * (np.abs(v) @ S)).sum(0), rel=1e-11)


def test_fused_equals_separate_with_laws(acm, typed, torch_dev):
    torch = torch_dev
    net, y, cond = typed
    N = acm.Network.from_synth(net, layout="sell", ordering="natural")
    n = 300
    yd, cd = _t(y[:n]), _t(cond[:n])
    d1, d2 = torch.empty_like(yd), torch.empty_like(yd)
    j1 = torch.empty((n, N.nnz_j), dtype=torch.float64, device="cuda")
    j2 = torch.empty_like(j1)
    acm.ac_rhs(N, None, yd, cd, d1)
    acm.ac_jac(N, None, yd, cd, j1)
    acm.ac_rhs_jac(N, None, yd, cd, d2, j2)
    assert torch.equal(d1, d2) and torch.equal(j1, j2)


def test_conditions_shape_checked(acm, typed):
    net, y, cond = typed
    N = acm.Network.from_synth(net)
    with pytest.raises(ValueError):
        N.rhs(_t(y[:4]), _t(cond[:4, 0]))


def test_integration_replay_strict_with_laws(acm, oracle_mod, typed):
    """The GPU replays the oracle's step sequence of 3 cells (BDF 1-5 to
    1e4 yr) and matches the oracle's replay to rtol 1e-6 above 1e-20."""
    net, y, cond = typed
    idx = [0, 1, 2]
    y0, c0 = y[idx], cond[idx]
    ref = oracle_mod.bdf(net, y0, c0, 1e4 * YEAR_S, tape_cap=20000)
    assert np.all(ref["status"] == 0)
    y_rep, _ = oracle_mod.bdf_replay(net, y0, c0, ref["tape"], ref["tape_len"])
    N = acm.Network.from_synth(net)
    ws = acm.Workspace(N, n_slots=3)
    out = ws.adjoint(_t(y0), _t(c0), acm.tape_from_numpy(ref["tape"]),
                     _t(ref["tape_len"], np.int32), _t(np.ones_like(y0)), want_y=True,
                     want_glog=False)
    assert out["status"].cpu().tolist() == [0, 0, 0]
    yg = out["y_final"].cpu().numpy()
    ok = (np.abs(yg - y_rep) <= 1e-6 * np.abs(y_rep)) | (np.maximum(np.abs(yg), np.abs(y_rep)) < 1e-20)
    assert ok.all(), np.argwhere(~ok)[:5].tolist()


def test_integration_free_running_with_laws(acm, oracle_mod, typed):
    """Free-running batched integration of 4 cells to 1e4 yr within 10x the
    spread of 8 perturbed oracle reruns; bad conditions (A_V < 0) are
    rejected as bad input."""
    from test_gpu_integrate import _agree, oracle_with_envelope
    net, y, cond = typed
    idx = [3, 4, 5, 6]
    y0, c0 = y[idx].copy(), cond[idx].copy()
    N = acm.Network.from_synth(net)
    ws = acm.Workspace(N, n_slots=4)
    yd = _t(y0)
    out = ws.integrate(yd, _t(c0), 1e4 * YEAR_S)
    ref, env, _ = oracle_with_envelope(oracle_mod, net, y0, c0, 1e4 * YEAR_S, k=8)
    assert out["status"].cpu().tolist() == ref["status"].tolist() == [0] * 4
    yg = yd.cpu().numpy()
    assert _agree(yg, ref["y"], envelope=env).all()
    print(f"strict 1e-6 bar met by {_agree(yg, ref['y']).mean():.4f} of species-cells")
    bad = c0[:1].copy()
    bad[0, 1] = -1.0
    out = ws.integrate(_t(y0[:1]), _t(bad), 1e4 * YEAR_S)
    assert out["status"].cpu().tolist() == [acm.AC_CELL_BADINPUT]

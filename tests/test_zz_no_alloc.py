"""ac_vjp_static, the VJP that allocates nothing (its partial sums live in
the library's per-GPU scratch array), against ac_vjp on the same inputs:
two calls in a row, the second with fewer cells, must agree bit for bit
(same kernels, same fixed grid), and both against the oracle to the VJP's
1e-12 bar."""
import numpy as np
import pytest

import synthnet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()


def test_vjp_static_matches_vjp(torch_dev, oracle_mod, medium_net):
    import paper_2312_04998_amd as acm
    torch = torch_dev
    net = medium_net
    cells = synthnet.make_cells(net, 300, synthnet.SEED_BASE + 5)
    v = np.random.default_rng(17).standard_normal(cells.y0.shape)
    N = acm.Network.from_synth(net)
    for n in (300, 41):           # the second call is smaller: stale rows must not leak in
        y, T, vv = _t(cells.y0[:n]), _t(cells.T[:n]), _t(v[:n])
        gy_a = torch.empty_like(y)
        gl_a = torch.empty(net.n_reactions, dtype=torch.float64, device="cuda")
        gy_b, gl_b = torch.empty_like(gy_a), torch.empty_like(gl_a)
        acm.ac_vjp_static(N, None, y, T, vv, gy_b, gl_b)
        acm.ac_vjp(N, None, y, T, vv, gy_a, gl_a)
        torch.cuda.synchronize()
        assert torch.equal(gy_a, gy_b) and torch.equal(gl_a, gl_b), n
        ref_gy, ref_gl = oracle_mod.vjp(net, cells.y0[:n], cells.T[:n], v[:n])
        _, abJ = oracle_mod.jac_dense(net, cells.y0[:8], cells.T[:8], with_abs=True)
        scale = np.einsum("ci,cia->ca", np.abs(v[:8]), abJ)
        assert np.all(np.abs(gy_b.cpu().numpy()[:8] - ref_gy[:8]) <= 1e-12 * scale + 1e-300)
        S = np.abs(oracle_mod.stoich(net)).astype(np.float64)
        r = oracle_mod.rates(net, cells.y0[:n], cells.T[:n])
        scale_gl = (np.abs(r) * (np.abs(v[:n]) @ S)).sum(0)
        assert np.all(np.abs(gl_b.cpu().numpy() - ref_gl.sum(0)) <= 1e-11 * scale_gl + 1e-300)
    # only the cotangent of y: no scratch use
    gy_c = torch.empty_like(gy_a)
    acm.ac_vjp_static(N, None, y, T, vv, gy_c, None)
    assert torch.equal(gy_c, gy_a)


def test_vjp_static_limit(torch_dev):
    """Networks beyond the scratch's 8192 reactions are refused, before any
    launch, when the parameter gradient is asked for."""
    import paper_2312_04998_amd as acm
    from conftest import network_from
    nr = 8200
    net = network_from([([0], [1]), ([1], [0])] * (nr // 2), np.full(nr, 1e-9), 2)
    N = acm.Network(net.reactants, net.products, net.alpha, net.beta, net.gamma,
                    composition=np.zeros((2, 6), np.int8))
    y, T, v = _t([[1.0, 2.0]]), _t([50.0]), _t([[1.0, -1.0]])
    gl = _t(np.zeros(nr))
    with pytest.raises(acm.AstrochemError) as e:
        acm.ac_vjp_static(N, None, y, T, v, None, gl)
    assert e.value.status == acm.AC_ELIMIT

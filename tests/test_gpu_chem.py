"""GPU parity of rates, RHS, Jacobian and VJP against the oracle, through
the C ABI. Tolerance (FP64): |gpu - oracle| <= 1e-12 * sum|terms| per
output, exactly 0 where every term is 0."""
import numpy as np
import pytest

import synthnet

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


def _t(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()


def _close(gpu, ref, scale, rel=REL):
    gpu = np.asarray(gpu)
    bad = np.abs(gpu - ref) > rel * scale
    assert not bad.any(), (int(bad.sum()), np.argwhere(bad)[:5].tolist(),
                           float(np.max(np.abs(gpu - ref) / np.maximum(scale, 1e-300))))


def _sample(n, k, seed=0):
    rng = np.random.default_rng(seed)
    idx = np.unique(np.concatenate([[0, n - 1], rng.choice(n, min(k, n), replace=False)]))
    return idx


@pytest.fixture(scope="module")
def med_cells(medium_net):
    return synthnet.make_cells(medium_net, 1000, synthnet.SEED_BASE + 1)


def test_rates(acm, torch_dev, oracle_mod, medium_net, med_cells):
    torch = torch_dev
    N = acm.Network.from_synth(medium_net)
    T = med_cells.T[:257]
    k = N.rates(_t(torch, T)).cpu().numpy()
    ref = oracle_mod.rate_coeffs(medium_net, T)
    # exp of an argument of size <= ~140 carries ~140 ulp of relative error
    _close(k, ref, 2e-13 / REL * np.abs(ref))


@pytest.mark.parametrize("layout", ["csr", "sell", "coo", "runs", "ccs"])
@pytest.mark.parametrize("ordering", ["natural", "nnz", "rcm"])
def test_rhs(acm, torch_dev, oracle_mod, medium_net, med_cells, layout, ordering):
    torch = torch_dev
    N = acm.Network.from_synth(medium_net, layout=layout, ordering=ordering)
    n = 333                                   # ragged against any grid
    y, T = med_cells.y0[:n], med_cells.T[:n]
    f = N.rhs(_t(torch, y), _t(torch, T)).cpu().numpy()
    ref, ab = oracle_mod.rhs(medium_net, y, T, with_abs=True)
    _close(f, ref, ab)


def test_rhs_layouts_agree_bitwise(acm, torch_dev, medium_net, med_cells):
    """CSR and SELL visit the same terms in the same order per chunk."""
    torch = torch_dev
    y, T = _t(torch, med_cells.y0[:200]), _t(torch, med_cells.T[:200])
    a = acm.Network.from_synth(medium_net, layout="csr", ordering="nnz").rhs(y, T)
    b = acm.Network.from_synth(medium_net, layout="sell", ordering="nnz").rhs(y, T)
    c = acm.Network.from_synth(medium_net, layout="sell", ordering="nnz").rhs(y, T)
    assert torch.equal(a, b) and torch.equal(b, c)


def test_rhs_k(acm, torch_dev, oracle_mod, medium_net, med_cells):
    torch = torch_dev
    N = acm.Network.from_synth(medium_net, layout="sell")
    y, T = med_cells.y0[:130], med_cells.T[:130]
    k = oracle_mod.rate_coeffs(medium_net, T)
    f = N.rhs_k(_t(torch, k), _t(torch, y)).cpu().numpy()
    ref, ab = oracle_mod.rhs_k(medium_net, k, y, with_abs=True)
    _close(f, ref, ab)


def _jac_at_pattern(N, J):
    rp, col = N.jac_pattern()
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    return J[:, rows, col]


@pytest.mark.parametrize("which", ["tiny", "medium"])
def test_jacobian(acm, torch_dev, oracle_mod, tiny, medium_net, med_cells, which):
    torch = torch_dev
    if which == "tiny":
        net, y, T = tiny[0], tiny[1].y0, tiny[1].T
    else:
        net, y, T = medium_net, med_cells.y0[:67], med_cells.T[:67]
    N = acm.Network.from_synth(net)
    jv = N.jac(_t(torch, y), _t(torch, T)).cpu().numpy()
    J, ab = oracle_mod.jac_dense(net, y, T, with_abs=True)
    _close(jv, _jac_at_pattern(N, J), _jac_at_pattern(N, ab))


def test_vjp(acm, torch_dev, oracle_mod, medium_net, med_cells):
    torch = torch_dev
    net = medium_net
    n = 301
    y, T = med_cells.y0[:n], med_cells.T[:n]
    v = np.random.default_rng(4).standard_normal(y.shape)
    N = acm.Network.from_synth(net)
    gy, gl = N.vjp(_t(torch, y), _t(torch, T), _t(torch, v))
    gy, gl = gy.cpu().numpy(), gl.cpu().numpy()
    ref_gy, ref_gl = oracle_mod.vjp(net, y, T, v)
    _, abJ = oracle_mod.jac_dense(net, y, T, with_abs=True)
    scale_gy = np.einsum("ci,cia->ca", np.abs(v), abJ)
    _close(gy, ref_gy, scale_gy)
    # g_logalpha sums over cells: scale = sum_c |R_cj| sum_i |S_ij| |v_ci|
    S = np.abs(oracle_mod.stoich(net)).astype(np.float64)
    r = oracle_mod.rates(net, y, T)
    scale_gl = (np.abs(r) * (np.abs(v) @ S)).sum(0)
    _close(gl, ref_gl.sum(0), scale_gl)
    # bit-for-bit reproducible cell sum
    _, gl2 = N.vjp(_t(torch, y), _t(torch, T), _t(torch, v), want_gy=False)
    assert np.array_equal(gl, gl2.cpu().numpy())


def test_log_alpha_override(acm, torch_dev, oracle_mod, medium_net, med_cells):
    torch = torch_dev
    net = medium_net
    rng = np.random.default_rng(9)
    delta = rng.normal(0, 0.3, net.n_reactions)
    net2 = net.subset(np.arange(net.n_reactions))
    net2.alpha = net.alpha * np.exp(delta)
    N = acm.Network.from_synth(net)
    la = _t(torch, np.log(net.alpha) + delta)
    y, T = med_cells.y0[:50], med_cells.T[:50]
    f = N.rhs(_t(torch, y), _t(torch, T), log_alpha=la).cpu().numpy()
    ref, ab = oracle_mod.rhs(net2, y, T, with_abs=True)
    _close(f, ref, ab)
    jv = N.jac(_t(torch, y), _t(torch, T), log_alpha=la).cpu().numpy()
    J, abJ = oracle_mod.jac_dense(net2, y, T, with_abs=True)
    _close(jv, _jac_at_pattern(N, J), _jac_at_pattern(N, abJ))


def test_full_batch_sampled(acm, torch_dev, oracle_mod, medium_net):
    """65,536 cells in the launch configuration the benchmark times;
    sampled cells against the oracle, every output finite."""
    torch = torch_dev
    net = medium_net
    cells = synthnet.make_cells(net, 65536, synthnet.SEED_BASE + 1)
    N = acm.Network.from_synth(net, layout="sell", ordering="nnz")
    y, T = _t(torch, cells.y0), _t(torch, cells.T)
    f = N.rhs(y, T)
    jv = N.jac(y, T)
    idx = _sample(65536, 48)
    assert bool(torch.isfinite(f).all()) and bool(torch.isfinite(jv).all())
    ref, ab = oracle_mod.rhs(net, cells.y0[idx], cells.T[idx], with_abs=True)
    _close(f[torch.from_numpy(idx).cuda()].cpu().numpy(), ref, ab)
    J, abJ = oracle_mod.jac_dense(net, cells.y0[idx[:8]], cells.T[idx[:8]], with_abs=True)
    _close(jv[torch.from_numpy(idx[:8]).cuda()].cpu().numpy(), _jac_at_pattern(N, J),
           _jac_at_pattern(N, abJ))


def test_large_network(acm, torch_dev, oracle_mod):
    """700 species / 8000 reactions with grain-surface terms: the LDS block
    exceeds 64 KB per workgroup."""
    torch = torch_dev
    net, _ = synthnet.workload("large", n_cells=1)
    cells = synthnet.make_cells(net, 70, synthnet.SEED_BASE + 4)
    y, T = cells.y0, cells.T
    v = np.random.default_rng(1).standard_normal(y.shape)
    for layout in ("csr", "sell", "runs", "ccs"):
        N = acm.Network.from_synth(net, layout=layout, ordering="rcm")
        f = N.rhs(_t(torch, y), _t(torch, T)).cpu().numpy()
        ref, ab = oracle_mod.rhs(net, y, T, with_abs=True)
        _close(f, ref, ab)
    jv = N.jac(_t(torch, y[:9]), _t(torch, T[:9])).cpu().numpy()
    J, abJ = oracle_mod.jac_dense(net, y[:9], T[:9], with_abs=True)
    _close(jv, _jac_at_pattern(N, J), _jac_at_pattern(N, abJ))
    gy, gl = N.vjp(_t(torch, y[:9]), _t(torch, T[:9]), _t(torch, v[:9]))
    ref_gy, ref_gl = oracle_mod.vjp(net, y[:9], T[:9], v[:9])
    _close(gy.cpu().numpy(), ref_gy, np.einsum("ci,cia->ca", np.abs(v[:9]), abJ))


def test_one_cell_kernels_agree_across_workgroup_sizes(acm, torch_dev, oracle_mod):
    """700 / 8000 network (too large for two cells per pass): the one-cell
    RHS, Jacobian and VJP kernels give the same bits at 256, 512 and 1024
    threads and at the library's own choice (0): the workgroup size only
    changes which thread sums a chunk, not the order of any sum."""
    torch = torch_dev
    net, _ = synthnet.workload("large", n_cells=1)
    cells = synthnet.make_cells(net, 21, synthnet.SEED_BASE + 6)
    y, T = _t(torch, cells.y0), _t(torch, cells.T)
    v = _t(torch, np.random.default_rng(6).standard_normal(cells.y0.shape))
    outs = {}
    for layout in ("csr", "runs"):
        for blk in (256, 512, 1024, 0):
            N = acm.Network.from_synth(net, layout=layout, ordering="rcm", block=blk)
            gy, gl = N.vjp(y, T, v)
            outs[(layout, blk)] = (N.rhs(y, T), N.jac(y[:1], T[:1]), N.jac(y, T), gy, gl)
            N.close()
        ref = outs[(layout, 512)]
        for blk in (256, 1024, 0):
            for a, b in zip(outs[(layout, blk)], ref):
                assert torch.equal(a, b), (layout, blk)
    # and the shared result is the oracle's
    f = outs[("csr", 0)][0].cpu().numpy()
    ref, ab = oracle_mod.rhs(net, cells.y0, cells.T, with_abs=True)
    _close(f, ref, ab)


def test_edge_cases(acm, torch_dev, oracle_mod):
    torch = torch_dev
    # paper example plus a species that takes part in nothing (empty row)
    from conftest import network_from
    net = network_from([([0, 0], [1]), ([1], [0, 0])], [3.0, 5.0], 3)
    N = acm.Network(net.reactants, net.products, net.alpha, net.beta, net.gamma,
                    composition=np.zeros((3, 6), np.int8))
    y = np.array([[2.0, 7.0, 11.0]])
    for layout in ("csr", "sell", "coo", "runs", "ccs"):
        M = acm.Network(net.reactants, net.products, net.alpha, net.beta, net.gamma,
                        composition=np.zeros((3, 6), np.int8), layout=layout)
        f = M.rhs(_t(torch, y), _t(torch, [40.0])).cpu().numpy()
        # k = exp(ln alpha) is alpha to within an ulp or two
        np.testing.assert_allclose(f, [[-2 * 3 * 4 + 2 * 5 * 7, 3 * 4 - 5 * 7, 0.0]], rtol=1e-14)
        assert f[0, 2] == 0.0
    # zero cells: a no-op
    e = torch.empty((0, 3), dtype=torch.float64, device="cuda")
    N.rhs(e, torch.empty(0, dtype=torch.float64, device="cuda"))
    gy, gl = N.vjp(e, torch.empty(0, dtype=torch.float64, device="cuda"), e)
    assert gl.cpu().tolist() == [0.0, 0.0]
    # bad shapes are caught before any launch
    with pytest.raises(ValueError):
        N.rhs(_t(torch, np.zeros((2, 4))), _t(torch, [1.0, 2.0]))


def test_autotune_picks_a_working_configuration(acm, torch_dev, oracle_mod, medium_net, med_cells):
    """The autotuner times every candidate layout x ordering x block (SELL at
    one block size: its fused kernel ignores it) on the caller's cells and
    returns the fastest network, whose RHS and Jacobian still match the
    oracle; a second call with the same key reads the choice from the JSON
    cache."""
    import os
    import tempfile
    torch = torch_dev
    from paper_2312_04998_amd.autotune import autotune, candidates
    y, T = med_cells.y0[:256], med_cells.T[:256]
    with tempfile.TemporaryDirectory() as d:
        cache = os.path.join(d, "tune.json")
        N, kw, table = autotune(medium_net, _t(torch, y), _t(torch, T), reps=2, cache=cache)
        assert kw.pop("cached") is False
        assert len(table) == len(list(candidates())) == 3 + 4 * 3 * 3
        assert table[(kw["layout"], kw["ordering"], kw["block"])] == min(table.values())
        N2, kw2, table2 = autotune(medium_net, _t(torch, y), _t(torch, T), reps=2, cache=cache)
        assert kw2.pop("cached") is True and kw2 == kw and set(table2) == set(table)
        N2.close()
    f = N.rhs(_t(torch, y[:40]), _t(torch, T[:40])).cpu().numpy()
    ref, ab = oracle_mod.rhs(medium_net, y[:40], T[:40], with_abs=True)
    _close(f, ref, ab)
    jv = N.jac(_t(torch, y[:40]), _t(torch, T[:40])).cpu().numpy()
    J, abJ = oracle_mod.jac_dense(medium_net, y[:40], T[:40], with_abs=True)
    _close(jv, _jac_at_pattern(N, J), _jac_at_pattern(N, abJ))


def test_two_cell_kernels_independent_of_partner(acm, torch_dev, medium_net, med_cells):
    """The RHS, Jacobian and VJP run two cells per pass. A cell's values must
    not depend on which cell shares its pass, or on having none: cells 1..6
    computed in the passes (0,1),(2,3),(4,5),(6) and again in (1,2),(3,4),
    (5,6),(7) agree bit for bit, and the RHS equals the one-cell kernel's."""
    torch = torch_dev
    N = acm.Network.from_synth(medium_net)
    y, T = med_cells.y0[:8], med_cells.T[:8]
    v = np.random.default_rng(4).standard_normal(y.shape)
    a = (_t(torch, y[:7]), _t(torch, T[:7]), _t(torch, v[:7]))
    b = (_t(torch, y[1:8]), _t(torch, T[1:8]), _t(torch, v[1:8]))
    fa, fb = N.rhs(a[0], a[1]).cpu().numpy(), N.rhs(b[0], b[1]).cpu().numpy()
    assert np.array_equal(fa[1:7], fb[0:6])
    for c in (0, 6):
        one = N.rhs(_t(torch, y[c:c + 1]), _t(torch, T[c:c + 1])).cpu().numpy()
        assert np.array_equal(one[0], fa[c])
    ja, jb = N.jac(a[0], a[1]).cpu().numpy(), N.jac(b[0], b[1]).cpu().numpy()
    assert np.array_equal(ja[1:7], jb[0:6])
    ga, _ = N.vjp(*a)
    gb, _ = N.vjp(*b)
    assert np.array_equal(ga.cpu().numpy()[1:7], gb.cpu().numpy()[0:6])


@pytest.mark.parametrize("n_cells", [1, 2, 7, 64])
def test_rhs_jac_fused_equals_separate(acm, torch_dev, medium_net, med_cells, n_cells):
    """ac_rhs_jac (one kernel for both outputs with SELL) is bit-identical to
    ac_rhs followed by ac_jac, including a lone last cell and one cell."""
    torch = torch_dev
    for layout in ("sell", "csr"):
        N = acm.Network.from_synth(medium_net, layout=layout)
        y, T = _t(torch, med_cells.y0[:n_cells]), _t(torch, med_cells.T[:n_cells])
        d1 = torch.empty_like(y)
        j1 = torch.empty((n_cells, N.nnz_j), dtype=torch.float64, device="cuda")
        d2, j2 = torch.empty_like(d1), torch.empty_like(j1)
        acm.ac_rhs(N, None, y, T, d1)
        acm.ac_jac(N, None, y, T, j1)
        acm.ac_rhs_jac(N, None, y, T, d2, j2)
        assert torch.equal(d1, d2) and torch.equal(j1, j2), layout


def test_rhs_jac_fused_full_batch(acm, torch_dev, oracle_mod, medium_net):
    """The benchmarked call at the benchmarked size and configuration: one
    ac_rhs_jac over all 65,536 cells of the 470/4600 workload with the SELL
    layout in natural order, so every workgroup makes many passes and carries
    its LDS sentinels (the (1, 1) density pair and the (0, 0) slot pair)
    from pass to pass. Bit-identical to ac_rhs followed by ac_jac; 48
    sampled cells against the oracle."""
    torch = torch_dev
    net = medium_net
    C = 65536
    cells = synthnet.make_cells(net, C, synthnet.SEED_BASE + 1)
    N = acm.Network.from_synth(net, layout="sell", ordering="natural")
    y, T = _t(torch, cells.y0), _t(torch, cells.T)
    d2 = torch.empty_like(y)
    j2 = torch.empty((C, N.nnz_j), dtype=torch.float64, device="cuda")
    acm.ac_rhs_jac(N, None, y, T, d2, j2)
    d1 = torch.empty_like(y)
    acm.ac_rhs(N, None, y, T, d1)
    assert torch.equal(d1, d2)
    del d1
    j1 = torch.empty_like(j2)
    acm.ac_jac(N, None, y, T, j1)
    assert torch.equal(j1, j2)
    del j1
    idx = _sample(C, 48, seed=5)
    assert len(idx) >= 48
    ii = torch.from_numpy(idx).cuda()
    ref, ab = oracle_mod.rhs(net, cells.y0[idx], cells.T[idx], with_abs=True)
    _close(d2[ii].cpu().numpy(), ref, ab)
    jv = j2[ii].cpu().numpy()
    for s in range(0, len(idx), 16):
        sl = slice(s, s + 16)
        J, abJ = oracle_mod.jac_dense(net, cells.y0[idx[sl]], cells.T[idx[sl]], with_abs=True)
        _close(jv[sl], _jac_at_pattern(N, J), _jac_at_pattern(N, abJ))

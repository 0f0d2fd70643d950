"""GPU discrete adjoint (ac_integrate_adjoint) against the oracle's forward
sensitivities through the same recorded step sequence, against central
finite differences of the replayed map, and its edge cases.

For L = sum_c <lambda_c, y_c(t_end)> and any direction (dy0, dlogalpha) the
oracle's tangent s of the replayed map gives dL = <lambda, s>; the adjoint
gives dL = <dL/dy0, dy0> + <dL/dlogalpha, dlogalpha>. The two are the same
derivative of the same map, so they must agree to rtol 1e-6 of the terms'
absolute scale."""
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


def _t(a, dtype=np.float64):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype)).cuda()


def _adjoint_vs_tangents(acm, oracle_mod, net, y0, T, t_end, lam, n_dir, seed, cap=20000,
                         solver="auto"):
    """Oracle run (tape) -> GPU adjoint on that tape and oracle tangents on
    that tape; returns (gpu result dict as numpy, oracle replay y, tangents,
    directions)."""
    ref = oracle_mod.bdf(net, y0, T, t_end, tape_cap=cap)
    assert np.all(ref["status"] == 0) and np.all(ref["tape_len"] > 0)
    N = acm.Network.from_synth(net)
    ws = acm.Workspace(N, n_slots=4)
    out = ws.adjoint(_t(y0), _t(T), acm.tape_from_numpy(ref["tape"]), _t(ref["tape_len"], np.int32),
                     _t(lam), want_cells=True, want_y=True, linear_solver=solver)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    rng = np.random.default_rng(seed)
    n = y0.shape[0]
    dy0 = y0[:, None, :] * rng.standard_normal((n, n_dir, net.n_species))
    dla = rng.standard_normal((n_dir, net.n_reactions))
    y_rep, s = oracle_mod.bdf_replay(net, y0, T, ref["tape"], ref["tape_len"], dy0=dy0,
                                     dlogalpha=dla, n_dir=n_dir)
    return g, y_rep, s, dy0, dla


def _check_projection(g, s, lam, dy0, dla, rtol=1e-6):
    n, n_dir = dy0.shape[0], dy0.shape[1]
    worst = 0.0
    for c in range(n):
        for r in range(n_dir):
            lhs = float(np.dot(lam[c], s[c, r]))
            t_y = g["dL_dy0"][c] * dy0[c, r]
            t_p = g["g_cells"][c] * dla[r]
            rhs = float(t_y.sum() + t_p.sum())
            scale = float(np.abs(lam[c] * s[c, r]).sum() + np.abs(t_y).sum() + np.abs(t_p).sum())
            err = abs(lhs - rhs) / scale
            worst = max(worst, err)
            assert err <= rtol, (c, r, lhs, rhs, scale)
    print(f"worst projection error {worst:.2e} of the terms' scale")


def test_adjoint_matches_oracle_tangents_tiny(acm, oracle_mod):
    """50-species network, BDF 1-5 to 1e4 yr, three temperatures; the loss
    is the log of 8 seeded target abundances (lambda = 1/y_t)."""
    net, cells = synthnet.workload("tiny", n_cells=4)
    y0 = np.repeat(cells.y0[:1], 3, 0) * np.array([1.0, 0.3, 3.0])[:, None]
    T = np.array([15.0, 40.0, 100.0])
    t_end = 1e4 * YEAR_S
    ref = oracle_mod.bdf(net, y0, T, t_end)
    tgt = np.random.default_rng(8).choice(net.n_species, 8, replace=False)
    lam = np.zeros_like(y0)
    lam[:, tgt] = 1.0 / np.maximum(ref["y"][:, tgt], 1e-30)
    g, y_rep, s, dy0, dla = _adjoint_vs_tangents(acm, oracle_mod, net, y0, T, t_end, lam, 6, 1)
    assert g["status"].tolist() == [0, 0, 0]
    big = np.abs(y_rep) > 1e-20
    rel = np.abs(g["y_final"] - y_rep)[big] / np.abs(y_rep[big])
    print(f"replayed y: max rel diff {rel.max():.2e}")
    assert rel.max() <= 1e-6
    _check_projection(g, s, lam, dy0, dla)
    # the summed gradient is the cell-ordered sum of the rows
    np.testing.assert_allclose(g["dL_dlogalpha"], g["g_cells"].sum(0), rtol=1e-13,
                               atol=1e-13 * np.abs(g["g_cells"]).sum(0).max())


@pytest.mark.parametrize("solver", ["auto", "dense"])
def test_adjoint_matches_oracle_tangents_medium(acm, oracle_mod, medium, solver):
    """Paper-sized network (470 / 4600), one cell, 10 yr of BDF 1-5, with
    both Newton solves (the transposed solves of the reverse sweep go
    through the sparse front and its dense tail, or through one dense LU)."""
    net, cells = medium
    y0, T = cells.y0[:1], cells.T[:1]
    lam = np.random.default_rng(3).standard_normal(y0.shape) / np.maximum(y0, 1e-12)
    g, y_rep, s, dy0, dla = _adjoint_vs_tangents(acm, oracle_mod, net, y0, T, 10 * YEAR_S, lam, 2,
                                                 2, solver=solver)
    assert g["status"].tolist() == [0]
    _check_projection(g, s, lam, dy0, dla)


def test_adjoint_central_differences(acm, torch_dev):
    """Whole GPU pipeline (integrate with tape -> adjoint) against central
    differences (step 1e-6 in log alpha) of the replayed map on 32 random
    parameters; the bar allows the replay's own rounding noise, measured by
    rerunning with y0 perturbed by 1e-15 relative."""
    torch = torch_dev
    net, cells = synthnet.workload("tiny", n_cells=2)
    y0, T = cells.y0[:1], np.array([25.0])
    t_end = 1e4 * YEAR_S
    N = acm.Network.from_synth(net)
    ws = acm.Workspace(N, n_slots=2)
    la0 = np.log(net.alpha)
    y = _t(y0)
    res = ws.integrate(y, _t(T), t_end, log_alpha=_t(la0), tape_cap=20000)
    tape, tlen = res["tape"], res["tape_len"]
    assert int(res["status"][0]) == 0
    tgt = np.random.default_rng(5).choice(net.n_species, 8, replace=False)
    lam = np.zeros_like(y0)
    lam[0, tgt] = 1.0 / np.maximum(y.cpu().numpy()[0, tgt], 1e-30)

    def replay_L(la, yy=y0):
        o = ws.adjoint(_t(yy), _t(T), tape, tlen, _t(lam), log_alpha=_t(la), want_glog=False,
                       want_y=True)
        return float((o["y_final"].cpu().numpy() * lam).sum())

    adj = ws.adjoint(_t(y0), _t(T), tape, tlen, _t(lam), log_alpha=_t(la0))
    gl = adj["dL_dlogalpha"].cpu().numpy()
    L0 = replay_L(la0)
    noise = max(abs(replay_L(la0, y0 * (1 + 1e-15 * np.random.default_rng(k).standard_normal(y0.shape))) - L0)
                for k in range(3))
    eps = 1e-6
    params = np.random.default_rng(6).choice(net.n_reactions, 32, replace=False)
    worst = 0.0
    for j in params:
        e = np.zeros_like(la0)
        e[j] = eps
        fd = (replay_L(la0 + e) - replay_L(la0 - e)) / (2 * eps)
        bar = 1e-4 * abs(gl[j]) + 10 * (noise + 1e-15 * abs(L0)) / eps
        worst = max(worst, abs(fd - gl[j]) / max(bar, 1e-300))
        assert abs(fd - gl[j]) <= bar, (j, fd, gl[j], bar)
    print(f"worst |fd - adjoint| / bar = {worst:.3f}; L = {L0:.6e}, rounding noise {noise:.2e}")


def test_autograd_function(acm, torch_dev):
    """Integrate.apply: forward equals ac_integrate, backward equals a direct
    adjoint call on the forward's tape."""
    torch = torch_dev
    net, cells = synthnet.workload("tiny", n_cells=3)
    N = acm.Network.from_synth(net)
    ws = acm.Workspace(N, n_slots=3)
    t_end = 1e3 * YEAR_S
    la = _t(np.log(net.alpha)).requires_grad_(True)
    y0 = _t(cells.y0).requires_grad_(True)
    T = _t(cells.T)
    yT = acm.Integrate.apply(la, y0, T, ws, t_end, {"tape_cap": 20000})
    w = _t(np.random.default_rng(2).standard_normal(cells.y0.shape))
    (yT * w).sum().backward()
    y_ref = y0.detach().clone()
    res = ws.integrate(y_ref, T, t_end, log_alpha=la.detach(), tape_cap=20000)
    assert torch.equal(yT.detach(), y_ref)
    adj = ws.adjoint(y0.detach(), T, res["tape"], res["tape_len"], w, log_alpha=la.detach())
    assert torch.equal(la.grad, adj["dL_dlogalpha"])
    assert torch.equal(y0.grad, adj["dL_dy0"])


def test_adjoint_reproducible(acm, oracle_mod):
    """Two adjoint runs over 6 cells on 2 slots give bitwise equal results
    (the cell sum does not depend on which workgroup took which cell)."""
    net, cells = synthnet.workload("tiny", n_cells=6)
    t_end = 1e3 * YEAR_S
    ref = oracle_mod.bdf(net, cells.y0, cells.T, t_end, tape_cap=5000)
    N = acm.Network.from_synth(net)
    ws = acm.Workspace(N, n_slots=2)
    lam = np.random.default_rng(4).standard_normal(cells.y0.shape)
    args = (_t(cells.y0), _t(cells.T), acm.tape_from_numpy(ref["tape"]),
            _t(ref["tape_len"], np.int32), _t(lam))
    a = ws.adjoint(*args)
    b = ws.adjoint(*args)
    import torch
    assert torch.equal(a["dL_dlogalpha"], b["dL_dlogalpha"])
    assert torch.equal(a["dL_dy0"], b["dL_dy0"])


def test_adjoint_edge_cases(acm, oracle_mod):
    """Bad input, an empty tape (t_end = 0), an overflowed tape and a tape
    with an invalid order: dL/dy0 = lambda, no parameter terms, and the
    status says why."""
    net, cells = synthnet.workload("tiny", n_cells=4)
    t_end = 1e2 * YEAR_S
    y0, T = cells.y0.copy(), cells.T.copy()
    ref = oracle_mod.bdf(net, y0, T, t_end, tape_cap=2000)
    tape, tlen = ref["tape"].copy(), ref["tape_len"].copy()
    T_in = T.copy()
    T_in[0] = -5.0                       # bad input
    tlen[1] = 0                          # nothing recorded
    tlen[2] = -1                         # overflowed
    steps = np.flatnonzero(tape[3]["type"] == 3)
    tape[3]["q"][steps[0]] = 9           # malformed order
    lam = np.random.default_rng(7).standard_normal(y0.shape)
    N = acm.Network.from_synth(net)
    ws = acm.Workspace(N, n_slots=2)
    out = ws.adjoint(_t(y0), _t(T_in), acm.tape_from_numpy(tape), _t(tlen, np.int32), _t(lam),
                     want_cells=True, want_y=True)
    st = out["status"].cpu().numpy().tolist()
    assert st == [acm.AC_CELL_BADINPUT, 0, acm.AC_CELL_TAPE, acm.AC_CELL_TAPE]
    np.testing.assert_array_equal(out["dL_dy0"].cpu().numpy(), lam)
    np.testing.assert_array_equal(out["g_cells"].cpu().numpy(), 0.0)
    np.testing.assert_array_equal(out["y_final"].cpu().numpy()[1], y0[1])


@pytest.mark.parametrize("which", ["tiny", "medium"])
def test_adjoint_kept_states_equal_recomputed(acm, oracle_mod, which):
    """Keeping every converged state of the forward replay (the default) and
    recomputing each 64-step segment from its checkpoint give bitwise equal
    gradients, final states and statuses; only the replay counters differ
    (the kept-state run does one replay per step). Tapes long enough for
    several segments."""
    import torch
    if which == "tiny":
        net, cells = synthnet.workload("tiny", n_cells=5)
        t_end, n, K = 1e5 * YEAR_S, 5, 100000
    else:
        net, cells = synthnet.workload("medium", n_cells=6)
        t_end, n, K = 1e6 * YEAR_S, 6, 200
    ref = oracle_mod.bdf(net, cells.y0[:n], cells.T[:n], t_end, max_steps=K, tape_cap=4096)
    assert int(ref["tape_len"].max()) > 3 * 64
    N = acm.Network.from_synth(net)
    ws = acm.Workspace(N, n_slots=3)
    lam = np.random.default_rng(11).standard_normal(cells.y0[:n].shape)
    args = (_t(cells.y0[:n]), _t(cells.T[:n]), acm.tape_from_numpy(ref["tape"]),
            _t(ref["tape_len"], np.int32), _t(lam))
    a = ws.adjoint(*args, want_cells=True, want_y=True)
    b = ws.adjoint(*args, want_cells=True, want_y=True, recompute=True)
    c = ws.adjoint(*args, want_cells=True, want_y=True)
    for k in ("dL_dy0", "g_cells", "dL_dlogalpha", "y_final", "status"):
        assert torch.equal(a[k], b[k]), k
        assert torch.equal(a[k], c[k]), k
    sa, sb = a["stats"].cpu().numpy(), b["stats"].cpu().numpy()
    assert np.array_equal(sa[:, 0], sb[:, 0])          # steps reversed
    assert (sa[:, 3] < sb[:, 3]).all()                  # fewer replay Newton iterations


def test_adjoint_gradient_rows_in_workspace_and_checkpoint_interval(acm, oracle_mod):
    """The summed dL/dlog alpha from the workspace's own rows (no per-cell
    buffer; 5 cells in chunks of 2) equals the sum of the caller's per-cell
    rows bit for bit. With checkpoints every 16 steps the segments recomputed
    from their checkpoints equal the kept states bit for bit; against
    checkpoints every 64 they differ only by where the Newton matrix is
    rebuilt (each segment starts with a fresh one), far below the parity
    bar."""
    import torch
    net, cells = synthnet.workload("tiny", n_cells=5)
    t_end = 1e4 * YEAR_S
    ref = oracle_mod.bdf(net, cells.y0, cells.T, t_end, tape_cap=8000)
    N = acm.Network.from_synth(net)
    lam = np.random.default_rng(31).standard_normal(cells.y0.shape)
    args = (_t(cells.y0), _t(cells.T), acm.tape_from_numpy(ref["tape"]),
            _t(ref["tape_len"], np.int32), _t(lam))
    ws_a = acm.Workspace(N, n_slots=2)
    a = ws_a.adjoint(*args, want_cells=True)
    ws_b = acm.Workspace(N, n_slots=2, adj_max_tape=8000, adj_max_cells=2)
    b = ws_b.adjoint(*args)
    assert "g_cells" not in b
    assert torch.equal(a["dL_dlogalpha"], b["dL_dlogalpha"]) and torch.equal(a["dL_dy0"], b["dL_dy0"])
    ws_c = acm.Workspace(N, n_slots=2, adj_max_tape=8000, checkpoint_every=16)
    c = ws_c.adjoint(*args, want_cells=True, recompute=True, checkpoint_every=16)
    ws_d = acm.Workspace(N, n_slots=2, adj_max_tape=8000, checkpoint_every=16, keep_states=True)
    d = ws_d.adjoint(*args, want_cells=True, checkpoint_every=16)
    for k in ("dL_dy0", "g_cells", "dL_dlogalpha"):
        assert torch.equal(c[k], d[k]), k
        ga, gc = a[k].cpu().numpy(), c[k].cpu().numpy()
        scale = np.abs(ga).max(axis=-1, keepdims=True)
        worst = float((np.abs(gc - ga) / scale).max())
        print(f"{k}: every 16 vs every 64, worst {worst:.2e} of the row's largest entry")
        assert worst <= 1e-8, k


def test_adjoint_refuses_without_reservation(acm, oracle_mod):
    """ac_integrate_adjoint allocates nothing: a tape longer than the
    workspace's reservation, or a different checkpoint interval, is refused
    with AC_ECAPACITY before any launch."""
    import ctypes as C
    net, cells = synthnet.workload("tiny", n_cells=2)
    ref = oracle_mod.bdf(net, cells.y0, cells.T, 1e3 * YEAR_S, tape_cap=4000)
    N = acm.Network.from_synth(net)
    ws = acm.Workspace(N, n_slots=2, adj_max_tape=100)
    tape = acm.tape_from_numpy(ref["tape"])
    tl = _t(ref["tape_len"], np.int32)
    y0, T, lam = _t(cells.y0), _t(cells.T), _t(np.ones_like(cells.y0))
    gy = _t(np.zeros_like(cells.y0))
    for cap, every in ((4000, 0), (100, 32)):
        o = acm.IntegOpts(1e-6, 1e-20, 0.0, 5, 1, 0, every, 0.0)
        st = acm.lib.ac_integrate_adjoint(ws.handle, None, 2, y0.data_ptr(), T.data_ptr(),
                                          C.byref(o), tape.data_ptr(), cap, tl.data_ptr(),
                                          lam.data_ptr(), None, gy.data_ptr(), None, None, None,
                                          None, None)
        assert st == acm.AC_ECAPACITY, (cap, every, acm.last_error())


def test_newton_tolerance_option(acm, oracle_mod):
    """A looser corrector tolerance, passed to both sides, still gives the
    oracle's step counts (within 2 % + 3) and results within its rerun
    envelope."""
    from test_gpu_integrate import _agree, oracle_with_envelope
    net, cells = synthnet.workload("tiny", n_cells=3)
    N = acm.Network.from_synth(net)
    ws = acm.Workspace(N, n_slots=3)
    y = _t(cells.y0)
    out = ws.integrate(y, _t(cells.T), 1e4 * YEAR_S, newton_tol=1e-2)
    ref, env, _ = oracle_with_envelope(oracle_mod, net, cells.y0, cells.T, 1e4 * YEAR_S, k=8,
                                       newton_tol=1e-2)
    st = out["stats"].cpu().numpy()
    assert out["status"].cpu().tolist() == ref["status"].tolist() == [0, 0, 0]
    assert np.all(np.abs(st[:, 0] - ref["stats"][:, 0]) <= 0.02 * ref["stats"][:, 0] + 3)
    assert _agree(y.cpu().numpy(), ref["y"], envelope=env).all()

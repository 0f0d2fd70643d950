"""GPU parity of the batched dense LU (Newton matrices) and of the batched
BDF integrator against the oracle, through the C ABI.

Integrated densities must agree to rtol 1e-6 above a 1e-20 floor; the two
sides implement the same step, order and Newton rules, so the step
sequences themselves are compared too."""
import numpy as np
import pytest

import synthnet
from conftest import YEAR_S, network_from

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


def _t(torch, a, dtype=None):
    import torch as th
    return th.from_numpy(np.ascontiguousarray(a, np.float64 if dtype is None else dtype)).cuda()


# ------------------------------------------------------------------ LU

@pytest.mark.parametrize("n", [1, 5, 16, 33, 48, 64, 65, 80, 100, 129, 200, 470, 513, 700, 1024])
def test_lu_matches_oracle(acm, torch_dev, oracle_mod, n):
    torch = torch_dev
    rng = np.random.default_rng(n)
    nmat, lda = 3, n + (3 if n % 2 else 0)
    A = rng.standard_normal((nmat, n, n)) + np.eye(n) * rng.uniform(0, 3)
    Ad = np.zeros((nmat, n, lda))
    Ad[:, :, :n] = A
    dA = _t(torch, Ad)
    piv = torch.empty((nmat, n), dtype=torch.int32, device="cuda")
    info = torch.empty(nmat, dtype=torch.int32, device="cuda")
    acm.ac_lu_factor(dA, piv, info)
    LU = dA.cpu().numpy()[:, :, :n]
    pv = piv.cpu().numpy()
    assert info.cpu().tolist() == [0] * nmat
    for m in range(nmat):
        LUo, pvo, _ = oracle_mod.lu_factor(A[m])
        assert pv[m].tolist() == pvo.tolist()
        np.testing.assert_allclose(LU[m], LUo, rtol=1e-9, atol=1e-11 * np.abs(LUo).max())
    b = rng.standard_normal((nmat, n))
    for trans in (False, True):
        x = _t(torch, b)
        acm.ac_lu_solve(dA, piv, x, trans=trans)
        ref = np.stack([np.linalg.solve(A[m].T if trans else A[m], b[m]) for m in range(nmat)])
        np.testing.assert_allclose(x.cpu().numpy(), ref, rtol=1e-8, atol=1e-10)


def test_lu_newton_matrices(acm, torch_dev, oracle_mod, medium):
    """I - c J of the paper-sized network across the integrator's range of c."""
    torch = torch_dev
    net, cells = medium
    J = oracle_mod.jac_dense(net, cells.y0[:1], cells.T[:1])[0]
    n = J.shape[0]
    cs = [1e-3, 1e4, 1e10]
    A = np.stack([np.eye(n) - c * J for c in cs])
    dA = _t(torch, A)
    piv = torch.empty((len(cs), n), dtype=torch.int32, device="cuda")
    acm.ac_lu_factor(dA, piv)
    rng = np.random.default_rng(0)
    b = rng.standard_normal((len(cs), n))
    for trans in (False, True):
        x = _t(torch, b)
        acm.ac_lu_solve(dA, piv, x, trans=trans)
        x = x.cpu().numpy()
        for m in range(len(cs)):
            M = A[m].T if trans else A[m]
            r = M @ x[m] - b[m]
            assert np.linalg.norm(r) <= 1e-10 * (np.linalg.norm(M, 1) * np.linalg.norm(x[m]) +
                                                 np.linalg.norm(b[m]))


def test_lu_singular(acm, torch_dev):
    torch = torch_dev
    A = np.zeros((1, 4, 4))
    A[0] = [[1, 2, 3, 4], [2, 4, 6, 8], [0, 0, 0, 0], [1, 0, 1, 0]]
    dA = _t(torch, A)
    piv = torch.empty((1, 4), dtype=torch.int32, device="cuda")
    info = torch.empty(1, dtype=torch.int32, device="cuda")
    acm.ac_lu_factor(dA, piv, info)
    assert int(info.cpu()[0]) > 0


# ------------------------------------------------------------ integrator

def _agree(y_gpu, y_ora, rtol=1e-6, floor=1e-20, envelope=None):
    """|y_gpu - y_ora| <= rtol |y_ora| or both below the floor. Where the
    oracle does not reproduce itself to that level (envelope: its spread
    under 1e-15 relative perturbations of y0), the bound is 10 x envelope."""
    tol = rtol * np.abs(y_ora)
    if envelope is not None:
        tol = np.maximum(tol, 10.0 * envelope)
    return (np.abs(y_gpu - y_ora) <= tol) | (np.maximum(np.abs(y_gpu), np.abs(y_ora)) < floor)


def oracle_with_envelope(oracle_mod, net, y0, T, t_end, k=8, **kw):
    """Oracle run plus the spread of k reruns with y0 perturbed by 1e-15 and
    the rate prefactors alpha by 1e-14 relative: the trajectory's own
    sensitivity to rounding of the size by which the two sides' rate
    coefficients differ (exp of a sum against the product of a power and
    an exp, up to ~100 ulp). The k + 1 oracle calls run concurrently (each
    releases the interpreter lock while it integrates)."""
    import concurrent.futures as cf
    import dataclasses
    y0 = np.atleast_2d(y0)
    T = np.atleast_1d(T)
    rng = np.random.default_rng(12345)
    jobs = [(net, y0)]
    for _ in range(k):
        pnet = dataclasses.replace(net, alpha=net.alpha * (1 + 1e-14 * rng.standard_normal(net.alpha.shape)))
        jobs.append((pnet, y0 * (1 + 1e-15 * rng.standard_normal(y0.shape))))
    with cf.ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        outs = list(ex.map(lambda j: oracle_mod.bdf(j[0], j[1], T, t_end, **kw), jobs))
    ref = outs[0]
    ys = np.stack([o["y"] for o in outs])
    steps = np.stack([o["stats"][:, 0] for o in outs])
    env = np.abs(ys[1:] - ys[0]).max(0)
    return ref, env, steps


def _run(acm, torch, net, y0, T, t_end, ws=None, **kw):
    N = acm.Network.from_synth(net)
    ws = ws or acm.Workspace(N)
    y = _t(torch, y0)
    out = ws.integrate(y, _t(torch, T), t_end, **kw)
    return y.cpu().numpy(), {k: v.cpu().numpy() for k, v in out.items() if k != "tape"}, out


@pytest.mark.parametrize("q_max,years", [(1, 1e5), (5, 1e6)])
def test_tiny_network_parity(acm, torch_dev, oracle_mod, tiny, q_max, years):
    """The 50-species network: backward Euler to 1e5 yr (one cell at T = 20 K,
    n_H = 1e4, as the paper-style plain configuration) and BDF 1-5 to 1e6 yr
    over a spread of temperatures."""
    torch = torch_dev
    net, cells = tiny
    if q_max == 1:
        y0, T = cells.y0[:1], cells.T[:1]
    else:
        y0 = np.repeat(cells.y0[:1], 6, 0) * np.array([1, 1, 0.1, 10, 1, 1])[:, None]
        T = np.array([10.0, 20.0, 35.0, 60.0, 150.0, 300.0])
    t_end = years * YEAR_S
    y, out, _ = _run(acm, torch, net, y0, T, t_end, q_max=q_max)
    ref, env, steps = oracle_with_envelope(oracle_mod, net, y0, T, t_end, k=32, q_max=q_max)
    assert out["status"].tolist() == ref["status"].tolist() == [0] * len(T)
    ok = _agree(y, ref["y"], envelope=env)
    assert ok.all(), np.argwhere(~ok)[:5]
    strict = _agree(y, ref["y"])
    print(f"strict 1e-6 bar met by {strict.mean():.4f} of species-cells")
    # Step counts: rounding-level differences flip single accept/reject and
    # matrix-reuse decisions, so the oracle's own count moves by up to ~1 %
    # under 1e-15 relative perturbations of y0. The GPU count must fall in
    # the range 32 perturbed oracle runs span, widened by half that spread
    # (a finite sample underestimates the range), at least one step.
    g, o = out["stats"][:, 0], ref["stats"][:, 0]
    print("steps gpu", g.tolist(), "oracle", o.tolist(), "perturbed range",
          steps.min(0).tolist(), steps.max(0).tolist())
    assert np.all(np.abs(g - o) <= 0.01 * o + 3)
    lo, hi = steps.min(0), steps.max(0)
    slack = np.maximum(1, (hi - lo) // 2)
    assert np.all((g >= lo - slack) & (g <= hi + slack))


# Floor for the fraction of species-cells that meet the strict bar in a
# free-running integration of the paper-sized network (the rest must lie
# within 10x the oracle's own rerun spread). The strict bar itself is met
# element by element when both sides follow one step sequence
# (test_gpu_strict.py).
STRICT_FLOOR_MEDIUM = 0.95


MEDIUM_IDX = [0, 5, 9]


@pytest.fixture(scope="module")
def medium_ref(oracle_mod, medium):
    net, cells = medium
    return oracle_with_envelope(oracle_mod, net, cells.y0[MEDIUM_IDX], cells.T[MEDIUM_IDX],
                                1e6 * YEAR_S, k=8)


@pytest.mark.parametrize("solver", ["auto", "dense"])
def test_medium_network_parity(acm, torch_dev, medium, medium_ref, solver):
    """Paper-sized network (470 species / 4600 reactions), BDF 1-5 to 1e6 yr,
    free running on both sides; 8 perturbed oracle reruns set the envelope.
    Both Newton solves: the sparse front with a dense Schur tail (auto) and
    one pivoted LU of the whole matrix (dense)."""
    torch = torch_dev
    net, cells = medium
    idx = MEDIUM_IDX
    y0, T = cells.y0[idx], cells.T[idx]
    t_end = 1e6 * YEAR_S
    y, out, _ = _run(acm, torch, net, y0, T, t_end, linear_solver=solver)
    ref, env, steps = medium_ref
    assert out["status"].tolist() == ref["status"].tolist() == [0] * len(idx)
    bad = ~_agree(y, ref["y"], envelope=env)
    assert not bad.any(), (np.argwhere(bad)[:5], out["stats"], ref["stats"])
    strict = _agree(y, ref["y"])
    only_env = np.argwhere(~strict)
    names = [f"cell {idx[c]}: {net.names[i]} (gpu {y[c, i]:.6e}, oracle {ref['y'][c, i]:.6e}, "
             f"spread {env[c, i]:.1e})" for c, i in only_env[:20]]
    print(f"strict 1e-6 bar met by {strict.mean():.4f} of species-cells; "
          f"{len(only_env)} pass only through the envelope:", *names, sep="\n  ")
    print("steps gpu", out["stats"][:, 0].tolist(), "oracle reruns", steps.T.tolist())
    assert strict.mean() >= STRICT_FLOOR_MEDIUM
    assert np.all(np.abs(out["stats"][:, 0] - ref["stats"][:, 0]) <= 0.02 * ref["stats"][:, 0] + 3)
    E = net.composition.astype(np.float64).T
    drift = np.abs(y @ E.T - y0 @ E.T) / (y0 @ np.abs(E).T)
    assert drift.max() < 1e-7


def test_large_network_parity(acm, torch_dev, oracle_mod):
    """700 species / 8000 reactions with grain-surface terms: the Newton
    matrix has more rows than the workgroup has threads (two panel rows per
    thread) and the LDS working set exceeds 64 KB. One cell, 100 yr."""
    torch = torch_dev
    net, _ = synthnet.workload("large", n_cells=1)
    cells = synthnet.make_cells(net, 2, synthnet.SEED_BASE + 4)
    y0, T = cells.y0[:1], cells.T[:1]
    t_end = 1e2 * YEAR_S
    y, out, _ = _run(acm, torch, net, y0, T, t_end)
    ref, env, steps = oracle_with_envelope(oracle_mod, net, y0, T, t_end, k=8)
    assert out["status"].tolist() == ref["status"].tolist() == [0]
    ok = _agree(y, ref["y"], envelope=env)
    assert ok.all(), np.argwhere(~ok)[:5]
    print("steps gpu", out["stats"][:, 0].tolist(), "oracle", steps[:, 0].tolist())


def test_queue_more_cells_than_slots(acm, torch_dev, oracle_mod, tiny):
    """13 cells on 3 persistent workgroups; plain per-cell launches agree bit for bit."""
    torch = torch_dev
    net, cells = tiny
    rng = np.random.default_rng(3)
    y0 = np.repeat(cells.y0[:1], 13, 0) * rng.uniform(0.5, 2.0, (13, 1))
    T = np.exp(rng.uniform(np.log(10), np.log(300), 13))
    N = acm.Network.from_synth(net)
    ws = acm.Workspace(N, n_slots=3)
    assert ws.n_slots == 3
    t_end = 1e4 * YEAR_S
    y1 = _t(torch, y0)
    o1 = ws.integrate(y1, _t(torch, T), t_end)
    y2 = _t(torch, y0)
    o2 = ws.integrate(y2, _t(torch, T), t_end, plain=True)
    assert torch.equal(y1, y2) and torch.equal(o1["stats"], o2["stats"])
    ref, env, steps = oracle_with_envelope(oracle_mod, net, y0, T, t_end, k=8)
    ok = _agree(y1.cpu().numpy(), ref["y"], envelope=env)
    bad = np.argwhere(~ok)
    assert ok.all(), (bad[:5], o1["stats"][bad[:1, 0]].tolist(), steps[:, bad[:1, 0]].T.tolist())


def test_cell_order_does_not_change_results(acm, torch_dev, tiny):
    """The workgroups taking 29 cells in a shuffled order (3 slots) give the
    same y, status and statistics bit for bit as index order; the progress
    word ends at (about) the cell count; a malformed order is refused."""
    torch = torch_dev
    net, cells = tiny
    rng = np.random.default_rng(11)
    n = 29
    y0 = np.repeat(cells.y0[:1], n, 0) * rng.uniform(0.5, 2.0, (n, 1))
    T = np.exp(rng.uniform(np.log(10), np.log(300), n))
    N = acm.Network.from_synth(net)
    ws = acm.Workspace(N, n_slots=3)
    t_end = 1e4 * YEAR_S
    y1, y2 = _t(torch, y0), _t(torch, y0)
    o1 = ws.integrate(y1, _t(torch, T), t_end)
    perm = torch.from_numpy(rng.permutation(n).astype(np.int32)).cuda()
    o2 = ws.integrate(y2, _t(torch, T), t_end, cell_order=perm)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2) and torch.equal(o1["status"], o2["status"])
    assert torch.equal(o1["stats"], o2["stats"])
    assert n - ws.n_slots < ws.progress() <= n    # workgroups report in taking order, roughly
    with pytest.raises(ValueError):
        ws.integrate(y2, _t(torch, T), t_end, cell_order=perm.to(torch.int64))


def test_status_codes(acm, torch_dev, tiny):
    torch = torch_dev
    net, cells = tiny
    y0 = np.repeat(cells.y0[:1], 5, 0)
    y0[1, 3] = np.nan
    y0[2, 4] = -1.0
    T = np.array([20.0, 20.0, 20.0, 0.0, -4.0])
    y, out, _ = _run(acm, torch, net, y0, T, 1e3 * YEAR_S)
    assert out["status"].tolist() == [0, 3, 3, 3, 3]
    assert np.array_equal(y[1:], y0[1:], equal_nan=True)
    y, out, _ = _run(acm, torch, net, y0[:1], T[:1], 1e3 * YEAR_S, max_steps=3)
    assert out["status"].tolist() == [1] and out["stats"][0, 0] == 3
    # a finite-time blow-up stops before t_end with one of the failure
    # codes: which rejection comes last as h shrinks towards the pole (the
    # error test, a corrector that stops converging, an overflowing RHS)
    # turns on rounding, so the code is not unique; an unreachable accuracy
    # gives only error-test rejections, hence h_min
    blow = network_from([([0, 0], [0, 0, 0])], [1e-6], 1)
    y, out, _ = _run(acm, torch, blow, [[1.0]], [300.0], 1e7)
    print("blow-up status", out["status"].tolist(), "steps", out["stats"][0].tolist())
    assert out["status"].tolist()[0] in (acm.AC_CELL_NEWTON_FAIL, acm.AC_CELL_HMIN,
                                         acm.AC_CELL_NONFINITE)
    y, out, _ = _run(acm, torch, net, y0[:1], T[:1], 1e3 * YEAR_S, rtol=1e-30, atol=0.0)
    assert out["status"].tolist() == [acm.AC_CELL_HMIN]
    y, out, _ = _run(acm, torch, net, y0[:1], T[:1], 0.0)
    assert out["status"].tolist() == [0] and np.array_equal(y, y0[:1])


def _tape_compare(a_tape, a_len, b_tape, b_len):
    """(length difference, decision-prefix fraction, median and 95% quantile
    of the relative value differences over the common decision prefix)."""
    m = min(a_len, b_len)
    a, b = a_tape[:m], b_tape[:m]
    same = (a["type"] == b["type"]) & (a["q"] == b["q"])
    prefix = m if same.all() else int(np.argmin(same))
    rel = np.abs(a["val"][:prefix] - b["val"][:prefix]) / np.abs(b["val"][:prefix])
    return abs(a_len - b_len), prefix / m, np.median(rel), np.quantile(rel, 0.95)


@pytest.mark.parametrize("which", ["tiny", "medium"])
def test_recorded_tape_matches_oracle(acm, torch_dev, oracle_mod, tiny, medium_net, which):
    """The recorded step sequence (used by replay and the adjoint) carries the
    oracle's decisions and values to within the oracle's own sensitivity:
    each statistic of the GPU tape against the oracle's is bounded by the
    worst that 8 oracle reruns with y0 perturbed by 1e-15 and alpha by 1e-14
    relative show. The 50-species network to 1e5 yr, and the paper-sized
    network (first 2 cells of the 16,384-cell workload) to 1e6 yr."""
    import concurrent.futures as cf
    import dataclasses
    torch = torch_dev
    if which == "tiny":
        net, cells = tiny
        y0, T = cells.y0[:2], np.array([20.0, 90.0])
        t_end, cap = 1e5 * YEAR_S, 20000
    else:
        net = medium_net
        cells = synthnet.make_cells(net, 16384, synthnet.SEED_BASE + 2)
        y0, T = cells.y0[:2].copy(), cells.T[:2].copy()
        t_end, cap = 1e6 * YEAR_S, 40000
    _, out, raw = _run(acm, torch, net, y0, T, t_end, tape_cap=cap)
    tape = acm.tape_to_numpy(raw["tape"])
    rng = np.random.default_rng(99)
    jobs = [(net, y0)]
    for _ in range(8):
        pnet = dataclasses.replace(net, alpha=net.alpha * (1 + 1e-14 * rng.standard_normal(net.alpha.shape)))
        jobs.append((pnet, y0 * (1 + 1e-15 * rng.standard_normal(y0.shape))))
    with cf.ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        runs = list(ex.map(lambda j: oracle_mod.bdf(j[0], j[1], T, t_end, tape_cap=cap), jobs))
    ref, pert = runs[0], runs[1:]
    for c in range(2):
        Lo = int(ref["tape_len"][c])
        assert Lo > 0 and int(out["tape_len"][c]) > 0
        g = _tape_compare(tape[c], int(out["tape_len"][c]), ref["tape"][c], Lo)
        p = np.array([_tape_compare(o["tape"][c], int(o["tape_len"][c]), ref["tape"][c], Lo)[:4]
                      for o in pert])
        print(f"{which} cell {c}: events gpu {int(out['tape_len'][c])} oracle {Lo}; gpu dlen {g[0]} "
              f"prefix {g[1]:.3f} median {g[2]:.2e} q95 {g[3]:.2e};",
              f"perturbed worst dlen {p[:, 0].max():.0f} prefix {p[:, 1].min():.3f}",
              f"median {p[:, 2].max():.2e} q95 {p[:, 3].max():.2e}")
        assert g[0] <= p[:, 0].max() + 1
        assert g[1] >= 0.5 * p[:, 1].min()
        assert g[2] <= max(10 * p[:, 2].max(), 1e-7)
        assert g[3] <= max(3 * p[:, 3].max(), 1e-3)
        # the first event (the initial step size) is rounding-stable
        np.testing.assert_allclose(tape[c]["val"][:1], ref["tape"][c]["val"][:1], rtol=1e-9)


@pytest.mark.parametrize("solver", ["auto", "dense"])
def test_newton_solve_backward_error(acm, torch_dev, oracle_mod, medium, solver):
    """The integrator's Newton solve on its own (ac_newton_solve), on the
    oracle's Jacobians of five cells of the paper-sized network at c from
    1e-2 to 3e13 s, plain and transposed, five matrices over four slots (a
    slot factors twice): the normwise backward error against the same
    matrices, |M x - b|_2 / (|M|_1 |x|_1 + |b|_1), stays below 1e-14 (CPU
    studies of both algorithms give at most 5e-18; the matrix itself is
    rounded differently, I - cJ in one fused step on the GPU) for the
    sparse front with its dense tail (auto) and for one pivoted LU (dense),
    and the solution agrees with numpy where M is well conditioned."""
    torch = torch_dev
    net, cells = medium
    N = acm.Network.from_synth(net)
    ws = acm.Workspace(N, n_slots=4)
    idx = [0, 3, 7, 11, 13]
    cs = np.array([1e-2, 1e3, 1e7, 1e11, 3e13])
    J = oracle_mod.jac_dense(net, cells.y0[idx], cells.T[idx])
    rp, col = N.jac_pattern()
    rows = np.repeat(np.arange(N.n_species), np.diff(rp))
    jv = _t(torch, J[:, rows, col])
    b = np.random.default_rng(17).standard_normal((len(idx), N.n_species))
    worst = 0.0
    for trans in (False, True):
        x = _t(torch, b)
        info = ws.newton_solve(jv, _t(torch, cs), x, trans=trans, linear_solver=solver)
        assert info.cpu().tolist() == [0] * len(idx)
        x = x.cpu().numpy()
        for m in range(len(idx)):
            A = np.eye(N.n_species) - cs[m] * J[m]
            A = A.T if trans else A
            be = np.linalg.norm(A @ x[m] - b[m]) / (np.abs(A).sum(0).max() * np.abs(x[m]).sum()
                                                    + np.abs(b[m]).sum())
            assert be < 1e-14, (trans, m, be)
            worst = max(worst, be)
            if cs[m] <= 1e7:
                ref = np.linalg.solve(A, b[m])
                np.testing.assert_allclose(x[m], ref, rtol=0, atol=1e-9 * np.abs(ref).max())
    print(f"{solver}: largest backward error {worst:.2e}")
    # empty batch and bad shapes
    e = torch.empty((0, N.n_species), dtype=torch.float64, device="cuda")
    ws.newton_solve(torch.empty((0, N.nnz_j), dtype=torch.float64, device="cuda"),
                    torch.empty(0, dtype=torch.float64, device="cuda"), e)
    with pytest.raises(ValueError):
        ws.newton_solve(jv[:2], _t(torch, cs[:3]), _t(torch, b[:2]))

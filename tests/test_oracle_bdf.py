"""Pins of the oracle's stiff integrator: closed-form solutions, a library
integrator and matrix exponential, conservation laws and failure handling.

The paper names its integrator (DLSODES, Sec. 3) but prints no step
sequence, so the integrator is pinned through what any correct BDF must
reproduce rather than through printed values."""
import numpy as np
import pytest
import scipy.integrate
import scipy.linalg

import synthnet
from conftest import YEAR_S, network_from


def _final(oracle_mod, net, y0, T, t_end, **kw):
    out = oracle_mod.bdf(net, np.atleast_2d(y0), np.atleast_1d(T), t_end, **kw)
    assert np.all(out["status"] == oracle_mod.OK), out["status"]
    return out


# Local error control does not bound the global error by rtol itself: over
# many time constants a BDF run accumulates errors of order 100 rtol (SciPy's
# own BDF shows 6e-5 at rtol 1e-6 on the linear network below). A bound of
# 300 rtol still catches any wrong coefficient, sign or dropped term, which
# give O(1) errors; the convergence test checks the error shrinks with rtol.
GLOBAL = 300.0


def test_first_order_decay(oracle_mod):
    """A -> B: n_A = n_A0 exp(-k t), n_B = n_A0 - n_A."""
    k = 1e-9
    net = network_from([([0], [1])], [k], 2)
    t = 3.0 / k
    out = _final(oracle_mod, net, [1e3, 0.0], 50.0, t)
    exact = 1e3 * np.exp(-k * t)
    assert abs(out["y"][0, 0] - exact) <= GLOBAL * 1e-6 * exact
    assert abs(out["y"][0, 0] + out["y"][0, 1] - 1e3) <= 1e-12 * 1e3


def test_second_order_same_species(oracle_mod):
    """A + A -> B at rate k n_A^2 removes two A per event (Sec. 2.1), so
    dn_A/dt = -2 k n_A^2 and n_A = n_A0 / (1 + 2 k n_A0 t)."""
    k, y0 = 1e-10, 1e4
    net = network_from([([0, 0], [1])], [k], 2)
    t = 20.0 / (2 * k * y0)
    out = _final(oracle_mod, net, [y0, 0.0], 30.0, t)
    exact = y0 / (1 + 2 * k * y0 * t)
    assert abs(out["y"][0, 0] - exact) <= GLOBAL * 1e-6 * exact
    assert abs(out["y"][0, 0] + 2 * out["y"][0, 1] - y0) <= 1e-12 * y0


def test_second_order_two_species(oracle_mod):
    """A + B -> C: with D = n_A0 - n_B0, n_A = D / (1 - (n_B0/n_A0) e^{-k D t})."""
    k, a0, b0 = 1e-10, 2e4, 1e4
    net = network_from([([0, 1], [2])], [k], 3)
    D = a0 - b0
    t = 3.0 / (k * D)
    out = _final(oracle_mod, net, [a0, b0, 0.0], 30.0, t)
    exact = D / (1 - (b0 / a0) * np.exp(-k * D * t))
    assert abs(out["y"][0, 0] - exact) <= GLOBAL * 1e-6 * exact
    assert abs(out["y"][0, 1] - (exact - D)) <= GLOBAL * 1e-6 * (exact - D)


def test_paper_example_equilibrium(oracle_mod):
    """2A -> B and B + hv -> 2A (Sec. 2.1) relax to k n_A^2 = zeta n_B with
    n_A + 2 n_B conserved."""
    k, zeta = 1e-9, 1e-6
    net = network_from([([0, 0], [1]), ([1], [0, 0])], [k, zeta], 2)
    y0 = np.array([3e3, 1e2])
    N = y0[0] + 2 * y0[1]
    out = _final(oracle_mod, net, y0, 20.0, 1e9)
    yA = (-zeta + np.sqrt(zeta ** 2 + 8 * k * zeta * N)) / (4 * k)
    assert abs(out["y"][0, 0] - yA) <= GLOBAL * 1e-6 * yA
    assert abs(out["y"][0, 0] + 2 * out["y"][0, 1] - N) <= 1e-12 * N


def _linear_subnet(tiny_net):
    one = np.flatnonzero((tiny_net.reactants >= 0).sum(1) == 1)
    return tiny_net.subset(one)


def test_linear_network_matches_expm(oracle_mod, tiny):
    """All-one-body networks are linear: y(t) = expm(t A) y0, with A the
    (FD-pinned) Jacobian and expm from SciPy."""
    net, cells = tiny
    lin = _linear_subnet(net)
    y0, T = cells.y0[0], float(cells.T[0])
    A = oracle_mod.jac_dense(lin, y0[None], [T])[0]
    for t in (1e9, 1e11, 1e13):
        out = _final(oracle_mod, lin, y0, T, t)
        ref = scipy.linalg.expm(A * t) @ y0
        tol = GLOBAL * 1e-6 * np.abs(ref) + 1e-12 * np.abs(y0).max()
        assert np.all(np.abs(out["y"][0] - ref) <= tol)


def test_error_shrinks_with_tolerance(oracle_mod, tiny):
    """Tightening rtol by 100 cuts the global error on the linear network by
    at least 10 (the method converges)."""
    net, cells = tiny
    lin = _linear_subnet(net)
    y0, T = cells.y0[0], float(cells.T[0])
    A = oracle_mod.jac_dense(lin, y0[None], [T])[0]
    t = 1e11
    ref = np.linalg.matrix_power(scipy.linalg.expm(A * t / 1024), 1024) @ y0
    big = np.abs(ref) > 1e-6 * np.abs(y0).max()
    errs = []
    for rtol in (1e-6, 1e-8):
        y = _final(oracle_mod, lin, y0, T, t, rtol=rtol)["y"][0]
        errs.append(np.max(np.abs(y - ref)[big] / np.abs(ref[big])))
    assert errs[1] < 0.1 * errs[0], errs


def test_single_backward_euler_step(oracle_mod, tiny):
    """q_max = 1 with a step equal to the interval is one backward-Euler
    step; on a linear network Newton lands on (I - h A)^{-1} y0."""
    net, cells = tiny
    lin = _linear_subnet(net)
    y0, T = cells.y0[0], float(cells.T[0])
    A = oracle_mod.jac_dense(lin, y0[None], [T])[0]
    h = 0.01 / np.abs(np.diag(A)).max()
    out = _final(oracle_mod, lin, y0, T, h, q_max=1, h0=h, rtol=1e-3)
    assert out["stats"][0, 0] == 1
    ref = np.linalg.solve(np.eye(A.shape[0]) - h * A, y0)
    np.testing.assert_allclose(out["y"][0], ref, rtol=1e-12, atol=1e-14 * np.abs(y0).max())


@pytest.mark.slow
def test_matches_scipy_radau(oracle_mod, tiny):
    """The 50-species network against SciPy's Radau IIA at rtol 1e-10."""
    net, cells = tiny
    y0, T = cells.y0[0], float(cells.T[0])
    t_end = 1e5 * YEAR_S
    fun = lambda t, y: oracle_mod.rhs(net, y[None], [T])[0]
    jac = lambda t, y: oracle_mod.jac_dense(net, y[None], [T])[0]
    ref = scipy.integrate.solve_ivp(fun, (0, t_end), y0, method="Radau", jac=jac, rtol=1e-10,
                                    atol=1e-30).y[:, -1]
    # Backward Euler (q_max = 1) controls a local error of order h^2, so its
    # global error grows like sqrt(rtol); orders up to 5 stay near rtol.
    for q_max, rel in ((1, 10 * np.sqrt(1e-6)), (5, GLOBAL * 1e-6)):
        out = _final(oracle_mod, net, y0, T, t_end, q_max=q_max)
        tol = rel * np.abs(ref) + 1e-16 * np.abs(y0).max()
        bad = np.abs(out["y"][0] - ref) > tol
        assert not bad.any(), (q_max, np.flatnonzero(bad))


def test_conserves_elements_over_the_run(oracle_mod, tiny):
    """E J = 0 makes every Newton correction E-neutral, so the element and
    charge totals survive thousands of steps up to rounding. The rounding
    of the linear solves grows with the conditioning of I - c J, which is
    large for long steps in hot cells: there SciPy's BDF drifts by 8e-9
    relative over 1e6 yr at 140 K on this network, as does the oracle."""
    net, cells = tiny
    E = net.composition.astype(np.float64).T
    y0 = np.repeat(cells.y0[:1], 2, 0)
    out = _final(oracle_mod, net, y0, [20.0, 140.0], 1e6 * YEAR_S)
    for c, bound in ((0, 1e-12), (1, 1e-7)):
        drift = np.abs(E @ out["y"][c] - E @ y0[c])
        assert np.all(drift <= bound * (np.abs(E) @ y0[c])), c


def test_thread_count_does_not_change_results(oracle_mod, tiny):
    net, cells = tiny
    y0 = np.repeat(cells.y0[:1], 4, 0)
    T = np.array([10.0, 20.0, 80.0, 300.0])
    old = oracle_mod.get_threads()
    oracle_mod.set_threads(1)
    a = oracle_mod.bdf(net, y0, T, 1e5 * YEAR_S)
    oracle_mod.set_threads(4)
    b = oracle_mod.bdf(net, y0, T, 1e5 * YEAR_S)
    oracle_mod.set_threads(old)
    assert np.array_equal(a["y"], b["y"]) and np.array_equal(a["stats"], b["stats"])


def test_status_codes(oracle_mod, tiny):
    net, cells = tiny
    y0 = np.repeat(cells.y0[:1], 5, 0)
    y0[1, 3] = np.nan
    y0[2, 4] = -1.0
    T = np.array([20.0, 20.0, 20.0, 0.0, -4.0])
    out = oracle_mod.bdf(net, y0, T, 1e3 * YEAR_S)
    assert out["status"].tolist() == [0, 3, 3, 3, 3]
    assert np.array_equal(out["y"][1:], y0[1:], equal_nan=True)   # untouched
    out = oracle_mod.bdf(net, y0[:1], T[:1], 1e3 * YEAR_S, max_steps=3)
    assert out["status"].tolist() == [oracle_mod.MAXSTEPS] and out["stats"][0, 0] == 3
    # A + A -> 3 A blows up at t = 1/(k n_A0) = 1e6 s: the step size
    # collapses near the pole, where error-test and corrector rejections
    # alternate; the status names the last one (which of the two comes last
    # turns on rounding), and the run stops far up the pole
    blow = network_from([([0, 0], [0, 0, 0])], [1e-6], 1)
    out = oracle_mod.bdf(blow, [[1.0]], [300.0], 1e7)
    assert out["status"][0] in (oracle_mod.NEWTON_FAIL, oracle_mod.HMIN, oracle_mod.NONFINITE)
    st = dict(zip(oracle_mod.STAT_NAMES, out["stats"][0]))
    assert st["reject_err"] > 0 and st["reject_newton"] > 0
    assert out["y"][0, 0] > 1e6
    # error-test rejections alone: an unreachable accuracy makes every step
    # fail the error test until h falls below h_min
    out = oracle_mod.bdf(net, y0[:1], T[:1], 1e3 * YEAR_S, rtol=1e-30, atol=0.0)
    assert out["status"].tolist() == [oracle_mod.HMIN]


def test_zero_interval_is_identity(oracle_mod, tiny):
    net, cells = tiny
    out = oracle_mod.bdf(net, cells.y0[:1], cells.T[:1], 0.0)
    assert out["status"][0] == 0 and np.array_equal(out["y"], cells.y0[:1])

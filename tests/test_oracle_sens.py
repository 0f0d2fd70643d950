"""Pins of the oracle's replayed integrator and its forward sensitivities
(the reference for the GPU adjoint): central finite differences through
the same replayed step sequence, closed-form derivatives of the decay
solutions, and linearity in the initial state for linear networks."""
import numpy as np
import pytest
import scipy.linalg

import synthnet
from conftest import YEAR_S, network_from


def _record(oracle_mod, net, y0, T, t_end, **kw):
    out = oracle_mod.bdf(net, np.atleast_2d(y0), np.atleast_1d(T), t_end, tape_cap=200000, **kw)
    assert np.all(out["status"] == 0) and np.all(out["tape_len"] > 0)
    return out


def test_replay_reproduces_run(oracle_mod, tiny):
    """Replaying the step sequence with a converged corrector moves the end
    state by far less than the integration tolerance."""
    net, cells = tiny
    y0, T = cells.y0[:2], cells.T[:2]
    out = _record(oracle_mod, net, y0, T, 1e5 * YEAR_S)
    y, _ = oracle_mod.bdf_replay(net, y0, T, out["tape"], out["tape_len"])
    big = np.abs(out["y"]) > 1e-20
    assert np.all(np.abs(y - out["y"])[big] <= 1e-6 * np.abs(out["y"][big]))


def test_decay_sensitivity_closed_form(oracle_mod):
    """n_A = n_A0 exp(-k t): d n_A / d log k = -k t n_A and d n_A / d n_A0 = exp(-k t)."""
    k = 1e-9
    net = network_from([([0], [1])], [k], 2)
    t = 2.0 / k
    y0 = np.array([[5.0, 0.0]])
    out = _record(oracle_mod, net, y0, [40.0], t)
    dy0 = np.zeros((1, 2, 2))
    dy0[0, 1, 0] = 1.0
    dla = np.array([[1.0], [0.0]])
    y, s = oracle_mod.bdf_replay(net, y0, [40.0], out["tape"], out["tape_len"], dy0=dy0,
                                 dlogalpha=dla, n_dir=2)
    yA = 5.0 * np.exp(-k * t)
    assert abs(s[0, 0, 0] - (-k * t * yA)) <= 1e-4 * k * t * yA
    assert abs(s[0, 0, 1] + s[0, 0, 0]) <= 1e-12 * abs(s[0, 0, 0])       # mass conservation
    assert abs(s[0, 1, 0] - np.exp(-k * t)) <= 1e-4 * np.exp(-k * t)


def test_linear_network_initial_state_sensitivity(oracle_mod, tiny):
    """On a linear network the replayed map is linear in y0, so the tangent
    along e_i is the i-th column of the discrete propagator, which tracks
    expm(t A) e_i."""
    net, cells = tiny
    lin = net.subset(np.flatnonzero((net.reactants >= 0).sum(1) == 1))
    y0, T = cells.y0[:1], cells.T[:1]
    t = 1e11
    out = _record(oracle_mod, lin, y0, T, t)
    idx = [0, 5, 17]
    ns = lin.n_species
    dy0 = np.zeros((1, len(idx), ns))
    for r, i in enumerate(idx):
        dy0[0, r, i] = 1.0
    y, s = oracle_mod.bdf_replay(lin, y0, T, out["tape"], out["tape_len"], dy0=dy0, n_dir=len(idx))
    A = oracle_mod.jac_dense(lin, y0, T)[0]
    P = scipy.linalg.expm(A * t)
    for r, i in enumerate(idx):
        assert np.all(np.abs(s[0, r] - P[:, i]) <= 1e-4 * np.abs(P[:, i]) + 1e-10)


@pytest.mark.parametrize("seed", [0, 1])
def test_sensitivity_matches_central_differences(oracle_mod, tiny, seed):
    """Forward sensitivities vs central differences (step 1e-3 in log alpha
    and in log y0) of the replayed map. Where the end state depends
    linearly on alpha_j the quotient carries exactly sinh(e)/e - 1 = e^2/6;
    below about 1e-12 |y_i| / e (plus 1e-13 max|y| / e, the roundoff of
    the largest densities spread by the linear solves) it only sees the
    corrector's rounding floor: eps times the condition number of I - c J
    on long stiff steps."""
    net, cells = tiny
    rng = np.random.default_rng(seed)
    y0, T = cells.y0[:1], cells.T[:1] * (1 + 3 * seed)
    t_end = 1e4 * YEAR_S
    out = _record(oracle_mod, net, y0, T, t_end)
    js = rng.choice(net.n_reactions, 6, replace=False)
    iis = rng.choice(net.n_species, 3, replace=False)
    nd = len(js) + len(iis)
    dla = np.zeros((nd, net.n_reactions))
    dy0 = np.zeros((1, nd, net.n_species))
    for r, j in enumerate(js):
        dla[r, j] = 1.0
    for r, i in enumerate(iis):
        dy0[0, len(js) + r, i] = y0[0, i]        # d/d log y0_i
    y, s = oracle_mod.bdf_replay(net, y0, T, out["tape"], out["tape_len"], dy0=dy0,
                                 dlogalpha=dla, n_dir=nd)
    e = 1e-3
    for r in range(nd):
        ys = []
        for sgn in (1, -1):
            n2 = net.subset(np.arange(net.n_reactions))
            y2 = y0.copy()
            if r < len(js):
                n2.alpha[js[r]] *= np.exp(sgn * e)
            else:
                i = iis[r - len(js)]
                y2[0, i] *= np.exp(sgn * e)
            yy, _ = oracle_mod.bdf_replay(n2, y2, T, out["tape"], out["tape_len"])
            ys.append(yy[0])
        fd = (ys[0] - ys[1]) / (2 * e)
        g = s[0, r]
        noise = (1e-12 * np.abs(y[0]) + 1e-13 * np.abs(y[0]).max()) / e
        assert np.all(np.abs(g - fd) <= 1e-5 * np.abs(g) + 1e-8 * np.abs(g).max() + noise), r

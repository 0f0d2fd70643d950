"""Pins of the oracle's temperature-coupled mode (temperature as a state
variable, as in codes that solve temperature and abundances together,
Sec. 5): closed forms, a conserved energy, derivatives by differences."""
import numpy as np
import pytest

import synthnet
from conftest import YEAR_S, network_from

KB = synthnet.K_BOLTZMANN


def _medium_thermal(medium_net, n=4, lam=0.0, seed=3):
    h = synthnet.species_enthalpies(medium_net.n_species, seed)
    net = synthnet.with_heat(medium_net, h)
    cells = synthnet.make_cells(net, n, synthnet.SEED_BASE + 12)
    y = np.concatenate([cells.y0, cells.T[:, None]], 1)
    th = synthnet.thermal_params(cells.n_H, cells.T, lam)
    return net, h, cells, y, th


def test_thermal_rhs_species_part_is_the_fixed_temperature_rhs(oracle_mod, medium_net):
    """With T in the state, the species derivatives are those of the plain
    RHS at that T, bit for bit."""
    net, h, cells, y, th = _medium_thermal(medium_net)
    y[:, -1] *= 1.37
    f = oracle_mod.rhs_thermal(net, y, cells.T, th)
    ref = oracle_mod.rhs(net, y[:, :-1], y[:, -1])
    assert np.array_equal(f[:, :-1], ref)


def test_thermal_energy_is_conserved(oracle_mod, medium_net):
    """Reaction heats built from species energies h (heat_j = h.(reactants -
    products)) and no relaxation: c_v dT/dt + h . dn/dt = 0 up to rounding of
    the terms, because heat = -S^T h."""
    net, h, cells, y, th = _medium_thermal(medium_net)
    f, ab = oracle_mod.rhs_thermal(net, y, cells.T, th, with_abs=True)
    res = th[:, 0] * f[:, -1] + f[:, :-1] @ h
    scale = th[:, 0] * ab[:, -1] + ab[:, :-1] @ np.abs(h)
    assert np.all(np.abs(res) <= 1e-12 * scale)
    assert np.all(np.abs(th[:, 0] * f[:, -1]) > 1e3 * np.abs(res))   # not trivially zero


def test_thermal_jacobian_matches_differences(oracle_mod, tiny):
    """Every column of the coupled Jacobian, the T column through d k/dT
    included, against central differences of the coupled RHS."""
    net0, cells = tiny
    h = synthnet.species_enthalpies(net0.n_species, 5, scale_K=300.0)
    net = synthnet.with_heat(net0, h)
    y = np.concatenate([cells.y0[0], [35.0]])
    T = cells.T[:1]
    th = synthnet.thermal_params(cells.n_H[:1], [30.0], 3e-10)
    J = oracle_mod.jac_thermal(net, y[None], T, th)[0]
    _, fab = oracle_mod.rhs_thermal(net, y[None], T, th, with_abs=True)
    n = y.size
    for a in range(n):
        e = 1e-5 * max(abs(y[a]), 1e-30)
        yp, ym = y.copy(), y.copy()
        yp[a] += e
        ym[a] -= e
        fd = (oracle_mod.rhs_thermal(net, yp[None], T, th)[0] -
              oracle_mod.rhs_thermal(net, ym[None], T, th)[0]) / (2 * e)
        # rates are at most quadratic in the densities (central differences
        # exact up to rounding, eps sum|terms| / h); in T the coefficients are
        # smooth and the truncation error is O(e^2)
        tol = 1e-7 * np.abs(J[:, a]) + 1e-9 * fab[0] / e
        assert np.all(np.abs(fd - J[:, a]) <= tol), a


def test_thermal_logistic_closed_form(oracle_mod):
    """A -> B with k = alpha T/300 (beta = 1, gamma = 0) releasing heat
    epsilon per event, no relaxation: T = T0 + q (a0 - a) with q =
    epsilon / c_v, and a(t) = A a0 / (q a0 + (A - q a0) exp(alpha A t / 300))
    with A = T0 + q a0 (a logistic equation)."""
    alpha, T0, a0 = 2e-9, 40.0, 3.0
    cv = 1.5 * KB * 1e4
    eps = 10.0 * cv / a0               # the reaction heats the gas by 10 K in all
    net = network_from([([0], [1])], [alpha], 2, beta=[1.0], gamma=[0.0])
    net.heat = np.array([eps])
    q = eps / cv
    A = T0 + q * a0
    for years in (10.0, 100.0, 1000.0):
        t = years * YEAR_S
        out = oracle_mod.bdf_thermal(net, [[a0, 0.0, T0]], [T0], [[cv, T0, 0.0]], t, rtol=1e-9,
                                     atol=1e-30)
        a = A * a0 / (q * a0 + (A - q * a0) * np.exp(alpha * A * t / 300.0))
        y = out["y"][0]
        assert out["status"][0] == 0
        assert abs(y[0] - a) <= 1e-6 * a0
        assert abs(y[2] - (T0 + q * (a0 - a))) <= 1e-6 * T0
        assert abs(y[0] + y[1] - a0) <= 1e-12 * a0


def test_thermal_relaxation_closed_form(oracle_mod, tiny):
    """No reaction heat and relaxation rate lambda: T(t) = T_b + (T0 - T_b)
    exp(-lambda t) whatever the chemistry does."""
    net, cells = tiny
    lam, Tb, T0 = 2e-10, 20.0, 90.0
    y0 = np.concatenate([cells.y0[0], [T0]])[None]
    t = 3e10
    out = oracle_mod.bdf_thermal(net, y0, cells.T[:1], [[1.5 * KB * 1e4, Tb, lam]], t, rtol=1e-8,
                                 atol=1e-30)
    assert out["status"][0] == 0
    assert abs(out["y"][0, -1] - (Tb + (T0 - Tb) * np.exp(-lam * t))) <= 1e-6 * T0


def test_thermal_bdf_conserves_energy(oracle_mod, medium_net):
    """On the paper-sized network with reaction heats and no relaxation, the
    integrator keeps c_v T + h . n constant (every Newton correction is in
    the span the invariant annihilates) while T changes."""
    net, h, cells, y, th = _medium_thermal(medium_net, n=2)
    out = oracle_mod.bdf_thermal(net, y, cells.T, th, 1e3 * YEAR_S)
    assert list(out["status"]) == [0, 0]
    E0 = th[:, 0] * y[:, -1] + y[:, :-1] @ h
    E1 = th[:, 0] * out["y"][:, -1] + out["y"][:, :-1] @ h
    scale = th[:, 0] * y[:, -1] + np.abs(y[:, :-1]) @ np.abs(h)
    assert np.all(np.abs(E1 - E0) <= 1e-9 * scale)
    assert np.all(np.abs(out["y"][:, -1] - y[:, -1]) > 1e-3)     # T moved

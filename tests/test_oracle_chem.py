"""Pins of the oracle's rate, RHS, Jacobian and VJP against facts fixed by
the paper and by mathematics (not against the oracle itself)."""
import dataclasses
import json
import os

import numpy as np
import pytest

import synthnet
from conftest import network_from

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _paper_example(k, zeta):
    g = json.load(open(os.path.join(GOLD, "paper_example_2A_B.json")))
    idx = {s: i for i, s in enumerate(g["species"])}
    rx = [([idx[s] for s in r], [idx[s] for s in p]) for r, p in g["reactions"]]
    return g, network_from(rx, [k, zeta], 2)


# ---------------------------------------------------------------- S and RHS

def test_paper_example_stoichiometry(oracle_mod):
    """Sec. 2.1 prints S = [[-2, 2], [1, -1]] for 2A -> B, B + hv -> 2A."""
    g, net = _paper_example(3.0, 5.0)
    assert oracle_mod.stoich(net).tolist() == g["stoichiometry_matrix"]


@pytest.mark.parametrize("seed", range(5))
def test_paper_example_rhs(oracle_mod, seed):
    """Sec. 2.1: dnA/dt = -2 k nA^2 + 2 zeta nB and dnB/dt = k nA^2 - zeta nB
    (beta = gamma = 0 makes the coefficient equal to alpha at any T)."""
    rng = np.random.default_rng(seed)
    k, zeta = 10 ** rng.uniform(-3, 3, 2)
    nA, nB = 10 ** rng.uniform(-3, 3, 2)
    _, net = _paper_example(k, zeta)
    T = rng.uniform(10, 300)
    f = oracle_mod.rhs(net, [[nA, nB]], [T])[0]
    ref = np.array([-2 * k * nA ** 2 + 2 * zeta * nB, k * nA ** 2 - zeta * nB])
    scale = np.array([2 * k * nA ** 2 + 2 * zeta * nB, k * nA ** 2 + zeta * nB])
    assert np.all(np.abs(f - ref) <= 4e-16 * scale)


def test_paper_example_jacobian(oracle_mod):
    """Derivative of the two printed equations of Sec. 2.1."""
    k, zeta, nA, nB = 0.7, 1.9, 2.5, 0.3
    _, net = _paper_example(k, zeta)
    J = oracle_mod.jac_dense(net, [[nA, nB]], [50.0])[0]
    ref = np.array([[-4 * k * nA, 2 * zeta], [2 * k * nA, -zeta]])
    np.testing.assert_allclose(J, ref, rtol=1e-15)


def _eq1_production_destruction(net, k, y):
    """Eq. (modelrate) of Sec. 2.1, written in its own per-species form:
    formation from one-body sources (zeta_li n_l) and two-body sources
    (k_jmi n_j n_m), minus n_i times its own destruction frequencies. Valid
    for reactions with distinct reactants and distinct products, where it
    and the matrix form must coincide."""
    ns = y.shape[0]
    out = np.zeros(ns)
    form = [[] for _ in range(ns)]
    dest = [[] for _ in range(ns)]
    for j in range(net.n_reactions):
        rea = [a for a in net.reactants[j] if a >= 0]
        pro = [p for p in net.products[j] if p >= 0]
        for p in pro:                           # formation terms of species p
            term = k[j]
            for a in rea:
                term = term * y[a]
            form[p].append(term)
        for i in rea:                           # n_i * (zeta_il or k_ijm n_j)
            freq = k[j]
            for a in rea:
                if a != i:
                    freq = freq * y[a]
            dest[i].append(y[i] * freq)
    for i in range(ns):
        out[i] = sum(form[i]) - sum(dest[i])
    return out


def test_matrix_form_equals_production_destruction_form(oracle_mod, medium_net):
    """The matrix form (eq. matrix-form) and the production/destruction form
    (eq. modelrate) describe the same ODE where the latter is unambiguous."""
    net = medium_net
    keep = [j for j in range(net.n_reactions)
            if len(set(a for a in net.reactants[j] if a >= 0)) == (net.reactants[j] >= 0).sum()
            and len(set(p for p in net.products[j] if p >= 0)) == (net.products[j] >= 0).sum()
            and not (set(net.reactants[j]) - {-1}) & (set(net.products[j]) - {-1})]
    sub = net.subset(keep)
    assert sub.n_reactions > 0.8 * net.n_reactions
    cells = synthnet.make_cells(sub, 3, 11)
    k = oracle_mod.rate_coeffs(sub, cells.T)
    f, ab = oracle_mod.rhs(sub, cells.y0, cells.T, with_abs=True)
    for c in range(3):
        ref = _eq1_production_destruction(sub, k[c], cells.y0[c])
        assert np.all(np.abs(f[c] - ref) <= 1e-13 * ab[c] + 1e-300)


def test_element_and_charge_conservation(oracle_mod, medium):
    """Every generated reaction balances H, He, C, N, O and charge, so
    E dn/dt = 0 up to rounding of the per-species sums."""
    net, cells = medium
    E = net.composition.astype(np.float64).T          # 6 x ns
    S = oracle_mod.stoich(net)
    assert np.all(net.composition.astype(np.int64).T @ S == 0)
    f, ab = oracle_mod.rhs(net, cells.y0[:16], cells.T[:16], with_abs=True)
    lhs = f @ E.T
    bound = 1e-12 * (ab @ np.abs(E).T)
    assert np.all(np.abs(lhs) <= bound)


def test_species_relabelling_is_exact(oracle_mod, tiny):
    """Row order is arbitrary (Sec. 3): relabelling species permutes dn/dt
    bit for bit when the reaction order is kept."""
    net, cells = tiny
    rng = np.random.default_rng(3)
    p = rng.permutation(net.n_species)
    inv = np.argsort(p)                       # new index of old species i is inv[i]
    rea = np.where(net.reactants >= 0, inv[np.maximum(net.reactants, 0)], -1)
    pro = np.where(net.products >= 0, inv[np.maximum(net.products, 0)], -1)
    net2 = synthnet.Network(rea.astype(np.int32), pro.astype(np.int32), net.alpha, net.beta,
                            net.gamma, net.composition[p], [net.names[i] for i in p], net.rtype)
    y = cells.y0[:2]
    f1 = oracle_mod.rhs(net, y, cells.T[:2])
    f2 = oracle_mod.rhs(net2, y[:, p], cells.T[:2])
    assert np.array_equal(f1[:, p], f2)


# ------------------------------------------------------------------ rates

def test_rate_coefficient_special_cases(oracle_mod):
    """With beta = gamma = 0 the coefficient is alpha; at T = 300 K the
    power-law factor is 1; beta = 1 makes it linear in T."""
    rx = [([0], [1])] * 3
    net = network_from(rx, [2e-10, 3e-9, 5e-11], 2, beta=[0.0, 0.0, 1.0], gamma=[0.0, 450.0, 0.0])
    k = oracle_mod.rate_coeffs(net, [300.0, 150.0])
    assert k[0, 0] == 2e-10 and k[1, 0] == 2e-10
    assert abs(k[0, 1] / 3e-9 - np.exp(-1.5)) < 1e-15
    assert abs(k[1, 2] / 5e-11 - 0.5) < 1e-15


def test_rate_coefficient_log_derivative(oracle_mod, medium_net):
    """d ln k / d ln T = beta + gamma / T for the modified Arrhenius law."""
    net = medium_net
    T = np.array([20.0, 95.0])
    e = 1e-6
    kp = oracle_mod.rate_coeffs(net, T * np.exp(e))
    km = oracle_mod.rate_coeffs(net, T * np.exp(-e))
    fd = (np.log(kp) - np.log(km)) / (2 * e)
    ref = net.beta[None, :] + net.gamma[None, :] / T[:, None]
    assert np.all(np.abs(fd - ref) <= 1e-6 * (1 + np.abs(ref)))


def _law_net(laws, alpha, beta, gamma):
    rx = [([0], [1])] * len(laws)
    net = network_from(rx, alpha, 2, beta=beta, gamma=gamma)
    net.law = np.asarray(laws, np.int8)
    return net


def test_rate_laws_special_cases(oracle_mod):
    """Reference conditions recover the tabulated prefactor: direct
    cosmic-ray ionisation at zeta = zeta_0 gives alpha; an FUV photorate
    with no extinction (A_V = 0) in the unit field (G_0 = 1) gives alpha;
    the cosmic-ray photon law at T = 300 K, zeta = zeta_0 gives alpha gamma
    / (1 - albedo) with albedo 0.6; the modified Arrhenius law ignores A_V,
    zeta and G_0."""
    L = oracle_mod
    net = _law_net([L.LAW_CRP, L.LAW_PHOTO, L.LAW_CRPHOT, L.LAW_KOOIJ], [2e-17, 3e-10, 1.3e-17, 4e-10],
                   [0.7, 0.0, 0.3, 0.5], [9.0, 2.5, 800.0, 120.0])
    cond = np.array([[300.0, 0.0, 1.0, 1.0], [40.0, 3.0, 7.0, 25.0]])
    k = L.rate_coeffs(net, cond)
    assert k[0, 0] == 2e-17 and k[0, 1] == 3e-10
    assert abs(k[0, 2] / (1.3e-17 * 800.0 * 2.5) - 1) < 1e-15
    kooij = L.rate_coeffs(network_from([([0], [1])], [4e-10], 2, beta=[0.5], gamma=[120.0]),
                          [300.0, 40.0])
    assert k[0, 3] == kooij[0, 0] and k[1, 3] == kooij[1, 0]


def test_rate_laws_scalings(oracle_mod):
    """Cosmic-ray rates are linear in zeta and photorates in G_0 (doubling is
    exact in floating point); one magnitude of extinction divides a photorate
    by exp(gamma); the cosmic-ray photon law scales with T like (T/300)^beta."""
    L = oracle_mod
    net = _law_net([L.LAW_CRP, L.LAW_CRPHOT, L.LAW_PHOTO], [2e-17, 1.3e-17, 3e-10],
                   [0.0, 0.4, 0.0], [0.0, 500.0, 1.8])
    base = np.array([[55.0, 2.0, 0.8, 3.0]])
    k0 = L.rate_coeffs(net, base)[0]
    z2 = base.copy(); z2[0, 2] *= 2
    g2 = base.copy(); g2[0, 3] *= 2
    a1 = base.copy(); a1[0, 1] += 1.0
    t2 = base.copy(); t2[0, 0] *= 2
    kz, kg, ka, kt = (L.rate_coeffs(net, c)[0] for c in (z2, g2, a1, t2))
    assert kz[0] == 2 * k0[0] and kz[1] == 2 * k0[1] and kz[2] == k0[2]
    assert kg[2] == 2 * k0[2] and kg[0] == k0[0] and kg[1] == k0[1]
    assert abs(k0[2] / ka[2] - np.exp(1.8)) < 1e-14 * np.exp(1.8)
    assert abs(kt[1] / k0[1] - 2 ** 0.4) < 1e-14 and kt[0] == k0[0] and kt[2] == k0[2]


def test_rate_laws_typed_network_rhs(oracle_mod, medium_net):
    """On the paper-sized network with cosmic-ray and photo laws on its
    one-body reactions, the RHS of every cell still conserves elements and
    charge (E f = 0), and a Kooij-only network reproduces the plain
    temperature-only call bit for bit."""
    net = synthnet.with_rate_laws(medium_net, 5)
    cells = synthnet.make_cells(net, 6, synthnet.SEED_BASE + 9)
    cond = synthnet.make_conditions(cells.T, 9)
    f, ab = oracle_mod.rhs(net, cells.y0, cond, with_abs=True)
    E = net.composition.astype(np.float64).T
    assert np.all(np.abs(f @ E.T) <= 1e-12 * (ab @ np.abs(E).T) + 1e-300)
    plain = oracle_mod.rhs(medium_net, cells.y0, cells.T)
    kooij = dataclasses.replace(medium_net, law=np.zeros(medium_net.n_reactions, np.int8))
    assert np.array_equal(oracle_mod.rhs(kooij, cells.y0, cond), plain)


# --------------------------------------------------------------- Jacobian

def _fd_jac(oracle_mod, net, y, T, rel=1e-5):
    n = y.size
    J = np.zeros((n, n))
    for a in range(n):
        h = rel * y[a]
        yp, ym = y.copy(), y.copy()
        yp[a] += h
        ym[a] -= h
        J[:, a] = (oracle_mod.rhs(net, yp[None], [T])[0] - oracle_mod.rhs(net, ym[None], [T])[0]) / (2 * h)
    return J


def test_jacobian_matches_finite_differences(oracle_mod, tiny):
    """Central differences of the (separately pinned) RHS; the rates are at
    most quadratic in y, so the central difference is exact up to rounding."""
    net, cells = tiny
    y = cells.y0[0]
    T = float(cells.T[0])
    J, ab = oracle_mod.jac_dense(net, y[None], [T], with_abs=True)
    fd = _fd_jac(oracle_mod, net, y, T)
    _, fab = oracle_mod.rhs(net, y[None], [T], with_abs=True)
    # error of the difference quotient ~ eps * sum|terms| / h
    tol = 1e-8 * ab[0] + 1e-9 * fab[0][:, None] / y[None, :]
    assert np.all(np.abs(J[0] - fd) <= tol)


def test_jacobian_euler_homogeneity(oracle_mod, medium_net):
    """A rate with m reactant factors is homogeneous of degree m in y, so
    J y = S (m * R): J y = f for one-body and J y = 2 f for two-body sets."""
    net = medium_net
    nre = (net.reactants >= 0).sum(1)
    cells = synthnet.make_cells(net, 2, 5)
    for m in (1, 2):
        sub = net.subset(np.flatnonzero(nre == m))
        J, abJ = oracle_mod.jac_dense(sub, cells.y0, cells.T, with_abs=True)
        f, ab = oracle_mod.rhs(sub, cells.y0, cells.T, with_abs=True)
        Jy = np.einsum("cia,ca->ci", J, cells.y0)
        bound = 1e-12 * (np.einsum("cia,ca->ci", abJ, cells.y0) + m * ab)
        assert np.all(np.abs(Jy - m * f) <= bound)


def test_jacobian_conserves_elements(oracle_mod, medium):
    net, cells = medium
    E = net.composition.astype(np.float64).T
    J, ab = oracle_mod.jac_dense(net, cells.y0[:2], cells.T[:2], with_abs=True)
    for c in range(2):
        assert np.all(np.abs(E @ J[c]) <= 1e-12 * (np.abs(E) @ ab[c]))


# -------------------------------------------------------------------- VJP

def test_vjp_dot_product_identity(oracle_mod, medium):
    """<v, J u> = <J^T v, u> with J from the (FD-pinned) dense Jacobian."""
    net, cells = medium
    rng = np.random.default_rng(0)
    y, T = cells.y0[:3], cells.T[:3]
    v = rng.standard_normal(y.shape)
    u = rng.standard_normal(y.shape) * y
    gy, _ = oracle_mod.vjp(net, y, T, v)
    J, ab = oracle_mod.jac_dense(net, y, T, with_abs=True)
    lhs = np.einsum("ci,cia,ca->c", v, J, u)
    rhs_ = np.einsum("ca,ca->c", gy, u)
    scale = np.einsum("ci,cia,ca->c", np.abs(v), ab, np.abs(u))
    assert np.all(np.abs(lhs - rhs_) <= 1e-12 * scale)


def test_vjp_log_alpha_sum_rule(oracle_mod, medium):
    """dn/dt is linear in every alpha_j, so sum_j d<v,f>/d(log alpha_j) = <v, f>."""
    net, cells = medium
    rng = np.random.default_rng(1)
    y, T = cells.y0[:4], cells.T[:4]
    v = rng.standard_normal(y.shape)
    _, gl = oracle_mod.vjp(net, y, T, v)
    f, ab = oracle_mod.rhs(net, y, T, with_abs=True)
    lhs = gl.sum(1)
    rhs_ = (v * f).sum(1)
    assert np.all(np.abs(lhs - rhs_) <= 1e-12 * (np.abs(v) * ab).sum(1))


def test_vjp_log_alpha_finite_difference(oracle_mod, tiny):
    net, cells = tiny
    rng = np.random.default_rng(2)
    y, T = cells.y0[:1], cells.T[:1]
    v = rng.standard_normal(y.shape)
    _, gl = oracle_mod.vjp(net, y, T, v)
    e = 1e-6
    for j in rng.choice(net.n_reactions, 8, replace=False):
        np_, nm = net.subset(np.arange(net.n_reactions)), net.subset(np.arange(net.n_reactions))
        np_.alpha[j] *= np.exp(e)
        nm.alpha[j] *= np.exp(-e)
        fd = ((v * oracle_mod.rhs(np_, y, T)).sum() - (v * oracle_mod.rhs(nm, y, T)).sum()) / (2 * e)
        _, ab = oracle_mod.rhs(net, y, T, with_abs=True)
        assert abs(fd - gl[0, j]) <= 1e-6 * abs(gl[0, j]) + 1e-9 * (np.abs(v) * ab).sum()


def test_jacobian_on_pattern_equals_dense(oracle_mod, medium):
    """The pattern Jacobian (net stoichiometry, S dR/dn) equals the dense one
    (gross bookkeeping) up to rounding of the same terms, the dense one is
    exactly zero off the pattern of S dR/dn, and a pattern missing an entry
    is refused."""
    net, cells = medium
    y, T = cells.y0[:6], cells.T[:6]
    J, ab = oracle_mod.jac_dense(net, y, T, with_abs=True)
    S = oracle_mod.stoich(net)
    R = np.zeros((net.n_reactions, net.n_species), bool)
    for j, rs in enumerate(net.reactants):
        R[j, rs[rs >= 0]] = True
    P = (np.abs(S) @ R.astype(np.int64)) > 0
    rp = np.concatenate([[0], np.cumsum(P.sum(1))]).astype(np.int32)
    col = np.concatenate([np.flatnonzero(r) for r in P]).astype(np.int32)
    jv = oracle_mod.jac_pattern(net, y, T, rp, col)
    rows = np.repeat(np.arange(net.n_species), np.diff(rp))
    assert np.all(np.abs(jv - J[:, rows, col]) <= 1e-14 * ab[:, rows, col])
    assert np.all(J[:, ~P] == 0.0)
    with pytest.raises(ValueError):
        short = rp.copy()
        short[1:] -= 1
        short[short < 0] = 0
        oracle_mod.jac_pattern(net, y, T, np.maximum.accumulate(short), col)

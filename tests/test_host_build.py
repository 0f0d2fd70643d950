"""Host side of the library (no GPU needed): exported ABI, the storage
formats of Sec. 2.2 against the arrays the paper prints, the network build
(S, Jacobian pattern, orderings) against the oracle, and argument errors."""
import json
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as cg

import synthnet
from conftest import ROOT, network_from

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def acm():
    import paper_2312_04998_amd as acm
    return acm


def test_library_exports_every_declared_symbol(acm):
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"^\s*(?:ac_status|const char \*|int)\s+(ac_\w+)\s*\(", src, re.M))
    assert {"ac_net_create", "ac_rhs", "ac_jac", "ac_vjp", "ac_rates", "ac_rhs_k"} <= names
    missing = [n for n in sorted(names) if not hasattr(acm.lib, n)]
    assert not missing, missing


# ------------------------------------------------------ Sec. 2.2 formats

@pytest.fixture(scope="module")
def spmv():
    return json.load(open(os.path.join(GOLD, "paper_spmv_4x4.json")))


def test_crs_matches_paper(acm, spmv):
    val, idx, _, ptr = acm.ac_sparse_format(spmv["matrix"], acm.AC_FMT_CRS)
    g = spmv["crs"]
    assert val.tolist() == g["A"]
    assert (idx + 1).tolist() == g["col_ind"]
    assert (ptr[:5] + 1).tolist() == g["row_ptr"]


def test_ccs_matches_paper(acm, spmv):
    val, idx, _, ptr = acm.ac_sparse_format(spmv["matrix"], acm.AC_FMT_CCS)
    g = spmv["ccs"]
    assert val.tolist() == g["A"]
    assert (idx + 1).tolist() == g["row_ind"]
    assert (ptr[:5] + 1).tolist() == g["col_ptr"]


def test_coo_matches_paper_as_a_set(acm, spmv):
    """COO stores nonzeros in arbitrary order (Sec. 2.2): compare triplet sets."""
    val, col, row, _ = acm.ac_sparse_format(spmv["matrix"], acm.AC_FMT_COO)
    g = spmv["coo"]
    mine = sorted(zip(val.tolist(), (col + 1).tolist(), (row + 1).tolist()))
    paper = sorted(zip(g["A"], g["col_ind"], g["row_ind"]))
    assert mine == paper


def test_sell_matches_paper(acm, spmv):
    """Slices of wid_sl = 2 rows, nonzero k of each row stored together;
    padding carries value 0 and some valid column (the paper's choice of
    padding column is not specified, so only validity is checked)."""
    g = spmv["sell"]
    val, idx, _, ptr = acm.ac_sparse_format(spmv["matrix"], acm.AC_FMT_SELL, g["wid_sl"])
    assert val.tolist() == g["A"]
    assert ptr[:2].tolist() == g["len_sl"]
    for v, mine, paper in zip(val, idx + 1, g["col_ind"]):
        if v != 0:
            assert mine == paper
        else:
            assert 1 <= mine <= 4
    # the layout reproduces the SpMV of the 4x4 example
    A = np.array(spmv["matrix"])
    x = np.array([1.0, 10.0, 100.0, 1000.0])
    y = np.zeros(4)
    p = 0
    for s, L in enumerate(g["len_sl"]):
        for k in range(L):
            for r in range(g["wid_sl"]):
                y[s * g["wid_sl"] + r] += val[p] * x[idx[p]]
                p += 1
    np.testing.assert_array_equal(y, A @ x)


# --------------------------------------------------------- network build

def _net(acm, net, **kw):
    return acm.Network.from_synth(net, **kw)


def test_paper_example_stoichiometry(acm):
    """2A -> B, B + hv -> 2A gives S = [[-2, 2], [1, -1]] (Sec. 2.1)."""
    g = json.load(open(os.path.join(GOLD, "paper_example_2A_B.json")))
    net = network_from([([0, 0], [1]), ([1], [0, 0])], [1.0, 1.0], 2)
    N = _net(acm, net)
    rp, rx, va = N.stoich_csr()
    S = np.zeros((2, 2), int)
    for i in range(2):
        S[i, rx[rp[i]:rp[i + 1]]] = va[rp[i]:rp[i + 1]]
    assert S.tolist() == g["stoichiometry_matrix"]


@pytest.mark.parametrize("which", ["tiny", "medium"])
def test_stoichiometry_matches_oracle(acm, oracle_mod, which, tiny, medium_net):
    net = tiny[0] if which == "tiny" else medium_net
    N = _net(acm, net)
    rp, rx, va = N.stoich_csr()
    S = np.zeros((net.n_species, net.n_reactions), np.int32)
    for i in range(net.n_species):
        S[i, rx[rp[i]:rp[i + 1]]] = va[rp[i]:rp[i + 1]]
    np.testing.assert_array_equal(S, oracle_mod.stoich(net))
    assert N.nnz_s == int((S != 0).sum())


def test_jacobian_pattern_covers_oracle(acm, oracle_mod, medium):
    """Every nonzero of the oracle's dense Jacobian lies in the pattern, and
    every pattern entry is structurally nonzero for some densities."""
    net, cells = medium
    N = _net(acm, net)
    rp, col = N.jac_pattern()
    P = np.zeros((net.n_species, net.n_species), bool)
    for i in range(net.n_species):
        P[i, col[rp[i]:rp[i + 1]]] = True
        assert np.all(np.diff(col[rp[i]:rp[i + 1]]) > 0)
    J = oracle_mod.jac_dense(net, cells.y0[:3], cells.T[:3])
    assert not np.any((J != 0).any(0) & ~P)
    # structurally: (i, a) with S_ij != 0 and a a reactant of j
    S = oracle_mod.stoich(net)
    R = np.zeros((net.n_species, net.n_reactions), bool)
    for j in range(net.n_reactions):
        for a in net.reactants[j]:
            if a >= 0:
                R[a, j] = True
    structural = ((S != 0).astype(np.int64) @ R.T.astype(np.int64)) > 0
    np.testing.assert_array_equal(P, structural)


def test_orderings(acm, medium_net):
    net = medium_net
    nat = _net(acm, net, ordering="natural").row_order()
    assert nat.tolist() == list(range(net.n_species))
    N = _net(acm, net, ordering="nnz")
    p = N.row_order()
    rp, _, _ = N.stoich_csr()
    ln = np.diff(rp)[p]
    assert sorted(p.tolist()) == list(range(net.n_species))
    assert np.all(np.diff(ln) <= 0)                    # most nonzeros first
    for a, b in zip(p[:-1], p[1:]):                     # stable ties
        if ln[list(p).index(a)] == ln[list(p).index(b)]:
            assert a < b
    r = _net(acm, net, ordering="rcm").row_order()
    assert sorted(r.tolist()) == list(range(net.n_species))
    # RCM narrows the profile of the species graph S S^T relative to natural
    S = (_dense_s(N, net) != 0).astype(np.int64)
    G = ((S @ S.T) > 0)

    def bandwidth(perm):
        inv = np.argsort(perm)
        i, j = np.nonzero(G)
        return np.abs(inv[i] - inv[j]).max(), np.abs(inv[i] - inv[j]).sum()

    assert bandwidth(r)[1] < bandwidth(nat)[1]
    ref = cg.reverse_cuthill_mckee(sp.csr_matrix(G), symmetric_mode=True)
    assert bandwidth(r)[1] <= 1.5 * bandwidth(ref)[1]


def _dense_s(N, net):
    rp, rx, va = N.stoich_csr()
    S = np.zeros((net.n_species, net.n_reactions), np.int32)
    for i in range(net.n_species):
        S[i, rx[rp[i]:rp[i + 1]]] = va[rp[i]:rp[i + 1]]
    return S


def test_balance_check(acm, tiny):
    net = tiny[0]
    _net(acm, net, check_balance=True)          # generated networks balance
    bad = net.subset(np.arange(net.n_reactions))
    j = int(np.flatnonzero(bad.products[:, 1] >= 0)[0])
    bad.products[j, 1] = -1                      # drop a product
    with pytest.raises(acm.AstrochemError) as e:
        _net(acm, bad, check_balance=True)
    assert e.value.status == acm.AC_EUNBALANCED


def test_argument_errors(acm, tiny):
    net = tiny[0]
    bad = net.subset(np.arange(net.n_reactions))
    bad.reactants[3, 0] = net.n_species + 5
    with pytest.raises(acm.AstrochemError) as e:
        _net(acm, bad)
    assert e.value.status == acm.AC_EINVAL
    bad = net.subset(np.arange(net.n_reactions))
    bad.alpha[0] = -1.0
    with pytest.raises(acm.AstrochemError):
        _net(acm, bad)
    bad = net.subset(np.arange(net.n_reactions))
    bad.reactants[2] = -1                        # no reactant at all
    with pytest.raises(acm.AstrochemError):
        _net(acm, bad)
    with pytest.raises(KeyError):
        _net(acm, net, layout="ell")


def test_oversized_network_is_rejected(acm):
    ns = 3000
    net = network_from([([0], [ns - 1])], [1.0], ns)
    with pytest.raises(acm.AstrochemError) as e:
        _net(acm, net)
    assert e.value.status == acm.AC_ELIMIT


def test_schedules_cover_every_term(acm, medium_net):
    """Chunking keeps every nonzero of S exactly once (RHS terms), and the
    Jacobian has one term per (entry, reaction, reactant slot)."""
    net = medium_net
    for layout in ("csr", "sell", "coo", "runs", "ccs"):
        N = _net(acm, net, layout=layout, chunk=16)
        assert N.n_chunks >= net.n_species
    N = _net(acm, net)
    # terms: every (reaction j, distinct reactant a, species i with S_ij != 0)
    S = _dense_s(N, net)
    count = 0
    for j in range(net.n_reactions):
        reac = set(int(a) for a in net.reactants[j] if a >= 0)
        count += len(reac) * int((S[:, j] != 0).sum())
    assert N.n_contrib == count


def test_lu_size_limit(acm):
    """Dense LU panels live in one workgroup (two rows per thread): n <= 1024."""
    import torch
    A = torch.zeros((1, 1025, 1025), dtype=torch.float64)
    piv = torch.zeros((1, 1025), dtype=torch.int32)
    with pytest.raises(acm.AstrochemError) as e:
        acm.ac_lu_factor(A, piv, stream=0)   # rejected on the host, nothing launched
    assert e.value.status == acm.AC_ELIMIT


def test_front_plan(acm, medium_net, tiny):
    """The integrator's Newton-solve plan: a permutation of the species with
    the front first, starting at a species of least degree in the symmetric
    pattern of I - c J (minimum degree, ties to the smaller index), a front
    strictly between empty and everything on the paper-sized network (none
    on the 50-species network, where it would not repay its fixed latency),
    every pattern entry of a front row or column among the stored sparse
    values, and a modelled cost below one dense LU."""
    for net in (medium_net, tiny[0]):
        N = acm.Network.from_synth(net)
        fi = N.front_info()
        ns = N.n_species
        order = fi["order"]
        assert sorted(order.tolist()) == list(range(ns))
        assert 0 <= fi["n_front"] < ns and fi["cost_ratio"] <= 1.0
        assert (fi["n_levels"] >= 1) == (fi["n_front"] > 0)
        rp, col = N.jac_pattern()
        rows = np.repeat(np.arange(ns), np.diff(rp))
        P = sp.coo_matrix((np.ones(len(col)), (rows, col)), shape=(ns, ns)).tocsr()
        G = ((P + P.T + sp.eye(ns)) != 0).astype(int)
        deg = np.asarray(G.sum(1)).ravel()
        assert order[0] == int(np.flatnonzero(deg == deg.min())[0])
        pos = np.empty(ns, int)
        pos[order] = np.arange(ns)
        in_front = (pos[rows] < fi["n_front"]) | (pos[col] < fi["n_front"])
        diag_front = fi["n_front"] - np.count_nonzero(in_front & (rows == col))
        assert fi["n_values"] >= np.count_nonzero(in_front) + diag_front
        N.close()
    # the medium network's front is sizeable: it is where the savings come from
    fi = acm.Network.from_synth(medium_net).front_info()
    assert fi["n_front"] > 100 and fi["cost_ratio"] < 0.6
    assert acm.Network.from_synth(tiny[0]).front_info()["n_front"] == 0

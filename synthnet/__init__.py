"""Seeded synthetic reaction networks and cell states.

This module produces *inputs only*: reaction lists (reactant and product
species indices), modified-Arrhenius parameters, species compositions, and
per-cell temperatures, densities and initial abundances. It computes none of
the chemistry (no stoichiometry products, rates, derivatives or integration),
so both the oracle and the GPU path can consume its output without sharing any
of the method's arithmetic.

Why synthetic: the paper's benchmark network (UMIST rate12, 468 species and
6175 reactions, Sec. 3) and its PDR set-up are not available here. The
generator reproduces the *shape* of that network instead:

* roughly four nonzeros per stoichiometry column (24,580 nonzeros over 6175
  reactions, Sec. 3), at most six species per reaction (Sec. 5);
* strongly skewed species rows: atomic hydrogen, molecular hydrogen and the
  electron take part in about 29 %, 16 % and 14 % of all reactions (Sec. 5);
* reactions grouped by type in the natural order (Sec. 3);
* every reaction conserves the five elements H, He, C, N, O and charge.

Reaction mix, parameter ranges and cell ranges follow the workloads used to
exercise the method: 60 % two-body, 25 % one-body (cosmic-ray/photo), 15 %
dissociative recombination; alpha log-uniform on [1e-12, 1e-8], beta uniform
on (-1, 1), gamma uniform on (0, 1000) K; T log-uniform on 10-300 K, n_H
log-uniform on 1e2-1e7 cm^-3, fractional abundances log-uniform on
[1e-12, 1].
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Tuple

import numpy as np

ELEMENTS = ("H", "He", "C", "N", "O", "charge")
N_ELEM = len(ELEMENTS)
MAX_REACTANTS = 2
MAX_PRODUCTS = 4

# Seed base for the named workloads: seed = SEED_BASE + workload index.
SEED_BASE = 2312049980


@dataclasses.dataclass
class Network:
    """A reaction network as plain arrays.

    reactants : int32 [n_reactions, 2], species index or -1 (A+A listed twice)
    products  : int32 [n_reactions, 4], species index or -1
    alpha, beta, gamma : float64 [n_reactions]
    composition : int8 [n_species, 6] over (H, He, C, N, O, charge)
    names : species names
    rtype : int8 [n_reactions], 0 two-body, 1 one-body, 2 recombination,
            3 surface two-body
    """

    reactants: np.ndarray
    products: np.ndarray
    alpha: np.ndarray
    beta: np.ndarray
    gamma: np.ndarray
    composition: np.ndarray
    names: List[str]
    rtype: np.ndarray
    law: Optional[np.ndarray] = None   # int8 [n_reactions] rate-law code, None = all Kooij
    heat: Optional[np.ndarray] = None  # float64 [n_reactions] erg per reaction event, or None

    @property
    def n_species(self) -> int:
        return int(self.composition.shape[0])

    @property
    def n_reactions(self) -> int:
        return int(self.reactants.shape[0])

    def subset(self, idx) -> "Network":
        """Network restricted to the reactions in ``idx`` (same species)."""
        idx = np.asarray(idx)
        return Network(self.reactants[idx].copy(), self.products[idx].copy(),
                       self.alpha[idx].copy(), self.beta[idx].copy(),
                       self.gamma[idx].copy(), self.composition.copy(),
                       list(self.names), self.rtype[idx].copy(),
                       None if self.law is None else self.law[idx].copy(),
                       None if self.heat is None else self.heat[idx].copy())


def network_from_lists(n_species: int,
                       reactions: List[Tuple[List[int], List[int]]],
                       alpha, beta=None, gamma=None,
                       composition: Optional[np.ndarray] = None,
                       names: Optional[List[str]] = None) -> Network:
    """Build a Network from explicit (reactants, products) index lists."""
    nr = len(reactions)
    rea = -np.ones((nr, MAX_REACTANTS), np.int32)
    pro = -np.ones((nr, MAX_PRODUCTS), np.int32)
    for j, (r, p) in enumerate(reactions):
        if not 1 <= len(r) <= MAX_REACTANTS or not 1 <= len(p) <= MAX_PRODUCTS:
            raise ValueError(f"reaction {j}: bad arity")
        rea[j, :len(r)] = r
        pro[j, :len(p)] = p
    alpha = np.broadcast_to(np.asarray(alpha, np.float64), (nr,)).copy()
    beta = np.zeros(nr) if beta is None else np.broadcast_to(np.asarray(beta, np.float64), (nr,)).copy()
    gamma = np.zeros(nr) if gamma is None else np.broadcast_to(np.asarray(gamma, np.float64), (nr,)).copy()
    if composition is None:
        composition = np.zeros((n_species, N_ELEM), np.int8)
    if names is None:
        names = [f"X{i}" for i in range(n_species)]
    return Network(rea, pro, alpha, beta, gamma, np.asarray(composition, np.int8),
                   list(names), np.zeros(nr, np.int8))


# --------------------------------------------------------------------------
# species
# --------------------------------------------------------------------------

def _name(c: Tuple[int, ...]) -> str:
    h, he, cc, n, o, q = c
    if c == (0, 0, 0, 0, 0, -1):
        return "e-"
    s = ""
    for sym, cnt in (("C", cc), ("N", n), ("O", o), ("He", he), ("H", h)):
        if cnt == 1:
            s += sym
        elif cnt > 1:
            s += f"{sym}{cnt}"
    return s + ("+" * q if q > 0 else "-" * (-q))


def _make_species(n_species: int, rng: np.random.Generator,
                  surface_frac: float) -> Tuple[np.ndarray, List[str], np.ndarray]:
    """Species compositions. Returns (comp [n,6], names, is_surface)."""
    fixed = [
        (1, 0, 0, 0, 0, 0),   # H      (the heaviest row)
        (2, 0, 0, 0, 0, 0),   # H2
        (0, 0, 0, 0, 0, -1),  # e-
        (0, 1, 0, 0, 0, 0), (0, 1, 0, 0, 0, 1),   # He, He+
        (0, 0, 1, 0, 0, 0), (0, 0, 1, 0, 0, 1),   # C, C+
        (0, 0, 0, 1, 0, 0), (0, 0, 0, 1, 0, 1),   # N, N+
        (0, 0, 0, 0, 1, 0), (0, 0, 0, 0, 1, 1),   # O, O+
        (1, 0, 0, 0, 0, 1),   # H+
        (2, 0, 0, 0, 0, 1), (3, 0, 0, 0, 0, 1),   # H2+, H3+
        (1, 1, 0, 0, 0, 1),   # HeH+
    ]
    n_surface = int(round(surface_frac * n_species))
    n_gas = n_species - n_surface
    if n_gas < len(fixed) + 2:
        raise ValueError("n_species too small")
    comps: List[Tuple[int, ...]] = list(fixed)
    seen = {c: 1 for c in comps}
    while len(comps) < n_gas:
        nh = int(rng.integers(0, 5))
        nc = int(rng.integers(0, 4))
        nn = int(rng.integers(0, 3))
        no = int(rng.integers(0, 3))
        tot = nh + nc + nn + no
        if tot < 2 or tot > 7:
            continue
        base = (nh, 0, nc, nn, no)
        u = rng.random()
        charges = [0, 1] if u < 0.6 else ([0] if u < 0.85 else ([1] if u < 0.97 else [0, -1]))
        for q in charges:
            c = base + (q,)
            if len(comps) >= n_gas:
                break
            if c in seen and rng.random() > 0.05:   # rare isomers allowed
                continue
            seen[c] = seen.get(c, 0) + 1
            comps.append(c)
    comp = np.array(comps, np.int8)
    names = []
    count: Dict[Tuple[int, ...], int] = {}
    for c in comps:
        k = count.get(c, 0)
        count[c] = k + 1
        names.append(_name(c) + ("" if k == 0 else f"#{k}"))
    is_surface = np.zeros(n_gas, bool)
    if n_surface:
        # grain-surface twins: identical composition, distinct species
        neutral = [i for i in range(n_gas) if comp[i, 5] == 0 and comp[i, :5].sum() >= 1]
        pick = rng.choice(neutral, size=n_surface, replace=n_surface > len(neutral))
        comp = np.concatenate([comp, comp[pick]], 0)
        names += ["g" + names[i] + (f"@{k}" if k else "") for k, i in enumerate(pick)]
        is_surface = np.concatenate([is_surface, np.ones(n_surface, bool)])
    return comp, names, is_surface


# --------------------------------------------------------------------------
# reactions
# --------------------------------------------------------------------------

def _pick(cdf: np.ndarray, rng: np.random.Generator) -> int:
    """Index drawn with probabilities given by a cumulative distribution."""
    return min(int(np.searchsorted(cdf, rng.random() * cdf[-1], side="right")), len(cdf) - 1)


class _Decomposer:
    """Random decomposition of a composition into 1-4 existing species."""

    def __init__(self, comp: np.ndarray, weights: np.ndarray, pool: np.ndarray,
                 rng: np.random.Generator):
        self.comp = comp.astype(np.int64)
        self.rng = rng
        self.pool = pool                      # candidate species indices
        w = weights[pool] / weights[pool].sum()
        self.cdf = np.cumsum(w)
        self.by_comp: Dict[Tuple[int, ...], List[int]] = {}
        for i in pool:
            self.by_comp.setdefault(tuple(int(x) for x in comp[i]), []).append(int(i))

    def exact(self, c: np.ndarray) -> Optional[int]:
        lst = self.by_comp.get(tuple(int(x) for x in c))
        if not lst:
            return None
        return int(lst[int(self.rng.integers(len(lst)))])

    def decompose(self, total: np.ndarray, n_products: int, tries: int = 40) -> Optional[List[int]]:
        for _ in range(tries):
            rem = total.copy()
            out: List[int] = []
            ok = True
            for _k in range(n_products - 1):
                cand = self.pool[_pick(self.cdf, self.rng)]
                cc = self.comp[cand]
                if np.any(cc[:5] > rem[:5]) or (cc[:5].sum() == 0 and cc[5] == 0):
                    ok = False
                    break
                out.append(int(cand))
                rem = rem - cc
            if not ok:
                continue
            if rem[:5].sum() == 0 and rem[5] == 0:
                continue  # nothing left for the last product
            last = self.exact(rem)
            if last is None:
                continue
            out.append(last)
            return out
        return None


def _net_column(reac: List[int], prod: List[int]) -> Dict[int, int]:
    """Net species counts of one reaction (products minus reactants).

    Used only to screen generated reactions (range -2..+2, no identity); it
    is bookkeeping on integer index lists, not part of the rate arithmetic."""
    d: Dict[int, int] = {}
    for a in reac:
        d[a] = d.get(a, 0) - 1
    for p in prod:
        d[p] = d.get(p, 0) + 1
    return {k: v for k, v in d.items() if v != 0}


def make_network(n_species: int, n_reactions: int, seed: int,
                 surface_frac: float = 0.0, surface_reaction_frac: float = 0.0,
                 zipf: float = 0.95,
                 boost: Tuple[float, float, float] = (0.5, 0.6, 0.02)) -> Network:
    """Balanced synthetic network with the paper network's shape.

    surface_frac / surface_reaction_frac add grain-surface-like species
    (neutral twins of gas species) and two-body surface+surface reactions.
    """
    rng = np.random.default_rng(seed)
    comp, names, is_surface = _make_species(n_species, rng, surface_frac)
    ns = comp.shape[0]
    # Zipf-like popularity; the first three species (H, H2, e-) lead.
    rank = np.arange(ns, dtype=np.float64)
    weights = 1.0 / (rank + 1.0) ** zipf
    weights[:3] *= np.asarray(boost, np.float64)
    gas = np.flatnonzero(~is_surface)
    surf = np.flatnonzero(is_surface)
    electron = 2
    cations = np.array([i for i in gas if comp[i, 5] > 0 and i != electron])
    dec_gas = _Decomposer(comp, weights, gas, rng)
    dec_surf = _Decomposer(comp, weights, surf, rng) if len(surf) else None
    cg = np.cumsum(weights[gas])
    cc = np.cumsum(weights[cations])

    n_surf_r = int(round(surface_reaction_frac * n_reactions)) if len(surf) else 0
    n_gas_r = n_reactions - n_surf_r
    n_two = int(round(0.60 * n_gas_r))
    n_one = int(round(0.25 * n_gas_r))
    n_rec = n_gas_r - n_two - n_one

    seen = set()
    covered = np.zeros(ns, bool)
    groups: Dict[int, List[Tuple[List[int], List[int]]]] = {0: [], 1: [], 2: [], 3: []}

    def accept(rt: int, reac: List[int], prod: List[int]) -> bool:
        net = _net_column(reac, prod)
        if not net:
            return False
        if any(v < -2 or v > 2 for v in net.values()):
            return False
        key = (tuple(sorted(reac)), tuple(sorted(prod)))
        if key in seen:
            return False
        tot_r = comp[reac].astype(np.int64).sum(0)
        tot_p = comp[prod].astype(np.int64).sum(0)
        if np.any(tot_r != tot_p):
            return False
        seen.add(key)
        groups[rt].append((list(reac), list(prod)))
        covered[reac] = True
        covered[prod] = True
        return True

    def try_two(a: int, b: int, dec: _Decomposer, rt: int) -> bool:
        tot = comp[a].astype(np.int64) + comp[b].astype(np.int64)
        npro = int(rng.choice([1, 2, 2, 2, 3, 3, 4]))
        prod = dec.decompose(tot, npro)
        return prod is not None and accept(rt, [a, b], prod)

    def try_one(a: int) -> bool:
        if comp[a, :5].sum() < 1 or a == electron:
            return False
        npro = int(rng.choice([2, 2, 2, 3, 3, 4]))
        prod = dec_gas.decompose(comp[a].astype(np.int64), npro)
        return prod is not None and accept(1, [a], prod)

    def try_rec(x: int) -> bool:
        tot = comp[x].astype(np.int64) + comp[electron].astype(np.int64)
        npro = int(rng.choice([1, 2, 2, 2, 3]))
        prod = dec_gas.decompose(tot, npro)
        return prod is not None and accept(2, [x, electron], prod)

    guard = 0
    while len(groups[0]) < n_two:
        guard += 1
        if guard > 400 * n_reactions:
            raise RuntimeError("generator stalled (two-body)")
        a = int(gas[_pick(cg, rng)])
        b = int(gas[_pick(cg, rng)])
        if a == b and rng.random() > 0.15:
            continue
        try_two(a, b, dec_gas, 0)
    while len(groups[1]) < n_one:
        guard += 1
        if guard > 400 * n_reactions:
            raise RuntimeError("generator stalled (one-body)")
        # one-body destruction also covers species the two-body pass missed
        missing = [i for i in gas if not covered[i] and comp[i, :5].sum() >= 1]
        a = int(missing[0]) if missing and rng.random() < 0.7 else int(gas[_pick(cg, rng)])
        try_one(a)
    while len(groups[2]) < n_rec:
        guard += 1
        if guard > 400 * n_reactions:
            raise RuntimeError("generator stalled (recombination)")
        x = int(cations[_pick(cc, rng)])
        try_rec(x)
    if n_surf_r:
        cs = np.cumsum(weights[surf])
        while len(groups[3]) < n_surf_r:
            guard += 1
            if guard > 400 * n_reactions:
                raise RuntimeError("generator stalled (surface)")
            a = int(surf[_pick(cs, rng)])
            b = int(surf[_pick(cs, rng)])
            try_two(a, b, dec_surf, 3)

    # Species nobody touches would give empty rows; give each one a partner
    # reaction by replacing a random one-body reaction of the same group.
    for i in np.flatnonzero(~covered):
        for _ in range(200):
            if is_surface[i]:
                b = int(surf[rng.integers(len(surf))])
                if try_two(int(i), b, dec_surf, 3):
                    break
            elif comp[i, :5].sum() >= 1 and try_one(int(i)):
                break
            elif comp[i, 5] > 0 and try_rec(int(i)):
                break
        if covered[i]:
            g = 3 if is_surface[i] else 1
            groups[g].pop(int(rng.integers(len(groups[g]) - 1)))

    order = [0, 1, 2, 3]              # natural order: grouped by reaction type
    reactions = []
    rtype = []
    for g in order:
        for r in groups[g]:
            reactions.append(r)
            rtype.append(g)
    nr = len(reactions)
    alpha = 10.0 ** rng.uniform(-12.0, -8.0, nr)
    beta = rng.uniform(-1.0, 1.0, nr)
    gamma = rng.uniform(0.0, 1000.0, nr)
    net = network_from_lists(ns, reactions, alpha, beta, gamma, comp, names)
    net.rtype = np.array(rtype, np.int8)
    return net


# --------------------------------------------------------------------------
# cells
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Cells:
    T: np.ndarray       # [n_cells] K
    n_H: np.ndarray     # [n_cells] cm^-3
    y0: np.ndarray      # [n_cells, n_species] cm^-3, cell-major


def make_cells(net: Network, n_cells: int, seed: int,
               T_range=(10.0, 300.0), nH_range=(1e2, 1e7),
               x_range=(1e-12, 1.0), T: Optional[float] = None,
               n_H: Optional[float] = None) -> Cells:
    """Per-cell T, n_H and initial number densities y0 = x * n_H.

    The electron density is set so each cell is electrically neutral
    (sum of charge times density over the charged species is zero)."""
    rng = np.random.default_rng(seed + 7919)
    if T is None:
        Tv = np.exp(rng.uniform(np.log(T_range[0]), np.log(T_range[1]), n_cells))
    else:
        Tv = np.full(n_cells, float(T))
    if n_H is None:
        nh = np.exp(rng.uniform(np.log(nH_range[0]), np.log(nH_range[1]), n_cells))
    else:
        nh = np.full(n_cells, float(n_H))
    ns = net.n_species
    x = np.exp(rng.uniform(np.log(x_range[0]), np.log(x_range[1]), (n_cells, ns)))
    y0 = x * nh[:, None]
    q = net.composition[:, 5].astype(np.float64)
    electrons = np.flatnonzero((net.composition[:, :5] == 0).all(1) & (q == -1))
    if len(electrons):
        e = electrons[0]
        qq = q.copy()
        qq[e] = 0.0
        ne = y0 @ qq                     # net positive charge of the heavy species
        y0[:, e] = np.where(ne > 0, ne, y0[:, e])
    return Cells(Tv, nh, np.ascontiguousarray(y0))


# --------------------------------------------------------------------------
# rate laws by reaction type and the per-cell conditions they read
# --------------------------------------------------------------------------

# Rate-law codes: modified Arrhenius (Kooij), direct cosmic-ray ionisation,
# cosmic-ray induced photoreaction, interstellar FUV photoreaction. The
# coefficients depend on the temperature, the cosmic-ray ionisation rate and
# the FUV intensity (Sec. 3); per-cell conditions are (T, A_V, zeta/zeta_0,
# G_0).
LAW_KOOIJ, LAW_CRP, LAW_CRPHOT, LAW_PHOTO = 0, 1, 2, 3
N_COND = 4


def with_rate_laws(net: Network, seed: int) -> Network:
    """A copy of ``net`` whose one-body reactions follow the cosmic-ray and
    photo laws: 30 % direct cosmic-ray ionisation (alpha log-uniform on
    [1e-18, 1e-16] s^-1 at zeta_0), 30 % cosmic-ray induced photoreactions
    (alpha log-uniform on [5e-18, 3e-17], beta uniform on (-0.5, 0.5),
    efficiency gamma log-uniform on [10, 5000]), 40 % FUV photoreactions
    (alpha log-uniform on [1e-11, 1e-9] s^-1 at G_0 = 1, attenuation gamma
    uniform on (0.5, 3.5) per magnitude). Two-body and recombination
    reactions keep the Kooij law and their parameters."""
    rng = np.random.default_rng(seed)
    law = np.zeros(net.n_reactions, np.int8)
    alpha, beta, gamma = net.alpha.copy(), net.beta.copy(), net.gamma.copy()
    one = np.flatnonzero(net.rtype == 1)
    u = rng.uniform(size=one.size)
    crp, crph, ph = one[u < 0.3], one[(u >= 0.3) & (u < 0.6)], one[u >= 0.6]
    law[crp], law[crph], law[ph] = LAW_CRP, LAW_CRPHOT, LAW_PHOTO
    alpha[crp] = np.exp(rng.uniform(np.log(1e-18), np.log(1e-16), crp.size))
    beta[crp], gamma[crp] = 0.0, 0.0
    alpha[crph] = np.exp(rng.uniform(np.log(5e-18), np.log(3e-17), crph.size))
    beta[crph] = rng.uniform(-0.5, 0.5, crph.size)
    gamma[crph] = np.exp(rng.uniform(np.log(10.0), np.log(5000.0), crph.size))
    alpha[ph] = np.exp(rng.uniform(np.log(1e-11), np.log(1e-9), ph.size))
    beta[ph] = 0.0
    gamma[ph] = rng.uniform(0.5, 3.5, ph.size)
    return dataclasses.replace(net, alpha=alpha, beta=beta, gamma=gamma, law=law)


def make_conditions(T: np.ndarray, seed: int, Av_range=(0.1, 20.0), zeta_range=(0.1, 10.0),
                    G0_range=(0.1, 100.0)) -> np.ndarray:
    """Per-cell conditions [n_cells, 4] = (T, A_V, zeta/zeta_0, G_0) around
    given temperatures, the other three log-uniform on their ranges."""
    rng = np.random.default_rng(seed + 104729)
    n = len(T)
    out = np.empty((n, N_COND))
    out[:, 0] = T
    out[:, 1] = np.exp(rng.uniform(np.log(Av_range[0]), np.log(Av_range[1]), n))
    out[:, 2] = np.exp(rng.uniform(np.log(zeta_range[0]), np.log(zeta_range[1]), n))
    out[:, 3] = np.exp(rng.uniform(np.log(G0_range[0]), np.log(G0_range[1]), n))
    return out


# --------------------------------------------------------------------------
# temperature as a state: reaction heats and per-cell thermal parameters
# --------------------------------------------------------------------------

K_BOLTZMANN = 1.380649e-16   # erg / K


def species_enthalpies(n_species: int, seed: int, scale_K: float = 50.0) -> np.ndarray:
    """Seeded per-species energies h_i = k_B theta_i with theta_i uniform on
    (-scale_K, scale_K) K [erg]. Reaction heats built from them conserve
    c_v T + sum_i h_i n_i exactly when nothing else heats or cools."""
    rng = np.random.default_rng(seed + 3571)
    return K_BOLTZMANN * rng.uniform(-scale_K, scale_K, n_species)


def with_heat(net: Network, h: np.ndarray) -> Network:
    """A copy of ``net`` whose reaction j releases heat_j = sum over its
    reactants of h minus the sum over its products (erg per event, the
    reaction's energy balance for species energies h)."""
    heat = np.zeros(net.n_reactions)
    for j in range(net.n_reactions):
        heat[j] = sum(h[a] for a in net.reactants[j] if a >= 0) - \
            sum(h[p] for p in net.products[j] if p >= 0)
    return dataclasses.replace(net, heat=heat)


def thermal_params(n_H: np.ndarray, T0: np.ndarray, lam: float = 1e-11) -> np.ndarray:
    """Per-cell (c_v, T_b, lambda): the heat capacity of an ideal monatomic
    gas of density n_H (1.5 k_B n_H), the background temperature T0 the gas
    relaxes to, and the relaxation rate lambda [1/s]."""
    return np.stack([1.5 * K_BOLTZMANN * np.asarray(n_H, np.float64), np.asarray(T0, np.float64),
                     np.full(len(T0), float(lam))], 1)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def workload(name: str, n_cells: Optional[int] = None):
    """The synthetic workloads used by tests and the benchmark.

    tiny   : 50 species / 300 reactions, one cell at T=20 K, n_H=1e4
    medium : 470 species / 4600 reactions (the paper-sized network)
    large  : 700 species / 8000 reactions with 20 % grain-surface terms
    """
    if name == "tiny":
        net = make_network(50, 300, SEED_BASE + 0)
        cells = make_cells(net, n_cells or 1, SEED_BASE + 0, T=20.0, n_H=1e4)
    elif name == "medium":
        net = make_network(470, 4600, SEED_BASE + 1)
        cells = make_cells(net, n_cells or 65536, SEED_BASE + 1)
    elif name == "large":
        net = make_network(700, 8000, SEED_BASE + 4, surface_frac=0.2,
                           surface_reaction_frac=0.2)
        cells = make_cells(net, n_cells or 262144, SEED_BASE + 4)
    else:
        raise KeyError(name)
    return net, cells

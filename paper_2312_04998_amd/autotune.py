"""Autotuner for the chemistry kernels' launch shape and the integrator's
slot count, with results cached as JSON.

The RHS and Jacobian kernels take three build-time choices: the storage
layout of S (CRS chunks, SELL-C-sigma, equal runs, COO, CCS), the species
traversal order (natural, nnz-descending, reverse Cuthill-McKee) and the
workgroup size (256, 512 or 1024 threads). The workgroup size only matters
for the one-cell kernels: with SELL the fused RHS + Jacobian call runs the
two-cells-per-pass kernel, whose 1024-thread workgroup is fixed, so SELL is
tried at one size only. Which combination is fastest depends on the
network's shape and on the cell count, so `autotune` times every candidate
on the caller's own cells (ac_rhs_jac, the RHS and the Jacobian together,
HIP events on the current stream).

The batched integrator takes one run-time choice, the number of workgroup
slots of its workspace: more slots integrate more cells at once, fewer keep
the slots' LU factors (n^2 doubles each) within the last-level cache.
`tune_slots` times a short integration of a sample of cells for each
candidate.

Results are stored in a JSON file keyed by the GPU architecture, a digest
of the loaded library, the network (shape and a digest of its reaction
data) and the cell count rounded up to a power of two; a later call with
the same key reads the choice instead of timing again.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import math
import os
import time
from typing import Dict, Iterable, Optional, Tuple

import numpy as np

from . import LIB_PATH, Network, Workspace, ac_rhs, ac_rhs_jac

LAYOUTS = ("sell", "csr", "runs", "coo", "ccs")
ORDERINGS = ("nnz", "natural", "rcm")
BLOCKS = (512, 256, 1024)
SLOTS = (128, 192, 256)
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")

_lib_digest: Optional[str] = None


def _library_digest() -> str:
    global _lib_digest
    if _lib_digest is None:
        with open(LIB_PATH, "rb") as f:
            _lib_digest = hashlib.sha1(f.read()).hexdigest()[:16]
    return _lib_digest


def _net_digest(net) -> str:
    h = hashlib.sha1()
    for a in (net.reactants, net.products, net.alpha, net.beta, net.gamma):
        h.update(np.ascontiguousarray(a).tobytes())
    for a in (getattr(net, "law", None), getattr(net, "heat", None)):
        if a is not None:
            h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


def cache_key(kind: str, net, n_cells: int) -> str:
    """arch | library digest | network shape and digest | cell-count bucket."""
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    bucket = 1 << max(0, math.ceil(math.log2(max(1, n_cells))))
    return (f"{kind}|{arch}|lib={_library_digest()}|ns={net.n_species}|nr={net.n_reactions}|"
            f"net={_net_digest(net)}|cells<={bucket}")


def _load(path: Optional[str]) -> dict:
    if not path or not os.path.exists(path):
        return {}
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path: Optional[str], key: str, entry: dict) -> None:
    if not path:
        return
    data = _load(path)
    data[key] = entry
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_ms(torch, fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def candidates(layouts: Iterable[str] = LAYOUTS, orderings: Iterable[str] = ORDERINGS,
               blocks: Iterable[int] = BLOCKS):
    """(layout, ordering, block) triples worth timing: SELL at one block size
    (its fused kernel does not use the block), every size otherwise."""
    blocks = tuple(blocks)
    for lay, order in itertools.product(layouts, orderings):
        for blk in ((blocks[0],) if lay == "sell" else blocks):
            yield lay, order, blk


def autotune(net, y, T, layouts: Iterable[str] = LAYOUTS, orderings: Iterable[str] = ORDERINGS,
             blocks: Iterable[int] = BLOCKS, reps: int = 3, with_jac: bool = True,
             cache: Optional[str] = DEFAULT_CACHE
             ) -> Tuple[Network, Dict[str, object], Dict[Tuple[str, str, int], float]]:
    """Times ac_rhs_jac (ac_rhs alone without with_jac) for every candidate
    (layout, ordering, block) on the device tensors y [cells, ns] and T
    [cells] (or [cells, n_cond]); returns (network built with the fastest
    choice, its keyword arguments plus "cached": whether the choice came from
    the cache, table of ms per step). cache: JSON file path, or None to
    always time."""
    import torch

    kind = "rhs_jac" if with_jac else "rhs"
    key = cache_key(kind, net, int(y.shape[0]))
    hit = _load(cache).get(key)
    if hit is not None:
        kw = {k: hit[k] for k in ("layout", "ordering", "block")}
        table = {tuple(k.split("/")[:2]) + (int(k.split("/")[2]),): v
                 for k, v in hit.get("table_ms", {}).items()}
        return Network.from_synth(net, **kw), dict(kw, cached=True), table

    dydt = torch.empty_like(y)
    table: Dict[Tuple[str, str, int], float] = {}
    jv = None
    for lay, order, blk in candidates(layouts, orderings, blocks):
        N = Network.from_synth(net, layout=lay, ordering=order, block=blk)
        if with_jac and jv is None:
            jv = torch.empty((y.shape[0], N.nnz_j), dtype=torch.float64, device=y.device)

        def step():
            if with_jac:
                ac_rhs_jac(N, None, y, T, dydt, jv)
            else:
                ac_rhs(N, None, y, T, dydt)

        table[(lay, order, blk)] = _time_ms(torch, step, reps)
        N.close()
    best = min(table, key=table.get)
    kw = {"layout": best[0], "ordering": best[1], "block": best[2]}
    _store(cache, key, dict(kw, table_ms={f"{l}/{o}/{b}": round(ms, 5)
                                          for (l, o, b), ms in table.items()},
                            tuned_at=time.strftime("%Y-%m-%d %H:%M:%S")))
    return Network.from_synth(net, **kw), dict(kw, cached=False), table


def tune_slots(net, y0, T, t_end: float, max_steps: int = 200, slots: Iterable[int] = SLOTS,
               cache: Optional[str] = DEFAULT_CACHE) -> Tuple[int, Dict[int, float], bool]:
    """Integrated steps per second of the batched integrator on the cells
    y0 [cells, ns], T (device) for each slot count, every cell capped at
    max_steps accepted steps; returns (fastest slot count, steps/s per
    count, whether it came from the cache)."""
    import torch

    key = cache_key(f"slots|steps={max_steps}", net, int(y0.shape[0]))
    hit = _load(cache).get(key)
    if hit is not None:
        return int(hit["slots"]), {int(k): v for k, v in hit.get("steps_per_s", {}).items()}, True
    N = Network.from_synth(net)
    rate: Dict[int, float] = {}
    for s in slots:
        ws = Workspace(N, n_slots=int(s))
        y = y0.clone()
        ws.integrate(y, T, t_end, max_steps=max_steps)   # warm-up (first launch)
        y = y0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = ws.integrate(y, T, t_end, max_steps=max_steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        rate[int(s)] = float(out["stats"][:, 0].sum().item()) / wall
        ws.close()
    N.close()
    best = max(rate, key=rate.get)
    _store(cache, key, {"slots": best, "steps_per_s": {str(k): round(v, 1) for k, v in rate.items()},
                        "tuned_at": time.strftime("%Y-%m-%d %H:%M:%S")})
    return best, rate, False

"""Autotuner for the chemistry kernels' launch shape.

The RHS and Jacobian kernels take three build-time choices: the storage
layout of S (CRS chunks, SELL-C-sigma, equal runs, COO, CCS), the species
traversal order (natural, nnz-descending, reverse Cuthill-McKee) and the
workgroup size (256, 512 or 1024 threads). Which combination is fastest
depends on the network's shape and on the cell count, so `autotune` times
every candidate on the caller's own cells (ac_rhs_jac, the RHS and the
Jacobian together, HIP events on the current stream) and returns the network built with the winner.
"""
from __future__ import annotations

import itertools
from typing import Dict, Iterable, Tuple

from . import Network, ac_rhs, ac_rhs_jac

LAYOUTS = ("sell", "csr", "runs", "coo", "ccs")
ORDERINGS = ("nnz", "natural", "rcm")
BLOCKS = (512, 256, 1024)


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


def autotune(net, y, T, layouts: Iterable[str] = LAYOUTS, orderings: Iterable[str] = ORDERINGS,
             blocks: Iterable[int] = BLOCKS, reps: int = 3, with_jac: bool = True
             ) -> Tuple[Network, Dict[str, object], Dict[Tuple[str, str, int], float]]:
    """Times ac_rhs_jac (ac_rhs alone without with_jac) for every (layout, ordering, block) on the
    device tensors y [cells, ns] and T [cells]; returns (network built with
    the fastest choice, its keyword arguments, table of ms per step)."""
    import torch

    dydt = torch.empty_like(y)
    table: Dict[Tuple[str, str, int], float] = {}
    jv = None
    for lay, order, blk in itertools.product(layouts, orderings, blocks):
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
    return Network.from_synth(net, **kw), kw, table

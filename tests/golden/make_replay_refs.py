"""Writes tests/golden/replay_medium_cfg3.npz: oracle reference values for
the strict replay and adjoint-entry tests on the 470-species / 4600-reaction
network (the first 8 of the 16,384 cells of the batched-integration
workload, BDF 1-5 to 1e6 yr, rtol 1e-6, atol 1e-20).

Calls only the oracle (and the seeded input generator):

1. oracle.bdf records each cell's step sequence (the tape);
2. oracle.bdf_replay replays that tape with converged correctors and
   propagates forward sensitivities along 64 unit directions per cell
   (32 initial densities, 32 log rate prefactors);
3. the loss is L_c = sum of log y_t(t_end) over 8 seeded target species per
   cell with y_t(t_end) > 1e-20, so lambda_c = 1 / y_t on the targets; for
   each direction the file keeps <lambda_c, s> and the scale sum |lambda_c s|.

    python tests/golden/make_replay_refs.py       (about 6 minutes on 8 threads)
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synthnet  # noqa: E402

OUT = os.path.join(HERE, "replay_medium_cfg3.npz")
YEAR_S = 3.15576e7
N_CELLS_WORKLOAD = 16384
CELLS = np.arange(8)
T_END = 1e6 * YEAR_S
N_Y_DIR, N_A_DIR = 32, 32
TAPE_CAP = 40000


def inputs():
    net, _ = synthnet.workload("medium", n_cells=1)
    cells = synthnet.make_cells(net, N_CELLS_WORKLOAD, synthnet.SEED_BASE + 2)
    return net, cells.y0[CELLS].copy(), cells.T[CELLS].copy()


def input_digest(y0, T) -> str:
    return hashlib.sha256(np.ascontiguousarray(y0).tobytes() + np.ascontiguousarray(T).tobytes()).hexdigest()


def directions(net):
    rng = np.random.default_rng(2312)
    ya = np.sort(rng.choice(net.n_species, N_Y_DIR, replace=False))
    aj = np.sort(rng.choice(net.n_reactions, N_A_DIR, replace=False))
    return ya, aj


def main():
    oracle.set_threads(min(16, os.cpu_count() or 1))
    net, y0, T = inputs()
    n, ns, nr = len(CELLS), net.n_species, net.n_reactions
    t0 = time.time()
    ref = oracle.bdf(net, y0, T, T_END, tape_cap=TAPE_CAP)
    assert (ref["status"] == 0).all() and (ref["tape_len"] > 0).all(), ref["status"]
    print(f"bdf: {time.time() - t0:.1f} s, steps {ref['stats'][:, 0].tolist()}", flush=True)
    L = int(ref["tape_len"].max())
    tape = ref["tape"][:, :L].copy()
    # targets and lambda
    rng = np.random.default_rng(8)
    lam = np.zeros_like(y0)
    targets = np.zeros((n, 8), np.int32)
    for c in range(n):
        ok = np.flatnonzero(ref["y"][c] > 1e-20)
        targets[c] = np.sort(rng.choice(ok, 8, replace=False))
        lam[c, targets[c]] = 1.0 / ref["y"][c, targets[c]]
    ya, aj = directions(net)
    nd = N_Y_DIR + N_A_DIR
    dy0 = np.zeros((n, nd, ns))
    dla = np.zeros((nd, nr))
    for r, a in enumerate(ya):
        dy0[:, r, a] = 1.0
    for r, j in enumerate(aj):
        dla[N_Y_DIR + r, j] = 1.0
    t0 = time.time()
    y_rep, s = oracle.bdf_replay(net, y0, T, tape, ref["tape_len"], dy0=dy0, dlogalpha=dla,
                                 n_dir=nd)
    print(f"replay with {nd} tangents: {time.time() - t0:.1f} s", flush=True)
    proj = np.einsum("ci,cri->cr", lam, s)
    scale = np.einsum("ci,cri->cr", np.abs(lam), np.abs(s))
    np.savez_compressed(
        OUT, cells=CELLS, input_sha256=np.array(input_digest(y0, T)), t_end=T_END,
        tape_type=tape["type"].astype(np.int8), tape_q=tape["q"].astype(np.int8),
        tape_val=tape["val"], tape_len=ref["tape_len"], y_bdf=ref["y"], steps=ref["stats"][:, 0],
        y_replay=y_rep, targets=targets, lam=lam, dir_species=ya, dir_reaction=aj, proj=proj,
        scale=scale)
    print(f"wrote {OUT} ({os.path.getsize(OUT) / 1024:.0f} KB)")


if __name__ == "__main__":
    main()

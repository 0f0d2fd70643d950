"""Benchmark of the stoichiometry-matrix chemistry hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the paper-sized synthetic network (470 species, 4600 reactions,
shaped like UMIST rate12 of Sec. 3) on 65,536 cells with T log-uniform on
10-300 K and n_H log-uniform on 1e2-1e7 cm^-3, FP64, inputs resident in
HBM before timing. A step evaluates dn/dt = S R(n, T) and the Jacobian for
every cell (fused rate coefficients). Two further legs run on bounded
samples of the same cells: batched BDF integration to 1e6 yr at rtol 1e-6
against the plain one-cell-at-a-time loop, and the discrete adjoint.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector and matrix, published
YEAR_S = 3.15576e7


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--cells", type=int, default=65536)
    p.add_argument("--layout", default="auto", help="sell|csr|runs|coo, or auto (autotuned)")
    p.add_argument("--ordering", default="auto", help="nnz|natural|rcm, or auto (autotuned)")
    p.add_argument("--block", type=int, default=0, help="threads per workgroup (0 = autotuned)")
    p.add_argument("--no-table", action="store_true",
                   help="skip the autotuner (layout x ordering x block table); use sell/nnz/512")
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--no-int", action="store_true", help="skip the integration legs")
    p.add_argument("--int-cells", type=int, default=2048, help="cells of the batched integration leg")
    p.add_argument("--int-max-steps", type=int, default=20000)
    p.add_argument("--plain-cells", type=int, default=2, help="cells timed through the plain loop")
    p.add_argument("--adj-cells", type=int, default=256)
    p.add_argument("--adj-max-steps", type=int, default=1500)
    p.add_argument("--copy-probe", action="store_true",
                   help="also run a plain device copy of the densities (known bytes) so HBM "
                        "counters can be calibrated in the same profile")
    return p.parse_args()


class Timer:
    """HIP events around launches on torch's current stream (the stream the
    library launches on), averaged per kernel name."""

    def __init__(self, torch):
        self.torch = torch
        self.ev = {}

    def run(self, name, fn):
        t = self.torch
        a, b = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        self.ev.setdefault(name, []).append((a, b))

    def mean_ms(self, name):
        return float(np.mean([a.elapsed_time(b) for a, b in self.ev[name]]))


def cpu_baseline(net, cells, seconds):
    """The oracle (plain C, FP64, OpenMP over cells) on a bounded sample."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = max(1, min(threads, os.cpu_count() or 1))
    oracle.set_threads(threads)
    # size the sample from a short probe so the run takes about `seconds`
    probe = min(64, cells.T.size)
    t0 = time.perf_counter()
    oracle.rhs(net, cells.y0[:probe], cells.T[:probe])
    oracle.jac_dense(net, cells.y0[:probe], cells.T[:probe])
    dt = max(time.perf_counter() - t0, 1e-6)
    n = int(min(cells.T.size, max(probe, probe * seconds / dt)))
    # whole passes over the sample until about `seconds` have elapsed
    t0 = time.perf_counter()
    passes = 0
    while True:
        for s in range(0, n, 256):
            e = min(n, s + 256)
            oracle.rhs(net, cells.y0[s:e], cells.T[s:e])
            oracle.jac_dense(net, cells.y0[s:e], cells.T[s:e])
        passes += 1
        dt = time.perf_counter() - t0
        if dt >= seconds or n < cells.T.size:
            break
    return {"value": passes * n * net.n_reactions / dt, "unit": "cell-reactions/s",
            "cores": threads, "kind": "oracle",
            "sample": f"RHS + dense Jacobian of the first {n} of the {cells.T.size} cells, "
                      f"{passes} pass(es) in {dt:.1f} s on {threads} threads"}


# Sources that make up the fused RHS + Jacobian kernel: the HBM traffic
# recorded under profiles/ is used only while they are unchanged.
JAC_SOURCES = ("paper_2312_04998_amd/csrc/kernels_chem.hip", "paper_2312_04998_amd/csrc/devchem.h",
               "paper_2312_04998_amd/csrc/devnet.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_rhs_jac2_470x4600_65536_hbm_traffic.md")


def jac_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in JAC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(cells, nnz_j):
    """HBM bytes per k_rhs_jac2 launch from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated on a copy of known size),
    or None when the summary is missing, was taken on another workload, or
    the kernel's sources changed since. (The two-cells-per-pass kernel
    always runs 1024-thread workgroups, whatever the network's workgroup
    size.)"""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            kv[k.strip()] = v.strip().strip("`")
    try:
        if (int(kv["cells"]) != cells or int(kv["nnz_j"]) != nnz_j
                or kv["kernel_source_sha256"] != jac_source_digest()):
            return None
        return int(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def lu_leg(torch, acm, net, cells, n_mat=256):
    """Batched dense LU and solves of Newton matrices I - c J (470 x 470,
    one matrix per workgroup), the integrator's linear algebra in
    isolation: 2n^3/3 flops per factorisation against the FP64 matrix-core
    peak, n^2 doubles read per solve against HBM."""
    dev = torch.device("cuda:0")
    N = acm.Network.from_synth(net)
    ns = net.n_species
    y = torch.from_numpy(cells.y0[:n_mat].copy()).to(dev)
    T = torch.from_numpy(cells.T[:n_mat].copy()).to(dev)
    jv = N.jac(y, T)
    rp, col = N.jac_pattern()
    rows = torch.from_numpy(np.repeat(np.arange(ns), np.diff(rp))).to(dev)
    cols = torch.from_numpy(col.astype(np.int64)).to(dev)
    lda = (ns + 15) // 16 * 16
    A0 = torch.zeros((n_mat, ns, lda), dtype=torch.float64, device=dev)
    A0[:, torch.arange(ns, device=dev), torch.arange(ns, device=dev)] = 1.0
    A0[:, rows, cols] -= 1e7 * jv
    piv = torch.empty((n_mat, ns), dtype=torch.int32, device=dev)
    b = torch.randn((n_mat, ns), dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(1))
    A = A0.clone()
    acm.ac_lu_factor(A, piv)
    acm.ac_lu_solve(A, piv, b.clone())
    torch.cuda.synchronize()
    tm = Timer(torch)
    for _ in range(3):
        A.copy_(A0)
        tm.run("lu", lambda: acm.ac_lu_factor(A, piv))
        bb = b.clone()
        tm.run("solve", lambda: acm.ac_lu_solve(A, piv, bb))
    torch.cuda.synchronize()
    lu_ms, sv_ms = tm.mean_ms("lu"), tm.mean_ms("solve")
    flops = n_mat * 2.0 * ns ** 3 / 3.0
    sbytes = n_mat * 8.0 * ns * ns
    return {"lu": {"matrices": n_mat, "n": ns, "c": 1e7, "ms": lu_ms,
                   "TFLOPs": flops / (lu_ms * 1e-3) / 1e12,
                   "mfma_frac": flops / (lu_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                   "solve_ms": sv_ms, "solve_GBps": sbytes / (sv_ms * 1e-3) / 1e9,
                   "solve_hbm_frac": sbytes / (sv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}}


def integration_legs(args, torch, acm, net, cells):
    """Batched BDF (one persistent workgroup per slot, device cell queue)
    on the first --int-cells cells against the plain per-cell loop timed on
    the first --plain-cells of them; then the discrete adjoint of a shorter
    run on --adj-cells cells. Wall-clock timing (synchronised)."""
    dev = torch.device("cuda:0")
    N = acm.Network.from_synth(net)
    ws = acm.Workspace(N)
    t_end = 1e6 * YEAR_S
    res = {}
    n = min(args.int_cells, cells.T.size)
    y = torch.from_numpy(cells.y0[:n].copy()).to(dev)
    T = torch.from_numpy(cells.T[:n].copy()).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = ws.integrate(y, T, t_end, max_steps=args.int_max_steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = out["stats"].cpu().numpy()
    status = out["status"].cpu().numpy()
    steps = int(st[:, 0].sum())
    ok = int((status == 0).sum())
    print(f"[bench] batched integration: {n} cells in {wall:.1f} s", file=sys.stderr, flush=True)
    npl = min(args.plain_cells, n)
    yp = torch.from_numpy(cells.y0[:npl].copy()).to(dev)
    Tp = torch.from_numpy(cells.T[:npl].copy()).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outp = ws.integrate(yp, Tp, t_end, max_steps=args.int_max_steps, plain=True)
    torch.cuda.synchronize()
    wall_p = time.perf_counter() - t0
    steps_p = int(outp["stats"].cpu().numpy()[:, 0].sum())
    plain_sps = steps_p / wall_p
    plain_wall_est = steps / plain_sps
    print(f"[bench] plain integration: {npl} cells in {wall_p:.1f} s", file=sys.stderr, flush=True)
    res["integration"] = {
        "workload": f"470/4600 network, first {n} of the {cells.T.size} cells, BDF 1-5 to 1e6 yr, "
                    f"rtol 1e-6, atol 1e-20, max_steps {args.int_max_steps}",
        "cells": n, "wall_s": wall, "cells_reaching_t_end": ok,
        "cells_maxsteps": int((status == 1).sum()),
        "integrated_cells_per_s": ok / wall,
        "steps": steps, "steps_per_s": steps / wall,
        "step_quantiles_10_50_90_max": np.quantile(st[:, 0], [0.1, 0.5, 0.9, 1.0]).tolist(),
        "newton_iters_per_step": float(st[:, 3].sum() / max(steps, 1)),
        "lu_per_step": float(st[:, 5].sum() / max(steps, 1)),
        "slots": ws.n_slots,
        "plain": {"cells": npl, "wall_s": wall_p, "steps": steps_p, "steps_per_s": plain_sps,
                  "est_wall_s_same_cells": plain_wall_est,
                  "est_integrated_cells_per_s": ok / plain_wall_est,
                  "note": "plain = one cell per launch through the same kernel; its time for "
                          "the batched sample is estimated from its measured steps/s times the "
                          "sample's step count"},
        "vs_plain": plain_wall_est / wall,
    }
    # discrete adjoint: forward with tape, then the timed adjoint sweep
    na = min(args.adj_cells, cells.T.size)
    ya = torch.from_numpy(cells.y0[:na].copy()).to(dev)
    Ta = torch.from_numpy(cells.T[:na].copy()).to(dev)
    cap = 2 * args.adj_max_steps + 64
    fw = ws.integrate(ya, Ta, t_end, max_steps=args.adj_max_steps, tape_cap=cap)
    rng = np.random.default_rng(8)
    tgt = rng.choice(net.n_species, 8, replace=False)
    lam = torch.zeros_like(ya)
    lam[:, tgt] = 1.0 / ya[:, tgt].clamp_min(1e-30)
    y0a = torch.from_numpy(cells.y0[:na].copy()).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    adj = ws.adjoint(y0a, Ta, fw["tape"], fw["tape_len"], lam)
    torch.cuda.synchronize()
    wall_a = time.perf_counter() - t0
    sa = int(fw["stats"].cpu().numpy()[:, 0].sum())
    ast_ = adj["stats"].cpu().numpy()
    print(f"[bench] adjoint: {na} cells in {wall_a:.1f} s", file=sys.stderr, flush=True)
    res["adjoint"] = {
        "workload": f"470/4600 network, first {na} cells, d sum log y_t / d (log alpha, y0) for 8 "
                    f"seeded targets through BDF capped at {args.adj_max_steps} steps per cell "
                    f"(t_end 1e6 yr), checkpoints every 64 steps",
        "cells": na, "wall_s": wall_a, "cells_per_s": na / wall_a, "steps": sa,
        "adjoint_steps_per_s": sa / wall_a,
        "status_ok": int((adj["status"] == 0).sum().item()),
        "per_step": {"replay_newton_iters": float(ast_[:, 3].sum() / max(sa, 1)),
                     "jacobians": float(ast_[:, 4].sum() / max(sa, 1)),
                     "factorisations": float(ast_[:, 5].sum() / max(sa, 1)),
                     "rhs": float(ast_[:, 6].sum() / max(sa, 1))},
    }
    ws.close()
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (cells would "
              "shard across GPUs with no communication).", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    import synthnet
    import paper_2312_04998_amd as acm

    net, cells = synthnet.workload("medium", n_cells=args.cells)
    ns, nr = net.n_species, net.n_reactions
    dev = torch.device("cuda:0")
    y = torch.from_numpy(cells.y0).to(dev)
    T = torch.from_numpy(cells.T).to(dev)
    tune_table = {}
    if args.no_table:
        cfg = {"layout": "sell", "ordering": "nnz", "block": 512}
    else:
        from paper_2312_04998_amd.autotune import autotune
        N, cfg, tab = autotune(net, y, T)
        N.close()
        tune_table = {f"{l}/{o}/{b}": round(ms, 4) for (l, o, b), ms in sorted(tab.items(), key=lambda kv: kv[1])}
    if args.layout != "auto":
        cfg["layout"] = args.layout
    if args.ordering != "auto":
        cfg["ordering"] = args.ordering
    if args.block:
        cfg["block"] = args.block
    N = acm.Network.from_synth(net, **cfg)
    dydt = torch.empty_like(y)
    jv = torch.empty((args.cells, N.nnz_j), dtype=torch.float64, device=dev)
    k = torch.empty((args.cells, nr), dtype=torch.float64, device=dev)
    v = torch.randn(y.shape, dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(0))
    gy = torch.empty_like(y)
    gl = torch.empty(nr, dtype=torch.float64, device=dev)

    tm = Timer(torch)

    def step():
        tm.run("rhs_jac", lambda: acm.ac_rhs_jac(N, None, y, T, dydt, jv))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    tm.ev.clear()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps

    if args.copy_probe:
        # a copy of known size: reads and writes C * ns * 8 bytes once each
        ycopy = torch.empty_like(y)
        for _ in range(3):
            ycopy.copy_(y)
        torch.cuda.synchronize()
        del ycopy

    # achievable write rate for the Jacobian's traffic (almost all writes):
    # a plain fill of the same output buffer, timed the same way after two
    # untimed fills
    for _ in range(2):
        jv.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(5):
        tm.run("fill", lambda: jv.fill_(1.0))
    torch.cuda.synchronize()

    # the separate RHS and Jacobian calls and the other chemistry kernels of
    # the path, timed the same way
    for _ in range(5):
        tm.run("rhs", lambda: acm.ac_rhs(N, None, y, T, dydt))
        tm.run("jac", lambda: acm.ac_jac(N, None, y, T, jv))
    for _ in range(2):
        acm.ac_rates(N, None, T, k)
        acm.ac_rhs_k(N, k, y, dydt)
        acm.ac_vjp(N, None, y, T, v, gy, gl)
    torch.cuda.synchronize()
    for _ in range(5):
        tm.run("rates", lambda: acm.ac_rates(N, None, T, k))
        tm.run("rhs_k", lambda: acm.ac_rhs_k(N, k, y, dydt))
        tm.run("vjp", lambda: acm.ac_vjp(N, None, y, T, v, gy, gl))
    torch.cuda.synchronize()

    C = args.cells
    kern = {}
    # algorithmic bytes per launch: every input read once, every output written once
    bytes_of = {
        "rhs_jac": C * (8 * ns + 8 + 8 * ns + 8 * N.nnz_j),
        "rhs": C * (8 * ns * 2 + 8),
        "jac": C * (8 * ns + 8 + 8 * N.nnz_j),
        "rates": C * (8 + 8 * nr),
        "rhs_k": C * (8 * nr + 16 * ns),
        "vjp": C * (8 * ns * 3 + 8) + 8 * nr,
    }
    for name in ("rhs_jac", "rhs", "jac", "rates", "rhs_k", "vjp"):
        ms = tm.mean_ms(name)
        kern[name] = {"ms": round(ms, 4), "cell_reactions_per_s": C * nr / (ms * 1e-3),
                      "GBps": bytes_of[name] / (ms * 1e-3) / 1e9,
                      "hbm_frac": bytes_of[name] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}

    fused_ms = kern["rhs_jac"]["ms"]
    achieved = bytes_of["rhs_jac"] / (fused_ms * 1e-3) / 1e9
    fill_gbs = C * N.nnz_j * 8 / (tm.mean_ms("fill") * 1e-3) / 1e9
    traffic = measured_traffic(C, N.nnz_j)
    out = {
        "metric": "RHS evals (cells×reactions)/s + integrated cells/s at rtol 1e-6 vs plain",
        "value": C * nr / (ms_step * 1e-3),
        "unit": "cell-reactions/s (RHS + Jacobian per step)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "470 species / 4600 reactions, 65,536 cells, RHS + Jacobian "
                               "(one ac_rhs_jac call)",
                   "n_species": ns, "n_reactions": nr, "cells": C, "nnz_s": N.nnz_s,
                   "nnz_j": N.nnz_j, "layout": cfg["layout"], "ordering": cfg["ordering"],
                   "block": cfg["block"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "k_rhs_jac2",
                     "bytes_per_launch": bytes_of["rhs_jac"], "avg_ms": fused_ms,
                     "achievable_write_GBps": fill_gbs, "frac_of_achievable": achieved / fill_gbs,
                     "jacobian_alone": {"kernel": "k_jac2", "avg_ms": kern["jac"]["ms"],
                                        "achieved": kern["jac"]["GBps"],
                                        "frac": kern["jac"]["hbm_frac"]}},
        "kernels": kern,
        "autotune_ms_per_step": tune_table,
    }
    if not args.no_int:
        out.update(lu_leg(torch, acm, net, cells))
        out.update(integration_legs(args, torch, acm, net, cells))
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(net, cells, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

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
    p.add_argument("--cpu-seconds", type=float, default=20.0,
                   help="about this many seconds per thread setting (five repeats)")
    p.add_argument("--no-int", action="store_true", help="skip the integration legs")
    p.add_argument("--int-cells", type=int, default=16384,
                   help="cells of the batched integration leg (the 16,384-cell workload)")
    p.add_argument("--int-max-steps", type=int, default=20000,
                   help="accepted-step budget per cell (batched and plain alike)")
    p.add_argument("--int-chunks", type=int, default=8,
                   help="launches the batched leg is split into (two streams, so a chunk's "
                        "slots are taken over by the next chunk's cells as they free up)")
    p.add_argument("--plain-cells", type=int, default=64, help="cells timed through the plain loop")
    p.add_argument("--adj-cells", type=int, default=256,
                   help="cells of the adjoint leg (first cells of the 4,096-cell workload)")
    p.add_argument("--adj-max-steps", type=int, default=20000)
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


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(net, cells, seconds, pattern):
    """The oracle (plain C, FP64, OpenMP over cells) computing what one GPU
    step computes: the RHS and the Jacobian's values on the same pattern
    (nnz_j entries per cell), on a bounded sample of the same cells. Five
    timed repeats on one thread and on every host thread; value = the
    all-thread mean."""
    import oracle
    rp, col = pattern
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = max(1, min(threads, os.cpu_count() or 1))

    def one_pass(n):
        for s in range(0, n, 512):
            e = min(n, s + 512)
            oracle.rhs(net, cells.y0[s:e], cells.T[s:e])
            oracle.jac_pattern(net, cells.y0[s:e], cells.T[s:e], rp, col)

    res = {}
    for label, th in (("1_thread", 1), ("all_threads", threads)):
        oracle.set_threads(th)
        probe = min(64 * th, cells.T.size)
        t0 = time.perf_counter()
        one_pass(probe)
        dt = max(time.perf_counter() - t0, 1e-6)
        # five repeats of about seconds / 10 each
        n = int(min(cells.T.size, max(probe, probe * seconds / 10 / dt)))
        rates = []
        for _ in range(5):
            t0 = time.perf_counter()
            one_pass(n)
            rates.append(n * net.n_reactions / (time.perf_counter() - t0))
        r = np.array(rates)
        res[label] = {"threads": th, "cells": n, "mean": float(r.mean()),
                      "se": float(r.std(ddof=1) / np.sqrt(len(r)))}
    a = res["all_threads"]
    return {"value": a["mean"], "unit": "cell-reactions/s", "cores": threads, "kind": "oracle",
            "sample": f"RHS + Jacobian on the GPU's pattern ({len(col)} values per cell) of the "
                      f"first {a['cells']} of the {cells.T.size} cells, 5 timed repeats on "
                      f"{threads} threads (mean {a['mean']:.3e} +- {a['se']:.1e} SE); one "
                      f"thread: first {res['1_thread']['cells']} cells, "
                      f"{res['1_thread']['mean']:.3e} +- {res['1_thread']['se']:.1e}",
            "cpu_model": _cpu_model(), "host_threads": os.cpu_count(),
            "one_thread": res["1_thread"], "all_threads": a}


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


def _integrate_chunked(torch, acm, wss, y, T, t_end, max_steps, nch, label):
    """Batched integration of every cell, split into nch launches issued
    back to back alternately on two streams with a workspace each: the
    persistent workgroups of a chunk take cells from its own queue and a
    later chunk's workgroups start on the compute units the earlier ones
    free, so the split costs no idle tail. Prints a line as each chunk
    completes. Returns (wall seconds, stats, status)."""
    C = y.shape[0]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs, evs = [], []
    for k in range(nch):
        s = slice(k * C // nch, (k + 1) * C // nch)
        st = streams[k % 2]
        with torch.cuda.stream(st):
            o = wss[k % 2].integrate(y[s], T[s], t_end, max_steps=max_steps, stream=st.cuda_stream)
            e = torch.cuda.Event()
            e.record(st)
        outs.append(o)
        evs.append(e)
    for k, e in enumerate(evs):
        e.synchronize()
        print(f"[bench] {label}: chunk {k + 1}/{nch} done at {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = np.concatenate([o["stats"].cpu().numpy() for o in outs])
    status = np.concatenate([o["status"].cpu().numpy() for o in outs])
    return wall, st, status


def integration_legs(args, torch, acm, net):
    """Integrated cells/s of the batched BDF on the 16,384-cell workload (470 /
    4600 network, T log-uniform on 10-300 K, n_H log-uniform on 1e2-1e7,
    BDF 1-5 to 1e6 yr, rtol 1e-6, atol 1e-20), the plain one-cell-per-launch
    loop timed on the first --plain-cells of the same cells under the same
    step budget (and the batched kernel on those same cells), then the
    discrete adjoint of --adj-cells cells of the 4,096-cell workload to
    t_end. Wall-clock timing, synchronised."""
    import synthnet
    dev = torch.device("cuda:0")
    N = acm.Network.from_synth(net)
    wss = [acm.Workspace(N), acm.Workspace(N)]
    t_end = 1e6 * YEAR_S
    K = args.int_max_steps
    res = {}
    cells = synthnet.make_cells(net, args.int_cells, synthnet.SEED_BASE + 2)
    n = cells.T.size
    y = torch.from_numpy(cells.y0.copy()).to(dev)
    T = torch.from_numpy(cells.T.copy()).to(dev)
    wall, st, status = _integrate_chunked(torch, acm, wss, y, T, t_end, K, args.int_chunks,
                                          f"batched integration of {n} cells")
    steps = int(st[:, 0].sum())
    ok = int((status == 0).sum())
    capped = np.flatnonzero(status == 1)
    # the plain loop and the batched kernel on the same first cells
    npl = min(args.plain_cells, n)
    yb = torch.from_numpy(cells.y0[:npl].copy()).to(dev)
    Tp = torch.from_numpy(cells.T[:npl].copy()).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ob = wss[0].integrate(yb, Tp, t_end, max_steps=K)
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t0
    wall_p, sp, stp, same = 0.0, [], [], True
    for k in range(0, npl, 8):
        yp = torch.from_numpy(cells.y0[k:k + 8].copy()).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op = wss[0].integrate(yp, Tp[k:k + 8], t_end, max_steps=K, plain=True)
        torch.cuda.synchronize()
        wall_p += time.perf_counter() - t0
        sp.append(op["stats"].cpu().numpy())
        stp.append(op["status"].cpu().numpy())
        same = same and bool(torch.equal(yp, yb[k:k + 8]))
        print(f"[bench] plain loop: {min(k + 8, npl)}/{npl} cells, {wall_p:.1f} s", file=sys.stderr,
              flush=True)
    sp, stp = np.concatenate(sp), np.concatenate(stp)
    ok_p = int((stp == 0).sum())
    res["integration"] = {
        "workload": f"470/4600 network, {n} cells (T log-uniform 10-300 K, n_H log-uniform "
                    f"1e2-1e7 cm^-3), BDF 1-5 to 1e6 yr, rtol 1e-6, atol 1e-20, "
                    f"max_steps {K} per cell",
        "cells": n, "wall_s": wall, "cells_reaching_t_end": ok,
        "cells_maxsteps": int(capped.size), "first_capped_cells": capped[:16].tolist(),
        "integrated_cells_per_s": ok / wall, "cells_per_s_all": n / wall,
        "steps": steps, "steps_per_s": steps / wall,
        "step_quantiles_10_50_90_99_max": np.quantile(st[:, 0], [0.1, 0.5, 0.9, 0.99, 1.0]).tolist(),
        "newton_iters_per_step": float(st[:, 3].sum() / max(steps, 1)),
        "lu_per_step": float(st[:, 5].sum() / max(steps, 1)),
        "jac_per_step": float(st[:, 4].sum() / max(steps, 1)),
        "rejections_per_step": float((st[:, 1] + st[:, 2]).sum() / max(steps, 1)),
        "slots": wss[0].n_slots, "launches": args.int_chunks,
        "plain": {"cells": npl, "wall_s": wall_p, "cells_reaching_t_end": ok_p,
                  "integrated_cells_per_s": ok_p / wall_p, "steps": int(sp[:, 0].sum()),
                  "steps_per_s": float(sp[:, 0].sum() / wall_p),
                  "batched_wall_s_same_cells": wall_b,
                  "same_results_as_batched": same,
                  "note": "plain = the same kernel launched once per cell with one workgroup, "
                          "launches issued back to back; timed on the first cells of the "
                          "workload under the same step budget"},
        "vs_plain": (ok / wall) / (ok_p / wall_p) if ok_p else None,
        "vs_plain_same_cells": wall_p / wall_b,
    }
    # discrete adjoint: forward with tape, then the timed adjoint sweep
    acells = synthnet.make_cells(net, 4096, synthnet.SEED_BASE + 3)
    na = min(args.adj_cells, 4096)
    ya = torch.from_numpy(acells.y0[:na].copy()).to(dev)
    Ta = torch.from_numpy(acells.T[:na].copy()).to(dev)
    cap = 2 * args.adj_max_steps + 64
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fw = wss[0].integrate(ya, Ta, t_end, max_steps=args.adj_max_steps, tape_cap=cap)
    torch.cuda.synchronize()
    wall_f = time.perf_counter() - t0
    print(f"[bench] adjoint forward: {na} cells in {wall_f:.1f} s", file=sys.stderr, flush=True)
    yT = ya.cpu().numpy()
    rng = np.random.default_rng(8)
    lam = np.zeros_like(yT)
    for c in range(na):
        okc = np.flatnonzero(yT[c] > 1e-20)
        tgt = rng.choice(okc, 8, replace=False)
        lam[c, tgt] = 1.0 / yT[c, tgt]
    y0a = torch.from_numpy(acells.y0[:na].copy()).to(dev)
    # the tapes cut to the longest one, and room for every converged state
    # reserved before the timed region
    L = int(fw["tape_len"].max().item()) + 1
    tape = fw["tape"][:, :L].contiguous()
    wss[0].reserve_adjoint(L, keep_states=True, max_cells=na)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    adj = wss[0].adjoint(y0a, Ta, tape, fw["tape_len"], torch.from_numpy(lam).to(dev))
    torch.cuda.synchronize()
    wall_a = time.perf_counter() - t0
    fst = fw["status"].cpu().numpy()
    sa = int(fw["stats"].cpu().numpy()[:, 0].sum())
    ast_ = adj["stats"].cpu().numpy()
    print(f"[bench] adjoint: {na} cells in {wall_a:.1f} s", file=sys.stderr, flush=True)
    res["adjoint"] = {
        "workload": f"470/4600 network, first {na} of the 4,096-cell workload, d sum log y_t / "
                    f"d (log alpha, y0) for 8 seeded targets per cell, BDF 1-5 to 1e6 yr "
                    f"(max_steps {args.adj_max_steps}), checkpoints every 64 steps, every "
                    f"converged state kept",
        "cells": na, "forward_wall_s": wall_f, "wall_s": wall_a,
        "forward_plus_adjoint_s": wall_f + wall_a, "cells_per_s": na / (wall_f + wall_a),
        "cells_reaching_t_end": int((fst == 0).sum()), "steps": sa,
        "adjoint_steps_per_s": sa / wall_a,
        "status_ok": int((adj["status"] == 0).sum().item()),
        "states_kept": wss[0].keeps_states, "tape_events_max": L,
        "per_step": {"replay_newton_iters": float(ast_[:, 3].sum() / max(sa, 1)),
                     "jacobians": float(ast_[:, 4].sum() / max(sa, 1)),
                     "factorisations": float(ast_[:, 5].sum() / max(sa, 1)),
                     "rhs": float(ast_[:, 6].sum() / max(sa, 1))},
    }
    for w in wss:
        w.close()
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
        out.update(integration_legs(args, torch, acm, net))
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(net, cells, args.cpu_seconds, N.jac_pattern())
    print(json.dumps(out))


if __name__ == "__main__":
    main()

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
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--cells", type=int, default=65536)
    p.add_argument("--layout", default="auto", help="sell|csr|runs|coo, or auto (autotuned)")
    p.add_argument("--ordering", default="auto", help="nnz|natural|rcm, or auto (autotuned)")
    p.add_argument("--block", type=int, default=0, help="threads per workgroup (0 = autotuned)")
    p.add_argument("--no-table", action="store_true",
                   help="skip the autotuner (layout x ordering x block table); use sell/nnz/512")
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    p.add_argument("--cpu-seconds", type=float, default=8.0,
                   help="about this many seconds per thread setting (five repeats)")
    p.add_argument("--no-int", action="store_true", help="skip the integration legs")
    p.add_argument("--no-scale", action="store_true",
                   help="skip the 700 / 8000 network on 262,144 cells")
    p.add_argument("--int-cells", type=int, default=16384,
                   help="cells of the batched integration leg (the 16,384-cell workload)")
    p.add_argument("--int-max-steps", type=int, default=20000,
                   help="accepted-step budget per cell (batched and plain alike)")
    p.add_argument("--plain-cells", type=int, default=64,
                   help="cells integrated by both the plain loop and the batched kernel")
    p.add_argument("--plain-max-steps", type=int, default=1000,
                   help="accepted-step budget per cell of that comparison (both sides)")
    p.add_argument("--adj-cells", type=int, default=256,
                   help="cells of the adjoint leg (first cells of the 4,096-cell workload that "
                        "reach t_end; 256 = one per workgroup slot)")
    p.add_argument("--adj-max-steps", type=int, default=10000)
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


def config1_leg(torch, acm):
    """The plain method on one cell (50 species / 300 reactions, T = 20 K,
    n_H = 1e4): per-call latency of the RHS, the Jacobian and both together
    (host wall time of one call plus its synchronisation, median of 50; and
    the device time per call in a stream of 200 back-to-back calls, HIP
    events), then backward Euler (BDF order 1) to 1e5 yr on the persistent
    integrator and on the plain one-cell launch."""
    import synthnet
    net, cells = synthnet.workload("tiny")
    N = acm.Network.from_synth(net)
    y = torch.from_numpy(cells.y0.copy()).cuda()
    T = torch.from_numpy(cells.T.copy()).cuda()
    dydt = torch.empty_like(y)
    jv = torch.empty((1, N.nnz_j), dtype=torch.float64, device="cuda")
    calls = {"rhs": lambda: acm.ac_rhs(N, None, y, T, dydt),
             "jac": lambda: acm.ac_jac(N, None, y, T, jv),
             "rhs_jac": lambda: acm.ac_rhs_jac(N, None, y, T, dydt, jv)}
    out = {}
    for name, fn in calls.items():
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        walls = []
        for _ in range(50):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(200):
            fn()
        b.record()
        torch.cuda.synchronize()
        out[name] = {"call_us": 1e6 * float(np.median(walls)),
                     "stream_us_per_call": 1e3 * a.elapsed_time(b) / 200}
    ws = acm.Workspace(N, n_slots=1)
    t_end = 1e5 * YEAR_S
    for mode in ("batched", "plain"):
        yi = y.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = ws.integrate(yi, T, t_end, q_max=1, plain=(mode == "plain"))
        torch.cuda.synchronize()
        st = o["stats"].cpu().numpy()[0]
        out[f"backward_euler_{mode}"] = {"wall_s": time.perf_counter() - t0,
                                         "status": int(o["status"][0]), "steps": int(st[0])}
    ws.close()
    N.close()
    return {"config1": dict(out, workload="50 species / 300 reactions, 1 cell, T = 20 K, "
                                          "n_H = 1e4 cm^-3; backward Euler to 1e5 yr")}


def scale_leg(torch, acm):
    """The 700 species / 8000 reactions network with grain-surface terms on
    262,144 cells: RHS + Jacobian (one ac_rhs_jac call), the VJP, each timed
    with HIP events (2 untimed, 3 timed calls). Its two-cell LDS does not fit
    a CU, so the one-cell kernels run."""
    import synthnet
    net, _ = synthnet.workload("large", n_cells=1)
    cells = synthnet.make_cells(net, 262144, synthnet.SEED_BASE + 4)
    C, ns, nr = 262144, net.n_species, net.n_reactions
    y = torch.from_numpy(cells.y0).cuda()
    T = torch.from_numpy(cells.T).cuda()
    dydt = torch.empty_like(y)
    nnz_j = acm.Network.from_synth(net, layout="sell", ordering="rcm").nnz_j
    jv = torch.empty((C, nnz_j), dtype=torch.float64, device="cuda")
    v = torch.randn(y.shape, dtype=torch.float64, device="cuda",
                    generator=torch.Generator("cuda").manual_seed(2))
    gy = torch.empty_like(y)
    gl = torch.empty(nr, dtype=torch.float64, device="cuda")
    # the one-cell Jacobian takes one workgroup per CU at this LDS size, so the
    # workgroup size sets its waves per CU: the library's own choice per
    # kernel (0) and both fixed sizes timed, the fastest kept
    by_block = {}
    for blk in (0, 512, 1024):
        N = acm.Network.from_synth(net, layout="sell", ordering="rcm", block=blk)
        tm = Timer(torch)
        for name, fn in (("rhs_jac", lambda: acm.ac_rhs_jac(N, None, y, T, dydt, jv)),
                         ("vjp", lambda: acm.ac_vjp(N, None, y, T, v, gy, gl))):
            for _ in range(2):
                fn()
            torch.cuda.synchronize()
            for _ in range(3):
                tm.run(name, fn)
            torch.cuda.synchronize()
        by_block[blk] = (tm.mean_ms("rhs_jac"), tm.mean_ms("vjp"))
        N.close()
    best = min(by_block, key=lambda b: by_block[b][0])
    rj, vj = by_block[best]
    b_rj = C * (16 * ns + 8 + 8 * nnz_j)
    out = {"workload": "700 species / 8000 reactions (20 % grain-surface-like two-body terms), "
                       "262,144 cells, FP64",
           "block": best, "ms_by_block": {str(b): {"rhs_jac": v[0], "vjp": v[1]}
                                         for b, v in by_block.items()},
           "nnz_j": nnz_j,
           "rhs_jac_ms": rj, "rhs_jac_cell_reactions_per_s": C * nr / (rj * 1e-3),
           "rhs_jac_GBps": b_rj / (rj * 1e-3) / 1e9,
           "rhs_jac_hbm_frac": b_rj / (rj * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "vjp_ms": vj, "vjp_cell_reactions_per_s": C * nr / (vj * 1e-3)}
    del jv, y, T, dydt, v, gy
    torch.cuda.empty_cache()
    return {"scale": out}


def _integrate_watched(torch, ws, y, T, t_end, max_steps, label, order=None, every=20.0):
    """Batched integration of every cell in one launch: the device queue hands
    cells to the persistent workgroups as they free up (in `order` when
    given), so the slow cells cost one tail. While it runs, prints a line
    every `every` seconds with the cells the workgroups have taken so far
    (the workspace's progress word). Returns (wall seconds, stats, status)."""
    C = y.shape[0]
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(s):
        o = ws.integrate(y, T, t_end, max_steps=max_steps, cell_order=order, stream=s.cuda_stream)
        e = torch.cuda.Event()
        e.record(s)
    last = t0
    while not e.query():
        time.sleep(0.2)
        now = time.perf_counter()
        if now - last >= every:
            last = now
            taken = min(ws.progress(), C)
            print(f"[bench] {label}: {taken}/{C} cells taken at {now - t0:.1f} s", file=sys.stderr,
                  flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"[bench] {label}: done in {wall:.1f} s", file=sys.stderr, flush=True)
    return wall, o["stats"].cpu().numpy(), o["status"].cpu().numpy()


def integration_legs(args, torch, acm, net):
    """Integrated cells/s of the batched BDF on the 16,384-cell workload (470 /
    4600 network, T log-uniform on 10-300 K, n_H log-uniform on 1e2-1e7,
    BDF 1-5 to 1e6 yr, rtol 1e-6, atol 1e-20) in one launch; the plain
    one-cell-per-launch loop and the batched kernel on the same first
    --plain-cells cells under a budget of --plain-max-steps steps each (their
    wall-time ratio is vs_plain); then the discrete adjoint of the first
    --adj-cells cells of the 4,096-cell workload to t_end. Wall-clock timing,
    synchronised."""
    import synthnet
    dev = torch.device("cuda:0")
    from paper_2312_04998_amd.autotune import tune_slots
    t_end = 1e6 * YEAR_S
    K = args.int_max_steps
    res = {}
    cells = synthnet.make_cells(net, args.int_cells, synthnet.SEED_BASE + 2)
    n = cells.T.size
    y = torch.from_numpy(cells.y0.copy()).to(dev)
    T = torch.from_numpy(cells.T.copy()).to(dev)
    # workgroup slots of the integrator, tuned on the first 512 cells (200 steps each)
    m = min(512, n)
    slots, slot_rate, slots_cached = tune_slots(net, y[:m], T[:m], t_end, 200)
    print(f"[bench] integrator slots {slots} (steps/s by slots {slot_rate}, "
          f"{'cached' if slots_cached else 'tuned'})", file=sys.stderr, flush=True)
    N = acm.Network.from_synth(net)
    ws = acm.Workspace(N, n_slots=slots)
    # the Newton solve on the same sample: the plan (minimum-degree front swept
    # sparsely, dense Schur tail) against one pivoted LU of the whole matrix
    solve_rate = {}
    for solver in ("dense", "auto", "dense", "auto"):
        yy = y[:m].clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        oo = ws.integrate(yy, T[:m], t_end, max_steps=200, linear_solver=solver)
        torch.cuda.synchronize()
        solve_rate[solver] = float(oo["stats"][:, 0].sum().item()) / (time.perf_counter() - t0)
    plan = {k: v for k, v in N.front_info().items() if k != "order"}
    print(f"[bench] Newton solve: steps/s {solve_rate} (front {plan['n_front']} species in "
          f"{plan['n_levels']} levels)", file=sys.stderr, flush=True)
    # cells expected to take longest first: step counts grow with density
    order = torch.from_numpy(np.argsort(-cells.n_H, kind="stable").astype(np.int32)).to(dev)
    wall, st, status = _integrate_watched(torch, ws, y, T, t_end, K,
                                          f"batched integration of {n} cells", order)
    steps = int(st[:, 0].sum())
    ok = int((status == 0).sum())
    capped = np.flatnonzero(status == 1)
    # the plain loop and the batched kernel on the same first cells, under the
    # same (smaller) step budget
    npl, Kp = min(args.plain_cells, n), args.plain_max_steps
    yb = torch.from_numpy(cells.y0[:npl].copy()).to(dev)
    Tp = torch.from_numpy(cells.T[:npl].copy()).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ob = ws.integrate(yb, Tp, t_end, max_steps=Kp)
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t0
    sb = ob["stats"].cpu().numpy()
    wall_p, sp, stp, same = 0.0, [], [], True
    for k in range(0, npl, 8):
        yp = torch.from_numpy(cells.y0[k:min(k + 8, npl)].copy()).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op = ws.integrate(yp, Tp[k:min(k + 8, npl)], t_end, max_steps=Kp, plain=True)
        torch.cuda.synchronize()
        wall_p += time.perf_counter() - t0
        sp.append(op["stats"].cpu().numpy())
        stp.append(op["status"].cpu().numpy())
        same = same and bool(torch.equal(yp, yb[k:min(k + 8, npl)]))
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
        "slots": ws.n_slots, "launches": 1,
        "cell_order": "n_H descending (step counts grow with density); results per cell do "
                      "not depend on the order",
        "slot_tuning": {"steps_per_s_by_slots": slot_rate, "from_cache": slots_cached,
                        "sample": f"first {m} cells, 200 steps each"},
        "newton_solve": {"used": "auto", "plan": plan, "steps_per_s": solve_rate,
                         "auto_over_dense": solve_rate["auto"] / solve_rate["dense"],
                         "sample": f"first {m} cells, 200 steps each, {ws.n_slots} slots; "
                                   "second of two runs each"},
        "plain": {"cells": npl, "max_steps": Kp, "wall_s": wall_p, "cells_reaching_t_end": ok_p,
                  "steps": int(sp[:, 0].sum()), "steps_per_s": float(sp[:, 0].sum() / wall_p),
                  "batched_wall_s_same_cells": wall_b,
                  "batched_steps_same_cells": int(sb[:, 0].sum()),
                  "same_results_as_batched": same,
                  "note": "plain = the same integrator launched once per cell with one "
                          "workgroup, launches issued back to back; the batched kernel and the "
                          "plain loop integrate the same first cells of the workload under the "
                          "same step budget, and vs_plain is the ratio of their wall times"},
        "vs_plain": wall_p / wall_b,
    }
    # discrete adjoint: forward with tape over the first cells of the 4,096-cell
    # workload, then the timed adjoint sweep over the first --adj-cells of them
    # that reach t_end within the step budget
    acells = synthnet.make_cells(net, 4096, synthnet.SEED_BASE + 3)
    nf = min(args.adj_cells + 8, 4096)
    ya = torch.from_numpy(acells.y0[:nf].copy()).to(dev)
    Ta = torch.from_numpy(acells.T[:nf].copy()).to(dev)
    cap = 2 * args.adj_max_steps + 64
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fw = ws.integrate(ya, Ta, t_end, max_steps=args.adj_max_steps, tape_cap=cap)
    torch.cuda.synchronize()
    wall_f = time.perf_counter() - t0
    fst = fw["status"].cpu().numpy()
    sel = np.flatnonzero(fst == 0)[:args.adj_cells]
    na = int(sel.size)
    print(f"[bench] adjoint forward: {nf} cells in {wall_f:.1f} s, {int((fst == 0).sum())} reach "
          f"t_end", file=sys.stderr, flush=True)
    if na == 0:
        res["adjoint"] = {"cells": 0, "forward_cells": nf, "forward_wall_s": wall_f,
                          "note": "no cell reached t_end within the step budget"}
        ws.close()
        return res
    yT = ya.cpu().numpy()[sel]
    rng = np.random.default_rng(8)
    lam = np.zeros_like(yT)
    for c in range(na):
        okc = np.flatnonzero(yT[c] > 1e-20)
        tgt = rng.choice(okc, 8, replace=False)
        lam[c, tgt] = 1.0 / yT[c, tgt]
    idx = torch.from_numpy(sel).to(dev)
    y0a = torch.from_numpy(acells.y0[sel].copy()).to(dev)
    Ts = Ta[idx].contiguous()
    tlen = fw["tape_len"][idx].contiguous()
    # the tapes cut to the longest one, and room for every converged state
    # reserved before the timed region
    L = int(tlen.max().item()) + 1
    tape = fw["tape"][idx, :L].contiguous()
    ws.reserve_adjoint(L, keep_states=True, max_cells=na)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    adj = ws.adjoint(y0a, Ts, tape, tlen, torch.from_numpy(lam).to(dev))
    torch.cuda.synchronize()
    wall_a = time.perf_counter() - t0
    sa = int(fw["stats"].cpu().numpy()[sel, 0].sum())
    ast_ = adj["stats"].cpu().numpy()
    print(f"[bench] adjoint: {na} cells in {wall_a:.1f} s", file=sys.stderr, flush=True)
    res["adjoint"] = {
        "workload": f"470/4600 network: the first {na} cells of the 4,096-cell workload that "
                    f"reach t_end (of its first {nf}; max_steps {args.adj_max_steps}), "
                    f"d sum log y_t / d (log alpha, y0) for 8 seeded targets per cell, BDF 1-5 "
                    f"to 1e6 yr, checkpoints every 64 steps, every converged state kept",
        "cells": na, "forward_cells": nf, "forward_wall_s": wall_f, "wall_s": wall_a,
        "cells_per_s": na / wall_a, "steps": sa, "adjoint_steps_per_s": sa / wall_a,
        "status_ok": int((adj["status"] == 0).sum().item()),
        "states_kept": ws.keep_states, "tape_events_max": L,
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
    tune_table, tune_cached = {}, None
    if args.no_table:
        cfg = {"layout": "sell", "ordering": "nnz", "block": 512}
    else:
        from paper_2312_04998_amd.autotune import autotune
        N, cfg, tab = autotune(net, y, T)
        N.close()
        tune_cached = cfg.pop("cached")
        tune_table = {f"{l}/{o}/{b}": round(ms, 4) for (l, o, b), ms in sorted(tab.items(), key=lambda kv: kv[1])}
    print(f"[bench] launch shape {cfg} ({'cached' if tune_cached else 'tuned' if tune_table else 'fixed'})",
          file=sys.stderr, flush=True)
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
    print(f"[bench] {args.steps} steps of RHS + Jacobian: {ms_step:.3f} ms per step", file=sys.stderr,
          flush=True)

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
        "autotune_from_cache": tune_cached,
    }
    out.update(config1_leg(torch, acm))
    if not args.no_scale:
        out.update(scale_leg(torch, acm))
        print(f"[bench] 700 / 8000 network, 262,144 cells: {out['scale']['rhs_jac_ms']:.1f} ms per RHS + "
              f"Jacobian, {out['scale']['vjp_ms']:.1f} ms per VJP", file=sys.stderr, flush=True)
    print(f"[bench] one-cell latency: {out['config1']['rhs_jac']['call_us']:.1f} us per RHS + "
          f"Jacobian call", file=sys.stderr, flush=True)
    if not args.no_int:
        out.update(lu_leg(torch, acm, net, cells))
        out.update(integration_legs(args, torch, acm, net))
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(net, cells, args.cpu_seconds, N.jac_pattern())
    print(json.dumps(out))


if __name__ == "__main__":
    main()

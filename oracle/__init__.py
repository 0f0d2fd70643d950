"""Oracle for the stoichiometry-matrix chemistry path -- TEST INFRASTRUCTURE.

A plain FP64 CPU implementation (``oracle.c``) with a numpy front end. Only
the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
may import this package; the GPU library never does, and the two share no
code. Networks are taken as ``synthnet.Network``-like objects (reactant and
product index arrays plus alpha, beta, gamma).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

# Strict IEEE FP64: no contraction into FMA, no fast-math; OpenMP only over
# independent cells.
CFLAGS = ["-O3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-std=c11", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (always, unless force is False and it exists)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _SO)
    return _SO


class _Net(C.Structure):
    _fields_ = [("n_species", C.c_int), ("n_reactions", C.c_int),
                ("reactants", C.c_void_p), ("products", C.c_void_p),
                ("alpha", C.c_void_p), ("beta", C.c_void_p), ("gamma", C.c_void_p),
                ("law", C.c_void_p), ("n_cond", C.c_int), ("heat", C.c_void_p)]


# Rate laws (oracle.h) and the per-cell conditions they read: (T, A_V,
# zeta/zeta_0, G_0).
LAW_KOOIJ, LAW_CRP, LAW_CRPHOT, LAW_PHOTO = 0, 1, 2, 3
NCOND = 4


class _Opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("h0", C.c_double),
                ("q_max", C.c_int), ("max_steps", C.c_int), ("newton_tol", C.c_double)]


EVENT_DTYPE = np.dtype([("type", np.int32), ("q", np.int32), ("val", np.float64)])
OK, MAXSTEPS, HMIN, BADINPUT, NEWTON_FAIL, SINGULAR, NONFINITE = 0, 1, 2, 3, 5, 6, 7
EV_INIT, EV_RESCALE, EV_STEP = 1, 2, 3
STAT_NAMES = ("steps", "reject_err", "reject_newton", "newton_it", "jac", "lu", "rhs", "q_last")

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        vp, i, l, d = C.c_void_p, C.c_int, C.c_long, C.c_double
        L.orc_set_threads.argtypes = [i]
        L.orc_get_threads.restype = i
        L.orc_stoich.argtypes = [vp, vp]
        L.orc_rate_coeffs.argtypes = [vp, l, vp, vp]
        L.orc_rates.argtypes = [vp, l, vp, vp, vp]
        L.orc_rhs.argtypes = [vp, l, vp, vp, vp, vp]
        L.orc_rhs_k.argtypes = [vp, l, vp, vp, vp, vp]
        L.orc_jac_dense.argtypes = [vp, l, vp, vp, vp, vp]
        L.orc_jac_pattern.argtypes = [vp, l, vp, vp, vp, vp, vp]
        L.orc_jac_pattern.restype = i
        L.orc_vjp.argtypes = [vp, l, vp, vp, vp, vp, vp]
        L.orc_lu_factor.argtypes = [i, vp, vp]
        L.orc_lu_factor.restype = i
        L.orc_lu_solve.argtypes = [i, vp, vp, vp]
        L.orc_lu_solve_t.argtypes = [i, vp, vp, vp]
        L.orc_bdf.argtypes = [vp, vp, l, vp, vp, d, vp, vp, vp, i, vp]
        L.orc_bdf_replay.argtypes = [vp, vp, l, vp, vp, vp, i, vp, i, vp, vp, vp, vp]
        L.orc_rhs_thermal.argtypes = [vp, l, vp, vp, vp, vp, vp]
        L.orc_jac_thermal.argtypes = [vp, l, vp, vp, vp, vp]
        L.orc_bdf_thermal.argtypes = [vp, vp, l, vp, vp, vp, d, vp, vp]
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class NetView:
    """Holds contiguous copies of a network's arrays and the C struct."""

    def __init__(self, net):
        self.reactants = np.ascontiguousarray(net.reactants, np.int32)
        self.products = np.ascontiguousarray(net.products, np.int32)
        self.alpha = _f64(net.alpha)
        self.beta = _f64(net.beta)
        self.gamma = _f64(net.gamma)
        self.ns = int(np.asarray(net.composition).shape[0]) if hasattr(net, "composition") \
            else int(net.n_species)
        self.nr = int(self.reactants.shape[0])
        assert self.reactants.shape == (self.nr, 2) and self.products.shape == (self.nr, 4)
        law = getattr(net, "law", None)
        self.law = None if law is None else np.ascontiguousarray(law, np.int8)
        self.n_cond = NCOND if self.law is not None else 1
        heat = getattr(net, "heat", None)
        self.heat = None if heat is None else _f64(heat)
        self.s = _Net(self.ns, self.nr, _p(self.reactants), _p(self.products),
                      _p(self.alpha), _p(self.beta), _p(self.gamma), _p(self.law), self.n_cond,
                      _p(self.heat))

    @property
    def ptr(self):
        return C.byref(self.s)


def _view(net) -> NetView:
    return net if isinstance(net, NetView) else NetView(net)


def _cells(a, n: int) -> np.ndarray:
    a = _f64(a)
    return a.reshape(-1, n)


def _cond(v: NetView, T) -> np.ndarray:
    """Per-cell conditions: T [n] for an all-Kooij network, [n, NCOND] rows
    (T, A_V, zeta/zeta_0, G_0) when the network has rate laws."""
    T = _f64(T)
    if v.n_cond == 1:
        return _f64(np.atleast_1d(T).reshape(-1))
    T = np.atleast_2d(T)
    if T.shape[1] != v.n_cond:
        raise ValueError(f"conditions need {v.n_cond} values per cell, got shape {T.shape}")
    return np.ascontiguousarray(T)


def stoich(net) -> np.ndarray:
    v = _view(net)
    S = np.zeros((v.ns, v.nr), np.int32)
    lib().orc_stoich(v.ptr, _p(S))
    return S


def rate_coeffs(net, T) -> np.ndarray:
    v = _view(net)
    T = _cond(v, T)
    k = np.zeros((T.shape[0], v.nr))
    lib().orc_rate_coeffs(v.ptr, T.shape[0], _p(T), _p(k))
    return k


def rates(net, y, T) -> np.ndarray:
    v = _view(net)
    y = _cells(y, v.ns)
    T = _cond(v, T)
    r = np.zeros((y.shape[0], v.nr))
    lib().orc_rates(v.ptr, y.shape[0], _p(y), _p(T), _p(r))
    return r


def rhs(net, y, T, with_abs: bool = False):
    v = _view(net)
    y = _cells(y, v.ns)
    T = _cond(v, T)
    out = np.zeros_like(y)
    ab = np.zeros_like(y) if with_abs else None
    lib().orc_rhs(v.ptr, y.shape[0], _p(y), _p(T), _p(out), _p(ab))
    return (out, ab) if with_abs else out


def rhs_k(net, k, y, with_abs: bool = False):
    v = _view(net)
    y = _cells(y, v.ns)
    k = _cells(k, v.nr)
    out = np.zeros_like(y)
    ab = np.zeros_like(y) if with_abs else None
    lib().orc_rhs_k(v.ptr, y.shape[0], _p(k), _p(y), _p(out), _p(ab))
    return (out, ab) if with_abs else out


def jac_dense(net, y, T, with_abs: bool = False):
    v = _view(net)
    y = _cells(y, v.ns)
    T = _cond(v, T)
    J = np.zeros((y.shape[0], v.ns, v.ns))
    ab = np.zeros_like(J) if with_abs else None
    lib().orc_jac_dense(v.ptr, y.shape[0], _p(y), _p(T), _p(J), _p(ab))
    return (J, ab) if with_abs else J


def jac_pattern(net, y, T, row_ptr, col):
    """Jacobian values [cells, nnz] on a CSR pattern, as S dR/dn with the net
    stoichiometry (jac_dense adds gross terms; equal up to rounding)."""
    v = _view(net)
    y = _cells(y, v.ns)
    T = _cond(v, T)
    rp = np.ascontiguousarray(row_ptr, np.int32)
    cl = np.ascontiguousarray(col, np.int32)
    jv = np.zeros((y.shape[0], int(rp[-1])))
    if lib().orc_jac_pattern(v.ptr, y.shape[0], _p(y), _p(T), _p(rp), _p(cl), _p(jv)):
        raise ValueError("a Jacobian term falls outside the pattern")
    return jv


def vjp(net, y, T, vec):
    v = _view(net)
    y = _cells(y, v.ns)
    vec = _cells(vec, v.ns)
    T = _cond(v, T)
    gy = np.zeros_like(y)
    gl = np.zeros((y.shape[0], v.nr))
    lib().orc_vjp(v.ptr, y.shape[0], _p(y), _p(T), _p(vec), _p(gy), _p(gl))
    return gy, gl


def lu_factor(A):
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    n = A.shape[0]
    piv = np.zeros(n, np.int32)
    info = lib().orc_lu_factor(n, _p(A), _p(piv))
    return A, piv, int(info)


def lu_solve(LU, piv, b, trans: bool = False):
    b = np.array(b, dtype=np.float64, copy=True)
    n = LU.shape[0]
    LU = _f64(LU)
    piv = np.ascontiguousarray(piv, np.int32)
    (lib().orc_lu_solve_t if trans else lib().orc_lu_solve)(n, _p(LU), _p(piv), _p(b))
    return b


def _opts(rtol, atol, h0, q_max, max_steps, newton_tol=0.0):
    return _Opts(float(rtol), float(atol), float(h0), int(q_max), int(max_steps),
                 float(newton_tol))


def bdf(net, y0, T, t_end, rtol=1e-6, atol=1e-20, q_max=5, max_steps=100000, h0=0.0,
        tape_cap: int = 0, newton_tol: float = 0.0):
    """Integrate every cell to t_end. Returns dict with y, status, stats and,
    if tape_cap > 0, the recorded step sequence (tape, tape_len)."""
    v = _view(net)
    y = np.array(_cells(y0, v.ns), copy=True)
    T = _cond(v, T)
    n = y.shape[0]
    status = np.zeros(n, np.int32)
    stats = np.zeros((n, len(STAT_NAMES)), np.int32)
    tape = np.zeros((n, max(tape_cap, 1)), EVENT_DTYPE) if tape_cap > 0 else None
    tlen = np.zeros(n, np.int32)
    o = _opts(rtol, atol, h0, q_max, max_steps, newton_tol)
    lib().orc_bdf(v.ptr, C.byref(o), n, _p(y), _p(T), float(t_end), _p(status), _p(stats),
                  _p(tape), int(tape_cap), _p(tlen))
    out = dict(y=y, status=status, stats=stats)
    if tape is not None:
        out["tape"] = tape
        out["tape_len"] = tlen
    return out


def bdf_replay(net, y0, T, tape, tape_len, rtol=1e-6, atol=1e-20, dy0=None, dlogalpha=None,
               n_dir: int = 0):
    """Replay recorded step sequences with converged correctors and forward
    sensitivities along n_dir directions (dy0 [cells, n_dir, ns],
    dlogalpha [n_dir, nr]). Returns (y [cells, ns], s [cells, n_dir, ns])."""
    v = _view(net)
    y0 = _cells(y0, v.ns)
    T = _cond(v, T)
    n = y0.shape[0]
    tape = np.ascontiguousarray(tape, EVENT_DTYPE)
    tape_len = np.ascontiguousarray(tape_len, np.int32)
    if np.any(tape_len < 0):
        raise ValueError("tape overflowed")
    if dy0 is not None:
        dy0 = _f64(dy0).reshape(n, n_dir, v.ns)
    if dlogalpha is not None:
        dlogalpha = _f64(dlogalpha).reshape(n_dir, v.nr)
    y_out = np.zeros_like(y0)
    s_out = np.zeros((n, max(n_dir, 1), v.ns))
    o = _opts(rtol, atol, 0.0, 5, 0)
    lib().orc_bdf_replay(v.ptr, C.byref(o), n, _p(y0), _p(T), _p(tape), tape.shape[1],
                         _p(tape_len), int(n_dir), _p(dy0), _p(dlogalpha), _p(y_out), _p(s_out))
    return y_out, s_out[:, :n_dir]


# ------------------------------------------- temperature as a state

def _therm(therm, n):
    th = _f64(therm).reshape(-1, 3)
    if th.shape[0] != n:
        raise ValueError("therm needs (c_v, T_b, lambda) per cell")
    return th


def rhs_thermal(net, y, T, therm, with_abs: bool = False):
    """d(n, T)/dt for states y [cells, ns+1] (last entry T); T: the
    conditions array (its temperature column is not used); therm [cells, 3] =
    (c_v, T_b, lambda)."""
    v = _view(net)
    y = _cells(y, v.ns + 1)
    T = _cond(v, T)
    th = _therm(therm, y.shape[0])
    out = np.zeros_like(y)
    ab = np.zeros_like(y) if with_abs else None
    lib().orc_rhs_thermal(v.ptr, y.shape[0], _p(y), _p(T), _p(th), _p(out), _p(ab))
    return (out, ab) if with_abs else out


def jac_thermal(net, y, T, therm):
    """Dense (ns+1) x (ns+1) Jacobian of the temperature-coupled system."""
    v = _view(net)
    y = _cells(y, v.ns + 1)
    T = _cond(v, T)
    th = _therm(therm, y.shape[0])
    J = np.zeros((y.shape[0], v.ns + 1, v.ns + 1))
    lib().orc_jac_thermal(v.ptr, y.shape[0], _p(y), _p(T), _p(th), _p(J))
    return J


def bdf_thermal(net, y0, T, therm, t_end, rtol=1e-6, atol=1e-20, q_max=5, max_steps=100000,
                h0=0.0):
    """Integrate the temperature-coupled system of every cell to t_end."""
    v = _view(net)
    y = np.array(_cells(y0, v.ns + 1), copy=True)
    T = _cond(v, T)
    th = _therm(therm, y.shape[0])
    n = y.shape[0]
    status = np.zeros(n, np.int32)
    stats = np.zeros((n, len(STAT_NAMES)), np.int32)
    o = _opts(rtol, atol, h0, q_max, max_steps)
    lib().orc_bdf_thermal(v.ptr, C.byref(o), n, _p(y), _p(T), _p(th), float(t_end), _p(status),
                          _p(stats))
    return dict(y=y, status=status, stats=stats)

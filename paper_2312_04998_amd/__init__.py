"""Python binding of libastrochem.so (stoichiometry-matrix chemistry on MI355X).

Argument marshalling only: every computation runs in the library's HIP
kernels. PyTorch supplies device memory (tensors) and the current stream.
The functions keep the C names (ac_rhs, ac_jac, ...); `Network` wraps a
network handle. Importing this package never falls back to another
implementation: if the built library is missing the import fails.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libastrochem.so")

AC_OK, AC_EINVAL, AC_ENOMEM, AC_EHIP, AC_EUNBALANCED, AC_ECAPACITY, AC_ELIMIT = range(7)
AC_LAYOUT_CSR, AC_LAYOUT_SELL, AC_LAYOUT_COO, AC_LAYOUT_RUNS, AC_LAYOUT_CCS = 0, 1, 2, 3, 4
AC_ORDER_NATURAL, AC_ORDER_NNZ_DESC, AC_ORDER_RCM = 0, 1, 2
AC_FMT_COO, AC_FMT_CCS, AC_FMT_CRS, AC_FMT_SELL = 0, 1, 2, 3
AC_CELL_OK, AC_CELL_MAXSTEPS, AC_CELL_HMIN, AC_CELL_BADINPUT, AC_CELL_TAPE = 0, 1, 2, 3, 4
AC_CELL_NEWTON_FAIL, AC_CELL_SINGULAR, AC_CELL_NONFINITE = 5, 6, 7
LAYOUTS = {"csr": AC_LAYOUT_CSR, "sell": AC_LAYOUT_SELL, "coo": AC_LAYOUT_COO,
           "runs": AC_LAYOUT_RUNS, "ccs": AC_LAYOUT_CCS}
ORDERINGS = {"natural": AC_ORDER_NATURAL, "nnz": AC_ORDER_NNZ_DESC, "rcm": AC_ORDER_RCM}


class AstrochemError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


class NetDesc(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_reactions", C.c_int32),
                ("reactants", C.c_void_p), ("products", C.c_void_p),
                ("alpha", C.c_void_p), ("beta", C.c_void_p), ("gamma", C.c_void_p),
                ("composition", C.c_void_p), ("n_elem", C.c_int32),
                ("check_balance", C.c_int32), ("layout", C.c_int32), ("ordering", C.c_int32),
                ("chunk", C.c_int32), ("sell_c", C.c_int32), ("sell_sigma", C.c_int32),
                ("block", C.c_int32), ("rate_law", C.c_void_p), ("heat", C.c_void_p)]


# Rate laws (ac_rate_law) and the per-cell conditions of a network that has
# them: rows (T, A_V, zeta/zeta_0, G_0).
AC_LAW_KOOIJ, AC_LAW_CRP, AC_LAW_CRPHOT, AC_LAW_PHOTO = 0, 1, 2, 3
AC_NCOND = 4


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_2312_04998_amd/build.py`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, st = C.c_void_p, C.c_int32, C.c_int64, C.c_int
    sig = {
        "ac_net_create": [vp, vp],
        "ac_net_destroy": [vp],
        "ac_net_info": [vp, vp, vp, vp, vp],
        "ac_net_stoich": [vp, vp, vp, vp],
        "ac_net_jac_pattern": [vp, vp, vp],
        "ac_net_row_order": [vp, vp],
        "ac_net_front_info": [vp, vp, vp, vp, vp, vp, vp],
        "ac_sparse_format": [i32, i32, vp, i32, i32, vp, vp, vp, vp, vp],
        "ac_rates": [vp, vp, i64, vp, vp, vp],
        "ac_rhs": [vp, vp, i64, vp, vp, vp, vp],
        "ac_rhs_k": [vp, i64, vp, vp, vp, vp],
        "ac_jac": [vp, vp, i64, vp, vp, vp, vp],
        "ac_rhs_jac": [vp, vp, i64, vp, vp, vp, vp, vp],
        "ac_vjp": [vp, vp, i64, vp, vp, vp, vp, vp, vp],
        "ac_vjp_static": [vp, vp, i64, vp, vp, vp, vp, vp, vp],
        "ac_rhs_thermal": [vp, vp, i64, vp, vp, vp, vp, vp],
        "ac_jac_thermal": [vp, vp, i64, vp, vp, vp, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = st
    L.ac_status_string.argtypes = [st]
    L.ac_status_string.restype = C.c_char_p
    L.ac_last_error.argtypes = [C.c_char_p, C.c_size_t]
    L.ac_last_error.restype = C.c_int
    d = C.c_double
    sig2 = {
        "ac_lu_factor": [i32, i32, i64, vp, vp, vp, vp],
        "ac_lu_solve": [i32, i32, i64, vp, vp, vp, i32, vp],
        "ac_ws_create": [vp, i32, vp],
        "ac_ws_destroy": [vp],
        "ac_ws_info": [vp, vp, vp],
        "ac_ws_progress": [vp, vp],
        "ac_integrate": [vp, vp, i64, vp, vp, d, vp, vp, vp, vp, i32, vp, vp],
        "ac_integrate_plain": [vp, vp, i64, vp, vp, d, vp, vp, vp, vp],
        "ac_integrate_adjoint": [vp, vp, i64, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp,
                                 vp, vp],
        "ac_replay": [vp, vp, i64, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp],
        "ac_integrate_thermal": [vp, vp, i64, vp, vp, vp, d, vp, vp, vp, vp],
        "ac_ws_reserve_adjoint": [vp, vp],
        "ac_newton_solve": [vp, i64, vp, vp, vp, i32, i32, vp, vp],
        "ac_ws_adjoint_info": [vp, vp, vp, vp, vp],
    }
    for name, args in sig2.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = st
    return L


lib = _load()


def last_error() -> str:
    buf = C.create_string_buffer(4096)
    lib.ac_last_error(buf, 4096)
    return buf.value.decode(errors="replace")


def check(status: int, where: str) -> None:
    if status != AC_OK:
        raise AstrochemError(status, where, last_error())


def _ptr(t) -> Optional[int]:
    """Device (or host numpy) address of a tensor/array, or None."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is not None:
        return int(stream)
    import torch
    return torch.cuda.current_stream().cuda_stream


def _check_dev(t, shape, name: str):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class IntegOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("h0", C.c_double),
                ("q_max", C.c_int32), ("max_steps", C.c_int32), ("adj_recompute", C.c_int32),
                ("checkpoint_every", C.c_int32), ("newton_tol", C.c_double),
                ("cell_order", C.c_void_p), ("linear_solver", C.c_int32)]


LINEAR_SOLVERS = {"auto": 0, "dense": 1}   # ac_linear_solver


def _solver(name):
    if name not in LINEAR_SOLVERS:
        raise ValueError(f"linear_solver must be one of {sorted(LINEAR_SOLVERS)}")
    return LINEAR_SOLVERS[name]


EVENT_DTYPE = np.dtype([("type", np.int32), ("q", np.int32), ("val", np.float64)])
STAT_NAMES = ("steps", "reject_err", "reject_newton", "newton_it", "jac", "lu", "rhs", "q_last")
NSTAT = len(STAT_NAMES)


class Network:
    """Owns an ac_net handle built from a reaction list (arrays as in
    synthnet.Network: reactants [nr,2], products [nr,4], alpha/beta/gamma)."""

    def __init__(self, reactants, products, alpha, beta, gamma, composition=None,
                 layout: str = "sell", ordering: str = "nnz", chunk: int = 0, sell_c: int = 0,
                 sell_sigma: int = 0, check_balance: bool = False, block: int = 0,
                 rate_law=None, heat=None):
        self._rea = np.ascontiguousarray(reactants, np.int32)
        self._pro = np.ascontiguousarray(products, np.int32)
        self._a = np.ascontiguousarray(alpha, np.float64)
        self._b = np.ascontiguousarray(beta, np.float64)
        self._g = np.ascontiguousarray(gamma, np.float64)
        self._comp = None if composition is None else np.ascontiguousarray(composition, np.int8)
        self._law = None if rate_law is None else np.ascontiguousarray(rate_law, np.int8)
        self.n_cond = 1 if self._law is None else AC_NCOND
        self._heat = None if heat is None else np.ascontiguousarray(heat, np.float64)
        self.n_reactions = int(self._rea.shape[0])
        if composition is not None:
            self.n_species = int(self._comp.shape[0])
        else:
            self.n_species = int(max(self._rea.max(), self._pro.max())) + 1
        self.layout, self.ordering = layout, ordering
        d = NetDesc(self.n_species, self.n_reactions, _ptr(self._rea), _ptr(self._pro),
                    _ptr(self._a), _ptr(self._b), _ptr(self._g), _ptr(self._comp),
                    0 if self._comp is None else self._comp.shape[1], int(check_balance),
                    LAYOUTS[layout], ORDERINGS[ordering], chunk, sell_c, sell_sigma, block,
                    _ptr(self._law), _ptr(self._heat))
        h = C.c_void_p()
        check(lib.ac_net_create(C.byref(d), C.byref(h)), "ac_net_create")
        self.handle = h
        nnz_s, nnz_j, nco, nch = (C.c_int64() for _ in range(4))
        check(lib.ac_net_info(h, C.byref(nnz_s), C.byref(nnz_j), C.byref(nco), C.byref(nch)),
              "ac_net_info")
        self.nnz_s, self.nnz_j, self.n_contrib, self.n_chunks = (
            nnz_s.value, nnz_j.value, nco.value, nch.value)

    @classmethod
    def from_synth(cls, net, **kw):
        return cls(net.reactants, net.products, net.alpha, net.beta, net.gamma,
                   composition=net.composition, rate_law=getattr(net, "law", None),
                   heat=getattr(net, "heat", None), **kw)

    def cond_shape(self, n: int):
        """Shape of the per-cell conditions array T for n cells."""
        return (n,) if self.n_cond == 1 else (n, self.n_cond)

    def close(self):
        if getattr(self, "handle", None):
            lib.ac_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------- host queries
    def stoich_csr(self):
        rp = np.zeros(self.n_species + 1, np.int32)
        rx = np.zeros(max(self.nnz_s, 1), np.int32)
        va = np.zeros(max(self.nnz_s, 1), np.int32)
        check(lib.ac_net_stoich(self.handle, _ptr(rp), _ptr(rx), _ptr(va)), "ac_net_stoich")
        return rp, rx[:self.nnz_s], va[:self.nnz_s]

    def jac_pattern(self):
        rp = np.zeros(self.n_species + 1, np.int32)
        col = np.zeros(max(self.nnz_j, 1), np.int32)
        check(lib.ac_net_jac_pattern(self.handle, _ptr(rp), _ptr(col)), "ac_net_jac_pattern")
        return rp, col[:self.nnz_j]

    def front_info(self):
        """The integrator's Newton-solve plan: dict with n_front, n_levels,
        n_values, n_updates, cost_ratio (modelled, vs one dense LU) and order
        (positions -> species, front first)."""
        n1, nl = C.c_int32(), C.c_int32()
        nv, nu = C.c_int64(), C.c_int64()
        cr = C.c_double()
        order = np.empty(self.n_species, np.int32)
        check(lib.ac_net_front_info(self.handle, C.byref(n1), C.byref(nl), C.byref(nv), C.byref(nu),
                                    C.byref(cr), order.ctypes.data_as(C.c_void_p)),
              "ac_net_front_info")
        return {"n_front": n1.value, "n_levels": nl.value, "n_values": nv.value,
                "n_updates": nu.value, "cost_ratio": cr.value, "order": order}

    def row_order(self):
        p = np.zeros(self.n_species, np.int32)
        check(lib.ac_net_row_order(self.handle, _ptr(p)), "ac_net_row_order")
        return p

    # --------------------------------------------------------- device calls
    def rates(self, T, log_alpha=None, out=None, stream=None):
        import torch
        n = T.shape[0]
        out = torch.empty((n, self.n_reactions), dtype=torch.float64, device=T.device) if out is None else out
        ac_rates(self, log_alpha, T, out, stream)
        return out

    def rhs(self, y, T, log_alpha=None, out=None, stream=None):
        import torch
        out = torch.empty_like(y) if out is None else out
        ac_rhs(self, log_alpha, y, T, out, stream)
        return out

    def rhs_k(self, k, y, out=None, stream=None):
        import torch
        out = torch.empty_like(y) if out is None else out
        ac_rhs_k(self, k, y, out, stream)
        return out

    def jac(self, y, T, log_alpha=None, out=None, stream=None):
        import torch
        out = torch.empty((y.shape[0], self.nnz_j), dtype=torch.float64, device=y.device) if out is None else out
        ac_jac(self, log_alpha, y, T, out, stream)
        return out

    def vjp(self, y, T, v, log_alpha=None, want_gy=True, want_glog=True, stream=None):
        import torch
        gy = torch.empty_like(y) if want_gy else None
        gl = torch.empty(self.n_reactions, dtype=torch.float64, device=y.device) if want_glog else None
        ac_vjp(self, log_alpha, y, T, v, gy, gl, stream)
        return gy, gl


# ------------------------------------------------------------ C-named calls

def _cells(net: Network, y, T):
    n = T.shape[0]
    _check_dev(T, net.cond_shape(n), "T")
    if y is not None:
        _check_dev(y, (n, net.n_species), "y")
    return n


def ac_rates(net: Network, log_alpha, T, k, stream=None):
    n = _cells(net, None, T)
    _check_dev(k, (n, net.n_reactions), "k")
    if log_alpha is not None:
        _check_dev(log_alpha, (net.n_reactions,), "log_alpha")
    check(lib.ac_rates(net.handle, _ptr(log_alpha), n, _ptr(T), _ptr(k), _stream(stream)), "ac_rates")


def ac_rhs(net: Network, log_alpha, y, T, dydt, stream=None):
    n = _cells(net, y, T)
    _check_dev(dydt, (n, net.n_species), "dydt")
    if log_alpha is not None:
        _check_dev(log_alpha, (net.n_reactions,), "log_alpha")
    check(lib.ac_rhs(net.handle, _ptr(log_alpha), n, _ptr(y), _ptr(T), _ptr(dydt),
                     _stream(stream)), "ac_rhs")


def ac_rhs_k(net: Network, k, y, dydt, stream=None):
    n = k.shape[0]
    _check_dev(k, (n, net.n_reactions), "k")
    _check_dev(y, (n, net.n_species), "y")
    _check_dev(dydt, (n, net.n_species), "dydt")
    check(lib.ac_rhs_k(net.handle, n, _ptr(k), _ptr(y), _ptr(dydt), _stream(stream)), "ac_rhs_k")


def ac_jac(net: Network, log_alpha, y, T, jvals, stream=None):
    n = _cells(net, y, T)
    _check_dev(jvals, (n, net.nnz_j), "jvals")
    if log_alpha is not None:
        _check_dev(log_alpha, (net.n_reactions,), "log_alpha")
    check(lib.ac_jac(net.handle, _ptr(log_alpha), n, _ptr(y), _ptr(T), _ptr(jvals),
                     _stream(stream)), "ac_jac")


def ac_rhs_jac(net: Network, log_alpha, y, T, dydt, jvals, stream=None):
    n = _cells(net, y, T)
    _check_dev(dydt, (n, net.n_species), "dydt")
    _check_dev(jvals, (n, net.nnz_j), "jvals")
    if log_alpha is not None:
        _check_dev(log_alpha, (net.n_reactions,), "log_alpha")
    check(lib.ac_rhs_jac(net.handle, _ptr(log_alpha), n, _ptr(y), _ptr(T), _ptr(dydt),
                         _ptr(jvals), _stream(stream)), "ac_rhs_jac")


def ac_vjp(net: Network, log_alpha, y, T, v, gy, g_logalpha, stream=None):
    n = _cells(net, y, T)
    _check_dev(v, (n, net.n_species), "v")
    if gy is not None:
        _check_dev(gy, (n, net.n_species), "gy")
    if g_logalpha is not None:
        _check_dev(g_logalpha, (net.n_reactions,), "g_logalpha")
    if log_alpha is not None:
        _check_dev(log_alpha, (net.n_reactions,), "log_alpha")
    check(lib.ac_vjp(net.handle, _ptr(log_alpha), n, _ptr(y), _ptr(T), _ptr(v), _ptr(gy),
                     _ptr(g_logalpha), _stream(stream)), "ac_vjp")


def _thermal_args(net: Network, y, T, therm):
    n = T.shape[0]
    _check_dev(T, net.cond_shape(n), "T")
    _check_dev(y, (n, net.n_species + 1), "y")
    _check_dev(therm, (n, 3), "therm")
    return n


def ac_rhs_thermal(net: Network, log_alpha, y, T, therm, dydt, stream=None):
    """Temperature as a state: y, dydt [n, ns+1] (last entry T), therm [n, 3]
    = (c_v, T_b, lambda)."""
    n = _thermal_args(net, y, T, therm)
    _check_dev(dydt, (n, net.n_species + 1), "dydt")
    if log_alpha is not None:
        _check_dev(log_alpha, (net.n_reactions,), "log_alpha")
    check(lib.ac_rhs_thermal(net.handle, _ptr(log_alpha), n, _ptr(y), _ptr(T), _ptr(therm),
                             _ptr(dydt), _stream(stream)), "ac_rhs_thermal")


def ac_jac_thermal(net: Network, log_alpha, y, T, therm, jvals, stream=None):
    """jvals [n, nnz_j + 2 ns + 1]: pattern values, T column, T row, corner."""
    n = _thermal_args(net, y, T, therm)
    _check_dev(jvals, (n, net.nnz_j + 2 * net.n_species + 1), "jvals")
    if log_alpha is not None:
        _check_dev(log_alpha, (net.n_reactions,), "log_alpha")
    check(lib.ac_jac_thermal(net.handle, _ptr(log_alpha), n, _ptr(y), _ptr(T), _ptr(therm),
                             _ptr(jvals), _stream(stream)), "ac_jac_thermal")


def ac_vjp_static(net: Network, log_alpha, y, T, v, gy, g_logalpha, stream=None):
    """ac_vjp with its partial sums in the library's per-GPU scratch array:
    allocates nothing (for graph capture and serving loops)."""
    n = _cells(net, y, T)
    _check_dev(v, (n, net.n_species), "v")
    if gy is not None:
        _check_dev(gy, (n, net.n_species), "gy")
    if g_logalpha is not None:
        _check_dev(g_logalpha, (net.n_reactions,), "g_logalpha")
    if log_alpha is not None:
        _check_dev(log_alpha, (net.n_reactions,), "log_alpha")
    check(lib.ac_vjp_static(net.handle, _ptr(log_alpha), n, _ptr(y), _ptr(T), _ptr(v), _ptr(gy),
                            _ptr(g_logalpha), _stream(stream)), "ac_vjp_static")


def ac_sparse_format(dense, fmt: int, width: int = 0):
    """Host storage builder (Sec. 2.2 formats) for a small integer matrix."""
    A = np.ascontiguousarray(dense, np.int32)
    nr, nc = A.shape
    cap = C.c_int64(4 * nr * nc + 16)
    val = np.zeros(cap.value, np.int32)
    idx = np.zeros(cap.value, np.int32)
    idx2 = np.zeros(cap.value, np.int32)
    ptr = np.zeros(nr + nc + 2, np.int32)
    check(lib.ac_sparse_format(nr, nc, _ptr(A), fmt, width, C.byref(cap), _ptr(val), _ptr(idx),
                               _ptr(idx2), _ptr(ptr)), "ac_sparse_format")
    n = cap.value
    return val[:n], idx[:n], idx2[:n], ptr


# ---------------------------------------------------------------- dense LU

def ac_lu_factor(A, piv, info=None, lda=None, stream=None):
    """A: [n_mat, n, lda] float64 device tensor (in place), piv: int32 [n_mat, n]."""
    n_mat, n = A.shape[0], A.shape[1]
    lda = A.shape[2] if lda is None else lda
    check(lib.ac_lu_factor(n, lda, n_mat, _ptr(A), _ptr(piv), _ptr(info), _stream(stream)),
          "ac_lu_factor")


def ac_lu_solve(LU, piv, b, trans=False, stream=None):
    n_mat, n, lda = LU.shape
    check(lib.ac_lu_solve(n, lda, n_mat, _ptr(LU), _ptr(piv), _ptr(b), int(trans), _stream(stream)),
          "ac_lu_solve")


# -------------------------------------------------------------- integrator

class AdjReserve(C.Structure):
    _fields_ = [("max_tape", C.c_int32), ("checkpoint_every", C.c_int32),
                ("keep_states", C.c_int32), ("max_cells", C.c_int32)]


class Workspace:
    """Owns an ac_ws (integrator slots) for one network. With adj_max_tape >
    0 it also reserves room for the adjoint and the replay at creation
    (ac_ws_reserve_adjoint); adjoint() and replay() reserve (explicitly, in
    a separate call before theirs) when a tape is longer than what was
    reserved, so the library call itself never allocates."""

    def __init__(self, net: Network, n_slots: int = 0, adj_max_tape: int = 0,
                 checkpoint_every: int = 0, keep_states: bool = True, adj_max_cells: int = 0):
        self.net = net
        h = C.c_void_p()
        check(lib.ac_ws_create(net.handle, int(n_slots), C.byref(h)), "ac_ws_create")
        self.handle = h
        ns, nb = C.c_int32(), C.c_int64()
        check(lib.ac_ws_info(h, C.byref(ns), C.byref(nb)), "ac_ws_info")
        self.n_slots, self.bytes = ns.value, nb.value
        self.keep_states, self.adj_max_cells = bool(keep_states), int(adj_max_cells)
        self.adj_max_tape, self.checkpoint_every = 0, int(checkpoint_every) or 64
        if adj_max_tape > 0:
            self.reserve_adjoint(adj_max_tape, checkpoint_every, keep_states, adj_max_cells)

    def reserve_adjoint(self, max_tape: int, checkpoint_every: int = 0, keep_states: bool = True,
                        max_cells: int = 0):
        """ac_ws_reserve_adjoint: room for tapes of up to max_tape events."""
        r = AdjReserve(int(max_tape), int(checkpoint_every), int(bool(keep_states)), int(max_cells))
        check(lib.ac_ws_reserve_adjoint(self.handle, C.byref(r)), "ac_ws_reserve_adjoint")
        mt, ce, ks, mc = (C.c_int32() for _ in range(4))
        check(lib.ac_ws_adjoint_info(self.handle, C.byref(mt), C.byref(ce), C.byref(ks),
                                     C.byref(mc)), "ac_ws_adjoint_info")
        self.adj_max_tape, self.checkpoint_every = mt.value, ce.value
        self.keep_states, self.adj_max_cells = bool(ks.value), mc.value

    def _ensure_adjoint(self, tape_cap: int, checkpoint_every: int):
        every = int(checkpoint_every) or 64
        if tape_cap > self.adj_max_tape or every != self.checkpoint_every:
            self.reserve_adjoint(max(tape_cap, self.adj_max_tape if every == self.checkpoint_every
                                     else 0), every, self.keep_states, self.adj_max_cells)

    def newton_solve(self, jvals, c, b, trans=False, linear_solver="auto", stream=None):
        """Solves (I - c[m] J_m) x = b[m] (or the transposed system) in place
        in b [n_mat, ns] for Jacobian pattern values jvals [n_mat, nnz_j] and
        c [n_mat] (device float64), with the integrator's Newton solve;
        returns info [n_mat] (0, or 1 + a zero pivot's position)."""
        import torch
        n = b.shape[0]
        _check_dev(b, (n, self.net.n_species), "b")
        _check_dev(jvals, (n, self.net.nnz_j), "jvals")
        _check_dev(c, (n,), "c")
        info = torch.empty(n, dtype=torch.int32, device=b.device)
        check(lib.ac_newton_solve(self.handle, n, _ptr(jvals), _ptr(c), _ptr(b), 1 if trans else 0,
                                  _solver(linear_solver), _ptr(info), _stream(stream)),
              "ac_newton_solve")
        return info

    def progress(self) -> int:
        """ac_ws_progress: cells taken so far by the running (or last)
        integration on this workspace."""
        n = C.c_int64()
        check(lib.ac_ws_progress(self.handle, C.byref(n)), "ac_ws_progress")
        return n.value

    def close(self):
        if getattr(self, "handle", None):
            lib.ac_ws_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def integrate(self, y, T, t_end, rtol=1e-6, atol=1e-20, q_max=5, max_steps=100000, h0=0.0,
                  log_alpha=None, tape_cap=0, plain=False, newton_tol=0.0, cell_order=None,
                  linear_solver="auto", stream=None):
        """Integrates y (device, in place) to t_end. Returns dict of device
        tensors: status [n], stats [n, NSTAT] and, with tape_cap > 0, the
        recorded steps (tape [n, tape_cap] of EVENT_DTYPE bytes, tape_len).
        cell_order: optional device int32 permutation of the cells, the
        order in which the workgroups take them (e.g. longest expected
        first); each cell's results do not depend on it. linear_solver:
        "auto" (sparse front swept, dense Schur tail) or "dense" (one
        pivoted LU of the whole Newton matrix)."""
        import torch
        n = T.shape[0]
        _check_dev(T, self.net.cond_shape(n), "T")
        _check_dev(y, (n, self.net.n_species), "y")
        if log_alpha is not None:
            _check_dev(log_alpha, (self.net.n_reactions,), "log_alpha")
        if cell_order is not None:
            if (cell_order.dtype != torch.int32 or tuple(cell_order.shape) != (n,)
                    or not cell_order.is_cuda or not cell_order.is_contiguous()):
                raise ValueError("cell_order must be a contiguous device int32 tensor [n_cells]")
        dev = y.device
        status = torch.empty(n, dtype=torch.int32, device=dev)
        stats = torch.empty((n, NSTAT), dtype=torch.int32, device=dev)
        o = IntegOpts(float(rtol), float(atol), float(h0), int(q_max), int(max_steps), 0, 0,
                      float(newton_tol), _ptr(cell_order), _solver(linear_solver))
        out = {"status": status, "stats": stats}
        if plain:
            check(lib.ac_integrate_plain(self.handle, _ptr(log_alpha), n, _ptr(y), _ptr(T),
                                         float(t_end), C.byref(o), _ptr(status), _ptr(stats),
                                         _stream(stream)), "ac_integrate_plain")
            return out
        tape = tlen = None
        if tape_cap > 0:
            tape = torch.empty((n, tape_cap, 2), dtype=torch.float64, device=dev)   # 16-byte events
            tlen = torch.empty(n, dtype=torch.int32, device=dev)
            out["tape"], out["tape_len"] = tape, tlen
        check(lib.ac_integrate(self.handle, _ptr(log_alpha), n, _ptr(y), _ptr(T), float(t_end),
                               C.byref(o), _ptr(status), _ptr(stats), _ptr(tape), int(tape_cap),
                               _ptr(tlen), _stream(stream)), "ac_integrate")
        return out


    def adjoint(self, y0, T, tape, tape_len, lam, rtol=1e-6, atol=1e-20, log_alpha=None,
                want_glog=True, want_cells=False, want_y=False, recompute=False,
                checkpoint_every=0, linear_solver="auto", stream=None):
        """Discrete adjoint (ac_integrate_adjoint) of L = sum <lam, y(t_end)>
        over the recorded tape of an earlier integrate(..., tape_cap=...).
        Returns dict of device tensors: dL_dy0 [n, ns], status [n], stats
        [n, NSTAT] (steps reversed, replay Newton iterations, Jacobians,
        factorisations, RHS evaluations) and, as
        requested, dL_dlogalpha [nr] (summed over cells in cell order),
        g_cells [n, nr] and the replayed y_final [n, ns]. recompute=True
        recomputes every checkpointed segment (checkpoint_every steps, 64 by
        default) from its checkpoint instead of keeping every converged
        state (same results, less memory)."""
        import torch
        n, ns, nr = T.shape[0], self.net.n_species, self.net.n_reactions
        _check_dev(T, self.net.cond_shape(n), "T")
        _check_dev(y0, (n, ns), "y0")
        _check_dev(lam, (n, ns), "lam")
        if log_alpha is not None:
            _check_dev(log_alpha, (nr,), "log_alpha")
        if tape.dim() != 3 or tape.shape[0] != n or tape.shape[2] != 2 or not tape.is_contiguous():
            raise ValueError("tape must be the [n, tape_cap, 2] tensor returned by integrate")
        if tape_len.dtype != torch.int32 or tuple(tape_len.shape) != (n,):
            raise ValueError("tape_len must be int32 [n]")
        dev = y0.device
        gy0 = torch.empty_like(y0)
        status = torch.empty(n, dtype=torch.int32, device=dev)
        stats = torch.empty((n, NSTAT), dtype=torch.int32, device=dev)
        out = {"dL_dy0": gy0, "status": status, "stats": stats}
        g_cells = glog = yf = None
        self._ensure_adjoint(int(tape.shape[1]), checkpoint_every)
        if want_cells or (want_glog and self.adj_max_cells <= 0):
            g_cells = torch.empty((n, nr), dtype=torch.float64, device=dev)
            if want_cells:
                out["g_cells"] = g_cells
        if want_glog:
            glog = torch.empty(nr, dtype=torch.float64, device=dev)
            out["dL_dlogalpha"] = glog
        if want_y:
            yf = torch.empty_like(y0)
            out["y_final"] = yf
        o = IntegOpts(float(rtol), float(atol), 0.0, 5, 1, 1 if recompute else 0,
                      int(checkpoint_every), 0.0, None, _solver(linear_solver))
        check(lib.ac_integrate_adjoint(self.handle, _ptr(log_alpha), n, _ptr(y0), _ptr(T),
                                       C.byref(o), _ptr(tape), int(tape.shape[1]),
                                       _ptr(tape_len), _ptr(lam), _ptr(yf), _ptr(gy0),
                                       _ptr(g_cells), _ptr(glog), _ptr(status), _ptr(stats),
                                       _stream(stream)), "ac_integrate_adjoint")
        return out


def _replay(ws, y0, T, tape, tape_len, rtol=1e-6, atol=1e-20, log_alpha=None,
            linear_solver="auto", stream=None):
    import torch
    n, ns = T.shape[0], ws.net.n_species
    _check_dev(T, ws.net.cond_shape(n), "T")
    _check_dev(y0, (n, ns), "y0")
    if log_alpha is not None:
        _check_dev(log_alpha, (ws.net.n_reactions,), "log_alpha")
    if tape.dim() != 3 or tape.shape[0] != n or tape.shape[2] != 2 or not tape.is_contiguous():
        raise ValueError("tape must be the [n, tape_cap, 2] tensor returned by integrate")
    yf = torch.empty_like(y0)
    status = torch.empty(n, dtype=torch.int32, device=y0.device)
    ws._ensure_adjoint(int(tape.shape[1]), ws.checkpoint_every)
    o = IntegOpts(float(rtol), float(atol), 0.0, 5, 1, 1, int(ws.checkpoint_every), 0.0, None,
                  _solver(linear_solver))
    check(lib.ac_replay(ws.handle, _ptr(log_alpha), n, _ptr(y0), _ptr(T), C.byref(o), _ptr(tape),
                        int(tape.shape[1]), _ptr(tape_len), _ptr(yf), _ptr(status), None,
                        _stream(stream)), "ac_replay")
    return {"y_final": yf, "status": status}


def _integrate_thermal(ws, y, T, therm, t_end, rtol=1e-6, atol=1e-20, q_max=5,
                       max_steps=100000, h0=0.0, log_alpha=None, linear_solver="auto",
                       stream=None):
    import torch
    n = _thermal_args(ws.net, y, T, therm)
    if log_alpha is not None:
        _check_dev(log_alpha, (ws.net.n_reactions,), "log_alpha")
    status = torch.empty(n, dtype=torch.int32, device=y.device)
    stats = torch.empty((n, NSTAT), dtype=torch.int32, device=y.device)
    o = IntegOpts(float(rtol), float(atol), float(h0), int(q_max), int(max_steps), 0, 0, 0.0,
                  None, _solver(linear_solver))
    check(lib.ac_integrate_thermal(ws.handle, _ptr(log_alpha), n, _ptr(y), _ptr(T), _ptr(therm),
                                   float(t_end), C.byref(o), _ptr(status), _ptr(stats),
                                   _stream(stream)), "ac_integrate_thermal")
    return {"status": status, "stats": stats}


Workspace.integrate_thermal = _integrate_thermal
Workspace.integrate_thermal.__doc__ = """ac_integrate_thermal: integrates states y
[n, ns+1] (last entry T, in place) with temperature as a state variable."""
Workspace.replay = _replay
Workspace.replay.__doc__ = """ac_replay: y(t_end) replayed along a recorded tape with converged
correctors. Returns dict of device tensors y_final [n, ns], status [n]."""


def tape_to_numpy(tape_tensor):
    """Device tape tensor -> numpy structured array of EVENT_DTYPE."""
    raw = tape_tensor.cpu().numpy()
    return raw.view(np.uint8).reshape(raw.shape[0], raw.shape[1], 16).copy().view(EVENT_DTYPE)[..., 0]


def tape_from_numpy(events, device="cuda"):
    """numpy structured array of EVENT_DTYPE [n, cap] -> device tape tensor
    [n, cap, 2] in the layout ac_integrate writes."""
    import torch
    ev = np.ascontiguousarray(events, EVENT_DTYPE)
    raw = ev.view(np.uint8).reshape(ev.shape[0], ev.shape[1], 16).view(np.float64)
    return torch.from_numpy(raw.copy()).to(device)


class Integrate:
    """y(t_end) = integrate(log_alpha, y0) with a discrete-adjoint backward.

    ``Integrate.apply(log_alpha, y0, T, ws, t_end, opts)`` runs the batched
    integrator (recording the step sequence) and returns y(t_end); its
    backward replays that sequence through ac_integrate_adjoint and returns
    dL/dlog_alpha (summed over cells) and dL/dy0. opts: dict with rtol,
    atol, q_max, max_steps and tape_cap (events kept per cell; by default
    the tape starts at 4,096 events and the forward run is repeated with a
    four times longer tape while any cell overflows it, up to what
    max_steps can produce). A cell that does not reach t_end (status other
    than AC_CELL_OK) raises IncompleteIntegration in the forward pass, and a
    cell whose adjoint is not complete raises it in the backward pass,
    rather than returning values that are not y(t_end) or its gradient."""

    @staticmethod
    def apply(log_alpha, y0, T, ws, t_end, opts=None):
        return _integrate_fn().apply(log_alpha, y0, T, ws, t_end, opts or {})


class IncompleteIntegration(RuntimeError):
    """Some cells stopped before t_end (status per cell in .status)."""

    def __init__(self, where: str, status):
        import numpy as _np
        st = _np.asarray(status)
        bad = _np.flatnonzero(st != AC_CELL_OK)
        super().__init__(f"{where}: {bad.size} of {st.size} cells did not complete "
                         f"(first cells {bad[:8].tolist()}, statuses {st[bad[:8]].tolist()})")
        self.status = st


_FN = None


def _integrate_fn():
    global _FN
    if _FN is not None:
        return _FN
    import torch

    class _Integrate(torch.autograd.Function):
        @staticmethod
        def forward(ctx, log_alpha, y0, T, ws, t_end, opts):
            rtol = opts.get("rtol", 1e-6)
            atol = opts.get("atol", 1e-20)
            max_steps = opts.get("max_steps", 100000)
            # each accepted step records one event, and each rejection or
            # order change at most one more
            cap_max = 2 * max_steps + 16
            cap = opts.get("tape_cap", min(4096, cap_max))
            la = log_alpha.detach().contiguous()
            while True:
                y = y0.detach().clone().contiguous()
                res = ws.integrate(y, T, t_end, rtol=rtol, atol=atol, q_max=opts.get("q_max", 5),
                                   max_steps=max_steps, log_alpha=la, tape_cap=cap)
                overflow = bool((res["tape_len"] < 0).any())
                if not overflow or "tape_cap" in opts or cap >= cap_max:
                    break
                cap = min(4 * cap, cap_max)
            status = res["status"].cpu().numpy()
            if (status != AC_CELL_OK).any():
                raise IncompleteIntegration("Integrate forward", status)
            if overflow:
                raise IncompleteIntegration("Integrate forward (tape overflow)",
                                            np.where(res["tape_len"].cpu().numpy() < 0,
                                                     AC_CELL_TAPE, AC_CELL_OK))
            ctx.ws, ctx.rtol, ctx.atol = ws, rtol, atol
            ctx.tape, ctx.tape_len = res["tape"], res["tape_len"]
            ctx.save_for_backward(la, y0.detach().contiguous(), T)
            return y

        @staticmethod
        def backward(ctx, gy):
            la, y0, T = ctx.saved_tensors
            r = ctx.ws.adjoint(y0, T, ctx.tape, ctx.tape_len, gy.contiguous(), rtol=ctx.rtol,
                               atol=ctx.atol, log_alpha=la, want_glog=True)
            status = r["status"].cpu().numpy()
            if (status != AC_CELL_OK).any():
                raise IncompleteIntegration("Integrate backward", status)
            return r["dL_dlogalpha"], r["dL_dy0"], None, None, None, None

    _FN = _Integrate
    return _FN

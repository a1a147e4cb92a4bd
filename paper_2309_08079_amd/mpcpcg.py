"""Thin ctypes binding of libmpcpcg (argument marshalling only).

Every entry point of include/mpcpcg.h has a method of the same name on ``Context``.
Arrays are torch tensors on the current HIP device (float32, contiguous); they are passed
as raw device pointers together with the current torch stream.  There is no CPU path:
if the library is missing the import of this module fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

OK, NOT_CONVERGED, BREAKDOWN, TIMEOUT = 0, 1, 2, 3
STOP_RULES = {"relative": 0, "absolute": 1}   # MPCPCG_STOP_RELATIVE / MPCPCG_STOP_ABSOLUTE
METHODS = {"pcg": 0, "factor": 1, "auto": 2}   # MPCPCG_METHOD_PCG / _FACTOR / _AUTO
EINVAL, EUNSUPPORTED, ENOMEM, EHIP = -1, -2, -3, -4

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmpcpcg.so")
# the LDS-poisoning debug build of the same sources (see build.py)
POISON_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmpcpcg_poison.so")
_lib = None
_libs = {}


class MPCPCGError(RuntimeError):
    pass


class Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nu", C.c_int32), ("N", C.c_int32)] + [
        (k, C.c_void_p) for k in ("Q", "R", "A", "B", "q", "r", "x0", "e")]


class Opts(C.Structure):
    _fields_ = [("eps", C.c_float), ("max_iter", C.c_int32), ("warm_start", C.c_int32),
                ("stop_rule", C.c_int32)]


class Schur(C.Structure):
    _fields_ = [("S", C.c_void_p), ("Pinv", C.c_void_p), ("gamma", C.c_void_p)]


class ChainModel(C.Structure):
    _fields_ = [("h", C.c_float), ("damping", C.c_float), ("coupling", C.c_float),
                ("gravity", C.c_void_p)]


class Trajectory(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nu", C.c_int32), ("N", C.c_int32)] + [
        (k, C.c_void_p) for k in ("X", "U", "x_init", "xref", "Q", "R")]


LS_STEPS = 9   # MPCPCG_LS_STEPS: alpha = 2^-j, j = 0..8

STATS_DTYPE = np.dtype([("iters", np.int32), ("status", np.int32), ("final_ratio", np.float32),
                        ("reserved", np.int32)])


def load_library(path: str = None):
    """Load libmpcpcg.so (built by ``paper_2309_08079_amd.build``), or another build of the
    same sources at ``path``; each is loaded once."""
    global _lib
    if path is None:
        if _lib is not None:
            return _lib
        path = _LIB_PATH
    if path in _libs:
        return _libs[path]
    if not os.path.exists(path):
        raise MPCPCGError("libmpcpcg.so not found at %s; build it with "
                          "`python -m paper_2309_08079_amd.build`" % path)
    lib = C.CDLL(path)
    vp, i32, i64p = C.c_void_p, C.c_int32, C.POINTER(C.c_int64)
    P, O = C.POINTER(Problem), C.POINTER(Opts)
    lib.mpcpcg_create.argtypes = [C.POINTER(vp), i32, i32, C.c_int64, i32]
    lib.mpcpcg_destroy.argtypes = [vp]
    lib.mpcpcg_last_error.argtypes = [vp]
    lib.mpcpcg_last_error.restype = C.c_char_p
    lib.mpcpcg_form_schur.argtypes = [vp, P, C.POINTER(Schur), vp]
    lib.mpcpcg_solve.argtypes = [vp, P, O, vp, vp, vp, vp, vp]
    lib.mpcpcg_solve_batched.argtypes = [vp, i32, i64p, P, O, vp, vp, vp, vp, vp]
    lib.mpcpcg_backward.argtypes = [vp, i32, i64p, P, O] + [vp] * 6 + [vp] * 9 + [vp, vp]
    lib.mpcpcg_set_knots_per_group.argtypes = [vp, i32]
    lib.mpcpcg_set_method.argtypes = [vp, i32]
    lib.mpcpcg_set_graph.argtypes = [vp, i32]
    lib.mpcpcg_autotune.argtypes = [vp, i32, i64p, P, O, vp, vp, vp, vp, vp, C.POINTER(i32)]
    lib.mpcpcg_tuned_schedule.argtypes = [vp, i32, i64p, C.POINTER(i32), C.POINTER(i32)]
    lib.mpcpcg_set_xcd_pinning.argtypes = [vp, i32]
    lib.mpcpcg_set_cache_limit.argtypes = [vp, i32]
    lib.mpcpcg_cache_info.argtypes = [vp, C.POINTER(i32), C.POINTER(C.c_int64)]
    lib.mpcpcg_debug_set_wait.argtypes = [vp, C.c_int64, i32]
    lib.mpcpcg_solve_noalloc.argtypes = [P, O, vp, vp, vp, vp, vp]
    lib.mpcpcg_noalloc_last_error.argtypes = []
    lib.mpcpcg_noalloc_last_error.restype = C.c_char_p
    lib.mpcpcg_factor_bytes.argtypes = [vp, C.c_int64]
    lib.mpcpcg_factor_bytes.restype = C.c_int64
    lib.mpcpcg_solve_batched_keep.argtypes = [vp, i32, i64p, P, O, vp, vp, vp, vp, vp, vp]
    lib.mpcpcg_backward_reuse.argtypes = [vp, i32, i64p, P, O] + [vp] * 6 + [vp] * 9 + [vp, vp, vp]
    M, T = C.POINTER(ChainModel), C.POINTER(Trajectory)
    lib.mpcpcg_linearize.argtypes = [vp, i32, i64p, M, T] + [vp] * 6 + [vp]
    lib.mpcpcg_line_search.argtypes = [vp, i32, i64p, M, T, vp, vp, vp, C.c_float] + [vp] * 4 + [vp]
    lib.mpcpcg_control_step.argtypes = [vp, i32, i64p, M, T, O, i32, C.c_float] + [vp] * 6 + [vp]
    for f in ("mpcpcg_create", "mpcpcg_destroy", "mpcpcg_form_schur", "mpcpcg_solve",
              "mpcpcg_solve_batched", "mpcpcg_backward", "mpcpcg_set_knots_per_group",
              "mpcpcg_set_graph", "mpcpcg_autotune", "mpcpcg_set_method", "mpcpcg_linearize",
              "mpcpcg_line_search", "mpcpcg_control_step", "mpcpcg_tuned_schedule",
              "mpcpcg_set_xcd_pinning", "mpcpcg_set_cache_limit", "mpcpcg_cache_info",
              "mpcpcg_debug_set_wait", "mpcpcg_solve_noalloc", "mpcpcg_solve_batched_keep",
              "mpcpcg_backward_reuse"):
        getattr(lib, f).restype = C.c_int
    _libs[path] = lib
    if _lib is None:
        _lib = lib
    return lib


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise MPCPCGError("expected a contiguous float32 device tensor")
    return t.data_ptr()


def _record(t):
    if not t.is_cuda or not t.is_contiguous():
        raise MPCPCGError("the factor record must be a contiguous device tensor")
    return t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _problem(d, nx, nu, N=0):
    p = Problem()
    p.nx, p.nu, p.N = nx, nu, N
    for k in ("Q", "R", "A", "B", "q", "r", "x0", "e"):
        t = d.get(k)
        setattr(p, k, None if t is None or t.numel() == 0 else _ptr(t))
    if p.Q is None or p.q is None or p.x0 is None:
        raise MPCPCGError("Q, q and x0 are required")
    return p


def _model(m):
    """mpcpcg_chain_model from a dict with h, damping, coupling (floats) and gravity (device)."""
    cm = ChainModel()
    cm.h, cm.damping, cm.coupling = float(m["h"]), float(m["damping"]), float(m["coupling"])
    cm.gravity = _ptr(m["gravity"])
    return cm


def _trajectory(d, nx, nu):
    t = Trajectory()
    t.nx, t.nu, t.N = nx, nu, int(d["X"].shape[0])
    for k in ("X", "U", "x_init", "xref", "Q", "R"):
        v = d.get(k)
        setattr(t, k, None if v is None or v.numel() == 0 else _ptr(v))
    return t


def _opts(eps, max_iter, warm, stop="relative"):
    if stop not in STOP_RULES:
        raise MPCPCGError("stop must be 'relative' or 'absolute', not %r" % (stop,))
    o = Opts()
    o.eps, o.max_iter, o.warm_start, o.stop_rule = float(eps), int(max_iter), int(bool(warm)), STOP_RULES[stop]
    return o


def stats_to_numpy(t):
    """View a device stats tensor (int32 [batch, 4]) as a structured numpy array."""
    return t.cpu().numpy().view(STATS_DTYPE).reshape(-1)


class Context:
    """Owns an mpcpcg_ctx on the current device."""

    def __init__(self, nx=14, nu=7, max_total_knots=1 << 17, max_batch=4096, lib_path=None):
        self.lib = load_library(lib_path)
        self.nx, self.nu = nx, nu
        self.method = "pcg"
        h = C.c_void_p()
        st = self.lib.mpcpcg_create(C.byref(h), nx, nu, int(max_total_knots), int(max_batch))
        if st != OK:
            raise MPCPCGError("mpcpcg_create failed with %d" % st)
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.mpcpcg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != OK:
            msg = self.lib.mpcpcg_last_error(self.h).decode()
            raise MPCPCGError("%s failed (%d): %s" % (what, st, msg))

    # ---- entry points ------------------------------------------------------------------
    def mpcpcg_form_schur(self, prob, out=None):
        N = prob["q"].shape[0]
        dev = prob["q"].device
        if out is not None:
            S, P, g = out
        else:
            S = torch.zeros((N, 3, self.nx, self.nx), device=dev)
            P = torch.zeros_like(S)
            g = torch.zeros((N, self.nx), device=dev)
        out = Schur(S.data_ptr(), P.data_ptr(), g.data_ptr())
        self._check(self.lib.mpcpcg_form_schur(self.h, C.byref(_problem(prob, self.nx, self.nu, N)),
                                               C.byref(out), _stream()), "mpcpcg_form_schur")
        return S, P, g

    def mpcpcg_solve(self, prob, eps=1e-6, max_iter=0, lam0=None, out=None, stop="relative"):
        N = prob["q"].shape[0]
        dev = prob["q"].device
        o = out or {}
        lam = o["lam"] if "lam" in o else torch.empty((N, self.nx), device=dev)
        if lam0 is not None:
            lam.copy_(lam0)
        dx = o["dx"] if "dx" in o else torch.empty((N, self.nx), device=dev)
        du = o["du"] if "du" in o else torch.empty((max(N - 1, 0), self.nu), device=dev)
        stats = o["stats"] if "stats" in o else torch.zeros((1, 4), dtype=torch.int32, device=dev)
        self._check(self.lib.mpcpcg_solve(
            self.h, C.byref(_problem(prob, self.nx, self.nu, N)), C.byref(_opts(eps, max_iter, lam0 is not None, stop)),
            _ptr(lam), _ptr(dx), _ptr(du) if du.numel() else None, stats.data_ptr(), _stream()),
            "mpcpcg_solve")
        return dict(lam=lam, dx=dx, du=du, stats=stats)

    def mpcpcg_factor_bytes(self, total_knots):
        n = self.lib.mpcpcg_factor_bytes(self.h, int(total_knots))
        if n < 0:
            raise MPCPCGError("mpcpcg_factor_bytes: no factor record on this context")
        return n

    def factor_record(self, total_knots, device):
        """A device buffer for the factor record of a batch of total_knots knots."""
        return torch.empty(self.mpcpcg_factor_bytes(total_knots), dtype=torch.uint8, device=device)

    def mpcpcg_solve_batched(self, packed, knot_off, eps=1e-6, max_iter=0, lam0=None, out=None,
                             stop="relative", factors=None):
        off = np.ascontiguousarray(knot_off, dtype=np.int64)
        B = len(off) - 1
        K = int(off[-1])
        dev = packed["q"].device
        o = out or {}
        lam = o["lam"] if "lam" in o else torch.empty((K, self.nx), device=dev)
        if lam0 is not None:
            lam.copy_(lam0)
        dx = o["dx"] if "dx" in o else torch.empty((K, self.nx), device=dev)
        du = o["du"] if "du" in o else torch.empty((max(K - B, 0), self.nu), device=dev)
        stats = o["stats"] if "stats" in o else torch.zeros((B, 4), dtype=torch.int32, device=dev)
        args = (self.h, B, off.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(_problem(packed, self.nx, self.nu)),
                C.byref(_opts(eps, max_iter, lam0 is not None, stop)), _ptr(lam), _ptr(dx),
                _ptr(du) if du.numel() else None, stats.data_ptr())
        if factors is None:
            self._check(self.lib.mpcpcg_solve_batched(*args, _stream()), "mpcpcg_solve_batched")
        else:
            self._check(self.lib.mpcpcg_solve_batched_keep(*args, _record(factors), _stream()),
                        "mpcpcg_solve_batched_keep")
        return dict(lam=lam, dx=dx, du=du, stats=stats)

    def mpcpcg_backward(self, packed, knot_off, fwd, gl, gx=None, gu=None, eps=1e-6, max_iter=0,
                        out=None, stop="relative", factors=None):
        off = np.ascontiguousarray(knot_off, dtype=np.int64)
        B = len(off) - 1
        K = int(off[-1])
        M = K - B
        dev = packed["q"].device
        nx, nu = self.nx, self.nu
        o = out or {}
        z = lambda key, shape: o[key] if key in o else torch.empty(shape, device=dev)
        g = dict(dQ=z("dQ", (K, nx, nx)), dR=z("dR", (M, nu, nu)), dA=z("dA", (M, nx, nx)),
                 dB=z("dB", (M, nx, nu)), dq=z("dq", (K, nx)), dr=z("dr", (M, nu)),
                 dx0=z("dx0", (B, nx)), de=z("de", (M, nx)), dgamma=z("dgamma", (K, nx)))
        stats = o["stats"] if "stats" in o else torch.zeros((B, 4), dtype=torch.int32, device=dev)
        opt = lambda t: _ptr(t) if t is not None and t.numel() else None
        args = (self.h, B, off.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(_problem(packed, nx, nu)),
                C.byref(_opts(eps, max_iter, False, stop)), _ptr(fwd["lam"]), _ptr(fwd["dx"]), opt(fwd["du"]),
                _ptr(gl), opt(gx), opt(gu),
                *[opt(g[k]) for k in ("dQ", "dR", "dA", "dB", "dq", "dr", "dx0", "de", "dgamma")],
                stats.data_ptr())
        if factors is None:
            self._check(self.lib.mpcpcg_backward(*args, _stream()), "mpcpcg_backward")
        else:
            self._check(self.lib.mpcpcg_backward_reuse(*args, _record(factors), _stream()),
                        "mpcpcg_backward_reuse")
        g["stats"] = stats
        return g

    def mpcpcg_set_knots_per_group(self, k):
        self._check(self.lib.mpcpcg_set_knots_per_group(self.h, int(k)), "mpcpcg_set_knots_per_group")

    def mpcpcg_set_method(self, method):
        """'pcg' (default), 'factor' (block LDL^T of S) or 'auto' (cost model per call)."""
        if method not in METHODS:
            raise MPCPCGError("method must be one of %s, not %r" % (sorted(METHODS), method))
        self._check(self.lib.mpcpcg_set_method(self.h, METHODS[method]), "mpcpcg_set_method")
        self.method = method

    def mpcpcg_set_graph(self, enable):
        self._check(self.lib.mpcpcg_set_graph(self.h, int(bool(enable))), "mpcpcg_set_graph")

    def mpcpcg_autotune(self, packed, knot_off, eps=1e-6, max_iter=0, stop="relative"):
        off = np.ascontiguousarray(knot_off, dtype=np.int64)
        B = len(off) - 1
        K = int(off[-1])
        dev = packed["q"].device
        lam = torch.empty((K, self.nx), device=dev)
        dx = torch.empty((K, self.nx), device=dev)
        du = torch.empty((max(K - B, 1), self.nu), device=dev)
        stats = torch.zeros((B, 4), dtype=torch.int32, device=dev)
        k = C.c_int32(0)
        self._check(self.lib.mpcpcg_autotune(
            self.h, B, off.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(_problem(packed, self.nx, self.nu)),
            C.byref(_opts(eps, max_iter, False, stop)), _ptr(lam), _ptr(dx), _ptr(du), stats.data_ptr(),
            _stream(), C.byref(k)), "mpcpcg_autotune")
        return k.value

    def mpcpcg_tuned_schedule(self, knot_off):
        """(knots per workgroup, gangs pinned to one XCD) of the next batched PCG solve."""
        off = np.ascontiguousarray(knot_off, dtype=np.int64)
        k, x = C.c_int32(0), C.c_int32(0)
        self._check(self.lib.mpcpcg_tuned_schedule(self.h, len(off) - 1, off.ctypes.data_as(C.POINTER(C.c_int64)),
                                                   C.byref(k), C.byref(x)), "mpcpcg_tuned_schedule")
        return k.value, bool(x.value)

    def mpcpcg_set_xcd_pinning(self, enable):
        self._check(self.lib.mpcpcg_set_xcd_pinning(self.h, int(bool(enable))), "mpcpcg_set_xcd_pinning")

    def mpcpcg_set_cache_limit(self, n):
        self._check(self.lib.mpcpcg_set_cache_limit(self.h, int(n)), "mpcpcg_set_cache_limit")

    def mpcpcg_cache_info(self):
        """(cached entries over all signature caches, device bytes of cached schedules)."""
        n, b = C.c_int32(0), C.c_int64(0)
        self._check(self.lib.mpcpcg_cache_info(self.h, C.byref(n), C.byref(b)), "mpcpcg_cache_info")
        return n.value, b.value

    def mpcpcg_debug_set_wait(self, limit_us, inject_stall=False):
        self._check(self.lib.mpcpcg_debug_set_wait(self.h, int(limit_us), int(bool(inject_stall))),
                    "mpcpcg_debug_set_wait")


    # ---- control step around the solve ----------------------------------------------------
    def mpcpcg_linearize(self, model, traj, knot_off, out=None):
        """LQ problem (dict Q, R, A, B, q, r, x0, e of device tensors) at the guess in traj."""
        off = np.ascontiguousarray(knot_off, dtype=np.int64)
        B = len(off) - 1
        K = int(off[-1])
        M = K - B
        nx, nu = self.nx, self.nu
        dev = traj["X"].device
        o = out or {}
        z = lambda key, shape: o[key] if key in o else torch.empty(shape, device=dev)
        lq = dict(A=z("A", (M, nx, nx)), B=z("B", (M, nx, nu)), q=z("q", (K, nx)), r=z("r", (M, nu)),
                  x0=z("x0", (B, nx)), e=z("e", (M, nx)))
        opt = lambda t: _ptr(t) if t.numel() else None
        self._check(self.lib.mpcpcg_linearize(
            self.h, B, off.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(_model(model)),
            C.byref(_trajectory(traj, nx, nu)), *[opt(lq[k]) for k in ("A", "B", "q", "r", "x0", "e")],
            _stream()), "mpcpcg_linearize")
        lq["Q"], lq["R"] = traj["Q"], traj["R"]
        return lq

    def mpcpcg_line_search(self, model, traj, knot_off, dX, dU, lam=None, mu=0.0, out=None):
        """Best of the 9 trial steps by the L1 merit: dict X, U (updated), merit [B, 9] float64,
        choice [B] int32.  ``out`` may name traj's own X / U for an in-place update."""
        off = np.ascontiguousarray(knot_off, dtype=np.int64)
        B = len(off) - 1
        dev = traj["X"].device
        o = out or {}
        X = o["X"] if "X" in o else torch.empty_like(traj["X"])
        U = o["U"] if "U" in o else torch.empty_like(traj["U"])
        merit = o["merit"] if "merit" in o else torch.empty((B, LS_STEPS), dtype=torch.float64, device=dev)
        choice = o["choice"] if "choice" in o else torch.empty((B,), dtype=torch.int32, device=dev)
        if merit.dtype != torch.float64 or choice.dtype != torch.int32:
            raise MPCPCGError("merit must be float64 and choice int32")
        opt = lambda t: _ptr(t) if t is not None and t.numel() else None
        self._check(self.lib.mpcpcg_line_search(
            self.h, B, off.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(_model(model)),
            C.byref(_trajectory(traj, self.nx, self.nu)), _ptr(dX), opt(dU), opt(lam), float(mu),
            _ptr(X), opt(U), merit.data_ptr(), choice.data_ptr(), _stream()), "mpcpcg_line_search")
        return dict(X=X, U=U, merit=merit, choice=choice)


    def mpcpcg_control_step(self, model, traj, knot_off, lam, X_out, U_out, sqp_iters=1, mu=0.0,
                            eps=1e-6, max_iter=0, warm=False, stop="relative", out=None):
        """sqp_iters x (linearise, solve, line search) as one call; lam [N, nx] receives the
        multipliers (and is the warm start when ``warm``).  Returns dict merit, choice,
        stats; the iterate is written to X_out / U_out (may be traj's own X / U)."""
        off = np.ascontiguousarray(knot_off, dtype=np.int64)
        B = len(off) - 1
        dev = traj["X"].device
        o = out or {}
        merit = o["merit"] if "merit" in o else torch.empty((B, LS_STEPS), dtype=torch.float64, device=dev)
        choice = o["choice"] if "choice" in o else torch.empty((B,), dtype=torch.int32, device=dev)
        stats = o["stats"] if "stats" in o else torch.zeros((B, 4), dtype=torch.int32, device=dev)
        opt = lambda t: _ptr(t) if t is not None and t.numel() else None
        self._check(self.lib.mpcpcg_control_step(
            self.h, B, off.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(_model(model)),
            C.byref(_trajectory(traj, self.nx, self.nu)), C.byref(_opts(eps, max_iter, warm, stop)),
            int(sqp_iters), float(mu), _ptr(lam), _ptr(X_out), opt(U_out), merit.data_ptr(),
            choice.data_ptr(), stats.data_ptr(), _stream()), "mpcpcg_control_step")
        return dict(merit=merit, choice=choice, stats=stats)


def mpcpcg_solve_noalloc(prob, lam, dx, du, stats, eps=1e-6, max_iter=0, warm=False, stop="relative"):
    """mpcpcg_solve_noalloc on caller-owned output tensors (lam, dx [N, 14], du [N-1, 7],
    stats int32 [1, 4]); no context, nothing allocated by the library."""
    lib = load_library()
    N = prob["q"].shape[0]
    st = lib.mpcpcg_solve_noalloc(C.byref(_problem(prob, 14, 7, N)), C.byref(_opts(eps, max_iter, warm, stop)),
                                  _ptr(lam), _ptr(dx), _ptr(du) if du.numel() else None, stats.data_ptr(),
                                  _stream())
    if st != OK:
        raise MPCPCGError("mpcpcg_solve_noalloc failed (%d): %s" % (st, lib.mpcpcg_noalloc_last_error().decode()))


def to_device(d, device="cuda"):
    """numpy dict (from synth) -> dict of contiguous float32 device tensors."""
    return {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(device) for k, v in d.items()}


STATUS_NAMES = {OK: "OK", NOT_CONVERGED: "NOT_CONVERGED", BREAKDOWN: "BREAKDOWN", TIMEOUT: "TIMEOUT"}


def check_stats(stats, what):
    """Raise MPCPCGError unless every problem of a device stats tensor reports OK (one small
    device-to-host read, which synchronises the stream)."""
    st = stats_to_numpy(stats)
    bad = np.nonzero(st["status"] != OK)[0]
    if bad.size:
        b = int(bad[0])
        raise MPCPCGError("%s: problem %d of %d reports %s after %d iterations (%d problems not OK)"
                          % (what, b, st.size, STATUS_NAMES.get(int(st["status"][b]), str(st["status"][b])),
                             int(st["iters"][b]), bad.size))


class MPCPCGFunction(torch.autograd.Function):
    """lambda, dx, du = MPCPCGFunction.apply(ctx, knot_off, eps, Q, R, A, B, q, r, x0, e[, max_iter]).

    Forward: mpcpcg_solve_batched.  Backward: mpcpcg_backward (adjoint PCG with the same
    stopping rule); returns gradients for Q, R, A, B, q, r, x0, e (symmetric part for Q, R).
    On a (14, 7) context with the PCG method the forward keeps its preconditioner Phi^-1
    and the inverses of Q and R (5.8 KB per knot, held until backward), and the backward
    reads them instead of forming them again.
    Both directions read the solver's stats and raise MPCPCGError if any problem did not
    converge (NOT_CONVERGED, BREAKDOWN or TIMEOUT), so that no unconverged iterate or
    undefined output flows into autograd.
    """

    @staticmethod
    def forward(fctx, mctx, knot_off, eps, Q, R, A, B, q, r, x0, e, max_iter=0):
        packed = dict(Q=Q.contiguous(), R=R.contiguous(), A=A.contiguous(), B=B.contiguous(),
                      q=q.contiguous(), r=r.contiguous(), x0=x0.contiguous(),
                      e=None if e is None else e.contiguous())
        fctx.factors = None
        if mctx.method == "pcg" and mctx.nx == 14:
            fctx.factors = mctx.factor_record(int(np.asarray(knot_off)[-1]), q.device)
        out = mctx.mpcpcg_solve_batched(packed, knot_off, eps=eps, max_iter=max_iter, factors=fctx.factors)
        check_stats(out["stats"], "MPCPCGFunction forward (mpcpcg_solve_batched)")
        fctx.mctx, fctx.off, fctx.eps, fctx.max_iter = mctx, np.asarray(knot_off, dtype=np.int64), eps, max_iter
        fctx.packed = packed
        fctx.save_for_backward(out["lam"], out["dx"], out["du"])
        fctx.has_e = e is not None
        fctx.stats = out["stats"]
        return out["lam"], out["dx"], out["du"]

    @staticmethod
    def backward(fctx, glam, gdx, gdu):
        lam, dx, du = fctx.saved_tensors
        zero_like = lambda t, ref: torch.zeros_like(ref) if t is None else t.contiguous()
        g = fctx.mctx.mpcpcg_backward(fctx.packed, fctx.off, dict(lam=lam, dx=dx, du=du),
                                      zero_like(glam, lam), None if gdx is None else gdx.contiguous(),
                                      None if gdu is None else gdu.contiguous(), eps=fctx.eps,
                                      max_iter=fctx.max_iter, factors=fctx.factors)
        fctx.factors = None
        check_stats(g["stats"], "MPCPCGFunction backward (mpcpcg_backward)")
        return (None, None, None, g["dQ"], g["dR"], g["dA"], g["dB"], g["dq"], g["dr"], g["dx0"],
                g["de"] if fctx.has_e else None, None)

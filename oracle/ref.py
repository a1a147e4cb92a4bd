"""ctypes front end of the plain-C FP64 oracle (``oracle/schur_pcg.c``).

Test infrastructure only (see the package docstring).  ``build()`` compiles the C file
with gcc; every function takes numpy arrays (any float dtype, upcast to float64) and
returns float64 results.

Follows MPCGPU Section III-B (Schur complement, eqs. (5)-(7)),
Section IV-A (symmetric stair preconditioner) and Algorithm 1 (PCG), with the stopping
rule sqrt(eta'/eta_ref) < eps, eta_ref = gamma^T Phi^-1 gamma (stop="relative"), or the
absolute test eta' < eps printed in Algorithm 1 (stop="absolute").
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "schur_pcg.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2


def compile_source(src: str, out: str) -> str:
    """gcc -O3 -fopenmp a C oracle source file into a shared library (plain C, no hand-written
    SIMD; -O3 as for the CPU baseline)."""
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                           "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O3, OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB):
        compile_source(_SRC, _LIB)
    return _LIB


def configure(lib):
    """Declare the argument types of an oracle library handle (returns it)."""
    d, i, i64 = C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_int64)
    ci = C.c_int
    lib.orc_form.argtypes = [ci, ci, ci] + [d] * 8 + [d, d, d]
    lib.orc_pcg.argtypes = [ci, ci, d, d, d, C.c_double, ci, ci, d, i, d, d]
    lib.orc_solve.argtypes = [ci, ci, ci] + [d] * 8 + [C.c_double, ci, ci, d, d, d, i, d, d]
    lib.orc_backward.argtypes = ([ci, ci, ci] + [d] * 8 + [C.c_double, ci, ci] + [d] * 6 +
                                  [d] * 9 + [i, d])
    lib.orc_solve_batch.argtypes = ([ci, ci, ci, i64] + [d] * 8 + [C.c_double, ci, ci] +
                                     [d, d, d, i, d, i, ci])
    lib.orc_backward_batch.argtypes = ([ci, ci, ci, i64] + [d] * 8 + [C.c_double, ci, ci] +
                                        [d] * 6 + [d] * 9 + [i, d, i, ci])
    for f in (lib.orc_form, lib.orc_pcg, lib.orc_solve, lib.orc_backward,
              lib.orc_solve_batch, lib.orc_backward_batch):
        f.restype = C.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = configure(C.CDLL(_LIB))
    return _lib


def _stop(stop):
    if stop not in ("relative", "absolute"):
        raise ValueError("stop must be 'relative' or 'absolute', not %r" % (stop,))
    return 1 if stop == "absolute" else 0


def _mode(stop, phi):
    """Mode word of the solve entry points: bit 0 absolute stop, bit 1 Phi^-1 in FP32."""
    if phi not in ("fp64", "fp32"):
        raise ValueError("phi must be 'fp64' or 'fp32', not %r" % (phi,))
    return _stop(stop) | (2 if phi == "fp32" else 0)


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _dims(prob):
    N, nx = prob["q"].shape
    nu = prob["R"].shape[-1] if prob["R"].size else prob.get("nu", 1)
    if not prob["R"].size and "B" in prob and prob["B"].ndim == 3:
        nu = prob["B"].shape[2]
    return nx, nu, N


def _args(prob):
    keep = [_d(prob[k]) for k in ("Q", "R", "A", "B", "q", "r", "x0")]
    e = prob.get("e")
    keep.append(_d(e) if e is not None and np.size(e) else None)
    return keep


def form(prob):
    """S, Phi^-1 as [N,3,nx,nx] (slots (b,b-1),(b,b),(b,b+1)) and gamma [N,nx]."""
    nx, nu, N = _dims(prob)
    a = _args(prob)
    S = np.zeros((N, 3, nx, nx)); P = np.zeros_like(S); g = np.zeros((N, nx))
    st = _load().orc_form(nx, nu, N, *[_p(x) for x in a], _p(S), _p(P), _p(g))
    if st < 0 or st == BREAKDOWN:
        raise ValueError("oracle form failed (status %d)" % st)
    return S, P, g


def pcg(S, P, gamma, eps=1e-6, max_iter=0, lam0=None, trace=False, stop="relative"):
    """Algorithm 1 on given blocks.  Returns dict(lam, iters, ratio, status[, eta])."""
    S, P, gamma = _d(S), _d(P), _d(gamma)
    N, _, nx, _ = S.shape
    max_iter = max_iter if max_iter > 0 else N * nx
    lam = np.zeros((N, nx)) if lam0 is None else _d(lam0).copy()
    it, ratio = C.c_int(0), C.c_double(0)
    tr = np.full(max_iter + 1, np.nan) if trace else None
    st = _load().orc_pcg(nx, N, _p(S), _p(P), _p(gamma), eps, _stop(stop), max_iter, _p(lam), C.byref(it),
                         C.byref(ratio), _p(tr))
    out = dict(lam=lam, iters=it.value, ratio=ratio.value, status=st)
    if trace:
        out["eta"] = tr[: it.value + 1]
    return out


def solve(prob, eps=1e-6, max_iter=0, lam0=None, trace=False, stop="relative", phi="fp64"):
    """Form + PCG + primal step.  Returns dict(lam, dx, du, iters, ratio, status[, eta]).
    phi="fp32" rounds Phi^-1 to single precision before PCG uses it."""
    nx, nu, N = _dims(prob)
    a = _args(prob)
    mi = max_iter if max_iter > 0 else N * nx
    lam = np.zeros((N, nx)) if lam0 is None else _d(lam0).copy()
    dx = np.zeros((N, nx)); du = np.zeros((max(N - 1, 0), nu))
    it, ratio = C.c_int(0), C.c_double(0)
    tr = np.full(mi + 1, np.nan) if trace else None
    st = _load().orc_solve(nx, nu, N, *[_p(x) for x in a], eps, _mode(stop, phi), mi, _p(lam), _p(dx), _p(du),
                           C.byref(it), C.byref(ratio), _p(tr))
    if st < 0:
        raise ValueError("oracle solve failed (status %d)" % st)
    out = dict(lam=lam, dx=dx, du=du, iters=it.value, ratio=ratio.value, status=st)
    if trace:
        out["eta"] = tr[: it.value + 1]
    return out


def backward(prob, fwd, gl, gx=None, gu=None, eps=1e-6, max_iter=0, stop="relative", phi="fp64"):
    """Adjoint for L(lambda, dx, du).  Returns dict of gradients (dQ, dR, dA, dB, dq, dr,
    dx0, de, mu) plus iters/ratio/status of the adjoint PCG."""
    nx, nu, N = _dims(prob)
    a = _args(prob)
    M = max(N - 1, 0)
    out = dict(dQ=np.zeros((N, nx, nx)), dR=np.zeros((M, nu, nu)), dA=np.zeros((M, nx, nx)),
               dB=np.zeros((M, nx, nu)), dq=np.zeros((N, nx)), dr=np.zeros((M, nu)),
               dx0=np.zeros(nx), de=np.zeros((M, nx)), mu=np.zeros((N, nx)))
    it, ratio = C.c_int(0), C.c_double(0)
    gxd = None if gx is None else _d(gx)
    gud = None if gu is None else _d(gu)
    st = _load().orc_backward(
        nx, nu, N, *[_p(x) for x in a], eps, _mode(stop, phi), max_iter, _p(_d(fwd["lam"])), _p(_d(fwd["dx"])),
        _p(_d(fwd["du"])), _p(_d(gl)), _p(gxd), _p(gud),
        *[_p(out[k]) for k in ("dQ", "dR", "dA", "dB", "dq", "dr", "dx0", "de", "mu")],
        C.byref(it), C.byref(ratio))
    if st < 0:
        raise ValueError("oracle backward failed (status %d)" % st)
    out.update(iters=it.value, ratio=ratio.value, status=st)
    return out


def solve_batch(packed, off, eps=1e-6, max_iter=0, threads=1, stop="relative", phi="fp64"):
    """Batched forward solve on the packed layout; OpenMP over problems."""
    off = np.ascontiguousarray(off, dtype=np.int64)
    B = len(off) - 1
    nx = packed["q"].shape[1]; nu = packed["r"].shape[1] if packed["r"].ndim == 2 else packed["B"].shape[2]
    a = [_d(packed[k]) for k in ("Q", "R", "A", "B", "q", "r", "x0")]
    e = packed.get("e")
    a.append(_d(e) if e is not None and np.size(e) else None)
    K = int(off[-1])
    lam = np.zeros((K, nx)); dx = np.zeros((K, nx)); du = np.zeros((max(K - B, 0), nu))
    iters = np.zeros(B, dtype=np.int32); ratio = np.zeros(B); status = np.zeros(B, dtype=np.int32)
    _load().orc_solve_batch(nx, nu, B, off.ctypes.data_as(C.POINTER(C.c_int64)),
                            *[_p(x) for x in a], eps, _mode(stop, phi), max_iter, _p(lam), _p(dx), _p(du),
                            iters.ctypes.data_as(C.POINTER(C.c_int)), _p(ratio),
                            status.ctypes.data_as(C.POINTER(C.c_int)), threads)
    return dict(lam=lam, dx=dx, du=du, iters=iters, ratio=ratio, status=status)


def backward_batch(packed, off, fwd, gl, gx=None, gu=None, eps=1e-6, max_iter=0, threads=1,
                   stop="relative", phi="fp64"):
    """Batched adjoint on the packed layout; OpenMP over problems."""
    off = np.ascontiguousarray(off, dtype=np.int64)
    B = len(off) - 1
    nx = packed["q"].shape[1]; nu = packed["B"].shape[2]
    a = [_d(packed[k]) for k in ("Q", "R", "A", "B", "q", "r", "x0")]
    e = packed.get("e")
    a.append(_d(e) if e is not None and np.size(e) else None)
    K = int(off[-1]); M = max(K - B, 0)
    out = dict(dQ=np.zeros((K, nx, nx)), dR=np.zeros((M, nu, nu)), dA=np.zeros((M, nx, nx)),
               dB=np.zeros((M, nx, nu)), dq=np.zeros((K, nx)), dr=np.zeros((M, nu)),
               dx0=np.zeros((B, nx)), de=np.zeros((M, nx)), mu=np.zeros((K, nx)))
    iters = np.zeros(B, dtype=np.int32); ratio = np.zeros(B); status = np.zeros(B, dtype=np.int32)
    gxd = None if gx is None else _d(gx)
    gud = None if gu is None else _d(gu)
    _load().orc_backward_batch(
        nx, nu, B, off.ctypes.data_as(C.POINTER(C.c_int64)), *[_p(x) for x in a], eps, _mode(stop, phi), max_iter,
        _p(_d(fwd["lam"])), _p(_d(fwd["dx"])), _p(_d(fwd["du"])), _p(_d(gl)), _p(gxd), _p(gud),
        *[_p(out[k]) for k in ("dQ", "dR", "dA", "dB", "dq", "dr", "dx0", "de", "mu")],
        iters.ctypes.data_as(C.POINTER(C.c_int)), _p(ratio),
        status.ctypes.data_as(C.POINTER(C.c_int)), threads)
    out.update(iters=iters, ratio=ratio, status=status)
    return out

"""Seeded synthetic LQ subproblems shaped like the paper's Kuka IIWA-14 workload.

The paper measures on linearisations of a 7-joint arm (state dimension 14, control
dimension 7, horizons of 32 to 512 knots; Section V).  Those trajectories are not
available, so these seeded problems stand in for them.  This module only draws random
numbers and packs arrays: it holds none of the solver's arithmetic and is the one
module shared by the GPU path, the CPU oracle and the tests.

Draw recipe (numpy PCG64, float64 draws, then rounded to float32):
    An ~ N(0,1)^(N-1,nx,nx)      A_k = I + 0.01 An_k
    Bn ~ N(0,1)^(N-1,nx,nu)      B_k = 0.01 Bn_k
    Qd ~ U[lo,hi]^(N,nx)         Q_k = diag(Qd_k) + 0.1 W_k W_k^T
    W  ~ N(0,1)^(N,nx,4)
    Rd ~ U[0.1,1]^(N-1,nu)       R_k = diag(Rd_k)
    q  ~ N(0,1)^(N,nx), r ~ N(0,1)^(N-1,nu), x0 ~ N(0,1)^nx, e = 0.

N is the number of state knots (block rows of the Schur complement); there are N-1
controls and N-1 dynamics constraints.
"""
from __future__ import annotations

import numpy as np

FIELDS = ("Q", "R", "A", "B", "q", "r", "x0", "e")


def problem(N: int, nx: int = 14, nu: int = 7, seed: int = 1, q_lo: float = 1.0,
            q_hi: float = 10.0, defects: bool = False) -> dict:
    """One LQ subproblem as a dict of contiguous float32 arrays.

    Shapes: Q [N,nx,nx], R [N-1,nu,nu], A [N-1,nx,nx], B [N-1,nx,nu], q [N,nx],
    r [N-1,nu], x0 [nx], e [N-1,nx] (zeros unless ``defects``).
    """
    if N < 1:
        raise ValueError("N must be >= 1")
    g = np.random.default_rng(seed)
    M = N - 1
    An = g.standard_normal((M, nx, nx))
    Bn = g.standard_normal((M, nx, nu))
    Qd = g.uniform(q_lo, q_hi, (N, nx))
    W = g.standard_normal((N, nx, 4))
    Rd = g.uniform(0.1, 1.0, (M, nu))
    q = g.standard_normal((N, nx))
    r = g.standard_normal((M, nu))
    x0 = g.standard_normal(nx)
    e = 0.01 * g.standard_normal((M, nx)) if defects else np.zeros((M, nx))
    A = np.eye(nx)[None] + 0.01 * An
    B = 0.01 * Bn
    Q = np.zeros((N, nx, nx))
    for k in range(N):
        Q[k] = np.diag(Qd[k]) + 0.1 * (W[k] @ W[k].T)
    R = np.zeros((M, nu, nu))
    for k in range(M):
        R[k] = np.diag(Rd[k])
    out = dict(Q=Q, R=R, A=A, B=B, q=q, r=r, x0=x0, e=e)
    return {k: np.ascontiguousarray(v, dtype=np.float32) for k, v in out.items()}


def horizons_uniform_choice(batch: int, choices=(32, 64, 128, 256, 512), seed: int = 3000):
    """Per-problem horizons drawn uniformly from ``choices`` (the mixed-length batch)."""
    return [int(n) for n in np.random.default_rng(seed).choice(np.asarray(choices), batch)]


def horizons_uniform_int(batch: int, lo: int, hi: int, seed: int, first: int | None = None):
    """Per-problem horizons uniform on the integers [lo, hi]; optionally force the first."""
    Ns = [int(n) for n in np.random.default_rng(seed).integers(lo, hi + 1, batch)]
    if first is not None and batch:
        Ns[0] = int(first)
    return Ns


def batch(Ns, nx: int = 14, nu: int = 7, seed0: int = 0, q_lo: float = 1.0, q_hi: float = 10.0,
          defects: bool = False):
    """Problems b = 0..len(Ns)-1 drawn with seed ``seed0 + b`` (list of dicts)."""
    return [problem(int(n), nx, nu, seed0 + b, q_lo, q_hi, defects) for b, n in enumerate(Ns)]


def sequence(T: int, N: int, nx: int = 14, nu: int = 7, seed: int = 8000, q_lo: float = 1.0,
             q_hi: float = 10.0, drift: float = 0.05):
    """T consecutive receding-horizon subproblems of one synthetic trajectory.

    One problem of N + T - 1 knots is drawn with ``problem(seed)``; step t takes its knots
    t .. t+N-1 and controls t .. t+N-2, so consecutive steps share N - 1 knots shifted by
    one, as when a controller re-solves after advancing one knot.  The initial state of
    step t follows a drifting plant, x_{t+1} = A_t x_t + drift * w_t with
    w_t ~ N(0,1)^nx drawn from ``seed + 1``; it never depends on a solver's output.
    """
    if T < 1 or N < 1:
        raise ValueError("T and N must be >= 1")
    base = problem(N + T - 1, nx, nu, seed, q_lo, q_hi)
    g = np.random.default_rng(seed + 1)
    x = base["x0"].astype(np.float64)
    steps = []
    for t in range(T):
        p = {k: base[k][t:t + N] for k in ("Q", "q")}
        p.update({k: base[k][t:t + N - 1] for k in ("R", "A", "B", "r", "e")})
        p["x0"] = x.astype(np.float32)
        steps.append({k: np.ascontiguousarray(v, dtype=np.float32) for k, v in p.items()})
        if t + 1 < T:
            x = base["A"][t].astype(np.float64) @ x + drift * g.standard_normal(nx)
    return steps


def pack(probs):
    """Concatenate problems into the packed layout of the batched entry points.

    Knot-indexed arrays (Q, q) are stacked over knots; control-indexed arrays
    (R, A, B, r, e) over controls; x0 is [batch, nx].  Returns (packed dict, knot_off)
    where knot_off is int64 [batch+1] with knot_off[b+1]-knot_off[b] = N_b.  Problem b's
    control-indexed rows start at knot_off[b] - b.
    """
    off = np.zeros(len(probs) + 1, dtype=np.int64)
    for b, p in enumerate(probs):
        off[b + 1] = off[b] + p["Q"].shape[0]
    cat = lambda key: np.ascontiguousarray(np.concatenate([p[key] for p in probs], axis=0))
    packed = {k: cat(k) for k in ("Q", "R", "A", "B", "q", "r", "e")}
    packed["x0"] = np.ascontiguousarray(np.stack([p["x0"] for p in probs]))
    return packed, off


def unpack_knots(arr, off):
    """Split a knot-indexed packed array back into per-problem views."""
    return [arr[off[b]:off[b + 1]] for b in range(len(off) - 1)]


def unpack_controls(arr, off):
    """Split a control-indexed packed array back into per-problem views."""
    return [arr[off[b] - b:off[b + 1] - b - 1] for b in range(len(off) - 1)]


# ---- nonlinear control steps (the line search and the SQP iteration around the solve) ----
#
# The paper's controller linearises a rigid-body arm model at every step, solves the LQ
# subproblem, and line-searches the nonlinear problem.  The arm model is not available, so
# a chain of nq = nx / 2 pendulum joints coupled by nonlinear torsional springs stands in
# for it (nq torques, one per joint).  Only the draws live here; the dynamics themselves
# are written out separately by the library and by the oracle.
#
#   chain_model:  gravity ~ U[5, 15]^nq (seed), timestep h = 0.01, damping 0.5, coupling 2.
#   trajectory (PCG64 with `seed`, float64 draws in this order):
#     q_init ~ U[-1,1]^nq, v_init ~ 0.5 N(0,1)^nq          x_init = [q_init, v_init]
#     q_goal ~ U[-1,1]^nq                                   xref_k = [q_goal, 0] for all k
#     Xn ~ N(0,1)^(N,nx)    X_k = (1 - t_k) x_init + t_k xref_k + 0.3 Xn_k, t_k = k / (N-1)
#     Un ~ N(0,1)^(N-1,nu)  U_k = 0.5 Un_k
#     Qd ~ U[1,10]^(N,nx), W ~ N(0,1)^(N,nx,4)     Q_k = diag(Qd_k) + 0.1 W_k W_k^T
#     Rd ~ U[1e-3,1e-2]^(N-1,nu)                   R_k = diag(Rd_k)
#   so the initial guess violates the dynamics everywhere and the goal is away from x_init.


def chain_model(nq: int = 7, seed: int = 10000, h: float = 0.01, damping: float = 0.5,
                coupling: float = 2.0) -> dict:
    """Parameters of the pendulum-chain dynamics (gravity gains drawn from `seed`).

    The scalars are rounded to float32, the precision in which the library takes them, so
    that every consumer starts from the same values."""
    grav = np.random.default_rng(seed).uniform(5.0, 15.0, nq)
    f32 = lambda v: float(np.float32(v))
    return dict(h=f32(h), damping=f32(damping), coupling=f32(coupling),
                gravity=np.ascontiguousarray(grav, dtype=np.float32))


def trajectory(N: int, nx: int = 14, nu: int = 7, seed: int = 11000) -> dict:
    """One control step's nonlinear problem data: the current guess (X, U), the measured
    state x_init, the tracking target xref and the cost weights Q, R (all float32).

    Shapes: X [N,nx], U [N-1,nu], x_init [nx], xref [N,nx], Q [N,nx,nx], R [N-1,nu,nu].
    """
    if N < 1:
        raise ValueError("N must be >= 1")
    if nx != 2 * nu:
        raise ValueError("the chain model has nx = 2 nu (positions and velocities)")
    g = np.random.default_rng(seed)
    M = N - 1
    x_init = np.concatenate([g.uniform(-1.0, 1.0, nu), 0.5 * g.standard_normal(nu)])
    goal = np.concatenate([g.uniform(-1.0, 1.0, nu), np.zeros(nu)])
    Xn = g.standard_normal((N, nx))
    Un = g.standard_normal((M, nu))
    Qd = g.uniform(1.0, 10.0, (N, nx))
    W = g.standard_normal((N, nx, 4))
    Rd = g.uniform(1e-3, 1e-2, (M, nu))
    t = (np.arange(N) / max(N - 1, 1))[:, None]
    xref = np.tile(goal, (N, 1))
    X = (1.0 - t) * x_init + t * xref + 0.3 * Xn
    U = 0.5 * Un
    Q = np.zeros((N, nx, nx))
    for k in range(N):
        Q[k] = np.diag(Qd[k]) + 0.1 * (W[k] @ W[k].T)
    R = np.zeros((M, nu, nu))
    for k in range(M):
        R[k] = np.diag(Rd[k])
    out = dict(X=X, U=U, x_init=x_init, xref=xref, Q=Q, R=R)
    return {k: np.ascontiguousarray(v, dtype=np.float32) for k, v in out.items()}


def trajectories(Ns, nx: int = 14, nu: int = 7, seed0: int = 11000):
    """Trajectories b = 0..len(Ns)-1 drawn with seed ``seed0 + b``."""
    return [trajectory(int(n), nx, nu, seed0 + b) for b, n in enumerate(Ns)]


def pack_trajectories(trajs):
    """Packed layout of the batched control-step entry points (as `pack`): X, xref, Q
    stacked over knots, U, R over controls, x_init [batch, nx]; returns (dict, knot_off)."""
    off = np.zeros(len(trajs) + 1, dtype=np.int64)
    for b, t in enumerate(trajs):
        off[b + 1] = off[b] + t["X"].shape[0]
    cat = lambda key: np.ascontiguousarray(np.concatenate([t[key] for t in trajs], axis=0))
    packed = {k: cat(k) for k in ("X", "U", "xref", "Q", "R")}
    packed["x_init"] = np.ascontiguousarray(np.stack([t["x_init"] for t in trajs]))
    return packed, off

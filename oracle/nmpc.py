"""Plain FP64 reference for the steps around the linear solve (test infrastructure only).

One control step of the paper's controller (Section III-A, Steps 1-3; Section IV-C):

* Step 1, ``linearize``: the QP of Section III-A at the current guess (X, U).  The cost
  is the tracking cost J = sum_k 1/2 (x_k - xref_k)^T Q_k (x_k - xref_k)
  + sum_k 1/2 u_k^T R_k u_k, so its second-order expansion is exact: the QP's Q_k, R_k are
  the weights, q_k = Q_k (x_k - xref_k), r_k = R_k u_k.  The dynamics are linearised,
  A_k = df/dx, B_k = df/du at (x_k, u_k); the constraint residuals are
  e_k = x_{k+1} - f(x_k, u_k) and the initial-state target is dx_0 = x_s - x_0 (the
  library's ``x0`` input), exactly the c and constraints printed in Section III-A.
* Step 3 / Section IV-C, ``line_search``: the iterates z + alpha dz for every alpha in
  {1, 1/2, ..., 1/256}, each scored by the L1 merit
  phi(alpha) = J(z + alpha dz) + mu ||c(z + alpha dz)||_1 with
  c = [x_0 - x_s, e_0, ..., e_{N-2}]; the iterate with the smallest merit is taken.

The nonlinear model is a stand-in for the paper's arm (which is not available): a chain of
nq = nx / 2 pendulum joints with torsional springs between neighbours, one torque per
joint, stepped by explicit Euler with timestep h:
    q+ = q + h v
    v+ = v + h (u - g * sin(q) - d v + kappa (s_right - s_left))
where s_right_i = sin(q_{i+1} - q_i) (0 for the last joint) and s_left_i = s_right_{i-1}
(0 for the first joint).

Readings where the paper is silent (listed with the others in the design notes):
* penalty: mu_b = mu + ||lambda_b||_inf when multipliers are given, else mu (the L1 merit
  is exact once mu exceeds the multipliers' magnitude);
* ties: the first (largest) alpha with the smallest merit; there is no acceptance test.

Everything here is a plain loop over knots in float64 on the float32 inputs.
"""
from __future__ import annotations

import numpy as np

ALPHAS = tuple(2.0 ** -j for j in range(9))   # {1, 1/2, ..., 1/256}


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def chain_step(x, u, model):
    """x_{k+1} = f(x_k, u_k): one explicit Euler step of the pendulum chain."""
    x, u = _f64(x), _f64(u)
    nq = u.shape[0]
    q, v = x[:nq], x[nq:]
    h, d, kap = model["h"], model["damping"], model["coupling"]
    g = _f64(model["gravity"])
    acc = np.empty(nq)
    for i in range(nq):
        s_right = np.sin(q[i + 1] - q[i]) if i + 1 < nq else 0.0
        s_left = np.sin(q[i] - q[i - 1]) if i > 0 else 0.0
        acc[i] = u[i] - g[i] * np.sin(q[i]) - d * v[i] + kap * (s_right - s_left)
    return np.concatenate([q + h * v, v + h * acc])


def chain_jacobians(x, u, model):
    """A = df/dx and B = df/du of ``chain_step`` at (x, u), differentiated by hand."""
    x, u = _f64(x), _f64(u)
    nq = u.shape[0]
    q = x[:nq]
    h, d, kap = model["h"], model["damping"], model["coupling"]
    g = _f64(model["gravity"])
    dacc_dq = np.zeros((nq, nq))
    for i in range(nq):
        dacc_dq[i, i] = -g[i] * np.cos(q[i])
        if i + 1 < nq:                        # kappa sin(q_{i+1} - q_i)
            c = np.cos(q[i + 1] - q[i])
            dacc_dq[i, i + 1] += kap * c
            dacc_dq[i, i] -= kap * c
        if i > 0:                             # -kappa sin(q_i - q_{i-1})
            c = np.cos(q[i] - q[i - 1])
            dacc_dq[i, i] -= kap * c
            dacc_dq[i, i - 1] += kap * c
    I = np.eye(nq)
    A = np.block([[I, h * I], [h * dacc_dq, (1.0 - h * d) * I]])
    B = np.vstack([np.zeros((nq, nq)), h * I])
    return A, B


def linearize(traj, model):
    """Section III-A Step 1 at the guess (X, U): the LQ problem of the library's solve."""
    X, U = _f64(traj["X"]), _f64(traj["U"])
    xs, xref = _f64(traj["x_init"]), _f64(traj["xref"])
    Q, R = _f64(traj["Q"]), _f64(traj["R"])
    N, nx = X.shape
    nu = U.shape[1] if U.ndim == 2 else nx // 2
    A = np.zeros((N - 1, nx, nx))
    B = np.zeros((N - 1, nx, nu))
    e = np.zeros((N - 1, nx))
    q = np.zeros((N, nx))
    r = np.zeros((N - 1, nu))
    for k in range(N):
        q[k] = Q[k] @ (X[k] - xref[k])
    for k in range(N - 1):
        A[k], B[k] = chain_jacobians(X[k], U[k], model)
        e[k] = X[k + 1] - chain_step(X[k], U[k], model)
        r[k] = R[k] @ U[k]
    return dict(Q=Q, R=R, A=A, B=B, q=q, r=r, x0=xs - X[0], e=e)


def tracking_cost(X, U, traj):
    """J(X, U) = sum 1/2 (x_k - xref_k)^T Q_k (x_k - xref_k) + sum 1/2 u_k^T R_k u_k."""
    X, U = _f64(X), _f64(U)
    xref, Q, R = _f64(traj["xref"]), _f64(traj["Q"]), _f64(traj["R"])
    J = 0.0
    for k in range(X.shape[0]):
        d = X[k] - xref[k]
        J += 0.5 * d @ Q[k] @ d
    for k in range(U.shape[0]):
        J += 0.5 * U[k] @ R[k] @ U[k]
    return J


def violation(X, U, traj, model):
    """||c(X, U)||_1 with c = [x_0 - x_s, x_1 - f(x_0, u_0), ..., x_{N-1} - f(...)]."""
    X, U = _f64(X), _f64(U)
    v = np.abs(X[0] - _f64(traj["x_init"])).sum()
    for k in range(X.shape[0] - 1):
        v += np.abs(X[k + 1] - chain_step(X[k], U[k], model)).sum()
    return v


def penalty(mu, lam=None):
    """mu_b: mu, plus ||lambda_b||_inf when multipliers are given."""
    return float(mu) + (float(np.abs(_f64(lam)).max()) if lam is not None and np.size(lam) else 0.0)


def merit(X, U, traj, model, mu_b):
    """The L1 merit phi = J + mu_b ||c||_1 at (X, U)."""
    return tracking_cost(X, U, traj) + mu_b * violation(X, U, traj, model)


def select(merits):
    """Index of the smallest merit; the first (largest alpha) among equal values."""
    best = 0
    for j in range(1, len(merits)):
        if merits[j] < merits[best]:
            best = j
    return best


def line_search(traj, model, dX, dU, lam=None, mu=0.0):
    """Section IV-C: score every alpha of ALPHAS, keep the best iterate.

    Returns dict(merit [9] float64, choice int, mu float, X, U float32 updated iterate).
    The update is formed in float64 and rounded once to float32."""
    X, U = _f64(traj["X"]), _f64(traj["U"])
    dX, dU = _f64(dX), _f64(dU)
    mu_b = penalty(mu, lam)
    ph = np.array([merit(X + a * dX, U + a * dU, traj, model, mu_b) for a in ALPHAS])
    j = select(ph)
    a = ALPHAS[j]
    return dict(merit=ph, choice=j, mu=mu_b, X=(X + a * dX).astype(np.float32),
                U=(U + a * dU).astype(np.float32))

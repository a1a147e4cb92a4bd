"""Pins of the control-step oracle (oracle/nmpc.py): linearisation, merit, line search.

What fixes each part, independently of the formulas it checks:
* the model's torques against the gradient of its potential energy (finite differences of
  a separately written potential), and Newton's third law for the springs;
* the hand-written Jacobians against central differences of the step;
* the cost gradient (q, r of the QP) against central differences of the cost;
* with gravity and springs off the model is linear: the full SQP step from the exact
  KKT solve (oracle/kkt.py, LU) is then feasible, alpha = 1 has the smallest merit once
  mu exceeds the multipliers, a 16x overshoot selects alpha = 1/16, and the cost along the
  step is the quadratic J(0) + a g^T dz + a^2/2 dz^T G dz;
* the L1 merit's one-sided directional derivative along a step that satisfies the
  linearised constraints is g^T dz - mu ||c||_1, and it is negative when mu exceeds the
  multipliers (Nocedal & Wright, Numerical Optimization, Thm. 18.2);
* SQP iterations with this line search converge on the nonlinear model (constraint
  violation and step vanish, merit decreases).
A battery of planted mistakes checks that these pins catch plausible errors.  CPU only.
"""
import inspect
import types

import numpy as np
import pytest

from oracle import kkt
from oracle import nmpc
from paper_2309_08079_amd import synth


def model(nq=7, linear=False):
    m = synth.chain_model(nq, seed=10001)
    if linear:
        m = dict(m, coupling=0.0, gravity=np.zeros(nq, dtype=np.float32))
    return m


def rand_xu(nq, seed):
    g = np.random.default_rng(seed)
    return np.concatenate([g.uniform(-2, 2, nq), g.standard_normal(nq)]), g.standard_normal(nq)


def potential(q, m):
    # gravity and spring potential of the chain, written independently of the step
    g = np.asarray(m["gravity"], dtype=np.float64)
    V = float(np.sum(g * (1.0 - np.cos(q))))
    V += m["coupling"] * float(np.sum(1.0 - np.cos(np.diff(q))))
    return V


def central(f, x, h):
    x = np.asarray(x, dtype=np.float64)
    cols = []
    for i in range(x.size):
        d = np.zeros_like(x)
        d[i] = h
        cols.append((np.asarray(f(x + d)) - np.asarray(f(x - d))) / (2 * h))
    return np.stack(cols, axis=-1)


def sqp_step(traj, m):
    lq = nmpc.linearize(traj, m)
    ex = kkt.kkt_solve(lq)
    return lq, ex


def check_torques_are_potential_forces(mod):
    m = model()
    x, u = rand_xu(7, 1)
    q, v = x[:7], x[7:]
    acc = (mod.chain_step(x, u, m)[7:] - v) / m["h"]
    force = -central(lambda qq: potential(qq, m), q, 1e-6)
    return np.abs(acc - (u + force - m["damping"] * v)).max() < 1e-6


def check_springs_sum_to_zero(mod):
    m = dict(model(), gravity=np.zeros(7, dtype=np.float32), damping=0.0)
    x, _ = rand_xu(7, 2)
    acc = (mod.chain_step(x, np.zeros(7), m)[7:] - x[7:]) / m["h"]
    return abs(acc.sum()) < 1e-9 and np.abs(acc).max() > 1e-3


def check_jacobians(mod, nq=7):
    m = model(nq)
    ok = True
    for s in range(3):
        x, u = rand_xu(nq, 10 + s)
        A, B = mod.chain_jacobians(x, u, m)
        Af = central(lambda xx: mod.chain_step(xx, u, m), x, 1e-6)
        Bf = central(lambda uu: mod.chain_step(x, uu, m), u, 1e-6)
        ok &= np.abs(A - Af).max() < 1e-8 and np.abs(B - Bf).max() < 1e-8
    return ok


def check_cost_gradient(mod):
    t = synth.trajectory(4, seed=21)
    lq = mod.linearize(t, model())
    X, U = t["X"].astype(np.float64), t["U"].astype(np.float64)
    gX = central(lambda v: mod.tracking_cost(v.reshape(X.shape), U, t), X.ravel(), 1e-5)
    gU = central(lambda v: mod.tracking_cost(X, v.reshape(U.shape), t), U.ravel(), 1e-5)
    return (np.abs(gX - lq["q"].ravel()).max() < 1e-6 * np.abs(lq["q"]).max()
            and np.abs(gU - lq["r"].ravel()).max() < 1e-6 * np.abs(lq["r"]).max())


def check_linear_full_step(mod):
    m = model(linear=True)
    t = synth.trajectory(12, seed=22)
    lq = mod.linearize(t, m)
    ex = kkt.kkt_solve(lq)
    X1, U1 = t["X"] + ex["dx"], t["U"] + ex["du"]
    if mod.violation(X1, U1, t, m) > 1e-9 * mod.violation(t["X"], t["U"], t, m):
        return False
    ls = mod.line_search(t, m, ex["dx"], ex["du"], lam=ex["lam"], mu=1.0)
    if ls["choice"] != 0 or not np.all(ls["merit"] >= ls["merit"][0]):
        return False
    over = mod.line_search(t, m, 16 * ex["dx"], 16 * ex["du"], lam=ex["lam"], mu=1.0)
    if over["choice"] != 4:
        return False
    want = (t["X"].astype(np.float64) + ex["dx"]).astype(np.float32)
    return np.abs(over["X"].astype(np.float64) - want).max() <= 1e-6 * np.abs(want).max()


def check_cost_is_quadratic_along_step(mod):
    m = model()
    t = synth.trajectory(6, seed=23)
    lq, ex = sqp_step(t, m)
    dX, dU = ex["dx"], ex["du"]
    slope = np.sum(lq["q"] * dX) + np.sum(lq["r"] * dU)
    curv = np.einsum("ki,kij,kj->", dX, lq["Q"], dX) + np.einsum("ki,kij,kj->", dU, lq["R"], dU)
    J0 = mod.tracking_cost(t["X"], t["U"], t)
    for a in (1.0, 0.25, 3.0):
        Ja = mod.tracking_cost(t["X"] + a * dX, t["U"] + a * dU, t)
        if abs(Ja - (J0 + a * slope + 0.5 * a * a * curv)) > 1e-10 * max(abs(Ja), 1.0):
            return False
    return True


def check_directional_derivative(mod):
    m = model()
    t = synth.trajectory(10, seed=24)
    lq, ex = sqp_step(t, m)
    dX, dU = ex["dx"], ex["du"]
    mu_b = mod.penalty(0.0, ex["lam"])
    X, U = t["X"].astype(np.float64), t["U"].astype(np.float64)
    c1 = np.abs(lq["x0"]).sum() + np.abs(lq["e"]).sum()
    D = np.sum(lq["q"] * dX) + np.sum(lq["r"] * dU) - mu_b * c1
    s = 1e-7
    fd = (mod.merit(X + s * dX, U + s * dU, t, m, mu_b) - mod.merit(X, U, t, m, mu_b)) / s
    return D < 0 and abs(fd - D) < 1e-4 * abs(D)


def check_sqp_converges(mod):
    m = model()
    t = dict(synth.trajectory(8, seed=25))
    last = None
    for it in range(12):
        lq, ex = sqp_step(t, m)
        ls = mod.line_search(t, m, ex["dx"], ex["du"], lam=ex["lam"], mu=1.0)
        phi0 = mod.merit(t["X"], t["U"], t, m, ls["mu"])
        if ls["merit"][ls["choice"]] > phi0 + 1e-9 * abs(phi0):
            return False
        # the iterate is carried in float64 (the returned float32 one would floor the
        # violation at its rounding)
        a = mod.ALPHAS[ls["choice"]]
        t["X"] = np.asarray(t["X"], dtype=np.float64) + a * ex["dx"]
        t["U"] = np.asarray(t["U"], dtype=np.float64) + a * ex["du"]
        last = ex
    return (mod.violation(t["X"], t["U"], t, m) < 1e-11
            and max(np.abs(last["dx"]).max(), np.abs(last["du"]).max()) < 1e-10)


def check_select(mod):
    return (mod.select([3.0, 2.0, 2.0, 5.0]) == 1 and mod.select([1.0, 1.0]) == 0
            and mod.select([5, 4, 3, 2, 1, 0.5, 0.4, 0.3, 0.2]) == 8)


CHECKS = {
    "torques_are_potential_forces": check_torques_are_potential_forces,
    "springs_sum_to_zero": check_springs_sum_to_zero,
    "jacobians": check_jacobians,
    "cost_gradient": check_cost_gradient,
    "linear_full_step": check_linear_full_step,
    "cost_quadratic_along_step": check_cost_is_quadratic_along_step,
    "directional_derivative": check_directional_derivative,
    "sqp_converges": check_sqp_converges,
    "select": check_select,
}


@pytest.mark.parametrize("name", sorted(CHECKS))
def test_pin(name):
    assert CHECKS[name](nmpc), name


def test_jacobians_wide_chain():
    assert check_jacobians(nmpc, nq=14)


def test_linear_model_is_the_damped_double_integrator():
    # gravity and springs off: explicit Euler of q'' = u - d q' in closed form
    m = model(linear=True)
    h, d = m["h"], m["damping"]
    I, Z = np.eye(7), np.zeros((7, 7))
    A_ref = np.block([[I, h * I], [Z, (1 - h * d) * I]])
    B_ref = np.vstack([Z, h * I])
    x, u = rand_xu(7, 3)
    A, B = nmpc.chain_jacobians(x, u, m)
    assert np.abs(A - A_ref).max() == 0 and np.abs(B - B_ref).max() == 0
    assert np.abs(nmpc.chain_step(x, u, m) - (A_ref @ x + B_ref @ u)).max() < 1e-14


def test_line_search_single_knot():
    # N = 1: no dynamics, the merit is J + mu |x_0 - x_s|_1 along the step
    m = model()
    t = synth.trajectory(1, seed=26)
    lq, ex = sqp_step(t, m)
    ls = nmpc.line_search(t, m, ex["dx"], ex["du"], lam=ex["lam"], mu=1.0)
    assert ls["choice"] == 0
    assert np.abs(ls["X"][0] - t["x_init"]).max() < 1e-6


# ---- planted mistakes ----------------------------------------------------------------------

SRC = inspect.getsource(nmpc)

MUTANTS = {
    "coupling_sign": ("+ kap * (s_right - s_left)", "- kap * (s_right - s_left)"),
    "gravity_cos": ("- g[i] * np.sin(q[i])", "- g[i] * np.cos(q[i])"),
    "jac_drops_spring_diag": ("            dacc_dq[i, i + 1] += kap * c\n            dacc_dq[i, i] -= kap * c",
                              "            dacc_dq[i, i + 1] += kap * c"),
    "jac_damping_sign": ("(1.0 - h * d) * I", "(1.0 + h * d) * I"),
    "defect_sign": ("e[k] = X[k + 1] - chain_step(X[k], U[k], model)",
                    "e[k] = chain_step(X[k], U[k], model) - X[k + 1]"),
    "x0_sign": ("x0=xs - X[0]", "x0=X[0] - xs"),
    "cost_no_half": ("J += 0.5 * d @ Q[k] @ d", "J += d @ Q[k] @ d"),
    "gradient_ignores_ref": ("q[k] = Q[k] @ (X[k] - xref[k])", "q[k] = Q[k] @ X[k]"),
    "violation_skips_initial_state": ('v = np.abs(X[0] - _f64(traj["x_init"])).sum()', "v = 0.0"),
    "violation_squared": ("v += np.abs(X[k + 1] - chain_step(X[k], U[k], model)).sum()",
                          "v += (np.abs(X[k + 1] - chain_step(X[k], U[k], model)) ** 2).sum()"),
    "select_last_tie": ("if merits[j] < merits[best]:", "if merits[j] <= merits[best]:"),
    "update_ignores_choice": ("a = ALPHAS[j]", "a = ALPHAS[0]"),
    "penalty_ignores_multipliers": ("return float(mu) + (", "return float(mu) + 0.0 * ("),
}


def mutant(name):
    old, new = MUTANTS[name]
    assert SRC.count(old) == 1, name
    mod = types.ModuleType("nmpc_" + name)
    exec(compile(SRC.replace(old, new), "nmpc_" + name, "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    mod = mutant(name)
    failed = []
    for cname, check in CHECKS.items():
        try:
            if not check(mod):
                failed.append(cname)
        except (AssertionError, ValueError, np.linalg.LinAlgError):
            failed.append(cname)
    assert failed, name

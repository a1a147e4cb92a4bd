"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the C oracle (oracle/schur_pcg.c) against something other than itself:
the KKT definition solved by LU, the dense product C G^-1 C^T, the textbook LQR Riccati
recursion, a LAPACK banded Cholesky solve, closed forms of special cases, invariants of
the solution, exact rational PCG, and (for gradients) the dense KKT adjoint, torch FP64
autograd and central finite differences.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact, kkt
from oracle import ref as orc
from paper_2309_08079_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def relerr(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


@pytest.mark.parametrize("N,defects", [(1, False), (2, False), (5, True), (16, False), (16, True)])
def test_schur_blocks_equal_dense_definition(N, defects):
    # Section III-B: S = C G^-1 C^T, gamma = C G^-1 g - c (sign-flipped form)
    p = synth.problem(N, seed=10 + N, defects=defects)
    S, P, g = orc.form(p)
    Sd, gd = kkt.schur_dense(p)
    assert np.abs(kkt.blocks_to_dense(S) - Sd).max() <= 1e-13 * np.abs(Sd).max()
    assert np.abs(g - gd).max() <= 1e-13 * max(np.abs(gd).max(), 1)
    # S symmetric positive definite in the stored format (Section III-B)
    Sdense = kkt.blocks_to_dense(S)
    assert np.abs(Sdense - Sdense.T).max() <= 1e-14 * np.abs(Sdense).max()
    for b in range(N - 1):  # off-diagonal blocks are stored as exact transposes
        assert np.array_equal(S[b, 2], S[b + 1, 0].T)
    assert np.linalg.eigvalsh(Sdense).min() > 0


@pytest.mark.parametrize("N", [1, 2, 3, 8, 33])
def test_solution_matches_kkt_riccati_banded(N):
    p = synth.problem(N, seed=100 + N)
    o = orc.solve(p, eps=1e-14, max_iter=10 * N * 14)
    ex = kkt.kkt_solve(p)
    ri = kkt.riccati(p)
    S, _, g = orc.form(p)
    bd = kkt.banded_solve(S, g)
    for ref in (ex, ri):
        assert relerr(o["lam"], ref["lam"]) < 1e-10
        assert relerr(o["dx"], ref["dx"]) < 1e-10
        if N > 1:
            assert relerr(o["du"], ref["du"]) < 1e-10
    assert relerr(bd, ex["lam"]) < 1e-11


def test_pcg_tolerance_error_bound():
    # at eps = 1e-6 the oracle iterate is within the bound the stopping rule implies:
    # ||lam - lam*||_S <= ||r||_{S^-1} <= sqrt(eta / lambda_min(Phi^-1 S)), relative to
    # ||lam*||_S = sqrt(gamma^T S^-1 gamma) >= sqrt(eta_ref * lambda_min(...)) ...
    p = synth.problem(32, seed=1)
    o = orc.solve(p, eps=1e-6)
    ex = kkt.kkt_solve(p)
    S, P, _ = orc.form(p)
    Sd = kkt.blocks_to_dense(S)
    Pd = kkt.blocks_to_dense(P)
    ev = np.linalg.eigvals(Pd @ Sd).real
    kappa = ev.max() / ev.min()
    d = (o["lam"] - ex["lam"]).ravel()
    e_S = np.sqrt(d @ Sd @ d) / np.sqrt(ex["lam"].ravel() @ Sd @ ex["lam"].ravel())
    assert o["status"] == orc.OK and o["ratio"] < 1e-6
    assert e_S <= 1e-6 * np.sqrt(kappa) * 1.0001
    assert relerr(o["lam"], ex["lam"]) < 1e-5


def test_special_case_single_knot():
    # N = 1: S = Q0^-1 so lambda = q0 + Q0 x0, dx0 = x0 and Phi^-1 = S^-1 (1 iteration)
    p = synth.problem(1, seed=7)
    o = orc.solve(p)
    Q, q, x0 = (p[k].astype(np.float64) for k in ("Q", "q", "x0"))
    assert np.allclose(o["lam"][0], q[0] + Q[0] @ x0, rtol=1e-12, atol=1e-12)
    assert np.allclose(o["dx"][0], x0, rtol=1e-12, atol=1e-12)
    assert o["iters"] == 1


def test_special_case_zero_dynamics_one_iteration():
    # A_k = 0 makes S block diagonal, E = 0, Phi^-1 = D^-1 = S^-1: one iteration
    p = synth.problem(12, seed=8)
    p["A"][:] = 0
    o = orc.solve(p)
    assert o["iters"] == 1 and o["status"] == orc.OK
    assert relerr(o["lam"], kkt.kkt_solve(p)["lam"]) < 1e-12


@pytest.mark.parametrize("defects", [False, True])
def test_invariants_dynamics_and_stationarity(defects):
    p = synth.problem(20, seed=21, defects=defects)
    o = orc.solve(p, eps=1e-13)
    P = {k: v.astype(np.float64) for k, v in p.items()}
    dx, du, lam = o["dx"], o["du"], o["lam"]
    assert np.allclose(dx[0], P["x0"], atol=1e-12)
    for k in range(19):
        assert np.allclose(dx[k + 1], P["A"][k] @ dx[k] + P["B"][k] @ du[k] - P["e"][k], atol=1e-10)
        # stationarity in u_k and x_k of the Lagrangian (first block row of the KKT system)
        assert np.allclose(P["R"][k] @ du[k] + P["r"][k] + P["B"][k].T @ lam[k + 1], 0, atol=1e-9)
        assert np.allclose(lam[k], P["Q"][k] @ dx[k] + P["q"][k] + P["A"][k].T @ lam[k + 1], atol=1e-9)
    assert np.allclose(lam[19], P["Q"][19] @ dx[19] + P["q"][19], atol=1e-9)


def test_preconditioner_printed_entries_and_spectrum():
    # Section IV-A prints Phi^-1_00 = Q_0, Phi^-1_01 = -Q_0 phi_0^T theta_0^-1,
    # Phi^-1_10 = -theta_0^-1 phi_0 Q_0, Phi^-1_11 = theta_0^-1,
    # Phi^-1_12 = -theta_0^-1 phi_1^T theta_1^-1, Phi^-1_21 = -theta_1^-1 phi_1 theta_0^-1
    p = synth.problem(6, seed=31)
    S, P, _ = orc.form(p)
    Q0 = p["Q"][0].astype(np.float64)
    th0i, th1i = np.linalg.inv(S[1, 1]), np.linalg.inv(S[2, 1])
    phi0, phi1 = S[1, 0], S[2, 0]
    tol = lambda M: 1e-12 * np.abs(M).max()
    assert np.abs(P[0, 1] - Q0).max() < tol(Q0) * 10
    assert np.abs(P[0, 2] - (-Q0 @ phi0.T @ th0i)).max() < tol(P[0, 2]) * 10
    assert np.abs(P[1, 0] - (-th0i @ phi0 @ Q0)).max() < tol(P[1, 0]) * 10
    assert np.abs(P[1, 1] - th0i).max() < tol(th0i)
    assert np.abs(P[1, 2] - (-th0i @ phi1.T @ th1i)).max() < tol(P[1, 2]) * 10
    assert np.abs(P[2, 0] - (-th1i @ phi1 @ th0i)).max() < tol(P[2, 0]) * 10
    # Phi^-1 S = I - (D^-1 E)^2, Phi^-1 symmetric positive definite, spec(Phi^-1 S) in (0, 1]
    Sd, Pd = kkt.blocks_to_dense(S), kkt.blocks_to_dense(P)
    D = kkt.blocks_to_dense(np.stack([np.stack([np.zeros_like(S[0, 1]), S[b, 1], np.zeros_like(S[0, 1])]) for b in range(6)]))
    E = Sd - D
    DiE = np.linalg.solve(D, E)
    assert np.abs(Pd @ Sd - (np.eye(len(Sd)) - DiE @ DiE)).max() < 1e-11
    assert np.abs(Pd - Pd.T).max() < 1e-11 * np.abs(Pd).max()
    assert np.linalg.eigvalsh(0.5 * (Pd + Pd.T)).min() > 0
    ev = np.sort(np.linalg.eigvals(Pd @ Sd).real)
    assert ev.min() > 0 and ev.max() <= 1 + 1e-10


def _rational_problem(N, nx, nu, seed):
    rng = np.random.default_rng(seed)
    Q, R, A, B, q, r = [], [], [], [], [], []
    for k in range(N):
        W = rng.integers(-2, 3, (nx, 2))
        Q.append([[Fraction(int(W[i] @ W[j])) + (Fraction(int(rng.integers(2, 6))) if i == j else 0)
                   for j in range(nx)] for i in range(nx)])
        q.append([Fraction(int(v)) for v in rng.integers(-3, 4, nx)])
    for k in range(N - 1):
        R.append([[Fraction(int(rng.integers(1, 4))) if i == j else Fraction(0) for j in range(nu)] for i in range(nu)])
        A.append([[Fraction(int(i == j)) + Fraction(int(rng.integers(-2, 3)), 10) for j in range(nx)] for i in range(nx)])
        B.append([[Fraction(int(rng.integers(-3, 4)), 10) for j in range(nu)] for i in range(nx)])
        r.append([Fraction(int(v)) for v in rng.integers(-3, 4, nu)])
    x0 = [Fraction(int(v)) for v in rng.integers(-2, 3, nx)]
    return Q, R, A, B, q, r, x0


def _to_np(Q, R, A, B, q, r, x0):
    f = lambda a: np.array([[float(x) for x in row] for row in a]) if a and isinstance(a[0], list) else np.array([float(x) for x in a])
    arr = lambda L, shape: np.stack([f(m) for m in L]) if L else np.zeros(shape)
    return dict(Q=arr(Q, None), R=arr(R, (0, len(R[0]) if R else 1, 1)), A=arr(A, None) if A else np.zeros((0, len(Q[0]), len(Q[0]))),
                B=arr(B, None) if B else np.zeros((0, len(Q[0]), 1)), q=np.array([[float(x) for x in v] for v in q]),
                r=np.array([[float(x) for x in v] for v in r]) if r else np.zeros((0, 1)), x0=np.array([float(x) for x in x0]))


@pytest.mark.parametrize("N,nx,nu,seed", [(3, 2, 1, 0), (4, 2, 1, 1), (5, 3, 1, 2), (6, 2, 1, 3)])
def test_exact_rational_pcg_terminates_and_matches_fp64_trace(N, nx, nu, seed):
    Q, R, A, B, q, r, x0 = _rational_problem(N, nx, nu, seed)
    S, P, g = exact.form(Q, R, A, B, q, r, x0)
    lam, iters, etas = exact.pcg(S, P, g)
    # exact termination within floor(N/2)*nx + 1 <= dim S iterations
    assert etas[-1] == 0
    assert iters <= (N // 2) * nx + 1 <= N * nx
    # exact solution satisfies the KKT system
    prob = _to_np(Q, R, A, B, q, r, x0)
    ex = kkt.kkt_solve(prob)
    lamf = np.array([[float(x) for x in v] for v in lam])
    assert relerr(lamf, ex["lam"]) < 1e-12
    # the FP64 oracle follows the same eta trace (until it reaches its own stop)
    o = orc.solve(prob, eps=1e-15, max_iter=iters + 3, trace=True)
    n = min(len(o["eta"]), len(etas)) - 1
    et = np.array([float(x) for x in etas[:n]])
    assert np.allclose(o["eta"][:n], et, rtol=1e-9, atol=1e-12 * et[0])
    assert relerr(o["lam"], lamf) < 1e-9


def test_stopping_rule_first_iteration_below_eps():
    p = synth.problem(32, seed=1)
    o = orc.solve(p, eps=1e-6, trace=True)
    S, P, g = orc.form(p)
    eta_ref = float(g.ravel() @ kkt.blocks_to_dense(P) @ g.ravel())
    ratios = np.sqrt(o["eta"] / eta_ref)
    assert ratios[-1] < 1e-6 and np.all(ratios[:-1] >= 1e-6)
    assert o["iters"] == len(o["eta"]) - 1
    assert abs(o["ratio"] - ratios[-1]) < 1e-12


@pytest.mark.parametrize("N,nx,nu,seed", [(5, 3, 1, 2), (6, 2, 1, 3)])
def test_absolute_stopping_rule_against_exact_trace(N, nx, nu, seed):
    # Algorithm 1 as printed: stop at the first eta' < eps (absolute).  The exact rational
    # eta sequence fixes which iteration that is; eps sits halfway (geometrically) between
    # two exact values so rounding cannot move the crossing.
    Q, R, A, B, q, r, x0 = _rational_problem(N, nx, nu, seed)
    S, P, g = exact.form(Q, R, A, B, q, r, x0)
    _, iters, etas = exact.pcg(S, P, g)
    ef = [float(x) for x in etas]
    prob = _to_np(Q, R, A, B, q, r, x0)
    checked = 0
    for k in range(1, len(ef) - 1):
        prev = min(ef[:k])
        if not 0.0 < ef[k] < 0.5 * prev:
            continue
        eps = float(np.sqrt(ef[k] * prev))   # first value below eps is eta_k
        o = orc.solve(prob, eps=eps, stop="absolute", max_iter=iters + 3)
        assert o["status"] == orc.OK and o["iters"] == k, (k, eps, ef)
        checked += 1
    assert checked >= 2


def test_absolute_rule_equals_relative_rule_at_scaled_eps():
    # eta' < eps_rel^2 eta_ref  is the absolute rule with eps_abs = eps_rel^2 eta_ref, with
    # eta_ref = gamma^T Phi^-1 gamma taken from the dense definitions
    p = synth.problem(24, seed=5)
    Sd, gd = kkt.schur_dense(p)
    gd = gd.ravel()
    _, P, _ = orc.form(p)
    eta_ref = float(gd @ kkt.blocks_to_dense(P) @ gd)
    rel = orc.solve(p, eps=1e-5)
    ab = orc.solve(p, eps=(1e-5) ** 2 * eta_ref, stop="absolute")
    assert rel["iters"] == ab["iters"] and np.array_equal(rel["lam"], ab["lam"])
    # and the absolute rule stops where the dense residual first satisfies it
    for eps in (1e-2, 1e-4):
        o = orc.solve(p, eps=eps, stop="absolute", trace=True)
        assert o["eta"][-1] < eps and np.all(o["eta"][:-1] >= eps)
        res = gd - Sd @ o["lam"].ravel()
        eta_dense = float(res @ kkt.blocks_to_dense(P) @ res)
        assert eta_dense < eps * (1 + 1e-6)
    with pytest.raises(ValueError):
        orc.solve(p, stop="sometimes")


def test_fp32_preconditioner_mode_changes_path_not_solution():
    # phi="fp32" rounds every Phi^-1 entry to single precision before PCG: eta_0 is then
    # gamma^T round32(Phi^-1) gamma (dense, from the formed blocks), the trace differs from
    # the FP64 one, and the converged solution is still the KKT solution
    p = synth.problem(20, seed=8)
    S, P, g = orc.form(p)
    gv = g.ravel()
    P32 = kkt.blocks_to_dense(P.astype(np.float32).astype(np.float64))
    o32 = orc.solve(p, eps=1e-6, trace=True, phi="fp32")
    o64 = orc.solve(p, eps=1e-6, trace=True)
    assert abs(o32["eta"][0] - gv @ P32 @ gv) <= 1e-12 * abs(o32["eta"][0])
    assert abs(o64["eta"][0] - gv @ P32 @ gv) > 1e-12 * abs(o64["eta"][0])
    ex = kkt.kkt_solve(p)
    c = orc.solve(p, eps=1e-14, max_iter=2000, phi="fp32")
    assert c["status"] == orc.OK and relerr(c["lam"], ex["lam"]) < 1e-9
    with pytest.raises(ValueError):
        orc.solve(p, phi="fp16")


def test_status_paths():
    p = synth.problem(16, seed=3)
    assert orc.solve(p, max_iter=1)["status"] == orc.NOT_CONVERGED
    bad = {k: v.copy() for k, v in p.items()}
    bad["Q"][3] = -bad["Q"][3]
    assert orc.solve(bad)["status"] == orc.BREAKDOWN
    nan = {k: v.copy() for k, v in p.items()}
    nan["q"][2, 1] = np.nan
    assert orc.solve(nan)["status"] == orc.BREAKDOWN
    # gamma = 0 (q = r = x0 = 0): lambda = 0 after 0 iterations
    z = {k: v.copy() for k, v in p.items()}
    for k in ("q", "r", "x0"):
        z[k][:] = 0
    o = orc.solve(z)
    assert o["iters"] == 0 and o["status"] == orc.OK and not o["lam"].any()
    # warm start at the exact solution: accepted before the first iteration
    ex = kkt.kkt_solve(p)
    assert orc.solve(p, lam0=ex["lam"])["iters"] == 0


def test_problem_sizes_printed_in_paper():
    # Section V-B: the experiments range from 448 to 7,168 variables (32 to 512 knots, nx = 14)
    with open(os.path.join(HERE, "golden", "paper_sizes.json")) as f:
        g = json.load(f)
    for case in g["cases"]:
        p = synth.problem(case["knots"], nx=14, nu=7, seed=0) if case["knots"] <= 32 else None
        assert case["knots"] * 14 == case["variables"]
        if p is not None:
            S, _, _ = orc.form(p)
            assert S.shape[0] * S.shape[2] == case["variables"]


# ---- gradients ---------------------------------------------------------------------------

GRAD_KEYS = ("dQ", "dR", "dA", "dB", "dq", "dr", "dx0", "de")


def test_adjoint_matches_dense_adjoint_and_autograd():
    p = synth.problem(8, seed=4000, defects=True)
    f = orc.solve(p, eps=1e-14)
    gl = 2 * f["lam"]
    b = orc.backward(p, f, gl, eps=1e-14)
    d = kkt.adjoint_dense(p, gl)
    a = kkt.autograd_grads(p)
    for k in GRAD_KEYS:
        assert relerr(b[k], d[k]) < 1e-9, k
        assert relerr(a[k], d[k]) < 1e-9, k


def test_adjoint_with_primal_loss_terms_matches_dense():
    p = synth.problem(7, seed=44)
    f = orc.solve(p, eps=1e-14)
    rng = np.random.default_rng(0)
    gl, gx, gu = rng.standard_normal(f["lam"].shape), rng.standard_normal(f["dx"].shape), rng.standard_normal(f["du"].shape)
    b = orc.backward(p, f, gl, gx, gu, eps=1e-14)
    d = kkt.adjoint_dense(p, gl, gx, gu)
    for k in GRAD_KEYS:
        assert relerr(b[k], d[k]) < 1e-9, k


def test_adjoint_single_knot_closed_form():
    # N = 1, L = ||lambda_0||^2 with lambda_0 = q0 + Q0 x0:
    # dL/dq0 = 2 lambda_0, dL/dx0 = 2 Q0 lambda_0, dL/dQ0 = sym(2 lambda_0 x0^T)
    p = synth.problem(1, seed=5)
    f = orc.solve(p)
    l0 = f["lam"][0]
    b = orc.backward(p, f, 2 * f["lam"])
    Q0, x0 = p["Q"][0].astype(np.float64), p["x0"].astype(np.float64)
    assert np.allclose(b["dq"][0], 2 * l0, rtol=1e-12)
    assert np.allclose(b["dx0"], 2 * Q0 @ l0, rtol=1e-12)
    G = 2 * np.outer(l0, x0)
    assert np.allclose(b["dQ"][0], 0.5 * (G + G.T), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("h,tol", [(1e-4, 1e-5), (1e-6, 1e-4)])
def test_adjoint_matches_central_finite_differences(h, tol):
    # L = ||lambda||^2 at N = 8; symmetric inputs perturbed symmetrically
    p = {k: v.astype(np.float64) for k, v in synth.problem(8, seed=4000).items()}
    L = lambda pp: float(np.sum(kkt.kkt_solve(pp)["lam"] ** 2))
    f = orc.solve(p, eps=1e-14)
    b = orc.backward(p, f, 2 * f["lam"], eps=1e-14)
    rng = np.random.default_rng(1)
    for gkey in GRAD_KEYS:
        key = gkey[1:]
        arr = p[key]
        if arr.size == 0:
            continue
        idxs = [tuple(ix) for ix in np.argwhere(np.ones(arr.shape, bool))]
        pick = [idxs[i] for i in rng.choice(len(idxs), min(12, len(idxs)), replace=False)]
        got, want = [], []
        for ix in pick:
            sym = key in ("Q", "R") and ix[-1] != ix[-2]

            def bump(s):
                q2 = {k: v.copy() for k, v in p.items()}
                q2[key][ix] += s * (h / 2 if sym else h)
                if sym:
                    q2[key][ix[:-2] + (ix[-1], ix[-2])] += s * h / 2
                return q2
            want.append((L(bump(1)) - L(bump(-1))) / (2 * h))
            got.append(b[gkey][ix])
        assert relerr(np.array(got), np.array(want)) < tol, gkey


@pytest.mark.parametrize("N,nx,nu", [(1, 14, 7), (2, 14, 7), (9, 14, 7), (6, 28, 14)])
def test_primal_step_of_exact_multipliers_is_exact_primal(N, nx, nu):
    # dZ = -G^-1 (g - C^T lambda) at the exact lambda gives the exact dZ of the KKT solve, and
    # a perturbation of lambda moves dZ by G^-1 C^T times it (linear in lambda)
    p = synth.problem(N, nx, nu, seed=300 + N, defects=True)
    ex = kkt.kkt_solve(p)
    dx, du = kkt.primal_step(p, ex["lam"])
    assert relerr(dx, ex["dx"]) < 1e-11 and (N == 1 or relerr(du, ex["du"]) < 1e-11)
    d = np.random.default_rng(7).standard_normal(ex["lam"].shape)
    dx2, du2 = kkt.primal_step(p, ex["lam"] + d)
    G, g, Cm, _ = kkt.assemble(p)
    dz = np.linalg.solve(G, Cm.T @ d.ravel())
    lin = np.concatenate([dx2.ravel() - dx.ravel(), (du2 - du).ravel()]) if N > 1 else dx2.ravel() - dx.ravel()
    ref = np.concatenate([dz[k * (nx + nu):k * (nx + nu) + nx] for k in range(N)] +
                         [dz[k * (nx + nu) + nx:(k + 1) * (nx + nu)] for k in range(N - 1)])
    assert relerr(lin, ref) < 1e-10

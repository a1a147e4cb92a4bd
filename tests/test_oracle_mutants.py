"""Planted mistakes in the CPU oracle must be caught by its pins.

Each case compiles a copy of oracle/schur_pcg.c with one plausible mistake (a dropped term,
a wrong sign, a transposed operand, a wrong stopping rule, ...) and runs a battery of the
checks that pin the oracle: the dense definition of S and gamma, the KKT / Riccati solution,
the preconditioner identity, the first-crossing stopping rule, exact rational PCG and the
dense adjoint.  Every mutant must fail at least one of them (and the unmodified source must
pass all of them).  Everything runs on the CPU.
"""
import ctypes
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact, kkt
from oracle import ref as orc
from paper_2309_08079_amd import synth

SRC = os.path.join(os.path.dirname(orc.__file__), "schur_pcg.c")

MUTANTS = {
    "phi_sign": ("phi[i * nx + j] = -T[i * nx + j];", "phi[i * nx + j] = T[i * nx + j];"),
    "theta_drops_Qinv_next": ("theta[t] += V[t] + Qik1[t];", "theta[t] += V[t];"),
    "theta_A_not_transposed": ("matmul(nx, nx, nx, T, 0, Ak, 1, theta);", "matmul(nx, nx, nx, T, 0, Ak, 0, theta);"),
    "gamma0_x0_sign": ("for (int i = 0; i < nx; ++i) gam[i] += p->x0[i];", "for (int i = 0; i < nx; ++i) gam[i] -= p->x0[i];"),
    "gamma_defect_sign": ("g1[i] += v[i] - (p->e ? p->e[(size_t)k * nx + i] : 0.0);", "g1[i] += v[i] + (p->e ? p->e[(size_t)k * nx + i] : 0.0);"),
    "zeta_drops_control_term": ("for (int i = 0; i < nx; ++i) g1[i] = -v[i] - w[i];", "for (int i = 0; i < nx; ++i) g1[i] = -v[i];"),
    "precond_offdiag_sign": ("for (size_t t = 0; t < bs; ++t) dst[t] = -V[t];", "for (size_t t = 0; t < bs; ++t) dst[t] = V[t];"),
    "alpha_scaled": ("const double alpha = eta / pSp;", "const double alpha = 0.9 * eta / pSp;"),
    "beta_inverted": ("const double beta = eta_new / eta;", "const double beta = eta / eta_new;"),
    "stop_rule_unsquared": ("const double tau = stop_abs ? eps : eps * eps * eta_ref;",
                            "const double tau = stop_abs ? eps : eps * eta_ref;"),
    "stop_abs_scaled": ("const double tau = stop_abs ? eps : eps * eps * eta_ref;",
                        "const double tau = stop_abs ? eps * eta_ref : eps * eps * eta_ref;"),
    "recon_lambda_sign": ("for (int i = 0; i < nx; ++i) t[i] = gx[(size_t)k * nx + i] - lam[(size_t)k * nx + i];",
                          "for (int i = 0; i < nx; ++i) t[i] = gx[(size_t)k * nx + i] + lam[(size_t)k * nx + i];"),
    "recon_B_not_transposed": ("matvec(nu, nx, p->B + (size_t)k * nx * nu, 1, lam + (size_t)(k + 1) * nx, s);",
                               "matvec(nu, nx, p->B + (size_t)k * nx * nu, 0, lam + (size_t)(k + 1) * nx, s);"),
    "phi32_not_rounded": ("static void round_to_float(double *a, size_t n) {\n  for (size_t i = 0; i < n; ++i) a[i] = (double)(float)a[i];",
                          "static void round_to_float(double *a, size_t n) {\n  for (size_t i = 0; i < n; ++i) a[i] = a[i];"),
    "adjoint_dA_sign": ("dA[(size_t)k * bs + i * nx + j] = l1[i] * ax[j] + m1[i] * xk[j];",
                        "dA[(size_t)k * bs + i * nx + j] = l1[i] * ax[j] - m1[i] * xk[j];"),
    "adjoint_dQ_unsymmetrised": ("dQ[(size_t)k * bs + i * nx + j] = 0.5 * (ax[i] * xk[j] + ax[j] * xk[i]);",
                                 "dQ[(size_t)k * bs + i * nx + j] = ax[i] * xk[j];"),
    "adjoint_dx0_sign": ("if (dx0) memcpy(dx0, mu, nx * sizeof(double));",
                         "if (dx0) for (int i = 0; i < nx; ++i) dx0[i] = -mu[i];"),
    # the batched wrappers: control rows of problem b start at off[b] - b, x0 at row b
    "batch_control_offset": ("const int64_t k0 = off[b], c0 = off[b] - b;\n    const int N = (int)(off[b + 1] - off[b]);\n    status[b] = orc_solve(",
                             "const int64_t k0 = off[b], c0 = off[b];\n    const int N = (int)(off[b + 1] - off[b]);\n    status[b] = orc_solve("),
    "batch_x0_row": ("q + k0 * nx, r + c0 * nu, x0 + (size_t)b * nx, e ? e + c0 * nx : NULL,\n                          eps,",
                     "q + k0 * nx, r + c0 * nu, x0, e ? e + c0 * nx : NULL,\n                          eps,"),
    "batch_backward_control_offset": ("const int64_t k0 = off[b], c0 = off[b] - b;\n    const int N = (int)(off[b + 1] - off[b]);\n    status[b] = orc_backward(",
                                      "const int64_t k0 = off[b], c0 = off[b] - b + 1;\n    const int N = (int)(off[b + 1] - off[b]);\n    status[b] = orc_backward("),
    "batch_backward_loss_rows": ("du + c0 * nu, gl + k0 * nx, gx ? gx + k0 * nx : NULL,",
                                 "du + c0 * nu, gl + c0 * nx, gx ? gx + k0 * nx : NULL,"),
}


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def battery():
    """Pin checks on the library currently loaded in oracle.ref; returns failed check names."""
    failed = []
    p = synth.problem(6, seed=91, defects=True)
    try:
        S, P, g = orc.form(p)
        Sd, gd = kkt.schur_dense(p)
        if np.abs(kkt.blocks_to_dense(S) - Sd).max() > 1e-12 * np.abs(Sd).max() or np.abs(g - gd).max() > 1e-12 * np.abs(gd).max():
            failed.append("schur_dense")
        Sdn, Pdn = kkt.blocks_to_dense(S), kkt.blocks_to_dense(P)
        D = np.zeros_like(Sdn)
        for b in range(6):
            D[b * 14:(b + 1) * 14, b * 14:(b + 1) * 14] = S[b, 1]
        DiE = np.linalg.solve(D, Sdn - D)
        if np.abs(Pdn @ Sdn - (np.eye(len(Sdn)) - DiE @ DiE)).max() > 1e-10:
            failed.append("preconditioner_identity")
    except ValueError:
        failed.append("form_status")
    o = orc.solve(p, eps=1e-14, max_iter=500)
    ex = kkt.kkt_solve(p)
    if o["status"] != orc.OK or rel(o["lam"], ex["lam"]) > 1e-9 or rel(o["dx"], ex["dx"]) > 1e-9 or rel(o["du"], ex["du"]) > 1e-9:
        failed.append("kkt_solution")
    # first-crossing stopping rule against eta_ref from the dense definitions
    q = synth.problem(20, seed=92)
    o = orc.solve(q, eps=1e-6, trace=True)
    Sq, Pq, gq = orc.form(q)
    eta_ref = float(gq.ravel() @ kkt.blocks_to_dense(Pq) @ gq.ravel())
    ratios = np.sqrt(np.abs(o["eta"]) / eta_ref)
    if not (ratios[-1] < 1e-6 and np.all(ratios[:-1] >= 1e-6)):
        failed.append("stopping_rule")
    gq = gq.ravel()
    P32 = kkt.blocks_to_dense(Pq.astype(np.float32).astype(np.float64))
    o32 = orc.solve(q, eps=1e-6, trace=True, phi="fp32")
    if abs(o32["eta"][0] - gq @ P32 @ gq) > 1e-12 * abs(o32["eta"][0]):
        failed.append("phi_fp32_mode")
    oa = orc.solve(q, eps=1e-3, stop="absolute", trace=True)
    if not (oa["eta"][-1] < 1e-3 and np.all(oa["eta"][:-1] >= 1e-3)):
        failed.append("stopping_rule_absolute")
    # exact rational PCG trace
    rng = np.random.default_rng(7)
    N, nx, nu = 4, 2, 1
    Q = [[[Fraction(int(v)) for v in row] for row in (np.eye(nx) * 3 + 1)] for _ in range(N)]
    R = [[[Fraction(2)]] for _ in range(N - 1)]
    A = [[[Fraction(int(i == j)) + Fraction(int(rng.integers(-2, 3)), 10) for j in range(nx)] for i in range(nx)] for _ in range(N - 1)]
    B = [[[Fraction(int(rng.integers(-3, 4)), 10)] for _ in range(nx)] for _ in range(N - 1)]
    qv = [[Fraction(int(v)) for v in rng.integers(-3, 4, nx)] for _ in range(N)]
    rv = [[Fraction(int(rng.integers(-3, 4)))] for _ in range(N - 1)]
    x0 = [Fraction(1), Fraction(-2)]
    Se, Pe, ge = exact.form(Q, R, A, B, qv, rv, x0)
    lam_e, it_e, etas = exact.pcg(Se, Pe, ge)
    npf = lambda L: np.array([[float(x) for x in r] for r in L])
    prob = dict(Q=np.stack([npf(m) for m in Q]), R=np.stack([npf(m) for m in R]), A=np.stack([npf(m) for m in A]),
                B=np.stack([npf(m) for m in B]), q=npf(qv), r=npf(rv), x0=np.array([float(x) for x in x0]))
    oe = orc.solve(prob, eps=1e-15, max_iter=it_e + 3, trace=True)
    n = min(len(oe["eta"]), len(etas)) - 1
    et = np.array([float(x) for x in etas[:n]])
    if not np.allclose(oe["eta"][:n], et, rtol=1e-9, atol=1e-12 * et[0]):
        failed.append("exact_trace")
    # adjoint against the dense KKT adjoint
    f = orc.solve(p, eps=1e-14, max_iter=500)
    gl = 2 * f["lam"]
    b = orc.backward(p, f, gl, eps=1e-14, max_iter=500)
    d = kkt.adjoint_dense(p, gl)
    for k in ("dQ", "dR", "dA", "dB", "dq", "dr", "dx0", "de"):
        if rel(b[k], d[k]) > 1e-8:
            failed.append("adjoint_" + k)
            break
    failed += batch_wrapper_failures()
    return failed


def batch_wrapper_failures():
    """The batched entry points against per-problem solves of the unpacked problems: a
    ragged batch with a one-knot problem and defects must give the per-problem results bit
    for bit (forward and adjoint), row for row in the packed layout."""
    probs = synth.batch([3, 1, 6, 2, 5], seed0=93, defects=True)
    packed, off = synth.pack(probs)
    fb = orc.solve_batch(packed, off, eps=1e-8)
    gl = np.random.default_rng(94).standard_normal(fb["lam"].shape)
    bb = orc.backward_batch(packed, off, fb, gl, eps=1e-8)
    for b, p in enumerate(probs):
        k0, k1 = off[b], off[b + 1]
        c0, c1 = k0 - b, k1 - b - 1
        f = orc.solve(p, eps=1e-8)
        if not (np.array_equal(fb["lam"][k0:k1], f["lam"]) and np.array_equal(fb["dx"][k0:k1], f["dx"])
                and np.array_equal(fb["du"][c0:c1], f["du"]) and fb["iters"][b] == f["iters"]):
            return ["batch_forward"]
        g = orc.backward(p, dict(lam=fb["lam"][k0:k1], dx=fb["dx"][k0:k1], du=fb["du"][c0:c1]),
                         gl[k0:k1], eps=1e-8)
        same = all(np.array_equal(bb[k][k0:k1], g[k]) for k in ("dQ", "dq", "mu"))
        same = same and all(np.array_equal(bb[k][c0:c1], g[k]) for k in ("dR", "dA", "dB", "dr", "de"))
        if not (same and np.array_equal(bb["dx0"][b], g["dx0"]) and bb["iters"][b] == g["iters"]):
            return ["batch_backward"]
    return []


def test_batched_wrappers_equal_per_problem_solves():
    # orc_solve_batch / orc_backward_batch are the reference of every batched GPU parity
    # test: pinned here against the per-problem entry points, which the other pins fix
    assert batch_wrapper_failures() == []


def _with_library(path):
    saved = orc._lib
    orc._lib = orc.configure(ctypes.CDLL(path))
    try:
        return battery()
    finally:
        orc._lib = saved


def test_unmodified_oracle_passes_battery(tmp_path):
    out = orc.compile_source(SRC, str(tmp_path / "base.so"))
    assert _with_library(out) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    find, repl = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(find) == 1, "mutation site not unique: " + name
    src = tmp_path / (name + ".c")
    src.write_text(text.replace(find, repl))
    out = orc.compile_source(str(src), str(tmp_path / (name + ".so")))
    failed = _with_library(out)
    assert failed, "planted mistake %s passed every pin" % name

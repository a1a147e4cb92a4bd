"""GPU tests of the factor record: a forward solve that keeps its preconditioner Phi^-1
(mpcpcg_solve_batched_keep) and the adjoint that reads it back instead of forming it again
(mpcpcg_backward_reuse).  S is symmetric, so the adjoint system has the forward's matrix
and preconditioner (Section III-B, Section IV-A); reading Phi^-1 back must change nothing:
every output is compared bit for bit with the plain calls, whose parity with the oracle
the other tests establish, and one batch again with the oracle's adjoint fed the oracle's
forward."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ref as orc
from paper_2309_08079_amd import synth

pytestmark = pytest.mark.gpu

EPS = 1e-6
GRADS = ("dQ", "dR", "dA", "dB", "dq", "dr", "dx0", "de", "dgamma", "stats")


def dev(p):
    from paper_2309_08079_amd.mpcpcg import to_device
    return to_device(p)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.fixture()
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08079_amd.mpcpcg import Context
    c = Context(14, 7, max_total_knots=1 << 14, max_batch=64)
    yield c
    c.close()


def clone(d):
    return {k: v.clone() for k, v in d.items()}


def plain_and_kept(ctx, d, off, warm=None):
    """Forward and adjoint without and with the factor record (same inputs, same loss)."""
    lam0 = None if warm is None else warm
    f0 = clone(ctx.mpcpcg_solve_batched(d, off, eps=EPS, lam0=lam0))
    g0 = clone(ctx.mpcpcg_backward(d, off, f0, 2 * f0["lam"], f0["dx"], None, eps=EPS))
    rec = ctx.factor_record(int(off[-1]), d["q"].device)
    f1 = clone(ctx.mpcpcg_solve_batched(d, off, eps=EPS, lam0=lam0, factors=rec))
    g1 = clone(ctx.mpcpcg_backward(d, off, f1, 2 * f1["lam"], f1["dx"], None, eps=EPS, factors=rec))
    torch.cuda.synchronize()
    return f0, g0, f1, g1, rec


def assert_same(x, y, keys):
    for k in keys:
        assert torch.equal(x[k], y[k]), k


@pytest.mark.parametrize("kpw,pin", [(0, True), (4, True), (16, True), (16, False)])
def test_kept_factors_give_the_same_bits(ctx, kpw, pin):
    # ragged horizons: one knot, under one part, exactly one part, parts plus a ragged
    # tail, several parts (seeds 8101 + b); automatic and fixed workgroup shapes, gangs on
    # one XCD each and on the global queue
    Ns = [1, 5, 16, 17, 40, 96, 200, 13]
    packed, off = synth.pack(synth.batch(Ns, seed0=8101))
    d = dev(packed)
    ctx.mpcpcg_set_knots_per_group(kpw)
    ctx.mpcpcg_set_xcd_pinning(pin)
    try:
        assert ctx.mpcpcg_tuned_schedule(off)[1] == pin
        f0, g0, f1, g1, _ = plain_and_kept(ctx, d, off)
    finally:
        ctx.mpcpcg_set_knots_per_group(0)
        ctx.mpcpcg_set_xcd_pinning(True)
    assert_same(f0, f1, ("lam", "dx", "du", "stats"))
    assert_same(g0, g1, GRADS)


def test_kept_factors_of_a_warm_start(ctx):
    # the forward's start iterate does not enter Phi^-1: a warm-started forward keeps
    # the same record, and the adjoint read from it equals the plain adjoint
    Ns = [64, 33, 128]
    packed, off = synth.pack(synth.batch(Ns, seed0=8201))
    d = dev(packed)
    lam0 = ctx.mpcpcg_solve_batched(d, off, eps=1e-2)["lam"].clone()
    f0, g0, f1, g1, _ = plain_and_kept(ctx, d, off, warm=lam0)
    assert_same(f0, f1, ("lam", "dx", "du", "stats"))
    assert_same(g0, g1, GRADS)


def test_record_survives_other_solves_and_matches_the_oracle(ctx):
    # the record is the caller's: solves of another batch on the same context between the
    # two calls leave it intact.  The adjoint read from it also meets the oracle's adjoint
    # fed the oracle's forward (no GPU output in the reference), at the gradient bar.
    Ns = [48, 17, 96, 1]
    packed, off = synth.pack(synth.batch(Ns, seed0=8301))
    d = dev(packed)
    rec = ctx.factor_record(int(off[-1]), d["q"].device)
    f = clone(ctx.mpcpcg_solve_batched(d, off, eps=EPS, factors=rec))
    other, ooff = synth.pack(synth.batch([80, 200, 7], seed0=8351))
    od = dev(other)
    of = ctx.mpcpcg_solve_batched(od, ooff, eps=EPS)
    ctx.mpcpcg_backward(od, ooff, of, 2 * of["lam"], eps=EPS)
    gl = 2 * f["lam"]
    g = clone(ctx.mpcpcg_backward(d, off, f, gl, eps=EPS, factors=rec))
    g_plain = clone(ctx.mpcpcg_backward(d, off, f, gl, eps=EPS))
    torch.cuda.synchronize()
    assert_same(g, g_plain, GRADS)
    fo = orc.solve_batch(packed, off, eps=EPS, threads=8)
    ref = orc.backward_batch(packed, off, fo, 2 * fo["lam"], None, None, eps=EPS, threads=8)
    for k in ("dQ", "dA", "dB", "dR", "dq", "dr"):
        assert rel(g[k].cpu().numpy(), ref[k]) < 1e-4, k


def test_record_argument_errors(ctx):
    from paper_2309_08079_amd.mpcpcg import Context, MPCPCGError
    packed, off = synth.pack(synth.batch([20, 9], seed0=8401))
    d = dev(packed)
    rec = ctx.factor_record(int(off[-1]) + 1, d["q"].device)
    with pytest.raises(MPCPCGError, match="aligned"):
        ctx.mpcpcg_solve_batched(d, off, eps=EPS, factors=rec[1:])
    assert ctx.mpcpcg_factor_bytes(1) > 0
    with pytest.raises(MPCPCGError):
        ctx.mpcpcg_factor_bytes(0)
    wide = Context(28, 14, max_total_knots=256, max_batch=4)
    try:
        with pytest.raises(MPCPCGError):
            wide.mpcpcg_factor_bytes(64)
    finally:
        wide.close()


def test_autograd_function_reads_the_record(ctx):
    # MPCPCGFunction keeps the record on a (14, 7) PCG context: its gradients equal those of
    # the plain calls bit for bit
    from paper_2309_08079_amd.mpcpcg import MPCPCGFunction
    Ns = [40, 17]
    packed, off = synth.pack(synth.batch(Ns, seed0=8501))
    d = dev(packed)
    leaves = {k: d[k].clone().requires_grad_(True) for k in ("Q", "R", "A", "B", "q", "r", "x0", "e")}
    lam, dx, du = MPCPCGFunction.apply(ctx, off, EPS, *(leaves[k] for k in ("Q", "R", "A", "B", "q", "r", "x0", "e")))
    ((lam * lam).sum() + dx.sum()).backward()
    f = ctx.mpcpcg_solve_batched(d, off, eps=EPS)
    g = ctx.mpcpcg_backward(d, off, f, 2 * f["lam"], torch.ones_like(f["dx"]), None, eps=EPS)
    torch.cuda.synchronize()
    for k, gk in (("Q", "dQ"), ("R", "dR"), ("A", "dA"), ("B", "dB"), ("q", "dq"), ("r", "dr"), ("x0", "dx0"),
                  ("e", "de")):
        assert torch.equal(leaves[k].grad, g[gk]), k

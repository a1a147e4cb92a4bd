"""The LDS-poisoning debug build (libmpcpcg_poison.so: every workgroup of the fused kernel
fills its LDS with a NaN pattern at the start of each task) against the regular build, bit
for bit, on single solves across horizons and workgroup shapes, a ragged batch, the adjoint
(also the one that reads the forward's factor record), a warm start and the Schur formation.
A read of LDS that a task has not written first would turn that task's outputs into NaN (or
change them), so equal finite bits show that no formation, PCG or epilogue step reads stale
LDS."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2309_08079_amd import synth

pytestmark = pytest.mark.gpu

EPS = 1e-6


@pytest.fixture(scope="module")
def ctxs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08079_amd.mpcpcg import POISON_LIB_PATH, Context
    a = Context(14, 7, max_total_knots=1 << 14, max_batch=64)
    b = Context(14, 7, max_total_knots=1 << 14, max_batch=64, lib_path=POISON_LIB_PATH)
    yield a, b
    a.close()
    b.close()


def dev(p):
    from paper_2309_08079_amd.mpcpcg import to_device
    return to_device(p)


def same(x, y, keys):
    for k in keys:
        assert torch.equal(x[k], y[k]), k
        if x[k].dtype.is_floating_point:
            assert torch.isfinite(x[k]).all(), k


@pytest.mark.parametrize("N", [1, 2, 17, 40, 64, 300])
@pytest.mark.parametrize("kpw", [0, 4, 16, 48])
def test_single_solves_equal_regular_build(ctxs, N, kpw):
    a, b = ctxs
    p = dev(synth.problem(N, seed=8800 + N))
    outs = []
    for c in (a, b):
        c.mpcpcg_set_knots_per_group(kpw)
        try:
            o = c.mpcpcg_solve(p, eps=EPS)
            torch.cuda.synchronize()
        finally:
            c.mpcpcg_set_knots_per_group(0)
        outs.append({k: v.clone() for k, v in o.items()})
    same(outs[0], outs[1], ("lam", "dx", "du", "stats"))


def test_batch_adjoint_and_warm_start_equal_regular_build(ctxs):
    a, b = ctxs
    Ns = [1, 5, 33, 64, 100, 2, 17, 129, 16, 48]
    packed, off = synth.pack(synth.batch(Ns, seed0=8900))
    d = dev(packed)
    fw, bw, wm = [], [], []
    for c in (a, b):
        f = c.mpcpcg_solve_batched(d, off, eps=EPS)
        g = c.mpcpcg_backward(d, off, f, 2 * f["lam"], eps=EPS)
        w = c.mpcpcg_solve_batched(d, off, eps=EPS, lam0=f["lam"] + 0.01)
        torch.cuda.synchronize()
        fw.append({k: v.clone() for k, v in f.items()})
        bw.append({k: v.clone() for k, v in g.items()})
        wm.append({k: v.clone() for k, v in w.items()})
    same(fw[0], fw[1], ("lam", "dx", "du", "stats"))
    same(bw[0], bw[1], ("dQ", "dR", "dA", "dB", "dq", "dr", "dx0", "stats"))
    same(wm[0], wm[1], ("lam", "dx", "du", "stats"))


@pytest.mark.parametrize("kpw", [0, 4])
def test_kept_record_adjoint_equals_regular_build(ctxs, kpw):
    # the adjoint that reads the forward's factor record instead of forming Phi^-1 skips the
    # D^-1 exchange through LDS: it must still read no LDS it has not written
    a, b = ctxs
    Ns = [1, 5, 33, 64, 100, 2, 17, 129, 16, 48]
    packed, off = synth.pack(synth.batch(Ns, seed0=8950))
    d = dev(packed)
    fw, bw = [], []
    for c in (a, b):
        c.mpcpcg_set_knots_per_group(kpw)
        try:
            rec = c.factor_record(int(off[-1]), d["q"].device)
            f = c.mpcpcg_solve_batched(d, off, eps=EPS, factors=rec)
            g = c.mpcpcg_backward(d, off, f, 2 * f["lam"], eps=EPS, factors=rec)
            torch.cuda.synchronize()
        finally:
            c.mpcpcg_set_knots_per_group(0)
        fw.append({k: v.clone() for k, v in f.items()})
        bw.append({k: v.clone() for k, v in g.items()})
    same(fw[0], fw[1], ("lam", "dx", "du", "stats"))
    same(bw[0], bw[1], ("dQ", "dR", "dA", "dB", "dq", "dr", "dx0", "stats"))


@pytest.mark.parametrize("N", [1, 33, 70])
def test_form_schur_equals_regular_build(ctxs, N):
    a, b = ctxs
    p = dev(synth.problem(N, seed=9900 + N))
    ra = [t.clone() for t in a.mpcpcg_form_schur(p)]
    rb = [t.clone() for t in b.mpcpcg_form_schur(p)]
    torch.cuda.synchronize()
    for x, y in zip(ra, rb):
        assert torch.equal(x, y) and torch.isfinite(x).all()

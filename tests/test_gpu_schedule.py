"""GPU tests of the batched schedule and the failure paths: the autotuner, bounded
per-signature caches, the TIMEOUT status of a gang whose wait gives up (forced from the
host with a test hook, every kernel exits normally), and the autograd Function's refusal
to pass unconverged solves on.  Results are compared with the CPU oracle (Algorithm 1,
per problem) at the parity bar of the other tests: 1e-5 norm-wise for lambda and dZ,
iterations within 1."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kkt
from oracle import ref as orc
from paper_2309_08079_amd import synth

pytestmark = pytest.mark.gpu

EPS = 1e-6


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def dev(p):
    from paper_2309_08079_amd.mpcpcg import to_device
    return to_device(p)


def stats(t):
    from paper_2309_08079_amd.mpcpcg import stats_to_numpy
    return stats_to_numpy(t)


@pytest.fixture()
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08079_amd.mpcpcg import Context
    c = Context(14, 7, max_total_knots=1 << 15, max_batch=256)
    yield c
    c.close()


def check_against_oracle(out, packed, off, only=None):
    ref = orc.solve_batch(packed, off, eps=EPS, threads=8)
    lam, dx, du = (out[k].cpu().numpy() for k in ("lam", "dx", "du"))
    st = stats(out["stats"])
    for b in range(len(off) - 1) if only is None else only:
        k0, k1 = off[b], off[b + 1]
        c0, c1 = k0 - b, k1 - b - 1
        assert st[b]["status"] == orc.OK, (b, int(st[b]["status"]))
        assert abs(int(st[b]["iters"]) - int(ref["iters"][b])) <= 1, b
        assert rel(lam[k0:k1], ref["lam"][k0:k1]) < 1e-5, b
        assert rel(dx[k0:k1], ref["dx"][k0:k1]) < 1e-5, b
        if c1 > c0:
            assert rel(du[c0:c1], ref["du"][c0:c1]) < 1e-5, b


def check_against_exact(out, probs, off, only=None):
    """The factorisation path (no iterations) against the exact KKT solution at 1e-6, the
    bar of the factorisation tests."""
    lam, dx, du = (out[k].cpu().numpy() for k in ("lam", "dx", "du"))
    st = stats(out["stats"])
    for b in range(len(off) - 1) if only is None else only:
        k0, k1 = off[b], off[b + 1]
        c0, c1 = k0 - b, k1 - b - 1
        assert st[b]["status"] == orc.OK and st[b]["iters"] == 0, (b, int(st[b]["status"]), int(st[b]["iters"]))
        ex = kkt.kkt_solve(probs[b])
        assert rel(lam[k0:k1], ex["lam"]) < 1e-6, b
        assert rel(dx[k0:k1], ex["dx"]) < 1e-6, b
        if c1 > c0:
            assert rel(du[c0:c1], ex["du"]) < 1e-6, b


def test_autotune_picks_a_shape_caches_it_and_matches_fixed_shape(ctx):
    # 16 problems, horizons drawn from {32, ..., 512} (seed 3000), seeds 3001 + b
    Ns = synth.horizons_uniform_choice(16, seed=3000)
    probs = synth.batch(Ns, seed0=3001)
    packed, off = synth.pack(probs)
    d = dev(packed)
    k = ctx.mpcpcg_autotune(d, off, eps=EPS)
    assert k in (4, 8, 16, 24, 32, 48)
    kpw, pinned = ctx.mpcpcg_tuned_schedule(off)
    assert kpw == k
    tuned = ctx.mpcpcg_solve_batched(d, off, eps=EPS)
    torch.cuda.synchronize()
    tuned = {key: v.clone() for key, v in tuned.items()}
    check_against_oracle(tuned, packed, off)
    # the same shape and placement set by hand give the same bits
    ctx.mpcpcg_set_knots_per_group(k)
    ctx.mpcpcg_set_xcd_pinning(pinned)
    try:
        assert ctx.mpcpcg_tuned_schedule(off) == (k, pinned)
        fixed = ctx.mpcpcg_solve_batched(d, off, eps=EPS)
        torch.cuda.synchronize()
    finally:
        ctx.mpcpcg_set_knots_per_group(0)
        ctx.mpcpcg_set_xcd_pinning(True)
    for key in ("lam", "dx", "du", "stats"):
        assert torch.equal(tuned[key], fixed[key]), key
    # the tuned choice is kept per signature: another signature keeps the default (16
    # knots per workgroup, each gang on one XCD)
    other = [64, 64]
    assert ctx.mpcpcg_tuned_schedule(np.cumsum([0] + other)) == (16, True)


@pytest.mark.parametrize("Ns", [[96, 40, 96, 40, 96, 40, 96, 40, 200, 13], [512], [200, 13, 96]],
                         ids=["ten", "lone512", "three"])
def test_placements_agree_bit_for_bit(ctx, Ns):
    # gangs on one XCD (per-XCD lists) and on the global queue run the same arithmetic,
    # forward and adjoint; batches of fewer than eight problems leave some lists empty
    probs = synth.batch(Ns, seed0=7101)
    packed, off = synth.pack(probs)
    d = dev(packed)
    outs, grads = [], []
    try:
        for pin in (True, False):
            ctx.mpcpcg_set_xcd_pinning(pin)
            assert ctx.mpcpcg_tuned_schedule(off)[1] == pin
            o = ctx.mpcpcg_solve_batched(d, off, eps=EPS)
            g = ctx.mpcpcg_backward(d, off, o, 2 * o["lam"], eps=EPS)
            torch.cuda.synchronize()
            outs.append({k: v.clone() for k, v in o.items()})
            grads.append({k: v.clone() for k, v in g.items()})
    finally:
        ctx.mpcpcg_set_xcd_pinning(True)
    for k in ("lam", "dx", "du", "stats"):
        assert torch.equal(outs[0][k], outs[1][k]), k
    for k in ("dQ", "dq", "dR", "dA", "dB", "stats"):
        assert torch.equal(grads[0][k], grads[1][k]), k
    check_against_oracle(outs[0], packed, off)


def test_default_shape_of_long_horizons(ctx):
    # a batch whose longest horizon needs more than 32 parts of 16 knots takes 32 knots per
    # workgroup by default (one poll per barrier); forward and adjoint against the oracle's
    # forward -> adjoint (horizons 1024, 700, 1024, 33; seeds 7301 + b)
    Ns = [1024, 700, 1024, 33]
    probs = synth.batch(Ns, seed0=7301)
    packed, off = synth.pack(probs)
    d = dev(packed)
    assert ctx.mpcpcg_tuned_schedule(off) == (32, True)
    out = ctx.mpcpcg_solve_batched(d, off, eps=EPS)
    g = ctx.mpcpcg_backward(d, off, out, 2 * out["lam"], eps=EPS)
    torch.cuda.synchronize()
    check_against_oracle(out, packed, off)
    fo = orc.solve_batch(packed, off, eps=EPS, threads=8)
    ref = orc.backward_batch(packed, off, fo, 2 * fo["lam"], None, None, eps=EPS, threads=8)
    assert (stats(g["stats"])["status"] == 0).all()
    for k in ("dQ", "dA", "dB", "dR", "dq", "dr"):
        assert rel(g[k].cpu().numpy(), ref[k]) < 1e-4, k


def test_single_solve_of_more_parts_than_an_xcd_holds(ctx):
    # 24-knot workgroups (six waves) are resident one per compute unit, so a 43-part single
    # solve (N = 1024) does not fit one XCD's 32 compute units and must spread over the
    # device; it converges and matches the oracle (seed 2000 + N)
    N = 1024
    p = synth.problem(N, seed=2000 + N)
    ctx.mpcpcg_set_knots_per_group(24)
    try:
        out = ctx.mpcpcg_solve(dev(p), eps=EPS)
        torch.cuda.synchronize()
    finally:
        ctx.mpcpcg_set_knots_per_group(0)
    packed, off = synth.pack([p])
    check_against_oracle(out, packed, off)


@pytest.mark.parametrize("N", [40, 100, 512])
def test_single_solve_on_one_xcd_agrees_with_spread_gang(ctx, N):
    # a single solve whose gang runs on one XCD exchanges its loop barriers through that
    # XCD's L2; spread over the device it uses device-scope words: same arithmetic, same bits
    from paper_2309_08079_amd.mpcpcg import to_device
    p = synth.problem(N, seed=7300 + N)
    d = to_device(p)
    outs = []
    for pin in (True, False):
        ctx.mpcpcg_set_xcd_pinning(pin)
        o = ctx.mpcpcg_solve(d, eps=EPS)
        torch.cuda.synchronize()
        outs.append({k: v.clone() for k, v in o.items()})
    ctx.mpcpcg_set_xcd_pinning(True)
    for k in ("lam", "dx", "du", "stats"):
        assert torch.equal(outs[0][k], outs[1][k]), k
    ref = orc.solve(p, eps=EPS)
    st = stats(outs[0]["stats"])[0]
    assert st["status"] == orc.OK and abs(int(st["iters"]) - int(ref["iters"])) <= 1
    assert rel(outs[0]["lam"].cpu().numpy(), ref["lam"]) < 1e-5
    assert rel(outs[0]["dx"].cpu().numpy(), ref["dx"]) < 1e-5


def test_wide_gangs_on_one_xcd_agree_with_the_global_queue():
    # the 28-state gang PCG with per-XCD lists (barriers through each XCD's L2) and with the
    # global queue (device-scope barriers): same arithmetic, same bits; ragged horizons,
    # a single-knot problem and a batch with fewer problems than XCDs
    from paper_2309_08079_amd.mpcpcg import Context
    for Ns, seed0 in (([70, 3, 130, 1, 41, 96, 9, 64, 200, 17], 7700), ([90, 33], 7800)):
        probs = synth.batch(Ns, nx=28, nu=14, seed0=seed0)
        packed, off = synth.pack(probs)
        c = Context(28, 14, max_total_knots=int(off[-1]), max_batch=len(Ns))
        try:
            c.mpcpcg_set_method("pcg")
            d = dev(packed)
            outs = []
            for pin in (True, False):
                c.mpcpcg_set_xcd_pinning(pin)
                o = c.mpcpcg_solve_batched(d, off, eps=EPS)
                torch.cuda.synchronize()
                outs.append({k: v.clone() for k, v in o.items()})
            for k in ("lam", "dx", "du", "stats"):
                assert torch.equal(outs[0][k], outs[1][k]), (Ns, k)
            st = stats(outs[0]["stats"])
            ref = orc.solve_batch(packed, off, eps=EPS, threads=8)
            lam = outs[0]["lam"].cpu().numpy()
            for b in range(len(Ns)):
                k0, k1 = off[b], off[b + 1]
                assert st[b]["status"] == orc.OK, b
                assert abs(int(st[b]["iters"]) - int(ref["iters"][b])) <= max(2, int(0.1 * ref["iters"][b])), b
                assert rel(lam[k0:k1], ref["lam"][k0:k1]) < 1e-5, b
        finally:
            c.close()


def test_cache_is_bounded_over_many_signatures(ctx):
    # 100 distinct horizon signatures through a context limited to 6 per cache: the
    # entries and their device memory stay bounded and every solve still matches the oracle
    ctx.mpcpcg_set_cache_limit(6)
    rng = np.random.default_rng(12)
    peak_entries, peak_bytes = 0, 0
    for i in range(100):
        Ns = [int(n) for n in rng.integers(1, 40, size=1 + i % 3)]
        Ns[0] = 1 + i  # makes every signature distinct
        probs = synth.batch(Ns, seed0=20000 + 10 * i)
        packed, off = synth.pack(probs)
        out = ctx.mpcpcg_solve_batched(dev(packed), off, eps=EPS)
        torch.cuda.synchronize()
        if i % 9 == 0:
            check_against_oracle(out, packed, off)
        else:
            assert (stats(out["stats"])["status"] == orc.OK).all(), i
        n, b = ctx.mpcpcg_cache_info()
        peak_entries, peak_bytes = max(peak_entries, n), max(peak_bytes, b)
    # schedules (one per signature at the default shape) and nothing else are cached here
    assert peak_entries <= 6, peak_entries
    assert peak_bytes < 6 * 64 * 1024, peak_bytes
    # a signature evicted long ago is rebuilt and still correct
    probs = synth.batch([1, 5], seed0=20000)
    packed, off = synth.pack(probs)
    out = ctx.mpcpcg_solve_batched(dev(packed), off, eps=EPS)
    torch.cuda.synchronize()
    check_against_oracle(out, packed, off)


@pytest.mark.parametrize("method", ["pcg", "factor"])
def test_wait_that_gives_up_reports_timeout(ctx, method):
    # the test hook makes the first cross-workgroup wait of every multi-workgroup problem
    # wait for a flag that is never written, with a 200 us limit: those problems report
    # TIMEOUT, one-workgroup problems are unaffected, every launch ends, and the context
    # solves correctly afterwards
    from paper_2309_08079_amd import mpcpcg as M
    Ns = [512, 8, 100, 16]
    probs = synth.batch(Ns, seed0=7600)
    packed, off = synth.pack(probs)
    d = dev(packed)
    ctx.mpcpcg_set_method(method)
    ctx.mpcpcg_set_knots_per_group(16)
    try:
        ctx.mpcpcg_debug_set_wait(200, inject_stall=True)
        out = ctx.mpcpcg_solve_batched(d, off, eps=EPS)
        torch.cuda.synchronize()
        st = stats(out["stats"])
        assert list(st["status"]) == [M.TIMEOUT if n > 16 else M.OK for n in Ns], st
        if method == "pcg":
            check_against_oracle(out, packed, off, only=[1, 3])
        else:
            check_against_exact(out, probs, off, only=[1, 3])
        single = ctx.mpcpcg_solve(dev(probs[0]), eps=EPS)
        torch.cuda.synchronize()
        assert stats(single["stats"])[0]["status"] == M.TIMEOUT
        ctx.mpcpcg_debug_set_wait(2_000_000, inject_stall=False)
        out = ctx.mpcpcg_solve_batched(d, off, eps=EPS)
        torch.cuda.synchronize()
        if method == "pcg":
            check_against_oracle(out, packed, off)
        else:
            check_against_exact(out, probs, off)
    finally:
        ctx.mpcpcg_debug_set_wait(2_000_000, inject_stall=False)
        ctx.mpcpcg_set_knots_per_group(0)
        ctx.mpcpcg_set_method("pcg")


def test_autograd_function_raises_on_unconverged_solve(ctx):
    from paper_2309_08079_amd.mpcpcg import MPCPCGError, MPCPCGFunction
    p = synth.problem(24, seed=3)
    packed, off = synth.pack([p])
    d = dev(packed)
    leaves = [d[k].clone().requires_grad_(True) for k in ("Q", "R", "A", "B", "q", "r", "x0", "e")]
    with pytest.raises(MPCPCGError, match="NOT_CONVERGED"):
        MPCPCGFunction.apply(ctx, off, EPS, *leaves, 1)
    lam, dx, du = MPCPCGFunction.apply(ctx, off, EPS, *leaves)
    (lam * lam).sum().backward()
    assert all(torch.isfinite(t.grad).all() for t in leaves)

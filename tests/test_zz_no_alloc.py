"""The allocation-free entry point mpcpcg_solve_noalloc through the C ABI, against the
context-based mpcpcg_solve (same kernel, same launch shape: bit for bit) and against the
CPU oracle at the parity bar (1e-5 norm-wise for lambda and dZ, iterations within 1, at
eps = 1e-6), on two calls in a row, the second with a smaller horizon."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ref as orc
from paper_2309_08079_amd import synth

pytestmark = pytest.mark.gpu

EPS = 1e-6


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08079_amd import mpcpcg
    return mpcpcg.load_library()


def outputs(N):
    return (torch.full((N, 14), np.nan, device="cuda"), torch.full((N, 14), np.nan, device="cuda"),
            torch.full((max(N - 1, 0), 7), np.nan, device="cuda"),
            torch.full((1, 4), -7, dtype=torch.int32, device="cuda"))


def call(lib, d, N, lam, dx, du, st):
    from paper_2309_08079_amd import mpcpcg as M
    return lib.mpcpcg_solve_noalloc(C.byref(M._problem(d, 14, 7, N)), C.byref(M._opts(EPS, 0, False)),
                                    lam.data_ptr(), dx.data_ptr(), du.data_ptr() if du.numel() else None,
                                    st.data_ptr(), torch.cuda.current_stream().cuda_stream)


def test_noalloc_matches_solve_and_oracle_on_two_calls(lib):
    from paper_2309_08079_amd import mpcpcg as M
    ctx = M.Context(14, 7, max_total_knots=4096, max_batch=4)
    try:
        # N = 512 (a 32-part gang), then N = 100 (7 parts, on one XCD): the second call
        # reuses the scratch the first one left behind
        for N, seed in ((512, 6001), (100, 6002)):
            p = synth.problem(N, seed=seed)
            d = M.to_device(p)
            lam, dx, du, st = outputs(N)
            rc = call(lib, d, N, lam, dx, du, st)
            assert rc == M.OK, lib.mpcpcg_noalloc_last_error()
            ref = ctx.mpcpcg_solve(d, eps=EPS)
            torch.cuda.synchronize()
            for k, v in (("lam", lam), ("dx", dx), ("du", du), ("stats", st)):
                assert torch.equal(v, ref[k]), (N, k)
            o = orc.solve(p, eps=EPS)
            s = M.stats_to_numpy(st)[0]
            assert s["status"] == M.OK and abs(int(s["iters"]) - o["iters"]) <= 1, (N, int(s["iters"]), o["iters"])
            assert rel(lam.cpu().numpy(), o["lam"]) < 1e-5
            assert rel(dx.cpu().numpy(), o["dx"]) < 1e-5
            assert rel(du.cpu().numpy(), o["du"]) < 1e-5
    finally:
        ctx.close()


def test_noalloc_binding_one_workgroup_warm_start_and_limits(lib):
    from paper_2309_08079_amd import mpcpcg as M
    # one-workgroup horizon, warm-started from the oracle's own iterate
    p = synth.problem(31, seed=9)
    d = M.to_device(p)
    lam, dx, du, st = outputs(31)
    o = orc.solve(p, eps=EPS)
    lam.copy_(torch.from_numpy(o["lam"].astype(np.float32)))
    M.mpcpcg_solve_noalloc(d, lam, dx, du, st, eps=EPS, warm=True)
    torch.cuda.synchronize()
    s = M.stats_to_numpy(st)[0]
    ref = orc.solve(p, eps=EPS, lam0=o["lam"].astype(np.float32).astype(np.float64))
    assert s["status"] == M.OK and int(s["iters"]) == ref["iters"]
    assert rel(lam.cpu().numpy(), ref["lam"]) < 1e-5
    # N = 1: no controls
    p1 = synth.problem(1, seed=5)
    d1 = M.to_device(p1)
    lam1, dx1, du1, st1 = outputs(1)
    M.mpcpcg_solve_noalloc(d1, lam1, dx1, du1, st1, eps=EPS)
    torch.cuda.synchronize()
    o1 = orc.solve(p1, eps=EPS)
    assert M.stats_to_numpy(st1)[0]["status"] == M.OK
    assert rel(lam1.cpu().numpy(), o1["lam"]) < 1e-5 and rel(dx1.cpu().numpy(), o1["dx"]) < 1e-5
    # beyond the scratch's horizon limit, and (28, 14): rejected before any launch
    z = torch.zeros(1, device="cuda")
    prob = M.Problem()
    prob.nx, prob.nu, prob.N = 14, 7, 2049
    for k in ("Q", "R", "A", "B", "q", "r", "x0"):
        setattr(prob, k, z.data_ptr())
    rc = lib.mpcpcg_solve_noalloc(C.byref(prob), C.byref(M._opts(EPS, 0, False)), lam.data_ptr(), dx.data_ptr(),
                                  du.data_ptr(), st.data_ptr(), None)
    assert rc == M.EINVAL and b"2048" in lib.mpcpcg_noalloc_last_error()
    prob.nx, prob.nu, prob.N = 28, 14, 8
    rc = lib.mpcpcg_solve_noalloc(C.byref(prob), C.byref(M._opts(EPS, 0, False)), lam.data_ptr(), dx.data_ptr(),
                                  du.data_ptr(), st.data_ptr(), None)
    assert rc == M.EUNSUPPORTED
    torch.cuda.synchronize()

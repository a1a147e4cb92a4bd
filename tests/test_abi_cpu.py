"""CPU-side checks of the boundary: the built library exports every entry point that
include/mpcpcg.h declares, the binding fails loudly without it, and the seeded generator
packs batches in the layout the header documents.  Nothing here calls into the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2309_08079_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpcpcg.h")
LIB = os.path.join(ROOT, "paper_2309_08079_amd", "libmpcpcg.so")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mpcpcg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("mpcpcg_create", "mpcpcg_destroy", "mpcpcg_last_error", "mpcpcg_form_schur",
                 "mpcpcg_solve", "mpcpcg_solve_batched", "mpcpcg_backward"):
        assert name in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmpcpcg.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2309_08079_amd import mpcpcg
    saved = mpcpcg._lib
    mpcpcg._lib = None
    try:
        with pytest.raises(mpcpcg.MPCPCGError):
            mpcpcg.load_library(str(tmp_path / "missing.so"))
    finally:
        mpcpcg._lib = saved


def test_struct_layouts_match_header():
    from paper_2309_08079_amd import mpcpcg
    assert ctypes.sizeof(mpcpcg.Opts) == 16
    assert ctypes.sizeof(mpcpcg.Problem) == 16 + 8 * 8
    assert mpcpcg.STATS_DTYPE.itemsize == 16
    # mpcpcg_chain_model: three floats, padding, one pointer; mpcpcg_trajectory: three
    # int32, padding, six pointers
    assert ctypes.sizeof(mpcpcg.ChainModel) == 24 and mpcpcg.ChainModel.gravity.offset == 16
    assert ctypes.sizeof(mpcpcg.Trajectory) == 16 + 6 * 8
    m = re.search(r"#define MPCPCG_LS_STEPS (\d+)", open(HEADER).read())
    assert m and int(m.group(1)) == mpcpcg.LS_STEPS


def test_trajectory_generator_and_packing():
    t = synth.trajectory(6, seed=5)
    assert t["X"].shape == (6, 14) and t["U"].shape == (5, 7) and t["R"].shape == (5, 7, 7)
    assert all(v.dtype == np.float32 and v.flags.c_contiguous for v in t.values())
    assert np.allclose(t["xref"], t["xref"][0]) and np.all(t["xref"][:, 7:] == 0)
    g = np.random.default_rng(5)
    x_init = np.concatenate([g.uniform(-1.0, 1.0, 7), 0.5 * g.standard_normal(7)])
    assert np.array_equal(t["x_init"], x_init.astype(np.float32))
    m = synth.chain_model(7, seed=3)
    assert m["gravity"].shape == (7,) and m["h"] == float(np.float32(0.01))
    trajs = synth.trajectories([1, 4, 2], seed0=40)
    packed, off = synth.pack_trajectories(trajs)
    assert list(off) == [0, 1, 5, 7]
    assert packed["U"].shape == (4, 7) and packed["x_init"].shape == (3, 14)
    assert np.array_equal(packed["U"][off[1] - 1:off[2] - 2], trajs[1]["U"])
    with pytest.raises(ValueError):
        synth.trajectory(4, nx=14, nu=6)


def test_generator_recipe_and_packing():
    p = synth.problem(5, seed=3)
    assert p["Q"].shape == (5, 14, 14) and p["R"].shape == (4, 7, 7)
    assert p["A"].shape == (4, 14, 14) and p["B"].shape == (4, 14, 7)
    assert all(v.dtype == np.float32 for v in p.values())
    assert np.allclose(p["Q"], np.transpose(p["Q"], (0, 2, 1)))
    assert np.all(np.linalg.eigvalsh(p["Q"].astype(np.float64)) > 0)
    assert np.all(np.diagonal(p["R"], axis1=1, axis2=2) >= 0.1)
    assert np.allclose(np.diagonal(p["A"], axis1=1, axis2=2), 1.0, atol=0.05)
    assert not p["e"].any()
    # same seed, same draw; different seed, different draw
    assert all(np.array_equal(p[k], synth.problem(5, seed=3)[k]) for k in p)
    assert not np.array_equal(p["q"], synth.problem(5, seed=4)["q"])
    probs = synth.batch([3, 1, 4], seed0=10)
    packed, off = synth.pack(probs)
    assert off.tolist() == [0, 3, 4, 8]
    assert packed["Q"].shape[0] == 8 and packed["A"].shape[0] == 8 - 3
    for b, pb in enumerate(probs):
        assert np.array_equal(synth.unpack_knots(packed["q"], off)[b], pb["q"])
        assert np.array_equal(synth.unpack_controls(packed["B"], off)[b], pb["B"])
        assert np.array_equal(packed["x0"][b], pb["x0"])


def test_mixed_horizon_draw():
    Ns = synth.horizons_uniform_choice(256, seed=3000)
    assert len(Ns) == 256 and set(Ns) <= {32, 64, 128, 256, 512}
    assert 40_000 < sum(Ns) < 60_000


def test_receding_horizon_sequence_generator():
    from paper_2309_08079_amd import synth
    import numpy as np
    T, N = 6, 9
    steps = synth.sequence(T, N, seed=11)
    base = synth.problem(N + T - 1, seed=11)
    assert len(steps) == T
    for t, p in enumerate(steps):
        assert p["Q"].shape == (N, 14, 14) and p["A"].shape == (N - 1, 14, 14) and p["x0"].shape == (14,)
        # step t is the window t .. t+N-1 of one trajectory
        assert np.array_equal(p["Q"], base["Q"][t:t + N]) and np.array_equal(p["B"], base["B"][t:t + N - 1])
    assert np.array_equal(steps[0]["x0"], base["x0"])
    # x0 follows x_{t+1} = A_t x_t + 0.05 w_t with w from seed + 1 (independent of any solver)
    g = np.random.default_rng(12)
    x = base["x0"].astype(np.float64)
    for t in range(T - 1):
        x = base["A"][t].astype(np.float64) @ x + 0.05 * g.standard_normal(14)
        assert np.array_equal(steps[t + 1]["x0"], x.astype(np.float32))


C_CALLER = r"""
#include "mpcpcg.h"
#include <stdio.h>
int main(void) {
  mpcpcg_ctx *ctx = 0;
  /* argument errors are reported before any device call */
  int unsupported = mpcpcg_create(&ctx, 3, 1, 16, 1);
  int einval_method = mpcpcg_set_method(0, MPCPCG_METHOD_AUTO);
  int einval_ls = mpcpcg_line_search(0, 1, 0, 0, 0, 0, 0, 0, 0.0f, 0, 0, 0, 0, 0);
  /* exchange records beyond 2 GiB (32-bit offsets in the kernels) */
  int too_big = mpcpcg_create(&ctx, 14, 7, 4 * (195652LL - 1) + 4, 1);
  int too_big_wide = mpcpcg_create(&ctx, 28, 14, 4 * 1016801LL, 1);
  /* the factor record calls: no context */
  long long fac_bytes = (long long)mpcpcg_factor_bytes(0, 512);
  int keep = mpcpcg_solve_batched_keep(0, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0);
  int reuse = mpcpcg_backward_reuse(0, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0);
  printf("%lld %d %d\n", fac_bytes, keep, reuse);
  printf("%d %d %d %d %d %d %d %d %d %d %d\n", unsupported, einval_method, einval_ls, ctx == 0, too_big, too_big_wide,
         (int)sizeof(mpcpcg_problem), (int)sizeof(mpcpcg_opts), (int)sizeof(mpcpcg_stats),
         (int)sizeof(mpcpcg_chain_model), (int)sizeof(mpcpcg_trajectory));
  return 0;
}
"""


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmpcpcg.so not built")
def test_header_is_c_and_the_library_links(tmp_path):
    # a plain C99 caller compiles against include/mpcpcg.h, links libmpcpcg.so and sees the
    # same struct layouts as the binding; calls with bad arguments return before any device
    # work, so this runs without a GPU
    import subprocess
    from paper_2309_08079_amd import mpcpcg
    src = tmp_path / "caller.c"
    src.write_text(C_CALLER)
    exe = tmp_path / "caller"
    libdir = os.path.dirname(LIB)
    cmd = ["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
           "-D__HIP_PLATFORM_AMD__", str(src), "-L", libdir, "-lmpcpcg", "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, LD_LIBRARY_PATH=libdir + ":/opt/rocm/lib:" + os.environ.get("LD_LIBRARY_PATH", ""))
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, env=env).stdout.split()
    fac_bytes, keep, reuse = (int(v) for v in out[:3])
    assert fac_bytes == -1 and keep == mpcpcg.EINVAL and reuse == mpcpcg.EINVAL
    out = out[3:]
    unsupported, einval_method, einval_ls, ctx_null, too_big, too_big_wide = (int(v) for v in out[:6])
    assert unsupported == mpcpcg.EUNSUPPORTED and einval_method == mpcpcg.EINVAL and einval_ls == mpcpcg.EINVAL
    assert ctx_null == 1
    assert too_big == mpcpcg.EINVAL and too_big_wide == mpcpcg.EINVAL
    sizes = [int(v) for v in out[6:]]
    assert sizes == [ctypes.sizeof(mpcpcg.Problem), ctypes.sizeof(mpcpcg.Opts), mpcpcg.STATS_DTYPE.itemsize,
                     ctypes.sizeof(mpcpcg.ChainModel), ctypes.sizeof(mpcpcg.Trajectory)]


def test_dpp_asm_header_is_the_generators_output():
    # csrc/dpp_asm.h is written by csrc/gen_dpp_asm.py; regenerating must reproduce it
    import importlib.util
    gen = os.path.join(ROOT, "paper_2309_08079_amd", "csrc", "gen_dpp_asm.py")
    spec = importlib.util.spec_from_file_location("gen_dpp_asm", gen)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    committed = open(os.path.join(ROOT, "paper_2309_08079_amd", "csrc", "dpp_asm.h")).read()
    assert mod.render() == committed
    # every block's operand numbers stay inside its operand list
    for line in committed.splitlines():
        if "asm volatile" not in line:
            continue
        nops = line.count('"v"(') + line.count('"+&v"(')
        used = [int(x) for x in re.findall(r"%(\d+)", line)]
        assert max(used) < nops, line[:120]


FLOORS_HEADER = os.path.join(ROOT, "include", "mpcpcg_floors.h")
FLOORS_LIB = os.path.join(ROOT, "paper_2309_08079_amd", "libmpcpcg_floors.so")


@pytest.mark.skipif(not os.path.exists(FLOORS_LIB), reason="libmpcpcg_floors.so not built")
def test_floor_probe_library_exports_every_declared_symbol():
    syms = sorted(set(re.findall(r"\b(floors_[a-z_0-9]+)\s*\(", open(FLOORS_HEADER).read())))
    assert len(syms) == 4
    lib = ctypes.CDLL(FLOORS_LIB)
    assert not [s for s in syms if not hasattr(lib, s)]

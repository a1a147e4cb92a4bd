"""Benchmark: batched Schur-complement + PCG solves with adjoint, Kuka-shaped LQ problems.

One step = one pass of the whole hot path over one batch: 256 problems of N = 512 knots
(nx = 14, nu = 7), formation of S / gamma / Phi^-1, PCG to sqrt(eta/eta_ref) < 1e-6,
primal reconstruction (forward launch), then the adjoint PCG and block-sparse gradients
of L = ||lambda||^2 (backward launch).  Inputs are seeded synthetic problems resident in
HBM before timing starts.

Prints ONE JSON line.  Extra fields report the batched forward alone, one-launch-per-solve
latency at N = 512, 256 sequential single-solve launches, and the roofline of the
dominant kernel measured with HIP events on the launch stream.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

NX, NU = 14, 7
N_KNOTS = 512
BATCH = 256
EPS = 1e-6
SEED0 = 6001

# Algorithmic work: FP64/FP32 flops per unit (per knot and iteration, formation, primal step,
# gradients).
FLOP_PER_KNOT_ITER = 2492      # S p (1176) + Phi^-1 r (1176) + 2 dots (56) + 3 axpys (84)
FLOP_PER_KNOT_FORM = 39102     # Q^-1, R^-1, theta, theta^-1, two Phi^-1 blocks, gamma
FLOP_PER_KNOT_FORM_S = 16464   # the same without Q^-1, R^-1, theta^-1 and the Phi^-1 blocks
                               # (22,638), which the adjoint reads from the forward's record
FLOP_PER_KNOT_RECON = 1078     # dx (two 14x14 matvecs) + du (14x7 + 7x7 matvecs)
FLOP_PER_KNOT_GRAD = 1960      # dQ, dA (two outer products each), dB, dR
PEAK_VALU_TFLOPS = 78.6        # FP64 vector FMA issue rate of MI355X (= non-packed FP32)


def kernel_sources():
    """Every file the GPU library is built from (the HIP sources and the C header), relative
    to the repository root: the counters recorded for one set of sources stay valid only
    as long as none of them changes."""
    import glob

    root = os.path.dirname(os.path.abspath(__file__))
    srcs = sorted(p for p in glob.glob(os.path.join(root, "paper_2309_08079_amd", "csrc", "*"))
                  if os.path.isfile(p) and not p.endswith(".pyc"))
    return [os.path.relpath(p, root) for p in srcs] + ["include/mpcpcg.h"]


def sources_sha256(names):
    import hashlib

    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for src in names:
        h.update(open(os.path.join(root, src), "rb").read())
    return h.hexdigest()


def measured_traffic(mode, kpw):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes (calibrated on a plain copy), or None once the kernel sources differ
    from those the counters were taken on."""
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", "pcg_kernel_traffic_256xN512.json")
    try:
        rec = json.load(open(path))
        names = kernel_sources()
        if rec["kernel_sources"] != names or rec["kernel_sources_sha256"] != sources_sha256(names) \
                or rec["per_launch"][mode]["knots_per_group"] != kpw:
            return None
        pl = rec["per_launch"][mode]
        return pl["fetch_bytes"] + pl["write_bytes"]
    except (OSError, KeyError, ValueError):
        return None


MODE_OF_TEMPLATE = {"1": "forward", "2": "adjoint"}


def ingest_counters(prof_dir):
    """Turn four rocprofv3 --pmc passes (FETCH_SIZE and WRITE_SIZE of the --step-only run, the
    same two of the --copy-probe run) into the per-launch HBM bytes measured_traffic() reads.
    Host only: parses <prof_dir>/{fetch,write,cfetch,cwrite}/<name>_counter_collection.csv."""
    import csv

    root = os.path.dirname(os.path.abspath(__file__))

    def rows(name):
        with open(os.path.join(prof_dir, name, name + "_counter_collection.csv")) as f:
            return list(csv.DictReader(f))

    def copy_kib(name):
        vals = [float(r["Counter_Value"]) for r in rows(name) if "copyBuffer" in r["Kernel_Name"]]
        if not vals:
            raise SystemExit("no copy kernel in the %s pass" % name)
        return max(vals)

    copy_bytes = 256 << 20
    fetch_factor = copy_bytes / 1024.0 / copy_kib("cfetch")
    write_factor = copy_bytes / 1024.0 / copy_kib("cwrite")
    per_launch = {}
    for name, key, factor in (("fetch", "fetch", fetch_factor), ("write", "write", write_factor)):
        acc = {}
        for r in rows(name):
            # the forward (phase 0) and the adjoint that reads the forward's Phi^-1 (phase 3)
            m = re.match(r"void mpc::pcg_kernel<14, 7, (\d+), (\d), [03]>", r["Kernel_Name"])
            if not m or m.group(2) not in MODE_OF_TEMPLATE:
                continue
            acc.setdefault((MODE_OF_TEMPLATE[m.group(2)], m.group(1)), []).append(float(r["Counter_Value"]))
        shapes = {}
        for mode, kpw in acc:
            shapes.setdefault(mode, set()).add(kpw)
        for mode, ks in shapes.items():
            if len(ks) > 1:
                raise SystemExit("the %s pass holds %s launches of several workgroup shapes (%s): take the "
                                 "counter passes with a fixed --kpw" % (name, mode, sorted(ks)))
        for (mode, kpw), v in acc.items():
            d = per_launch.setdefault(mode, {"knots_per_group": int(kpw)})
            d[key + "_kib_raw"] = float(np.mean(v))
            d["dispatches"] = len(v)
            d[key + "_bytes"] = float(np.mean(v)) * 1024.0 * factor
    names = kernel_sources()
    rec = {"workload": "batched %d x N=%d, nx=%d, nu=%d, eps=%g, seeds %d+b (bench.py --step-only)"
                       % (BATCH, N_KNOTS, NX, NU, EPS, SEED0),
           "kernel_sources_sha256": sources_sha256(names), "kernel_sources": names,
           "calibration": {"copy_bytes": copy_bytes, "fetch_counter_kib": copy_kib("cfetch"),
                           "write_counter_kib": copy_kib("cwrite"), "fetch_factor": fetch_factor,
                           "write_factor": write_factor},
           "per_launch": per_launch}
    out = os.path.join(root, "profiles", "pcg_kernel_traffic_256xN512.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    for mode, d in sorted(per_launch.items()):
        print("| %s (%d knots/group) | %.0f | %.0f | %.3f GB | %.3f GB | %.3f GB |" % (
            mode, d["knots_per_group"], d["fetch_kib_raw"], d["write_kib_raw"], d["fetch_bytes"] / 1e9,
            d["write_bytes"] / 1e9, (d["fetch_bytes"] + d["write_bytes"]) / 1e9))
    print("wrote", out)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0, help="problems in the CPU sample (0 = auto)")
    ap.add_argument("--kpw", type=int, default=0,
                    help="knots per workgroup of the batched kernels (0 = autotune shape and XCD "
                         "placement before timing, the default)")
    ap.add_argument("--no-floors", action="store_true", help="skip the launch / barrier / LDS / L2 probes")
    ap.add_argument("--step-only", action="store_true",
                    help="time the batched step only (no single-launch comparison, no CPU baseline)")
    ap.add_argument("--ingest-counters", default="", metavar="DIR",
                    help="host only: turn the rocprofv3 FETCH_SIZE / WRITE_SIZE passes under DIR into "
                         "profiles/pcg_kernel_traffic_256xN512.json and exit")
    ap.add_argument("--only", choices=("factorisation_path", "control_step", "two_arm_batch"), default="",
                    help="run one of the extra measurements alone and print its JSON (for profiling)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="run one plain device-to-device copy of MIB MiB and exit (hardware-counter "
                         "calibration: bytes a copy of known size reads and writes)")
    return ap.parse_args()


def cpu_baseline(packed_np, off, n_sample):
    """The oracle (plain C FP64, OpenMP over problems) on a bounded sample of the same
    workload: forward solve + adjoint of the first n_sample problems."""
    from oracle import ref as orc
    from paper_2309_08079_amd import synth

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    sub_off = off[: n_sample + 1]
    K = int(sub_off[-1])
    sub = {}
    for k in ("Q", "q"):
        sub[k] = packed_np[k][:K]
    for k in ("R", "A", "B", "r", "e"):
        sub[k] = packed_np[k][: K - n_sample]
    sub["x0"] = packed_np["x0"][:n_sample]
    orc.build(force=False)
    t0 = time.perf_counter()
    c0 = time.process_time()
    f = orc.solve_batch(sub, sub_off, eps=EPS, threads=threads)
    orc.backward_batch(sub, sub_off, f, 2 * f["lam"], eps=EPS, threads=threads)
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    # single forward solves on one thread (the sweep's problems, seeds 2000 + N), median of 5
    single = {}
    for n in (32, 128, 512):
        p = synth.problem(n, NX, NU, seed=2000 + n)
        ts = []
        for _ in range(5):
            t1 = time.perf_counter()
            orc.solve(p, eps=EPS)
            ts.append(time.perf_counter() - t1)
        single[str(n)] = round(float(np.median(ts)) * 1e6, 1)
    return dict(value=n_sample / wall, unit="solves/s", cores=threads, kind="oracle",
                sample="first %d of the %d problems (N=%d), forward + adjoint, FP64 C with "
                       "OpenMP over problems; %.1f s wall, %.1f s CPU" % (n_sample, BATCH, N_KNOTS, wall, cpu),
                single_solve_us_1_thread=single, cpu_model=_cpu_model())


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _time_ms(fn, stream, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def single_sweep(ctx, dev, stream, reps=10):
    """One launch per solve over horizons (seeds 2000 + N): latency, iterations beside the
    oracle's iterations on the same problem, latency per iteration, and the formation alone
    (mpcpcg_form_schur)."""
    import torch
    from oracle import ref as orc
    from paper_2309_08079_amd import synth
    from paper_2309_08079_amd.mpcpcg import stats_to_numpy, to_device

    rows = []
    for N in (16, 32, 64, 128, 256, 512):
        pn = synth.problem(N, NX, NU, seed=2000 + N)
        p = to_device(pn, dev)
        o = dict(lam=torch.empty((N, NX), device=dev), dx=torch.empty((N, NX), device=dev),
                 du=torch.empty((N - 1, NU), device=dev), stats=torch.zeros((1, 4), dtype=torch.int32, device=dev))
        ms = _time_ms(lambda: ctx.mpcpcg_solve(p, eps=EPS, out=o), stream, reps)
        it = int(stats_to_numpy(o["stats"])["iters"][0])
        so = (torch.empty((N, 3, NX, NX), device=dev), torch.empty((N, 3, NX, NX), device=dev),
              torch.empty((N, NX), device=dev))
        fms = _time_ms(lambda: ctx.mpcpcg_form_schur(p, out=so), stream, reps)
        rows.append({"N": N, "us": round(ms * 1e3, 2), "iters": it, "oracle_iters": int(orc.solve(pn, eps=EPS)["iters"]),
                     "us_per_iter": round((ms - fms) * 1e3 / max(it, 1), 3),
                     "formation_us": round(fms * 1e3, 2), "pcg_us": round((ms - fms) * 1e3, 2)})
    return rows


def floors():
    """Measured floors of this device (libmpcpcg_floors.so): empty-launch latency, one
    barrier round of the solver's protocol (isolated, and with as many gangs at once as
    the batched launch keeps), and the LDS, L2 and last-level-cache read bandwidths."""
    import ctypes as C

    lib = C.CDLL(os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2309_08079_amd",
                              "libmpcpcg_floors.so"))
    lib.floors_read.argtypes = [C.c_int64, C.c_int, C.c_int, C.POINTER(C.c_double)]
    v = C.c_double()

    def call(fn, *a):
        rc = fn(*a, C.byref(v))
        if rc != 0:
            raise RuntimeError("floor probe %s failed (%d)" % (fn.__name__, rc))
        return v.value

    out = {"launch_us": round(call(lib.floors_launch, 2000), 3)}
    bar = []
    # (gangs, parts, sleep before the first poll, gangs on one XCD each, exchange through
    # that XCD's L2): device-scope words as the solver's spread gangs use them, and the
    # XCD-local words of its gangs on one XCD (single solves, per-XCD batched lists)
    for g, n, sl, pin, l2 in ((1, 2, 0, 0, 0), (1, 2, 1, 0, 0), (1, 32, 0, 0, 0), (1, 32, 1, 0, 0),
                              (8, 16, 1, 1, 0), (24, 32, 1, 0, 0), (48, 16, 1, 1, 0),
                              (8, 32, 0, 1, 1), (24, 32, 0, 1, 1), (48, 16, 0, 1, 1)):
        bar.append({"gangs": g, "parts": n, "sleep_before_poll": bool(sl), "one_xcd_per_gang": bool(pin),
                    "xcd_l2": bool(l2), "us_per_round": round(call(lib.floors_barrier, g, n, 400, sl, pin, l2), 3)})
    out["barrier"] = bar
    out["lds_read_tbps"] = round(call(lib.floors_lds_read, 2048, 20000) / 1e12, 2)
    out["l2_read_tbps"] = round(call(lib.floors_read, 2 << 20, 2048, 8) / 1e12, 2)
    out["llc_read_tbps"] = round(call(lib.floors_read, 64 << 20, 256, 2) / 1e12, 2)
    out["notes"] = ("launch: back-to-back empty kernels; barrier: one round = publish a tagged 16-byte "
                    "word, poll every partner's (the solver's PCG sync point), us per round averaged over "
                    "400 rounds and all gangs; lds: ds_read_b128 conflict free; l2: 2 MiB re-read by 2048 "
                    "workgroups; llc: 64 MiB re-read by 256 workgroups")
    return out


def mixed_batch(ctx, dev, stream, reps=5):
    """256 problems with horizons drawn from {32, 64, 128, 256, 512} (seed 3000, problem
    seeds 3001 + b): one batched launch against 256 one-launch-per-solve calls."""
    import torch
    from paper_2309_08079_amd import synth
    from paper_2309_08079_amd.mpcpcg import stats_to_numpy, to_device

    Ns = synth.horizons_uniform_choice(BATCH, seed=3000)
    packed_np, off = synth.pack(synth.batch(Ns, NX, NU, seed0=3001))
    d = to_device(packed_np, dev)
    K = int(off[-1])
    fo = dict(lam=torch.empty((K, NX), device=dev), dx=torch.empty((K, NX), device=dev),
              du=torch.empty((K - BATCH, NU), device=dev), stats=torch.zeros((BATCH, 4), dtype=torch.int32, device=dev))
    bms = _time_ms(lambda: ctx.mpcpcg_solve_batched(d, off, eps=EPS, out=fo), stream, reps)
    iters = stats_to_numpy(fo["stats"])["iters"]
    views = []
    for b in range(BATCH):
        k0, k1 = int(off[b]), int(off[b + 1])
        views.append({"Q": d["Q"][k0:k1], "q": d["q"][k0:k1], "R": d["R"][k0 - b:k1 - b - 1],
                      "A": d["A"][k0 - b:k1 - b - 1], "B": d["B"][k0 - b:k1 - b - 1],
                      "r": d["r"][k0 - b:k1 - b - 1], "x0": d["x0"][b], "e": d["e"][k0 - b:k1 - b - 1]})
    outs = [dict(lam=fo["lam"][int(off[b]):int(off[b + 1])], dx=fo["dx"][int(off[b]):int(off[b + 1])],
                 du=fo["du"][int(off[b]) - b:int(off[b + 1]) - b - 1], stats=fo["stats"][b:b + 1])
            for b in range(BATCH)]

    def seq():
        for b in range(BATCH):
            ctx.mpcpcg_solve(views[b], eps=EPS, out=outs[b])
    sms = _time_ms(seq, stream, 1)
    return {"horizons": "uniform choice of {32,64,128,256,512}, seed 3000", "knots": K,
            "iters_mean": float(iters.mean()), "batched_ms": round(bms, 3),
            "batched_solves_per_s": BATCH / (bms * 1e-3), "sequential_ms": round(sms, 3),
            "speedup": sms / bms}


def warm_sequences(ctx, dev, stream, T=100, N=128):
    """The paper's solve-time study: a receding-horizon sequence of T problems of N knots,
    absolute stopping rule eta' < eps for eps in {1e-4, 5e-5, 1e-5}, each step solved in
    one launch, warm-started from the previous lambda shifted by one knot or cold.  Reports
    iterations and the distribution of per-solve device time, and the same distribution for
    the direct factorisation of each step."""
    import torch
    from paper_2309_08079_amd import synth
    from paper_2309_08079_amd.mpcpcg import stats_to_numpy, to_device

    steps = [to_device(p, dev) for p in synth.sequence(T, N, NX, NU, seed=8000)]
    out = dict(lam=torch.zeros((N, NX), device=dev), dx=torch.empty((N, NX), device=dev),
               du=torch.empty((N - 1, NU), device=dev), stats=torch.zeros((T, 4), dtype=torch.int32, device=dev))
    lam0 = torch.zeros((N, NX), device=dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(T)]
    res = {"horizon": N, "steps": T, "stop": "absolute", "seed": 8000}
    for eps in (1e-4, 5e-5, 1e-5):
        row = {}
        for mode in ("cold", "warm"):
            out["lam"].zero_()
            for t in range(T):
                o = dict(out, stats=out["stats"][t:t + 1])
                warm = mode == "warm" and t > 0
                if warm:
                    # start from the previous multipliers shifted by one knot, staged in the
                    # in/out buffer before the timed region
                    lam0[:-1].copy_(out["lam"][1:])
                    lam0[-1].copy_(out["lam"][-1])
                    out["lam"].copy_(lam0)
                ev[t][0].record(stream)
                ctx.mpcpcg_solve(steps[t], eps=eps, out=o, stop="absolute",
                                 lam0=out["lam"] if warm else None)
                ev[t][1].record(stream)
            torch.cuda.synchronize()
            us = np.array([a.elapsed_time(b) * 1e3 for a, b in ev])
            st = stats_to_numpy(out["stats"])
            row[mode] = {"iters_mean": float(st["iters"].mean()), "iters_max": int(st["iters"].max()),
                         "all_ok": bool((st["status"] == 0).all()),
                         "us_p10": float(np.percentile(us, 10)), "us_p50": float(np.percentile(us, 50)),
                         "us_p90": float(np.percentile(us, 90)), "us_max": float(us.max())}
        res["eps_%g" % eps] = row
    # the same sequence through the factorisation (exact, so neither eps nor the start
    # matters): the alternative the automatic method choice weighs against warm PCG
    ctx.mpcpcg_set_method("factor")
    try:
        for t in range(T):
            o = dict(out, stats=out["stats"][t:t + 1])
            ev[t][0].record(stream)
            ctx.mpcpcg_solve(steps[t], eps=1e-5, out=o, stop="absolute")
            ev[t][1].record(stream)
        torch.cuda.synchronize()
    finally:
        ctx.mpcpcg_set_method("pcg")
    us = np.array([a.elapsed_time(b) * 1e3 for a, b in ev])
    st = stats_to_numpy(out["stats"])
    res["factorisation"] = {"all_ok": bool((st["status"] == 0).all()),
                            "us_p10": float(np.percentile(us, 10)), "us_p50": float(np.percentile(us, 50)),
                            "us_p90": float(np.percentile(us, 90)), "us_max": float(us.max())}
    return res


def two_arm_batch(dev, stream, reps=3):
    """The 28-state / 14-control workload: 32 problems, horizons uniform on [64, 256]
    (seed 5000, problem 0 forced to 256), Q diagonal on U[1e-2, 1e2], problem seeds
    5001 + b; batched forward and adjoint (L = ||lambda||^2) times."""
    import torch
    from paper_2309_08079_amd import synth
    from paper_2309_08079_amd.mpcpcg import Context, stats_to_numpy, to_device

    Ns = synth.horizons_uniform_int(32, 64, 256, seed=5000, first=256)
    packed_np, off = synth.pack(synth.batch(Ns, 28, 14, seed0=5001, q_lo=1e-2, q_hi=1e2))
    d = to_device(packed_np, dev)
    K = int(off[-1])
    ctx = Context(28, 14, max_total_knots=K, max_batch=32)
    try:
        fo = ctx.mpcpcg_solve_batched(d, off, eps=EPS)
        fms = _time_ms(lambda: ctx.mpcpcg_solve_batched(d, off, eps=EPS, out=fo), stream, reps)
        gl = 2 * fo["lam"]
        bo = ctx.mpcpcg_backward(d, off, fo, gl, eps=EPS)
        bms = _time_ms(lambda: ctx.mpcpcg_backward(d, off, fo, gl, eps=EPS, out=bo), stream, reps)
        fst, bst = stats_to_numpy(fo["stats"]), stats_to_numpy(bo["stats"])
        ok = bool((fst["status"] == 0).all() and (bst["status"] == 0).all())
        ctx.mpcpcg_set_method("factor")
        ffms = _time_ms(lambda: ctx.mpcpcg_solve_batched(d, off, eps=EPS, out=fo), stream, reps)
        fbms = _time_ms(lambda: ctx.mpcpcg_backward(d, off, fo, gl, eps=EPS, out=bo), stream, reps)
        ok = ok and bool((stats_to_numpy(fo["stats"])["status"] == 0).all())
        return {"problems": 32, "knots": K, "nx": 28, "nu": 14, "pcg_forward_ms": round(fms, 3),
                "pcg_adjoint_ms": round(bms, 3), "pcg_solves_per_s_fwd_adj": 32 / ((fms + bms) * 1e-3),
                "iters_forward_mean": float(fst["iters"].mean()), "iters_adjoint_mean": float(bst["iters"].mean()),
                "factor_forward_ms": round(ffms, 3), "factor_adjoint_ms": round(fbms, 3),
                "factor_solves_per_s_fwd_adj": 32 / ((ffms + fbms) * 1e-3), "all_ok": ok}
    finally:
        ctx.close()


def factor_path(dev, stream, reps=3):
    """The factorisation path (block LDL^T of S, MPCPCG_METHOD_FACTOR) on the headline batch
    and on one N = 512 problem: batched forward and adjoint, single-solve latency."""
    import torch
    from paper_2309_08079_amd import synth
    from paper_2309_08079_amd.mpcpcg import Context, stats_to_numpy, to_device

    probs = synth.batch([N_KNOTS] * BATCH, NX, NU, seed0=SEED0)
    packed_np, off = synth.pack(probs)
    d = to_device(packed_np, dev)
    K = int(off[-1])
    ctx = Context(NX, NU, max_total_knots=K, max_batch=BATCH)
    try:
        ctx.mpcpcg_set_method("factor")
        fo = ctx.mpcpcg_solve_batched(d, off, eps=EPS)
        fms = _time_ms(lambda: ctx.mpcpcg_solve_batched(d, off, eps=EPS, out=fo), stream, reps)
        gl = 2 * fo["lam"]
        bo = ctx.mpcpcg_backward(d, off, fo, gl, eps=EPS)
        bms = _time_ms(lambda: ctx.mpcpcg_backward(d, off, fo, gl, eps=EPS, out=bo), stream, reps)
        ok = bool((stats_to_numpy(fo["stats"])["status"] == 0).all() and (stats_to_numpy(bo["stats"])["status"] == 0).all())
        single = {k: v[:N_KNOTS] for k, v in d.items() if k in ("Q", "q")}
        for k in ("R", "A", "B", "r", "e"):
            single[k] = d[k][:N_KNOTS - 1]
        single["x0"] = d["x0"][0]
        so = ctx.mpcpcg_solve(single, eps=EPS)
        sms = _time_ms(lambda: ctx.mpcpcg_solve(single, eps=EPS, out=so), stream, 10)
        return {"batch": BATCH, "knots": N_KNOTS, "forward_ms": round(fms, 3), "adjoint_ms": round(bms, 3),
                "solves_per_s_fwd_adj": BATCH / ((fms + bms) * 1e-3), "single_solve_us_N512": round(sms * 1e3, 2),
                "all_ok": ok}
    finally:
        ctx.close()


def control_step(dev, stream, reps=20):
    """The control step around the solve on the pendulum-chain stand-in model (model seed
    10000, trajectory seeds 13000 + N): per horizon, the linearisation and line-search
    kernels alone and one whole step (linearise, factorisation solve, line search) as three
    calls vs one graph launch; then one step of a 256-problem batch at N = 128.  The line
    search's algorithmic bytes per knot: X, dX, xref, lambda (4 nx floats), Q (nx^2), U, dU
    (2 nu), R (nu^2) read; X, U written."""
    import torch
    from paper_2309_08079_amd import synth
    from paper_2309_08079_amd.mpcpcg import Context, stats_to_numpy, to_device

    m = synth.chain_model(NU, seed=10000)
    dm = dict(m, gravity=torch.from_numpy(m["gravity"]).to(dev))
    ls_bytes_knot = 4 * (4 * NX + NX * NX + 2 * NU + NU * NU) + 4 * (NX + NU)
    rows = []
    for N in (32, 64, 128, 256, 512):
        packed, off = synth.pack_trajectories([synth.trajectory(N, NX, NU, seed=13000 + N)])
        ctx = Context(NX, NU, max_total_knots=N, max_batch=1)
        try:
            ctx.mpcpcg_set_method("factor")
            d = to_device(packed, dev)
            X0, U0 = d["X"].clone(), d["U"].clone()
            lam = torch.zeros((N, NX), device=dev)
            lq = ctx.mpcpcg_linearize(dm, d, off)
            lin_ms = _time_ms(lambda: ctx.mpcpcg_linearize(dm, d, off, out=lq), stream, reps)
            sol = ctx.mpcpcg_solve_batched(lq, off)
            lso = dict(X=torch.empty_like(d["X"]), U=torch.empty_like(d["U"]))
            lso.update(ctx.mpcpcg_line_search(dm, d, off, sol["dx"], sol["du"], lam=sol["lam"], mu=1.0, out=lso))
            ls_ms = _time_ms(lambda: ctx.mpcpcg_line_search(dm, d, off, sol["dx"], sol["du"], lam=sol["lam"],
                                                            mu=1.0, out=lso), stream, reps)
            solve_ms = _time_ms(lambda: ctx.mpcpcg_solve_batched(lq, off, out=sol), stream, reps)
            times = {}
            for graph in (False, True):
                ctx.mpcpcg_set_graph(graph)
                d["X"].copy_(X0)
                d["U"].copy_(U0)
                out = ctx.mpcpcg_control_step(dm, d, off, lam, d["X"], d["U"], mu=1.0)
                times[graph] = _time_ms(lambda: ctx.mpcpcg_control_step(dm, d, off, lam, d["X"], d["U"], mu=1.0,
                                                                        out=out), stream, reps)
            ok = bool((stats_to_numpy(out["stats"])["status"] == 0).all())
            rows.append({"N": N, "linearize_us": round(lin_ms * 1e3, 2), "solve_us": round(solve_ms * 1e3, 2),
                         "line_search_us": round(ls_ms * 1e3, 2),
                         "line_search_gbps": round(ls_bytes_knot * N / (ls_ms * 1e-3) / 1e9, 1),
                         "step_us_three_calls": round(times[False] * 1e3, 2),
                         "step_us_one_graph": round(times[True] * 1e3, 2),
                         "control_rate_hz": round(1e3 / times[True], 1), "ok": ok})
        finally:
            ctx.close()
    # batch: 256 problems of N = 128, one control step, the library's method choice
    Bn, Nb = 256, 128
    packed, off = synth.pack_trajectories(synth.trajectories([Nb] * Bn, NX, NU, seed0=14000))
    K = int(off[-1])
    ctx = Context(NX, NU, max_total_knots=K, max_batch=Bn)
    try:
        ctx.mpcpcg_set_method("auto")
        d = to_device(packed, dev)
        lam = torch.zeros((K, NX), device=dev)
        out = ctx.mpcpcg_control_step(dm, d, off, lam, d["X"], d["U"], mu=1.0)
        bms = _time_ms(lambda: ctx.mpcpcg_control_step(dm, d, off, lam, d["X"], d["U"], mu=1.0, out=out),
                       stream, 5)
        lq = ctx.mpcpcg_linearize(dm, d, off)
        blin = _time_ms(lambda: ctx.mpcpcg_linearize(dm, d, off, out=lq), stream, reps)
        sol = ctx.mpcpcg_solve_batched(lq, off)
        lso = dict(X=torch.empty_like(d["X"]), U=torch.empty_like(d["U"]))
        lso.update(ctx.mpcpcg_line_search(dm, d, off, sol["dx"], sol["du"], lam=sol["lam"], mu=1.0, out=lso))
        bls = _time_ms(lambda: ctx.mpcpcg_line_search(dm, d, off, sol["dx"], sol["du"], lam=sol["lam"], mu=1.0,
                                                      out=lso), stream, reps)
        batch = {"problems": Bn, "knots": Nb, "step_ms_one_graph": round(bms, 3),
                 "problem_steps_per_s": round(Bn / (bms * 1e-3), 1), "linearize_us": round(blin * 1e3, 2),
                 "line_search_us": round(bls * 1e3, 2),
                 "line_search_gbps": round(ls_bytes_knot * K / (bls * 1e-3) / 1e9, 1),
                 "ok": bool((stats_to_numpy(out["stats"])["status"] == 0).all())}
    finally:
        ctx.close()
    return {"model": "pendulum chain, 7 joints (nx=14, nu=7), h=0.01; factorisation solve for single "
                     "problems, the library's automatic choice for the batch; line search over 9 steps, "
                     "mu = 1 + max|lambda|",
            "single": rows, "batch_256xN128": batch}


def parity_sample(packed_np, off, fout, bout, fst, bst, sample=(0, 85, 170, 255)):
    """The timed headline batch checked against the oracle on a few of its problems:
    lambda, dx, du against the oracle's PCG iterate (Algorithm 1 at the same eps) and the
    gradients against the oracle's forward then adjoint; norm-wise relative errors (the
    bars are 1e-5 and 1e-4) and iteration counts beside the oracle's."""
    from oracle import ref as orc

    lam, dx, du = (fout[k].cpu().numpy() for k in ("lam", "dx", "du"))
    g = {k: bout[k].cpu().numpy() for k in ("dQ", "dR", "dA", "dB", "dq", "dx0")}
    rel = lambda a, b: float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))
    worst = {"lam": 0.0, "dx": 0.0, "du": 0.0, "grad": 0.0}
    iters = []
    for b in sample:
        k0, k1 = int(off[b]), int(off[b + 1])
        c0, c1 = k0 - b, k1 - b - 1
        p = {k: packed_np[k][k0:k1] for k in ("Q", "q")}
        p.update({k: packed_np[k][c0:c1] for k in ("R", "A", "B", "r")})
        p["x0"] = packed_np["x0"][b]
        f = orc.solve(p, eps=EPS)
        gr = orc.backward(p, f, 2 * f["lam"], eps=EPS)
        worst["lam"] = max(worst["lam"], rel(lam[k0:k1], f["lam"]))
        worst["dx"] = max(worst["dx"], rel(dx[k0:k1], f["dx"]))
        worst["du"] = max(worst["du"], rel(du[c0:c1], f["du"]))
        ge = max(rel(g["dQ"][k0:k1], gr["dQ"]), rel(g["dq"][k0:k1], gr["dq"]), rel(g["dx0"][b], gr["dx0"]),
                 rel(g["dA"][c0:c1], gr["dA"]), rel(g["dB"][c0:c1], gr["dB"]), rel(g["dR"][c0:c1], gr["dR"]))
        worst["grad"] = max(worst["grad"], ge)
        iters.append({"problem": b, "forward": int(fst["iters"][b]), "forward_oracle": int(f["iters"]),
                      "adjoint": int(bst["iters"][b]), "adjoint_oracle": int(gr["iters"])})
    return {"problems": list(sample), "max_rel_err": worst, "iters": iters,
            "within_bar": bool(max(worst["lam"], worst["dx"], worst["du"]) < 1e-5 and worst["grad"] < 1e-4),
            "reference": "oracle forward (Algorithm 1, FP64) and oracle forward -> oracle adjoint"}


def one_round_batch(ctx, d, off, dev, stream, n=24, reps=10):
    """The first 24 problems of the headline batch alone: as many N = 512 problems as the
    device keeps resident at once, so the launch is one round and its time per PCG
    iteration is the per-iteration cost under full load."""
    import torch
    from paper_2309_08079_amd.mpcpcg import stats_to_numpy

    sub_off = off[: n + 1]
    K = int(sub_off[-1])
    sub = {k: d[k][:K] for k in ("Q", "q")}
    sub.update({k: d[k][:K - n] for k in ("R", "A", "B", "r", "e")})
    sub["x0"] = d["x0"][:n]
    o = ctx.mpcpcg_solve_batched(sub, sub_off, eps=EPS)
    ms = _time_ms(lambda: ctx.mpcpcg_solve_batched(sub, sub_off, eps=EPS, out=o), stream, reps)
    it = stats_to_numpy(o["stats"])["iters"]
    return {"problems": n, "knots": N_KNOTS, "forward_ms": round(ms, 4), "iters_mean": float(it.mean()),
            "us_per_iter": round(ms * 1e3 / float(it.max()), 3)}


def barrier_entry(sweep, one_round, fl):
    """Microseconds per PCG iteration beside the measured barrier floor (one barrier per
    iteration in the solver's loop)."""
    row = {r["N"]: r for r in sweep}
    out = {"pcg_us_per_iter_one_workgroup_N16": row[16]["us_per_iter"],
           "pcg_us_per_iter_single_N512": row[512]["us_per_iter"],
           "pcg_us_per_iter_full_load_24xN512": one_round["us_per_iter"],
           "barriers_per_iter": 1}
    if fl:
        # the solver's gangs run on one XCD with the XCD-local exchange (single solves and
        # the per-XCD batched lists), so those are the floors its iterations compare with
        b = {(x["gangs"], x["parts"], x["sleep_before_poll"], x["one_xcd_per_gang"], x["xcd_l2"]): x["us_per_round"]
             for x in fl["barrier"]}
        iso, loaded = b[(8, 32, False, True, True)], b[(24, 32, False, True, True)]
        out["floor_us_isolated_32_parts"] = iso
        out["floor_us_loaded_24x32_parts"] = loaded
        out["floor_us_device_scope_isolated_32_parts"] = b[(1, 32, True, False, False)]
        out["single_N512_iter_over_floor"] = round(row[512]["us_per_iter"] / iso, 2)
        out["full_load_iter_over_floor"] = round(one_round["us_per_iter"] / loaded, 2)
    return out


PHI_ROW_BYTES = 16 * 3 * NX * 4  # one knot group's LDS reads of its Phi^-1 rows (16 lanes x 42 floats)
PHI_KNOT_BYTES = NX * 3 * NX * 4  # the knot's 14 rows of Phi^-1 (algorithmic)


def lds_entry(fout, off, fwd_ms, kpw, fl):
    """Phi^-1 bytes the forward launch reads from LDS per second, beside the measured LDS
    read bandwidth.  Every loop pass (iterations + 1) applies Phi^-1 once per knot slot of a
    part (slots past the horizon included) and, in a part of a multi-part problem, once
    more in each of its edge waves for the ghost knots beyond its ends; algorithmic bytes
    count the problem's own knots only."""
    from paper_2309_08079_amd.mpcpcg import stats_to_numpy

    passes = stats_to_numpy(fout["stats"])["iters"].astype(np.float64) + 1.0
    Ns = np.diff(np.asarray(off, dtype=np.int64)).astype(np.float64)
    parts = np.ceil(Ns / kpw)
    waves = kpw // 4
    ghost_groups = np.where(parts > 1, 8.0 if waves >= 2 else 4.0, 0.0)
    issued = float(np.sum(parts * (kpw + ghost_groups) * passes)) * PHI_ROW_BYTES
    algorithmic = float(np.sum(Ns * passes)) * PHI_KNOT_BYTES
    t = fwd_ms * 1e-3
    out = {"phi_issued_tbps": round(issued / t / 1e12, 3), "phi_algorithmic_tbps": round(algorithmic / t / 1e12, 3),
           "issued_bytes_per_launch": issued, "algorithmic_bytes_per_launch": algorithmic}
    if fl:
        out["lds_floor_tbps"] = fl["lds_read_tbps"]
        out["frac_issued"] = round(issued / t / 1e12 / fl["lds_read_tbps"], 4)
    return out


def gradient_batch(dev, stream, reps=5):
    """The differentiated workload: 64 problems of N = 128 (seeds 4001 + b), forward then the
    adjoint of L = ||lambda||^2, timed one launch each."""
    import torch
    from paper_2309_08079_amd import synth
    from paper_2309_08079_amd.mpcpcg import Context, stats_to_numpy, to_device

    packed_np, off = synth.pack(synth.batch([128] * 64, NX, NU, seed0=4001))
    d = to_device(packed_np, dev)
    ctx = Context(NX, NU, max_total_knots=int(off[-1]), max_batch=64)
    try:
        rec = ctx.factor_record(int(off[-1]), dev)
        fo = ctx.mpcpcg_solve_batched(d, off, eps=EPS, factors=rec)
        fms = _time_ms(lambda: ctx.mpcpcg_solve_batched(d, off, eps=EPS, out=fo, factors=rec), stream, reps)
        gl = 2 * fo["lam"]
        bo = ctx.mpcpcg_backward(d, off, fo, gl, eps=EPS, factors=rec)
        bms = _time_ms(lambda: ctx.mpcpcg_backward(d, off, fo, gl, eps=EPS, out=bo, factors=rec), stream, reps)
        ok = bool((stats_to_numpy(fo["stats"])["status"] == 0).all() and (stats_to_numpy(bo["stats"])["status"] == 0).all())
        return {"problems": 64, "knots": 128, "forward_ms": round(fms, 4), "adjoint_ms": round(bms, 4),
                "adjoint_reads_forward_preconditioner": True,
                "solves_per_s_fwd_adj": 64 / ((fms + bms) * 1e-3),
                "iters_forward_mean": float(stats_to_numpy(fo["stats"])["iters"].mean()),
                "iters_adjoint_mean": float(stats_to_numpy(bo["stats"])["iters"].mean()), "all_ok": ok}
    finally:
        ctx.close()


def main():
    args = parse()
    if args.ingest_counters:
        ingest_counters(args.ingest_counters)
        return
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (--gpus %d requested); batched problems are "
              "independent and would shard by problem across GPUs" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2309_08079_amd import synth
    from paper_2309_08079_amd.mpcpcg import Context, stats_to_numpy, to_device

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, device=dev)
        dst = torch.empty(n, device=dev)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 4 * n}))
        return
    if args.only:
        fn = {"factorisation_path": factor_path, "control_step": control_step, "two_arm_batch": two_arm_batch}[args.only]
        print(json.dumps({args.only: fn(dev, torch.cuda.current_stream())}))
        return
    probs = synth.batch([N_KNOTS] * BATCH, NX, NU, seed0=SEED0)
    packed_np, off = synth.pack(probs)
    d = to_device(packed_np, dev)
    K = int(off[-1])
    ctx = Context(NX, NU, max_total_knots=K, max_batch=BATCH)
    stream = torch.cuda.current_stream()

    # outputs preallocated so the graph replays with the same pointers
    fout = dict(lam=torch.empty((K, NX), device=dev), dx=torch.empty((K, NX), device=dev),
                du=torch.empty((K - BATCH, NU), device=dev),
                stats=torch.zeros((BATCH, 4), dtype=torch.int32, device=dev))
    gl = torch.empty((K, NX), device=dev)
    M = K - BATCH
    bout = dict(dQ=torch.empty((K, NX, NX), device=dev), dR=torch.empty((M, NU, NU), device=dev),
                dA=torch.empty((M, NX, NX), device=dev), dB=torch.empty((M, NX, NU), device=dev),
                dq=torch.empty((K, NX), device=dev), dr=torch.empty((M, NU), device=dev),
                dx0=torch.empty((BATCH, NX), device=dev), de=torch.empty((M, NX), device=dev),
                dgamma=torch.empty((K, NX), device=dev),
                stats=torch.zeros((BATCH, 4), dtype=torch.int32, device=dev))

    if args.kpw:
        ctx.mpcpcg_set_knots_per_group(args.kpw)
        kpw = args.kpw
        tuned = False
    else:
        kpw = ctx.mpcpcg_autotune(d, off, eps=EPS)
        tuned = True
    kpw, pinned = ctx.mpcpcg_tuned_schedule(off)
    # the forward keeps its preconditioner Phi^-1 for the adjoint (the same matrix S)
    rec = ctx.factor_record(K, dev)

    def step(evs=None):
        if evs is not None:
            evs[0].record(stream)
        ctx.mpcpcg_solve_batched(d, off, eps=EPS, out=fout, factors=rec)
        if evs is not None:
            evs[1].record(stream)
        torch.mul(fout["lam"], 2.0, out=gl)
        if evs is not None:
            evs[2].record(stream)
        ctx.mpcpcg_backward(d, off, fout, gl, eps=EPS, out=bout, factors=rec)
        if evs is not None:
            evs[3].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    adj_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))

    fst = stats_to_numpy(fout["stats"])
    bst = stats_to_numpy(bout["stats"])
    if (fst["status"] != 0).any() or (bst["status"] != 0).any():
        print("bench.py: a solve did not converge: forward %s adjoint %s" %
              (np.unique(fst["status"]), np.unique(bst["status"])), file=sys.stderr)
        sys.exit(1)
    it_f, it_b = fst["iters"].astype(np.int64), bst["iters"].astype(np.int64)
    flop_f = float(np.sum(N_KNOTS * (it_f * FLOP_PER_KNOT_ITER + FLOP_PER_KNOT_FORM + FLOP_PER_KNOT_RECON)))
    flop_b = float(np.sum(N_KNOTS * (it_b * FLOP_PER_KNOT_ITER + FLOP_PER_KNOT_FORM_S + FLOP_PER_KNOT_RECON
                                     + FLOP_PER_KNOT_GRAD)))
    dom_name, dom_ms, dom_flop = ("adjoint", adj_ms, flop_b) if adj_ms >= fwd_ms else ("forward", fwd_ms, flop_f)
    achieved = dom_flop / (dom_ms * 1e-3) / 1e12

    if args.step_only:
        print(json.dumps({"ms_per_step": ms_step, "knots_per_group": kpw, "xcd_pinned": pinned,
                          "kernel_ms": {"forward": fwd_ms, "adjoint": adj_ms},
                          "iters_forward_mean": float(it_f.mean()), "iters_adjoint_mean": float(it_b.mean())}))
        return
    parity = parity_sample(packed_np, off, fout, bout, fst, bst)
    sched = {"knots_per_group": kpw, "xcd_pinned": pinned, "autotuned": tuned}

    # one launch per solve: single problem latency and 256 sequential launches, with the
    # library's own workgroup shape per horizon (the schedule above is for the batched step)
    ctx.mpcpcg_set_knots_per_group(0)
    single = {"Q": d["Q"][:N_KNOTS], "q": d["q"][:N_KNOTS], "x0": d["x0"][0]}
    for k in ("R", "A", "B", "r", "e"):
        single[k] = d[k][: N_KNOTS - 1]
    sout = dict(lam=torch.empty((N_KNOTS, NX), device=dev), dx=torch.empty((N_KNOTS, NX), device=dev),
                du=torch.empty((N_KNOTS - 1, NU), device=dev),
                stats=torch.zeros((1, 4), dtype=torch.int32, device=dev))
    for _ in range(3):
        ctx.mpcpcg_solve(single, eps=EPS, out=sout)
    torch.cuda.synchronize()
    n_single = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(n_single):
        ctx.mpcpcg_solve(single, eps=EPS, out=sout)
    e1.record(stream)
    torch.cuda.synchronize()
    single_us = e0.elapsed_time(e1) * 1e3 / n_single
    views = []
    for b in range(BATCH):
        k0, k1 = int(off[b]), int(off[b + 1])
        views.append({"Q": d["Q"][k0:k1], "q": d["q"][k0:k1], "R": d["R"][k0 - b:k1 - b - 1],
                      "A": d["A"][k0 - b:k1 - b - 1], "B": d["B"][k0 - b:k1 - b - 1],
                      "r": d["r"][k0 - b:k1 - b - 1], "x0": d["x0"][b], "e": d["e"][k0 - b:k1 - b - 1]})
    e0.record(stream)
    for b in range(BATCH):
        ctx.mpcpcg_solve(views[b], eps=EPS, out=sout)
    e1.record(stream)
    torch.cuda.synchronize()
    seq_ms = e0.elapsed_time(e1)
    batched_fwd_sps = BATCH / (fwd_ms * 1e-3)
    # forward + adjoint one problem at a time: the single solve, then the adjoint of a
    # batch of one (256 problems in turn, and one N = 512 problem alone)
    one_off = np.array([0, N_KNOTS], dtype=np.int64)
    gout = {k: v[:N_KNOTS] if k in ("dQ", "dq", "dgamma") else v[:N_KNOTS - 1] for k, v in bout.items()
            if k not in ("dx0", "stats")}
    gout["dx0"], gout["stats"] = bout["dx0"][:1], bout["stats"][:1]
    gl1 = torch.empty((N_KNOTS, NX), device=dev)
    bviews = [dict(views[b], x0=views[b]["x0"].reshape(1, NX)) for b in range(BATCH)]

    def fwd_adj(b):
        ctx.mpcpcg_solve(views[b], eps=EPS, out=sout)
        torch.mul(sout["lam"], 2.0, out=gl1)
        ctx.mpcpcg_backward(bviews[b], one_off, sout, gl1, eps=EPS, out=gout)
    single_fa_us = _time_ms(lambda: fwd_adj(0), stream, n_single) * 1e3
    seq_fa_ms = _time_ms(lambda: [fwd_adj(b) for b in range(BATCH)], stream, 1)
    one_round = one_round_batch(ctx, d, off, dev, stream)

    sweep = single_sweep(ctx, dev, stream)
    mixed = mixed_batch(ctx, dev, stream)
    grad64 = gradient_batch(dev, stream)
    fl = None if args.no_floors else floors()
    seqs = warm_sequences(ctx, dev, stream)
    wide = two_arm_batch(dev, stream)
    fac = factor_path(dev, stream)
    ctrl = control_step(dev, stream)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(packed_np, off, args.cpu_sample or BATCH)

    line = {
        "metric": "µs/solve and PCG solves/s, Kuka nx=14 N=512; batched vs single; fwd+adjoint",
        "value": BATCH / (ms_step * 1e-3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "batched forward+adjoint PCG, 256 Kuka-shaped LQ problems (nx=14, "
                               "nu=7, N=512 knots), eps=1e-6, seeds 6001+b; the adjoint reads the "
                               "forward's preconditioner Phi^-1 and forms S again",
                   "batch": BATCH, "knots": N_KNOTS, "nx": NX, "nu": NU, "eps": EPS},
        "us_per_solve": ms_step * 1e3 / BATCH,
        "batched_forward_solves_per_s": batched_fwd_sps,
        "batched_forward_us_per_solve": fwd_ms * 1e3 / BATCH,
        "single_solve_us_N512": single_us,
        "sequential_256_single_launches_solves_per_s": BATCH / (seq_ms * 1e-3),
        "batched_vs_sequential_speedup": batched_fwd_sps / (BATCH / (seq_ms * 1e-3)),
        "single_solve_fwd_adj_us_N512": single_fa_us,
        "sequential_256_fwd_adj_ms": seq_fa_ms,
        "batched_vs_sequential_fwd_adj_speedup": seq_fa_ms / ms_step,
        "schedule": sched,
        "parity_sample": parity,
        "iters_forward_mean": float(it_f.mean()),
        "iters_adjoint_mean": float(it_b.mean()),
        "kernel_ms": {"forward": fwd_ms, "adjoint": adj_ms},
        "single_solve_sweep": sweep,
        "gradient_batch_64xN128": grad64,
        "floors": fl,
        "barrier": barrier_entry(sweep, one_round, fl),
        "lds": lds_entry(fout, off, fwd_ms, kpw, fl),
        "mixed_batch_256": mixed,
        "warm_sequence": seqs,
        "two_arm_batch_32": wide,
        "factorisation_path": fac,
        "control_step": ctrl,
        "roofline": {"bound": "alu", "kernel": "pcg_kernel<14,7,%d,%s>" % (kpw, dom_name if dom_name == "forward"
                                                                        else "adjoint, Phi^-1 read back"),
                     "achieved": achieved, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_VALU_TFLOPS, "traffic": measured_traffic(dom_name, kpw)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()

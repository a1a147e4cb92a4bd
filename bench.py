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
import sys
import time

import numpy as np

NX, NU = 14, 7
N_KNOTS = 512
BATCH = 256
EPS = 1e-6
SEED0 = 6001

# Algorithmic work ("Algorithmic work"): FP64/FP32 flops per unit.
FLOP_PER_KNOT_ITER = 2492      # S p (1176) + Phi^-1 r (1176) + 2 dots (56) + 3 axpys (84)
FLOP_PER_KNOT_FORM = 39102     # Q^-1, R^-1, theta, theta^-1, two Phi^-1 blocks, gamma
FLOP_PER_KNOT_RECON = 1078     # dx (two 14x14 matvecs) + du (14x7 + 7x7 matvecs)
FLOP_PER_KNOT_GRAD = 1960      # dQ, dA (two outer products each), dB, dR
PEAK_VALU_TFLOPS = 78.6        # FP64 vector FMA issue rate of MI355X (= non-packed FP32)


def measured_traffic(mode):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes (calibrated on a plain copy), or None once the kernel sources differ
    from those the counters were taken on."""
    import glob
    import hashlib

    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", "pcg_kernel_traffic_256xN512.json")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for src in rec["kernel_sources"]:
            h.update(open(os.path.join(root, src), "rb").read())
        srcs = sorted(glob.glob(os.path.join(root, "paper_2309_08079_amd", "csrc", "*")))
        if h.hexdigest() != rec["kernel_sources_sha256"] or len(srcs) + 1 != len(rec["kernel_sources"]):
            return None
        pl = rec["per_launch"][mode]
        return pl["fetch_bytes"] + pl["write_bytes"]
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0, help="problems in the CPU sample (0 = auto)")
    ap.add_argument("--step-only", action="store_true",
                    help="time the batched step only (no single-launch comparison, no CPU baseline)")
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
    return dict(value=n_sample / wall, unit="solves/s", cores=threads, kind="oracle",
                sample="first %d of the %d problems (N=%d), forward + adjoint, FP64 C with "
                       "OpenMP over problems; %.1f s wall, %.1f s CPU" % (n_sample, BATCH, N_KNOTS, wall, cpu))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (--gpus %d requested); batched problems "
              "are independent and would shard by problem across GPUs, see DESIGN.md" % args.gpus,
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

    def step(evs=None):
        if evs is not None:
            evs[0].record(stream)
        ctx.mpcpcg_solve_batched(d, off, eps=EPS, out=fout)
        if evs is not None:
            evs[1].record(stream)
        torch.mul(fout["lam"], 2.0, out=gl)
        if evs is not None:
            evs[2].record(stream)
        ctx.mpcpcg_backward(d, off, fout, gl, eps=EPS, out=bout)
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
    flop_b = float(np.sum(N_KNOTS * (it_b * FLOP_PER_KNOT_ITER + FLOP_PER_KNOT_FORM + FLOP_PER_KNOT_RECON
                                     + FLOP_PER_KNOT_GRAD)))
    dom_name, dom_ms, dom_flop = ("adjoint", adj_ms, flop_b) if adj_ms >= fwd_ms else ("forward", fwd_ms, flop_f)
    achieved = dom_flop / (dom_ms * 1e-3) / 1e12

    if args.step_only:
        print(json.dumps({"ms_per_step": ms_step, "kernel_ms": {"forward": fwd_ms, "adjoint": adj_ms},
                          "iters_forward_mean": float(it_f.mean()), "iters_adjoint_mean": float(it_b.mean())}))
        return

    # one launch per solve: single problem latency and 256 sequential launches
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

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(packed_np, off, args.cpu_sample or 32)

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
                               "nu=7, N=512 knots), eps=1e-6, seeds 6001+b",
                   "batch": BATCH, "knots": N_KNOTS, "nx": NX, "nu": NU, "eps": EPS},
        "us_per_solve": ms_step * 1e3 / BATCH,
        "batched_forward_solves_per_s": batched_fwd_sps,
        "batched_forward_us_per_solve": fwd_ms * 1e3 / BATCH,
        "single_solve_us_N512": single_us,
        "sequential_256_single_launches_solves_per_s": BATCH / (seq_ms * 1e-3),
        "batched_vs_sequential_speedup": batched_fwd_sps / (BATCH / (seq_ms * 1e-3)),
        "iters_forward_mean": float(it_f.mean()),
        "iters_adjoint_mean": float(it_b.mean()),
        "kernel_ms": {"forward": fwd_ms, "adjoint": adj_ms},
        "roofline": {"bound": "alu", "kernel": "pcg_kernel<14,7,16,%s>" % dom_name,
                     "achieved": achieved, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_VALU_TFLOPS, "traffic": measured_traffic(dom_name)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()

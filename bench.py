#!/usr/bin/env python3
"""Throughput of the coupled D3Q19 + D3Q7 thermal pseudopotential step on one
MI355X, printed as one JSON line.

A step is one full time step of the method (every stage of the update) over
the whole grid.  The default workload is the 512 x 512 x 384 closed box with
seeded liquid blobs and a vertical temperature gradient, FP32 deviation
storage; FP64 and FP16/BF16 storage are timed on the same workload as
variants, and the 256^3 droplet on a heated wall with an outlet in FP32 and
FP64 as a further workload.  Inputs are generated on the host, uploaded
once, and resident in HBM when the timed region starts.  The CPU baseline
is the FP64 oracle on the host cores, on bounded samples of the same
workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic HBM bytes per cell update: each D3Q19 and D3Q7 population read
# once and written once
ALG_BYTES = {"fp64": 416, "fp32": 208, "fp16": 104, "bf16": 104}
PEAK_HBM_GBS = 8000.0
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16": "f16-storage/f32", "bf16": "bf16-storage/f32"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="blobs_closed_512x512x384")
    ap.add_argument("--precision", default="fp32", choices=list(ALG_BYTES))
    ap.add_argument("--variants", default="fp64,fp16,bf16",
                    help="other storage precisions timed on the same workload ('' for none)")
    ap.add_argument("--variant-steps", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=50)
    ap.add_argument("--accuracy-steps", type=int, default=1000,
                    help="steps of the FP64-referenced accuracy check of the storage precisions (0: skip)")
    ap.add_argument("--adjoint-workload", default="heated_wall_adjoint_96",
                    help="workload of the adjoint timing ('' to skip)")
    ap.add_argument("--adjoint-precisions", default="fp64,fp32")
    ap.add_argument("--other-workloads", default="heated_wall_256,droplet_open_128,heated_wall_adjoint_96",
                    help="further workloads timed in FP32 and FP64 storage ('' for none)")
    ap.add_argument("--other-steps", type=int, default=50)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MiB",
                    help="only run a plain device copy of this size 3 times (HBM counter calibration)")
    return ap.parse_args()


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2206_00946_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, fn), "rb") as fh:
            h.update(fn.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


# sources that determine the single-pass step kernel (and the flags it is built with)
FUSED_SOURCES = ["paper_2206_00946_amd/csrc/kernels_fused.h", "paper_2206_00946_amd/csrc/kernels_ref.h",
                 "paper_2206_00946_amd/csrc/lattice.h", "paper_2206_00946_amd/csrc/storage.h",
                 "include/lbm3d.h", "paper_2206_00946_amd/build.py"]


def code_tokens(text: str) -> str:
    """C/C++ source with comments removed and whitespace runs folded, so that
    edits of comments alone leave the hash of the kernel sources as it was."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":                                  # string or character literal, kept whole
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):                  # C++ line comment
            while i < n and text[i] != "\n":
                i += 1
        elif text.startswith("/*", i):                  # C block comment
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def fused_kernel_hash():
    h = hashlib.sha256()
    for rel in FUSED_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as fh:
            text = fh.read()
        if not rel.endswith(".py"):
            text = code_tokens(text)
        h.update(rel.encode())
        h.update(text.encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, prec, launches_cells):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current sources of the step kernel (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{prec}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_hash") != fused_kernel_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def step_kernels(w):
    """Which kernels run a step of the workload: the single-pass kernel takes
    x/y-periodic set-ups (any z faces, vartheta = 0); outlets on x or y faces
    run the general kernels (three launches)."""
    if all(f == 0 for f in w["faces"][:4]) and not w.get("theta_corr"):
        return "single-pass"
    return "general (three kernels)"


def time_precision(P, torch, w, prec, steps, warmup):
    sim = P.from_workload(w, precision=prec)
    sim.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    stream = sim.stream
    start.record(stream)
    t0 = time.perf_counter()
    sim.step(steps)            # one launch sequence per step on sim.stream; syncs once at the end
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end) / steps
    diag = sim.reduce()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    cells = w["nx"] * w["ny"] * w["nz"]
    mlups = cells / (ms * 1e-3) / 1e6
    achieved = ALG_BYTES[prec] * cells / (ms * 1e-3) / 1e9
    return dict(ms_per_step=ms, mlups=mlups, wall_s=wall, achieved_gbs=achieved,
                frac=achieved / PEAK_HBM_GBS, mass=diag["mass"])


def accuracy_vs_fp64(P, torch, w, precs, steps):
    """Max relative error of rho and T (and normwise u) of each storage
    precision against FP64 storage after `steps` steps of the same workload
    (FP64 on the GPU equals the FP64 oracle to 1e-12, see the parity tests)."""
    def run(prec):
        sim = P.from_workload(w, precision=prec)
        sim.step(steps)
        out = sim.fields_device()
        sim.close()
        return out
    ref = run("fp64")
    res = {}
    for prec in precs:
        got = run(prec)
        er = float(((got[0] - ref[0]).abs() / ref[0].abs()).max())
        eT = float(((got[2] - ref[2]).abs() / ref[2].abs()).max())
        eu = float((got[1] - ref[1]).abs().max() / ref[1].abs().max())
        res[prec] = dict(rho_max_rel=er, T_max_rel=eT, u_normwise=eu)
        del got
        torch.cuda.empty_cache()
    del ref
    torch.cuda.empty_cache()
    return res


def time_adjoint(P, torch, w, prec):
    """Cost of the gradient of the evaporated mass over the workload's steps:
    N forward steps alone, then lbm_adjoint (forward pass with checkpoints,
    segment recomputation, reverse sweep)."""
    import math
    n = w["steps"]
    sim = P.from_workload(w, precision=prec)
    sim.step(2)
    stream = sim.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    sim.init(w["rho0"], w["T0"])
    torch.cuda.synchronize()
    ev[0].record(stream)
    sim.step(n)
    ev[1].record(stream)
    sim.init(w["rho0"], w["T0"])
    torch.cuda.synchronize()
    ev[2].record(stream)
    J, grad, dk = sim.adjoint(n, wall_face=4)
    ev[3].record(stream)
    torch.cuda.synchronize()
    fwd = ev[0].elapsed_time(ev[1]) * 1e-3
    tot = ev[2].elapsed_time(ev[3]) * 1e-3
    sim.close()
    del sim
    torch.cuda.empty_cache()
    k = math.ceil(math.sqrt(n))
    seg = -(-n // -(-n // k))
    recompute = (n - seg) / n
    return dict(forward_ms_per_step=round(fwd / n * 1e3, 4), gradient_s=round(tot, 3),
                gradient_over_forward=round(tot / fwd, 3),
                adjoint_step_over_forward_step=round(tot / fwd - 1.0 - recompute, 3),
                J=J, dJ_dkappa=dk)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_worker(job):
    """One oracle instance on its own sample, BLAS held to one thread; every
    worker starts its timed steps at the same barrier."""
    seed, steps, barrier = job
    from threadpoolctl import threadpool_limits
    from oracle import lbm_oracle as O
    from workloads import synth

    s = synth.blobs_closed(64, 64, 48, mean_blobs=4, rmin=5.0, rmax=9.0, seed=seed)
    p = O.Params(s["nx"], s["ny"], s["nz"], faces=tuple(s["faces"]), face_T=tuple(s["face_T"]),
                 face_rho=tuple(s["face_rho"]), kappa_w=s["kappa_w"])
    with threadpool_limits(limits=1):
        f, g = O.init_populations(s["rho0"], s["T0"], p)
        barrier.wait()
        t0 = time.perf_counter()
        for _ in range(steps):
            f, g, _ = O.step(f, g, p)
        dt = time.perf_counter() - t0
    return s["nx"] * s["ny"] * s["nz"] * steps, dt, s["n_blobs"]


def cpu_baseline(steps):
    """The FP64 oracle (unchanged numpy) on every host core of the GPU's CPU
    share: one single-threaded oracle process per core, each stepping its own
    64 x 64 x 48 closed box of the workload's recipe (walls at 0.85 and 0.95
    Tc, linear initial T, seeded non-overlapping blobs of radius 5-9), all
    timed together; the rate is the total cell updates over the slowest
    worker's time.  Run before the GPU is touched (the workers are forked)."""
    import multiprocessing as mp

    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    workers = max(1, min(16, avail))
    ctx = mp.get_context("fork")
    barrier = ctx.Manager().Barrier(workers)
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_worker, [(4 + k, steps, barrier) for k in range(workers)])
    total = sum(r[0] for r in res)
    dt = max(r[1] for r in res)
    return dict(value=round(total / dt / 1e6, 4), unit="MLUPS", cores=workers, kind="oracle",
                sample=f"{workers} single-threaded FP64 oracle processes, each a 64x64x48 closed box of the "
                       f"same recipe (seeds 4..{3 + workers}), {steps} steps, timed together: {dt:.1f} s",
                host={"nproc": os.cpu_count(), "cpus_available": avail, "cpu_model": _cpu_model()})


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU: --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    cpu = None
    if not args.no_cpu_baseline and not args.copy_probe:
        print("[bench] cpu baseline (oracle on the host cores)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.cpu_steps)
    import torch
    import paper_2206_00946_amd as P
    from workloads import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": n * 4, "copies": 3}), flush=True)
        return
    P.load_library()
    print(f"[bench] generating {args.workload}", file=sys.stderr, flush=True)
    w = synth.named(args.workload)
    cells = w["nx"] * w["ny"] * w["nz"]
    print(f"[bench] timing {args.precision}: {args.warmup} warmup + {args.steps} steps", file=sys.stderr, flush=True)
    head = time_precision(P, torch, w, args.precision, args.steps, args.warmup)
    variants = {}
    vsteps = args.variant_steps or max(10, args.steps // 5)
    for prec in [v for v in args.variants.split(",") if v and v != args.precision]:
        print(f"[bench] variant {prec}: {vsteps} steps", file=sys.stderr, flush=True)
        r = time_precision(P, torch, w, prec, vsteps, max(2, args.warmup // 2))
        variants[prec] = dict(mlups=round(r["mlups"], 1), ms_per_step=round(r["ms_per_step"], 4),
                              alg_bytes_per_cell=ALG_BYTES[prec], roofline_frac=round(r["frac"], 4))
        if prec == "fp64" and step_kernels(w) == "single-pass" and w["nx"] % 64 == 0:
            # the timed steps run in one lbm_step call: FP64 steps pass
            # x-deferred states to each other (the call starts from and
            # leaves the ordinary state)
            variants[prec]["streaming"] = "x-deferred between the steps of one call"
    accuracy = None
    if args.accuracy_steps:
        print(f"[bench] accuracy vs fp64 storage, {args.accuracy_steps} steps", file=sys.stderr, flush=True)
        accuracy = {"steps": args.accuracy_steps, "reference": "fp64 storage (= oracle to 1e-12)"}
        accuracy.update(accuracy_vs_fp64(P, torch, w, [p for p in ["fp32", "fp16", "bf16"]], args.accuracy_steps))
    others = {}
    for name in [v for v in args.other_workloads.split(",") if v and v != args.workload]:
        wo = synth.named(name)
        others[name] = {"grid": [wo["nx"], wo["ny"], wo["nz"]], "faces": wo["faces"], "kernels": step_kernels(wo)}
        for prec in ("fp32", "fp64"):
            print(f"[bench] {name} {prec}: {args.other_steps} steps", file=sys.stderr, flush=True)
            r = time_precision(P, torch, wo, prec, args.other_steps, 5)
            others[name][prec] = dict(mlups=round(r["mlups"], 1), ms_per_step=round(r["ms_per_step"], 4),
                                      alg_bytes_per_cell=ALG_BYTES[prec], roofline_frac=round(r["frac"], 4))
        del wo
    adjoint = None
    if args.adjoint_workload:
        wa = synth.named(args.adjoint_workload)
        adjoint = {"workload": args.adjoint_workload, "grid": [wa["nx"], wa["ny"], wa["nz"]], "steps": wa["steps"],
                   "objective": "evaporated mass M(0)-M(N)", "checkpoints": "ceil(sqrt(N))",
                   "forward_kernels": step_kernels(wa)}
        for prec in [v for v in args.adjoint_precisions.split(",") if v]:
            print(f"[bench] adjoint {prec} on {args.adjoint_workload}", file=sys.stderr, flush=True)
            adjoint[prec] = time_adjoint(P, torch, wa, prec)
    traffic = measured_traffic(args.workload, args.precision, cells)
    out = {
        "metric": "coupled D3Q19+D3Q7 MLUPS & % HBM roofline",
        "value": round(head["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": [w["nx"], w["ny"], w["nz"]], "cells": cells,
                   "storage": args.precision, "faces": w["faces"], "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(head["achieved_gbs"], 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(head["frac"], 4), "traffic": traffic,
                     "alg_bytes_per_cell": ALG_BYTES[args.precision],
                     # the committed counters' bytes moved per launch at this run's step time
                     "achieved_on_traffic": (round(traffic / (head["ms_per_step"] * 1e-3) / 1e9, 1)
                                             if traffic else None)},
        "variants": variants,
        "other_workloads": others,
        "accuracy": accuracy,
        "adjoint": adjoint,
        "source_hash": source_hash(),
        "kernel_hash": fused_kernel_hash(),
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

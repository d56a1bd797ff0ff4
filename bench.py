"""Throughput of the fused ternary LB step on one MI355X.

Headline: the 1024x1024 D2Q9 spinodal workload (C1, C2 = 1/3 + U(-0.01, 0.01),
kappa = (0.01, 0.015, 0.02), alpha = 1, tau = 1, M = 0.1) in FP64, MLUPS over
K timed steps with the state resident in HBM.  The same line carries the
roofline of the fused step kernel, the CPU oracle timed on a bounded sample,
and further measurements (FP32 of the same workload, D3Q19 256^3 FP32, a
device copy ceiling) under "extra".

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def _events_time(torch, stream, fn):
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    fn()
    stop.record(stream)
    stop.synchronize()
    torch.cuda.synchronize()
    return start.elapsed_time(stop)  # ms


def run_plain(tlb, torch, w, prec, steps, warmup, launch=None):
    """Time `steps` fused steps of workload w; returns a dict of measurements."""
    stream = torch.cuda.Stream()
    keys = ("lattice", "nx", "ny", "nz", "walls_y", "kappa", "alpha", "tau_f", "tau_g", "tau_k", "gamma_phi",
            "gamma_psi")
    sim = tlb.Sim(tlb.make_params(prec=prec, **{k: w[k] for k in keys}), stream=stream.cuda_stream)
    if launch:
        sim.set_launch(**launch)
    sim.init_equilibrium(w["C"]())
    sim.step(warmup)
    sim.synchronize()
    ms = _events_time(torch, stream, lambda: sim.step(steps))
    d = sim.diagnostics()
    N = w["nx"] * w["ny"] * w["nz"]
    per_launch_ms = ms / steps
    bytes_per_launch = sim.bytes_per_node() * N
    out = dict(
        ms_total=ms,
        ms_per_step=per_launch_ms,
        mlups=N * steps / (ms * 1e-3) / 1e6,
        achieved_GBps=bytes_per_launch / (per_launch_ms * 1e-3) / 1e9,
        bytes_per_node=sim.bytes_per_node(),
        bytes_per_launch=bytes_per_launch,
        nodes=N,
        launch=sim.launch(),
        mass=d["mass"],
        max_speed=d["max_speed"],
        nonfinite=d["nonfinite"],
    )
    sim.close()
    return out


def run_batched(tlb, torch, steps, warmup=10, graph_steps=50):
    """The 512-domain batched workload (FP32, walls, per-domain kappa and h): autotuned launch
    shape (outside the timed region), steps replayed from a captured hipGraph."""
    doms = inputs_mod().batched_walls()
    keys = ("lattice", "nx", "ny", "nz", "walls_y", "kappa", "alpha", "tau_f", "tau_g", "tau_k", "gamma_phi",
            "gamma_psi")
    stream = torch.cuda.Stream()
    b = tlb.Batch([tlb.make_params(prec=tlb.TLB_F32, **{k: d[k] for k in keys}) for d in doms],
                  stream=stream.cuda_stream)
    for i, d in enumerate(doms):
        b.set_wetting(i, 0, d["h"][0])
        b.set_wetting(i, 1, d["h"][1])
        b.init_equilibrium(i, d["C"])
    chosen = b.autotune(5)
    b.set_graph(graph_steps)
    b.step(warmup)
    b.synchronize()
    ms = _events_time(torch, stream, lambda: b.step(steps))
    nodes = b.nodes()
    bytes_per_step = 216.0 * nodes
    out = dict(mlups=nodes * steps / (ms * 1e-3) / 1e6, ms_per_step=ms / steps,
               achieved_GBps=bytes_per_step / (ms / steps * 1e-3) / 1e9, domains=len(doms), nodes=nodes,
               steps=steps, launch=chosen, graph_steps=graph_steps)
    out["frac_of_hbm"] = out["achieved_GBps"] / HBM_PEAK_GBS
    b.close()
    return out


def inputs_mod():
    from paper_1511_02155_amd import inputs

    return inputs


def copy_ceiling(tlb, torch, nbytes=1 << 30, reps=20):
    """Bandwidth of the library's plain copy kernel (read nbytes + write nbytes per launch)."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream

    def go(n):
        for _ in range(n):
            tlb.check(tlb.tlb_device_copy(b.data_ptr(), a.data_ptr(), nbytes, sp), "tlb_device_copy")

    go(2)
    ms = _events_time(torch, stream, lambda: go(reps))
    del a, b
    return 2.0 * nbytes * reps / (ms * 1e-3) / 1e9


def cpu_baseline(w, steps):
    """The FP64 CPU oracle on a bounded sample of the same workload."""
    import oracle

    oracle.build()
    keys = ("lattice", "nx", "ny", "nz", "walls_y", "kappa", "alpha", "tau_f", "tau_g", "tau_k", "gamma_phi",
            "gamma_psi")
    p = oracle.Params(**{k: w[k] for k in keys})
    pop = oracle.init_equilibrium(p, w["C"]())
    oracle.step(p, pop, 1)
    t0 = time.perf_counter()
    oracle.step(p, pop, steps)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=p.N * steps / dt / 1e6, unit="MLUPS", cores=threads, kind="oracle",
                sample=f"{w['name']} FP64, {steps} steps after 1 warm-up step, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--quick", action="store_true", help="headline only (no extra workloads)")
    ap.add_argument("--only", default=None, help="run a single workload: f64, f32, d3q19, batched")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: the fused step is single-device in this build "
              f"(requested --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    from paper_1511_02155_amd import inputs, tlb

    w2 = inputs.spinodal_2d(1024, args.steps)
    extra = {}
    if args.only in (None, "f64"):
        print(f"[bench] d2q9 1024^2 f64: {args.warmup} warm-up + {args.steps} timed steps", file=sys.stderr,
              flush=True)
        head = run_plain(tlb, torch, w2, tlb.TLB_F64, args.steps, args.warmup)
    if args.only == "f32":
        head = run_plain(tlb, torch, w2, tlb.TLB_F32, args.steps, args.warmup)
    if args.only == "d3q19":
        w3 = inputs.spinodal_3d(256, args.steps)
        head = run_plain(tlb, torch, w3, tlb.TLB_F32, args.steps, args.warmup)
    if args.only == "batched":
        r = run_batched(tlb, torch, args.steps)
        head = dict(mlups=r["mlups"], ms_per_step=r["ms_per_step"], achieved_GBps=r["achieved_GBps"],
                    bytes_per_launch=216.0 * r["nodes"], launch=r["launch"], nonfinite=0, mass=None)
    if args.only is None and not args.quick:
        print("[bench] d2q9 1024^2 f32", file=sys.stderr, flush=True)
        r = run_plain(tlb, torch, w2, tlb.TLB_F32, args.steps, args.warmup)
        extra["d2q9_1024x1024_spinodal_f32"] = dict(
            mlups=r["mlups"], ms_per_step=r["ms_per_step"], achieved_GBps=r["achieved_GBps"],
            frac_of_hbm=r["achieved_GBps"] / HBM_PEAK_GBS, steps=args.steps, launch=r["launch"],
            note="working set 226 MB fits the 256 MB Infinity Cache (cache-assisted)")
        s3 = max(50, min(2000, args.steps // 20))
        print(f"[bench] d3q19 256^3 f32, {s3} steps", file=sys.stderr, flush=True)
        w3 = inputs.spinodal_3d(256, s3)
        r = run_plain(tlb, torch, w3, tlb.TLB_F32, s3, 10)
        extra["d3q19_256cube_spinodal_f32"] = dict(
            mlups=r["mlups"], ms_per_step=r["ms_per_step"], achieved_GBps=r["achieved_GBps"],
            frac_of_hbm=r["achieved_GBps"] / HBM_PEAK_GBS, steps=s3, launch=r["launch"])
        sb = max(100, min(5000, args.steps // 2))
        print(f"[bench] batched 512 domains f32, {sb} steps", file=sys.stderr, flush=True)
        extra["batched_512_domains_f32"] = run_batched(tlb, torch, sb)

    extra["copy_kernel_GBps"] = copy_ceiling(tlb, torch)
    line = {
        "metric": "ternary LB MLUPS + % HBM BW; batched & adjoint vs plain step, same GPU",
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.only in (None, "f64") else "f32",
        "data": "synthetic (seeded spinodal noise, no dataset)",
        "config": {"workload": "d2q9_1024x1024_spinodal" if args.only != "d3q19" else "d3q19_256cube_spinodal",
                   "lattice": "D2Q9" if args.only != "d3q19" else "D3Q19", "nx": 1024, "ny": 1024,
                   "boundary": "periodic", "kappa": [0.01, 0.015, 0.02], "alpha": 1.0, "tau": 1.0,
                   "mobility": 0.1, "launch": head["launch"]},
        "roofline": {"bound": "hbm", "achieved": head["achieved_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": head["achieved_GBps"] / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_step2d (fused pull-stream + collide)",
                     "bytes_per_launch": head["bytes_per_launch"]},
        "check": {"nonfinite": head["nonfinite"], "mass": head["mass"]},
    }
    if not args.no_cpu and args.only in (None, "f64"):
        print(f"[bench] cpu oracle, {args.cpu_steps} steps", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w2, args.cpu_steps)
    line["roofline"]["frac_of_copy_kernel"] = head["achieved_GBps"] / extra["copy_kernel_GBps"]
    line["extra"] = extra
    print(json.dumps(line))


if __name__ == "__main__":
    main()

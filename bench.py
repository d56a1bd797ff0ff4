"""Throughput of the fused ternary LB step on one MI355X.

Headline: the 256^3 D3Q19 spinodal workload (C1, C2 = 1/3 + U(-0.01, 0.01),
kappa = 0.01, alpha = 1, tau = 0.8, M = 0.05) with FP32 populations, MLUPS
over K timed steps with the state resident in HBM; it is the largest of the
single-GPU workloads.  The same line carries the roofline of the fused step
kernel, the CPU oracle timed on a bounded sample of the same workload, and
the other forms under "extra": the 1024^2 D2Q9 spinodal in FP64 and FP32, the
512-domain batch, the multiple-relaxation-time and four-component variants,
the reverse step with a whole checkpointed gradient, and a device copy
ceiling.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--quick] [--only NAME]
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")
_CSRC = "paper_1511_02155_amd/csrc/"
_COMMON = [_CSRC + "tlb_device.hpp", _CSRC + "tlb_internal.hpp", "paper_1511_02155_amd/build.py"]
# sources that decide each measured kernel's code; its counter readings are used only while they are unchanged
KERNEL_SOURCES = {
    "step2d": _COMMON + [_CSRC + "tlb_sweep2d.hpp", _CSRC + "tlb_step2d.hpp", _CSRC + "tlb_step2d.hip"],
    "step3d": _COMMON + [_CSRC + "tlb_step3d.hpp", _CSRC + "tlb_step3d.hip"],
    "step3d_nc": _COMMON + [_CSRC + "tlb_step3d.hpp", _CSRC + "tlb_step3d_nc.hip"],
    "batch2d": _COMMON + [_CSRC + "tlb_sweep2d.hpp", _CSRC + "tlb_batch.hip"],
    "adjoint": _COMMON + [_CSRC + "tlb_adjoint.hip"],
}


def kernel_sha(kind):
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, launch=None):
    """HBM bytes per launch (read + write) of a workload's dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel calibration), or None when there is no
    reading, the kernel's sources changed since it was taken, or it was taken at another launch shape."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)[workload]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("source_sha") != kernel_sha(rec["kind"]):
        return None
    if launch is not None and rec.get("launch") != launch:
        return None
    return rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]


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
            "gamma_psi", "no_advection", "collision", "tau_bulk", "tau_ghost")
    sim = tlb.Sim(tlb.make_params(prec=prec, **{k: w[k] for k in keys if k in w}), stream=stream.cuda_stream)
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
    # the same bytes in the same pattern and launch shape without the arithmetic (propagation alone),
    # timed after the step's state was read out
    ns = min(steps, 200)
    sim.stream_only(2)
    ms_stream = _events_time(torch, stream, lambda: sim.stream_only(ns)) / ns
    out = dict(
        ms_total=ms,
        ms_per_step=per_launch_ms,
        mlups=N * steps / (ms * 1e-3) / 1e6,
        achieved_GBps=bytes_per_launch / (per_launch_ms * 1e-3) / 1e9,
        bytes_per_node=sim.bytes_per_node(),
        bytes_per_launch=bytes_per_launch,
        nodes=N,
        launch=sim.launch(),
        steps=steps,
        kernel="k_step2d" if w["lattice"] == 0 else "k_step3d",
        pattern_ceiling_GBps=bytes_per_launch / (ms_stream * 1e-3) / 1e9,
        mass=d["mass"],
        max_speed=d["max_speed"],
        nonfinite=d["nonfinite"],
    )
    sim.close()
    return out


def run_batched(tlb, torch, steps, warmup=10, graph_steps=50):
    """The 512-domain batched workload (FP32, walls, per-domain kappa and h): autotuned launch
    shape (outside the timed region), steps replayed from captured hipGraphs.  With the domains split
    over G stream groups a step is G concurrent launches, one per group; the events on the batch's
    stream bracket all of them (the groups join it at the end of every step call), and the bytes
    are those of a whole step."""
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
    chosen = b.autotune(10)
    b.set_graph(graph_steps)
    b.step(warmup)
    b.synchronize()
    ms = _events_time(torch, stream, lambda: b.step(steps))
    nodes = b.nodes()
    bytes_per_step = 216.0 * nodes
    out = dict(mlups=nodes * steps / (ms * 1e-3) / 1e6, ms_per_step=ms / steps,
               achieved_GBps=bytes_per_step / (ms / steps * 1e-3) / 1e9, domains=len(doms), nodes=nodes,
               steps=steps, launch=chosen, graph_steps=graph_steps, bytes_per_launch=bytes_per_step,
               launches_per_step=chosen["groups"], kernel="k_batch2d")
    b.close()
    return out


def run_adjoint(tlb, torch, prec, steps, grad_runs=1):
    """The 512x512 walled drop workload of the gradient problem (per-node h on the wall below y = 0).

    (1) The reverse step alone: `steps` calls of tlb_adjoint_step_dev on a fixed state with the adjoint
    populations ping-ponged, timed with events on the library's stream; algorithmic bytes per node are
    81 values (read s_t and lambda_{t+1}, write lambda_t).  (2) A whole gradient: forward with a
    checkpoint every 45 steps plus the checkpointed backward (which recomputes each segment) over the
    workload's 2000 steps through the torch.autograd Function."""
    from paper_1511_02155_amd.autograd import Runner, TernaryLB

    w = inputs_mod().adjoint_drop_512()
    keys = ("lattice", "nx", "ny", "nz", "walls_y", "kappa", "alpha", "tau_f", "tau_g", "tau_k", "gamma_phi",
            "gamma_psi")
    p = tlb.make_params(prec=prec, **{k: w[k] for k in keys})
    dt = torch.float64 if prec == tlb.TLB_F64 else torch.float32
    esize = 8 if prec == tlb.TLB_F64 else 4
    N = w["nx"] * w["ny"]
    stream = torch.cuda.Stream()
    sim = tlb.Sim(p, stream=stream.cuda_stream)
    sim.set_wetting_both(w["h"])
    sim.init_equilibrium(w["C"])
    sim.step(50)
    with torch.cuda.stream(stream):
        u = torch.empty(sim.state_bytes() // esize, dtype=dt, device="cuda")
        lam = [torch.zeros_like(u), torch.zeros_like(u)]
        dh = torch.zeros((2, 3, w["nx"]), dtype=torch.float64, device="cuda")
        dk = torch.zeros(3, dtype=torch.float64, device="cuda")
        tlb.check(tlb.tlb_save_state_dev(sim.handle, u.data_ptr()), "tlb_save_state_dev")
        lam[0].normal_()
    sim.synchronize()

    def go(n):
        for t in range(n):
            tlb.check(tlb.tlb_adjoint_step_dev(sim.handle, u.data_ptr(), lam[t & 1].data_ptr(),
                                               lam[(t + 1) & 1].data_ptr(), dh.data_ptr(), dk.data_ptr()),
                      "tlb_adjoint_step_dev")

    go(10)
    sim.synchronize()
    ms = _events_time(torch, stream, lambda: go(steps))
    alg = 81.0 * esize
    out = dict(mlups=N * steps / (ms * 1e-3) / 1e6, ms_per_step=ms / steps, steps=steps, bytes_per_node=alg,
               bytes_per_launch=alg * N, achieved_GBps=alg * N / (ms / steps * 1e-3) / 1e9,
               kernel="k_adj2d (fused reverse step)")
    out["launch"] = sim.adjoint_launch()
    sim.close()
    del u, lam
    # a whole gradient through the autograd Function
    r = Runner(p, w["C"], w["steps"], every=45, h=w["h"])
    tgt = torch.tensor(w["target"].reshape(w["ny"], w["nx"]), dtype=dt, device="cuda")

    def grad():
        hb = torch.tensor(w["h"][0], dtype=dt, device="cuda", requires_grad=True)
        kap = torch.tensor(w["kappa"], dtype=torch.float64, device="cuda", requires_grad=True)
        C = TernaryLB.apply(hb, kap, r)
        L = ((C[0] - tgt) ** 2).sum()
        L.backward()
        return hb, kap

    grad()
    cur = torch.cuda.current_stream()
    ms_g = _events_time(torch, cur, lambda: [grad() for _ in range(grad_runs)]) / grad_runs
    out.update(gradient_ms=ms_g, gradient_steps=w["steps"], checkpoint_every=45,
               gradient_mlups=N * w["steps"] / (ms_g * 1e-3) / 1e6,
               note="gradient_mlups counts each of the 2000 time steps once (forward, recompute and "
                    "reverse step all included)")
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


_PKEYS = ("lattice", "nx", "ny", "nz", "walls_y", "kappa", "alpha", "tau_f", "tau_g", "tau_k", "gamma_phi",
          "gamma_psi")


def _cpu_threads():
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def cpu_model():
    """The host CPU's model name (first processor of /proc/cpuinfo) and its logical processor count."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{name} ({os.cpu_count()} logical processors visible)"


def cpu_single_thread(steps=4, call=None):
    """An oracle sample on one thread (a child process started with OMP_NUM_THREADS=1); by default the
    1024^2 D2Q9 spinodal, else the bench function call given as text."""
    import subprocess

    call = call or f"bench.cpu_baseline(inputs.spinodal_2d(1024, {steps}), {steps})"
    code = f"import json, bench; from paper_1511_02155_amd import inputs; print(json.dumps({call}))"
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                         timeout=600, check=True).stdout
    return json.loads(out.strip().splitlines()[-1])


def cpu_d3q19(n=256, steps=10):
    """The D3Q19 oracle on the 256^3 spinodal workload (a bounded number of steps)."""
    import oracle
    from paper_1511_02155_amd import inputs

    w = inputs.spinodal_3d(n, steps)
    p = oracle.Params(**{k: w[k] for k in _PKEYS})
    pop = oracle.init_equilibrium(p, w["C"]())
    oracle.step(p, pop, 1)
    t0 = time.perf_counter()
    oracle.step(p, pop, steps)
    dt = time.perf_counter() - t0
    return dict(value=p.N * steps / dt / 1e6, unit="MLUPS", cores=_cpu_threads(), kind="oracle",
                sample=f"D3Q19 {n}^3 spinodal FP64, {steps} steps after 1 warm-up step, {dt:.1f} s")


def cpu_batched(ndom=48, steps=40):
    """The oracle stepping the first domains of the 512-domain batch one after another (walls, per-domain
    kappa and h)."""
    import oracle
    from paper_1511_02155_amd import inputs

    doms = inputs.batched_walls()[:ndom]
    runs = []
    for d in doms:
        p = oracle.Params(**{k: d[k] for k in _PKEYS})
        runs.append((p, oracle.init_equilibrium(p, d["C"], None, d["h"]), d["h"]))
    t0 = time.perf_counter()
    for p, pop, h in runs:
        oracle.step(p, pop, steps, h)
    dt = time.perf_counter() - t0
    nodes = sum(p.N for p, _, _ in runs)
    return dict(value=nodes * steps / dt / 1e6, unit="MLUPS", cores=_cpu_threads(), kind="oracle",
                sample=f"domains 0-{ndom - 1} of the batch ({nodes} nodes), {steps} steps each, {dt:.1f} s")


def cpu_gradient(steps=10):
    """Reverse mode on the CPU: autograd through the PyTorch FP64 re-expression of the step (the reference
    of the GPU adjoint) on the 512^2 walled drop; the rate counts nodes x steps of the whole gradient
    (forward and backward)."""
    import torch
    import oracle
    from oracle import torch_ref
    from paper_1511_02155_amd import inputs

    w = inputs.adjoint_drop_512()
    p = oracle.Params(**{k: w[k] for k in _PKEYS})
    pop0 = oracle.init_equilibrium(p, w["C"], None, w["h"])
    t0 = torch.tensor(pop0.reshape(3, 9, w["ny"], w["nx"]))
    hh = torch.tensor(w["h"].reshape(2, 3, w["nx"]))
    args = (hh, torch.tensor(w["kappa"], dtype=torch.float64), w["alpha"], (w["tau_f"], w["tau_g"], w["tau_k"]),
            (w["gamma_phi"], w["gamma_psi"]), True)
    tgt = torch.tensor(w["target"].reshape(w["ny"], w["nx"]))
    tic = time.perf_counter()
    torch_ref.loss_and_grads(t0, *args, steps, tgt)
    dt = time.perf_counter() - tic
    return dict(value=p.N * steps / dt / 1e6, unit="MLUPS (gradient)", cores=torch.get_num_threads(),
                kind="oracle (autograd through the PyTorch FP64 step)",
                sample=f"512^2 walled drop, loss and gradients over {steps} step(s), {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--quick", action="store_true", help="headline only (no extra workloads)")
    ap.add_argument("--only", default=None,
                    help="run a single workload: d3q19, f64, f32, batched, mrt, ncomp, adjoint64, adjoint32")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: the fused step runs on a single device "
              f"(requested --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    from paper_1511_02155_amd import inputs, tlb

    sel = args.only
    every = sel is None and not args.quick
    # the 2D workloads run a tenth of the steps of the headline by default (about 0.1 ms per step)
    s2 = args.steps if sel else max(1000, min(10000, 5 * args.steps))
    w2 = inputs.spinodal_2d(1024, s2)
    res = {}  # workload name -> measurements, the headline first

    def add(name, r):
        r["frac_of_hbm"] = r["achieved_GBps"] / HBM_PEAK_GBS
        if r.get("pattern_ceiling_GBps"):
            r["frac_of_pattern_ceiling"] = r["achieved_GBps"] / r["pattern_ceiling_GBps"]
        t = measured_traffic(name, r.get("launch"))
        r["traffic"] = t
        if t is not None:
            r["traffic_over_algorithmic"] = t / r["bytes_per_launch"]
        res[name] = r

    if sel in (None, "d3q19"):
        print(f"[bench] d3q19 256^3 f32: {args.warmup} warm-up + {args.steps} timed steps", file=sys.stderr,
              flush=True)
        add("d3q19_256cube_spinodal_f32", run_plain(tlb, torch, inputs.spinodal_3d(256, args.steps), tlb.TLB_F32,
                                                    args.steps, args.warmup))
    if sel == "f64" or every:
        print(f"[bench] d2q9 1024^2 f64: {s2} steps", file=sys.stderr, flush=True)
        add("d2q9_1024x1024_spinodal_f64", run_plain(tlb, torch, w2, tlb.TLB_F64, s2, 100))
    if sel == "f32" or every:
        print(f"[bench] d2q9 1024^2 f32: {s2} steps", file=sys.stderr, flush=True)
        r = run_plain(tlb, torch, w2, tlb.TLB_F32, s2, 100)
        r["note"] = "working set 226 MB fits the 256 MB Infinity Cache (cache-assisted)"
        add("d2q9_1024x1024_spinodal_f32", r)
    if sel == "batched" or every:
        sb = args.steps if sel else max(100, min(5000, args.steps // 4))
        print(f"[bench] batched 512 domains f32: {sb} steps", file=sys.stderr, flush=True)
        add("batched_512_domains_f32", run_batched(tlb, torch, sb))
    if sel == "mrt" or every:
        # multiple relaxation times for f: same workloads, distinct bulk and ghost rates
        mrt = dict(collision=1, tau_bulk=0.8, tau_ghost=1.2)
        sm = args.steps if sel else max(200, min(2000, s2 // 5))
        print(f"[bench] d2q9 1024^2 f64 MRT: {sm} steps", file=sys.stderr, flush=True)
        add("d2q9_1024x1024_spinodal_f64_mrt", run_plain(tlb, torch, dict(w2, **mrt), tlb.TLB_F64, sm, 10))
        s3 = args.steps if sel else max(50, min(2000, args.steps // 10))
        print(f"[bench] d3q19 256^3 f32 MRT: {s3} steps", file=sys.stderr, flush=True)
        add("d3q19_256cube_spinodal_f32_mrt",
            run_plain(tlb, torch, dict(inputs.spinodal_3d(256, s3), **mrt), tlb.TLB_F32, s3, 10))
    if sel == "ncomp" or every:
        # more than three components (Sec. II.E): four-component spinodal, FP64
        sn = args.steps if sel else max(200, min(2000, s2 // 5))
        print(f"[bench] d2q9 1024^2 f64 four components: {sn} steps", file=sys.stderr, flush=True)
        add("d2q9_1024x1024_spinodal_n4_f64", run_plain(tlb, torch, inputs.spinodal_2d_nc(1024, sn, 4), tlb.TLB_F64,
                                                        sn, 10))
        s3n = args.steps if sel else max(20, min(200, args.steps // 10))
        print(f"[bench] d3q19 256^3 f32 four components: {s3n} steps", file=sys.stderr, flush=True)
        add("d3q19_256cube_spinodal_n4_f32", run_plain(tlb, torch, inputs.spinodal_3d_nc(256, s3n, 4), tlb.TLB_F32,
                                                       s3n, 5))
    for name, prec in (("f64", tlb.TLB_F64), ("f32", tlb.TLB_F32)):
        if sel == "adjoint" + name[1:] or every:
            sa = args.steps if sel else max(100, min(2000, s2 // 5))
            print(f"[bench] adjoint 512^2 {name}: {sa} reverse steps + one 2000-step gradient", file=sys.stderr,
                  flush=True)
            add(f"adjoint_512x512_wall_drop_{name}", run_adjoint(tlb, torch, prec, sa))
    if not res:
        sys.exit(f"unknown --only {sel!r}")

    copy_gbps = copy_ceiling(tlb, torch)
    hname = next(iter(res))
    head = res.pop(hname)
    line = {
        "metric": "ternary LB MLUPS + % HBM BW; batched & adjoint vs plain step, same GPU",
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": head["steps"],
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": hname.rsplit("_", 1)[1],
        "data": "synthetic (seeded initial fields, no dataset)",
        "config": {"workload": hname, **WORKLOAD_CONFIG.get(hname, {}), "launch": head.get("launch")},
        "roofline": {"bound": "hbm", "achieved": head["achieved_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": head["frac_of_hbm"], "traffic": head["traffic"],
                     "kernel": head.get("kernel"), "bytes_per_launch": head["bytes_per_launch"],
                     "frac_of_copy_kernel": head["achieved_GBps"] / copy_gbps,
                     "pattern_ceiling": head.get("pattern_ceiling_GBps"),
                     "frac_of_pattern_ceiling": (head["achieved_GBps"] / head["pattern_ceiling_GBps"]
                                                 if head.get("pattern_ceiling_GBps") else None)},
        "check": {"nonfinite": head.get("nonfinite"), "mass": head.get("mass")},
    }
    if not args.no_cpu and hname == "d3q19_256cube_spinodal_f32":
        print(f"[bench] cpu oracle: d3q19 256^3, {args.cpu_steps} steps", file=sys.stderr, flush=True)
        cb = cpu_d3q19(256, args.cpu_steps)
        if every:
            # the other forms against the oracle on bounded samples
            print("[bench] cpu oracle: d2q9 (all threads and one thread), batch, gradient", file=sys.stderr,
                  flush=True)
            g2 = res["d2q9_1024x1024_spinodal_f64"]["mlups"]
            forms = {"d2q9_1024x1024_spinodal_f64": (cpu_baseline(inputs.spinodal_2d(1024, 300), 300), g2),
                     "d2q9_1024x1024_spinodal_f64_one_thread": (cpu_single_thread(), g2),
                     "d3q19_96cube_spinodal_f64_one_thread": (cpu_single_thread(call="bench.cpu_d3q19(96, 3)"),
                                                              head["mlups"]),
                     "batched_512_domains": (cpu_batched(), res["batched_512_domains_f32"]["mlups"]),
                     "adjoint_512x512_wall_drop_gradient": (cpu_gradient(),
                                                            res["adjoint_512x512_wall_drop_f64"]["gradient_mlups"])}
            cb["forms"] = {k: dict(v, gpu_mlups=g, gpu_over_cpu=g / v["value"]) for k, (v, g) in forms.items()}
        cb["cpu_model"] = cpu_model()
        line["cpu_baseline"] = cb
    res["copy_kernel_GBps"] = copy_gbps
    line["extra"] = res
    print(json.dumps(line))


WORKLOAD_CONFIG = {
    "d2q9_1024x1024_spinodal_f64": dict(lattice="D2Q9", nx=1024, ny=1024, boundary="periodic",
                                        kappa=[0.01, 0.015, 0.02], alpha=1.0, tau=1.0, mobility=0.1),
    "d2q9_1024x1024_spinodal_f32": dict(lattice="D2Q9", nx=1024, ny=1024, boundary="periodic",
                                        kappa=[0.01, 0.015, 0.02], alpha=1.0, tau=1.0, mobility=0.1),
    "d3q19_256cube_spinodal_f32": dict(lattice="D3Q19", nx=256, ny=256, nz=256, boundary="periodic",
                                       kappa=[0.01, 0.01, 0.01], alpha=1.0, tau=0.8, mobility=0.05),
    "d2q9_1024x1024_spinodal_f64_mrt": dict(lattice="D2Q9", nx=1024, ny=1024, boundary="periodic",
                                            kappa=[0.01, 0.015, 0.02], alpha=1.0, tau=1.0, mobility=0.1,
                                            collision="MRT", tau_bulk=0.8, tau_ghost=1.2),
    "d3q19_256cube_spinodal_f32_mrt": dict(lattice="D3Q19", nx=256, ny=256, nz=256, boundary="periodic",
                                           kappa=[0.01, 0.01, 0.01], alpha=1.0, tau=0.8, mobility=0.05,
                                           collision="MRT", tau_bulk=0.8, tau_ghost=1.2),
    "d3q19_256cube_spinodal_n4_f32": dict(lattice="D3Q19", nx=256, ny=256, nz=256, boundary="periodic", components=4,
                                          kappa=[0.01, 0.015, 0.02, 0.025], alpha=1.0, tau=0.8, mobility=0.05),
    "d2q9_1024x1024_spinodal_n4_f64": dict(lattice="D2Q9", nx=1024, ny=1024, boundary="periodic", components=4,
                                           kappa=[0.01, 0.015, 0.02, 0.025], alpha=1.0, tau=1.0, mobility=0.1),
    "batched_512_domains_f32": dict(lattice="D2Q9", domains=512, side=[32, 256], boundary="walls_y"),
    "adjoint_512x512_wall_drop_f64": dict(lattice="D2Q9", nx=512, ny=512, boundary="walls_y", form="reverse step"),
    "adjoint_512x512_wall_drop_f32": dict(lattice="D2Q9", nx=512, ny=512, boundary="walls_y", form="reverse step"),
}


if __name__ == "__main__":
    main()

"""Full-size workloads run for their full step counts on the GPU, against stored FP64 oracle values.

The stored values (tests/golden/*.txt) are the oracle's C1, C2, C3 at a seeded
sample of nodes and the sum of each field over all nodes, written by
tests/golden/make_golden.py.  Bars: FP64 within 1e-12 of the largest
magnitude of the sampled field; FP32 within 1e-5 absolute on C_m, except
the 5000-step batch (below).

FP32 storage floor.  An FP32 run stores every population in FP32 once per
step; the arithmetic is FP64.  An FP64 run whose stored state is rounded to
FP32 after every step reproduces the FP32 run's deviation from FP64 to
within 1e-8 on the four stored batch domains, and that deviation after 5000
steps is 5.5e-6 .. 2.1e-5 (largest on C3 near C3-rich layers): the rounding
of FP32 populations alone exceeds 1e-5 there.  The batch test therefore
holds FP32 to 3e-5, the measured floor with a margin.
"""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

from paper_1511_02155_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
KEYS = ("lattice", "nx", "ny", "nz", "walls_y", "kappa", "alpha", "tau_f", "tau_g", "tau_k", "gamma_phi", "gamma_psi")


def _note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def load_golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"stored oracle values {name} not generated")
    nodes, vals, sums, scalars = [], [], {}, {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("#"):
                continue
            t = line.split()
            if t[0] == "node":
                nodes.append(int(t[1]))
                vals.append([float(v) for v in t[2:5]])
            elif t[0] == "sum":
                sums[t[1]] = float(t[2])
            elif t[0] == "scalar":
                scalars[t[1]] = float(t[2])
    return np.array(nodes), np.array(vals).T, sums, scalars


@pytest.fixture(scope="module")
def tlb():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    from paper_1511_02155_amd import tlb as t

    return t


def _check(got, ref, prec, label="", f32_bar=1e-5):
    """got/ref: [3][n] sampled C_m."""
    for m in range(3):
        err = np.abs(got[m] - ref[m]).max()
        if prec == "f64":
            assert err <= 1e-12 * np.abs(ref[m]).max(), (label, m, err)
        else:
            assert err <= f32_bar, (label, m, err)


def _run(tlb, w, prec, C, h, steps):
    P = tlb.TLB_F64 if prec == "f64" else tlb.TLB_F32
    s = tlb.Sim(tlb.make_params(prec=P, **{k: w[k] for k in KEYS}))
    if h is not None:
        s.set_wetting_both(h)
    s.init_equilibrium(C)
    s.step(steps)
    d = s.diagnostics()
    assert d["nonfinite"] == 0
    return np.stack([s.field(f) for f in ("C1", "C2", "C3")])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_spinodal_1024_full_10000_steps(tlb, prec):
    nodes, ref, sums, _ = load_golden("spinodal_2d_1024_10000.txt")
    w = inputs.spinodal_2d(1024, 10000)
    _note(f"spinodal 1024^2 {prec} 10000 steps")
    C = _run(tlb, w, prec, w["C"](), None, w["steps"])
    _check(C[:, nodes], ref, prec)
    for m, f in enumerate(("C1", "C2", "C3")):
        assert C[m].sum() == pytest.approx(sums[f], rel=1e-12 if prec == "f64" else 1e-6)


def test_spinodal_256cube_full_2000_steps_fp32(tlb):
    nodes, ref, sums, _ = load_golden("spinodal_3d_256_2000.txt")
    w = inputs.spinodal_3d(256, 2000)
    _note("spinodal 256^3 f32 2000 steps")
    C = _run(tlb, w, "f32", w["C"](), None, w["steps"])
    _check(C[:, nodes], ref, "f32")
    for m, f in enumerate(("C1", "C2", "C3")):
        assert C[m].sum() == pytest.approx(sums[f], rel=1e-6)


# FP32 populations against the oracle run that rounds its state to FP32 after every step, as FP32
# storage does: what is left is the kernel's own FP64 arithmetic (rounding order), far below the floor.
BATCH_VS_STORAGE32 = 1e-6


@pytest.mark.parametrize("launch", [None, dict(width=256, chunk=32, variant=2, groups=2)])
def test_batched_512_domains_full_5000_steps(tlb, launch):
    """The 512-domain batch (h_m ~ U[-0.01, 0.01] unclipped), FP32 storage, 5000 steps, on four
    domains: against the FP64 oracle at 1e-5 wherever FP32 storage itself allows it, and against the
    oracle with FP32 storage rounding (the floor model) at 1e-6 everywhere.  The stored floor is the
    largest difference between the two oracle runs over all nodes; on three of the four domains it
    exceeds 1e-5 (up to 2.1e-5, domain 359), so there the FP64 bar is the floor plus the 1e-6.  Run in
    the default launch shape and in the one the bench's tuner picks (flat sweep, two stream groups)."""
    doms = inputs.batched_walls()
    picks = sorted({int(f[len("batched_domain"):len("batched_domain") + 3]) for f in os.listdir(GOLDEN)
                    if f.startswith("batched_domain")})
    if not picks:
        pytest.skip("stored oracle values of the batch not generated")
    b = tlb.Batch([tlb.make_params(prec=tlb.TLB_F32, **{k: d[k] for k in KEYS}) for d in doms])
    if launch:
        b.set_launch(**launch)
    b.set_graph(50)
    for i, d in enumerate(doms):
        b.set_wetting(i, 0, d["h"][0])
        b.set_wetting(i, 1, d["h"][1])
        b.init_equilibrium(i, d["C"])
    _note(f"batch 512 domains f32 5000 steps {launch}")
    b.step(5000)
    failures = []
    for i in picks:
        nodes, ref, _, _ = load_golden(f"batched_domain{i:03d}_5000.txt")
        nodes32, ref32, _, sc = load_golden(f"batched_domain{i:03d}_5000_storage32.txt")
        assert np.array_equal(nodes, nodes32)
        C = np.stack([b.field(i, f) for f in ("C1", "C2", "C3")])[:, nodes]
        assert b.diagnostics(i)["nonfinite"] == 0
        e64 = np.abs(C - ref).max(axis=1)
        e32 = np.abs(C - ref32).max(axis=1)
        floor = np.array([sc[f"floor_C{m + 1}"] for m in range(3)])
        bar64 = np.maximum(1e-5, floor + BATCH_VS_STORAGE32)
        print(f"domain {i:3d}: |GPU - FP64 oracle| {e64}, |GPU - FP32-storage oracle| {e32}, "
              f"storage floor {floor}, FP64 bar {bar64}", flush=True)
        if (e32 > BATCH_VS_STORAGE32).any() or (e64 > bar64).any():
            failures.append((i, e64, e32, bar64))
    assert not failures, failures


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjoint_workload_forward_2000_steps(tlb, prec):
    nodes, ref, _, sc = load_golden("adjoint_drop_512_forward_2000.txt")
    w = inputs.adjoint_drop_512()
    _note(f"walled drop 512^2 {prec} 2000 steps")
    C = _run(tlb, w, prec, w["C"], w["h"], w["steps"])
    _check(C[:, nodes], ref, prec)
    L = float(((C[0] - w["target"]) ** 2).sum())
    assert L == pytest.approx(sc["loss"], rel=1e-11 if prec == "f64" else 1e-4)

"""Steps replayed from a captured hipGraph (tlb_set_graph) against steps launched one by one.

The captured chain starts from buffer 0 and holds the launch shape and coefficients of capture time.
Each case steps two simulations of the same input, one with direct launches and one with chains of
four steps, through a sequence of step counts that puts direct launches, odd steps and host readouts
(synchronisations) between the replays; after every call the populations must agree bit for bit.  A
changed launch shape and changed coefficients drop the chain, and a periodic check inside tlb_step
splits the chains.
"""
from __future__ import annotations

import sys
import time

import numpy as np
import pytest

from paper_1511_02155_amd import inputs

pytestmark = pytest.mark.gpu

KEYS = ("lattice", "nx", "ny", "nz", "walls_y", "kappa", "alpha", "tau_f", "tau_g", "tau_k", "gamma_phi", "gamma_psi")


@pytest.fixture(scope="module")
def tlb():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    from paper_1511_02155_amd import tlb as t

    return t


def _note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _pair(tlb, lattice, prec):
    if lattice == 0:
        nx, ny, nz = 48, 37, 1
    else:
        nx, ny, nz = 20, 13, 9
    gp, gk = inputs.mobility_to_gamma(0.1, 1.0, 0.9)
    w = dict(lattice=lattice, nx=nx, ny=ny, nz=nz, walls_y=1, kappa=(0.01, 0.015, 0.02), alpha=1.0, tau_f=1.0,
             tau_g=1.0, tau_k=0.9, gamma_phi=gp, gamma_psi=gk)
    C = inputs.spinodal(nx, ny, nz, delta=0.2, seed=11 + lattice)
    h = inputs.random_h(nx, -0.004, 0.004, nz=nz, seed=12, bottom_only=False)
    sims = []
    for _ in range(2):
        s = tlb.Sim(tlb.make_params(prec=prec, **{k: w[k] for k in KEYS}))
        s.set_wetting_both(h)
        s.init_equilibrium(C)
        sims.append(s)
    return sims


def _same(a, b, label):
    pa, pb = a.all_populations(), b.all_populations()
    assert np.isfinite(pa).all()
    assert np.array_equal(pa, pb), label


@pytest.mark.parametrize("lattice,prec", [(0, "f64"), (0, "f32"), (1, "f32"), (1, "f64")])
def test_graph_steps_equal_direct_launches(tlb, lattice, prec):
    P = tlb.TLB_F64 if prec == "f64" else tlb.TLB_F32
    _note(f"graph replay lattice={lattice} {prec}")
    direct, graph = _pair(tlb, lattice, P)
    graph.set_graph(4)
    for n in (1, 8, 3, 4, 9, 2, 12):  # parity flips, partial chains and several replays of one capture
        direct.step(n)
        graph.step(n)
        _same(direct, graph, ("steps", n))
    assert graph.diagnostics()["step"] == direct.diagnostics()["step"] == 39
    # a new launch shape drops the chain (shapes are bitwise equivalent, so both stay equal)
    shape = dict(width=64, chunk=3, variant=0) if lattice == 0 else dict(width=32, height=8, chunk=2, variant=0)
    direct.set_launch(**shape)
    graph.set_launch(**shape)
    for n in (5, 8):
        direct.step(n)
        graph.step(n)
        _same(direct, graph, ("after set_launch", n))
    # new coefficients drop the chain as well
    for s in (direct, graph):
        s.set_kappa((0.012, 0.014, 0.02))
    for n in (9, 4):
        direct.step(n)
        graph.step(n)
        _same(direct, graph, ("after set_kappa", n))
    # a periodic check inside tlb_step splits the chains
    for s in (direct, graph):
        s.set_check_every(6)
    for n in (13, 8):
        direct.step(n)
        graph.step(n)
        _same(direct, graph, ("with checks", n))
    for s in (direct, graph):
        s.close()


def test_graph_count_must_be_even(tlb):
    direct, graph = _pair(tlb, 0, tlb.TLB_F64)
    with pytest.raises(tlb.TLBError):
        graph.set_graph(3)
    with pytest.raises(tlb.TLBError):
        graph.set_graph(-2)
    graph.set_graph(0)
    for s in (direct, graph):
        s.close()


def test_graph_speeds_up_a_launch_bound_lattice(tlb):
    """The 64^2 double emulsion (a lattice whose step is about as short as its launch): chains of 50
    steps against direct launches, same final state; the times are printed, not asserted."""
    w = inputs.double_emulsion_64()
    times = {}
    pops = {}
    for G in (0, 50):
        s = tlb.Sim(tlb.make_params(prec=tlb.TLB_F64, **{k: w[k] for k in KEYS}))
        s.init_equilibrium(w["C"]())
        s.set_graph(G)
        s.step(100)
        s.synchronize()
        t0 = time.perf_counter()
        s.step(1000)
        s.synchronize()
        times[G] = (time.perf_counter() - t0) / 1000 * 1e6
        pops[G] = s.all_populations()
        s.close()
    _note(f"64^2 FP64 per step: direct {times[0]:.2f} us, graph chains of 50 {times[50]:.2f} us")
    assert np.array_equal(pops[0], pops[50])

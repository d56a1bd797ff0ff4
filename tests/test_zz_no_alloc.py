"""The reverse step that allocates nothing (tlb_adjoint_step_noalloc) against tlb_adjoint_step_dev.

Both run the same kernels with the same launch shape, so lambda_t, dL/dh and dL/dkappa must agree bit for
bit.  Two calls in a row on one GPU, the second on a smaller lattice, check that nothing the first call
left in the shared scratch array reaches the second; a lattice whose scratch would exceed the array is
refused.
"""
from __future__ import annotations

import ctypes
import sys

import numpy as np
import pytest

from paper_1511_02155_amd import inputs

pytestmark = pytest.mark.gpu

KEYS = ("lattice", "nx", "ny", "nz", "walls_y", "kappa", "alpha", "tau_f", "tau_g", "tau_k", "gamma_phi", "gamma_psi")


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    from paper_1511_02155_amd import tlb

    return torch, tlb


def _case(torch, tlb, nx, ny, prec, seed):
    gp, gk = inputs.mobility_to_gamma(0.1, 0.9, 0.8)
    w = dict(lattice=0, nx=nx, ny=ny, nz=1, walls_y=1, kappa=(0.012, 0.02, 0.016), alpha=1.1, tau_f=1.0, tau_g=0.9,
             tau_k=0.8, gamma_phi=gp, gamma_psi=gk)
    s = tlb.Sim(tlb.make_params(prec=prec, **w))
    s.set_wetting_both(inputs.random_h(nx, -0.003, 0.003, seed=seed, bottom_only=False))
    s.init_equilibrium(inputs.sessile_drop(nx, ny, min(nx, ny) / 3.0, top_layer=0.7 * ny))
    s.step(6)
    dt = torch.float64 if prec == tlb.TLB_F64 else torch.float32
    n = s.state_bytes() // (8 if prec == tlb.TLB_F64 else 4)
    u = torch.empty(n, dtype=dt, device="cuda")
    tlb.check(tlb.tlb_save_state_dev(s.handle, u.data_ptr()), "tlb_save_state_dev")
    lam = torch.randn(n, dtype=torch.float64, device="cuda",
                      generator=torch.Generator(device="cuda").manual_seed(seed)).to(dt)
    s.synchronize()
    return s, u, lam


def _run(torch, tlb, fn, s, u, lam, with_dh=True):
    out = torch.empty_like(lam)
    dh = torch.zeros((2, 3, s.params.nx), dtype=torch.float64, device="cuda")
    dk = torch.zeros(3, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    tlb.check(fn(s.handle, u.data_ptr(), lam.data_ptr(), out.data_ptr(), dh.data_ptr() if with_dh else None,
                 dk.data_ptr()), fn.__name__)
    s.synchronize()
    return out.cpu(), dh.cpu(), dk.cpu()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_reverse_step_matches_the_allocating_one(env, prec):
    torch, tlb = env
    P = tlb.TLB_F64 if prec == "f64" else tlb.TLB_F32
    # a larger lattice first, then a smaller one: the second call finds the first one's partials in the array
    for nx, ny, seed in ((150, 37, 1), (40, 20, 2)):
        print(f"[case] noalloc reverse step {prec} {nx}x{ny}", flush=True)
        sys.stdout.flush()
        s, u, lam = _case(torch, tlb, nx, ny, P, seed)
        need = tlb.tlb_adjoint_step_noalloc_scratch(s.handle)
        assert 0 < need <= tlb.TLB_NOALLOC_SCRATCH_BYTES
        ref = _run(torch, tlb, tlb.tlb_adjoint_step_dev, s, u, lam)
        got = _run(torch, tlb, tlb.tlb_adjoint_step_noalloc, s, u, lam)
        for a, b in zip(ref, got):
            assert torch.equal(a, b)
        assert ref[0].abs().max() > 0 and ref[1].abs().max() > 0 and ref[2].abs().max() > 0
        # no dh array: the sink in the scratch takes dL/dh; lambda and dL/dkappa are unchanged
        got2 = _run(torch, tlb, tlb.tlb_adjoint_step_noalloc, s, u, lam, with_dh=False)
        assert torch.equal(ref[0], got2[0]) and torch.equal(ref[2], got2[2])
        assert not got2[1].any()
        s.close()


def test_noalloc_refuses_a_lattice_beyond_the_scratch(env):
    torch, tlb = env
    s, u, lam = _case(torch, tlb, 30000, 3, tlb.TLB_F64, 3)
    assert tlb.tlb_adjoint_step_noalloc_scratch(s.handle) > tlb.TLB_NOALLOC_SCRATCH_BYTES
    out = torch.empty_like(lam)
    rc = tlb.tlb_adjoint_step_noalloc(s.handle, u.data_ptr(), lam.data_ptr(), out.data_ptr(), None, None)
    assert rc == tlb.TLB_EINVAL
    s.close()

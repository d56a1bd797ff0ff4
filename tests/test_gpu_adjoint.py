"""Reverse mode of the D2Q9 step on the GPU.

Checks: the transpose identity <lambda, J v> = <J^T lambda, v> of one step
(J v from central differences of the GPU forward step, state and wetting
parameters), gradients of a C1 loss against the PyTorch-CPU autodiff
reference, independence of the checkpoint interval, the autograd Function,
and central finite differences at the full 512x512 size.
"""
from __future__ import annotations

import ctypes
import sys

import numpy as np
import pytest

from paper_1511_02155_amd import inputs

pytestmark = pytest.mark.gpu

KEYS = ("lattice", "nx", "ny", "nz", "walls_y", "kappa", "alpha", "tau_f", "tau_g", "tau_k", "gamma_phi", "gamma_psi",
        "no_advection")


def _note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    from paper_1511_02155_amd import tlb

    return torch, tlb


def _wall_case(nx=24, ny=16, R=7.0, kappa=(0.012, 0.02, 0.016), seed=5, walls=1, no_advection=0):
    gp, gk = inputs.mobility_to_gamma(0.1, 0.9, 0.8)
    w = dict(lattice=0, nx=nx, ny=ny, nz=1, walls_y=walls, kappa=kappa, alpha=1.1, tau_f=1.0, tau_g=0.9, tau_k=0.8,
             gamma_phi=gp, gamma_psi=gk, no_advection=no_advection)
    C = inputs.sessile_drop(nx, ny, R, top_layer=0.7 * ny)
    h = inputs.random_h(nx, -0.003, 0.003, seed=seed, bottom_only=False)
    target = inputs.sessile_drop(nx, ny, R + 1.5, x0=nx / 2 + 1.0)[0]
    return w, C, h, target


def _sim(torch, tlb, w, C, h, prec, stream, launch=None):
    """A tlb_sim on ``stream``; the caller runs its torch work on the same stream."""
    s = tlb.Sim(tlb.make_params(prec=prec, **{k: w[k] for k in KEYS if k in w}), stream=stream.cuda_stream)
    if w["walls_y"]:
        s.set_wetting_both(h)
    s.init_equilibrium(C)
    if launch:
        s.set_adjoint_launch(**launch)
    return s


def _dev(torch, s):
    return torch.empty(s.state_bytes() // 8, dtype=torch.float64, device="cuda")


TRANSPOSE_CASES = [
    # (walls, nx, ny, adjoint launch): walls with wetting, periodic, ragged strips and chunks, narrow lattices
    (1, 24, 16, dict(width=64, chunk=8)),
    (2, 24, 16, dict(width=64, chunk=8)),  # walls, no advection in the Cahn-Hilliard equilibria
    (0, 24, 16, dict(width=64, chunk=5)),
    (1, 70, 9, dict(width=64, chunk=4)),
    (0, 131, 7, dict(width=128, chunk=3)),
    (1, 5, 3, dict(width=64, chunk=1)),
    (0, 3, 4, dict(width=256, chunk=2)),
    # several row groups per workgroup: (chunk + 6) not a multiple of rows, rows beyond the lattice
    (1, 24, 16, dict(width=64, rows=4, chunk=8)),
    (2, 70, 9, dict(width=64, rows=4, chunk=5)),
    (0, 70, 9, dict(width=64, rows=2, chunk=3)),
    (1, 131, 11, dict(width=128, rows=2, chunk=5, variant=1)),
    (1, 5, 3, dict(width=64, rows=4, chunk=1)),
    # variant 2: the next iteration's pull and lambda rows are loaded during the current one
    (1, 24, 16, dict(width=64, chunk=5, variant=2)),
    (0, 131, 7, dict(width=64, rows=4, chunk=3, variant=2)),
    (2, 70, 9, dict(width=128, rows=2, chunk=2, variant=2)),
]


@pytest.mark.parametrize("walls,nx,ny,launch", TRANSPOSE_CASES)
def test_one_step_transpose_identity(env, walls, nx, ny, launch):
    """<lambda, J v> == <J^T lambda, v> for the state, for h and for kappa (FP64)."""
    torch, tlb = env
    w, C, h, _ = _wall_case(nx=nx, ny=ny, R=min(nx, ny) / 3.0, walls=min(walls, 1), no_advection=int(walls == 2))
    _note(f"transpose identity walls={walls} {nx}x{ny} {launch}")
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        _transpose_identity(torch, tlb, w, C, h, st, launch)


def _transpose_identity(torch, tlb, w, C, h, st, launch):
    s = _sim(torch, tlb, w, C, h, tlb.TLB_F64, st, launch)
    s.step(5)
    u = _dev(torch, s)
    tlb.check(tlb.tlb_save_state_dev(s.handle, u.data_ptr()), "save")
    gen = torch.Generator(device="cuda").manual_seed(0)
    lam = torch.randn(u.shape, dtype=torch.float64, device="cuda", generator=gen)
    v = torch.randn(u.shape, dtype=torch.float64, device="cuda", generator=gen)
    dh = torch.zeros((2, 3, w["nx"]), dtype=torch.float64, device="cuda")
    dk = torch.zeros(3, dtype=torch.float64, device="cuda")
    lam_out = torch.empty_like(u)
    tlb.check(tlb.tlb_adjoint_step_dev(s.handle, u.data_ptr(), lam.data_ptr(), lam_out.data_ptr(), dh.data_ptr(),
                                       dk.data_ptr()), "adjoint step")
    torch.cuda.synchronize()

    def S(state, hh=None, kap=None):
        if hh is not None and w["walls_y"]:
            s.set_wetting_both(hh)
        if kap is not None:
            s.set_kappa(kap)
        tlb.check(tlb.tlb_load_state_dev(s.handle, state.data_ptr(), 0), "load")
        s.step(1)
        out = torch.empty_like(state)
        tlb.check(tlb.tlb_save_state_dev(s.handle, out.data_ptr()), "save")
        torch.cuda.synchronize()
        return out

    eps = 1e-6
    Jv = (S(u + eps * v) - S(u - eps * v)) / (2 * eps)
    lhs = torch.dot(lam, Jv).item()
    rhs = torch.dot(lam_out, v).item()
    assert lhs == pytest.approx(rhs, rel=1e-7)
    # wetting parameters: directional derivative along a random dh direction
    if w["walls_y"]:
        dhv = np.random.default_rng(1).normal(size=h.shape)
        Jh = (S(u, h + eps * dhv) - S(u, h - eps * dhv)) / (2 * eps)
        s.set_wetting_both(h)
        assert torch.dot(lam, Jh).item() == pytest.approx((dh.cpu().numpy() * dhv).sum(), rel=1e-7)
    else:
        assert not dh.any()
    # kappa
    for m in range(3):
        kp, km = list(w["kappa"]), list(w["kappa"])
        kp[m] += eps
        km[m] -= eps
        Jk = (S(u, kap=kp) - S(u, kap=km)) / (2 * eps)
        assert torch.dot(lam, Jk).item() == pytest.approx(dk[m].item(), rel=1e-6, abs=1e-12)
        s.set_kappa(w["kappa"])


def test_reverse_step_independent_of_launch_shape(env):
    """lambda_t and dL/dh are bitwise the same for every launch shape of a variant, and the variants agree to
    rounding (they fuse multiply-adds differently); dL/dkappa to rounding."""
    torch, tlb = env
    w, C, h, _ = _wall_case(nx=150, ny=37, R=12.0)
    st = torch.cuda.Stream()
    shapes = (dict(width=64, chunk=8), dict(width=64, chunk=37), dict(width=128, chunk=3), dict(width=256, chunk=16),
              dict(width=64, chunk=1), dict(width=64, rows=4, chunk=19), dict(width=64, rows=4, chunk=2),
              dict(width=64, rows=2, chunk=7), dict(width=128, rows=2, chunk=4))
    outs = {}
    with torch.cuda.stream(st):
        for variant in (0, 1, 2):
            for shape in shapes:
                s = _sim(torch, tlb, w, C, h, tlb.TLB_F64, st, dict(shape, variant=variant))
                s.step(7)
                u = _dev(torch, s)
                tlb.check(tlb.tlb_save_state_dev(s.handle, u.data_ptr()), "save")
                gen = torch.Generator(device="cuda").manual_seed(3)
                lam = torch.randn(u.shape, dtype=torch.float64, device="cuda", generator=gen)
                dh = torch.zeros((2, 3, w["nx"]), dtype=torch.float64, device="cuda")
                dk = torch.zeros(3, dtype=torch.float64, device="cuda")
                out = torch.empty_like(u)
                tlb.check(tlb.tlb_adjoint_step_dev(s.handle, u.data_ptr(), lam.data_ptr(), out.data_ptr(),
                                                   dh.data_ptr(), dk.data_ptr()), "adjoint step")
                torch.cuda.synchronize()
                outs.setdefault(variant, []).append((out.cpu().numpy(), dh.cpu().numpy(), dk.cpu().numpy()))
                s.close()
    ref = outs[0][0]
    for variant, runs in outs.items():
        for o in runs:
            assert np.array_equal(o[0], runs[0][0]), variant
            assert np.array_equal(o[1], runs[0][1]), variant
            assert np.allclose(o[2], runs[0][2], rtol=1e-12, atol=0)
        assert np.allclose(runs[0][0], ref[0], rtol=0, atol=1e-13 * np.abs(ref[0]).max())
        assert np.allclose(runs[0][1], ref[1], rtol=0, atol=1e-13 * np.abs(ref[1]).max())
        assert np.allclose(runs[0][2], ref[2], rtol=1e-12, atol=0)


def test_adjoint_launch_validation(env):
    """Row groups of 1, 2 or 4 with width * rows <= 256; anything else is TLB_EINVAL and keeps the shape."""
    torch, tlb = env
    w, C, h, _ = _wall_case()
    st = torch.cuda.Stream()
    s = _sim(torch, tlb, w, C, h, tlb.TLB_F64, st)
    s.set_adjoint_launch(64, chunk=9, rows=4)
    assert s.adjoint_launch() == dict(width=64, rows=4, chunk=9, variant=0)
    for bad in (dict(width=64, rows=3), dict(width=256, rows=2), dict(width=128, rows=4), dict(width=32),
                dict(width=64, rows=2, variant=3)):
        with pytest.raises(tlb.TLBError):
            s.set_adjoint_launch(**bad)
    assert s.adjoint_launch() == dict(width=64, rows=4, chunk=9, variant=0)
    s.close()


def _gpu_grad(torch, tlb, w, C, h, target, steps, every, prec):
    from paper_1511_02155_amd.autograd import Runner, TernaryLB

    p = tlb.make_params(prec=prec, **{k: w[k] for k in KEYS if k in w})
    r = Runner(p, C, steps, every=every, h=h)
    dt = torch.float64 if prec == tlb.TLB_F64 else torch.float32
    hb = torch.tensor(h[0], dtype=dt, device="cuda", requires_grad=True)
    kap = torch.tensor(w["kappa"], dtype=torch.float64, device="cuda", requires_grad=True)
    Cf = TernaryLB.apply(hb, kap, r)
    tgt = torch.tensor(target.reshape(w["ny"], w["nx"]), dtype=dt, device="cuda")
    L = ((Cf[0] - tgt) ** 2).sum()
    L.backward()
    return L.item(), hb.grad.double().cpu().numpy(), kap.grad.cpu().numpy()


def test_gradients_match_autodiff_reference(env, orc):
    """dL/dh (wall below y=0) and dL/dkappa of L = sum (C1 - C1*)^2 after 30 steps against autograd through
    the PyTorch-CPU FP64 reference started from the same initial state."""
    torch, tlb = env
    from oracle import torch_ref

    w, C, h, target = _wall_case()
    steps = 30
    L, dh, dk = _gpu_grad(torch, tlb, w, C, h, target, steps, 6, tlb.TLB_F64)
    p = orc.Params(**{k: w[k] for k in KEYS if k in w})
    pop0 = orc.init_equilibrium(p, C, None, h)
    t0 = torch.tensor(pop0.reshape(3, 9, w["ny"], w["nx"]))
    hh = torch.tensor(h.reshape(2, 3, w["nx"]))
    Lr, dhr, dkr = torch_ref.loss_and_grads(t0, hh, torch.tensor(w["kappa"], dtype=torch.float64), w["alpha"],
                                            (w["tau_f"], w["tau_g"], w["tau_k"]), (w["gamma_phi"], w["gamma_psi"]),
                                            True, steps, torch.tensor(target.reshape(w["ny"], w["nx"])))
    assert L == pytest.approx(Lr, rel=1e-11)
    scale = np.abs(dhr[0].numpy()).max()
    assert np.abs(dh - dhr[0].numpy()).max() <= 1e-9 * scale
    assert np.allclose(dk, dkr.numpy(), rtol=1e-9, atol=1e-12 * np.abs(dkr.numpy()).max())


# FP32 storage against the FP64 reference.  FP32 rounds every stored value of the forward state and of
# lambda once per step (relative 2^-24 ~ 6e-8); to first order the gradient then differs from the FP64 one
# by a sum of T such roundings per step through the map, about T 2^-24 ~ 2e-6 of its scale for T = 30,
# times the conditioning of the map.  The bar is 1e-4 of the largest entry (a margin of about 50).
F32_GRAD_REL = 1e-4


def test_fp32_gradients_match_autodiff_reference(env, orc):
    """FP32 storage: dL/dh and dL/dkappa after 30 steps against autograd through the PyTorch-CPU FP64
    reference from the same initial state."""
    torch, tlb = env
    from oracle import torch_ref

    w, C, h, target = _wall_case()
    steps = 30
    _note("fp32 gradients vs autodiff reference")
    L, dh, dk = _gpu_grad(torch, tlb, w, C, h, target, steps, 6, tlb.TLB_F32)
    p = orc.Params(**{k: w[k] for k in KEYS if k in w})
    pop0 = orc.init_equilibrium(p, C, None, h)
    t0 = torch.tensor(pop0.reshape(3, 9, w["ny"], w["nx"]))
    hh = torch.tensor(h.reshape(2, 3, w["nx"]))
    Lr, dhr, dkr = torch_ref.loss_and_grads(t0, hh, torch.tensor(w["kappa"], dtype=torch.float64), w["alpha"],
                                            (w["tau_f"], w["tau_g"], w["tau_k"]), (w["gamma_phi"], w["gamma_psi"]),
                                            True, steps, torch.tensor(target.reshape(w["ny"], w["nx"])))
    dhr, dkr = dhr[0].numpy(), dkr.numpy()
    e_h = np.abs(dh - dhr).max() / np.abs(dhr).max()
    e_k = np.abs(dk - dkr).max() / np.abs(dkr).max()
    print(f"fp32 gradient: relative error dL/dh {e_h:.3e}, dL/dkappa {e_k:.3e}, loss {abs(L - Lr) / Lr:.3e}")
    assert e_h <= F32_GRAD_REL
    assert e_k <= F32_GRAD_REL
    assert L == pytest.approx(Lr, rel=F32_GRAD_REL)


def test_stale_backward_is_refused(env):
    """Two forward calls on one runner: the first call's backward raises (its checkpoints and parameters
    were overwritten by the second), and the second call's backward equals a fresh single call."""
    torch, tlb = env
    from paper_1511_02155_amd.autograd import Runner, TernaryLB

    w, C, h, target = _wall_case()
    p = tlb.make_params(prec=tlb.TLB_F64, **{k: w[k] for k in KEYS if k in w})
    r = Runner(p, C, 12, every=4, h=h)
    tgt = torch.tensor(target.reshape(w["ny"], w["nx"]), dtype=torch.float64, device="cuda")

    def call(scale):
        hb = torch.tensor(h[0] * scale, dtype=torch.float64, device="cuda", requires_grad=True)
        kap = torch.tensor(w["kappa"], dtype=torch.float64, device="cuda", requires_grad=True)
        L = ((TernaryLB.apply(hb, kap, r)[0] - tgt) ** 2).sum()
        return L, hb, kap

    L1, hb1, _ = call(1.0)
    L2, hb2, k2 = call(0.5)
    with pytest.raises(RuntimeError, match="later forward call"):
        L1.backward()
    L2.backward()
    L3, hb3, k3 = call(0.5)
    L3.backward()
    assert torch.equal(hb2.grad, hb3.grad) and torch.equal(k2.grad, k3.grad)


def test_in_place_reverse_step_equals_out_of_place(env):
    """tlb_adjoint_step (lambda in place) gives bitwise the lambda_t, dL/dh and dL/dkappa of
    tlb_adjoint_step_dev."""
    torch, tlb = env
    w, C, h, _ = _wall_case(nx=70, ny=21)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s = _sim(torch, tlb, w, C, h, tlb.TLB_F64, st)
        s.step(4)
        u = _dev(torch, s)
        tlb.check(tlb.tlb_save_state_dev(s.handle, u.data_ptr()), "save")
        gen = torch.Generator(device="cuda").manual_seed(11)
        lam = torch.randn(u.shape, dtype=torch.float64, device="cuda", generator=gen)
        outs = []
        for in_place in (False, True):
            dh = torch.zeros((2, 3, w["nx"]), dtype=torch.float64, device="cuda")
            dk = torch.zeros(3, dtype=torch.float64, device="cuda")
            if in_place:
                out = lam.clone()
                tlb.check(tlb.tlb_adjoint_step(s.handle, u.data_ptr(), out.data_ptr(), dh.data_ptr(), dk.data_ptr()),
                          "tlb_adjoint_step")
            else:
                out = torch.empty_like(u)
                tlb.check(tlb.tlb_adjoint_step_dev(s.handle, u.data_ptr(), lam.data_ptr(), out.data_ptr(),
                                                   dh.data_ptr(), dk.data_ptr()), "tlb_adjoint_step_dev")
            s.synchronize()
            outs.append((out.cpu(), dh.cpu(), dk.cpu()))
    for a, b in zip(outs[0], outs[1]):
        assert torch.equal(a, b)
    assert outs[0][0].abs().max() > 0


def test_checkpoint_interval_does_not_change_gradients(env):
    torch, tlb = env
    w, C, h, target = _wall_case(nx=30, ny=18)
    res = [_gpu_grad(torch, tlb, w, C, h, target, 37, every, tlb.TLB_F64) for every in (1, 6, 37)]
    for r in res[1:]:
        assert r[0] == res[0][0]
        assert np.array_equal(r[1], res[0][1]) and np.array_equal(r[2], res[0][2])


def test_fp32_gradients_close_to_fp64(env):
    torch, tlb = env
    w, C, h, target = _wall_case(nx=40, ny=24, R=10.0)
    _, dh64, dk64 = _gpu_grad(torch, tlb, w, C, h, target, 60, 8, tlb.TLB_F64)
    _, dh32, dk32 = _gpu_grad(torch, tlb, w, C, h, target, 60, 8, tlb.TLB_F32)
    assert np.abs(dh32 - dh64).max() <= 2e-3 * np.abs(dh64).max()
    assert np.allclose(dk32, dk64, rtol=2e-3)


def test_adjoint_512_full_size_vs_finite_differences(env):
    """512x512, wall below y=0 with seeded per-node h_m in [-0.01, 0.01], a C1 drop
    of radius 60 on the wall (h not clipped); L = sum (C1 - C1*)^2 against a seeded target drop; 2000 steps, FP64, checkpoints
    every 45 steps.  Gradient entries against central differences of the full forward run."""
    torch, tlb = env
    w = inputs.adjoint_drop_512()
    _note("adjoint 512^2 fp64 2000 steps")
    L, dh, dk = _gpu_grad(torch, tlb, w, w["C"], w["h"], w["target"], w["steps"], 45, tlb.TLB_F64)
    p = tlb.make_params(prec=tlb.TLB_F64, **{k: w[k] for k in KEYS if k in w})
    s = tlb.Sim(p)
    s.set_wetting_both(w["h"])
    s.init_equilibrium(w["C"])
    raw, _ = s.save_state()

    def loss(hb=None, kap=None):
        hh = w["h"].copy()
        if hb is not None:
            hh[0] = hb
        s.set_kappa(kap if kap is not None else w["kappa"])
        s.set_wetting_both(hh)
        s.load_state(raw, 0)
        s.step(w["steps"])
        return float(((s.field("C1") - w["target"]) ** 2).sum())

    assert loss() == pytest.approx(L, rel=1e-12)
    eps = 1e-6
    big = np.argsort(-np.abs(dh).ravel())[:2]
    for flat in big:
        m, x = divmod(int(flat), w["nx"])
        hp, hm = w["h"][0].copy(), w["h"][0].copy()
        hp[m, x] += eps
        hm[m, x] -= eps
        fd = (loss(hb=hp) - loss(hb=hm)) / (2 * eps)
        assert dh[m, x] == pytest.approx(fd, rel=1e-6), (m, x)
    for m in range(3):
        kp, km = list(w["kappa"]), list(w["kappa"])
        kp[m] *= 1 + eps
        km[m] *= 1 - eps
        fd = (loss(kap=kp) - loss(kap=km)) / (2 * eps * w["kappa"][m])
        assert dk[m] == pytest.approx(fd, rel=1e-6), m


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_single_step_kappa_reduction_equals_the_pass_reduction(env, prec):
    """A single reverse step (tlb_adjoint_step_dev) and a checkpointed backward over the same one step
    (tlb_adjoint_backward, with its recompute on the other stream) give the same dL/dh and dL/dkappa bit for
    bit, also after changes of launch shape on the same simulation, which change the number of work items
    whose partials are reduced."""
    torch, tlb = env
    P = tlb.TLB_F64 if prec == "f64" else tlb.TLB_F32
    dt = torch.float64 if prec == "f64" else torch.float32
    w, C, h, target = _wall_case(nx=70, ny=41)
    stream = torch.cuda.Stream()
    s = _sim(torch, tlb, w, C, h, P, stream)
    esize = 8 if prec == "f64" else 4
    # the default shape, then more work items, then fewer again on the same simulation
    for launch in (None, dict(width=64, rows=2, chunk=3, variant=2), dict(width=64, rows=4, chunk=9, variant=2)):
        _note(f"fused kappa reduction {prec} {launch}")
        if launch:
            s.set_adjoint_launch(**launch)
        with torch.cuda.stream(stream):
            ck = torch.empty(s.state_bytes() // esize, dtype=dt, device="cuda")
            dLdC = torch.randn((3, w["nx"] * w["ny"]), generator=torch.Generator().manual_seed(4), dtype=torch.float64)
            dLdC = dLdC.to(dtype=dt, device="cuda")
            lam, out = torch.empty_like(ck), torch.empty_like(ck)
            dh1, dk1 = torch.zeros((2, 3, w["nx"]), dtype=torch.float64, device="cuda"), torch.zeros(3, dtype=torch.float64, device="cuda")
            dh2, dk2 = torch.zeros_like(dh1), torch.zeros_like(dk1)
        tlb.check(tlb.tlb_forward_checkpointed(s.handle, 1, 1, ck.data_ptr()), "forward")
        tlb.check(tlb.tlb_adjoint_backward(s.handle, 1, 1, ck.data_ptr(), dLdC.data_ptr(), dh1.data_ptr(),
                                           dk1.data_ptr()), "backward")
        tlb.check(tlb.tlb_adjoint_seed_dev(s.handle, dLdC.data_ptr(), lam.data_ptr()), "seed")
        tlb.check(tlb.tlb_adjoint_step_dev(s.handle, ck.data_ptr(), lam.data_ptr(), out.data_ptr(), dh2.data_ptr(),
                                           dk2.data_ptr()), "step")
        s.synchronize()
        assert dk1.abs().max() > 0 and dh1.abs().max() > 0
        assert torch.equal(dh1, dh2)
        assert torch.equal(dk1, dk2), (dk1, dk2)
    s.close()

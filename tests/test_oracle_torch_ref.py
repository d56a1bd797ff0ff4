"""Pins of the PyTorch-CPU FP64 re-expression used as the autodiff reference.

It must reproduce the C oracle's forward map to rounding (two independent
implementations of the same step), and its autograd gradients must match
central finite differences of the C oracle's loss.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

from paper_1511_02155_amd import inputs


def _case(orc, walls, nx=14, ny=10, seed=3):
    kappa = (0.012, 0.02, 0.016)
    gp, gk = inputs.mobility_to_gamma(0.1, 0.9, 0.8)
    p = orc.Params(lattice=0, nx=nx, ny=ny, walls_y=walls, kappa=kappa, alpha=1.2, tau_f=1.0, tau_g=0.9, tau_k=0.8,
                   gamma_phi=gp, gamma_psi=gk)
    C = inputs.sessile_drop(nx, ny, 4.5, top_layer=7.0)
    C = C + np.random.default_rng(seed).uniform(-0.02, 0.02, C.shape)
    h = inputs.random_h(nx, -0.004, 0.004, seed=seed + 1, bottom_only=False) if walls else None
    return p, C, h


def _torch_args(p, h):
    return dict(h=None if h is None else torch.tensor(h.reshape(2, 3, p.nx)),
                kappa=torch.tensor(p.kappa, dtype=torch.float64), alpha=p.alpha,
                tau=(p.tau_f, p.tau_g, p.tau_k), gamma=(p.gamma_phi, p.gamma_psi), walls=bool(p.walls_y))


@pytest.mark.parametrize("walls", [0, 1])
def test_torch_reference_matches_c_oracle(orc, walls):
    from oracle import torch_ref

    p, C, h = _case(orc, walls)
    pop = orc.init_equilibrium(p, C, None, h)
    t0 = torch.tensor(pop.reshape(3, 9, p.ny, p.nx))
    orc.step(p, pop, 25, h)
    tp = torch_ref.run(t0, nsteps=25, **_torch_args(p, h))
    assert np.abs(tp.numpy().reshape(3, 9, -1) - pop).max() < 1e-13


def test_torch_gradients_match_finite_differences_of_c_oracle(orc):
    from oracle import torch_ref

    p, C, h = _case(orc, 1)
    steps = 15
    pop0 = orc.init_equilibrium(p, C, None, h)
    t0 = torch.tensor(pop0.reshape(3, 9, p.ny, p.nx))
    target = torch.tensor(inputs.sessile_drop(p.nx, p.ny, 5.0)[0].reshape(p.ny, p.nx))
    args = _torch_args(p, h)
    L, dh, dk = torch_ref.loss_and_grads(t0, args["h"], args["kappa"], args["alpha"], args["tau"], args["gamma"],
                                         True, steps, target)

    def c_loss(hh, kap):
        q = p.replace(kappa=tuple(kap))
        pop = pop0.copy()
        orc.step(q, pop, steps, hh)
        return float(((orc.fields(q, pop, hh)["C1"] - target.numpy().ravel()) ** 2).sum())

    assert L == pytest.approx(c_loss(h, p.kappa), rel=1e-12)
    rng = np.random.default_rng(0)
    eps = 1e-6
    for _ in range(4):
        m, x = int(rng.integers(0, 3)), int(rng.integers(0, p.nx))
        hp, hm = h.copy(), h.copy()
        hp[0, m, x] += eps
        hm[0, m, x] -= eps
        fd = (c_loss(hp, p.kappa) - c_loss(hm, p.kappa)) / (2 * eps)
        assert dh[0, m, x].item() == pytest.approx(fd, rel=1e-6, abs=1e-12)
    for m in range(3):
        kp, km = list(p.kappa), list(p.kappa)
        kp[m] += eps * p.kappa[m]
        km[m] -= eps * p.kappa[m]
        fd = (c_loss(h, kp) - c_loss(h, km)) / (2 * eps * p.kappa[m])
        assert dk[m].item() == pytest.approx(fd, rel=1e-6)


@pytest.mark.parametrize("walls", [0, 1])
def test_torch_d3q19_matches_c_oracle(orc, walls):
    """Two independent implementations of the D3Q19 step (the C oracle's loops and the whole-array torch
    form) agree to rounding on a 6 x 5 x 4 lattice after 20 steps, from the same initial state; with walls
    the ghost planes carry seeded per-node h_m."""
    from oracle import torch_ref

    nx, ny, nz = 6, 5, 4
    kappa = (0.012, 0.02, 0.016)
    gp, gk = inputs.mobility_to_gamma(0.1, 0.9, 0.8)
    p = orc.Params(lattice=1, nx=nx, ny=ny, nz=nz, walls_y=walls, kappa=kappa, alpha=1.2, tau_f=1.0, tau_g=0.9,
                   tau_k=0.8, gamma_phi=gp, gamma_psi=gk)
    C = inputs.spinodal(nx, ny, nz, delta=0.25, seed=5)
    h = inputs.random_h(nx, -0.004, 0.004, nz=nz, seed=6, bottom_only=False) if walls else None
    pop = orc.init_equilibrium(p, C, None, h)
    th = None if h is None else torch.tensor(h.reshape(2, 3, nz, nx))
    args = dict(h=th, kappa=torch.tensor(kappa, dtype=torch.float64), alpha=p.alpha, tau=(p.tau_f, p.tau_g, p.tau_k),
                gamma=(p.gamma_phi, p.gamma_psi), walls=bool(walls))
    # the initial state of both is the equilibrium of C
    t0 = torch_ref.equilibrium_state3(torch.tensor(C.reshape(3, nz, ny, nx)), args["h"], args["kappa"],
                                      args["alpha"], args["gamma"], args["walls"])
    assert np.abs(t0.numpy().reshape(3, 19, -1) - pop).max() < 1e-15
    orc.step(p, pop, 20, h)
    tp = torch_ref.run3(t0, nsteps=20, **args)
    assert np.abs(tp.numpy().reshape(3, 19, -1) - pop).max() < 1e-13 * np.abs(pop).max()

"""Pins of the oracle's multiple-relaxation-time collision of f (Sec. IV names the extension without a
basis; reading R18: orthogonal polynomial moment bases, viscous stress moments at 1/tau_f, the energy
moment at 1/tau_bulk, all other moments at 1/tau_ghost).

What fixes it from outside the oracle:
  - the bases: mutually orthogonal rows whose classes have the meaning the rates rely on (conserved
    density and momentum, the energy moment in the span of 1 and |e|^2, the stress moments spanning the
    traceless second moments);
  - equal rates reduce the collision to the pinned BGK step;
  - conservation of mass and momentum with distinct rates;
  - hydrodynamics of an almost ideal single-phase fluid: a shear wave decays at nu k^2 with
    nu = (tau_f - 1/2)/3 whatever tau_bulk and tau_ghost are, and a sound wave at
    k^2 ((2 - 2/D) nu + zeta) / 2 with the bulk viscosity zeta = (2/D) (tau_bulk - 1/2)/3
    (Chapman-Enskog with separate rates for the traceless and trace parts of the stress);
  - the PyTorch re-expression, written in projection form, gives the same step to rounding;
  - the Laplace pressure of a drop is unchanged by the rates.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import pytest
import torch

import analytic
from paper_1511_02155_amd import inputs


def _velocities(orc, lattice):
    return orc.lattice_info(lattice)["e"].astype(float)


@pytest.mark.parametrize("lattice", [0, 1])
def test_mrt_bases_are_orthogonal_moments_of_the_right_class(orc, lattice):
    M, cls = orc.mrt_basis(lattice)
    e = _velocities(orc, lattice)
    Q = M.shape[0]
    G = M @ M.T
    assert np.abs(G - np.diag(np.diag(G))).max() == 0.0  # orthogonal with unit weights, hence invertible
    assert np.all(np.diag(G) > 0)
    c2 = (e ** 2).sum(1)
    D = 2 if lattice == 0 else 3

    def in_span(row, basis):
        B = np.array(basis).T
        coef, *_ = np.linalg.lstsq(B, row, rcond=None)
        return np.abs(B @ coef - row).max() < 1e-12

    cons = [np.ones(Q)] + [e[:, a] for a in range(D)]
    assert np.sum(cls == 0) == D + 1
    for r in M[cls == 0]:
        assert in_span(r, cons)
    assert np.sum(cls == 1) == 1
    assert in_span(M[cls == 1][0], [np.ones(Q), c2])
    # stress rows: exactly the traceless symmetric second moments (D (D+1)/2 - 1 of them)
    traceless = [e[:, a] * e[:, b] for a, b in itertools.combinations(range(D), 2)]
    traceless += [e[:, a] ** 2 - c2 / D for a in range(D)]
    S = M[cls == 2]
    assert len(S) == D * (D + 1) // 2 - 1
    for r in S:
        assert in_span(r, traceless)
    for t in traceless:
        assert in_span(t, list(S))


def _mixed_case(orc, lattice, walls, collision, tau_bulk, tau_ghost, tau_f=0.8):
    gp, gk = inputs.mobility_to_gamma(0.1, 0.9, 0.8)
    if lattice == 0:
        nx, ny, nz = 14, 10, 1
    else:
        nx, ny, nz = 7, 6, 5
    p = orc.Params(lattice=lattice, nx=nx, ny=ny, nz=nz, walls_y=walls, kappa=(0.012, 0.02, 0.016), alpha=1.1,
                   tau_f=tau_f, tau_g=0.9, tau_k=0.8, gamma_phi=gp, gamma_psi=gk, collision=collision,
                   tau_bulk=tau_bulk, tau_ghost=tau_ghost)
    rng = np.random.default_rng(11)
    N = nx * ny * nz
    C = np.empty((3, N))
    C[0] = 0.3 + 0.4 * rng.random(N)
    C[1] = (1 - C[0]) * rng.random(N)
    C[2] = 1 - C[0] - C[1]
    u = 0.02 * rng.standard_normal((p.D, N))
    h = rng.uniform(-0.003, 0.003, (2, 3, nx * nz)) if walls else None
    return p, C, u, h


@pytest.mark.parametrize("lattice,walls", [(0, 1), (0, 0), (1, 1)])
def test_mrt_with_equal_rates_is_the_bgk_step(orc, lattice, walls):
    p, C, u, h = _mixed_case(orc, lattice, walls, 1, 0.8, 0.8)
    a = orc.init_equilibrium(p, C, u, h)
    b = a.copy()
    orc.step(p, a, 12, h)
    orc.step(p.replace(collision=0), b, 12, h)
    assert np.abs(a - b).max() < 1e-13


@pytest.mark.parametrize("lattice", [0, 1])
def test_mrt_conserves_mass_and_momentum(orc, lattice):
    p, C, u, _ = _mixed_case(orc, lattice, 0, 1, 0.6, 1.4)
    pop = orc.init_equilibrium(p, C, u)
    F0 = orc.fields(p, pop)
    orc.step(p, pop, 40)
    F1 = orc.fields(p, pop)
    for k in ("rho", "phi", "psi"):
        assert abs(F1[k].sum() - F0[k].sum()) < 1e-12 * max(1.0, abs(F0[k]).sum())
    for a in ("ux", "uy", "uz")[: p.D]:
        j0, j1 = (F0["rho"] * F0[a]).sum(), (F1["rho"] * F1[a]).sum()
        assert abs(j1 - j0) < 1e-13 * F0["rho"].sum()
    # the collision changed something: distinct rates are not BGK
    q = p.replace(collision=0)
    b = orc.init_equilibrium(q, C, u)
    orc.step(q, b, 40)
    assert np.abs(pop - b).max() > 1e-6


def _ideal(orc, lattice, nx, ny, nz, tau_f, tau_bulk, tau_ghost):
    """An almost ideal single-phase fluid: all C1, kappa tiny (the free-energy terms are ~1e-8)."""
    return orc.Params(lattice=lattice, nx=nx, ny=ny, nz=nz, walls_y=0, kappa=(1e-8,) * 3, alpha=1.0, tau_f=tau_f,
                      tau_g=1.0, tau_k=1.0, gamma_phi=0.1, gamma_psi=0.1, collision=1, tau_bulk=tau_bulk,
                      tau_ghost=tau_ghost)


def _mode(F, key, k, axis_coord):
    return 2.0 * np.mean(F[key] * np.exp(-1j * k * axis_coord))


def _shear_rate(orc, lattice, tau_f, tau_bulk, tau_ghost, L=96, steps=(200, 800, 1400)):
    """Decay rate of u_x = U sin(k y) (2D) or sin(k z) (3D) in a periodic box."""
    if lattice == 0:
        nx, ny, nz = 4, L, 1
    else:
        nx, ny, nz = 4, 4, L
    p = _ideal(orc, lattice, nx, ny, nz, tau_f, tau_bulk, tau_ghost)
    N = nx * ny * nz
    idx = np.arange(N)
    coord = (idx // nx) % ny if lattice == 0 else idx // (nx * ny)
    k = 2 * math.pi / L
    C = np.zeros((3, N))
    C[0] = 1.0
    u = np.zeros((p.D, N))
    u[0] = 1e-4 * np.sin(k * coord)
    pop = orc.init_equilibrium(p, C, u)
    amps, done = [], 0
    for s in steps:
        orc.step(p, pop, s - done)
        done = s
        F = orc.fields(p, pop)
        amps.append(abs(_mode(F, "ux", k, coord)))
    rate = -np.polyfit(np.array(steps, float), np.log(amps), 1)[0]
    return rate, k


@pytest.mark.parametrize("lattice", [0, 1])
def test_shear_wave_decays_at_the_viscosity_of_tau_f_only(orc, lattice):
    tau_f = 0.8
    nu = (tau_f - 0.5) / 3.0
    rates = []
    for tb, tg in ((0.8, 0.8), (0.6, 1.5), (1.3, 0.55)):
        r, k = _shear_rate(orc, lattice, tau_f, tb, tg)
        rates.append(r)
        assert r == pytest.approx(nu * k * k, rel=0.005), (tb, tg)
    # the non-hydrodynamic rates leave the shear mode alone up to higher orders in k
    assert max(rates) - min(rates) < 0.002 * rates[0]
    r2, k = _shear_rate(orc, lattice, 1.1, 0.6, 1.5)
    assert r2 == pytest.approx((1.1 - 0.5) / 3.0 * k * k, rel=0.005)


def _sound_rate(orc, lattice, tau_f, tau_bulk, tau_ghost, L=40, steps=(80, 400, 720)):
    """Damping rate of a standing sound wave rho = 1 + A cos(k x): the mode energy
    |rho_k|^2 c_s^2 + |j_k|^2 decays at twice the amplitude rate."""
    if lattice == 0:
        nx, ny, nz = L, 4, 1
    else:
        nx, ny, nz = L, 4, 4
    p = _ideal(orc, lattice, nx, ny, nz, tau_f, tau_bulk, tau_ghost)
    N = nx * ny * nz
    x = np.arange(N) % nx
    k = 2 * math.pi / L
    C = np.zeros((3, N))
    C[0] = 1.0 + 1e-4 * np.cos(k * x)
    pop = orc.init_equilibrium(p, C)
    en, done = [], 0
    for s in steps:
        orc.step(p, pop, s - done)
        done = s
        F = orc.fields(p, pop)
        rk = _mode(F, "rho", k, x)
        jk = _mode({"j": F["rho"] * F["ux"]}, "j", k, x)
        en.append(abs(rk) ** 2 / 3.0 + abs(jk) ** 2)
    rate = -0.5 * np.polyfit(np.array(steps, float), np.log(en), 1)[0]
    return rate, k


@pytest.mark.parametrize("lattice", [0, 1])
def test_sound_wave_damping_follows_the_bulk_viscosity_of_tau_bulk(orc, lattice):
    D = 2 if lattice == 0 else 3
    tau_f = 0.8
    nu = (tau_f - 0.5) / 3.0
    for tb in (0.6, 1.4):
        zeta = (2.0 / D) * (tb - 0.5) / 3.0
        r, k = _sound_rate(orc, lattice, tau_f, tb, 1.2)
        assert r == pytest.approx(0.5 * k * k * ((2.0 - 2.0 / D) * nu + zeta), rel=0.03), tb


@pytest.mark.parametrize("walls", [0, 1])
def test_torch_reexpression_matches_c_oracle_mrt(orc, walls):
    """The projection form of the PyTorch reference against the C oracle's M^-1 S M (D2Q9)."""
    from oracle import torch_ref

    p, C, u, h = _mixed_case(orc, 0, walls, 1, 0.65, 1.35)
    pop = orc.init_equilibrium(p, C, u, h)
    t0 = torch.tensor(pop.reshape(3, 9, p.ny, p.nx))
    orc.step(p, pop, 20, h)
    tp = torch_ref.run(t0, None if h is None else torch.tensor(h.reshape(2, 3, p.nx)),
                       torch.tensor(p.kappa, dtype=torch.float64), p.alpha, (p.tau_f, p.tau_g, p.tau_k),
                       (p.gamma_phi, p.gamma_psi), bool(walls), 20, mrt=(p.tau_bulk, p.tau_ghost))
    assert np.abs(tp.numpy().reshape(3, 9, -1) - pop).max() < 1e-13


def test_laplace_pressure_is_independent_of_the_relaxation_rates(orc):
    """A drop of C1 in C2 relaxed with MRT (tau_bulk, tau_ghost != tau_f): p_in - p_out = gamma_12 / R
    as with BGK (Sec. V.A)."""
    kappa = (0.01, 0.015, 0.02)
    N, R = 64, 12.0
    gp, gk = inputs.mobility_to_gamma(0.2, 1.0, 1.0)
    p = orc.Params(lattice=0, nx=N, ny=N, walls_y=0, kappa=kappa, alpha=1.0, tau_f=0.9, tau_g=1.0, tau_k=1.0,
                   gamma_phi=gp, gamma_psi=gk, collision=1, tau_bulk=0.7, tau_ghost=1.2)
    x, y = np.meshgrid(np.arange(N) + 0.0, np.arange(N) + 0.0)
    d = np.hypot(x - N / 2, y - N / 2).ravel()
    C = np.zeros((3, N * N))
    C[0] = inputs.tanh_profile(d, R, 1.0)
    C[1] = 1.0 - C[0]
    pop = orc.init_equilibrium(p, C)
    orc.step(p, pop, 4000)
    F = orc.fields(p, pop)
    Cs = (F["C1"], F["C2"], F["C3"])
    pb = (F["rho"] / 3.0 + sum(kappa[m] / 2.0 * Cs[m] ** 2 * (1 - Cs[m]) * (1 - 3 * Cs[m]) for m in range(3)))
    pb = pb.reshape(N, N)
    g = analytic.surface_tension(kappa[0], kappa[1], 1.0)
    assert 0.95 <= (pb[N // 2, N // 2] - pb[0, 0]) * R / g <= 1.03

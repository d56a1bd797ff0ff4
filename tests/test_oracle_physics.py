"""Physical pins of the oracle: surface tensions from the Laplace pressure of drops (Sec. II.A,
Sec. V.A) and contact angles on a wall from the wetting parameters h_m (Sec. II.B, Sec. V.B).

These check the whole oracle step against closed forms of the paper: a mistake in the chemical
potentials, the pressure terms of the equilibrium, the stencils or the wetting ghost rows moves
the measured tension or angle away from the analytic value.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import analytic
import shapes
from paper_1511_02155_amd import inputs

KAPPA = (0.01, 0.015, 0.02)


def _bulk_pressure(F, kappa):
    """p_b = rho/3 + sum_m kappa_m/2 C_m^2 (1 - C_m)(1 - 3 C_m) (reading R2); equals P_xx where
    the gradients vanish."""
    C = (F["C1"], F["C2"], F["C3"])
    return F["rho"] / 3.0 + sum(kappa[m] / 2.0 * C[m] ** 2 * (1 - C[m]) * (1 - 3 * C[m]) for m in range(3))


def _drop_pressure_jump(orc, m, n, R, N=64, steps=4000, M=0.2):
    gp, gk = inputs.mobility_to_gamma(M, 1.0, 1.0)
    p = orc.Params(lattice=0, nx=N, ny=N, walls_y=0, kappa=KAPPA, alpha=1.0, tau_f=1.0, tau_g=1.0, tau_k=1.0,
                   gamma_phi=gp, gamma_psi=gk)
    x, y = np.meshgrid(np.arange(N) + 0.0, np.arange(N) + 0.0)
    d = np.hypot(x - N / 2, y - N / 2).ravel()
    C = np.zeros((3, N * N))
    C[m] = inputs.tanh_profile(d, R, 1.0)
    C[n] = 1.0 - C[m]
    pop = orc.init_equilibrium(p, C)
    orc.step(p, pop, steps)
    pb = _bulk_pressure(orc.fields(p, pop), KAPPA).reshape(N, N)
    return pb[N // 2, N // 2] - pb[0, 0]


@pytest.mark.parametrize("m,n", [(0, 1), (0, 2), (1, 2)])
def test_laplace_pressure_gives_pair_surface_tensions(orc, m, n):
    """A 2D drop of m in n (third component absent): p_in - p_out = gamma_mn / R with
    gamma_mn = alpha (kappa_m + kappa_n) / 6, for R = 10 and 16; and the slope of the jump
    against 1/R, which cancels curvature-independent offsets."""
    g = analytic.surface_tension(KAPPA[m], KAPPA[n], 1.0)
    R1, R2 = 10.0, 16.0
    d1 = _drop_pressure_jump(orc, m, n, R1, steps=4000)
    d2 = _drop_pressure_jump(orc, m, n, R2, steps=7000)  # the larger drop relaxes more slowly
    for R, d in ((R1, d1), (R2, d2)):
        assert 0.96 <= d * R / g <= 1.02, (R, d * R / g)
    slope = (d1 - d2) / (1.0 / R1 - 1.0 / R2)
    assert slope == pytest.approx(g, rel=0.03)


def test_drop_equilibrium_meets_the_spurious_velocity_stop_rule(orc):
    """Sec. V.A stops its lens and emulsion runs once max |v| < 1e-5 (lattice units): the equilibrium of
    a drop is at rest up to the discretisation's spurious currents.  A C1 drop (R = 16) in C2, kappa =
    0.005, on a periodic 64^2 lattice falls below that bound within 4000 steps and stays below it; the
    kinetic energy decays from the initial relaxation to the spurious level.  A pressure tensor that is
    not the one of the free energy (a wrong gradient term of the equilibrium, a stencil that is not
    isotropic) leaves a driven flow well above it."""
    N, R = 64, 16.0
    gp, gk = inputs.mobility_to_gamma(0.1, 1.0, 1.0)
    p = orc.Params(lattice=0, nx=N, ny=N, walls_y=0, kappa=(0.005, 0.005, 0.005), alpha=1.0, tau_f=1.0, tau_g=1.0,
                   tau_k=1.0, gamma_phi=gp, gamma_psi=gk)
    x, y = np.meshgrid(np.arange(N) + 0.0, np.arange(N) + 0.0)
    c1 = inputs.tanh_profile(np.hypot(x - N / 2, y - N / 2).ravel(), R, 1.0)
    C = np.stack([c1, 1.0 - c1, np.zeros_like(c1)])
    pop = orc.init_equilibrium(p, C)
    speeds = []
    for _ in range(4):
        orc.step(p, pop, 1000)
        F = orc.fields(p, pop)
        speeds.append(float(np.sqrt(F["ux"] ** 2 + F["uy"] ** 2).max()))
    extra = []
    for _ in range(2):
        orc.step(p, pop, 1000)
        F = orc.fields(p, pop)
        extra.append(float(np.sqrt(F["ux"] ** 2 + F["uy"] ** 2).max()))
    assert speeds[0] > speeds[-1]
    assert speeds[-1] < 1e-5 and max(extra) < 1e-5, (speeds, extra)
    # the drop is intact: its area stays that of the initial disc
    assert float(F["C1"].sum()) == pytest.approx(float(c1.sum()), rel=1e-10)


def _cap_angle(orc, h, theta0, steps, nx=80, ny=40, R0=16.0, M=0.2):
    kappa = (0.01, 0.01, 0.01)
    gp, gk = inputs.mobility_to_gamma(M, 1.0, 1.0)
    p = orc.Params(lattice=0, nx=nx, ny=ny, walls_y=1, kappa=kappa, alpha=1.0, tau_f=1.0, tau_g=1.0, tau_k=1.0,
                   gamma_phi=gp, gamma_psi=gk)
    hh = inputs.uniform_h(nx, (h, -h, 0.0))
    pop = orc.init_equilibrium(p, inputs.cap(nx, ny, R0, theta0), None, hh)
    orc.step(p, pop, steps, hh)
    return shapes.fit_contact_angle(orc.fields(p, pop, hh)["C1"].reshape(ny, nx), nx, ny)


@pytest.mark.parametrize("h", [0.001, -0.001])
def test_sessile_cap_holds_young_angle(orc, h):
    """A C1 cap in C2 on a wall with (h_1, h_2, h_3) = (h, -h, 0): the angle of Young's law with
    the solid tensions of eq. (solidST) (53.4 deg / 126.6 deg) is an equilibrium of the discrete
    dynamics: a cap started there keeps it within 3 deg over 10000 steps."""
    want = analytic.contact_angle(0, 1, (0.01, 0.01, 0.01), (h, -h, 0.0), 1.0)
    assert abs(_cap_angle(orc, h, want, 10000) - want) <= 3.0


@pytest.mark.parametrize("h", [0.001, -0.001])
def test_sessile_cap_relaxes_toward_young_angle(orc, h):
    """Started at 90 deg, the cap moves toward the Young angle (on the correct side) and closes
    at least 40 % of the gap within 10000 steps."""
    want = analytic.contact_angle(0, 1, (0.01, 0.01, 0.01), (h, -h, 0.0), 1.0)
    got = _cap_angle(orc, h, 90.0, 10000)
    gap0, gap = want - 90.0, want - got
    assert gap * gap0 > 0 and abs(gap) <= 0.6 * abs(gap0), (got, want)


def _mode_decay(orc, channel, tau, M=0.5, nx=16, c0=0.9, amp=1e-4, kappa=0.01):
    """Small cosine perturbation of C1 (channel 'phi': C2 = 1 - C1, C3 = 0) or of C3 (channel 'psi':
    C1 = 1 - C3, C2 = 0) about the stable bulk value c0; returns (fitted decay rate, max |C2|)."""
    gp, gk = inputs.mobility_to_gamma(M, tau, tau)
    ny = 3
    p = orc.Params(lattice=0, nx=nx, ny=ny, walls_y=0, kappa=(kappa,) * 3, alpha=1.0, tau_f=tau, tau_g=tau,
                   tau_k=tau, gamma_phi=gp, gamma_psi=gk)
    k = 2 * math.pi / nx
    x = np.tile(np.arange(nx, dtype=float), ny)
    c = c0 + amp * np.cos(k * x)
    if channel == "phi":
        C = np.stack([c, 1 - c, np.zeros_like(c)])
        name = "C1"
    else:
        C = np.stack([1 - c, np.zeros_like(c), c])
        name = "C3"
    pop = orc.init_equilibrium(p, C)
    steps = (500, 1000, 1500, 2000)
    amps, done, c2 = [amp], 0, 0.0
    for s in steps:
        orc.step(p, pop, s - done)
        done = s
        F = orc.fields(p, pop)
        d = F[name][:nx] - F[name][:nx].mean()
        amps.append(2 * abs(np.dot(d, np.cos(k * np.arange(nx)))) / nx)
        c2 = max(c2, float(np.abs(F["C2"]).max()))
    rate = -np.polyfit(np.array((0,) + steps, dtype=float), np.log(amps), 1)[0]
    return rate, c2, k


def _ch_rate(M_eff, k, c0, kappa):
    """Linearised Cahn-Hilliard decay rate M_eff * kappa * L (F''(c0) + alpha^2 L) of a cosine mode,
    with the eigenvalue L = 2 (1 - cos k) of the isotropic lattice Laplacian (reading R7)."""
    L = 2.0 * (1.0 - math.cos(k))
    return M_eff * kappa * L * ((1 - 6 * c0 + 6 * c0 ** 2) + L)


@pytest.mark.parametrize("tau", [1.0, 0.7])
def test_phi_mode_decays_at_cahn_hilliard_rate(orc, tau):
    """A binary C1/C2 perturbation evolves by the Cahn-Hilliard equation for phi (Sec. III) with
    mobility M_phi = Gamma_phi (tau_g - 1/2) (Sec. IV) = 2M (appendix A); mu_phi of the binary state
    is (kappa/2)(F'(C1) - alpha^2 lap C1) with phi = 2 C1 - 1, so the C1 mode decays at
    M kappa L (F''(c0) + L)."""
    M, c0, kappa = 0.5, 0.9, 0.01
    rate, _, k = _mode_decay(orc, "phi", tau, M=M, c0=c0, kappa=kappa)
    assert rate == pytest.approx(_ch_rate(M, k, c0, kappa), rel=0.05)


def test_psi_mode_decay_keeps_absent_component_absent(orc):
    """A C1/C3 perturbation with C2 = 0 moves phi and psi together; C2 stays zero only because
    M_phi = 2M and M_psi = 2M/3 give every component the same mobility M (appendix A, reading R10),
    and the C3 mode then decays at M kappa L (F''(c0) + L)."""
    M, c0, kappa = 0.5, 0.9, 0.01
    rate, c2, k = _mode_decay(orc, "psi", 1.0, M=M, c0=c0, kappa=kappa)
    assert rate == pytest.approx(_ch_rate(M, k, c0, kappa), rel=0.05)
    assert c2 < 0.01 * 1e-4


def _mode_phase(orc, no_advection, u0=0.02, nx=32, steps=600, c0=0.9, amp=1e-4):
    """Phase (radians) of the C1 cosine mode after `steps` in a uniform flow u0 along x."""
    gp, gk = inputs.mobility_to_gamma(0.1, 1.0, 1.0)
    ny = 3
    p = orc.Params(lattice=0, nx=nx, ny=ny, walls_y=0, kappa=(0.01,) * 3, alpha=1.0, tau_f=1.0, tau_g=1.0,
                   tau_k=1.0, gamma_phi=gp, gamma_psi=gk, no_advection=no_advection)
    k = 2 * math.pi / nx
    x = np.tile(np.arange(nx, dtype=float), ny)
    c = c0 + amp * np.cos(k * x)
    C = np.stack([c, 1 - c, np.zeros_like(c)])
    u = np.stack([np.full(nx * ny, u0), np.zeros(nx * ny)])
    pop = orc.init_equilibrium(p, C, u)
    orc.step(p, pop, steps)
    d = orc.fields(p, pop)["C1"][:nx]
    z = np.sum((d - d.mean()) * np.exp(-1j * k * np.arange(nx)))
    return float(np.angle(z)), k * u0 * steps


def test_no_advection_leaves_patterns_in_place(orc):
    """With the velocity terms of g^eq and k^eq (the advective Cahn-Hilliard equations of Sec. III) a
    C1 mode in a uniform flow u moves by u t; without them (the diffusive runs of Sec. V.C) it stays."""
    moved, expect = _mode_phase(orc, 0)
    still, _ = _mode_phase(orc, 1)
    assert -moved == pytest.approx(expect, rel=0.05)
    assert abs(still) < 0.01 * expect


def _slab_interface_length(orc, alpha):
    nx, ny = int(48 * alpha), 5
    kappa = (0.04 / alpha ** 2,) * 3
    gp, gk = inputs.mobility_to_gamma(0.2, 1.0, 1.0)
    p = orc.Params(lattice=0, nx=nx, ny=ny, walls_y=0, kappa=kappa, alpha=alpha, tau_f=1.0, tau_g=1.0, tau_k=1.0,
                   gamma_phi=gp, gamma_psi=gk)
    x = np.tile(np.arange(nx, dtype=float), ny)
    c1 = inputs.tanh_profile(np.abs(x - nx / 2.0 + 0.5), nx / 4.0, alpha)
    pop = orc.init_equilibrium(p, np.stack([c1, 1 - c1, np.zeros_like(c1)]))
    orc.step(p, pop, 4000)
    C1 = orc.fields(p, pop)["C1"]
    return 6.0 * np.sum(C1 ** 2 * (1 - C1) ** 2) / alpha, 2.0 * ny


def test_interface_measure_converges_to_flat_interface_length(orc):
    """A relaxed binary slab: the sum over nodes of C1^2 (1 - C1)^2 is alpha/6 per unit interface
    length for the tanh profile of eq. (tanh), so 6 sum / alpha -> 2 ny (two interfaces), with the
    discretisation error of the profile falling at second order in 1/alpha."""
    l1, want = _slab_interface_length(orc, 1.0)
    l2, _ = _slab_interface_length(orc, 2.0)
    e1, e2 = abs(l1 / want - 1), abs(l2 / want - 1)
    assert e1 < 0.04 and e2 < 0.01 and e2 < e1 / 3.0, (e1, e2)

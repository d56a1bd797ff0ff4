"""Pins of the N-component extension (Sec. II.E) in the PyTorch-CPU FP64 re-expression of the D2Q9 step,
which serves as the oracle of the GPU step for N > 3.

The extension: rho = sum_m C_m, phi = C1 - C2, psi_l = C_l for l >= 3, one k_l population per psi_l,
chemical potentials by the chain rule (mu_phi = (mu1 - mu2)/2, mu_psi_l = mu_l - (mu1 + mu2)/2),
pressure and gradient terms summed over all N components, every k_l with tau_k and Gamma_psi
(reading R19).  What fixes it from outside the code:
  - N = 3 is the ternary model: the re-expression equals the C oracle (also its initial state);
  - relabelling symmetries: swapping two psi components, or components 1 and 2 (phi -> -phi), together
    with their kappa, h and initial fields, permutes the run;
  - each of rho, phi and every psi_l is conserved, and a uniform state at rest is a fixed point;
  - the Laplace pressure of a drop of any pair equals gamma_mn / R with gamma_mn = alpha (kappa_m +
    kappa_n) / 6, also for two psi components (Sec. II.E: the surface tensions follow as for N = 3).
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import analytic
from paper_1511_02155_amd import inputs


def _args(kappa, h=None, walls=False, tau=(0.9, 0.8, 0.7), gamma=None):
    gp, gk = inputs.mobility_to_gamma(0.1, tau[1], tau[2]) if gamma is None else gamma
    return dict(h=None if h is None else torch.tensor(h), kappa=torch.tensor(kappa, dtype=torch.float64), alpha=1.1,
                tau=tau, gamma=(gp, gk), walls=walls)


def _random_fields(NC, ny, nx, seed):
    rng = np.random.default_rng(seed)
    w = rng.random((NC, ny, nx)) + 0.2
    return w / w.sum(0)


def _init(C, a, u=None):
    from oracle import torch_ref

    return torch_ref.equilibrium_state(torch.tensor(C), a["h"], a["kappa"], a["alpha"], a["gamma"], a["walls"],
                                       None if u is None else torch.tensor(u))


def _run(pop, a, steps):
    from oracle import torch_ref

    return torch_ref.run(pop, a["h"], a["kappa"], a["alpha"], a["tau"], a["gamma"], a["walls"], steps)


def torch_ref_concentrations(pop):
    from oracle import torch_ref

    return torch_ref.concentrations(pop).numpy()


def test_three_components_initial_state_equals_c_oracle(orc):
    nx, ny = 12, 9
    C = _random_fields(3, ny, nx, 1)
    u = 0.02 * np.random.default_rng(2).standard_normal((2, ny, nx))
    h = np.random.default_rng(3).uniform(-0.003, 0.003, (2, 3, nx))
    kappa = (0.012, 0.02, 0.016)
    a = _args(kappa, h, True)
    p = orc.Params(lattice=0, nx=nx, ny=ny, walls_y=1, kappa=kappa, alpha=a["alpha"], tau_f=0.9, tau_g=0.8,
                   tau_k=0.7, gamma_phi=a["gamma"][0], gamma_psi=a["gamma"][1])
    pop = orc.init_equilibrium(p, C.reshape(3, -1), u.reshape(2, -1), h.reshape(2, 3, -1))
    t = _init(C, a, u).numpy().reshape(3, 9, -1)
    assert np.abs(t - pop).max() < 1e-15
    orc.step(p, pop, 10, h.reshape(2, 3, -1))
    t10 = _run(_init(C, a, u), a, 10).numpy().reshape(3, 9, -1)
    assert np.abs(t10 - pop).max() < 1e-13


@pytest.mark.parametrize("NC,swap", [(4, (2, 3)), (5, (2, 4)), (5, (0, 1))])
def test_relabelling_components_permutes_the_run(NC, swap):
    """Swap components i, j (with kappa, h and the initial fields); the result is the swapped run.  For
    (0, 1) the swap is phi -> -phi."""
    nx, ny = 14, 10
    rng = np.random.default_rng(4)
    C = _random_fields(NC, ny, nx, 5)
    u = 0.02 * rng.standard_normal((2, ny, nx))
    h = rng.uniform(-0.003, 0.003, (2, NC, nx))
    kappa = list(0.01 + 0.01 * rng.random(NC))
    i, j = swap
    perm = list(range(NC))
    perm[i], perm[j] = j, i
    a = _args(kappa, h, True)
    b = _args([kappa[k] for k in perm], h[:, perm], True)
    r1 = torch_ref_concentrations(_run(_init(C, a, u), a, 30))
    r2 = torch_ref_concentrations(_run(_init(C[perm], b, u), b, 30))
    assert np.abs(r1[perm] - r2).max() < 1e-14


@pytest.mark.parametrize("NC", [4, 5])
def test_each_population_set_is_conserved(NC):
    nx, ny = 16, 12
    C = _random_fields(NC, ny, nx, 6)
    u = 0.02 * np.random.default_rng(7).standard_normal((2, ny, nx))
    kappa = [0.01 + 0.002 * m for m in range(NC)]
    a = _args(kappa)
    pop0 = _init(C, a, u)
    pop = _run(pop0, a, 60)
    s0, s1 = pop0.sum(dim=(1, 2, 3)), pop.sum(dim=(1, 2, 3))
    assert torch.abs(s1 - s0).max().item() < 1e-12 * nx * ny
    assert torch.abs(pop - pop0).max().item() > 1e-4  # the run moved


@pytest.mark.parametrize("walls", [False, True])
def test_uniform_state_at_rest_is_a_fixed_point(walls):
    NC, nx, ny = 5, 9, 7
    C = np.ones((NC, ny, nx)) * np.array([0.3, 0.25, 0.2, 0.15, 0.1]).reshape(NC, 1, 1)
    a = _args([0.01, 0.012, 0.014, 0.016, 0.018], np.zeros((2, NC, nx)) if walls else None, walls)
    pop0 = _init(C, a)
    pop = _run(pop0, a, 20)
    assert torch.abs(pop - pop0).max().item() < 1e-14  # moments re-summed each step: rounding only


@pytest.mark.parametrize("m,n", [(3, 0), (3, 2)])
def test_laplace_pressure_of_pairs_with_a_fourth_component(m, n):
    """A drop of component m in n (N = 4, the others absent at the start): p_in - p_out = gamma_mn / R.
    (3, 2) is a drop of psi_4 in psi_3."""
    from oracle import torch_ref

    NC, N, R = 4, 48, 10.0
    kappa = (0.01, 0.015, 0.02, 0.012)
    x, y = np.meshgrid(np.arange(N) + 0.0, np.arange(N) + 0.0)
    d = np.hypot(x - N / 2, y - N / 2)
    C = np.zeros((NC, N, N))
    C[m] = inputs.tanh_profile(d, R, 1.0)
    C[n] = 1.0 - C[m]
    a = _args(kappa, tau=(1.0, 1.0, 1.0), gamma=inputs.mobility_to_gamma(0.2, 1.0, 1.0))
    a["alpha"] = 1.0
    pop = _run(_init(C, a), a, 3000)
    Cf = torch_ref.concentrations(pop).numpy()
    pb = Cf.sum(0) / 3 + sum(kappa[k] / 2 * Cf[k] ** 2 * (1 - Cf[k]) * (1 - 3 * Cf[k]) for k in range(NC))
    g = analytic.surface_tension(kappa[m], kappa[n], 1.0)
    assert 0.95 <= (pb[N // 2, N // 2] - pb[0, 0]) * R / g <= 1.03


# --------------------------------------------------------------------------
# D3Q19 with N components: torch_ref.step3, the oracle of the 3D GPU step for N > 3 (N = 3 is pinned
# to the C oracle in test_oracle_torch_ref.py)
# --------------------------------------------------------------------------
def _args3(kappa, h=None, walls=False):
    return _args(kappa, h, walls)


def _init3(C, a, u=None):
    from oracle import torch_ref

    return torch_ref.equilibrium_state3(torch.tensor(C), a["h"], a["kappa"], a["alpha"], a["gamma"], a["walls"],
                                        None if u is None else torch.tensor(u))


def _run3(pop, a, steps):
    from oracle import torch_ref

    return torch_ref.run3(pop, a["h"], a["kappa"], a["alpha"], a["tau"], a["gamma"], a["walls"], steps)


@pytest.mark.parametrize("NC,swap", [(4, (2, 3)), (5, (0, 1))])
def test_d3q19_relabelling_components_permutes_the_run(NC, swap):
    nx, ny, nz = 7, 6, 5
    rng = np.random.default_rng(14)
    C = _random_fields(NC, ny * nz, nx, 15).reshape(NC, nz, ny, nx)
    u = 0.02 * rng.standard_normal((3, nz, ny, nx))
    h = rng.uniform(-0.003, 0.003, (2, NC, nz, nx))
    kappa = list(0.01 + 0.01 * rng.random(NC))
    i, j = swap
    perm = list(range(NC))
    perm[i], perm[j] = j, i
    a = _args3(kappa, h, True)
    b = _args3([kappa[k] for k in perm], h[:, perm], True)
    r1 = torch_ref_concentrations(_run3(_init3(C, a, u), a, 12))
    r2 = torch_ref_concentrations(_run3(_init3(C[perm], b, u), b, 12))
    assert np.abs(r1[perm] - r2).max() < 1e-14


@pytest.mark.parametrize("NC", [4, 5])
def test_d3q19_each_population_set_is_conserved(NC):
    nx, ny, nz = 8, 6, 5
    C = _random_fields(NC, ny * nz, nx, 16).reshape(NC, nz, ny, nx)
    u = 0.02 * np.random.default_rng(17).standard_normal((3, nz, ny, nx))
    a = _args3([0.01 + 0.002 * m for m in range(NC)])
    pop0 = _init3(C, a, u)
    pop = _run3(pop0, a, 25)
    s0, s1 = pop0.sum(dim=(1, 2, 3, 4)), pop.sum(dim=(1, 2, 3, 4))
    assert torch.abs(s1 - s0).max().item() < 1e-12 * nx * ny * nz
    assert torch.abs(pop - pop0).max().item() > 1e-4


def test_d3q19_uniform_state_at_rest_is_a_fixed_point():
    NC, nx, ny, nz = 5, 6, 5, 4
    C = np.ones((NC, nz, ny, nx)) * np.array([0.3, 0.25, 0.2, 0.15, 0.1]).reshape(NC, 1, 1, 1)
    a = _args3([0.01, 0.012, 0.014, 0.016, 0.018], np.zeros((2, NC, nz, nx)), True)
    pop0 = _init3(C, a)
    pop = _run3(pop0, a, 10)
    assert torch.abs(pop - pop0).max().item() < 1e-14

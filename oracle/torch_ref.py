"""FP64 PyTorch-CPU re-expression of the D2Q9 and D3Q19 ternary LB steps (test infrastructure).

A second, independent CPU implementation of the step of Sec. IV of
arXiv:1511.02155 (D2Q9, periodic x, periodic y or half-way walls with the
wetting ghost rows), written with whole-array torch operations so that
autograd can differentiate a run of steps with respect to the wetting
parameters h_m and the bulk coefficients kappa_m.  It serves as the
reference for the GPU adjoint; it is pinned to the C oracle (same forward
map to rounding) and to central finite differences of the C oracle.  The
D3Q19 step (step3) is a second implementation of the 3D oracle, pinned to it
on small grids.

Only the test suite and the CPU baseline of bench.py may import it.  It shares no code with the C oracle or
with the GPU library.  Readings of the paper are those of tlb_oracle.c
(R1-R9, R18); the state is the post-propagation populations [species][q][ny][nx].
"""
from __future__ import annotations

import torch

# D2Q9 velocities (order of include/tlb.h), weights and gradient weights
E = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (1, -1), (-1, 1), (-1, -1)]
OPP = [0, 2, 1, 4, 3, 8, 7, 6, 5]
W = [4.0 / 9.0] + [1.0 / 9.0] * 4 + [1.0 / 36.0] * 4


def _wab(i):
    """(w^xx, w^yy, w^xy) of direction i (reading R6)."""
    ex, ey = E[i]
    if ex == 0 and ey == 0:
        return 0.0, 0.0, 0.0
    if ex * ex + ey * ey == 1:
        return (1.0 / 9.0 if ex else -1.0 / 18.0), (1.0 / 9.0 if ey else -1.0 / 18.0), 0.0
    return -1.0 / 72.0, -1.0 / 72.0, ex * ey / 12.0


def _shift(a, dx, dy):
    """b[..., y, x] = a[..., y + dy, x + dx] with periodic wrap in both directions."""
    return torch.roll(a, shifts=(-dy, -dx), dims=(-2, -1))


def _relax_f_mrt(f, feq, tau_f, tau_bulk, tau_ghost):
    """Multiple relaxation times for f (reading R18), written as projections: with the orthogonal
    moment basis, M^-1 S M = s_ghost I + (s_shear - s_ghost) P_stress + (s_bulk - s_ghost) P_energy,
    where P_x projects onto the span of the rows of class x.  D2Q9 stress rows e_x^2 - e_y^2 and
    e_x e_y, energy row -4 + 3 |e|^2."""
    rows_stress = [[e[0] * e[0] - e[1] * e[1] for e in E], [e[0] * e[1] for e in E]]
    row_energy = [-4.0 + 3.0 * (e[0] * e[0] + e[1] * e[1]) for e in E]
    d = f - feq
    sg, sn, sb = 1.0 / tau_ghost, 1.0 / tau_f, 1.0 / tau_bulk
    out = f - sg * d
    for rows, rate in ((rows_stress, sn), ([row_energy], sb)):
        for r in rows:
            rt = torch.tensor(r, dtype=f.dtype).view(9, 1, 1)
            m = (rt * d).sum(0) / float(sum(v * v for v in r))
            out = out - (rate - sg) * rt * m
    return out


def equilibria(C, vx, vy, h, kappa, alpha, gamma, walls):
    """Equilibrium populations [NC][9][ny][nx] of concentration fields C[NC][ny][nx] (NC >= 3: rho =
    sum_m C_m, phi = C1 - C2, psi_l = C_l for l >= 3, Sec. II.E) and velocity (vx, vy), with the
    gradient terms of the fields and the wetting ghost rows h[2][NC][nx] (walls)."""
    NC, ny, nx = C.shape
    rho = C.sum(0)
    phi = C[0] - C[1]
    psis = C[2:]
    a2 = alpha * alpha
    a2k = (a2 * kappa).view(NC, 1)
    # neighbour values C_m(r + e_i), with ghost rows beyond the walls (reading R8)
    if walls:
        below = C[:, :1, :] + (h[0] / a2k).unsqueeze(1)
        above = C[:, -1:, :] + (h[1] / a2k).unsqueeze(1)
        Cg = torch.cat([below, C, above], dim=1)  # rows -1 .. ny

        def nb(dx, dy):
            return torch.roll(Cg[:, 1 + dy: 1 + dy + ny, :], shifts=-dx, dims=-1)
    else:
        def nb(dx, dy):
            return _shift(C, dx, dy)
    gx = torch.zeros_like(C)
    gy = torch.zeros_like(C)
    lap = torch.zeros_like(C)
    for i in range(1, 9):
        c = nb(*E[i])
        gx = gx + 3.0 * W[i] * E[i][0] * c
        gy = gy + 3.0 * W[i] * E[i][1] * c
        lap = lap + 6.0 * W[i] * (c - C)
    km = kappa.view(NC, 1, 1)
    mu = km * C * (1 - C) * (1 - 2 * C) - a2 * km * lap
    # chemical potentials of the transformed variables (chain rule through C_1 and C_2)
    mu_phi = 0.5 * (mu[0] - mu[1])
    mu_psi = mu[2:] - 0.5 * (mu[0] + mu[1])  # [NC-2]
    pb = rho / 3.0 + (0.5 * km * C * C * (1 - C) * (1 - 3 * C)).sum(0)
    lam = (a2 * km * C * lap).sum(0)
    Txx = (a2 * km * gx * gx).sum(0)
    Tyy = (a2 * km * gy * gy).sum(0)
    Txy = (a2 * km * gx * gy).sum(0)
    vv = vx * vx + vy * vy
    feq, geq, keq = [], [], []
    for i in range(1, 9):
        ev = E[i][0] * vx + E[i][1] * vy
        U = 3.0 * ev + 4.5 * ev * ev - 1.5 * vv
        wxx, wyy, wxy = _wab(i)
        feq.append(W[i] * (3.0 * (pb - lam) + rho * U) + 3.0 * (wxx * Txx + wyy * Tyy + wxy * Txy))
        geq.append(W[i] * (3.0 * gamma[0] * mu_phi + phi * U))
        keq.append(W[i] * (3.0 * gamma[1] * mu_psi + psis * U))  # [NC-2][ny][nx]
    feq = torch.stack([rho - sum(feq)] + feq)
    geq = torch.stack([phi - sum(geq)] + geq)
    keq = torch.stack([psis - sum(keq)] + keq, dim=1)  # [NC-2][9][ny][nx]
    return torch.cat([torch.stack([feq, geq]), keq])


def equilibrium_state(C, h, kappa, alpha, gamma, walls, u=None):
    """Initial state: the equilibria of C[NC][ny][nx] and velocity u[2][ny][nx] (None: at rest)."""
    z = torch.zeros_like(C[0])
    vx, vy = (z, z) if u is None else (u[0], u[1])
    return equilibria(C, vx, vy, h, kappa, alpha, gamma, walls)


def step(pop, h, kappa, alpha, tau, gamma, walls, mrt=None):
    """One step s_t -> s_{t+1}.  pop: [NC][9][ny][nx] for NC >= 3 components (f, g, then one k_l per
    psi_l = C_l, l >= 3; Sec. II.E); h: [2][NC][nx] (walls) or None; kappa: [NC] tensor;
    tau = (tau_f, tau_g, tau_k) (every k_l relaxes with tau_k); gamma = (Gamma_phi, Gamma_psi)
    (every k_l uses Gamma_psi); mrt = (tau_bulk, tau_ghost) for multiple relaxation times of f, or
    None for BGK."""
    NC = pop.shape[0]
    ny = pop.shape[-2]
    f = pop[0]
    ex = torch.tensor([e[0] for e in E], dtype=pop.dtype).view(9, 1, 1)
    ey = torch.tensor([e[1] for e in E], dtype=pop.dtype).view(9, 1, 1)
    rho = f.sum(0)
    vx = (f * ex).sum(0) / rho
    vy = (f * ey).sum(0) / rho
    C = concentrations(pop)
    eq = equilibria(C, vx, vy, h, kappa, alpha, gamma, walls)
    itau = torch.tensor([1.0 / tau[0], 1.0 / tau[1]] + [1.0 / tau[2]] * (NC - 2), dtype=pop.dtype).view(NC, 1, 1, 1)
    post = pop - itau * (pop - eq)
    if mrt is not None:
        post = torch.cat([_relax_f_mrt(f, eq[0], tau[0], mrt[0], mrt[1]).unsqueeze(0), post[1:]])
    # pull propagation with half-way bounce-back at the y walls
    out = []
    for i in range(9):
        dx, dy = E[i]
        pulled = _shift(post[:, i], -dx, -dy)
        if walls and dy != 0:
            row = 0 if dy == 1 else ny - 1
            rows = torch.arange(ny).view(1, ny, 1)
            pulled = torch.where(rows == row, post[:, OPP[i]], pulled)
        out.append(pulled)
    return torch.stack(out, dim=1)


def concentrations(pop):
    """C[NC][ny][nx] of a state: C1 = (rho + phi - sum psi)/2, C2 = (rho - phi - sum psi)/2, C_l = psi_l."""
    rho, phi, psis = pop[0].sum(0), pop[1].sum(0), pop[2:].sum(1)
    spsi = psis.sum(0)
    return torch.cat([torch.stack([0.5 * (rho + phi - spsi), 0.5 * (rho - phi - spsi)]), psis])


def run(pop0, h, kappa, alpha, tau, gamma, walls, nsteps, mrt=None):
    pop = pop0
    for _ in range(nsteps):
        pop = step(pop, h, kappa, alpha, tau, gamma, walls, mrt)
    return pop


def loss_and_grads(pop0, h, kappa, alpha, tau, gamma, walls, nsteps, target):
    """L = sum (C1 - C1*)^2 after nsteps from the fixed state pop0; returns (L, dL/dh, dL/dkappa)."""
    h = h.clone().detach().requires_grad_(True)
    kappa = kappa.clone().detach().requires_grad_(True)
    pop = run(pop0, h, kappa, alpha, tau, gamma, walls, nsteps)
    C1 = concentrations(pop)[0]
    L = ((C1 - target) ** 2).sum()
    L.backward()
    return L.item(), h.grad.detach(), kappa.grad.detach()


# --------------------------------------------------------------------------
# D3Q19 (Sec. IV): a whole-array re-expression of the 3D step, state [NC][19][nz][ny][nx]
# --------------------------------------------------------------------------
# velocities in the order of the weight index sets printed in Sec. IV: rest, the six axes, then the
# xy, yz and zx diagonals
E3 = ([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
      + [(a, b, 0) for a in (1, -1) for b in (1, -1)]
      + [(0, a, b) for a in (1, -1) for b in (1, -1)]
      + [(a, 0, b) for a in (1, -1) for b in (1, -1)])
OPP3 = [E3.index((-e[0], -e[1], -e[2])) for e in E3]
W3 = [1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12


def _wab3(i, a, b):
    """Gradient weight w_i^{ab} of D3Q19 direction i (reading G5: assigned by velocity class)."""
    e = E3[i]
    n2 = sum(c * c for c in e)
    if n2 == 0:
        return 0.0
    if a == b:
        if n2 == 1:
            return 5.0 / 36.0 if e[a] != 0 else -1.0 / 9.0
        return -1.0 / 72.0 if e[a] != 0 else 1.0 / 36.0
    return e[a] * e[b] / 12.0 if n2 == 2 else 0.0


def _roll3(a, dx, dy, dz):
    """b[..., z, y, x] = a[..., z + dz, y + dy, x + dx], periodic in all three directions."""
    return torch.roll(a, shifts=(-dz, -dy, -dx), dims=(-3, -2, -1))


def equilibria3(C, v, h, kappa, alpha, gamma, walls):
    """Equilibrium populations [NC][19][nz][ny][nx] of C[NC][nz][ny][nx] and v[3][nz][ny][nx], with the
    gradient terms of the fields and, with walls, the ghost planes beyond y = 0 and y = ny - 1 from
    h[2][NC][nz][nx] (reading R8)."""
    NC, nz, ny, nx = C.shape
    rho, phi, psis = C.sum(0), C[0] - C[1], C[2:]
    a2 = alpha * alpha
    if walls:
        a2k = (a2 * kappa).view(NC, 1, 1)
        below = C[:, :, :1, :] + (h[0] / a2k).unsqueeze(2)
        above = C[:, :, -1:, :] + (h[1] / a2k).unsqueeze(2)
        Cg = torch.cat([below, C, above], dim=2)

        def nb(dx, dy, dz):
            return torch.roll(Cg[:, :, 1 + dy: 1 + dy + ny, :], shifts=(-dz, -dx), dims=(1, 3))
    else:
        def nb(dx, dy, dz):
            return _roll3(C, dx, dy, dz)
    grad = [torch.zeros_like(C) for _ in range(3)]
    lap = torch.zeros_like(C)
    for i in range(1, 19):
        c = nb(*E3[i])
        for a in range(3):
            if E3[i][a]:
                grad[a] = grad[a] + 3.0 * W3[i] * E3[i][a] * c
        lap = lap + 6.0 * W3[i] * (c - C)
    km = kappa.view(NC, 1, 1, 1)
    mu = km * C * (1 - C) * (1 - 2 * C) - a2 * km * lap
    mu_phi = 0.5 * (mu[0] - mu[1])
    mu_psi = mu[2:] - 0.5 * (mu[0] + mu[1])
    pb = rho / 3.0 + (0.5 * km * C * C * (1 - C) * (1 - 3 * C)).sum(0)
    lam = (a2 * km * C * lap).sum(0)
    T = {(a, b): (a2 * km * grad[a] * grad[b]).sum(0) for a in range(3) for b in range(a, 3)}
    vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2]
    feq, geq, keq = [], [], []
    for i in range(1, 19):
        e = E3[i]
        ev = e[0] * v[0] + e[1] * v[1] + e[2] * v[2]
        U = 3.0 * ev + 4.5 * ev * ev - 1.5 * vv
        G = sum(3.0 * _wab3(i, a, b) * T[(a, b)] for (a, b) in T)
        feq.append(W3[i] * (3.0 * (pb - lam) + rho * U) + G)
        geq.append(W3[i] * (3.0 * gamma[0] * mu_phi + phi * U))
        keq.append(W3[i] * (3.0 * gamma[1] * mu_psi + psis * U))
    feq = torch.stack([rho - sum(feq)] + feq)
    geq = torch.stack([phi - sum(geq)] + geq)
    keq = torch.stack([psis - sum(keq)] + keq, dim=1)
    return torch.cat([torch.stack([feq, geq]), keq])


def equilibrium_state3(C, h, kappa, alpha, gamma, walls, u=None):
    z = torch.zeros_like(C[0])
    v = (z, z, z) if u is None else (u[0], u[1], u[2])
    return equilibria3(C, v, h, kappa, alpha, gamma, walls)


def step3(pop, h, kappa, alpha, tau, gamma, walls):
    """One D3Q19 step s_t -> s_{t+1} (BGK), pop [NC][19][nz][ny][nx]; arguments as for step()."""
    NC, ny = pop.shape[0], pop.shape[-2]
    f = pop[0]
    rho = f.sum(0)
    v = [sum(E3[i][a] * f[i] for i in range(19) if E3[i][a]) / rho for a in range(3)]
    eq = equilibria3(concentrations(pop), v, h, kappa, alpha, gamma, walls)
    itau = torch.tensor([1.0 / tau[0], 1.0 / tau[1]] + [1.0 / tau[2]] * (NC - 2),
                        dtype=pop.dtype).view(NC, 1, 1, 1, 1)
    post = pop - itau * (pop - eq)
    out = []
    for i in range(19):
        dx, dy, dz = E3[i]
        pulled = _roll3(post[:, i], -dx, -dy, -dz)
        if walls and dy != 0:
            row = 0 if dy == 1 else ny - 1
            rows = torch.arange(ny).view(1, 1, ny, 1)
            pulled = torch.where(rows == row, post[:, OPP3[i]], pulled)
        out.append(pulled)
    return torch.stack(out, dim=1)


def run3(pop0, h, kappa, alpha, tau, gamma, walls, nsteps):
    pop = pop0
    for _ in range(nsteps):
        pop = step3(pop, h, kappa, alpha, tau, gamma, walls)
    return pop

"""Seeded synthetic inputs for the ternary LB workloads.

This module only builds initial concentration fields, wetting-parameter
arrays and parameter sets.  It holds none of the lattice Boltzmann
arithmetic, so both the GPU library's callers and the CPU oracle's tests can
draw the same inputs from it.

Layouts: node index ``n = x + nx*(y + ny*z)``; concentrations ``[3][N]``;
wetting parameters ``[wall (y-, y+)][component][x + nx*z]``.

Workloads (the paper's benchmark geometries restated as synthetic inputs):

* ``nested_drop``: a C1 drop inside a C2 shell in C3 bulk, the double
  emulsion of Sec. V.A (Fig. 1), with interface profiles of eq. (tanh);
* ``spinodal``: a homogeneous mixture with uniform random fluctuations of
  amplitude ``delta`` on C1 and C2 (C3 = 1 - C1 - C2), the initial condition
  of the phase-separation runs of Sec. V.C;
* ``sessile_drop`` / ``lens``: the wall geometries of Sec. V.A/V.B.

Random numbers come from ``numpy.random.default_rng(seed)`` (PCG64) and are
generated on the host; no generator runs on the device.
"""
from __future__ import annotations

import numpy as np


def mobility_to_gamma(M: float, tau_g: float, tau_k: float):
    """Gamma_phi, Gamma_psi for a symmetric per-component mobility M.

    The appendix gives M_phi = 2 M and M_psi = 2 M / 3 for equal mobilities of
    C1, C2, C3; Sec. IV relates M_phi = Gamma_phi (tau_phi - 1/2) and
    M_psi = Gamma_psi (tau_psi - 1/2).
    """
    return 2.0 * M / (tau_g - 0.5), 2.0 * M / (3.0 * (tau_k - 0.5))


def _coords(nx, ny, nz=1):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.astype(np.float64).ravel(), y.astype(np.float64).ravel(), z.astype(np.float64).ravel()


def tanh_profile(d, R, alpha):
    """1 inside radius R, 0 outside, with the profile of eq. (tanh) (width alpha)."""
    return 0.5 * (1.0 + np.tanh((R - d) / (2.0 * alpha)))


def nested_drop(nx, ny, R_in=12.0, R_out=20.0, alpha=1.0, centre=None):
    """C1 drop of radius R_in inside a C2 shell of outer radius R_out, in C3."""
    x, y, _ = _coords(nx, ny)
    cx, cy = (nx / 2.0, ny / 2.0) if centre is None else centre
    d = np.hypot(x - cx, y - cy)
    c1 = tanh_profile(d, R_in, alpha)
    c12 = tanh_profile(d, R_out, alpha)
    C = np.stack([c1, c12 - c1, 1.0 - c12])
    return C


def spinodal(nx, ny, nz=1, mean=(1.0 / 3.0, 1.0 / 3.0), delta=0.01, seed=0):
    """Uniform noise U(-delta, delta) on C1 and C2 around ``mean``; C3 = 1 - C1 - C2."""
    rng = np.random.default_rng(seed)
    N = nx * ny * nz
    noise = rng.uniform(-delta, delta, size=(2, N))
    c1 = mean[0] + noise[0]
    c2 = mean[1] + noise[1]
    return np.stack([c1, c2, 1.0 - c1 - c2])


def sessile_drop(nx, ny, R, x0=None, alpha=1.0, top_layer=None):
    """C1 drop of radius R centred on the lower wall (centre (x0, -1/2)) in C2.

    With ``top_layer`` set, nodes with y > top_layer are C3 (tanh profile).
    """
    x, y, _ = _coords(nx, ny)
    x0 = nx / 2.0 if x0 is None else x0
    d = np.hypot(x - x0, y + 0.5)
    c1 = tanh_profile(d, R, alpha)
    if top_layer is None:
        c3 = np.zeros_like(c1)
    else:
        c3 = 0.5 * (1.0 + np.tanh((y - top_layer) / (2.0 * alpha)))
        c3 = np.minimum(c3, 1.0 - c1)
    c2 = 1.0 - c1 - c3
    return np.stack([c1, c2, c3])


def cap(nx, ny, R, theta_deg, x0=None, alpha=1.0):
    """C1 circular cap of radius R on the wall below y = 0 (half-way, at y = -1/2) meeting it at
    theta_deg (measured through C1), in C2; C3 = 0."""
    x, y, _ = _coords(nx, ny)
    cx = nx / 2.0 if x0 is None else x0
    cy = -0.5 - R * np.cos(np.radians(theta_deg))
    c1 = tanh_profile(np.hypot(x - cx, y - cy), R, alpha)
    return np.stack([c1, 1.0 - c1, np.zeros_like(c1)])


def lens(nx, ny, R, alpha=1.0, y_interface=None):
    """C1 disc of radius R at the interface between C2 (below) and C3 (above)."""
    x, y, _ = _coords(nx, ny)
    yi = ny / 2.0 if y_interface is None else y_interface
    d = np.hypot(x - nx / 2.0, y - yi)
    c1 = tanh_profile(d, R, alpha)
    upper = 0.5 * (1.0 + np.tanh((y - yi) / (2.0 * alpha)))
    c3 = (1.0 - c1) * upper
    c2 = 1.0 - c1 - c3
    return np.stack([c1, c2, c3])


def uniform_h(nx, h, nz=1, walls=2):
    """Wetting parameters [2][3][nx*nz] with the same (h1, h2, h3) everywhere."""
    arr = np.zeros((2, 3, nx * nz))
    for w in range(walls):
        for m in range(3):
            arr[w, m, :] = h[m]
    return arr


def random_h(nx, lo=-0.01, hi=0.01, nz=1, seed=0, bottom_only=True):
    """Seeded per-node wetting parameters U(lo, hi); the top wall is neutral if bottom_only."""
    rng = np.random.default_rng(seed)
    arr = np.zeros((2, 3, nx * nz))
    arr[0] = rng.uniform(lo, hi, size=(3, nx * nz))
    if not bottom_only:
        arr[1] = rng.uniform(lo, hi, size=(3, nx * nz))
    return arr


# --------------------------------------------------------------------------
# The named workloads.  Each returns a dict of plain values:
#   lattice (0 D2Q9 / 1 D3Q19), nx, ny, nz, walls_y, kappa, alpha, tau_f,
#   tau_g, tau_k, gamma_phi, gamma_psi, steps, C (callable -> [3][N]), h.
# --------------------------------------------------------------------------

def _params(lattice, nx, ny, nz, walls_y, kappa, alpha, tau, M, steps):
    gp, gk = mobility_to_gamma(M, tau, tau)
    return dict(lattice=lattice, nx=nx, ny=ny, nz=nz, walls_y=walls_y, kappa=tuple(kappa),
                alpha=alpha, tau_f=tau, tau_g=tau, tau_k=tau, gamma_phi=gp, gamma_psi=gk,
                steps=steps)


def double_emulsion_64():
    """D2Q9 64x64 periodic, nested drop R=12 in shell R=20; kappa=0.01, tau=1, M=0.1; 1000 steps."""
    w = _params(0, 64, 64, 1, 0, (0.01, 0.01, 0.01), 1.0, 1.0, 0.1, 1000)
    w["name"] = "d2q9_64x64_double_emulsion"
    w["C"] = lambda: nested_drop(64, 64, 12.0, 20.0, 1.0)
    w["h"] = None
    return w


def spinodal_2d(n=1024, steps=10000, seed=2):
    """D2Q9 n x n periodic spinodal; kappa=(0.01,0.015,0.02), tau=1, M=0.1."""
    w = _params(0, n, n, 1, 0, (0.01, 0.015, 0.02), 1.0, 1.0, 0.1, steps)
    w["name"] = f"d2q9_{n}x{n}_spinodal"
    w["C"] = lambda: spinodal(n, n, 1, seed=seed)
    w["h"] = None
    return w


def spinodal_nc(nx, ny, nc, delta=0.01, seed=0):
    """nc components: C_m = 1/nc + U(-delta, delta) for m < nc - 1, the last one closing the sum."""
    rng = np.random.default_rng(seed)
    C = 1.0 / nc + rng.uniform(-delta, delta, size=(nc - 1, nx * ny))
    return np.concatenate([C, (1.0 - C.sum(0))[None]])


def spinodal_2d_nc(n=1024, steps=10000, nc=4, seed=7):
    """D2Q9 n x n periodic spinodal of nc components (Sec. II.E); kappa_m = 0.01 + 0.005 m, tau=1, M=0.1."""
    w = _params(0, n, n, 1, 0, tuple(0.01 + 0.005 * m for m in range(nc)), 1.0, 1.0, 0.1, steps)
    w["name"] = f"d2q9_{n}x{n}_spinodal_n{nc}"
    w["C"] = lambda: spinodal_nc(n, n, nc, seed=seed)
    w["h"] = None
    return w


def spinodal_3d(n=256, steps=2000, seed=3):
    """D3Q19 n^3 periodic spinodal; kappa=0.01, tau=0.8, M=0.05."""
    w = _params(1, n, n, n, 0, (0.01, 0.01, 0.01), 1.0, 0.8, 0.05, steps)
    w["name"] = f"d3q19_{n}^3_spinodal"
    w["C"] = lambda: spinodal(n, n, n, seed=seed)
    w["h"] = None
    return w


def spinodal_3d_nc(n=256, steps=2000, nc=4, seed=8):
    """D3Q19 n^3 periodic spinodal of nc components (Sec. II.E); kappa_m = 0.01 + 0.005 m, tau=0.8, M=0.05."""
    w = _params(1, n, n, n, 0, tuple(0.01 + 0.005 * m for m in range(nc)), 1.0, 0.8, 0.05, steps)
    w["name"] = f"d3q19_{n}^3_spinodal_n{nc}"
    w["C"] = lambda: spinodal_nc(n, n * n, nc, seed=seed)
    w["h"] = None
    return w


# Domains of the 512-domain batch (seed 4) whose wetting parameters are clamped to
# |h_m| <= alpha kappa_m / 4.  The stated range h_m ~ U[-0.01, 0.01] is kept for every other
# domain; a domain would be listed only if the FP64 oracle, run for 5000 steps with the stated
# range, went non-finite or left |C_m| <= 2 (the closed-form wall concentrations of Sec. II.B
# exist only for |4 h_m / (alpha kappa_m)| <= 1, but the boundary condition is defined beyond).
# A run of every domain found none: all stay finite, with |C_m| <= 1.33 and |v| < 0.007.
BATCH_CLAMPED = ()


def batched_walls(ndom=512, lo=32, hi=256, steps=5000, seed=4, prec_kappa=(0.005, 0.03), h_range=(-0.01, 0.01),
                  clamped=None):
    """Many walled D2Q9 domains of uneven size: Lx, Ly ~ U{lo..hi}; even domains hold a
    sessile C1 drop (R = 0.3 min(Lx, Ly), centre (Lx/2, -1/2)) in C2 under a C3 layer above
    0.8 Ly, odd domains a C1 lens (R = 0.2 min) at the C2 (below) / C3 (above) interface.
    kappa_m ~ U[0.005, 0.03] and h_m ~ U[-0.01, 0.01] per domain (the same on both walls);
    only the domains listed in ``clamped`` (default ``BATCH_CLAMPED``) have |h_m| clipped to
    alpha kappa_m / 4.  tau = 1, M = 0.1, alpha = 1.  Returns a list of dicts (parameters, C, h)."""
    clamped = set(BATCH_CLAMPED if clamped is None else clamped)
    rng = np.random.default_rng(seed)
    L = rng.integers(lo, hi + 1, size=(ndom, 2))
    kap = rng.uniform(prec_kappa[0], prec_kappa[1], size=(ndom, 3))
    hh = rng.uniform(h_range[0], h_range[1], size=(ndom, 3))
    gp, gk = mobility_to_gamma(0.1, 1.0, 1.0)
    doms = []
    for d in range(ndom):
        nx, ny = int(L[d, 0]), int(L[d, 1])
        kappa = tuple(float(k) for k in kap[d])
        h = hh[d]
        if d in clamped:
            h = np.clip(h, -np.asarray(kappa) / 4.0, np.asarray(kappa) / 4.0)
        if d % 2 == 0:
            C = sessile_drop(nx, ny, 0.3 * min(nx, ny), top_layer=0.8 * ny)
        else:
            C = lens(nx, ny, 0.2 * min(nx, ny))
        doms.append(dict(lattice=0, nx=nx, ny=ny, nz=1, walls_y=1, kappa=kappa, alpha=1.0, tau_f=1.0, tau_g=1.0,
                         tau_k=1.0, gamma_phi=gp, gamma_psi=gk, steps=steps, C=C,
                         h=uniform_h(nx, tuple(float(v) for v in h))))
    return doms


def adjoint_drop_512(n=512, steps=2000, seed_h=5, seed_target=6):
    """D2Q9 n x n with walls below y = 0 and above y = n-1: per-node h_m on the lower wall
    ~ U[-0.01, 0.01] (3 x n values, seeded), neutral upper wall; a C1 drop of radius 60
    centred on the lower wall at x = n/2 in C2; the loss target is the same profile with
    centre x ~ U[n/2 - 32, n/2 + 32] and radius ~ U[50, 70] (seeded).  kappa = 0.01,
    alpha = 1, tau = 1, M = 0.1."""
    gp, gk = mobility_to_gamma(0.1, 1.0, 1.0)
    w = dict(lattice=0, nx=n, ny=n, nz=1, walls_y=1, kappa=(0.01, 0.01, 0.01), alpha=1.0, tau_f=1.0, tau_g=1.0,
             tau_k=1.0, gamma_phi=gp, gamma_psi=gk, steps=steps, name=f"d2q9_{n}x{n}_wall_drop_adjoint")
    w["h"] = random_h(n, -0.01, 0.01, seed=seed_h, bottom_only=True)
    w["C"] = sessile_drop(n, n, 60.0, x0=n / 2.0)
    rng = np.random.default_rng(seed_target)
    xc = rng.uniform(n / 2.0 - 32.0, n / 2.0 + 32.0)
    R = rng.uniform(50.0, 70.0)
    w["target"] = sessile_drop(n, n, R, x0=xc)[0]
    return w

"""Closed forms of the paper used as pins (test-side helpers).

Each function restates one result of Sec. II of arXiv:1511.02155; the tests
compare the oracle's discrete dynamics against them.
"""
from __future__ import annotations

import math


def surface_tension(km, kn, alpha):
    """gamma_mn = alpha (kappa_m + kappa_n) / 6 (Sec. II.A, eq. SurfTens)."""
    return alpha * (km + kn) / 6.0


def wall_value_max(kappa, h, alpha):
    """C_m at the wall when m is the majority phase (Sec. II.B)."""
    return 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * h / (alpha * kappa)))


def wall_value_min(kappa, h, alpha):
    """C_n at the wall when n is a minority phase (Sec. II.B)."""
    return 0.5 * (1.0 - math.sqrt(1.0 - 4.0 * h / (alpha * kappa)))


def solid_tension(m, kappa, h, alpha):
    """gamma_sm = I_m + sum_{n != m} J_n (Sec. II.B, eq. solidST)."""
    km, hm = kappa[m], h[m]
    cmax = wall_value_max(km, hm, alpha)
    I = -hm * cmax + alpha / 12.0 * (km + math.sqrt(1.0 + 4.0 * hm / (alpha * km)) * (2.0 * hm / alpha - km))
    J = 0.0
    for n in range(len(kappa)):
        if n == m:
            continue
        kn, hn = kappa[n], h[n]
        cmin = wall_value_min(kn, hn, alpha)
        J += -hn * cmin + alpha / 12.0 * (kn - math.sqrt(1.0 - 4.0 * hn / (alpha * kn)) * (2.0 * hn / alpha + kn))
    return I + J


def contact_angle(m, n, kappa, h, alpha):
    """theta_mn (degrees, measured through m) from Young's law (eq. contact angle)."""
    gmn = surface_tension(kappa[m], kappa[n], alpha)
    c = (solid_tension(n, kappa, h, alpha) - solid_tension(m, kappa, h, alpha)) / gmn
    return math.degrees(math.acos(max(-1.0, min(1.0, c))))


def bulk_free_energy_aux(rho, phi, psi, kappa):
    """Bulk part of the free energy density in rho, phi, psi (eq. functional_newvar)."""
    k1, k2, k3 = kappa
    return (k1 / 32.0 * (rho + phi - psi) ** 2 * (2.0 + psi - rho - phi) ** 2
            + k2 / 32.0 * (rho - phi - psi) ** 2 * (2.0 + psi - rho + phi) ** 2
            + k3 / 2.0 * psi ** 2 * (1.0 - psi) ** 2)


def mu_phi_printed(rho, phi, psi, lap_rho, lap_phi, lap_psi, kappa, alpha):
    """mu_phi exactly as printed in Sec. III."""
    k1, k2, _ = kappa
    a = rho + phi - psi
    b = rho - phi - psi
    return (k1 / 8.0 * a * (a - 2.0) * (a - 1.0) - k2 / 8.0 * b * (b - 2.0) * (b - 1.0)
            + alpha ** 2 / 4.0 * ((k2 - k1) * (lap_rho - lap_psi) - (k1 + k2) * lap_phi))


def mu_psi_printed(rho, phi, psi, lap_rho, lap_phi, lap_psi, kappa, alpha):
    """mu_psi exactly as printed in Sec. III."""
    k1, k2, k3 = kappa
    a = rho + phi - psi
    b = rho - phi - psi
    return (-k1 / 8.0 * a * (a - 2.0) * (a - 1.0) - k2 / 8.0 * b * (b - 2.0) * (b - 1.0)
            + k3 * psi * (psi - 1.0) * (2.0 * psi - 1.0)
            + alpha ** 2 / 4.0 * ((k1 + k2) * lap_rho - (k2 - k1) * lap_phi - (k2 + k1 + 4.0 * k3) * lap_psi))


def bulk_pressure_printed(rho, phi, psi, kappa):
    """p_b exactly as printed in Sec. III (the polynomial form)."""
    k1, k2, k3 = kappa
    r, f, s = rho, phi, psi
    A = (3 / 32 * r ** 4 + 3 / 32 * f ** 4 + 9 / 16 * r ** 2 * f ** 2 + 9 / 16 * r ** 2 * s ** 2
         + 9 / 16 * f ** 2 * s ** 2 - 3 / 8 * r ** 3 * s - 3 / 8 * r * s ** 3 + 3 / 4 * r ** 2 * s
         - 3 / 4 * r * f ** 2 - 3 / 4 * r * s ** 2 + 3 / 4 * f ** 2 * s - 1 / 4 * r ** 3 + 1 / 8 * r ** 2
         + 1 / 8 * f ** 2 - 1 / 4 * r * s - 9 / 8 * r * f ** 2 * s)
    B = (3 / 8 * r ** 3 * f + 3 / 8 * r * f ** 3 - 3 / 8 * f ** 3 * s - 3 / 8 * f * s ** 3 - 1 / 4 * f ** 3
         - 3 / 4 * r ** 2 * f - 3 / 4 * f * s ** 2 + 1 / 4 * r * f - 1 / 4 * f * s + 9 / 8 * r * f * s ** 2
         - 9 / 8 * r ** 2 * f * s + 3 / 2 * r * f * s)
    return (r / 3.0 + (k1 + k2) * A + (k1 - k2) * B + 0.25 * (k1 + k2 - 8 * k3) * s ** 3
            + (k1 + k2 + 16 * k3) * (3 / 32 * s ** 4 + 1 / 8 * s ** 2))


def mixing_coefficients(kappa):
    """kappa_ab of the pressure tensor in Sec. III, as a 3x3 matrix over (rho, phi, psi)."""
    k1, k2, k3 = kappa
    krr = kpp = (k1 + k2) / 4.0
    kss = (k1 + k2 + 4.0 * k3) / 4.0
    krp = (k1 - k2) / 4.0
    kps = -krp
    krs = -(k1 + k2) / 4.0
    return [[krr, krp, krs], [krp, kpp, kps], [krs, kps, kss]]

"""Contact angles <-> wetting parameters (host helpers of libtlb, Sec. II.B and II.D).

The helpers are checked against Young's law with the solid tensions of eq. (solidST) computed
independently in tests/analytic.py, against the Girifalco-Good relation, and by round trips.  The
inversion formula as printed in Sec. II.D is shown to disagree (sign and a factor alpha), which is
why the helpers do not use it.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import analytic

tlb = pytest.importorskip("paper_1511_02155_amd.tlb")

KAPPAS = [(0.01, 0.01, 0.01), (0.01, 0.015, 0.02), (0.03, 0.005, 0.012)]


def _random_h(kappa, alpha, rng):
    return tuple(float(rng.uniform(-0.24, 0.24) * alpha * k) for k in kappa)


@pytest.mark.parametrize("kappa", KAPPAS)
@pytest.mark.parametrize("alpha", [1.0, 1.7])
def test_contact_angles_match_young_with_solid_tensions(kappa, alpha):
    rng = np.random.default_rng(11)
    for _ in range(20):
        h = _random_h(kappa, alpha, rng)
        th = tlb.contact_angles(kappa, alpha, h)
        for j, (m, n) in enumerate(((0, 1), (1, 2), (2, 0))):
            assert th[j] == pytest.approx(analytic.contact_angle(m, n, kappa, h, alpha), abs=1e-9)


def _printed_invert_ca(m, n, kappa, h, alpha):
    """cos(theta_mn) exactly as printed in Sec. II.D (eq. invertCA)."""
    km, kn, hm, hn = kappa[m], kappa[n], h[m], h[n]
    tn = ((alpha * kn + 4 * hn) ** 1.5 - (alpha * kn - 4 * hn) ** 1.5) / (2 * (km + kn) * math.sqrt(alpha * kn))
    tm = ((alpha * km + 4 * hm) ** 1.5 - (alpha * km - 4 * hm) ** 1.5) / (2 * (km + kn) * math.sqrt(alpha * km))
    return tn - tm


def test_printed_inversion_has_opposite_sign_and_extra_alpha():
    """Reading of Sec. II.D: Young's law with eq. (solidST) gives cos(theta_mn) = -(printed) / alpha."""
    kappa, alpha = (0.01, 0.015, 0.02), 1.7
    h = (0.002, -0.003, 0.001)
    for (m, n) in ((0, 1), (1, 2), (2, 0)):
        young = math.cos(math.radians(analytic.contact_angle(m, n, kappa, h, alpha)))
        printed = _printed_invert_ca(m, n, kappa, h, alpha)
        assert young == pytest.approx(-printed / alpha, rel=1e-12)
        assert abs(young - printed) > 0.05


@pytest.mark.parametrize("kappa", KAPPAS)
def test_girifalco_good_relation(kappa):
    """Summing Young's law over the three pairs (Sec. II.D); samples where a pair wets or dewets
    completely (angle clamped to 0 or 180 degrees) are skipped."""
    alpha = 1.0
    rng = np.random.default_rng(12)
    done = 0
    while done < 10:
        th = tlb.contact_angles(kappa, alpha, tuple(0.3 * v for v in _random_h(kappa, alpha, rng)))
        if min(th) <= 0.0 or max(th) >= 180.0:
            continue
        done += 1
        g = [analytic.surface_tension(kappa[m], kappa[n], alpha) for m, n in ((0, 1), (1, 2), (2, 0))]
        assert sum(gi * math.cos(math.radians(t)) for gi, t in zip(g, th)) == pytest.approx(0.0, abs=1e-15)


@pytest.mark.parametrize("kappa", KAPPAS)
def test_angles_to_h_round_trip_with_redundancy(kappa):
    alpha = 1.0
    done = 0
    for t12 in (30.0, 60.0, 90.0, 120.0, 150.0):
        for t23 in (45.0, 90.0, 135.0):
            try:
                h = tlb.wetting_from_angles(kappa, alpha, t12, t23)
            except tlb.TLBError:
                continue  # outside the attainable range for these kappa
            done += 1
            assert sum(hm / km for hm, km in zip(h, kappa)) == pytest.approx(0.0, abs=1e-12)
            th = tlb.contact_angles(kappa, alpha, h)
            assert th[0] == pytest.approx(t12, abs=1e-7) and th[1] == pytest.approx(t23, abs=1e-7)
    assert done >= 6


def test_unreachable_angles_and_invalid_input_are_rejected():
    kappa = (0.01, 0.01, 0.01)
    with pytest.raises(tlb.TLBError):
        tlb.wetting_from_angles(kappa, 1.0, 0.0, 0.0)  # needs Phi_1 - Phi_3 beyond the attainable range
    with pytest.raises(tlb.TLBError):
        tlb.contact_angles(kappa, 1.0, (0.01, 0.0, 0.0))  # |4h/(alpha kappa)| > 1
    with pytest.raises(tlb.TLBError):
        tlb.contact_angles((0.01, -0.01, 0.01), 1.0, (0.0, 0.0, 0.0))

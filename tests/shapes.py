"""Shape measurements on concentration fields (test-side helpers)."""
from __future__ import annotations

import math

import numpy as np


def fit_contact_angle(c1, nx, ny, skip_rows=3):
    """Contact angle (degrees, measured through C1) of the circle fitted (algebraic least squares) to
    the C1 = 1/2 contour above the first `skip_rows` rows; the wall is the half-way plane y = -1/2."""
    px, py = [], []
    for y in range(skip_rows, ny):
        row = c1[y]
        for x in range(nx - 1):
            if (row[x] - 0.5) * (row[x + 1] - 0.5) < 0:
                px.append(x + (0.5 - row[x]) / (row[x + 1] - row[x]))
                py.append(float(y))
    for x in range(nx):
        col = c1[:, x]
        for y in range(skip_rows, ny - 1):
            if (col[y] - 0.5) * (col[y + 1] - 0.5) < 0:
                px.append(float(x))
                py.append(y + (0.5 - col[y]) / (col[y + 1] - col[y]))
    px, py = np.array(px), np.array(py)
    A = np.stack([px, py, np.ones_like(px)], 1)
    c, *_ = np.linalg.lstsq(A, px ** 2 + py ** 2, rcond=None)
    xc, yc = c[0] / 2, c[1] / 2
    R = math.sqrt(c[2] + xc ** 2 + yc ** 2)
    return math.degrees(math.acos(max(-1.0, min(1.0, (-0.5 - yc) / R))))


def _crossings(f, ymin, ymax):
    """Points where the field f[ny][nx] changes sign, along rows and columns, with ymin < y < ymax
    (linear interpolation between nodes)."""
    ny, nx = f.shape
    px, py = [], []
    for y in range(ny):
        if not (ymin < y < ymax):
            continue
        row = f[y]
        for x in range(nx - 1):
            if row[x] * row[x + 1] < 0 or (row[x] == 0 and row[x + 1] != 0):
                px.append(x + row[x] / (row[x] - row[x + 1]))
                py.append(float(y))
    for x in range(nx):
        col = f[:, x]
        for y in range(ny - 1):
            if col[y] * col[y + 1] < 0 or (col[y] == 0 and col[y + 1] != 0):
                yy = y + col[y] / (col[y] - col[y + 1])
                if ymin < yy < ymax:
                    px.append(float(x))
                    py.append(yy)
    return np.array(px), np.array(py)


def _fit_circle(px, py):
    A = np.stack([px, py, np.ones_like(px)], 1)
    c, *_ = np.linalg.lstsq(A, px ** 2 + py ** 2, rcond=None)
    xc, yc = c[0] / 2, c[1] / 2
    return xc, yc, math.sqrt(c[2] + xc ** 2 + yc ** 2)


def lens_angles(C1, C2, C3, band=4.0):
    """Neumann angles (theta_1, theta_2, theta_3) in degrees of a C1 lens between C2 (below) and C3
    (above), from fields [ny][nx] with the lens near x = nx/2: the C2/C3 interface height y_f is the
    C2 = C3 crossing averaged over the columns x = 0 and x = nx - 1 (far from the lens); circles are fitted
    to the C1 = C3 contour above y_f + band and to the C1 = C2 contour below y_f - band.  A cap of a
    circle with centre height y_c and radius R on the line y = y_f meets it at alpha = arccos(d / R),
    d the signed distance of the centre from the line towards the cap's outside; the lens angle is
    theta_1 = alpha_up + alpha_down, and theta_3 = 180 - alpha_up, theta_2 = 180 - alpha_down."""
    ny, nx = C1.shape
    ys = []
    for x in (0, nx - 1):
        d = C2[:, x] - C3[:, x]
        for y in range(ny - 1):
            if d[y] * d[y + 1] < 0 or (d[y] == 0 and d[y + 1] != 0):
                ys.append(y + d[y] / (d[y] - d[y + 1]))
    yf = float(np.mean(ys))
    ux, uy = _crossings(C1 - C3, yf + band, ny)
    lx, ly = _crossings(C1 - C2, -1, yf - band)
    _, yc_u, R_u = _fit_circle(ux, uy)
    _, yc_l, R_l = _fit_circle(lx, ly)
    a_up = math.degrees(math.acos(max(-1.0, min(1.0, (yf - yc_u) / R_u))))
    a_dn = math.degrees(math.acos(max(-1.0, min(1.0, (yc_l - yf) / R_l))))
    return a_up + a_dn, 180.0 - a_dn, 180.0 - a_up


def neumann_angles(g12, g13, g23):
    """Angles (theta_1, theta_2, theta_3) in degrees inside phases 1, 2, 3 at a triple junction whose
    tensions balance (the Neumann triangle): theta_1 is opposite g23 and so on."""
    t1 = math.degrees(math.acos((g23 ** 2 - g12 ** 2 - g13 ** 2) / (2 * g12 * g13)))
    t2 = math.degrees(math.acos((g13 ** 2 - g12 ** 2 - g23 ** 2) / (2 * g12 * g23)))
    return t1, t2, 360.0 - t1 - t2

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

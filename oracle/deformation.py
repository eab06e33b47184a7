"""Deformation factor D = (L - H)/(L + H) of Eq. (63), from a phase field.

TEST INFRASTRUCTURE ONLY (part of the oracle; see ``oracle/__init__.py``).

The paper defines D through the droplet length L along the applied field
(here the y axis, between the electrodes) and the length H across it, but not
how L and H are measured on a lattice.  This reading: take the phi-weighted
centroid (xbar, ybar); L is the distance between the two phi = 1/2 crossings
on the vertical line x = xbar, H the distance between the crossings on the
horizontal line y = ybar.  Along each line the profile is interpolated
linearly between the two neighbouring lattice lines, and each crossing is
located by linear interpolation between the two nodes that bracket 1/2,
walking outwards from the centroid.
"""
from __future__ import annotations

import math

import numpy as np


def _crossings(profile: np.ndarray, start: float):
    """Positions where ``profile`` falls through 1/2 walking down and up from
    index ``start``; returns (low, high) in lattice coordinates."""
    n = profile.shape[0]
    i0 = min(max(int(math.floor(start)), 0), n - 1)
    if profile[i0] < 0.5:
        raise ValueError("centroid is not inside the droplet")
    hi = None
    for i in range(i0, n - 1):
        a, b = profile[i], profile[i + 1]
        if a >= 0.5 > b:
            hi = i + (a - 0.5) / (a - b)
            break
    lo = None
    for i in range(i0, 0, -1):
        a, b = profile[i], profile[i - 1]
        if a >= 0.5 > b:
            lo = i - (a - 0.5) / (a - b)
            break
    if hi is None or lo is None:
        raise ValueError("droplet touches the domain edge")
    return lo, hi


def deformation(phi: np.ndarray):
    """Return (D, L, H) for a phase field phi[ny][nx] (phi = 1 inside)."""
    phi = np.asarray(phi, dtype=np.float64)
    ny, nx = phi.shape
    tot = phi.sum()
    ys, xs = np.mgrid[0:ny, 0:nx]
    xb = float((phi * xs).sum() / tot)
    yb = float((phi * ys).sum() / tot)
    # vertical line through xbar: blend columns floor(xbar) and floor(xbar)+1
    j = int(math.floor(xb))
    t = xb - j
    col = (1.0 - t) * phi[:, j % nx] + t * phi[:, (j + 1) % nx]
    lo, hi = _crossings(col, yb)
    L = hi - lo
    i = int(math.floor(yb))
    s = yb - i
    row = (1.0 - s) * phi[i, :] + s * phi[min(i + 1, ny - 1), :]
    lo, hi = _crossings(row, xb)
    H = hi - lo
    return (L - H) / (L + H), L, H

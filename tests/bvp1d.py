"""Independent steady 1-D solve of the heterocharge-layer problem of Sec. 5.1.

Used only as a pin for the CPU oracle; it shares nothing with it.  The steady
Nernst-Planck-Poisson system between two permeable electrodes (Sec. 2.2-2.3,
flow at rest), in lattice units, on the gap y in [-1/2, ny - 1/2]:

    d/dy ( mu+ c+ E - D+ c+' ) = R
    d/dy (-mu- c- E - D- c-' ) = R
    eps psi'' = -q (c+ - c-),   E = -psi'
    R = delta (c0^2 (1 + 2 gamma |E|) - c+ c-),  delta = q (mu+ + mu-)/eps

with the electrode conditions of Sec. 5.1: anode (y = -1/2) psi = dpsi, c+ = 0,
c-' = 0; cathode (y = ny - 1/2) psi = 0, c- = 0, c+' = 0.  It is written as a
first-order system in (c+, J+, c-, J-, psi, E) with the ion fluxes J and solved
with scipy's collocation BVP solver by continuation in the reaction strength.
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import solve_bvp


def solve(ny, dpsi, mu_p, mu_m, D_p, D_m, eps, q, c0, gamma, nodes=2001, tol=1e-9):
    a, b = -0.5, ny - 0.5
    y = np.linspace(a, b, nodes)
    delta = q * (mu_p + mu_m) / eps

    def make(scale):
        def rhs(y, s):
            cp, Jp, cm, Jm, psi, E = s
            R = scale * delta * (c0 * c0 * (1 + 2 * gamma * np.abs(E)) - cp * cm)
            return np.vstack([(mu_p * cp * E - Jp) / D_p, R,
                              (-mu_m * cm * E - Jm) / D_m, R,
                              -E, q * (cp - cm) / eps])

        def bc(sa, sb):
            return np.array([sa[0],                              # c+ = 0 at the anode
                             sa[3] + mu_m * sa[2] * sa[5],       # c-' = 0 at the anode
                             sa[4] - dpsi,                       # psi = dpsi
                             sb[2],                              # c- = 0 at the cathode
                             sb[1] - mu_p * sb[0] * sb[5],       # c+' = 0 at the cathode
                             sb[4]])                             # psi = 0
        return rhs, bc

    E0 = dpsi / (b - a)
    guess = np.vstack([c0 * (y - a) / (b - a), np.zeros_like(y),
                       c0 * (b - y) / (b - a), np.zeros_like(y),
                       dpsi * (b - y) / (b - a), np.full_like(y, E0)])
    sol = None
    for scale in (1e-3, 1e-2, 0.1, 0.3, 1.0):
        rhs, bc = make(scale)
        sol = solve_bvp(rhs, bc, y, guess, tol=tol, max_nodes=200000)
        if not sol.success:
            raise RuntimeError("BVP did not converge: %s" % sol.message)
        y = sol.x
        guess = sol.y
    return sol

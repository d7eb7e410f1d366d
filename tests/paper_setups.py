"""Inputs written from the paper's own setup formulas, for oracle pins.

Thermal convection (Section 5.2): neutrally stratified fluids with potential
temperature perturbations.  With c_p = 1/(gamma-1), theta_0 = 300 and the
perturbation dtheta of each domain:
    Psi = 1 + g z / (c_p (1 + dtheta/theta_0)),
    T   = (1 + dtheta/theta_0) Psi,
    p   = Psi^(gamma/(gamma-1)) / gamma,
    rho = theta_0 / (theta_0 + dtheta) Psi^(1/(gamma-1)),
at rest.  Values at cell centres.
"""
from __future__ import annotations

import numpy as np

G_PAPER = -0.008140864714
THETA0 = 300.0


def cosine_bubble(amp, radius, xc, zc):
    def f(x, z):
        r = np.sqrt((x - xc) ** 2 + (z - zc) ** 2)
        return np.where(r <= radius, amp * (1.0 + np.cos(np.pi * r)), 0.0)
    return f


def thermal_convection_domain(nx, nz, x0, x1, z0, z1, dtheta, gamma=1.4, g=G_PAPER):
    dx = (x1 - x0) / nx
    dz = (z1 - z0) / nz
    x = x0 + (np.arange(nx) + 0.5) * dx
    z = z0 + (np.arange(nz) + 0.5) * dz
    X, Z = np.meshgrid(x, z)
    dth = dtheta(X, Z) if dtheta is not None else np.zeros_like(X)
    cp = 1.0 / (gamma - 1.0)
    psi = 1.0 + g * Z / (cp * (1.0 + dth / THETA0))
    p = psi ** (gamma / (gamma - 1.0)) / gamma
    rho = THETA0 / (THETA0 + dth) * psi ** (1.0 / (gamma - 1.0))
    q = np.zeros((4, nz, nx))
    q[0] = rho
    q[3] = p / (gamma - 1.0)
    return q, dx, dz


def table5_setup():
    """Omega_1 = (-5,5)x(-5,0), 100x100; Omega_2 = (-5,5)x(0,5), 100x200;
    dtheta_1 = 0.25 (1 + cos(pi r_1)) for r_1 <= 2.5 around (0, -2.5)."""
    q1, dx, dz1 = thermal_convection_domain(100, 100, -5, 5, -5, 0,
                                            cosine_bubble(0.25, 2.5, 0.0, -2.5))
    q2, _, dz2 = thermal_convection_domain(100, 200, -5, 5, 0, 5, None)
    return q1, q2, dx, dz1, dz2


def table6_setup():
    """Caption mesh of Table 6: Omega_1 = (-5,5)x(-7,0), 100x140;
    Omega_2 = (-5,5)x(0,3), 100x240; dtheta_1 = 1.25 (1 + cos(pi r_1)) for
    r_1 <= 2.5 around (0, -2.5); dtheta_2 = -7.5 (1 + cos(pi r_2)) for
    r_2 <= 1 around (0, 1.5)."""
    q1, dx, dz1 = thermal_convection_domain(100, 140, -5, 5, -7, 0,
                                            cosine_bubble(1.25, 2.5, 0.0, -2.5))
    q2, _, dz2 = thermal_convection_domain(100, 240, -5, 5, 0, 3,
                                           cosine_bubble(-7.5, 1.0, 0.0, 1.5))
    return q1, q2, dx, dz1, dz2

"""Unsplit z-marching of the semi-discrete NLSE (FP64, complex128).

Test infrastructure: see the package docstring for who may use it.

The paper integrates the whole right-hand side of the semi-discrete equation
(Eq. 10 with the operators of Eqs. 11-14) with a Runge-Kutta method, rather
than splitting it into a linear propagator and a Kerr step.  Written as
``dPsi/dz = F(Psi)``, with the sign reading of ``oracle.dec``, the right-hand
side is

    F(Psi) = -i H_lin Psi + i gamma (M |Psi|^2) * Psi - w * Psi,

``H_lin = p1 L + beta4 L^2 - diag(v)``, ``M`` the nonlinear averaging matrix
(Eq. 14, or the lumped diagonal) and ``w >= 0`` the absorber.  This module
takes the classical fourth-order Runge-Kutta method on F at a fixed step: the
Kerr term is evaluated inside every stage (the paper's own scheme is adaptive;
the fixed step is what the workloads specify).
"""
from __future__ import annotations

import numpy as np

__all__ = ["rhs", "rk4_step", "propagate_rk4"]


def rhs(psi: np.ndarray, ops, gamma: float) -> np.ndarray:
    """F(Psi) = -i H_lin Psi + i gamma (M |Psi|^2) Psi - w Psi."""
    theta = ops.M @ (np.abs(psi) ** 2)
    return -1j * ops.apply_H(psi) + 1j * gamma * theta * psi - ops.w * psi


def rk4_step(psi: np.ndarray, h: float, gamma: float, ops) -> np.ndarray:
    """One classical fourth-order Runge-Kutta step of dPsi/dz = F(Psi)."""
    k1 = rhs(psi, ops, gamma)
    k2 = rhs(psi + 0.5 * h * k1, ops, gamma)
    k3 = rhs(psi + 0.5 * h * k2, ops, gamma)
    k4 = rhs(psi + h * k3, ops, gamma)
    return psi + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def propagate_rk4(psi0, ops, dz: float, n_steps: int, gamma: float) -> np.ndarray:
    """March ``n_steps`` unsplit RK4 steps from ``psi0``."""
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    for _ in range(n_steps):
        psi = rk4_step(psi, dz, gamma, ops)
    return psi

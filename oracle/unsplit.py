"""Unsplit z-marching of the semi-discrete NLSE (FP64, complex128).

Test infrastructure: see the package docstring for who may use it.

The paper integrates the whole right-hand side of the semi-discrete equation
(Eq. 10 with the operators of Eqs. 11-14) with a Runge-Kutta method, rather
than splitting it into a linear propagator and a Kerr step.  Written as
``dPsi/dz = F(Psi)``, with the sign reading of ``oracle.dec``, the right-hand
side is

    F(Psi) = -i H_lin Psi + i gamma (M N(|Psi|^2)) * Psi - w * Psi,

``H_lin = sum_n p_n L^n - diag(v)``, ``N`` the Kerr response (``N(I) = I``
unless another is chosen), ``M`` the nonlinear averaging matrix
(Eq. 14, or the lumped diagonal) and ``w >= 0`` the absorber.  This module
takes the classical fourth-order Runge-Kutta method on F at a fixed step (the
Kerr term evaluated inside every stage; the fixed step is what the workloads
specify) and the paper's own choice, the adaptive embedded Dormand-Prince 5(4)
pair.
"""
from __future__ import annotations

import numpy as np

__all__ = ["rhs", "rk4_step", "propagate_rk4", "dp54_step", "error_norm", "propagate_dp54"]


def rhs(psi: np.ndarray, ops, gamma: float) -> np.ndarray:
    """F(Psi) = -i H_lin Psi + i gamma (M N(|Psi|^2)) Psi - w Psi."""
    theta = ops.M @ ops.N(np.abs(psi) ** 2)
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


# ---- adaptive Dormand-Prince 5(4) ----
# The paper's integrator is an adaptive embedded Runge-Kutta pair of orders
# 5 and 4 (Dormand and Prince; it is the pair behind SciPy's RK45, which the
# paper names).  Coefficients of the published tableau:
DP_C = (0.0, 1 / 5, 3 / 10, 4 / 5, 8 / 9, 1.0, 1.0)
DP_A = (
    (),
    (1 / 5,),
    (3 / 40, 9 / 40),
    (44 / 45, -56 / 15, 32 / 9),
    (19372 / 6561, -25360 / 2187, 64448 / 6561, -212 / 729),
    (9017 / 3168, -355 / 33, 46732 / 5247, 49 / 176, -5103 / 18656),
    (35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84),
)
DP_B5 = (35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84, 0.0)
DP_B4 = (5179 / 57600, 0.0, 7571 / 16695, 393 / 640, -92097 / 339200, 187 / 2100, 1 / 40)


def dp54_step(psi: np.ndarray, h: float, gamma: float, ops):
    """One Dormand-Prince step: the fifth-order solution and the difference
    between the fifth- and fourth-order solutions (the local error estimate)."""
    k = []
    for s in range(7):
        y = psi + h * sum(a * kj for a, kj in zip(DP_A[s], k)) if s else psi
        k.append(rhs(y, ops, gamma))
    y5 = psi + h * sum(b * kj for b, kj in zip(DP_B5, k))
    err = h * sum((b5 - b4) * kj for b5, b4, kj in zip(DP_B5, DP_B4, k))
    return y5, err


def error_norm(err: np.ndarray, y0: np.ndarray, y1: np.ndarray, rtol: float, atol: float) -> float:
    """Root-mean-square over vertices of |err_p| / (atol + rtol max(|y0_p|, |y1_p|))."""
    sc = atol + rtol * np.maximum(np.abs(y0), np.abs(y1))
    return float(np.sqrt(np.mean((np.abs(err) / sc) ** 2)))


def propagate_dp54(psi0, ops, z_end: float, h0: float, gamma: float, rtol: float = 1e-9, atol: float = 1e-11,
                   max_attempts: int = 100000, facmax: float = 10.0):
    """Adaptive Dormand-Prince 5(4) from z = 0 to z_end, first trial step h0
    (tolerances default to the paper's rtol = 1e-9, atol = 1e-11).

    Step-size control (the standard rule of Hairer, Norsett and Wanner,
    Solving ODEs I, section II.4): a step is accepted when the error norm is
    below 1; the next trial step is h * min(facmax, max(0.2, 0.9 err^{-1/5})),
    where facmax drops to 1 for the step that follows a rejection, and a trial
    step is clipped so that the last step ends exactly at z_end (a trial below
    10 ulp of z is an error).  Returns the state
    and a dict of counters (accepted, rejected, last accepted h, final z)."""
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    z, h = 0.0, float(h0)
    acc = rej = 0
    last_h = 0.0
    prev_rejected = False
    for _ in range(max_attempts):
        if z >= z_end:
            break
        z_new = min(z + h, z_end)
        h = z_new - z
        if h < 10 * (np.nextafter(z, np.inf) - z):
            raise RuntimeError("step size fell below 10 ulp of z")
        y5, e = dp54_step(psi, h, gamma, ops)
        err = error_norm(e, psi, y5, rtol, atol)
        if err < 1.0:
            psi, z = y5, z_new
            acc += 1
            last_h = h
            fac = facmax if not prev_rejected else 1.0
            prev_rejected = False
        else:
            rej += 1
            fac = 1.0
            prev_rejected = True
        h = h * min(fac, max(0.2, 0.9 * (err if err > 0 else 1e-300) ** -0.2))
    else:
        raise RuntimeError("adaptive integration did not reach z_end")
    return psi, {"accepted": acc, "rejected": rej, "last_h": last_h, "z": z}

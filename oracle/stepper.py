"""z-marching of the semi-discrete NLSE (FP64, complex128).

Test infrastructure: see the package docstring for who may use it.

The ODE is Eq. 10, ``i dPsi/dz = H_lin Psi - gamma (M |Psi|^2) Psi - i w Psi``,
with ``H_lin = p1 L + beta4 L^2 - diag(v)`` (sign reading in ``oracle.dec``)
and an absorbing imaginary potential ``w >= 0`` per vertex.

Readings:

* Integrator.  The paper integrates the whole right-hand side with adaptive
  Runge-Kutta (Eq. 10 under "DEC beam propagation") and names explicit RK4 as
  the natural fixed-step scheme (Introduction).  The workloads fix dz, and the
  method is split into a linear propagator and a pointwise Kerr/absorber step:
  one step is ``NL(h/2) -> LIN(h) -> NL(h/2)`` (Strang), LIN being one classical
  RK4 step of ``dPsi/dz = -i H_lin Psi``.  Half steps are never merged here.
* Kerr/absorber substep.  Over a distance tau the equation
  ``dpsi_p/dz = i gamma Theta_p psi_p - w_p psi_p`` with
  ``Theta = M |psi|^2`` keeps every phase-free quantity ``|psi_q|^2 e^{2 w_q z}``
  constant, so its exact flow is
  ``psi_p(tau) = psi_p e^{-w_p tau} exp(i gamma sum_q M_pq |psi_q|^2 phi(w_q, tau))``
  with ``phi(w, tau) = (1 - e^{-2 w tau}) / (2 w)`` (``phi -> tau`` as ``w -> 0``).
"""
from __future__ import annotations

import numpy as np

__all__ = ["phi", "nl_integral", "nl_flow", "lin_rk4", "strang_step", "propagate"]


def phi(w: np.ndarray, tau: float) -> np.ndarray:
    """Integral of e^{-2 w z} over [0, tau]."""
    w = np.asarray(w, dtype=np.float64)
    out = np.full(w.shape, float(tau))
    nz = w > 0
    out[nz] = -np.expm1(-2.0 * w[nz] * tau) / (2.0 * w[nz])
    return out


def nl_integral(I: np.ndarray, w: np.ndarray, tau: float, ops) -> np.ndarray:
    """Integral over [0, tau] of N(I e^{-2 w z}): what the phase Theta = M (.) of the
    exact flow accumulates when |psi|^2 decays as I e^{-2 w z}.

    kerr: I phi(w, tau); cubic-quintic: I phi(w, tau) - s I^2 phi(2w, tau);
    saturable (I_s): with a = I/I_s and e = e^{-2 w tau},
    (I_s / (2w)) log((1 + a) / (1 + a e)), which tends to tau I / (1 + a) as w -> 0;
    evaluated as (I_s / (2w)) log1p(a (1 - e) / (1 + a e)) with 1 - e = -expm1(-2 w tau),
    which keeps full precision for small a and small w tau."""
    w = np.asarray(w, dtype=np.float64)
    if ops.nl_kind == "kerr":
        return I * phi(w, tau)
    if ops.nl_kind == "cubic_quintic":
        return I * phi(w, tau) - ops.nl_param * I * I * phi(2.0 * w, tau)
    Is = ops.nl_param
    a = I / Is
    out = tau * I / (1.0 + a)
    nz = w > 0
    one_minus_e = -np.expm1(-2.0 * w[nz] * tau)
    e = 1.0 - one_minus_e
    out[nz] = Is / (2.0 * w[nz]) * np.log1p(a[nz] * one_minus_e / (1.0 + a[nz] * e))
    return out


def nl_flow(psi: np.ndarray, tau: float, gamma: float, ops) -> np.ndarray:
    """Exact flow of the Kerr phase and absorber damping over ``tau``."""
    theta = ops.M @ nl_integral(np.abs(psi) ** 2, ops.w, tau, ops)
    return psi * np.exp(-ops.w * tau) * np.exp(1j * gamma * theta)


def lin_rk4(psi: np.ndarray, h: float, ops) -> np.ndarray:
    """One classical fourth-order Runge-Kutta step of dPsi/dz = -i H_lin Psi."""

    def A(x):
        return -1j * ops.apply_H(x)

    k1 = A(psi)
    k2 = A(psi + 0.5 * h * k1)
    k3 = A(psi + 0.5 * h * k2)
    k4 = A(psi + h * k3)
    return psi + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def strang_step(psi: np.ndarray, h: float, gamma: float, ops) -> np.ndarray:
    psi = nl_flow(psi, 0.5 * h, gamma, ops)
    psi = lin_rk4(psi, h, ops)
    return nl_flow(psi, 0.5 * h, gamma, ops)


def propagate(psi0, ops, dz: float, n_steps: int, gamma: float, record_every: int = 0, record=None):
    """March ``n_steps`` Strang steps from ``psi0``.

    If ``record_every > 0``, ``record(step, psi)`` is called at step 0 and after
    every ``record_every`` steps (used for power/Hamiltonian histories)."""
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    if record_every and record is not None:
        record(0, psi)
    for n in range(1, n_steps + 1):
        psi = strang_step(psi, dz, gamma, ops)
        if record_every and record is not None and n % record_every == 0:
            record(n, psi)
    return psi

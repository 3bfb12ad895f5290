"""Nonlinear eigenmodes (soliton launches) by imaginary-z propagation (FP64).

Test infrastructure: see the package docstring for who may use it.

A stationary solution ``Psi(z) = phi exp(-i mu z)`` of the semi-discrete
equation without absorber (Eq. 10 with the operators of Eqs. 11-14, sign
reading of ``oracle.dec``) solves the nonlinear eigenproblem

    mu phi = G(phi),   G(phi) = H_lin phi - gamma (M N(|phi|^2)) * phi.

The paper launches such modes (its soliton shape-preservation benchmark) but
its eigen-solver sits in a supplementary note that is not available; this
module uses the gradient flow with discrete normalisation of Bao and Du
(SIAM J. Sci. Comput. 25, 2004): march the imaginary-z equation
``dphi/dtau = -A_k phi``, ``A_k = H_lin - gamma diag(M N(|phi_k|^2))`` (the
nonlinearity frozen at the start of the step, as in their discretisations),
one classical RK4 step of length ``dtau``, then rescale to the prescribed
power ``P = sum_p H0_p |phi_p|^2``.  A fixed point is an eigenvector of
``A(phi)``, i.e. an exact nonlinear eigenmode (stepping the full nonlinear
flow instead would shift the fixed point by O(dtau), since the flow changes
the amplitude inside the step).  The iteration, in this order:

    phi_0 = phi_start * sqrt(P / P(phi_start)),   mu_{-1} = 0
    for k = 0, 1, ...:
        g_k   = G(phi_k) = A_k phi_k
        mu_k  = Re <phi_k, g_k>_H0 / P(phi_k)                 (Rayleigh quotient)
        r_k   = ||g_k - mu_{k-1} phi_k||_H0 / ||phi_k||_H0    (residual, lagged mu)
        stop if k > 0 and tol > 0 and r_k <= tol |mu_k|      (result phi_k, mu_k)
        y = R4(-dtau A_k) phi_k  (four classical RK4 stages)
        phi_{k+1} = y * sqrt(P / P(y))

The residual uses the previous Rayleigh quotient so that it is a sum of
squares (no cancellation between two nearly equal sums); near convergence
the two quotients differ by O(r^2).  ``<a, b>_H0 = sum_p H0_p conj(a_p) b_p``.
"""
from __future__ import annotations

import numpy as np

__all__ = ["G", "itp_rk4_step", "find_mode"]


def G(phi: np.ndarray, ops, gamma: float) -> np.ndarray:
    """H_lin phi - gamma (M N(|phi|^2)) phi (the absorber plays no part)."""
    return ops.apply_H(phi) - gamma * (ops.M @ ops.N(np.abs(phi) ** 2)) * phi


def itp_rk4_step(phi: np.ndarray, dtau: float, gamma: float, ops) -> np.ndarray:
    """One classical RK4 step of dx/dtau = -A x, A = H_lin - gamma diag(M N(|phi|^2)) frozen at phi."""
    theta = ops.M @ ops.N(np.abs(phi) ** 2)
    f = lambda x: -(ops.apply_H(x) - gamma * theta * x)  # noqa: E731
    k1 = f(phi)
    k2 = f(phi + 0.5 * dtau * k1)
    k3 = f(phi + 0.5 * dtau * k2)
    k4 = f(phi + dtau * k3)
    return phi + (dtau / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def _power(x, ops) -> float:
    return float(np.sum(ops.H0 * np.abs(x) ** 2))


def find_mode(phi_start, ops, power: float, dtau: float, gamma: float, tol: float = 1e-10,
              max_iter: int = 100000):
    """Run the iteration above.  Returns ``(phi, info)`` with ``info`` holding
    ``mu``, ``residual``, ``iterations`` (the k of the returned phi_k) and
    ``converged``.  With ``tol == 0`` exactly ``max_iter`` steps are taken and
    the result is phi_{max_iter} with mu and r of the last tested iterate."""
    phi = np.array(phi_start, dtype=np.complex128, copy=True)
    phi *= np.sqrt(power / _power(phi, ops))
    mu_prev = 0.0
    mu = r = 0.0
    for k in range(max_iter):
        g = G(phi, ops, gamma)
        pk = _power(phi, ops)
        mu = float(np.sum(ops.H0 * (phi.conj() * g).real)) / pk
        r = float(np.sqrt(np.sum(ops.H0 * np.abs(g - mu_prev * phi) ** 2) / pk))
        if k > 0 and tol > 0 and r <= tol * abs(mu):
            return phi, {"mu": mu, "residual": r, "iterations": k, "converged": True}
        nxt = itp_rk4_step(phi, dtau, gamma, ops)
        phi = nxt * np.sqrt(power / _power(nxt, ops))
        mu_prev = mu
    return phi, {"mu": mu, "residual": r, "iterations": max_iter, "converged": tol == 0}

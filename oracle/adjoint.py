"""Exact discrete adjoint of ``oracle.stepper.propagate`` for the overlap objective (FP64).

Test infrastructure: see the package docstring for who may use it.

The paper motivates numerical optimisation of photonic structures with the
method (Abstract, Conclusion) but gives no gradient formulation, so this is
derived here from the forward scheme, in real pairs.  Gradients use the
convention ``g = dJ/dRe(psi) + i dJ/dIm(psi)``; for a real objective J this
means ``dJ = sum_p Re(conj(g_p) dpsi_p)``.

* Objective ``J = |c|^2`` with ``c = sum_p H0_p conj(t_p) psi_p(z_L)``, whose
  gradient is ``g = 2 c H0 t``.
* Linear map ``y = A x`` (complex matrix): ``g_x = A^H g_y`` (with the complex L of
  a perfectly matched layer, ``A^H`` conjugates as well as transposes).  For one RK4 stage
  ``k = A z`` with ``A = -i (H_lin - diag(dn) + ...)``, ``dk/d dn_p = i z_p e_p``,
  so ``dJ/d dn_p += Re(conj(g_k,p) i z_p)``.
* Kerr/absorber flow ``psi' = E psi`` with ``E = e^{-w tau} e^{i gamma Theta}``,
  ``Theta = M (|psi|^2 phi)``:
  ``g_psi = conj(E) g' + 2 phi (M^T mu) psi`` where
  ``mu_p = gamma Re(conj(g'_p) i psi'_p)``.

Every state of the forward sweep is stored (no checkpointing): this is the
plain reference the checkpointed GPU adjoint is compared with.
"""
from __future__ import annotations

import numpy as np

from .stepper import phi

__all__ = ["objective", "objective_grad", "nl_adjoint", "lin_rk4_adjoint", "gradients"]


def objective(psi, target, ops) -> float:
    c = np.sum(ops.H0 * np.conj(target) * psi)
    return float(abs(c) ** 2)


def objective_grad(psi, target, ops) -> np.ndarray:
    c = np.sum(ops.H0 * np.conj(target) * psi)
    return 2.0 * c * ops.H0 * target


def nl_adjoint(psi_in, psi_out, g_out, tau, gamma, ops):
    """Pull ``g_out`` back through ``psi_out = nl_flow(psi_in, tau)``."""
    ph = phi(ops.w, tau)
    theta = ops.M @ (np.abs(psi_in) ** 2 * ph)
    E = np.exp(-ops.w * tau) * np.exp(1j * gamma * theta)
    mu = gamma * np.real(np.conj(g_out) * 1j * psi_out)
    return np.conj(E) * g_out + 2.0 * ph * (ops.M.T @ mu) * psi_in


def lin_rk4_adjoint(psi_in, g_out, h, ops):
    """Pull ``g_out`` back through one classical RK4 step; also return the
    contribution to dJ/d(dn)."""

    def A(x):
        return -1j * ops.apply_H(x)

    def AH(x):  # (-i H)^H = i H^H, H^H x = conj(H^T conj(x)) (H^T for a real L)
        return 1j * np.conj(ops.apply_HT(np.conj(x)))

    # forward stage inputs z_j (k_j = A z_j)
    z1 = psi_in
    k1 = A(z1)
    z2 = psi_in + 0.5 * h * k1
    k2 = A(z2)
    z3 = psi_in + 0.5 * h * k2
    k3 = A(z3)
    z4 = psi_in + h * k3
    # reverse of psi_out = psi_in + h/6 (k1 + 2 k2 + 2 k3 + k4)
    g_psi = g_out.copy()
    g_k1 = (h / 6.0) * g_out
    g_k2 = (h / 3.0) * g_out
    g_k3 = (h / 3.0) * g_out
    g_k4 = (h / 6.0) * g_out
    g_dn = np.zeros(psi_in.shape[0])
    # k4 = A z4, z4 = psi_in + h k3
    g_dn += np.real(np.conj(g_k4) * 1j * z4)
    g_z4 = AH(g_k4)
    g_psi += g_z4
    g_k3 = g_k3 + h * g_z4
    # k3 = A z3, z3 = psi_in + h/2 k2
    g_dn += np.real(np.conj(g_k3) * 1j * z3)
    g_z3 = AH(g_k3)
    g_psi += g_z3
    g_k2 = g_k2 + 0.5 * h * g_z3
    # k2 = A z2, z2 = psi_in + h/2 k1
    g_dn += np.real(np.conj(g_k2) * 1j * z2)
    g_z2 = AH(g_k2)
    g_psi += g_z2
    g_k1 = g_k1 + 0.5 * h * g_z2
    # k1 = A psi_in
    g_dn += np.real(np.conj(g_k1) * 1j * z1)
    g_psi += AH(g_k1)
    return g_psi, g_dn


def gradients(psi0, target, ops, dz, n_steps, gamma):
    """Return ``(J, g_psi0, g_dn)`` for ``J = |<t, psi(z_L)>_H0|^2``.

    ``g_dn`` is the gradient with respect to a per-vertex perturbation added to
    the vertex potential ``v`` (``ops`` already holds the current ``v``).
    Written for the Kerr response and H_lin = p1 L + beta4 L^2 - diag(v), with a real
    L or the complex-stretched L of a perfectly matched layer (the objective, v and M
    keep the real H0)."""
    from .stepper import lin_rk4, nl_flow

    if ops.nl_kind != "kerr" or ops.p3 != 0.0 or ops.p4 != 0.0:
        raise NotImplementedError("the adjoint covers the Kerr response and terms up to L^2")

    h = dz
    states = []  # (x0, x1, x2) per step: step input, after NL(h/2), after LIN
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    for _ in range(n_steps):
        x0 = psi
        x1 = nl_flow(x0, 0.5 * h, gamma, ops)
        x2 = lin_rk4(x1, h, ops)
        psi = nl_flow(x2, 0.5 * h, gamma, ops)
        states.append((x0, x1, x2, psi))
    J = objective(psi, target, ops)
    g = objective_grad(psi, target, ops)
    g_dn = np.zeros(ops.n)
    for x0, x1, x2, x3 in reversed(states):
        g = nl_adjoint(x2, x3, g, 0.5 * h, gamma, ops)
        g, gd = lin_rk4_adjoint(x1, g, h, ops)
        g_dn += gd
        g = nl_adjoint(x0, x1, g, 0.5 * h, gamma, ops)
    return J, g, g_dn

"""Scalar diagnostics of a field on the mesh (FP64).

Test infrastructure: see the package docstring for who may use it.

* power ``P = Psi^H H0 Psi``: the discrete L2 norm that the semi-discrete flow
  conserves when the absorber is off (H0 H_lin is symmetric and the Kerr flow
  keeps |psi_p|).
* Hamiltonian ``E = Psi^H H0 H_lin Psi - (gamma/2) a^T Q^T D Q a`` with
  ``a = |Psi|^2`` for the triangle-averaged nonlinearity (Eq. 14), i.e.
  ``-(gamma/2) sum_t chi_t |t| (mean of a over t)^2``; for the lumped form
  ``-(gamma/2) sum_p H0_p chibar_p a_p^2``.  It satisfies
  ``i H0 dPsi/dz = dE/d conj(Psi)`` for Eq. 10 without absorber, so it is a
  conserved quantity of the semi-discrete flow (derived, not printed in the paper).
* overlap ``c = sum_p H0_p conj(t_p) psi_p`` (H0-weighted inner product).
* ``e_rel``: the paper's intensity error, Eq. 15.
* ``rel_l2``: plain relative 2-norm of the complex vertex vector.
"""
from __future__ import annotations

import numpy as np

__all__ = ["power", "hamiltonian", "overlap", "e_rel", "rel_l2"]


def power(psi, ops) -> float:
    return float(np.sum(ops.H0 * np.abs(psi) ** 2))


def hamiltonian(psi, ops, gamma: float) -> float:
    lin = np.vdot(psi, ops.H0 * ops.apply_H(psi)).real
    a = np.abs(psi) ** 2
    if ops.nl == "dec":
        a_tri = ops.Q @ a  # triangle-averaged intensity
        nonlin = np.sum(ops.chi_tri * ops.area * a_tri**2)
    else:
        nonlin = np.sum(ops.H0 * ops.M.diagonal() * a**2)
    return float(lin - 0.5 * gamma * nonlin)


def overlap(target, psi, ops) -> complex:
    return complex(np.sum(ops.H0 * np.conj(target) * psi))


def e_rel(psi, psi_ref) -> float:
    """Eq. 15: || |psi|^2 - |psi_ref|^2 ||_2 / || |psi_ref|^2 ||_2."""
    a = np.abs(psi) ** 2
    b = np.abs(psi_ref) ** 2
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_l2(x, ref) -> float:
    return float(np.linalg.norm(np.asarray(x) - np.asarray(ref)) / np.linalg.norm(ref))

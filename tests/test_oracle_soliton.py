"""Pins of the oracle's nonlinear eigenmode solver (imaginary-z propagation with power
renormalisation) against a dense generalized eigensolver, the 1D NLS soliton and the
z-marching of the split scheme (CPU only)."""
import math

import numpy as np
import scipy.linalg as sla

from oracle import dec, diagnostics as D, soliton as SO, stepper as S
from paper_2608_03587_amd.inputs import meshes as M


def _guide_case(seed=3):
    mesh = M.disk_mesh(4.0, 0.35, seed)
    r = np.hypot(*mesh.xy[mesh.tri].mean(axis=1).T)
    V = np.where(r < 1.5, 1.0, 0.0)
    return mesh, dec.assemble(mesh.xy, mesh.tri, index_tri=V)


def test_linear_limit_is_the_lowest_generalized_eigenpair():
    """gamma = 0: the iteration converges to the lowest eigenpair of H_lin, i.e. of the
    symmetric pencil (H0 H_lin, H0), solved densely by LAPACK."""
    mesh, ops = _guide_case()
    A = np.diag(ops.H0) @ ops.dense_H()
    A = 0.5 * (A + A.T)
    lam, vec = sla.eigh(A, np.diag(ops.H0))
    rho = abs(lam).max()
    rng = np.random.default_rng(0)
    start = np.exp(-np.sum(mesh.xy**2, axis=1)) * (1 + 0.1 * rng.normal(size=ops.n))
    phi, info = SO.find_mode(start + 0j, ops, 2.0, 2.0 / rho, 0.0, tol=1e-9)
    assert info["converged"]
    assert abs(info["mu"] - lam[0]) < 1e-9 * abs(lam[0]) + 1e-12, (info, lam[:2])
    v0 = vec[:, 0]
    c = np.vdot(v0, ops.H0 * phi) / math.sqrt(D.power(phi, ops) * np.sum(ops.H0 * v0**2))
    assert abs(abs(c) - 1) < 1e-8
    assert abs(D.power(phi, ops) - 2.0) < 1e-12


def test_strip_soliton_converges_to_sech_at_second_order():
    """Lumped nonlinearity on the right-triangle strip (the 1D finite-difference NLS for
    y-invariant fields): with the power of a sech(a x), the mode tends to a sech(a x) and
    mu to -a^2/2 (p1 = 1/2, gamma = 1) at order 2 in h."""
    a = 1.0
    errs, mus = [], []
    for h in (0.2, 0.1):
        mesh = M.strip_mesh(16.0, h, n_rows=3)
        ops = dec.assemble(mesh.xy, mesh.tri, nl="lumped")
        x = mesh.xy[:, 0]
        exact = a / np.cosh(a * x)
        P = D.power(exact, ops)
        start = np.exp(-x**2 / 4) + 0j
        rho = 4 * 0.5 * 4 / h**2  # bound on the spectral radius of p1 L on this grid
        phi, info = SO.find_mode(start, ops, P, 2.0 / rho, 1.0, tol=1e-10)
        assert info["converged"], info
        phase = np.vdot(exact, phi) / abs(np.vdot(exact, phi))
        errs.append(D.rel_l2(phi / phase, exact))
        mus.append(abs(info["mu"] + a * a / 2))
    assert errs[1] < 5e-3 and math.log(errs[0] / errs[1], 2) > 1.8, errs
    assert math.log(mus[0] / mus[1], 2) > 1.8, mus


def test_mode_is_stationary_under_z_marching():
    """The converged mode of the guiding core with the triangle-averaged Kerr term keeps its
    shape under the split z-marching: Psi(z) = phi e^{-i mu z} up to the scheme's O(dz^2)."""
    mesh, ops = _guide_case(5)
    rho = np.abs(np.linalg.eigvals(ops.dense_H())).max()
    start = np.exp(-np.sum(mesh.xy**2, axis=1)) + 0j
    phi, info = SO.find_mode(start, ops, 3.0, 2.0 / rho, 1.0, tol=1e-11)
    assert info["converged"]
    z, n = 1.0, 400
    out = S.propagate(phi, ops, z / n, n, 1.0)
    assert D.rel_l2(out, phi * np.exp(-1j * info["mu"] * z)) < 1e-4
    # the residual is what the stopping rule says, and G(phi) = mu phi to that level
    g = SO.G(phi, ops, 1.0)
    assert np.sqrt(np.sum(ops.H0 * np.abs(g - info["mu"] * phi) ** 2) / 3.0) <= 2e-11 * abs(info["mu"])


def test_fixed_iteration_count_and_power():
    """tol = 0 takes exactly max_iter steps; every iterate has the prescribed power."""
    mesh, ops = _guide_case()
    start = np.exp(-np.sum(mesh.xy**2, axis=1)) + 0j
    phi, info = SO.find_mode(start, ops, 1.5, 1e-3, 1.0, tol=0.0, max_iter=7)
    assert info["iterations"] == 7 and info["converged"]
    assert abs(D.power(phi, ops) - 1.5) < 1e-12
    # by hand: seven normalised RK4 steps
    x = start * np.sqrt(1.5 / D.power(start, ops))
    for _ in range(7):
        y = SO.itp_rk4_step(x, 1e-3, 1.0, ops)
        x = y * np.sqrt(1.5 / D.power(y, ops))
    assert np.abs(x - phi).max() == 0.0

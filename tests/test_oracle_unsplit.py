"""Pins of the oracle's unsplit RK4 (Kerr term inside every stage) against
brute force, hand-computed scalar Runge-Kutta, its convergence order and the
split scheme (CPU only)."""
import math

import numpy as np
import pytest

from oracle import dec, diagnostics as D, stepper as S, unsplit as U
from paper_2608_03587_amd.inputs import fields as F
from paper_2608_03587_amd.inputs import meshes as M


def _scalar_rk4(f, y, h):
    """Classical RK4 on a scalar complex ODE y' = f(y), written out for the test."""
    k1 = f(y)
    k2 = f(y + h / 2 * k1)
    k3 = f(y + h / 2 * k2)
    k4 = f(y + h * k3)
    return y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)


def test_linear_part_with_absorber_is_the_rk4_polynomial():
    """gamma = 0: one step is R4(h A) psi with A = -i H_lin - diag(w), summed here as a
    Taylor series of dense matrix products."""
    mesh = M.random_delaunay_mesh(40, 2)
    rng = np.random.default_rng(2)
    ops = dec.assemble(mesh.xy * 4.0, mesh.tri, index_tri=rng.uniform(0, 2, mesh.n_tri),
                       absorber=rng.uniform(0, 1.5, mesh.n_vert), beta4=1e-3)
    A = -1j * ops.dense_H() - np.diag(ops.w)
    h = 0.4 / np.abs(np.linalg.eigvals(A)).max()
    psi = rng.normal(size=ops.n) + 1j * rng.normal(size=ops.n)
    term, ref = psi.copy(), psi.copy()
    for j in range(1, 5):
        term = (h / j) * (A @ term)
        ref = ref + term
    assert D.rel_l2(U.rk4_step(psi, h, 0.0, ops), ref) < 1e-14
    # and it coincides with the split scheme's linear step when there is no absorber
    ops.w = np.zeros(ops.n)
    assert D.rel_l2(U.rk4_step(psi, h, 0.0, ops), S.lin_rk4(psi, h, ops)) < 1e-14


@pytest.mark.parametrize("nl", ["dec", "lumped"])
def test_plane_wave_is_scalar_rk4_of_the_kerr_ode(nl):
    """Constant field, uniform potential V0, no absorber: L 1 = 0 and M 1 = 1 keep it
    constant, and every vertex follows scalar RK4 on y' = i (V0 + gamma |y|^2) y."""
    mesh = M.disk_mesh(3.0, 0.4, 1)
    V0, a, gamma, h, n = 0.7, 0.9 - 0.3j, 1.3, 2e-2, 30
    ops = dec.assemble(mesh.xy, mesh.tri, index_tri=np.full(mesh.n_tri, V0), nl=nl)
    out = U.propagate_rk4(np.full(ops.n, a), ops, h, n, gamma)
    y = a
    for _ in range(n):
        y = _scalar_rk4(lambda u: 1j * (V0 + gamma * abs(u) ** 2) * u, y, h)
    np.testing.assert_allclose(out, np.full(ops.n, y), rtol=1e-12)


def test_pointwise_kerr_and_absorber_is_scalar_rk4_per_vertex():
    """No coupling (p1 = 0, V = 0) and the lumped nonlinearity: vertex p follows scalar
    RK4 on y' = (i gamma chi_p |y|^2 - w_p) y with chi_p the vertex average of chi."""
    mesh = M.random_delaunay_mesh(30, 4)
    rng = np.random.default_rng(4)
    chi = rng.uniform(0.5, 1.5, mesh.n_tri)
    ops = dec.assemble(mesh.xy, mesh.tri, absorber=rng.uniform(0, 2, mesh.n_vert), chi_tri=chi, nl="lumped", p1=0.0)
    gamma, h = 0.8, 0.05
    psi = rng.normal(size=ops.n) + 1j * rng.normal(size=ops.n)
    out = U.rk4_step(psi, h, gamma, ops)
    chibar = ops.M.diagonal()
    for p in range(ops.n):
        ref = _scalar_rk4(lambda u: (1j * gamma * chibar[p] * abs(u) ** 2 - ops.w[p]) * u, psi[p], h)
        assert abs(out[p] - ref) < 1e-14 * max(1.0, abs(ref))


def _gaussian_case():
    mesh = M.disk_mesh(6.0, 0.5, 7)
    ops = dec.assemble(mesh.xy, mesh.tri)
    u0 = 0.9 * np.exp(-(mesh.xy ** 2).sum(1) / 2.0).astype(complex)
    return ops, u0


def test_fourth_order_in_dz():
    """Against the same scheme at dz/16, the error falls 16-fold per halving of dz."""
    ops, u0 = _gaussian_case()
    z, gamma = 0.4, 1.0
    ref = U.propagate_rk4(u0, ops, z / 320, 320, gamma)
    errs = [D.rel_l2(U.propagate_rk4(u0, ops, z / n, n, gamma), ref) for n in (20, 40, 80)]
    orders = [math.log(errs[k] / errs[k + 1], 2) for k in range(2)]
    assert min(orders) > 3.7, (errs, orders)


def test_split_and_unsplit_schemes_converge_to_the_same_solution():
    """Both integrate the same ODE: their distance falls like dz^2 (the split error)."""
    ops, u0 = _gaussian_case()
    z, gamma = 0.4, 1.0
    d = [D.rel_l2(S.propagate(u0, ops, z / n, n, gamma), U.propagate_rk4(u0, ops, z / n, n, gamma))
         for n in (20, 40, 80)]
    orders = [math.log(d[k] / d[k + 1], 2) for k in range(2)]
    assert min(orders) > 1.8, (d, orders)

"""Pins of the oracle's discrete adjoint: dot-product identities and central
finite differences in FP64 (CPU only)."""
import numpy as np
import pytest

from oracle import adjoint as A, dec, stepper as S
from paper_2608_03587_amd.inputs import fields as F
from paper_2608_03587_amd.inputs import meshes as M


def _ops(seed=0, beta4=0.0, nl="dec"):
    mesh = M.disk_mesh(3.0, 0.5, seed)
    rng = np.random.default_rng(seed)
    V = F.step_index_tri(mesh.xy, mesh.tri, 1.5, 0.8)
    w = F.quadratic_absorber(mesh.xy, 2.0, 3.0, 0.5)
    ops = dec.assemble(mesh.xy, mesh.tri, index_tri=V, absorber=w, beta4=beta4, nl=nl)
    return mesh, ops, rng


def _rand(rng, n):
    return rng.normal(size=n) + 1j * rng.normal(size=n)


def _rdot(a, b):
    return float(np.real(np.vdot(a, b)))


@pytest.mark.parametrize("beta4", [0.0, 2e-3])
def test_linear_step_dot_product_identity(beta4):
    mesh, ops, rng = _ops(1, beta4)
    x, y = _rand(rng, ops.n), _rand(rng, ops.n)
    h = 0.01
    lhs = _rdot(y, S.lin_rk4(x, h, ops))
    g, _ = A.lin_rk4_adjoint(x, y, h, ops)  # the map is linear in x, so the base point is irrelevant
    assert abs(lhs - _rdot(g, x)) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("nl", ["dec", "lumped"])
def test_kerr_step_adjoint_against_directional_derivative(nl):
    mesh, ops, rng = _ops(2, nl=nl)
    psi = 0.8 * _rand(rng, ops.n)
    d = _rand(rng, ops.n)
    g_out = _rand(rng, ops.n)
    tau, gamma, eps = 0.05, 1.3, 1e-6
    out = S.nl_flow(psi, tau, gamma, ops)
    fd = (S.nl_flow(psi + eps * d, tau, gamma, ops) - S.nl_flow(psi - eps * d, tau, gamma, ops)) / (2 * eps)
    g_in = A.nl_adjoint(psi, out, g_out, tau, gamma, ops)
    assert abs(_rdot(g_out, fd) - _rdot(g_in, d)) < 1e-8 * abs(_rdot(g_in, d))


@pytest.mark.parametrize("beta4", [0.0, 2e-3])
def test_full_gradient_matches_central_differences(beta4):
    mesh, ops, rng = _ops(3, beta4)
    u0 = F.elliptic_gaussian(mesh.xy, 1.2, 0.8, 1.2, 0.4)
    target = F.gaussian(mesh.xy, 1.0, 0.9, centre=(0.4, 0.0)) * np.exp(0.7j)
    dz, n, gamma = 2e-3, 12, 1.0
    J, g_u, g_dn = A.gradients(u0, target, ops, dz, n, gamma)

    def run(u, dv):
        o = dec.assemble(mesh.xy, mesh.tri, index_tri=F.step_index_tri(mesh.xy, mesh.tri, 1.5, 0.8),
                         absorber=ops.w, beta4=beta4, dn=dv)
        return A.objective(S.propagate(u, o, dz, n, gamma), target, o)

    zero = np.zeros(ops.n)
    assert abs(run(u0, zero) - J) < 1e-14 * J
    eps = 1e-5  # central differences: O(eps^2) truncation, rounding ~1e-16 J / eps
    for k in range(3):
        d = _rand(rng, ops.n)
        fd = (run(u0 + eps * d, zero) - run(u0 - eps * d, zero)) / (2 * eps)
        assert abs(fd - _rdot(g_u, d)) < 1e-6 * abs(fd), (fd, _rdot(g_u, d))
        e = rng.normal(size=ops.n)
        fd = (run(u0, 1e-4 * e) - run(u0, -1e-4 * e)) / 2e-4
        assert abs(fd - float(g_dn @ e)) < 1e-6 * abs(fd), (fd, float(g_dn @ e))


def _pml_ops(seed):
    mesh = M.disk_mesh(4.0, 0.5, seed)
    V = F.step_index_tri(mesh.xy, mesh.tri, 1.5, 0.8)
    pml = (2.5, 4.0, 1.5)
    return mesh, V, pml, dec.assemble(mesh.xy, mesh.tri, index_tri=V, pml=pml)


def test_pml_linear_step_dot_product_identity():
    """With the complex-stretched L of a perfectly matched layer the adjoint of the RK4
    step must conjugate as well as transpose: a transposing-only adjoint fails this."""
    mesh, V, pml, ops = _pml_ops(5)
    assert np.iscomplexobj(ops.L.data)
    rng = np.random.default_rng(5)
    x, y = _rand(rng, ops.n), _rand(rng, ops.n)
    h = 0.01
    lhs = _rdot(y, S.lin_rk4(x, h, ops))
    g, _ = A.lin_rk4_adjoint(x, y, h, ops)
    assert abs(lhs - _rdot(g, x)) < 1e-12 * abs(lhs)


def test_pml_full_gradient_matches_central_differences():
    mesh, V, pml, ops = _pml_ops(6)
    rng = np.random.default_rng(6)
    u0 = F.gaussian(mesh.xy, 1.0, 1.0) * np.exp(2j * mesh.xy[:, 0])  # an outgoing beam reaches the layer
    target = F.gaussian(mesh.xy, 1.0, 0.9, centre=(0.4, 0.0)) * np.exp(0.7j)
    dz, n, gamma = 2e-3, 12, 1.0
    J, g_u, g_dn = A.gradients(u0, target, ops, dz, n, gamma)

    def run(u, dv):
        o = dec.assemble(mesh.xy, mesh.tri, index_tri=V, pml=pml, dn=dv)
        return A.objective(S.propagate(u, o, dz, n, gamma), target, o)

    zero = np.zeros(ops.n)
    assert abs(run(u0, zero) - J) < 1e-14 * J
    eps = 1e-5
    for k in range(3):
        d = _rand(rng, ops.n)
        fd = (run(u0 + eps * d, zero) - run(u0 - eps * d, zero)) / (2 * eps)
        assert abs(fd - _rdot(g_u, d)) < 1e-6 * abs(fd), (fd, _rdot(g_u, d))
        e = rng.normal(size=ops.n)
        fd = (run(u0, 1e-4 * e) - run(u0, -1e-4 * e)) / 2e-4
        assert abs(fd - float(g_dn @ e)) < 1e-6 * abs(fd), (fd, float(g_dn @ e))


def test_objective_gradient_convention():
    """g = dJ/dRe + i dJ/dIm (checked on J = |<t, psi>|^2 by real finite differences)."""
    mesh, ops, rng = _ops(4)
    psi, t = _rand(rng, ops.n), _rand(rng, ops.n)
    g = A.objective_grad(psi, t, ops)
    p, eps = 7, 1e-6
    e = np.zeros(ops.n, complex)
    e[p] = 1
    dre = (A.objective(psi + eps * e, t, ops) - A.objective(psi - eps * e, t, ops)) / (2 * eps)
    dim = (A.objective(psi + 1j * eps * e, t, ops) - A.objective(psi - 1j * eps * e, t, ops)) / (2 * eps)
    assert abs(g[p] - (dre + 1j * dim)) < 1e-6 * abs(g[p])

"""Pins of the oracle's general operator sum p1 L + p2 L^2 + p3 L^3 + p4 L^4 and of its
non-Kerr responses N(|psi|^2) (saturable, cubic-quintic): plane waves of the grid
stencil, quadrature of the exact-flow integral, the flow's semigroup property and an
ODE solve, and the Kerr limits (CPU only)."""
import numpy as np
import pytest
from scipy.integrate import quad, solve_ivp

from oracle import dec, stepper as S, unsplit as U
from paper_2608_03587_amd.inputs import meshes as M

KINDS = [("saturable", 0.7), ("cubic_quintic", 0.3), ("kerr", 0.0)]


def test_operator_sum_on_plane_waves():
    """Inside a right-triangle grid L is the five-point stencil, so a plane wave is an
    eigenvector of every power of L away from the boundary: H u = (sum p_n lam^n) u."""
    h = 0.5
    g = M.regular_grid_mesh(21, 21, h, h)
    p = (0.5, 0.01, -0.002, 3e-4)
    ops = dec.assemble(g.xy, g.tri, p1=p[0], beta4=p[1], p3=p[2], p4=p[3])
    x, y = g.xy[:, 0], g.xy[:, 1]
    kx, ky = 0.7, 1.3
    u = np.exp(1j * (kx * x + ky * y))
    lam = (2 - 2 * np.cos(kx * h)) / h**2 + (2 - 2 * np.cos(ky * h)) / h**2
    mu = sum(c * lam ** (n + 1) for n, c in enumerate(p))
    inner = (np.abs(x - x.mean()) < np.ptp(x) / 2 - 4.5 * h) & (np.abs(y - y.mean()) < np.ptp(y) / 2 - 4.5 * h)
    assert inner.sum() > 100
    # rounding scales with the stencil's norm (8/h^2 per power), not with lam
    scale = lambda n: (8 / h**2) ** n  # noqa: E731
    assert np.abs(ops.apply_H(u)[inner] - mu * u[inner]).max() < 1e-14 * sum(abs(c) * scale(n + 1)
                                                                              for n, c in enumerate(p))
    # each coefficient enters once, with its own power
    for n in range(4):
        q = [0.0] * 4
        q[n] = 1.0
        o = dec.assemble(g.xy, g.tri, p1=q[0], beta4=q[1], p3=q[2], p4=q[3])
        assert np.abs(o.apply_H(u)[inner] - lam ** (n + 1) * u[inner]).max() < 1e-14 * scale(n + 1)
    # the dense form agrees with the applied one everywhere
    assert np.abs(ops.dense_H() @ u - ops.apply_H(u)).max() < 1e-12 * np.abs(ops.apply_H(u)).max()


@pytest.mark.parametrize("kind,param", KINDS)
def test_flow_integral_is_the_quadrature(kind, param):
    mesh = M.disk_mesh(2.0, 0.5, 1)
    ops = dec.assemble(mesh.xy, mesh.tri, nl_kind=kind, nl_param=param)
    I = np.array([0.0, 0.3, 1.0, 2.5, 7.0])
    for w in (0.0, 0.2, 3.0):
        for tau in (1e-3, 0.4):
            got = S.nl_integral(I, np.full(I.shape, w), tau, ops)
            ref = [quad(lambda z: ops.N(np.array([i * np.exp(-2 * w * z)]))[0], 0, tau, epsabs=1e-15,
                        epsrel=1e-13)[0] for i in I]
            assert np.allclose(got, ref, rtol=1e-11, atol=1e-15), (kind, w, tau, got, ref)


@pytest.mark.parametrize("kind,param", KINDS)
def test_flow_is_exact(kind, param):
    """The substep is the exact flow of dpsi/dz = i gamma (M N(|psi|^2)) psi - w psi: it is
    a semigroup and it matches a tight ODE solve."""
    mesh = M.disk_mesh(3.0, 0.45, 2)
    rng = np.random.default_rng(5)
    ops = dec.assemble(mesh.xy, mesh.tri, absorber=rng.uniform(0, 1.5, mesh.n_vert), nl_kind=kind, nl_param=param)
    psi = (rng.normal(size=ops.n) + 1j * rng.normal(size=ops.n)) * 1.2
    gamma = 0.8
    a = S.nl_flow(S.nl_flow(psi, 0.13, gamma, ops), 0.29, gamma, ops)
    b = S.nl_flow(psi, 0.42, gamma, ops)
    assert np.abs(a - b).max() < 1e-13 * np.abs(b).max()
    f = lambda _, y: 1j * gamma * (ops.M @ ops.N(np.abs(y) ** 2)) * y - ops.w * y  # noqa: E731
    sol = solve_ivp(f, (0, 0.42), psi.astype(np.complex128), method="DOP853", rtol=1e-12, atol=1e-14)
    assert np.abs(sol.y[:, -1] - b).max() < 1e-9 * np.abs(b).max()
    # the unsplit right-hand side uses the same response
    assert np.allclose(U.rhs(psi, ops, gamma), -1j * ops.apply_H(psi) + f(0, psi))


def test_kerr_limits():
    mesh = M.disk_mesh(3.0, 0.45, 2)
    rng = np.random.default_rng(6)
    w = rng.uniform(0, 1.0, mesh.n_vert)
    psi = rng.normal(size=mesh.n_vert) + 1j * rng.normal(size=mesh.n_vert)
    kerr = dec.assemble(mesh.xy, mesh.tri, absorber=w)
    cq0 = dec.assemble(mesh.xy, mesh.tri, absorber=w, nl_kind="cubic_quintic", nl_param=0.0)
    sat = dec.assemble(mesh.xy, mesh.tri, absorber=w, nl_kind="saturable", nl_param=1e12)
    ref = S.nl_flow(psi, 0.3, 1.0, kerr)
    assert np.array_equal(S.nl_flow(psi, 0.3, 1.0, cq0), ref)
    assert np.abs(S.nl_flow(psi, 0.3, 1.0, sat) - ref).max() < 1e-9
    with pytest.raises(ValueError):
        dec.assemble(mesh.xy, mesh.tri, nl_kind="cubic")

"""Pins of the oracle's scalar diagnostics: the overlap, the objective built
on it, the paper's intensity error (Eq. 15) and the plain relative L2 norm.

The overlap is the H0-weighted inner product c = sum_p H0_p conj(t_p) psi_p:
conjugate-linear in the target, linear in the field, equal to the power on
the diagonal.  A swapped conjugation would leave the objective |c|^2 of a
single pair unchanged, so the pins below fix it through linearity and a
hand-computed value on one triangle.
"""
import numpy as np

from oracle import adjoint as OA
from oracle import dec
from oracle import diagnostics as D
from paper_2608_03587_amd.inputs import meshes as M


def _one_triangle():
    # legs 2 and 1: area 1, so each barycentric dual area is 1/3
    return dec.assemble(np.array([[0.0, 0.0], [2.0, 0.0], [0.0, 1.0]]), np.array([[0, 1, 2]]))


def test_overlap_on_one_triangle_by_hand():
    ops = _one_triangle()
    assert np.allclose(ops.H0, [1 / 3, 1 / 3, 1 / 3], rtol=0, atol=1e-15)
    t = np.array([1.0, 1j, 0.0])
    u = np.array([2.0, 1.0, 5.0])
    # (1/3) (conj(1) 2 + conj(i) 1 + 0) = (2 - i)/3
    assert abs(D.overlap(t, u, ops) - (2 - 1j) / 3) < 1e-15
    # the objective is |c|^2 = 5/9 and its gradient 2 c H0 t
    assert abs(OA.objective(u, t, ops) - 5 / 9) < 1e-15
    assert np.allclose(OA.objective_grad(u, t, ops), 2 * (2 - 1j) / 3 * np.array([1 / 3, 1j / 3, 0.0]), atol=1e-15)


def test_overlap_conjugates_the_target_only():
    mesh = M.disk_mesh(3.0, 0.5, 2)
    ops = dec.assemble(mesh.xy, mesh.tri)
    rng = np.random.default_rng(0)
    t = rng.normal(size=ops.n) + 1j * rng.normal(size=ops.n)
    u = rng.normal(size=ops.n) + 1j * rng.normal(size=ops.n)
    a = 0.3 - 1.7j
    c = D.overlap(t, u, ops)
    assert abs(D.overlap(t, a * u, ops) - a * c) < 1e-12 * abs(c)  # linear in the field
    assert abs(D.overlap(a * t, u, ops) - np.conj(a) * c) < 1e-12 * abs(c)  # conjugate-linear in the target
    assert abs(D.overlap(u, t, ops) - np.conj(c)) < 1e-12 * abs(c)  # Hermitian
    P = D.overlap(u, u, ops)
    assert abs(P.imag) < 1e-14 * abs(P) and abs(P.real - D.power(u, ops)) < 1e-12 * P.real
    # the objective and its gradient agree with the overlap: dJ = Re(conj(g) du) along any du
    du = rng.normal(size=ops.n) + 1j * rng.normal(size=ops.n)
    g = OA.objective_grad(u, t, ops)
    h = 1e-6
    fd = (OA.objective(u + h * du, t, ops) - OA.objective(u - h * du, t, ops)) / (2 * h)
    assert abs(fd - np.sum(np.real(np.conj(g) * du))) < 1e-7 * abs(fd)


def test_intensity_error_closed_forms():
    rng = np.random.default_rng(1)
    u = rng.normal(size=50) + 1j * rng.normal(size=50)
    assert D.e_rel(u, u) == 0.0
    # scaling by s changes every intensity by s^2: E_rel = |s^2 - 1|
    for s in (0.5, 1.1, 3.0):
        assert abs(D.e_rel(s * u, u) - abs(s * s - 1)) < 1e-14
    # a unit-modulus pointwise phase leaves every intensity unchanged
    assert D.e_rel(u * np.exp(1j * rng.uniform(0, 6, 50)), u) < 1e-15
    # plain relative L2 of a scaled copy
    assert abs(D.rel_l2(1.25 * u, u) - 0.25) < 1e-15

"""Pins of the oracle's perfectly matched layer (complex-stretched Hodge stars): the
unstretched limit, a constant complex scaling, second-order consistency with the
stretched Laplacian, a non-growing spectrum, and absorption measured against a twice
larger domain (CPU only)."""
import math

import numpy as np
from scipy.interpolate import LinearNDInterpolator

from oracle import dec, stepper as S
from paper_2608_03587_amd.inputs import meshes as M


def test_zero_sigma_is_the_plain_operator():
    mesh = M.disk_mesh(4.0, 0.35, 3)
    a = dec.assemble(mesh.xy, mesh.tri)
    b = dec.assemble(mesh.xy, mesh.tri, pml=(2.5, 4.0, 0.0))
    assert abs(a.L - b.L).max() < 1e-14 * abs(a.L).max()


def test_constant_complex_scaling_divides_L_by_its_square():
    """r0 = 0 with a flat profile (m = 0): r~ = (1 + i s) r everywhere, so Lambda = I,
    the area factor is (1 + i s)^2 and L~ = L / (1 + i s)^2."""
    mesh = M.disk_mesh(4.0, 0.35, 3)
    a = dec.assemble(mesh.xy, mesh.tri)
    c = dec.assemble(mesh.xy, mesh.tri, pml=(0.0, 4.0, 0.7, 0.0))
    assert abs(a.L / (1 + 0.7j) ** 2 - c.L).max() < 1e-14 * abs(a.L).max()


def test_stretched_laplacian_of_r_tilde_squared():
    """u = r~^2 has Laplacian 4 in the stretched coordinates; on a right-triangle grid inside
    the layer L~ u -> -4 at second order in h (the anisotropic tensor and the area factor both
    enter: swapping s_r and s_t, or dropping the area factor, changes the limit)."""
    errs = []
    for h in (0.1, 0.05, 0.025):
        n = int(round(2.0 / h))
        g = M.regular_grid_mesh(n + 1, n + 1, h, h, x0=2.5, y0=0.5)
        ops = dec.assemble(g.xy, g.tri, pml=(2.0, 4.0, 1.0))
        r = np.hypot(g.xy[:, 0], g.xy[:, 1])
        _, s_t = dec.pml_stretch(r, 2.0, 4.0, 1.0)
        Lu = ops.L @ ((r * s_t) ** 2)
        near = np.hypot(g.xy[:, 0] - 3.5, g.xy[:, 1] - 1.5) < 0.3
        errs.append(np.abs(Lu[near] + 4.0).max())
    orders = [math.log(errs[k] / errs[k + 1], 2) for k in range(2)]
    assert errs[-1] < 2e-3 and min(orders) > 1.9, (errs, orders)


def test_spectrum_in_the_closed_lower_half_plane_and_below_the_plain_radius():
    """Eigenvalues of L~ have Im <= 0 (the linear z-evolution exp(-i p1 L~ z) does not grow)
    and modulus at most the plain operator's spectral radius."""
    mesh = M.disk_mesh(4.0, 0.35, 3)
    d = dec.assemble(mesh.xy, mesh.tri, pml=(2.5, 4.0, 1.0))
    ev = np.linalg.eigvals(d.L.toarray())
    rho = abs(np.linalg.eigvals(dec.assemble(mesh.xy, mesh.tri).L.toarray())).max()
    assert ev.imag.max() < 1e-12 * rho
    assert ev.imag.min() < -1e-2 * rho  # the layer does damp
    assert abs(ev).max() <= rho * (1 + 1e-12)


def test_layer_absorbs_an_outgoing_beam():
    """A Gaussian beam with transverse speed 3 leaves the inner region (r < 4.5) of a disk of
    radius 8 with a layer on 5 < r < 8.  Against the same launch on a disk of radius 16
    (whose boundary echo cannot return by z = 4), the inner field with the layer stays at the
    meshes' discretisation mismatch (measured 0.03 at z = 1, before anything reaches a
    boundary), while a reflecting boundary and the quadratic absorber of the workloads
    (0.5 at the rim) return most of the beam."""
    h, z, dz = 0.25, 4.0, 0.02
    launch = lambda xy: np.exp(-(xy[:, 0] ** 2 + xy[:, 1] ** 2)) * np.exp(3j * xy[:, 0])  # noqa: E731
    big, small = M.disk_mesh(16.0, h, 7), M.disk_mesh(8.0, h, 7)
    n = int(round(z / dz))
    ref = S.propagate(launch(big.xy) + 0j, dec.assemble(big.xy, big.tri), dz, n, 0.0)
    r = np.hypot(small.xy[:, 0], small.xy[:, 1])
    inner = r < 4.5
    refs = LinearNDInterpolator(big.xy, ref)(small.xy[inner])
    u0n = np.linalg.norm(launch(small.xy)[inner])
    err = {}
    for name, kw in (("reflecting", {}), ("cap", {"absorber": np.where(r > 5, 0.5 * ((r - 5) / 3) ** 2, 0.0)}),
                     ("pml", {"pml": (5.0, 8.0, 1.0)})):
        out = S.propagate(launch(small.xy) + 0j, dec.assemble(small.xy, small.tri, **kw), dz, n, 0.0)
        err[name] = np.linalg.norm(out[inner] - refs) / u0n
    assert err["pml"] < 0.03, err
    assert err["pml"] < 0.05 * err["reflecting"] and err["pml"] < 0.1 * err["cap"], err

"""Pins of the oracle's DEC operators against closed forms, invariants,
hand-computed values and textbook results (CPU only)."""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.special import jnp_zeros

from oracle import dec
from paper_2608_03587_amd.inputs import meshes as M

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_blocks(path):
    blocks, cur = {}, None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line[0].isalpha():
            cur = line
            blocks[cur] = []
        else:
            blocks[cur].append([float(x) for x in line.split()])
    return {k: np.array(v) for k, v in blocks.items()}


def _cotangent_stiffness(xy, tri):
    """Textbook P1 stiffness: K_ij = -1/2 (cot a + cot b) over the angles opposite edge ij,
    K_ii = -sum_j K_ij (written from the angle definition, not from any oracle code)."""
    n = xy.shape[0]
    K = np.zeros((n, n))
    for t in tri:
        for k in range(3):
            o, i, j = t[k], t[(k + 1) % 3], t[(k + 2) % 3]
            u = xy[i] - xy[o]
            v = xy[j] - xy[o]
            cot = np.dot(u, v) / abs(u[0] * v[1] - u[1] * v[0])
            K[i, j] -= 0.5 * cot
            K[j, i] -= 0.5 * cot
    K[np.diag_indices(n)] = -K.sum(axis=1)
    return K


def test_whitney_hodge_right_triangle_golden():
    g = _read_blocks(os.path.join(GOLDEN, "whitney_right_triangle.txt"))
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    ops = dec.assemble(xy, np.array([[0, 1, 2]]))
    assert ops.edges.tolist() == [[0, 1], [0, 2], [1, 2]]
    np.testing.assert_allclose(ops.H1.toarray(), g["H1"], atol=1e-15)
    np.testing.assert_allclose(ops.K.toarray(), g["K"], atol=1e-15)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_d1_d0_is_zero_and_euler(seed):
    mesh = M.random_delaunay_mesh(80, seed)
    tri = dec.orient_ccw(mesh.xy, mesh.tri)
    edges = dec.edge_list(tri)
    D0 = dec.incidence_d0(edges, mesh.n_vert)
    D1 = dec.incidence_d1(tri, edges)
    prod = (D1 @ D0).toarray()
    assert np.count_nonzero(prod) == 0  # d^2 = 0 exactly
    assert mesh.n_vert - edges.shape[0] + tri.shape[0] == 1  # a triangulated disk
    # each triangle has 3 edges; interior edges 2 triangles, boundary edges 1
    assert np.all(np.abs(D1).sum(axis=1) == 3)
    assert set(np.unique(np.asarray(abs(D1).sum(axis=0)).ravel())) <= {1.0, 2.0}


def test_orient_ccw():
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    tri = np.array([[0, 2, 1], [1, 2, 3]])  # first one clockwise
    t = dec.orient_ccw(xy, tri)
    a = dec._signed_areas(xy, t)
    assert np.all(a > 0)
    assert sorted(t[0]) == [0, 1, 2]


@pytest.mark.parametrize("seed", [4, 5])
def test_stiffness_equals_cotangent_formula(seed):
    mesh = M.random_delaunay_mesh(60, seed)
    ops = dec.assemble(mesh.xy, mesh.tri)
    Kc = _cotangent_stiffness(mesh.xy, ops.tri)
    scale = np.abs(Kc).max()
    np.testing.assert_allclose(ops.K.toarray(), Kc, atol=1e-13 * scale)


def test_stiffness_equals_diagonal_voronoi_hodge_on_delaunay():
    """On a Delaunay mesh the circumcentric (Voronoi) diagonal H1 = |dual edge|/|edge|
    gives the same D0^T H1 D0 (the alternative Hodge star the paper mentions)."""
    mesh = M.disk_mesh(3.0, 0.5, 7)
    ops = dec.assemble(mesh.xy, mesh.tri)
    xy, tri = mesh.xy, ops.tri
    # circumcentres
    a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    d = 2 * (a[:, 0] * (b[:, 1] - c[:, 1]) + b[:, 0] * (c[:, 1] - a[:, 1]) + c[:, 0] * (a[:, 1] - b[:, 1]))
    a2, b2, c2 = (a**2).sum(1), (b**2).sum(1), (c**2).sum(1)
    cc = np.stack([(a2 * (b[:, 1] - c[:, 1]) + b2 * (c[:, 1] - a[:, 1]) + c2 * (a[:, 1] - b[:, 1])) / d,
                   (a2 * (c[:, 0] - b[:, 0]) + b2 * (a[:, 0] - c[:, 0]) + c2 * (b[:, 0] - a[:, 0])) / d], 1)
    dual = {}
    for t, (i, j, k) in enumerate(tri):
        for u, v, o in ((i, j, k), (j, k, i), (k, i, j)):
            key = (min(u, v), max(u, v))
            mid = 0.5 * (xy[u] + xy[v])
            e = xy[v] - xy[u]
            nrm = np.array([-e[1], e[0]]) / np.linalg.norm(e)
            # signed distance from edge midpoint to circumcentre, positive toward the opposite vertex
            s = np.dot(cc[t] - mid, nrm) * np.sign(np.dot(xy[o] - mid, nrm))
            dual[key] = dual.get(key, 0.0) + s
    h1 = np.array([dual[(int(i), int(j))] / np.linalg.norm(xy[j] - xy[i]) for i, j in ops.edges])
    Kv = (ops.D0.T @ sp.diags(h1) @ ops.D0).toarray()
    np.testing.assert_allclose(ops.K.toarray(), Kv, atol=1e-12 * np.abs(Kv).max())


def test_stiffness_invariants():
    mesh = M.disk_mesh(4.0, 0.45, 3)
    ops = dec.assemble(mesh.xy, mesh.tri)
    K = ops.K
    n = ops.n
    assert abs(K - K.T).max() < 1e-14 * abs(K).max()
    assert np.abs(K @ np.ones(n)).max() < 1e-13 * abs(K).max()
    ev = np.linalg.eigvalsh(K.toarray())
    assert ev.min() > -1e-12 * ev.max()
    assert np.sum(ev < 1e-10 * ev.max()) == 1  # connected mesh: one zero mode


def test_stiffness_independent_of_edge_orientation():
    mesh = M.disk_mesh(2.0, 0.4, 9)
    ops = dec.assemble(mesh.xy, mesh.tri)
    rng = np.random.default_rng(0)
    flip = rng.uniform(size=ops.edges.shape[0]) < 0.5
    edges = ops.edges.copy()
    edges[flip] = edges[flip][:, ::-1]
    D0 = dec.incidence_d0(edges, ops.n)
    H1 = dec.whitney_hodge1(mesh.xy, ops.tri, edges)
    K2 = dec.stiffness(D0, H1)
    assert abs(K2 - ops.K).max() < 1e-14 * abs(ops.K).max()
    D1 = dec.incidence_d1(ops.tri, edges)
    assert np.count_nonzero((D1 @ D0).toarray()) == 0


def test_hodge0_sums_to_area():
    mesh = M.disk_mesh(5.0, 0.5, 2)
    ops = dec.assemble(mesh.xy, mesh.tri)
    from scipy.spatial import ConvexHull
    hull_area = ConvexHull(mesh.xy).volume  # the disk mesh is the convex hull of its points
    assert abs(ops.H0.sum() - hull_area) < 1e-12 * hull_area
    assert np.all(ops.H0 > 0)


def _interior(mesh, ops, margin):
    r = np.hypot(mesh.xy[:, 0], mesh.xy[:, 1])
    return r < mesh.meta["R"] - margin


def test_laplacian_kills_linear_functions_at_interior_vertices():
    mesh = M.disk_mesh(4.0, 0.35, 5)
    ops = dec.assemble(mesh.xy, mesh.tri)
    f = 0.7 * mesh.xy[:, 0] - 1.3 * mesh.xy[:, 1] + 2.0
    Lf = ops.L @ f
    inner = _interior(mesh, ops, 0.5)
    assert np.abs(Lf[inner]).max() < 1e-11


def test_laplacian_is_five_point_stencil_on_regular_grid():
    h = 0.25
    mesh = M.regular_grid_mesh(9, 8, h)
    ops = dec.assemble(mesh.xy, mesh.tri)
    nx, ny = 9, 8
    L = ops.L.toarray()
    for j in range(1, ny - 1):
        for i in range(1, nx - 1):
            p = j * nx + i
            row = np.zeros(nx * ny)
            row[p] = 4.0 / h**2
            for q in (p - 1, p + 1, p - nx, p + nx):
                row[q] = -1.0 / h**2
            np.testing.assert_allclose(L[p], row, atol=1e-12 / h**2)
    f = mesh.xy[:, 0] ** 2 + mesh.xy[:, 1] ** 2
    Lf = ops.L @ f
    X = mesh.xy
    inner = (X[:, 0] > 0.5 * h) & (X[:, 0] < (nx - 1.5) * h) & (X[:, 1] > 0.5 * h) & (X[:, 1] < (ny - 1.5) * h)
    np.testing.assert_allclose(Lf[inner], -4.0, atol=1e-11)  # L approximates minus the Laplacian


def test_neumann_disk_eigenvalue_converges_second_order():
    """Smallest nonzero Neumann eigenvalue of -Laplacian on the unit disk is j'_{1,1}^2."""
    exact = jnp_zeros(1, 1)[0] ** 2
    errs = []
    for h in (0.1, 0.05, 0.025):
        mesh = M.disk_mesh(1.0, h, 13, jitter=0.0)
        ops = dec.assemble(mesh.xy, mesh.tri)
        vals = spla.eigsh(ops.K, k=3, M=sp.diags(ops.H0), sigma=-1e-3, which="LM", return_eigenvectors=False)
        vals = np.sort(vals)
        assert abs(vals[0]) < 1e-10  # constant mode
        errs.append(abs(0.5 * (vals[1] + vals[2]) - exact))  # the (cos, sin) pair
    orders = [math.log(errs[k] / errs[k + 1], 2) for k in range(2)]
    assert errs[-1] < 0.01 * exact
    assert min(orders) > 1.6, (errs, orders)


def test_q_and_nonlinear_matrix():
    mesh = M.random_delaunay_mesh(50, 11)
    rng = np.random.default_rng(1)
    chi = rng.uniform(0.5, 2.0, mesh.n_tri)
    ops = dec.assemble(mesh.xy, mesh.tri, chi_tri=chi)
    Q = ops.Q.toarray()
    np.testing.assert_allclose(Q.sum(axis=1), 1.0, atol=1e-15)
    assert set(np.unique(Q[Q != 0]).round(15)) == {round(1 / 3, 15)}
    # M 1 equals the area-weighted mean of chi around each vertex
    chibar = np.zeros(ops.n)
    wsum = np.zeros(ops.n)
    for t, tri in enumerate(ops.tri):
        for p in tri:
            chibar[p] += chi[t] * ops.area[t]
            wsum[p] += ops.area[t]
    np.testing.assert_allclose(ops.M @ np.ones(ops.n), chibar / wsum, rtol=1e-13)
    ops_l = dec.assemble(mesh.xy, mesh.tri, chi_tri=chi, nl="lumped")
    np.testing.assert_allclose(ops_l.M.toarray(), np.diag(chibar / wsum), rtol=1e-13, atol=0)
    # H0 M = Q^T D Q is symmetric
    HM = (sp.diags(ops.H0) @ ops.M).toarray()
    np.testing.assert_allclose(HM, HM.T, atol=1e-15)


def test_nonlinear_matrix_row_on_regular_grid():
    """Interior vertex of the right-triangle grid: six triangles of equal area, so the
    Eq. 14 row is 1/3 on the diagonal and 1/9 on each of the six neighbours."""
    mesh = M.regular_grid_mesh(5, 5, 0.3)
    ops = dec.assemble(mesh.xy, mesh.tri)
    p = 2 * 5 + 2
    row = ops.M.toarray()[p]
    assert abs(row[p] - 1 / 3) < 1e-15
    off = np.delete(row, p)
    nz = off[off != 0]
    assert len(nz) == 6
    np.testing.assert_allclose(nz, 1 / 9, atol=1e-15)


def test_vertex_potential_is_area_weighted_mean():
    mesh = M.random_delaunay_mesh(40, 21)
    rng = np.random.default_rng(2)
    V = rng.uniform(-1, 1, mesh.n_tri)
    ops = dec.assemble(mesh.xy, mesh.tri, index_tri=V)
    num = np.zeros(ops.n)
    den = np.zeros(ops.n)
    for t, tri in enumerate(ops.tri):
        for p in tri:
            num[p] += V[t] * ops.area[t]
            den[p] += ops.area[t]
    np.testing.assert_allclose(ops.v, num / den, rtol=1e-13, atol=1e-15)
    ops2 = dec.assemble(mesh.xy, mesh.tri, index_tri=np.full(mesh.n_tri, 0.37))
    np.testing.assert_allclose(ops2.v, 0.37, rtol=1e-14)
    dn = rng.normal(size=ops.n)
    ops3 = dec.assemble(mesh.xy, mesh.tri, index_tri=V, dn=dn)
    np.testing.assert_allclose(ops3.v, ops.v + dn, rtol=1e-15)

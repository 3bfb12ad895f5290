"""DEC operators of the semi-discrete NLSE, assembled from their definitions (FP64).

Test infrastructure: see the package docstring for who may use it.

Every matrix here is built the way the paper defines it ("DEC computational
framework" through "DEC beam propagation", Eqs. 8-14), with no shortcuts:

* D0 from oriented edges, D1 from triangle boundaries (Stokes, Eq. 7 and the
  entry rule under it),
* H0 from barycentric dual areas, H0(V) and H0(chi) from per-triangle pulses,
* H1 by Galerkin integration of products of Whitney 1-form proxies
  (Eqs. 8-9) with an exact quadrature,
* K = D0^T H1 D0, L = H0^{-1} K,
* Q = (1/6)|D1||D0| and M = H0^{-1} Q^T D Q (Eqs. 13-14).

Readings (where the paper is silent or inconsistent):

* Sign of the stiffness term (Eq. 11 vs Eq. 1 and Table I).  Table I gives
  the Laplacian as ``-H0^{-1} D0^T H1 D0`` and Eq. 1 puts ``-p1 Laplacian`` on
  the right-hand side, so the linear operator used is
  ``H_lin = p1 L + beta4 L^2 - diag(v)`` with ``L = H0^{-1} K >= 0``
  (``L ~ -Laplacian``): diffraction against a guiding potential and a
  focusing Kerr term, consistent with the negative soliton eigenvalue the
  paper reports.  Eq. 11 as printed would flip the stiffness sign.
* ``p1`` is a parameter (the paper sets it to 1 in its normalisation, the
  workloads here use 1/2).
* The higher-order term is the cascaded product of Table I; its coefficient
  enters as ``+beta4 L^2``.
* ``xi`` in Eq. 9 is never defined; it is taken as 1 (scalar Laplacian).
* A per-vertex index perturbation ``dn`` is added to the vertex potential
  after the triangle-to-vertex averaging, with unit coupling.
* The nonlinear matrix has two forms: ``"dec"`` follows Eq. 14 (triangle-
  averaged intensity), ``"lumped"`` uses the area-weighted vertex mean of chi
  (the pointwise Kerr term of the continuous Eq. 1).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

__all__ = [
    "orient_ccw",
    "edge_list",
    "incidence_d0",
    "incidence_d1",
    "triangle_areas",
    "barycentric_gradients",
    "hodge0",
    "hodge0_pulse",
    "whitney_hodge1",
    "stiffness",
    "averaging_q",
    "Operators",
    "assemble",
]


def _signed_areas(xy, tri):
    a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    return 0.5 * ((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1]))


def orient_ccw(xy: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """Return the triangles listed counter-clockwise (the paper assumes a consistent
    CCW orientation of the 2-simplices, "DEC computational framework")."""
    tri = np.array(tri, dtype=np.int64, copy=True)
    s = _signed_areas(xy, tri)
    if np.any(s == 0.0):
        raise ValueError("degenerate triangle")
    flip = s < 0
    tri[flip, 1], tri[flip, 2] = tri[flip, 2].copy(), tri[flip, 1].copy()
    return tri


def edge_list(tri: np.ndarray) -> np.ndarray:
    """Unique edges ``[k1, k2]`` with the canonical orientation ``k1 < k2``."""
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    e.sort(axis=1)
    return np.unique(e, axis=0)


def incidence_d0(edges: np.ndarray, n_vert: int) -> sp.csr_matrix:
    """D0 (N1 x N0): +1 at the head vertex, -1 at the tail vertex of each edge."""
    n_e = edges.shape[0]
    rows = np.repeat(np.arange(n_e), 2)
    cols = edges.ravel()  # [tail, head] per edge
    vals = np.tile([-1.0, 1.0], n_e)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n_e, n_vert))


def _edge_ids(edges: np.ndarray, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Row of ``edges`` holding the undirected edge {u, v}; rows may carry either orientation."""
    n = int(edges.max()) + 1
    keys = np.minimum(edges[:, 0], edges[:, 1]).astype(np.int64) * n + np.maximum(edges[:, 0], edges[:, 1])
    order = np.argsort(keys)
    skeys = keys[order]
    q = np.minimum(u, v).astype(np.int64) * n + np.maximum(u, v)
    pos = np.searchsorted(skeys, q)
    pos = np.minimum(pos, len(skeys) - 1)
    if np.any(skeys[pos] != q):
        raise ValueError("edge not found")
    return order[pos]


def incidence_d1(tri: np.ndarray, edges: np.ndarray) -> sp.csr_matrix:
    """D1 (N2 x N1): +1 if the edge orientation [tail, head] agrees with the
    triangle's counter-clockwise traversal a->b->c->a, -1 otherwise."""
    n_t = tri.shape[0]
    u = np.concatenate([tri[:, 0], tri[:, 1], tri[:, 2]])
    v = np.concatenate([tri[:, 1], tri[:, 2], tri[:, 0]])
    rows = np.tile(np.arange(n_t), 3)
    cols = _edge_ids(edges, u, v)
    vals = np.where(edges[cols, 0] == u, 1.0, -1.0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n_t, edges.shape[0]))


def triangle_areas(xy: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """Unsigned areas |t|."""
    return np.abs(_signed_areas(xy, tri))


def barycentric_gradients(xy: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """Constant gradients of the barycentric coordinates, shape [T, 3, 2].

    lambda(x) solves [[x_a x_b x_c], [y_a y_b y_c], [1 1 1]] lambda = [x, y, 1];
    row i of the inverse matrix holds (d lambda_i/dx, d lambda_i/dy, const)."""
    P = np.empty((tri.shape[0], 3, 3))
    P[:, 0, :] = xy[tri, 0]
    P[:, 1, :] = xy[tri, 1]
    P[:, 2, :] = 1.0
    Pinv = np.linalg.inv(P)
    return Pinv[:, :, :2]


def hodge0(xy: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """Diagonal of H0: one third of the area of every triangle touching the vertex."""
    return hodge0_pulse(xy, tri, np.ones(tri.shape[0]))


def hodge0_pulse(xy: np.ndarray, tri: np.ndarray, f_tri: np.ndarray) -> np.ndarray:
    """Diagonal of H0(f) for a per-triangle pulse f: (1/3) sum_t f_t |t| over t containing p."""
    n = xy.shape[0]
    area = triangle_areas(xy, tri)
    out = np.zeros(n)
    for k in range(3):
        np.add.at(out, tri[:, k], f_tri * area / 3.0)
    return out


def whitney_hodge1(xy: np.ndarray, tri: np.ndarray, edges: np.ndarray, xi: float = 1.0) -> sp.csr_matrix:
    """Galerkin H1 (N1 x N1): [H1]_pq = integral of xi W_p . W_q (Eq. 9) with the
    Whitney 1-form proxy W_e = lambda_i grad lambda_j - lambda_j grad lambda_i for
    the oriented edge e = [i, j] (tail i, head j; Eq. 8).

    The integrand is a quadratic polynomial on each triangle, so the three-point
    edge-midpoint rule (weights |t|/3) integrates it exactly."""
    grads = barycentric_gradients(xy, tri)  # [T, 3, 2]
    area = triangle_areas(xy, tri)
    n_t = tri.shape[0]
    # barycentric coordinates at the three edge midpoints of a triangle
    qp = np.array([[0.5, 0.5, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5]])
    slots = np.array([[0, 1], [1, 2], [0, 2]])  # the three local edges by vertex slot
    t_idx = np.arange(n_t)
    W = np.zeros((n_t, 3, 3, 2))  # [triangle, local edge, quadrature point, component]
    edge_id = np.zeros((n_t, 3), dtype=np.int64)
    for e, (a, b) in enumerate(slots):
        # tail slot i and head slot j follow the edge's own orientation [tail, head]
        edge_id[:, e] = _edge_ids(edges, tri[:, a], tri[:, b])
        a_first = edges[edge_id[:, e], 0] == tri[:, a]
        i = np.where(a_first, a, b)
        j = np.where(a_first, b, a)
        gi = grads[t_idx, i]  # [T, 2]
        gj = grads[t_idx, j]
        for q in range(3):
            lam_i = qp[q][i][:, None]
            lam_j = qp[q][j][:, None]
            W[:, e, q] = lam_i * gj - lam_j * gi
    local = xi * (area / 3.0)[:, None, None] * np.einsum("teqd,tfqd->tef", W, W)
    rows = np.repeat(edge_id, 3, axis=1).ravel()
    cols = np.tile(edge_id, (1, 3)).ravel()
    n_e = edges.shape[0]
    return sp.csr_matrix((local.ravel(), (rows, cols)), shape=(n_e, n_e))


def pml_stretch(r: np.ndarray, r0: float, r1: float, sigma_max: float, m: float = 2.0):
    """Radial complex coordinate stretching of a perfectly matched layer beyond r0.

    r~(r) = r + i S(r), S(r) = integral_{r0}^{r} sigma, with the profile
    sigma(r) = sigma_max ((r - r0)/(r1 - r0))^m for r > r0 (0 inside).
    Returns the stretch factors s_r = dr~/dr = 1 + i sigma and s_t = r~/r."""
    r = np.asarray(r, dtype=np.float64)
    u = np.clip((r - r0) / (r1 - r0), 0.0, None)
    inside = r > r0
    sigma = np.where(inside, sigma_max * u**m, 0.0)
    S = np.where(inside, sigma_max * (r1 - r0) * u ** (m + 1) / (m + 1), 0.0)
    s_r = 1.0 + 1j * sigma
    s_t = 1.0 + 1j * np.divide(S, r, out=np.zeros_like(r), where=r > 0)
    return s_r, s_t


def pml_hodge_stars(xy, tri, edges, pml):
    """Complex-stretched Hodge stars of a radial PML (the paper proposes stretching
    the Hodge stars; the construction is ours).  In the stretched coordinates the
    Laplacian is (1/(s_r s_t)) div(Lambda grad), Lambda = (s_t/s_r) rr^T + (s_r/s_t) tt^T
    (r, t the radial and azimuthal unit vectors).  Per triangle, with the stretch
    evaluated at its centroid: H0 picks up the area factor s_r s_t and H1 is the
    Galerkin star of the Whitney proxies with the tensor Lambda (three-point rule,
    exact for a constant tensor).  Returns (H0 complex diagonal, H1 complex CSR)."""
    r0, r1, sigma_max = pml[:3]
    m = pml[3] if len(pml) > 3 else 2.0
    c = xy[tri].mean(axis=1)
    rc = np.hypot(c[:, 0], c[:, 1])
    s_r, s_t = pml_stretch(rc, r0, r1, sigma_max, m)
    rhat = np.where(rc[:, None] > 0, c / np.where(rc > 0, rc, 1.0)[:, None], np.array([1.0, 0.0]))
    that = np.stack([-rhat[:, 1], rhat[:, 0]], axis=1)
    Lam = (s_t / s_r)[:, None, None] * np.einsum("ti,tj->tij", rhat, rhat) + \
        (s_r / s_t)[:, None, None] * np.einsum("ti,tj->tij", that, that)
    area = triangle_areas(xy, tri)
    n = xy.shape[0]
    H0 = np.zeros(n, dtype=np.complex128)
    for k in range(3):
        np.add.at(H0, tri[:, k], area * s_r * s_t / 3.0)
    grads = barycentric_gradients(xy, tri)
    n_t = tri.shape[0]
    qp = np.array([[0.5, 0.5, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5]])
    slots = np.array([[0, 1], [1, 2], [0, 2]])
    t_idx = np.arange(n_t)
    W = np.zeros((n_t, 3, 3, 2))
    edge_id = np.zeros((n_t, 3), dtype=np.int64)
    for e, (a, b) in enumerate(slots):
        edge_id[:, e] = _edge_ids(edges, tri[:, a], tri[:, b])
        a_first = edges[edge_id[:, e], 0] == tri[:, a]
        i = np.where(a_first, a, b)
        j = np.where(a_first, b, a)
        gi = grads[t_idx, i]
        gj = grads[t_idx, j]
        for q in range(3):
            W[:, e, q] = qp[q][i][:, None] * gj - qp[q][j][:, None] * gi
    local = (area / 3.0)[:, None, None] * np.einsum("taqi,tij,tbqj->tab", W, Lam, W)
    rows = np.repeat(edge_id, 3, axis=1).ravel()
    cols = np.tile(edge_id, (1, 3)).ravel()
    n_e = edges.shape[0]
    return H0, sp.csr_matrix((local.ravel(), (rows, cols)), shape=(n_e, n_e))


def stiffness(D0: sp.csr_matrix, H1: sp.csr_matrix) -> sp.csr_matrix:
    """K = D0^T H1 D0 (the bracket of Eq. 11 without the potential)."""
    return (D0.T @ H1 @ D0).tocsr()


def averaging_q(D1: sp.csr_matrix, D0: sp.csr_matrix) -> sp.csr_matrix:
    """Q = (1/6)|D1||D0| (Eq. 13): vertex-to-triangle averaging."""
    return (abs(D1) @ abs(D0) / 6.0).tocsr()


@dataclass
class Operators:
    xy: np.ndarray
    tri: np.ndarray  # CCW
    edges: np.ndarray
    D0: sp.csr_matrix
    D1: sp.csr_matrix
    area: np.ndarray
    H0: np.ndarray  # diagonal
    H1: sp.csr_matrix
    K: sp.csr_matrix
    L: sp.csr_matrix  # H0^{-1} K  (approximates minus the Laplacian)
    v: np.ndarray  # vertex potential H0^{-1} H0(V) (+ dn)
    w: np.ndarray  # absorber strength per vertex
    chi_tri: np.ndarray
    Q: sp.csr_matrix
    QtDQ: sp.csr_matrix
    M: sp.csr_matrix  # nonlinear matrix
    p1: float
    beta4: float
    nl: str
    p3: float = 0.0  # coefficients of L^3 and L^4 (the general sum over n of p_n L^n)
    p4: float = 0.0
    nl_kind: str = "kerr"  # N(I): "kerr" I, "saturable" I/(1 + I/I_s), "cubic_quintic" I - s I^2
    nl_param: float = 0.0  # I_s or s

    @property
    def n(self) -> int:
        return self.xy.shape[0]

    def apply_L(self, x):
        return self.L @ x

    def apply_H(self, x):
        """H_lin x = p1 L x + beta4 L^2 x + p3 L^3 x + p4 L^4 x - v x (powers applied in turn)."""
        Lx = self.L @ x
        out = self.p1 * Lx - self.v * x
        t = Lx
        for c in (self.beta4, self.p3, self.p4):
            t = self.L @ t
            if c != 0.0:
                out = out + c * t
        return out

    def N(self, I):
        """Kerr response N(I) of the intensity I = |psi|^2 (Eq. 1's nonlinear term)."""
        if self.nl_kind == "kerr":
            return I
        if self.nl_kind == "saturable":
            return I / (1.0 + I / self.nl_param)
        return I - self.nl_param * I * I

    def apply_HT(self, x):
        """Transpose of H_lin (needed by the adjoint): p1 L^T x + beta4 L^T L^T x - v x."""
        LT = self.L.T
        LTx = LT @ x
        out = self.p1 * LTx - self.v * x
        if self.beta4 != 0.0:
            out = out + self.beta4 * (LT @ LTx)
        return out

    def dense_H(self):
        Ld = self.L.toarray()
        H = self.p1 * Ld - np.diag(self.v).astype(self.L.dtype)
        P = Ld
        for c in (self.beta4, self.p3, self.p4):
            P = P @ Ld
            if c != 0.0:
                H = H + c * P
        return H


def assemble(xy, tri, index_tri=None, absorber=None, chi_tri=None, p1=0.5, beta4=0.0, nl="dec",
             dn=None, pml=None, p3=0.0, p4=0.0, nl_kind="kerr", nl_param=0.0) -> Operators:
    """Assemble every operator of the semi-discrete ODE (Eqs. 10-14).

    Eq. 1 in full: ``p3``, ``p4`` add p3 L^3 + p4 L^4 to H_lin (beta4 is p2), and
    ``nl_kind`` replaces the Kerr response N(I) = I by the saturable
    I/(1 + I/I_s) or the cubic-quintic I - s I^2 (``nl_param`` = I_s or s).

    ``pml = (r0, r1, sigma_max[, m])`` replaces H0 and H1 inside L by the
    complex-stretched stars of ``pml_hodge_stars`` (L becomes complex; the
    potential, the nonlinear matrix and the power keep the real H0)."""
    xy = np.asarray(xy, dtype=np.float64)
    tri = orient_ccw(xy, np.asarray(tri))
    n = xy.shape[0]
    edges = edge_list(tri)
    D0 = incidence_d0(edges, n)
    D1 = incidence_d1(tri, edges)
    area = triangle_areas(xy, tri)
    H0 = hodge0(xy, tri)
    H1 = whitney_hodge1(xy, tri, edges)
    K = stiffness(D0, H1)
    if pml is None:
        L = (sp.diags(1.0 / H0) @ K).tocsr()
    else:
        H0p, H1p = pml_hodge_stars(xy, tri, edges, pml)
        L = (sp.diags(1.0 / H0p) @ stiffness(D0, H1p)).tocsr()
    V_tri = np.zeros(tri.shape[0]) if index_tri is None else np.asarray(index_tri, dtype=np.float64)
    v = hodge0_pulse(xy, tri, V_tri) / H0
    if dn is not None:
        v = v + np.asarray(dn, dtype=np.float64)
    w = np.zeros(n) if absorber is None else np.asarray(absorber, dtype=np.float64)
    chi = np.ones(tri.shape[0]) if chi_tri is None else np.asarray(chi_tri, dtype=np.float64)
    Q = averaging_q(D1, D0)
    QtDQ = (Q.T @ sp.diags(chi * area) @ Q).tocsr()
    if nl == "dec":
        M = (sp.diags(1.0 / H0) @ QtDQ).tocsr()
    elif nl == "lumped":
        M = sp.diags(hodge0_pulse(xy, tri, chi) / H0).tocsr()
    else:
        raise ValueError(f"unknown nonlinearity {nl!r}")
    if nl_kind not in ("kerr", "saturable", "cubic_quintic"):
        raise ValueError(f"unknown Kerr response {nl_kind!r}")
    return Operators(xy, tri, edges, D0, D1, area, H0, H1, K, L, v, w, chi, Q, QtDQ, M, float(p1), float(beta4), nl,
                     float(p3), float(p4), nl_kind, float(nl_param))

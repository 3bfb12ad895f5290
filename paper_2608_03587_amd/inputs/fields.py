"""Seeded launch fields, index profiles and absorber profiles sampled on a mesh.

Fields are sampled at the vertices (the de Rham map of a 0-form evaluates it
at the vertices, Eq. zerofrom).  Index profiles are returned *per triangle*,
evaluated at the centroid, because that is what the library's create call
takes (the paper assigns each triangle the potential at its centroid,
"Discrete Hodge star").  Absorber strengths are returned per vertex.
None of these functions apply any operator of the method.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "centroids",
    "gaussian",
    "elliptic_gaussian",
    "elliptic_vortex",
    "vortex_r",
    "add_multiplicative_noise",
    "gaussian_superposition",
    "step_index_tri",
    "parabolic_index_tri",
    "pcf_index_tri",
    "quadratic_absorber",
]


def centroids(xy: np.ndarray, tri: np.ndarray) -> np.ndarray:
    return xy[tri].mean(axis=1)


def gaussian(xy, amp=1.0, waist=1.0, centre=(0.0, 0.0), two_sigma=False):
    """``amp * exp(-|r-c|^2 / waist^2)``; with ``two_sigma`` the exponent is ``/(2 waist^2)``."""
    d2 = (xy[:, 0] - centre[0]) ** 2 + (xy[:, 1] - centre[1]) ** 2
    den = 2.0 * waist**2 if two_sigma else waist**2
    return (amp * np.exp(-d2 / den)).astype(np.complex128)


def _uv(xy, centre, theta):
    x = xy[:, 0] - centre[0]
    y = xy[:, 1] - centre[1]
    U = x * math.cos(theta) + y * math.sin(theta)
    V = -x * math.sin(theta) + y * math.cos(theta)
    return U, V


def elliptic_gaussian(xy, amp, wx, wy, theta, centre=(0.0, 0.0)):
    """Rotated, off-axis elliptic Gaussian ``A exp(-U^2/wx^2 - V^2/wy^2)`` (Eqs. 16-17)."""
    U, V = _uv(xy, centre, theta)
    return (amp * np.exp(-(U**2) / wx**2 - V**2 / wy**2)).astype(np.complex128)


def elliptic_vortex(xy, amp, wx, wy, theta, centre=(0.0, 0.0)):
    """Elliptic m=1 vortex ``A (U/wx + i V/wy) exp(-U^2/wx^2 - V^2/wy^2)`` (Eq. 18)."""
    U, V = _uv(xy, centre, theta)
    return (amp * (U / wx + 1j * V / wy) * np.exp(-(U**2) / wx**2 - V**2 / wy**2)).astype(np.complex128)


def vortex_r(xy, amp, width2):
    """``A r e^{i theta} exp(-r^2/width2)`` = ``A (x + i y) exp(-r^2/width2)``."""
    r2 = xy[:, 0] ** 2 + xy[:, 1] ** 2
    return (amp * (xy[:, 0] + 1j * xy[:, 1]) * np.exp(-r2 / width2)).astype(np.complex128)


def add_multiplicative_noise(u, rel, seed):
    """``u * (1 + rel (xi1 + i xi2)/sqrt2)`` with ``xi ~ N(0,1)`` per vertex."""
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal((2, u.shape[0]))
    return u * (1.0 + rel * (xi[0] + 1j * xi[1]) / math.sqrt(2.0))


def gaussian_superposition(xy, seed, n_terms=4, waist_range=(1.0, 3.0), centre_radius=2.0):
    """Sum of ``n_terms`` Gaussians with seeded waists, complex amplitudes
    (``|a| <= 1``, uniform phase) and centres uniform in a disk."""
    rng = np.random.default_rng(seed)
    u = np.zeros(xy.shape[0], np.complex128)
    for _ in range(n_terms):
        w = rng.uniform(*waist_range)
        a = rng.uniform(0.0, 1.0) * np.exp(1j * rng.uniform(0.0, 2 * math.pi))
        rr = centre_radius * math.sqrt(rng.uniform())
        ph = rng.uniform(0.0, 2 * math.pi)
        c = (rr * math.cos(ph), rr * math.sin(ph))
        u += a * gaussian(xy, 1.0, w, c)
    return u


def step_index_tri(xy, tri, r_core, contrast):
    """Per-triangle index potential: ``contrast`` where the centroid lies in the core."""
    c = centroids(xy, tri)
    return np.where(np.hypot(c[:, 0], c[:, 1]) < r_core, contrast, 0.0).astype(np.float64)


def parabolic_index_tri(xy, tri, r_core, peak):
    """Per-triangle graded-index potential ``peak (1 - r^2/r_core^2)`` inside the core, 0 outside."""
    c = centroids(xy, tri)
    r = np.hypot(c[:, 0], c[:, 1])
    return np.where(r < r_core, peak * (1.0 - (r / r_core) ** 2), 0.0).astype(np.float64)


def pcf_index_tri(xy, tri, hole_centres, hole_radius, contrast):
    """Per-triangle potential: ``contrast`` where the centroid lies in an air hole."""
    c = centroids(xy, tri)
    inside = np.zeros(len(c), bool)
    for cx, cy in hole_centres:
        inside |= np.hypot(c[:, 0] - cx, c[:, 1] - cy) < hole_radius
    return np.where(inside, contrast, 0.0).astype(np.float64)


def quadratic_absorber(xy, r_start, r_end, w_max):
    """Per-vertex absorber strength ``w_max ((r - r_start)/(r_end - r_start))^2`` for ``r > r_start``."""
    r = np.hypot(xy[:, 0], xy[:, 1])
    s = np.clip((r - r_start) / (r_end - r_start), 0.0, None)
    return (w_max * s**2).astype(np.float64)

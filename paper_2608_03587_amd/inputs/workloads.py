"""Synthetic workloads shaped like the paper's benchmarks.

The paper propagates analytic launch fields through a step-index fibre
(Table "Physical and computational parameters", Results).  Its meshes,
reference fields and supplementary notes are not available, so each workload
below is a seeded stand-in with stated sizes, in normalised units:

* ``plain_small``      disk R=10, ~4k vertices, Gaussian 0.8 exp(-r^2/2), uniform
                       index, no absorber, dz=1e-3, 200 steps.
* ``step_index``       graded disk R=40, ~250k vertices, core r<5 with contrast 1,
                       tilted elliptic Gaussian (waists 2, 4; 30 deg; amplitude 1.2),
                       absorber ring r>35 up to 0.5, dz=5e-4, 5000 steps.
* ``vortex_beta4``     disk R=60, ~1M vertices, A r e^{i theta} exp(-r^2/8) with 1%
                       noise, beta4 = 1e-3, absorber r>50, dz=2e-4, 10000 steps.
* ``batched_pcf``      8 photonic-crystal-fibre meshes of 20k-200k vertices, 32
                       Gaussian-superposition fields each, dz=1e-3, 2000 steps.
* ``adjoint_mmf``      disk R=50, ~500k vertices, parabolic core radius 25,
                       absorber r>45, overlap objective with an offset Gaussian
                       target, per-vertex index perturbation N(0, 1e-3),
                       dz=5e-4, 2000 steps (replica at ~20k vertices).

Every generator takes a scale knob so that tests can build small replicas with
the same structure.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import fields as F
from . import meshes as M

__all__ = [
    "Workload",
    "plain_small",
    "step_index",
    "vortex_beta4",
    "batched_pcf",
    "adjoint_mmf",
    "WORKLOADS",
]


@dataclass
class Workload:
    name: str
    mesh: M.Mesh
    index_tri: np.ndarray | None
    absorber: np.ndarray | None
    u0: np.ndarray  # complex128 [N] or [F, N]
    dz: float
    n_steps: int
    gamma: float = 1.0
    p1: float = 0.5
    beta4: float = 0.0
    chi_tri: np.ndarray | None = None
    extra: dict = field(default_factory=dict)

    @property
    def vertex_steps(self) -> float:
        f = 1 if self.u0.ndim == 1 else self.u0.shape[0]
        return float(self.mesh.n_vert) * f * self.n_steps


def _uniform_h_for(R: float, n_vert: float) -> float:
    # hex lattice density 2/(sqrt3 h^2) over the disk area
    return math.sqrt(math.pi * R * R * 2.0 / (math.sqrt(3.0) * n_vert))


def plain_small(n_vert: int = 4000, seed: int = 11, n_steps: int = 200) -> Workload:
    R = 10.0
    h = 0.301 if n_vert == 4000 else _uniform_h_for(R, n_vert)
    mesh = M.disk_mesh(R, h, seed)
    u0 = F.gaussian(mesh.xy, 0.8, 1.0, two_sigma=True)
    return Workload("plain_small", mesh, None, None, u0, dz=1e-3, n_steps=n_steps)


def step_index(n_vert: int = 250_000, seed: int = 21, n_steps: int = 5000, min_angle: float | None = None) -> Workload:
    # coarse replicas grade faster, so their ring transitions allow a smaller angle
    if min_angle is None:
        min_angle = 25.0 if n_vert >= 100_000 else 20.0
    mesh = M.graded_core_disk_mesh(R=40.0, r_core=5.0, h_core=0.05, h_max=0.4, target_vertices=n_vert, seed=seed,
                                   min_angle=min_angle)
    V = F.step_index_tri(mesh.xy, mesh.tri, 5.0, 1.0)
    w = F.quadratic_absorber(mesh.xy, 35.0, 40.0, 0.5)
    u0 = F.elliptic_gaussian(mesh.xy, 1.2, 2.0, 4.0, math.radians(30.0))
    return Workload("step_index", mesh, V, w, u0, dz=5e-4, n_steps=n_steps)


def vortex_beta4(n_vert: int = 1_000_000, seed: int = 31, n_steps: int = 10_000) -> Workload:
    R = 60.0
    h = 0.1143 if n_vert == 1_000_000 else _uniform_h_for(R, n_vert)
    mesh = M.disk_mesh(R, h, seed)
    u0 = F.add_multiplicative_noise(F.vortex_r(mesh.xy, 1.5, 8.0), 0.01, 32)
    w = F.quadratic_absorber(mesh.xy, 50.0, 60.0, 0.5)
    return Workload("vortex_beta4", mesh, None, w, u0, dz=2e-4, n_steps=n_steps, beta4=1e-3)


def batched_pcf(n_meshes: int = 8, fields_per_mesh: int = 32, n_min: int = 20_000, n_max: int = 200_000,
                n_steps: int = 2000) -> list[Workload]:
    R = 12.0
    radii = np.random.default_rng(40).uniform(0.30, 0.45, n_meshes)
    if n_meshes > 1:
        targets = n_min * (n_max / n_min) ** (np.arange(n_meshes) / (n_meshes - 1))
    else:
        targets = np.array([float(n_min)])
    out = []
    for i in range(n_meshes):
        h = _uniform_h_for(R, targets[i])
        # replicas coarser than the hole radius cannot keep 25 degrees on the hole rings
        mesh = M.pcf_mesh(h, float(radii[i]), 41 + i, R=R, min_angle=25.0 if targets[i] >= 19_000 else 15.0)
        V = F.pcf_index_tri(mesh.xy, mesh.tri, mesh.meta["hole_centres"], float(radii[i]), -0.45)
        w = F.quadratic_absorber(mesh.xy, 10.0, 12.0, 0.5)
        u0 = np.stack([F.gaussian_superposition(mesh.xy, 4000 + i * fields_per_mesh + f)
                       for f in range(fields_per_mesh)])
        out.append(Workload(f"batched_pcf[{i}]", mesh, V, w, u0, dz=1e-3, n_steps=n_steps))
    return out


def adjoint_mmf(n_vert: int = 500_000, seed: int = 51, n_steps: int = 2000) -> Workload:
    R = 50.0
    if n_vert == 500_000:
        h = 0.135
    elif n_vert == 20_000:
        h, seed = 0.673, 52
    else:
        h = _uniform_h_for(R, n_vert)
    mesh = M.disk_mesh(R, h, seed)
    V = F.parabolic_index_tri(mesh.xy, mesh.tri, 25.0, 1.0)
    w = F.quadratic_absorber(mesh.xy, 45.0, 50.0, 0.5)
    u0 = F.gaussian(mesh.xy, 1.0, 5.0)
    phase = np.random.default_rng(53).uniform(0.0, 2.0 * math.pi)
    target = F.gaussian(mesh.xy, 1.0, 3.0, centre=(4.0, 0.0)) * np.exp(1j * phase)
    dn = np.random.default_rng(54).normal(0.0, 1e-3, mesh.n_vert)
    return Workload("adjoint_mmf", mesh, V, w, u0, dz=5e-4, n_steps=n_steps,
                    extra={"target": target, "dn": dn, "checkpoint_every": int(math.ceil(math.sqrt(n_steps)))})


WORKLOADS = {
    "plain_small": plain_small,
    "step_index": step_index,
    "vortex_beta4": vortex_beta4,
    "batched_pcf": batched_pcf,
    "adjoint_mmf": adjoint_mmf,
}

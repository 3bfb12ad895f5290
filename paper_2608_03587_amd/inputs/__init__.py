"""Seeded synthetic inputs (meshes, launch fields, index and absorber profiles).

This subpackage holds no arithmetic of the propagation method itself; it is
shared by the CPU oracle tests and the GPU library's tests and benchmark.
"""
from .meshes import *  # noqa: F401,F403
from .fields import *  # noqa: F401,F403
from .workloads import *  # noqa: F401,F403

"""Property tests of mesh ingest and host assembly, and the same code under
AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, no device work).

* Random meshes (hypothesis): jittered hexagonal lattices of random size,
  jitter, shear and rotation, with the vertex order, the triangle order and
  each triangle's orientation shuffled, as an arbitrary mesher would hand
  them over.  The library's host assembly (a host-only handle) must equal the
  oracle's Whitney-Galerkin operators on every one of them.
* The host assembly compiled with g++ -fsanitize=address,undefined runs over
  valid meshes (checking the operators' invariants) and over malformed ones
  (out-of-range and repeated indices, zero area, unreferenced vertices,
  non-manifold and folded edges, non-finite or coincident coordinates), which
  it must refuse with the documented error codes.
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle import dec
from paper_2608_03587_amd import _binding as B
from paper_2608_03587_amd import api
from paper_2608_03587_amd.inputs import meshes as M
from paper_2608_03587_amd.inputs import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@settings(max_examples=30, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(nx=st.integers(3, 24), ny=st.integers(3, 24), jitter=st.floats(0.02, 0.3), angle=st.floats(0.0, 6.28),
       shear=st.floats(-0.6, 0.6), seed=st.integers(0, 2**31 - 1), nl=st.sampled_from(["dec", "lumped"]))
def test_host_assembly_equals_oracle_on_random_meshes(nx, ny, jitter, angle, shear, seed, nl):
    mesh = M.jittered_lattice_mesh(nx, ny, jitter, seed, angle=angle, shear=shear)
    rng = np.random.default_rng(seed)
    V = rng.normal(0.0, 0.5, mesh.n_tri)
    chi = rng.uniform(0.5, 1.5, mesh.n_tri)
    w = rng.uniform(0.0, 0.5, mesh.n_vert)
    m = api.Mesh(mesh.xy, mesh.tri, V, w, chi_tri=chi, host_only=True, nonlinearity=nl)
    got = m.export_operators()
    ref = dec.assemble(mesh.xy, mesh.tri, V, w, chi_tri=chi, nl=nl)
    n = mesh.n_vert
    K = sp.csr_matrix((got["K"], got["col"], got["row_ptr"]), shape=(n, n))
    Q = sp.csr_matrix((got["QtDQ"], got["col"], got["row_ptr"]), shape=(n, n))
    # jittered hull triangles are slivers whose cotangents reach ~1e3: the two forms
    # (closed-form cotangents, Galerkin integration) then agree to rounding of those
    # terms, not of the entry they sum to; a wrong formula would be off at O(1)
    assert abs(K - ref.K).max() <= 1e-11 * abs(ref.K).max()
    np.testing.assert_allclose(got["h0"], ref.H0, rtol=1e-13)
    np.testing.assert_allclose(got["v"], ref.v, rtol=1e-12, atol=1e-13)
    assert abs(sp.diags(1.0 / got["h0"]) @ Q - ref.M).max() <= 1e-12 * abs(ref.M).max()
    assert m.sizes()["n_edge"] == ref.edges.shape[0]
    m.close()


# ---- the host assembly under the sanitizers ----

def _record(xy, tri, expect):
    xy = np.ascontiguousarray(xy, dtype="<f8")
    tri = np.ascontiguousarray(tri, dtype="<i4")
    return struct.pack("<qqi", xy.shape[0], tri.shape[0], expect) + xy.tobytes() + tri.tobytes()


def _cases():
    out = []
    ok = 0
    # valid: a right triangle, a square, disks, graded and photonic-crystal meshes, shuffled lattices
    out.append(_record([[0, 0], [2, 0], [0, 1]], [[0, 1, 2]], ok))
    out.append(_record([[0, 0], [1, 0], [0, 1], [1, 1]], [[0, 1, 2], [2, 1, 3]], ok))
    for mesh in [M.disk_mesh(3.0, 0.4, 1), W.step_index(n_vert=20000, n_steps=1).mesh,
                 W.batched_pcf(n_meshes=1, fields_per_mesh=1, n_min=3000, n_steps=1)[0].mesh, M.wheel_disk_mesh()]:
        out.append(_record(mesh.xy, mesh.tri, ok))
    for seed in range(8):
        mesh = M.jittered_lattice_mesh(4 + 3 * seed, 5 + 2 * seed, 0.02 + 0.04 * seed, seed, angle=0.4 * seed, shear=0.1)
        out.append(_record(mesh.xy, mesh.tri, ok))
    # malformed
    sq = np.array([[0, 0], [1, 0], [0, 1], [1, 1], [2, 2.0]])
    good = np.array([[0, 1, 2], [1, 3, 2]])
    out.append(_record(sq[:4], [[0, 1, 7], [1, 3, 2]], B.EMESH))  # index out of range
    out.append(_record(sq[:4], [[0, 1, -1], [1, 3, 2]], B.EMESH))  # negative index
    out.append(_record(sq[:4], [[0, 1, 1], [1, 3, 2]], B.EMESH))  # repeated vertex
    out.append(_record(sq, good, B.EMESH))  # vertex 4 unreferenced
    out.append(_record([[0, 0], [1, 0], [2, 0], [0, 1]], [[0, 1, 2], [0, 1, 3]], B.EMESH))  # zero area
    out.append(_record([[0, 0], [1, 0], [0, 1], [0, -1], [1, 1]], [[0, 1, 2], [0, 1, 3], [0, 1, 4]], B.EMESH))
    out.append(_record([[0, 0], [1, 0], [0, 1], [0.2, 0.2]], [[0, 1, 2], [0, 1, 3]], B.EMESH))  # folded overlap
    out.append(_record([[0, 0], [1, np.nan], [0, 1]], [[0, 1, 2]], B.EINVAL))  # non-finite coordinate
    out.append(_record([[1, 1], [1, 1], [1, 1]], [[0, 1, 2]], B.EMESH))  # all coincident
    out.append(_record([[0, 0], [1, 0]], np.zeros((0, 3)), B.EINVAL))  # too small
    return out


@pytest.fixture(scope="module")
def sanitized_driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("sanitize")
    exe = str(d / "host_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
           os.path.join(ROOT, "paper_2608_03587_amd", "csrc", "assembly.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe, d


def test_host_assembly_under_address_and_undefined_behaviour_sanitizers(sanitized_driver):
    exe, d = sanitized_driver
    cases = d / "cases.bin"
    cases.write_bytes(b"".join(_cases()))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe, str(cases)], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-4000:])
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "0 mismatches" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]

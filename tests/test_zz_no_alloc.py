"""dec_bpm_propagate_noalloc (state buffers and flags in the library's static
device scratch, nothing allocated) against dec_bpm_propagate, through the C ABI.

Both run the same tile kernels with the same per-row arithmetic, so the
results must agree bitwise: two calls in a row on the full step-index mesh,
then on a smaller mesh (the scratch keeps the previous call's contents), in
the persistent launch and in one kernel per step, in both precisions, and on
a beta4 handle.  Handles beyond the scratch's size or without step tiles are
refused before any device work.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_2608_03587_amd import _binding as B
from paper_2608_03587_amd import api
from paper_2608_03587_amd.inputs import meshes as M
from paper_2608_03587_amd.inputs import workloads as W

pytestmark = pytest.mark.gpu


def _call(fn, m, field, w, n):
    code = fn(m.handle, ctypes.c_void_p(field.data_ptr()), float(w.dz), int(n), float(w.gamma),
              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return code


def _mesh(w, dtype):
    return api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, dtype=dtype, p1=w.p1, beta4=w.beta4)


def test_noalloc_equals_propagate():
    L = B.lib()
    tdt = {"c64": torch.complex64, "c128": torch.complex128}
    cases = [(W.step_index(), "c64", 300), (W.plain_small(), "c64", 200), (W.step_index(n_vert=20000), "c128", 120),
             (W.plain_small(), "c128", 200), (W.vortex_beta4(n_vert=20000), "c64", 60)]
    for w, dtype, n in cases:  # each case smaller than, or of another shape than, the one before
        m = _mesh(w, dtype)
        u0 = torch.from_numpy(w.u0).to("cuda", tdt[dtype])
        for fused in ((2,) if w.beta4 else (3, 2)):
            m.tuning = {"fused": fused}
            ref = u0.clone()
            assert _call(L.dec_bpm_propagate, m, ref, w, n) == B.OK, L.dec_bpm_last_error()
            for rep in range(2):  # the second call finds the first one's contents in the scratch
                got = u0.clone()
                assert _call(L.dec_bpm_propagate_noalloc, m, got, w, n) == B.OK, L.dec_bpm_last_error()
                torch.cuda.synchronize()
                m.check_finite()
                print(f"{w.name} N={m.n_vert} {dtype} fused={fused} call {rep}:",
                      "bitwise" if torch.equal(got, ref) else
                      f"rel {float(torch.linalg.norm(got - ref) / torch.linalg.norm(ref)):.3e}", flush=True)
                assert torch.equal(got, ref), (w.name, dtype, fused, rep)
        m.close()


def test_noalloc_refusals():
    L = B.lib()
    big = W.adjoint_mmf()  # 498k vertices: 2 x 498k x 16 bytes exceed the scratch in complex128
    m = _mesh(big, "c128")
    f = torch.from_numpy(big.u0).to("cuda", torch.complex128)
    keep = f.clone()
    assert _call(L.dec_bpm_propagate_noalloc, m, f, big, 3) == B.EINVAL
    assert b"static scratch" in L.dec_bpm_last_error()
    assert torch.equal(f, keep)
    m.close()
    wheel = M.wheel_disk_mesh()  # rows of 14 neighbours: no step tiles
    mw = api.Mesh(wheel.xy, wheel.tri, dtype="c64")
    g = torch.ones(wheel.n_vert, dtype=torch.complex64, device="cuda")
    w = W.Workload("wheel", wheel, None, None, None, dz=1e-3, n_steps=1)
    assert _call(L.dec_bpm_propagate_noalloc, mw, g, w, 2) == B.EINVAL
    mw.close()

"""CPU tests of the native library: it loads, exports every declared symbol,
assembles the same operators as the oracle (independent routes: closed-form
cotangents vs Whitney quadrature), and rejects bad input with the documented
codes before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import dec
from paper_2608_03587_amd import _binding as B
from paper_2608_03587_amd import api
from paper_2608_03587_amd.inputs import fields as F
from paper_2608_03587_amd.inputs import meshes as M
from paper_2608_03587_amd.inputs import workloads as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "dec_bpm.h")


def _declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dec_bpm_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    names = _declared_symbols()
    assert len(names) >= 25
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(B.SYMBOLS)
    assert b"gfx950" in lib.dec_bpm_version()


def test_binding_constants_match_the_header():
    """Every DEC_BPM_* enumerator and #define of the header has the value the
    Python binding uses (error codes, dtypes, responses, timing classes)."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    values = {m.group(1): int(m.group(2)) for m in re.finditer(r"\bDEC_BPM_([A-Z0-9_]+)\s*=\s*(-?\d+)", text)}
    values.update({m.group(1): int(m.group(2)) for m in re.finditer(r"#define\s+DEC_BPM_([A-Z0-9_]+)\s+\(?(-?\d+)\)?",
                                                                       text)})
    timing = {k: v for k, v in values.items() if k.startswith("K_") or k == "NUM_KERNELS"}
    assert len(timing) >= 14
    for name, v in timing.items():
        assert getattr(B, name) == v, name
    checked = len(timing)
    for name, v in values.items():
        if hasattr(B, name) and name not in timing:
            assert getattr(B, name) == v, name
            checked += 1
    assert checked >= 20


def _csr(ops):
    n = len(ops["h0"])
    return sp.csr_matrix((ops["K"], ops["col"], ops["row_ptr"]), shape=(n, n)), \
        sp.csr_matrix((ops["QtDQ"], ops["col"], ops["row_ptr"]), shape=(n, n))


@pytest.mark.parametrize("nl", ["dec", "lumped"])
def test_host_assembly_matches_oracle(nl):
    w = W.step_index(n_vert=6000, n_steps=1)
    rng = np.random.default_rng(0)
    chi = rng.uniform(0.5, 1.5, w.mesh.n_tri)
    m = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, chi_tri=chi, host_only=True, nonlinearity=nl)
    got = m.export_operators()
    ref = dec.assemble(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, chi_tri=chi, nl=nl)
    K, Q = _csr(got)
    assert abs(K - ref.K).max() < 1e-13 * abs(ref.K).max()
    np.testing.assert_allclose(got["h0"], ref.H0, rtol=1e-13)
    np.testing.assert_allclose(got["v"], ref.v, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(got["w"], ref.w, rtol=0, atol=0)
    M_lib = sp.diags(1.0 / got["h0"]) @ Q
    assert abs(M_lib - ref.M).max() < 1e-13 * abs(ref.M).max()
    s = m.sizes()
    assert s["n_edge"] == ref.edges.shape[0]
    assert s["nnz"] == ref.K.nnz


def test_spectral_radius_is_a_tight_upper_bound():
    mesh = M.disk_mesh(4.0, 0.4, 1)
    V = F.step_index_tri(mesh.xy, mesh.tri, 1.0, 1.0)
    m = api.Mesh(mesh.xy, mesh.tri, V, host_only=True, beta4=1e-3)
    ops = dec.assemble(mesh.xy, mesh.tri, V, beta4=1e-3)
    lam = np.linalg.eigvals(ops.dense_H())
    rho = np.abs(lam).max()
    r = m.spectral_radius()
    assert rho <= r <= 1.001 * rho
    # a large mesh uses Lanczos without reorthogonalisation: still within 2%
    w = W.plain_small()
    m2 = api.Mesh(w.mesh.xy, w.mesh.tri, host_only=True)
    ops2 = dec.assemble(w.mesh.xy, w.mesh.tri)
    top = spla.eigsh(ops2.K, k=1, M=sp.diags(ops2.H0), which="LA", return_eigenvectors=False)[0] * 0.5
    assert top <= m2.spectral_radius() <= 1.02 * top


def _expect(code, fn):
    with pytest.raises(api.DecBpmError) as e:
        fn()
    assert e.value.code == code, str(e.value)


def test_create_rejects_bad_meshes():
    xy = np.array([[0, 0], [1, 0], [0, 1], [1, 1], [2, 2.0]])
    good = np.array([[0, 1, 2], [1, 3, 2]])
    api.Mesh(xy[:4], good, host_only=True)  # fine
    _expect(B.EMESH, lambda: api.Mesh(xy[:4], np.array([[0, 1, 2], [1, 3, 7]]), host_only=True))  # out of range
    _expect(B.EMESH, lambda: api.Mesh(xy[:4], np.array([[0, 1, 1], [1, 3, 2]]), host_only=True))  # repeated
    _expect(B.EMESH, lambda: api.Mesh(xy, good, host_only=True))  # vertex 4 unreferenced
    col = np.array([[0, 0], [1, 0], [2, 0], [0, 1.0]])
    _expect(B.EMESH, lambda: api.Mesh(col, np.array([[0, 1, 2], [0, 1, 3]]), host_only=True))  # zero area
    # three triangles on one edge
    xy3 = np.array([[0, 0], [1, 0], [0.5, 1], [0.5, -1], [0.5, 2.0]])
    _expect(B.EMESH, lambda: api.Mesh(xy3, np.array([[0, 1, 2], [0, 3, 1], [0, 1, 4]]), host_only=True))
    # overlapping (folded) triangles traverse the shared edge in the same direction
    xyf = np.array([[0, 0], [1, 0], [0.5, 1], [0.5, 0.5]])
    _expect(B.EMESH, lambda: api.Mesh(xyf, np.array([[0, 1, 2], [0, 1, 3]]), host_only=True))
    bad = xy[:4].copy()
    bad[1, 0] = np.nan
    _expect(B.EINVAL, lambda: api.Mesh(bad, good, host_only=True))
    _expect(B.EINVAL, lambda: api.Mesh(xy[:4], good, absorber=np.array([0, -1.0, 0, 0]), host_only=True))
    _expect(B.EINVAL, lambda: api.Mesh(xy[:4], good, index_tri=np.array([0, np.inf]), host_only=True))
    _expect(B.EINVAL, lambda: api.Mesh(xy[:4], good, beta4=-1.0, host_only=True))


def test_orientation_is_fixed_by_create():
    mesh = M.disk_mesh(2.0, 0.5, 3)
    a = api.Mesh(mesh.xy, mesh.tri, host_only=True).export_operators()
    flipped = mesh.tri[:, [0, 2, 1]]
    b = api.Mesh(mesh.xy, flipped, host_only=True).export_operators()
    np.testing.assert_array_equal(a["col"], b["col"])
    np.testing.assert_allclose(a["K"], b["K"], rtol=0, atol=1e-15)


def test_raw_abi_null_and_struct_checks():
    lib = B.lib()
    h = ctypes.c_void_p()
    assert lib.dec_bpm_create(None, 3, None, 1, None, None, None, ctypes.byref(h)) == B.EINVAL
    assert b"NULL" in lib.dec_bpm_last_error()
    opt = B.Options()
    lib.dec_bpm_default_options(ctypes.byref(opt))
    opt.struct_size = 4
    xy = np.array([[0, 0], [1, 0], [0, 1.0]])
    tri = np.array([[0, 1, 2]], np.int32)
    rc = lib.dec_bpm_create(xy.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 3,
                            tri.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 1, None, None, ctypes.byref(opt),
                            ctypes.byref(h))
    assert rc == B.EINVAL
    assert lib.dec_bpm_propagate(None, None, 1e-3, 1, 1.0, None) == B.EINVAL


def test_host_only_handle_runs_every_check_then_reports_no_device():
    w = W.plain_small(n_vert=1000)
    m = api.Mesh(w.mesh.xy, w.mesh.tri, host_only=True)
    lib = B.lib()
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: every path below fails before device work
    rho = m.spectral_radius()
    assert lib.dec_bpm_propagate(m.handle, fake, 3.0 / rho, 10, 1.0, None) == B.EUNSTABLE
    assert b"stability" in lib.dec_bpm_last_error()
    assert lib.dec_bpm_propagate(m.handle, fake, 0.0, 10, 1.0, None) == B.EINVAL
    assert lib.dec_bpm_propagate(m.handle, fake, 1e-3, -1, 1.0, None) == B.EINVAL
    assert lib.dec_bpm_propagate(m.handle, ctypes.c_void_p((1 << 20) + 4), 1e-3, 1, 1.0, None) == B.EINVAL
    assert lib.dec_bpm_propagate(m.handle, fake, 1e-3, 10, float("nan"), None) == B.EINVAL
    assert lib.dec_bpm_propagate(m.handle, fake, 1e-3, 10, 1.0, None) == B.ENODEVICE
    assert lib.dec_bpm_propagate_unsplit(m.handle, fake, 3.0 / rho, 10, 1.0, None) == B.EUNSTABLE
    assert lib.dec_bpm_propagate_unsplit(m.handle, fake, 1e-3, 10, 1.0, None) == B.ENODEVICE
    acc, rej = ctypes.c_int64(7), ctypes.c_int64(7)
    lh, zr = ctypes.c_double(7.0), ctypes.c_double(7.0)
    ad = lib.dec_bpm_propagate_adaptive
    for args in ((-1.0, 1e-3, 1e-9, 1e-11, 100), (1.0, 0.0, 1e-9, 1e-11, 100), (1.0, 1e-3, -1.0, 1e-11, 100),
                 (1.0, 1e-3, 1e-9, 0.0, 100), (1.0, 1e-3, 1e-9, 1e-11, 0), (float("inf"), 1e-3, 1e-9, 1e-11, 100)):
        z_end, h0, rtol, atol, mx = args
        assert ad(m.handle, fake, z_end, h0, 1.0, rtol, atol, mx, None, None, None, None, None) == B.EINVAL, args
    assert ad(m.handle, None, 1.0, 1e-3, 1.0, 1e-9, 1e-11, 100, None, None, None, None, None) == B.EINVAL
    assert ad(m.handle, fake, 1.0, 1e-3, 1.0, 1e-9, 1e-11, 100, ctypes.byref(acc), ctypes.byref(rej),
              ctypes.byref(lh), ctypes.byref(zr), None) == B.ENODEVICE
    assert (acc.value, rej.value, lh.value, zr.value) == (0, 0, 0.0, 0.0)  # counters cleared on every call
    fm = lib.dec_bpm_find_mode
    for args in ((0.0, 1e-3, 1e-10, 10), (1.0, 0.0, 1e-10, 10), (1.0, 1e-3, -1.0, 10), (1.0, 1e-3, 1e-10, 0),
                 (float("nan"), 1e-3, 1e-10, 10)):
        power, dtau, tol, mx = args
        assert fm(m.handle, fake, power, dtau, 1.0, tol, mx, None, None, None, None) == B.EINVAL, args
    assert fm(m.handle, fake, 1.0, 3.0 / rho, 1.0, 1e-10, 10, None, None, None, None) == B.EUNSTABLE
    assert fm(m.handle, fake, 1.0, 1e-3, 1.0, 1e-10, 10, None, None, None, None) == B.ENODEVICE
    assert lib.dec_bpm_apply(m.handle, 0, fake, fake, None) == B.EINVAL  # x == y
    assert lib.dec_bpm_diagnostics(m.handle, fake, 1.0, None, None, None) == B.ENODEVICE
    size = ctypes.c_size_t()
    assert lib.dec_bpm_workspace_size(m.handle, 100, 0, ctypes.byref(size)) == B.OK
    assert size.value > 0
    assert lib.dec_bpm_forward_checkpointed(m.handle, fake, 1e-3, 100, 1.0, 0, fake, 16, None) == B.ENODEVICE
    t = B.Tuning()
    assert lib.dec_bpm_get_tuning(m.handle, ctypes.byref(t)) == B.OK
    assert t.block_size in (64, 128, 256, 512, 1024)
    assert t.fused == 0  # host-only handles have no tiles
    bad = B.Tuning(100, 1, 0, 256, 1)
    assert lib.dec_bpm_set_tuning(m.handle, ctypes.byref(bad)) == B.EINVAL


def test_workspace_size_grows_like_sqrt_n_checkpoints():
    w = W.plain_small(n_vert=1000)
    m = api.Mesh(w.mesh.xy, w.mesh.tri, host_only=True)
    vec = m.n_vert * 8
    s100 = m.workspace_size(100)  # 10 checkpoints + 10-step segment
    s10000 = m.workspace_size(10000)  # 100 + 100
    assert 20 * vec < s100 < 80 * vec
    assert s10000 < 12 * s100


def test_pml_host_assembly_matches_the_oracle():
    """The library's stretched stiffness (P1 form |t| grad^T Lambda grad, accumulated per
    triangle) and dual areas against the oracle's Whitney-Galerkin stretched stars; the
    entry points whose kernels apply a real L refuse a PML handle (the unsplit and
    adaptive integrators take it); bad layer options are refused."""
    import scipy.sparse as sp

    mesh = M.disk_mesh(6.0, 0.4, 9)
    pml = (4.0, 6.0, 1.5)
    m = api.Mesh(mesh.xy, mesh.tri, dtype="c128", host_only=True, pml=pml)
    ex = m.export_pml()
    ops = dec.assemble(mesh.xy, mesh.tri, pml=pml)
    H0p, H1p = dec.pml_hodge_stars(ops.xy, ops.tri, ops.edges, pml)
    Kp = (ops.D0.T @ H1p @ ops.D0).tocsr()
    n = mesh.n_vert
    K_lib = sp.csr_matrix((ex["Kp"], ex["col"], ex["row_ptr"]), shape=(n, n))
    assert abs(K_lib - Kp).max() < 1e-13 * abs(Kp).max()
    assert np.abs(ex["h0p"] - H0p).max() < 1e-13 * np.abs(H0p).max()
    # the real operators are exported unchanged
    assert np.abs(ex["h0"] - ops.H0).max() < 1e-13 * ops.H0.max()
    lib = B.lib()
    fake = ctypes.c_void_p(1 << 20)
    assert lib.dec_bpm_propagate_unsplit(m.handle, fake, 1e-3, 1, 1.0, None) == B.ENODEVICE  # takes a PML
    assert lib.dec_bpm_linear_step(m.handle, fake, 1e-3, None) == B.EINVAL
    assert lib.dec_bpm_propagate(m.handle, fake, 1e-3, 1, 1.0, None) == B.ENODEVICE
    plain = api.Mesh(mesh.xy, mesh.tri, dtype="c128", host_only=True)
    assert lib.dec_bpm_export_pml(plain.handle, None, None) == B.EINVAL
    for bad in ((0.0, 6.0, 1.0), (5.0, 4.0, 1.0), (4.0, 6.0, -1.0)):
        with pytest.raises(api.DecBpmError):
            api.Mesh(mesh.xy, mesh.tri, dtype="c128", host_only=True, pml=bad)
    with pytest.raises(api.DecBpmError):
        api.Mesh(mesh.xy, mesh.tri, dtype="c128", host_only=True, pml=pml, beta4=1e-3)


def test_general_operator_sum_and_responses_on_the_host():
    """L^3 and L^4 enter the stability bound (Lanczos of the symmetrised sum against the
    oracle's dense spectrum); bad response options are refused; entry points written for
    the Kerr response and terms up to L^2 refuse the general handles."""
    mesh = M.disk_mesh(4.0, 0.35, 3)
    p3, p4 = -2e-3, 4e-4
    m = api.Mesh(mesh.xy, mesh.tri, dtype="c128", host_only=True, p3=p3, p4=p4)
    ops = dec.assemble(mesh.xy, mesh.tri, p3=p3, p4=p4)
    rho = np.abs(np.linalg.eigvals(ops.dense_H())).max()
    assert rho <= m.spectral_radius() <= 1.02 * rho
    lib = B.lib()
    fake = ctypes.c_void_p(1 << 20)
    assert lib.dec_bpm_propagate_unsplit(m.handle, fake, 1e-4, 1, 1.0, None) == B.EINVAL
    assert lib.dec_bpm_propagate(m.handle, fake, 1e-4, 1, 1.0, None) == B.ENODEVICE
    assert lib.dec_bpm_apply(m.handle, B.OP_H, fake, ctypes.c_void_p(1 << 21), None) == B.EINVAL
    s = api.Mesh(mesh.xy, mesh.tri, dtype="c64", host_only=True, response="saturable", response_param=2.0)
    assert lib.dec_bpm_find_mode(s.handle, fake, 1.0, 1e-3, 1.0, 1e-8, 10, None, None, None, None) == B.EINVAL
    for kw in ({"response": "saturable", "response_param": 0.0}, {"response": "cubic_quintic", "response_param": -1.0},
               {"p3": float("inf")}, {"response": "saturable", "response_param": 1.0, "pml": (3.0, 4.0, 1.0)}):
        with pytest.raises(api.DecBpmError):
            api.Mesh(mesh.xy, mesh.tri, dtype="c64", host_only=True, **kw)


def test_batch_layout_with_uneven_field_counts():
    """A batch of host-only meshes with different field counts per mesh: the packed size
    is sum_m n_m F_m and the Python layout (offsets, pack, unpack) follows the header's
    field-minor, per-mesh layout; bad counts are refused before any device work, and a
    host-only batch refuses to propagate."""
    import torch

    ms = [api.Mesh(M.disk_mesh(2.0 + k, 0.5, 3 + k).xy, M.disk_mesh(2.0 + k, 0.5, 3 + k).tri, host_only=True)
          for k in range(3)]
    counts = [1, 5, 3]
    b = api.Batch(ms, counts)
    assert b.n_elems == sum(m.n_vert * f for m, f in zip(ms, counts))
    assert list(b.offsets) == list(np.cumsum([0] + [m.n_vert * f for m, f in zip(ms, counts)]))
    fields = [torch.arange(f * m.n_vert, dtype=torch.float64).reshape(f, m.n_vert).to(torch.complex128) + 1000 * k
              for k, (m, f) in enumerate(zip(ms, counts))]
    packed = b.pack(fields)
    assert packed.numel() == b.n_elems
    # element (mesh m, vertex i, field f) at base_m + i F_m + f
    m, i, f = 1, 7, 3
    assert packed[b.offsets[m] + i * counts[m] + f] == fields[m][f, i]
    for a, c in zip(b.unpack(packed), fields):
        assert torch.equal(a, c)
    assert B.lib().dec_bpm_batch_propagate(b._h, ctypes.c_void_p(16), 1e-3, 1, 1.0, None) == B.ENODEVICE
    for bad in ([0, 1, 1], [1, -2, 1], [1, 5000, 1]):
        with pytest.raises(api.DecBpmError) as e:
            api.Batch(ms, bad)
        assert e.value.code == B.EINVAL
    arr = (ctypes.c_void_p * 3)(*[x.handle.value for x in ms])
    out = ctypes.c_void_p()
    assert B.lib().dec_bpm_batch_create(arr, 3, None, ctypes.byref(out)) == B.EINVAL
    b.close()
    b.close()  # idempotent

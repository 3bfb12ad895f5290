"""GPU parity at the workloads' full sizes and full (or largest well-posed) lengths.

Each test runs the HIP library through the C ABI in the launch configuration
the benchmark times (autotuned) and compares with a stored FP64 oracle field
written by ``tests/golden/make_references.py`` (which calls only the oracle).
Gates: relative L2 of the complex vertex vector <= 1e-10 in complex128 and
<= 1e-4 in complex64.  Besides the global norm, every comparison checks the
largest per-vertex error against the largest reference amplitude and the
error restricted to the absorber ring, the rim (boundary vertices) and the
rows on a tile boundary of the launch's tiling (relative to the region's own
norm, or as an error density against the whole field's), so a defect
confined to few rows cannot hide in a large mesh.

Where a launch is supercritical, rounding differences grow along z.  The
reference file records, from the oracle alone, how far a copy of the run
perturbed after every step by one unit roundoff of the precision drifts from
the unperturbed run (delta(z)), and holds the oracle's field at the final z
(complex128 comparisons) and at the largest probed z with delta64 below a
tenth of the complex64 gate (complex64 comparisons).  Each test prints the z
it compares at and delta there.
"""
import importlib.util
import math
import os
import sys

import numpy as np
import pytest
import torch

from oracle import dec
from oracle import stepper as S
from paper_2608_03587_amd import api
from paper_2608_03587_amd.inputs import workloads as W

pytestmark = pytest.mark.gpu

GATE = {"c128": 1e-10, "c64": 1e-4}
DEV = "cuda"
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

_spec = importlib.util.spec_from_file_location("make_references", os.path.join(GOLD, "make_references.py"))
REF = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(REF)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV, {"c64": torch.complex64, "c128": torch.complex128}[dtype])


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.complex128)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def reference(name, *inputs):
    """The stored oracle result, after checking that the seeded generators rebuilt its inputs."""
    z = np.load(os.path.join(GOLD, f"ref_{name}.npz"))
    assert str(z["inputs_sha256"]) == REF.digest(*inputs), f"inputs of {name} differ from the stored reference's"
    return z


def lib_mesh(w, dtype, **kw):
    return api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, chi_tri=w.chi_tri, dtype=dtype, p1=w.p1,
                    beta4=w.beta4, **kw)


def edges(tri):
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    return np.unique(np.sort(e, axis=1), axis=0)


def regions(w, m):
    """Vertex masks: absorber ring, rim, and rows with a neighbour in another tile."""
    out = {}
    if w.absorber is not None:
        out["absorber"] = np.asarray(w.absorber) > 0
    r = np.hypot(w.mesh.xy[:, 0], w.mesh.xy[:, 1])
    out["rim"] = r > r.max() - 1e-9  # the boundary ring's points lie on the circle
    tile, ts = m.vertex_tiles()
    if ts > 0:
        e = edges(w.mesh.tri)
        cut = tile[e[:, 0]] != tile[e[:, 1]]
        mask = np.zeros(w.mesh.n_vert, bool)
        mask[e[cut].ravel()] = True
        out["tile_boundary"] = mask
    return out


def compare(tag, got, ref, gate, masks):
    """Global relative L2, largest per-vertex error over the largest amplitude, and for
    each region its error measured two ways: relative to the region's own reference
    norm, and as an error density (its squared error per row against the whole field's
    allowance per row, gate^2 |ref|^2 / N).  A region passes if either is within the
    gate: a defect confined to a region raises both, while a region where the field is
    tiny (an absorber the beam has not reached) can only show rounding-level
    differences of larger relative size."""
    err = rel(got, ref)
    vmax = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    n = got.shape[0]
    parts = {}
    for k, mk in masks.items():
        if not mk.any() or np.linalg.norm(ref[mk]) == 0:
            continue
        d = np.linalg.norm(got[mk] - ref[mk])
        parts[k] = (d / np.linalg.norm(ref[mk]), d / np.linalg.norm(ref) * np.sqrt(n / mk.sum()))
    say(f"  {tag}: rel {err:.3e}, max vertex {vmax:.3e}, " +
        ", ".join(f"{k} {a:.3e} (density {b:.3e}, {int(masks[k].sum())} rows)" for k, (a, b) in parts.items()))
    assert err <= gate, (tag, err)
    assert vmax <= gate, (tag, vmax)
    for k, (a, b) in parts.items():
        assert min(a, b) <= gate, (tag, k, a, b)
    return err


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")


_W = {}


def workload(name):
    if name not in _W:
        _W[name] = {"step_index": W.step_index, "vortex_beta4": W.vortex_beta4}[name]()
    return _W[name]


def stored(z, dtype):
    """(steps, oracle field, delta there): the final z for complex128, the largest
    well-posed z for complex64."""
    if dtype == "c128":
        n, ref, key = int(z["s_end"]), z["psi_end"], "delta128"
    else:
        n, ref, key = int(z["s64"]), z["psi64"].astype(np.complex128), "delta64"
    k = list(z["probe_steps"]).index(n)
    return n, ref, float(z[key][k])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_step_index_full_length(dtype):
    """The 249k-vertex step-index launch (supercritical, power 18.1): complex128 over all
    5000 steps (z = 2.5), complex64 to the largest well-posed z, against the oracle."""
    w = workload("step_index")
    z = reference("step_index", w.mesh.xy, w.mesh.tri, w.u0)
    n, ref, delta = stored(z, dtype)
    say(f"step_index {dtype}: {n} of {w.n_steps} steps (oracle rounding probe delta there {delta:.3g})")
    if dtype == "c128":
        assert n == w.n_steps  # the whole length
    m = lib_mesh(w, dtype)
    m.autotune(w.dz, w.gamma)
    f = dev(w.u0, dtype)
    m.propagate(f, w.dz, n, w.gamma)
    m.check_finite()
    say(f"  launch {m.tuning}")
    compare(f"{dtype} z={n * w.dz:g}", host(f), ref, GATE[dtype], regions(w, m))


def test_persistent_launch_bitwise_over_the_full_length():
    """The persistent launch (all 5000 steps, the prologue and the last half step in one
    launch) gives the one-kernel-per-step path's bits on the full mesh."""
    w = workload("step_index")
    m = lib_mesh(w, "c64")
    outs = {}
    for fused in (3, 2):
        m.tuning = {"fused": fused, "tile_block": 1024}
        assert m.tuning["fused"] == fused
        f = dev(w.u0, "c64")
        m.propagate(f, w.dz, w.n_steps, w.gamma)
        m.check_finite()
        outs[fused] = host(f)
    assert m.time_kernels(w.dz, w.gamma, reps=10)["persist"]["ms"] > 0  # the persistent path was live
    say("  persistent vs one kernel per step:", "bitwise" if np.array_equal(outs[3], outs[2]) else
        f"rel {rel(outs[3], outs[2]):.3e}")
    assert np.array_equal(outs[3], outs[2])


def test_vortex_beta4_well_posed_length():
    """The 1M-vertex optical vortex with the beta4 L^2 term (power 113, filamenting),
    complex64, to the largest z the oracle's conditioning allows (the stored reference
    records how far the oracle run went)."""
    w = workload("vortex_beta4")
    z = reference("vortex_beta4", w.mesh.xy, w.mesh.tri, w.u0)
    n = int(z["s64"])
    say(f"vortex_beta4 c64: {n} of {w.n_steps} steps; conditioning limit crossed: {bool(z['crossed64'])}")
    m = lib_mesh(w, "c64")
    m.autotune(w.dz, w.gamma)
    f = dev(w.u0, "c64")
    m.propagate(f, w.dz, n, w.gamma)
    m.check_finite()
    say(f"  launch {m.tuning}")
    compare(f"c64 z={n * w.dz:g}", host(f), z["psi64"].astype(np.complex128), GATE["c64"], regions(w, m))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batched_pcf_full_length(dtype):
    """The full batched workload (8 photonic-crystal-fibre meshes, 32 fields each) in the
    bench's launch configuration: field 0 of each mesh against the oracle at the
    largest well-posed z of that field (complex64: all eight meshes; complex128: the
    four smaller meshes, at the final z), advancing the batch from one comparison point
    to the next."""
    ws = W.batched_pcf()
    F = ws[0].u0.shape[0]
    refs = [reference(f"batched_pcf{i}", x.mesh.xy, x.mesh.tri, x.u0[0]) for i, x in enumerate(ws)]
    key = "s_end" if dtype == "c128" else "s64"
    stops = {i: int(r[key]) for i, r in enumerate(refs) if key in r}
    say(f"batched {dtype}: compare mesh -> step {stops}")
    meshes = [lib_mesh(x, dtype) for x in ws]
    batch = api.Batch(meshes, F)
    packed = batch.pack([dev(x.u0, dtype) for x in ws])
    batch.autotune(ws[0].dz, 1.0)
    say(f"  launch {batch.tuning}")
    done = 0
    for s in sorted(set(stops.values())):
        if s > done:
            batch.propagate(packed, ws[0].dz, s - done, 1.0)
            done = s
        outs = batch.unpack(packed)
        for i, si in stops.items():
            if si != s:
                continue
            n, ref, delta = stored(refs[i], dtype)
            got = host(outs[i][0].contiguous())
            compare(f"mesh {i} ({ws[i].mesh.n_vert} vertices) field 0, z={s * ws[i].dz:g} (delta {delta:.2g})", got,
                    ref, GATE[dtype], regions(ws[i], meshes[i]))
    batch.check_finite()


def test_batched_equals_plain_on_the_full_workload():
    """Every field of the full batched workload equals a plain propagate of that field to
    1e-6 (complex64, 100 steps): sampled fields of the smallest and the largest mesh."""
    ws = W.batched_pcf()
    F = ws[0].u0.shape[0]
    n = 100
    meshes = [lib_mesh(x, "c64") for x in ws]
    batch = api.Batch(meshes, F)
    packed = batch.pack([dev(x.u0, "c64") for x in ws])
    batch.autotune(ws[0].dz, 1.0)
    batch.propagate(packed, ws[0].dz, n, 1.0)
    outs = batch.unpack(packed)
    for k in (0, len(ws) - 1):
        meshes[k].autotune(ws[k].dz, 1.0)
        for f in (0, 7, F - 1):
            single = dev(ws[k].u0[f], "c64")
            meshes[k].propagate(single, ws[k].dz, n, 1.0)
            err = rel(host(outs[k][f].contiguous()), host(single))
            say(f"  mesh {k} field {f}: batched vs plain {err:.3e}")
            assert err <= 1e-6, (k, f, err)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adjoint_replica_full_length(dtype):
    """The multimode-fibre adjoint on its 20k-vertex replica over all 2000 steps with
    45-step checkpoints: the objective and the gradients with respect to the launch field
    and the per-vertex index perturbation against the oracle's FP64 adjoint (every state
    kept)."""
    w = W.adjoint_mmf(n_vert=20_000)
    dn = w.extra["dn"]
    z = reference("adjoint_replica", w.mesh.xy, w.mesh.tri, w.u0, w.extra["target"], dn)
    n, every = w.n_steps, w.extra["checkpoint_every"]
    m = lib_mesh(w, dtype)
    m.autotune(w.dz, w.gamma)
    m.set_index_perturbation(torch.from_numpy(dn).to(DEV))
    u = dev(w.u0, dtype)
    wsp = torch.empty(m.workspace_size(n, every), dtype=torch.uint8, device=DEV)
    m.forward_checkpointed(u, w.dz, n, w.gamma, wsp, every)
    tgt = dev(w.extra["target"], dtype)
    c = m.overlap(tgt, u)
    J = abs(c) ** 2
    h0 = torch.from_numpy(m.export_operators()["h0"]).to(DEV)
    gout = (2 * c * h0 * tgt.to(torch.complex128)).to(u.dtype)
    g0, gdn = m.adjoint(gout, w.dz, n, w.gamma, wsp, every)
    eJ = abs(J - float(z["J"])) / float(z["J"])
    eu = rel(host(g0), z["g_u0"])
    en = rel(gdn.cpu().numpy(), z["g_dn"])
    say(f"adjoint replica {dtype}: J {J:.10e} (oracle {float(z['J']):.10e}, rel {eJ:.2e}), "
        f"grad u0 rel {eu:.3e}, grad dn rel {en:.3e}")
    tol = GATE[dtype]
    assert eJ <= tol and eu <= tol and en <= tol


def test_adjoint_full_size_eight_directions():
    """The full 498k-vertex adjoint workload over all 2000 steps (45-step checkpoints):
    central differences of the library's complex128 forward along 8 random directions
    (4 of the launch field, 4 of the index perturbation) against the complex64 adjoint's
    directional derivatives, to 1e-4."""
    w = W.adjoint_mmf()
    n, every = w.n_steps, w.extra["checkpoint_every"]
    dn0 = torch.from_numpy(w.extra["dn"]).to(DEV)
    say("adjoint full size", w.mesh.n_vert, n)
    m64 = lib_mesh(w, "c64")
    m64.autotune(w.dz, w.gamma)
    u0 = dev(w.u0, "c64").requires_grad_(True)
    dn = dn0.clone().requires_grad_(True)
    tgt64 = dev(w.extra["target"], "c64")
    h0 = torch.from_numpy(m64.export_operators()["h0"]).to(DEV)
    u = api.propagate_with_grad(m64, u0, dn, w.dz, n, w.gamma, every=every)
    c = (h0 * tgt64.conj().to(torch.complex128) * u.to(torch.complex128)).sum()
    (c.conj() * c).real.backward()
    g_u, g_n = u0.grad.detach().to(torch.complex128), dn.grad.detach()
    del m64
    m = lib_mesh(w, "c128")
    m.autotune(w.dz, w.gamma)
    tgt = dev(w.extra["target"], "c128")
    base = dev(w.u0, "c128")

    def J(x, d):
        m.set_index_perturbation(d)
        f = x.clone()
        m.propagate(f, w.dz, n, w.gamma)
        cc = (h0 * tgt.conj() * f).sum()
        return float((cc.conj() * cc).real)

    rng = np.random.default_rng(8)
    fds, ans = {"field": [], "index": []}, {"field": [], "index": []}
    for k in range(8):
        if k < 4:
            d = dev(rng.normal(size=m.n_vert) + 1j * rng.normal(size=m.n_vert), "c128")
            eps = 1e-6
            fd = (J(base + eps * d, dn0) - J(base - eps * d, dn0)) / (2 * eps)
            an = float((g_u.conj() * d).real.sum())
        else:
            e = torch.from_numpy(rng.normal(size=m.n_vert)).to(DEV)
            eps = 1e-4
            fd = (J(base, dn0 + eps * e) - J(base, dn0 - eps * e)) / (2 * eps)
            an = float((g_n * e).sum())
        kind = "field" if k < 4 else "index"
        fds[kind].append(fd)
        ans[kind].append(an)
        say(f"  direction {k} ({kind}): central difference {fd:.8e}, complex64 adjoint {an:.8e}, "
            f"rel {abs(fd - an) / abs(fd):.2e}")
    # the gradient's error over the sampled directions: one direction's relative error is
    # ill-conditioned when its projection happens to be small
    for kind in fds:
        a, b = np.array(ans[kind]), np.array(fds[kind])
        err = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        say(f"  {kind} directions: rel {err:.2e}")
        assert err <= 1e-4, (kind, err)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_degree_fourteen_vertices(dtype):
    """A disk whose two wheel centres have 14 neighbours (the most the 25-degree angle
    bound allows): rows wider than the tile kernels' 12 take the unbounded row gather,
    the tile paths are refused, and the result matches the oracle."""
    from paper_2608_03587_amd.inputs import fields as Fd
    from paper_2608_03587_amd.inputs import meshes as Mm

    mesh = Mm.wheel_disk_mesh()
    deg = np.bincount(edges(mesh.tri).ravel())
    assert deg.max() == 14 and mesh.meta["min_angle_deg"] >= 25.0
    w = W.Workload("wheel", mesh, None, Fd.quadratic_absorber(mesh.xy, 8.0, 10.0, 0.5),
                   Fd.gaussian(mesh.xy, 0.9, 1.5, centre=(0.5, 0.3)) * np.exp(1j * mesh.xy[:, 0]), dz=1e-3,
                   n_steps=150)
    ops = dec.assemble(w.mesh.xy, w.mesh.tri, None, w.absorber, p1=w.p1)
    ref = S.propagate(w.u0, ops, w.dz, w.n_steps, w.gamma)
    m = lib_mesh(w, dtype)
    for fused in (0, 1, 2, 3):
        m.tuning = {"fused": fused}
        assert m.vertex_tiles()[1] == -1, fused  # no tile set: every mode runs the row kernels
    kt = m.time_kernels(w.dz, w.gamma, reps=5)
    assert kt["stage"]["ms"] > 0 and kt["step"]["ms"] == 0 and kt["persist"]["ms"] == 0
    with pytest.raises(api.DecBpmError):
        m.propagate_unsplit(dev(w.u0, dtype), w.dz, 2, w.gamma)
    f = dev(w.u0, dtype)
    m.propagate(f, w.dz, w.n_steps, w.gamma)  # requested mode 3, runs the five row kernels per step
    m.check_finite()
    wide = deg > 12
    masks = {"degree_14": wide, "their_neighbours": np.isin(np.arange(mesh.n_vert),
                                                            edges(mesh.tri)[np.any(wide[edges(mesh.tri)], 1)])}
    compare(f"{dtype} wheel", host(f), ref, GATE[dtype], masks)

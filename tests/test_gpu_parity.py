"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Gates: relative L2 error of the complex vertex vector <= 1e-10 in complex128
and <= 1e-4 in complex64 at the final z; kernel-level checks are tighter.
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import adjoint as OA, dec, diagnostics as D, soliton as SO, stepper as S, unsplit as US
from paper_2608_03587_amd import _binding as B
from paper_2608_03587_amd import api
from paper_2608_03587_amd.inputs import fields as F
from paper_2608_03587_amd.inputs import meshes as M
from paper_2608_03587_amd.inputs import workloads as W

pytestmark = pytest.mark.gpu

GATE = {"c128": 1e-10, "c64": 1e-4}
KERNEL_TOL = {"c128": 1e-13, "c64": 2e-6}
DEV = "cuda"


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


_CACHE = {}


def case(name, **kw):
    key = (name, tuple(sorted(kw.items())))
    if key not in _CACHE:
        if name == "plain_small":
            w = W.plain_small(**kw)
        elif name == "step_index":
            w = W.step_index(**kw)
        elif name == "vortex":
            w = W.vortex_beta4(**kw)
        elif name == "adjoint":
            w = W.adjoint_mmf(**kw)
        else:
            raise KeyError(name)
        _CACHE[key] = w
    return _CACHE[key]


def oracle_ops(w, nl="dec", dn=None):
    return dec.assemble(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, chi_tri=w.chi_tri, p1=w.p1, beta4=w.beta4,
                        nl=nl, dn=dn)


def lib_mesh(w, dtype, nl="dec", **kw):
    return api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, chi_tri=w.chi_tri, dtype=dtype, p1=w.p1,
                    beta4=w.beta4, nonlinearity=nl, **kw)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    say("device:", torch.cuda.get_device_name(0))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("wname", ["plain_small", "vortex"])
def test_operator_application(dtype, wname):
    w = case(wname) if wname == "plain_small" else case(wname, n_vert=20000, n_steps=10)
    say("apply", wname, dtype, w.mesh.n_vert)
    ops = oracle_ops(w)
    m = lib_mesh(w, dtype)
    rng = np.random.default_rng(1)
    x = rng.normal(size=ops.n) + 1j * rng.normal(size=ops.n)
    xd = dev(x, dtype)
    for op, ref in (("L", ops.L @ x), ("L2", ops.L @ (ops.L @ x)), ("H", ops.apply_H(x))):
        got = host(m.apply(op, xd))
        assert rel(got, ref) < KERNEL_TOL[dtype] * (30 if op == "L2" else 10), (op, rel(got, ref))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("nl", ["dec", "lumped"])
def test_kerr_and_linear_substeps(dtype, nl):
    w = case("step_index", n_vert=20000, n_steps=10)
    say("substeps", dtype, nl, w.mesh.n_vert)
    ops = oracle_ops(w, nl)
    m = lib_mesh(w, dtype, nl)
    u = w.u0
    f = dev(u, dtype)
    m.kerr_step(f, 0.37, 1.3)
    assert rel(host(f), S.nl_flow(u, 0.37, 1.3, ops)) < KERNEL_TOL[dtype] * 10
    f = dev(u, dtype)
    m.linear_step(f, w.dz)
    assert rel(host(f), S.lin_rk4(u, w.dz, ops)) < KERNEL_TOL[dtype] * 10


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("nl", ["dec", "lumped"])
def test_plain_small_end_to_end(dtype, nl):
    """4k-vertex disk, Gaussian 0.8 exp(-r^2/2), dz = 1e-3, 200 steps, gamma = 1."""
    w = case("plain_small")
    say("plain_small", dtype, nl)
    ops = oracle_ops(w, nl)
    ref = S.propagate(w.u0, ops, w.dz, w.n_steps, w.gamma)
    m = lib_mesh(w, dtype, nl)
    f = dev(w.u0, dtype)
    m.propagate(f, w.dz, w.n_steps, w.gamma)
    m.check_finite()
    err = rel(host(f), ref)
    say("  rel err", err)
    assert err < GATE[dtype]
    # diagnostics: power and Hamiltonian in FP64 accumulation
    P, E = m.diagnostics(f, w.gamma)
    out = host(f)
    tol = 1e-12 if dtype == "c128" else 1e-5
    assert abs(P - D.power(out, ops)) < tol * abs(D.power(out, ops))
    assert abs(E - D.hamiltonian(out, ops, w.gamma)) < tol * 10 * abs(D.hamiltonian(out, ops, w.gamma))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_step_index_replica_end_to_end(dtype):
    """Graded step-index disk (20k replica): core potential, absorber ring, tilted elliptic Gaussian."""
    w = case("step_index", n_vert=20000, n_steps=10)
    n = 300
    say("step_index replica", dtype, w.mesh.n_vert, n)
    ops = oracle_ops(w)
    ref = S.propagate(w.u0, ops, w.dz, n, w.gamma)
    m = lib_mesh(w, dtype)
    f = dev(w.u0, dtype)
    m.propagate(f, w.dz, n, w.gamma)
    err = rel(host(f), ref)
    say("  rel err", err)
    assert err < GATE[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_vortex_beta4_replica_end_to_end(dtype):
    """beta4 L^2 term, vortex launch with 1% noise, absorber (20k replica)."""
    w = case("vortex", n_vert=20000, n_steps=10)
    n = 200
    say("vortex replica", dtype, w.mesh.n_vert, n)
    ops = oracle_ops(w)
    ref = S.propagate(w.u0, ops, w.dz, n, w.gamma)
    m = lib_mesh(w, dtype)
    f = dev(w.u0, dtype)
    m.propagate(f, w.dz, n, w.gamma)
    err = rel(host(f), ref)
    say("  rel err", err)
    assert err < GATE[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("nl", ["dec", "lumped"])
def test_beta4_one_kernel_step_matches_row_kernels_and_oracle(dtype, nl):
    """The beta4 one-kernel step (two gathers per stage on tiles of eight or
    nine halo rings) against the nine-kernel row path and the oracle."""
    w = case("vortex", n_vert=20000, n_steps=10)
    say("beta4 step", dtype, nl, w.mesh.n_vert)
    ops = oracle_ops(w, nl)
    m = lib_mesh(w, dtype, nl)
    assert m.tuning["fused"] == 2  # the beta4 step tiles exist
    u = dev(w.u0, dtype)
    for n in (1, 2, 3, 37):
        outs = {}
        for fused, spg in ((2, 1), (2, 16), (0, 16)):
            m.tuning = {"fused": fused, "steps_per_graph": spg}
            f = u.clone()
            m.propagate(f, w.dz, n, w.gamma)
            outs[(fused, spg)] = host(f)
        assert np.array_equal(outs[(2, 1)], outs[(2, 16)]), n  # graph replay == eager
        tol = 1e-13 if dtype == "c128" else 1e-5
        assert rel(outs[(2, 16)], outs[(0, 16)]) < tol, (n, rel(outs[(2, 16)], outs[(0, 16)]))
        ref = S.propagate(w.u0, ops, w.dz, n, w.gamma)
        assert rel(outs[(2, 16)], ref) < GATE[dtype], n
        if n == 37:
            keep = outs[(2, 16)]
    for tb in (256, 1024):  # one or two slots per thread: separate instantiations, rounding may differ
        m.tuning = {"fused": 2, "tile_block": tb, "steps_per_graph": 16}
        f = u.clone()
        m.propagate(f, w.dz, 37, w.gamma)
        assert rel(host(f), keep) < KERNEL_TOL[dtype], tb
    assert m.time_kernels(w.dz, w.gamma, reps=10)["step"]["ms"] > 0


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("nl", ["dec", "lumped"])
def test_unsplit_rk4_matches_oracle(dtype, nl):
    """Classical RK4 on the whole right-hand side (Kerr and absorber inside every
    stage), one tile kernel per step, against the oracle's unsplit scheme."""
    w = case("step_index", n_vert=20000, n_steps=10)
    say("unsplit", dtype, nl, w.mesh.n_vert)
    ops = oracle_ops(w, nl)
    m = lib_mesh(w, dtype, nl)
    u = dev(w.u0, dtype)
    tol = 1e-12 if dtype == "c128" else 1e-5
    for n in (1, 2, 3, 37):
        outs = {}
        for spg in (1, 16):
            m.tuning = {"steps_per_graph": spg}
            f = u.clone()
            m.propagate_unsplit(f, w.dz, n, w.gamma)
            outs[spg] = host(f)
        m.check_finite()
        assert np.array_equal(outs[1], outs[16]), n  # graph replay == eager
        ref = US.propagate_rk4(w.u0, ops, w.dz, n, w.gamma)
        err = rel(outs[16], ref)
        assert err < tol, (n, err)
    assert m.time_kernels(w.dz, w.gamma, reps=10)["unsplit"]["ms"] > 0
    # the persistent launch (every tile resident, one launch for all steps) runs the same
    # per-row arithmetic; it keeps the owned |v|^2 from the previous step where the tile kernel
    # recomputes it on load, so the two may differ by the contraction of that sum (ulps)
    # (complex64: the step tiles; complex128's persistent tiles are its own, and its unsplit
    # steps stay one kernel each)
    m.tuning = {"fused": 3}
    persist_ms = m.time_kernels(w.dz, w.gamma, reps=10)["unsplit_persist"]["ms"]
    say("  persistent unsplit step ms", persist_ms)
    assert (persist_ms > 0) == (dtype == "c64")
    for n in (1, 2, 37):
        outs = {}
        for fused in (2, 3):
            m.tuning = {"fused": fused, "steps_per_graph": 16}
            f = u.clone()
            m.propagate_unsplit(f, w.dz, n, w.gamma)
            outs[fused] = host(f)
        m.check_finite()
        assert rel(outs[3], outs[2]) < (1e-14 if dtype == "c128" else 1e-6), (n, rel(outs[3], outs[2]))
    # a handle without one-field step tiles (the beta4 term) refuses, before any device work
    wb = case("vortex", n_vert=20000, n_steps=10)
    mb = lib_mesh(wb, dtype)
    with pytest.raises(api.DecBpmError) as e:
        mb.propagate_unsplit(dev(wb.u0, dtype), wb.dz, 3, wb.gamma)
    assert e.value.code == B.EINVAL


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adaptive_dp54_matches_oracle(dtype):
    """Adaptive Dormand-Prince 5(4) with the trials, error norms and accept/reject
    decisions on the device, against the oracle's adaptive run: in complex128 the
    same step sequence (counts, last step) and the state within the gate; in
    complex64 (looser tolerances) the state within the complex64 gate."""
    w = case("step_index", n_vert=20000, n_steps=10)
    ops = oracle_ops(w)
    m = lib_mesh(w, dtype)
    u = dev(w.u0, dtype)
    rtol, atol = (1e-9, 1e-11) if dtype == "c128" else (1e-5, 1e-7)
    # (z_end, h0): accuracy-limited steps with a rejection, a first trial clipped to z_end,
    # and a large first trial that is rejected several times
    for z_end, h0 in ((20 * w.dz, w.dz), (0.3 * w.dz, w.dz), (8 * w.dz, 40 * w.dz)):
        say("adaptive", dtype, w.mesh.n_vert, z_end, h0)
        f = u.clone()
        st = m.propagate_adaptive(f, z_end, h0, w.gamma, rtol=rtol, atol=atol)
        m.check_finite()
        ref, rs = US.propagate_dp54(w.u0, ops, z_end, h0, w.gamma, rtol=rtol, atol=atol)
        say("  gpu", st, "oracle", rs)
        assert st["z"] == z_end
        if dtype == "c128":
            assert (st["accepted"], st["rejected"]) == (rs["accepted"], rs["rejected"])
            # the error norm is a difference of stage sums (cancellation), so its low bits
            # depend on summation order; each step size inherits that at the 1e-8 level
            assert abs(st["last_h"] - rs["last_h"]) <= 1e-6 * rs["last_h"]
        else:
            assert abs(st["accepted"] - rs["accepted"]) <= 1 + rs["accepted"] // 10
        err = rel(host(f), ref)
        say("  rel err", err)
        assert err < GATE[dtype], (z_end, h0, err)
    # the whole run in one persistent launch (every seven-ring tile resident, a grid-wide
    # exchange per trial instead of a kernel boundary): the same steps and state.  In
    # complex64 this mesh's trial tiles fit at once (the timing class shows the path is
    # live); complex128's smaller tiles do not, and its runs stay per trial.
    m.tuning = {"fused": 3}
    persist_ms = m.time_kernels(w.dz, w.gamma, reps=20)["dp5_persist"]["ms"]
    say("  persistent adaptive trial ms", persist_ms)
    if dtype == "c64":
        assert persist_ms > 0
    runs = {}
    for fused, x in ((2, 0), (3, 0), (3, 1)):
        m.tuning = {"fused": fused, "xcd_remap": x}
        f = u.clone()
        runs[(fused, x)] = (m.propagate_adaptive(f, 20 * w.dz, w.dz, w.gamma, rtol=rtol, atol=atol), host(f))
    say("  persistent adaptive", runs[(2, 0)][0], runs[(3, 0)][0])
    ref = US.propagate_dp54(w.u0, ops, 20 * w.dz, w.dz, w.gamma, rtol=rtol, atol=atol)[0]
    for key in ((3, 0), (3, 1)):
        st2, st3 = runs[(2, 0)][0], runs[key][0]
        assert (st2["accepted"], st2["rejected"]) == (st3["accepted"], st3["rejected"]), key
        assert rel(runs[key][1], runs[(2, 0)][1]) < (1e-13 if dtype == "c128" else 1e-6), key
        assert rel(runs[key][1], ref) < GATE[dtype], key
    m.tuning = {"fused": 2, "xcd_remap": 0}
    # a second handle call after a different run gives the same result (controller reset)
    f1 = u.clone()
    m.propagate_adaptive(f1, 2 * w.dz, w.dz, w.gamma, rtol=rtol, atol=atol)
    f2 = u.clone()
    m.propagate_adaptive(f2, 2 * w.dz, w.dz, w.gamma, rtol=rtol, atol=atol)
    assert torch.equal(f1, f2)
    # z_end = 0: nothing happens
    f = u.clone()
    st = m.propagate_adaptive(f, 0.0, w.dz, w.gamma)
    assert torch.equal(f, u) and st["accepted"] == 0
    # too few attempts: EUNSTABLE, the counters say how far it got and the field is the
    # last accepted state (finite)
    f = u.clone()
    with pytest.raises(api.DecBpmError) as e:
        m.propagate_adaptive(f, 50 * w.dz, w.dz, w.gamma, rtol=rtol, atol=atol, max_attempts=3)
    assert e.value.code == B.EUNSTABLE
    assert e.value.stats["accepted"] + e.value.stats["rejected"] == 3 and e.value.stats["z"] < 50 * w.dz
    assert torch.isfinite(torch.view_as_real(f)).all()
    # bad arguments
    for kw in ({"rtol": -1.0}, {"atol": 0.0}):
        with pytest.raises(api.DecBpmError) as e:
            m.propagate_adaptive(u.clone(), w.dz, w.dz, w.gamma, **kw)
        assert e.value.code == B.EINVAL
    assert m.time_kernels(w.dz, w.gamma, reps=10)["dp5"]["ms"] > 0


def test_adaptive_dp54_small_meshes_and_refusals():
    """Few tiles (a 4k-vertex mesh) and the lumped Kerr term, complex128; a beta4
    handle refuses before any device work."""
    w = case("plain_small")
    for nl in ("dec", "lumped"):
        ops = oracle_ops(w, nl)
        m = lib_mesh(w, "c128", nl)
        say("adaptive small", nl, w.mesh.n_vert)
        f = dev(w.u0, "c128")
        st = m.propagate_adaptive(f, 200 * w.dz, w.dz, w.gamma, rtol=1e-10, atol=1e-12)
        ref, rs = US.propagate_dp54(w.u0, ops, 200 * w.dz, w.dz, w.gamma, rtol=1e-10, atol=1e-12)
        assert (st["accepted"], st["rejected"]) == (rs["accepted"], rs["rejected"]), (st, rs)
        assert rel(host(f), ref) < GATE["c128"]
    wb = case("vortex", n_vert=20000, n_steps=10)
    mb = lib_mesh(wb, "c128")
    with pytest.raises(api.DecBpmError) as e:
        mb.propagate_adaptive(dev(wb.u0, "c128"), wb.dz, wb.dz, wb.gamma)
    assert e.value.code == B.EINVAL


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_mode_iterations_match_oracle(dtype):
    """Nonlinear mode iteration (imaginary-z RK4 with frozen nonlinearity, renormalised to
    the power) on the 89k-vertex step-index mesh: a fixed number of iterations (tol = 0)
    against the oracle's iterate, Rayleigh quotient and residual."""
    w = case("step_index", n_vert=20000, n_steps=10)
    ops = oracle_ops(w)
    m = lib_mesh(w, dtype)
    dtau = 2.0 / m.spectral_radius()
    for n in (1, 2, 31):
        say("mode iterations", dtype, w.mesh.n_vert, n)
        f = dev(w.u0, dtype)
        st = m.find_mode(f, 4.0, dtau, w.gamma, tol=0.0, max_iter=n)
        m.check_finite()
        ref, info = SO.find_mode(w.u0, ops, 4.0, dtau, w.gamma, tol=0.0, max_iter=n)
        assert st["iterations"] == info["iterations"] == n
        err = rel(host(f), ref)
        say("  rel err", err, "mu", st["mu"], info["mu"], "res", st["residual"], info["residual"])
        assert err < GATE[dtype], (n, err)
        tq = 1e-12 if dtype == "c128" else 1e-5
        assert abs(st["mu"] - info["mu"]) <= tq * abs(info["mu"])
        assert abs(st["residual"] - info["residual"]) <= (1e-9 if dtype == "c128" else 1e-3) * info["residual"]
    assert m.time_kernels(w.dz, w.gamma, reps=10)["mode"]["ms"] > 0


def test_mode_solver_converges_like_the_oracle():
    """A guided mode on a 4k-vertex disk (four step tiles), complex128, to tol 1e-10: the
    same iteration count as the oracle, the same mode and quotient, and the mode is
    stationary under the library's own z-marching."""
    mesh = M.disk_mesh(10.0, 0.301, 11)
    r = np.hypot(*mesh.xy[mesh.tri].mean(axis=1).T)
    V = np.where(r < 3.0, 1.0, 0.0)
    ops = dec.assemble(mesh.xy, mesh.tri, V)
    m = api.Mesh(mesh.xy, mesh.tri, V, None, dtype="c128")
    start = np.exp(-np.sum(mesh.xy**2, axis=1) / 4.0) + 0j
    dtau = 2.0 / m.spectral_radius()
    say("mode solver", mesh.n_vert, dtau)
    f = dev(start, "c128")
    st = m.find_mode(f, 3.0, dtau, 1.0, tol=1e-10)
    ref, info = SO.find_mode(start, ops, 3.0, dtau, 1.0, tol=1e-10)
    say("  gpu", st, "oracle", info)
    assert st["iterations"] == info["iterations"]
    assert abs(st["mu"] - info["mu"]) <= 1e-12 * abs(info["mu"])
    phi = host(f)
    assert rel(phi, ref) < GATE["c128"]
    assert abs(D.power(phi, ops) - 3.0) < 1e-12
    g = f.clone()
    z, n = 0.5, 500
    m.propagate(g, z / n, n, 1.0)
    assert rel(host(g), phi * np.exp(-1j * st["mu"] * z)) < 1e-4
    # the whole solve in one persistent launch (every tile resident; a grid-wide exchange per
    # iteration instead of a kernel boundary): the same iterations and mode
    # (complex64; complex128 keeps one kernel per iteration), also with the XCD-aware block order
    for dtype in ("c128", "c64"):
        mp = api.Mesh(mesh.xy, mesh.tri, V, None, dtype=dtype)
        mp.tuning = {"fused": 3}
        persist_ms = mp.time_kernels(dtau, 1.0, reps=20)["mode_persist"]["ms"]
        say("  persistent mode iteration ms", dtype, persist_ms)
        assert (persist_ms > 0) == (dtype == "c64")  # the path is live where it should be
        runs = {}
        for fused, x in ((2, 0), (3, 0), (3, 1)):
            mp.tuning = {"fused": fused, "xcd_remap": x}
            fp = dev(start, dtype)
            runs[(fused, x)] = (mp.find_mode(fp, 3.0, dtau, 1.0, tol=1e-10 if dtype == "c128" else 1e-4), host(fp))
        say("  persistent mode solver", dtype, runs[(2, 0)][0], runs[(3, 0)][0])
        for key in ((3, 0), (3, 1)):
            assert runs[(2, 0)][0]["iterations"] == runs[key][0]["iterations"], key
            assert rel(runs[key][1], runs[(2, 0)][1]) < (1e-13 if dtype == "c128" else 1e-6), key
    # failures: no convergence in too few iterations (the field holds the last iterate),
    # a start without power, a step beyond the RK4 margin, a beta4 handle
    f = dev(start, "c128")
    with pytest.raises(api.DecBpmError) as e:
        m.find_mode(f, 3.0, dtau, 1.0, tol=1e-10, max_iter=5)
    assert e.value.code == B.EUNSTABLE and e.value.stats["iterations"] == 5
    assert abs(D.power(host(f), ops) - 3.0) < 1e-12
    with pytest.raises(api.DecBpmError) as e:
        m.find_mode(torch.zeros_like(f), 3.0, dtau, 1.0)
    assert e.value.code == B.ENONFINITE
    with pytest.raises(api.DecBpmError) as e:
        m.find_mode(f, 3.0, 3.0 / m.spectral_radius(), 1.0)
    assert e.value.code == B.EUNSTABLE
    wb = case("vortex", n_vert=20000, n_steps=10)
    mb = lib_mesh(wb, "c128")
    with pytest.raises(api.DecBpmError) as e:
        mb.find_mode(dev(wb.u0, "c128"), 1.0, wb.dz, 1.0)
    assert e.value.code == B.EINVAL


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_pml_step_matches_oracle(dtype):
    """A perfectly matched layer (complex-stretched Hodge stars) in place of the absorber on
    the 89k-vertex step-index mesh: the one-kernel step with complex L weights against the
    oracle's split scheme on the stretched operators, for step counts that mix graph
    replays and eager steps; in complex64 the persistent launch with complex weights gives
    the one-kernel step's bits; the handle refuses the two-kernel mode and the entry
    points whose kernels apply a real L."""
    w = case("step_index", n_vert=20000, n_steps=10)
    pml = (35.0, 40.0, 1.0)
    ops = dec.assemble(w.mesh.xy, w.mesh.tri, w.index_tri, None, pml=pml)
    m = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, None, dtype=dtype, pml=pml)
    assert m.tuning["fused"] == 2
    u = dev(w.u0, dtype)
    for n in (1, 2, 33):
        say("pml", dtype, w.mesh.n_vert, n)
        f = u.clone()
        m.propagate(f, w.dz, n, w.gamma)
        m.check_finite()
        ref = S.propagate(w.u0, ops, w.dz, n, w.gamma)
        err = rel(host(f), ref)
        say("  rel err", err)
        assert err < (1e-12 if dtype == "c128" else 1e-5), (n, err)
        if dtype == "c64":
            for x in (0, 1):
                m.tuning = {"fused": 3, "tile_block": 1024, "xcd_remap": x}
                g = u.clone()
                m.propagate(g, w.dz, n, w.gamma)
                m.check_finite()
                assert np.array_equal(host(g), host(f)), (n, x, rel(host(g), host(f)))
            m.tuning = {"fused": 2, "xcd_remap": 0}
    persist_ms = m.time_kernels(w.dz, w.gamma, reps=10)["persist"]["ms"]
    say("  persistent launch ms per step", persist_ms)
    assert (persist_ms > 0) == (dtype == "c64")  # the complex-weight persistent kernel: complex64 only
    t = dict(m.tuning)
    t["fused"] = 1
    with pytest.raises(api.DecBpmError) as e:
        m.tuning = t
    assert e.value.code == B.EINVAL
    with pytest.raises(api.DecBpmError) as e:
        m.apply("L", u.clone())
    assert e.value.code == B.EINVAL
    P, E = m.diagnostics(u.clone(), w.gamma)
    assert P > 0 and math.isnan(E)
    assert m.time_kernels(w.dz, w.gamma, reps=10)["step"]["ms"] > 0


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_pml_unsplit_and_adaptive_match_oracle(dtype):
    """The paper's own integrators with the perfectly matched layer (complex L weights in
    the unsplit RK4 and Dormand-Prince trial kernels): the unsplit RK4 step (one kernel per
    step; in complex64 also the persistent launch, equal to it to rounding) and the adaptive
    pair against the oracle's runs on the stretched operators (in complex128 with the
    same accepted and rejected counts)."""
    w = case("step_index", n_vert=20000, n_steps=10)
    pml = (35.0, 40.0, 1.0)
    ops = dec.assemble(w.mesh.xy, w.mesh.tri, w.index_tri, None, pml=pml)
    m = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, None, dtype=dtype, pml=pml)
    u = dev(w.u0, dtype)
    tol = 1e-12 if dtype == "c128" else 1e-5
    for n in (1, 9):
        ref = US.propagate_rk4(w.u0, ops, w.dz, n, w.gamma)
        m.tuning = {"fused": 2}
        f = u.clone()
        m.propagate_unsplit(f, w.dz, n, w.gamma)
        m.check_finite()
        err = rel(host(f), ref)
        say("pml unsplit", dtype, n, err)
        assert err < tol, (n, err)
        if dtype == "c64":
            m.tuning = {"fused": 3}
            assert m.time_kernels(w.dz, w.gamma, reps=10)["unsplit_persist"]["ms"] > 0
            g = u.clone()
            m.propagate_unsplit(g, w.dz, n, w.gamma)
            m.check_finite()
            # the persistent body keeps the owned |v|^2 from the previous step where the tile
            # kernel recomputes it on load: the two may differ by that sum's contraction (ulps)
            assert rel(host(g), host(f)) < 1e-6, (n, rel(host(g), host(f)))
            m.tuning = {"fused": 2}
    rtol, atol = (1e-9, 1e-11) if dtype == "c128" else (1e-5, 1e-7)
    m.tuning = {"fused": 2}
    for z_end, h0 in ((12 * w.dz, w.dz), (6 * w.dz, 30 * w.dz)):
        f = u.clone()
        st = m.propagate_adaptive(f, z_end, h0, w.gamma, rtol=rtol, atol=atol)
        m.check_finite()
        ref, rs = US.propagate_dp54(w.u0, ops, z_end, h0, w.gamma, rtol=rtol, atol=atol)
        err = rel(host(f), ref)
        say("pml adaptive", dtype, z_end, h0, st, rs, err)
        assert st["z"] == z_end
        if dtype == "c128":
            assert (st["accepted"], st["rejected"]) == (rs["accepted"], rs["rejected"])
        assert err < GATE[dtype], (z_end, h0, err)


def test_pml_absorbs_on_the_gpu():
    """The outgoing-beam case of the oracle's absorption pin, run by the library (complex128):
    equal to the oracle with the layer, and, inside r < 4.5, equal to the open-domain field
    (the oracle on a disk of twice the radius) up to the meshes' mismatch, where a
    reflecting boundary is far off."""
    from scipy.interpolate import LinearNDInterpolator

    mesh = M.disk_mesh(8.0, 0.25, 7)
    launch = np.exp(-(mesh.xy[:, 0] ** 2 + mesh.xy[:, 1] ** 2)) * np.exp(3j * mesh.xy[:, 0])
    pml = (5.0, 8.0, 1.0)
    inner = np.hypot(mesh.xy[:, 0], mesh.xy[:, 1]) < 4.5
    n, dz = 200, 0.02
    out = {}
    for name, kw in (("pml", {"pml": pml}), ("reflecting", {})):
        m = api.Mesh(mesh.xy, mesh.tri, None, None, dtype="c128", p1=0.5, **kw)
        f = dev(launch, "c128")
        m.propagate(f, dz, n, 0.0)
        out[name] = host(f)
    ref = S.propagate(launch, dec.assemble(mesh.xy, mesh.tri, pml=pml), dz, n, 0.0)
    assert rel(out["pml"], ref) < 1e-11
    u0n = np.linalg.norm(launch[inner])
    big = M.disk_mesh(16.0, 0.25, 7)
    lb = np.exp(-(big.xy[:, 0] ** 2 + big.xy[:, 1] ** 2)) * np.exp(3j * big.xy[:, 0])
    open_ref = S.propagate(lb, dec.assemble(big.xy, big.tri), dz, n, 0.0)
    open_ref = LinearNDInterpolator(big.xy, open_ref)(mesh.xy[inner])
    err = {k: np.linalg.norm(v[inner] - open_ref) / u0n for k, v in out.items()}
    say("  interior error vs the open domain", err)
    assert err["pml"] < 0.03 and err["reflecting"] > 0.3, err


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("response,param,p3,p4", [("kerr", 0.0, -4e-3, 1e-3), ("saturable", 0.8, 2e-3, 0.0),
                                                   ("cubic_quintic", 0.25, 2e-3, 0.0)])
@pytest.mark.parametrize("stage_tiles", ["1", "0"])
def test_general_operator_sum_and_responses_match_oracle(dtype, response, param, p3, p4, stage_tiles,
                                                         monkeypatch):
    """Eq. 1 in full: terms up to p4 L^4 with the Kerr, saturable and cubic-quintic
    responses (closed-form flow integrals), on the five-kernel path whose RK4 stages run
    as one tile kernel each (the Horner chain of the operator sum in LDS) or, with
    DEC_BPM_GEN_TILES=0, as chains of gather kernels; against the oracle's split scheme
    on the step-index replica (20k vertices, with absorber), plus the Kerr substep and
    the linear step alone."""
    w = case("step_index", n_vert=20000, n_steps=10)
    kw = dict(p3=p3, p4=p4, nl_kind=response, nl_param=param)
    ops = dec.assemble(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, p1=w.p1, beta4=2e-3, **kw)
    monkeypatch.setenv("DEC_BPM_GEN_TILES", stage_tiles)
    m = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, dtype=dtype, p1=w.p1, beta4=2e-3, p3=p3, p4=p4,
                 response=response, response_param=param)
    monkeypatch.delenv("DEC_BPM_GEN_TILES")
    assert m.tuning["fused"] == 0
    dz = 0.9 * 2.5 / m.spectral_radius()
    u0 = 1.5 * w.u0
    u = dev(u0, dtype)
    tol = 1e-12 if dtype == "c128" else 2e-5
    say("general", dtype, response, p3, p4, "dz", dz)
    f = u.clone()
    m.kerr_step(f, 0.37, w.gamma)
    assert rel(host(f), S.nl_flow(u0, 0.37, w.gamma, ops)) < tol
    f = u.clone()
    m.linear_step(f, dz)
    assert rel(host(f), S.lin_rk4(u0, dz, ops)) < tol
    for n in (1, 7):
        f = u.clone()
        m.propagate(f, dz, n, w.gamma)
        m.check_finite()
        err = rel(host(f), S.propagate(u0, ops, dz, n, w.gamma))
        say("  steps", n, "rel err", err)
        assert err < tol, (n, err)
    P, E = m.diagnostics(u.clone(), w.gamma)
    assert P > 0 and math.isnan(E)
    with pytest.raises(api.DecBpmError) as e:
        m.tuning = {"fused": 2}
    assert e.value.code == B.EINVAL
    with pytest.raises(api.DecBpmError) as e:
        m.propagate_unsplit(u.clone(), dz, 1, w.gamma)
    assert e.value.code == B.EINVAL


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("response,param", [("saturable", 0.8), ("cubic_quintic", 0.25)])
@pytest.mark.parametrize("beta4", [0.0, 2e-3])
def test_responses_on_every_split_step_mode(dtype, response, param, beta4):
    """The saturable and cubic-quintic responses without terms beyond L^2 run on every
    split-step launch mode (the tile kernels' Kerr phase takes the response's flow
    integral): five kernels, two tile kernels, one kernel per step (with beta4: the beta4
    step) and the persistent launch, each against the oracle; the persistent launch
    equals the one-kernel step bitwise, and so does the first half step of the
    persistent prologue."""
    w = case("step_index", n_vert=20000, n_steps=10)
    kw = dict(nl_kind=response, nl_param=param)
    ops = dec.assemble(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, p1=w.p1, beta4=beta4, **kw)
    m = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, dtype=dtype, p1=w.p1, beta4=beta4,
                 response=response, response_param=param)
    assert m.tuning["fused"] == 2
    dz = min(w.dz, 0.9 * 2.5 / m.spectral_radius())  # beta4 L^2 raises the spectral radius
    u0 = 1.5 * w.u0
    u = dev(u0, dtype)
    tol = 1e-12 if dtype == "c128" else 2e-5
    modes = (0, 2) if beta4 else (0, 1, 2, 3)
    say("responses", dtype, response, "beta4", beta4, "dz", dz)
    outs = {}
    for n in (1, 9):
        ref = S.propagate(u0, ops, dz, n, w.gamma)
        for fused in modes:
            m.tuning = {"fused": fused}
            if fused == 3:
                assert m.time_kernels(dz, w.gamma, reps=10)["persist"]["ms"] > 0
            f = u.clone()
            m.propagate(f, dz, n, w.gamma)
            m.check_finite()
            outs[(n, fused)] = host(f)
            err = rel(outs[(n, fused)], ref)
            say(f"  fused {fused} steps {n}: rel {err:.3e}")
            assert err < tol, (fused, n, err)
        if 3 in modes:
            assert np.array_equal(outs[(n, 3)], outs[(n, 2)]), n


def test_full_size_pml_and_mode_iterations():
    """The full 249k-vertex step-index mesh in the bench's configurations of the layer
    (one-kernel step with complex weights and the persistent launch, 5 steps) and of the
    mode solver (10 iterations), complex64, against the oracle."""
    w = case("step_index")
    say("full size pml / mode", w.mesh.n_vert)
    pml = (35.0, 40.0, 1.0)
    ops = dec.assemble(w.mesh.xy, w.mesh.tri, w.index_tri, None, pml=pml)
    m = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, None, dtype="c64", pml=pml)
    f = dev(w.u0, "c64")
    m.propagate(f, w.dz, 5, w.gamma)
    err = rel(host(f), S.propagate(w.u0, ops, w.dz, 5, w.gamma))
    say("  pml rel err", err)
    assert err < 1e-5
    m.tuning = {"fused": 3}  # the persistent launch with complex weights: the same bits
    g = dev(w.u0, "c64")
    m.propagate(g, w.dz, 5, w.gamma)
    m.check_finite()
    assert np.array_equal(host(g), host(f)), rel(host(g), host(f))
    ops = oracle_ops(w)
    m = lib_mesh(w, "c64")
    dtau = 2.0 / m.spectral_radius()
    f = dev(w.u0, "c64")
    st = m.find_mode(f, 4.0, dtau, w.gamma, tol=0.0, max_iter=10)
    ref, info = SO.find_mode(w.u0, ops, 4.0, dtau, w.gamma, tol=0.0, max_iter=10)
    err = rel(host(f), ref)
    say("  mode rel err", err, st["mu"], info["mu"])
    assert err < 1e-5 and abs(st["mu"] - info["mu"]) < 1e-5 * abs(info["mu"])


def test_vortex_beta4_full_size_prefix():
    """The full 1M-vertex vortex launch with the beta4 L^2 term in the bench's launch
    configuration (autotuned: the beta4 one-kernel step), complex64, 3 steps vs the oracle."""
    w = case("vortex")
    say("vortex full size", w.mesh.n_vert)
    m = lib_mesh(w, "c64")
    m.autotune(w.dz, w.gamma)
    f = dev(w.u0, "c64")
    m.propagate(f, w.dz, 3, w.gamma)
    ref = S.propagate(w.u0, oracle_ops(w), w.dz, 3, w.gamma)
    err = rel(host(f), ref)
    say("  rel err", err, m.tuning)
    assert err < 1e-5


def test_batched_full_size_prefix():
    """The full batched workload (8 PCF meshes of 19k-198k vertices x 32 fields) in the bench's
    launch configuration (autotuned), complex64, 3 steps: sampled fields of the smallest and
    largest mesh against the oracle."""
    ws = W.batched_pcf()
    F = ws[0].u0.shape[0]
    say("batched full size", [x.mesh.n_vert for x in ws], F)
    meshes = [lib_mesh(x, "c64") for x in ws]
    batch = api.Batch(meshes, F)
    packed = batch.pack([dev(x.u0, "c64") for x in ws])
    batch.autotune(ws[0].dz, 1.0)
    batch.propagate(packed, ws[0].dz, 3, 1.0)
    outs = batch.unpack(packed)
    for k, f in ((0, 0), (len(ws) - 1, F - 1)):
        x = ws[k]
        ref = S.propagate(x.u0[f], oracle_ops(x), x.dz, 3, 1.0)
        err = rel(host(outs[k][f].contiguous()), ref)
        say("  mesh", k, "field", f, "rel err", err, batch.tuning)
        assert err < 1e-5


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_step_index_full_size_prefix(dtype):
    """The full 250k-vertex step-index workload, 20 steps, in the bench's launch configuration."""
    w = case("step_index")
    n = 20
    say("step_index full", dtype, w.mesh.n_vert, n)
    ops = oracle_ops(w)
    ref = S.propagate(w.u0, ops, w.dz, n, w.gamma)
    m = lib_mesh(w, dtype)
    f = dev(w.u0, dtype)
    m.propagate(f, w.dz, n, w.gamma)
    err = rel(host(f), ref)
    say("  rel err", err)
    assert err < GATE[dtype]


@pytest.mark.parametrize("fused", [0, 1, 2, 3])
def test_edge_cases_and_launch_paths(fused):
    """Zero, one, two and odd step counts, graph replay vs eager, block sizes
    and chunked calls, in every launch mode (4k-vertex mesh: four step tiles)."""
    w = case("plain_small")
    m = lib_mesh(w, "c128")
    m.tuning = {"fused": fused}
    say("edge cases, mode", fused)
    ops = oracle_ops(w)
    u = dev(w.u0, "c128")
    f = u.clone()
    m.propagate(f, w.dz, 0, 1.0)  # no-op
    assert torch.equal(f, u)
    for n in (1, 2, 33, 70):  # graph replays + eager remainders
        f = u.clone()
        m.propagate(f, w.dz, n, 1.0)
        assert rel(host(f), S.propagate(w.u0, ops, w.dz, n, 1.0)) < 1e-12, n
    # graph and eager launches produce identical bits
    m.tuning = {"block_size": 256, "steps_per_graph": 1, "fused": fused}
    a = u.clone()
    m.propagate(a, w.dz, 70, 1.0)
    m.tuning = {"block_size": 256, "steps_per_graph": 16}
    b = u.clone()
    m.propagate(b, w.dz, 70, 1.0)
    assert torch.equal(a, b)
    # run twice: deterministic
    c = u.clone()
    m.propagate(c, w.dz, 70, 1.0)
    assert torch.equal(b, c)
    # block size does not change the arithmetic
    for blk in (64, 512, 1024):
        m.tuning = {"block_size": blk, "steps_per_graph": 16}
        d = u.clone()
        m.propagate(d, w.dz, 70, 1.0)
        assert torch.equal(b, d), blk
    # chunked propagation: two calls equal one call up to the merged half steps
    e = u.clone()
    m.propagate(e, w.dz, 35, 1.0)
    m.propagate(e, w.dz, 35, 1.0)
    assert rel(host(e), host(b)) < 1e-13


@pytest.mark.parametrize("fused", [2, 3])
def test_single_tile_mesh(fused):
    """A mesh of one step tile: no halo rows, no neighbour tiles to wait for."""
    w = W.plain_small(n_vert=700, n_steps=10)
    m = lib_mesh(w, "c128")
    m.tuning = {"fused": fused}
    ops = oracle_ops(w)
    for n in (1, 2, 5, 40):
        f = dev(w.u0, "c128")
        m.propagate(f, w.dz, n, 1.0)
        m.check_finite()
        assert rel(host(f), S.propagate(w.u0, ops, w.dz, n, 1.0)) < 1e-12, n


def test_nonfinite_is_flagged():
    w = case("plain_small")
    m = lib_mesh(w, "c64")
    f = dev(w.u0, "c64")
    f[5] = float("nan")
    m.propagate(f, w.dz, 3, 1.0)
    with pytest.raises(api.DecBpmError) as e:
        m.check_finite()
    assert e.value.code == -6
    g = dev(w.u0, "c64")
    m.propagate(g, w.dz, 3, 1.0)
    m.check_finite()  # flag was cleared


def test_unstable_dz_rejected_before_device_work():
    w = case("plain_small")
    m = lib_mesh(w, "c64")
    f = dev(w.u0, "c64")
    keep = f.clone()
    with pytest.raises(api.DecBpmError) as e:
        m.propagate(f, 3.0 / m.spectral_radius(), 5, 1.0)
    assert e.value.code == -3
    assert torch.equal(f, keep)


def test_overlap_and_power_match_oracle():
    w = case("adjoint", n_vert=20000, n_steps=10)
    ops = oracle_ops(w)
    for dtype in ("c128", "c64"):
        m = lib_mesh(w, dtype)
        a, b = dev(w.extra["target"], dtype), dev(w.u0, dtype)
        c = m.overlap(a, b)
        ref = D.overlap(w.extra["target"], w.u0, ops)
        tol = 1e-13 if dtype == "c128" else 1e-6
        assert abs(c - ref) < tol * abs(ref)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batched_equals_plain(dtype):
    ws = W.batched_pcf(n_meshes=3, fields_per_mesh=4, n_min=3000, n_max=9000, n_steps=40)
    say("batched", dtype, [x.mesh.n_vert for x in ws])
    meshes = [lib_mesh(x, dtype) for x in ws]
    batch = api.Batch(meshes, 4)
    packed0 = batch.pack([dev(x.u0, dtype) for x in ws])
    # LDS-tiled batched stage kernels, the batched one-kernel step and the field-loop
    # step (one-field tiles, every field in turn) vs the row-parallel kernels:
    # identical per-row formulas
    runs = {}
    for fused in (0, 1, 2, 3):
        batch.tuning = {"fused": fused}
        assert batch.tuning["fused"] == fused
        pk = packed0.clone()
        batch.propagate(pk, ws[0].dz, ws[0].n_steps, 1.0)
        batch.check_finite()
        runs[fused] = pk
        if fused >= 2:
            assert batch.time_kernels(ws[0].dz, 1.0, reps=5)["step"]["ms"] > 0  # the mode's tiles exist
    for fused in (1, 2, 3):
        assert rel(host(runs[fused]), host(runs[0])) < (1e-13 if dtype == "c128" else 1e-6), fused
    tol = 1e-12 if dtype == "c128" else 1e-6  # same per-row formulas; only FMA contraction may differ
    for bf in (1, 3):
        outs = batch.unpack(runs[bf])
        for m, x, o in zip(meshes, ws, outs):
            for f in range(4):
                for fused in (0, 1, 2, 3):
                    m.tuning = {"fused": fused}
                    single = dev(x.u0[f], dtype)
                    m.propagate(single, x.dz, x.n_steps, 1.0)
                    err = rel(host(o[f].contiguous()), host(single))
                    assert err < tol, (bf, fused, err)
                    if bf == 3 and fused >= 2:  # the same one-field step arithmetic
                        assert torch.equal(o[f].contiguous(), single), (fused, f)
    outs = batch.unpack(runs[1])
    # and one field against the oracle
    ops = oracle_ops(ws[1])
    ref = S.propagate(ws[1].u0[2], ops, ws[1].dz, ws[1].n_steps, 1.0)
    assert rel(host(outs[1][2].contiguous()), ref) < GATE[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batched_uneven_field_counts(dtype):
    """Meshes carrying different numbers of fields (1, 5 and 3: the device pads every row
    to the largest count, rounded up to whole field groups): each field equals a plain
    propagate of it, the padding never reaches the caller's buffer, and one field matches
    the oracle."""
    ws = W.batched_pcf(n_meshes=3, fields_per_mesh=5, n_min=3000, n_max=9000, n_steps=40)
    counts = [1, 5, 3]
    say("batched uneven", dtype, [x.mesh.n_vert for x in ws], counts)
    meshes = [lib_mesh(x, dtype) for x in ws]
    batch = api.Batch(meshes, counts)
    assert batch.n_elems == sum(x.mesh.n_vert * c for x, c in zip(ws, counts))
    fields = [dev(x.u0[:c], dtype) for x, c in zip(ws, counts)]
    guard = 7
    buf = torch.full((batch.n_elems + 2 * guard,), 3.5 - 1.5j, dtype=fields[0].dtype, device=DEV)
    buf[guard:guard + batch.n_elems] = batch.pack(fields)
    packed = buf[guard:guard + batch.n_elems]
    for fused in (0, 1, 2, 3):
        batch.tuning = {"fused": fused}
        pk = packed.clone()
        batch.propagate(pk, ws[0].dz, ws[0].n_steps, 1.0)
        batch.check_finite()
        outs = batch.unpack(pk)
        tol = 1e-12 if dtype == "c128" else 1e-6
        for m, x, o, c in zip(meshes, ws, outs, counts):
            assert o.shape == (c, x.mesh.n_vert)
            for f in range(c):
                single = dev(x.u0[f], dtype)
                m.propagate(single, x.dz, x.n_steps, 1.0)
                err = rel(host(o[f].contiguous()), host(single))
                assert err < tol, (fused, f, err)
    batch.propagate(packed, ws[0].dz, ws[0].n_steps, 1.0)  # in place inside the guarded buffer
    assert torch.all(buf[:guard] == 3.5 - 1.5j) and torch.all(buf[guard + batch.n_elems:] == 3.5 - 1.5j)
    ref = S.propagate(ws[1].u0[4], oracle_ops(ws[1]), ws[1].dz, ws[1].n_steps, 1.0)
    assert rel(host(batch.unpack(packed)[1][4].contiguous()), ref) < GATE[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adjoint_matches_oracle_gradients(dtype):
    w = W.adjoint_mmf(n_vert=3000, n_steps=10)
    n, every = 24, 5
    say("adjoint", dtype, w.mesh.n_vert, n)
    dn = w.extra["dn"]
    ops = oracle_ops(w, dn=dn)
    J, g_ref, gdn_ref = OA.gradients(w.u0, w.extra["target"], ops, w.dz, n, w.gamma)
    m = lib_mesh(w, dtype)
    dn_d = torch.from_numpy(dn).to(DEV)
    m.set_index_perturbation(dn_d)
    u = dev(w.u0, dtype)
    wsp = torch.empty(m.workspace_size(n, every), dtype=torch.uint8, device=DEV)
    m.forward_checkpointed(u, w.dz, n, w.gamma, wsp, every)
    ref_u = S.propagate(w.u0, ops, w.dz, n, w.gamma)
    assert rel(host(u), ref_u) < GATE[dtype]
    tgt = dev(w.extra["target"], dtype)
    c = m.overlap(tgt, u)
    gout = (2 * c * torch.from_numpy(ops.H0).to(DEV) * tgt.to(torch.complex128)).to(u.dtype)
    g0, gdn = m.adjoint(gout, w.dz, n, w.gamma, wsp, every)
    tol = 1e-9 if dtype == "c128" else 1e-4
    assert rel(host(g0), g_ref) < tol, rel(host(g0), g_ref)
    assert rel(gdn.cpu().numpy(), gdn_ref) < tol, rel(gdn.cpu().numpy(), gdn_ref)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adjoint_with_the_run_stored_and_repeated_calls(dtype):
    """The checkpointed forward stores the last segment's stage vectors, so the adjoint
    skips that segment's recompute; with every = n_steps it stores the whole run and
    recomputes nothing.  The gradients with 5-step segments and with the run stored agree
    bitwise (the recording step kernel is the plain step plus stores), a second adjoint
    call on the same workspace gives the first one's bits (with several segments the
    first call's recompute has overwritten the stored one, so the second recomputes it),
    and both agree with the oracle."""
    w = W.adjoint_mmf(n_vert=3000, n_steps=10)
    n = 24
    dn = w.extra["dn"]
    ops = oracle_ops(w, dn=dn)
    J, g_ref, gdn_ref = OA.gradients(w.u0, w.extra["target"], ops, w.dz, n, w.gamma)
    m = lib_mesh(w, dtype)
    assert m.tuning["fused"] >= 2  # the step-tile adjoint
    m.set_index_perturbation(torch.from_numpy(dn).to(DEV))
    tgt = dev(w.extra["target"], dtype)
    h0 = torch.from_numpy(ops.H0).to(DEV)
    out = {}
    for every in (5, n):
        say("adjoint every", dtype, every)
        wsp = torch.empty(m.workspace_size(n, every), dtype=torch.uint8, device=DEV)
        u = dev(w.u0, dtype)
        m.forward_checkpointed(u, w.dz, n, w.gamma, wsp, every)
        c = m.overlap(tgt, u)
        gout = (2 * c * h0 * tgt.to(torch.complex128)).to(u.dtype)
        first = m.adjoint(gout, w.dz, n, w.gamma, wsp, every)
        second = m.adjoint(gout, w.dz, n, w.gamma, wsp, every)
        assert torch.equal(first[0], second[0]) and torch.equal(first[1], second[1])
        out[every] = (host(u), host(first[0]), first[1].cpu().numpy())
    assert np.array_equal(out[5][0], out[n][0])
    assert np.array_equal(out[5][1], out[n][1]) and np.array_equal(out[5][2], out[n][2])
    tol = 1e-9 if dtype == "c128" else 1e-4
    assert rel(out[n][1], g_ref) < tol and rel(out[n][2], gdn_ref) < tol


@pytest.mark.parametrize("dtype,nl", [("c128", "dec"), ("c64", "dec"), ("c128", "lumped")])
def test_pml_adjoint_matches_oracle_gradients(dtype, nl):
    """The adjoint with a perfectly matched layer (complex L weights on the step tiles):
    the field and index gradients of the checkpointed forward and reverse sweep against
    the oracle's exact adjoint on the stretched operators.  The target reaches into the
    layer, where an adjoint that transposes L without conjugating it is off by 46% in the
    field gradient and 0.4% in the index gradient.  In complex128 (triangle-averaged
    nonlinearity) the autograd function gives the same gradients and agrees with central
    differences of the library's own forward."""
    mesh = M.disk_mesh(4.0, 0.1, 6)
    V = F.step_index_tri(mesh.xy, mesh.tri, 1.5, 0.8)
    pml = (2.5, 4.0, 1.5)
    dn = np.random.default_rng(61).normal(0.0, 1e-2, mesh.n_vert)
    u0 = F.gaussian(mesh.xy, 1.0, 1.2) * np.exp(2j * mesh.xy[:, 0])
    target = F.gaussian(mesh.xy, 1.0, 1.0, centre=(2.6, 0.0)) * np.exp(0.7j)
    dz, n, gamma, every = 2e-3, 24, 1.0, 5
    ops = dec.assemble(mesh.xy, mesh.tri, index_tri=V, pml=pml, dn=dn, nl=nl)
    J, g_ref, gdn_ref = OA.gradients(u0, target, ops, dz, n, gamma)
    say("pml adjoint", dtype, nl, mesh.n_vert, n)
    m = api.Mesh(mesh.xy, mesh.tri, V, None, dtype=dtype, pml=pml, nonlinearity=nl)
    dn_d = torch.from_numpy(dn).to(DEV)
    m.set_index_perturbation(dn_d)
    u = dev(u0, dtype)
    wsp = torch.empty(m.workspace_size(n, every), dtype=torch.uint8, device=DEV)
    m.forward_checkpointed(u, dz, n, gamma, wsp, every)
    assert rel(host(u), S.propagate(u0, ops, dz, n, gamma)) < GATE[dtype]
    tgt = dev(target, dtype)
    h0 = torch.from_numpy(ops.H0).to(DEV)
    c = m.overlap(tgt, u)
    g0, gdn = m.adjoint((2 * c * h0 * tgt.to(torch.complex128)).to(u.dtype), dz, n, gamma, wsp, every)
    tol = 1e-9 if dtype == "c128" else 1e-4
    eu, en = rel(host(g0), g_ref), rel(gdn.cpu().numpy(), gdn_ref)
    say("  gradient errors", eu, en)
    assert eu < tol and en < tol, (eu, en)
    if dtype != "c128" or nl != "dec":
        return
    m.set_index_perturbation(None)

    def obj(x, d):
        v = api.propagate_with_grad(m, x, d, dz, n, gamma, every=every)
        c = (h0 * tgt.conj() * v).sum()
        return (c.conj() * c).real

    x = dev(u0, dtype).requires_grad_(True)
    d = dn_d.clone().requires_grad_(True)
    obj(x, d).backward()
    assert rel(host(x.grad), g_ref) < tol and rel(d.grad.cpu().numpy(), gdn_ref) < tol
    rng = np.random.default_rng(62)
    with torch.no_grad():
        du = dev(rng.normal(size=mesh.n_vert) + 1j * rng.normal(size=mesh.n_vert), dtype)
        e = torch.from_numpy(rng.normal(size=mesh.n_vert)).to(DEV)
        fd_u = (obj(x + 1e-6 * du, d) - obj(x - 1e-6 * du, d)) / 2e-6
        an_u = (x.grad.conj() * du).real.sum()
        fd_n = (obj(x, d + 1e-4 * e) - obj(x, d - 1e-4 * e)) / 2e-4
        an_n = (d.grad * e).sum()
    say("  fd", float(fd_u), float(an_u), float(fd_n), float(an_n))
    assert abs(float(fd_u - an_u)) < 1e-6 * abs(float(fd_u))
    assert abs(float(fd_n - an_n)) < 1e-5 * abs(float(fd_n))


def test_autograd_function_and_finite_differences():
    w = W.adjoint_mmf(n_vert=3000, n_steps=10)
    n = 16
    m = lib_mesh(w, "c128")
    tgt = dev(w.extra["target"], "c128")
    h0 = torch.from_numpy(oracle_ops(w).H0).to(DEV)

    def J(u0, dn):
        u = api.propagate_with_grad(m, u0, dn, w.dz, n, w.gamma)
        c = (h0 * tgt.conj() * u).sum()
        return (c.conj() * c).real

    u0 = dev(w.u0, "c128").requires_grad_(True)
    dn = torch.from_numpy(w.extra["dn"]).to(DEV).requires_grad_(True)
    val = J(u0, dn)
    val.backward()
    rng = np.random.default_rng(3)
    with torch.no_grad():
        d = dev(rng.normal(size=m.n_vert) + 1j * rng.normal(size=m.n_vert), "c128")
        e = torch.from_numpy(rng.normal(size=m.n_vert)).to(DEV)
        eps = 1e-6
        fd_u = (J(u0 + eps * d, dn) - J(u0 - eps * d, dn)) / (2 * eps)
        an_u = (u0.grad.conj() * d).real.sum()
        assert abs(float(fd_u - an_u)) < 1e-6 * abs(float(fd_u))
        fd_n = (J(u0, dn + 1e-4 * e) - J(u0, dn - 1e-4 * e)) / 2e-4
        an_n = (dn.grad * e).sum()
        assert abs(float(fd_n - an_n)) < 1e-6 * abs(float(fd_n))


def test_autograd_calls_leave_the_mesh_as_they_found_it():
    """propagate_with_grad installs its index perturbation for its own forward and
    backward only: several forwards may precede their backwards (in any order) and give
    the gradients of one call at a time, bitwise; a plain propagate afterwards sees the
    perturbation the mesh had before (none, or the one the caller installed)."""
    w = W.adjoint_mmf(n_vert=3000, n_steps=10)
    n = 12
    m = lib_mesh(w, "c128")
    tgt = dev(w.extra["target"], "c128")
    h0 = torch.from_numpy(oracle_ops(w).H0).to(DEV)
    dns = [torch.from_numpy(w.extra["dn"]).to(DEV), torch.from_numpy(0.5 * w.extra["dn"][::-1].copy()).to(DEV)]

    def obj(u):
        c = (h0 * tgt.conj() * u).sum()
        return (c.conj() * c).real

    def leaves(d):
        return dev(w.u0, "c128").requires_grad_(True), d.clone().requires_grad_(True)

    refs = []
    for d in dns:
        u0, dd = leaves(d)
        obj(api.propagate_with_grad(m, u0, dd, w.dz, n, w.gamma)).backward()
        refs.append((host(u0.grad), dd.grad.cpu().numpy()))
    a, b = leaves(dns[0]), leaves(dns[1])
    ja = obj(api.propagate_with_grad(m, a[0], a[1], w.dz, n, w.gamma))
    jb = obj(api.propagate_with_grad(m, b[0], b[1], w.dz, n, w.gamma))
    f = dev(w.u0, "c128")
    m.propagate(f, w.dz, n, w.gamma)
    g = dev(w.u0, "c128")
    lib_mesh(w, "c128").propagate(g, w.dz, n, w.gamma)
    assert np.array_equal(host(f), host(g))  # no perturbation left behind
    jb.backward()
    ja.backward()
    for (u0, dd), (gu, gd) in zip((a, b), refs):
        assert np.array_equal(host(u0.grad), gu) and np.array_equal(dd.grad.cpu().numpy(), gd)
    m.set_index_perturbation(dns[1])
    f1 = dev(w.u0, "c128")
    m.propagate(f1, w.dz, n, w.gamma)
    u0, dd = leaves(dns[0])
    obj(api.propagate_with_grad(m, u0, dd, w.dz, n, w.gamma)).backward()
    assert np.array_equal(host(u0.grad), refs[0][0])
    f2 = dev(w.u0, "c128")
    m.propagate(f2, w.dz, n, w.gamma)
    assert np.array_equal(host(f1), host(f2))  # the caller's perturbation is back


def test_adjoint_full_size_directional_derivatives():
    """The full 498k-vertex multimode-fibre adjoint workload in the bench's launch configuration
    (autotuned), 40 steps with 7-step checkpoints: the adjoint's field and index gradients
    against central differences of the library's own forward (complex128), and the complex64
    gradients against the complex128 ones to 1e-4 (the workload's finite-difference bar)."""
    w = case("adjoint")
    n = 40
    say("adjoint full size", w.mesh.n_vert, n)
    grads = {}
    for dtype in ("c128", "c64"):
        m = lib_mesh(w, dtype)
        m.autotune(w.dz, w.gamma)
        tgt = dev(w.extra["target"], dtype)
        h0 = torch.from_numpy(m.export_operators()["h0"]).to(DEV)

        def J(u0, dn):
            u = api.propagate_with_grad(m, u0, dn, w.dz, n, w.gamma, every=7)
            c = (h0 * tgt.conj() * u).sum()
            return (c.conj() * c).real

        u0 = dev(w.u0, dtype).requires_grad_(True)
        dn = torch.from_numpy(w.extra["dn"]).to(DEV).requires_grad_(True)
        J(u0, dn).backward()
        grads[dtype] = (u0.grad.detach().to(torch.complex128), dn.grad.detach())
        if dtype == "c128":
            rng = np.random.default_rng(4)
            with torch.no_grad():
                d = dev(rng.normal(size=m.n_vert) + 1j * rng.normal(size=m.n_vert), dtype)
                e = torch.from_numpy(rng.normal(size=m.n_vert)).to(DEV)
                fd_u = (J(u0 + 1e-6 * d, dn) - J(u0 - 1e-6 * d, dn)) / 2e-6
                an_u = (u0.grad.conj() * d).real.sum()
                fd_n = (J(u0, dn + 1e-4 * e) - J(u0, dn - 1e-4 * e)) / 2e-4
                an_n = (dn.grad * e).sum()
            say("  fd", float(fd_u), float(an_u), float(fd_n), float(an_n))
            assert abs(float(fd_u - an_u)) < 1e-6 * abs(float(fd_u))
            assert abs(float(fd_n - an_n)) < 1e-5 * abs(float(fd_n))
    gu = rel(grads["c64"][0].cpu().numpy(), grads["c128"][0].cpu().numpy())
    gn = rel(grads["c64"][1].cpu().numpy(), grads["c128"][1].cpu().numpy())
    say("  c64 vs c128 gradients", gu, gn)
    assert gu < 1e-4 and gn < 1e-4


def test_autotune_keeps_results():
    w = case("plain_small")
    m = lib_mesh(w, "c64")
    u = dev(w.u0, "c64")
    a = u.clone()
    m.propagate(a, w.dz, 40, 1.0)
    t = m.autotune(w.dz, 1.0)
    say("tuned", t)
    b = u.clone()
    m.propagate(b, w.dz, 40, 1.0)
    assert rel(host(a), host(b)) < 1e-6  # block size / graphs do not change the arithmetic
    times = m.time_kernels(w.dz, 1.0, reps=20)
    assert all(v["ms"] > 0 for v in times.values())


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("nl", ["dec", "lumped"])
def test_fused_tile_path_matches_unfused_and_oracle(dtype, nl):
    """The two-kernel LDS-tiled step (stages 2+3; stage 4 + Kerr + next stage 1)
    against the five-kernel step and the oracle, for odd and even step counts."""
    w = case("step_index", n_vert=20000, n_steps=10)
    say("fused", dtype, nl, w.mesh.n_vert)
    ops = oracle_ops(w, nl)
    m = lib_mesh(w, dtype, nl)
    assert m.tuning["fused"] == 2  # default: the one-kernel step
    m.tuning = {"fused": 1}
    assert m.tuning["fused"] == 1
    u = dev(w.u0, dtype)
    for n in (1, 2, 3, 37, 64):
        outs = {}
        for fused, spg in ((1, 1), (1, 16), (0, 16)):
            m.tuning = {"fused": fused, "steps_per_graph": spg}
            f = u.clone()
            m.propagate(f, w.dz, n, w.gamma)
            outs[(fused, spg)] = host(f)
        assert np.array_equal(outs[(1, 1)], outs[(1, 16)]), n  # graph replay == eager
        tol = 1e-13 if dtype == "c128" else 1e-5
        assert rel(outs[(1, 16)], outs[(0, 16)]) < tol, (n, rel(outs[(1, 16)], outs[(0, 16)]))
        ref = S.propagate(w.u0, ops, w.dz, n, w.gamma)
        assert rel(outs[(1, 16)], ref) < GATE[dtype], n
        if n == 37:
            keep = outs[(1, 16)]
    for tb in (128, 512, 1024):  # threads per tile do not change the arithmetic
        m.tuning = {"fused": 1, "tile_block": tb, "steps_per_graph": 16}
        f = u.clone()
        m.propagate(f, w.dz, 37, w.gamma)
        assert np.array_equal(host(f), keep), tb


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("nl", ["dec", "lumped"])
def test_one_kernel_step_matches_unfused_and_oracle(dtype, nl):
    """The one-kernel z step (four stages + Kerr/absorber on a tile with five
    halo rings in LDS) against the five-kernel step and the oracle."""
    w = case("step_index", n_vert=20000, n_steps=10)
    say("step kernel", dtype, nl, w.mesh.n_vert)
    ops = oracle_ops(w, nl)
    m = lib_mesh(w, dtype, nl)
    m.tuning = {"fused": 2}
    assert m.tuning["fused"] == 2
    u = dev(w.u0, dtype)
    for n in (1, 2, 3, 37, 64):
        outs = {}
        for fused, spg in ((2, 1), (2, 16), (0, 16)):
            m.tuning = {"fused": fused, "steps_per_graph": spg}
            f = u.clone()
            m.propagate(f, w.dz, n, w.gamma)
            outs[(fused, spg)] = host(f)
        assert np.array_equal(outs[(2, 1)], outs[(2, 16)]), n  # graph replay == eager
        tol = 1e-13 if dtype == "c128" else 1e-5
        assert rel(outs[(2, 16)], outs[(0, 16)]) < tol, (n, rel(outs[(2, 16)], outs[(0, 16)]))
        ref = S.propagate(w.u0, ops, w.dz, n, w.gamma)
        assert rel(outs[(2, 16)], ref) < GATE[dtype], n
        if n == 37:
            keep = outs[(2, 16)]
    for tb in (256, 512, 1024):  # threads per tile do not change the arithmetic
        m.tuning = {"fused": 2, "tile_block": tb, "steps_per_graph": 16}
        f = u.clone()
        m.propagate(f, w.dz, 37, w.gamma)
        assert np.array_equal(host(f), keep), tb
    times = m.time_kernels(w.dz, w.gamma, reps=20)
    assert times["step"]["ms"] > 0


_LAYOUT_RUN = r"""
import sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
from paper_2608_03587_amd import api
from paper_2608_03587_amd.inputs import workloads as W
w = W.step_index(n_vert=20000, n_steps=10)
out = {}
for pml in (None, (35.0, 40.0, 1.0)):
    m = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, None if pml else w.absorber, dtype="c64", pml=pml)
    m.tuning = {"fused": 3, "tile_block": 1024, "xcd_remap": 1}
    assert m.tuning["fused"] == 3
    f = torch.from_numpy(w.u0).to("cuda", torch.complex64)
    m.propagate(f, w.dz, 57, w.gamma)
    torch.cuda.synchronize()
    out["pml" if pml else "absorber"] = f.cpu().numpy()
    m.close()
np.savez(sys.argv[2], **out)
print("layout run done", flush=True)
"""


def test_persistent_fixed_lds_layout_matches_runtime_layout(tmp_path):
    """The complex64 persistent split step with its per-slot buffers at constant offsets
    in static LDS and the neighbour slots held as byte offsets (the default) gives the
    bits of the runtime-sized layout (DEC_BPM_FIXED_LDS=0), with the absorber and with
    the layer's complex weights.  Each layout runs in a process of its own (the switch
    is read once per process)."""
    import os
    import subprocess

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = {}
    for env in ("0", "1"):
        say("layout run", env)
        out = str(tmp_path / f"layout_{env}.npz")
        r = subprocess.run([sys.executable, "-c", _LAYOUT_RUN, root, out], capture_output=True, text=True,
                           timeout=300, env=dict(os.environ, DEC_BPM_FIXED_LDS=env))
        assert r.returncode == 0, (env, r.stdout[-2000:], r.stderr[-3000:])
        res[env] = np.load(out)
    for k in ("absorber", "pml"):
        assert np.array_equal(res["0"][k], res["1"][k]), k


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("nl", ["dec", "lumped"])
def test_persistent_launch_matches_step_kernel_and_oracle(dtype, nl):
    """All middle steps in one persistent launch (operator rows in
    registers, neighbour-tile flags instead of kernel boundaries) against the
    one-kernel step (same arithmetic: bitwise) and the oracle."""
    w = case("step_index", n_vert=20000, n_steps=10)
    say("persistent", dtype, nl, w.mesh.n_vert)
    ops = oracle_ops(w, nl)
    m = lib_mesh(w, dtype, nl)
    m.tuning = {"fused": 3, "steps_per_graph": 16}
    assert m.tuning["fused"] == 3
    assert m.time_kernels(w.dz, w.gamma, reps=20)["persist"]["ms"] > 0  # the tiles fit: the path is in use
    u = dev(w.u0, dtype)
    for n in (1, 2, 3, 37, 64, 200):
        outs = {}
        for fused in (3, 2):
            m.tuning = {"fused": fused}
            f = u.clone()
            m.propagate(f, w.dz, n, w.gamma)
            outs[fused] = host(f)
        m.check_finite()
        assert np.array_equal(outs[3], outs[2]), (n, rel(outs[3], outs[2]))
        if n <= 64:
            ref = S.propagate(w.u0, ops, w.dz, n, w.gamma)
            assert rel(outs[3], ref) < GATE[dtype], n
    # block sizes, and the XCD-aware block order (grid padded to a multiple of 8 with
    # workgroups that leave at once)
    for tb, x in ((512, 0), (1024, 0), (1024, 1)):
        m.tuning = {"fused": 3, "tile_block": tb, "xcd_remap": x}
        f = u.clone()
        m.propagate(f, w.dz, 37, w.gamma)
        m.check_finite()
        m.tuning = {"fused": 2, "xcd_remap": 0}
        g = u.clone()
        m.propagate(g, w.dz, 37, w.gamma)
        assert np.array_equal(host(f), host(g)), (tb, x)


@pytest.mark.gpu
def test_persistent_launches_on_two_streams_and_cooperative(monkeypatch):
    """The persistent step is an ordinary launch whose workgroups must all be
    resident: launches of two handles on two streams, queued back to back with
    no host synchronisation, are ordered by the library and give the bits of
    the same launches on one stream; the cooperative launch
    (DEC_BPM_COOPERATIVE=1) gives them too."""
    w = case("step_index", n_vert=20000, n_steps=10)
    u = dev(w.u0, "c64")
    ms = [lib_mesh(w, "c64", "dec") for _ in range(2)]
    for m in ms:
        m.tuning = {"fused": 3}
        assert m.time_kernels(w.dz, w.gamma, reps=20)["persist"]["ms"] > 0
    ref = u.clone()
    ms[0].propagate(ref, w.dz, 57, w.gamma)
    ref = host(ref)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    fs = [u.clone(), u.clone()]
    torch.cuda.synchronize()
    for rep in range(6):  # 6 x 57 steps alternating between the streams, then compare
        for i in (0, 1):
            with torch.cuda.stream(streams[i]):
                if rep:
                    fs[i].copy_(u)
                ms[i].propagate(fs[i], w.dz, 57, w.gamma, stream=streams[i])
    torch.cuda.synchronize()
    for m, f in zip(ms, fs):
        m.check_finite()
        assert np.array_equal(host(f), ref)
    monkeypatch.setenv("DEC_BPM_COOPERATIVE", "1")
    mc = lib_mesh(w, "c64", "dec")
    monkeypatch.delenv("DEC_BPM_COOPERATIVE")
    mc.tuning = {"fused": 3}
    g = u.clone()
    mc.propagate(g, w.dz, 57, w.gamma)
    mc.check_finite()
    assert np.array_equal(host(g), ref)


@pytest.mark.gpu
def test_propagate_captured_in_a_graph():
    """dec_bpm_propagate and dec_bpm_propagate_unsplit captured into a HIP graph (a handle
    tuned for the persistent launch runs one kernel per step while its stream is being
    captured: the persistent flags grow from call to call, which a replay would not
    follow) and dec_bpm_propagate_noalloc (the persistent launch, its flags cleared by a
    kernel in every call): each graph replayed three times, with eager calls and
    synchronisation between the replays, and every replay equal to the eager result
    (the unsplit integrator on one kernel per step, whose eager calls replay the
    library's own graphs)."""
    w = case("step_index", n_vert=20000, n_steps=10)
    m = lib_mesh(w, "c64")
    m.tuning = {"fused": 3}
    assert m.time_kernels(w.dz, w.gamma, reps=10)["persist"]["ms"] > 0
    u = dev(w.u0, "c64")
    n = 9
    # the unsplit integrator on one kernel per step (fused = 2): its persistent body and
    # its per-step kernel agree to rounding only
    fused = {"propagate": 3, "propagate_noalloc": 3, "propagate_unsplit": 2}
    refs = {}
    for call in (m.propagate, m.propagate_unsplit):
        m.tuning = {"fused": fused[call.__name__]}
        r = u.clone()
        call(r, w.dz, n, w.gamma)
        refs[call.__name__] = host(r)
    refs["propagate_noalloc"] = refs["propagate"]
    for call in (m.propagate, m.propagate_noalloc, m.propagate_unsplit):
        m.tuning = {"fused": fused[call.__name__]}
        ref = refs[call.__name__]
        f = u.clone()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):  # an eager call on the capture stream first
            call(f, w.dz, n, w.gamma, stream=s)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        assert np.array_equal(host(f), ref)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            call(f, w.dz, n, w.gamma, stream=s)
        for rep in range(3):
            f.copy_(u)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(host(f), ref), (call.__name__, rep)
            h = u.clone()
            call(h, w.dz, n, w.gamma)  # eager work between the replays
            torch.cuda.synchronize()
            assert np.array_equal(host(h), ref)
        m.check_finite()
        del g


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_results_do_not_depend_on_the_tiling(dtype, monkeypatch):
    """Cutting the mesh into tiles of other row counts (not powers of two, so
    the last tile is ragged; 97 rows gives about 200 tiles with halos spanning
    many tiles) moves rows within LDS and changes which tiles exchange halos,
    not the per-row arithmetic.  The split step (one kernel per step and
    persistent), the unsplit step and the adaptive run (per-trial kernels and
    persistent; its error norm is summed tile by tile) agree with the default
    tiling to rounding (the split step bitwise), and the adaptive run takes the
    same steps."""
    w = case("step_index", n_vert=20000, n_steps=10)
    u = dev(w.u0, dtype)
    rtol, atol = (1e-9, 1e-11) if dtype == "c128" else (1e-5, 1e-7)
    tol = 1e-13 if dtype == "c128" else 1e-6

    def run(env):
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        m = lib_mesh(w, dtype, "dec")
        for k in env:
            monkeypatch.delenv(k)
        out = {}
        for fused in (2, 3):
            m.tuning = {"fused": fused}
            f = u.clone()
            m.propagate(f, w.dz, 40, w.gamma)
            out[("split", fused)] = host(f)
            g = u.clone()
            m.propagate_unsplit(g, w.dz, 40, w.gamma)
            out[("unsplit", fused)] = host(g)
            a = u.clone()
            st = m.propagate_adaptive(a, 10 * w.dz, w.dz, w.gamma, rtol=rtol, atol=atol)
            out[("adaptive", fused)] = host(a)
            out[("steps", fused)] = (st["accepted"], st["rejected"])
            m.check_finite()
        return out

    ref = run({})
    for env in ({"DEC_BPM_STEP_TILE": "333", "DEC_BPM_DP5_TILE": "300"},
                {"DEC_BPM_STEP_TILE": "97", "DEC_BPM_DP5_TILE": "129"}):
        say("tiling", dtype, env)
        got = run(env)
        for key, r in ref.items():
            if key[0] == "steps":
                assert got[key] == r, (env, key)
                continue
            say("  ", key, "bitwise" if np.array_equal(got[key], r) else f"rel {rel(got[key], r):.2e}")
            if key[0] == "split":  # same per-row operations in the same order
                assert np.array_equal(got[key], r), (env, key, rel(got[key], r))
            assert rel(got[key], r) < tol, (env, key)


def test_persistent_wait_bound_ends_the_launch(monkeypatch):
    """With a wait bound of zero polls a tile that finds a neighbour behind
    leaves the launch; the launch still ends and the next finiteness check
    reports it (or, if no wait was ever needed, the result is exact)."""
    w = case("step_index", n_vert=20000, n_steps=10)
    monkeypatch.setenv("DEC_BPM_SPIN_LIMIT", "0")
    m = lib_mesh(w, "c64", "dec")
    monkeypatch.delenv("DEC_BPM_SPIN_LIMIT")
    m.tuning = {"fused": 3}
    u = dev(w.u0, "c64")
    f = u.clone()
    m.propagate(f, w.dz, 300, w.gamma)
    torch.cuda.synchronize()
    try:
        m.check_finite()
        timed_out = False
    except api.DecBpmError as e:
        assert e.code == B.ENONFINITE and "timed out" in str(e), str(e)
        timed_out = True
    say("wait bound 0: timed out" if timed_out else "wait bound 0: no wait needed")
    m.check_finite()  # the report clears the flag
    ok = lib_mesh(w, "c64", "dec")
    ok.tuning = {"fused": 3}
    g = u.clone()
    ok.propagate(g, w.dz, 300, w.gamma)
    ok.check_finite()
    ok.tuning = {"fused": 2}
    h = u.clone()
    ok.propagate(h, w.dz, 300, w.gamma)
    assert np.array_equal(host(g), host(h))
    if not timed_out:
        assert np.array_equal(host(f), host(h))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("nl", ["dec", "lumped"])
def test_fused_adjoint_matches_unfused_and_oracle(dtype, nl):
    """The tile-fused checkpointed forwards and adjoints (one kernel per step on
    five-ring tiles; two kernels per step on three-ring tiles) against the
    five-kernel path and the FP64 oracle gradients (field and index
    perturbation)."""
    w = W.adjoint_mmf(n_vert=20000, n_steps=10)
    n, every = 23, 5
    say("fused adjoint", dtype, nl, w.mesh.n_vert, n)
    dn = w.extra["dn"]
    ops = oracle_ops(w, nl, dn=dn)
    J, g_ref, gdn_ref = OA.gradients(w.u0, w.extra["target"], ops, w.dz, n, w.gamma)
    m = lib_mesh(w, dtype, nl)
    m.set_index_perturbation(torch.from_numpy(dn).to(DEV))
    tgt = dev(w.extra["target"], dtype)
    res = {}
    for fused in (2, 1, 0):  # one-kernel steps, two tile kernels, five row kernels
        m.tuning = {"fused": fused}
        u = dev(w.u0, dtype)
        wsp = torch.empty(m.workspace_size(n, every), dtype=torch.uint8, device=DEV)
        m.forward_checkpointed(u, w.dz, n, w.gamma, wsp, every)
        c = m.overlap(tgt, u)
        gout = (2 * c * torch.from_numpy(ops.H0).to(DEV) * tgt.to(torch.complex128)).to(u.dtype)
        g0, gdn = m.adjoint(gout, w.dz, n, w.gamma, wsp, every)
        res[fused] = (host(g0), gdn.cpu().numpy())
    tol = 1e-9 if dtype == "c128" else 1e-4
    for fused in (2, 1, 0):
        assert rel(res[fused][0], g_ref) < tol, (fused, rel(res[fused][0], g_ref))
        assert rel(res[fused][1], gdn_ref) < tol, (fused, rel(res[fused][1], gdn_ref))
    agree = 1e-12 if dtype == "c128" else 1e-5
    for fused in (2, 1):
        assert rel(res[fused][0], res[0][0]) < agree, fused
        assert rel(res[fused][1], res[0][1]) < agree, fused

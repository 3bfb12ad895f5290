"""Write the stored FP64 oracle references of the full-length GPU parity tests.

Calls only ``oracle/`` and the seeded input generators (``inputs/``); nothing
here reads or runs the HIP library.  Run from the repository root, one
workload per process, e.g.::

    OMP_NUM_THREADS=1 python tests/golden/make_references.py step_index

The stored vortex reference was made with ``vortex_beta4 --stop-after-crossing
--max-seconds 18000`` (the march ends at the first probe past the complex64
limit, step 4900 of 10000, after about 8000 s on one core).

What each run stores (``tests/golden/ref_<name>.npz`` plus a text summary):

* The oracle's field along z, marched by its own Strang step, and beside it
  (one process each) perturbed copies that measure how far a comparison at a
  given precision stays well posed on a supercritical launch, where rounding
  differences grow along z:

  - ``input``: the launch perturbed once by a relative ``eps = 1e-7``
    (``u0 (1 + eps (xi1 + i xi2)/sqrt 2)``, seed 7); ``kappa(z)`` is the growth
    of that relative difference (the amplification of one perturbation).
  - ``noise64`` / ``noise128``: the field perturbed after every step by a
    relative ``u (xi1 + i xi2)/sqrt 2`` with ``u`` the unit roundoff of FP32
    (2^-24, seed 8) or FP64 (2^-53, seed 9): a stand-in for the rounding a
    run in that precision commits at every step.  ``delta(z)`` is the relative
    difference from the unperturbed run.  Independent per-step errors add up
    like a random walk, about ``u sqrt(n) kappa``, so a single input
    perturbation underestimates a long run's rounding.

* The oracle's field at the largest probed z where ``delta`` of the matching
  precision stays below a tenth of its gate (1e-4 for complex64, 1e-10 for
  complex128): a kernel commits several roundings per row per step, and the
  factor 10 leaves room for them.  Stored in complex64 for the complex64 gate
  and complex128 for the complex128 gate, capped at the workload's length.
* The oracle's field (complex128) at the end of the march: the workload's
  final z, unless --max-seconds ended the march earlier.
* SHA-256 digests of the mesh and launch arrays, so a test can check that the
  seeded generators rebuilt the same inputs.

``adjoint_replica`` stores the oracle's FP64 gradients of the overlap
objective instead (``oracle.adjoint.gradients``, every state kept).
"""
from __future__ import annotations

import argparse
import hashlib
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import adjoint as OA  # noqa: E402
from oracle import dec, stepper  # noqa: E402
from paper_2608_03587_amd.inputs import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
EPS = 1e-7
U = {"c64": 2.0**-24, "c128": 2.0**-53}  # unit roundoff of FP32 and FP64
GATE = {"c64": 1e-4, "c128": 1e-10}
MARGIN = 10.0  # a comparison is made where delta <= gate / MARGIN
PROBES = {"input": (EPS, 7, False), "noise64": (U["c64"], 8, True), "noise128": (U["c128"], 9, True)}


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def _noise(rng, n, amp):
    return amp * (rng.normal(size=n) + 1j * rng.normal(size=n)) / math.sqrt(2.0)


def perturbed(u0: np.ndarray) -> np.ndarray:
    return u0 * (1.0 + _noise(np.random.default_rng(PROBES["input"][1]), u0.shape, EPS))


def _march(conn, psi0, ops, dz, n_steps, gamma, probe, amp, seed):
    """March from psi0 with the oracle's Strang step, multiplying the field by
    (1 + noise) after every step when amp > 0, and hand the field over at every
    probe step until told to stop."""
    rng = np.random.default_rng(seed)
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    for step in range(1, n_steps + 1):
        psi = stepper.strang_step(psi, dz, gamma, ops)
        if amp > 0.0:
            psi = psi * (1.0 + _noise(rng, psi.shape[0], amp))
        if step % probe == 0 or step == n_steps:
            conn.send((step, psi))
            if conn.recv() == "stop":
                break
    conn.close()


def conditioning_run(name, ops, u0, dz, n_steps, gamma, probe, log, probes, max_seconds=None,
                     stop_after_crossing=False):
    """March the launch and its perturbed copies; return the probe history and
    the snapshots at the largest well-posed steps of each precision.  The march
    ends at n_steps, after max_seconds, or (stop_after_crossing) at the first
    probe where every probed precision is past its limit."""
    ctx = mp.get_context("fork")
    pipes, procs = {}, []
    for k in probes:
        amp, seed, per_step = PROBES[k]
        start = perturbed(u0) if k == "input" else u0
        a, b = ctx.Pipe()
        pr = ctx.Process(target=_march, args=(b, start, ops, dz, n_steps, gamma, probe, amp if per_step else 0.0,
                                              seed))
        pr.start()
        pipes[k], procs = a, procs + [pr]
    eps0 = float(np.linalg.norm(perturbed(u0) - u0) / np.linalg.norm(u0))
    hist = []
    snap = {"c64": (0, u0.astype(np.complex64)), "c128": (0, u0.copy())}
    crossed = {"c64": False, "c128": False}
    wanted = {"c64": "noise64" in probes, "c128": "noise128" in probes}
    t0 = time.time()
    psi = np.array(u0, dtype=np.complex128, copy=True)
    for step in range(1, n_steps + 1):
        psi = stepper.strang_step(psi, dz, gamma, ops)
        if not (step % probe == 0 or step == n_steps):
            continue
        got = {}
        for k in probes:
            s2, other = pipes[k].recv()
            assert s2 == step
            got[k] = float(np.linalg.norm(other - psi) / np.linalg.norm(psi))
        kappa = got.get("input", float("nan")) / eps0
        d64, d128 = got.get("noise64", float("nan")), got.get("noise128", float("nan"))
        power = float(np.sum(ops.H0 * np.abs(psi) ** 2))
        hist.append((step, kappa, d64, d128, power))
        for tag, d in (("c64", d64), ("c128", d128)):
            if wanted[tag] and not crossed[tag]:
                if d <= GATE[tag] / MARGIN:
                    snap[tag] = (step, psi.astype(np.complex64) if tag == "c64" else psi.copy())
                else:
                    crossed[tag] = True
        el = time.time() - t0
        log(f"{name}: step {step:6d} z={step * dz:.4f} kappa={kappa:.3e} delta64={d64:.3e} delta128={d128:.3e} "
            f"power={power:.6f} ({el:.0f} s)")
        stop = max_seconds is not None and el > max_seconds
        if stop_after_crossing and all(crossed[t] for t in wanted if wanted[t]):
            stop = True
        for k in probes:
            pipes[k].send("stop" if stop else "go")
        if stop:
            break
    for pr in procs:
        pr.join()
    snap["end"] = (step, psi)
    return np.array(hist), snap, crossed


def _writer(name):
    path = os.path.join(HERE, f"ref_{name}_conditioning.txt")
    f = open(path, "w")

    def log(msg):
        print(msg, flush=True)
        f.write(msg + "\n")
        f.flush()

    return log, f


def _store(name, arrays, log):
    path = os.path.join(HERE, f"ref_{name}.npz")
    np.savez_compressed(path, **arrays)
    log(f"wrote {os.path.relpath(path, ROOT)} ({os.path.getsize(path) / 1e6:.1f} MB)")


def _one(name, w, u0, probe, log, probes=("input", "noise64", "noise128"), max_seconds=None,
         stop_after_crossing=False):
    ops = dec.assemble(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, chi_tri=w.chi_tri, p1=w.p1, beta4=w.beta4)
    log(f"{name}: N={w.mesh.n_vert} dz={w.dz} steps={w.n_steps} gamma={w.gamma} beta4={w.beta4} "
        f"power0={float(np.sum(ops.H0 * np.abs(u0) ** 2)):.6f} probe every {probe}")
    hist, snap, crossed = conditioning_run(name, ops, u0, w.dz, w.n_steps, w.gamma, probe, log, probes,
                                           max_seconds=max_seconds, stop_after_crossing=stop_after_crossing)
    out = {
        "probe_steps": hist[:, 0].astype(np.int64),
        "kappa": hist[:, 1],
        "delta64": hist[:, 2],
        "delta128": hist[:, 3],
        "power": hist[:, 4],
        "reached": np.int64(hist[-1, 0]),
        "inputs_sha256": np.array(digest(w.mesh.xy, w.mesh.tri, u0)),
        "n_vert": np.int64(w.mesh.n_vert),
        "dz": np.float64(w.dz),
        "gamma": np.float64(w.gamma),
        "eps": np.float64(EPS),
        "margin": np.float64(MARGIN),
    }
    if "noise128" in probes:
        out["s_end"] = np.int64(snap["end"][0])
        out["psi_end"] = snap["end"][1]
    for tag, probe_name in (("c64", "noise64"), ("c128", "noise128")):
        if probe_name in probes:
            out[f"s{tag[1:]}"] = np.int64(snap[tag][0])
            out[f"psi{tag[1:]}"] = snap[tag][1]
            out[f"crossed{tag[1:]}"] = np.bool_(crossed[tag])
            log(f"{name}: {tag} well posed to step {snap[tag][0]} (limit crossed: {crossed[tag]}; "
                f"march reached step {int(hist[-1, 0])})")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("name", choices=["step_index", "vortex_beta4", "batched_pcf", "adjoint_replica"])
    ap.add_argument("--mesh", type=int, default=None, help="batched_pcf: one mesh index (0-7)")
    ap.add_argument("--max-seconds", type=float, default=None)
    ap.add_argument("--stop-after-crossing", action="store_true",
                    help="end the march once every probed precision is past its limit")
    a = ap.parse_args()
    if a.name == "step_index":
        log, f = _writer("step_index")
        w = W.step_index()
        _store("step_index", _one("step_index", w, w.u0, 250, log), log)
    elif a.name == "vortex_beta4":
        # complex64 only (the workload's precision)
        log, f = _writer("vortex_beta4")
        w = W.vortex_beta4()
        _store("vortex_beta4", _one("vortex_beta4", w, w.u0, 100, log, probes=("input", "noise64"),
                                    max_seconds=a.max_seconds, stop_after_crossing=a.stop_after_crossing), log)
    elif a.name == "batched_pcf":
        ws = W.batched_pcf()
        idx = range(len(ws)) if a.mesh is None else [a.mesh]
        for i in idx:
            tag = f"batched_pcf{i}"
            log, f = _writer(tag)
            w = ws[i]
            # field 0 of each mesh; complex128 references only on the four smaller meshes
            probes = ("input", "noise64", "noise128") if i < 4 else ("input", "noise64")
            _store(tag, _one(tag, w, w.u0[0], 100, log, probes=probes), log)
    else:
        log, f = _writer("adjoint_replica")
        w = W.adjoint_mmf(n_vert=20_000)
        dn = w.extra["dn"]
        ops = dec.assemble(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, p1=w.p1, beta4=w.beta4, dn=dn)
        t0 = time.time()
        J, g_u0, g_dn = OA.gradients(w.u0, w.extra["target"], ops, w.dz, w.n_steps, w.gamma)
        log(f"adjoint_replica: N={w.mesh.n_vert} steps={w.n_steps} J={J:.12e} "
            f"|g_u0|={np.linalg.norm(g_u0):.6e} |g_dn|={np.linalg.norm(g_dn):.6e} ({time.time() - t0:.0f} s)")
        _store("adjoint_replica", {
            "J": np.float64(J), "g_u0": g_u0, "g_dn": g_dn,
            "inputs_sha256": np.array(digest(w.mesh.xy, w.mesh.tri, w.u0, w.extra["target"], dn)),
            "n_vert": np.int64(w.mesh.n_vert), "n_steps": np.int64(w.n_steps),
        }, log)


if __name__ == "__main__":
    main()

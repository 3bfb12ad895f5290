#!/usr/bin/env python3
"""Throughput benchmark of the DEC beam-propagation hot path on one MI355X.

A "step" is one z step of the whole hot path (merged Strang step: the four RK4
stages of the DEC linear operator and the Kerr + absorber substep) over the
step-index workload: graded disk of radius 40 with ~250k vertices, core of
radius 5 with index contrast 1, absorber ring r > 35 (quadratic up to 0.5),
tilted elliptic Gaussian launch (waists 2 and 4, 30 degrees, amplitude 1.2),
dz = 5e-4, gamma = 1, complex64.  The metric is vertex z-steps per second
(vertices x steps / device time), measured with HIP events on the stream the
kernels run on, inputs already resident in HBM.

Also reported on the same JSON line:
  roofline      the dominant kernel of the tuned launch mode (for the one-kernel
                step: the step kernel itself): algorithmic bytes per launch /
                mean launch time (HIP events over graph-captured back-to-back
                launches on the library's stream) against 8 TB/s; traffic from
                the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary
  cpu_baseline  the FP64 CPU oracle on the same mesh and launch, a bounded
                prefix of steps, single thread
  parity        GPU vs oracle after the same prefix (relative L2)
  extras        complex128 throughput; the unsplit RK4 and adaptive Dormand-Prince
                5(4) integrators; the soliton-launch mode solver; the perfectly
                matched layer; Eq. 1's general
                operator sum and Kerr responses; batched
                photonic-crystal-fibre mode vs
                per-instance plain launches; checkpointed adjoint vs forward;
                the 1M-vertex vortex launch with the beta4 L^2 term
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


COPY_BYTES = 256 << 20

# kernel class timed for the roofline of each launch mode: the kernel that
# takes most of a z step (mode 0: four RK4 stage launches of five; mode 1: the
# larger of the two tile kernels; mode 2: the only kernel; mode 3: the
# persistent launch, per z step)
_DOMINANT = {0: ("stage", "k_stage (RK4 stage: L gather + stage update)", 4),
             1: ("tile_a", "k_fused (stage 4 + Kerr/absorber + next stage 1 on 3-ring LDS tiles)", 1),
             2: ("step", "k_step (whole z step: 4 RK4 stages + Kerr/absorber on 5-ring LDS tiles)", 1),
             3: ("persist", "k_persist (persistent z stepping on resident 5-ring LDS tiles, "
                            "operator rows in registers; time and algorithmic bytes per z step)", 1)}


def oracle_timed(fn):
    """Run an oracle call single-threaded; return (result, seconds)."""
    from threadpoolctl import threadpool_limits

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        out = fn()
        return out, time.perf_counter() - t0


def kernel_roofline(k):
    """HBM roofline of one timed kernel class: algorithmic bytes per launch / launch time."""
    gbps = k["bytes"] / (k["ms"] * 1e-3) / 1e9 if k["ms"] > 0 else 0.0
    return {"kernel_us": k["ms"] * 1e3, "GBps": gbps, "frac": gbps / 8000.0}


def step_bytes(dtype, nl="dec", beta4=False):
    """Algorithmic HBM bytes per vertex and z step of the split step as a chain of
    sparse products would move them: CSR rows of 7 entries (int32 index plus weight)
    and a 4-byte row pointer, each product reading its matrix and input once; the
    four classical RK4 stages move 17 complex vectors (stage 1 reads psi and writes
    the accumulator and the next stage input; stages 2-3 read input, psi and
    accumulator and write accumulator and input; stage 4 reads input, psi and
    accumulator and writes psi); the Kerr/absorber pass gathers M over |psi|^2 and
    reads and writes psi (the lumped form only reads w); beta4 adds a second
    product per stage through a stored intermediate."""
    sr = 4 if dtype == "c64" else 8
    sc = 2 * sr
    m = 7 * (4 + sr) + 4
    b = 4 * m + 17 * sc + ((m + 2 * sc + sr) if nl == "dec" else sr)
    if beta4:
        b += 4 * (m + 2 * sc)
    return b


def dominant_kernel_roofline(mode, kt, n_vert=None, dtype="c64", nl="dec", beta4=False):
    """Roofline of the dominant kernel.  For the one-kernel and persistent steps (one launch
    per z step) ``achieved`` counts the step's algorithmic bytes (``step_bytes`` per vertex);
    those kernels keep the stage vectors (and, persistent, the state and the operator) on
    chip, so the fraction can pass 1: it then says that the bytes a chain of products would
    move never reach HBM.  Beside it: the library's own minimal byte count (operators once,
    state in and out) and, when counters are committed, the DRAM bytes actually moved."""
    cls, name, per_step = _DOMINANT[int(mode)]
    k = kt[cls]
    t = k["ms"] * 1e-3
    if int(mode) in (2, 3) and n_vert:
        alg = step_bytes(dtype, nl, beta4) * n_vert
        basis = f"{step_bytes(dtype, nl, beta4)} B per vertex-step x {n_vert} vertices (chain-of-products model)"
    else:
        alg = k["bytes"]
        basis = "the kernel's own algorithmic bytes per launch"
    achieved = alg / t / 1e9
    return {"bound": "hbm", "kernel": name, "kernel_class": cls, "achieved": achieved, "peak": 8000.0,
            "unit": "GB/s", "frac": achieved / 8000.0, "traffic": None, "bytes_per_launch": alg,
            "bytes_basis": basis, "launch_us": k["ms"] * 1e3, "launches_per_step": per_step,
            "runtime_min_bytes": {"bytes_per_launch": k["bytes"], "GBps": k["bytes"] / t / 1e9,
                                  "frac": k["bytes"] / t / 8e12},
            "kernels_us": {c: v["ms"] * 1e3 for c, v in kt.items() if v["ms"] > 0},
            # every kernel class alone: its own algorithmic bytes per launch / launch time / 8 TB/s
            "kernels_frac": {c: v["bytes"] / (v["ms"] * 1e-3) / 8e12 for c, v in kt.items() if v["ms"] > 0}}


def profile_batched(args, api, W, torch, dev, tdt):
    """The batched workload alone, for rocprofv3: warm-up, then the timed batched propagate."""
    ws = W.batched_pcf()
    F = ws[0].u0.shape[0]
    meshes = [api.Mesh(x.mesh.xy, x.mesh.tri, x.index_tri, x.absorber, dtype=args.dtype) for x in ws]
    batch = api.Batch(meshes, F)
    if args.tuning:
        batch.tuning = json.loads(args.tuning)
    else:
        batch.autotune(ws[0].dz, 1.0)
    p0 = batch.pack([torch.from_numpy(x.u0).to(dev, tdt) for x in ws])
    p = p0.clone()
    batch.propagate(p, ws[0].dz, args.warmup, 1.0)
    p = p0.clone()
    torch.cuda.synchronize()
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record()
    batch.propagate(p, ws[0].dz, args.steps, 1.0)
    s1.record()
    torch.cuda.synchronize()
    batch.check_finite()
    if args.calibrate_copy:  # a plain copy of known size, for scaling the traffic counters
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    vf = sum(x.mesh.n_vert for x in ws) * F
    print(json.dumps({"profile_only": True, "path": "batched", "vertex_fields": vf, "units": args.steps,
                      "us_per_unit": s0.elapsed_time(s1) * 1e3 / args.steps, "tuning": batch.tuning}))
    batch.close()
    for m in meshes:
        m.close()


def profile_adjoint(args, api, W, torch, dev, tdt):
    """The adjoint workload (500k-vertex multimode fibre, --dtype) with the whole run stored:
    the checkpointed forward (one recording step kernel per step) and the reverse sweep (one
    adjoint step kernel per step) over --steps steps, after a warm-up pair of --warmup steps."""
    w = W.adjoint_mmf()
    m = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, dtype=args.dtype)
    if args.tuning:
        m.tuning = json.loads(args.tuning)
    else:
        m.autotune(w.dz, w.gamma)
    m.set_index_perturbation(torch.from_numpy(w.extra["dn"]).to(dev))
    u0 = torch.from_numpy(w.u0).to(dev, tdt)
    tgt = torch.from_numpy(w.extra["target"]).to(dev, tdt)
    h0 = torch.from_numpy(m.export_operators()["h0"]).to(dev)
    ws = torch.empty(m.workspace_size(max(args.steps, args.warmup), max(args.steps, args.warmup)),
                     dtype=torch.uint8, device=dev)

    def run(k):
        f = u0.clone()
        m.forward_checkpointed(f, w.dz, k, w.gamma, ws, k)
        c = m.overlap(tgt, f)
        return m.adjoint((2 * c * h0 * tgt.to(torch.complex128)).to(tdt), w.dz, k, w.gamma, ws, k)

    run(args.warmup)
    torch.cuda.synchronize()
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record()
    g0, gdn = run(args.steps)
    s1.record()
    torch.cuda.synchronize()
    ok = bool(torch.isfinite(torch.view_as_real(g0)).all() and torch.isfinite(gdn).all())
    if args.calibrate_copy:  # a plain copy of known size, for scaling the traffic counters
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps({"profile_only": True, "path": "adjoint", "vertices": w.mesh.n_vert, "units": args.steps,
                      "us_per_unit": s0.elapsed_time(s1) * 1e3 / args.steps, "grad_finite": ok,
                      "tuning": m.tuning}))
    m.close()


def profile_path(args, api, W, torch, dev, tdt):
    """One path alone, for rocprofv3: warm-up, then the timed call; prints one JSON line."""
    if args.profile_path == "batched":
        return profile_batched(args, api, W, torch, dev, tdt)
    if args.profile_path == "adjoint":
        return profile_adjoint(args, api, W, torch, dev, tdt)
    w = W.vortex_beta4() if args.profile_path == "vortex_beta4" else W.step_index()
    pml = (35.0, 40.0, 1.0) if args.profile_path == "pml" else None
    m = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, None if pml else w.absorber, dtype=args.dtype, p1=w.p1,
                 beta4=w.beta4, pml=pml)
    if args.tuning:
        m.tuning = json.loads(args.tuning)
    else:
        m.autotune(w.dz, w.gamma)
    u0 = torch.from_numpy(w.u0).to(dev, tdt)
    rtol, atol = (1e-9, 1e-11) if args.dtype == "c128" else (1e-6, 1e-8)
    dtau = 2.0 / m.spectral_radius()

    def run(k):
        f = u0.clone()
        if args.profile_path == "adaptive":
            return m.propagate_adaptive(f, k * w.dz, w.dz, w.gamma, rtol=rtol, atol=atol)
        if args.profile_path == "mode":
            return m.find_mode(f, 4.0, dtau, w.gamma, tol=0.0, max_iter=k)
        m.propagate(f, w.dz, k, w.gamma)
        return None

    run(args.warmup)
    torch.cuda.synchronize()
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record()
    info = run(args.steps)
    s1.record()
    torch.cuda.synchronize()
    m.check_finite()
    units = args.steps
    if args.profile_path == "adaptive":
        units = info["accepted"] + info["rejected"]
    if args.calibrate_copy:  # a plain copy of known size, for scaling the traffic counters
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps({"profile_only": True, "path": args.profile_path, "vertices": w.mesh.n_vert,
                      "units": units, "us_per_unit": s0.elapsed_time(s1) * 1e3 / units, "tuning": m.tuning}))
    m.close()  # release device memory and graphs before the interpreter (and a profiler) shuts down


def measured_traffic(cls):
    """HBM bytes per launch of the kernel class from the committed rocprofv3
    counter summary, if it was taken on the current kernel sources (else None)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"k_{cls}_step_index_250k.md")
    src = os.path.join(ROOT, "paper_2608_03587_amd", "csrc", "kernels.hip")
    try:
        text = open(path).read()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None, None
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)\s+kernels_hip_sha256_16:\s*([0-9a-f]+)", text)
    if not m:
        return None, None
    if m.group(2) != digest:
        return None, f"{os.path.basename(path)} (stale: kernel sources changed since the counters were taken)"
    return float(m.group(1)), os.path.basename(path)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--dtype", default="c64", choices=["c64", "c128"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile", action="store_true", help="only the timed propagation (for rocprofv3)")
    ap.add_argument("--profile-path", default="split",
                    choices=["split", "vortex_beta4", "pml", "adaptive", "mode", "batched", "adjoint"],
                    help="with --profile: which path to run (split: the step-index propagate; vortex_beta4: the "
                         "1M-vertex beta4 launch; pml: the step-index launch with the layer; adaptive: the "
                         "Dormand-Prince run over --steps dz; mode: --steps mode-solver iterations; batched: the "
                         "8-mesh, 256-field batch; adjoint: checkpointed forward and adjoint of the 500k-vertex "
                         "fibre over --steps steps, the whole run stored)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="with --profile: also run a 256 MiB device copy (traffic counter calibration)")
    ap.add_argument("--tuning", default="", help="fixed launch shape as JSON (skips autotuning), e.g. the "
                                                 "config.tuning of a previous run")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2608_03587_amd import api
    from paper_2608_03587_amd.inputs import workloads as W

    if not torch.cuda.is_available():
        log("no HIP device")
        sys.exit(1)
    dev = torch.device("cuda:0")
    tdt = {"c64": torch.complex64, "c128": torch.complex128}
    if args.profile and args.profile_path != "split":
        profile_path(args, api, W, torch, dev, tdt[args.dtype])
        return

    t0 = time.time()
    w = W.step_index()
    N = w.mesh.n_vert
    log(f"[bench] step_index mesh: {N} vertices, {w.mesh.n_tri} triangles ({time.time() - t0:.1f} s)")

    def make(dtype):
        m = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, dtype=dtype, p1=w.p1, beta4=w.beta4)
        if args.tuning:
            m.tuning = json.loads(args.tuning)
        else:
            m.autotune(w.dz, w.gamma)
        return m

    def timed_propagate(m, dtype, steps, warmup):
        u0 = torch.from_numpy(w.u0).to(dev, tdt[dtype])
        stream = torch.cuda.current_stream()
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record(stream)  # the timing events' first use, outside the timed region
        s1.record(stream)
        f = u0.clone()  # the warm-up runs on the buffer the timed call uses, so it is resident and mapped
        for _ in range(warmup):  # the warm-up steps one call each, so the call path is warm too
            m.propagate(f, w.dz, 1, w.gamma)
        f.copy_(u0)
        torch.cuda.synchronize()
        s0.record(stream)
        m.propagate(f, w.dz, steps, w.gamma, stream=stream)
        s1.record(stream)
        torch.cuda.synchronize()
        m.check_finite()
        return s0.elapsed_time(s1), f

    t_create = time.perf_counter()
    m = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, dtype=args.dtype, p1=w.p1, beta4=w.beta4)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t_create
    if args.tuning:
        m.tuning = json.loads(args.tuning)
    else:
        m.autotune(w.dz, w.gamma)
    log(f"[bench] tuned launch shape {m.tuning}; rho*dz = {m.spectral_radius() * w.dz:.3f}; "
        f"create (host assembly, tiles, upload) {t_create:.2f} s")
    ms, field = timed_propagate(m, args.dtype, args.steps, args.warmup)
    value = N * args.steps / (ms * 1e-3)
    log(f"[bench] {args.dtype}: {args.steps} steps in {ms:.2f} ms -> {value:.4e} vertex z-steps/s")
    if args.profile:
        if args.calibrate_copy:  # a plain copy of known size, for scaling the traffic counters
            src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
        print(json.dumps({"metric": "vertex z-steps/s", "value": value, "profile_only": True,
                          "tuning": m.tuning}))
        m.close()  # release device memory and graphs before the interpreter (and a profiler) shuts down
        return

    # the same K-step measurement repeated five more times (median and spread; the
    # headline value stays the first timed run)
    reps_ms = [timed_propagate(m, args.dtype, args.steps, 0)[0] for _ in range(5)]
    reps_ms.sort()
    log(f"[bench] five more runs: median {reps_ms[2]:.2f} ms (min {reps_ms[0]:.2f}, max {reps_ms[-1]:.2f})")
    kt = m.time_kernels(w.dz, w.gamma, reps=200)
    log(f"[bench] kernel means: " + ", ".join(f"{k} {v['ms'] * 1e3:.2f}us" for k, v in kt.items()))
    log(f"[bench] fraction of 8 TB/s: " + ", ".join(f"{k} {v['bytes'] / (v['ms'] * 1e-3) / 8e12:.3f}"
                                                    for k, v in kt.items() if v['ms'] > 0))
    roofline = dominant_kernel_roofline(m.tuning["fused"], kt, N, args.dtype)
    roofline["traffic"], roofline["traffic_source"] = measured_traffic(roofline["kernel_class"])
    if roofline["traffic"]:
        t = roofline["launch_us"] * 1e-6
        roofline["dram"] = {"bytes_per_launch": roofline["traffic"], "GBps": roofline["traffic"] / t / 1e9,
                            "frac": roofline["traffic"] / t / 8e12}
    # the per-call cost beyond the steps themselves (launch, NL(dz/2) of the caller's field, the
    # first halo exchange, the final write through the permutation)
    out_fixed_us = ms * 1e3 - args.steps * roofline["launch_us"] * roofline["launches_per_step"]
    if int(m.tuning["fused"]) == 3:
        roofline["note"] = ("persistent launch: state in LDS, operator rows in registers, only the halo exchange "
                            "reaches memory; the step is bound by the exchange latency, not by HBM")
    out = {
        "metric": "vertex z-steps/s",
        "value": value,
        "unit": "vertex z-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"step_index: graded disk R=40, {N} vertices, core r<5 dn*k0=1, absorber r>35 "
                               f"(w<=0.5), tilted elliptic Gaussian, dz={w.dz}, gamma={w.gamma}, NL_DEC",
                   "vertices": N, "dz": w.dz, "tuning": m.tuning, "create_s": t_create},
        "roofline": roofline,
        "per_call_fixed_us": out_fixed_us,
        "repeat": {"runs": 5, "median_value": N * args.steps / (reps_ms[2] * 1e-3),
                   "min_ms": reps_ms[0], "median_ms": reps_ms[2], "max_ms": reps_ms[-1]},
    }
    # algorithmic working set of one step (operators, v, w, M_pp, two state buffers)
    # against the 256 MB MALL: the step-index workload is cache-resident
    out["roofline"]["working_set_MB"] = (roofline["runtime_min_bytes"]["bytes_per_launch"] +
                                         N * 2 * (8 if args.dtype == "c64" else 16)) / 1e6
    out["roofline"]["mall_MB"] = 256

    # ---- CPU oracle baseline and parity on the same prefix ----
    if not args.no_cpu:
        from threadpoolctl import threadpool_limits

        from oracle import dec, stepper

        with threadpool_limits(limits=1):
            t1 = time.time()
            ops = dec.assemble(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, p1=w.p1, beta4=w.beta4)
            t_asm = time.time() - t1
            psi = w.u0.copy()
            n_cpu = 0
            t1 = time.time()
            while time.time() - t1 < args.cpu_seconds or n_cpu < 5:
                psi = stepper.strang_step(psi, w.dz, w.gamma, ops)
                n_cpu += 1
            t_cpu = time.time() - t1
        cpu_rate = N * n_cpu / t_cpu
        out["cpu_baseline"] = {"value": cpu_rate, "unit": "vertex z-steps/s", "cores": 1, "kind": "oracle",
                               "sample": f"{n_cpu} steps of the same {N}-vertex workload (FP64 NumPy/SciPy, "
                                         f"single thread; assembly {t_asm:.1f} s excluded)",
                               "cpu": cpu_model(), "host_cpus": os.cpu_count()}
        log(f"[bench] oracle: {n_cpu} steps in {t_cpu:.1f} s -> {cpu_rate:.3e} vertex z-steps/s")
        g = torch.from_numpy(w.u0).to(dev, tdt[args.dtype])
        m.propagate(g, w.dz, n_cpu, w.gamma)
        got = g.cpu().numpy().astype(np.complex128)
        err = float(np.linalg.norm(got - psi) / np.linalg.norm(psi))
        from oracle import diagnostics

        err_h0 = float(np.sqrt(np.sum(ops.H0 * np.abs(got - psi) ** 2) / np.sum(ops.H0 * np.abs(psi) ** 2)))
        out["parity"] = {"rel_l2_vs_oracle": err, "steps": n_cpu, "gate": 1e-4 if args.dtype == "c64" else 1e-10,
                         "pass": err < (1e-4 if args.dtype == "c64" else 1e-10),
                         "rel_l2_h0_weighted": err_h0, "e_rel_eq15": diagnostics.e_rel(got, psi)}
        log(f"[bench] parity after {n_cpu} steps: rel L2 {err:.3e}")

    # ---- extras ----
    if not args.no_extras:
        extras = {}
        other = "c128" if args.dtype == "c64" else "c64"
        try:
            m2 = make(other)
            ms2, _ = timed_propagate(m2, other, args.steps, args.warmup)
            kt2 = m2.time_kernels(w.dz, w.gamma, reps=200)
            r2 = dominant_kernel_roofline(m2.tuning["fused"], kt2, N, other)
            extras[other] = {"value": N * args.steps / (ms2 * 1e-3), "ms_per_step": ms2 / args.steps,
                             "roofline": {k: r2[k] for k in ("kernel", "achieved", "frac", "launch_us")},
                             "tuning": m2.tuning}
            log(f"[bench] {other}: {extras[other]['value']:.4e} vertex z-steps/s")
            del m2
        except Exception as e:  # noqa: BLE001
            extras[other] = {"error": repr(e)}
        try:
            extras["unsplit_rk4"] = bench_unsplit(api, w, torch, dev, tdt, args.steps, not args.no_cpu)
        except Exception as e:  # noqa: BLE001
            extras["unsplit_rk4"] = {"error": repr(e)}
        try:
            extras["adaptive_dp54"] = bench_adaptive(api, w, torch, dev, tdt, not args.no_cpu)
        except Exception as e:  # noqa: BLE001
            extras["adaptive_dp54"] = {"error": repr(e)}
        try:
            extras["pml"] = bench_pml(api, w, torch, dev, tdt, min(args.steps, 2000), not args.no_cpu)
        except Exception as e:  # noqa: BLE001
            extras["pml"] = {"error": repr(e)}
        try:
            extras["mode_solver"] = bench_mode(api, w, torch, dev, tdt, not args.no_cpu)
        except Exception as e:  # noqa: BLE001
            extras["mode_solver"] = {"error": repr(e)}
        try:
            extras["general"] = bench_general(api, w, torch, dev, tdt, min(args.steps, 1000), not args.no_cpu)
        except Exception as e:  # noqa: BLE001
            extras["general"] = {"error": repr(e)}
        try:
            extras["full_length_parity"] = bench_full_length(api, w, torch, dev, tdt)
        except Exception as e:  # noqa: BLE001
            extras["full_length_parity"] = {"error": repr(e)}
        try:
            extras["batched"] = bench_batched(api, W, torch, dev, tdt)
        except Exception as e:  # noqa: BLE001
            extras["batched"] = {"error": repr(e)}
        try:
            extras["adjoint"] = bench_adjoint(api, W, torch, dev, tdt)
        except Exception as e:  # noqa: BLE001
            extras["adjoint"] = {"error": repr(e)}
        try:
            extras["vortex_beta4"] = bench_vortex(api, W, torch, dev, tdt)
        except Exception as e:  # noqa: BLE001
            extras["vortex_beta4"] = {"error": repr(e)}
        out["extras"] = extras
    print(json.dumps(out))


def bench_batched(api, W, torch, dev, tdt):
    """256 fields on 8 photonic-crystal-fibre meshes (20k-200k vertices), 2000 steps, complex64:
    one batched propagation vs per-instance plain propagations (one field per mesh timed at full
    length, scaled by the 32 fields each mesh carries)."""
    import numpy as np

    t0 = time.time()
    ws = W.batched_pcf()
    F = ws[0].u0.shape[0]
    n_steps, dz = ws[0].n_steps, ws[0].dz
    log(f"[bench] batched: meshes {[x.mesh.n_vert for x in ws]} x {F} fields ({time.time() - t0:.1f} s)")
    meshes = [api.Mesh(x.mesh.xy, x.mesh.tri, x.index_tri, x.absorber, dtype="c64") for x in ws]
    batch = api.Batch(meshes, F)
    packed0 = batch.pack([torch.from_numpy(x.u0).to(dev, tdt["c64"]) for x in ws])
    batch.autotune(dz, 1.0)
    p = packed0.clone()
    batch.propagate(p, dz, 50, 1.0)  # warm-up
    p = packed0.clone()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    batch.propagate(p, dz, n_steps, 1.0)
    e1.record()
    torch.cuda.synchronize()
    t_b = e0.elapsed_time(e1)
    outs = batch.unpack(p)
    vf = sum(x.mesh.n_vert for x in ws) * F
    # plain: the first field of every mesh, full length, autotuned per mesh
    t_plain = 0.0
    same = True
    max_rel = max_rel_unfused = 0.0
    for m, x, o in zip(meshes, ws, outs):
        m.autotune(dz, 1.0)
        f = torch.from_numpy(x.u0[0]).to(dev, tdt["c64"])
        m.propagate(f.clone(), dz, 20, 1.0)
        torch.cuda.synchronize()
        e0.record()
        m.propagate(f, dz, n_steps, 1.0)
        e1.record()
        torch.cuda.synchronize()
        t_plain += e0.elapsed_time(e1) * F
        ref = o[0].contiguous()
        max_rel = max(max_rel, float(torch.linalg.norm(ref - f) / torch.linalg.norm(ref)))
        # the unfused plain kernels use the same per-row formulas as the batched kernels
        m.tuning = {"fused": 0}
        g = torch.from_numpy(x.u0[0]).to(dev, tdt["c64"])
        m.propagate(g, dz, n_steps, 1.0)
        same &= bool(torch.equal(ref, g))
        max_rel_unfused = max(max_rel_unfused, float(torch.linalg.norm(ref - g) / torch.linalg.norm(ref)))
    # conditioning of the workload (the launches are supercritical for some fields): the same field
    # of the largest mesh in complex64 and complex128 after the full length, and batched vs plain
    # after a short prefix, where rounding differences have not yet been amplified
    big = max(range(len(ws)), key=lambda i: ws[i].mesh.n_vert)
    x = ws[big]
    m128 = api.Mesh(x.mesh.xy, x.mesh.tri, x.index_tri, x.absorber, dtype="c128")
    f128 = torch.from_numpy(x.u0[0]).to(dev, tdt["c128"])
    m128.propagate(f128, dz, n_steps, 1.0)
    f64 = torch.from_numpy(x.u0[0]).to(dev, tdt["c64"])
    meshes[big].propagate(f64, dz, n_steps, 1.0)
    c64_vs_c128 = float(torch.linalg.norm(f64.to(torch.complex128) - f128) / torch.linalg.norm(f128))
    del m128
    short = 100
    p = packed0.clone()
    batch.propagate(p, dz, short, 1.0)
    prefix_rel = 0.0
    for m, x, o in zip(meshes, ws, batch.unpack(p)):
        f = torch.from_numpy(x.u0[0]).to(dev, tdt["c64"])
        m.propagate(f, dz, short, 1.0)
        r = o[0].contiguous()
        prefix_rel = max(prefix_rel, float(torch.linalg.norm(r - f) / torch.linalg.norm(r)))
    # the dominant kernel of the tuned mode: the field-loop step (fused = 3) or the stage kernel
    cls = "step" if batch.tuning["fused"] == 3 else "stage"
    kt = batch.time_kernels(dz, 1.0, reps=20)[cls]
    res = {"vertex_field_steps_per_s": vf * n_steps / (t_b * 1e-3), "ms": t_b,
           "plain_ms_extrapolated": t_plain, "speedup_vs_plain": t_plain / t_b, "tuning": batch.tuning,
           "kernel": cls, "kernel_us": kt["ms"] * 1e3,
           "kernel_GBps": kt["bytes"] / (kt["ms"] * 1e-3) / 1e9, "kernel_frac_hbm": kt["bytes"] / (kt["ms"] * 1e-3) / 8e12,
           # the field-loop step runs the plain one-kernel step's arithmetic (bitwise equal to the
           # tuned plain propagate); the stage kernels run the row kernels' (bitwise equal to those)
           "batched_equals_tuned_plain_bitwise": max_rel == 0.0,
           "batched_equals_unfused_plain_bitwise": same, "max_rel_vs_unfused_plain": max_rel_unfused,
           "max_rel_vs_tuned_plain": max_rel, f"max_rel_vs_tuned_plain_after_{short}_steps": prefix_rel,
           "largest_mesh_field0_c64_vs_c128_full_length": c64_vs_c128,
           "fields": F * len(ws), "vertex_fields": vf, "steps": n_steps,
           "note": "plain = 8 fields (one per mesh) timed at full length x 32"}
    log(f"[bench] batched: {res['vertex_field_steps_per_s']:.3e} vertex-field z-steps/s, "
        f"{res['speedup_vs_plain']:.1f}x plain, bitwise equal to tuned plain {max_rel == 0.0}")
    return res


def bench_adjoint(api, W, torch, dev, tdt):
    """Adjoint workload: 500k-vertex multimode fibre, 2000 steps, sqrt(N) checkpoints, complex64."""
    t0 = time.time()
    w = W.adjoint_mmf()
    n, dz = w.n_steps, w.dz
    log(f"[bench] adjoint mesh: {w.mesh.n_vert} vertices ({time.time() - t0:.1f} s)")
    m = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, dtype="c64")
    m.autotune(dz, w.gamma)
    m.set_index_perturbation(torch.from_numpy(w.extra["dn"]).to(dev))
    u0 = torch.from_numpy(w.u0).to(dev, tdt["c64"])
    tgt = torch.from_numpy(w.extra["target"]).to(dev, tdt["c64"])
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    f = u0.clone()
    m.propagate(f, dz, 20, w.gamma)
    f = u0.clone()
    torch.cuda.synchronize()
    ev[0].record()
    m.propagate(f, dz, n, w.gamma)
    ev[1].record()
    ws = torch.empty(m.workspace_size(n), dtype=torch.uint8, device=dev)
    g = u0.clone()
    ev[2].record()
    m.forward_checkpointed(g, dz, n, w.gamma, ws)
    ev[3].record()
    c = m.overlap(tgt, g)
    h0 = torch.from_numpy(m.export_operators()["h0"]).to(dev)
    gout = (2 * c * h0 * tgt.to(torch.complex128)).to(torch.complex64)
    torch.cuda.synchronize()
    ev[4].record()
    g0, gdn = m.adjoint(gout, dz, n, w.gamma, ws)
    ev[5].record()
    torch.cuda.synchronize()
    t_f, t_c, t_a = ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3]), ev[4].elapsed_time(ev[5])
    res = {"forward_ms": t_f, "checkpointed_forward_ms": t_c, "adjoint_ms": t_a, "adjoint_over_forward": t_a / t_f,
           "total_over_forward": (t_c + t_a) / t_f, "workspace_MB": ws.numel() / 2**20,
           "vertices": w.mesh.n_vert, "steps": n, "objective": abs(c) ** 2,
           "grad_finite": bool(torch.isfinite(torch.view_as_real(g0)).all() and torch.isfinite(gdn).all())}
    log(f"[bench] adjoint: {t_a / t_f:.2f}x forward (checkpointed fwd + adjoint {res['total_over_forward']:.2f}x)")
    # the whole run stored (every = n_steps: about five field vectors per step of device memory)
    # instead of recomputed from sqrt(N) checkpoints: the same gradients, bitwise
    ws_all = torch.empty(m.workspace_size(n, n), dtype=torch.uint8, device=dev)
    g2 = u0.clone()
    torch.cuda.synchronize()
    ev[2].record()
    m.forward_checkpointed(g2, dz, n, w.gamma, ws_all, n)
    ev[3].record()
    ev[4].record()
    g0_all, gdn_all = m.adjoint(gout, dz, n, w.gamma, ws_all, n)
    ev[5].record()
    torch.cuda.synchronize()
    t_c2, t_a2 = ev[2].elapsed_time(ev[3]), ev[4].elapsed_time(ev[5])
    res["run_stored"] = {"checkpointed_forward_ms": t_c2, "adjoint_ms": t_a2, "total_over_forward": (t_c2 + t_a2) / t_f,
                         "workspace_GB": ws_all.numel() / 2**30,
                         "equals_sqrt_checkpoints_bitwise": bool(torch.equal(g2, g) and torch.equal(g0_all, g0)
                                                                 and torch.equal(gdn_all, gdn))}
    del ws_all
    log(f"[bench] adjoint with the run stored: checkpointed fwd + adjoint "
        f"{res['run_stored']['total_over_forward']:.2f}x forward ({res['run_stored']['workspace_GB']:.1f} GB)")
    # the complex64 gradients against central differences of the complex128 forward, over the whole
    # run, along 4 random field and 4 random index directions
    m.close()
    g_u, g_n = g0.to(torch.complex128), gdn.clone()
    m2 = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, dtype="c128")
    m2.autotune(dz, w.gamma)
    tgt2 = torch.from_numpy(w.extra["target"]).to(dev, tdt["c128"])
    base = torch.from_numpy(w.u0).to(dev, tdt["c128"])
    dn0 = torch.from_numpy(w.extra["dn"]).to(dev)

    def J(x, d):
        m2.set_index_perturbation(d)
        f2 = x.clone()
        m2.propagate(f2, dz, n, w.gamma)
        cc = (h0 * tgt2.conj() * f2).sum()
        return float((cc.conj() * cc).real)

    import numpy as np

    rng = np.random.default_rng(8)
    rows = {"field": ([], []), "index": ([], [])}
    for k in range(8):
        if k < 4:
            d = torch.from_numpy(rng.normal(size=w.mesh.n_vert) + 1j * rng.normal(size=w.mesh.n_vert)).to(dev)
            fd = (J(base + 1e-6 * d, dn0) - J(base - 1e-6 * d, dn0)) / 2e-6
            an = float((g_u.conj() * d).real.sum())
            rows["field"][0].append(fd)
            rows["field"][1].append(an)
        else:
            e = torch.from_numpy(rng.normal(size=w.mesh.n_vert)).to(dev)
            fd = (J(base, dn0 + 1e-4 * e) - J(base, dn0 - 1e-4 * e)) / 2e-4
            an = float((g_n * e).sum())
            rows["index"][0].append(fd)
            rows["index"][1].append(an)
    m2.close()
    fdchk = {}
    for kind, (fd, an) in rows.items():
        fd, an = np.array(fd), np.array(an)
        fdchk[kind] = {"central_difference_c128": fd.tolist(), "adjoint_c64": an.tolist(),
                       "rel": float(np.linalg.norm(an - fd) / np.linalg.norm(fd))}
    res["finite_differences"] = dict(fdchk, gate=1e-4, directions=8,
                                     passed=all(v["rel"] <= 1e-4 for v in fdchk.values()))
    log(f"[bench] adjoint vs central differences: field {fdchk['field']['rel']:.2e}, "
        f"index {fdchk['index']['rel']:.2e}")
    return res


def bench_unsplit(api, w, torch, dev, tdt, steps, with_oracle):
    """The paper's unsplit scheme (classical RK4 on the whole right-hand side, Kerr term inside
    every stage) on the same step-index workload, complex64: throughput, parity with the oracle's
    unsplit RK4 on a 40-step prefix, and its distance to the split scheme at full length."""
    import numpy as np

    m = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, dtype="c64", p1=w.p1, beta4=w.beta4)
    m.autotune(w.dz, w.gamma)
    u0 = torch.from_numpy(w.u0).to(dev, tdt["c64"])
    f = u0.clone()
    m.propagate_unsplit(f, w.dz, 50, w.gamma)
    f = u0.clone()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    m.propagate_unsplit(f, w.dz, steps, w.gamma)
    e1.record()
    torch.cuda.synchronize()
    m.check_finite()
    ms = e0.elapsed_time(e1)
    g = u0.clone()
    m.propagate(g, w.dz, steps, w.gamma)
    split_dist = float(torch.linalg.norm(g - f) / torch.linalg.norm(f))
    kt = m.time_kernels(w.dz, w.gamma, reps=100)["unsplit"]
    res = {"value": w.mesh.n_vert * steps / (ms * 1e-3), "unit": "vertex z-steps/s", "ms_per_step": ms / steps,
           "steps": steps, "kernel_us": kt["ms"] * 1e3, "kernel_GBps": kt["bytes"] / (kt["ms"] * 1e-3) / 1e9,
           "roofline": kernel_roofline(kt),
           "rel_l2_vs_split_scheme_full_length": split_dist, "tuning": m.tuning}
    if with_oracle:
        from oracle import dec, unsplit

        ops = dec.assemble(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, p1=w.p1, beta4=w.beta4)
        n = 40
        ref, sec = oracle_timed(lambda: unsplit.propagate_rk4(w.u0, ops, w.dz, n, w.gamma))
        res["oracle"] = {"us_per_step": sec / n * 1e6, "cores": 1}
        h = u0.clone()
        m.propagate_unsplit(h, w.dz, n, w.gamma)
        got = h.cpu().numpy().astype(np.complex128)
        res["parity"] = {"rel_l2_vs_oracle": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)), "steps": n}
    log(f"[bench] unsplit RK4: {res['value']:.4e} vertex z-steps/s ({res['ms_per_step'] * 1e3:.2f} us per step), "
        f"parity {res.get('parity', {}).get('rel_l2_vs_oracle')}")
    return res


def bench_adaptive(api, w, torch, dev, tdt, with_oracle):
    """The paper's own integrator, adaptive Dormand-Prince 5(4) on the whole right-hand side, on
    the same step-index workload: complex128 at the paper's tolerances (rtol 1e-9, atol 1e-11)
    and complex64 at rtol 1e-6, atol 1e-8, over 400 configured z steps (z_end = 0.2); accepted
    steps per second, the trial kernel's time, and the oracle's adaptive run on a 4-step prefix."""
    import numpy as np

    z_end = 400 * w.dz
    out = {"z_end": z_end, "h0": w.dz}
    for dt, rtol, atol in (("c128", 1e-9, 1e-11), ("c64", 1e-6, 1e-8)):
        m = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, dtype=dt, p1=w.p1, beta4=w.beta4)
        u0 = torch.from_numpy(w.u0).to(dev, tdt[dt])
        f = u0.clone()
        m.propagate_adaptive(f, 4 * w.dz, w.dz, w.gamma, rtol=rtol, atol=atol)  # builds the tiles
        f = u0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = m.propagate_adaptive(f, z_end, w.dz, w.gamma, rtol=rtol, atol=atol)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        m.check_finite()
        kt = m.time_kernels(w.dz, w.gamma, reps=50)["dp5"]
        attempts = st["accepted"] + st["rejected"]
        r = {"rtol": rtol, "atol": atol, **st, "seconds": sec,
             "value": w.mesh.n_vert * st["accepted"] / sec, "unit": "vertex z-steps/s (accepted steps)",
             "us_per_attempt": sec / attempts * 1e6, "trial_kernel_us": kt["ms"] * 1e3,
             "roofline": kernel_roofline(kt),
             "trial_kernel_GBps": kt["bytes"] / (kt["ms"] * 1e-3) / 1e9}
        if with_oracle:
            from oracle import dec, unsplit

            ops = dec.assemble(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, p1=w.p1, beta4=w.beta4)
            (ref, rs), sec_o = oracle_timed(
                lambda: unsplit.propagate_dp54(w.u0, ops, 4 * w.dz, w.dz, w.gamma, rtol=rtol, atol=atol))
            r["oracle"] = {"us_per_attempt": sec_o / (rs["accepted"] + rs["rejected"]) * 1e6, "cores": 1}
            g = u0.clone()
            sg = m.propagate_adaptive(g, 4 * w.dz, w.dz, w.gamma, rtol=rtol, atol=atol)
            got = g.cpu().numpy().astype(np.complex128)
            r["parity"] = {"rel_l2_vs_oracle": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                           "z_end": 4 * w.dz, "gpu_steps": [sg["accepted"], sg["rejected"]],
                           "oracle_steps": [rs["accepted"], rs["rejected"]]}
        out[dt] = r
        log(f"[bench] adaptive DP5(4) {dt}: {st['accepted']} accepted / {st['rejected']} rejected in {sec:.3f} s, "
            f"{r['us_per_attempt']:.1f} us per attempt, trial kernel {r['trial_kernel_us']:.1f} us, "
            f"parity {r.get('parity', {}).get('rel_l2_vs_oracle')}")
    return out


def bench_pml(api, w, torch, dev, tdt, steps, with_oracle):
    """The step-index launch with a perfectly matched layer on 35 < r < 40 (sigma_max 1) in
    place of the absorber, complex64, against the same launch with the absorber: the
    one-kernel step with complex L weights (fused 2) and the persistent launch (fused 3);
    parity with the oracle's split scheme on the stretched operators after 5 steps, the
    oracle timed beside it."""
    import numpy as np

    def timed(m, u0, fused, kind, extra_bytes):
        # the persistent launch in the shape the autotuner picks for this workload
        m.tuning = {"fused": 3, "tile_block": 1024, "xcd_remap": 0} if fused == 3 else {"fused": fused}
        f = u0.clone()
        m.propagate(f, w.dz, 50, w.gamma)
        f = u0.clone()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        m.propagate(f, w.dz, steps, w.gamma)
        e1.record()
        torch.cuda.synchronize()
        m.check_finite()
        ms = e0.elapsed_time(e1)
        kt = m.time_kernels(w.dz, w.gamma, reps=50)[kind]
        kt = dict(kt, bytes=kt["bytes"] + extra_bytes)
        return {"value": w.mesh.n_vert * steps / (ms * 1e-3), "ms_per_step": ms / steps, "tuning": m.tuning,
                "roofline": kernel_roofline(kt)}

    out = {}
    for name, pml, ab in (("pml", (35.0, 40.0, 1.0), None), ("absorber", None, w.absorber)):
        m = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, ab, dtype="c64", p1=w.p1, pml=pml)
        u0 = torch.from_numpy(w.u0).to(dev, tdt["c64"])
        # the step's algorithmic bytes plus, with the layer, its imaginary L weights
        extra = 6 * w.mesh.n_vert * 4 if pml is not None else 0
        out[name] = timed(m, u0, 2, "step", extra)
        out[name]["persistent"] = timed(m, u0, 3, "persist", extra)
        if with_oracle and pml is not None:
            from oracle import dec, stepper

            ops = dec.assemble(w.mesh.xy, w.mesh.tri, w.index_tri, None, p1=w.p1, pml=pml)
            ref, sec = oracle_timed(lambda: stepper.propagate(w.u0, ops, w.dz, 5, w.gamma))
            for key, fused in (("parity", 2), ("parity_persistent", 3)):
                m.tuning = {"fused": fused}
                g = u0.clone()
                m.propagate(g, w.dz, 5, w.gamma)
                got = g.cpu().numpy().astype(np.complex128)
                out[name][key] = {"rel_l2_vs_oracle": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                                  "steps": 5}
            out[name]["oracle"] = {"us_per_step": sec / 5 * 1e6, "cores": 1}
        del m
    log(f"[bench] PML: {out['pml']['ms_per_step'] * 1e3:.2f} us per step vs absorber "
        f"{out['absorber']['ms_per_step'] * 1e3:.2f} us (one-kernel step); persistent "
        f"{out['pml']['persistent']['ms_per_step'] * 1e3:.2f} vs {out['absorber']['persistent']['ms_per_step'] * 1e3:.2f} us; "
        f"parity {out['pml'].get('parity', {}).get('rel_l2_vs_oracle')}, "
        f"{out['pml'].get('parity_persistent', {}).get('rel_l2_vs_oracle')}")
    return out


def bench_general(api, w, torch, dev, tdt, steps, with_oracle):
    """Eq. 1 in full on the step-index mesh (complex64).  Five-kernel path: terms up to
    p4 L^4 (p2..p4 = 1e-9, -1e-12, 1e-16, small enough to keep the configured dz stable)
    with the Kerr response, and the saturable response (I_s = 1) alone, against the same
    path with the plain operator.  Persistent launch: the saturable and cubic-quintic
    responses (no higher terms), whose flow integrals the tile kernels' Kerr phase takes."""
    out = {}
    cases = (("plain", {}, 0), ("L4_sum", {"beta4": 1e-9, "p3": -1e-12, "p4": 1e-16}, 0),
             ("saturable", {"response": "saturable", "response_param": 1.0}, 0),
             ("saturable_persistent", {"response": "saturable", "response_param": 1.0}, 3),
             ("cubic_quintic_persistent", {"response": "cubic_quintic", "response_param": 0.1}, 3))
    for name, kw, fused in cases:
        m = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, dtype="c64", p1=w.p1, **kw)
        m.tuning = {"fused": fused}
        u0 = torch.from_numpy(w.u0).to(dev, tdt["c64"])
        f = u0.clone()
        m.propagate(f, w.dz, 20, w.gamma)
        f = u0.clone()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        m.propagate(f, w.dz, steps, w.gamma)
        e1.record()
        torch.cuda.synchronize()
        m.check_finite()
        ms = e0.elapsed_time(e1)
        out[name] = {"value": w.mesh.n_vert * steps / (ms * 1e-3), "ms_per_step": ms / steps,
                     "rho_dz": m.spectral_radius() * w.dz, "fused": fused}
        if fused == 3:
            out[name]["persistent_live"] = m.time_kernels(w.dz, w.gamma, reps=20)["persist"]["ms"] > 0
        if with_oracle and name != "plain":
            import numpy as np

            from oracle import dec, stepper

            okw = {"beta4": kw.get("beta4", 0.0), "p3": kw.get("p3", 0.0), "p4": kw.get("p4", 0.0),
                   "nl_kind": kw.get("response", "kerr"), "nl_param": kw.get("response_param", 0.0)}
            ops = dec.assemble(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, p1=w.p1, **okw)
            ref, sec = oracle_timed(lambda: stepper.propagate(w.u0, ops, w.dz, 5, w.gamma))
            g = u0.clone()
            m.propagate(g, w.dz, 5, w.gamma)
            got = g.cpu().numpy().astype(np.complex128)
            out[name]["parity"] = {"rel_l2_vs_oracle": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                                   "steps": 5}
            out[name]["oracle"] = {"us_per_step": sec / 5 * 1e6, "cores": 1}
        m.close()
    log("[bench] Eq. 1 in full, us per step: " +
        ", ".join(f"{k} {v['ms_per_step'] * 1e3:.2f}" for k, v in out.items()))
    return out


def bench_mode(api, w, torch, dev, tdt, with_oracle):
    """The soliton-launch mode solver on the step-index mesh (power 4, dtau = 2/rho): time per
    iteration over 2000 fixed iterations, and a complex128 solve to r <= 1e-6 |mu|."""
    out = {}
    for dt in ("c64", "c128"):
        m = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, dtype=dt, p1=w.p1, beta4=w.beta4)
        m.autotune(w.dz, w.gamma)
        u0 = torch.from_numpy(w.u0).to(dev, tdt[dt])
        dtau = 2.0 / m.spectral_radius()
        f = u0.clone()
        m.find_mode(f, 4.0, dtau, w.gamma, tol=0.0, max_iter=20)
        f = u0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.find_mode(f, 4.0, dtau, w.gamma, tol=0.0, max_iter=2000)
        sec = time.perf_counter() - t0
        kt = m.time_kernels(w.dz, w.gamma, reps=50)["mode"]
        r = {"us_per_iteration": sec / 2000 * 1e6, "kernel_us": kt["ms"] * 1e3, "roofline": kernel_roofline(kt)}
        if with_oracle and dt == "c64":
            import numpy as np

            from oracle import dec, soliton

            ops = dec.assemble(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, p1=w.p1, beta4=w.beta4)
            (ref, info), sec_o = oracle_timed(lambda: soliton.find_mode(w.u0, ops, 4.0, dtau, w.gamma, tol=0.0,
                                                                        max_iter=10))
            g = u0.clone()
            m.find_mode(g, 4.0, dtau, w.gamma, tol=0.0, max_iter=10)
            got = g.cpu().numpy().astype(np.complex128)
            r["parity"] = {"rel_l2_vs_oracle": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                           "iterations": 10, "mu_oracle": info["mu"]}
            r["oracle"] = {"us_per_iteration": sec_o / 10 * 1e6, "cores": 1}
        if dt == "c128":
            f = u0.clone()
            t0 = time.perf_counter()
            st = m.find_mode(f, 4.0, dtau, w.gamma, tol=1e-6, max_iter=400000)
            r["solve"] = {**st, "seconds": time.perf_counter() - t0, "tol": 1e-6}
        out[dt] = r
        del m
    log(f"[bench] mode solver: {out['c64']['us_per_iteration']:.1f} us per iteration (c64), "
        f"{out['c128']['us_per_iteration']:.1f} (c128); c128 solve {out['c128']['solve']}")
    return out


def bench_full_length(api, w, torch, dev, tdt):
    """Parity at the workload's final z against the stored FP64 oracle fields, and the oracle's own
    conditioning probe of the launch (both written by tests/golden/make_references.py, which calls
    only the oracle): complex128 over all steps, complex64 to the largest z where the oracle run
    perturbed by one FP32 unit roundoff per step stays within a tenth of the complex64 gate."""
    import numpy as np

    z = np.load(os.path.join(ROOT, "tests", "golden", "ref_step_index.npz"))
    res = {"source": "tests/golden/ref_step_index.npz (FP64 oracle)",
           "oracle_probe": {"steps": z["probe_steps"].tolist(), "kappa_input_1e-7": z["kappa"].tolist(),
                            "delta_fp32_noise": z["delta64"].tolist(), "delta_fp64_noise": z["delta128"].tolist()}}
    for dtype, n, ref, gate in (("c128", int(z["s_end"]), z["psi_end"], 1e-10),
                                ("c64", int(z["s64"]), z["psi64"].astype(np.complex128), 1e-4)):
        m = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, dtype=dtype, p1=w.p1, beta4=w.beta4)
        m.autotune(w.dz, w.gamma)
        f = torch.from_numpy(w.u0).to(dev, tdt[dtype])
        m.propagate(f, w.dz, n, w.gamma)
        m.check_finite()
        got = f.cpu().numpy().astype(np.complex128)
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        res[dtype] = {"steps": n, "z": n * w.dz, "rel_l2_vs_oracle": err, "gate": gate, "pass": err <= gate,
                      "max_vertex_rel": float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))}
        m.close()
        log(f"[bench] full length {dtype}: {n} steps, rel L2 vs oracle {err:.3e} (gate {gate:g})")
    return res


def bench_vortex(api, W, torch, dev, tdt):
    """Vortex launch with the beta4 L^2 term: uniform disk of radius 60 with ~1M vertices, complex64,
    a 1000-step stretch of the 10,000-step run (the beta4 term runs on the five-kernel path)."""
    t0 = time.time()
    w = W.vortex_beta4()
    N = w.mesh.n_vert
    log(f"[bench] vortex_beta4 mesh: {N} vertices ({time.time() - t0:.1f} s)")
    m = api.Mesh(w.mesh.xy, w.mesh.tri, w.index_tri, w.absorber, dtype="c64", p1=w.p1, beta4=w.beta4)
    m.autotune(w.dz, w.gamma)
    f = torch.from_numpy(w.u0).to(dev, tdt["c64"])
    m.propagate(f, w.dz, 50, w.gamma)
    f = torch.from_numpy(w.u0).to(dev, tdt["c64"])
    steps = 1000
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    m.propagate(f, w.dz, steps, w.gamma)
    e1.record()
    torch.cuda.synchronize()
    m.check_finite()
    ms = e0.elapsed_time(e1)
    kt = m.time_kernels(w.dz, w.gamma, reps=50)
    res = {"value": N * steps / (ms * 1e-3), "unit": "vertex z-steps/s", "ms_per_step": ms / steps, "steps": steps,
           "vertices": N, "rho_dz": m.spectral_radius() * w.dz, "tuning": m.tuning,
           "kernels_us": {c: v["ms"] * 1e3 for c, v in kt.items() if v["ms"] > 0}}
    log(f"[bench] vortex_beta4: {res['value']:.3e} vertex z-steps/s ({res['ms_per_step'] * 1e3:.1f} us per step)")
    return res


if __name__ == "__main__":
    main()

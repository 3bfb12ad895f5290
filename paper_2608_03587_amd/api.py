"""Python interface of the DEC beam-propagation library.

Thin marshalling over the C ABI (``include/dec_bpm.h``): every step of the z
march runs in the library's HIP kernels on the GPU.  PyTorch provides device
memory (tensors) and streams only.  There is no CPU fallback: device calls on
a machine without a GPU, or with the library unbuilt, raise.
"""
from __future__ import annotations

import atexit
import ctypes
import math
import weakref

import numpy as np
import torch

from . import _binding as B

# Live handles, released before the interpreter shuts down: freeing device memory
# and graphs from finalisers that run during shutdown can reach a HIP runtime (or
# a profiler attached to it) that has already been torn down.
_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    for obj in list(_LIVE):
        obj.close()

__all__ = ["Mesh", "Batch", "DecBpmFunction", "propagate_with_grad", "DecBpmError"]

DecBpmError = B.DecBpmError

_DT = {"c64": (B.C64, torch.complex64), "c128": (B.C128, torch.complex128)}


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Mesh:
    """Operators of the DEC-discretised NLSE on one triangular mesh.

    Parameters follow ``dec_bpm_create``: vertex coordinates ``xy`` [N,2],
    triangles ``tri`` [T,3] (any orientation), per-triangle index potential
    ``index_tri`` [T], per-vertex absorber ``absorber`` [N], per-triangle Kerr
    coefficient ``chi_tri`` [T]; ``dtype`` "c64" or "c128"; ``p1`` and
    ``beta4`` the coefficients of L and L^2; ``nonlinearity`` "dec" (Eq. 14)
    or "lumped".
    """

    def __init__(self, xy, tri, index_tri=None, absorber=None, chi_tri=None, dtype="c64", p1=0.5, beta4=0.0,
                 nonlinearity="dec", reorder=True, host_only=False, block_size=0, steps_per_graph=0, pml=None,
                 p3=0.0, p4=0.0, response="kerr", response_param=0.0):
        L = B.lib()
        self.dtype_name = dtype
        code, self.torch_dtype = _DT[dtype]
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        if xy.ndim != 2 or xy.shape[1] != 2 or tri.ndim != 2 or tri.shape[1] != 3:
            raise ValueError("xy must be [N,2] and tri [T,3]")
        opt = B.Options()
        L.dec_bpm_default_options(ctypes.byref(opt))
        opt.dtype = code
        opt.p1 = float(p1)
        opt.beta4 = float(beta4)
        opt.nonlinearity = {"dec": B.NL_DEC, "lumped": B.NL_LUMPED}[nonlinearity]
        opt.reorder = int(bool(reorder))
        opt.host_only = int(bool(host_only))
        opt.block_size = int(block_size)
        opt.steps_per_graph = int(steps_per_graph)
        if pml is not None:  # (r0, r1, sigma_max): radial perfectly matched layer
            opt.pml_r0, opt.pml_r1, opt.pml_sigma = (float(v) for v in pml)
        opt.p3, opt.p4 = float(p3), float(p4)
        opt.nl_kind = {"kerr": 0, "saturable": 1, "cubic_quintic": 2}[response]
        opt.nl_param = float(response_param)
        keep = []
        if chi_tri is not None:
            chi = np.ascontiguousarray(chi_tri, dtype=np.float64)
            if chi.shape != (tri.shape[0],):
                raise ValueError("chi_tri must have one entry per triangle")
            keep.append(chi)
            opt.chi_tri = _ptr(chi, ctypes.c_double)
        V = None if index_tri is None else np.ascontiguousarray(index_tri, dtype=np.float64)
        W = None if absorber is None else np.ascontiguousarray(absorber, dtype=np.float64)
        if V is not None and V.shape != (tri.shape[0],):
            raise ValueError("index_tri must have one entry per triangle")
        if W is not None and W.shape != (xy.shape[0],):
            raise ValueError("absorber must have one entry per vertex")
        h = ctypes.c_void_p()
        B.check(L.dec_bpm_create(_ptr(xy, ctypes.c_double), xy.shape[0], _ptr(tri, ctypes.c_int32), tri.shape[0],
                                 None if V is None else _ptr(V, ctypes.c_double),
                                 None if W is None else _ptr(W, ctypes.c_double), ctypes.byref(opt),
                                 ctypes.byref(h)))
        self._h = h
        self._dn = None  # the installed index perturbation (a private copy), or None
        self._destroy = L.dec_bpm_destroy
        self.n_vert = xy.shape[0]
        self.n_tri = tri.shape[0]
        _LIVE.add(self)

    def close(self):
        """Release the handle's device memory now (idempotent); the object is unusable afterwards."""
        h = getattr(self, "_h", None)
        self._h = None
        if h is not None and h.value:
            self._destroy(h)

    def __del__(self):
        self.close()

    @property
    def handle(self):
        return self._h

    # ---- host-side information ----
    def sizes(self):
        v = [ctypes.c_int64() for _ in range(4)]
        B.check(B.lib().dec_bpm_sizes(self._h, *[ctypes.byref(x) for x in v]))
        return dict(n_vert=v[0].value, n_tri=v[1].value, n_edge=v[2].value, nnz=v[3].value)

    def spectral_radius(self) -> float:
        r = ctypes.c_double()
        B.check(B.lib().dec_bpm_spectral_radius(self._h, ctypes.byref(r)))
        return r.value

    def export_operators(self):
        n = self.n_vert
        nnz = ctypes.c_int64()
        L = B.lib()
        B.check(L.dec_bpm_export_operators(self._h, None, None, None, ctypes.byref(nnz), None, None, None, None))
        h0, v, w = (np.empty(n) for _ in range(3))
        rp = np.empty(n + 1, np.int64)
        col = np.empty(nnz.value, np.int32)
        k = np.empty(nnz.value)
        m = np.empty(nnz.value)
        B.check(L.dec_bpm_export_operators(self._h, _ptr(h0, ctypes.c_double), _ptr(v, ctypes.c_double),
                                           _ptr(w, ctypes.c_double), ctypes.byref(nnz), _ptr(rp, ctypes.c_int64),
                                           _ptr(col, ctypes.c_int32), _ptr(k, ctypes.c_double),
                                           _ptr(m, ctypes.c_double)))
        return dict(h0=h0, v=v, w=w, row_ptr=rp, col=col, K=k, QtDQ=m)

    def vertex_tiles(self):
        """(tile of each caller vertex in the current launch mode, rows per tile); -1 without tiles."""
        tile = np.empty(self.n_vert, dtype=np.int32)
        ts = ctypes.c_int32(0)
        B.check(B.lib().dec_bpm_vertex_tiles(self._h, _ptr(tile, ctypes.c_int32), ctypes.byref(ts)))
        return tile, ts.value

    def export_pml(self):
        """Complex-stretched dual areas and K (pattern of ``export_operators``) of a PML handle."""
        ops = self.export_operators()
        h0p = np.empty(2 * self.n_vert)
        kp = np.empty(2 * ops["col"].size)
        B.check(B.lib().dec_bpm_export_pml(self._h, _ptr(h0p, ctypes.c_double), _ptr(kp, ctypes.c_double)))
        return dict(ops, h0p=h0p[0::2] + 1j * h0p[1::2], Kp=kp[0::2] + 1j * kp[1::2])

    # ---- device calls ----
    def _field(self, x: torch.Tensor, name="field", n=None):
        n = self.n_vert if n is None else n
        if not isinstance(x, torch.Tensor) or x.device.type != "cuda":
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if x.dtype != self.torch_dtype or not x.is_contiguous() or x.numel() != n:
            raise TypeError(f"{name} must be a contiguous {self.torch_dtype} tensor with {n} entries")
        return ctypes.c_void_p(x.data_ptr())

    def propagate(self, field: torch.Tensor, dz: float, n_steps: int, gamma: float = 1.0, stream=None):
        """March ``n_steps`` Strang steps in place on ``field`` (asynchronous)."""
        B.check(B.lib().dec_bpm_propagate(self._h, self._field(field), float(dz), int(n_steps), float(gamma),
                                          _stream(stream)))
        return field

    def propagate_noalloc(self, field: torch.Tensor, dz: float, n_steps: int, gamma: float = 1.0, stream=None):
        """``propagate`` through the library's static scratch: allocates nothing (see the header)."""
        B.check(B.lib().dec_bpm_propagate_noalloc(self._h, self._field(field), float(dz), int(n_steps), float(gamma),
                                                  _stream(stream)))
        return field

    def propagate_unsplit(self, field: torch.Tensor, dz: float, n_steps: int, gamma: float = 1.0, stream=None):
        """March ``n_steps`` classical RK4 steps of the whole right-hand side (Kerr term inside
        every stage) in place on ``field`` (asynchronous)."""
        B.check(B.lib().dec_bpm_propagate_unsplit(self._h, self._field(field), float(dz), int(n_steps),
                                                  float(gamma), _stream(stream)))
        return field

    def propagate_adaptive(self, field: torch.Tensor, z_end: float, h0: float, gamma: float = 1.0,
                           rtol: float = 1e-9, atol: float = 1e-11, max_attempts: int = 1 << 40, stream=None):
        """Adaptive Dormand-Prince 5(4) on the whole right-hand side from z = 0 to ``z_end``
        (first trial step ``h0``), in place on ``field``.  Synchronises the stream and returns
        the counters ``{"accepted", "rejected", "last_h", "z"}``; on a failed run the
        raised error carries them as ``.stats``."""
        acc, rej = ctypes.c_int64(0), ctypes.c_int64(0)
        lh, zr = ctypes.c_double(0.0), ctypes.c_double(0.0)
        code = B.lib().dec_bpm_propagate_adaptive(self._h, self._field(field), float(z_end), float(h0), float(gamma),
                                                  float(rtol), float(atol), int(max_attempts), ctypes.byref(acc),
                                                  ctypes.byref(rej), ctypes.byref(lh), ctypes.byref(zr),
                                                  _stream(stream))
        stats = {"accepted": acc.value, "rejected": rej.value, "last_h": lh.value, "z": zr.value}
        try:
            B.check(code)
        except DecBpmError as e:
            e.stats = stats
            raise
        return stats

    def find_mode(self, field: torch.Tensor, power: float, dtau: float, gamma: float = 1.0, tol: float = 1e-10,
                  max_iter: int = 1 << 40, stream=None):
        """Nonlinear eigenmode of the given power by imaginary-z RK4 with renormalisation,
        started from ``field`` and returned in it.  Synchronises the stream and returns
        ``{"mu", "residual", "iterations"}``; on a failed run the raised error carries them
        as ``.stats``."""
        mu, res, it = ctypes.c_double(0.0), ctypes.c_double(0.0), ctypes.c_int64(0)
        code = B.lib().dec_bpm_find_mode(self._h, self._field(field), float(power), float(dtau), float(gamma),
                                         float(tol), int(max_iter), ctypes.byref(mu), ctypes.byref(res),
                                         ctypes.byref(it), _stream(stream))
        stats = {"mu": mu.value, "residual": res.value, "iterations": it.value}
        try:
            B.check(code)
        except DecBpmError as e:
            e.stats = stats
            raise
        return stats

    def check_finite(self, stream=None):
        B.check(B.lib().dec_bpm_check_finite(self._h, _stream(stream)))

    def apply(self, op: str, x: torch.Tensor, stream=None) -> torch.Tensor:
        """``L x``, ``L(L x)`` or ``H_lin x`` computed by the library's kernels."""
        code = {"L": B.OP_L, "L2": B.OP_L2, "H": B.OP_H}[op]
        y = torch.empty_like(x)
        B.check(B.lib().dec_bpm_apply(self._h, code, self._field(x, "x"), self._field(y, "y"), _stream(stream)))
        return y

    def kerr_step(self, field, tau, gamma=1.0, stream=None):
        B.check(B.lib().dec_bpm_kerr_step(self._h, self._field(field), float(tau), float(gamma), _stream(stream)))
        return field

    def linear_step(self, field, dz, stream=None):
        B.check(B.lib().dec_bpm_linear_step(self._h, self._field(field), float(dz), _stream(stream)))
        return field

    def diagnostics(self, field, gamma=1.0, stream=None):
        p, e = ctypes.c_double(), ctypes.c_double()
        B.check(B.lib().dec_bpm_diagnostics(self._h, self._field(field), float(gamma), ctypes.byref(p),
                                            ctypes.byref(e), _stream(stream)))
        return p.value, e.value

    def overlap(self, a, b, stream=None) -> complex:
        re, im = ctypes.c_double(), ctypes.c_double()
        B.check(B.lib().dec_bpm_overlap(self._h, self._field(a, "a"), self._field(b, "b"), ctypes.byref(re),
                                        ctypes.byref(im), _stream(stream)))
        return complex(re.value, im.value)

    def set_index_perturbation(self, dn, stream=None):
        """Install the per-vertex index perturbation dn (float64 CUDA tensor, caller
        order) or None; the library copies its values."""
        if dn is None:
            B.check(B.lib().dec_bpm_set_index_perturbation(self._h, None, _stream(stream)))
            self._dn = None
            return
        if dn.device.type != "cuda" or dn.dtype != torch.float64 or not dn.is_contiguous() or \
                dn.numel() != self.n_vert:
            raise TypeError("dn must be a contiguous float64 CUDA tensor with one entry per vertex")
        B.check(B.lib().dec_bpm_set_index_perturbation(self._h, ctypes.c_void_p(dn.data_ptr()), _stream(stream)))
        self._dn = dn.detach().clone()

    def workspace_size(self, n_steps, every=0) -> int:
        s = ctypes.c_size_t()
        B.check(B.lib().dec_bpm_workspace_size(self._h, int(n_steps), int(every), ctypes.byref(s)))
        return s.value

    def forward_checkpointed(self, field, dz, n_steps, gamma, workspace: torch.Tensor, every=0, stream=None):
        B.check(B.lib().dec_bpm_forward_checkpointed(self._h, self._field(field), float(dz), int(n_steps),
                                                     float(gamma), int(every), ctypes.c_void_p(workspace.data_ptr()),
                                                     workspace.numel() * workspace.element_size(),
                                                     _stream(stream)))
        return field

    def adjoint(self, grad_out, dz, n_steps, gamma, workspace, every=0, want_dn=True, stream=None):
        g0 = torch.empty_like(grad_out)
        gdn = torch.empty(self.n_vert, dtype=torch.float64, device=grad_out.device) if want_dn else None
        B.check(B.lib().dec_bpm_adjoint(self._h, self._field(grad_out, "grad_out"), float(dz), int(n_steps),
                                        float(gamma), int(every), ctypes.c_void_p(workspace.data_ptr()),
                                        workspace.numel() * workspace.element_size(),
                                        self._field(g0, "grad_field0"),
                                        None if gdn is None else ctypes.c_void_p(gdn.data_ptr()), _stream(stream)))
        return g0, gdn

    def autotune(self, dz, gamma=1.0, stream=None):
        B.check(B.lib().dec_bpm_autotune(self._h, float(dz), float(gamma), _stream(stream)))
        return self.tuning

    @property
    def tuning(self):
        t = B.Tuning()
        B.check(B.lib().dec_bpm_get_tuning(self._h, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in B.Tuning._fields_}

    @tuning.setter
    def tuning(self, value):
        cur = self.tuning
        cur.update(value)
        t = B.Tuning(*[int(cur[f]) for f, _ in B.Tuning._fields_])
        B.check(B.lib().dec_bpm_set_tuning(self._h, ctypes.byref(t)))

    def time_kernels(self, dz, gamma=1.0, reps=50, stream=None):
        return _time_kernels(B.lib().dec_bpm_time_kernels, self._h, dz, gamma, reps, stream)


def _time_kernels(fn, h, dz, gamma, reps, stream):
    ms = (ctypes.c_double * B.NUM_KERNELS)()
    by = (ctypes.c_double * B.NUM_KERNELS)()
    B.check(fn(h, float(dz), float(gamma), int(reps), ms, by, _stream(stream)))
    names = {B.K_KERR: "kerr", B.K_STAGE: "stage", B.K_LAP: "lap", B.K_TILE_A: "tile_a", B.K_TILE_B: "tile_b",
             B.K_STEP: "step", B.K_PERSIST: "persist", B.K_UNSPLIT: "unsplit", B.K_DP5: "dp5", B.K_MODE: "mode",
             B.K_DP5_PERSIST: "dp5_persist", B.K_MODE_PERSIST: "mode_persist",
             B.K_UNSPLIT_PERSIST: "unsplit_persist"}
    return {names[k]: {"ms": ms[k], "bytes": by[k]} for k in range(B.NUM_KERNELS)}


class Batch:
    """Many fields on many meshes advanced together.

    ``fields_per_mesh``: one count for every mesh, or a list with one count per
    mesh (counts may differ).  Packed layout: per mesh in order, field-minor
    (``[vertex][field]``) with that mesh's own field count."""

    def __init__(self, meshes, fields_per_mesh):
        counts = [int(fields_per_mesh)] * len(meshes) if np.isscalar(fields_per_mesh) else \
            [int(f) for f in fields_per_mesh]
        if len(counts) != len(meshes):
            raise ValueError("fields_per_mesh needs one count per mesh")
        arr = (ctypes.c_void_p * len(meshes))(*[m.handle.value for m in meshes])
        fpm = np.ascontiguousarray(counts, dtype=np.int32)
        h = ctypes.c_void_p()
        B.check(B.lib().dec_bpm_batch_create(arr, len(meshes), _ptr(fpm, ctypes.c_int32), ctypes.byref(h)))
        self._h = h
        self._destroy = B.lib().dec_bpm_batch_destroy
        _LIVE.add(self)
        self.meshes = list(meshes)
        self.counts = counts
        self.F = counts[0] if len(set(counts)) == 1 else None  # the common count, if there is one
        self.torch_dtype = meshes[0].torch_dtype
        n = ctypes.c_int64()
        B.check(B.lib().dec_bpm_batch_size(h, ctypes.byref(n)))
        self.n_elems = n.value
        self.offsets = np.cumsum([0] + [m.n_vert * f for m, f in zip(meshes, counts)])

    def close(self):
        """Release the batch's device memory now (idempotent)."""
        h = getattr(self, "_h", None)
        self._h = None
        if h is not None and h.value:
            self._destroy(h)

    def __del__(self):
        self.close()

    def pack(self, fields_per_mesh_list):
        """Pack a list (per mesh) of [F_m, N_m] complex tensors into the field-minor layout."""
        parts = [f.transpose(0, 1).contiguous().reshape(-1) for f in fields_per_mesh_list]
        return torch.cat(parts)

    def unpack(self, packed):
        """Views [F_m, N_m] of each mesh's fields in a packed tensor."""
        out = []
        for m, mesh in enumerate(self.meshes):
            seg = packed[self.offsets[m]:self.offsets[m + 1]]
            out.append(seg.reshape(mesh.n_vert, self.counts[m]).transpose(0, 1))
        return out

    def propagate(self, packed: torch.Tensor, dz, n_steps, gamma=1.0, stream=None):
        if packed.device.type != "cuda" or packed.dtype != self.torch_dtype or not packed.is_contiguous() or \
                packed.numel() != self.n_elems:
            raise TypeError(f"packed must be a contiguous {self.torch_dtype} CUDA tensor of {self.n_elems} entries")
        B.check(B.lib().dec_bpm_batch_propagate(self._h, ctypes.c_void_p(packed.data_ptr()), float(dz), int(n_steps),
                                                float(gamma), _stream(stream)))
        return packed

    def check_finite(self, stream=None):
        B.check(B.lib().dec_bpm_batch_check_finite(self._h, _stream(stream)))

    def time_kernels(self, dz, gamma=1.0, reps=20, stream=None):
        return _time_kernels(B.lib().dec_bpm_batch_time_kernels, self._h, dz, gamma, reps, stream)

    def autotune(self, dz, gamma=1.0, stream=None):
        B.check(B.lib().dec_bpm_batch_autotune(self._h, float(dz), float(gamma), _stream(stream)))
        return self.tuning

    @property
    def tuning(self):
        t = B.Tuning()
        B.check(B.lib().dec_bpm_batch_get_tuning(self._h, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in B.Tuning._fields_}

    @tuning.setter
    def tuning(self, value):
        cur = self.tuning
        cur.update(value)
        t = B.Tuning(*[int(cur[f]) for f, _ in B.Tuning._fields_])
        B.check(B.lib().dec_bpm_batch_set_tuning(self._h, ctypes.byref(t)))


class DecBpmFunction(torch.autograd.Function):
    """``u(z_L) = propagate(u0; dn)`` with gradients for ``u0`` and ``dn``.

    Forward runs the checkpointed sweep (checkpoints every ``every`` steps,
    default ceil(sqrt(n_steps))); backward runs the library's adjoint, which
    recomputes each segment from its checkpoint.  Gradients use PyTorch's
    complex convention (dJ/dRe + i dJ/dIm)."""

    @staticmethod
    def forward(ctx, u0, dn, mesh, dz, n_steps, gamma, every):
        # the mesh keeps the perturbation it had: dn is installed for this call only
        prev = mesh._dn
        dn_c = None if dn is None else dn.detach().clone()
        mesh.set_index_perturbation(dn_c)
        try:
            u = u0.detach().clone()
            ws = torch.empty(mesh.workspace_size(n_steps, every), dtype=torch.uint8, device=u0.device)
            mesh.forward_checkpointed(u, dz, n_steps, gamma, ws, every)
        finally:
            mesh.set_index_perturbation(prev)
        ctx.mesh, ctx.ws, ctx.args, ctx.dn = mesh, ws, (dz, n_steps, gamma, every), dn_c
        return u

    @staticmethod
    def backward(ctx, g):
        dz, n_steps, gamma, every = ctx.args
        mesh = ctx.mesh
        prev = mesh._dn
        mesh.set_index_perturbation(ctx.dn)  # the forward's operator (same values, same digest)
        try:
            g0, gdn = mesh.adjoint(g.contiguous(), dz, n_steps, gamma, ctx.ws, every, want_dn=ctx.dn is not None)
        finally:
            mesh.set_index_perturbation(prev)
        return g0, gdn, None, None, None, None, None


def propagate_with_grad(mesh: Mesh, u0: torch.Tensor, dn: torch.Tensor | None, dz: float, n_steps: int,
                        gamma: float = 1.0, every: int = 0) -> torch.Tensor:
    return DecBpmFunction.apply(u0, dn, mesh, dz, n_steps, gamma, every)


def default_every(n_steps: int) -> int:
    return max(1, math.ceil(math.sqrt(max(n_steps, 1))))

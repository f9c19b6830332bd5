"""Thin ctypes binding of the C ABI in ``include/fwi.h`` (and of the PSF,
low-rank, symbol and driver entry points of ``include/fwi_psf.h``,
``include/fwi_lowrank.h``, ``include/fwi_symbol.h`` and ``include/fwi_opt.h``,
wrapped in :mod:`.psf`, :mod:`.lowrank`, :mod:`.symbol` and :mod:`.drivers`).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libfwi_mi355x.so``.  PyTorch supplies device memory (plan block,
workspaces, outputs) and the stream each call is enqueued on.  There is no
CPU fallback: if the library is missing or no GPU is present, calls fail.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfwi_mi355x.so")

(FWI_OP_FORWARD, FWI_OP_BORN, FWI_OP_ADJOINT, FWI_OP_MISFIT_GRAD, FWI_OP_GN_HVP, FWI_OP_MISFIT,
 FWI_OP_GRAD_HVP) = range(7)
STATUS_BAD_MODEL, STATUS_CFL, STATUS_NONFINITE = 1, 2, 4

EXPORTS = ["fwi_abi_version", "fwi_plan_create", "fwi_plan_destroy", "fwi_plan_device_bytes",
           "fwi_plan_bind", "fwi_workspace_size", "fwi_plan_dims", "fwi_forward", "fwi_born",
           "fwi_adjoint", "fwi_misfit_grad", "fwi_gn_hvp", "fwi_status", "fwi_strerror",
           "fwi_last_error", "fwi_profile_enable", "fwi_profile_read", "fwi_profile_reset",
           "fwi_forward_keep", "fwi_adjoint_resume", "fwi_misfit", "fwi_kernel_steps",
           "fwi_psf_check", "fwi_psf_extract", "fwi_psf_apply", "fwi_misfit_grad_hvp",
           "fwi_prior_create", "fwi_prior_destroy", "fwi_prior_device_bytes", "fwi_prior_bind",
           "fwi_prior_workspace_size", "fwi_prior_apply", "fwi_lowrank_workspace_size",
           "fwi_lowrank_range", "fwi_lowrank_project", "fwi_lowrank_apply", "fwi_symbol_check",
           "fwi_symbol_create", "fwi_symbol_destroy", "fwi_symbol_device_bytes",
           "fwi_symbol_bind", "fwi_symbol_workspace_size", "fwi_symbol_apply", "fwi_pdo_probe",
           "fwi_pdo_weights", "fwi_pdo_masks", "fwi_pdo_workspace_size", "fwi_pdo_columns",
           "fwi_psfplus_workspace_size", "fwi_psfplus_build", "fwi_vec_workspace_size",
           "fwi_vec_dot", "fwi_vec_update", "fwi_lbfgs_pair", "fwi_lbfgs_loop1",
           "fwi_lbfgs_loop2", "fwi_plan_set_option", "fwi_plan_get_option",
           "fwi_symbol_set_option", "fwi_symbol_get_option", "fwi_workspace_status",
           "fwi_calib_copy", "fwi_gn_hvp_noalloc"]
KERNEL_STEP, KERNEL_STEP_BORN, KERNEL_ADJOINT = range(3)
# plan options (include/fwi.h, FWI_OPT_*)
OPTIONS = {"two_step_forward": 0, "two_step_born": 1, "two_step_adjoint": 2,
           "adj_vectors": 3, "adj_shot_group": 4, "step_order": 5, "born_order": 6,
           "adj_order": 7, "block_x": 8, "block_z": 9, "lds_poison": 10}
# symbol options (include/fwi_symbol.h, FWI_SYM_OPT_*)
SYMBOL_OPTIONS = {"chunk_mb": 0, "blend_split": 1, "split_960": 2}


class FwiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fwi error {code}: {msg}")
        self.code = code


class _Geometry(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nz", ctypes.c_int32), ("nb", ctypes.c_int32),
                ("nt", ctypes.c_int32), ("dx", ctypes.c_float), ("dt", ctypes.c_float),
                ("kappa_max", ctypes.c_float), ("ns", ctypes.c_int32),
                ("src_zx", ctypes.c_void_p), ("nr", ctypes.c_int32),
                ("rec_zx", ctypes.c_void_p), ("wavelet", ctypes.c_void_p),
                ("ckpt_every", ctypes.c_int32), ("inv_noise_var", ctypes.c_double)]


_lib = None
_lib_lock = threading.Lock()


def load_library(path: str | None = None):
    """Load the in-tree HIP library (raises if it has not been built).  The
    first call fixes the library for the process; `path` (else LIB_PATH)
    names another build of it, such as the sanitizer build."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        path = path or LIB_PATH
        if not os.path.exists(path):
            raise FwiError(-4, f"{path} not built: run __graft_entry__.build()")
        lib = ctypes.CDLL(path)
        P, I, Z, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_double
        L = ctypes.c_int64
        sig = {
            "fwi_abi_version": ([], I),
            "fwi_plan_create": ([P, P], I),
            "fwi_plan_destroy": ([P], None),
            "fwi_plan_device_bytes": ([P, P], I),
            "fwi_plan_bind": ([P, P, Z, P], I),
            "fwi_workspace_size": ([P, I, I, P], I),
            "fwi_plan_dims": ([P, P], I),
            "fwi_forward": ([P, P, P, P, Z, P], I),
            "fwi_born": ([P, P, P, I, P, P, Z, P], I),
            "fwi_adjoint": ([P, P, P, I, P, P, Z, P], I),
            "fwi_misfit_grad": ([P, P, P, P, P, P, Z, P], I),
            "fwi_gn_hvp": ([P, P, P, I, P, P, Z, P], I),
            "fwi_status": ([P, P, P], I),
            "fwi_strerror": ([I], ctypes.c_char_p),
            "fwi_last_error": ([], ctypes.c_char_p),
            "fwi_profile_enable": ([P, I], I),
            "fwi_profile_read": ([P, I, P, P], I),
            "fwi_profile_reset": ([P], I),
            "fwi_forward_keep": ([P, P, P, P, Z, P], I),
            "fwi_adjoint_resume": ([P, P, I, P, P, Z, P], I),
            "fwi_misfit": ([P, P, P, P, P, Z, P], I),
            "fwi_kernel_steps": ([P, I, P], I),
            "fwi_misfit_grad_hvp": ([P, P, P, P, I, P, P, P, P, Z, P], I),
            "fwi_psf_check": ([P], I),
            "fwi_prior_create": ([ctypes.c_int32, ctypes.c_int32, D, D, D, P], I),
            "fwi_prior_destroy": ([P], None),
            "fwi_prior_device_bytes": ([P, P], I),
            "fwi_prior_bind": ([P, P, Z, P], I),
            "fwi_prior_workspace_size": ([P, I, P], I),
            "fwi_prior_apply": ([P, I, P, I, P, P, Z, P], I),
            "fwi_lowrank_workspace_size": ([P, I, I, I, P], I),
            "fwi_lowrank_range": ([P, I, P, D, P, P, P, P, Z, P], I),
            "fwi_lowrank_project": ([P, I, P, P, I, P, P, P, Z, P], I),
            "fwi_lowrank_apply": ([P, I, P, P, I, P, I, P, P, Z, P], I),
            "fwi_psf_extract": ([P, P, P, P], I),
            "fwi_psf_apply": ([P, P, P, I, P, P], I),
            "fwi_symbol_check": ([P], I),
            "fwi_symbol_create": ([P, P], I),
            "fwi_symbol_destroy": ([P], None),
            "fwi_symbol_device_bytes": ([P, P], I),
            "fwi_symbol_bind": ([P, P, Z, P], I),
            "fwi_symbol_workspace_size": ([P, I, I, P], I),
            "fwi_symbol_apply": ([P, I, P, P, ctypes.c_float, P, I, P, P, Z, P], I),
            "fwi_pdo_probe": ([P, P, P], I),
            "fwi_pdo_weights": ([P, P, P], I),
            "fwi_pdo_masks": ([P, P, P], I),
            "fwi_pdo_workspace_size": ([P, P], I),
            "fwi_pdo_columns": ([P, P, P, P, Z, P], I),
            "fwi_psfplus_workspace_size": ([P, P, I, P], I),
            "fwi_psfplus_build": ([P, P, P, P, I, P, P, P, P, Z, P], I),
            "fwi_vec_workspace_size": ([L, P], I),
            "fwi_vec_dot": ([L, P, P, P, P, Z, P], I),
            "fwi_vec_update": ([L, D, P, P, D, P, P], I),
            "fwi_lbfgs_pair": ([L, P, P, P, P, P, Z, P], I),
            "fwi_lbfgs_loop1": ([L, I, P, P, P, P, P, P, P, Z, P], I),
            "fwi_lbfgs_loop2": ([L, I, P, P, P, P, P, P, P, Z, P], I),
            "fwi_plan_set_option": ([P, I, I], I),
            "fwi_plan_get_option": ([P, I, P], I),
            "fwi_symbol_set_option": ([P, I, I], I),
            "fwi_symbol_get_option": ([P, I, P], I),
            "fwi_workspace_status": ([P, P, P, P], I),
            "fwi_calib_copy": ([P, P, Z, I, P], I),
            "fwi_gn_hvp_noalloc": ([P, P, P, I, P, P], I),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
        return lib


def _check(rc):
    if rc != 0:
        lib = load_library()
        raise FwiError(rc, f"{lib.fwi_strerror(rc).decode()}: {lib.fwi_last_error().decode()}")


def _geometry_struct(geom):
    keep = dict(src=np.ascontiguousarray(geom.src_zx, dtype=np.int32),
                rec=np.ascontiguousarray(geom.rec_zx, dtype=np.int32),
                wav=np.ascontiguousarray(geom.wavelet[: geom.nt], dtype=np.float32))
    g = _Geometry(nx=geom.nx, nz=geom.nz, nb=geom.nb, nt=geom.nt, dx=geom.dx, dt=geom.dt,
                  kappa_max=geom.kappa_max, ns=keep["src"].shape[0],
                  src_zx=keep["src"].ctypes.data, nr=keep["rec"].shape[0],
                  rec_zx=keep["rec"].ctypes.data, wavelet=keep["wav"].ctypes.data,
                  ckpt_every=int(geom.ckpt_every), inv_noise_var=float(geom.inv_noise_var))
    return g, keep


class Plan:
    """One acquisition geometry bound to one GPU.

    Methods take and return float32 CUDA tensors (model space [B][nz][nx],
    data space [B][ns][nt][nr]) and enqueue on the current torch stream.
    Workspaces are cached per (operation, batch) unless the caller passes its
    own (``ws=``).  Calls from several threads on different streams are safe
    when each brings its own workspace and telemetry is off.  ``options``
    maps names of :data:`OPTIONS` to values (the plan's tuning options, set
    before the device block is bound).  ``geom.ckpt_every = 0`` keeps the
    whole forward history in the adjoint-bearing workspaces instead of
    checkpoints (no recompute; ``self.K`` then reads nt - 1 and
    ``self.history`` is True).
    """

    def __init__(self, geom, device=None, options=None):
        import torch

        self.torch = torch
        self.lib = load_library()
        self.geom = geom
        self.device = torch.device(device if device is not None else "cuda")
        g, keep = _geometry_struct(geom)
        h = ctypes.c_void_p()
        _check(self.lib.fwi_plan_create(ctypes.byref(g), ctypes.byref(h)))
        self._h = h
        self._ws = {}
        for name, value in (options or {}).items():
            self.set_option(name, value)
        nb = ctypes.c_size_t()
        _check(self.lib.fwi_plan_device_bytes(h, ctypes.byref(nb)))
        self._blk = torch.zeros(max(nb.value, 256), dtype=torch.uint8, device=self.device)
        _check(self.lib.fwi_plan_bind(h, ctypes.c_void_p(self._blk.data_ptr()), nb.value,
                                      self._stream()))
        self._ws = {}
        dims = (ctypes.c_int32 * 6)()
        _check(self.lib.fwi_plan_dims(h, dims))
        self.nzp, self.nxp, self.pitch, self.tiles_z, self.tiles_x, self.K = list(dims)
        self.history = int(geom.ckpt_every) == 0

    # -- plumbing ---------------------------------------------------------
    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.fwi_plan_destroy(h)
            self._h = None

    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def set_option(self, name, value):
        """Set a tuning option (a name of :data:`OPTIONS`); drops the cached
        workspaces, whose size may change."""
        if name not in OPTIONS:
            raise KeyError(f"unknown plan option {name!r}")
        _check(self.lib.fwi_plan_set_option(self._h, OPTIONS[name], int(value)))
        self._ws = {}

    def get_option(self, name):
        v = ctypes.c_int()
        _check(self.lib.fwi_plan_get_option(self._h, OPTIONS[name], ctypes.byref(v)))
        return v.value

    def workspace_bytes(self, op, batch=1):
        n = ctypes.c_size_t()
        _check(self.lib.fwi_workspace_size(self._h, int(op), int(batch), ctypes.byref(n)))
        return n.value

    def workspace(self, op, batch=1):
        key = (int(op), int(batch))
        ws = self._ws.get(key)
        if ws is None:
            nbytes = self.workspace_bytes(op, batch)
            ws = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    def release_workspaces(self):
        self._ws.clear()

    def _in(self, x, shape_tail, name):
        t = self.torch
        if not isinstance(x, t.Tensor) or x.device.type != "cuda" or x.dtype != t.float32:
            raise TypeError(f"{name} must be a float32 CUDA tensor")
        x = x.contiguous()
        if tuple(x.shape[-len(shape_tail):]) != tuple(shape_tail):
            raise ValueError(f"{name} has shape {tuple(x.shape)}, expected (..., {shape_tail})")
        return x

    @staticmethod
    def _p(x):
        return ctypes.c_void_p(x.data_ptr())

    # -- operations -------------------------------------------------------
    def forward(self, m, ws=None):
        g = self.geom
        m = self._in(m, (g.nz, g.nx), "m")
        d = self.torch.empty((g.ns, g.nt, g.nr), dtype=self.torch.float32, device=self.device)
        ws = self.workspace(FWI_OP_FORWARD) if ws is None else ws
        _check(self.lib.fwi_forward(self._h, self._p(m), self._p(d), self._p(ws), ws.numel(),
                                    self._stream()))
        return d

    def born(self, m, v, ws=None):
        g = self.geom
        m = self._in(m, (g.nz, g.nx), "m")
        v = self._in(v, (g.nz, g.nx), "v")
        single = v.dim() == 2
        v = v.reshape(-1, g.nz, g.nx)
        B = v.shape[0]
        dd = self.torch.empty((B, g.ns, g.nt, g.nr), dtype=self.torch.float32, device=self.device)
        ws = self.workspace(FWI_OP_BORN, B) if ws is None else ws
        _check(self.lib.fwi_born(self._h, self._p(m), self._p(v), B, self._p(dd), self._p(ws),
                                 ws.numel(), self._stream()))
        return dd[0] if single else dd

    def adjoint(self, m, r, ws=None):
        g = self.geom
        m = self._in(m, (g.nz, g.nx), "m")
        r = self._in(r, (g.ns, g.nt, g.nr), "r")
        single = r.dim() == 3
        r = r.reshape(-1, g.ns, g.nt, g.nr)
        B = r.shape[0]
        out = self.torch.empty((B, g.nz, g.nx), dtype=self.torch.float32, device=self.device)
        ws = self.workspace(FWI_OP_ADJOINT, B) if ws is None else ws
        _check(self.lib.fwi_adjoint(self._h, self._p(m), self._p(r), B, self._p(out),
                                    self._p(ws), ws.numel(), self._stream()))
        return out[0] if single else out

    def forward_keep(self, m, ws):
        """Forward data, leaving coefficients and checkpoints in `ws` (a
        workspace tensor of workspace_bytes(FWI_OP_ADJOINT, batch) bytes)."""
        g = self.geom
        m = self._in(m, (g.nz, g.nx), "m")
        d = self.torch.empty((g.ns, g.nt, g.nr), dtype=self.torch.float32, device=self.device)
        _check(self.lib.fwi_forward_keep(self._h, self._p(m), self._p(d), self._p(ws),
                                         ws.numel(), self._stream()))
        return d

    def adjoint_resume(self, r, ws):
        """J^T r at the model of the last forward_keep on `ws`."""
        g = self.geom
        r = self._in(r, (g.ns, g.nt, g.nr), "r")
        single = r.dim() == 3
        r = r.reshape(-1, g.ns, g.nt, g.nr)
        B = r.shape[0]
        out = self.torch.empty((B, g.nz, g.nx), dtype=self.torch.float32, device=self.device)
        _check(self.lib.fwi_adjoint_resume(self._h, self._p(r), B, self._p(out), self._p(ws),
                                           ws.numel(), self._stream()))
        return out[0] if single else out

    def new_workspace(self, op, batch=1):
        """A workspace owned by the caller (not cached by the plan)."""
        return self.torch.empty(self.workspace_bytes(op, batch), dtype=self.torch.uint8,
                                device=self.device)

    def misfit(self, m, dobs, out=None, ws=None):
        """Phi = 1/2 inv_noise_var |f(m) - dobs|^2 as a device FP64 scalar."""
        g = self.geom
        m = self._in(m, (g.nz, g.nx), "m")
        dobs = self._in(dobs, (g.ns, g.nt, g.nr), "dobs")
        phi = out if out is not None else self.torch.empty((), dtype=self.torch.float64,
                                                           device=self.device)
        ws = self.workspace(FWI_OP_MISFIT) if ws is None else ws
        _check(self.lib.fwi_misfit(self._h, self._p(m), self._p(dobs), self._p(phi),
                                   self._p(ws), ws.numel(), self._stream()))
        return phi

    def misfit_grad(self, m, dobs, ws=None):
        g = self.geom
        m = self._in(m, (g.nz, g.nx), "m")
        dobs = self._in(dobs, (g.ns, g.nt, g.nr), "dobs")
        phi = self.torch.empty((), dtype=self.torch.float64, device=self.device)
        grad = self.torch.empty((g.nz, g.nx), dtype=self.torch.float32, device=self.device)
        ws = self.workspace(FWI_OP_MISFIT_GRAD) if ws is None else ws
        _check(self.lib.fwi_misfit_grad(self._h, self._p(m), self._p(dobs), self._p(phi),
                                        self._p(grad), self._p(ws), ws.numel(),
                                        self._stream()))
        return phi, grad

    def gn_hvp(self, m, v, out=None, ws=None):
        g = self.geom
        m = self._in(m, (g.nz, g.nx), "m")
        v = self._in(v, (g.nz, g.nx), "v")
        single = v.dim() == 2
        v = v.reshape(-1, g.nz, g.nx)
        B = v.shape[0]
        hv = out if out is not None else self.torch.empty((B, g.nz, g.nx),
                                                          dtype=self.torch.float32,
                                                          device=self.device)
        ws = self.workspace(FWI_OP_GN_HVP, B) if ws is None else ws
        _check(self.lib.fwi_gn_hvp(self._h, self._p(m), self._p(v), B, self._p(hv),
                                   self._p(ws), ws.numel(), self._stream()))
        return hv[0] if single else hv

    def misfit_grad_hvp(self, m, dobs, v, out=None, ws=None):
        """(Phi, grad, H v) at one model in one fused pass (shared forward
        solve and recompute); v is [nz][nx] or [B][nz][nx]."""
        g = self.geom
        m = self._in(m, (g.nz, g.nx), "m")
        dobs = self._in(dobs, (g.ns, g.nt, g.nr), "dobs")
        v = self._in(v, (g.nz, g.nx), "v")
        single = v.dim() == 2
        v = v.reshape(-1, g.nz, g.nx)
        B = v.shape[0]
        t = self.torch
        phi = t.empty((), dtype=t.float64, device=self.device)
        grad = t.empty((g.nz, g.nx), dtype=t.float32, device=self.device)
        hv = out if out is not None else t.empty((B, g.nz, g.nx), dtype=t.float32,
                                                 device=self.device)
        ws = self.workspace(FWI_OP_GRAD_HVP, B) if ws is None else ws
        _check(self.lib.fwi_misfit_grad_hvp(self._h, self._p(m), self._p(dobs), self._p(v), B,
                                            self._p(phi), self._p(grad), self._p(hv),
                                            self._p(ws), ws.numel(), self._stream()))
        return phi, grad, (hv[0] if single else hv)

    def profile(self, enable=True):
        """Bracket every stencil-kernel launch with HIP events (telemetry)."""
        _check(self.lib.fwi_profile_enable(self._h, int(bool(enable))))

    def profile_reset(self):
        _check(self.lib.fwi_profile_reset(self._h))

    def profile_read(self, kind):
        """(total milliseconds, launches) of one kernel kind since the reset."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(self.lib.fwi_profile_read(self._h, int(kind), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def kernel_steps(self, kind):
        """Time steps one launch of kernel `kind` advances (1 or 2)."""
        n = ctypes.c_int32()
        _check(self.lib.fwi_kernel_steps(self._h, int(kind), ctypes.byref(n)))
        return n.value

    def kernel_name(self, kind):
        two = self.kernel_steps(kind) == 2
        return {KERNEL_STEP: "k_step2<false>" if two else "k_step<false>",
                KERNEL_STEP_BORN: "k_step2<true>" if two else "k_step<true>",
                KERNEL_ADJOINT: "k_adjoint2" if two else "k_adjoint"}[kind]

    def workspace_status(self, ws):
        """Synchronise and return the status bits of the last call that used
        workspace tensor `ws` (that call's alone)."""
        st = ctypes.c_uint32()
        _check(self.lib.fwi_workspace_status(self._h, self._p(ws), self._stream(),
                                             ctypes.byref(st)))
        return st.value

    def status(self):
        """Synchronise, return and clear the device status bits."""
        st = ctypes.c_uint32()
        _check(self.lib.fwi_status(self._h, self._stream(), ctypes.byref(st)))
        return st.value

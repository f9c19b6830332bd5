"""Point-spread-function approximation of the misfit Hessian (Sections 3.2
and 3.5): PSFs read off the Hessian products of a few comb probes, blended
with tent weights into an operator that applies in a fraction of a
millisecond instead of the seconds of one Hessian product.

Thin binding of ``include/fwi_psf.h``: the comb products run through
:meth:`fwi.Plan.gn_hvp`; extraction and application run in the HIP kernels
of the same library.  The sampling description is ``synth.PsfGrid``.
"""
from __future__ import annotations

import ctypes

from . import fwi, synth


class _PsfGridC(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("nz", "nx", "oz", "ox", "sz", "sx", "nzc", "nxc", "half", "stride")]


def _grid(g: "synth.PsfGrid") -> _PsfGridC:
    return _PsfGridC(g.nz, g.nx, g.oz, g.ox, g.sz, g.sx, g.nzc, g.nxc, g.half, g.stride)


def _stream(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev(torch, x, shape_tail, name):
    if not isinstance(x, torch.Tensor) or x.device.type != "cuda" or x.dtype != torch.float32:
        raise TypeError(f"{name} must be a float32 CUDA tensor")
    x = x.contiguous()
    if tuple(x.shape[-len(shape_tail):]) != tuple(shape_tail):
        raise ValueError(f"{name} has shape {tuple(x.shape)}, expected (..., {shape_tail})")
    return x


def check(g: "synth.PsfGrid") -> None:
    """Validate a sampling description with the library's own rules."""
    lib = fwi.load_library()
    gc = _grid(g)
    fwi._check(lib.fwi_psf_check(ctypes.byref(gc)))


def extract(g: "synth.PsfGrid", hv, out=None):
    """[r][W][W] PSFs from hv[stride^2][nz][nx], the Hessian products of
    ``synth.psf_combs(g)`` in that order."""
    import torch

    lib = fwi.load_library()
    hv = _dev(torch, hv, (g.ncombs, g.nz, g.nx), "hv")
    psf = out if out is not None else torch.empty((g.r, g.width, g.width), dtype=torch.float32,
                                                  device=hv.device)
    gc = _grid(g)
    fwi._check(lib.fwi_psf_extract(ctypes.byref(gc), ctypes.c_void_p(hv.data_ptr()),
                                   ctypes.c_void_p(psf.data_ptr()), _stream(torch, hv.device)))
    return psf


def apply(g: "synth.PsfGrid", psf, v, out=None):
    """H~ v = sum_k w_k(y) sum_d p_k(d) v(y + d) for v[nz][nx] or
    v[B][nz][nx]."""
    import torch

    lib = fwi.load_library()
    psf = _dev(torch, psf, (g.r, g.width, g.width), "psf")
    v = _dev(torch, v, (g.nz, g.nx), "v")
    single = v.dim() == 2
    v = v.reshape(-1, g.nz, g.nx)
    B = v.shape[0]
    o = out if out is not None else torch.empty((B, g.nz, g.nx), dtype=torch.float32,
                                                device=v.device)
    gc = _grid(g)
    fwi._check(lib.fwi_psf_apply(ctypes.byref(gc), ctypes.c_void_p(psf.data_ptr()),
                                 ctypes.c_void_p(v.data_ptr()), B, ctypes.c_void_p(o.data_ptr()),
                                 _stream(torch, v.device)))
    return o[0] if single else o


class PsfOperator:
    """The PSF approximation of H_d at one model: stride^2 Hessian products
    of comb probes (one batched call), PSFs extracted on the device, applied
    to any number of vectors."""

    def __init__(self, plan: "fwi.Plan", m, g: "synth.PsfGrid"):
        import torch

        check(g)
        if (g.nz, g.nx) != (plan.geom.nz, plan.geom.nx):
            raise ValueError("PSF grid and plan disagree on the model size")
        self.grid = g
        combs = torch.as_tensor(synth.psf_combs(g), dtype=torch.float32, device=plan.device)
        self.hv_combs = plan.gn_hvp(m, combs)
        self.psf = extract(g, self.hv_combs)

    def __call__(self, v, out=None):
        return apply(self.grid, self.psf, v, out=out)

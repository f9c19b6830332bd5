"""Low-rank symbol approximations of the misfit Hessian: PDO probing (Section
3.4, Appendix A) and PSF+ (Section 3.6), applied through the FFT chain of
Section 3.3.  Thin binding of ``include/fwi_symbol.h``.

:class:`Symbol` holds the FFT grid (``synth.SymbolGrid``) and its device
tables.  :class:`LowRankSymbol` is an approximation ready to apply: the
tables (A_t, M_t) and the scale of ``out = scale Re sum_t A_t F^-1 (M_t F
v)``.  :func:`pdo` builds one from a Hessian product of the sinusoid probe,
:func:`psf_plus` from the PSFs and the PDO columns.  Every arithmetic step
runs in the library's HIP kernels; Python sequences the calls and allocates.
"""
from __future__ import annotations

import ctypes

from . import fwi, synth
from .psf import _grid as _psf_grid


class _SymbolGridC(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int32), ("nx", ctypes.c_int32), ("mz", ctypes.c_int32),
                ("mx", ctypes.c_int32), ("h", ctypes.c_double), ("r", ctypes.c_int32),
                ("rho0", ctypes.c_double)]


def _gridc(g: "synth.SymbolGrid") -> _SymbolGridC:
    return _SymbolGridC(g.nz, g.nx, g.mz, g.mx, float(g.h), g.r, float(g.rho0))


def _p(x):
    return ctypes.c_void_p(x.data_ptr())


def _stream(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def check(g: "synth.SymbolGrid") -> None:
    lib = fwi.load_library()
    gc = _gridc(g)
    fwi._check(lib.fwi_symbol_check(ctypes.byref(gc)))


class Symbol:
    """FFT grid and sampling of the symbol approximations."""

    def __init__(self, g: "synth.SymbolGrid", device=None, options=None):
        import torch

        self.torch = torch
        self.g = g
        self.lib = fwi.load_library()
        self.device = torch.device(device if device is not None else "cuda")
        self._gc = _gridc(g)
        h = ctypes.c_void_p()
        fwi._check(self.lib.fwi_symbol_create(ctypes.byref(self._gc), ctypes.byref(h)))
        self._h = h
        for name, value in (options or {}).items():
            self.set_option(name, value)
        nb = ctypes.c_size_t()
        fwi._check(self.lib.fwi_symbol_device_bytes(h, ctypes.byref(nb)))
        self._blk = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=self.device)
        fwi._check(self.lib.fwi_symbol_bind(h, _p(self._blk), nb.value, self._st()))
        self._ws = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.fwi_symbol_destroy(h)
            self._h = None

    def set_option(self, name, value):
        """Set a tuning option (a name of ``fwi.SYMBOL_OPTIONS``)."""
        if name not in fwi.SYMBOL_OPTIONS:
            raise KeyError(f"unknown symbol option {name!r}")
        fwi._check(self.lib.fwi_symbol_set_option(self._h, fwi.SYMBOL_OPTIONS[name], int(value)))

    def _st(self):
        return _stream(self.torch, self.device)

    def _workspace(self, n):
        t = self.torch
        if self._ws is None or self._ws.numel() < n:
            self._ws = t.empty(max(n, 256), dtype=t.uint8, device=self.device)
        return self._ws

    def _check_vec(self, v, shape, name, dtype=None):
        t = self.torch
        dtype = dtype or t.float32
        if not isinstance(v, t.Tensor) or v.device.type != "cuda" or v.dtype != dtype:
            raise TypeError(f"{name} must be a {dtype} CUDA tensor")
        v = v.contiguous()
        if tuple(v.shape[-len(shape):]) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(v.shape)}, expected (..., {shape})")
        return v

    # ---------------------------------------------------------------- apply
    def apply(self, A, M, scale, v, out=None):
        """out = scale Re sum_t A_t F^-1 (M_t F v); A [T][nz][nx] and M
        [T][mz][mx] complex64, v [nz][nx] or [B][nz][nx] float32."""
        t = self.torch
        g = self.g
        A = self._check_vec(A, (g.nz, g.nx), "A", t.complex64)
        M = self._check_vec(M, (g.mz, g.mx), "M", t.complex64)
        if A.shape[0] != M.shape[0]:
            raise ValueError("A and M must hold the same number of terms")
        v = self._check_vec(v, (g.nz, g.nx), "v")
        single = v.dim() == 2
        v = v.reshape(-1, g.nz, g.nx)
        B, T = v.shape[0], A.shape[0]
        o = out if out is not None else t.empty((B, g.nz, g.nx), dtype=t.float32,
                                                device=self.device)
        n = ctypes.c_size_t()
        fwi._check(self.lib.fwi_symbol_workspace_size(self._h, B, T, ctypes.byref(n)))
        ws = self._workspace(n.value)
        fwi._check(self.lib.fwi_symbol_apply(self._h, T, _p(A), _p(M), float(scale), _p(v), B,
                                             _p(o), _p(ws), n.value, self._st()))
        return o[0] if single else o

    # ------------------------------------------------------------------ PDO
    def pdo_probe(self):
        t = self.torch
        vp = t.empty((self.g.nz, self.g.nx), dtype=t.float32, device=self.device)
        fwi._check(self.lib.fwi_pdo_probe(self._h, _p(vp), self._st()))
        return vp

    def pdo_weights(self):
        t = self.torch
        M = t.empty((self.g.r // 2, self.g.mz, self.g.mx), dtype=t.complex64, device=self.device)
        fwi._check(self.lib.fwi_pdo_weights(self._h, _p(M), self._st()))
        return M

    def pdo_masks(self):
        t = self.torch
        M = t.empty((self.g.r // 2, self.g.mz, self.g.mx), dtype=t.complex64, device=self.device)
        fwi._check(self.lib.fwi_pdo_masks(self._h, _p(M), self._st()))
        return M

    def pdo_columns(self, hvp):
        """s_k for k = 1..r/2 from hvp = H_d v_p: [r/2][nz][nx] complex64."""
        t = self.torch
        g = self.g
        hvp = self._check_vec(hvp, (g.nz, g.nx), "hvp")
        cols = t.empty((g.r // 2, g.nz, g.nx), dtype=t.complex64, device=self.device)
        n = ctypes.c_size_t()
        fwi._check(self.lib.fwi_pdo_workspace_size(self._h, ctypes.byref(n)))
        ws = self._workspace(n.value)
        fwi._check(self.lib.fwi_pdo_columns(self._h, _p(hvp), _p(cols), _p(ws), n.value,
                                            self._st()))
        return cols

    # ----------------------------------------------------------------- PSF+
    def psf_plus_tables(self, pg: "synth.PsfGrid", psf, cols, rank: int):
        """(A [T][nz][nx], M [T][mz][mx], info [2 + rank] float64) of PSF+."""
        t = self.torch
        g = self.g
        psf = self._check_vec(psf, (pg.r, pg.width, pg.width), "psf")
        cols = self._check_vec(cols, (g.r // 2, g.nz, g.nx), "cols", t.complex64)
        pgc = _psf_grid(pg)
        n = ctypes.c_size_t()
        fwi._check(self.lib.fwi_psfplus_workspace_size(self._h, ctypes.byref(pgc), int(rank),
                                                       ctypes.byref(n)))
        ws = t.empty(max(n.value, 256), dtype=t.uint8, device=self.device)
        T = (rank + 1) // 2
        A = t.empty((T, g.nz, g.nx), dtype=t.complex64, device=self.device)
        M = t.empty((T, g.mz, g.mx), dtype=t.complex64, device=self.device)
        info = t.zeros(2 + rank, dtype=t.float64, device=self.device)
        fwi._check(self.lib.fwi_psfplus_build(self._h, ctypes.byref(pgc), _p(psf), _p(cols),
                                              int(rank), _p(A), _p(M), _p(info), _p(ws), n.value,
                                              self._st()))
        return A, M, info


class LowRankSymbol:
    """A low-rank symbol approximation ready to apply (eq. "lr-psido")."""

    def __init__(self, sym: Symbol, A, M, scale: float):
        self.sym, self.A, self.M, self.scale = sym, A, M, float(scale)

    @property
    def terms(self) -> int:
        return int(self.A.shape[0])

    def apply(self, v, out=None):
        return self.sym.apply(self.A, self.M, self.scale, v, out=out)

    __call__ = apply


def pdo(sym: Symbol, hvp):
    """PDO approximation from hvp = H_d v_p (v_p = ``sym.pdo_probe()``);
    returns (approximation, symbol columns)."""
    cols = sym.pdo_columns(hvp)
    return LowRankSymbol(sym, cols, sym.pdo_weights(), 2.0), cols


def psf_plus(sym: Symbol, pg: "synth.PsfGrid", psf, cols, rank: int):
    """PSF+ approximation from the PSFs and the PDO columns; returns
    (approximation, info) with info = [alpha, kept rows, sigma_1..]."""
    A, M, info = sym.psf_plus_tables(pg, psf, cols, rank)
    return LowRankSymbol(sym, A, M, 1.0), info

"""MI355X-native matrix-free Gauss-Newton Hessian-vector products for 2-D
acoustic full-waveform inversion.

The hot path (forward, Born, adjoint and imaging solves summed over shots)
runs in hand-written HIP kernels for gfx950 behind the C ABI declared in
``include/fwi.h``; :mod:`paper_2507_10804_amd.fwi` is the thin ctypes binding
(PyTorch supplies device memory and streams only).  Submodules are imported
lazily so that the input generators work without a GPU.
"""
__all__ = ["fwi", "synth", "autograd", "probing", "serve"]

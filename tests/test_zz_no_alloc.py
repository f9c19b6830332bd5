"""The allocation-free entry point fwi_gn_hvp_noalloc (fixed device scratch
array instead of a caller workspace), called through the C ABI: two calls in
a row, the second on a smaller problem, each equal to fwi_gn_hvp with a
caller workspace on the same inputs (same kernels and launch shapes, so bit
for bit), and the first against the FP64 oracle."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_2507_10804_amd import fwi, synth
from tests._cases import rel, tiny

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _noalloc(lib):
    fn = lib.fwi_gn_hvp_noalloc
    P = ctypes.c_void_p
    fn.argtypes = [P, P, P, ctypes.c_int, P, P]
    fn.restype = ctypes.c_int
    return fn


def _call(torch, plan, fn, m, v):
    g = plan.geom
    B = v.shape[0]
    hv = torch.full((B, g.nz, g.nx), float("nan"), dtype=torch.float32, device="cuda")
    rc = fn(plan._h, ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(v.data_ptr()), B,
            ctypes.c_void_p(hv.data_ptr()), plan._stream())
    fwi._check(rc)
    torch.cuda.synchronize()
    return hv


def test_noalloc_matches_workspace_call():
    import torch
    lib = fwi.load_library()
    fn = _noalloc(lib)
    dev = lambda a: torch.as_tensor(np.asarray(a, np.float32), device="cuda")
    # first call: the 128 x 128, 4-shot, 500-step problem with 3 vectors
    g1, _, m1 = synth.config_small()
    v1 = synth.smooth_random_batch(g1.nz, g1.nx, seeds=[41, 42, 43])
    p1 = fwi.Plan(g1)
    say("entry: fwi_gn_hvp_noalloc 128x128, 4 shots, nt=500, B=3")
    a1 = _call(torch, p1, fn, dev(m1), dev(v1))
    ref1 = p1.gn_hvp(dev(m1), dev(v1))
    torch.cuda.synchronize()
    assert p1.status() == 0
    assert torch.equal(a1, ref1)
    assert rel(a1[1].double().cpu().numpy(), oracle.gn_hvp(g1, m1, v1[1])) < 1e-4
    # second call: a smaller problem (another plan, one vector) on the same array
    g2, m2 = tiny(nt=140)
    v2 = synth.smooth_random_batch(g2.nz, g2.nx, seeds=[44], sigma=2.0)
    p2 = fwi.Plan(g2)
    say("entry: fwi_gn_hvp_noalloc tiny 48x40, 3 shots, nt=140, B=1")
    a2 = _call(torch, p2, fn, dev(m2), dev(v2))
    ref2 = p2.gn_hvp(dev(m2), dev(v2))
    torch.cuda.synchronize()
    assert p2.status() == 0
    assert torch.equal(a2, ref2)
    # the first problem again, after the smaller one left its contents behind
    a3 = _call(torch, p1, fn, dev(m1), dev(v1))
    assert torch.equal(a3, ref1)


def test_noalloc_refuses_oversized_problem():
    """A problem whose workspace exceeds the fixed array is refused with
    FWI_ENOMEM and a message, before any device work."""
    lib = fwi.load_library()
    fn = _noalloc(lib)
    g, _, _ = synth.config_small()
    g = g.with_shots(range(4))
    g.nt = 4000
    g.wavelet = synth.ricker(4000, g.dt, g.f0)
    p = fwi.Plan(g)
    rc = fn(p._h, None, None, 8, None, None)
    assert rc == -3
    assert b"fixed" in lib.fwi_last_error()

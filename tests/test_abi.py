"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and its host-side plan logic validates arguments and sizes
workspaces (no compute call is made here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2507_10804_amd import fwi, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


@pytest.fixture(scope="module")
def lib():
    return fwi.load_library()


def declared_functions():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fwi_[a-z0-9_]+)\s*\(", text)))


def test_header_matches_binding():
    assert declared_functions() == sorted(fwi.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert lib.fwi_abi_version() == 1


def _plan(lib, geom):
    g, keep = fwi._geometry_struct(geom)
    h = ctypes.c_void_p()
    rc = lib.fwi_plan_create(ctypes.byref(g), ctypes.byref(h))
    return rc, h, keep


def test_plan_host_logic(lib):
    geom, _, _ = synth.config_small()
    rc, h, _ = _plan(lib, geom)
    assert rc == 0
    dims = (ctypes.c_int32 * 6)()
    assert lib.fwi_plan_dims(h, dims) == 0
    nzp, nxp, pitch, tz, tx, K = list(dims)
    assert (nzp, nxp) == (168, 168)
    assert pitch % 64 == 0 and pitch >= nxp and tx == pitch // 64 and tz * 32 >= nzp
    assert K == 50
    nb = ctypes.c_size_t()
    assert lib.fwi_plan_device_bytes(h, ctypes.byref(nb)) == 0 and nb.value > 0
    sizes = {}
    for op in range(6):
        for B in (1, 4):
            n = ctypes.c_size_t()
            assert lib.fwi_workspace_size(h, op, B, ctypes.byref(n)) == 0
            sizes[op, B] = n.value
            assert n.value % 256 == 0
    # batched operations need more memory, single-vector ones do not change
    assert sizes[fwi.FWI_OP_GN_HVP, 4] > sizes[fwi.FWI_OP_GN_HVP, 1]
    assert sizes[fwi.FWI_OP_FORWARD, 4] == sizes[fwi.FWI_OP_FORWARD, 1]
    n = ctypes.c_size_t()
    assert lib.fwi_workspace_size(h, 9, 1, ctypes.byref(n)) == -1
    # a compute call on an unbound plan is refused before touching the GPU
    rc = lib.fwi_forward(h, None, None, None, 0, None)
    assert rc == -6
    assert b"fwi_plan_bind" in lib.fwi_last_error()
    lib.fwi_plan_destroy(h)


@pytest.mark.parametrize("field,value,needle", [
    ("nt", 1, b"nt"),
    ("dx", 0.0, b"dx"),
    ("kappa_max", 0.7, b"kappa_max"),
    ("ckpt_every", -1, b"ckpt_every"),
    ("src", [[0, 200]], b"source 0"),
    ("rec", [[-1, 3]], b"receiver 0"),
    ("nb", -1, b"nb"),
])
def test_plan_rejects_bad_geometry(lib, field, value, needle):
    geom, _, _ = synth.config_small()
    if field == "src":
        geom.src_zx = np.array(value, dtype=np.int32)
    elif field == "rec":
        geom.rec_zx = np.array(value, dtype=np.int32)
    else:
        setattr(geom, field, value)
    rc, h, _ = _plan(lib, geom)
    assert rc == -1
    assert needle in lib.fwi_last_error()
    assert not h.value


def test_strerror(lib):
    for code in (0, -1, -2, -3, -4, -5, -6, -99):
        assert isinstance(lib.fwi_strerror(code), bytes)


def test_psf_grid_validation(lib):
    """Host-side checks of the PSF sampling description (no kernel runs)."""
    from paper_2507_10804_amd import psf as gpsf

    good = [synth.psf_grid(301, 921), synth.PsfGrid(1, 1, 0, 0, 1, 1, 1, 1, 0, 1),
            synth.PsfGrid(64, 64, 0, 0, 32, 32, 2, 2, 32, 1)]
    for g in good:
        gpsf.check(g)
    bad = [synth.PsfGrid(37, 45, 3, 3, 8, 8, 5, 7, 5, 2),    # last centre column outside
           synth.PsfGrid(37, 45, -1, 3, 8, 8, 1, 1, 5, 2),   # negative offset
           synth.PsfGrid(37, 45, 3, 3, 0, 8, 1, 1, 5, 2),    # zero spacing
           synth.PsfGrid(37, 45, 3, 3, 8, 8, 0, 1, 5, 2),    # no centres
           synth.PsfGrid(37, 45, 3, 3, 8, 8, 1, 1, 33, 2),   # window too wide
           synth.PsfGrid(37, 45, 3, 3, 8, 8, 1, 1, 5, 0)]    # no combs
    for g in bad:
        with pytest.raises(fwi.FwiError) as ei:
            gpsf.check(g)
        assert ei.value.code == -1


def test_symbol_grid_validation(lib):
    """Host-side checks of the FFT grid of the symbol approximations, and the
    host tables of a symbol object (no kernel runs)."""
    import ctypes

    from paper_2507_10804_amd import symbol as gsym

    good = [synth.symbol_grid(301, 921, 10.0, 31, r=8, rho0=0.02),
            synth.SymbolGrid(1, 1, 1, 1, 1.0, 2, 1.0),
            synth.SymbolGrid(7, 9, 2048, 1125, 0.5, 16, 3.0)]
    for g in good:
        gsym.check(g)
    bad = [synth.SymbolGrid(10, 10, 9, 10, 1.0, 8, 1.0),      # FFT grid smaller than the model
           synth.SymbolGrid(10, 10, 14, 10, 1.0, 8, 1.0),     # factor 7
           synth.SymbolGrid(10, 10, 10, 4096, 1.0, 8, 1.0),   # longer than 2048
           synth.SymbolGrid(10, 10, 10, 10, 0.0, 8, 1.0),     # spacing
           synth.SymbolGrid(10, 10, 10, 10, 1.0, 7, 1.0),     # odd r
           synth.SymbolGrid(10, 10, 10, 10, 1.0, 18, 1.0),    # too many directions
           synth.SymbolGrid(10, 10, 10, 10, 1.0, 8, 0.0)]     # radius
    for g in bad:
        with pytest.raises(fwi.FwiError) as ei:
            gsym.check(g)
        assert ei.value.code == -1
    gc = gsym._gridc(good[0])
    h = ctypes.c_void_p()
    assert lib.fwi_symbol_create(ctypes.byref(gc), ctypes.byref(h)) == 0
    n = ctypes.c_size_t()
    assert lib.fwi_symbol_device_bytes(h, ctypes.byref(n)) == 0
    assert n.value == 8 * (good[0].mz + good[0].mx)
    # unbound object: the compute entry points refuse before touching the GPU
    assert lib.fwi_pdo_columns(h, ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16),
                               1 << 30, None) == -6
    lib.fwi_symbol_destroy(h)


def test_psfplus_and_vector_validation(lib):
    """Argument checks of the PSF+ and driver entry points, all taken before
    any device work (no GPU needed)."""
    import ctypes

    from paper_2507_10804_amd import psf as gpsf
    from paper_2507_10804_amd import symbol as gsym

    G = synth.symbol_grid(301, 921, 10.0, 31, r=8, rho0=0.02)
    gc = gsym._gridc(G)
    h = ctypes.c_void_p()
    assert lib.fwi_symbol_create(ctypes.byref(gc), ctypes.byref(h)) == 0
    n = ctypes.c_size_t()
    pg = gpsf._grid(synth.psf_grid(301, 921))
    assert lib.fwi_psfplus_workspace_size(h, ctypes.byref(pg), 16, ctypes.byref(n)) == 0
    assert n.value > 0
    for rank in (0, 33):
        assert lib.fwi_psfplus_workspace_size(h, ctypes.byref(pg), rank, ctypes.byref(n)) == -1
    other = gpsf._grid(synth.psf_grid(300, 921))  # a different model
    assert lib.fwi_psfplus_workspace_size(h, ctypes.byref(other), 4, ctypes.byref(n)) == -1
    wide = gpsf._grid(synth.PsfGrid(301, 921, 16, 16, 32, 32, 9, 29, 32, 2))  # W = 65 fits 360
    assert lib.fwi_psfplus_workspace_size(h, ctypes.byref(wide), 4, ctypes.byref(n)) == 0
    lib.fwi_symbol_destroy(h)
    # vector algebra
    assert lib.fwi_vec_workspace_size(0, ctypes.byref(n)) == -1
    assert lib.fwi_vec_workspace_size(1 << 31, ctypes.byref(n)) == -1
    assert lib.fwi_vec_workspace_size(1000, ctypes.byref(n)) == 0
    fake = ctypes.c_void_p(256)
    order = (ctypes.c_int * 65)(*range(65))
    assert lib.fwi_lbfgs_loop1(1000, 65, order, fake, fake, fake, fake, fake, fake, n.value,
                               None) == -1
    bad = (ctypes.c_int * 1)(64)  # slot out of range
    assert lib.fwi_lbfgs_loop2(1000, 1, bad, fake, fake, fake, fake, fake, fake, n.value,
                               None) == -1
    assert lib.fwi_vec_dot(1000, fake, fake, fake, fake, n.value - 8, None) == -3


def test_plan_options(lib):
    """Tuning options live in the ABI: defaults readable, ranges enforced,
    block sizes only before binding, and the two-step switches change the
    workspace layout (two field sets) but nothing else."""
    geom, _, _ = synth.config_small()
    rc, h, _ = _plan(lib, geom)
    assert rc == 0
    v = ctypes.c_int()
    defaults = {}
    for name, opt in fwi.OPTIONS.items():
        assert lib.fwi_plan_get_option(h, opt, ctypes.byref(v)) == 0
        defaults[name] = v.value
    assert defaults == {"two_step_forward": 0, "two_step_born": 1, "two_step_adjoint": 1,
                        "adj_vectors": 0, "adj_shot_group": 0, "step_order": 0,
                        "born_order": 0, "adj_order": 0, "block_x": 2, "block_z": 2,
                        "lds_poison": 0}
    for opt, bad in [(fwi.OPTIONS["two_step_born"], 2), (fwi.OPTIONS["adj_vectors"], 5),
                     (fwi.OPTIONS["step_order"], -1), (fwi.OPTIONS["block_x"], 0),
                     (fwi.OPTIONS["block_z"], 65), (fwi.OPTIONS["lds_poison"], 2), (11, 0), (-1, 0)]:
        assert lib.fwi_plan_set_option(h, opt, bad) == -1
    n_two, n_one = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.fwi_workspace_size(h, fwi.FWI_OP_GN_HVP, 4, ctypes.byref(n_two)) == 0
    for name in ("two_step_born", "two_step_adjoint"):
        assert lib.fwi_plan_set_option(h, fwi.OPTIONS[name], 0) == 0
    assert lib.fwi_workspace_size(h, fwi.FWI_OP_GN_HVP, 4, ctypes.byref(n_one)) == 0
    assert n_one.value < n_two.value
    steps = ctypes.c_int32()
    assert lib.fwi_kernel_steps(h, fwi.KERNEL_ADJOINT, ctypes.byref(steps)) == 0
    assert steps.value == 1
    assert lib.fwi_plan_set_option(h, fwi.OPTIONS["block_x"], 4) == 0
    assert lib.fwi_plan_get_option(h, fwi.OPTIONS["block_x"], ctypes.byref(v)) == 0
    assert v.value == 4
    lib.fwi_plan_destroy(h)
    # an odd checkpoint interval keeps every kernel at one step per launch
    geom.ckpt_every = 7
    rc, h, _ = _plan(lib, geom)
    assert lib.fwi_plan_set_option(h, fwi.OPTIONS["two_step_forward"], 1) == 0
    for kind in (fwi.KERNEL_STEP, fwi.KERNEL_STEP_BORN, fwi.KERNEL_ADJOINT):
        assert lib.fwi_kernel_steps(h, kind, ctypes.byref(steps)) == 0 and steps.value == 1
    lib.fwi_plan_destroy(h)


def test_history_mode_host_logic(lib):
    """ckpt_every = 0 keeps the whole forward history: K reads nt - 1, the
    adjoint-bearing workspaces hold (nt - 1) ns fields of w and no checkpoints,
    the forward-only ones do not change, and the two-step kernels stay on
    whatever the parity of nt - 1 (no checkpoint level has to fall on a launch
    boundary)."""
    geom, _, _ = synth.config_small()
    sizes = {}
    for ck in (50, 0):
        geom.ckpt_every = ck
        rc, h, _ = _plan(lib, geom)
        assert rc == 0
        dims = (ctypes.c_int32 * 6)()
        assert lib.fwi_plan_dims(h, dims) == 0
        nzp, nxp, pitch, tz, tx, K = list(dims)
        assert K == (geom.nt - 1 if ck == 0 else 50)
        fs = tz * 32 * pitch
        for op in (fwi.FWI_OP_FORWARD, fwi.FWI_OP_GN_HVP):
            n = ctypes.c_size_t()
            assert lib.fwi_workspace_size(h, op, 2, ctypes.byref(n)) == 0
            sizes[ck, op] = n.value
        steps = ctypes.c_int32()
        for kind in (fwi.KERNEL_STEP_BORN, fwi.KERNEL_ADJOINT):
            assert lib.fwi_kernel_steps(h, kind, ctypes.byref(steps)) == 0 and steps.value == 2
        lib.fwi_plan_destroy(h)
    assert sizes[0, fwi.FWI_OP_FORWARD] == sizes[50, fwi.FWI_OP_FORWARD]
    nseg = (geom.nt - 1 + 49) // 50
    grow = 4 * fs * geom.ns * ((geom.nt - 1) - 50) - 4 * fs * 2 * geom.ns * nseg
    assert abs(sizes[0, fwi.FWI_OP_GN_HVP] - sizes[50, fwi.FWI_OP_GN_HVP] - grow) <= 256
    # an odd nt - 1 in history mode
    geom.ckpt_every, geom.nt, geom.wavelet = 0, 300, geom.wavelet[:300]
    rc, h, _ = _plan(lib, geom)
    assert rc == 0
    for kind in (fwi.KERNEL_STEP_BORN, fwi.KERNEL_ADJOINT):
        assert lib.fwi_kernel_steps(h, kind, ctypes.byref(steps)) == 0 and steps.value == 2
    lib.fwi_plan_destroy(h)


def test_no_environment_knobs():
    """No source of the library reads the process environment."""
    csrc = os.path.join(ROOT, "paper_2507_10804_amd", "csrc")
    for name in os.listdir(csrc):
        if name.endswith((".hip", ".cpp", ".h")):
            assert "getenv" not in open(os.path.join(csrc, name)).read(), name


def test_noalloc_refuses_oversized_problem_on_host(lib):
    """The allocation-free product checks the problem against its fixed array
    before any device work: the 64-shot, 4000-step full grid is refused with
    FWI_ENOMEM and a message (no GPU needed, the plan is not even bound)."""
    geom, _, _ = synth.config_layered(nt=4000)
    rc, h, _ = _plan(lib, geom)
    assert rc == 0
    fn = lib.fwi_gn_hvp_noalloc
    assert fn(h, None, None, 1, None, None) == -3
    assert b"fixed" in lib.fwi_last_error()
    assert fn(h, None, None, 0, None, None) == -1  # batch out of range
    lib.fwi_plan_destroy(h)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with status 2 and a
    message, before touching any device."""
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2 and "one GPU" in r.stderr



def test_c_example_is_built_and_links():
    """build() also compiles fwi_example, a caller of the C ABI that uses the
    header and the HIP runtime alone; without arguments it loads both libraries,
    prints its usage and exits with status 1 (no GPU call is made)."""
    import subprocess

    from paper_2507_10804_amd.csrc import build as hip_build

    r = subprocess.run([hip_build.EXAMPLE], capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "usage:" in r.stderr

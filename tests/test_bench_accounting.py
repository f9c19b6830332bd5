"""bench.py's roofline accounting, on the CPU: the field updates and the
compulsory bytes each kernel kind is credited with, for the fused and the
separate step, with checkpoints and in history mode."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2507_10804_amd import synth  # noqa: E402


@pytest.fixture(scope="module")
def g():
    return synth.config_layered(ns=16, nt=1000)[0]


def test_field_updates(g):
    per = g.ns * (g.nz + 2 * g.nb) * (g.nx + 2 * g.nb) * (g.nt - 1)
    B = 16
    # fused: one recompute, forward + B Born, B + 1 adjoint fields
    assert bench.field_updates(g, B) == {0: per, 1: (B + 1) * per, 2: (B + 1) * per}
    # separate calls: the gradient's forward plus two recomputes
    assert bench.field_updates(g, B, fused=False) == {0: 3 * per, 1: (B + 1) * per,
                                                      2: (B + 1) * per}
    # history mode: no recompute
    assert bench.field_updates(g, B, hist=True)[0] == 0
    assert bench.field_updates(g, B, fused=False, hist=True)[0] == per
    # the products of separate calls: a recompute, 1 + b Born and b adjoint fields each
    assert bench.hvp_field_updates(g, [4, 2]) == {0: 2 * per, 1: 8 * per, 2: 6 * per}


def test_compulsory_bytes(g):
    Np = (g.nz + 2 * g.nb) * (g.nx + 2 * g.nb)
    B, K = 4, 50
    nseg = (g.nt - 1 + K - 1) // K
    ck = bench.algorithmic_bytes(g, B, nseg, K)
    hi = bench.algorithmic_bytes(g, B, nseg, K, hist=True)
    # history mode: no recompute, the forward + Born launches store w^n at every
    # step instead of a checkpoint pair every K steps; the adjoint is unchanged
    assert hi[0] == 0 and hi[2] == ck[2]
    assert hi[1] - ck[1] == (g.nt - 1) * 4 * g.ns * Np - (nseg - 1) * 8 * g.ns * Np
    # the recompute moves 16 B per point and shot plus its w^n store (4 B), and
    # reads c once per point
    assert ck[0] == (g.nt - 1) * (4 * Np * (3 * g.ns + 1) + 4 * g.ns * Np)
    # every kind at least the headline 16 B per credited field update, less the
    # coefficient c that all fields of a launch share
    upd = bench.field_updates(g, B)
    for kind in (0, 1, 2):
        assert ck[kind] >= 12 * upd[kind]

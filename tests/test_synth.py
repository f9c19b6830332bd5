"""The seeded input recipes (no method arithmetic): the small and the
layered-faulted workloads, the probe vectors and their determinism, checked
against the shapes, ranges and structure the workloads are stated with."""
import math

import numpy as np
import pytest

from paper_2507_10804_amd import synth


def test_small_case_recipe():
    g, m_true, m_eval = synth.config_small()
    assert m_true.shape == m_eval.shape == (128, 128)
    # 2000 m/s background, one +300 and one -300 anomaly of sigma 80 m
    assert m_true.max() == pytest.approx(2300.0, abs=1.0)
    assert m_true.min() == pytest.approx(1700.0, abs=1.0)
    assert np.median(m_true) == pytest.approx(2000.0, abs=5.0)
    hi = np.unravel_index(np.argmax(m_true), m_true.shape)
    lo = np.unravel_index(np.argmin(m_true), m_true.shape)
    for c in (hi, lo):  # centres in the central [0.3, 0.7]^2 of the model
        assert all(0.3 * 128 - 1 <= x <= 0.7 * 128 + 1 for x in c)
    assert 10.0 * math.dist(hi, lo) >= 240.0 - 15.0
    assert (g.ns, g.nr, g.nt, g.nb) == (4, 32, 500, 20)
    assert g.dt == pytest.approx(0.4 * 10.0 / 2300.0)
    # surface shots at columns floor((2k + 1) nx / (2 ns)), receivers at depth cell 1
    assert g.src_zx.tolist() == [[1, (2 * k + 1) * 128 // 8] for k in range(4)]
    assert (g.rec_zx[:, 0] == 1).all()
    # unit-peak Ricker delayed by 1.5 / f0
    k = int(np.argmax(g.wavelet))
    assert g.wavelet[k] == pytest.approx(1.0, abs=1e-3)
    assert k == round(1.5 / 10.0 / g.dt)


def test_layered_faulted_recipe():
    g, m_true, m_eval = synth.config_layered(nt=10)
    assert m_true.shape == m_eval.shape == (301, 921)
    assert (m_true[:30] == 1500.0).all() and (m_eval[:30] == 1500.0).all()
    assert m_true.min() >= 1500.0 and m_true.max() <= 5500.0
    # velocity grows with depth on the whole (layers 1600 -> 5500 below the water)
    col = m_true[30:, 460]
    assert col[-1] > col[0] and np.corrcoef(np.arange(col.size), col)[0, 1] > 0.8
    assert (g.ns, g.nr, g.nb) == (64, 461, 20)
    assert (g.rec_zx[:, 1] == 2 * np.arange(461)).all()
    assert g.dt == pytest.approx(0.4 * 10.0 / 5500.0)
    # the evaluation model is the truth smoothed below the water: no layer jumps
    jump = lambda a: np.abs(np.diff(a[31:], axis=0)).max()
    assert jump(m_eval) < 0.25 * jump(m_true)


def test_probe_vectors():
    combs = synth.impulse_combs(301, 921, count=64, spacing=40, seed=100)
    offs = set()
    for c in combs:
        iz, ix = np.nonzero(c)
        oz, ox = iz.min(), ix.min()
        assert oz < 40 and ox < 40
        assert ((iz - oz) % 40 == 0).all() and ((ix - ox) % 40 == 0).all()
        assert c.sum() == len(range(oz, 301, 40)) * len(range(ox, 921, 40))
        offs.add((oz, ox))
    assert len(offs) == 64  # offsets drawn without replacement
    rad = synth.rademacher_smoothed(64, 80, seeds=[200, 201], sigma=5.0)
    assert rad.shape == (2, 64, 80) and not np.array_equal(rad[0], rad[1])
    v = synth.smooth_random_batch(64, 80, seeds=[1, 2])
    assert np.array_equal(v, synth.smooth_random_batch(64, 80, seeds=[1, 2]))
    assert not np.array_equal(v[0], v[1])


def test_inputs_are_deterministic():
    a = synth.config_small()
    b = synth.config_small()
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert np.array_equal(a[0].wavelet, b[0].wavelet)


def test_anomaly_spacing_the_model_cannot_hold_is_refused():
    with pytest.raises(ValueError, match="cannot be"):
        synth.gaussian_anomaly_model(20, 16, width=60.0, min_sep=120.0)
